// CSR SpMM Y = A W (Alg. 1: the products A X^[0] and A W^[k] for a sparse
// operator).  HBM-bound on the (col, val) stream and, for banded matrices,
// bound by the L2-to-CU gathers of W rows.  A group of G lanes (G = next
// power of two >= number of block columns) owns one row: the group loads G
// (col, val) pairs coalesced, broadcasts them with __shfl, and every lane
// gathers one column of the W row (the group reads the whole W row, ncols * s
// contiguous bytes).  Row blocks are remapped so that each XCD (hardware
// dispatches block b to XCD b % 8) walks one contiguous range of rows: a
// banded matrix then keeps its W window inside that XCD's L2.
#include <algorithm>

#include "internal.h"

namespace lobpcg {

// G = lanes per stored entry (next power of two >= ncols); a row is owned by a
// group of GS = max(G, 16) lanes, which holds NP = GS / G "slots" that take
// stored entries in turn.  The group loads its row's (col, val) pairs in
// chunks of GS (one per lane, coalesced), four chunks up front, broadcasts
// them with __shfl, and issues all gathers of a chunk before accumulating.
// Slot partial sums are combined with xor shuffles at the end.
template <typename TV, typename TW, int G>
__global__ __launch_bounds__(256) void k_spmm_csr(const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci,
                                                  const TV* __restrict__ val,
                                                  const TW* __restrict__ W, int64_t ldw,
                                                  TW* __restrict__ Y, int64_t ldy, int ncols,
                                                  int64_t n, int per_xcd) {
  constexpr int GS = (G < 16) ? 16 : G;
  constexpr int NP = GS / G;
  constexpr int RPB = 256 / GS;
  // narrow blocks (G <= 2) take four chunks per pass: a row's entries then
  // fit one pass, and every gather of the pass is in flight together
  constexpr int NCH = (G <= 2) ? 4 : 2;
  const int b = blockIdx.x;
  const int lb = (b & 7) * per_xcd + (b >> 3);
  const int64_t row = (int64_t)lb * RPB + threadIdx.x / GS;
  const int lg = threadIdx.x & (GS - 1);
  const int slot = lg / G;
  const int c = lg & (G - 1);
  const int gbase = (threadIdx.x & 63) & ~(GS - 1);
  if (row >= n) return;  // the whole group shares the row
  const bool active = c < ncols;
  const int e0 = rp[row], e1 = rp[row + 1];
  TW acc = TW(0);
  for (int e = e0; e < e1; e += NCH * GS) {
    int colr[NCH];
    TV vr[NCH];
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      const int ee = e + k * GS + lg;
      const bool ok = ee < e1;
      colr[k] = ok ? ci[ee] : 0;
      vr[k] = ok ? val[ee] : TV(0);
    }
    if constexpr (G <= 4) {
      // all gathers of the pass first, then the products in the same order
      // as below (entries past the row end contribute 0 * 0)
      TW w[NCH][G];
      TV vv[NCH][G];
#pragma unroll
      for (int k = 0; k < NCH; ++k) {
        const int base_e = e + k * GS;
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int t = slot + NP * u;
          const int cidx = __shfl(colr[k], gbase + t, 64);
          vv[k][u] = __shfl(vr[k], gbase + t, 64);
          w[k][u] = (active && base_e + t < e1) ? W[(int64_t)cidx * ldw + c] : TW(0);
        }
      }
#pragma unroll
      for (int k = 0; k < NCH; ++k)
#pragma unroll
        for (int u = 0; u < G; ++u) acc += (TW)vv[k][u] * w[k][u];
      continue;
    }
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      const int base_e = e + k * GS;
      if (base_e >= e1) break;
      constexpr int UB = (G < 8) ? G : 8;  // gathers in flight per batch
#pragma unroll
      for (int u0 = 0; u0 < G; u0 += UB) {
        TW w[UB];
        TV vv[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int t = slot + NP * (u0 + u);
          const int cidx = __shfl(colr[k], gbase + t, 64);
          vv[u] = __shfl(vr[k], gbase + t, 64);
          w[u] = (active && base_e + t < e1) ? W[(int64_t)cidx * ldw + c] : TW(0);
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) acc += (TW)vv[u] * w[u];
      }
    }
  }
#pragma unroll
  for (int off = G; off < GS; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (slot == 0 && active) Y[row * ldy + c] = acc;
}

template <typename TV, typename TW, int G>
static hipError_t spmm_launch(const int32_t* rp, const int32_t* ci, const TV* val, const TW* W,
                              int64_t ldw, TW* Y, int64_t ldy, int ncols, int64_t n,
                              hipStream_t s) {
  constexpr int GS = (G < 16) ? 16 : G;
  constexpr int RPB = 256 / GS;
  const int64_t nb = (n + RPB - 1) / RPB;
  const int64_t nbp = (nb + 7) / 8 * 8;
  hipLaunchKernelGGL((k_spmm_csr<TV, TW, G>), dim3((unsigned)nbp), dim3(256), 0, s, rp, ci, val,
                     W, ldw, Y, ldy, ncols, n, (int)(nbp / 8));
  return hipGetLastError();
}

template <typename TV, typename TW>
static hipError_t spmm_any(const int32_t* rp, const int32_t* ci, const TV* val, const TW* W,
                           int64_t ldw, TW* Y, int64_t ldy, int ncols, int64_t n, hipStream_t s) {
  if (n < 1 || ncols < 1) return hipErrorInvalidValue;
  // columns beyond 64 are processed in slices of 64
  for (int c0 = 0; c0 < ncols; c0 += 64) {
    const int nc = std::min(64, ncols - c0);
    hipError_t e;
    if (nc <= 1) e = spmm_launch<TV, TW, 1>(rp, ci, val, W + c0, ldw, Y + c0, ldy, nc, n, s);
    else if (nc <= 2) e = spmm_launch<TV, TW, 2>(rp, ci, val, W + c0, ldw, Y + c0, ldy, nc, n, s);
    else if (nc <= 4) e = spmm_launch<TV, TW, 4>(rp, ci, val, W + c0, ldw, Y + c0, ldy, nc, n, s);
    else if (nc <= 8) e = spmm_launch<TV, TW, 8>(rp, ci, val, W + c0, ldw, Y + c0, ldy, nc, n, s);
    else if (nc <= 16) e = spmm_launch<TV, TW, 16>(rp, ci, val, W + c0, ldw, Y + c0, ldy, nc, n, s);
    else if (nc <= 32) e = spmm_launch<TV, TW, 32>(rp, ci, val, W + c0, ldw, Y + c0, ldy, nc, n, s);
    else e = spmm_launch<TV, TW, 64>(rp, ci, val, W + c0, ldw, Y + c0, ldy, nc, n, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t spmm_csr_f64(const int32_t* rp, const int32_t* ci, const double* val, const double* W,
                        int64_t ldw, double* Y, int64_t ldy, int ncols, int64_t n, hipStream_t s) {
  return spmm_any<double, double>(rp, ci, val, W, ldw, Y, ldy, ncols, n, s);
}
hipError_t spmm_csr_f32(const int32_t* rp, const int32_t* ci, const float* val, const float* W,
                        int64_t ldw, float* Y, int64_t ldy, int ncols, int64_t n, hipStream_t s) {
  return spmm_any<float, float>(rp, ci, val, W, ldw, Y, ldy, ncols, n, s);
}

}  // namespace lobpcg
