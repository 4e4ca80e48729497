// CSR SpMM Y = A W (Alg. 1: the products A X^[0] and A W^[k] for a sparse
// operator).  The (col, val) stream is read from HBM once; every stored entry
// then needs one row of W (ncols * s contiguous bytes), gathered through L2.
// For the banded workloads the W window stays in L2 (hit rate ~90 %, HBM
// traffic within 1 % of the algorithmic bytes), and what bounds the kernel is
// the rate of L1 misses a CU keeps in flight: one 64- or 128-byte request per
// stored entry whatever the column count, ~0.2 requests per clock per CU at
// ~250 cycles of L2 latency.  Two kernels:
//   * k_spmm_csr_vec (2 fp64 / 4 fp32 columns per lane, 16-byte loads; the
//     block's (col, val) range staged in LDS): the fewest instructions and
//     wave slots per gathered row, used whenever W and ldw allow 16-byte
//     loads and the block has at least 5 (fp64) or 9 (fp32) columns;
//   * k_spmm_csr (one column per lane, (col, val) broadcast by shuffles):
//     narrow or misaligned blocks.
// Row blocks are remapped so that each XCD (hardware dispatches block b to
// XCD b % 8) walks one contiguous range of rows: a banded matrix then keeps
// its W window inside that XCD's L2.  The (col, val) stream is loaded with the
// non-temporal hint so that it does not evict W rows from L2.
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


// 16-byte vector of CPL elements (CPL * sizeof(T) == 16)
template <typename T, int CPL>
struct Vec16;
template <>
struct Vec16<double, 2> {
  typedef double __attribute__((ext_vector_type(2))) type;
};
template <>
struct Vec16<float, 4> {
  typedef float __attribute__((ext_vector_type(4))) type;
};

constexpr int kVecCap = 2048;  // (col, val) entries staged in LDS per pass

// A group of G lanes owns one row; lane l holds columns [l CPL, l CPL + CPL)
// and gathers them with one 16-byte load per stored entry (lanes whose
// columns run past ncols load element by element, or nothing).  The block's
// rows are consecutive, so their stored entries form one contiguous range:
// it is copied to LDS in passes of kVecCap entries (coalesced, non-temporal),
// and every group reads its row's (col, val) pairs from there as broadcasts.
// Entries are accumulated in CSR order, UN gathers in flight per lane.
// Requires W and ldw aligned to CPL elements (16 bytes).
template <typename TV, typename TW, int G, int CPL, int UN>
__global__ __launch_bounds__(256) void k_spmm_csr_vec(const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci,
                                                      const TV* __restrict__ val,
                                                      const TW* __restrict__ W, int64_t ldw,
                                                      TW* __restrict__ Y, int64_t ldy, int ncols,
                                                      int64_t n, int per_xcd) {
  typedef typename Vec16<TW, CPL>::type VT;
  constexpr int RPB = 256 / G;
  __shared__ int32_t scol[kVecCap];
  __shared__ TV sval[kVecCap];
  const int b = blockIdx.x;
  const int lb = (b & 7) * per_xcd + (b >> 3);
  const int64_t r0 = (int64_t)lb * RPB;
  if (r0 >= n) return;  // whole block
  const int64_t rl = min((int64_t)RPB, n - r0);
  const int myr = threadIdx.x / G;
  const int c = (threadIdx.x % G) * CPL;
  const int nv = max(0, min(CPL, ncols - c));  // columns this lane owns
  const int64_t row = r0 + myr;
  const int B0 = rp[r0], B1 = rp[r0 + rl];
  int e0 = 0, e1 = 0;
  if (myr < rl && nv > 0) {
    e0 = rp[row];
    e1 = rp[row + 1];
  }
  TW acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = TW(0);
  for (int p0 = B0; p0 < B1; p0 += kVecCap) {
    const int p1 = min(p0 + kVecCap, B1);
    __syncthreads();  // the previous pass is consumed
    for (int i = p0 + (int)threadIdx.x; i < p1; i += 256) {
      scol[i - p0] = __builtin_nontemporal_load(ci + i);
      sval[i - p0] = __builtin_nontemporal_load(val + i);
    }
    __syncthreads();
    const int a = max(e0, p0) - p0, z = min(e1, p1) - p0;
    for (int e = a; e < z; e += UN) {
      TW w[UN][CPL];
      TW vv[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const bool ok = e + u < z;
        const int col = ok ? scol[e + u] : 0;  // past the row end: row 0, weight 0
        vv[u] = ok ? (TW)sval[e + u] : TW(0);
        const TW* src = W + (int64_t)col * ldw + c;
        if (nv == CPL) {
          const VT t = *reinterpret_cast<const VT*>(src);
#pragma unroll
          for (int q = 0; q < CPL; ++q) w[u][q] = t[q];
        } else {
#pragma unroll
          for (int q = 0; q < CPL; ++q) w[u][q] = (q < nv) ? src[q] : TW(0);
        }
      }
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[q] += vv[u] * w[u][q];
    }
  }
  if (myr < rl) {
    TW* dst = Y + row * ldy + c;
#pragma unroll
    for (int q = 0; q < CPL; ++q)
      if (q < nv) dst[q] = acc[q];
  }
}

template <typename TV, typename TW, int G>
static hipError_t spmm_vec_launch(const int32_t* rp, const int32_t* ci, const TV* val, const TW* W,
                                  int64_t ldw, TW* Y, int64_t ldy, int ncols, int64_t n,
                                  hipStream_t s) {
  constexpr int CPL = 16 / (int)sizeof(TW);
  constexpr int UN = (G <= 4 && sizeof(TW) == 8) ? 8 : 4;
  constexpr int RPB = 256 / G;
  const int64_t nb = (n + RPB - 1) / RPB;
  const int64_t nbp = (nb + 7) / 8 * 8;
  hipLaunchKernelGGL((k_spmm_csr_vec<TV, TW, G, CPL, UN>), dim3((unsigned)nbp), dim3(256), 0, s, rp,
                     ci, val, W, ldw, Y, ldy, ncols, n, (int)(nbp / 8));
  return hipGetLastError();
}

// ---- banded matrices: W staged in LDS, slab by slab ----
// A workgroup of kSlabThreads takes kSlabBlockRows consecutive rows (4 lanes
// per row, 4 of the 16 columns per lane, kSlabUnits rows per thread).  The W
// rows that its entries reference lie in the block's column window
// [win.x, win.y] (computed once per operator); it walks that window in slabs
// of kSlabLds bytes (1024 fp64 or 2048 fp32 W rows of 16 columns), staging
// each slab in LDS once, and every row consumes the entries whose column
// falls in the slab (its columns are sorted, so they are the next ones of the
// row).  The W gathers then come from LDS, but each (col, val) load now
// reads 16 rows' entries at once, slab after slab: on the n = 1e6 banded
// matrix (band +-5000, 16 fp64 columns) this path takes 1.4 ms against the
// gather kernel's 0.38 ms (2.6 ms when every row's next entry was loaded
// together per round), so it is not the default (LOBPCG_OPT_SPMM_SLAB).
template <typename TV, typename TW>
__global__ __launch_bounds__(kSlabThreads) void k_spmm_slab(const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const TV* __restrict__ val,
                                                            const TW* __restrict__ W, int64_t ldw,
                                                            TW* __restrict__ Y, int64_t ldy,
                                                            int ncols, int64_t n,
                                                            const int2* __restrict__ win,
                                                            int per_xcd) {
  // W rows in LDS at a stride of 17 elements: the 16 rows a wave reads at
  // once then start on different banks (at 16 they shared two bank groups)
  constexpr int LS = 17;
  constexpr int SW = kSlabLds / (LS * (int)sizeof(TW));  // W rows per slab
  constexpr int U = kSlabUnits;
  constexpr int RG = kSlabThreads / 4;  // rows taken at once
  extern __shared__ char slab_smem[];
  TW* Ws = reinterpret_cast<TW*>(slab_smem);
  const int b = blockIdx.x;
  const int lb = (b & 7) * per_xcd + (b >> 3);  // XCD b % 8 walks a contiguous range
  const int64_t r0 = (int64_t)lb * kSlabBlockRows;
  if (r0 >= n) return;  // whole block
  const int lane = threadIdx.x & 3, rg = threadIdx.x >> 2;
  int p[U], e[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = r0 + rg + (int64_t)RG * u;
    p[u] = (i < n) ? rp[i] : 0;
    e[u] = (i < n) ? rp[i + 1] : 0;
  }
  TW acc[U][4];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[u][q] = TW(0);
  const int2 w = win[lb];
  if (w.y >= w.x) {
    const int s_lo = w.x / SW, s_hi = w.y / SW;
    for (int s = s_lo; s <= s_hi; ++s) {
      const int64_t c0 = (int64_t)s * SW;
      __syncthreads();  // the previous slab is consumed
      for (int q = threadIdx.x; q < SW * 16; q += kSlabThreads) {
        const int rr = q >> 4, cc = q & 15;
        const int64_t wr = c0 + rr;
        Ws[rr * LS + cc] = (wr < n && cc < ncols) ? W[wr * ldw + cc] : TW(0);
      }
      __syncthreads();
      const int64_t cend = c0 + SW;
      // each row takes its next entries while their columns lie in this slab
#pragma unroll
      for (int u = 0; u < U; ++u) {
        while (p[u] < e[u]) {
          const int col = ci[p[u]];
          if (col >= cend) break;
          const TW v = (TW)val[p[u]];
          const TW* wr = Ws + (col - c0) * LS + 4 * lane;
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[u][q] += v * wr[q];
          ++p[u];
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = r0 + rg + (int64_t)RG * u;
    if (i < n) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 4 * lane + q;
        if (c < ncols) Y[i * ldy + c] = acc[u][q];
      }
    }
  }
}

template <typename TV, typename TW>
static hipError_t spmm_slab_launch(const int32_t* rp, const int32_t* ci, const TV* val,
                                   const TW* W, int64_t ldw, TW* Y, int64_t ldy, int ncols,
                                   int64_t n, const int2* win, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_spmm_slab<TV, TW>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kSlabLds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t nb = (n + kSlabBlockRows - 1) / kSlabBlockRows;
  const int64_t nbp = (nb + 7) / 8 * 8;
  hipLaunchKernelGGL((k_spmm_slab<TV, TW>), dim3((unsigned)nbp), dim3(kSlabThreads), kSlabLds, s,
                     rp, ci, val, W, ldw, Y, ldy, ncols, n, win, (int)(nbp / 8));
  return hipGetLastError();
}

// Column window of each kSlabBlockRows-row block: win[b] = (smallest first
// column, largest last column) over its rows, (INT_MAX, -1) for a block of
// empty rows; *unsorted = 1 if some row's columns decrease.
__global__ __launch_bounds__(256) void k_csr_windows(const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, int64_t n,
                                                     int2* __restrict__ win,
                                                     int* __restrict__ unsorted) {
  __shared__ int slo[256], shi[256];
  const int64_t r0 = (int64_t)blockIdx.x * kSlabBlockRows;
  const int64_t r1 = min(n, r0 + kSlabBlockRows);
  int lo = INT_MAX, hi = -1;
  bool bad = false;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
    const int a = rp[i], z = rp[i + 1];
    if (z > a) {
      lo = min(lo, ci[a]);
      hi = max(hi, ci[z - 1]);
      for (int q = a + 1; q < z; ++q) bad |= ci[q] < ci[q - 1];
    }
  }
  if (bad) *unsorted = 1;
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      slo[threadIdx.x] = min(slo[threadIdx.x], slo[threadIdx.x + w]);
      shi[threadIdx.x] = max(shi[threadIdx.x], shi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) win[blockIdx.x] = make_int2(slo[0], shi[0]);
}

template <typename TV, typename TW>
static hipError_t spmm_any(const int32_t* rp, const int32_t* ci, const TV* val, const TW* W,
                           int64_t ldw, TW* Y, int64_t ldy, int ncols, int64_t n, const int2* win,
                           hipStream_t s) {
  if (n < 1 || ncols < 1) return hipErrorInvalidValue;
  if (win != nullptr) {
    for (int c0 = 0; c0 < ncols; c0 += 16) {
      hipError_t e = spmm_slab_launch<TV, TW>(rp, ci, val, W + c0, ldw, Y + c0, ldy,
                                              std::min(16, ncols - c0), n, win, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  constexpr int CPL = 16 / (int)sizeof(TW);
  // 16-byte loads need W and its row stride aligned to CPL elements; the
  // vector kernel is used from 5 (fp64) / 9 (fp32) columns, below which the
  // one-column-per-lane kernel is as fast, up to 16 lanes per row
  const bool aligned = (reinterpret_cast<uintptr_t>(W) % 16) == 0 && ldw % CPL == 0;
  const int vec_min = (CPL == 2) ? 5 : 9;
  const int slice = aligned ? 16 * CPL : 64;
  for (int c0 = 0; c0 < ncols; c0 += slice) {
    const int nc = std::min(slice, ncols - c0);
    const TW* Wc = W + c0;
    TW* Yc = Y + c0;
    hipError_t e;
    if (aligned && nc >= vec_min) {
      const int lanes = (nc + CPL - 1) / CPL;
      if (lanes <= 4) e = spmm_vec_launch<TV, TW, 4>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
      else if (lanes <= 8) e = spmm_vec_launch<TV, TW, 8>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
      else e = spmm_vec_launch<TV, TW, 16>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
    } else if (nc <= 1) e = spmm_launch<TV, TW, 1>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
    else if (nc <= 2) e = spmm_launch<TV, TW, 2>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
    else if (nc <= 4) e = spmm_launch<TV, TW, 4>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
    else if (nc <= 8) e = spmm_launch<TV, TW, 8>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
    else if (nc <= 16) e = spmm_launch<TV, TW, 16>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
    else if (nc <= 32) e = spmm_launch<TV, TW, 32>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
    else e = spmm_launch<TV, TW, 64>(rp, ci, val, Wc, ldw, Yc, ldy, nc, n, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t spmm_csr_f64(const int32_t* rp, const int32_t* ci, const double* val, const double* W,
                        int64_t ldw, double* Y, int64_t ldy, int ncols, int64_t n, const int2* win,
                        hipStream_t s) {
  return spmm_any<double, double>(rp, ci, val, W, ldw, Y, ldy, ncols, n, win, s);
}
hipError_t spmm_csr_f32(const int32_t* rp, const int32_t* ci, const float* val, const float* W,
                        int64_t ldw, float* Y, int64_t ldy, int ncols, int64_t n, const int2* win,
                        hipStream_t s) {
  return spmm_any<float, float>(rp, ci, val, W, ldw, Y, ldy, ncols, n, win, s);
}
hipError_t csr_windows(const int32_t* rp, const int32_t* ci, int64_t n, int2* win, int* unsorted,
                       hipStream_t s) {
  const int64_t nb = (n + kSlabBlockRows - 1) / kSlabBlockRows;
  if (nb < 1) return hipSuccess;
  hipLaunchKernelGGL(k_csr_windows, dim3((unsigned)nb), dim3(256), 0, s, rp, ci, n, win, unsorted);
  return hipGetLastError();
}

}  // namespace lobpcg
