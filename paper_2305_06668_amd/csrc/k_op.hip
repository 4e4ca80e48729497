// Operator application Y = A W for the matrix kinds the solver accepts
// (Alg. 1: the products A X^[0] and A W^[k]; the method is matrix-free,
// Sec. 3.1, so the operator is an input, not part of the method).
//
//   * CSR SpMM: HBM-bound on the (col, val) stream.  A group of G lanes
//     (G = next power of two >= number of block columns) owns one row: the
//     group loads G (col, val) pairs coalesced, broadcasts them with
//     __shfl, and every lane gathers one column of the W row (the group
//     reads the whole W row, ncols*8 contiguous bytes).  Row blocks are
//     remapped so that each XCD (hardware dispatches block b to XCD b % 8)
//     walks one contiguous range of rows: a banded matrix then keeps its W
//     window inside that XCD's L2.
//   * dense: HBM-bound on A; a wave owns R rows, lanes stride the columns,
//     and the ncols partial sums are reduced across the wave at the end.
#include "internal.h"

namespace lobpcg {

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

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
  constexpr int NCH = 2;
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

// ---------------------------------------------------------------------------
// dense: Y (n x ncols) = A (n x n, lda) W (n x ncols), R rows per wave,
// up to MC columns per launch.

template <typename T, int R, int MC>
__global__ __launch_bounds__(256) void k_dense(const T* __restrict__ A, int64_t lda,
                                               const T* __restrict__ W, int64_t ldw,
                                               T* __restrict__ Y, int64_t ldy, int ncols,
                                               int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t r0 = gw * R;
  if (r0 >= n) return;
  T acc[R][MC];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < MC; ++j) acc[r][j] = T(0);
  const T* arow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) arow[r] = A + min(r0 + r, n - 1) * lda;
  for (int64_t c = lane; c < n; c += 64) {
    T w[MC];
#pragma unroll
    for (int j = 0; j < MC; ++j) w[j] = (j < ncols) ? W[c * ldw + j] : T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T a = arow[r][c];
#pragma unroll
      for (int j = 0; j < MC; ++j) acc[r][j] += a * w[j];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      T v = acc[r][j];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
      acc[r][j] = v;
    }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r0 + r < n)
#pragma unroll
        for (int j = 0; j < MC; ++j)
          if (j < ncols) Y[(r0 + r) * ldy + j] = acc[r][j];
  }
}

template <typename T>
static hipError_t dense_any(const T* A, int64_t lda, const T* W, int64_t ldw, T* Y, int64_t ldy,
                            int ncols, int64_t n, hipStream_t s) {
  if (n < 1 || ncols < 1) return hipErrorInvalidValue;
  constexpr int R = 4;
  const int64_t waves = (n + R - 1) / R;
  const int grid = cdiv(waves, 4);
  for (int c0 = 0; c0 < ncols; c0 += 8) {
    const int nc = std::min(8, ncols - c0);
    if (nc <= 4)
      hipLaunchKernelGGL((k_dense<T, R, 4>), dim3(grid), dim3(256), 0, s, A, lda, W + c0, ldw,
                         Y + c0, ldy, nc, n);
    else
      hipLaunchKernelGGL((k_dense<T, R, 8>), dim3(grid), dim3(256), 0, s, A, lda, W + c0, ldw,
                         Y + c0, ldy, nc, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t dense_apply_f64(const double* A, int64_t lda, const double* W, int64_t ldw, double* Y,
                           int64_t ldy, int ncols, int64_t n, hipStream_t s) {
  return dense_any<double>(A, lda, W, ldw, Y, ldy, ncols, n, s);
}
hipError_t dense_apply_f32(const float* A, int64_t lda, const float* W, int64_t ldw, float* Y,
                           int64_t ldy, int ncols, int64_t n, hipStream_t s) {
  return dense_any<float>(A, lda, W, ldw, Y, ldy, ncols, n, s);
}

// ---------------------------------------------------------------------------
// CSR structure check (run once when the operator is set): row pointers
// non-decreasing from 0 to nnz, every column index inside [0, n).

__global__ void k_csr_check(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            int64_t n, int64_t nnz, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) atomicOr(bad, 1);
  if (i >= n) return;
  const int32_t e0 = rp[i], e1 = rp[i + 1];
  if (e1 < e0 || e0 < 0 || (int64_t)e1 > nnz) {
    atomicOr(bad, 2);
    return;
  }
  for (int32_t e = e0; e < e1; ++e) {
    const int32_t c = ci[e];
    if (c < 0 || (int64_t)c >= n) {
      atomicOr(bad, 4);
      return;
    }
  }
}
hipError_t csr_check(const int32_t* rp, const int32_t* ci, int64_t n, int64_t nnz, int* bad,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_csr_check, dim3(cdiv(n, 256)), dim3(256), 0, s, rp, ci, n, nnz, bad);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gershgorin bound max_i sum_j |a_ij| (used by the precision switch)

__device__ __forceinline__ double block_max(double v, double* sh) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
  return r;
}

__global__ __launch_bounds__(256) void k_csr_rowabs(const int32_t* __restrict__ rp,
                                                    const double* __restrict__ val, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double sh[4];
  double best = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s += fabs(val[e]);
    best = fmax(best, s);
  }
  best = block_max(best, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = best;
}

__global__ __launch_bounds__(256) void k_dense_rowabs(const double* __restrict__ A, int64_t lda,
                                                      int64_t n, double* __restrict__ part) {
  __shared__ double sh[4];
  double best = 0.0;
  // one wave per row
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) s += fabs(A[i * lda + j]);
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    best = fmax(best, s);
  }
  best = block_max(best, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = best;
}

__global__ void k_max_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  __shared__ double sh[4];
  double best = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) best = fmax(best, part[i]);
  best = block_max(best, sh);
  if (threadIdx.x == 0) *out = best;
}

hipError_t csr_norm_bound(const int32_t* rp, const double* val, int64_t n, double* part,
                          double* out, hipStream_t s) {
  const int grid = (int)std::min<int64_t>(kStreamBlocks, cdiv(n, 256));
  hipLaunchKernelGGL(k_csr_rowabs, dim3(grid), dim3(256), 0, s, rp, val, n, part);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, part, grid, out);
  return hipGetLastError();
}

hipError_t dense_norm_bound(const double* A, int64_t lda, int64_t n, double* part, double* out,
                            hipStream_t s) {
  const int grid = (int)std::min<int64_t>(kStreamBlocks, cdiv(n, 4));
  hipLaunchKernelGGL(k_dense_rowabs, dim3(grid), dim3(256), 0, s, A, lda, n, part);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, part, grid, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagonals (inputs of the Jacobi preconditioner)

__global__ void k_csr_diag(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ val, int64_t n, double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] == i) v += val[e];
  d[i] = v;
}
hipError_t csr_diag(const int32_t* rp, const int32_t* ci, const double* val, int64_t n,
                    double* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_csr_diag, dim3(cdiv(n, 256)), dim3(256), 0, s, rp, ci, val, n, diag);
  return hipGetLastError();
}

__global__ void k_dense_diag(const double* __restrict__ A, int64_t lda, int64_t n,
                             double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = A[i * lda + i];
}
hipError_t dense_diag(const double* A, int64_t lda, int64_t n, double* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_diag, dim3(cdiv(n, 256)), dim3(256), 0, s, A, lda, n, diag);
  return hipGetLastError();
}

__global__ void k_kron_diag(const double* __restrict__ A, const double* __restrict__ Vp,
                            int64_t na, double* __restrict__ d) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= na * na) return;
  const int64_t i = idx / na, j = idx - i * na;
  d[idx] = A[i * na + i] + A[j * na + j] + Vp[idx];
}
hipError_t kronsum_diag(const double* A, const double* Vp, int64_t na, double* diag,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_kron_diag, dim3(cdiv(na * na, 256)), dim3(256), 0, s, A, Vp, na, diag);
  return hipGetLastError();
}

}  // namespace lobpcg
