// Operator application Y = A W for the matrix kinds the solver accepts
// (Alg. 1: the products A X^[0] and A W^[k]; the method is matrix-free,
// Sec. 3.1, so the operator is an input, not part of the method).
//
//   * CSR SpMM: in k_spmm.hip.
//   * dense: HBM-bound on A; a wave owns R rows, lanes stride the columns,
//     and the ncols partial sums are reduced across the wave at the end.
#include "internal.h"

namespace lobpcg {

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

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

// Vector form for aligned operands: a wave owns R = 8 rows; lanes take
// VE = 16 / sizeof(T) adjacent columns per step (one 16-byte load per row),
// so each W row fetched (as 16-byte vectors, from L2) serves 8 rows of A,
// and the ncols x R sums are reduced across the wave once at the end, one
// output value per lane.  Fewer rows per wave re-read W more often (4 rows:
// half the rate); splitting a row group's columns over 2 or 4 waves, with a
// reduction through LDS, ran 30-45 % slower.  Walking A by column strips
// instead (A symmetric, Y = A^T W, lanes owning output rows, W rows shared
// through LDS) ran at 0.3 TB/s: every step moves to another row of A.
// Sharing each chunk of W rows among a workgroup's 4 waves through LDS
// (double-buffered, one barrier per 512 columns) ran 15 % slower: the W
// re-reads from L2 are not what bounds this kernel.  With 8 fp64 columns
// the 64 accumulators leave room for one wave per SIMD, so A is prefetched
// a step ahead and read with the non-temporal hint (737 -> 661 us at
// n = 2e4 in isolation).
template <typename T>
struct alignas(16) DVec {
  T v[16 / sizeof(T)];
};
// the same 16 bytes as a vector type (what the non-temporal load takes)
template <typename T>
struct NtVec;
template <>
struct NtVec<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
};
template <>
struct NtVec<float> {
  typedef float __attribute__((ext_vector_type(4))) type;
};

template <typename T, int R, int MC, bool FULLW>
__global__ __launch_bounds__(256) void k_dense_vec(const T* __restrict__ A, int64_t lda,
                                                   const T* __restrict__ W, int64_t ldw,
                                                   T* __restrict__ Y, int64_t ldy, int ncols,
                                                   int64_t n) {
  constexpr int VE = 16 / sizeof(T);
  constexpr int WV = MC / VE;  // 16-byte vectors per W row
  static_assert(MC % VE == 0 && R * MC <= 64, "tile shape");
  typedef DVec<T> V;
  const int lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * R;
  if (r0 >= n) return;
  T acc[R][MC];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < MC; ++j) acc[r][j] = T(0);
  const T* arow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) arow[r] = A + min(r0 + r, n - 1) * lda;
  constexpr int64_t kStep = 64 * VE;
  const int64_t nfull = (n / kStep) * kStep;
  // A is read once: non-temporal loads keep it from evicting W from L2, and
  // the next step's A vectors are loaded before this step's products (one
  // step in flight ahead; fully unrolled steps ran 3 % slower)
  typedef typename NtVec<T>::type VN;
  auto load_a = [&](int64_t c, V* dst) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const VN t = __builtin_nontemporal_load(reinterpret_cast<const VN*>(arow[r] + c));
#pragma unroll
      for (int u = 0; u < VE; ++u) dst[r].v[u] = t[u];
    }
  };
  // (prefetch only where occupancy is one wave per SIMD anyway: fp64 with 8
  // columns; elsewhere its registers would cost a wave)
  constexpr bool PF = sizeof(T) == 8 && MC == 8;
  V anext[PF ? R : 1];
  if (PF && nfull > 0) load_a(lane * VE, anext);
#pragma unroll 1
  for (int64_t c0 = 0; c0 < nfull; c0 += kStep) {
    const int64_t c = c0 + lane * VE;
    V a[R];
    if constexpr (PF) {
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = anext[r];
      if (c0 + kStep < nfull) load_a(c + kStep, anext);
    } else {
      load_a(c, a);
    }
    // W rows as 16-byte vectors; a vector that would reach past column
    // ncols (the block may be a column slice of a wider buffer) is read value
    // by value
    V w[VE][WV];
#pragma unroll
    for (int e = 0; e < VE; ++e)
#pragma unroll
      for (int q = 0; q < WV; ++q) {
        const T* src = W + (c + e) * ldw + q * VE;
        if (FULLW || (q + 1) * VE <= ncols) {
          w[e][q] = *reinterpret_cast<const V*>(src);
        } else {
#pragma unroll
          for (int u = 0; u < VE; ++u) w[e][q].v[u] = (q * VE + u < ncols) ? src[u] : T(0);
        }
      }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int e = 0; e < VE; ++e)
#pragma unroll
        for (int j = 0; j < MC; ++j) acc[r][j] += a[r].v[e] * w[e][j / VE].v[j % VE];
  }
  // ragged tail (fewer than 64 VE columns): value by value
  for (int64_t c = nfull + lane; c < n; c += 64) {
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
  T mine = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      T v = acc[r][j];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
      if (lane == r * MC + j) mine = v;
    }
  const int r = lane / MC, j = lane % MC;
  if (r < R && r0 + r < n && j < ncols) Y[(r0 + r) * ldy + j] = mine;
}

template <typename T>
static hipError_t dense_any(const T* A, int64_t lda, const T* W, int64_t ldw, T* Y, int64_t ldy,
                            int ncols, int64_t n, T* pack, hipStream_t s) {
  if (n < 1 || ncols < 1) return hipErrorInvalidValue;
  constexpr int VE = 16 / sizeof(T);
  // a block that is not a compact 8-column one is packed (8 columns at a
  // time, zero-padded) into `pack` first: strided rows and partial widths
  // cost the vector kernel 25-70 % (n = 2e4: 904 / 1271 us at ld 24 with 8
  // and 7 columns, against 737 us compact)
  if (pack != nullptr && lda % VE == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
      !(ldw == 8 && ncols == 8 && reinterpret_cast<uintptr_t>(W) % 16 == 0)) {
    const int gridv = cdiv(cdiv(n, 8), 4);
    for (int c0 = 0; c0 < ncols; c0 += 8) {
      const int nc = std::min(8, ncols - c0);
      hipError_t e = (sizeof(T) == 8)
                         ? pack8_f64(reinterpret_cast<const double*>(W + c0), ldw, nc, n,
                                     reinterpret_cast<double*>(pack), s)
                         : pack8_f32(reinterpret_cast<const float*>(W + c0), ldw, nc, n,
                                     reinterpret_cast<float*>(pack), s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_dense_vec<T, 8, 8, true>), dim3(gridv), dim3(256), 0, s, A, lda, pack,
                         (int64_t)8, Y + c0, ldy, nc, n);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const bool vec = lda % VE == 0 && ldw % VE == 0 &&
                   reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(W) % 16 == 0;
  if (vec) {
    constexpr int RV = 8;
    const int gridv = cdiv(cdiv(n, RV), 4);
    for (int c0 = 0; c0 < ncols; c0 += 8) {
      const int nc = std::min(8, ncols - c0);
      // W + c0 stays 16-byte aligned (c0 is a multiple of 8); only the block's
      // nc columns of each W row are read
      if (nc == 8)
        hipLaunchKernelGGL((k_dense_vec<T, RV, 8, true>), dim3(gridv), dim3(256), 0, s, A, lda,
                           W + c0, ldw, Y + c0, ldy, nc, n);
      else if (nc == 4)
        hipLaunchKernelGGL((k_dense_vec<T, RV, 4, true>), dim3(gridv), dim3(256), 0, s, A, lda,
                           W + c0, ldw, Y + c0, ldy, nc, n);
      else if (nc < 4)
        hipLaunchKernelGGL((k_dense_vec<T, RV, 4, false>), dim3(gridv), dim3(256), 0, s, A, lda,
                           W + c0, ldw, Y + c0, ldy, nc, n);
      else
        hipLaunchKernelGGL((k_dense_vec<T, RV, 8, false>), dim3(gridv), dim3(256), 0, s, A, lda,
                           W + c0, ldw, Y + c0, ldy, nc, n);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
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
                           int64_t ldy, int ncols, int64_t n, double* pack, hipStream_t s) {
  return dense_any<double>(A, lda, W, ldw, Y, ldy, ncols, n, pack, s);
}
hipError_t dense_apply_f32(const float* A, int64_t lda, const float* W, int64_t ldw, float* Y,
                           int64_t ldy, int ncols, int64_t n, float* pack, hipStream_t s) {
  return dense_any<float>(A, lda, W, ldw, Y, ldy, ncols, n, pack, s);
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
