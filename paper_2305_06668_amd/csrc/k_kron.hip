// Matrix-free Kronecker-sum operator H = A (x) I + I (x) A + diag(vec V)
// applied to a row-major block: vector entry (i, j) of column b lives at
// W[(i * na + j) * ldw + b], so
//   Y[i][j][b] = sum_k A[i][k] W[k][j][b] + sum_k A[j][k] W[i][k][b]
//              + V[i][j] W[i][j][b].
// For each column b both sums are dense products of na x na matrices,
// A W_b and W_b A (A symmetric), so the operator is two GEMMs sharing one
// accumulator: a workgroup owns an output tile of 32 i x 32 j x 8 columns
// and walks k in chunks of 16, staging A[i-tile][k], A[k][j-tile],
// W[k][j-tile][b] and W[i-tile][k][b] in LDS; each of the 4 waves owns two
// columns b and the four 16 x 16 (i, j) sub-tiles of each, and issues per
// 4-deep k step two MFMA 16x16x4 per sub-tile (one per term).  The tile is
// staged back through LDS so the diagonal term and the stores run along
// contiguous (j, b) rows.  4 na flops per output entry: na = 4096, 8 columns
// (n = 16.8M) is 2.2 TFLOP per application.
#include <algorithm>

#include "internal.h"

namespace lobpcg {

namespace {

constexpr int kTI = 32, kTJ = 32, kBB = 8, kKC = 16;

__device__ __forceinline__ d4 kmma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 kmma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct KAcc;
template <> struct KAcc<double> { typedef d4 type; };
template <> struct KAcc<float> { typedef f4 type; };
// accumulator register r of lane l holds row 4 r + l / 16 (f64) or
// 4 (l / 16) + r (f32) of the 16 x 16 tile, column l % 16
template <typename T> __device__ __forceinline__ int krow(int r, int lane);
template <> __device__ __forceinline__ int krow<double>(int r, int lane) { return 4 * r + (lane >> 4); }
template <> __device__ __forceinline__ int krow<float>(int r, int lane) { return 4 * (lane >> 4) + r; }

template <typename T>
struct KronSmem {
  T ai[kTI][kKC + 1];          // A[i0 + ii][k0 + kk]
  T aj[kKC][kTJ + 1];          // A[k0 + kk][j0 + jj]
  T xk[kKC][kTJ][kBB];         // W[(k0 + kk) na + j0 + jj][b0 + bb]
  T xi[kTI][kKC][kBB];         // W[(i0 + ii) na + k0 + kk][b0 + bb]
};

template <typename T>
__global__ __launch_bounds__(256) void k_kron_mfma(const T* __restrict__ A,
                                                   const T* __restrict__ Vp, int64_t na,
                                                   const T* __restrict__ W, int64_t ldw,
                                                   T* __restrict__ Y, int64_t ldy, int nc) {
  typedef typename KAcc<T>::type AccT;
  __shared__ KronSmem<T> sm;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int64_t j0 = (int64_t)blockIdx.x * kTJ, i0 = (int64_t)blockIdx.y * kTI;
  const int b0 = blockIdx.z * kBB;
  AccT acc[2][2][2];  // [b local 2 wave + bw][si][sj]
#pragma unroll
  for (int bw = 0; bw < 2; ++bw)
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[bw][si][sj][e] = T(0);
  for (int64_t k0 = 0; k0 < na; k0 += kKC) {
    __syncthreads();
    for (int t = threadIdx.x; t < kTI * kKC; t += 256) {
      const int ii = t / kKC, kk = t % kKC;
      const int64_t i = i0 + ii, k = k0 + kk;
      sm.ai[ii][kk] = (i < na && k < na) ? A[i * na + k] : T(0);
    }
    for (int t = threadIdx.x; t < kKC * kTJ; t += 256) {
      const int kk = t / kTJ, jj = t % kTJ;
      const int64_t k = k0 + kk, j = j0 + jj;
      sm.aj[kk][jj] = (k < na && j < na) ? A[k * na + j] : T(0);
    }
    for (int t = threadIdx.x; t < kKC * kTJ * kBB; t += 256) {
      const int bb = t % kBB, jj = (t / kBB) % kTJ, kk = t / (kBB * kTJ);
      const int64_t k = k0 + kk, j = j0 + jj;
      sm.xk[kk][jj][bb] =
          (k < na && j < na && b0 + bb < nc) ? W[(k * na + j) * ldw + b0 + bb] : T(0);
    }
    for (int t = threadIdx.x; t < kTI * kKC * kBB; t += 256) {
      const int bb = t % kBB, kk = (t / kBB) % kKC, ii = t / (kBB * kKC);
      const int64_t i = i0 + ii, k = k0 + kk;
      sm.xi[ii][kk][bb] =
          (i < na && k < na && b0 + bb < nc) ? W[(i * na + k) * ldw + b0 + bb] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < kKC; k4 += 4) {
      const int kk = k4 + g;
      T ai[2], aj[2];
#pragma unroll
      for (int si = 0; si < 2; ++si) ai[si] = sm.ai[16 * si + r][kk];
#pragma unroll
      for (int sj = 0; sj < 2; ++sj) aj[sj] = sm.aj[kk][16 * sj + r];
#pragma unroll
      for (int bw = 0; bw < 2; ++bw) {
        const int bb = 2 * wave + bw;
        T xk[2], xi[2];
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) xk[sj] = sm.xk[kk][16 * sj + r][bb];
#pragma unroll
        for (int si = 0; si < 2; ++si) xi[si] = sm.xi[16 * si + r][kk][bb];
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
          for (int sj = 0; sj < 2; ++sj) {
            // A W_b: A-operand A[i][k], B-operand W_b[k][j]
            acc[bw][si][sj] = kmma(ai[si], xk[sj], acc[bw][si][sj]);
            // W_b A: A-operand W_b[i][k], B-operand A[k][j]
            acc[bw][si][sj] = kmma(xi[si], aj[sj], acc[bw][si][sj]);
          }
      }
    }
  }
  // stage the tile through LDS (reusing the W areas) and store along (j, b)
  __syncthreads();
  T* so = &sm.xk[0][0][0];  // [ii][jj][bb]: kTI * kTJ * kBB values = xk + xi
  static_assert(sizeof(sm.xk) + sizeof(sm.xi) >= sizeof(T) * kTI * kTJ * kBB, "staging area");
#pragma unroll
  for (int bw = 0; bw < 2; ++bw)
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ii = 16 * si + krow<T>(e, lane), jj = 16 * sj + r;
          so[(ii * kTJ + jj) * kBB + 2 * wave + bw] = acc[bw][si][sj][e];
        }
  __syncthreads();
  for (int t = threadIdx.x; t < kTI * kTJ * kBB; t += 256) {
    const int bb = t % kBB, jj = (t / kBB) % kTJ, ii = t / (kBB * kTJ);
    const int64_t i = i0 + ii, j = j0 + jj;
    if (i < na && j < na && b0 + bb < nc) {
      const int64_t e = i * na + j;
      Y[e * ldy + b0 + bb] = so[t] + Vp[e] * W[e * ldw + b0 + bb];
    }
  }
}

}  // namespace

template <typename T>
static hipError_t kron_any(const T* A, const T* Vp, int64_t na, const T* W, int64_t ldw, T* Y,
                           int64_t ldy, int nc, hipStream_t s) {
  if (na < 1 || nc < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((na + kTJ - 1) / kTJ), (unsigned)((na + kTI - 1) / kTI),
                  (unsigned)((nc + kBB - 1) / kBB));
  hipLaunchKernelGGL((k_kron_mfma<T>), grid, dim3(256), 0, s, A, Vp, na, W, ldw, Y, ldy, nc);
  return hipGetLastError();
}

hipError_t kronsum_apply_f64(const double* A, const double* Vp, int64_t na, const double* W,
                             int64_t ldw, double* Y, int64_t ldy, int ncols, hipStream_t s) {
  return kron_any<double>(A, Vp, na, W, ldw, Y, ldy, ncols, s);
}
hipError_t kronsum_apply_f32(const float* A, const float* Vp, int64_t na, const float* W,
                             int64_t ldw, float* Y, int64_t ldy, int ncols, hipStream_t s) {
  return kron_any<float>(A, Vp, na, W, ldw, Y, ldy, ncols, s);
}

}  // namespace lobpcg
