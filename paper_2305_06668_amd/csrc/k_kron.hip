// Matrix-free Kronecker-sum operator H = A (x) I + I (x) A + diag(vec V)
// applied to a row-major block: vector entry (i, j) of column b lives at
// W[(i * na + j) * ldw + b], so
//   Y[i][j][b] = sum_k A[i][k] W[k][j][b] + sum_k A[j][k] W[i][k][b]
//              + V[i][j] W[i][j][b].
// Reference (untiled) version: one thread per output entry.
#include "internal.h"

namespace lobpcg {

template <typename T>
__global__ __launch_bounds__(256) void k_kron_naive(const T* __restrict__ A,
                                                    const T* __restrict__ Vp, int64_t na,
                                                    const T* __restrict__ W, int64_t ldw,
                                                    T* __restrict__ Y, int64_t ldy, int nc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = na * na * nc;
  if (idx >= total) return;
  const int b = (int)(idx % nc);
  const int64_t ij = idx / nc;
  const int64_t i = ij / na, j = ij - i * na;
  T s = Vp[ij] * W[ij * ldw + b];
  for (int64_t k = 0; k < na; ++k) {
    s += A[i * na + k] * W[(k * na + j) * ldw + b];
    s += A[j * na + k] * W[(i * na + k) * ldw + b];
  }
  Y[ij * ldy + b] = s;
}

template <typename T>
static hipError_t kron_any(const T* A, const T* Vp, int64_t na, const T* W, int64_t ldw, T* Y,
                           int64_t ldy, int nc, hipStream_t s) {
  if (na < 1 || nc < 1) return hipErrorInvalidValue;
  const int64_t total = na * na * nc;
  hipLaunchKernelGGL((k_kron_naive<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A,
                     Vp, na, W, ldw, Y, ldy, nc);
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
