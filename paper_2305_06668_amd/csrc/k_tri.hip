// Tridiagonal preconditioner (Sec. 4.4, Table 1: the diagonal plus the upper
// and lower diagonal elements of A, where the paper solves with LAPACK's
// Gaussian elimination).  Column j of R (n x nact, row-major, leading
// dimension ld) is replaced in place by the solution w of T_j w = r with
//   T_j = tridiag(e, t, e),  t_i = max(|d_i - theta_j|, |e_{i-1}| + |e_i| + delta_j),
// e_i = a_{i,i+1}, d = diag(A), delta_j = kPrecondGuard max(1, |theta_j|):
// symmetric and strictly diagonally dominant with a positive diagonal, so
// elimination without pivoting is stable.
//
// Partition method over P balanced chunks [s_c, e_c) of at least 64 rows:
//   k_tri_bound   thread (c, j): an LU sweep down and a UL sweep up over the
//                 chunk give its first and last unknowns as affine functions
//                 of the two unknowns just outside it,
//                   x_i = y_i + v_i x_{s-1} + w_i x_e   (i = s, e - 1);
//   k_tri_reduced workgroup j: the 2P boundary unknowns b_c = (x_s, x_{e-1})
//                 form a block tridiagonal system with 2 x 2 blocks, solved
//                 by block Thomas in LDS;
//   k_tri_final   thread (c, j): the chunk's own system with the neighbours'
//                 boundary values on the right-hand side, by Thomas (the
//                 forward factors kept in `scr`, n x nact fp64, the forward
//                 right-hand side in R itself).
// Every sum and factor is fp64; in the fp32 phase R is read and written in
// fp32.
#include <algorithm>

#include "internal.h"

namespace lobpcg {

__device__ __forceinline__ void chunk_bounds(int64_t n, int P, int c, int64_t* s, int64_t* e) {
  *s = (int64_t)c * n / P;
  *e = (int64_t)(c + 1) * n / P;
}

__device__ __forceinline__ double tri_diag(double d, double th, double off, double delta) {
  return fmax(fabs(d - th), off + delta);
}

// Operands of row i for column j, loaded kU rows ahead of the dependent
// recurrences (every sweep is latency-bound on its divisions; the loads are
// not).
constexpr int kU = 8;

// bnd[(c * nact + j) * 6 + {0..5}] = y_s, v_s, w_s, y_e, v_e, w_e
template <typename T>
__global__ __launch_bounds__(256) void k_tri_bound(const T* __restrict__ R, int64_t ld, int nact,
                                                   int64_t n, int P, const double* __restrict__ theta,
                                                   const double* __restrict__ d,
                                                   const double* __restrict__ e,
                                                   const double* __restrict__ off,
                                                   double* __restrict__ bnd) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * nact) return;
  const int c = t / nact, j = t - c * nact;
  int64_t s, en;
  chunk_bounds(n, P, c, &s, &en);
  const double th = theta[j];
  const double delta = kPrecondGuard * fmax(1.0, fabs(th));
  const double a_s = (s > 0) ? e[s - 1] : 0.0;  // coupling to x_{s-1}
  const double c_e = e[en - 1];                 // coupling to x_e (e[n-1] = 0)
  // LU sweep down: last-row values
  double cp = 0.0, ry = 0.0, rv = 0.0, den = 1.0;
  for (int64_t i0 = s; i0 < en; i0 += kU) {
    double tt[kU], ea[kU], ec[kU], rr[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = min(i0 + u, en - 1);
      tt[u] = tri_diag(d[i], th, off[i], delta);
      ea[u] = (i > s) ? e[i - 1] : 0.0;
      ec[u] = e[i];
      rr[u] = (double)R[i * ld + j];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (i0 + u >= en) break;
      den = tt[u] - ea[u] * cp;
      const double inv = 1.0 / den;
      ry = (rr[u] - ea[u] * ry) * inv;
      rv = ((i0 + u == s ? -a_s : 0.0) - ea[u] * rv) * inv;
      cp = ec[u] * inv;
    }
  }
  const double y_e = ry, v_e = rv, w_e = -c_e / den;
  // UL sweep up: first-row values
  double ap = 0.0, sy = 0.0, sw = 0.0;
  den = 1.0;
  for (int64_t i0 = en - 1; i0 >= s; i0 -= kU) {
    double tt[kU], ea[kU], ec[kU], rr[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = max(i0 - u, s);
      tt[u] = tri_diag(d[i], th, off[i], delta);
      ea[u] = (i > 0) ? e[i - 1] : 0.0;
      ec[u] = (i < en - 1) ? e[i] : 0.0;
      rr[u] = (double)R[i * ld + j];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (i0 - u < s) break;
      den = tt[u] - ec[u] * ap;
      const double inv = 1.0 / den;
      sy = (rr[u] - ec[u] * sy) * inv;
      sw = ((i0 - u == en - 1 ? -c_e : 0.0) - ec[u] * sw) * inv;
      ap = ea[u] * inv;
    }
  }
  const double y_s = sy, v_s = -a_s / den, w_s = sw;
  double* o = bnd + (int64_t)t * 6;
  o[0] = y_s;
  o[1] = v_s;
  o[2] = w_s;
  o[3] = y_e;
  o[4] = v_e;
  o[5] = w_e;
}

// Block Thomas on b_c = (f_c, l_c):
//   b_c - Lo_c b_{c-1} - Up_c b_{c+1} = y_c,
//   Lo_c = [[0, v_s], [0, v_e]],  Up_c = [[w_s, 0], [w_e, 0]].
// One workgroup per column: the column's boundary data are staged in LDS,
// one thread runs the sequential elimination there, and the solution b_c is
// written to xb[(c * nact + j) * 2 + {0, 1}].
__global__ __launch_bounds__(256) void k_tri_reduced(int nact, int P, const double* __restrict__ bnd,
                                                     double* __restrict__ xb) {
  extern __shared__ double lds[];  // P * 6 boundary data, then P * 4 factors
  const int j = blockIdx.x;
  double* q = lds;
  double* f = lds + (int64_t)P * 6;
  for (int idx = threadIdx.x; idx < P * 6; idx += blockDim.x) {
    const int c = idx / 6, k = idx - c * 6;
    q[idx] = bnd[((int64_t)c * nact + j) * 6 + k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // G_{c-1} = [[G0, 0], [G1, 0]] (its right column is always 0), g_{c-1}
    double G0 = 0.0, G1 = 0.0, g0 = 0.0, g1 = 0.0;
    for (int c = 0; c < P; ++c) {
      const double* b = q + c * 6;
      const double ys = b[0], vs = b[1], ws = b[2], ye = b[3], ve = b[4], we = b[5];
      // S = I - Lo G_{c-1} = [[1 - vs G1, 0], [-ve G1, 1]]
      const double S00 = 1.0 - vs * G1;
      const double S10 = -ve * G1;
      const double i00 = 1.0 / S00;
      // rhs = y + Lo g_{c-1}
      const double r0 = ys + vs * g1, r1 = ye + ve * g1;
      // S^-1 = [[i00, 0], [-S10 i00, 1]]
      G0 = i00 * ws;
      G1 = -S10 * i00 * ws + we;
      g0 = i00 * r0;
      g1 = -S10 * i00 * r0 + r1;
      double* o = f + c * 4;
      o[0] = G0;
      o[1] = G1;
      o[2] = g0;
      o[3] = g1;
    }
    // back substitution: b_c = g_c + G_c b_{c+1} (b_P = 0); G_c b = G f_{c+1}
    double bf = 0.0;
    for (int c = P - 1; c >= 0; --c) {
      double* o = f + c * 4;
      const double n0 = o[2] + o[0] * bf;
      const double n1 = o[3] + o[1] * bf;
      o[2] = n0;
      o[3] = n1;
      bf = n0;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < P; c += blockDim.x) {
    xb[((int64_t)c * nact + j) * 2 + 0] = f[c * 4 + 2];
    xb[((int64_t)c * nact + j) * 2 + 1] = f[c * 4 + 3];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_tri_final(T* __restrict__ R, int64_t ld, int nact, int64_t n,
                                                   int P, const double* __restrict__ theta,
                                                   const double* __restrict__ d,
                                                   const double* __restrict__ e,
                                                   const double* __restrict__ off,
                                                   const double* __restrict__ xb,
                                                   double* __restrict__ scr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * nact) return;
  const int c = t / nact, j = t - c * nact;
  int64_t s, en;
  chunk_bounds(n, P, c, &s, &en);
  const double th = theta[j];
  const double delta = kPrecondGuard * fmax(1.0, fabs(th));
  // neighbours' boundary values: x_{s-1} = l_{c-1}, x_e = f_{c+1}
  const double xl = (c > 0) ? xb[((int64_t)(c - 1) * nact + j) * 2 + 1] : 0.0;
  const double xf = (c < P - 1) ? xb[((int64_t)(c + 1) * nact + j) * 2 + 0] : 0.0;
  const double a_s = (s > 0) ? e[s - 1] : 0.0;
  const double c_e = e[en - 1];
  double cp = 0.0, rp = 0.0;
  for (int64_t i0 = s; i0 < en; i0 += kU) {
    double tt[kU], ea[kU], ec[kU], rr[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = min(i0 + u, en - 1);
      tt[u] = tri_diag(d[i], th, off[i], delta);
      ea[u] = (i > s) ? e[i - 1] : 0.0;
      ec[u] = e[i];
      rr[u] = (double)R[i * ld + j];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = i0 + u;
      if (i >= en) break;
      const double den = tt[u] - ea[u] * cp;
      const double inv = 1.0 / den;
      double r = rr[u];
      if (i == s) r -= a_s * xl;
      if (i == en - 1) r -= c_e * xf;
      rp = (r - ea[u] * rp) * inv;
      cp = ec[u] * inv;
      scr[i * nact + j] = cp;
      R[i * ld + j] = (T)rp;  // (in the fp32 phase at the blocks' precision)
    }
  }
  double x = 0.0;
  for (int64_t i0 = en - 1; i0 >= s; i0 -= kU) {
    double rr[kU], cc[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = max(i0 - u, s);
      rr[u] = (double)R[i * ld + j];
      cc[u] = scr[i * nact + j];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = i0 - u;
      if (i < s) break;
      x = (i == en - 1) ? rr[u] : rr[u] - cc[u] * x;
      R[i * ld + j] = (T)x;
    }
  }
}

int tri_chunks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kTriMaxChunks, n / 64)); }

template <typename T>
static hipError_t tri_apply_any(T* R, int64_t ld, int nact, int64_t n, const double* theta,
                                const double* d, const double* e, const double* off,
                                double* bnd, double* xb, double* scr, hipStream_t s) {
  if (n < 1 || nact < 1 || nact > 64 || ld < nact) return hipErrorInvalidValue;
  const int P = tri_chunks(n);
  const int threads = P * nact;
  const int grid = (threads + 255) / 256;
  hipLaunchKernelGGL((k_tri_bound<T>), dim3(grid), dim3(256), 0, s, R, ld, nact, n, P, theta, d, e,
                     off, bnd);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_tri_reduced, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kTriMaxChunks * 10 * (int)sizeof(double));
    (void)hipGetLastError();
    attr = true;
  }
  hipLaunchKernelGGL(k_tri_reduced, dim3(nact), dim3(256), (size_t)P * 10 * sizeof(double), s, nact, P,
                     bnd, xb);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_tri_final<T>), dim3(grid), dim3(256), 0, s, R, ld, nact, n, P, theta, d, e,
                     off, xb, scr);
  return hipGetLastError();
}

hipError_t tri_apply_f64(double* R, int64_t ld, int nact, int64_t n, const double* theta,
                         const double* d, const double* e, const double* off, double* bnd,
                         double* xb, double* scr, hipStream_t s) {
  return tri_apply_any<double>(R, ld, nact, n, theta, d, e, off, bnd, xb, scr, s);
}
hipError_t tri_apply_f32(float* R, int64_t ld, int nact, int64_t n, const double* theta,
                         const double* d, const double* e, const double* off, double* bnd,
                         double* xb, double* scr, hipStream_t s) {
  return tri_apply_any<float>(R, ld, nact, n, theta, d, e, off, bnd, xb, scr, s);
}

// ---- the off-diagonal e_i = a_{i,i+1} and off_i = |e_{i-1}| + |e_i| ------

__global__ void k_tri_off_csr(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const double* __restrict__ val, int64_t n, double* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k)
    if ((int64_t)ci[k] == i + 1) v += val[k];
  e[i] = v;
}

__global__ void k_tri_off_dense(const double* __restrict__ A, int64_t lda, int64_t n,
                                double* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  e[i] = (i + 1 < n) ? A[i * lda + i + 1] : 0.0;
}

// H = A (x) I + I (x) A + diag(vec V): entry (i na + j, i na + j + 1) is
// A[j][j+1] inside a block of na rows, 0 across blocks
__global__ void k_tri_off_kron(const double* __restrict__ A, int64_t na, double* __restrict__ e) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= na * na) return;
  const int64_t j = r % na;
  e[r] = (j + 1 < na) ? A[j * na + j + 1] : 0.0;
}

__global__ void k_tri_rowoff(const double* __restrict__ e, int64_t n, double* __restrict__ off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  off[i] = fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0);
}

static hipError_t rowoff(const double* e, int64_t n, double* off, hipStream_t s) {
  hipLaunchKernelGGL(k_tri_rowoff, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, e, n, off);
  return hipGetLastError();
}

hipError_t tri_offdiag_csr(const int32_t* rp, const int32_t* ci, const double* val, int64_t n,
                           double* e, double* off, hipStream_t s) {
  hipLaunchKernelGGL(k_tri_off_csr, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rp, ci, val, n,
                     e);
  hipError_t err = hipGetLastError();
  return err != hipSuccess ? err : rowoff(e, n, off, s);
}
hipError_t tri_offdiag_dense(const double* A, int64_t lda, int64_t n, double* e, double* off,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_tri_off_dense, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, lda, n,
                     e);
  hipError_t err = hipGetLastError();
  return err != hipSuccess ? err : rowoff(e, n, off, s);
}
hipError_t tri_offdiag_kron(const double* A, int64_t na, double* e, double* off, hipStream_t s) {
  const int64_t n = na * na;
  hipLaunchKernelGGL(k_tri_off_kron, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, na, e);
  hipError_t err = hipGetLastError();
  return err != hipSuccess ? err : rowoff(e, n, off, s);
}

}  // namespace lobpcg
