// Kernels of the generalized problem A x = lambda B x (Sec. 3.3): the
// residual R = A X - B X Theta with the preconditioned active columns, the
// column statistics of the true-residual check, and the small coefficient
// matrices of the B-orthogonal projection and of the B-Cholesky.  Blocks are
// row-major fp64; reductions over n run in a fixed order (per-block
// partials, then blocks summed in index order), so results are bitwise
// reproducible.
#include <algorithm>

#include "internal.h"

namespace lobpcg {

constexpr int kGenBlocks = 1024;

// Per-block partials: part[b * m + j] = sum over the block's rows of r_ij^2.
// W~ (columns [0, m - a0) of Wout, leading dimension ldw) = T_j R[:, j] for
// j >= a0, T_j = 1 (precond 0), 1 / g(|dA - theta_j dB|) (1) or the signed
// form (2), g the Jacobi guard.
__global__ __launch_bounds__(256) void k_gen_residual(const double* __restrict__ AX,
                                                      const double* __restrict__ BX, int64_t ld, int m,
                                                      const double* __restrict__ theta, int a0,
                                                      int precond, const double* __restrict__ dA,
                                                      const double* __restrict__ dB,
                                                      double* __restrict__ Wout, int64_t ldw, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double red[256];
  __shared__ double th[64];
  for (int j = threadIdx.x; j < m; j += blockDim.x) th[j] = theta[j];
  __syncthreads();
  // thread (row slot, column): 256 / m rows per pass
  const int mm = m;
  const int rows_per = 256 / mm;
  const int j = threadIdx.x % mm;
  const int rs = threadIdx.x / mm;
  double acc = 0.0;
  if (rs < rows_per) {
    for (int64_t i = (int64_t)blockIdx.x * rows_per + rs; i < n; i += (int64_t)gridDim.x * rows_per) {
      const double r = AX[i * ld + j] - th[j] * BX[i * ld + j];
      acc += r * r;
      if (j >= a0) {
        double w = r;
        if (precond != 0) {
          const double delta = kPrecondGuard * fmax(1.0, fabs(th[j]));
          double den = dA[i] - th[j] * dB[i];
          if (precond == 1) den = fabs(den);
          if (fabs(den) < delta) den = (den < 0.0) ? -delta : delta;
          w = r / den;
        }
        Wout[i * ldw + (j - a0)] = w;
      }
    }
  }
  // fixed-order reduction of the row slots of each column
  red[threadIdx.x] = (rs < rows_per) ? acc : 0.0;
  __syncthreads();
  if (threadIdx.x < mm) {
    double s = 0.0;
    for (int q = 0; q < rows_per; ++q) s += red[q * mm + threadIdx.x];
    part[(int64_t)blockIdx.x * mm + threadIdx.x] = s;
  }
}

// out[o] = sum over blocks of part[b * cnt + o], in block order
__global__ void k_gen_sum(const double* __restrict__ part, int nblk, int cnt, double* __restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= cnt) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * cnt + o];
  out[o] = s;
}

static int gen_blocks(int64_t n, int m) {
  const int rows_per = 256 / m;
  return (int)std::max<int64_t>(1, std::min<int64_t>(kGenBlocks, (n + rows_per - 1) / rows_per));
}

hipError_t gen_residual(const double* AX, const double* BX, int64_t ld, int m, const double* theta,
                        int a0, int precond, const double* dA, const double* dB, double* Wout,
                        int64_t ldw, int64_t n, double* part, double* resn2, hipStream_t s) {
  if (m < 1 || m > 64 || n < 1) return hipErrorInvalidValue;
  const int nb = gen_blocks(n, m);
  hipLaunchKernelGGL(k_gen_residual, dim3(nb), dim3(256), 0, s, AX, BX, ld, m, theta, a0, precond, dA,
                     dB, Wout, ldw, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gen_sum, dim3(1), dim3(64), 0, s, part, nb, m, resn2);
  return hipGetLastError();
}

// Column statistics of the true check: part rows of 3m values, out[0:m] =
// x^T B x, out[m:2m] = x^T A x, out[2m:3m] = ||A x - theta B x||^2.
__global__ __launch_bounds__(256) void k_gen_colstats(const double* __restrict__ X, int64_t ldx,
                                                      const double* __restrict__ AX,
                                                      const double* __restrict__ BX, int64_t ldm, int m,
                                                      const double* __restrict__ theta, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double red[3][256];
  const int rows_per = 256 / m;
  const int j = threadIdx.x % m;
  const int rs = threadIdx.x / m;
  double sb = 0.0, sa = 0.0, sr = 0.0;
  if (rs < rows_per) {
    const double th = theta[j];
    for (int64_t i = (int64_t)blockIdx.x * rows_per + rs; i < n; i += (int64_t)gridDim.x * rows_per) {
      const double x = X[i * ldx + j], ax = AX[i * ldm + j], bx = BX[i * ldm + j];
      sb += x * bx;
      sa += x * ax;
      const double r = ax - th * bx;
      sr += r * r;
    }
  }
  const bool live = rs < rows_per;
  red[0][threadIdx.x] = live ? sb : 0.0;
  red[1][threadIdx.x] = live ? sa : 0.0;
  red[2][threadIdx.x] = live ? sr : 0.0;
  __syncthreads();
  if (threadIdx.x < m) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int q = 0; q < rows_per; ++q) {
      t0 += red[0][q * m + threadIdx.x];
      t1 += red[1][q * m + threadIdx.x];
      t2 += red[2][q * m + threadIdx.x];
    }
    double* o = part + (int64_t)blockIdx.x * 3 * m;
    o[threadIdx.x] = t0;
    o[m + threadIdx.x] = t1;
    o[2 * m + threadIdx.x] = t2;
  }
}

hipError_t gen_colstats(const double* X, int64_t ldx, const double* AX, const double* BX, int64_t ldm,
                        int m, const double* theta, int64_t n, double* part, double* out,
                        hipStream_t s) {
  if (m < 1 || m > 64 || n < 1) return hipErrorInvalidValue;
  const int nb = gen_blocks(n, m);
  hipLaunchKernelGGL(k_gen_colstats, dim3(nb), dim3(256), 0, s, X, ldx, AX, BX, ldm, m, theta, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gen_sum, dim3(1), dim3(256), 0, s, part, nb, 3 * m, out);
  return hipGetLastError();
}

// coef ((ny + nw) x nw) = [-C; I] for W <- [Y W] coef = W - Y C, and
// *cmax = max |C| (C: ny x nw, row-major)
__global__ void k_gen_proj_coef(const double* __restrict__ C, int ny, int nw, double* __restrict__ coef,
                                double* __restrict__ cmax) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int idx = threadIdx.x; idx < (ny + nw) * nw; idx += blockDim.x) {
    const int i = idx / nw, j = idx - i * nw;
    if (i < ny) {
      const double c = C[i * nw + j];
      coef[idx] = -c;
      mx = fmax(mx, fabs(c));
    } else {
      coef[idx] = (i - ny == j) ? 1.0 : 0.0;
    }
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int t = 0; t < (int)blockDim.x; ++t) r = fmax(r, red[t]);
    *cmax = r;
  }
}

hipError_t gen_proj_coef(const double* C, int ny, int nw, double* coef, double* cmax, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_proj_coef, dim3(1), dim3(256), 0, s, C, ny, nw, coef, cmax);
  return hipGetLastError();
}

// out (p x p) = L^-T for the lower factor L (p x p, row-major); one thread
// per column of L^-1, forward substitution
__global__ void k_gen_lt_inv(const double* __restrict__ L, int p, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= p) return;
  double col[kMaxBlock];
  for (int i = 0; i < p; ++i) {
    double s = (i == j) ? 1.0 : 0.0;
    for (int k = j; k < i; ++k) s -= L[i * p + k] * col[k];
    col[i] = (i < j) ? 0.0 : s / L[i * p + i];
  }
  // (L^-1)[i][j] = col[i]; out = (L^-1)^T: out[j][i] = col[i]
  for (int i = 0; i < p; ++i) out[j * p + i] = col[i];
}

hipError_t gen_lt_inv(const double* L, int p, double* out, hipStream_t s) {
  if (p < 1 || p > kMaxBlock) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gen_lt_inv, dim3(1), dim3(64), 0, s, L, p, out);
  return hipGetLastError();
}

// *out = max_i |x_i| over len values: per-block maxima, then one block
__global__ __launch_bounds__(256) void k_max_abs_part(const double* __restrict__ x, int64_t len,
                                                      double* __restrict__ part) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    mx = fmax(mx, fabs(x[i]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

hipError_t vec_max_abs(const double* x, int64_t len, double* part, double* out, hipStream_t s) {
  if (len < 1) return hipErrorInvalidValue;
  const int nb = (int)std::min<int64_t>(1024, (len + 255) / 256);
  hipLaunchKernelGGL(k_max_abs_part, dim3(nb), dim3(256), 0, s, x, len, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_max_abs_part, dim3(1), dim3(256), 0, s, part, (int64_t)nb, out);
  return hipGetLastError();
}

}  // namespace lobpcg
