// Streaming kernels of the learned preconditioner's training driver: column
// gathers, block projections, column dot products, the per-column scalars of
// the training objective, and the vector updates of the block MINRES that
// produces the near-exact Jacobi-Davidson corrections.  All fp64.  The
// blocks are row-major n x nc (nc <= 64); the elementwise kernels give a
// workgroup 256 / nc whole rows, one element per thread, so a wave's loads
// are one contiguous run; the column dots reduce in two fixed-order stages.
#include <algorithm>

#include "internal.h"

namespace lobpcg {

namespace {

constexpr int kDotBlocks = 1024;

inline int cdiv64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Element (i, j) of this thread in an n x nc block: a workgroup covers
// 256 / nc whole rows (grid rows_grid(n, nc)).
struct Elem {
  int64_t i;
  int j;
  bool ok;
};
__device__ __forceinline__ Elem elem_of(int nc, int64_t n) {
  const int rpb = 256 / nc;
  const int r = (int)threadIdx.x / nc;
  const int64_t i = (int64_t)blockIdx.x * rpb + r;
  return {i, (int)threadIdx.x - r * nc, r < rpb && i < n};
}
inline int rows_grid(int64_t n, int nc) { return std::max(1, cdiv64(n, 256 / nc)); }

// Out[:, j] = In[:, cols[j]]
__global__ void k_gather_cols(const double* __restrict__ In, int64_t ldi,
                              const int* __restrict__ cols, int nc, int64_t n,
                              double* __restrict__ Out, int64_t ldo) {
  const Elem x = elem_of(nc, n);
  if (x.ok) Out[x.i * ldo + x.j] = In[x.i * ldi + cols[x.j]];
}

// Out = In - X C  (X: n x m, C: m x nc row-major, staged in LDS); the
// lanes of one row read the same X entries together
__global__ __launch_bounds__(256) void k_project(const double* __restrict__ In, int64_t ldi,
                                                 const double* __restrict__ X, int64_t ldx, int m,
                                                 const double* __restrict__ C, int nc, int64_t n,
                                                 double* __restrict__ Out, int64_t ldo) {
  __shared__ double Cs[kMaxBlock * 64];
  for (int q = threadIdx.x; q < m * nc; q += 256) Cs[q] = C[q];
  __syncthreads();
  const Elem x = elem_of(nc, n);
  if (!x.ok) return;
  const double* xr = X + x.i * ldx;
  double s = In[x.i * ldi + x.j];
  for (int t = 0; t < m; ++t) s -= xr[t] * Cs[t * nc + x.j];
  Out[x.i * ldo + x.j] = s;
}

struct DotArgs {
  const double* P[3];
  const double* Q[3];
  int64_t ldp[3], ldq[3];
  int npairs, nc;
  int64_t n;
};

// part[(pair nc + col) nblk + b] = sum over block b's rows of P[i][col] Q[i][col].
// Lane = (row offset rr < 64 / nc, column j): a wave reads 64 / nc whole
// rows per step; the partials of a column are added over (wave, rr) in a
// fixed order.
__global__ __launch_bounds__(256) void k_coldots_part(DotArgs a, double* __restrict__ part) {
  __shared__ double red[3][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nc = a.nc, rpw = 64 / nc;
  const int rr = lane / nc, j = lane - rr * nc;
  double s[3] = {0.0, 0.0, 0.0};
  if (rr < rpw) {
    const int64_t step = (int64_t)gridDim.x * 4 * rpw;
    for (int64_t i = ((int64_t)blockIdx.x * 4 + wave) * rpw + rr; i < a.n; i += step) {
#pragma unroll
      for (int pr = 0; pr < 3; ++pr)
        if (pr < a.npairs) s[pr] += a.P[pr][i * a.ldp[pr] + j] * a.Q[pr][i * a.ldq[pr] + j];
    }
  }
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) red[pr][threadIdx.x] = s[pr];
  __syncthreads();
  if ((int)threadIdx.x < a.npairs * nc) {
    const int pr = (int)threadIdx.x / nc, jj = (int)threadIdx.x - pr * nc;
    double t = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int r = 0; r < rpw; ++r) t += red[pr][64 * w + r * nc + jj];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}
// out[idx] = sum over the nblk partials of output idx (one workgroup each,
// fixed-order tree)
__global__ __launch_bounds__(256) void k_coldots_final(const double* __restrict__ part, int nblk,
                                                       double* __restrict__ out) {
  __shared__ double red[256];
  const double* p = part + (size_t)blockIdx.x * nblk;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += p[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Training objective per column (see mlp_objective_scalars).  With sdots
// (u.tau, tau.tau per column) and mu > 0 the supervised term
// mu (1 - (u.tau)^2 / (u.u tau.tau)) joins the loss, and its gradient in u,
// -2 mu c / (a e) tau + 2 mu c^2 / (a^2 e) u (c = u.tau, a = u.u, e =
// tau.tau; divided by nc like the rest), the coefficients of tau (coef4) and u.
__global__ void k_obj_scalars(const double* __restrict__ dots, const double* __restrict__ theta,
                              const double* __restrict__ ref, int nc, double* __restrict__ coef,
                              double* __restrict__ out, const double* __restrict__ sdots,
                              double mu, double* __restrict__ coef4) {
  const int j = threadIdx.x;
  if (j >= nc) return;
  const double uu = dots[j], ru = dots[nc + j], uau = dots[2 * nc + j];
  const double nu2 = uu, nu = sqrt(uu);
  const double b = ru / nu;
  const double cq = uau / nu2;
  const double h = 0.5 * (cq - theta[j]);
  const double S = hypot(h, b);
  // Delta = S - h, written b^2 / (S + h) when h > 0 (the difference cancels)
  const double D = h > 0.0 ? b * b / (S + h) : S - h;
  // dL/db = -(b / S) / (D nc); dL/dcq = (D / (2 S)) / (D nc) = 1 / (2 S nc)
  const double cb = -b / (S * D * nc);
  const double cc = 1.0 / (2.0 * S * nc);
  double cu = -cb * b / nu2 - cc * 2.0 * cq / nu2;
  double ct = 0.0, lsup = 0.0;
  if (sdots != nullptr && mu != 0.0) {
    const double c = sdots[j], e = sdots[nc + j];
    if (e > 0.0 && uu > 0.0) {
      lsup = mu * (1.0 - c * c / (uu * e));
      ct = -2.0 * mu * c / (uu * e * nc);
      cu += 2.0 * mu * c * c / (uu * uu * e * nc);
    }
  }
  coef[j] = cb / nu;           // r
  coef[nc + j] = cu;           // u
  coef[2 * nc + j] = cc * 2.0 / nu2;  // P A u
  if (coef4 != nullptr) coef4[j] = ct;  // tau
  out[j] = D;
  out[nc + j] = (ref ? log(ref[j]) : 0.0) - log(D) + lsup;
}

// Out = a R + b U + c Z (+ d Tau)  (per-column coefficients)
__global__ void k_combine3(const double* __restrict__ R, const double* __restrict__ U,
                           const double* __restrict__ Z, const double* __restrict__ Tau,
                           const double* __restrict__ coef, const double* __restrict__ coef4,
                           int nc, int64_t n, double* __restrict__ Out) {
  const Elem x = elem_of(nc, n);
  if (!x.ok) return;
  const int64_t e = x.i * nc + x.j;
  double o = coef[x.j] * R[e] + coef[nc + x.j] * U[e] + coef[2 * nc + x.j] * Z[e];
  if (Tau != nullptr) o += coef4[x.j] * Tau[e];
  Out[e] = o;
}

// R = AX - X diag(theta)
__global__ void k_residual(const double* __restrict__ X, const double* __restrict__ AX,
                           const double* __restrict__ theta, int m, int64_t n,
                           double* __restrict__ R) {
  const Elem x = elem_of(m, n);
  if (!x.ok) return;
  const int64_t e = x.i * m + x.j;
  R[e] = AX[e] - theta[x.j] * X[e];
}

// ---- block MINRES (Paige-Saunders recurrence, one system per column) ----
// Per-column state, updated by k_mr_scalars.
struct MrState {
  double beta1, beta, oldb, dbar, epsln, oldeps, phibar, cs, sn, phi, delta, denom, alfa;
  int done;
};

// V = Y / beta
__global__ void k_mr_scale(const double* __restrict__ Y, const MrState* __restrict__ st, int nc,
                           int64_t n, double* __restrict__ V) {
  const Elem x = elem_of(nc, n);
  if (!x.ok) return;
  const int64_t e = x.i * nc + x.j;
  V[e] = st[x.j].done ? 0.0 : Y[e] / st[x.j].beta;
}

// Y = (AV - theta V) - x (x^T (AV - theta V)) - (beta / oldb) R1 [itn > 1]
__global__ void k_mr_y(const double* __restrict__ AV, const double* __restrict__ V,
                       const double* __restrict__ Xc, const double* __restrict__ theta,
                       const double* __restrict__ dots, const double* __restrict__ R1,
                       const MrState* __restrict__ st, int first, int nc, int64_t n,
                       double* __restrict__ Y) {
  const Elem x = elem_of(nc, n);
  if (!x.ok) return;
  const int j = x.j;
  const int64_t e = x.i * nc + j;
  const double xd = dots[j] - theta[j] * dots[nc + j];  // x^T (A v - theta v)
  double y = AV[e] - theta[j] * V[e] - xd * Xc[e];
  if (!first && !st[j].done) y -= (st[j].beta / st[j].oldb) * R1[e];
  Y[e] = y;
}

// Y -= (alfa / beta) R2   (alfa = dots[j] stored into the state)
__global__ void k_mr_y2(const double* __restrict__ dots, const double* __restrict__ R2,
                        MrState* __restrict__ st, int nc, int64_t n, double* __restrict__ Y) {
  const Elem x = elem_of(nc, n);
  if (!x.ok || st[x.j].done) return;
  const int64_t e = x.i * nc + x.j;
  Y[e] -= (dots[x.j] / st[x.j].beta) * R2[e];
}

__global__ void k_mr_init(const double* __restrict__ bnorm2, int nc, MrState* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= nc) return;
  MrState s{};
  s.beta1 = sqrt(bnorm2[j]);
  s.beta = s.beta1;
  s.oldb = 0.0;
  s.phibar = s.beta1;
  s.cs = -1.0;
  s.sn = 0.0;
  s.done = !(s.beta1 > 0.0);
  st[j] = s;
}

// Givens recurrence of one MINRES step; alfa = dots_a[j], new beta^2 = dots_b[j].
__global__ void k_mr_scalars(const double* __restrict__ alfa, const double* __restrict__ beta2,
                             int nc, MrState* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= nc) return;
  MrState s = st[j];
  if (s.done) {
    s.phi = 0.0;
    s.denom = 0.0;
    st[j] = s;
    return;
  }
  s.alfa = alfa[j];
  s.oldb = s.beta;
  s.beta = sqrt(beta2[j]);
  s.oldeps = s.epsln;
  s.delta = s.cs * s.dbar + s.sn * s.alfa;
  const double gbar = s.sn * s.dbar - s.cs * s.alfa;
  s.epsln = s.sn * s.beta;
  s.dbar = -s.cs * s.beta;
  double gamma = sqrt(gbar * gbar + s.beta * s.beta);
  gamma = fmax(gamma, 1e-300);
  s.cs = gbar / gamma;
  s.sn = s.beta / gamma;
  s.phi = s.cs * s.phibar;
  s.phibar = s.sn * s.phibar;
  s.denom = 1.0 / gamma;
  if (!(s.beta > 1e-300 * s.beta1)) s.done = 1;  // exact invariant subspace: stop this column
  st[j] = s;
}

// Wn = (V - oldeps W1 - delta W2) denom ; T += phi Wn
__global__ void k_mr_update(const double* __restrict__ V, const double* __restrict__ W1,
                            const double* __restrict__ W2, const MrState* __restrict__ st, int nc,
                            int64_t n, double* __restrict__ Wn, double* __restrict__ T) {
  const Elem x = elem_of(nc, n);
  if (!x.ok) return;
  const MrState& s = st[x.j];
  const int64_t e = x.i * nc + x.j;
  const double w = (V[e] - s.oldeps * W1[e] - s.delta * W2[e]) * s.denom;
  Wn[e] = w;
  T[e] += s.phi * w;
}

// Y = -(r - x (x^T r)) given dots = x^T r
__global__ void k_mr_rhs(const double* __restrict__ Rc, const double* __restrict__ Xc,
                         const double* __restrict__ dots, int nc, int64_t n,
                         double* __restrict__ Y) {
  const Elem x = elem_of(nc, n);
  if (!x.ok) return;
  const int64_t e = x.i * nc + x.j;
  Y[e] = -(Rc[e] - dots[x.j] * Xc[e]);
}

}  // namespace

size_t mr_state_bytes() { return sizeof(MrState); }

hipError_t gather_cols(const double* In, int64_t ldi, const int* cols, int nc, int64_t n,
                       double* Out, int64_t ldo, hipStream_t s) {
  if (nc <= 0 || nc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_cols, dim3(rows_grid(n, nc)), dim3(256), 0, s, In, ldi, cols, nc, n,
                     Out, ldo);
  return hipGetLastError();
}
hipError_t project_block(const double* In, int64_t ldi, const double* X, int64_t ldx, int m,
                         const double* C, int nc, int64_t n, double* Out, int64_t ldo,
                         hipStream_t s) {
  if (m > kMaxBlock || nc <= 0 || nc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_project, dim3(rows_grid(n, nc)), dim3(256), 0, s, In, ldi, X, ldx, m, C, nc,
                     n, Out, ldo);
  return hipGetLastError();
}
hipError_t coldots(int npairs, const double* const* P, const int64_t* ldp, const double* const* Q,
                   const int64_t* ldq, int nc, int64_t n, double* part, double* out,
                   hipStream_t s) {
  DotArgs a{};
  for (int k = 0; k < npairs; ++k) {
    a.P[k] = P[k];
    a.Q[k] = Q[k];
    a.ldp[k] = ldp[k];
    a.ldq[k] = ldq[k];
  }
  if (npairs < 1 || npairs > 3 || nc <= 0 || nc > 64) return hipErrorInvalidValue;
  a.npairs = npairs;
  a.nc = nc;
  a.n = n;
  const int grid = std::max(1, std::min(kDotBlocks, cdiv64(n, 256)));
  hipLaunchKernelGGL(k_coldots_part, dim3(grid), dim3(256), 0, s, a, part);
  hipLaunchKernelGGL(k_coldots_final, dim3(npairs * nc), dim3(256), 0, s, part, grid, out);
  return hipGetLastError();
}
hipError_t objective_scalars(const double* dots, const double* theta, const double* ref, int nc,
                             double* coef, double* out, const double* sdots, double mu,
                             double* coef4, hipStream_t s) {
  hipLaunchKernelGGL(k_obj_scalars, dim3(1), dim3(64), 0, s, dots, theta, ref, nc, coef, out, sdots,
                     mu, coef4);
  return hipGetLastError();
}
hipError_t combine3(const double* R, const double* U, const double* Z, const double* Tau,
                    const double* coef, const double* coef4, int nc, int64_t n, double* Out,
                    hipStream_t s) {
  if (nc <= 0 || nc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_combine3, dim3(rows_grid(n, nc)), dim3(256), 0, s, R, U, Z, Tau, coef, coef4,
                     nc, n, Out);
  return hipGetLastError();
}
hipError_t residual_block(const double* X, const double* AX, const double* theta, int m,
                          int64_t n, double* R, hipStream_t s) {
  if (m <= 0 || m > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_residual, dim3(rows_grid(n, m)), dim3(256), 0, s, X, AX, theta, m, n, R);
  return hipGetLastError();
}
hipError_t mr_init(const double* bnorm2, int nc, void* st, hipStream_t s) {
  hipLaunchKernelGGL(k_mr_init, dim3(1), dim3(64), 0, s, bnorm2, nc, static_cast<MrState*>(st));
  return hipGetLastError();
}
hipError_t mr_rhs(const double* Rc, const double* Xc, const double* dots, int nc, int64_t n,
                  double* Y, hipStream_t s) {
  if (nc <= 0 || nc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mr_rhs, dim3(rows_grid(n, nc)), dim3(256), 0, s, Rc, Xc, dots, nc, n, Y);
  return hipGetLastError();
}
hipError_t mr_scale(const double* Y, const void* st, int nc, int64_t n, double* V, hipStream_t s) {
  if (nc <= 0 || nc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mr_scale, dim3(rows_grid(n, nc)), dim3(256), 0, s, Y,
                     static_cast<const MrState*>(st), nc, n, V);
  return hipGetLastError();
}
hipError_t mr_y(const double* AV, const double* V, const double* Xc, const double* theta,
                const double* dots, const double* R1, const void* st, int first, int nc, int64_t n,
                double* Y, hipStream_t s) {
  if (nc <= 0 || nc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mr_y, dim3(rows_grid(n, nc)), dim3(256), 0, s, AV, V, Xc, theta, dots, R1,
                     static_cast<const MrState*>(st), first, nc, n, Y);
  return hipGetLastError();
}
hipError_t mr_y2(const double* dots, const double* R2, void* st, int nc, int64_t n, double* Y,
                 hipStream_t s) {
  if (nc <= 0 || nc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mr_y2, dim3(rows_grid(n, nc)), dim3(256), 0, s, dots, R2,
                     static_cast<MrState*>(st), nc, n, Y);
  return hipGetLastError();
}
hipError_t mr_scalars(const double* alfa, const double* beta2, int nc, void* st, hipStream_t s) {
  hipLaunchKernelGGL(k_mr_scalars, dim3(1), dim3(64), 0, s, alfa, beta2, nc,
                     static_cast<MrState*>(st));
  return hipGetLastError();
}
hipError_t mr_update(const double* V, const double* W1, const double* W2, const void* st, int nc,
                     int64_t n, double* Wn, double* T, hipStream_t s) {
  if (nc <= 0 || nc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mr_update, dim3(rows_grid(n, nc)), dim3(256), 0, s, V, W1, W2,
                     static_cast<const MrState*>(st), nc, n, Wn, T);
  return hipGetLastError();
}

}  // namespace lobpcg
