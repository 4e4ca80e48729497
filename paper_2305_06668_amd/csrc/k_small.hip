// Small dense fp64 linear algebra of the LOBPCG step, one workgroup each,
// everything resident in LDS (gfx950: 160 KB per workgroup):
//   * cyclic Jacobi eigensolver in parallel (round-robin) order for the
//     p x p Rayleigh-Ritz matrix, p <= 96 (Alg. 1, "solve a u = lambda u";
//     the paper calls LAPACK dsyev, Sec. 3.1);
//   * shifted Cholesky of an overlap matrix (Sec. 3.2: retry with
//     alpha * eps * ||X|| added to the diagonal, alpha = 100, 1000, ...);
//   * the implicit P coefficients u_p = ortho(u_x[:, act] - E[:, act]; u_x)
//     in R^p (Alg. 1 and the "Basis selection" paragraph of Sec. 3.1);
//   * the controller of ortho(W; Y) on n-vectors (Alg. 2 inside Alg. 3): it
//     reads the overlap G = [Y W]^T W of the current W and emits the small
//     coefficient matrix that the streaming kernel applies next.
#include "internal.h"

namespace lobpcg {

constexpr double kEps = 0x1.0p-52;  // double precision machine epsilon
constexpr double kShiftAlpha0 = 100.0;
constexpr double kShiftGrowth = 10.0;
constexpr int kShiftRetries = 20;
constexpr int kJacobiMaxSweeps = 40;

__device__ __forceinline__ uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// LDS writes of one wave visible to the same wave's later reads
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Cholesky of an n x n symmetric matrix (n <= 16) held by one wave in
// registers: lane l keeps column c = l & 15, rows r = (l >> 4) + 4 t
// (t = 0..3), in g[t]; only r >= c is read, and rows or columns from n to 15
// are those of the identity.  Right-looking, column by column: the pivot is
// read from its lane, column k of L is formed in its four lanes and handed
// to the others by lane shuffles, then the trailing entries are updated.
// Every entry takes the same operations in the same order as the LDS
// factorizations: G[r][k] / l_kk (KDIV) or G[r][k] * (1 / l_kk), and
// G[r][c] - L[r][k] L[c][k] as one fused multiply-add.  On return g holds L
// (diagonal included).  False, uniform over the wave, when a pivot is not
// > 0 (or, with CHECKINF, not finite); linv (LDS, may be null) receives
// 1 / l_kk when !KDIV.
template <bool KDIV, bool CHECKINF>
__device__ __forceinline__ bool reg_chol16(double (&g)[4], int n, double* linv) {
  const int l = threadIdx.x & 63, c = l & 15, rb = l >> 4;
  for (int k = 0; k < n; ++k) {
    // register k >> 2 of lane k + 16 (k & 3) (a select: no indexed registers)
    const int tk = k >> 2;
    const double gk = (tk == 0) ? g[0] : (tk == 1) ? g[1] : (tk == 2) ? g[2] : g[3];
    const double gkk = readlane_f64(gk, k + 16 * (k & 3));
    if (!(gkk > 0.0)) return false;
    if (CHECKINF && !(gkk < INFINITY)) return false;
    const double lkk = sqrt(gkk);
    const double inv = KDIV ? 0.0 : 1.0 / lkk;
    if (c == k) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = rb + 4 * t;
        if (r > k) g[t] = KDIV ? g[t] / lkk : g[t] * inv;
        else if (r == k) g[t] = lkk;
      }
    }
    if (!KDIV && linv != nullptr && l == 0) linv[k] = inv;
    // lr[t] = L[rb + 4t][k] (lane k + 16 rb, register t); lc[t] from lane
    // k + 16 (c & 3): L[c][k] is its register c >> 2
    double lr[4], lc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      lr[t] = __shfl(g[t], k + 16 * rb);
      lc[t] = __shfl(g[t], k + 16 * (c & 3));
    }
    const int tc = c >> 2;
    const double lck = (tc == 0) ? lc[0] : (tc == 1) ? lc[1] : (tc == 2) ? lc[2] : lc[3];
    if (c > k) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (rb + 4 * t >= c) g[t] = fma(-lr[t], lck, g[t]);
    }
  }
  return true;
}

// One wave (all 64 lanes): L = chol(S + shift I) for the n x n (n <= 16)
// matrix S in LDS (lower triangle read), written to L in LDS (lower
// triangle; the strict upper one zeroed when ZUP).  wave_chol16_lds is the
// out-of-line form, so that the large single-workgroup kernels keep their
// own register budgets.  Returns false (uniform) on a pivot that is not > 0
// (or, CHECKINF, not finite).
template <bool KDIV, bool CHECKINF, bool ZUP>
__device__ __forceinline__ bool wave_chol16_body(const double* S, int lds_, int n, double shift,
                                                 double* L, int ldl, double* linv) {
  const int l = threadIdx.x & 63, c = l & 15, rb = l >> 4;
  double g[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = rb + 4 * t;
    g[t] = (r < n && c < n) ? ((r >= c) ? S[r * lds_ + c] + (r == c ? shift : 0.0) : 0.0)
                            : (r == c ? 1.0 : 0.0);
  }
  const bool ok = reg_chol16<KDIV, CHECKINF>(g, n, linv);
  if (ok || ZUP) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = rb + 4 * t;
      if (r < n && c < n) {
        if (r >= c) L[r * ldl + c] = g[t];
        else if (ZUP) L[r * ldl + c] = 0.0;
      }
    }
  }
  return ok;
}
template <bool KDIV, bool CHECKINF, bool ZUP>
__device__ __noinline__ bool wave_chol16_lds(const double* S, int lds_, int n, double shift, double* L,
                                             int ldl, double* linv) {
  return wave_chol16_body<KDIV, CHECKINF, ZUP>(S, lds_, n, shift, L, ldl, linv);
}

// ---------------------------------------------------------------------------
// block-wide helpers (every thread of the block calls them)

__device__ __forceinline__ double blk_reduce_max(double v, double* scratch) {
  // scratch: blockDim.x / 64 doubles
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[w] = v;
  __syncthreads();
  double r = scratch[0];
  for (int i = 1; i < nw; ++i) r = fmax(r, scratch[i]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double blk_reduce_sum_ordered(double v, double* scratch) {
  // deterministic: each wave reduces by a fixed xor tree, waves in order
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[w] = v;
  __syncthreads();
  double r = scratch[0];
  for (int i = 1; i < nw; ++i) r += scratch[i];
  __syncthreads();
  return r;
}

// C (p x q) = A^T B, A: n x p, B: n x q
__device__ __forceinline__ void blk_gemm_tn(const double* A, int lda, const double* B, int ldb, int n, int p,
                            int q, double* C, int ldc) {
  for (int idx = threadIdx.x; idx < p * q; idx += blockDim.x) {
    const int i = idx / q, j = idx - i * q;
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += A[r * lda + i] * B[r * ldb + j];
    C[i * ldc + j] = s;
  }
  __syncthreads();
}

// X (n x q) -= Y (n x p) C (p x q)
__device__ __forceinline__ void blk_sub_mm(double* X, int ldx, const double* Y, int ldy, const double* C, int ldc,
                           int n, int p, int q) {
  for (int idx = threadIdx.x; idx < n * q; idx += blockDim.x) {
    const int r = idx / q, j = idx - r * q;
    double s = 0.0;
    for (int k = 0; k < p; ++k) s += Y[r * ldy + k] * C[k * ldc + j];
    X[r * ldx + j] -= s;
  }
  __syncthreads();
}

// scale columns of X (n x q) to unit norm; exact-zero columns are replaced
// by SplitMix64 columns (entry i of column j: splitmix64(seed + j n + i)).
__device__ __forceinline__ void blk_normalize(double* X, int ldx, int n, int q, double* tmp, int* zeros) {
  for (int j = threadIdx.x; j < q; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += X[r * ldx + j] * X[r * ldx + j];
    if (s == 0.0) {
      for (int r = 0; r < n; ++r) {
        const uint64_t z = sm64(kZeroColumnSeed + (uint64_t)j * (uint64_t)n + (uint64_t)r);
        X[r * ldx + j] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
      }
      s = 0.0;
      for (int r = 0; r < n; ++r) s += X[r * ldx + j] * X[r * ldx + j];
      atomicAdd(zeros, 1);
    }
    tmp[j] = sqrt(s);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * q; idx += blockDim.x) {
    const int j = idx % q;
    X[idx / q * ldx + j] /= tmp[j];
  }
  __syncthreads();
}

// Cholesky L L^T = M + shift I (lower, n x n); returns true on success.
// Breaks down when a pivot is not > 0 (NaN included), like LAPACK potrf.
// Every thread calls it and M must be complete on entry.  Wave 0 alone
// factors (REG != 0 and n <= 16: in registers, by an out-of-line call in
// the Rayleigh-Ritz kernel, whose register budget is full, inline in the
// ortho controller; otherwise column by column in LDS with wave-level
// syncs) while the other
// waves wait at the closing barriers: two workgroup barriers per
// factorization.  Each entry takes the same operations in the same order as
// a column-parallel factorization by the whole workgroup.
// REG: 0 column by column in LDS, 1 registers (out of line), 2 registers (inline)
template <int REG = 1>
__device__ __forceinline__ bool blk_chol(const double* M, int ldm, int n, double shift, double* L, int ldl,
                         int* flag) {
  if (REG != 0 && threadIdx.x < 64 && n <= 16) {
    const bool ok = (REG == 1) ? wave_chol16_lds<true, false, true>(M, ldm, n, shift, L, ldl, nullptr)
                               : wave_chol16_body<true, false, true>(M, ldm, n, shift, L, ldl, nullptr);
    if (threadIdx.x == 0) *flag = ok ? 0 : 1;
  } else if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    for (int idx = l; idx < n * n; idx += 64) {
      const int i = idx / n, j = idx - i * n;
      L[i * ldl + j] = (j <= i) ? (M[i * ldm + j] + (i == j ? shift : 0.0)) : 0.0;
    }
    int bad = 0;
    wave_sync();
    for (int j = 0; j < n; ++j) {
      const double d = L[j * ldl + j];
      if (!(d > 0.0)) {  // uniform across the wave
        bad = 1;
        break;
      }
      const double ljj = sqrt(d);
      if (l == 0) L[j * ldl + j] = ljj;
      for (int i = j + 1 + l; i < n; i += 64) L[i * ldl + j] /= ljj;
      wave_sync();
      const int rem = n - j - 1;
      for (int idx = l; idx < rem * rem; idx += 64) {
        const int i = j + 1 + idx / rem, k = j + 1 + idx % rem;
        if (k <= i) L[i * ldl + k] -= L[i * ldl + j] * L[k * ldl + j];
      }
      wave_sync();
    }
    if (l == 0) *flag = bad;
  }
  __syncthreads();
  const bool ok = (*flag == 0);
  __syncthreads();  // the flag is rewritten by the next call
  return ok;
}

struct ShiftCount {
  int factorizations, failed, shifted, svqb;
};

// Sec. 3.2 / Alg. 2: plain Cholesky, then shifts alpha*eps*||X||_F with
// ||X||_F = sqrt(trace M), alpha = 100, x10 per retry.
template <int REG = 1>
__device__ __forceinline__ bool blk_shifted_chol(const double* M, int ldm, int n, double* L, int ldl, int* flag,
                                 ShiftCount* c, double* scratch, int retries = kShiftRetries) {
  if (threadIdx.x == 0) c->factorizations++;
  if (blk_chol<REG>(M, ldm, n, 0.0, L, ldl, flag)) return true;
  if (threadIdx.x == 0) c->failed++;
  double tr = 0.0;
  for (int i = 0; i < n; ++i) tr += M[i * ldm + i];
  const double normx = sqrt(fmax(tr, 0.0));
  double alpha = kShiftAlpha0;
  for (int t = 0; t < retries; ++t) {
    if (threadIdx.x == 0) c->factorizations++;
    if (blk_chol<REG>(M, ldm, n, alpha * kEps * normx, L, ldl, flag)) {
      if (threadIdx.x == 0) c->shifted++;
      return true;
    }
    if (threadIdx.x == 0) c->failed++;
    alpha *= kShiftGrowth;
  }
  return false;
}

// Linv = L^-1 (lower), one column per thread by forward substitution.
__device__ __forceinline__ void blk_tri_inv(const double* L, int ldl, int n, double* Li, int ldi) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      if (i < j) {
        Li[i * ldi + j] = 0.0;
        continue;
      }
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= L[i * ldl + k] * Li[k * ldi + j];
      Li[i * ldi + j] = s / L[i * ldl + i];
    }
  }
  __syncthreads();
}

// X (n x q) <- X L^-T, one row per thread: z_j = (x_j - sum_{k<j} z_k L_jk) / L_jj
__device__ __forceinline__ void blk_trsm_rt(double* X, int ldx, int n, int q, const double* L, int ldl) {
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    for (int j = 0; j < q; ++j) {
      double s = X[r * ldx + j];
      for (int k = 0; k < j; ++k) s -= X[r * ldx + k] * L[j * ldl + k];
      X[r * ldx + j] = s / L[j * ldl + j];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi on the symmetric n x n matrix A (LDS, stride lda),
// accumulating V (stride ldv, initialised here to I).  Round-robin pairing:
// in round r the pairs are {pp-1, r} and {(r+k) mod (pp-1), (r-k) mod (pp-1)}
// for k = 1 .. pp/2-1, with pp = n rounded up to even (index n is a dummy).
// Two phases per round: (1) one thread per pair computes its rotation from
// the current 2x2 block; (2) every 2x2 block {i0,i1} x {j0,j1} of two pairs
// is rotated in place from both sides by one thread (it is closed under
// J^T A J, so no double buffer is needed), and V's column pairs likewise.
// A rotation is skipped when |a_pq| <= 2^-53 sqrt(|a_pp a_qq|) or
// |a_pq| <= 2^-60 ||A||_F; the sweep loop stops after a sweep without any
// rotation.  Returns the number of sweeps.  Must run with blockDim.x == 1024.

__device__ __forceinline__ int blk_jacobi(double* A, int lda, double* V, int ldv, int n, double* cs, int* pr,
                          int* rot_flag, double* scratch) {
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx - i * n;
    V[i * ldv + j] = (i == j) ? 1.0 : 0.0;
  }
  double fro = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const double v = A[(idx / n) * lda + idx % n];
    fro += v * v;
  }
  fro = sqrt(blk_reduce_sum_ordered(fro, scratch));
  const double abs_tol = 0x1.0p-60 * fro;
  if (n < 2) return 0;
  const int pp = n + (n & 1);
  const int npairs = pp / 2;
  double* cc = cs;            // cos per pair
  double* ss = cs + 64;       // sin per pair
  double* tt = cs + 128;      // tan per pair
  int sweep = 0;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (; sweep < kJacobiMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) *rot_flag = 0;
    __syncthreads();
    for (int r = 0; r < pp - 1; ++r) {
      for (int k = threadIdx.x; k < npairs; k += blockDim.x) {
        int i, j;
        if (k == 0) {
          i = pp - 1;
          j = r;
        } else {
          i = r + k;
          if (i >= pp - 1) i -= pp - 1;
          j = r - k;
          if (j < 0) j += pp - 1;
        }
        if (i > j) {
          const int t = i;
          i = j;
          j = t;
        }
        double c = 1.0, sn = 0.0, tn = 0.0;
        if (j < n) {
          const double apq = A[i * lda + j];
          const double app = A[i * lda + i], aqq = A[j * lda + j];
          if (fabs(apq) > 0x1.0p-53 * sqrt(fabs(app * aqq)) && fabs(apq) > abs_tol) {
            const double tau = (aqq - app) / (2.0 * apq);
            tn = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                              : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tn * tn);
            sn = tn * c;
            *rot_flag = 1;
          }
        }
        pr[2 * k] = i;
        pr[2 * k + 1] = j;
        cc[k] = c;
        ss[k] = sn;
        tt[k] = tn;
      }
      __syncthreads();
      // Phase 2 (needs blockDim == 1024: a 32 x 32 thread grid).  Thread
      // (ty, tx) owns the 2x2 blocks (P, Q) for P in {ty, ty+32}, Q in
      // {tx, tx+32} with P <= Q, and V's column pair Q on the rows ty,
      // ty+32, ty+64; every load of an item is issued before its arithmetic.
#pragma unroll
      for (int hq = 0; hq < 2; ++hq) {
        const int Q = tx + 32 * hq;
        if (Q >= npairs) continue;
        const double cQ = cc[Q], sQ = ss[Q], tQ = tt[Q];
        const int j0 = pr[2 * Q], j1 = pr[2 * Q + 1];
        const bool vj1 = j1 < n;
#pragma unroll
        for (int hp = 0; hp < 2; ++hp) {
          const int P = ty + 32 * hp;
          if (P >= npairs || P > Q) continue;
          if (P == Q) {
            if (sQ == 0.0) continue;  // skipped or dummy pair
            const double a01 = A[j0 * lda + j1];
            const double a00 = A[j0 * lda + j0], a11 = A[j1 * lda + j1];
            A[j0 * lda + j0] = a00 - tQ * a01;
            A[j1 * lda + j1] = a11 + tQ * a01;
            A[j0 * lda + j1] = 0.0;
            A[j1 * lda + j0] = 0.0;
            continue;
          }
          const double cP = cc[P], sP = ss[P];
          if (sP == 0.0 && sQ == 0.0) continue;
          const int i0 = pr[2 * P], i1 = pr[2 * P + 1];
          const bool vi1 = i1 < n;
          const double b00 = A[i0 * lda + j0];
          const double b01 = vj1 ? A[i0 * lda + j1] : 0.0;
          const double b10 = vi1 ? A[i1 * lda + j0] : 0.0;
          const double b11 = (vi1 && vj1) ? A[i1 * lda + j1] : 0.0;
          // rows (J^T A): i0' = c i0 - s i1, i1' = s i0 + c i1
          const double t00 = cP * b00 - sP * b10, t01 = cP * b01 - sP * b11;
          const double t10 = sP * b00 + cP * b10, t11 = sP * b01 + cP * b11;
          // columns (A J): j0' = c j0 - s j1, j1' = s j0 + c j1
          const double n00 = cQ * t00 - sQ * t01, n01 = sQ * t00 + cQ * t01;
          const double n10 = cQ * t10 - sQ * t11, n11 = sQ * t10 + cQ * t11;
          A[i0 * lda + j0] = n00;
          A[j0 * lda + i0] = n00;
          if (vj1) {
            A[i0 * lda + j1] = n01;
            A[j1 * lda + i0] = n01;
          }
          if (vi1) {
            A[i1 * lda + j0] = n10;
            A[j0 * lda + i1] = n10;
          }
          if (vi1 && vj1) {
            A[i1 * lda + j1] = n11;
            A[j1 * lda + i1] = n11;
          }
        }
        if (sQ != 0.0) {
          // rows ty, ty + 32, ty + 64 (clamped reads, guarded writes)
          const int r0 = ty, r1 = ty + 32, r2 = ty + 64;
          const int q1 = (r1 < n) ? r1 : r0, q2 = (r2 < n) ? r2 : r0;
          const double a0 = V[r0 * ldv + j0], b0 = V[r0 * ldv + j1];
          const double a1 = V[q1 * ldv + j0], b1 = V[q1 * ldv + j1];
          const double a2 = V[q2 * ldv + j0], b2 = V[q2 * ldv + j1];
          if (r0 < n) {
            V[r0 * ldv + j0] = cQ * a0 - sQ * b0;
            V[r0 * ldv + j1] = sQ * a0 + cQ * b0;
          }
          if (r1 < n) {
            V[r1 * ldv + j0] = cQ * a1 - sQ * b1;
            V[r1 * ldv + j1] = sQ * a1 + cQ * b1;
          }
          if (r2 < n) {
            V[r2 * ldv + j0] = cQ * a2 - sQ * b2;
            V[r2 * ldv + j1] = sQ * a2 + cQ * b2;
          }
        }
      }
      __syncthreads();
    }
    const int any = *rot_flag;
    __syncthreads();
    if (!any) break;
    // stop without a confirming sweep when no pair would rotate any more
    if (threadIdx.x == 0) *rot_flag = 0;
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      const int i = idx / n, j = idx - i * n;
      if (j <= i) continue;
      const double apq = A[i * lda + j];
      if (fabs(apq) > 0x1.0p-53 * sqrt(fabs(A[i * lda + i] * A[j * lda + j])) && fabs(apq) > abs_tol)
        *rot_flag = 1;
    }
    __syncthreads();
    const int more = *rot_flag;
    __syncthreads();
    if (!more) break;
  }
  return sweep + 1;
}

// evals ascending (ties by index) -> perm[rank] = index
__device__ __forceinline__ void blk_sort_evals(const double* A, int lda, int n, int* perm) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double li = A[i * lda + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j * lda + j];
      if (lj < li || (lj == li && j < i)) ++rank;
    }
    perm[rank] = i;
  }
  __syncthreads();
}

// LDS layout shared by the eig-based kernels
struct EigLds {
  double* A;  // p x (p+1)
  double* V;  // p x (p+1)
  double* cs;
  int* pr;
  int* perm;
  double* scratch;
  int* flags;
};

// The second area holds V during the Jacobi sweeps and, in k_small_rr, the
// R^p orthonormalisation work arrays afterwards (X p x na, C m x na, M, L and
// an SVQB workspace), hence its size max(p (p+1), 2 p m + 3 m^2 + 2 m).
__host__ __device__ inline int eig_area2(int p, int m) {
  const int a = p * (p + 1), b = 2 * p * m + 3 * m * m + 2 * m;
  return a > b ? a : b;
}
__device__ __forceinline__ EigLds eig_lds(double* smem, int p, int m) {
  EigLds L;
  const int ld = p + 1;
  L.A = smem;
  L.V = L.A + p * ld;
  L.cs = L.V + eig_area2(p, m);   // 3 * 64
  L.scratch = L.cs + 3 * 64;      // 16
  L.pr = (int*)(L.scratch + 16);  // 2 * 64
  L.perm = L.pr + 2 * 64;         // 128
  L.flags = L.perm + 128;         // 8
  return L;
}
static size_t eig_lds_bytes(int p, int m) {
  return sizeof(double) * (size_t)(p * (p + 1) + eig_area2(p, m) + 3 * 64 + 16) +
         sizeof(int) * (2 * 64 + 128 + 8);
}

__device__ __forceinline__ void load_sym(const double* a, int p, double* A, int lda) {
  for (int idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
    const int i = idx / p, j = idx - i * p;
    A[i * lda + j] = 0.5 * (a[i * p + j] + a[j * p + i]);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Lowest nev eigenpairs of a symmetric p x p matrix by the tridiagonal
// route (the Rayleigh-Ritz solve of Alg. 1; the paper calls LAPACK for it,
// Sec. 3.1).  Jacobi needs p - 1 dependent rounds per sweep, each a chain
// of square roots and divisions followed by a full-matrix update; this path
// has one short chain per reflector and per Sturm count instead:
//   1. Householder reduction A = Q T Q^T by the workgroup: reflector k,
//      H_k = I - beta_k v_k v_k^T, maps column k below the diagonal to
//      alpha_k e_{k+1} (v_k kept in that column, Q = H_0 H_1 ... H_{p-3});
//   2. the nev lowest eigenvalues of T by multisection on Sturm counts
//      (counts of negative pivots of T - x I with LAPACK's pivmin guard),
//      G points per eigenvalue and round;
//   3. their vectors by block inverse iteration: a solve with the
//      partial-pivoting LU of T - lambda_j I from a SplitMix64 start
//      (pivots below eps ||T|| raised to eps ||T||, one thread per vector),
//      Cholesky-QR of the nev vectors, a second solve;
//   4. back-transformation u = Q z, one wave per vector;
//   5. Cholesky-QR, twice, of the nev vectors.
// Inverse iteration returns the vectors of a cluster of close or repeated
// eigenvalues as independent mixtures of the cluster's eigenvectors, which
// drift towards each other with further solves; orthonormalising them in
// ascending order between and after the solves keeps them an orthonormal
// eigenbasis of the cluster (residuals and orthogonality ~1e-15 ||A|| on
// repeated and 1e-14-separated eigenvalues, where three plain solves
// followed by Cholesky-QR lose two digits).
// Returns false when a Cholesky-QR breaks down (A is destroyed); the
// callers then reload A and run Jacobi.

constexpr int kEigLdsBytes = 152 * 1024;  // dynamic LDS of the eigensolver kernels
constexpr int kMsPoints = 32;              // multisection points per eigenvalue


template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Sum over the 64 lanes (all active), the same bits in every lane: within
// each row of 16 by DPP (swap neighbours, swap pairs, mirror 8, mirror 16;
// each step adds the same two operands on both partners), then the four row
// sums in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// LDS layout after the p x (p+1) A area, in doubles
struct TriLayout {
  int ldz, nb;
  int d, e, inve, e2, beta, vv, ww, ev, linv, G, Z, ws, sw, total;
};
__host__ __device__ inline TriLayout tri_layout(int p, int nev) {
  TriLayout t;
  t.ldz = nev + 1;
  int o = 0;
  t.d = o; o += p;
  t.e = o; o += p;
  t.inve = o; o += p;
  t.e2 = o; o += p;
  t.beta = o; o += p;
  t.vv = o; o += p;
  t.ww = o; o += p;
  t.ev = o; o += nev;
  t.linv = o; o += nev;
  t.G = o; o += nev * (nev + 1);
  t.Z = o; o += p * t.ldz;
  t.ws = o;
  const int avail = kEigLdsBytes / 8 - p * (p + 1) - o;
  const int per = 4 * p + (p + 7) / 8 + 1;  // U0^-1, U1, U2, multipliers + pivot flags
  int nb = avail / per;
  if (nb > nev) nb = nev;
  t.nb = nb;
  if (nb < 1) {
    t.sw = o;
    t.total = o;
    return t;
  }
  o += 4 * p * nb;
  t.sw = o;
  o += (p * nb + 7) / 8;
  t.total = o;
  return t;
}

// Householder reduction by the whole workgroup, three barriers per step:
// wave 0 forms reflector k from row k (= column k, the trailing block is
// kept symmetric); each wave takes rows i of p = beta A v, its lanes
// splitting the row; every thread then updates trailing entries with
// w = p - K v, K = beta/2 p^T v (formed by every wave in the same order).
__device__ void blk_tridiag(double* A, int lda, int p, double* d, double* e, double* beta, double* vv,
                            double* pp) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, nw = blockDim.x >> 6;
  for (int k = 0; k + 2 < p; ++k) {
    const int k1 = k + 1, s = p - k1;
    if (wave == 0) {
      double x[2];
      double tail = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        x[h] = (i > k && i < p) ? A[k * lda + i] : 0.0;
        if (i > k1) tail += x[h] * x[h];
      }
      const double x1 = A[k * lda + k1];
      tail = wave_sum(tail);
      double alpha = x1, b = 0.0;
      if (tail > 0.0) {
        const double nrm = sqrt(x1 * x1 + tail);
        alpha = (x1 >= 0.0) ? -nrm : nrm;
        b = 1.0 / (nrm * (nrm + fabs(x1)));  // 2 / v^T v for v = x - alpha e_1
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        if (i > k && i < p) {
          const double v = (b != 0.0 && i == k1) ? x1 - alpha : x[h];
          A[i * lda + k] = v;  // reflector k, kept for the back-transformation
          vv[i] = v;
        }
      }
      if (lane == 0) {
        d[k] = A[k * lda + k];
        e[k] = alpha;
        beta[k] = b;
      }
    }
    __syncthreads();
    const double b = beta[k];
    if (b == 0.0) continue;  // H_k = I (uniform)
    for (int i = k1 + wave; i < p; i += nw) {
      double acc = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = k1 + lane + 64 * h;
        if (j < p) acc += A[i * lda + j] * vv[j];
      }
      acc = wave_sum(acc);
      if (lane == 0) pp[i] = b * acc;
    }
    __syncthreads();
    double kp = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = k1 + lane + 64 * h;
      if (i < p) kp += pp[i] * vv[i];
    }
    const double K = 0.5 * b * wave_sum(kp);
    for (int idx = tid; idx < s * s; idx += blockDim.x) {
      const int jj = idx / s, ii = idx - jj * s;
      const int j = k1 + jj, i = k1 + ii;
      const double vj = vv[j], vi = vv[i];
      const double wi = pp[i] - K * vi, wj = pp[j] - K * vj;
      A[j * lda + i] -= vj * wi + wj * vi;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (p >= 2) {
      d[p - 2] = A[(p - 2) * lda + p - 2];
      e[p - 2] = A[(p - 1) * lda + p - 2];
    }
    d[p - 1] = A[(p - 1) * lda + p - 1];
  }
  __syncthreads();
}

// 1 / q to ~1 ulp: the hardware reciprocal and one Newton step (the Sturm
// count only needs each step to a few ulps, Kahan's backward-error argument)
__device__ __forceinline__ double rcp_nr(double q) {
  const double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}

// number of eigenvalues of T below x (negative pivots of T - x I)
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int p, double x,
                                           double pivmin) {
  double q = d[0] - x;
  int c = 0;
  if (q <= pivmin) {
    ++c;
    q = fmin(q, -pivmin);
  }
#pragma unroll 4
  for (int i = 1; i < p; ++i) {
    q = (d[i] - x) - e2[i - 1] * rcp_nr(q);
    if (q <= pivmin) {
      ++c;
      q = fmin(q, -pivmin);
    }
  }
  return c;
}

// eigenvalues 0 .. nev-1 (ascending) of T into ev; every thread calls it
__device__ void blk_multisection(const double* d, const double* e2, int p, int nev, double gl, double gu,
                                 double tnorm, double pivmin, double* ev) {
  int G = kMsPoints;
  while (G > 1 && G * nev > (int)blockDim.x) G >>= 1;
  const int t = threadIdx.x & (G - 1);
  const int gi = threadIdx.x / G, ngroups = blockDim.x / G;
  const int lane = threadIdx.x & 63;
  const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (lane & ~(G - 1)));
  for (int j = gi; j < nev; j += ngroups) {
    double lo = gl, hi = gu;
    for (int round = 0; round < 256; ++round) {
      const double w = hi - lo;
      if (w <= 2.0 * kEps * fmax(fabs(lo), fabs(hi)) || w <= kEps * tnorm) break;
      const double h = w / (double)(G + 1);
      const double x = lo + (double)(t + 1) * h;
      const int c = sturm_count(d, e2, p, x, pivmin);
      const int k = __popcll(__ballot(c <= j) & gmask);
      const double nlo = (k > 0) ? lo + (double)k * h : lo;
      const double nhi = (k < G) ? lo + (double)(k + 1) * h : hi;
      if (nlo == lo && nhi == hi) break;
      lo = nlo;
      hi = nhi;
    }
    if (t == 0) ev[j] = lo + 0.5 * (hi - lo);
  }
}

// one inverse-iteration solve of (T - lam I) z = Z[:, j] for the vectors
// j = j0 + t, t < nb (thread t); factor = true builds the LU, else reuses it.
// The loads of the next step are issued before the current step's stores.
__device__ void tri_invit_solve(const double* __restrict__ d, const double* __restrict__ e,
                                const double* __restrict__ inve, int p, double lam, double tol, double* Z,
                                int ldz, int j, double* ws, uint8_t* sw, int nb, int t, bool factor) {
  double* U0 = ws;
  double* U1 = ws + p * nb;
  double* U2 = ws + 2 * p * nb;
  double* LM = ws + 3 * p * nb;
  double y = Z[j];
  double bnx = (p > 1) ? Z[ldz + j] : 0.0;
  if (factor) {
    double c0 = d[0] - lam, c1 = (p > 1) ? e[0] : 0.0;
    for (int i = 0; i + 1 < p; ++i) {
      const double ei = e[i];
      const double dn = d[i + 1] - lam;
      const double en = (i + 2 < p) ? e[i + 1] : 0.0;
      const double ie = inve[i];
      const double bn = bnx;
      if (i + 2 < p) bnx = Z[(i + 2) * ldz + j];
      if (fabs(c0) >= fabs(ei)) {
        if (fabs(c0) < tol) c0 = (c0 < 0.0) ? -tol : tol;
        const double li = ei / c0;
        U0[i * nb + t] = 1.0 / c0;
        U1[i * nb + t] = c1;
        U2[i * nb + t] = 0.0;
        LM[i * nb + t] = li;
        sw[i * nb + t] = 0;
        Z[i * ldz + j] = y;
        y = bn - li * y;
        c0 = dn - li * c1;
        c1 = en;
      } else {
        const double li = c0 * ie;
        U0[i * nb + t] = ie;
        U1[i * nb + t] = dn;
        U2[i * nb + t] = en;
        LM[i * nb + t] = li;
        sw[i * nb + t] = 1;
        Z[i * ldz + j] = bn;
        y = y - li * bn;
        const double nc0 = c1 - li * dn;
        c1 = -li * en;
        c0 = nc0;
      }
    }
    if (fabs(c0) < tol) c0 = (c0 < 0.0) ? -tol : tol;
    U0[(p - 1) * nb + t] = 1.0 / c0;
    U1[(p - 1) * nb + t] = 0.0;
    U2[(p - 1) * nb + t] = 0.0;
  } else {
    double lmx = LM[t];
    uint8_t swx = sw[t];
    for (int i = 0; i + 1 < p; ++i) {
      const double bn = bnx, li = lmx;
      const uint8_t si = swx;
      if (i + 2 < p) bnx = Z[(i + 2) * ldz + j];
      if (i + 1 < p) {
        lmx = LM[(i + 1) * nb + t];
        swx = sw[(i + 1) * nb + t];
      }
      if (si == 0) {
        Z[i * ldz + j] = y;
        y = bn - li * y;
      } else {
        Z[i * ldz + j] = bn;
        y = y - li * bn;
      }
    }
  }
  Z[(p - 1) * ldz + j] = y;
  double z1 = 0.0, z2 = 0.0, zmax = 0.0;
  double zx = Z[(p - 1) * ldz + j], u0x = U0[(p - 1) * nb + t], u1x = U1[(p - 1) * nb + t],
         u2x = U2[(p - 1) * nb + t];
  for (int i = p - 1; i >= 0; --i) {
    const double zr = zx, u0 = u0x, u1 = u1x, u2 = u2x;
    if (i > 0) {
      zx = Z[(i - 1) * ldz + j];
      u0x = U0[(i - 1) * nb + t];
      u1x = U1[(i - 1) * nb + t];
      u2x = U2[(i - 1) * nb + t];
    }
    const double zi = (zr - u1 * z1 - u2 * z2) * u0;
    Z[i * ldz + j] = zi;
    zmax = fmax(zmax, fabs(zi));
    z2 = z1;
    z1 = zi;
  }
  const double sc = (zmax > 0.0 && zmax < INFINITY) ? 1.0 / zmax : 1.0;
#pragma unroll 4
  for (int i = 0; i < p; ++i) Z[i * ldz + j] *= sc;
}

// G (lower, n x n, stride ldg) <- Z^T Z for Z (p x n, stride ldz), every
// thread; ends with a barrier
__device__ void blk_gram_lower(const double* Z, int ldz, int p, int n, double* G, int ldg) {
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int r = idx / n, c = idx - r * n;
    if (c > r) continue;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = 0;
    for (; i + 4 <= p; i += 4) {
      s0 += Z[i * ldz + r] * Z[i * ldz + c];
      s1 += Z[(i + 1) * ldz + r] * Z[(i + 1) * ldz + c];
      s2 += Z[(i + 2) * ldz + r] * Z[(i + 2) * ldz + c];
      s3 += Z[(i + 3) * ldz + r] * Z[(i + 3) * ldz + c];
    }
    for (; i < p; ++i) s0 += Z[i * ldz + r] * Z[i * ldz + c];
    G[r * ldg + c] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
}

// Z <- Z L^-T with L L^T = G (the Gram Z^T Z from blk_gram_lower), by one
// wave; G is overwritten by L (n <= 16: factored in registers by
// reg_chol16).  False when a pivot is not > 0.
template <int NR>
__device__ bool wave_cholqr(double* Z, int ldz, int p, int n, double* G, int ldg, double* linv) {
  const int l = threadIdx.x & 63;
  wave_sync();
  if (n <= 16) {
    if (!wave_chol16_lds<false, true, false>(G, ldg, n, 0.0, G, ldg, linv)) return false;
    wave_sync();
  } else {
    for (int k = 0; k < n; ++k) {
      const double gkk = G[k * ldg + k];
      if (!(gkk > 0.0) || !(gkk < INFINITY)) return false;
      const double lkk = sqrt(gkk), inv = 1.0 / lkk;
#pragma unroll
      for (int h = 0; h < NR; ++h) {
        const int r = l + 64 * h;
        if (r > k && r < n) G[r * ldg + k] *= inv;
      }
      if (l == 0) {
        G[k * ldg + k] = lkk;
        linv[k] = inv;
      }
      wave_sync();
      // trailing update, lane c owning column c: G[r][c] -= L[r][k] L[c][k], r >= c > k
#pragma unroll
      for (int h = 0; h < NR; ++h) {
        const int c = l + 64 * h;
        if (c > k && c < n) {
          const double lck = G[c * ldg + k];
          for (int r0 = c; r0 < n; r0 += 4) {
            double lk[4], gc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int r = min(r0 + u, n - 1);
              lk[u] = G[r * ldg + k];
              gc[u] = G[r * ldg + c];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (r0 + u < n) G[(r0 + u) * ldg + c] = gc[u] - lk[u] * lck;
          }
        }
      }
      wave_sync();
    }
  }
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int i = l + 64 * h;
    if (i < p) {
      for (int jj = 0; jj < n; ++jj) {
        double s0 = Z[i * ldz + jj], s1 = 0.0;
        int k = 0;
        for (; k + 2 <= jj; k += 2) {
          s0 -= Z[i * ldz + k] * G[jj * ldg + k];
          s1 -= Z[i * ldz + k + 1] * G[jj * ldg + k + 1];
        }
        if (k < jj) s0 -= Z[i * ldz + k] * G[jj * ldg + k];
        Z[i * ldz + jj] = (s0 + s1) * linv[jj];
      }
    }
  }
  wave_sync();
  return true;
}

// The whole path (1-5).  A: p x lda in LDS (destroyed); base: the area after
// A laid out by tri_layout(p, nev), whose ev and Z receive the result.  Every
// thread calls it; the return value is uniform.
__device__ bool blk_tri_eigh(double* A, int lda, int p, int nev, double* base, const TriLayout& L,
                             int* flag) {
  double* d = base + L.d;
  double* e = base + L.e;
  double* inve = base + L.inve;
  double* e2 = base + L.e2;
  double* beta = base + L.beta;
  double* ev = base + L.ev;
  double* Z = base + L.Z;
  const int ldz = L.ldz;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  blk_tridiag(A, lda, p, d, e, beta, base + L.vv, base + L.ww);
  // Gershgorin interval, ||T||, pivmin (every thread, same order)
  double gl = INFINITY, gu = -INFINITY, emax2 = 0.0;
  for (int i = 0; i < p; ++i) {
    const double r = ((i > 0) ? fabs(e[i - 1]) : 0.0) + ((i + 1 < p) ? fabs(e[i]) : 0.0);
    gl = fmin(gl, d[i] - r);
    gu = fmax(gu, d[i] + r);
    if (i + 1 < p) emax2 = fmax(emax2, e[i] * e[i]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  if (!(tnorm < INFINITY)) return false;
  if (tnorm == 0.0) {  // the zero matrix
    for (int idx = threadIdx.x; idx < p * nev; idx += blockDim.x) {
      const int i = idx / nev, j = idx - i * nev;
      Z[i * ldz + j] = (i == j) ? 1.0 : 0.0;
    }
    for (int j = threadIdx.x; j < nev; j += blockDim.x) ev[j] = 0.0;
    __syncthreads();
    return true;
  }
  const double pivmin = 0x1.0p-1022 * fmax(1.0, emax2);
  const double tol = kEps * tnorm;
  const double widen = 2.1 * (kEps * tnorm * p + 2.0 * pivmin);
  gl -= widen;
  gu += widen;
  for (int i = threadIdx.x; i + 1 < p; i += blockDim.x) {
    e2[i] = e[i] * e[i];
    const double piv = (fabs(e[i]) < tol) ? ((e[i] < 0.0) ? -tol : tol) : e[i];
    inve[i] = (e[i] == 0.0) ? 0.0 : 1.0 / piv;
  }
  __syncthreads();
  blk_multisection(d, e2, p, nev, gl, gu, tnorm, pivmin, ev);
  // start vectors
  for (int idx = threadIdx.x; idx < p * nev; idx += blockDim.x) {
    const int i = idx / nev, j = idx - i * nev;
    const uint64_t z = sm64(kZeroColumnSeed ^ (0x5EEDull << 32) ^ ((uint64_t)j * (uint64_t)p + (uint64_t)i));
    Z[i * ldz + j] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
  }
  __syncthreads();
  // two solves with a Cholesky-QR between them (block inverse iteration);
  // with several batches the LU is rebuilt for the second solve
  const int nb = L.nb;
  for (int it = 0; it < 2; ++it) {
    for (int j0 = 0; j0 < nev; j0 += nb) {
      const int t = threadIdx.x;
      if (t < nb && j0 + t < nev) {
        const int j = j0 + t;
        tri_invit_solve(d, e, inve, p, ev[j], tol, Z, ldz, j, base + L.ws,
                        reinterpret_cast<uint8_t*>(base + L.sw), nb, t, it == 0 || nb < nev);
      }
      __syncthreads();
    }
    if (it == 0) {
      blk_gram_lower(Z, ldz, p, nev, base + L.G, nev + 1);
      if (wave == 0) {
        const bool ok = (p <= 64) ? wave_cholqr<1>(Z, ldz, p, nev, base + L.G, nev + 1, base + L.linv)
                                  : wave_cholqr<2>(Z, ldz, p, nev, base + L.G, nev + 1, base + L.linv);
        if (lane == 0) *flag = ok ? 1 : 0;
      }
      __syncthreads();
      const bool ok = *flag != 0;
      __syncthreads();
      if (!ok) return false;
    }
  }
  // u = H_0 H_1 ... H_{p-3} z, one wave per vector
  const int nw = blockDim.x >> 6;
  for (int j = wave; j < nev; j += nw) {
    double z[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      z[h] = (i < p) ? Z[i * ldz + j] : 0.0;
    }
#pragma unroll 2
    for (int k = p - 3; k >= 0; --k) {
      const double b = beta[k];  // 0 for H_k = I: then s = 0
      double v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        v[h] = (i > k && i < p) ? A[i * lda + k] : 0.0;
      }
      const double s = b * wave_sum(v[0] * z[0] + v[1] * z[1]);
      z[0] -= s * v[0];
      z[1] -= s * v[1];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i < p) Z[i * ldz + j] = z[h];
    }
  }
  __syncthreads();
  // Cholesky-QR twice, with the A area as Gram scratch.  One pass leaves
  // the vectors orthonormal to a few units of rounding when the Gram is
  // well conditioned, yet the second pass is kept: the P coefficients are
  // the small differences u_x - E, and dropping it whenever the columns'
  // cosines were below 1e-3 doubled the iterations of a dense generalized
  // solve (n = 2000, 4 pairs: 51 against 25, the lowest pair lagging).
  for (int pass = 0; pass < 2; ++pass) {
    blk_gram_lower(Z, ldz, p, nev, A, lda);
    if (wave == 0) {
      const bool ok = (p <= 64) ? wave_cholqr<1>(Z, ldz, p, nev, A, lda, base + L.linv)
                                : wave_cholqr<2>(Z, ldz, p, nev, A, lda, base + L.linv);
      if (lane == 0) *flag = ok ? 1 : 0;
    }
    __syncthreads();
    const bool ok = *flag != 0;
    __syncthreads();
    if (!ok) return false;
  }
  return true;
}

__global__ __launch_bounds__(1024) void k_small_eigh(const double* __restrict__ a, int p,
                                                    double* __restrict__ evals,
                                                    double* __restrict__ evecs, int* sweeps) {
  extern __shared__ double smem[];
  __shared__ int tflag;
  const int ld = p + 1;
  const TriLayout T = tri_layout(p, p);
  if (T.nb >= 1) {
    load_sym(a, p, smem, ld);
    double* base = smem + p * ld;
    if (blk_tri_eigh(smem, ld, p, p, base, T, &tflag)) {
      for (int idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
        const int i = idx / p, j = idx - i * p;
        const double sg = (base[T.Z + j * T.ldz + j] < 0.0) ? -1.0 : 1.0;
        evecs[i * p + j] = sg * base[T.Z + i * T.ldz + j];
      }
      for (int j = threadIdx.x; j < p; j += blockDim.x) evals[j] = base[T.ev + j];
      if (threadIdx.x == 0 && sweeps != nullptr) *sweeps = 0;
      return;
    }
  }
  EigLds L = eig_lds(smem, p, 1);
  load_sym(a, p, L.A, ld);
  const int sw = blk_jacobi(L.A, ld, L.V, ld, p, L.cs, L.pr, L.flags, L.scratch);
  blk_sort_evals(L.A, ld, p, L.perm);
  for (int idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
    const int i = idx / p, j = idx - i * p;
    const double sg = (L.V[j * ld + L.perm[j]] < 0.0) ? -1.0 : 1.0;
    evecs[i * p + j] = sg * L.V[i * ld + L.perm[j]];
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x) evals[j] = L.A[L.perm[j] * ld + L.perm[j]];
  if (threadIdx.x == 0 && sweeps != nullptr) *sweeps = sw;
}

hipError_t small_eigh(const double* a, int p, double* evals, double* evecs, int* sweeps,
                      hipStream_t s) {
  if (p < 1 || p > kMaxP) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_small_eigh, hipFuncAttributeMaxDynamicSharedMemorySize,
                              152 * 1024);
    (void)hipGetLastError();
    attr = true;
  }
  hipLaunchKernelGGL(k_small_eigh, dim3(1), dim3(1024), kEigLdsBytes, s, a, p, evals, evecs, sweeps);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// SVQB (Stathopoulos-Wu) coefficient for an n x n overlap M: X <- X U S^-1/2,
// eigenvalues clamped below eps * max.  Writes the n x n coefficient to Cf.
// Uses Ws (2 * n * (n+1) doubles) as Jacobi workspace.
__device__ __forceinline__ bool blk_svqb_coef(const double* M, int ldm, int n, double* Cf, int ldc, double* Ws,
                              double* cs, int* pr, int* flag, int* perm, double* scratch) {
  const int ld = n + 1;
  double* A = Ws;
  double* U = Ws + n * ld;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx - i * n;
    A[i * ld + j] = M[i * ldm + j];
  }
  __syncthreads();
  blk_jacobi(A, ld, U, ld, n, cs, pr, flag, scratch);
  double smax = 0.0;
  for (int i = 0; i < n; ++i) smax = fmax(smax, A[i * ld + i]);
  if (!(smax > 0.0)) return false;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx - i * n;
    const double sj = fmax(A[j * ld + j], kEps * smax);
    Cf[i * ldc + j] = U[i * ld + j] / sqrt(sj);
  }
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz coefficients (Alg. 1): eig of sym(a); u_x = lowest m
// eigenvectors; optionally u_p = ortho(u_x[:, a0:m] - E[:, a0:m]; u_x) in R^p
// by Alg. 3 / Alg. 2 (the same readings as on n-vectors).

// sym(a) into A (stride lda), with the pending column scaling of the W block
// (see small_rr in internal.h) applied from both sides when pend != nullptr
__device__ void load_rr_matrix(const double* a, int p, double* A, int lda, const OrthoState* pend,
                               int woff) {
  load_sym(a, p, A, lda);
  if (pend != nullptr) {
    const int nws = pend->nw;
    for (int idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
      const int i = idx / p, j = idx - i * p;
      const double di = (i >= woff && i < woff + nws) ? pend->dscale[i - woff] : 1.0;
      const double dj = (j >= woff && j < woff + nws) ? pend->dscale[j - woff] : 1.0;
      A[i * lda + j] *= di * dj;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_small_rr(const double* __restrict__ a, int p, int m,
                                                  int a0, int want_up, double tau,
                                                  const OrthoState* __restrict__ pend, int woff,
                                                  double* __restrict__ theta_all,
                                                  double* __restrict__ U, int* __restrict__ info,
                                                  int jacobi) {
  extern __shared__ double smem[];
  EigLds L = eig_lds(smem, p, m);
  const int ld = p + 1;
  __shared__ ShiftCount cnt;
  __shared__ int zeros;
  __shared__ int stalled, passes, grams, updates, tflag;
  if (threadIdx.x == 0) {
    cnt.factorizations = cnt.failed = cnt.shifted = cnt.svqb = 0;
    zeros = stalled = passes = grams = updates = 0;
  }
  const bool scaled = (pend != nullptr) && pend->pending_scale;
  double* Us = L.A;  // sorted eigenvectors u_x (first m columns), stride ld
  int sw = 0;
  const TriLayout T = tri_layout(p, m);
  bool tri = false;
  if (!jacobi && T.nb >= 1) {
    load_rr_matrix(a, p, L.A, ld, scaled ? pend : nullptr, woff);
    double* base = L.A + p * ld;
    tri = blk_tri_eigh(L.A, ld, p, m, base, T, &tflag);
    if (tri) {
      for (int j = threadIdx.x; j < m; j += blockDim.x) theta_all[j] = base[T.ev + j];
      // orientation: u[j][j] >= 0, so that u_x - E is the small update X_new - X_old
      for (int idx = threadIdx.x; idx < p * m; idx += blockDim.x) {
        const int i = idx / m, j = idx - i * m;
        const double sg = (base[T.Z + j * T.ldz + j] < 0.0) ? -1.0 : 1.0;
        Us[i * ld + j] = sg * base[T.Z + i * T.ldz + j];
      }
      __syncthreads();
    }
  }
  if (!tri) {
    load_rr_matrix(a, p, L.A, ld, scaled ? pend : nullptr, woff);
    sw = blk_jacobi(L.A, ld, L.V, ld, p, L.cs, L.pr, L.flags, L.scratch);
    blk_sort_evals(L.A, ld, p, L.perm);
    for (int j = threadIdx.x; j < m; j += blockDim.x) theta_all[j] = L.A[L.perm[j] * ld + L.perm[j]];
    __syncthreads();
    for (int idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
      const int i = idx / p, j = idx - i * p;
      const double sg = (L.V[j * ld + L.perm[j]] < 0.0) ? -1.0 : 1.0;
      Us[i * ld + j] = sg * L.V[i * ld + L.perm[j]];
    }
    __syncthreads();
  }
  const int na = want_up ? (m - a0) : 0;
  const int q = m + na;
  // u_x (row scaling for a pending W scaling is applied when U is written)
  for (int idx = threadIdx.x; idx < p * m; idx += blockDim.x) {
    const int i = idx / m, j = idx - i * m;
    const double di = (scaled && i >= woff && i < woff + pend->nw) ? pend->dscale[i - woff] : 1.0;
    U[i * q + j] = di * Us[i * ld + j];
  }
  int bad = 0;
  if (na > 0) {
    // V area becomes: X (p x na), C (m x na), M (na x na), Lc (na x na), Li, svqb workspace
    double* X = L.V;
    const int ldx = na;
    double* C = X + p * na;
    double* M = C + m * na;
    double* Lc = M + na * na;
    double* Ws = Lc + na * na;
    // u~_p = u_x[:, a0:m] - E[:, a0:m]
    for (int idx = threadIdx.x; idx < p * na; idx += blockDim.x) {
      const int i = idx / na, j = idx - i * na;
      X[i * ldx + j] = Us[i * ld + a0 + j] - ((i == a0 + j) ? 1.0 : 0.0);
    }
    __syncthreads();
    blk_normalize(X, ldx, p, na, L.cs, &zeros);
    blk_gemm_tn(Us, ld, X, ldx, p, m, na, C, na);  // C = u_x^T X
    for (int pass = 0; pass < 4; ++pass) {
      if (threadIdx.x == 0) passes++;
      blk_sub_mm(X, ldx, Us, ld, C, na, p, m, na);
      // ortho(X): normalise, then Gram / check / shifted Cholesky / X L^-T
      blk_normalize(X, ldx, p, na, L.cs, &zeros);
      for (int it = 0; it < 6; ++it) {
        blk_gemm_tn(X, ldx, X, ldx, p, na, na, M, na);
        if (threadIdx.x == 0) grams++;
        double dev = 0.0;
        for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
          const int i = idx / na, j = idx - i * na;
          const double v = 0.5 * (M[i * na + j] + M[j * na + i]) - (i == j ? 1.0 : 0.0);
          dev = fmax(dev, fabs(v));
        }
        dev = blk_reduce_max(dev, L.scratch);
        if (dev <= tau) break;
        if (it == 5) {
          if (threadIdx.x == 0) stalled++;
          break;
        }
        for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
          const int i = idx / na, j = idx - i * na;
          M[idx] = 0.5 * (M[i * na + j] + M[j * na + i]);
        }
        __syncthreads();
        // symmetrised copy is in place; compute Cholesky
        if (blk_shifted_chol(M, na, na, Lc, na, L.flags, &cnt, L.scratch)) {
          blk_trsm_rt(X, ldx, p, na, Lc, na);
        } else {
          if (threadIdx.x == 0) cnt.svqb++;
          if (!blk_svqb_coef(M, na, na, Lc, na, Ws, L.cs, L.pr, L.flags, L.perm, L.scratch)) {
            bad = 1;
            break;
          }
          // X <- X Cf (Cf in Lc), through the Ws area as a copy of X
          for (int idx = threadIdx.x; idx < p * na; idx += blockDim.x) Ws[idx] = X[idx];
          __syncthreads();
          for (int idx = threadIdx.x; idx < p * na; idx += blockDim.x) {
            const int r = idx / na, j = idx - r * na;
            double acc = 0.0;
            for (int k = 0; k < na; ++k) acc += Ws[r * na + k] * Lc[k * na + j];
            X[r * ldx + j] = acc;
          }
          __syncthreads();
        }
        if (threadIdx.x == 0) updates++;
      }
      if (bad) break;
      blk_gemm_tn(Us, ld, X, ldx, p, m, na, C, na);
      double cm = 0.0;
      for (int idx = threadIdx.x; idx < m * na; idx += blockDim.x) cm = fmax(cm, fabs(C[idx]));
      cm = blk_reduce_max(cm, L.scratch);
      if (cm <= tau) break;
      if (pass == 3 && threadIdx.x == 0) stalled++;
    }
    for (int idx = threadIdx.x; idx < p * na; idx += blockDim.x) {
      const int i = idx / na, j = idx - i * na;
      const double di = (scaled && i >= woff && i < woff + pend->nw) ? pend->dscale[i - woff] : 1.0;
      U[i * q + m + j] = di * X[i * ldx + j];
    }
  }
  if (threadIdx.x == 0) {
    info[0] = sw;
    info[1] = bad;
    info[2] = grams;
    info[3] = cnt.factorizations;
    info[4] = cnt.failed;
    info[5] = cnt.shifted;
    info[6] = updates;
    info[7] = passes;
    info[8] = stalled;
    info[9] = cnt.svqb;
    info[10] = zeros;
    info[11] = (tri || jacobi) ? 0 : 1;  // Jacobi fallback of the eigensolve
  }
}

hipError_t small_rr(const double* a, int p, int m, int a0, int want_up, double tau,
                    const OrthoState* pend, int woff, double* theta_all, double* U, int* info,
                    int jacobi, hipStream_t s) {
  if (p < 1 || p > kMaxP || m < 1 || m > p || a0 < 0 || a0 > m) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    // dynamic + static LDS must stay within the 160 KB of a workgroup
    (void)hipFuncSetAttribute((const void*)k_small_rr, hipFuncAttributeMaxDynamicSharedMemorySize,
                              152 * 1024);
    (void)hipGetLastError();
    attr = true;
  }
  hipLaunchKernelGGL(k_small_rr, dim3(1), dim3(1024), kEigLdsBytes, s, a, p, m, a0, want_up, tau,
                     pend, woff, theta_all, U, info, jacobi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// standalone shifted Cholesky (p <= 64)

__global__ __launch_bounds__(256) void k_small_chol(const double* __restrict__ M, int p,
                                                    double* __restrict__ Lout, int* info) {
  __shared__ double Ms[64 * 65];
  __shared__ double Ls[64 * 65];
  __shared__ double scratch[16];
  __shared__ int flag;
  __shared__ ShiftCount cnt;
  if (threadIdx.x == 0) cnt.factorizations = cnt.failed = cnt.shifted = cnt.svqb = 0;
  for (int idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
    const int i = idx / p, j = idx - i * p;
    Ms[i * 65 + j] = 0.5 * (M[i * p + j] + M[j * p + i]);
  }
  __syncthreads();
  const bool ok = blk_shifted_chol<0>(Ms, 65, p, Ls, 65, &flag, &cnt, scratch);
  for (int idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
    const int i = idx / p, j = idx - i * p;
    Lout[idx] = ok ? Ls[i * 65 + j] : 0.0;
  }
  if (threadIdx.x == 0) {
    info[0] = ok ? 0 : 1;
    info[1] = cnt.factorizations;
    info[2] = cnt.failed;
    info[3] = cnt.shifted;
  }
}

hipError_t small_cholesky(const double* M, int p, double* L, int* info, hipStream_t s) {
  if (p < 1 || p > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_small_chol, dim3(1), dim3(256), 0, s, M, p, L, info);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ortho(W; Y) controller.  G = [Y W]^T W, (ny + nw) x nw: rows [0, ny) are
// C = Y^T W, rows [ny, ny+nw) are M = W^T W.  The coefficient written to
// `coef` ((ny+nw) x nw) is applied by the streaming kernel as
// W <- [Y W] coef, after which G is recomputed and this kernel runs again.
//
// Phases (reading of Alg. 3 as a do-while around Alg. 2, both with column
// normalisation first):
//   START  raw W~: normalise (D0) and project: coef = [-C D0; D0]
//          (no Y: behave as BEGIN)
//   BEGIN  start of ortho(X): D = diag(M)^-1/2, M' = D M D;
//          ||M' - I|| <= tau -> ortho done on X = W D: Alg. 3 check on C D;
//          else shifted Cholesky M' = L L^T, coef = [0; D L^-T] -> LOOP
//   LOOP   ||M - I|| <= tau (or pass cap) -> Alg. 3 check on C;
//          else shifted Cholesky, coef = [0; L^-T]
//   Alg. 3 check: ||C|| <= tau (or no Y) -> finished; else project
//          coef = [-C; I] (scaled by the pending D) -> BEGIN
//   FINAL  a pending diagonal scaling was applied: finished.

enum { kPhFinal = 5, kPhYCheck = 6 };

// Bound on ||L^-1||_2 for the n x n lower factor L (stride ldl) with its
// inverse Li (stride ldi): 1 / (1 - e) when e = ||I - L||_F < 1/2 (Neumann
// series), else ||Li||_F.  *e_out receives e.  Every thread gets the result.
__device__ double blk_inv_bound(const double* L, int ldl, const double* Li, int ldi, int n,
                                double* e_out, double* scratch) {
  double se = 0.0, si = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx - i * n;
    if (j > i) continue;
    const double d = (i == j ? 1.0 : 0.0) - L[i * ldl + j];
    se += d * d;
    const double v = Li[i * ldi + j];
    si += v * v;
  }
  se = blk_reduce_sum_ordered(se, scratch);
  si = blk_reduce_sum_ordered(si, scratch);
  const double e = sqrt(se);
  *e_out = e;
  return (e < 0.5) ? 1.0 / (1.0 - e) : sqrt(si);
}

__global__ __launch_bounds__(1024) void k_ortho_ctl(const double* __restrict__ G,
                                                   OrthoState* __restrict__ gst,
                                                   double* __restrict__ coef) {
  __shared__ OrthoState st;
  __shared__ double Gs[kMaxP * kMaxBlock];
  __shared__ double Ms[kMaxBlock * (kMaxBlock + 1)];
  __shared__ double Ls[kMaxBlock * (kMaxBlock + 1)];
  __shared__ double Li[kMaxBlock * (kMaxBlock + 1)];
  __shared__ double Ws[2 * kMaxBlock * (kMaxBlock + 1)];
  __shared__ double D[kMaxBlock];
  __shared__ double cs[3 * 64];
  __shared__ int pr[2 * 64];
  __shared__ int perm[64];
  __shared__ double scratch[16];
  __shared__ int flag, nonfinite, zero_mask;
  __shared__ ShiftCount cnt;
  if (threadIdx.x == 0) {
    st = *gst;
    nonfinite = 0;
    zero_mask = 0;
    cnt.factorizations = cnt.failed = cnt.shifted = cnt.svqb = 0;
  }
  __syncthreads();
  if (st.done) return;
  const int ny = st.ny, nw = st.nw, nr = ny + nw;
  const int ldm = kMaxBlock + 1;
  for (int idx = threadIdx.x; idx < nr * nw; idx += blockDim.x) {
    const double v = G[idx];
    Gs[idx] = v;
    if (!isfinite(v)) nonfinite = 1;
  }
  __syncthreads();
  if (st.state == kPhFinal) {
    if (threadIdx.x == 0) {
      st.done = 1;
      st.skip_sum = 1;
      st.state = kPhDone;
      *gst = st;
    }
    return;
  }
  if (threadIdx.x == 0) st.grams++;  // (a no-overlap apply only precedes kPhFinal)
  if (nonfinite) {
    if (threadIdx.x == 0) {
      st.error = kOrthoErrNonfinite;
      st.done = 1;
      st.skip_sum = 1;
      *gst = st;
    }
    return;
  }
  // symmetrised M
  for (int idx = threadIdx.x; idx < nw * nw; idx += blockDim.x) {
    const int i = idx / nw, j = idx - i * nw;
    Ms[i * ldm + j] = 0.5 * (Gs[(ny + i) * nw + j] + Gs[(ny + j) * nw + i]);
  }
  __syncthreads();
  int phase = st.state;
  if (phase == kPhStart && ny == 0) phase = kPhBegin;

  // helper lambdas are avoided: explicit code per phase
  bool check_outer = false;
  bool have_scale = false;  // D pending (BEGIN passed its check)
  bool capped = false;
  double growth = st.growth;  // amplification of errors by the current Alg. 2 call
  if (phase == kPhStart || phase == kPhBegin) {
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
      const double d = Ms[j * ldm + j];
      if (d == 0.0) atomicOr(&zero_mask, 1 << j);
      D[j] = (d > 0.0) ? 1.0 / sqrt(d) : 0.0;
    }
    __syncthreads();
    if (zero_mask) {
      if (threadIdx.x == 0) {
        st.error = kOrthoErrZero;
        st.zero_mask = zero_mask;
        st.done = 1;
        st.skip_sum = 1;
        *gst = st;
      }
      return;
    }
  }
  if (phase == kPhStart) {
    // normalise + first projection (Alg. 3, first pass)
    for (int idx = threadIdx.x; idx < nr * nw; idx += blockDim.x) {
      const int i = idx / nw, j = idx - i * nw;
      coef[idx] = (i < ny) ? -Gs[i * nw + j] * D[j] : ((i - ny == j) ? D[j] : 0.0);
    }
    if (threadIdx.x == 0) {
      st.passes++;
      st.outer = 1;
      st.w_only = 0;
      st.no_gram = 0;
      st.skip_sum = 0;
      st.state = kPhBegin;
      *gst = st;
    }
    return;
  }
  if (phase == kPhBegin) {
    // M' = D M D, Alg. 2 check on the normalised X; the normalisation is
    // the first factor of this Alg. 2 call's growth
    double dmax = 0.0;
    for (int j = threadIdx.x; j < nw; j += blockDim.x) dmax = fmax(dmax, D[j]);
    growth = blk_reduce_max(dmax, scratch);
    for (int idx = threadIdx.x; idx < nw * nw; idx += blockDim.x) {
      const int i = idx / nw, j = idx - i * nw;
      Ms[i * ldm + j] *= D[i] * D[j];
    }
    if (threadIdx.x == 0) st.inner = 1;
    __syncthreads();
  } else if (phase == kPhLoop || phase == kPhYCheck) {
    if (threadIdx.x == 0 && phase == kPhLoop) st.inner++;
    for (int j = threadIdx.x; j < nw; j += blockDim.x) D[j] = 1.0;
    __syncthreads();
  }
  if (phase == kPhYCheck) {
    // a cheap exit ended Alg. 2 with the last update; only the Alg. 3
    // check of Y^T W (in the overlap that update formed) remains
    check_outer = true;
  } else {
  double dev = 0.0;
  for (int idx = threadIdx.x; idx < nw * nw; idx += blockDim.x) {
    const int i = idx / nw, j = idx - i * nw;
    dev = fmax(dev, fabs(Ms[i * ldm + j] - (i == j ? 1.0 : 0.0)));
  }
  dev = blk_reduce_max(dev, scratch);
  const bool ortho_ok = dev <= st.tau;
  capped = !ortho_ok && st.inner >= st.max_inner;
  if (ortho_ok || capped) {
    if (capped && threadIdx.x == 0) st.stalled++;
    check_outer = true;
    have_scale = (phase == kPhBegin);
  } else {
    // shifted Cholesky of M (= M' in BEGIN)
    const bool ok = blk_shifted_chol<2>(Ms, ldm, nw, Ls, ldm, &flag, &cnt, scratch, st.shift_retries);
    if (ok) {
      blk_tri_inv(Ls, ldm, nw, Li, ldm);
      // coef W part: D L^-T, i.e. coef[ny+i][j] = D_i Linv[j][i]
      for (int idx = threadIdx.x; idx < nr * nw; idx += blockDim.x) {
        const int i = idx / nw, j = idx - i * nw;
        coef[idx] = (i < ny) ? 0.0 : D[i - ny] * Li[j * ldm + (i - ny)];
      }
      // cheap exits: e = ||I - L||_F bounds kappa(L) <= (1 + e) / (1 - e)
      // and ||L^-1||; when the pass provably reached tau the overlap of the
      // new W is not formed (Alg. 2), and when the growth of the whole
      // Alg. 2 call also keeps Y^T W below tau, neither is Y^T W (Alg. 3)
      double e = 1.0;
      const double b = blk_inv_bound(Ls, ldm, Li, ldm, nw, &e, scratch);
      growth *= b;
      const double kap = (1.0 + e) / (1.0 - e);
      const bool exit2 = st.cheap_exit && cnt.shifted == 0 && e < 0.5 &&
                         st.cexit * kap * kap <= st.tau;
      const bool exit3 = exit2 && (ny == 0 || st.cexit * growth <= st.tau);
      if (threadIdx.x == 0) {
        st.factorizations += cnt.factorizations;
        st.failed += cnt.failed;
        st.shifted += cnt.shifted;
        st.svqb += cnt.svqb;
        st.updates++;
        st.w_only = 1;
        st.growth = growth;
        if (exit2) st.cheap_exits += (exit3 && ny > 0) ? 2 : 1;
        st.no_gram = exit3 ? 1 : 0;
        st.skip_sum = st.no_gram;
        st.state = exit3 ? kPhFinal : (exit2 ? kPhYCheck : kPhLoop);
        *gst = st;
      }
      return;
    } else {
      if (threadIdx.x == 0) cnt.svqb++;
      const bool sv = blk_svqb_coef(Ms, ldm, nw, Li, ldm, Ws, cs, pr, &flag, perm, scratch);
      if (!sv) {
        if (threadIdx.x == 0) {
          st.error = kOrthoErrFailed;
          st.done = 1;
          st.skip_sum = 1;
          st.factorizations += cnt.factorizations;
          st.failed += cnt.failed;
          *gst = st;
        }
        return;
      }
      for (int idx = threadIdx.x; idx < nr * nw; idx += blockDim.x) {
        const int i = idx / nw, j = idx - i * nw;
        coef[idx] = (i < ny) ? 0.0 : D[i - ny] * Li[(i - ny) * ldm + j];
      }
    }
    if (threadIdx.x == 0) {
      st.factorizations += cnt.factorizations;
      st.failed += cnt.failed;
      st.shifted += cnt.shifted;
      st.svqb += cnt.svqb;
      st.updates++;
      st.w_only = 1;
      st.growth = INFINITY;  // SVQB: no growth bound, no cheap exit
      st.no_gram = 0;
      st.skip_sum = 0;
      st.state = kPhLoop;
      *gst = st;
    }
    return;
  }
  }
  // Alg. 3: the growth of the finished Alg. 2 call may already bound Y^T W
  // below tau (cheap exit); else check C D (D = 1 unless BEGIN's
  // normalisation is pending)
  const bool grow_ok = st.cheap_exit && ny > 0 && !capped && phase != kPhYCheck &&
                       st.cexit * growth <= st.tau;
  double cm = 0.0;
  for (int idx = threadIdx.x; idx < ny * nw; idx += blockDim.x) {
    const int j = idx % nw;
    cm = fmax(cm, fabs(Gs[idx] * D[j]));
  }
  cm = blk_reduce_max(cm, scratch);
  if (grow_ok && threadIdx.x == 0) st.cheap_exits++;
  const bool y_ok = (ny == 0) || grow_ok || (cm <= st.tau);
  if (y_ok || st.outer >= st.max_outer) {
    if (!y_ok && threadIdx.x == 0) st.stalled++;
    if (have_scale && st.fold_scale) {
      // leave the normalisation pending: the caller folds it into the next
      // Rayleigh-Ritz coefficients instead of spending a pass on it
      if (threadIdx.x == 0) {
        for (int j = 0; j < nw; ++j) st.dscale[j] = D[j];
        st.pending_scale = 1;
        st.done = 1;
        st.skip_sum = 1;
        st.state = kPhDone;
        *gst = st;
      }
    } else if (have_scale) {
      // apply the pending normalisation, then finish
      for (int idx = threadIdx.x; idx < nr * nw; idx += blockDim.x) {
        const int i = idx / nw, j = idx - i * nw;
        coef[idx] = (i < ny) ? 0.0 : ((i - ny == j) ? D[j] : 0.0);
      }
      if (threadIdx.x == 0) {
        st.w_only = 1;
        st.no_gram = 1;  // the next round only finishes
        st.skip_sum = 1;
        st.state = kPhFinal;
        *gst = st;
      }
    } else if (threadIdx.x == 0) {
      st.done = 1;
      st.skip_sum = 1;
      st.state = kPhDone;
      *gst = st;
    }
    return;
  }
  // project again: W <- W D - Y (C D)
  for (int idx = threadIdx.x; idx < nr * nw; idx += blockDim.x) {
    const int i = idx / nw, j = idx - i * nw;
    coef[idx] = (i < ny) ? -Gs[i * nw + j] * D[j] : ((i - ny == j) ? D[j] : 0.0);
  }
  if (threadIdx.x == 0) {
    st.passes++;
    st.outer++;
    st.w_only = 0;
    st.no_gram = 0;
    st.skip_sum = 0;
    st.state = kPhBegin;
    *gst = st;
  }
}

__global__ void k_ortho_init(OrthoState* st, int ny, int nw, double tau, int max_inner,
                             int max_outer, int shift_retries, int fold_scale, double cexit) {
  OrthoState s;
  s.state = kPhStart;
  s.done = 0;
  s.inner = 0;
  s.outer = 0;
  s.w_only = 0;
  s.error = 0;
  s.zero_mask = 0;
  s.grams = s.factorizations = s.failed = s.shifted = s.updates = s.stalled = s.svqb = s.passes = 0;
  s.ny = ny;
  s.nw = nw;
  s.max_inner = max_inner;
  s.max_outer = max_outer;
  s.shift_retries = shift_retries;
  s.fold_scale = fold_scale;
  s.pending_scale = 0;
  s.cheap_exit = cexit > 0.0 ? 1 : 0;
  s.cheap_exits = 0;
  s.no_gram = 0;
  s.skip_sum = 0;
  s.cexit = cexit;
  s.growth = INFINITY;
  s.tau = tau;
  for (int j = 0; j < kMaxBlock; ++j) s.dscale[j] = 1.0;
  *st = s;
}

hipError_t ortho_init(OrthoState* st, int ny, int nw, double tau, int max_inner, int max_outer,
                      int shift_retries, int fold_scale, double cexit, hipStream_t s) {
  if (nw < 1 || nw > kMaxBlock || ny < 0 || ny + nw > kMaxP || shift_retries < 0)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ortho_init, dim3(1), dim3(1), 0, s, st, ny, nw, tau, max_inner, max_outer,
                     shift_retries, fold_scale, cexit);
  return hipGetLastError();
}

hipError_t ortho_ctl(const double* G, OrthoState* st, double* coef, hipStream_t s) {
  // 1024 threads: the SVQB fallback runs the Jacobi sweep, which assumes them
  hipLaunchKernelGGL(k_ortho_ctl, dim3(1), dim3(1024), 0, s, G, st, coef);
  return hipGetLastError();
}

}  // namespace lobpcg
