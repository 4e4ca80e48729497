// Internal declarations shared by the kernels and the host driver.
// Layout conventions: blocks of vectors are row-major (entry (i, j) of an
// n x c block with leading dimension ld is at ptr[i * ld + j]); small
// matrices are dense row-major.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>

namespace lobpcg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kMaxBlock = 32;            // RR block m
constexpr int kMaxP = 3 * kMaxBlock;     // RR subspace m + 2 m_act
constexpr int kGramMaxCols = 128;        // p, q limit of the Gram kernel
constexpr int kGramBlocks = 512;         // stage-1 workgroups of the Gram (768, 3 per CU, ran 4-8 % slower)
constexpr int kStreamBlocks = 1024;      // persistent grid of streaming kernels
constexpr double kPrecondGuard = 1e-8;   // |d - theta| floor, relative to max(1, |theta|)
constexpr uint64_t kZeroColumnSeed = 0x2305066680000000ull;
constexpr uint64_t kDefaultX0Seed = 0x2305066600000001ull;

enum PrecondKind { kPrecNone = 0, kPrecDiag = 1, kPrecDiagSigned = 2, kPrecLearned = 3, kPrecTridiag = 4 };

// learned preconditioner: per-entry MLP 3 -> 128 -> 128 -> 1
constexpr int kMlpHidden = 128;
constexpr int kMlpFeat = 3;
constexpr int kMlpParams = kMlpHidden * kMlpFeat + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpHidden + 1;
constexpr int kMlpBlocks = 256;  // persistent grid of the MLP kernels
constexpr int kMlpSuper = 256;   // entries per screened super tile of the bf16 transform
constexpr double kMlpWindow = 16.0;  // the net acts where |d - theta| <= kMlpWindow * rho

// Device-side state of one ortho(W; Y) call (Alg. 2 nested in Alg. 3).
// Written only by the one-workgroup controller kernel; the streaming kernels
// read `done` and return at once when it is set.
struct OrthoState {
  int state;    // OrthoPhase
  int done;     // 1: nothing left to apply
  int inner;    // overlap evaluations in the current Alg. 2 loop
  int outer;    // Alg. 3 passes
  int w_only;   // the pending coefficient has no Y part
  int error;    // 0, kOrthoErrZero (zero column met), kOrthoErrNonfinite, kOrthoErrFailed
  int zero_mask;  // bit j: column j of W was exactly zero
  int grams, factorizations, failed, shifted, updates, stalled, svqb, passes;
  int ny, nw;   // current shape
  int max_inner, max_outer;
  int shift_retries;  // shifted Cholesky attempts after a failed plain one, then SVQB
  int fold_scale;     // input: a final diagonal column scaling may be left pending
  int pending_scale;  // output: W must still be scaled by dscale (folded into the next RR)
  // cheap exits (Sec. 3.2's estimates after Alg. 2 and Alg. 3): when set,
  // a factor whose conditioning bound shows the pass already reached tau
  // skips the overlap that would only confirm it
  int cheap_exit;     // input: 0/1
  int cheap_exits;    // overlaps skipped
  int no_gram;        // the pending apply need not form the overlap
  int skip_sum;       // done || no_gram: the overlap's second stage skips itself
  double cexit;       // input: c(n) * unit roundoff of the block precision
  double growth;      // amplification of errors by the current Alg. 2 call
  double tau;
  double dscale[kMaxBlock];
};
enum OrthoPhase { kPhStart = 0, kPhBegin = 1, kPhLoop = 2, kPhOuter = 3, kPhDone = 4 };
enum { kOrthoErrZero = 1, kOrthoErrNonfinite = 2, kOrthoErrFailed = 3 };

// ---- streaming kernels (k_blas.hip) -------------------------------------
// Copies nwords 32-bit words from src (device) to dst (coherent host memory
// mapped for the device), makes them visible to the host, then stores seq
// to *flag (same memory).  One workgroup; nwords <= 1024.
hipError_t post_status(const void* src, int nwords, uint32_t* dst, uint32_t* flag, uint32_t seq,
                       hipStream_t s);
// C (p x q) = A^T B over n rows, fp64 result; `part` needs kGramBlocks*p*q.
hipError_t gram_f64(const double* A, int64_t lda, int p, const double* B, int64_t ldb, int q,
                    int64_t n, double* part, double* C, const int* skip, hipStream_t s);
hipError_t gram_f32(const float* A, int64_t lda, int p, const float* B, int64_t ldb, int q,
                    int64_t n, double* part, double* C, const int* skip, hipStream_t s);

// Out (n x q) = In (n x p) Coef (p x q); Out may alias columns of In when
// every row of Out lies inside the same row of In.  skip: optional flag.
hipError_t tsmm_f64(const double* In, int64_t ldi, int p, const double* Coef, int q, double* Out,
                    int64_t ldo, int64_t n, const int* skip, hipStream_t s);
hipError_t tsmm_f32(const float* In, int64_t ldi, int p, const double* Coef, int q, float* Out,
                    int64_t ldo, int64_t n, const int* skip, hipStream_t s);

// One pass of ortho(W; Y) on base = [Y | W]: W <- [Y W] coef in place and
// G = [Y W]^T W of the new W (skipped when st->done).
hipError_t ortho_apply_f64(double* base, int64_t ld, int ny, int nw, const double* coef,
                           const OrthoState* st, int64_t n, double* part, double* G,
                           hipStream_t s);
hipError_t ortho_apply_f32(float* base, int64_t ld, int ny, int nw, const double* coef,
                           const OrthoState* st, int64_t n, double* part, double* G,
                           hipStream_t s);

// Rotation + residual + preconditioner (one pass over V and AV).
struct RotateArgs {
  int64_t n, ldv, ldo;
  int p, m, q, a0, precond;
  const double* U;      // p x q
  const double* theta;  // m
  const double* diag;   // n (may be null for kPrecNone)
  double* part;         // kStreamBlocks * m partial norms
  double* resnorm2;     // m
};
hipError_t rotate_f64(const double* V, const double* AV, double* Vout, double* AVout,
                      const RotateArgs& a, hipStream_t s);
hipError_t rotate_f32(const float* V, const float* AV, float* Vout, float* AVout,
                      const RotateArgs& a, hipStream_t s);

// Column statistics for the true residual: out[0:m] = x^T x, out[m:2m] =
// x^T (Ax), out[2m:3m] = ||Ax - theta x||^2.
hipError_t colstats_f64(const double* X, int64_t ldx, const double* AX, int64_t ldax, int m,
                        const double* theta, int64_t n, double* part, double* out, hipStream_t s);

// Fill column `col` of an n x * block with SplitMix64 uniforms in [-0.5, 0.5):
// entry i = (splitmix64(seed + col_id * n + i) >> 11) * 2^-53 - 0.5.
hipError_t fill_splitmix(double* X, int64_t ld, int col, int col_id, int64_t n, uint64_t seed,
                         hipStream_t s);

hipError_t fill_splitmix_f32(float* X, int64_t ld, int col, int col_id, int64_t n, uint64_t seed,
                             hipStream_t s);

// Copy the first k columns of X to out (ld_out) with each column's sign set so
// its largest-magnitude entry (lowest index on ties) is positive.
hipError_t copy_signfix(const double* X, int64_t ldx, int k, int64_t n, double* out,
                        int64_t ldout, int64_t* part_idx, double* part_val, hipStream_t s);

// Precision conversions of an n x c block.
hipError_t convert_f64_to_f32(const double* in, int64_t ldi, float* out, int64_t ldo, int c,
                              int64_t n, hipStream_t s);
hipError_t convert_f32_to_f64(const float* in, int64_t ldi, double* out, int64_t ldo, int c,
                              int64_t n, hipStream_t s);
hipError_t convert_vec_f64_to_f32(const double* in, float* out, int64_t len, hipStream_t s);

// ---- operators (k_op.hip) -----------------------------------------------
// kSlabBlockRows-row blocks of the banded CSR path (win: one int2 per block,
// from csr_windows; nullptr selects the gather kernels)
constexpr int kSlabBlockRows = 2048;
constexpr int kSlabThreads = 1024;
constexpr int kSlabUnits = kSlabBlockRows * 4 / kSlabThreads;  // rows per thread
constexpr int kSlabLds = 128 * 1024;                            // bytes of W per slab
hipError_t spmm_csr_f64(const int32_t* rp, const int32_t* ci, const double* val, const double* W,
                        int64_t ldw, double* Y, int64_t ldy, int ncols, int64_t n, const int2* win,
                        hipStream_t s);
hipError_t spmm_csr_f32(const int32_t* rp, const int32_t* ci, const float* val, const float* W,
                        int64_t ldw, float* Y, int64_t ldy, int ncols, int64_t n, const int2* win,
                        hipStream_t s);
hipError_t csr_windows(const int32_t* rp, const int32_t* ci, int64_t n, int2* win, int* unsorted,
                       hipStream_t s);
// pack (optional, n x 8 values): scratch for a compact copy of W when W is
// not a compact 8-column block
hipError_t dense_apply_f64(const double* A, int64_t lda, const double* W, int64_t ldw, double* Y,
                           int64_t ldy, int ncols, int64_t n, double* pack, hipStream_t s);
hipError_t dense_apply_f32(const float* A, int64_t lda, const float* W, int64_t ldw, float* Y,
                           int64_t ldy, int ncols, int64_t n, float* pack, hipStream_t s);
// out (n x 8) = columns [0, nc) of W (n rows, leading dimension ldw), zero
// padded to 8: the operators' compact copy of a strided or partial block
hipError_t pack8_f64(const double* W, int64_t ldw, int nc, int64_t n, double* out, hipStream_t s);
hipError_t pack8_f32(const float* W, int64_t ldw, int nc, int64_t n, float* out, hipStream_t s);
// pack (optional, na^2 x 8 values): scratch for a compact copy of W when W
// is not a compact 8-column block
hipError_t kronsum_apply_f64(const double* A, const double* Vp, int64_t na, const double* W,
                             int64_t ldw, double* Y, int64_t ldy, int ncols, double* pack,
                             hipStream_t s);
hipError_t kronsum_apply_f32(const float* A, const float* Vp, int64_t na, const float* W,
                             int64_t ldw, float* Y, int64_t ldy, int ncols, float* pack,
                             hipStream_t s);
// Sets bits of *bad (device int, zeroed by the caller) on a malformed CSR.
hipError_t csr_check(const int32_t* rp, const int32_t* ci, int64_t n, int64_t nnz, int* bad,
                     hipStream_t s);
hipError_t csr_diag(const int32_t* rp, const int32_t* ci, const double* val, int64_t n,
                    double* diag, hipStream_t s);
hipError_t dense_diag(const double* A, int64_t lda, int64_t n, double* diag, hipStream_t s);
hipError_t kronsum_diag(const double* A, const double* Vp, int64_t na, double* diag,
                        hipStream_t s);
// Gershgorin bound max_i sum_j |a_ij| of the operator (device result in *out,
// via `part` partials of kStreamBlocks doubles).
hipError_t csr_norm_bound(const int32_t* rp, const double* val, int64_t n, double* part,
                          double* out, hipStream_t s);
hipError_t dense_norm_bound(const double* A, int64_t lda, int64_t n, double* part, double* out,
                            hipStream_t s);

// ---- lobpcg_gram_noalloc (noalloc.hip) -----------------------------------
// Looks up (once per device, with that device current) the device address of
// the static partial-sum array of lobpcg_gram_noalloc; *out receives it.
// Returns a LOBPCG_* status; *err gets a message on failure.
int noalloc_setup(int device, double** out, std::string* err);

// ---- generalized problem (k_gen.hip) -------------------------------------
// resn2[j] = ||A X - B X theta||^2 per column (AX, BX: n x m, ld); columns
// j >= a0 of R, preconditioned (0 none, 1 |dA - theta dB|, 2 signed, with
// the Jacobi guard), go to Wout[:, j - a0] (ldw).  part: 1024 m doubles.
hipError_t gen_residual(const double* AX, const double* BX, int64_t ld, int m, const double* theta,
                        int a0, int precond, const double* dA, const double* dB, double* Wout,
                        int64_t ldw, int64_t n, double* part, double* resn2, hipStream_t s);
// out[0:m] = x^T B x, out[m:2m] = x^T A x, out[2m:3m] = ||A x - theta B x||^2
// (X: ldx; AX, BX: ldm).  part: 3072 m doubles.
hipError_t gen_colstats(const double* X, int64_t ldx, const double* AX, const double* BX, int64_t ldm,
                        int m, const double* theta, int64_t n, double* part, double* out,
                        hipStream_t s);
// coef = [-C; I] ((ny + nw) x nw) and *cmax = max |C| (C: ny x nw)
hipError_t gen_proj_coef(const double* C, int ny, int nw, double* coef, double* cmax, hipStream_t s);
// out = L^-T (p x p, p <= kMaxBlock)
hipError_t gen_lt_inv(const double* L, int p, double* out, hipStream_t s);
// *out = max |x_i| (part: 1024 doubles; out must not lie in part)
hipError_t vec_max_abs(const double* x, int64_t len, double* part, double* out, hipStream_t s);

// ---- tridiagonal preconditioner (k_tri.hip) ------------------------------
constexpr int kTriMaxChunks = 1024;
// Chunks of the partition method for order n (balanced, >= 64 rows each).
int tri_chunks(int64_t n);
// In place: R[:, 0:nact] (ld) <- T_j^-1 R[:, j], T_j = tridiag(e, t, e) with
// t_i = max(|d_i - theta_j|, off_i + delta_j).  e: n values (e[n-1] = 0),
// off_i = |e_{i-1}| + |e_i|; bnd: 6 kTriMaxChunks nact doubles, xb: 2
// kTriMaxChunks nact doubles; scr: n nact doubles.
hipError_t tri_apply_f64(double* R, int64_t ld, int nact, int64_t n, const double* theta,
                         const double* d, const double* e, const double* off, double* bnd,
                         double* xb, double* scr, hipStream_t s);
hipError_t tri_apply_f32(float* R, int64_t ld, int nact, int64_t n, const double* theta,
                         const double* d, const double* e, const double* off, double* bnd,
                         double* xb, double* scr, hipStream_t s);
hipError_t tri_offdiag_csr(const int32_t* rp, const int32_t* ci, const double* val, int64_t n,
                           double* e, double* off, hipStream_t s);
hipError_t tri_offdiag_dense(const double* A, int64_t lda, int64_t n, double* e, double* off,
                             hipStream_t s);
hipError_t tri_offdiag_kron(const double* A, int64_t na, double* e, double* off, hipStream_t s);

// ---- small dense fp64 kernels (k_small.hip) -----------------------------
// Eigen-decomposition of sym(a) (p x p): evals ascending, evecs p x p.
hipError_t small_eigh(const double* a, int p, double* evals, double* evecs, int* sweeps,
                      hipStream_t s);
// Rayleigh-Ritz coefficients: eig of sym(a) (p x p); theta = lowest m
// values; U (p x q) = [u_x | u_p] where u_p = ortho(u_x[:, a0:m] - E[:, a0:m]; u_x)
// (q = m + (want_up ? m - a0 : 0)).  info[0] = Jacobi sweeps, info[1] = 0 ok,
// info[2..] ortho counters for the R^p orthonormalisation.
// `pend` (may be null): when pend->pending_scale is set, the columns
// [woff, woff + pend->nw) of V are taken as scaled by pend->dscale: a is
// scaled as D a D and the rows of U as D U, so the scaling never needs its
// own pass over V.
hipError_t small_rr(const double* a, int p, int m, int a0, int want_up, double tau,
                    const OrthoState* pend, int woff, double* theta_all, double* U, int* info,
                    int jacobi, hipStream_t s);
// Shifted Cholesky (p x p, p <= 64): L lower with L L^T = M + sigma I.
hipError_t small_cholesky(const double* M, int p, double* L, int* info, hipStream_t s);
// One controller step of ortho(W; Y): reads G = [Y W]^T W ((ny+nw) x nw),
// updates the state and writes the next coefficient ((ny+nw) x nw).
hipError_t ortho_ctl(const double* G, OrthoState* st, double* coef, hipStream_t s);
// cexit > 0 turns the cheap exits on (cexit = c(n) times the unit roundoff
// of the blocks' precision).
hipError_t ortho_init(OrthoState* st, int ny, int nw, double tau, int max_inner, int max_outer,
                      int shift_retries, int fold_scale, double cexit, hipStream_t s);

// ---- learned preconditioner (k_mlp.hip) ---------------------------------
// In place: R[:, 0:nact] (n rows, leading dimension ld) <- learned
// preconditioned columns for Ritz values theta[0:nact]; diag, rho (off-
// diagonal absolute row sums) and *s (mean |diag|) describe the operator;
// w holds kMlpParams fp32 weights; mask[j] != 0 (optional, device) or bit j
// of mbits selects the Jacobi step for column j; flags[j] (optional) is set
// to 1 where a net output was not finite (that entry then takes the Jacobi
// step).  The bf16 form clears flags[0 .. nact) itself; the fp32 form
// expects them cleared.
hipError_t mlp_apply_f64(double* R, int64_t ld, int nact, int64_t n, const double* theta,
                         const double* diag, const double* rho, const double* s, const float* w,
                         const int* mask, uint64_t mbits, int* flags, hipStream_t st);
hipError_t mlp_apply_f32(float* R, int64_t ld, int nact, int64_t n, const double* theta,
                         const double* diag, const double* rho, const double* s, const float* w,
                         const int* mask, uint64_t mbits, int* flags, hipStream_t st);
// The same transform with layer 2 on bf16 MFMA (fp32 accumulate): the
// solver's inference path.
// tflags: device scratch of tiles_cap >= ceil(n nact / kMlpSuper) ints,
// one flag per super tile of kMlpSuper entries (written by the screening
// pass, read by the MFMA pass)
hipError_t mlp_apply_bf16_f64(double* R, int64_t ld, int nact, int64_t n, const double* theta,
                              const double* diag, const double* rho, const double* s,
                              const float* w, const int* mask, uint64_t mbits, int* flags,
                              int* tflags, int64_t tiles_cap, hipStream_t st);
hipError_t mlp_apply_bf16_f32(float* R, int64_t ld, int nact, int64_t n, const double* theta,
                              const double* diag, const double* rho, const double* s,
                              const float* w, const int* mask, uint64_t mbits, int* flags,
                              int* tflags, int64_t tiles_cap, hipStream_t st);
// grad (kMlpParams doubles) = d/dweights of sum_e G_e w_e(weights), with w
// the learned columns of R; part needs kMlpBlocks * kMlpParams doubles.
hipError_t mlp_grad(const double* R, const double* G, int64_t ld, int nact, int64_t n,
                    const double* theta, const double* diag, const double* rho, const double* s,
                    const float* w, double* part, double* grad, hipStream_t st);
// One Adam step (step count t >= 1) on the fp32 weights.
hipError_t mlp_adam(float* w, float* m, float* v, const double* g, int t, double lr,
                    hipStream_t st);
hipError_t offdiag_abs_csr(const int32_t* rp, const int32_t* ci, const double* val, int64_t n,
                           double* rho, hipStream_t st);
hipError_t offdiag_abs_dense(const double* A, int64_t lda, int64_t n, double* rho,
                             hipStream_t st);
hipError_t offdiag_abs_kron(const double* A, int64_t na, double* ra_tmp, double* rho,
                            hipStream_t st);
// *out = mean |d| (part: 1024 doubles)
hipError_t abs_mean(const double* d, int64_t n, double* part, double* out, hipStream_t st);

}  // namespace lobpcg
