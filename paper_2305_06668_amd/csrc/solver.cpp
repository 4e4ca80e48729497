// Host driver of the block LOBPCG (Alg. 1 of arXiv:2305.06668) and the C ABI
// declared in include/lobpcg.h.
//
// Per iteration the host launches, on one stream:
//   Gram a = V^T AV -> small RR kernel (Jacobi eig + u_p) -> rotate (X, AX,
//   P, AP, R, W~ in one pass) -> [read back the m residual norms: the one
//   per-iteration host sync] -> ortho(W~; [X P]) as rounds of
//   (controller, block update, Gram) driven by device-side state -> the
//   operator on W.
// V = [X | P | W] and AV = [AX | AP | AW] are row-major blocks with leading
// dimension m + np + nw, double-buffered; Y = [X | P] is a column prefix so
// that ortho(W; Y) works on one buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

using namespace lobpcg;

size_t lobpcg_ctx::op32_elems() const {
  switch (op) {
    case kOpCsr: return (size_t)nnz;
    case kOpDense: return (size_t)n * (size_t)n;
    case kOpKron: return 2 * (size_t)na * (size_t)na;
    default: return 0;
  }
}

Layout lobpcg_ctx::plan(int m, int prec) const {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  if (method == LOBPCG_METHOD_DAVIDSON) {
    // basis and its products (n x max_dim), the rotation's [X | W~] and A X
    // (n x 2m), the explicit product of a true-residual check (n x m)
    const size_t basis = (size_t)n * dav_dim(m) * sizeof(double);
    const size_t side = (size_t)n * 2 * m * sizeof(double);
    L.V[0] = take(basis);
    L.AV[0] = take(basis);
    L.V[1] = take(side);
    L.AV[1] = take(side);
    L.dscr = take((size_t)n * m * sizeof(double));
  } else {
    const size_t blk = (size_t)n * 3 * m * sizeof(double);
    L.V[0] = take(blk);
    L.V[1] = take(blk);
    L.AV[0] = take(blk);
    L.AV[1] = take(blk);
  }
  if (bop != kOpNone) {
    const size_t blk = (size_t)n * 3 * m * sizeof(double);
    L.BV[0] = take(blk);
    L.BV[1] = take(blk);
    L.bdiag = take((size_t)n * sizeof(double));
  }
  L.diag = take((size_t)n * sizeof(double));
  L.rho = take((size_t)n * sizeof(double));
  if (pkind == LOBPCG_PRECOND_TRIDIAG) {
    L.tri_e = take((size_t)n * sizeof(double));
    L.tri_off = take((size_t)n * sizeof(double));
    L.tri_scr = take((size_t)n * std::max(m, 1) * sizeof(double));
    L.tri_bnd = take((size_t)kTriMaxChunks * kMaxBlock * 6 * sizeof(double));
    L.tri_xb = take((size_t)kTriMaxChunks * kMaxBlock * 6 * sizeof(double));
  }
  L.ltiles = take((size_t)ltiles_cap() * sizeof(int));
  if (op == kOpKron || op == kOpDense) L.kpack = take((size_t)n * 8 * sizeof(double));
  if (op == kOpCsr && slab_mode == 1)
    L.cwin = take(((size_t)(n + kSlabBlockRows - 1) / kSlabBlockRows + 1) * 8);
  const size_t gblk = (size_t)std::min<int64_t>(kGramBlocks, (n + 63) / 64) + 1;
  const size_t part =
      std::max({gblk * kGramMaxCols * kGramMaxCols, (size_t)kStreamBlocks * 3 * 64,
                (size_t)kStreamBlocks * kMaxP * kMaxBlock});
  L.part = take(part * sizeof(double));
  // small area
  size_t so = 0;
  auto stake = [&](size_t bytes) {
    const size_t o = so;
    so = align_up(so + bytes);
    return o;
  };
  L.a = stake(sizeof(double) * kGramMaxCols * kGramMaxCols);
  // read back once per iteration as one block: residual norms (64),
  // Ritz values (two slots of 64), RR info (64 ints), learned-path flags
  // (64 ints)
  L.rb = stake(kReadbackBytes);
  L.resn2 = L.rb;
  L.theta = L.rb + 512;
  L.info = L.rb + 1536;
  L.lflags = L.rb + 1792;
  L.U = stake(sizeof(double) * kMaxP * 64);
  L.G = stake(sizeof(double) * kMaxP * kMaxBlock);
  L.coef = stake(sizeof(double) * kMaxP * kMaxBlock);
  L.cols = stake(sizeof(double) * 3 * 64);
  L.ost = stake(sizeof(OrthoState));
  L.pidx = stake(sizeof(int64_t) * 256 * 64);
  L.pval = stake(sizeof(double) * 256 * 64);
  L.eye = stake(sizeof(double) * 64 * 64);
  L.lscale = stake(sizeof(double) * 4);
  L.small = take(so);
  if (prec == LOBPCG_PREC_FP32 && method != LOBPCG_METHOD_DAVIDSON) {
    const size_t blk32 = (size_t)n * 3 * m * sizeof(float);
    L.V32[0] = take(blk32);
    L.V32[1] = take(blk32);
    L.AV32[0] = take(blk32);
    L.AV32[1] = take(blk32);
    L.op32 = take(op32_elems() * sizeof(float));
  }
  L.total = off;
  return L;
}

int lobpcg_ctx::ensure_layout(int m) {
  if (ws == nullptr) return fail(LOBPCG_ERR_WORKSPACE, "no workspace set");
  Layout L = plan(m);
  if (lay_block != m || L.total != lay.total) {
    if (L.total > ws_bytes)
      return fail(LOBPCG_ERR_WORKSPACE, "workspace smaller than lobpcg_workspace_size");
    lay = L;
    lay_block = m;
    diag_ready = false;
    lfeat_ready = false;
    tri_ready = false;
    bdiag_ready = false;
    op32_ready = false;
    cwin_ready = false;
  }
  return LOBPCG_OK;
}

// The banded CSR path's column windows when LOBPCG_OPT_SPMM_SLAB selects
// it, computed once per operator and workspace layout (one read-back);
// nullptr for the gather kernels, also when some row's columns are not
// sorted.
const int2* lobpcg_ctx::csr_slab_windows() {
  if (op != kOpCsr || slab_mode != 1 || ws == nullptr || lay_block <= 0 || lay.cwin == 0)
    return nullptr;
  int2* win = reinterpret_cast<int2*>(ws + lay.cwin);
  const int64_t nb = (n + kSlabBlockRows - 1) / kSlabBlockRows;
  if (!cwin_ready) {
    int* flag = reinterpret_cast<int*>(win + nb);
    std::vector<int2> hw(nb + 1);
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), stream);
    if (e == hipSuccess) e = csr_windows(rp, ci, n, win, flag, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hw.data(), win, sizeof(int2) * (nb + 1), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return nullptr;
    slab_ok = hw[nb].x == 0;  // sorted columns
    cwin_ready = true;
  }
  return slab_ok ? win : nullptr;
}

int lobpcg_ctx::apply_op(const double* W, int64_t ldw, int nc, double* Y, int64_t ldy) {
  hipError_t e = hipSuccess;
  switch (op) {
    case kOpCsr: e = spmm_csr_f64(rp, ci, val, W, ldw, Y, ldy, nc, n, csr_slab_windows(), stream); break;
    case kOpDense:
      e = dense_apply_f64(A, lda, W, ldw, Y, ldy, nc, n,
                          (ws && lay_block > 0 && lay.kpack) ? dptr(lay.kpack) : nullptr, stream);
      break;
    case kOpKron:
      e = kronsum_apply_f64(A, Vpot, na, W, ldw, Y, ldy, nc,
                            (ws && lay_block > 0 && lay.kpack) ? dptr(lay.kpack) : nullptr,
                            stream);
      break;
    default: return fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  }
  if (e != hipSuccess) return hip_fail(e, "operator");
  stats.matvec_columns += nc;
  return LOBPCG_OK;
}

// fp32 operator (mixed-precision phase): copies made by ensure_op32
int lobpcg_ctx::apply_op(const float* W, int64_t ldw, int nc, float* Y, int64_t ldy) {
  const float* o32 = reinterpret_cast<const float*>(ws + lay.op32);
  hipError_t e = hipSuccess;
  switch (op) {
    case kOpCsr: e = spmm_csr_f32(rp, ci, o32, W, ldw, Y, ldy, nc, n, csr_slab_windows(), stream); break;
    case kOpDense:
      e = dense_apply_f32(o32, n, W, ldw, Y, ldy, nc, n,
                          lay.kpack ? reinterpret_cast<float*>(dptr(lay.kpack)) : nullptr, stream);
      break;
    case kOpKron:
      e = kronsum_apply_f32(o32, o32 + na * na, na, W, ldw, Y, ldy, nc,
                            lay.kpack ? reinterpret_cast<float*>(dptr(lay.kpack)) : nullptr,
                            stream);
      break;
    default: return fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  }
  if (e != hipSuccess) return hip_fail(e, "operator (fp32)");
  stats.matvec_columns += nc;
  return LOBPCG_OK;
}

int lobpcg_ctx::ensure_op32() {
  if (op32_ready) return LOBPCG_OK;
  float* o32 = reinterpret_cast<float*>(ws + lay.op32);
  double* part = dptr(lay.part);
  double* nb = small_ptr<double>(lay.cols);
  double* h = reinterpret_cast<double*>(pinned);
  switch (op) {
    case kOpCsr:
      HIPCHK(convert_vec_f64_to_f32(val, o32, nnz, stream));
      HIPCHK(csr_norm_bound(rp, val, n, part, nb, stream));
      break;
    case kOpDense:
      HIPCHK(convert_f64_to_f32(A, lda, o32, n, (int)n, n, stream));
      HIPCHK(dense_norm_bound(A, lda, n, part, nb, stream));
      break;
    case kOpKron:
      HIPCHK(convert_vec_f64_to_f32(A, o32, na * na, stream));
      HIPCHK(convert_vec_f64_to_f32(Vpot, o32 + na * na, na * na, stream));
      // ||H|| <= 2 max_i sum_j |A_ij| + max |V_ij| (the diag(vec V) term
      // contributes its largest entry, not a row sum of V)
      HIPCHK(dense_norm_bound(A, na, na, part, nb, stream));
      HIPCHK(vec_max_abs(Vpot, na * na, part, nb + 1, stream));
      break;
    default: return fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  }
  HIPCHK(hipMemcpyAsync(h, nb, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  norm_bound = (op == kOpKron) ? 2.0 * h[0] + h[1] : h[0];
  op32_ready = true;
  return LOBPCG_OK;
}

int lobpcg_ctx::ensure_diag() {
  if (diag_ready) return LOBPCG_OK;
  double* d = dptr(lay.diag);
  if (user_diag != nullptr) {
    HIPCHK(hipMemcpyAsync(d, user_diag, sizeof(double) * n, hipMemcpyDeviceToDevice, stream));
  } else {
    switch (op) {
      case kOpCsr: HIPCHK(csr_diag(rp, ci, val, n, d, stream)); break;
      case kOpDense: HIPCHK(dense_diag(A, lda, n, d, stream)); break;
      case kOpKron: HIPCHK(kronsum_diag(A, Vpot, na, d, stream)); break;
      default: return fail(LOBPCG_ERR_BAD_STATE, "no operator set");
    }
  }
  diag_ready = true;
  return LOBPCG_OK;
}

// The tridiagonal preconditioner's off-diagonal e_i = a_{i,i+1} and the row
// off-sums |e_{i-1}| + |e_i|, from the operator.
int lobpcg_ctx::ensure_tri() {
  if (tri_ready) return LOBPCG_OK;
  if (lay.tri_e == 0) return fail(LOBPCG_ERR_WORKSPACE, "workspace not sized for the tridiagonal preconditioner");
  int rc = ensure_diag();
  if (rc) return rc;
  double* e = dptr(lay.tri_e);
  double* off = dptr(lay.tri_off);
  switch (op) {
    case kOpCsr: HIPCHK(tri_offdiag_csr(rp, ci, val, n, e, off, stream)); break;
    case kOpDense: HIPCHK(tri_offdiag_dense(A, lda, n, e, off, stream)); break;
    case kOpKron: HIPCHK(tri_offdiag_kron(A, na, e, off, stream)); break;
    default: return fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  }
  tri_ready = true;
  return LOBPCG_OK;
}

static hipError_t tri_apply_t(double* R, int64_t ld, int nact, int64_t n, const double* th,
                              const double* d, const double* e, const double* off, double* bnd,
                              double* xb, double* scr, hipStream_t s) {
  return tri_apply_f64(R, ld, nact, n, th, d, e, off, bnd, xb, scr, s);
}
static hipError_t tri_apply_t(float* R, int64_t ld, int nact, int64_t n, const double* th,
                              const double* d, const double* e, const double* off, double* bnd,
                              double* xb, double* scr, hipStream_t s) {
  return tri_apply_f32(R, ld, nact, n, th, d, e, off, bnd, xb, scr, s);
}

template <typename T>
int lobpcg_ctx::tri_apply(T* R, int64_t ld, int nact, const double* th) {
  if (nact > lay_block || nact > kMaxBlock)
    return fail(LOBPCG_ERR_INVALID_ARG, "tridiagonal preconditioner: nact exceeds the block");
  HIPCHK(tri_apply_t(R, ld, nact, n, th, dptr(lay.diag), dptr(lay.tri_e), dptr(lay.tri_off),
                     dptr(lay.tri_bnd), dptr(lay.tri_xb), dptr(lay.tri_scr), stream));
  return LOBPCG_OK;
}

// Inputs of the learned preconditioner besides diag(A): the off-diagonal
// absolute row sums and s = mean |diag|.
int lobpcg_ctx::ensure_learned_features() {
  if (lfeat_ready) return LOBPCG_OK;
  int rc = ensure_diag();
  if (rc) return rc;
  double* rho = dptr(lay.rho);
  switch (op) {
    case kOpCsr: HIPCHK(offdiag_abs_csr(rp, ci, val, n, rho, stream)); break;
    case kOpDense: HIPCHK(offdiag_abs_dense(A, lda, n, rho, stream)); break;
    case kOpKron: HIPCHK(offdiag_abs_kron(A, na, dptr(lay.part), rho, stream)); break;
    default: return fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  }
  double* sc = small_ptr<double>(lay.lscale);
  HIPCHK(abs_mean(dptr(lay.diag), n, dptr(lay.part) + (op == kOpKron ? na : 0), sc, stream));
  double* hp = reinterpret_cast<double*>(pinned);
  HIPCHK(hipMemcpyAsync(hp, sc, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  lscale_host = hp[0];
  if (!(lscale_host > 0.0) || !std::isfinite(lscale_host))
    return fail(LOBPCG_ERR_INVALID_ARG, "learned preconditioner needs a nonzero diagonal");
  lfeat_ready = true;
  return LOBPCG_OK;
}

// typed dispatch of the streaming kernels
static hipError_t gram_t(const double* A, int64_t lda, int p, const double* B, int64_t ldb, int q,
                         int64_t n, double* part, double* C, const int* skip, hipStream_t s) {
  return gram_f64(A, lda, p, B, ldb, q, n, part, C, skip, s);
}
static hipError_t gram_t(const float* A, int64_t lda, int p, const float* B, int64_t ldb, int q,
                         int64_t n, double* part, double* C, const int* skip, hipStream_t s) {
  return gram_f32(A, lda, p, B, ldb, q, n, part, C, skip, s);
}
static hipError_t mlp_apply_t(bool bf16, double* R, int64_t ld, int nact, int64_t n,
                              const double* theta, const double* diag, const double* rho,
                              const double* s, const float* w, const int* mask,
                              uint64_t mbits, int* flags, int* tflags, int64_t tiles_cap,
                              hipStream_t st) {
  return bf16 ? mlp_apply_bf16_f64(R, ld, nact, n, theta, diag, rho, s, w, mask, mbits, flags,
                                   tflags, tiles_cap, st)
              : mlp_apply_f64(R, ld, nact, n, theta, diag, rho, s, w, mask, mbits, flags, st);
}
static hipError_t mlp_apply_t(bool bf16, float* R, int64_t ld, int nact, int64_t n,
                              const double* theta, const double* diag, const double* rho,
                              const double* s, const float* w, const int* mask,
                              uint64_t mbits, int* flags, int* tflags, int64_t tiles_cap,
                              hipStream_t st) {
  return bf16 ? mlp_apply_bf16_f32(R, ld, nact, n, theta, diag, rho, s, w, mask, mbits, flags,
                                   tflags, tiles_cap, st)
              : mlp_apply_f32(R, ld, nact, n, theta, diag, rho, s, w, mask, mbits, flags, st);
}
static hipError_t rotate_t(const double* V, const double* AV, double* Vo, double* AVo,
                           const RotateArgs& a, hipStream_t s) {
  return rotate_f64(V, AV, Vo, AVo, a, s);
}
static hipError_t rotate_t(const float* V, const float* AV, float* Vo, float* AVo,
                           const RotateArgs& a, hipStream_t s) {
  return rotate_f32(V, AV, Vo, AVo, a, s);
}
static hipError_t ortho_apply_t(double* b, int64_t ld, int ny, int nw, const double* coef,
                                const OrthoState* st, int64_t n, double* part, double* G,
                                hipStream_t s) {
  return ortho_apply_f64(b, ld, ny, nw, coef, st, n, part, G, s);
}
static hipError_t ortho_apply_t(float* b, int64_t ld, int ny, int nw, const double* coef,
                                const OrthoState* st, int64_t n, double* part, double* G,
                                hipStream_t s) {
  return ortho_apply_f32(b, ld, ny, nw, coef, st, n, part, G, s);
}
static hipError_t fill_t(double* X, int64_t ld, int col, int id, int64_t n, uint64_t seed,
                         hipStream_t s) {
  return fill_splitmix(X, ld, col, id, n, seed, s);
}
static hipError_t fill_t(float* X, int64_t ld, int col, int id, int64_t n, uint64_t seed,
                         hipStream_t s) {
  return fill_splitmix_f32(X, ld, col, id, n, seed, s);
}

// Status read-back of `bytes` of device memory once the queued work ran.
int lobpcg_ctx::readback(const void* src, size_t bytes, const void** out) {
  if (bytes > kPostBytes || bytes % 4 != 0) return fail(LOBPCG_ERR_INVALID_ARG, "read-back size");
  if (post == nullptr) {
    HIPCHK(hipMemcpyAsync(pinned, src, bytes, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    *out = pinned;
    return LOBPCG_OK;
  }
  // a kernel copies the block into coherent host memory and then raises the
  // sequence word; the host spins on that word instead of synchronising the
  // stream (which costs a copy-engine transfer and a wake-up per read-back)
  if (++post_seq == 0) post_seq = 1;
  const uint32_t seq = post_seq;
  HIPCHK(post_status(src, (int)(bytes / 4), post_dev, post_dev + kPostBytes / 4, seq, stream));
  volatile uint32_t* flag = post + kPostBytes / 4;
  const auto t0 = std::chrono::steady_clock::now();
  unsigned k = 0;
  while (*flag != seq) {
    __builtin_ia32_pause();
    if ((++k & 255) != 0) continue;
    // every few microseconds: a failed stream ends the wait, a drained one
    // must have posted (its kernels have completed)
    const hipError_t q = hipStreamQuery(stream);
    if (q == hipSuccess) {
      if (*flag == seq) break;
      return fail(LOBPCG_ERR_DEVICE, "status post missing after the stream drained");
    }
    if (q != hipErrorNotReady) return hip_fail(q, "stream");
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(300))
      return fail(LOBPCG_ERR_DEVICE, "status post timed out");
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  *out = post;
  return LOBPCG_OK;
}

// ortho(W; Y) (Alg. 3 around Alg. 2) on base = [Y | W] rows, ld: rounds of
// (controller kernel, block update with the next overlap) driven by the
// device-side state, read back every few rounds.
template <typename T>
int lobpcg_ctx::ortho_run(T* base, int64_t ld, int ny, int nw, lobpcg_ortho_info* info,
                          bool fold, double tau_run) {
  OrthoState* st = small_ptr<OrthoState>(lay.ost);
  double* G = small_ptr<double>(lay.G);
  double* coef = small_ptr<double>(lay.coef);
  double* part = dptr(lay.part);
  const int nr = ny + nw;
  const double t = (tau_run > 0.0) ? tau_run : tau;
  for (int attempt = 0; attempt < 3; ++attempt) {
    // cheap exits: c(n) times the unit roundoff of the blocks' precision
    const double unit = (sizeof(T) == sizeof(float)) ? 0x1.0p-23 : 0x1.0p-52;
    const double cexit =
        cheap_exit ? std::max(4.0, 0.02 * std::sqrt((double)n)) * unit : 0.0;
    HIPCHK(ortho_init(st, ny, nw, t, ortho_max_inner, ortho_max_outer, shift_retries, fold ? 1 : 0,
                      cexit, stream));
    // the overlap [Y W~]^T W~ of the raw W~, by its own kernel: fused into
    // the rotation it held the rotation at two waves per SIMD (fp64), which
    // cost more than the separate pass (434 us against 328 + 91 us per
    // iteration at n = 1e6, m = 16)
    HIPCHK(gram_t(base, ld, nr, base + ny, ld, nw, n, part, G, nullptr, stream));
    int rounds = 0;
    bool finished = false;
    OrthoState hs{};
    while (!finished) {
      const int batch = (rounds == 0) ? kOrthoRounds : 2;
      for (int r = 0; r < batch; ++r) {
        HIPCHK(ortho_ctl(G, st, coef, stream));
        HIPCHK(ortho_apply_t(base, ld, ny, nw, coef, st, n, part, G, stream));
      }
      rounds += batch;
      const void* rbp = nullptr;
      const int rc = readback(st, sizeof(OrthoState), &rbp);
      if (rc) return rc;
      std::memcpy(&hs, rbp, sizeof(OrthoState));
      if (hs.done) finished = true;
      else if (rounds >= kOrthoHardCap) return fail(LOBPCG_ERR_ORTHO_FAILED, "ortho did not finish");
    }
    const OrthoState s = hs;
    stats.ortho_grams += s.grams;
    stats.ortho_factorizations += s.factorizations;
    stats.ortho_failed += s.failed;
    stats.ortho_shifted += s.shifted;
    stats.ortho_stalled += s.stalled;
    stats.ortho_svqb += s.svqb;
    stats.against_passes += s.passes;
    stats.ortho_cheap_exits += s.cheap_exits;
    if (info != nullptr) {
      info->cheap_exits += s.cheap_exits;
      info->grams += s.grams;
      info->factorizations += s.factorizations;
      info->failed += s.failed;
      info->shifted += s.shifted;
      info->updates += s.updates;
      info->passes += s.passes;
      info->stalled += s.stalled;
      info->svqb += s.svqb;
    }
    if (s.error == 0) return LOBPCG_OK;
    if (s.error == kOrthoErrNonfinite) return fail(LOBPCG_ERR_NONFINITE, "non-finite overlap");
    if (s.error == kOrthoErrFailed) return fail(LOBPCG_ERR_ORTHO_FAILED, "shifted Cholesky and SVQB failed");
    // exact zero columns: replace by SplitMix64 columns and start again
    for (int j = 0; j < nw; ++j)
      if (s.zero_mask & (1 << j)) HIPCHK(fill_t(base + ny, ld, j, j, n, kZeroColumnSeed, stream));
  }
  return fail(LOBPCG_ERR_ORTHO_FAILED, "zero columns persist");
}

int lobpcg_ctx::true_residuals(const double* X, int64_t ldx, int m, double* scratch,
                               const double* theta_rr, std::vector<double>& th,
                               std::vector<double>& rn) {
  int rc = apply_op(X, ldx, m, scratch, m);
  if (rc) return rc;
  double* cols = small_ptr<double>(lay.cols);
  double* thd = small_ptr<double>(lay.theta) + 64;  // second theta slot
  double* part = dptr(lay.part);
  double* h = reinterpret_cast<double*>(pinned);
  HIPCHK(colstats_f64(X, ldx, scratch, m, m, theta_rr, n, part, cols, stream));
  HIPCHK(hipMemcpyAsync(h, cols, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  th.assign(m, 0.0);
  for (int j = 0; j < m; ++j) th[j] = h[m + j] / h[j];
  std::vector<double> tmp(th);
  HIPCHK(hipMemcpyAsync(thd, tmp.data(), sizeof(double) * m, hipMemcpyHostToDevice, stream));
  HIPCHK(colstats_f64(X, ldx, scratch, m, m, thd, n, part, cols, stream));
  HIPCHK(hipMemcpyAsync(h, cols, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  rn.assign(m, 0.0);
  for (int j = 0; j < m; ++j) rn[j] = std::sqrt(h[2 * m + j]);
  stats.true_checks++;
  return LOBPCG_OK;
}

static int leading_converged(const std::vector<double>& r, double tol) {
  int c = 0;
  for (double v : r) {
    if (v <= tol) ++c;
    else break;
  }
  return c;
}

// Reading R22's bookkeeping for one Rayleigh-Ritz step: true when R9's
// check is to run although the recurrence has not converged (the largest
// residual of the sought active columns, within 100 tol, has not fallen by
// 1 % over `window` steps)
static bool stall_step(const std::vector<double>& rnorm, int m_conv, int k, double tol,
                       int window, double& best, int& since) {
  if (window <= 0) return false;
  double ract = 0.0;
  for (int j = m_conv; j < k; ++j) ract = std::max(ract, rnorm[j]);
  if (ract < 0.99 * best) {
    best = ract;
    since = 0;
  } else {
    ++since;
  }
  // only near the tolerance: a plateau far above it is slow convergence,
  // which a restart (P dropped) would only slow down
  return since >= window && ract <= 100.0 * tol;
}

// One precision phase of Alg. 1, starting from the block X stored in V0
// (leading dimension m, not yet orthonormal).  `low` selects the fp32 phase
// (reading of the mixed-precision extension): no locking, ortho threshold
// 1e-6, and the phase ends when every residual is within 100 fp32 roundoffs
// of ||A|| or has stalled (no 10% decrease over 3 iterations).  The fp64
// phase ends on the true-residual check (every sought column's ||A x -
// theta x|| <= tol, recomputed from an explicit product A X) or max_iter.
template <typename T>
int lobpcg_ctx::run_phase(T* V0, T* V1, T* AV0, T* AV1, int k, double tol, bool low, int& iter,
                          PhaseOut& out) {
  const int m = block;
  T* V[2] = {V0, V1};
  T* AV[2] = {AV0, AV1};
  double* a = small_ptr<double>(lay.a);
  double* theta = small_ptr<double>(lay.theta);
  double* U = small_ptr<double>(lay.U);
  double* resn2 = small_ptr<double>(lay.resn2);
  int* info = small_ptr<int>(lay.info);
  double* part = dptr(lay.part);
  double* h = reinterpret_cast<double*>(pinned);
  const double tau_phase = low ? 1e-6 : tau;
  const double lock_tol = low ? -1.0 : tol;  // nothing locks in the fp32 phase
  const double switch_level = 100.0 * 0x1.0p-24 * (norm_bound > 0.0 ? norm_bound : 1.0);
  // learned preconditioner: a column whose residual did not decrease over
  // the step that used its learned W takes the Jacobi step for the next 3
  // iterations (so does a column where the net produced a non-finite value)
  const bool learned = (pkind == LOBPCG_PRECOND_LEARNED);
  const bool tri = (pkind == LOBPCG_PRECOND_TRIDIAG);
  std::vector<int> fb_left(m, 0);
  std::vector<char> used_learned(m, 0);
  std::vector<double> r_before(m, 0.0);
  int prev_a0 = 0, prev_nact = 0;
  int* lflags = small_ptr<int>(lay.lflags);
  if (learned) HIPCHK(hipMemsetAsync(lflags, 0, sizeof(int) * 64, stream));
  int rc = ortho_run<T>(V[0], m, 0, m, nullptr, true, tau_phase);
  if (rc) return rc;
  rc = apply_op(V[0], m, m, AV[0], m);
  if (rc) return rc;
  // a column scaling left pending by the last ortho of W (or of X0) is
  // folded into the next Rayleigh-Ritz coefficients
  const OrthoState* pend = small_ptr<OrthoState>(lay.ost);
  int pend_woff = 0;
  bool pend_valid = true;

  int c = 0;           // current buffer
  int L = m;           // its leading dimension (= number of columns in V)
  bool first = true;   // V = [X] only (initial RR, or restart after a true check)
  bool just_restarted = false;  // the convergence test waits one iteration after a restart
  int m_conv = 0;
  double prev_max = INFINITY;
  int stall = 0;
  // fp64 phase: the recurrence's residuals (A X carried as [AX AW AP] U)
  // can settle on a floor left by its rounding rather than by convergence;
  // without 1 % progress of the largest sought active one over
  // stall_window iterations, within 100 tol, the explicit check runs anyway
  double best_act = INFINITY;
  int since_best = 0;
  std::vector<double> rnorm(m), th_rr(m), th_t, rn_t;
  out.converged = false;
  for (;;) {
    // ---- Rayleigh-Ritz in V (Alg. 1) ----
    HIPCHK(gram_t(V[c], L, L, AV[c], L, L, n, part, a, nullptr, stream));
    const int want_up = first ? 0 : 1;
    int a0 = m_conv;
    int nact = m - a0;
    HIPCHK(small_rr(a, L, m, a0, want_up, tau_phase, pend_valid ? pend : nullptr, pend_woff, theta,
                    U, info, rr_jacobi, stream));
    int q = m + (want_up ? nact : 0);
    int ldo = q + nact;
    RotateArgs ra{};
    ra.n = n;
    ra.ldv = L;
    ra.ldo = ldo;
    ra.p = L;
    ra.m = m;
    ra.q = q;
    ra.a0 = a0;
    // learned and tridiagonal: W~ = R here, transformed below; once the
    // learned budget is spent the next iteration takes the fused Jacobi step
    const bool learned_now = learned && !(learned_budget > 0 && iter + 1 > learned_budget);
    ra.precond = (learned_now || tri) ? kPrecNone : (learned ? kPrecDiag : pkind);
    ra.U = U;
    ra.theta = theta;
    ra.diag = dptr(lay.diag);
    ra.part = part;
    ra.resnorm2 = resn2;
    HIPCHK(rotate_t(V[c], AV[c], V[1 - c], AV[1 - c], ra, stream));
    // one read-back: resn2 at hb[0], theta at hb[64], info at hb[192], flags
    // at hb[224]
    const void* rbp = nullptr;
    rc = readback(resn2, kReadbackBytes, &rbp);
    if (rc) return rc;
    const double* hb = static_cast<const double*>(rbp);
    const int* hinfo = reinterpret_cast<const int*>(hb + 192);
    if (hinfo[1] != 0) return fail(LOBPCG_ERR_ORTHO_FAILED, "R^p orthonormalisation of u_p failed");
    stats.rr_eig_fallbacks += hinfo[11];
    double rmax = 0.0;
    for (int j = 0; j < m; ++j) {
      rnorm[j] = std::sqrt(hb[j]);
      th_rr[j] = hb[64 + j];
      if (!std::isfinite(rnorm[j]) || !std::isfinite(th_rr[j]))
        return fail(LOBPCG_ERR_NONFINITE, "non-finite Ritz value or residual");
      rmax = std::max(rmax, rnorm[j]);
    }
    if (learned) {
      const int* hfl = reinterpret_cast<const int*>(hb + 224);
      for (int j = 0; j < prev_nact; ++j)
        if (hfl[j]) {
          stats.learned_nonfinite++;
          fb_left[prev_a0 + j] = 3;
          used_learned[prev_a0 + j] = 0;
        }
      for (int j = 0; j < m; ++j) {
        if (used_learned[j] && !(rnorm[j] < r_before[j])) {
          fb_left[j] = 3;
          stats.learned_fallbacks++;
        }
        used_learned[j] = 0;
      }
      prev_nact = 0;
    }
    if (low) {
      stall = (rmax > 0.9 * prev_max) ? stall + 1 : 0;
      prev_max = std::min(prev_max, rmax);
      if (rmax <= switch_level || stall >= 3 || iter >= max_iter) {
        out.X = V[1 - c];
        out.ld = ldo;
        return LOBPCG_OK;
      }
    }
    int newc = std::max(m_conv, leading_converged(rnorm, lock_tol));
    // after a restart the convergence test waits one iteration, and that
    // iteration keeps at least the k-th column active
    if (just_restarted) newc = std::min(newc, k - 1);
    just_restarted = false;
    const bool stalled =
        !low && stall_step(rnorm, m_conv, k, tol, stall_window, best_act, since_best);
    if (!low && (newc >= k || stalled)) {
      if (stalled && newc < k) stats.stall_checks++;
      best_act = INFINITY;
      since_best = 0;
      // convergence is confirmed on an explicit product A X, not the
      // recurrence's residuals
      // the implicit-P recurrence lets X's orthonormality drift by rounding
      // (about 1e-12 after hundreds of iterations): re-orthonormalise X
      // (Alg. 2) before the explicit product that judges it
      rc = ortho_run<T>(V[1 - c], ldo, 0, m, nullptr, false, tau);
      if (rc) return rc;
      const double* Xd = reinterpret_cast<const double*>(V[1 - c]);
      double* scratch = reinterpret_cast<double*>(AV[c]);
      rc = true_residuals(Xd, ldo, m, scratch, theta, th_t, rn_t);
      if (rc) return rc;
      double worst = 0.0;
      for (int j = 0; j < k; ++j) worst = std::max(worst, rn_t[j]);
      if (worst <= tol && stats.restarts >= force_restarts) {
        out.converged = true;
        out.X = V[1 - c];
        out.ld = ldo;
        break;
      }
      // restart as Alg. 1 starts: Rayleigh-Ritz on V = [X] with the explicit
      // product AV = [A X] (true_residuals left it in AV[c] at leading
      // dimension m), P dropped, locking recounted; the next convergence
      // test comes one iteration later, an iteration with at most k - 1
      // locked columns
      stats.restarts++;
      HIPCHK(hipMemcpy2DAsync(V[c], sizeof(T) * m, V[1 - c], sizeof(T) * ldo, sizeof(T) * m, n,
                              hipMemcpyDeviceToDevice, stream));
      L = m;
      first = true;
      m_conv = 0;
      pend_valid = false;  // the copied X is fully scaled
      just_restarted = true;
      continue;
    }
    if (newc != m_conv) {
      // locking changed the active set: rebuild u_p, P and W~ for it
      stats.relocks++;
      m_conv = newc;
      a0 = m_conv;
      nact = m - a0;
      HIPCHK(small_rr(a, L, m, a0, want_up, tau_phase, pend_valid ? pend : nullptr, pend_woff,
                      theta, U, info, rr_jacobi, stream));
      q = m + (want_up ? nact : 0);
      ldo = q + nact;
      ra.ldo = ldo;
      ra.q = q;
      ra.a0 = a0;
      HIPCHK(rotate_t(V[c], AV[c], V[1 - c], AV[1 - c], ra, stream));
    }
    if (iter >= max_iter) {
      rc = ortho_run<T>(V[1 - c], ldo, 0, m, nullptr, false, tau);
      if (rc) return rc;
      const double* Xd = reinterpret_cast<const double*>(V[1 - c]);
      rc = true_residuals(Xd, ldo, m, reinterpret_cast<double*>(AV[c]), theta, th_t, rn_t);
      if (rc) return rc;
      out.X = V[1 - c];
      out.ld = ldo;
      break;
    }
    ++iter;
    // ---- W = ortho(T R; [X P]) and AW = A W (Alg. 1) ----
    if (learned && !learned_now && stats.learned_budget_iter < 0) stats.learned_budget_iter = iter;
    if (learned_now) {
      // the fallback columns go to the kernels as a bit set (no copy); the
      // bf16 transform clears its flags itself
      uint64_t mbits = 0;
      for (int j = a0; j < m; ++j) {
        const bool jac = fb_left[j] > 0;
        if (jac) --fb_left[j];
        if (jac) mbits |= uint64_t(1) << (j - a0);
        used_learned[j] = jac ? 0 : 1;
        r_before[j] = rnorm[j];
      }
      if (!learned_bf16) HIPCHK(hipMemsetAsync(lflags, 0, sizeof(int) * 64, stream));
      HIPCHK(mlp_apply_t(learned_bf16 != 0, V[1 - c] + q, ldo, nact, n, theta + a0,
                         dptr(lay.diag), dptr(lay.rho), small_ptr<double>(lay.lscale), lweights,
                         nullptr, mbits, lflags, reinterpret_cast<int*>(ws + lay.ltiles),
                         ltiles_cap(), stream));
      prev_a0 = a0;
      prev_nact = nact;
    }
    if (tri) {
      rc = tri_apply<T>(V[1 - c] + q, ldo, nact, theta + a0);
      if (rc) return rc;
    }
    rc = ortho_run<T>(V[1 - c], ldo, q, nact, nullptr, true, tau_phase);
    if (rc) return rc;
    pend_valid = true;
    pend_woff = q;
    rc = apply_op(V[1 - c] + q, ldo, nact, AV[1 - c] + q, ldo);
    if (rc) return rc;
    c = 1 - c;
    L = ldo;
    first = false;
  }
  if (!low) {
    res_evals.assign(th_t.begin(), th_t.begin() + m);
    res_resn.assign(rn_t.begin(), rn_t.begin() + m);
    stats.m_conv = m_conv;
  }
  return LOBPCG_OK;
}

// Block Davidson (Sec. 2, X^{k+1} = RR(X^1, T^1 R^1, ..., T^k R^k); Sec. 4
// keeps 25 vectors per root): the basis V (n x max_dim, leading dimension
// max_dim) starts as ortho(X0) and grows by each active preconditioned
// residual block, made orthonormal to it by Alg. 3 (the ortho controller
// on [V | W]).  Per iteration: Gram a = V^T AV over the p basis columns,
// the RR eigensolve, the rotation into the side buffer ([X | W~], A X),
// locking and the true-residual test as in run_phase (readings R8, R9),
// then W~ is copied behind the basis, orthonormalised and multiplied by A.
// When the next block would exceed max_dim the history is truncated: the
// basis restarts from the current Ritz vectors X (and A X).
int lobpcg_ctx::run_davidson(int k, double tol, int& iter, PhaseOut& out) {
  const int m = block;
  const int md = dav_dim(m);
  double* V = dptr(lay.V[0]);
  double* AV = dptr(lay.AV[0]);
  double* V1 = dptr(lay.V[1]);
  double* AV1 = dptr(lay.AV[1]);
  double* scr = dptr(lay.dscr);
  double* a = small_ptr<double>(lay.a);
  double* theta = small_ptr<double>(lay.theta);
  double* U = small_ptr<double>(lay.U);
  double* resn2 = small_ptr<double>(lay.resn2);
  int* info = small_ptr<int>(lay.info);
  double* part = dptr(lay.part);
  const size_t sd = sizeof(double);

  int rc = ortho_run<double>(V, md, 0, m, nullptr, false, tau);
  if (rc) return rc;
  rc = apply_op(V, md, m, AV, md);
  if (rc) return rc;
  int p = m;  // basis columns
  int m_conv = 0;
  bool just_restarted = false;
  double best_act = INFINITY;  // reading R22
  int since_best = 0;
  stats.max_basis = p;
  std::vector<double> rnorm(m), th_t, rn_t;
  out.converged = false;
  for (;;) {
    HIPCHK(gram_f64(V, md, p, AV, md, p, n, part, a, nullptr, stream));
    int a0 = m_conv;
    int nact = m - a0;
    HIPCHK(small_rr(a, p, m, a0, 0, tau, nullptr, 0, theta, U, info, rr_jacobi, stream));
    int ldo = m + nact;
    RotateArgs ra{};
    ra.n = n;
    ra.ldv = md;
    ra.ldo = ldo;
    ra.p = p;
    ra.m = m;
    ra.q = m;
    ra.a0 = a0;
    ra.precond = (pkind == LOBPCG_PRECOND_TRIDIAG) ? kPrecNone : pkind;
    ra.U = U;
    ra.theta = theta;
    ra.diag = dptr(lay.diag);
    ra.part = part;
    ra.resnorm2 = resn2;
    HIPCHK(rotate_f64(V, AV, V1, AV1, ra, stream));
    const void* rbp = nullptr;
    rc = readback(resn2, kReadbackBytes, &rbp);
    if (rc) return rc;
    const double* hb = static_cast<const double*>(rbp);
    const int* hinfo = reinterpret_cast<const int*>(hb + 192);
    if (hinfo[1] != 0) return fail(LOBPCG_ERR_ORTHO_FAILED, "Rayleigh-Ritz eigensolve failed");
    stats.rr_eig_fallbacks += hinfo[11];
    for (int j = 0; j < m; ++j) {
      rnorm[j] = std::sqrt(hb[j]);
      if (!std::isfinite(rnorm[j]) || !std::isfinite(hb[64 + j]))
        return fail(LOBPCG_ERR_NONFINITE, "non-finite Ritz value or residual");
    }
    int newc = std::max(m_conv, leading_converged(rnorm, tol));
    if (just_restarted) newc = std::min(newc, k - 1);
    just_restarted = false;
    const bool stalled = stall_step(rnorm, m_conv, k, tol, stall_window, best_act, since_best);
    if (newc >= k || stalled) {
      if (stalled && newc < k) stats.stall_checks++;
      best_act = INFINITY;
      since_best = 0;
      rc = ortho_run<double>(V1, ldo, 0, m, nullptr, false, tau);
      if (rc) return rc;
      rc = true_residuals(V1, ldo, m, scr, theta, th_t, rn_t);
      if (rc) return rc;
      double worst = 0.0;
      for (int j = 0; j < k; ++j) worst = std::max(worst, rn_t[j]);
      if (worst <= tol && stats.restarts >= force_restarts) {
        out.converged = true;
        out.X = V1;
        out.ld = ldo;
        break;
      }
      // restart from X with the explicit product (reading R9)
      stats.restarts++;
      HIPCHK(hipMemcpy2DAsync(V, sd * md, V1, sd * ldo, sd * m, n, hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipMemcpy2DAsync(AV, sd * md, scr, sd * m, sd * m, n, hipMemcpyDeviceToDevice, stream));
      p = m;
      m_conv = 0;
      just_restarted = true;
      continue;
    }
    if (newc != m_conv) {
      // locking changed the active set: W~ for the new one
      stats.relocks++;
      m_conv = newc;
      a0 = m_conv;
      nact = m - a0;
      HIPCHK(small_rr(a, p, m, a0, 0, tau, nullptr, 0, theta, U, info, rr_jacobi, stream));
      ldo = m + nact;
      ra.ldo = ldo;
      ra.a0 = a0;
      HIPCHK(rotate_f64(V, AV, V1, AV1, ra, stream));
    }
    if (iter >= max_iter) {
      rc = ortho_run<double>(V1, ldo, 0, m, nullptr, false, tau);
      if (rc) return rc;
      rc = true_residuals(V1, ldo, m, scr, theta, th_t, rn_t);
      if (rc) return rc;
      out.X = V1;
      out.ld = ldo;
      break;
    }
    ++iter;
    if (p + nact > md) {
      // history truncation: restart the basis from the Ritz vectors
      stats.history_restarts++;
      HIPCHK(hipMemcpy2DAsync(V, sd * md, V1, sd * ldo, sd * m, n, hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipMemcpy2DAsync(AV, sd * md, AV1, sd * ldo, sd * m, n, hipMemcpyDeviceToDevice, stream));
      p = m;
    }
    if (pkind == LOBPCG_PRECOND_TRIDIAG) {
      rc = tri_apply<double>(V1 + m, ldo, nact, theta + a0);
      if (rc) return rc;
    }
    HIPCHK(hipMemcpy2DAsync(V + p, sd * md, V1 + m, sd * ldo, sd * nact, n, hipMemcpyDeviceToDevice,
                            stream));
    rc = ortho_run<double>(V, md, p, nact, nullptr, false, tau);
    if (rc) return rc;
    rc = apply_op(V + p, md, nact, AV + p, md);
    if (rc) return rc;
    p += nact;
    stats.max_basis = std::max(stats.max_basis, p);
  }
  res_evals.assign(th_t.begin(), th_t.begin() + m);
  res_resn.assign(rn_t.begin(), rn_t.begin() + m);
  stats.m_conv = m_conv;
  return LOBPCG_OK;
}

// ---- the generalized problem A x = lambda B x (Sec. 3.3) ----------------

int lobpcg_ctx::apply_b(const double* W, int64_t ldw, int nc, double* Y, int64_t ldy) {
  hipError_t e = hipSuccess;
  switch (bop) {
    case kOpCsr: e = spmm_csr_f64(brp, bci, bval, W, ldw, Y, ldy, nc, n, nullptr, stream); break;
    case kOpDense:
      e = dense_apply_f64(Bd, ldb, W, ldw, Y, ldy, nc, n,
                          (ws && lay_block > 0 && lay.kpack) ? dptr(lay.kpack) : nullptr, stream);
      break;
    default: return fail(LOBPCG_ERR_BAD_STATE, "no B operator set");
  }
  if (e != hipSuccess) return hip_fail(e, "B operator");
  stats.b_matvec_columns += nc;
  return LOBPCG_OK;
}

int lobpcg_ctx::ensure_bdiag() {
  if (bdiag_ready) return LOBPCG_OK;
  double* d = dptr(lay.bdiag);
  switch (bop) {
    case kOpCsr: HIPCHK(csr_diag(brp, bci, bval, n, d, stream)); break;
    case kOpDense: HIPCHK(dense_diag(Bd, ldb, n, d, stream)); break;
    default: return fail(LOBPCG_ERR_BAD_STATE, "no B operator set");
  }
  bdiag_ready = true;
  return LOBPCG_OK;
}

// One B-Cholesky pass with the application reused (Sec. 3.3): M = X^T (BX),
// M = L L^T (shifted on failure, Sec. 3.2), X <- X L^-T, BX <- BX L^-T; X
// and BX are n x nc with leading dimension ld.
int lobpcg_ctx::b_orthonormalize(double* X, double* BX, int64_t ld, int nc) {
  double* M = small_ptr<double>(lay.a);
  double* Lf = small_ptr<double>(lay.G);
  double* coef = small_ptr<double>(lay.coef);
  int* info = small_ptr<int>(lay.info);
  HIPCHK(gram_f64(X, ld, nc, BX, ld, nc, n, dptr(lay.part), M, nullptr, stream));
  HIPCHK(small_cholesky(M, nc, Lf, info, stream));
  HIPCHK(gen_lt_inv(Lf, nc, coef, stream));
  HIPCHK(tsmm_f64(X, ld, nc, coef, nc, X, ld, n, nullptr, stream));
  HIPCHK(tsmm_f64(BX, ld, nc, coef, nc, BX, ld, n, nullptr, stream));
  const void* rbp = nullptr;
  int rc = readback(info, 16, &rbp);
  if (rc) return rc;
  const int* hi = static_cast<const int*>(rbp);
  stats.ortho_factorizations += hi[1];
  stats.ortho_failed += hi[2];
  if (hi[0] != 0) return fail(LOBPCG_ERR_ORTHO_FAILED, "B-overlap not positive definite");
  return LOBPCG_OK;
}

// Alg. 1 for the generalized problem (reading of Sec. 3.3): the basis
// V = [X | P | W] is B-orthonormal and B V is carried in its own buffers.
// Per iteration: Gram a = V^T AV, the RR kernel, the rotation of V and AV
// (its residual is replaced), B V U for [BX BP], the generalized residual
// R = A X - B X Theta with the preconditioned W~, then
// W^ = ortho(W~, (BX, BP)) (the B-orthogonal projection W - [X P]([BX BP]^T
// W) and Euclidean Alg. 2 passes until ||[BX BP]^T W|| <= tau), one
// application B W^, one B-Cholesky reusing it, and A W.
int lobpcg_ctx::run_generalized(int k, double tol, int& iter, PhaseOut& out) {
  const int m = block;
  double* V[2] = {dptr(lay.V[0]), dptr(lay.V[1])};
  double* AV[2] = {dptr(lay.AV[0]), dptr(lay.AV[1])};
  double* BV[2] = {dptr(lay.BV[0]), dptr(lay.BV[1])};
  double* a = small_ptr<double>(lay.a);
  double* theta = small_ptr<double>(lay.theta);
  double* U = small_ptr<double>(lay.U);
  double* resn2 = small_ptr<double>(lay.resn2);
  int* info = small_ptr<int>(lay.info);
  double* part = dptr(lay.part);
  double* C = small_ptr<double>(lay.G);
  double* coef = small_ptr<double>(lay.coef);
  double* cols = small_ptr<double>(lay.cols);
  const size_t sd = sizeof(double);
  const int gp = (pkind == LOBPCG_PRECOND_NONE) ? 0 : (pkind == LOBPCG_PRECOND_DIAG_SIGNED ? 2 : 1);

  // X0: Euclidean Alg. 2, then B-orthonormalised with one B application
  int rc = ortho_run<double>(V[0], m, 0, m, nullptr, false, tau);
  if (rc) return rc;
  rc = apply_b(V[0], m, m, BV[0], m);
  if (rc) return rc;
  rc = b_orthonormalize(V[0], BV[0], m, m);
  if (rc) return rc;
  rc = apply_op(V[0], m, m, AV[0], m);
  if (rc) return rc;

  int c = 0, L = m, m_conv = 0;
  bool first = true, just_restarted = false;
  double best_act = INFINITY;  // reading R22
  int since_best = 0;
  std::vector<double> rnorm(m);
  std::vector<double> th_t(m), rn_t(m);
  out.converged = false;
  // the explicit products of a true check: X (B-orthonormalised again), A X
  // and B X land in V[c], AV[c] and BV[c] (leading dimension m), which the
  // restart then uses as its basis
  auto true_check = [&](double* X, int64_t ldx) -> int {
    int r = apply_b(X, ldx, m, BV[c], m);
    if (r) return r;
    HIPCHK(hipMemcpy2DAsync(V[c], sd * m, X, sd * ldx, sd * m, n, hipMemcpyDeviceToDevice, stream));
    r = b_orthonormalize(V[c], BV[c], m, m);
    if (r) return r;
    r = apply_op(V[c], m, m, AV[c], m);
    if (r) return r;
    // Rayleigh quotients, then the residuals with them
    double* thd = small_ptr<double>(lay.theta) + 64;
    HIPCHK(gen_colstats(V[c], m, AV[c], BV[c], m, m, theta, n, part, cols, stream));
    const void* rbp = nullptr;
    r = readback(cols, sd * 3 * m, &rbp);
    if (r) return r;
    const double* h = static_cast<const double*>(rbp);
    for (int j = 0; j < m; ++j) th_t[j] = h[m + j] / h[j];
    HIPCHK(hipMemcpyAsync(thd, th_t.data(), sd * m, hipMemcpyHostToDevice, stream));
    HIPCHK(gen_colstats(V[c], m, AV[c], BV[c], m, m, thd, n, part, cols, stream));
    r = readback(cols, sd * 3 * m, &rbp);
    if (r) return r;
    h = static_cast<const double*>(rbp);
    for (int j = 0; j < m; ++j) rn_t[j] = std::sqrt(std::max(h[2 * m + j], 0.0));
    stats.true_checks++;
    return LOBPCG_OK;
  };

  for (;;) {
    HIPCHK(gram_f64(V[c], L, L, AV[c], L, L, n, part, a, nullptr, stream));
    const int want_up = first ? 0 : 1;
    int a0 = m_conv;
    int nact = m - a0;
    HIPCHK(small_rr(a, L, m, a0, want_up, tau, nullptr, 0, theta, U, info, rr_jacobi, stream));
    int q = m + (want_up ? nact : 0);
    int ldo = q + nact;
    RotateArgs ra{};
    ra.n = n;
    ra.ldv = L;
    ra.ldo = ldo;
    ra.p = L;
    ra.m = m;
    ra.q = q;
    ra.a0 = a0;
    ra.precond = kPrecNone;
    ra.U = U;
    ra.theta = theta;
    ra.diag = dptr(lay.diag);
    ra.part = part;
    ra.resnorm2 = resn2;
    auto rotate_all = [&]() -> int {
      HIPCHK(rotate_f64(V[c], AV[c], V[1 - c], AV[1 - c], ra, stream));
      HIPCHK(tsmm_f64(BV[c], L, L, U, q, BV[1 - c], ldo, n, nullptr, stream));
      HIPCHK(gen_residual(AV[1 - c], BV[1 - c], ldo, m, theta, a0, gp, dptr(lay.diag),
                          dptr(lay.bdiag), V[1 - c] + q, ldo, n, part, resn2, stream));
      return LOBPCG_OK;
    };
    rc = rotate_all();
    if (rc) return rc;
    const void* rbp = nullptr;
    rc = readback(resn2, kReadbackBytes, &rbp);
    if (rc) return rc;
    const double* hb = static_cast<const double*>(rbp);
    const int* hinfo = reinterpret_cast<const int*>(hb + 192);
    if (hinfo[1] != 0) return fail(LOBPCG_ERR_ORTHO_FAILED, "R^p orthonormalisation of u_p failed");
    stats.rr_eig_fallbacks += hinfo[11];
    for (int j = 0; j < m; ++j) {
      rnorm[j] = std::sqrt(hb[j]);
      if (!std::isfinite(rnorm[j]) || !std::isfinite(hb[64 + j]))
        return fail(LOBPCG_ERR_NONFINITE, "non-finite Ritz value or residual");
    }
    int newc = std::max(m_conv, leading_converged(rnorm, tol));
    if (just_restarted) newc = std::min(newc, k - 1);
    just_restarted = false;
    const bool stalled = stall_step(rnorm, m_conv, k, tol, stall_window, best_act, since_best);
    if (newc >= k || stalled) {
      if (stalled && newc < k) stats.stall_checks++;
      best_act = INFINITY;
      since_best = 0;
      rc = true_check(V[1 - c], ldo);
      if (rc) return rc;
      double worst = 0.0;
      for (int j = 0; j < k; ++j) worst = std::max(worst, rn_t[j]);
      if (worst <= tol && stats.restarts >= force_restarts) {
        out.converged = true;
        out.X = V[c];
        out.ld = m;
        break;
      }
      // restart from the checked X, A X, B X (now in V[c], AV[c], BV[c])
      stats.restarts++;
      L = m;
      first = true;
      m_conv = 0;
      just_restarted = true;
      continue;
    }
    if (newc != m_conv) {
      stats.relocks++;
      m_conv = newc;
      a0 = m_conv;
      nact = m - a0;
      HIPCHK(small_rr(a, L, m, a0, want_up, tau, nullptr, 0, theta, U, info, rr_jacobi, stream));
      q = m + (want_up ? nact : 0);
      ldo = q + nact;
      ra.ldo = ldo;
      ra.q = q;
      ra.a0 = a0;
      rc = rotate_all();
      if (rc) return rc;
    }
    if (iter >= max_iter) {
      rc = true_check(V[1 - c], ldo);
      if (rc) return rc;
      out.X = V[c];
      out.ld = m;
      break;
    }
    ++iter;
    // W^ = ortho(W~, (BX, BP)) with Y = [X P] = columns [0, q) of V[1-c]
    double* Vn = V[1 - c];
    double* BVn = BV[1 - c];
    double* W = Vn + q;
    HIPCHK(gram_f64(BVn, ldo, q, W, ldo, nact, n, part, C, nullptr, stream));
    double cmax = INFINITY;
    for (int pass = 0; pass < ortho_max_outer; ++pass) {
      HIPCHK(gen_proj_coef(C, q, nact, coef, cols, stream));
      HIPCHK(tsmm_f64(Vn, ldo, q + nact, coef, nact, W, ldo, n, nullptr, stream));
      stats.against_passes++;
      rc = ortho_run<double>(W, ldo, 0, nact, nullptr, false, tau);
      if (rc) return rc;
      HIPCHK(gram_f64(BVn, ldo, q, W, ldo, nact, n, part, C, nullptr, stream));
      HIPCHK(gen_proj_coef(C, q, nact, coef, cols, stream));
      const void* cp = nullptr;
      rc = readback(cols, sizeof(double), &cp);
      if (rc) return rc;
      cmax = *static_cast<const double*>(cp);
      if (cmax <= tau) break;
    }
    if (!(cmax <= tau)) stats.ortho_stalled++;
    // one application of B, one B-Cholesky reusing it, then A W
    rc = apply_b(W, ldo, nact, BVn + q, ldo);
    if (rc) return rc;
    rc = b_orthonormalize(W, BVn + q, ldo, nact);
    if (rc) return rc;
    rc = apply_op(W, ldo, nact, AV[1 - c] + q, ldo);
    if (rc) return rc;
    c = 1 - c;
    L = ldo;
    first = false;
  }
  res_evals.assign(th_t.begin(), th_t.begin() + m);
  res_resn.assign(rn_t.begin(), rn_t.begin() + m);
  stats.m_conv = m_conv;
  return LOBPCG_OK;
}

int lobpcg_ctx::solve(int k, double tol) {
  const auto t0 = std::chrono::steady_clock::now();
  if (op == kOpNone) return fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  const int m = block;
  if (m < 1) return fail(LOBPCG_ERR_BAD_STATE, "block size unknown: set an initial guess or query the workspace");
  if (k < 1 || k > m) return fail(LOBPCG_ERR_INVALID_ARG, "need 1 <= k <= block");
  if (!(tol > 0.0)) return fail(LOBPCG_ERR_INVALID_ARG, "tol must be > 0");
  int rc = ensure_layout(m);
  if (rc) return rc;
  std::memset(&stats, 0, sizeof(stats));
  stats.precision_switch_iter = -1;
  stats.learned_budget_iter = -1;
  stats.stall_checks = 0;
  have_result = false;
  if (pkind != LOBPCG_PRECOND_NONE) {
    rc = ensure_diag();
    if (rc) return rc;
  }
  if (pkind == LOBPCG_PRECOND_TRIDIAG) {
    rc = ensure_tri();
    if (rc) return rc;
  }
  if (pkind == LOBPCG_PRECOND_LEARNED) {
    if (lweights == nullptr)
      return fail(LOBPCG_ERR_BAD_STATE, "learned preconditioner selected but no weights set");
    rc = ensure_learned_features();
    if (rc) return rc;
  }
  double* V[2] = {dptr(lay.V[0]), dptr(lay.V[1])};
  double* AV[2] = {dptr(lay.AV[0]), dptr(lay.AV[1])};
  const bool dav = (method == LOBPCG_METHOD_DAVIDSON);
  if (dav && (precision != LOBPCG_PREC_FP64 || pkind == LOBPCG_PRECOND_LEARNED))
    return fail(LOBPCG_ERR_UNSUPPORTED, "block Davidson runs in fp64 with the Jacobi preconditioners");
  if (dav && dav_dim(m) < 2 * m)
    return fail(LOBPCG_ERR_INVALID_ARG, "Davidson basis limit below 2 * block");
  const int ld0 = dav ? dav_dim(m) : m;  // the basis of block Davidson is n x max_dim

  // ---- initial block (Alg. 1 input) ----
  if (X0 != nullptr) {
    HIPCHK(hipMemcpy2DAsync(V[0], sizeof(double) * ld0, X0, sizeof(double) * ldx0,
                            sizeof(double) * m, n, hipMemcpyDeviceToDevice, stream));
  } else if (!X0_host.empty()) {
    HIPCHK(hipMemcpy2DAsync(V[0], sizeof(double) * ld0, X0_host.data(), sizeof(double) * m,
                            sizeof(double) * m, n, hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
  } else {
    for (int j = 0; j < m; ++j) HIPCHK(fill_splitmix(V[0], ld0, j, j, n, kDefaultX0Seed, stream));
  }
  int iter = 0;
  PhaseOut po{};
  if (bop != kOpNone) {
    if (dav || precision != LOBPCG_PREC_FP64 ||
        (pkind != LOBPCG_PRECOND_NONE && pkind != LOBPCG_PRECOND_DIAG &&
         pkind != LOBPCG_PRECOND_DIAG_SIGNED))
      return fail(LOBPCG_ERR_UNSUPPORTED,
                  "the generalized problem runs LOBPCG in fp64 with the Jacobi preconditioners");
    if (pkind != LOBPCG_PRECOND_NONE) {
      rc = ensure_bdiag();
      if (rc) return rc;
    }
    rc = run_generalized(k, tol, iter, po);
    if (rc) return rc;
    res_k = k;
    res_X = reinterpret_cast<const double*>(po.X);
    res_ld = po.ld;
    have_result = true;
    stats.iterations = iter;
    stats.converged = po.converged ? 1 : 0;
    stats.ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return po.converged ? LOBPCG_OK : LOBPCG_NOT_CONVERGED;
  }
  if (dav) {
    rc = run_davidson(k, tol, iter, po);
    if (rc) return rc;
    res_k = k;
    res_X = reinterpret_cast<const double*>(po.X);
    res_ld = po.ld;
    have_result = true;
    stats.iterations = iter;
    stats.converged = po.converged ? 1 : 0;
    stats.ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return po.converged ? LOBPCG_OK : LOBPCG_NOT_CONVERGED;
  }
  if (precision == LOBPCG_PREC_FP32) {
    rc = ensure_op32();
    if (rc) return rc;
    float* V32[2] = {reinterpret_cast<float*>(ws + lay.V32[0]), reinterpret_cast<float*>(ws + lay.V32[1])};
    float* AV32[2] = {reinterpret_cast<float*>(ws + lay.AV32[0]),
                      reinterpret_cast<float*>(ws + lay.AV32[1])};
    HIPCHK(convert_f64_to_f32(V[0], m, V32[0], m, m, n, stream));
    rc = run_phase<float>(V32[0], V32[1], AV32[0], AV32[1], k, tol, true, iter, po);
    if (rc) return rc;
    // switch: promote the fp32 Ritz vectors; phase 2 re-orthonormalises them
    // in fp64 and recomputes A X explicitly (P is dropped)
    HIPCHK(convert_f32_to_f64(reinterpret_cast<const float*>(po.X), po.ld, V[0], m, m, n, stream));
    stats.precision_switch_iter = iter;
  }
  rc = run_phase<double>(V[0], V[1], AV[0], AV[1], k, tol, false, iter, po);
  if (rc) return rc;
  res_k = k;
  res_X = reinterpret_cast<const double*>(po.X);
  res_ld = po.ld;
  have_result = true;
  stats.iterations = iter;
  stats.converged = po.converged ? 1 : 0;
  stats.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return po.converged ? LOBPCG_OK : LOBPCG_NOT_CONVERGED;
}

// ===========================================================================
// C ABI

#define GUARD(h)                                          \
  if ((h) == nullptr) return LOBPCG_ERR_INVALID_ARG;      \
  hipError_t dev_e_ = hipSetDevice((h)->device);          \
  if (dev_e_ != hipSuccess) return (h)->hip_fail(dev_e_, "hipSetDevice");

extern "C" {

int lobpcg_create(int64_t n, int device, lobpcg_t* out) {
  if (out == nullptr) return LOBPCG_ERR_INVALID_ARG;
  *out = nullptr;
  if (n < 1) return LOBPCG_ERR_INVALID_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return LOBPCG_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return LOBPCG_ERR_DEVICE;
  lobpcg_ctx* h = new (std::nothrow) lobpcg_ctx();
  if (h == nullptr) return LOBPCG_ERR_DEVICE;
  h->n = n;
  h->device = device;
  // the static scratch of lobpcg_gram_noalloc: its device address is taken
  // here, once per device, so that the entry point itself does no set-up
  if (noalloc_setup(device, nullptr, &h->err) != LOBPCG_OK) {
    delete h;
    return LOBPCG_ERR_DEVICE;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&h->pinned), kPinnedBytes, hipHostMallocDefault) !=
      hipSuccess) {
    delete h;
    return LOBPCG_ERR_DEVICE;
  }
  // coherent host memory for the status posts; without it the status
  // read-backs take the copy + stream synchronisation path
  if (hipHostMalloc(reinterpret_cast<void**>(&h->post), kPostBytes + 256, hipHostMallocCoherent) ==
      hipSuccess) {
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&h->post_dev), h->post, 0) != hipSuccess) {
      (void)hipHostFree(h->post);
      h->post = nullptr;
      h->post_dev = nullptr;
    } else {
      h->post[kPostBytes / 4] = 0;
    }
  } else {
    h->post = nullptr;
    (void)hipGetLastError();
  }
  *out = h;
  return LOBPCG_OK;
}

int lobpcg_destroy(lobpcg_t h) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  hipSetDevice(h->device);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->post) (void)hipHostFree(h->post);
  if (h->lweights) (void)hipFree(h->lweights);
  delete h;
  return LOBPCG_OK;
}

int lobpcg_set_stream(lobpcg_t h, void* s) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  h->stream = reinterpret_cast<hipStream_t>(s);
  return LOBPCG_OK;
}

int lobpcg_set_option(lobpcg_t h, int key, double v) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  switch (key) {
    case LOBPCG_OPT_TAU_ORTHO:
      if (!(v > 0.0)) return h->fail(LOBPCG_ERR_INVALID_ARG, "tau must be > 0");
      h->tau = v;
      return LOBPCG_OK;
    case LOBPCG_OPT_MAX_ITER:
      if (v < 0 || v > 1e9) return h->fail(LOBPCG_ERR_INVALID_ARG, "bad max_iter");
      h->max_iter = (int)v;
      return LOBPCG_OK;
    case LOBPCG_OPT_PRECISION:
      if (v != LOBPCG_PREC_FP64 && v != LOBPCG_PREC_FP32)
        return h->fail(LOBPCG_ERR_INVALID_ARG, "bad precision");
      h->precision = (int)v;
      return LOBPCG_OK;
    case LOBPCG_OPT_ORTHO_MAX_PASSES:
      if (v < 1 || v > 50) return h->fail(LOBPCG_ERR_INVALID_ARG, "bad pass cap");
      h->ortho_max_inner = (int)v;
      return LOBPCG_OK;
    case LOBPCG_OPT_ORTHO_Y_MAX_PASSES:
      if (v < 1 || v > 50) return h->fail(LOBPCG_ERR_INVALID_ARG, "bad pass cap");
      h->ortho_max_outer = (int)v;
      return LOBPCG_OK;
    case LOBPCG_OPT_TRACE:
      h->trace = (v != 0.0);
      return LOBPCG_OK;
    case LOBPCG_OPT_LEARNED_BF16:
      h->learned_bf16 = (v != 0.0);
      return LOBPCG_OK;
    case LOBPCG_OPT_RR_JACOBI:
      h->rr_jacobi = (v != 0.0);
      return LOBPCG_OK;
    case LOBPCG_OPT_SHIFT_RETRIES:
      if (v < 0 || v > 20 || v != (int)v)
        return h->fail(LOBPCG_ERR_INVALID_ARG, "shift retries must be an integer in [0, 20]");
      h->shift_retries = (int)v;
      return LOBPCG_OK;
    case LOBPCG_OPT_METHOD:
      if (v != LOBPCG_METHOD_LOBPCG && v != LOBPCG_METHOD_DAVIDSON)
        return h->fail(LOBPCG_ERR_INVALID_ARG, "bad method");
      h->method = (int)v;
      h->lay_block = -1;  // the workspace layout depends on the method
      return LOBPCG_OK;
    case LOBPCG_OPT_DAVIDSON_MAX_DIM:
      if (v < 0 || v > kMaxP || v != (int)v)
        return h->fail(LOBPCG_ERR_INVALID_ARG, "Davidson basis limit must be an integer in [0, 96]");
      h->dav_max_dim = (int)v;
      h->lay_block = -1;
      return LOBPCG_OK;
    case LOBPCG_OPT_CHEAP_EXIT:
      h->cheap_exit = (v != 0.0);
      return LOBPCG_OK;
    case LOBPCG_OPT_LEARNED_BUDGET:
      if (v < 0 || v > 1e9 || v != (int)v)
        return h->fail(LOBPCG_ERR_INVALID_ARG, "learned budget must be a non-negative integer");
      h->learned_budget = (int)v;
      return LOBPCG_OK;
    case LOBPCG_OPT_SPMM_SLAB:
      if (v != 0 && v != 1)
        return h->fail(LOBPCG_ERR_INVALID_ARG, "CSR product path must be 0 or 1");
      h->slab_mode = (int)v;
      h->cwin_ready = false;
      h->lay_block = -1;  // the workspace layout holds the column windows in mode 1
      return LOBPCG_OK;
    case LOBPCG_OPT_STALL_WINDOW:
      if (v < 0 || v > 1e9 || v != (int)v)
        return h->fail(LOBPCG_ERR_INVALID_ARG, "stall window must be a non-negative integer");
      h->stall_window = (int)v;
      return LOBPCG_OK;
    case LOBPCG_OPT_FORCE_RESTARTS:
      if (v < 0 || v > 100 || v != (int)v)
        return h->fail(LOBPCG_ERR_INVALID_ARG, "forced restarts must be an integer in [0, 100]");
      h->force_restarts = (int)v;
      return LOBPCG_OK;
    default: return h->fail(LOBPCG_ERR_INVALID_ARG, "unknown option");
  }
}

int lobpcg_workspace_size(lobpcg_t h, int k, int block, int precision, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (block < 1 || block > kMaxBlock || 3 * (int64_t)block > h->n)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "need 1 <= block <= 32 and 3*block <= n");
  if (k < 1 || k > block) return h->fail(LOBPCG_ERR_INVALID_ARG, "need 1 <= k <= block");
  if (precision != LOBPCG_PREC_FP64 && precision != LOBPCG_PREC_FP32)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad precision");
  *bytes = h->plan(block, precision).total;
  if (h->X0 == nullptr && h->X0_host.empty()) h->block = block;
  return LOBPCG_OK;
}

int lobpcg_set_workspace(lobpcg_t h, void* p, size_t bytes) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (p == nullptr || (reinterpret_cast<uintptr_t>(p) % kAlign) != 0)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "workspace must be non-null and 256-byte aligned");
  h->ws = reinterpret_cast<char*>(p);
  h->ws_bytes = bytes;
  h->lay_block = -1;
  h->diag_ready = false;
  h->lfeat_ready = false;
  h->have_result = false;
  return LOBPCG_OK;
}

int lobpcg_set_operator_csr(lobpcg_t h, const int32_t* row_ptr, const int32_t* col,
                            const double* val, int64_t nnz) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (row_ptr == nullptr || (nnz > 0 && (col == nullptr || val == nullptr)) || nnz < 0 ||
      nnz > INT32_MAX)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad CSR arrays");
  {
    // validate the structure on the device before any kernel indexes with it
    hipError_t e = hipSetDevice(h->device);
    int* bad = nullptr;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&bad), sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), h->stream);
    if (e == hipSuccess) e = csr_check(row_ptr, col, h->n, nnz, bad, h->stream);
    int hb = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (bad != nullptr) (void)hipFree(bad);
    if (e != hipSuccess) return h->hip_fail(e, "CSR check");
    if (hb != 0)
      return h->fail(LOBPCG_ERR_INVALID_ARG,
                     "malformed CSR (row_ptr must rise from 0 to nnz, columns in [0, n))");
  }
  h->op = kOpCsr;
  h->rp = row_ptr;
  h->ci = col;
  h->val = val;
  h->nnz = nnz;
  h->cwin_ready = false;
  if (h->slab_mode == 1) h->lay_block = -1;  // the layout holds its column windows
  h->diag_ready = false;
  h->lfeat_ready = false;
  h->tri_ready = false;
  h->op32_ready = false;
  h->have_result = false;
  return LOBPCG_OK;
}

int lobpcg_set_operator_dense(lobpcg_t h, const double* A, int64_t lda) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (A == nullptr || lda < h->n) return h->fail(LOBPCG_ERR_INVALID_ARG, "bad dense operator");
  h->op = kOpDense;
  h->A = A;
  h->lda = lda;
  h->diag_ready = false;
  h->lfeat_ready = false;
  h->tri_ready = false;
  h->op32_ready = false;
  h->have_result = false;
  return LOBPCG_OK;
}

int lobpcg_set_operator_kronsum(lobpcg_t h, int64_t na, const double* A, const double* V) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (A == nullptr || V == nullptr || na < 1 || na * na != h->n)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad Kronecker-sum operator (need na*na == n)");
  h->op = kOpKron;
  h->A = A;
  h->na = na;
  h->Vpot = V;
  h->diag_ready = false;
  h->lfeat_ready = false;
  h->tri_ready = false;
  h->op32_ready = false;
  h->have_result = false;
  return LOBPCG_OK;
}

int lobpcg_set_operator_b_csr(lobpcg_t h, const int32_t* row_ptr, const int32_t* col,
                              const double* val, int64_t nnz) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  h->have_result = false;
  h->bdiag_ready = false;
  if (row_ptr == nullptr) {  // back to the standard problem
    h->bop = kOpNone;
    return LOBPCG_OK;
  }
  if (nnz < 1 || nnz > INT32_MAX || col == nullptr || val == nullptr)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad CSR arrays for B");
  {
    hipError_t e = hipSetDevice(h->device);
    int* bad = nullptr;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&bad), sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), h->stream);
    if (e == hipSuccess) e = csr_check(row_ptr, col, h->n, nnz, bad, h->stream);
    int hb = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (bad != nullptr) (void)hipFree(bad);
    if (e != hipSuccess) return h->hip_fail(e, "CSR check (B)");
    if (hb != 0) return h->fail(LOBPCG_ERR_INVALID_ARG, "malformed CSR for B");
  }
  h->bop = kOpCsr;
  h->brp = row_ptr;
  h->bci = col;
  h->bval = val;
  h->bnnz = nnz;
  return LOBPCG_OK;
}

int lobpcg_set_operator_b_dense(lobpcg_t h, const double* B, int64_t ldb) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  h->have_result = false;
  h->bdiag_ready = false;
  if (B == nullptr) {
    h->bop = kOpNone;
    return LOBPCG_OK;
  }
  if (ldb < h->n) return h->fail(LOBPCG_ERR_INVALID_ARG, "bad dense B");
  h->bop = kOpDense;
  h->Bd = B;
  h->ldb = ldb;
  return LOBPCG_OK;
}

int lobpcg_set_preconditioner(lobpcg_t h, int kind, const double* diag) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (kind != LOBPCG_PRECOND_NONE && kind != LOBPCG_PRECOND_DIAG &&
      kind != LOBPCG_PRECOND_DIAG_SIGNED && kind != LOBPCG_PRECOND_LEARNED &&
      kind != LOBPCG_PRECOND_TRIDIAG)
    return h->fail(LOBPCG_ERR_UNSUPPORTED, "preconditioner kind not available");
  h->pkind = kind;
  h->user_diag = diag;
  h->diag_ready = false;
  h->lfeat_ready = false;
  h->tri_ready = false;
  return LOBPCG_OK;
}

int lobpcg_set_learned_weights(lobpcg_t h, const float* w, int64_t count) {
  GUARD(h);
  if (w == nullptr || count != kMlpParams)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "learned weights: need LOBPCG_LEARNED_NPARAMS floats");
  if (h->lweights == nullptr) {
    hipError_t e = hipMalloc(&h->lweights, sizeof(float) * kMlpParams);
    if (e != hipSuccess) {
      h->lweights = nullptr;
      return h->hip_fail(e, "hipMalloc(weights)");
    }
  }
  // on the handle's stream (after any solve still reading the old weights),
  // complete before the host buffer is handed back
  hipError_t e = hipMemcpyAsync(h->lweights, w, sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "hipMemcpyAsync(weights)");
  return LOBPCG_OK;
}

int lobpcg_set_initial_guess(lobpcg_t h, const double* X0, int64_t ld, int block) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (X0 == nullptr || block < 1 || block > kMaxBlock || ld < block || 3 * (int64_t)block > h->n)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad initial guess (block <= 32, 3*block <= n)");
  h->X0 = X0;
  h->ldx0 = ld;
  h->block = block;
  h->X0_host.clear();
  h->X0_host.shrink_to_fit();
  return LOBPCG_OK;
}

int lobpcg_set_initial_guess_host(lobpcg_t h, const double* X0, int64_t ld, int block) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (X0 == nullptr || block < 1 || block > kMaxBlock || ld < h->n || 3 * (int64_t)block > h->n)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad initial guess (block <= 32, 3*block <= n, ld >= n)");
  try {
    h->X0_host.assign((size_t)h->n * block, 0.0);
  } catch (...) {
    return h->fail(LOBPCG_ERR_INVALID_ARG, "initial guess: host allocation failed");
  }
  // column-major in, row-major (the device layout) kept
  const int64_t n = h->n;
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < block; ++j) h->X0_host[(size_t)i * block + j] = X0[(size_t)j * ld + i];
  h->X0 = nullptr;
  h->ldx0 = 0;
  h->block = block;
  return LOBPCG_OK;
}

int lobpcg_solve(lobpcg_t h, int k, double tol) {
  GUARD(h);
  return h->solve(k, tol);
}

int lobpcg_get_eigenpairs(lobpcg_t h, int k, double* evals, double* evecs, int64_t ldv,
                          double* resnorms) {
  GUARD(h);
  if (!h->have_result) return h->fail(LOBPCG_ERR_BAD_STATE, "no solve result");
  if (k < 1 || k > (int)h->res_evals.size()) return h->fail(LOBPCG_ERR_INVALID_ARG, "bad k");
  for (int j = 0; j < k; ++j) {
    if (evals) evals[j] = h->res_evals[j];
    if (resnorms) resnorms[j] = h->res_resn[j];
  }
  if (evecs != nullptr) {
    if (ldv < k) return h->fail(LOBPCG_ERR_INVALID_ARG, "ldv < k");
    hipError_t e = copy_signfix(h->res_X, h->res_ld, k, h->n, evecs, ldv,
                                h->small_ptr<int64_t>(h->lay.pidx),
                                h->small_ptr<double>(h->lay.pval), h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "copy_signfix");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->hip_fail(e, "sync");
  }
  return LOBPCG_OK;
}

int lobpcg_get_eigenpairs_host(lobpcg_t h, int k, double* evals, double* evecs, int64_t ldv,
                               double* resnorms) {
  GUARD(h);
  if (!h->have_result) return h->fail(LOBPCG_ERR_BAD_STATE, "no solve result");
  if (k < 1 || k > (int)h->res_evals.size()) return h->fail(LOBPCG_ERR_INVALID_ARG, "bad k");
  if (evecs != nullptr && ldv < h->n) return h->fail(LOBPCG_ERR_INVALID_ARG, "ldv < n");
  for (int j = 0; j < k; ++j) {
    if (evals) evals[j] = h->res_evals[j];
    if (resnorms) resnorms[j] = h->res_resn[j];
  }
  if (evecs == nullptr) return LOBPCG_OK;
  // sign-fixed row-major copy staged in the AV area of the workspace (the
  // result itself lives in a V buffer), then transposed on the host
  double* stage = h->dptr(h->lay.AV[0]);
  hipError_t e = copy_signfix(h->res_X, h->res_ld, k, h->n, stage, k,
                              h->small_ptr<int64_t>(h->lay.pidx), h->small_ptr<double>(h->lay.pval),
                              h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "copy_signfix");
  std::vector<double> tmp;
  try {
    tmp.resize((size_t)h->n * k);
  } catch (...) {
    return h->fail(LOBPCG_ERR_INVALID_ARG, "get_eigenpairs_host: host allocation failed");
  }
  e = hipMemcpyAsync(tmp.data(), stage, sizeof(double) * tmp.size(), hipMemcpyDeviceToHost,
                     h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "eigenvector read-back");
  for (int64_t i = 0; i < h->n; ++i)
    for (int j = 0; j < k; ++j) evecs[(size_t)j * ldv + i] = tmp[(size_t)i * k + j];
  return LOBPCG_OK;
}

int lobpcg_get_stats(lobpcg_t h, lobpcg_stats* out) {
  if (h == nullptr || out == nullptr) return LOBPCG_ERR_INVALID_ARG;
  *out = h->stats;
  return LOBPCG_OK;
}

const char* lobpcg_status_string(int s) {
  switch (s) {
    case LOBPCG_OK: return "ok";
    case LOBPCG_NOT_CONVERGED: return "not converged (max_iter reached)";
    case LOBPCG_ERR_INVALID_ARG: return "invalid argument";
    case LOBPCG_ERR_BAD_STATE: return "bad call order";
    case LOBPCG_ERR_DEVICE: return "HIP device error";
    case LOBPCG_ERR_WORKSPACE: return "workspace missing or too small";
    case LOBPCG_ERR_ORTHO_FAILED: return "orthonormalisation failed";
    case LOBPCG_ERR_NONFINITE: return "non-finite values";
    case LOBPCG_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* lobpcg_last_error(lobpcg_t h) {
  if (h == nullptr) return "null handle";
  return h->err.c_str();
}

// ---- step entry points ----------------------------------------------------

int lobpcg_apply_operator(lobpcg_t h, const double* W, int64_t ldw, int ncols, double* Y,
                          int64_t ldy) {
  GUARD(h);
  if (W == nullptr || Y == nullptr || ncols < 1 || ncols > 64 || ldw < ncols || ldy < ncols)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad apply arguments");
  // with a workspace, plan its layout so that the operator can use its
  // scratch (the Kronecker operator packs strided blocks there); without
  // one, or if it is too small, the operator runs without scratch
  if (h->ws != nullptr) {
    const int m = h->lay_block > 0 ? h->lay_block : (h->block > 0 ? h->block : 1);
    if (h->ensure_layout(m) != LOBPCG_OK) h->err.clear();
  }
  return h->apply_op(W, ldw, ncols, Y, ldy);
}

static int need_ws(lobpcg_t h) {
  if (h->ws == nullptr) return h->fail(LOBPCG_ERR_WORKSPACE, "no workspace set");
  const int m = h->lay_block > 0 ? h->lay_block : (h->block > 0 ? h->block : 1);
  return h->ensure_layout(m);
}

int lobpcg_apply_operator_f32(lobpcg_t h, const float* W, int64_t ldw, int ncols, float* Y,
                              int64_t ldy) {
  GUARD(h);
  if (W == nullptr || Y == nullptr || ncols < 1 || ncols > 64 || ldw < ncols || ldy < ncols)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad apply arguments");
  if (h->op == kOpNone) return h->fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  if (h->precision != LOBPCG_PREC_FP32)
    return h->fail(LOBPCG_ERR_BAD_STATE, "the fp32 operator needs LOBPCG_OPT_PRECISION = LOBPCG_PREC_FP32");
  int rc = need_ws(h);
  if (rc) return rc;
  rc = h->ensure_op32();
  if (rc) return rc;
  return h->apply_op(W, ldw, ncols, Y, ldy);
}

int lobpcg_learned_apply(lobpcg_t h, double* R, int64_t ldr, int nact, const double* theta,
                         const int* mask) {
  GUARD(h);
  if (R == nullptr || theta == nullptr || nact < 1 || nact > 64 || ldr < nact)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad learned_apply arguments");
  if (h->lweights == nullptr) return h->fail(LOBPCG_ERR_BAD_STATE, "no learned weights set");
  if (h->op == kOpNone) return h->fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  int rc = need_ws(h);
  if (rc) return rc;
  rc = h->ensure_learned_features();
  if (rc) return rc;
  hipError_t e = mlp_apply_t(h->learned_bf16 != 0, R, ldr, nact, h->n, theta,
                             h->dptr(h->lay.diag), h->dptr(h->lay.rho),
                             h->small_ptr<double>(h->lay.lscale), h->lweights, mask, 0,
                             nullptr, reinterpret_cast<int*>(h->ws + h->lay.ltiles),
                             h->ltiles_cap(), h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "learned apply");
  return LOBPCG_OK;
}

int lobpcg_tridiag_apply(lobpcg_t h, double* R, int64_t ldr, int nact, const double* theta) {
  GUARD(h);
  if (R == nullptr || theta == nullptr || nact < 1 || nact > kMaxBlock || ldr < nact)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad tridiag_apply arguments");
  if (h->op == kOpNone) return h->fail(LOBPCG_ERR_BAD_STATE, "no operator set");
  if (h->pkind != LOBPCG_PRECOND_TRIDIAG)
    return h->fail(LOBPCG_ERR_BAD_STATE, "select LOBPCG_PRECOND_TRIDIAG first");
  int rc = need_ws(h);
  if (rc) return rc;
  rc = h->ensure_tri();
  if (rc) return rc;
  return h->tri_apply<double>(R, ldr, nact, theta);
}

int lobpcg_gram(lobpcg_t h, const double* A, int64_t lda, int p, const double* B, int64_t ldb,
                int q, double* C) {
  GUARD(h);
  if (A == nullptr || B == nullptr || C == nullptr || p < 1 || q < 1 || p > kGramMaxCols ||
      q > kGramMaxCols || lda < p || ldb < q)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad gram arguments");
  int rc = need_ws(h);
  if (rc) return rc;
  hipError_t e = gram_f64(A, lda, p, B, ldb, q, h->n, h->dptr(h->lay.part), C, nullptr, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "gram");
  return LOBPCG_OK;
}

int lobpcg_ortho(lobpcg_t h, double* X, int64_t ldx, int ncols, lobpcg_ortho_info* info) {
  GUARD(h);
  if (X == nullptr || ncols < 1 || ncols > kMaxBlock || ldx < ncols)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad ortho arguments");
  int rc = need_ws(h);
  if (rc) return rc;
  if (info) std::memset(info, 0, sizeof(*info));
  return h->ortho_run<double>(X, ldx, 0, ncols, info);
}

int lobpcg_ortho_against(lobpcg_t h, double* X, int64_t ldx, int ncols, const double* Y,
                         int64_t ldy, int ycols, lobpcg_ortho_info* info) {
  GUARD(h);
  if (X == nullptr || Y == nullptr || ncols < 1 || ncols > kMaxBlock || ycols < 0 ||
      ycols + ncols > kMaxP || ldx < ycols + ncols || ldx != ldy || X != Y + ycols)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "ortho_against needs X == Y + ycols in one buffer");
  int rc = need_ws(h);
  if (rc) return rc;
  if (info) std::memset(info, 0, sizeof(*info));
  return h->ortho_run<double>(const_cast<double*>(Y), ldx, ycols, ncols, info);
}

int lobpcg_small_eigh(lobpcg_t h, const double* a, int p, double* evals, double* evecs) {
  GUARD(h);
  if (a == nullptr || evals == nullptr || evecs == nullptr || p < 1 || p > kMaxP)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad small_eigh arguments");
  hipError_t e = small_eigh(a, p, evals, evecs, nullptr, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "small_eigh");
  return LOBPCG_OK;
}

int lobpcg_small_cholesky(lobpcg_t h, const double* M, int p, double* L, int* shifts) {
  GUARD(h);
  if (M == nullptr || L == nullptr || p < 1 || p > 64)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad small_cholesky arguments");
  int rc = need_ws(h);
  if (rc) return rc;
  int* info = h->small_ptr<int>(h->lay.info);
  hipError_t e = small_cholesky(M, p, L, info, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "small_cholesky");
  int hi[4];
  e = hipMemcpyAsync(hi, info, sizeof(hi), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "small_cholesky readback");
  if (shifts) *shifts = hi[2];
  return hi[0] == 0 ? LOBPCG_OK : h->fail(LOBPCG_ERR_ORTHO_FAILED, "all shifted retries failed");
}

int lobpcg_rotate(lobpcg_t h, const double* V, const double* AV, int64_t ldv, int p,
                  const double* U, int m, int q, const double* theta, int a0, double* Vout,
                  double* AVout, int64_t ldo, double* resnorm2) {
  GUARD(h);
  if (V == nullptr || AV == nullptr || U == nullptr || theta == nullptr || Vout == nullptr ||
      AVout == nullptr || resnorm2 == nullptr || p < 1 || p > kMaxP || m < 1 || q < m || q > 64 ||
      a0 < 0 || a0 > m || ldv < p || ldo < q + (m - a0))
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad rotate arguments");
  int rc = need_ws(h);
  if (rc) return rc;
  if (h->pkind != LOBPCG_PRECOND_NONE) {
    if (h->op == kOpNone && h->user_diag == nullptr)
      return h->fail(LOBPCG_ERR_BAD_STATE, "preconditioner needs diag(A)");
    rc = h->ensure_diag();
    if (rc) return rc;
  }
  RotateArgs ra{};
  ra.n = h->n;
  ra.ldv = ldv;
  ra.ldo = ldo;
  ra.p = p;
  ra.m = m;
  ra.q = q;
  ra.a0 = a0;
  ra.precond = h->pkind;
  ra.U = U;
  ra.theta = theta;
  ra.diag = h->dptr(h->lay.diag);
  ra.part = h->dptr(h->lay.part);
  ra.resnorm2 = resnorm2;
  hipError_t e = rotate_f64(V, AV, Vout, AVout, ra, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "rotate");
  return LOBPCG_OK;
}

}  // extern "C"
