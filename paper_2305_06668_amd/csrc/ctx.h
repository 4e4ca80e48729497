// Solver handle shared by the host driver (solver.cpp) and the training
// driver of the learned preconditioner (learner.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lobpcg.h"
#include "internal.h"

namespace lobpcg {

constexpr size_t kAlign = 256;
// controller rounds launched before the first check: two applications and
// the deciding controller round cover most calls (a no-op round still costs
// ~13 us of launches; a further check costs a ~30 us read-back)
constexpr int kOrthoRounds = 3;
constexpr size_t kReadbackBytes = 2048;  // resn2, theta (2 slots), info, learned flags
constexpr size_t kPostBytes = 4096;      // largest status block posted to the host
constexpr int kOrthoHardCap = 64;   // rounds before giving up
constexpr size_t kPinnedBytes = 1 << 16;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum OpKind { kOpNone = 0, kOpCsr = 1, kOpDense = 2, kOpKron = 3 };

struct Layout {
  size_t V[2], AV[2], diag, rho, ltiles, part, small, total;
  size_t kpack = 0;  // dense / Kronecker operator: n x 8 packed copy of a W block
  size_t cwin = 0;   // CSR operator: column window per block of the banded path (+ a flag)
  size_t dscr = 0;   // block Davidson: n x m scratch for the explicit product A X
  // tridiagonal preconditioner: off-diagonal, row off-sums, forward factors,
  // chunk boundary data
  size_t tri_e = 0, tri_off = 0, tri_scr = 0, tri_bnd = 0, tri_xb = 0;
  // generalized problem: B V (double-buffered like V) and diag(B)
  size_t BV[2] = {0, 0}, bdiag = 0;
  size_t V32[2], AV32[2], op32;  // mixed precision only (0 otherwise)
  // inside small (byte offsets)
  size_t a, rb, theta, U, G, coef, resn2, cols, info, ost, pidx, pval, eye, lflags, lscale;
};

}  // namespace lobpcg

using lobpcg::Layout;

struct lobpcg_ctx {
  int64_t n = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  // options
  double tau = 1e-14;
  int max_iter = 1000;
  int precision = LOBPCG_PREC_FP64;
  int ortho_max_inner = 6;
  int ortho_max_outer = 4;
  int trace = 0;
  int rr_jacobi = 0;     // Rayleigh-Ritz eigensolver: 0 tridiagonal, 1 Jacobi
  int shift_retries = 20;  // shifted Cholesky retries before SVQB (ortho controller)
  int force_restarts = 0;  // test hook: true checks that count as failed
  int cheap_exit = 0;      // cheap exits of the ortho loops
  int method = LOBPCG_METHOD_LOBPCG;
  int dav_max_dim = 0;     // 0: min(25 m, kMaxP)
  int learned_budget = 200;  // iterations that use the learned step (0: no limit)
  int stall_window = 20;     // fp64 phase: iterations without 1 % progress before a true check (0: off)
  int slab_mode = 0;         // CSR products: 0 gather kernels, 1 banded path (columns sorted)
  bool cwin_ready = false;   // the column windows of the current CSR operator are computed
  bool slab_ok = false;      // ... and the columns are sorted within rows
  int learned_bf16 = 1;  // learned preconditioner inference: layer 2 on bf16 MFMA
  // operator
  int op = lobpcg::kOpNone;
  const int32_t* rp = nullptr;
  const int32_t* ci = nullptr;
  const double* val = nullptr;
  int64_t nnz = 0;
  const double* A = nullptr;
  int64_t lda = 0;
  int64_t na = 0;
  const double* Vpot = nullptr;
  // the second operator B of A x = lambda B x (Sec. 3.3); kOpNone: standard
  int bop = lobpcg::kOpNone;
  const int32_t* brp = nullptr;
  const int32_t* bci = nullptr;
  const double* bval = nullptr;
  int64_t bnnz = 0;
  const double* Bd = nullptr;
  int64_t ldb = 0;
  bool bdiag_ready = false;
  // preconditioner
  int pkind = LOBPCG_PRECOND_DIAG;
  const double* user_diag = nullptr;
  bool diag_ready = false;
  float* lweights = nullptr;     // learned preconditioner weights (library-owned device copy)
  bool lfeat_ready = false;      // off-diagonal row sums and mean |diag| computed
  bool tri_ready = false;        // tridiagonal off-diagonal extracted
  double lscale_host = 0.0;
  // initial guess (device, row-major; or a host copy, row-major)
  const double* X0 = nullptr;
  int64_t ldx0 = 0;
  std::vector<double> X0_host;
  int block = 0;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout lay{};
  int lay_block = -1;
  // pinned host buffer
  char* pinned = nullptr;
  // results
  bool have_result = false;
  int res_k = 0;
  const double* res_X = nullptr;
  int64_t res_ld = 0;
  std::vector<double> res_evals, res_resn;
  lobpcg_stats stats{};
  std::string err;
  // fp32 operator copies (mixed precision) and the operator norm bound
  bool op32_ready = false;
  double norm_bound = -1.0;

  // coherent host memory (kPostBytes of data, then the sequence word) that a
  // kernel writes status blocks into; post_dev is its device address
  uint32_t* post = nullptr;
  uint32_t* post_dev = nullptr;
  uint32_t post_seq = 0;

  // ---- helpers ----
  double* dptr(size_t off) const { return reinterpret_cast<double*>(ws + off); }
  // super-tile flags of the bf16 learned transform: up to 64 columns
  int64_t ltiles_cap() const { return (n * 64 + lobpcg::kMlpSuper - 1) / lobpcg::kMlpSuper; }
  template <typename T> T* small_ptr(size_t off) const {
    return reinterpret_cast<T*>(ws + lay.small + off);
  }
  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip_fail(hipError_t e, const char* where) {
    err = std::string(where) + ": " + hipGetErrorString(e);
    return LOBPCG_ERR_DEVICE;
  }
  Layout plan(int m) const { return plan(m, precision); }
  Layout plan(int m, int prec) const;
  size_t op32_elems() const;
  int ensure_layout(int m);
  int apply_op(const double* W, int64_t ldw, int nc, double* Y, int64_t ldy);
  // brings `bytes` (a multiple of 4, at most kPostBytes) of device memory
  // at src to the host once the work queued before it has run; *out points
  // at the host copy until the next read-back
  int readback(const void* src, size_t bytes, const void** out);
  int apply_op(const float* W, int64_t ldw, int nc, float* Y, int64_t ldy);
  template <typename T>
  int ortho_run(T* base, int64_t ld, int ny, int nw, lobpcg_ortho_info* info, bool fold = false,
                double tau_run = -1.0);
  int ensure_diag();
  int ensure_learned_features();
  int ensure_tri();
  template <typename T>
  int tri_apply(T* R, int64_t ld, int nact, const double* theta);
  int ensure_op32();
  const int2* csr_slab_windows();
  int true_residuals(const double* X, int64_t ldx, int m, double* scratch, const double* theta_rr,
                     std::vector<double>& th, std::vector<double>& rn);
  struct PhaseOut {
    const void* X;  // final Ritz vectors of the phase (first m columns)
    int64_t ld;
    bool converged;
  };
  template <typename T>
  int run_phase(T* V0, T* V1, T* AV0, T* AV1, int k, double tol, bool low, int& iter,
                PhaseOut& out);
  int solve(int k, double tol);
  int dav_dim(int m) const {
    const int d = dav_max_dim > 0 ? dav_max_dim : 25 * m;
    return d < lobpcg::kMaxP ? d : lobpcg::kMaxP;
  }
  int run_davidson(int k, double tol, int& iter, PhaseOut& out);
  int apply_b(const double* W, int64_t ldw, int nc, double* Y, int64_t ldy);
  int ensure_bdiag();
  int b_orthonormalize(double* X, double* BX, int64_t ld, int nc);
  int run_generalized(int k, double tol, int& iter, PhaseOut& out);
};

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)
