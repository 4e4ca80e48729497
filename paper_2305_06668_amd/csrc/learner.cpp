// Training driver of the learned preconditioner (C ABI part declared in
// include/lobpcg.h): snapshots of Ritz blocks, near-exact Jacobi-Davidson
// corrections by block MINRES, the training objective with its analytic
// gradient, and Adam.  Every vector operation runs in the kernels of
// k_learn.hip / k_mlp.hip / k_blas.hip and the operator of a solver handle;
// the host only sequences launches and reads back per-column scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

namespace lobpcg {
// k_learn.hip
size_t mr_state_bytes();
hipError_t gather_cols(const double* In, int64_t ldi, const int* cols, int nc, int64_t n,
                       double* Out, int64_t ldo, hipStream_t s);
hipError_t project_block(const double* In, int64_t ldi, const double* X, int64_t ldx, int m,
                         const double* C, int nc, int64_t n, double* Out, int64_t ldo,
                         hipStream_t s);
hipError_t coldots(int npairs, const double* const* P, const int64_t* ldp, const double* const* Q,
                   const int64_t* ldq, int nc, int64_t n, double* part, double* out,
                   hipStream_t s);
hipError_t objective_scalars(const double* dots, const double* theta, const double* ref, int nc,
                             double* coef, double* out, const double* sdots, double mu,
                             double* coef4, hipStream_t s);
hipError_t combine3(const double* R, const double* U, const double* Z, const double* Tau,
                    const double* coef, const double* coef4, int nc, int64_t n, double* Out,
                    hipStream_t s);
hipError_t residual_block(const double* X, const double* AX, const double* theta, int m,
                          int64_t n, double* R, hipStream_t s);
hipError_t mr_init(const double* bnorm2, int nc, void* st, hipStream_t s);
hipError_t mr_rhs(const double* Rc, const double* Xc, const double* dots, int nc, int64_t n,
                  double* Y, hipStream_t s);
hipError_t mr_scale(const double* Y, const void* st, int nc, int64_t n, double* V, hipStream_t s);
hipError_t mr_y(const double* AV, const double* V, const double* Xc, const double* theta,
                const double* dots, const double* R1, const void* st, int first, int nc, int64_t n,
                double* Y, hipStream_t s);
hipError_t mr_y2(const double* dots, const double* R2, void* st, int nc, int64_t n, double* Y,
                 hipStream_t s);
hipError_t mr_scalars(const double* alfa, const double* beta2, int nc, void* st, hipStream_t s);
hipError_t mr_update(const double* V, const double* W1, const double* W2, const void* st, int nc,
                     int64_t n, double* Wn, double* T, hipStream_t s);
}  // namespace lobpcg

using namespace lobpcg;

namespace {

constexpr int kDotPart = 1024 * 3 * kMaxBlock;  // coldots partials
constexpr int kNumWork = 8;                    // n x m work blocks

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform01(uint64_t& s) { return ((splitmix(s) >> 11) + 0.5) * 0x1.0p-53; }
double normal01(uint64_t& s) {
  const double u1 = uniform01(s), u2 = uniform01(s);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

struct Snapshot {
  lobpcg_ctx* h = nullptr;
  int64_t n = 0;
  int m = 0;
  double* X = nullptr;      // n x m
  double* R = nullptr;      // n x m
  double* theta = nullptr;  // m
  double* ref = nullptr;    // m: Delta of the MINRES corrections
  double* Tp = nullptr;     // n x m: (I - X X^T) times the MINRES corrections
  std::vector<double> th_h, rn_h, ref_h, relres_h;
};

}  // namespace

struct lobpcg_learner {
  int device = 0;
  float* w = nullptr;
  float* mo = nullptr;
  float* vo = nullptr;
  double* grad = nullptr;
  double* gpart = nullptr;  // kMlpBlocks * kMlpParams (also the Gram partials)
  double* small = nullptr;  // per-column scalars
  int* dcols = nullptr;
  int* dones = nullptr;     // mask of ones (Jacobi reference)
  void* mrst = nullptr;
  double* pinned = nullptr;
  int adam_t = 0;
  double mu = 0.0;  // weight of the supervised term (alignment with the corrections)
  std::vector<Snapshot> snaps;
  size_t work_elems = 0;
  double* work[kNumWork] = {};
  std::string err;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip_fail(hipError_t e, const char* where) {
    err = std::string(where) + ": " + hipGetErrorString(e);
    return LOBPCG_ERR_DEVICE;
  }
  int ensure_work(size_t elems);
  int decrease(Snapshot& S, const double* W0, bool run_mlp, const int* mask, int nc,
               const double* Rc, const double* thc, const double* refc, const double* Tc,
               bool want_grad, hipStream_t st);
  int objective(Snapshot& S, const int* cols, int nc, double* loss, double* grad_host,
                double* dl, double* dj, bool dev_grad = false);
  int minres(Snapshot& S, int maxit, double rtol);
  // small-area slots (doubles)
  double* s_dots() { return small; }                      // 3 * 64
  double* s_coef() { return small + 192; }                // 3 * 64
  double* s_out() { return small + 384; }                 // 2 * 64
  double* s_C() { return small + 512; }                   // 32 * 64
  double* s_thc() { return small + 512 + 2048; }          // 64
  double* s_refc() { return small + 512 + 2048 + 64; }    // 64
  double* s_sdots() { return small + 2688; }              // 2 * 64: u.tau, tau.tau
  double* s_coef4() { return small + 2816; }              // 64: coefficient of tau
  double* s_dpart() { return small + 4096; }              // kDotPart
};

int lobpcg_learner::ensure_work(size_t elems) {
  if (elems <= work_elems) return LOBPCG_OK;
  for (auto& p : work) {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
  work_elems = 0;
  for (auto& p : work) HIPCHK(hipMalloc(&p, sizeof(double) * elems));
  work_elems = elems;
  return LOBPCG_OK;
}

// Delta (and the loss terms) of the columns W (n x nc): W0 is copied into
// work[1] and, when run_mlp, transformed by the learned preconditioner from
// the residual columns Rc.  With Tc (the columns' projected corrections) and
// mu != 0 the supervised term joins the loss.  Leaves U = work[2],
// AU = work[3] and, with want_grad, the gradient of the loss in `grad`.
int lobpcg_learner::decrease(Snapshot& S, const double* W0, bool run_mlp, const int* mask, int nc,
                             const double* Rc, const double* thc, const double* refc,
                             const double* Tc, bool want_grad, hipStream_t st) {
  const int64_t n = S.n;
  const int m = S.m;
  lobpcg_ctx* h = S.h;
  double* W = work[1];
  double* U = work[2];
  double* AU = work[3];
  double* Z = work[4];
  double* G = work[5];
  HIPCHK(hipMemcpyAsync(W, W0, sizeof(double) * n * nc, hipMemcpyDeviceToDevice, st));
  if (run_mlp)
    HIPCHK(mlp_apply_f64(W, nc, nc, n, thc, h->dptr(h->lay.diag), h->dptr(h->lay.rho),
                         h->small_ptr<double>(h->lay.lscale), w, mask, 0, nullptr, st));
  HIPCHK(gram_f64(S.X, m, m, W, nc, nc, n, gpart, s_C(), nullptr, st));
  HIPCHK(project_block(W, nc, S.X, m, m, s_C(), nc, n, U, nc, st));
  int rc = h->apply_op(U, nc, nc, AU, nc);
  if (rc) return fail(rc, std::string("operator: ") + h->err);
  const double* P[3] = {U, Rc, U};
  const double* Q[3] = {U, U, AU};
  const int64_t ld[3] = {nc, nc, nc};
  HIPCHK(coldots(3, P, ld, Q, ld, nc, n, s_dpart(), s_dots(), st));
  const bool sup = Tc != nullptr && mu != 0.0;
  if (sup) {
    const double* Ps[2] = {U, Tc};
    const double* Qs[2] = {Tc, Tc};
    HIPCHK(coldots(2, Ps, ld, Qs, ld, nc, n, s_dpart(), s_sdots(), st));
  }
  HIPCHK(objective_scalars(s_dots(), thc, refc, nc, s_coef(), s_out(), sup ? s_sdots() : nullptr,
                           mu, s_coef4(), st));
  if (!want_grad) return LOBPCG_OK;
  HIPCHK(gram_f64(S.X, m, m, AU, nc, nc, n, gpart, s_C(), nullptr, st));
  HIPCHK(project_block(AU, nc, S.X, m, m, s_C(), nc, n, Z, nc, st));
  HIPCHK(combine3(Rc, U, Z, sup ? Tc : nullptr, s_coef(), s_coef4(), nc, n, G, st));
  HIPCHK(mlp_grad(Rc, G, nc, nc, n, thc, h->dptr(h->lay.diag), h->dptr(h->lay.rho),
                  h->small_ptr<double>(h->lay.lscale), w, gpart, grad, st));
  return LOBPCG_OK;
}

int lobpcg_learner::objective(Snapshot& S, const int* cols, int nc, double* loss,
                              double* grad_host, double* dl, double* dj, bool dev_grad) {
  const int64_t n = S.n;
  hipStream_t st = S.h->stream;
  double* Rc = work[0];
  int* hc = reinterpret_cast<int*>(pinned + 20000);
  std::memcpy(hc, cols, sizeof(int) * nc);
  HIPCHK(hipMemcpyAsync(dcols, hc, sizeof(int) * nc, hipMemcpyHostToDevice, st));
  HIPCHK(gather_cols(S.R, S.m, dcols, nc, n, Rc, nc, st));
  HIPCHK(gather_cols(S.theta, S.m, dcols, nc, 1, s_thc(), nc, st));
  HIPCHK(gather_cols(S.ref, S.m, dcols, nc, 1, s_refc(), nc, st));
  double* Tc = nullptr;
  if (mu != 0.0) {
    Tc = work[6];
    HIPCHK(gather_cols(S.Tp, S.m, dcols, nc, n, Tc, nc, st));
  }
  int rc = decrease(S, Rc, true, nullptr, nc, Rc, s_thc(), s_refc(), Tc,
                    dev_grad || grad_host != nullptr, st);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(pinned, s_out(), sizeof(double) * 2 * 64, hipMemcpyDeviceToHost, st));
  if (grad_host)
    HIPCHK(hipMemcpyAsync(pinned + 256, grad, sizeof(double) * kMlpParams, hipMemcpyDeviceToHost,
                          st));
  HIPCHK(hipStreamSynchronize(st));
  double L = 0.0;
  for (int j = 0; j < nc; ++j) L += pinned[nc + j];
  *loss = L / nc;
  if (dl) std::memcpy(dl, pinned, sizeof(double) * nc);
  if (grad_host) std::memcpy(grad_host, pinned + 256, sizeof(double) * kMlpParams);
  if (dj) {
    rc = decrease(S, Rc, true, dones, nc, Rc, s_thc(), nullptr, nullptr, false, st);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(pinned, s_out(), sizeof(double) * nc, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(dj, pinned, sizeof(double) * nc);
  }
  return LOBPCG_OK;
}

// Block MINRES (Paige-Saunders) on (I - x x^T)(A - theta I)(I - x x^T) t = -(I - x x^T) r
// for every column of the snapshot; the corrections' Delta go to S.ref.
int lobpcg_learner::minres(Snapshot& S, int maxit, double rtol) {
  const int64_t n = S.n;
  const int nc = S.m;
  hipStream_t st = S.h->stream;
  double* V = work[0];
  double* AV = work[1];
  double* R1 = work[2];
  double* R2 = work[3];
  double* Yn = work[4];
  double* Wc = work[5];
  double* W2 = work[6];
  double* T = work[7];
  const size_t bytes = sizeof(double) * n * nc;
  const int64_t ld[3] = {nc, nc, nc};
  {
    const double* P[1] = {S.X};
    const double* Q[1] = {S.R};
    HIPCHK(coldots(1, P, ld, Q, ld, nc, n, s_dpart(), s_dots(), st));
    HIPCHK(mr_rhs(S.R, S.X, s_dots(), nc, n, R2, st));
    const double* P2[1] = {R2};
    HIPCHK(coldots(1, P2, ld, P2, ld, nc, n, s_dpart(), s_dots(), st));
    HIPCHK(mr_init(s_dots(), nc, mrst, st));
  }
  HIPCHK(hipMemsetAsync(T, 0, bytes, st));
  HIPCHK(hipMemsetAsync(Wc, 0, bytes, st));
  HIPCHK(hipMemsetAsync(W2, 0, bytes, st));
  const size_t sb = mr_state_bytes();
  std::vector<char> hst(sb * nc);
  auto read_state = [&](int j, double* beta1, double* phibar) {
    const double* p = reinterpret_cast<const double*>(hst.data() + sb * j);
    *beta1 = p[0];
    *phibar = p[6];
  };
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    HIPCHK(mr_scale(R2, mrst, nc, n, V, st));
    int rc = S.h->apply_op(V, nc, nc, AV, nc);
    if (rc) return fail(rc, std::string("operator: ") + S.h->err);
    {
      const double* P[2] = {S.X, S.X};
      const double* Q[2] = {AV, V};
      HIPCHK(coldots(2, P, ld, Q, ld, nc, n, s_dpart(), s_dots(), st));
    }
    HIPCHK(mr_y(AV, V, S.X, S.theta, s_dots(), R1, mrst, it == 1, nc, n, Yn, st));
    {
      const double* P[1] = {V};
      const double* Q[1] = {Yn};
      HIPCHK(coldots(1, P, ld, Q, ld, nc, n, s_dpart(), s_coef(), st));  // alfa
    }
    HIPCHK(mr_y2(s_coef(), R2, mrst, nc, n, Yn, st));
    {
      const double* P[1] = {Yn};
      HIPCHK(coldots(1, P, ld, P, ld, nc, n, s_dpart(), s_dots(), st));  // beta^2
    }
    HIPCHK(mr_scalars(s_coef(), s_dots(), nc, mrst, st));
    // w1 = w2, w2 = w, w = (v - oldeps w1 - delta w2) denom, written over w1
    HIPCHK(mr_update(V, W2, Wc, mrst, nc, n, W2, T, st));
    std::swap(Wc, W2);  // Wc = new w, W2 = previous w
    double* old_r1 = R1;
    R1 = R2;
    R2 = Yn;
    Yn = old_r1;
    if (it % 10 == 0 || it == maxit) {
      HIPCHK(hipMemcpyAsync(hst.data(), mrst, sb * nc, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      bool all = true;
      for (int j = 0; j < nc; ++j) {
        double b1, pb;
        read_state(j, &b1, &pb);
        if (pb > rtol * b1) all = false;
      }
      if (all) break;
    }
  }
  HIPCHK(hipMemcpyAsync(hst.data(), mrst, sb * nc, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  S.relres_h.assign(nc, 0.0);
  for (int j = 0; j < nc; ++j) {
    double b1, pb;
    read_state(j, &b1, &pb);
    S.relres_h[j] = b1 > 0.0 ? pb / b1 : 0.0;
  }
  // the corrections' components outside span(X), kept for the supervised term
  HIPCHK(gram_f64(S.X, nc, nc, T, nc, nc, n, gpart, s_C(), nullptr, st));
  HIPCHK(project_block(T, nc, S.X, nc, nc, s_C(), nc, n, S.Tp, nc, st));
  // Delta of the corrections (no net); T lives in work[7], untouched by decrease
  int rc = decrease(S, T, false, nullptr, nc, S.R, S.theta, nullptr, nullptr, false, st);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(S.ref, s_out(), sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(pinned, s_out(), sizeof(double) * nc, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  S.ref_h.assign(pinned, pinned + nc);
  return LOBPCG_OK;
}

#define LGUARD(L)                                         \
  if ((L) == nullptr) return LOBPCG_ERR_INVALID_ARG;      \
  hipError_t dev_e_ = hipSetDevice((L)->device);          \
  if (dev_e_ != hipSuccess) return (L)->hip_fail(dev_e_, "hipSetDevice");

extern "C" {

int lobpcg_learner_create(int device, uint64_t seed, lobpcg_learner_t* out) {
  if (out == nullptr) return LOBPCG_ERR_INVALID_ARG;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return LOBPCG_ERR_DEVICE;
  auto* L = new lobpcg_learner();
  L->device = device;
  auto bad = [&](hipError_t e) {
    if (e == hipSuccess) return false;
    lobpcg_learner_destroy(L);
    return true;
  };
  if (bad(hipMalloc(&L->w, sizeof(float) * kMlpParams))) return LOBPCG_ERR_DEVICE;
  if (bad(hipMalloc(&L->mo, sizeof(float) * kMlpParams))) return LOBPCG_ERR_DEVICE;
  if (bad(hipMalloc(&L->vo, sizeof(float) * kMlpParams))) return LOBPCG_ERR_DEVICE;
  if (bad(hipMalloc(&L->grad, sizeof(double) * kMlpParams))) return LOBPCG_ERR_DEVICE;
  const size_t gp = std::max<size_t>((size_t)kMlpBlocks * kMlpParams,
                                     (size_t)kGramBlocks * kMaxBlock * 64);
  if (bad(hipMalloc(&L->gpart, sizeof(double) * gp))) return LOBPCG_ERR_DEVICE;
  if (bad(hipMalloc(&L->small, sizeof(double) * (4096 + kDotPart)))) return LOBPCG_ERR_DEVICE;
  if (bad(hipMalloc(&L->dcols, sizeof(int) * 64))) return LOBPCG_ERR_DEVICE;
  if (bad(hipMalloc(&L->dones, sizeof(int) * 64))) return LOBPCG_ERR_DEVICE;
  if (bad(hipMalloc(&L->mrst, mr_state_bytes() * 64))) return LOBPCG_ERR_DEVICE;
  if (bad(hipHostMalloc(reinterpret_cast<void**>(&L->pinned), sizeof(double) * 32768)))
    return LOBPCG_ERR_DEVICE;
  std::vector<int> ones(64, 1);
  if (bad(hipMemcpy(L->dones, ones.data(), sizeof(int) * 64, hipMemcpyHostToDevice)))
    return LOBPCG_ERR_DEVICE;
  // initial weights
  std::vector<float> w(kMlpParams, 0.0f);
  uint64_t s = seed;
  const int H = kMlpHidden, F = kMlpFeat;
  float* W1 = w.data();
  float* W2 = W1 + H * F + H;
  float* W3 = W2 + H * H + H;
  for (int i = 0; i < H * F; ++i) W1[i] = (float)(normal01(s) / std::sqrt((double)F));
  for (int i = 0; i < H * H; ++i) W2[i] = (float)(normal01(s) / std::sqrt((double)H));
  for (int i = 0; i < H; ++i) W3[i] = (float)(0.1 * normal01(s) / std::sqrt((double)H));
  w[kMlpParams - 1] = -3.0f;
  int rc = lobpcg_learner_set_weights(L, w.data(), kMlpParams);
  if (rc) {
    lobpcg_learner_destroy(L);
    return rc;
  }
  *out = L;
  return LOBPCG_OK;
}

int lobpcg_learner_destroy(lobpcg_learner_t L) {
  if (L == nullptr) return LOBPCG_ERR_INVALID_ARG;
  (void)hipSetDevice(L->device);
  for (auto& S : L->snaps) {
    (void)hipFree(S.X);
    (void)hipFree(S.R);
    (void)hipFree(S.theta);
    (void)hipFree(S.ref);
    (void)hipFree(S.Tp);
  }
  for (auto p : L->work)
    if (p) (void)hipFree(p);
  void* bufs[] = {L->w, L->mo, L->vo, L->grad, L->gpart, L->small, L->dcols, L->dones, L->mrst};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  if (L->pinned) (void)hipHostFree(L->pinned);
  delete L;
  return LOBPCG_OK;
}

int lobpcg_learner_set_supervision(lobpcg_learner_t L, double mu) {
  if (L == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (!(mu >= 0.0) || !(mu < INFINITY)) return L->fail(LOBPCG_ERR_INVALID_ARG, "mu must be finite and >= 0");
  L->mu = mu;
  return LOBPCG_OK;
}

int lobpcg_learner_set_weights(lobpcg_learner_t L, const float* w, int64_t count) {
  LGUARD(L);
  if (w == nullptr || count != kMlpParams)
    return L->fail(LOBPCG_ERR_INVALID_ARG, "need LOBPCG_LEARNED_NPARAMS weights");
  hipError_t e = hipMemcpy(L->w, w, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(L->mo, 0, sizeof(float) * kMlpParams);
  if (e == hipSuccess) e = hipMemset(L->vo, 0, sizeof(float) * kMlpParams);
  // the fills run on the null stream, which does not order work on
  // non-blocking streams: finish them before training can start elsewhere
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return L->hip_fail(e, "set_weights");
  L->adam_t = 0;
  return LOBPCG_OK;
}

int lobpcg_learner_get_weights(lobpcg_learner_t L, float* w, int64_t count) {
  LGUARD(L);
  if (w == nullptr || count != kMlpParams)
    return L->fail(LOBPCG_ERR_INVALID_ARG, "need LOBPCG_LEARNED_NPARAMS weights");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(w, L->w, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return L->hip_fail(e, "get_weights");
  return LOBPCG_OK;
}

int lobpcg_learner_add_snapshot(lobpcg_learner_t L, lobpcg_t h, const double* X, int64_t ldx,
                                int m, int minres_maxiter, double minres_rtol, int* index) {
  LGUARD(L);
  if (h == nullptr || X == nullptr || m < 1 || m > kMaxBlock || ldx < m || minres_maxiter < 0 ||
      !(minres_rtol > 0.0))
    return L->fail(LOBPCG_ERR_INVALID_ARG, "bad snapshot arguments");
  if (h->device != L->device) return L->fail(LOBPCG_ERR_INVALID_ARG, "handle on another device");
  if (h->op == kOpNone || h->ws == nullptr || h->block < 1)
    return L->fail(LOBPCG_ERR_BAD_STATE, "handle needs an operator and a workspace");
  int rc = h->ensure_layout(h->block);
  if (rc == LOBPCG_OK) rc = h->ensure_learned_features();
  if (rc) return L->fail(rc, std::string("handle: ") + h->err);
  const int64_t n = h->n;
  rc = L->ensure_work((size_t)n * kMaxBlock);
  if (rc) return rc;
  Snapshot S;
  S.h = h;
  S.n = n;
  S.m = m;
  hipStream_t st = h->stream;
  auto cleanup = [&]() {
    (void)hipFree(S.X);
    (void)hipFree(S.R);
    (void)hipFree(S.theta);
    (void)hipFree(S.ref);
    (void)hipFree(S.Tp);
  };
  hipError_t e = hipMalloc(&S.X, sizeof(double) * n * m);
  if (e == hipSuccess) e = hipMalloc(&S.R, sizeof(double) * n * m);
  if (e == hipSuccess) e = hipMalloc(&S.theta, sizeof(double) * m);
  if (e == hipSuccess) e = hipMalloc(&S.ref, sizeof(double) * m);
  if (e == hipSuccess) e = hipMalloc(&S.Tp, sizeof(double) * n * m);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(S.X, sizeof(double) * m, X, sizeof(double) * ldx, sizeof(double) * m, n,
                         hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) {
    cleanup();
    return L->hip_fail(e, "snapshot buffers");
  }
  // theta_j = x_j^T A x_j, R = A X - X diag(theta)
  double* AX = L->work[0];
  rc = h->apply_op(S.X, m, m, AX, m);
  if (rc) {
    cleanup();
    return L->fail(rc, std::string("operator: ") + h->err);
  }
  const int64_t ld[2] = {m, m};
  const double* P[2] = {S.X, S.X};
  const double* Q[2] = {AX, S.X};
  e = coldots(2, P, ld, Q, ld, m, n, L->s_dpart(), L->s_dots(), st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L->pinned, L->s_dots(), sizeof(double) * 2 * m, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    cleanup();
    return L->hip_fail(e, "snapshot theta");
  }
  S.th_h.resize(m);
  for (int j = 0; j < m; ++j) S.th_h[j] = L->pinned[j] / L->pinned[m + j];
  std::memcpy(L->pinned, S.th_h.data(), sizeof(double) * m);
  e = hipMemcpyAsync(S.theta, L->pinned, sizeof(double) * m, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = residual_block(S.X, AX, S.theta, m, n, S.R, st);
  const double* P1[1] = {S.R};
  if (e == hipSuccess) e = coldots(1, P1, ld, P1, ld, m, n, L->s_dpart(), L->s_dots(), st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L->pinned, L->s_dots(), sizeof(double) * m, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    cleanup();
    return L->hip_fail(e, "snapshot residual");
  }
  S.rn_h.resize(m);
  for (int j = 0; j < m; ++j) S.rn_h[j] = std::sqrt(L->pinned[j]);
  rc = L->minres(S, minres_maxiter, minres_rtol);
  if (rc) {
    cleanup();
    return rc;
  }
  L->snaps.push_back(S);
  if (index) *index = (int)L->snaps.size() - 1;
  return LOBPCG_OK;
}

int lobpcg_learner_snapshot_info(lobpcg_learner_t L, int snap, double* theta, double* resnorm,
                                 double* ref_decrease, double* minres_relres) {
  if (L == nullptr) return LOBPCG_ERR_INVALID_ARG;
  if (snap < 0 || snap >= (int)L->snaps.size())
    return L->fail(LOBPCG_ERR_INVALID_ARG, "no such snapshot");
  const Snapshot& S = L->snaps[snap];
  const size_t b = sizeof(double) * S.m;
  if (theta) std::memcpy(theta, S.th_h.data(), b);
  if (resnorm) std::memcpy(resnorm, S.rn_h.data(), b);
  if (ref_decrease) std::memcpy(ref_decrease, S.ref_h.data(), b);
  if (minres_relres) std::memcpy(minres_relres, S.relres_h.data(), b);
  return LOBPCG_OK;
}

int lobpcg_learner_objective(lobpcg_learner_t L, int snap, const int* cols, int ncols,
                             double* loss, double* grad, double* learned_decrease,
                             double* jacobi_decrease) {
  LGUARD(L);
  if (snap < 0 || snap >= (int)L->snaps.size())
    return L->fail(LOBPCG_ERR_INVALID_ARG, "no such snapshot");
  Snapshot& S = L->snaps[snap];
  if (cols == nullptr || loss == nullptr || ncols < 1 || ncols > S.m)
    return L->fail(LOBPCG_ERR_INVALID_ARG, "bad column list");
  for (int j = 0; j < ncols; ++j)
    if (cols[j] < 0 || cols[j] >= S.m) return L->fail(LOBPCG_ERR_INVALID_ARG, "bad column index");
  return L->objective(S, cols, ncols, loss, grad, learned_decrease, jacobi_decrease);
}

constexpr double kTrainResidualFloor = 1e-9;

int lobpcg_learner_train(lobpcg_learner_t L, int steps, int cols_per_step, double lr,
                         uint64_t seed, double* loss_first, double* loss_last) {
  LGUARD(L);
  if (L->snaps.empty()) return L->fail(LOBPCG_ERR_BAD_STATE, "no snapshots");
  if (steps < 1 || cols_per_step < 1 || !(lr > 0.0))
    return L->fail(LOBPCG_ERR_INVALID_ARG, "bad training arguments");
  // Columns whose residual is at rounding level carry no training signal:
  // their R (and so the learned step and the MINRES correction) is the
  // rounding of the product A X, ~eps sqrt(n) ||A||.  Only columns with
  // ||r_j|| > kTrainResidualFloor max(1, |theta_j|) are sampled.
  std::vector<std::vector<int>> elig(L->snaps.size());
  std::vector<int> usable;
  for (size_t q = 0; q < L->snaps.size(); ++q) {
    const Snapshot& S = L->snaps[q];
    for (int j = 0; j < S.m; ++j)
      if (S.rn_h[j] > kTrainResidualFloor * std::max(1.0, std::fabs(S.th_h[j]))) elig[q].push_back(j);
    if (!elig[q].empty()) usable.push_back((int)q);
  }
  if (usable.empty()) return L->fail(LOBPCG_ERR_BAD_STATE, "no snapshot column above the residual floor");
  uint64_t s = seed;
  const int tail = std::max(1, steps / 10);
  double first = 0.0, last = 0.0;
  for (int t = 0; t < steps; ++t) {
    const int q = usable[splitmix(s) % usable.size()];
    Snapshot& S = L->snaps[q];
    std::vector<int> perm(elig[q]);
    const int ne = (int)perm.size();
    const int nc = std::min(cols_per_step, ne);
    for (int j = 0; j < nc; ++j) std::swap(perm[j], perm[j + splitmix(s) % (ne - j)]);
    std::sort(perm.begin(), perm.begin() + nc);
    double loss = 0.0;
    int rc = L->objective(S, perm.data(), nc, &loss, nullptr, nullptr, nullptr, true);
    if (rc) return rc;
    L->adam_t++;
    hipError_t e = mlp_adam(L->w, L->mo, L->vo, L->grad, L->adam_t, lr, S.h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S.h->stream);
    if (e != hipSuccess) return L->hip_fail(e, "adam step");
    if (t < tail) first += loss / tail;
    if (t >= steps - tail) last += loss / tail;
  }
  if (loss_first) *loss_first = first;
  if (loss_last) *loss_last = last;
  return LOBPCG_OK;
}

const char* lobpcg_learner_last_error(lobpcg_learner_t L) {
  return L ? L->err.c_str() : "null learner";
}

}  // extern "C"
