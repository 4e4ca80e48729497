// lobpcg_gram_noalloc: the Gram product of lobpcg_gram for callers that
// cannot allocate (code under stream capture, serving loops): the
// partial sums of the n-reduction live in a file-scope device array instead
// of the caller's workspace.
//
// `scratch` holds kGramBlocks partial p x q sums for p, q <= 64 (16 MiB); the
// library takes its device address once per device (hipGetSymbolAddress, in
// lobpcg_create) and passes that address to the kernels.  Every call on one
// GPU uses the same array: calls that overlap on a GPU (two streams, two
// threads) race; calls in stream order do not, since the first stage writes
// every partial it uses before the second stage reads it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.h"

namespace {
constexpr int kNoAllocMaxCols = 64;
constexpr size_t kNoAllocParts = (size_t)lobpcg::kGramBlocks * kNoAllocMaxCols * kNoAllocMaxCols;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[kNoAllocParts];

namespace lobpcg {

// Device address of `scratch` on the current device (which must be
// `device`), looked up once per device.
int noalloc_setup(int device, double** out, std::string* err) {
  if (device < 0 || device >= kMaxDevices) {
    if (err) *err = "device index beyond the library's table";
    return LOBPCG_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      if (err) *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return LOBPCG_ERR_DEVICE;
    }
    g_scratch[device] = static_cast<double*>(p);
  }
  if (out) *out = g_scratch[device];
  return LOBPCG_OK;
}

}  // namespace lobpcg

extern "C" int lobpcg_gram_noalloc(lobpcg_t h, const double* A, int64_t lda, int p,
                                   const double* B, int64_t ldb, int q, double* C) {
  if (h == nullptr) return LOBPCG_ERR_INVALID_ARG;
  const hipError_t de = hipSetDevice(h->device);
  if (de != hipSuccess) return h->hip_fail(de, "hipSetDevice");
  if (A == nullptr || B == nullptr || C == nullptr || p < 1 || q < 1 || lda < p || ldb < q)
    return h->fail(LOBPCG_ERR_INVALID_ARG, "bad gram arguments");
  if (p > kNoAllocMaxCols || q > kNoAllocMaxCols)
    return h->fail(LOBPCG_ERR_INVALID_ARG,
                   "lobpcg_gram_noalloc: p and q must be <= 64 (its static scratch holds 512 "
                   "partial 64 x 64 sums); use lobpcg_gram for larger products");
  double* part = nullptr;
  const int rc = lobpcg::noalloc_setup(h->device, &part, &h->err);
  if (rc != LOBPCG_OK) return rc;
  const hipError_t e = lobpcg::gram_f64(A, lda, p, B, ldb, q, h->n, part, C, nullptr, h->stream);
  if (e != hipSuccess) return h->hip_fail(e, "gram (no-alloc)");
  return LOBPCG_OK;
}
