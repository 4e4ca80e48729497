// Matrix-free Kronecker-sum operator H = A (x) I + I (x) A + diag(vec V)
// applied to a row-major block: vector entry (i, j) of column b lives at
// W[(i * na + j) * ldw + b], so
//   Y[i][j][b] = sum_k A[i][k] W[k][j][b] + sum_k A[j][k] W[i][k][b]
//              + V[i][j] W[i][j][b].
// For each column b both sums are dense products of na x na matrices,
// A W_b and W_b A (A symmetric), so the operator is two GEMMs sharing one
// accumulator: a workgroup owns an output tile of 32 i x 32 j x 8 columns
// and walks k in chunks of 16.  Every LDS operand tile is stored k-major
// ([k][i], [k][j], [b][k][j], [b][k][i]) so that the 16 lanes that feed one
// MFMA operand row read 16 consecutive values, with an XOR swizzle of the
// row position by k so that the four k rows a wave reads at once fall in
// different banks.  The next chunk is loaded into registers (as pairs of
// values) while the MFMAs of the current one run.  Each of the 4 waves owns
// two columns b and the four 16 x 16 (i, j) sub-tiles of each, and issues
// per 4-deep k step two MFMA 16x16x4 per sub-tile (one per term).  The tile
// is staged back through LDS so the diagonal term and the stores run along
// contiguous (j, b) rows.  4 na flops per output entry: na = 4096, 8 columns
// (n = 16.8M) is 2.2 TFLOP per application.
#include <algorithm>
#include <cstddef>
#include <cstdint>

#include "internal.h"

namespace lobpcg {

namespace {

constexpr int kTI = 32, kTJ = 32, kBB = 8, kKC = 16;

__device__ __forceinline__ d4 kmma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 kmma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct KAcc;
template <> struct KAcc<double> { typedef d4 type; };
template <> struct KAcc<float> { typedef f4 type; };
// accumulator register r of lane l holds row 4 r + l / 16 (f64) or
// 4 (l / 16) + r (f32) of the 16 x 16 tile, column l % 16
template <typename T> __device__ __forceinline__ int krow(int r, int lane);
template <> __device__ __forceinline__ int krow<double>(int r, int lane) { return 4 * r + (lane >> 4); }
template <> __device__ __forceinline__ int krow<float>(int r, int lane) { return 4 * (lane >> 4) + r; }

// position of element x of LDS row k (of the tile of column b): rows of 32
// values, swizzled so that (1) the rows k4 .. k4 + 3 read together by one
// MFMA operand load fall in different banks (fp64: 256-byte rows, halves
// swapped on odd k; fp32: 128-byte rows, halves swapped on k = 2, 3 mod 4)
// and (2) the staging stores, whose 16-lane groups span 4 column pairs and
// 4 k rows, spread over the banks (bits 1-3 permuted by b and k, which keeps
// the 16 values one MFMA operand row reads contiguous and pairs adjacent)
template <typename T> __device__ __forceinline__ int kswz(int x, int k, int b);
template <> __device__ __forceinline__ int kswz<double>(int x, int k, int b) {
  return x ^ ((k & 1) << 4) ^ (((k >> 1) & 1) << 1) ^ ((b >> 1) << 2);
}
template <> __device__ __forceinline__ int kswz<float>(int x, int k, int b) {
  return x ^ (((k >> 1) & 1) << 4) ^ ((b >> 1) << 2);
}

template <typename T>
struct alignas(16) KronSmem {
  T ai[kKC][kTI];          // A[i0 + ii][k0 + kk] at [kk][swz(ii)]
  T aj[kKC][kTJ];          // A[k0 + kk][j0 + jj] at [kk][swz(jj)]
  T xk[kBB][kKC][kTJ];     // W[(k0 + kk) na + j0 + jj][b0 + bb] at [bb][kk][swz(jj)]
  T xi[kBB][kKC][kTI];     // W[(i0 + ii) na + k0 + kk][b0 + bb] at [bb][kk][swz(ii)]
};

template <typename T> struct Pair { T x, y; };
template <> struct __attribute__((aligned(16))) Pair<double> { double x, y; };
template <> struct __attribute__((aligned(8))) Pair<float> { float x, y; };

// values staged per thread and chunk, in pairs: W for the A W_b term
// (16 k x 32 j x 4 column pairs), W for the W_b A term (32 i x 16 k x 4
// column pairs), A rows of the i tile (32 i x 8 k pairs), A rows of the k
// chunk (16 k x 16 j pairs)
constexpr int kPXK = kKC * kTJ * (kBB / 2) / 256;  // 8
constexpr int kPXI = kTI * kKC * (kBB / 2) / 256;  // 8
static_assert(kTI * (kKC / 2) == 256 && kKC * (kTJ / 2) == 256, "one A pair per thread");

// VEC: pairs are loaded as one aligned 2-value load (ldw, na even, W and A
// aligned); otherwise value by value.  Out-of-range (i, j, k, b) read as 0.
template <typename T, bool VEC>
__device__ __forceinline__ Pair<T> ld_pair(const T* __restrict__ p, bool v0, bool v1) {
  Pair<T> r;
  if (VEC && v1) {
    r = *reinterpret_cast<const Pair<T>*>(p);
  } else {
    r.x = v0 ? p[0] : T(0);
    r.y = v1 ? p[1] : T(0);
  }
  return r;
}

template <typename T, bool VEC>
struct KronStage {
  Pair<T> xk[kPXK], xi[kPXI], ai, aj;

  // nc: the columns of W that may be read (a zero-padded packed block
  // allows all 8)
  __device__ __forceinline__ void load(const T* __restrict__ A, const T* __restrict__ W,
                                       int64_t na, int64_t ldw, int nc, int64_t i0, int64_t j0,
                                       int b0, int64_t k0, int t) {
#pragma unroll
    for (int u = 0; u < kPXK; ++u) {
      const int q = t + 256 * u;
      const int bp = q & 3, jj = (q >> 2) & (kTJ - 1), kk = q >> 7;
      const int64_t k = k0 + kk, j = j0 + jj;
      const int b = b0 + 2 * bp;
      const bool in = k < na && j < na;
      xk[u] = ld_pair<T, VEC>(W + (k * na + j) * ldw + b, in && b < nc, in && b + 1 < nc);
    }
#pragma unroll
    for (int u = 0; u < kPXI; ++u) {
      const int q = t + 256 * u;
      const int bp = q & 3, kk = (q >> 2) & (kKC - 1), ii = q >> 6;
      const int64_t i = i0 + ii, k = k0 + kk;
      const int b = b0 + 2 * bp;
      const bool in = i < na && k < na;
      xi[u] = ld_pair<T, VEC>(W + (i * na + k) * ldw + b, in && b < nc, in && b + 1 < nc);
    }
    {
      const int kp = t & 7, ii = t >> 3;
      const int64_t i = i0 + ii, k = k0 + 2 * kp;
      ai = ld_pair<T, VEC>(A + i * na + k, i < na && k < na, i < na && k + 1 < na);
    }
    {
      const int jp = t & 15, kk = t >> 4;
      const int64_t k = k0 + kk, j = j0 + 2 * jp;
      aj = ld_pair<T, VEC>(A + k * na + j, k < na && j < na, k < na && j + 1 < na);
    }
  }

  __device__ __forceinline__ void store(KronSmem<T>& sm, int t) const {
#pragma unroll
    for (int u = 0; u < kPXK; ++u) {
      const int q = t + 256 * u;
      const int bp = q & 3, jj = (q >> 2) & (kTJ - 1), kk = q >> 7;
      const int x = kswz<T>(jj, kk, 2 * bp);
      sm.xk[2 * bp][kk][x] = xk[u].x;
      sm.xk[2 * bp + 1][kk][x] = xk[u].y;
    }
#pragma unroll
    for (int u = 0; u < kPXI; ++u) {
      const int q = t + 256 * u;
      const int bp = q & 3, kk = (q >> 2) & (kKC - 1), ii = q >> 6;
      const int x = kswz<T>(ii, kk, 2 * bp);
      sm.xi[2 * bp][kk][x] = xi[u].x;
      sm.xi[2 * bp + 1][kk][x] = xi[u].y;
    }
    {
      const int kp = t & 7, ii = t >> 3;
      sm.ai[2 * kp][kswz<T>(ii, 2 * kp, 0)] = ai.x;
      sm.ai[2 * kp + 1][kswz<T>(ii, 2 * kp + 1, 0)] = ai.y;
    }
    {
      const int jp = t & 15, kk = t >> 4;
      // the swizzle leaves bit 0 alone, so the pair stays adjacent and aligned
      *reinterpret_cast<Pair<T>*>(&sm.aj[kk][kswz<T>(2 * jp, kk, 0)]) = aj;
    }
  }
};

template <typename T, bool VEC>
__global__ __launch_bounds__(256, 2) void k_kron_mfma(const T* __restrict__ A,
                                                      const T* __restrict__ Vp, int64_t na,
                                                      const T* __restrict__ W, int64_t ldw,
                                                      T* __restrict__ Y, int64_t ldy, int nc,
                                                      int ncl) {
  typedef typename KAcc<T>::type AccT;
  __shared__ KronSmem<T> sm;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int64_t j0 = (int64_t)blockIdx.x * kTJ, i0 = (int64_t)blockIdx.y * kTI;
  const int b0 = blockIdx.z * kBB;
  AccT acc[2][2][2];  // [b local 2 wave + bw][si][sj]
#pragma unroll
  for (int bw = 0; bw < 2; ++bw)
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[bw][si][sj][e] = T(0);
  KronStage<T, VEC> st;
  st.load(A, W, na, ldw, ncl, i0, j0, b0, 0, t);
  st.store(sm, t);
  __syncthreads();
  for (int64_t k0 = 0; k0 < na; k0 += kKC) {
    // the next chunk's loads are in flight while this chunk's MFMAs run
    const bool more = k0 + kKC < na;
    if (more) st.load(A, W, na, ldw, ncl, i0, j0, b0, k0 + kKC, t);
    // k steps not unrolled: 228 registers (all four unrolled hold 256 and
    // spill, two unrolled run 2 % slower)
#pragma unroll 1
    for (int k4 = 0; k4 < kKC; k4 += 4) {
      const int kk = k4 + g;
      T ai[2], aj[2], xk[2][2], xi[2][2];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int x = kswz<T>(16 * s2 + r, kk, 0);
        ai[s2] = sm.ai[kk][x];
        aj[s2] = sm.aj[kk][x];
#pragma unroll
        for (int bw = 0; bw < 2; ++bw) {
          const int xb = kswz<T>(16 * s2 + r, kk, 2 * wave + bw);
          xk[bw][s2] = sm.xk[2 * wave + bw][kk][xb];
          xi[bw][s2] = sm.xi[2 * wave + bw][kk][xb];
        }
      }
      // A W_b: A-operand A[i][k], B-operand W_b[k][j]
#pragma unroll
      for (int bw = 0; bw < 2; ++bw)
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
          for (int sj = 0; sj < 2; ++sj) acc[bw][si][sj] = kmma(ai[si], xk[bw][sj], acc[bw][si][sj]);
      // W_b A: A-operand W_b[i][k], B-operand A[k][j]
#pragma unroll
      for (int bw = 0; bw < 2; ++bw)
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
          for (int sj = 0; sj < 2; ++sj) acc[bw][si][sj] = kmma(xi[bw][si], aj[sj], acc[bw][si][sj]);
    }
    __syncthreads();
    if (more) {
      st.store(sm, t);
      __syncthreads();
    }
  }
  // stage the tile through LDS (reusing the W areas) and store along (j, b)
  T* so = &sm.xk[0][0][0];  // [ii][jj][bb]: kTI * kTJ * kBB values = xk + xi
  static_assert(sizeof(sm.xk) + sizeof(sm.xi) >= sizeof(T) * kTI * kTJ * kBB, "staging area");
  static_assert(offsetof(KronSmem<T>, xi) == offsetof(KronSmem<T>, xk) + sizeof(sm.xk), "contiguous");
#pragma unroll
  for (int bw = 0; bw < 2; ++bw)
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ii = 16 * si + krow<T>(e, lane), jj = 16 * sj + r;
          so[(ii * kTJ + jj) * kBB + 2 * wave + bw] = acc[bw][si][sj][e];
        }
  __syncthreads();
  for (int q = t; q < kTI * kTJ * kBB; q += 256) {
    const int bb = q % kBB, jj = (q / kBB) % kTJ, ii = q / (kBB * kTJ);
    const int64_t i = i0 + ii, j = j0 + jj;
    if (i < na && j < na && b0 + bb < nc) {
      const int64_t e = i * na + j;
      Y[e * ldy + b0 + bb] = so[q] + Vp[e] * W[e * ldw + b0 + bb];
    }
  }
}

}  // namespace

// packs columns [0, nc) of W (n rows, leading dimension ldw) into out
// (n x 8, zero-padded): the MFMA kernel then reads whole 64-byte rows
template <typename T>
__global__ __launch_bounds__(256) void k_kron_pack8(const T* __restrict__ W, int64_t ldw, int nc,
                                                    int64_t n, T* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    Pair<T> v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q].x = (2 * q < nc) ? W[i * ldw + 2 * q] : T(0);
      v[q].y = (2 * q + 1 < nc) ? W[i * ldw + 2 * q + 1] : T(0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) reinterpret_cast<Pair<T>*>(out + i * 8)[q] = v[q];
  }
}

template <typename T>
static hipError_t kron_launch(const T* A, const T* Vp, int64_t na, const T* W, int64_t ldw, T* Y,
                              int64_t ldy, int nc, int ncl, hipStream_t s) {
  const dim3 grid((unsigned)((na + kTJ - 1) / kTJ), (unsigned)((na + kTI - 1) / kTI),
                  (unsigned)((nc + kBB - 1) / kBB));
  const bool vec = (ldw % 2 == 0) && (na % 2 == 0) &&
                   (reinterpret_cast<uintptr_t>(W) % (2 * sizeof(T)) == 0) &&
                   (reinterpret_cast<uintptr_t>(A) % (2 * sizeof(T)) == 0);
  if (vec)
    hipLaunchKernelGGL((k_kron_mfma<T, true>), grid, dim3(256), 0, s, A, Vp, na, W, ldw, Y, ldy, nc,
                       ncl);
  else
    hipLaunchKernelGGL((k_kron_mfma<T, false>), grid, dim3(256), 0, s, A, Vp, na, W, ldw, Y, ldy,
                       nc, ncl);
  return hipGetLastError();
}

// A block that is not already a compact 8-column one is packed first (per
// 8 columns) into `pack` (na^2 x 8, optional): strided rows cost the MFMA
// kernel half again its time (na = 4096: 64 ms at ld 24 against 43 ms).
template <typename T>
static hipError_t kron_any(const T* A, const T* Vp, int64_t na, const T* W, int64_t ldw, T* Y,
                           int64_t ldy, int nc, T* pack, hipStream_t s) {
  if (na < 1 || nc < 1) return hipErrorInvalidValue;
  const bool compact = ldw == 8 && nc == 8 && reinterpret_cast<uintptr_t>(W) % 16 == 0;
  if (pack == nullptr || compact) return kron_launch<T>(A, Vp, na, W, ldw, Y, ldy, nc, nc, s);
  const int64_t n = na * na;
  const int pgrid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  for (int c0 = 0; c0 < nc; c0 += 8) {
    const int m = std::min(8, nc - c0);
    hipLaunchKernelGGL((k_kron_pack8<T>), dim3(pgrid), dim3(256), 0, s, W + c0, ldw, m, n, pack);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = kron_launch<T>(A, Vp, na, pack, 8, Y + c0, ldy, m, 8, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
static hipError_t pack8_any(const T* W, int64_t ldw, int nc, int64_t n, T* out, hipStream_t s) {
  if (n < 1 || nc < 1 || nc > 8 || W == nullptr || out == nullptr) return hipErrorInvalidValue;
  const int pgrid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL((k_kron_pack8<T>), dim3(pgrid), dim3(256), 0, s, W, ldw, nc, n, out);
  return hipGetLastError();
}
hipError_t pack8_f64(const double* W, int64_t ldw, int nc, int64_t n, double* out, hipStream_t s) {
  return pack8_any<double>(W, ldw, nc, n, out, s);
}
hipError_t pack8_f32(const float* W, int64_t ldw, int nc, int64_t n, float* out, hipStream_t s) {
  return pack8_any<float>(W, ldw, nc, n, out, s);
}

hipError_t kronsum_apply_f64(const double* A, const double* Vp, int64_t na, const double* W,
                             int64_t ldw, double* Y, int64_t ldy, int ncols, double* pack,
                             hipStream_t s) {
  return kron_any<double>(A, Vp, na, W, ldw, Y, ldy, ncols, pack, s);
}
hipError_t kronsum_apply_f32(const float* A, const float* Vp, int64_t na, const float* W,
                             int64_t ldw, float* Y, int64_t ldy, int ncols, float* pack,
                             hipStream_t s) {
  return kron_any<float>(A, Vp, na, W, ldw, Y, ldy, ncols, pack, s);
}

}  // namespace lobpcg
