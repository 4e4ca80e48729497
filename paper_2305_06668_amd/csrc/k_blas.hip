// Tall-skinny block kernels of the LOBPCG step (Alg. 1-3 of arXiv:2305.06668):
//   * gram    C = A^T B over the n rows (the RR matrix V^T AV, the overlaps
//             X^T X and Y^T X of Alg. 2 / Alg. 3),
//   * tsmm    Out = In Coef with a small coefficient matrix (X L^-T of
//             Alg. 2, X - Y Y^T X of Alg. 3),
//   * rotate  [X P] = V [u_x u_p], [AX AP] = AV [u_x u_p], R = AX - X Theta,
//             W~ = T R in one pass (eq. neweigv, "Reuse of applications").
//
// All of them are HBM-streaming contractions whose short dimension (<= 96)
// is the RR subspace; they run on the fp64 (or fp32) MFMA 16x16x4 units with
// the tall dimension n as the reduction (Gram) or the M dimension (tsmm,
// rotate).  Row chunks are staged in LDS for the M-dimension kernels; the
// Gram reads its fragments straight from global memory (each 16-lane group
// reads 128 contiguous bytes of one row).  Reductions over n are two-stage
// with a fixed order, so results are bit-reproducible run to run.
#include "internal.h"

namespace lobpcg {

// ---------------------------------------------------------------------------
// MFMA helpers.  Operand layout of v_mfma_*_16x16x4 (64 lanes): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator register r of lane l
// holds D[row][l % 16] with row = 4 r + l / 16 for f64 and 4 (l / 16) + r for
// f32.

__device__ __forceinline__ d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct AccOf;
template <> struct AccOf<double> { typedef d4 type; };
template <> struct AccOf<float> { typedef f4 type; };

template <typename T> __device__ __forceinline__ int acc_row(int r, int lane);
template <> __device__ __forceinline__ int acc_row<double>(int r, int lane) { return 4 * r + (lane >> 4); }
template <> __device__ __forceinline__ int acc_row<float>(int r, int lane) { return 4 * (lane >> 4) + r; }

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Gram: stage 1.  Grid (nblk, ngroups).  Block b reduces rows [b*rpb, ...);
// group g owns output row-tiles [g*MTI, g*MTI + MTI) and every column tile.
// Each of the 4 waves takes every 4th 4-row step of the block's rows.

template <typename T, int MTI, int MTJ>
// occupancy bound for up to 3 x 3 tiles (the Rayleigh-Ritz Gram at m = 16):
// 3 waves per SIMD without spills (fp64 240 -> 168 registers); larger tile
// counts would spill, so they keep the default
__global__ __launch_bounds__(256, (MTI <= 3 && MTJ <= 3) ? 3 : 1) void k_gram_part(const T* __restrict__ A, int64_t lda, int p,
                                                   const T* __restrict__ B, int64_t ldb, int q,
                                                   int64_t n, int64_t rpb,
                                                   double* __restrict__ part,
                                                   const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  typedef typename AccOf<T>::type AccT;
  __shared__ double red[MTI * MTJ * 256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane >> 4, cc = lane & 15;
  const int ti0 = blockIdx.y * MTI;
  const int TI = (p + 15) >> 4, TJ = (q + 15) >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = min(n, r0 + rpb);

  int ca[MTI], cb[MTJ];
  bool va[MTI], vb[MTJ];
#pragma unroll
  for (int ti = 0; ti < MTI; ++ti) {
    ca[ti] = (ti0 + ti) * 16 + cc;
    va[ti] = (ti0 + ti < TI) && (ca[ti] < p);
  }
#pragma unroll
  for (int tj = 0; tj < MTJ; ++tj) {
    cb[tj] = tj * 16 + cc;
    vb[tj] = (tj < TJ) && (cb[tj] < q);
  }
  AccT acc[MTI][MTJ];
#pragma unroll
  for (int ti = 0; ti < MTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) acc[ti][tj] = AccT{0, 0, 0, 0};

  int64_t base = r0 + wave * 4;
  // four steps at a time: all fragments of the four steps are loaded before
  // their MFMAs, which keeps 4 (MTI + MTJ) loads in flight per lane
  constexpr int U = 4;
  for (; base + 16 * (U - 1) + 4 <= r1; base += 16 * U) {
    T a[U][MTI], b[U][MTJ];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = base + 16 * u + kr;
#pragma unroll
      for (int ti = 0; ti < MTI; ++ti) a[u][ti] = va[ti] ? A[row * lda + ca[ti]] : T(0);
#pragma unroll
      for (int tj = 0; tj < MTJ; ++tj) b[u][tj] = vb[tj] ? B[row * ldb + cb[tj]] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int ti = 0; ti < MTI; ++ti)
#pragma unroll
        for (int tj = 0; tj < MTJ; ++tj) acc[ti][tj] = mma(a[u][ti], b[u][tj], acc[ti][tj]);
  }
  // remaining steps whose 4 rows all exist: no row checks
  for (; base + 4 <= r1; base += 16) {
    const int64_t row = base + kr;
    T a[MTI], b[MTJ];
#pragma unroll
    for (int ti = 0; ti < MTI; ++ti) a[ti] = va[ti] ? A[row * lda + ca[ti]] : T(0);
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) b[tj] = vb[tj] ? B[row * ldb + cb[tj]] : T(0);
#pragma unroll
    for (int ti = 0; ti < MTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < MTJ; ++tj) acc[ti][tj] = mma(a[ti], b[tj], acc[ti][tj]);
  }
  // tail with row checks
  for (; base < r1; base += 16) {
    const int64_t row = base + kr;
    const bool rv = row < r1;
    T a[MTI], b[MTJ];
#pragma unroll
    for (int ti = 0; ti < MTI; ++ti) a[ti] = (rv && va[ti]) ? A[row * lda + ca[ti]] : T(0);
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) b[tj] = (rv && vb[tj]) ? B[row * ldb + cb[tj]] : T(0);
#pragma unroll
    for (int ti = 0; ti < MTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < MTJ; ++tj) acc[ti][tj] = mma(a[ti], b[tj], acc[ti][tj]);
  }

  // fixed-order reduction over the 4 waves
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int ti = 0; ti < MTI; ++ti)
#pragma unroll
        for (int tj = 0; tj < MTJ; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = (ti * MTJ + tj) * 256 + acc_row<T>(r, lane) * 16 + cc;
            const double v = (double)acc[ti][tj][r];
            red[idx] = (w == 0) ? v : red[idx] + v;
          }
    }
    __syncthreads();
  }
  const int nrow = min(MTI, TI - ti0) * 16;
  double* dst = part + (int64_t)blockIdx.x * p * q;
  for (int idx = threadIdx.x; idx < nrow * q; idx += 256) {
    const int il = idx / q, j = idx - il * q;
    const int i = ti0 * 16 + il;
    if (i < p) dst[i * q + j] = red[((il >> 4) * MTJ + (j >> 4)) * 256 + (il & 15) * 16 + (j & 15)];
  }
}

// Stage 2: C[o] = sum over blocks b of part[b][o], fixed order: block x owns
// 16 consecutive outputs; thread (s, o) with s = tid / 16 sums the blocks
// b = s, s + 16, s + 32, ... in order; the 16 slice sums are added in slice
// order.  Loads of one b are 16 consecutive doubles (coalesced).
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int nblk,
                                                   int pq, double* __restrict__ C,
                                                   const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  __shared__ double red[16][17];
  const int o = blockIdx.x * 16 + (threadIdx.x & 15);
  const int sl = threadIdx.x >> 4;
  double acc = 0.0;
  if (o < pq) {
    int b = sl;
    for (; b + 48 < nblk; b += 64) {
      const double v0 = part[(int64_t)b * pq + o];
      const double v1 = part[(int64_t)(b + 16) * pq + o];
      const double v2 = part[(int64_t)(b + 32) * pq + o];
      const double v3 = part[(int64_t)(b + 48) * pq + o];
      acc += v0;
      acc += v1;
      acc += v2;
      acc += v3;
    }
    for (; b < nblk; b += 16) acc += part[(int64_t)b * pq + o];
  }
  red[sl][threadIdx.x & 15] = acc;
  __syncthreads();
  if (threadIdx.x < 16 && o < pq) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += red[i][threadIdx.x];
    C[o] = t;
  }
}

static hipError_t sum_parts(const double* part, int nblk, int pq, double* C, const int* skip,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_sum_parts, dim3(cdiv(pq, 16)), dim3(256), 0, s, part, nblk, pq, C, skip);
  return hipGetLastError();
}

template <typename T, int MTI, int MTJ>
static hipError_t gram_launch(const T* A, int64_t lda, int p, const T* B, int64_t ldb, int q,
                              int64_t n, double* part, double* C, const int* skip, hipStream_t s) {
  int nblk = (int)std::min<int64_t>(kGramBlocks, (n + 63) / 64);
  if (nblk < 1) nblk = 1;
  int64_t rpb = (n + nblk - 1) / nblk;
  rpb = (rpb + 15) / 16 * 16;
  nblk = (int)((n + rpb - 1) / rpb);
  if (nblk < 1) nblk = 1;
  const int TI = (p + 15) / 16;
  dim3 grid(nblk, (TI + MTI - 1) / MTI);
  hipLaunchKernelGGL((k_gram_part<T, MTI, MTJ>), grid, dim3(256), 0, s, A, lda, p, B, ldb, q, n,
                     rpb, part, skip);
  return sum_parts(part, nblk, p * q, C, skip, s);
}

template <typename T>
static hipError_t gram_any(const T* A, int64_t lda, int p, const T* B, int64_t ldb, int q,
                           int64_t n, double* part, double* C, const int* skip, hipStream_t s) {
  if (p < 1 || q < 1 || p > kGramMaxCols || q > kGramMaxCols || n < 1) return hipErrorInvalidValue;
  // row-tile group size: every row tile when the accumulators fit (<= 16
  // 16x16 tiles per wave), else groups of 16 / TJ row tiles
  const int TI = (p + 15) / 16;
  switch ((q + 15) / 16) {
    case 1:
      switch (std::min(TI, 8)) {
        case 1: return gram_launch<T, 1, 1>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 2: return gram_launch<T, 2, 1>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 3: return gram_launch<T, 3, 1>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 4: return gram_launch<T, 4, 1>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 5: return gram_launch<T, 5, 1>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 6: return gram_launch<T, 6, 1>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 7: return gram_launch<T, 7, 1>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        default: return gram_launch<T, 8, 1>(A, lda, p, B, ldb, q, n, part, C, skip, s);
      }
    case 2:
      switch (std::min(TI, 8)) {
        case 1: return gram_launch<T, 1, 2>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 2: return gram_launch<T, 2, 2>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 3: return gram_launch<T, 3, 2>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 4: return gram_launch<T, 4, 2>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 5: return gram_launch<T, 5, 2>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 6: return gram_launch<T, 6, 2>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 7: return gram_launch<T, 7, 2>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        default: return gram_launch<T, 8, 2>(A, lda, p, B, ldb, q, n, part, C, skip, s);
      }
    case 3:
      switch (std::min(TI, 5)) {
        case 1: return gram_launch<T, 1, 3>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 2: return gram_launch<T, 2, 3>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 3: return gram_launch<T, 3, 3>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 4: return gram_launch<T, 4, 3>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        default: return gram_launch<T, 5, 3>(A, lda, p, B, ldb, q, n, part, C, skip, s);
      }
    case 4:
      switch (std::min(TI, 4)) {
        case 1: return gram_launch<T, 1, 4>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 2: return gram_launch<T, 2, 4>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 3: return gram_launch<T, 3, 4>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        default: return gram_launch<T, 4, 4>(A, lda, p, B, ldb, q, n, part, C, skip, s);
      }
    case 5:
      switch (std::min(TI, 3)) {
        case 1: return gram_launch<T, 1, 5>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        case 2: return gram_launch<T, 2, 5>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        default: return gram_launch<T, 3, 5>(A, lda, p, B, ldb, q, n, part, C, skip, s);
      }
    case 6:
      switch (std::min(TI, 2)) {
        case 1: return gram_launch<T, 1, 6>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        default: return gram_launch<T, 2, 6>(A, lda, p, B, ldb, q, n, part, C, skip, s);
      }
    case 7:
      switch (std::min(TI, 2)) {
        case 1: return gram_launch<T, 1, 7>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        default: return gram_launch<T, 2, 7>(A, lda, p, B, ldb, q, n, part, C, skip, s);
      }
    case 8:
      switch (std::min(TI, 2)) {
        case 1: return gram_launch<T, 1, 8>(A, lda, p, B, ldb, q, n, part, C, skip, s);
        default: return gram_launch<T, 2, 8>(A, lda, p, B, ldb, q, n, part, C, skip, s);
      }
  }
  return hipErrorInvalidValue;
}

hipError_t gram_f64(const double* A, int64_t lda, int p, const double* B, int64_t ldb, int q,
                    int64_t n, double* part, double* C, const int* skip, hipStream_t s) {
  return gram_any<double>(A, lda, p, B, ldb, q, n, part, C, skip, s);
}
hipError_t gram_f32(const float* A, int64_t lda, int p, const float* B, int64_t ldb, int q,
                    int64_t n, double* part, double* C, const int* skip, hipStream_t s) {
  return gram_any<float>(A, lda, p, B, ldb, q, n, part, C, skip, s);
}

// ---------------------------------------------------------------------------
// Staging of a 64-row chunk (rows row0 .. row0+rows-1, p columns) into LDS
// with an odd row stride p+1 (no bank conflicts on the column-wise fragment
// reads).

// 16-byte vector of T
template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct Vec16<float> { typedef float __attribute__((ext_vector_type(4))) type; };

// Rows of p elements at stride ld starting at a 16-byte aligned address
// with p and ld multiples of the vector width: the chunk is then read as
// 16-byte vectors (6 per thread for 64 x 48 fp64), all issued before the
// LDS stores.  Rows past `rows` are zero-filled like the scalar path.
template <typename T>
__device__ __forceinline__ bool stage_rows_vec(const T* __restrict__ In, int64_t ld, int p,
                                               int64_t row0, int rows, T* __restrict__ tile) {
  typedef typename Vec16<T>::type V;
  constexpr int VE = 16 / sizeof(T);
  constexpr int B = 8;
  if (p % VE != 0 || ld % VE != 0 || (reinterpret_cast<uintptr_t>(In) & 15) != 0) return false;
  const int ldt = p + 1;
  const int pv = p / VE;
  const int total = 64 * pv;
  for (int base = threadIdx.x; base < total; base += 256 * B) {
    V v[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int idx = base + 256 * i;
      const int r = idx / pv, cv = idx - r * pv;
      if (idx < total && r < rows)
        v[i] = *reinterpret_cast<const V*>(In + (row0 + r) * ld + cv * VE);
      else
        for (int e = 0; e < VE; ++e) v[i][e] = T(0);
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int idx = base + 256 * i;
      if (idx < total) {
        const int r = idx / pv, cv = idx - r * pv;
#pragma unroll
        for (int e = 0; e < VE; ++e) tile[r * ldt + cv * VE + e] = v[i][e];
      }
    }
  }
  return true;
}

// Rows 0 .. rows-1 of an LDS tile (ncols elements at stride ldt) to global
// rows row0.. at stride ld: 16-byte vector stores when the global rows are
// aligned for them, else one element per thread and step.
template <typename T>
__device__ __forceinline__ void write_rows(const T* __restrict__ tile, int ldt, int ncols, int rows,
                                           T* __restrict__ Out, int64_t ld, int64_t row0) {
  typedef typename Vec16<T>::type V;
  constexpr int VE = 16 / sizeof(T);
  if (ncols % VE == 0 && ld % VE == 0 && (reinterpret_cast<uintptr_t>(Out) & 15) == 0) {
    const int cvn = ncols / VE;
    for (int idx = threadIdx.x; idx < rows * cvn; idx += 256) {
      const int r = idx / cvn, cv = idx - r * cvn;
      V v;
#pragma unroll
      for (int e = 0; e < VE; ++e) v[e] = tile[r * ldt + cv * VE + e];
      *reinterpret_cast<V*>(Out + (row0 + r) * ld + cv * VE) = v;
    }
  } else {
    for (int idx = threadIdx.x; idx < rows * ncols; idx += 256) {
      const int r = idx / ncols, c = idx - r * ncols;
      Out[(row0 + r) * ld + c] = tile[r * ldt + c];
    }
  }
}

template <typename T>
__device__ __forceinline__ void stage_rows(const T* __restrict__ In, int64_t ld, int p,
                                           int64_t row0, int rows, T* __restrict__ tile) {
  if (stage_rows_vec<T>(In, ld, p, row0, rows, tile)) return;
  // batches of 12 independent loads per thread before their LDS stores, so
  // that many global loads are in flight per thread.  Element idx of the
  // tile is (idx / p, idx % p); the thread's (row, column) is divided out
  // once and then advanced by 256 elements (dr rows and dc columns, with a
  // carry) per step, so no division sits in the loop.
  const int ldt = p + 1;
  const int total = 64 * p;
  constexpr int B = 12;
  const int dr = 256 / p, dc = 256 - dr * p;
  int r = threadIdx.x / p, c = threadIdx.x - (threadIdx.x / p) * p;
  for (int base = threadIdx.x; base < total; base += 256 * B) {
    T v[B];
    int rr[B], cc[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      rr[i] = r;
      cc[i] = c;
      const int idx = base + 256 * i;
      v[i] = (idx < total && r < rows) ? In[(row0 + r) * ld + c] : T(0);
      r += dr;
      c += dc;
      if (c >= p) {
        c -= p;
        ++r;
      }
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int idx = base + 256 * i;
      if (idx < total) tile[rr[i] * ldt + cc[i]] = v[i];
    }
  }
}

// ---------------------------------------------------------------------------
// ortho apply: one streaming pass of ortho(W; Y) (Alg. 2 / Alg. 3).  With
// base = [Y | W] (nr = ny + nw columns, leading dimension ld):
//   W <- [Y W] coef                (in place; coef is (ny + nw) x nw)
//   part[block] = [Y W]^T W        (of the NEW W, per-block partial)
// The new W rows are written back into the LDS tile so that the overlap is
// accumulated with MFMA straight from LDS (K = 4 rows per MFMA).  Skips
// itself when the controller has finished (st->done), and the overlap when
// the controller does not need it (st->no_gram: a cheap exit, or a final
// diagonal scaling).

template <typename T, int MTI, int MTJ>
// 4 waves per SIMD for one column tile and up to 5 row tiles (fp64 136 -> 108
// registers, no spills); wider instances would spill and keep the default
__global__ __launch_bounds__(256, (MTJ == 1 && MTI <= 5) ? 4 : 1) void k_ortho_apply(T* base, int64_t ld, int ny, int nw,
                                                     const double* __restrict__ coef,
                                                     const OrthoState* __restrict__ st, int64_t n,
                                                     double* __restrict__ part) {
  typedef typename AccOf<T>::type AccT;
  if (st->done) return;
  const int w_only = st->w_only;
  const bool gram = st->no_gram == 0;  // the controller may not need the overlap
  const int nr = ny + nw;
  extern __shared__ double smem_d[];
  double* red = smem_d;                          // MTI * MTJ * 256 doubles
  T* cf = reinterpret_cast<T*>(red + MTI * MTJ * 256);
  T* tile = cf + ((nr * nw + 1) & ~1);
  const int ldt = nr + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, cc = lane & 15;
  for (int i = threadIdx.x; i < nr * nw; i += 256) cf[i] = (T)coef[i];
  AccT G[MTI][MTJ];
#pragma unroll
  for (int I = 0; I < MTI; ++I)
#pragma unroll
    for (int J = 0; J < MTJ; ++J) G[I][J] = AccT{0, 0, 0, 0};
  const int kbeg = w_only ? (ny & ~3) : 0;  // coefficient rows < ny are zero then
  const int64_t nchunks = (n + 63) / 64;
  for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    __syncthreads();
    const int64_t row0 = chunk * 64;
    const int rows = (int)min<int64_t>(64, n - row0);
    stage_rows<T>(base, ld, nr, row0, rows, tile);
    __syncthreads();
    AccT acc[MTJ];
#pragma unroll
    for (int J = 0; J < MTJ; ++J) acc[J] = AccT{0, 0, 0, 0};
    const int arow = wave * 16 + cc;
    for (int k = kbeg; k < nr; k += 4) {
      const int kk = k + g;
      const bool kv = kk < nr;
      const T a = kv ? tile[arow * ldt + kk] : T(0);
#pragma unroll
      for (int J = 0; J < MTJ; ++J) {
        const int col = J * 16 + cc;
        const T b = (kv && col < nw) ? cf[kk * nw + col] : T(0);
        acc[J] = mma(a, b, acc[J]);
      }
    }
    __syncthreads();  // every wave is done reading the old W columns
#pragma unroll
    for (int J = 0; J < MTJ; ++J) {
      const int col = J * 16 + cc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wave * 16 + acc_row<T>(r, lane);
        if (rl < rows && col < nw) {
          const T v = (T)acc[J][r];
          base[(row0 + rl) * ld + ny + col] = v;
          tile[rl * ldt + ny + col] = v;
        }
      }
    }
    if (!gram) continue;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rl = wave * 16 + 4 * r + g;  // K = 4 rows per MFMA, any row order
      T bj[MTJ];
#pragma unroll
      for (int J = 0; J < MTJ; ++J) {
        const int cj = J * 16 + cc;
        bj[J] = (cj < nw) ? tile[rl * ldt + ny + cj] : T(0);
      }
#pragma unroll
      for (int I = 0; I < MTI; ++I) {
        const int ci = I * 16 + cc;
        const T ai = (ci < nr) ? tile[rl * ldt + ci] : T(0);
#pragma unroll
        for (int J = 0; J < MTJ; ++J) G[I][J] = mma(ai, bj[J], G[I][J]);
      }
    }
  }
  if (!gram) return;
  // fixed-order reduction over the waves, then the block partial
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int I = 0; I < MTI; ++I)
#pragma unroll
        for (int J = 0; J < MTJ; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = (I * MTJ + J) * 256 + acc_row<T>(r, lane) * 16 + cc;
            const double v = (double)G[I][J][r];
            red[idx] = (w == 0) ? v : red[idx] + v;
          }
    }
    __syncthreads();
  }
  double* dst = part + (int64_t)blockIdx.x * nr * nw;
  for (int idx = threadIdx.x; idx < nr * nw; idx += 256) {
    const int i = idx / nw, j = idx - i * nw;
    dst[idx] = red[((i >> 4) * MTJ + (j >> 4)) * 256 + (i & 15) * 16 + (j & 15)];
  }
}

template <typename T, int MTI, int MTJ>
static hipError_t ortho_apply_launch(T* base, int64_t ld, int ny, int nw, const double* coef,
                                     const OrthoState* st, int64_t n, double* part, double* G,
                                     hipStream_t s) {
  static bool attr = false;
  const int nr = ny + nw;
  const size_t sm = sizeof(double) * (size_t)(MTI * MTJ * 256) +
                    sizeof(T) * (size_t)(((nr * nw + 1) & ~1) + 64 * (nr + 1));
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_ortho_apply<T, MTI, MTJ>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
    (void)hipGetLastError();
    attr = true;
  }
  // up to 4 workgroups per CU (the partials, grid x nr x nw doubles, fit
  // the workspace's kStreamBlocks x kMaxP x kMaxBlock for every nr <= kMaxP,
  // nw <= kMaxBlock); 512 left registers and LDS for 4 - 5 per CU unused
  const int64_t nchunks = (n + 63) / 64;
  const int grid = (int)std::min<int64_t>(nchunks, kStreamBlocks);
  hipLaunchKernelGGL((k_ortho_apply<T, MTI, MTJ>), dim3(grid), dim3(256), sm, s, base, ld, ny, nw,
                     coef, st, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return sum_parts(part, grid, nr * nw, G, &st->skip_sum, s);
}

template <typename T>
static hipError_t ortho_apply_any(T* base, int64_t ld, int ny, int nw, const double* coef,
                                  const OrthoState* st, int64_t n, double* part, double* G,
                                  hipStream_t s) {
  const int nr = ny + nw;
  if (nw < 1 || nw > kMaxBlock || ny < 0 || nr > kMaxP || n < 1) return hipErrorInvalidValue;
  const int TI = (nr + 15) / 16;
  if (nw <= 16) {
    switch (TI) {
      case 1: return ortho_apply_launch<T, 1, 1>(base, ld, ny, nw, coef, st, n, part, G, s);
      case 2: return ortho_apply_launch<T, 2, 1>(base, ld, ny, nw, coef, st, n, part, G, s);
      case 3: return ortho_apply_launch<T, 3, 1>(base, ld, ny, nw, coef, st, n, part, G, s);
      case 4: return ortho_apply_launch<T, 4, 1>(base, ld, ny, nw, coef, st, n, part, G, s);
      case 5: return ortho_apply_launch<T, 5, 1>(base, ld, ny, nw, coef, st, n, part, G, s);
      default: return ortho_apply_launch<T, 6, 1>(base, ld, ny, nw, coef, st, n, part, G, s);
    }
  }
  switch (TI) {
    case 2: return ortho_apply_launch<T, 2, 2>(base, ld, ny, nw, coef, st, n, part, G, s);
    case 3: return ortho_apply_launch<T, 3, 2>(base, ld, ny, nw, coef, st, n, part, G, s);
    case 4: return ortho_apply_launch<T, 4, 2>(base, ld, ny, nw, coef, st, n, part, G, s);
    case 5: return ortho_apply_launch<T, 5, 2>(base, ld, ny, nw, coef, st, n, part, G, s);
    default: return ortho_apply_launch<T, 6, 2>(base, ld, ny, nw, coef, st, n, part, G, s);
  }
}

hipError_t ortho_apply_f64(double* base, int64_t ld, int ny, int nw, const double* coef,
                           const OrthoState* st, int64_t n, double* part, double* G,
                           hipStream_t s) {
  return ortho_apply_any<double>(base, ld, ny, nw, coef, st, n, part, G, s);
}
hipError_t ortho_apply_f32(float* base, int64_t ld, int ny, int nw, const double* coef,
                           const OrthoState* st, int64_t n, double* part, double* G,
                           hipStream_t s) {
  return ortho_apply_any<float>(base, ld, ny, nw, coef, st, n, part, G, s);
}

// ---------------------------------------------------------------------------
// tsmm: Out (n x q) = In (n x p) Coef (p x q).  Persistent grid; each block
// loads Coef once (converted to T) and walks 64-row chunks; wave w owns the
// chunk's rows [16w, 16w+16).

template <typename T, int MTJ>
__global__ __launch_bounds__(256) void k_tsmm(const T* In, int64_t ldi, int p,
                                              const double* __restrict__ Coef, int q, T* Out,
                                              int64_t ldo, int64_t n,
                                              const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  typedef typename AccOf<T>::type AccT;
  extern __shared__ double smem_d[];
  T* cf = reinterpret_cast<T*>(smem_d);
  T* tile = cf + ((p * q + 1) & ~1);
  const int ldt = p + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane >> 4, cc = lane & 15;
  for (int i = threadIdx.x; i < p * q; i += 256) cf[i] = (T)Coef[i];
  const int64_t nchunks = (n + 63) / 64;
  for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    __syncthreads();
    const int64_t row0 = chunk * 64;
    const int rows = (int)min<int64_t>(64, n - row0);
    stage_rows<T>(In, ldi, p, row0, rows, tile);
    __syncthreads();
    AccT acc[MTJ];
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) acc[tj] = AccT{0, 0, 0, 0};
    const int arow = wave * 16 + cc;
    for (int k = 0; k < p; k += 4) {
      const int kk = k + kr;
      const bool kv = kk < p;
      const T a = kv ? tile[arow * ldt + kk] : T(0);
#pragma unroll
      for (int tj = 0; tj < MTJ; ++tj) {
        const int col = tj * 16 + cc;
        const T b = (kv && col < q) ? cf[kk * q + col] : T(0);
        acc[tj] = mma(a, b, acc[tj]);
      }
    }
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) {
      const int col = tj * 16 + cc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = wave * 16 + acc_row<T>(r, lane);
        if (rr < rows && col < q) Out[(row0 + rr) * ldo + col] = (T)acc[tj][r];
      }
    }
  }
}

template <typename T>
static size_t tsmm_smem(int p, int q) {
  return sizeof(T) * (size_t)(((p * q + 1) & ~1) + 64 * (p + 1));
}

template <typename T, int MTJ>
static hipError_t tsmm_launch(const T* In, int64_t ldi, int p, const double* Coef, int q, T* Out,
                              int64_t ldo, int64_t n, const int* skip, hipStream_t s) {
  const size_t sm = tsmm_smem<T>(p, q);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_tsmm<T, MTJ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              152 * 1024);
    (void)hipGetLastError();
    attr = true;
  }
  const int64_t nchunks = (n + 63) / 64;
  const int grid = (int)std::min<int64_t>(nchunks, kStreamBlocks);
  hipLaunchKernelGGL((k_tsmm<T, MTJ>), dim3(grid), dim3(256), sm, s, In, ldi, p, Coef, q, Out, ldo,
                     n, skip);
  return hipGetLastError();
}

template <typename T>
static hipError_t tsmm_any(const T* In, int64_t ldi, int p, const double* Coef, int q, T* Out,
                           int64_t ldo, int64_t n, const int* skip, hipStream_t s) {
  if (p < 1 || q < 1 || p > kMaxP + 32 || q > 64 || n < 1) return hipErrorInvalidValue;
  switch ((q + 15) / 16) {
    case 1: return tsmm_launch<T, 1>(In, ldi, p, Coef, q, Out, ldo, n, skip, s);
    case 2: return tsmm_launch<T, 2>(In, ldi, p, Coef, q, Out, ldo, n, skip, s);
    case 3: return tsmm_launch<T, 3>(In, ldi, p, Coef, q, Out, ldo, n, skip, s);
    default: return tsmm_launch<T, 4>(In, ldi, p, Coef, q, Out, ldo, n, skip, s);
  }
}

hipError_t tsmm_f64(const double* In, int64_t ldi, int p, const double* Coef, int q, double* Out,
                    int64_t ldo, int64_t n, const int* skip, hipStream_t s) {
  return tsmm_any<double>(In, ldi, p, Coef, q, Out, ldo, n, skip, s);
}
hipError_t tsmm_f32(const float* In, int64_t ldi, int p, const double* Coef, int q, float* Out,
                    int64_t ldo, int64_t n, const int* skip, hipStream_t s) {
  return tsmm_any<float>(In, ldi, p, Coef, q, Out, ldo, n, skip, s);
}

// ---------------------------------------------------------------------------
// rotate: the whole per-row work of one LOBPCG update in a single pass.

__device__ __forceinline__ double precond_apply(double r, double d, double th, int kind) {
  if (kind == kPrecNone) return r;
  double den = d - th;
  const double delta = kPrecondGuard * fmax(1.0, fabs(th));
  if (kind == kPrecDiag) {
    den = fabs(den);
    if (den < delta) den = delta;
  } else if (fabs(den) < delta) {
    den = (den < 0.0) ? -delta : delta;
  }
  return r / den;
}

// dynamic LDS of k_rotate for a coefficient stride ldc; the stride is padded
// to 16 (mod 32) when that still fits in 150 KB (it does for every shape
// but the largest fp64 ones)
// The tile area holds the two staged input tiles (64 x (p+1) each) and,
// after them, the output tile (64 x (no+1), no = q + m - a0 <= 2q).
__host__ __device__ inline size_t rotate_smem_bytes(int p, int q, int ldc, size_t tsize) {
  size_t tiles = 2 * 64 * (size_t)(p + 1) * tsize;
  const size_t out = 64 * (size_t)(2 * q + 1) * tsize;
  if (out > tiles) tiles = out;
  return tsize * (size_t)((p * ldc + 1) & ~1) + tiles;
}
__host__ __device__ inline int rotate_ldc(int p, int q, size_t tsize) {
  const int padded = q + ((16 - q % 32) + 32) % 32;
  return rotate_smem_bytes(p, q, padded, tsize) <= 150 * 1024 ? padded : q;
}

// Register prefetch of the next chunk's rows (PF): thread t holds vectors
// t, t + 256, ... of the 64 x p tile read as 16-byte vectors, at most
// kPfVec of them per tile (p <= 64); they are loaded while the current
// chunk is multiplied and written, and stored to LDS at the next chunk.
template <typename T>
struct PfTile {
  static constexpr int VE = 16 / (int)sizeof(T);
  static constexpr int kPfVec = 64 * 64 / VE / 256;
  typename Vec16<T>::type v[kPfVec];
};
template <typename T>
__device__ __forceinline__ void pf_load(const T* __restrict__ In, int64_t ld, int p, int64_t row0,
                                        int rows, PfTile<T>& t) {
  constexpr int VE = PfTile<T>::VE;
  const int pv = p / VE, total = 64 * pv;
#pragma unroll
  for (int i = 0; i < PfTile<T>::kPfVec; ++i) {
    const int idx = threadIdx.x + 256 * i;
    const int r = idx / pv, cv = idx - r * pv;
    if (idx < total && r < rows)
      t.v[i] = *reinterpret_cast<const typename Vec16<T>::type*>(In + (row0 + r) * ld + cv * VE);
    else
      for (int e = 0; e < VE; ++e) t.v[i][e] = T(0);
  }
}
template <typename T>
__device__ __forceinline__ void pf_store(const PfTile<T>& t, int p, T* __restrict__ tile) {
  constexpr int VE = PfTile<T>::VE;
  const int pv = p / VE, total = 64 * pv, ldt = p + 1;
#pragma unroll
  for (int i = 0; i < PfTile<T>::kPfVec; ++i) {
    const int idx = threadIdx.x + 256 * i;
    if (idx < total) {
      const int r = idx / pv, cv = idx - r * pv;
#pragma unroll
      for (int e = 0; e < VE; ++e) tile[r * ldt + cv * VE + e] = t.v[i][e];
    }
  }
}

// 4 waves per SIMD for every instance (fp64 MTJ = 4: 3), without spills; the
// prefetching instances are bound to 2 blocks per CU by their LDS anyway
template <typename T, int MTJ, bool PF>
__global__ __launch_bounds__(256, (PF ? 2 : (MTJ <= 3 ? 4 : 3))) void k_rotate(const T* __restrict__ V,
                                                                   const T* __restrict__ AV,
                                                                   T* __restrict__ Vout,
                                                                   T* __restrict__ AVout,
                                                                   RotateArgs a) {
  typedef typename AccOf<T>::type AccT;
  extern __shared__ double smem_d[];
  __shared__ double nred[4][64];
  const int p = a.p, q = a.q, m = a.m;
  const int na = m - a.a0;
  const int no = q + na;  // output columns [X' P' W~]
  // coefficient stride = 16 (mod 32): the four k rows a wave reads per MFMA
  // step fall in different LDS banks
  const int ldc = rotate_ldc(p, q, sizeof(T));
  T* cf = reinterpret_cast<T*>(smem_d);
  T* tV = cf + ((p * ldc + 1) & ~1);
  T* tA = tV + 64 * (p + 1);
  T* tO = tV;  // output tile, reuses the staging area: 64 x (no + 1) <= 2 * 64 * (p + 1)
  const int ldt = p + 1, ldto = no + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane >> 4, cc = lane & 15;
  for (int i = threadIdx.x; i < p * q; i += 256) cf[(i / q) * ldc + i % q] = (T)a.U[i];
  double th[MTJ];
  double nacc[MTJ];
#pragma unroll
  for (int tj = 0; tj < MTJ; ++tj) {
    const int col = tj * 16 + cc;
    th[tj] = (col < m) ? a.theta[col] : 0.0;
    nacc[tj] = 0.0;
  }
  const int64_t n = a.n;
  const int64_t nchunks = (n + 63) / 64;
  PfTile<T> pfv, pfa;
  if (PF && blockIdx.x < nchunks) {
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int rws = (int)min<int64_t>(64, n - r0);
    pf_load<T>(V, a.ldv, p, r0, rws, pfv);
    pf_load<T>(AV, a.ldv, p, r0, rws, pfa);
  }
  for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    __syncthreads();
    const int64_t row0 = chunk * 64;
    const int rows = (int)min<int64_t>(64, n - row0);
    if (PF) {
      pf_store<T>(pfv, p, tV);
      pf_store<T>(pfa, p, tA);
      const int64_t nx = chunk + gridDim.x;
      if (nx < nchunks) {
        // the next chunk's loads are in flight during this chunk's work
        const int64_t r0 = nx * 64;
        const int rws = (int)min<int64_t>(64, n - r0);
        pf_load<T>(V, a.ldv, p, r0, rws, pfv);
        pf_load<T>(AV, a.ldv, p, r0, rws, pfa);
      }
    } else {
      stage_rows<T>(V, a.ldv, p, row0, rows, tV);
      stage_rows<T>(AV, a.ldv, p, row0, rows, tA);
    }
    __syncthreads();
    AccT ax[MTJ], aa[MTJ];
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) {
      ax[tj] = AccT{0, 0, 0, 0};
      aa[tj] = AccT{0, 0, 0, 0};
    }
    const int arow = wave * 16 + cc;
    for (int k = 0; k < p; k += 4) {
      const int kk = k + kr;
      const bool kv = kk < p;
      const T xv = kv ? tV[arow * ldt + kk] : T(0);
      const T av = kv ? tA[arow * ldt + kk] : T(0);
#pragma unroll
      for (int tj = 0; tj < MTJ; ++tj) {
        const int col = tj * 16 + cc;
        const T b = (kv && col < q) ? cf[kk * ldc + col] : T(0);
        ax[tj] = mma(xv, b, ax[tj]);
        aa[tj] = mma(av, b, aa[tj]);
      }
    }
    // The outputs go through LDS (the staging area becomes the output tile)
    // and leave as 16-byte vectors along contiguous rows: first
    // [X' P' W~] (no columns), then [AX' AP'] (q columns).
    __syncthreads();
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) {
      const int col = tj * 16 + cc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = wave * 16 + acc_row<T>(r, lane);
        if (col < q) {
          const T xo = (T)ax[tj][r];
          const T ao = (T)aa[tj][r];
          const bool live = rr < rows;
          tO[rr * ldto + col] = live ? xo : T(0);
          if (col < m) {
            T w = T(0);
            if (live) {
              const double res = (double)ao - th[tj] * (double)xo;
              nacc[tj] += res * res;
              if (col >= a.a0) {
                const double d = (a.precond == kPrecNone) ? 0.0 : a.diag[row0 + rr];
                w = (T)precond_apply(res, d, th[tj], a.precond);
              }
            }
            if (col >= a.a0) tO[rr * ldto + q + (col - a.a0)] = w;
          }
        }
      }
    }
    __syncthreads();
    write_rows<T>(tO, ldto, no, rows, Vout, a.ldo, row0);
    __syncthreads();
    const int ldtq = q + 1;
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) {
      const int col = tj * 16 + cc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = wave * 16 + acc_row<T>(r, lane);
        if (col < q) tO[rr * ldtq + col] = (rr < rows) ? (T)aa[tj][r] : T(0);
      }
    }
    __syncthreads();
    write_rows<T>(tO, ldtq, q, rows, AVout, a.ldo, row0);
  }
  // per-column residual partial: sum the 4 lane groups (fixed xor order), then waves
#pragma unroll
  for (int tj = 0; tj < MTJ; ++tj) {
    double v = nacc[tj];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    nacc[tj] = v;
  }
  __syncthreads();
  if (kr == 0) {
#pragma unroll
    for (int tj = 0; tj < MTJ; ++tj) nred[wave][tj * 16 + cc] = nacc[tj];
  }
  __syncthreads();
  if (threadIdx.x < m) {
    const int c = threadIdx.x;
    a.part[(int64_t)blockIdx.x * m + c] = ((nred[0][c] + nred[1][c]) + nred[2][c]) + nred[3][c];
  }
}

template <typename T>
static size_t rotate_smem(int p, int q) {
  return rotate_smem_bytes(p, q, rotate_ldc(p, q, sizeof(T)), sizeof(T));
}

template <typename T, int MTJ, bool PF>
static void rotate_kernel_launch(const T* V, const T* AV, T* Vout, T* AVout, const RotateArgs& a,
                                 int grid, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_rotate<T, MTJ, PF>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)hipGetLastError();
    attr = true;
  }
  hipLaunchKernelGGL((k_rotate<T, MTJ, PF>), dim3(grid), dim3(256), rotate_smem<T>(a.p, a.q), s, V,
                     AV, Vout, AVout, a);
}

template <typename T, int MTJ>
static hipError_t rotate_launch(const T* V, const T* AV, T* Vout, T* AVout, const RotateArgs& a,
                                hipStream_t s) {
  const int64_t nchunks = (a.n + 63) / 64;
  const int grid = (int)std::min<int64_t>(nchunks, kStreamBlocks);
  // register prefetch (fp64): 16-byte rows (p, ld and both bases aligned),
  // p <= 64.  The fp32 instances keep the staged path: their prefetch
  // registers would cost a block per CU (4 fit by LDS without them, 3 with)
  constexpr int VE = 16 / (int)sizeof(T);
  const bool pf = sizeof(T) == 8 && a.p <= 64 && a.p % VE == 0 && a.ldv % VE == 0 &&
                  (reinterpret_cast<uintptr_t>(V) & 15) == 0 &&
                  (reinterpret_cast<uintptr_t>(AV) & 15) == 0;
  // (fp64 with four column tiles would spill: it keeps the staged path)
  if constexpr (sizeof(T) != 8 || MTJ == 4) {
    rotate_kernel_launch<T, MTJ, false>(V, AV, Vout, AVout, a, grid, s);
  } else {
    if (pf) rotate_kernel_launch<T, MTJ, true>(V, AV, Vout, AVout, a, grid, s);
    else rotate_kernel_launch<T, MTJ, false>(V, AV, Vout, AVout, a, grid, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return sum_parts(a.part, grid, a.m, a.resnorm2, nullptr, s);
}

template <typename T>
static hipError_t rotate_any(const T* V, const T* AV, T* Vout, T* AVout, const RotateArgs& a,
                             hipStream_t s) {
  if (a.p < 1 || a.p > kMaxP || a.q < a.m || a.q > 64 || a.m < 1 || a.m > 64 || a.a0 < 0 ||
      a.a0 > a.m || a.n < 1 || a.ldo < a.q + (a.m - a.a0) || a.ldv < a.p)
    return hipErrorInvalidValue;
  switch ((a.q + 15) / 16) {
    case 1: return rotate_launch<T, 1>(V, AV, Vout, AVout, a, s);
    case 2: return rotate_launch<T, 2>(V, AV, Vout, AVout, a, s);
    case 3: return rotate_launch<T, 3>(V, AV, Vout, AVout, a, s);
    default: return rotate_launch<T, 4>(V, AV, Vout, AVout, a, s);
  }
}

hipError_t rotate_f64(const double* V, const double* AV, double* Vout, double* AVout,
                      const RotateArgs& a, hipStream_t s) {
  return rotate_any<double>(V, AV, Vout, AVout, a, s);
}
hipError_t rotate_f32(const float* V, const float* AV, float* Vout, float* AVout,
                      const RotateArgs& a, hipStream_t s) {
  return rotate_any<float>(V, AV, Vout, AVout, a, s);
}

// ---------------------------------------------------------------------------
// Column statistics (true residual).  Lane c of every wave owns column c.

__global__ __launch_bounds__(256) void k_colstats(const double* __restrict__ X, int64_t ldx,
                                                  const double* __restrict__ AX, int64_t ldax,
                                                  int m, const double* __restrict__ theta,
                                                  int64_t n, double* __restrict__ part) {
  __shared__ double red[4][3][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double sxx = 0.0, sxa = 0.0, srr = 0.0;
  if (lane < m) {
    const double th = theta[lane];
    for (int64_t row = (int64_t)blockIdx.x * 4 + wave; row < n; row += (int64_t)gridDim.x * 4) {
      const double x = X[row * ldx + lane];
      const double ax = AX[row * ldax + lane];
      const double r = ax - th * x;
      sxx += x * x;
      sxa += x * ax;
      srr += r * r;
    }
  }
  red[wave][0][lane] = sxx;
  red[wave][1][lane] = sxa;
  red[wave][2][lane] = srr;
  __syncthreads();
  if (threadIdx.x < 3 * m) {
    const int k = threadIdx.x / m, c = threadIdx.x - k * m;
    part[(int64_t)blockIdx.x * 3 * m + k * m + c] =
        ((red[0][k][c] + red[1][k][c]) + red[2][k][c]) + red[3][k][c];
  }
}

hipError_t colstats_f64(const double* X, int64_t ldx, const double* AX, int64_t ldax, int m,
                        const double* theta, int64_t n, double* part, double* out, hipStream_t s) {
  if (m < 1 || m > 64) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(kStreamBlocks, (n + 3) / 4);
  hipLaunchKernelGGL(k_colstats, dim3(grid), dim3(256), 0, s, X, ldx, AX, ldax, m, theta, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return sum_parts(part, grid, 3 * m, out, nullptr, s);
}

// ---------------------------------------------------------------------------
// SplitMix64 column fill.

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_fill_splitmix(double* X, int64_t ld, int col, int col_id, int64_t n,
                                uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t z = splitmix64(seed + (uint64_t)col_id * (uint64_t)n + (uint64_t)i);
  X[i * ld + col] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

hipError_t fill_splitmix(double* X, int64_t ld, int col, int col_id, int64_t n, uint64_t seed,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_fill_splitmix, dim3(cdiv(n, 256)), dim3(256), 0, s, X, ld, col, col_id, n,
                     seed);
  return hipGetLastError();
}

__global__ void k_fill_splitmix_f32(float* X, int64_t ld, int col, int col_id, int64_t n,
                                    uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t z = splitmix64(seed + (uint64_t)col_id * (uint64_t)n + (uint64_t)i);
  X[i * ld + col] = (float)((double)(z >> 11) * 0x1.0p-53 - 0.5);
}

hipError_t fill_splitmix_f32(float* X, int64_t ld, int col, int col_id, int64_t n, uint64_t seed,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_fill_splitmix_f32, dim3(cdiv(n, 256)), dim3(256), 0, s, X, ld, col, col_id,
                     n, seed);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sign normalisation: argmax |x| per column (lowest index on ties), then copy.

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  return (v > bv) || (v == bv && i < bi);
}

__global__ __launch_bounds__(256) void k_colargmax(const double* __restrict__ X, int64_t ldx,
                                                   int k, int64_t n, int64_t* pidx,
                                                   double* pval) {
  __shared__ double sv[4][64];
  __shared__ int64_t si[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double bv = -1.0;
  int64_t bi = n;
  if (lane < k) {
    for (int64_t row = (int64_t)blockIdx.x * 4 + wave; row < n; row += (int64_t)gridDim.x * 4) {
      const double v = fabs(X[row * ldx + lane]);
      if (better(v, row, bv, bi)) {
        bv = v;
        bi = row;
      }
    }
  }
  sv[wave][lane] = bv;
  si[wave][lane] = bi;
  __syncthreads();
  if (threadIdx.x < k) {
    const int c = threadIdx.x;
    double v = sv[0][c];
    int64_t i = si[0][c];
    for (int w = 1; w < 4; ++w)
      if (better(sv[w][c], si[w][c], v, i)) {
        v = sv[w][c];
        i = si[w][c];
      }
    pval[(int64_t)blockIdx.x * k + c] = v;
    pidx[(int64_t)blockIdx.x * k + c] = i;
  }
}

__global__ void k_argmax_final(const double* __restrict__ X, int64_t ldx, int k, int nblk,
                               int64_t* pidx, double* pval) {
  const int c = threadIdx.x;
  if (c >= k) return;
  double v = pval[c];
  int64_t i = pidx[c];
  for (int b = 1; b < nblk; ++b)
    if (better(pval[(int64_t)b * k + c], pidx[(int64_t)b * k + c], v, i)) {
      v = pval[(int64_t)b * k + c];
      i = pidx[(int64_t)b * k + c];
    }
  // sign of the winning entry, stored as +1 / -1 in pval[c]
  pval[c] = (X[i * ldx + c] < 0.0) ? -1.0 : 1.0;
}

__global__ void k_copy_sign(const double* __restrict__ X, int64_t ldx, int k, int64_t n,
                            const double* __restrict__ sign, double* out, int64_t ldout) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx / k;
  const int c = (int)(idx - i * k);
  out[i * ldout + c] = sign[c] * X[i * ldx + c];
}

hipError_t copy_signfix(const double* X, int64_t ldx, int k, int64_t n, double* out,
                        int64_t ldout, int64_t* part_idx, double* part_val, hipStream_t s) {
  if (k < 1 || k > 64) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(256, (n + 3) / 4);
  hipLaunchKernelGGL(k_colargmax, dim3(grid), dim3(256), 0, s, X, ldx, k, n, part_idx, part_val);
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(64), 0, s, X, ldx, k, grid, part_idx, part_val);
  hipLaunchKernelGGL(k_copy_sign, dim3(cdiv(n * k, 256)), dim3(256), 0, s, X, ldx, k, n,
                     (const double*)part_val, out, ldout);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// conversions

template <typename A, typename B>
__global__ void k_convert(const A* __restrict__ in, int64_t ldi, B* __restrict__ out, int64_t ldo,
                          int c, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * c) return;
  const int64_t i = idx / c;
  const int j = (int)(idx - i * c);
  out[i * ldo + j] = (B)in[i * ldi + j];
}

hipError_t convert_f64_to_f32(const double* in, int64_t ldi, float* out, int64_t ldo, int c,
                              int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, float>), dim3(cdiv(n * c, 256)), dim3(256), 0, s, in, ldi,
                     out, ldo, c, n);
  return hipGetLastError();
}
hipError_t convert_f32_to_f64(const float* in, int64_t ldi, double* out, int64_t ldo, int c,
                              int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<float, double>), dim3(cdiv(n * c, 256)), dim3(256), 0, s, in, ldi,
                     out, ldo, c, n);
  return hipGetLastError();
}
hipError_t convert_vec_f64_to_f32(const double* in, float* out, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, float>), dim3(cdiv(len, 256)), dim3(256), 0, s, in,
                     (int64_t)1, out, (int64_t)1, 1, len);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// status post: the block goes to coherent host memory with vector stores,
// every thread fences its stores at system scope, and after the barrier
// one thread stores the sequence word the host waits for
__global__ __launch_bounds__(256) void k_post_status(const uint32_t* __restrict__ src, int nwords,
                                                     uint32_t* dst, uint32_t* flag, uint32_t seq) {
  for (int i = threadIdx.x; i < nwords; i += 256) dst[i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) *reinterpret_cast<volatile uint32_t*>(flag) = seq;
}

hipError_t post_status(const void* src, int nwords, uint32_t* dst, uint32_t* flag, uint32_t seq,
                       hipStream_t s) {
  if (nwords < 0 || nwords > 1024 || src == nullptr || dst == nullptr || flag == nullptr)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_post_status, dim3(1), dim3(256), 0, s,
                     reinterpret_cast<const uint32_t*>(src), nwords, dst, flag, seq);
  return hipGetLastError();
}

}  // namespace lobpcg
