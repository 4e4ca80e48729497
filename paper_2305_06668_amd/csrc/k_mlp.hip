// Learned preconditioner: inference and training kernels.
//
// The preconditioned column is w_i = r_i / sqrt((d_i - theta)^2 + c_i^2)
// with c_i = s softplus(y_i), y_i the output of a per-entry MLP
// 3 -> 128 -> 128 -> 1 (SiLU) on the features
//   phi = (log(|d_i - theta| / s + 1e-6), theta / s, log(rho_i / s + 1e-6)),
// rho_i the off-diagonal absolute row sum and s = mean |d|.  The denominator
// is floored at the Jacobi guard delta = 1e-8 max(1, |theta|).  Outside the
// window |d_i - theta| <= 16 rho_i, c = 0 by definition (the regulariser
// only matters where d_i is within a few couplings of theta), and a tile
// with no entry inside the window skips the net.  A column flagged in
// `mask` or in the bit set `mbits`, and any entry whose net output is not
// finite, takes c = 0: the
// guarded absolute Jacobi step (the diagonal fallback).
//
// fp32 path (k_mlp_apply, and the forward inside training): a workgroup of
// 512 threads (eight waves, two per SIMD) holds W2 (128 x 128 fp32, rows
// swizzled against bank conflicts) and the
// small layers in LDS and walks tiles of 64 entries (entry e = row * nact +
// column, contiguous in the row-major block).  Layer 2 is a 64 x 128 x 128
// product per tile on v_mfma_f32_16x16x4f32: wave w computes entries
// 16 (w & 3) + [0, 16) against neurons 64 (w >> 2) + [0, 64); layer 3 is
// reduced over a wave's 16 neuron lanes with xor shuffles and over the two
// neuron halves through LDS.  Tiles are screened eight at a time (one entry
// per thread, a ballot per wave); only tiles with an entry inside the window
// run the net, the others take the Jacobi step in the screening pass.
//
// Training (k_mlp_grad): that forward pass, then the analytic backward pass
// for an output gradient dL/dw given per entry, its two contractions (dW2,
// dH1) on the same MFMA; per-tile sums are formed in fp32 and accumulated
// across tiles in fp64 per workgroup; k_grad_reduce adds the workgroup
// partials in a fixed order, k_adam updates the fp32 master weights.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace lobpcg {

namespace {

constexpr int kH = kMlpHidden;
constexpr int kTE = 64;          // entries per tile
constexpr int oW1 = 0, oB1 = kH * kMlpFeat, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH;
static_assert(oB3 + 1 == kMlpParams, "parameter layout");

// fp32 activations; the reciprocal is v_rcp_f32 (1 ulp) rather than a
// full division
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}
__device__ __forceinline__ double softplus_d(double y) {
  return fmax(y, 0.0) + log1p(exp(-fabs(y)));
}

// Per-entry inputs of one tile entry.
struct EntryIn {
  bool valid;
  bool inside;   // |d_i - theta_j| <= kMlpWindow rho_i
  int64_t row;
  int col;
  double dm;     // d_i - theta_j
  double theta;
};

struct EntryOut {
  double c;      // regulariser (0 on fallback)
  double q;      // dm^2 + c^2, floored
  bool floored;
};

__device__ __forceinline__ EntryOut regularise(const EntryIn& in, float y, double s, bool jacobi,
                                               int* flags) {
  EntryOut o{};
  if (!in.inside) jacobi = true;
  double c = s * softplus_d((double)y);
  if (!jacobi && !isfinite(c)) {
    if (flags) flags[in.col] = 1;
    jacobi = true;
  }
  if (jacobi) c = 0.0;
  const double delta = kPrecondGuard * fmax(1.0, fabs(in.theta));
  const double q = in.dm * in.dm + c * c;
  o.floored = q < delta * delta;
  o.q = o.floored ? delta * delta : q;
  o.c = c;
  return o;
}

// ---- fp32 MFMA tile kernels (512 threads) ----
constexpr int kGT = 512;
constexpr int gW2 = 0;                // W2 [k][j]
constexpr int gH1 = gW2 + kH * kH;    // H1 [e][j]
constexpr int gDZ = gH1 + kTE * kH;   // dZ2 [e][k] (training)
constexpr int gW1 = gDZ + kTE * kH;   // [f][j] (three feature rows of kH, a fourth unused)
constexpr int gB1 = gW1 + kH * 4;
constexpr int gB2 = gB1 + kH;
constexpr int gW3 = gB2 + kH;
constexpr int gB3 = gW3 + kH;         // 4 floats
constexpr int gPhi = gB3 + 4;         // [e][4]
constexpr int gYP = gPhi + kTE * 4;   // [2][e] layer-3 partials of the two neuron halves
constexpr int gDY = gYP + 2 * kTE;    // [e]
constexpr int gP1 = gDY + kTE;        // [4][j][4] dW1 (3), db1 per entry tile
constexpr int gP2 = gP1 + 4 * kH * 4; // [4][k][2] dW3, db2 per entry tile
constexpr int gAct = gP2 + 4 * kH * 2;  // [8] ints: tile of the screened group has an entry inside
constexpr int gEnd = gAct + 8;
constexpr int kGroup = kGT / kTE;     // tiles screened together, one per wave
// then doubles: per entry r, dL/dw, d - theta, theta; per neuron the fp64
// sums dW1 (3), db1, db2, dW3; dB3
constexpr int dR = 0, dG = kTE, dDM = 2 * kTE, dTH = 3 * kTE, dRow = 4 * kTE,
              dB3 = dRow + 6 * kH, dEnd = dB3 + 2;
constexpr size_t kTileBytes = sizeof(float) * gEnd + sizeof(double) * dEnd;
static_assert(gEnd % 2 == 0 && kTileBytes <= 160 * 1024, "LDS budget");

// Rows of 128 floats with column bits 1..4 xor-ed by the row's low four bits
// (row bit 0 into column bit 4, bits 1..3 into bits 1..3).  The LDS serves a
// wave in two halves of 32 lanes over 32 banks, and within a half both
// operand patterns -- 16 rows x 2 columns and 2 rows x 16 columns -- then
// hit 32 distinct banks: the bank-conflict cycles fell from 36 % (forward)
// and 22 % (gradient) of the LDS-active cycles, with the row bits xor-ed
// into column bits 2..5, to 0.4 % and 5 % (the launch times did not move).
__device__ __forceinline__ int swz(int row, int col) {
  return row * kH + (col ^ (((row & 1) << 4) | (((row >> 1) & 7) << 1)));
}

__device__ __forceinline__ void load_weights(const float* __restrict__ wts, float* L) {
  for (int idx = threadIdx.x; idx < kH * kH; idx += kGT)
    L[gW2 + swz(idx >> 7, idx & 127)] = wts[oW2 + idx];
  for (int idx = threadIdx.x; idx < kH; idx += kGT) {
    // feature-major: lanes of consecutive neurons read consecutive words
    L[gW1 + 0 * kH + idx] = wts[oW1 + idx * 3 + 0];
    L[gW1 + 1 * kH + idx] = wts[oW1 + idx * 3 + 1];
    L[gW1 + 2 * kH + idx] = wts[oW1 + idx * 3 + 2];
    L[gB1 + idx] = wts[oB1 + idx];
    L[gB2 + idx] = wts[oB2 + idx];
    L[gW3 + idx] = wts[oW3 + idx];
  }
  if (threadIdx.x == 0) L[gB3] = wts[oB3];
}

// Features of tile entry e into LDS, with the entry's d - theta and theta
// and (R, G given) its r and dL/dw; returns whether the entry is inside the
// window.  Not inlined: the constants of the fp64 log stay out of the
// callers' tile loops.
__device__ __noinline__ bool tile_entry(float* L, double* Ld, int e, int64_t ent, int64_t total,
                                        int nact, const double* __restrict__ R,
                                        const double* __restrict__ G, int64_t ld,
                                        const double* __restrict__ diag,
                                        const double* __restrict__ rho,
                                        const double* __restrict__ theta, double s) {
  float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
  double r = 0.0, gg = 0.0, dm = 0.0, th = 0.0;
  bool inside = false;
  if (ent < total) {
    const int64_t row = ent / nact;
    const int col = (int)(ent - row * nact);
    th = theta[col];
    dm = diag[row] - th;
    const double rr = rho[row];
    inside = fabs(dm) <= kMlpWindow * rr;
    f0 = (float)log(fabs(dm) / s + 1e-6);
    f1 = (float)(th / s);
    f2 = (float)log(rr / s + 1e-6);
    if (R != nullptr) {
      r = R[row * ld + col];
      gg = G[row * ld + col];
    }
  }
  L[gPhi + e * 4 + 0] = f0;
  L[gPhi + e * 4 + 1] = f1;
  L[gPhi + e * 4 + 2] = f2;
  Ld[dR + e] = r;
  Ld[dG + e] = gg;
  Ld[dDM + e] = dm;
  Ld[dTH + e] = th;
  return inside;
}

// Screening of the group of kGroup tiles from tile t0: thread tid takes
// entry t0 kTE + tid (wave w = tile t0 + w) and the wave's ballot records
// whether its tile has an entry inside the window.  Without a Jacobi target
// (J == nullptr) that is all; with one, the entries of tiles with none
// inside take the guarded Jacobi step there (the learned step with c = 0).
// The caller syncs before reading the flags.
template <typename T>
__device__ __forceinline__ void screen_group(float* L, int64_t t0, int64_t total, int nact,
                                             const double* __restrict__ diag,
                                             const double* __restrict__ rho,
                                             const double* __restrict__ theta, T* __restrict__ J,
                                             int64_t ld) {
  const int64_t ent = t0 * kTE + threadIdx.x;
  const bool valid = ent < total;
  int64_t row = 0;
  int col = 0;
  double dm = 0.0, th = 0.0;
  bool ins = false;
  if (valid) {
    row = ent / nact;
    col = (int)(ent - row * nact);
    th = theta[col];
    dm = diag[row] - th;
    ins = fabs(dm) <= kMlpWindow * rho[row];
  }
  const bool act = __ballot(ins) != 0;
  if ((threadIdx.x & 63) == 0) reinterpret_cast<int*>(L + gAct)[threadIdx.x >> 6] = act ? 1 : 0;
  if (J != nullptr && valid && !act) {
    const double delta = kPrecondGuard * fmax(1.0, fabs(th));
    T* p = J + row * ld + col;
    *p = (T)((double)*p / sqrt(fmax(dm * dm, delta * delta)));
  }
}

// Layer 1 into H1 (all threads), then layer 2 on MFMA: wave w's
// z[tt][r] = Z2[e = 16 (w & 3) + 4 g + r][k = 16 (4 (w >> 2) + tt) + c],
// and the layer-3 partial of each entry over the wave's 64 neurons into
// L[gYP + (w >> 2) kTE + e].  One barrier inside; the caller syncs before
// reading the partials.
__device__ __forceinline__ void mfma_forward(float* L, f4 (&z)[4], int w, int c, int g) {
  const int mt = w & 3, n0 = 4 * (w >> 2);
  for (int idx = threadIdx.x; idx < kTE * kH; idx += kGT) {
    const int e = idx >> 7, j = idx & 127;
    const float* w1 = L + gW1 + j;
    const float* ph = L + gPhi + e * 4;
    L[gH1 + swz(e, j)] = silu(L[gB1 + j] + w1[0] * ph[0] + w1[kH] * ph[1] + w1[2 * kH] * ph[2]);
  }
  __syncthreads();
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    const float b = L[gB2 + 16 * (n0 + tt) + c];
    z[tt] = f4{b, b, b, b};
  }
#pragma unroll 4
  for (int j4 = 0; j4 < kH; j4 += 4) {
    const float a = L[gH1 + swz(16 * mt + c, j4 + g)];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
      z[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L[gW2 + swz(16 * (n0 + tt) + c, j4 + g)],
                                                   z[tt], 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float p = 0.0f;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) p = fmaf(L[gW3 + 16 * (n0 + tt) + c], silu(z[tt][r]), p);
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) p += __shfl_xor(p, off, 16);
    if (c == 0) L[gYP + (w >> 2) * kTE + 16 * mt + 4 * g + r] = p;
  }
}

// The learned step of tile entry e (valid), written over R.
template <typename T>
__device__ __noinline__ void apply_entry(const double* Ld, int e, int64_t ent, int nact,
                                         T* __restrict__ R, int64_t ld, float y, double s,
                                         bool inside, const int* __restrict__ mask,
                                         uint64_t mbits, int* __restrict__ flags) {
  EntryIn in{};
  in.valid = true;
  in.inside = inside;
  in.row = ent / nact;
  in.col = (int)(ent - in.row * nact);
  in.dm = Ld[dDM + e];
  in.theta = Ld[dTH + e];
  const bool jac = ((mbits >> in.col) & 1) != 0 || (mask != nullptr && mask[in.col] != 0);
  const EntryOut o = regularise(in, y, s, jac, flags);
  T* p = R + in.row * ld + in.col;
  *p = (T)((double)*p / sqrt(o.q));
}

// Inference: R (n x nact, leading dimension ld) is replaced by the learned
// preconditioned columns.
template <typename T>
__global__ __launch_bounds__(kGT) void k_mlp_apply(T* __restrict__ R, int64_t ld, int nact,
                                                   int64_t n, const double* __restrict__ theta,
                                                   const double* __restrict__ diag,
                                                   const double* __restrict__ rho,
                                                   const double* __restrict__ sptr,
                                                   const float* __restrict__ wts,
                                                   const int* __restrict__ mask, uint64_t mbits,
                                                   int* __restrict__ flags) {
  extern __shared__ float L[];
  double* Ld = reinterpret_cast<double*>(L + gEnd);
  load_weights(wts, L);
  const double s = *sptr;
  const int tid = threadIdx.x;
  const int64_t total = n * nact;
  const int64_t ntiles = (total + kTE - 1) / kTE;
  for (int64_t t0 = (int64_t)blockIdx.x * kGroup; t0 < ntiles; t0 += (int64_t)gridDim.x * kGroup) {
    __syncthreads();  // previous group's flag reads done
    // the net only matters inside the window: tiles without such entries
    // take the Jacobi step here and skip it
    screen_group(L, t0, total, nact, diag, rho, theta, R, ld);
    __syncthreads();
    for (int u = 0; u < kGroup; ++u) {
      if (reinterpret_cast<const int*>(L + gAct)[u] == 0) continue;  // uniform in the workgroup
      // lane indices opaque to the compiler (see k_mlp_grad)
      int lid = tid;
      asm volatile("" : "+v"(lid));
      const int w = lid >> 6, c = lid & 15, g = (lid >> 4) & 3;
      const int64_t ent = (t0 + u) * kTE + tid;
      bool inside = false;
      __syncthreads();  // weights loaded / previous tile's LDS reads done
      if (tid < kTE)
        inside = tile_entry(L, Ld, tid, ent, total, nact, nullptr, nullptr, 0, diag, rho, theta, s);
      __syncthreads();
      f4 z[4];
      mfma_forward(L, z, w, c, g);
      __syncthreads();
      if (tid < kTE && ent < total)
        apply_entry(Ld, tid, ent, nact, R, ld, L[gB3] + L[gYP + tid] + L[gYP + kTE + tid], s,
                    inside, mask, mbits, flags);
    }
  }
}

// Training: per-workgroup partial gradients (kMlpParams doubles each) of
// sum_e G_e w_e, where w is the learned column of R and G = dL/dw is given
// (same layout as R).  The tile's three 64 x 128 x 128 contractions on
// v_mfma_f32_16x16x4f32 (fp32 in, fp32 accumulate):
//   forward  Z2  = H1 W2^T   wave w: entry tile w & 3, neuron tiles 4 (w >> 2) + [0, 4)
//   dW2      dW2 = dZ2^T H1  wave w: neuron tile w (rows k), all eight column tiles j
//   dH1      dH1 = dZ2 W2    wave w: entry tile w & 3, column tiles 4 (w >> 2) + [0, 4)
// The activations, layers 1 and 3 and the regulariser's derivative stay on
// the vector units.  Per-tile sums are fp32 (the MFMA accumulators, xor
// shuffles, and LDS partials added in a fixed order); they are accumulated
// across tiles in fp64 per workgroup (registers for dW2, LDS for the rest).

// dL/dy of tile entry e (0 outside the window or where the floor or the
// fallback holds): w = r q^-1/2, q = dm^2 + c^2, c = s softplus(y).
__device__ __noinline__ float entry_dy(const double* Ld, int e, bool inside, float y, double s) {
  if (!inside) return 0.0f;
  EntryIn in{};
  in.valid = true;
  in.inside = true;
  in.dm = Ld[dDM + e];
  in.theta = Ld[dTH + e];
  const EntryOut o = regularise(in, y, s, false, nullptr);
  if (o.floored || !(o.c > 0.0)) return 0.0f;
  const double sg = 1.0 / (1.0 + exp(-(double)y));
  return (float)(-Ld[dG + e] * Ld[dR + e] * o.c * s * sg / (o.q * sqrt(o.q)));
}

__global__ __launch_bounds__(kGT) void k_mlp_grad(const double* __restrict__ R,
                                                  const double* __restrict__ G, int64_t ld,
                                                  int nact, int64_t n,
                                                  const double* __restrict__ theta,
                                                  const double* __restrict__ diag,
                                                  const double* __restrict__ rho,
                                                  const double* __restrict__ sptr,
                                                  const float* __restrict__ wts,
                                                  double* __restrict__ part) {
  extern __shared__ float L[];
  double* Ld = reinterpret_cast<double*>(L + gEnd);
  const int tid = threadIdx.x;
  load_weights(wts, L);
  for (int idx = tid; idx < 6 * kH + 2; idx += kGT) Ld[dRow + idx] = 0.0;
  const double s = *sptr;
  const int64_t total = n * nact;
  const int64_t ntiles = (total + kTE - 1) / kTE;
  double aW2[8][4];  // dW2[k = 16 w + 4 g + r][j = 16 t + c]
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) aW2[t][r] = 0.0;
  for (int64_t t0 = (int64_t)blockIdx.x * kGroup; t0 < ntiles; t0 += (int64_t)gridDim.x * kGroup) {
    __syncthreads();  // previous group's flag reads done
    // entries outside the window have dL/dy = 0: tiles without any inside are skipped
    screen_group<double>(L, t0, total, nact, diag, rho, theta, nullptr, 0);
    __syncthreads();
    for (int u = 0; u < kGroup; ++u) {
      if (reinterpret_cast<const int*>(L + gAct)[u] == 0) continue;  // uniform in the workgroup
      const int64_t tile = t0 + u;
      // the lane indices are re-derived per tile, opaque to the compiler: the
      // swizzled LDS addresses built from them are recomputed inside the loop
      // instead of being hoisted into (and spilled from) registers
      int lid = tid;
      asm volatile("" : "+v"(lid));
      const int w = lid >> 6, c = lid & 15, g = (lid >> 4) & 3;
      const int mt = w & 3, n0 = 4 * (w >> 2);
      bool inside = false;
      __syncthreads();  // previous tile's LDS reads done
      if (tid < kTE)
        inside = tile_entry(L, Ld, tid, tile * kTE + tid, total, nact, R, G, ld, diag, rho, theta, s);
      __syncthreads();
      f4 z[4];  // Z2[e = 16 (w & 3) + 4 g + r][k = 16 (4 (w >> 2) + tt) + c]
      mfma_forward(L, z, w, c, g);
      __syncthreads();
      if (tid < kTE)
        L[gDY + tid] =
            entry_dy(Ld, tid, inside, L[gB3] + L[gYP + tid] + L[gYP + kTE + tid], s);
      __syncthreads();
      if (tid == 0) {
        float t = 0.0f;
        for (int e = 0; e < kTE; ++e) t += L[gDY + e];
        Ld[dB3] += (double)t;
      }
      // dz2 = dy w3 silu'(z2) into LDS; dW3 += dy h2, db2 += dz2 (this entry tile)
      {
        float pW3[4], pB2[4];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) pW3[tt] = pB2[tt] = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = 16 * mt + 4 * g + r;
          const float dy = L[gDY + e];
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            const int k = 16 * (n0 + tt) + c;
            const float zz = z[tt][r], sg = sigm(zz);
            const float dz = dy * L[gW3 + k] * (sg * (1.0f + zz * (1.0f - sg)));
            L[gDZ + swz(e, k)] = dz;
            pW3[tt] = fmaf(dy, zz * sg, pW3[tt]);
            pB2[tt] += dz;
          }
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          pW3[tt] += __shfl_xor(pW3[tt], 16);
          pB2[tt] += __shfl_xor(pB2[tt], 16);
          pW3[tt] += __shfl_xor(pW3[tt], 32);
          pB2[tt] += __shfl_xor(pB2[tt], 32);
          if (g == 0) {
            float* q = L + gP2 + (mt * kH + 16 * (n0 + tt) + c) * 2;
            q[0] = pW3[tt];
            q[1] = pB2[tt];
          }
        }
      }
      __syncthreads();
      // dW2 = dZ2^T H1 for neuron tile w (fp32 per tile, fp64 across tiles)
      {
        f4 acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 2
        for (int e4 = 0; e4 < kTE; e4 += 4) {
          const float a = L[gDZ + swz(e4 + g, 16 * w + c)];
#pragma unroll
          for (int t = 0; t < 8; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L[gH1 + swz(e4 + g, 16 * t + c)],
                                                          acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) aW2[t][r] += (double)acc[t][r];
      }
      // dH1 = dZ2 W2, then dz1 = dh1 silu'(z1); dW1 += dz1 phi, db1 += dz1
      {
        f4 dh[4];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) dh[tt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
        for (int k4 = 0; k4 < kH; k4 += 4) {
          const float a = L[gDZ + swz(16 * mt + c, k4 + g)];
#pragma unroll
          for (int tt = 0; tt < 4; ++tt)
            dh[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, L[gW2 + swz(k4 + g, 16 * (n0 + tt) + c)],
                                                          dh[tt], 0, 0, 0);
        }
        float p0[4], p1[4], p2[4], pb[4];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) p0[tt] = p1[tt] = p2[tt] = pb[tt] = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float* ph = L + gPhi + (16 * mt + 4 * g + r) * 4;
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            const int j = 16 * (n0 + tt) + c;
            const float* w1 = L + gW1 + j;
            const float z1 = L[gB1 + j] + w1[0] * ph[0] + w1[kH] * ph[1] + w1[2 * kH] * ph[2];
            const float dz1 = dh[tt][r] * dsilu(z1);
            p0[tt] = fmaf(dz1, ph[0], p0[tt]);
            p1[tt] = fmaf(dz1, ph[1], p1[tt]);
            p2[tt] = fmaf(dz1, ph[2], p2[tt]);
            pb[tt] += dz1;
          }
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
#pragma unroll
          for (int off = 16; off <= 32; off <<= 1) {
            p0[tt] += __shfl_xor(p0[tt], off);
            p1[tt] += __shfl_xor(p1[tt], off);
            p2[tt] += __shfl_xor(p2[tt], off);
            pb[tt] += __shfl_xor(pb[tt], off);
          }
          if (g == 0) {
            float* q = L + gP1 + (mt * kH + 16 * (n0 + tt) + c) * 4;
            q[0] = p0[tt];
            q[1] = p1[tt];
            q[2] = p2[tt];
            q[3] = pb[tt];
          }
        }
      }
      __syncthreads();
      if (tid < kH) {
        float q[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const float* p1 = L + gP1 + (m * kH + tid) * 4;
          const float* p2 = L + gP2 + (m * kH + tid) * 2;
          q[0] += p1[0];
          q[1] += p1[1];
          q[2] += p1[2];
          q[3] += p1[3];
          q[4] += p2[1];
          q[5] += p2[0];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) Ld[dRow + k * kH + tid] += (double)q[k];
      }
    }
  }
  __syncthreads();
  double* out = part + (size_t)blockIdx.x * kMlpParams;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      out[oW2 + (16 * (tid >> 6) + 4 * ((tid >> 4) & 3) + r) * kH + 16 * t + (tid & 15)] = aW2[t][r];
  if (tid < kH) {
    out[oW1 + tid * 3 + 0] = Ld[dRow + 0 * kH + tid];
    out[oW1 + tid * 3 + 1] = Ld[dRow + 1 * kH + tid];
    out[oW1 + tid * 3 + 2] = Ld[dRow + 2 * kH + tid];
    out[oB1 + tid] = Ld[dRow + 3 * kH + tid];
    out[oB2 + tid] = Ld[dRow + 4 * kH + tid];
    out[oW3 + tid] = Ld[dRow + 5 * kH + tid];
  }
  if (tid == 0) out[oB3] = Ld[dB3];
}

// Inference with layer 2 on bf16 MFMA (v_mfma_f32_16x16x32_bf16, fp32
// accumulate); layers 1 and 3, the features and the epilogue stay fp32 /
// fp64.  One wave computes 32 entries (two 16-row M tiles) against all 128
// neurons (eight 16-column N tiles); the B fragments of W2^T (8 x 4 x 8 bf16
// per lane) are read from LDS (W2 as bf16, rows padded to 136 values) once
// per K step and shared by both M tiles.  Lane (g = lane / 16,
// r = lane % 16) evaluates layer 1 for entry r of each M tile at the hidden
// units 32 ks + 8 g + [0, 8) -- exactly its A fragments, so every h1 value is
// computed once.  The accumulator row of lane (g, r), element i, is entry
// 4 g + i and its column is neuron r of the N tile; layer 3 sums over the
// 16 lanes of a segment with xor shuffles.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kMlpTilesPerWave = 2;  // 16-entry M tiles per wave iteration
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// Screening pass of the bf16 transform: a wave takes a super tile of
// kMlpSuper entries (4 per lane, loaded together) and, when none of them is
// inside the window, takes the Jacobi step for all of them (the formula of
// the tile epilogue with c = 0); it records per super tile whether one of
// its entries is inside (tflags[st] = 1) for the MFMA kernel.  (A list
// appended with an atomic counter serialised ~2000 same-address atomics
// per launch in L2.)
template <typename T>
__global__ __launch_bounds__(256) void k_mlp_screen(T* __restrict__ R, int64_t ld, int nact, int64_t n,
                                                    const double* __restrict__ theta,
                                                    const double* __restrict__ diag,
                                                    const double* __restrict__ rho,
                                                    int* __restrict__ flags,
                                                    int* __restrict__ tflags) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the MFMA pass (next on the stream) sets flags[j] for non-finite outputs
  if (flags != nullptr && blockIdx.x == 0 && (int)threadIdx.x < nact) flags[threadIdx.x] = 0;
  const int64_t total = n * nact;
  const int64_t nst = (total + kMlpSuper - 1) / kMlpSuper;
  constexpr int Q = kMlpSuper / 64;
  const bool small = total < (int64_t)INT32_MAX;  // 32-bit index arithmetic
  for (int64_t st = (int64_t)blockIdx.x * 4 + wave; st < nst; st += (int64_t)gridDim.x * 4) {
    int64_t srow[Q];
    int scol[Q];
    double sdm[Q], sth[Q], srr[Q];
    T sr[Q];
    bool sval[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t ent = st * kMlpSuper + 64 * q + lane;
      sval[q] = ent < total;
      if (small) {
        const uint32_t e32 = (uint32_t)(sval[q] ? ent : 0);
        srow[q] = e32 / (uint32_t)nact;
        scol[q] = (int)(e32 - (uint32_t)srow[q] * (uint32_t)nact);
      } else {
        const int64_t e = sval[q] ? ent : 0;
        srow[q] = e / nact;
        scol[q] = (int)(e - srow[q] * nact);
      }
    }
    // every operand of the super tile in flight at once (R too: it is
    // needed on the Jacobi path, which most super tiles take)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      sth[q] = theta[scol[q]];
      sdm[q] = diag[srow[q]];
      srr[q] = rho[srow[q]];
      sr[q] = sval[q] ? R[srow[q] * ld + scol[q]] : T(0);
    }
    bool any = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      sdm[q] -= sth[q];
      any |= sval[q] && fabs(sdm[q]) <= kMlpWindow * srr[q];
    }
    const bool listed = __ballot(any) != 0;
    if (lane == 0) tflags[st] = listed ? 1 : 0;
    if (listed) continue;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (!sval[q]) continue;
      const float dm = (float)sdm[q];
      const float delta = (float)(kPrecondGuard * fmax(1.0, fabs(sth[q])));
      const float qq = fmaxf(dm * dm + 0.0f * 0.0f, delta * delta);
      R[srow[q] * ld + scol[q]] = (T)((double)sr[q] * (double)__frsqrt_rn(qq));
    }
  }
}

template <typename T, int MT>
__global__ __launch_bounds__(256, 2) void k_mlp_apply_bf16(T* __restrict__ R, int64_t ld, int nact,
                                                        int64_t n,
                                                        const double* __restrict__ theta,
                                                        const double* __restrict__ diag,
                                                        const double* __restrict__ rho,
                                                        const double* __restrict__ sptr,
                                                        const float* __restrict__ wts,
                                                        const int* __restrict__ mask,
                                                        uint64_t mbits,
                                                        int* __restrict__ flags,
                                                        const int* __restrict__ tflags) {
  constexpr int kBS = kH + 8;  // padded row stride of the bf16 W2 copy
  __shared__ float4 w1s[kH];  // (W1[k][0..2], b1[k])
  __shared__ __attribute__((aligned(16))) __bf16 w2s[kH * kBS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  for (int k = threadIdx.x; k < kH; k += blockDim.x)
    w1s[k] = make_float4(wts[oW1 + 3 * k], wts[oW1 + 3 * k + 1], wts[oW1 + 3 * k + 2], wts[oB1 + k]);
  for (int idx = threadIdx.x; idx < kH * kH; idx += blockDim.x)
    w2s[(idx / kH) * kBS + (idx % kH)] = (__bf16)wts[oW2 + idx];
  float b2r[8], w3r[8];
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    b2r[nt] = wts[oB2 + 16 * nt + r];
    w3r[nt] = wts[oW3 + 16 * nt + r];
  }
  const float b3 = wts[oB3];
  const double s = *sptr;
  const double inv_s = 1.0 / s;
  __syncthreads();
  const int64_t total = n * nact;
  constexpr int E = 16 * MT;  // entries per wave tile
  const int64_t nwt = (total + E - 1) / E;
  // the super tiles (kSE entries) that k_mlp_screen flagged as holding
  // entries inside the window, each taken as kSE / E tiles
  constexpr int kSE = kMlpSuper, kTS = kSE / E;
  // wave w takes super tiles w, w + nw, w + 2 nw, ...: their flags are read
  // 64 at a time (one per lane) and the flagged ones processed in order
  const int64_t nst = (total + kSE - 1) / kSE;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave, nw = (int64_t)gridDim.x * 4;
  for (int64_t jb = 0; gw + jb * nw < nst; jb += 64) {
    const int64_t mine = gw + (jb + lane) * nw;
    uint64_t pend = __ballot(mine < nst && tflags[mine] != 0);
    while (pend != 0) {
      const int bit = __builtin_ctzll(pend);
      pend &= pend - 1;
      const int64_t st = gw + (jb + bit) * nw;
      for (int u = 0; u < kTS; ++u) {
        const int64_t wt = st * kTS + u;
        if (wt >= nwt) break;
        // keep the weight reads inside the loop (LDS re-reads are cheap; holding
        // every fragment in registers for the whole kernel would cap occupancy)
        asm volatile("" ::: "memory");
        // lane l < E owns entry l of the tile: its operands are loaded once
        const int64_t ent = wt * E + lane;
        const bool valid = lane < E && ent < total;
        int64_t row = 0;
        int col = 0;
        double th = 0.0, dmd = 0.0, rr = 0.0;
        if (valid) {
          row = ent / nact;
          col = (int)(ent - row * nact);
          th = theta[col];
          dmd = diag[row] - th;
          rr = rho[row];
        }
        const bool inside = valid && fabs(dmd) <= kMlpWindow * rr;
        // the net only acts inside the window: a tile without such entries takes
        // the Jacobi step everywhere and skips it
        float yv = 0.0f;
        if (__ballot(inside) != 0) {
          // features (fp32 logs of the fp64 difference d - theta); the four
          // lanes that hold an entry's A rows read them with shuffles
          float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
          if (valid) {
            f0 = __logf((float)(fabs(dmd) * inv_s) + 1e-6f);
            f1 = (float)(th * inv_s);
            f2 = __logf((float)(rr * inv_s) + 1e-6f);
          }
          float ph[MT][3];
    #pragma unroll
          for (int t = 0; t < MT; ++t) {
            ph[t][0] = __shfl(f0, 16 * t + r, 64);
            ph[t][1] = __shfl(f1, 16 * t + r, 64);
            ph[t][2] = __shfl(f2, 16 * t + r, 64);
          }
          f32x4 acc[MT][8];
    #pragma unroll
          for (int t = 0; t < MT; ++t)
    #pragma unroll
            for (int nt = 0; nt < 8; ++nt) acc[t][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            bf16x8 bq[8];
    #pragma unroll
            for (int nt = 0; nt < 8; ++nt)
              bq[nt] =
                  *reinterpret_cast<const bf16x8*>(w2s + (16 * nt + r) * kBS + 32 * ks + 8 * g);
    #pragma unroll
            for (int t = 0; t < MT; ++t) {
              bf16x8 a;
    #pragma unroll
              for (int j = 0; j < 8; ++j) {
                const float4 w = w1s[32 * ks + 8 * g + j];
                const float z = w.w + w.x * ph[t][0] + w.y * ph[t][1] + w.z * ph[t][2];
                a[j] = (__bf16)silu_fast(z);
              }
    #pragma unroll
              for (int nt = 0; nt < 8; ++nt)
                acc[t][nt] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bq[nt], acc[t][nt], 0, 0, 0);
            }
          }
          // layer 3: y of entry 16 t + 4 g + i, summed over the 16 lanes of segment g
          float y[MT][4];
    #pragma unroll
          for (int t = 0; t < MT; ++t) {
    #pragma unroll
            for (int i = 0; i < 4; ++i) y[t][i] = 0.0f;
    #pragma unroll
            for (int nt = 0; nt < 8; ++nt)
    #pragma unroll
              for (int i = 0; i < 4; ++i)
                y[t][i] = fmaf(w3r[nt], silu_fast(acc[t][nt][i] + b2r[nt]), y[t][i]);
    #pragma unroll
            for (int i = 0; i < 4; ++i)
    #pragma unroll
              for (int off = 8; off >= 1; off >>= 1) y[t][i] += __shfl_xor(y[t][i], off, 16);
          }
          // entry L's y sits in segment (L % 16) / 4, slot (t = L / 16, i = L % 4)
          const int src = 16 * ((lane & 15) >> 2);
    #pragma unroll
          for (int t = 0; t < MT; ++t)
    #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float v = __shfl(y[t][i], src, 64);
              if ((lane >> 4) == t && (lane & 3) == i) yv = v;
            }
          yv += b3;
        }
        // epilogue: w = r / sqrt((d - theta)^2 + c^2), floored at the guard
        if (valid) {
          bool jac = !inside || ((mbits >> col) & 1) != 0 || (mask != nullptr && mask[col] != 0);
          float c = 0.0f;
          if (!jac) {
            // c = s softplus(y), fp32 (the net itself ran in bf16)
            c = (float)s * (fmaxf(yv, 0.0f) + __logf(1.0f + __expf(-fabsf(yv))));
            if (!isfinite(c)) {
              if (flags) flags[col] = 1;
              c = 0.0f;
            }
          }
          const float dm = (float)dmd;
          const float delta = (float)(kPrecondGuard * fmax(1.0, fabs(th)));
          const float q = fmaxf(dm * dm + c * c, delta * delta);
          T* p = R + row * ld + col;
          *p = (T)((double)*p * (double)__frsqrt_rn(q));
        }
      }
    }
  }
}

__global__ void k_grad_reduce(const double* __restrict__ part, int nblk, double* __restrict__ g) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kMlpParams) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * kMlpParams + idx];
  g[idx] = s;
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const double* __restrict__ g, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kMlpParams) return;
  const float gi = (float)g[idx];
  const float mi = b1 * m[idx] + (1.0f - b1) * gi;
  const float vi = b2 * v[idx] + (1.0f - b2) * gi * gi;
  m[idx] = mi;
  v[idx] = vi;
  w[idx] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- features of the operator ------------------------------------------
__global__ void k_csr_offdiag_abs(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const double* __restrict__ val, int64_t n,
                                  double* __restrict__ rho) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] != i) s += fabs(val[e]);
  rho[i] = s;
}

// one wave per row
__global__ void k_dense_offdiag_abs(const double* __restrict__ A, int64_t lda, int64_t n,
                                    double* __restrict__ rho) {
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64)
    if (j != i) s += fabs(A[i * lda + j]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) rho[i] = s;
}

// H = A (x) I + I (x) A + diag(V): rho_(i,j) = ra_i + ra_j with ra the
// off-diagonal absolute row sums of A (computed first into rho[0..na)).
__global__ void k_kron_offdiag_abs(const double* __restrict__ ra, int64_t na,
                                   double* __restrict__ rho) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= na * na) return;
  const int64_t i = idx / na, j = idx - i * na;
  rho[idx] = ra[i] + ra[j];
}

// mean |d| in two fixed-order stages
__global__ void k_absmean_part(const double* __restrict__ d, int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += fabs(d[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_absmean_final(const double* __restrict__ part, int nblk, int64_t n,
                                double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[b];
  *out = s / (double)n;
}

inline int cdiv64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// workgroups of the fp32 tile kernels: one per group of kGroup tiles, at most kMlpBlocks
int mlp_grid(int64_t total) {
  const int64_t groups = (total + kTE * kGroup - 1) / (kTE * kGroup);
  return (int)std::min<int64_t>(groups, kMlpBlocks);
}

}  // namespace

template <typename T>
static hipError_t mlp_apply_bf16_t(T* R, int64_t ld, int nact, int64_t n, const double* theta,
                                   const double* diag, const double* rho, const double* s,
                                   const float* w, const int* mask, uint64_t mbits, int* flags,
                                   int* tflags, int64_t tiles_cap, hipStream_t st) {
  if (n <= 0 || nact <= 0) return hipSuccess;
  constexpr int MT = kMlpTilesPerWave;
  const int64_t nst = (n * nact + kMlpSuper - 1) / kMlpSuper;
  if (tflags == nullptr || nst > tiles_cap) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  const int sgrid = (int)std::min<int64_t>((nst + 3) / 4, 4096);
  hipLaunchKernelGGL((k_mlp_screen<T>), dim3(sgrid), dim3(256), 0, st, R, ld, nact, n, theta, diag,
                     rho, flags, tflags);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // two waves per SIMD (the MFMA path holds ~240 registers): 2 blocks per CU
  hipLaunchKernelGGL((k_mlp_apply_bf16<T, MT>), dim3(512), dim3(256), 0, st, R, ld, nact, n, theta,
                     diag, rho, s, w, mask, mbits, flags, tflags);
  return hipGetLastError();
}

hipError_t mlp_apply_bf16_f64(double* R, int64_t ld, int nact, int64_t n, const double* theta,
                              const double* diag, const double* rho, const double* s,
                              const float* w, const int* mask, uint64_t mbits, int* flags,
                              int* tflags, int64_t tiles_cap, hipStream_t st) {
  return mlp_apply_bf16_t(R, ld, nact, n, theta, diag, rho, s, w, mask, mbits, flags, tflags,
                          tiles_cap, st);
}
hipError_t mlp_apply_bf16_f32(float* R, int64_t ld, int nact, int64_t n, const double* theta,
                              const double* diag, const double* rho, const double* s,
                              const float* w, const int* mask, uint64_t mbits, int* flags,
                              int* tflags, int64_t tiles_cap, hipStream_t st) {
  return mlp_apply_bf16_t(R, ld, nact, n, theta, diag, rho, s, w, mask, mbits, flags, tflags,
                          tiles_cap, st);
}

template <typename T>
static hipError_t mlp_apply_t(T* R, int64_t ld, int nact, int64_t n, const double* theta,
                              const double* diag, const double* rho, const double* s,
                              const float* w, const int* mask, uint64_t mbits, int* flags,
                              hipStream_t st) {
  if (n <= 0 || nact <= 0) return hipSuccess;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_apply<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileBytes);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_mlp_apply<T>, dim3(mlp_grid(n * nact)), dim3(kGT), kTileBytes, st, R, ld,
                     nact, n, theta, diag, rho, s, w, mask, mbits, flags);
  return hipGetLastError();
}

hipError_t mlp_apply_f64(double* R, int64_t ld, int nact, int64_t n, const double* theta,
                         const double* diag, const double* rho, const double* s, const float* w,
                         const int* mask, uint64_t mbits, int* flags, hipStream_t st) {
  return mlp_apply_t(R, ld, nact, n, theta, diag, rho, s, w, mask, mbits, flags, st);
}
hipError_t mlp_apply_f32(float* R, int64_t ld, int nact, int64_t n, const double* theta,
                         const double* diag, const double* rho, const double* s, const float* w,
                         const int* mask, uint64_t mbits, int* flags, hipStream_t st) {
  return mlp_apply_t(R, ld, nact, n, theta, diag, rho, s, w, mask, mbits, flags, st);
}

hipError_t mlp_grad(const double* R, const double* G, int64_t ld, int nact, int64_t n,
                    const double* theta, const double* diag, const double* rho, const double* s,
                    const float* w, double* part, double* grad, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_grad),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileBytes);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int grid = (n > 0 && nact > 0) ? mlp_grid(n * nact) : 0;
  if (grid > 0)
    hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(kGT), kTileBytes, st, R, G, ld, nact, n,
                       theta, diag, rho, s, w, part);
  hipLaunchKernelGGL(k_grad_reduce, dim3(cdiv64(kMlpParams, 256)), dim3(256), 0, st, part, grid,
                     grad);
  return hipGetLastError();
}

hipError_t mlp_adam(float* w, float* m, float* v, const double* g, int t, double lr,
                    hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const float c1 = (float)(1.0 - std::pow(b1, t)), c2 = (float)(1.0 - std::pow(b2, t));
  hipLaunchKernelGGL(k_adam, dim3(cdiv64(kMlpParams, 256)), dim3(256), 0, st, w, m, v, g,
                     (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
  return hipGetLastError();
}

hipError_t offdiag_abs_csr(const int32_t* rp, const int32_t* ci, const double* val, int64_t n,
                           double* rho, hipStream_t st) {
  hipLaunchKernelGGL(k_csr_offdiag_abs, dim3(cdiv64(n, 256)), dim3(256), 0, st, rp, ci, val, n,
                     rho);
  return hipGetLastError();
}
hipError_t offdiag_abs_dense(const double* A, int64_t lda, int64_t n, double* rho,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_dense_offdiag_abs, dim3(cdiv64(n, 4)), dim3(256), 0, st, A, lda, n, rho);
  return hipGetLastError();
}
hipError_t offdiag_abs_kron(const double* A, int64_t na, double* ra_tmp, double* rho,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_dense_offdiag_abs, dim3(cdiv64(na, 4)), dim3(256), 0, st, A, na, na,
                     ra_tmp);
  hipLaunchKernelGGL(k_kron_offdiag_abs, dim3(cdiv64(na * na, 256)), dim3(256), 0, st, ra_tmp, na,
                     rho);
  return hipGetLastError();
}
hipError_t abs_mean(const double* d, int64_t n, double* part, double* out, hipStream_t st) {
  const int grid = (int)std::min<int64_t>(std::max<int64_t>(cdiv64(n, 256), 1), 1024);
  hipLaunchKernelGGL(k_absmean_part, dim3(grid), dim3(256), 0, st, d, n, part);
  hipLaunchKernelGGL(k_absmean_final, dim3(1), dim3(64), 0, st, part, grid, n, out);
  return hipGetLastError();
}

}  // namespace lobpcg
