// lod.hip -- learned level of detail for the ray caster.
//
// The paper truncates the octree at one camera-wide maximum level derived
// from the pixel size (Sec. 2).  Here a small network predicts, per 16 x 16
// pixel tile, the shallowest truncation level whose image stays within a
// relative tolerance of the full-depth image, so coarse-enough regions stop
// the descent early:
//   features  16 probe rays per tile, walked at a coarse level: column
//             integral, the chord-weighted histogram of subtree depths,
//             log-density statistics, pixel footprint;
//   network   32 -> 64 -> 64 -> 64 -> 16 (16 classes = levels 1..16), ReLU,
//             bf16 weights and activations, fp32 accumulation on
//             v_mfma_f32_16x16x32_bf16;
//   plan      (in the network's kernel) softmax; level = first class whose
//             cumulative probability reaches q; tiles whose top probability
//             is below a confidence threshold fall back to full depth; a
//             seeded fraction of tiles is audited (where the tile render
//             cut a cell, rendered again at full depth and compared, pixels
//             off by more than the tolerance overwritten and counted);
//   training  labels from plain renders at every level, cross-entropy with
//             an extra penalty on the probability of too-shallow levels,
//             backward on the MFMA units, Adam on fp32 master weights.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace amr {
namespace lod {

constexpr int kIn = 32, kHid = 64, kOut = 16, kCls = 16, kLv0 = 1, kTile = 16;
// subtree-depth histogram of the probe features: levels 7..16
constexpr int kBins = 10, kBin0 = 7;
// packets checked by one wave of the audit repair launch
constexpr int kRepairPackets = 16;
// The plan's counters (tiles, fallbacks, audited, level sum) are added into
// kStatSlots copies on separate 128-byte lines, picked by block index, so
// that the blocks' atomics do not all wait on one address; the repair launch
// folds the copies into the caller's statistics.
constexpr int kStatSlots = 32, kSlotU64 = 16;
// parameter offsets (floats) in the fp32 master buffer; the bf16 weight
// buffer uses the same offsets
constexpr int oW1 = 0, oB1 = oW1 + kIn * kHid, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid * kHid, oW4 = oB3 + kHid, oB4 = oW4 + kHid * kOut, kParams = oB4 + kOut;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16, round to nearest even (inputs are finite)
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

__device__ inline f32x4 mfma(const u16x8& a, const u16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// MFMA operand layout (v_mfma_f32_16x16x32_bf16): lane l owns A row l % 16
// and B column l % 16, eight consecutive k starting at 8 (l / 16); it
// receives D rows 4 (l / 16) .. +3 of column l % 16.

// One 16 x 16 output block of a 16-row activation tile (A, row-major in LDS,
// row stride lda, K = nk * 32, rows k < kvalid) times B = W^T:
// B[k][n] = W[(col0 + n) * ldw + k].
__device__ inline f32x4 block_lds_x_wt(const uint16_t* A, int lda, const uint16_t* W, int ldw, int col0, int nk,
                                       int kvalid) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < nk; ++ks) {
    u16x8 a, b;
    for (int j = 0; j < 8; ++j) {
      const int k = ks * 32 + g * 8 + j;
      a[j] = k < kvalid ? A[r * lda + k] : (uint16_t)0;
      b[j] = k < kvalid ? W[(col0 + r) * ldw + k] : (uint16_t)0;
    }
    acc = mfma(a, b, acc);
  }
  return acc;
}

// ------------------------------------------------- lane exchange (DPP)
// x from another lane of the same 16-lane row, by a DPP move (a VALU
// operation, no trip through LDS); lanes without a source read 0.
template <int kCtrl>
__device__ inline float dpp_f32(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, 0xF, 0xF, false));
}
// DPP controls: quad_perm [1,0,3,2] and [2,3,0,1] pair lanes l ^ 1 and l ^ 2;
// row_half_mirror pairs l with 7 - l inside each 8 lanes, row_mirror l with
// 15 - l.  After the two quad steps every lane of a quad holds the same
// value, and after the half mirror every lane of an 8-lane half, so each
// level pairs the same two partial results as an xor butterfly would: the
// reductions below give every lane of the row the same value, bit for bit
// that of the butterfly (addition and max are commutative).
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
__device__ inline float row16_sum(float x) {
  x += dpp_f32<kDppXor1>(x);
  x += dpp_f32<kDppXor2>(x);
  x += dpp_f32<kDppHalfMirror>(x);
  x += dpp_f32<kDppMirror>(x);
  return x;
}
__device__ inline float row16_max(float x) {
  x = fmaxf(x, dpp_f32<kDppXor1>(x));
  x = fmaxf(x, dpp_f32<kDppXor2>(x));
  x = fmaxf(x, dpp_f32<kDppHalfMirror>(x));
  x = fmaxf(x, dpp_f32<kDppMirror>(x));
  return x;
}
// Inclusive prefix sum over the lanes of a row (row_shr by 1, 2, 4, 8: lane
// r adds lane r - d, or 0 below d).
__device__ inline float row16_scan(float x) {
  x += dpp_f32<0x111>(x);
  x += dpp_f32<0x112>(x);
  x += dpp_f32<0x114>(x);
  x += dpp_f32<0x118>(x);
  return x;
}

// ------------------------------------------------------------------ plan
// SplitMix64 finaliser (Steele, Lea and Flood, 2014), high 32 bits: the
// audited-tile selection.
__device__ inline uint32_t hash32(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return (uint32_t)((x ^ (x >> 31)) >> 32);
}

struct PlanArgs {
  float q, conf_thresh;
  int full_level;
  float audit_frac;
  uint64_t audit_seed;
  const int8_t* forced;            // optional per-tile levels that replace the prediction
  int8_t* level;                   // out: per-tile level
  uint8_t* audit;                  // out: per-tile audit flag
  unsigned long long* slots;       // kStatSlots x {tiles, fallbacks, audited, level sum}, kSlotU64 apart
};

// Level of one tile from its kCls class logits, computed by the 16 lanes of
// a lane group, lane r holding class r (zc): the first class whose
// cumulative softmax probability reaches q, or full depth when the top
// probability is below the confidence threshold.  Max, sum and the
// cumulative sum are reductions and a scan inside the 16-lane row (DPP);
// every lane of the group returns the same level.
__device__ inline int plan_group(float zc, int64_t t, const PlanArgs& A, bool& fallback) {
  static_assert(kCls == 16, "one class per lane of a 16-lane group");
  const float m = row16_max(zc);
  const float e = expf(zc - m);
  const float sum = row16_sum(e);
  const float pc = e / sum;
  const float pmax = row16_max(pc);
  const float cdf = row16_scan(pc);  // inclusive scan over the classes
  const unsigned long long hit = __ballot(cdf >= A.q);
  const unsigned grp = (unsigned)(hit >> (threadIdx.x & 48)) & 0xFFFFu;  // this lane group's classes
  int L = kLv0 + (grp ? __ffs(grp) - 1 : kCls - 1);
  fallback = !(pmax >= A.conf_thresh) || A.conf_thresh >= 1.f;
  if (fallback) L = A.full_level;
  if (A.forced) L = A.forced[t];
  if (L > A.full_level) L = A.full_level;
  if (L < 0) L = 0;
  return L;
}

__device__ inline bool audit_draw(int64_t t, const PlanArgs& A) {
  return A.audit_frac >= 1.f || (double)hash32(A.audit_seed * 0x100000001b3ULL + (uint64_t)t) <
                                    (double)A.audit_frac * 4294967296.0;
}

// --------------------------------------------------------------- forward
// A 16-row activation tile (A, row-major in LDS, row stride kHid, K = nk *
// 32) times this lane's B operand held in registers (b[ks]: the eight
// weights of column l % 16, rows ks * 32 + 8 (l / 16) .. +7).
__device__ inline f32x4 lds_rows_x_regs(const uint16_t* A, const u16x8* b, int nk) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < nk; ++ks) {
    u16x8 a;
    for (int j = 0; j < 8; ++j) a[j] = A[r * kHid + ks * 32 + g * 8 + j];
    acc = mfma(a, b[ks], acc);
  }
  return acc;
}

// One block = 16 samples, kFwdWaves = 4 waves.  Wave v computes columns
// 16 v .. 16 v + 15 of each hidden layer, with its weight columns and biases
// loaded into registers once at the start; the block exchanges the layers'
// activations through LDS.  Every wave computes the 16 logits (one column
// block) of the 16 samples.  X: [n][32] bf16.  Wb: bf16 weights, P: fp32
// parameters (biases).  logits: [n][16] fp32 (written by wave 0).  acts
// (optional): [3][n][64] bf16 post-ReLU activations, for the backward pass.
// kPlan: wave v then plans samples 4 g + v (plan_group, lane group g) and the
// block adds its counts to one of the statistics slots.
constexpr int kFwdWaves = 4;
static_assert(kFwdWaves * 16 == kHid, "one column block of the hidden layers per wave");
template <bool kPlan>
__global__ __launch_bounds__(64 * kFwdWaves) void k_fwd(const uint16_t* __restrict__ X, int64_t n,
                                                        const uint16_t* __restrict__ Wb,
                                                        const float* __restrict__ P, float* __restrict__ logits,
                                                        uint16_t* __restrict__ acts, PlanArgs plan) {
  static_assert(kIn == 32 && kHid == 64 && kOut == 16, "operand layout of this kernel");
  __shared__ uint16_t act[2][16 * kHid];
  __shared__ unsigned long long cnt[kFwdWaves][4];
  const int lane = threadIdx.x & 63, v = (int)(threadIdx.x >> 6), r = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 16;
  const int col = v * 16 + r;
  // this lane's B operands: rows ks * 32 + 8 g + j of its column
  u16x8 b1[1], b2[2], b3[2], b4[2];
  for (int j = 0; j < 8; ++j) {
    b1[0][j] = Wb[oW1 + (g * 8 + j) * kHid + col];
    for (int ks = 0; ks < 2; ++ks) {
      const int k = ks * 32 + g * 8 + j;
      b2[ks][j] = Wb[oW2 + k * kHid + col];
      b3[ks][j] = Wb[oW3 + k * kHid + col];
      b4[ks][j] = Wb[oW4 + k * kOut + r];
    }
  }
  const float bias[3] = {P[oB1 + col], P[oB2 + col], P[oB3 + col]};
  const float bias4 = P[oB4 + r];
  // the input rows (row stride kHid)
  for (int e = (int)threadIdx.x; e < 16 * kIn; e += 64 * kFwdWaves) {
    const int row = e / kIn, k = e % kIn;
    act[0][row * kHid + k] = r0 + row < n ? X[(r0 + row) * kIn + k] : (uint16_t)0;
  }
  __syncthreads();
  for (int L = 0; L < 3; ++L) {
    const uint16_t* in = act[L & 1];
    uint16_t* out = act[(L + 1) & 1];
    const f32x4 acc = L == 0 ? lds_rows_x_regs(in, b1, 1) : lds_rows_x_regs(in, L == 1 ? b2 : b3, 2);
    for (int i = 0; i < 4; ++i) {
      const int row = g * 4 + i;
      float x = acc[i] + bias[L];
      x = x > 0.f ? x : 0.f;
      const uint16_t h = f2bf(x);
      out[row * kHid + col] = h;
      if (acts && r0 + row < n) acts[((int64_t)L * n + r0 + row) * kHid + col] = h;
    }
    __syncthreads();
  }
  const f32x4 acc = lds_rows_x_regs(act[1], b4, 2);
  if (v == 0)
    for (int i = 0; i < 4; ++i) {
      const int64_t row = r0 + g * 4 + i;
      if (row < n) logits[row * kOut + r] = acc[i] + bias4;
    }
  if (!kPlan) return;
  // wave v plans sample 4 g + v: lane group g holds its 16 class logits
  const float z = (v == 0 ? acc[0] : v == 1 ? acc[1] : v == 2 ? acc[2] : acc[3]) + bias4;
  const int64_t row = r0 + g * 4 + v;
  const int64_t tr = row < n ? row : n - 1;  // rows past n plan a copy and store nothing
  bool fb;
  const int L = plan_group(z, tr, plan, fb);
  unsigned long long nv = 0, nf = 0, na = 0, lsum = 0;  // counted by lane r = 0 of each group
  if (r == 0 && row < n) {
    const bool au = audit_draw(row, plan);
    plan.level[row] = (int8_t)L;
    plan.audit[row] = au ? 1 : 0;
    nv = 1;
    nf = fb ? 1 : 0;
    na = au ? 1 : 0;
    lsum = (unsigned long long)L;
  }
  for (int off = 32; off >= 16; off >>= 1) {  // the four group leaders (lanes 0, 16, 32, 48)
    nv += __shfl_xor(nv, off, 64);
    nf += __shfl_xor(nf, off, 64);
    na += __shfl_xor(na, off, 64);
    lsum += __shfl_xor(lsum, off, 64);
  }
  if (lane == 0) {
    cnt[v][0] = nv;
    cnt[v][1] = nf;
    cnt[v][2] = na;
    cnt[v][3] = lsum;
  }
  __syncthreads();
  if (threadIdx.x < 4) {  // the block's counts, one atomic each
    unsigned long long t = 0;
    for (int w = 0; w < kFwdWaves; ++w) t += cnt[w][threadIdx.x];
    if (t) atomicAdd(&plan.slots[(blockIdx.x % kStatSlots) * kSlotU64 + threadIdx.x], t);
  }
}

// ------------------------------------------------------------------ loss
// Cross-entropy over the 10 level classes plus lambda times the probability
// of the levels shallower than the label.  dlogits = gradient * scale.
__global__ void k_loss(const float* __restrict__ logits, const int8_t* __restrict__ labels, int64_t n, float lambda,
                       float scale, float* __restrict__ dlogits, float* __restrict__ loss_sum) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float loss = 0.f;
  if (s < n) {
    const float* z = logits + s * kOut;
    float m = z[0];
    for (int c = 1; c < kCls; ++c) m = fmaxf(m, z[c]);
    float p[kCls], sum = 0.f;
    for (int c = 0; c < kCls; ++c) {
      p[c] = expf(z[c] - m);
      sum += p[c];
    }
    int y = labels[s];
    y = y < 0 ? 0 : (y >= kCls ? kCls - 1 : y);
    float S = 0.f, py = 0.f;
    for (int c = 0; c < kCls; ++c) {
      p[c] /= sum;
      if (c < y) S += p[c];
      if (c == y) py = p[c];
    }
    loss = -logf(fmaxf(py, 1e-30f)) + lambda * S;
    float* d = dlogits + s * kOut;
    for (int c = 0; c < kOut; ++c) {
      float gz = 0.f;
      if (c < kCls) gz = p[c] - (c == y ? 1.f : 0.f) + lambda * p[c] * ((c < y ? 1.f : 0.f) - S);
      d[c] = gz * scale;
    }
  }
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_down(loss, off, 64);
  if ((threadIdx.x & 63) == 0 && loss_sum) atomicAdd(loss_sum, loss);
}

// ------------------------------------------------------- backward (data)
// Per 16 samples: dZ4 = bf16(dlogits); dZ3 = (dZ4 W4^T) * [A3 > 0]; ... down
// to dZ1.  dz: [4] planes, dz[0..2] [n][64] (layers 1..3), dz[3] [n][16].
__global__ __launch_bounds__(64) void k_bwd_data(const uint16_t* __restrict__ Wb, const uint16_t* __restrict__ acts,
                                                 const float* __restrict__ dlogits, int64_t n,
                                                 uint16_t* __restrict__ dz) {
  __shared__ uint16_t hA[16 * kHid];
  __shared__ uint16_t hB[16 * kHid];
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 16;
  uint16_t* dz1 = dz;
  uint16_t* dz4 = dz + 3 * n * kHid;
  for (int e = lane; e < 16 * kOut; e += 64) {
    const int row = e / kOut, k = e % kOut;
    const uint16_t h = r0 + row < n ? f2bf(dlogits[(r0 + row) * kOut + k]) : (uint16_t)0;
    hA[row * kHid + k] = h;
    if (r0 + row < n) dz4[(r0 + row) * kOut + k] = h;
  }
  __syncthreads();
  uint16_t* in = hA;
  uint16_t* out = hB;
  const int wofs[3] = {oW4, oW3, oW2}, wout[3] = {kOut, kHid, kHid};
  for (int L = 2; L >= 0; --L) {  // produces dZ_{L+1} (layer L+1 of 1..3)
    const int step = 2 - L;
    for (int cb = 0; cb < kHid / 16; ++cb) {
      f32x4 acc = block_lds_x_wt(in, kHid, Wb + wofs[step], wout[step], cb * 16, wout[step] > 32 ? 2 : 1,
                                 wout[step]);
      const int col = cb * 16 + r;
      for (int i = 0; i < 4; ++i) {
        const int row = g * 4 + i;
        const bool live = r0 + row < n;
        const uint16_t a = live ? acts[((int64_t)L * n + r0 + row) * kHid + col] : (uint16_t)0;
        const float v = bf2f(a) > 0.f ? acc[i] : 0.f;
        const uint16_t h = f2bf(v);
        out[row * kHid + col] = h;
        if (live) dz1[((int64_t)L * n + r0 + row) * kHid + col] = h;
      }
    }
    __syncthreads();
    uint16_t* t = in;
    in = out;
    out = t;
  }
}

// ----------------------------------------------------- backward (weights)
// gW[i][o] += sum over samples of X[s][i] dZ[s][o] for the samples of this
// block's slice (K = samples on the MFMA); gb[o] += sum of dZ[s][o].
__global__ __launch_bounds__(64) void k_wgrad(const uint16_t* __restrict__ Xin, int in_dim,
                                              const uint16_t* __restrict__ dZ, int out_dim, int64_t n,
                                              int64_t slice, float* __restrict__ gW, float* __restrict__ gb) {
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int tiles_o = out_dim / 16;
  const int ti = blockIdx.x / tiles_o, to = blockIdx.x % tiles_o;
  const int64_t s0 = (int64_t)blockIdx.y * slice;
  const int64_t s1 = s0 + slice < n ? s0 + slice : n;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int64_t k0 = s0; k0 < s1; k0 += 32) {
    u16x8 a, b;
    for (int j = 0; j < 8; ++j) {
      const int64_t s = k0 + g * 8 + j;
      const bool ok = s < s1;
      a[j] = ok ? Xin[s * in_dim + ti * 16 + r] : (uint16_t)0;
      b[j] = ok ? dZ[s * out_dim + to * 16 + r] : (uint16_t)0;
      if (ti == 0 && ok) bsum += bf2f(b[j]);
    }
    acc = mfma(a, b, acc);
  }
  for (int i = 0; i < 4; ++i) atomicAdd(&gW[(ti * 16 + g * 4 + i) * out_dim + to * 16 + r], acc[i]);
  if (ti == 0) {
    // lanes r, r+16, r+32, r+48 hold partial sums of column to*16 + r
    bsum += __shfl_xor(bsum, 16, 64);
    bsum += __shfl_xor(bsum, 32, 64);
    if (g == 0) atomicAdd(&gb[to * 16 + r], bsum);
  }
}

// ------------------------------------------------------------------ Adam
__global__ void k_adam(float* __restrict__ P, float* __restrict__ G, float* __restrict__ M, float* __restrict__ V,
                       uint16_t* __restrict__ Wb, int np, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const float gk = G[k];
  const float m = b1 * M[k] + (1.f - b1) * gk;
  const float v = b2 * V[k] + (1.f - b2) * gk * gk;
  M[k] = m;
  V[k] = v;
  const float p = P[k] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  P[k] = p;
  Wb[k] = f2bf(p);
  G[k] = 0.f;
}

__global__ void k_zero_f32(float* p, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0.f;
}

// -------------------------------------------------------------- features
struct FeatVis {
  static constexpr bool kNeedsLength = true;
  const float AMR_GLOBAL* rho;
  const uint8_t AMR_GLOBAL* md;
  float x = 0.f;
  int depth = 0;
  float col = 0.f, len = 0.f, slg = 0.f, slg2 = 0.f;
  float hist[kBins];
  __device__ void fetch(int32_t node) {
    x = rho[node];
    depth = md[node];
  }
  __device__ void fetch0(int32_t node, float v0) {
    x = v0;  // rho is field 0
    depth = md[node];
  }
  __device__ void seg(int32_t, int, float l, int32_t, int32_t, int32_t) {
    col += x * l;
    len += l;
    const float lg = __log2f(fmaxf(x, 1e-30f));  // log2; scaled to log10 after the walk
    slg += l * lg;
    slg2 += l * lg * lg;
    int b = depth - kBin0;
    b = b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
    for (int c = 0; c < kBins; ++c) hist[c] += c == b ? l : 0.f;
  }
};

// One block = one wave = 4 tiles x 16 probe rays at pixel (16 tx + 4 a + 2,
// 16 ty + 4 b + 2) (clamped to the image), each ray walked whole with the
// tree truncated at level lc (probes are short at a coarse level, so a
// split into spans would only repeat the ray set-up).
__global__ __launch_bounds__(64) void k_features(TreeView T, CameraView C, int lc, int tiles_x, int tiles_y,
                                                 float foot_log2, uint16_t* __restrict__ feat,
                                                 unsigned long long* __restrict__ zero_stats,
                                                 unsigned long long* __restrict__ zero_slots) {
  // the LOD render's statistics and counter slots start from zero here (the
  // plan and the repair add to them later on the stream)
  if (zero_stats && blockIdx.x == 0) {
    if (threadIdx.x < 8) zero_stats[threadIdx.x] = 0;
    for (int e = (int)threadIdx.x; e < kStatSlots * kSlotU64; e += (int)blockDim.x) zero_slots[e] = 0;
  }
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (lane >> 4), probe = lane & 15;
  const int ntiles = tiles_x * tiles_y;
  const int tt = tile < ntiles ? tile : ntiles - 1;
  const int ty = tt / tiles_x, tx = tt % tiles_x;
  int i = tx * kTile + (probe & 3) * 4 + 2, j = ty * kTile + (probe >> 2) * 4 + 2;
  i = i < C.W ? i : C.W - 1;
  j = j < C.H ? j : C.H - 1;
  FeatVis v;
  v.rho = T.val;
  v.md = T.maxdepth;
  for (int c = 0; c < kBins; ++c) v.hist[c] = 0.f;
  Ray R;
  Entry E;
  int32_t nseg = 0;
  const bool hit = setup_ray(C, i, j, R, E);
  if (hit) nseg = walk_fast<FeatVis, true>(T, R, E, lc, v);  // the whole ray, to the box
  constexpr float kLog10_2 = 0.30102999566398120f;
  v.slg *= kLog10_2;
  v.slg2 *= kLog10_2 * kLog10_2;
  // reduce over the 16 probes of the tile
  float cmax = v.col;
  float s[15];
  s[0] = v.col;
  s[1] = v.len;
  s[2] = v.slg;
  s[3] = v.slg2;
  s[4] = hit ? 1.f : 0.f;
  for (int c = 0; c < kBins; ++c) s[5 + c] = v.hist[c];
  for (int q = 0; q < 15; ++q) s[q] = row16_sum(s[q]);
  const float segs = row16_sum((float)nseg);
  cmax = row16_max(cmax);
  if (tile >= ntiles) return;
  const float mean_col = s[0] / 16.f;
  const float L = s[1];
  const float mlg = L > 0.f ? s[2] / L : 0.f;
  const float vlg = L > 0.f ? fmaxf(s[3] / L - mlg * mlg, 0.f) : 0.f;
  float f[2];
  for (int h = 0; h < 2; ++h) {
    const int k = probe + 16 * h;
    float x = 0.f;
    if (k == 0) x = log10f(1e-12f + mean_col);
    else if (k == 1) x = log10f(1e-12f + cmax) - log10f(1e-12f + mean_col);
    else if (k >= 2 && k < 2 + kBins) x = L > 0.f ? s[5 + (k - 2)] / L : 0.f;
    else if (k == 12) x = mlg;
    else if (k == 13) x = vlg;
    else if (k == 14) x = foot_log2;
    else if (k == 15) x = s[4] / 16.f;
    else if (k == 16) x = segs / (16.f * 64.f);
    f[h] = x;
  }
  feat[(int64_t)tile * kIn + probe] = f2bf(f[0]);
  feat[(int64_t)tile * kIn + probe + 16] = f2bf(f[1]);
}

// ---------------------------------------------------------------- labels
// Per tile: the first level L (class L - 1) whose image is within tol of the
// full-depth image at every pixel of the tile.  imgs: 16 device pointers
// (levels 1..16); the last is the reference.
struct ImgPtrs {
  const float* p[kCls];
};
__global__ __launch_bounds__(64) void k_labels(ImgPtrs I, int W, int H, int tiles_x, int ntiles, float tol,
                                               int8_t* __restrict__ labels) {
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;
  const int lane = threadIdx.x;
  const int ty = tile / tiles_x, tx = tile % tiles_x;
  int label = kCls - 1;
  for (int c = 0; c < kCls - 1; ++c) {
    float e = 0.f;
    for (int q = lane; q < kTile * kTile; q += 64) {
      const int i = tx * kTile + (q & 15), j = ty * kTile + (q >> 4);
      if (i >= W || j >= H) continue;
      const int64_t pix = (int64_t)j * W + i;
      const float ref = I.p[kCls - 1][pix], x = I.p[c][pix];
      const float d = fabsf(x - ref);
      const float r = ref != 0.f ? d / fabsf(ref) : (d == 0.f ? 0.f : 3.4e38f);
      e = fmaxf(e, r);
    }
    for (int off = 32; off > 0; off >>= 1) e = fmaxf(e, __shfl_xor(e, off, 64));
    if (e <= tol) {
      label = c;
      break;
    }
  }
  if (lane == 0) labels[tile] = (int8_t)label;
}

// ----------------------------------------------------- render and audit
// 8 x 8 packets (inside one 16 x 16 tile), tree truncated at the tile's
// level, every ray walked in two spans by the block's two waves exactly as
// the default plain render does (a tile at full depth is bit-identical to
// it), packet rows dispatched from the middle of the image out.  The walk
// records whether any ray cut a cell (stopped descending at a cell that has
// children).  For a packet of an audited tile (a tile below full depth
// picked for checking) that cut none, the image is the full-depth image
// exactly (the same cells, chords and summation order) and is copied to the
// full-depth planes; one that cut a cell is walked again at full depth by
// the same block right away (stats[5] counts these), so that walk overlaps
// the rest of the image instead of following it (k_render_tiles below).

// One walk of a packet's rays with the tree truncated at lw: wave w walks
// span w of its lane's ray (cut tracking on), wave 1 leaves its partial sums
// in part for wave 0.
template <int OP, bool STD>
__device__ __forceinline__ void tile_walk(const RenderArgs& A, int i, int j, bool in, int w, int lw, float* part,
                                          Partial& P, bool& cut) {
  partial_init<OP>(P);
  cut = false;
  Ray R;
  Entry E;
  if (in && setup_ray(A.c, i, j, R, E) && span_setup(R, E, A.t.base < lw ? A.t.base : lw, 2, w)) {
    if (w == 1)  // the last span runs to the box
      walk_span<OP, true, true, STD>(A.t, R, E, lw, A.field, A.wfield, A.los, P, &cut);
    else
      walk_span<OP, false, true, STD>(A.t, R, E, lw, A.field, A.wfield, A.los, P, &cut);
  }
  if (w == 1) {
    float* q = part + (threadIdx.x & 63);
    q[0] = P.s0;
    q[64] = P.c0;
    q[128] = P.s1;
    q[192] = P.c1;
  }
}

template <int OP>
__device__ __forceinline__ void tile_finish(const float* part, Partial& P, float& o, float& x) {
  const float* q = part + (threadIdx.x & 63);
  partial_merge<OP>(P, Partial{q[0], q[64], q[128], q[192]});
  o = 0.f;
  x = 0.f;
  partial_finish<OP>(P, o, x);
}

// STD: the render may take walk_span's kStd walk (std_walk).
template <int OP, bool STD = false>
__global__ __launch_bounds__(128, OP == kOpWMean ? 7 : 8) void k_render_tiles(RenderArgs A, const int8_t* __restrict__ level,
                                                      const uint8_t* __restrict__ audit, int tiles_x,
                                                      float* __restrict__ full_out, float* __restrict__ full_aux,
                                                      unsigned long long* __restrict__ stats) {
  __shared__ float part[4 * 64];
  const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
  const int packet = center_out((int)blockIdx.x, A.packets_x, A.packets_y);
  const int ty = packet / A.packets_x, tx = packet - ty * A.packets_x;
  const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
  const bool in = ty < A.packets_y && i < A.c.W && j < A.c.H;
  const int64_t pix = (int64_t)j * A.c.W + i;
  // a packet lies inside one tile: its level and audit flag are block-uniform
  const int t = (ty * 8 / kTile) * tiles_x + (tx * 8 / kTile);
  const int L = level[t];
  const bool audited = audit[t] && L < A.max_level;
  Partial P;
  bool cut;
  float o, x;
  tile_walk<OP, STD>(A, i, j, in, w, L, part, P, cut);
  // (also the barrier for part) did a ray of either span cut a cell?
  const bool again = audited ? __syncthreads_or(cut ? 1 : 0) != 0 : (__syncthreads(), false);
  if (w == 0 && in) {
    tile_finish<OP>(part, P, o, x);
    A.out[pix] = o;
    if (OP == kOpWMean && A.aux) A.aux[pix] = x;
    if (audited && !again) {  // no cell cut: this is the full-depth image
      full_out[pix] = o;
      if (OP == kOpWMean) full_aux[pix] = x;
    }
  }
  if (!again) return;  // block-uniform
  if (threadIdx.x == 0) atomicAdd(&stats[5], 1ull);
  __syncthreads();  // wave 0 has read part before wave 1 writes it again
  tile_walk<OP, STD>(A, i, j, in, w, A.max_level, part, P, cut);
  __syncthreads();
  if (w == 0 && in) {
    tile_finish<OP>(part, P, o, x);
    full_out[pix] = o;
    if (OP == kOpWMean) full_aux[pix] = x;
  }
}

template <int OP>
__global__ __launch_bounds__(64) void k_audit_repair(RenderArgs A, const int8_t* __restrict__ level,
                                                     const uint8_t* __restrict__ audit, int tiles_x, float tol,
                                                     const float* __restrict__ full_out,
                                                     const float* __restrict__ full_aux, unsigned long long* stats,
                                                     const unsigned long long* __restrict__ slots) {
  const int lane = threadIdx.x & 63;
  const int np = A.packets_x * A.packets_y;
  if (blockIdx.x == 0) {  // the plan's counters: sum of the slots
    static_assert(kStatSlots <= 64, "one lane per slot");
    unsigned long long v[4] = {0, 0, 0, 0};
    if (lane < kStatSlots)
      for (int k = 0; k < 4; ++k) v[k] = slots[lane * kSlotU64 + k];
    for (int off = 32; off > 0; off >>= 1)
      for (int k = 0; k < 4; ++k) v[k] += __shfl_xor(v[k], off, 64);
    if (lane == 0) {
      stats[0] = v[0];
      stats[1] = v[1];
      stats[2] = v[2];
      stats[4] = v[3];
    }
  }
  static_assert(kRepairPackets <= 64, "one lane per packet reads the flags");
  // kRepairPackets consecutive packets per wave: lane k reads the flags of
  // packet k's tile (one round trip), then the wave walks the flagged ones
  const int pk = (int)blockIdx.x * kRepairPackets + lane;
  bool flagged = false;
  if (lane < kRepairPackets && pk < np) {
    const int ty = pk / A.packets_x, tx = pk - ty * A.packets_x;
    const int t = (ty * 8 / kTile) * tiles_x + (tx * 8 / kTile);
    flagged = audit[t] && level[t] < A.max_level;
  }
  unsigned long long todo = __ballot(flagged);
  unsigned long long nbad = 0;
  while (todo) {
    const int k = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const int packet = (int)blockIdx.x * kRepairPackets + k;
    const int ty = packet / A.packets_x, tx = packet - ty * A.packets_x;
    const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
    if (i >= A.c.W || j >= A.c.H) continue;
    const int64_t pix = (int64_t)j * A.c.W + i;
    const float o = A.out[pix], of = full_out[pix];
    const float d = fabsf(o - of);
    const bool bad = of != 0.f ? d > tol * fabsf(of) : d != 0.f;
    if (bad) {
      A.out[pix] = of;
      if (OP == kOpWMean && A.aux) A.aux[pix] = full_aux[pix];
      ++nbad;
    }
  }
  for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off, 64);
  if (lane == 0 && nbad) atomicAdd(&stats[3], nbad);
}

}  // namespace lod
}  // namespace amr

using namespace amr;
using namespace amr::lod;

struct amr_lod_model {
  float* P = nullptr;   // fp32 master parameters
  float* G = nullptr;   // gradients
  float* M = nullptr;   // Adam moments
  float* V = nullptr;
  uint16_t* Wb = nullptr;  // bf16 copy
  int64_t step = 0;
  amr_lod_config cfg;
};

namespace {

amr_status upload_params(amr_lod_model* m, const std::vector<float>& p) {
  std::vector<uint16_t> b(kParams);
  for (int k = 0; k < kParams; ++k) b[k] = f2bf(p[k]);
  if (hipMemcpy(m->P, p.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->Wb, b.data(), sizeof(uint16_t) * kParams, hipMemcpyHostToDevice) != hipSuccess)
    return fail(AMR_EHIP, "parameter upload failed");
  return AMR_OK;
}

amr_lod_model* alloc_model() {
  amr_lod_model* m = new (std::nothrow) amr_lod_model();
  if (!m) return nullptr;
  hipError_t e = hipMalloc((void**)&m->P, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->G, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->M, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->V, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->Wb, sizeof(uint16_t) * kParams);
  if (e == hipSuccess) e = hipMemset(m->G, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMemset(m->M, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMemset(m->V, 0, sizeof(float) * kParams);
  if (e != hipSuccess) {
    amr_lod_free(m);
    return nullptr;
  }
  return m;
}

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

const uint32_t kMagic = 0x414d524cu;  // "AMRL"
const uint32_t kVersion = 1;

}  // namespace

extern "C" {

int32_t amr_lod_param_count(void) { return kParams; }

amr_status amr_lod_create(const amr_lod_config* cfg, uint64_t seed, amr_lod_model** out) {
  if (!out) return fail(AMR_EINVAL, "null output");
  *out = nullptr;
  amr_lod_model* m = alloc_model();
  if (!m) return fail(AMR_ENOMEM, "model allocation failed");
  if (cfg) m->cfg = *cfg;
  else m->cfg = amr_lod_config{7, 0.99f, 0.5f, 1e-3f, 0.02f, 0};
  // He-normal weights from a counter-based SplitMix64 stream, zero biases
  std::vector<float> p(kParams, 0.f);
  struct L {
    int ofs, fan_in, fan_out;
  } layers[4] = {{oW1, kIn, kHid}, {oW2, kHid, kHid}, {oW3, kHid, kHid}, {oW4, kHid, kOut}};
  uint64_t ctr = 0;
  for (const L& l : layers) {
    const double sd = std::sqrt(2.0 / l.fan_in) * (l.ofs == oW4 ? 0.25 : 1.0);
    for (int k = 0; k < l.fan_in * l.fan_out; ++k) {
      const double u1 = ((mix64(seed * 0x9e3779b97f4a7c15ULL + 2 * ctr + 1) >> 11) + 0.5) * 0x1.0p-53;
      const double u2 = ((mix64(seed * 0x9e3779b97f4a7c15ULL + 2 * ctr + 2) >> 11) + 0.5) * 0x1.0p-53;
      ++ctr;
      p[l.ofs + k] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
  }
  amr_status st = upload_params(m, p);
  if (st) {
    amr_lod_free(m);
    return st;
  }
  *out = m;
  return AMR_OK;
}

void amr_lod_free(amr_lod_model* m) {
  if (!m) return;
  if (m->P) (void)hipFree(m->P);
  if (m->G) (void)hipFree(m->G);
  if (m->M) (void)hipFree(m->M);
  if (m->V) (void)hipFree(m->V);
  if (m->Wb) (void)hipFree(m->Wb);
  delete m;
}

amr_status amr_lod_get_config(const amr_lod_model* m, amr_lod_config* cfg) {
  if (!m || !cfg) return fail(AMR_EINVAL, "null argument");
  *cfg = m->cfg;
  return AMR_OK;
}
amr_status amr_lod_set_config(amr_lod_model* m, const amr_lod_config* cfg) {
  if (!m || !cfg) return fail(AMR_EINVAL, "null argument");
  m->cfg = *cfg;
  return AMR_OK;
}

amr_status amr_lod_get_params(const amr_lod_model* m, float* host) {
  if (!m || !host) return fail(AMR_EINVAL, "null argument");
  if (hipMemcpy(host, m->P, sizeof(float) * kParams, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(AMR_EHIP, "download failed");
  return AMR_OK;
}
amr_status amr_lod_set_params(amr_lod_model* m, const float* host) {
  if (!m || !host) return fail(AMR_EINVAL, "null argument");
  std::vector<float> p(host, host + kParams);
  return upload_params(m, p);
}
amr_status amr_lod_get_grads(const amr_lod_model* m, float* host) {
  if (!m || !host) return fail(AMR_EINVAL, "null argument");
  if (hipMemcpy(host, m->G, sizeof(float) * kParams, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(AMR_EHIP, "download failed");
  return AMR_OK;
}

amr_status amr_lod_save(const amr_lod_model* m, const char* path) {
  if (!m || !path) return fail(AMR_EINVAL, "null argument");
  std::vector<float> p(kParams), a(kParams), b(kParams);
  if (hipMemcpy(p.data(), m->P, sizeof(float) * kParams, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(a.data(), m->M, sizeof(float) * kParams, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(b.data(), m->V, sizeof(float) * kParams, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(AMR_EHIP, "download failed");
  FILE* f = fopen(path, "wb");
  if (!f) return fail(AMR_EINVAL, "cannot open file");
  const uint32_t hdr[4] = {kMagic, kVersion, (uint32_t)kParams, (uint32_t)sizeof(amr_lod_config)};
  bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1 && fwrite(&m->cfg, sizeof(m->cfg), 1, f) == 1 &&
            fwrite(&m->step, sizeof(m->step), 1, f) == 1 && fwrite(p.data(), 4, kParams, f) == (size_t)kParams &&
            fwrite(a.data(), 4, kParams, f) == (size_t)kParams && fwrite(b.data(), 4, kParams, f) == (size_t)kParams;
  ok = (fclose(f) == 0) && ok;
  return ok ? AMR_OK : fail(AMR_EINVAL, "write failed");
}

amr_status amr_lod_load(const char* path, amr_lod_model** out) {
  if (!path || !out) return fail(AMR_EINVAL, "null argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(AMR_EINVAL, "cannot open file");
  uint32_t hdr[4];
  amr_lod_config cfg;
  int64_t step = 0;
  std::vector<float> p(kParams), a(kParams), b(kParams);
  bool ok = fread(hdr, sizeof(hdr), 1, f) == 1;
  if (ok && (hdr[0] != kMagic || hdr[1] != kVersion || hdr[2] != (uint32_t)kParams ||
             hdr[3] != (uint32_t)sizeof(amr_lod_config))) {
    fclose(f);
    return fail(AMR_EMODEL, "LOD model file has another format or version");
  }
  ok = ok && fread(&cfg, sizeof(cfg), 1, f) == 1 && fread(&step, sizeof(step), 1, f) == 1 &&
       fread(p.data(), 4, kParams, f) == (size_t)kParams && fread(a.data(), 4, kParams, f) == (size_t)kParams &&
       fread(b.data(), 4, kParams, f) == (size_t)kParams;
  fclose(f);
  if (!ok) return fail(AMR_EMODEL, "truncated LOD model file");
  amr_lod_model* m = alloc_model();
  if (!m) return fail(AMR_ENOMEM, "model allocation failed");
  m->cfg = cfg;
  m->step = step;
  amr_status st = upload_params(m, p);
  if (!st && (hipMemcpy(m->M, a.data(), 4 * kParams, hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(m->V, b.data(), 4 * kParams, hipMemcpyHostToDevice) != hipSuccess))
    st = fail(AMR_EHIP, "upload failed");
  if (st) {
    amr_lod_free(m);
    return st;
  }
  *out = m;
  return AMR_OK;
}

int64_t amr_lod_tiles(int32_t W, int32_t H) {
  return (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
}

namespace {
amr_status launch_features(const amr_tree* t, const amr_camera* cam, int32_t coarse_level, uint16_t* feat,
                           unsigned long long* zero_stats, unsigned long long* zero_slots, amr_stream s) {
  amr_status cs = check_render_common(t, cam);
  if (cs) return cs;
  if (!feat) return fail(AMR_EINVAL, "null argument");
  if (coarse_level < 0 || coarse_level > kMaxLevel) return fail(AMR_EINVAL, "bad level");
  const int tx = (cam->W + kTile - 1) / kTile, ty = (cam->H + kTile - 1) / kTile;
  // log2 of the pixel footprint in units of the coarse cell side: the
  // camera record's step length over |F| (perspective, at unit distance) or
  // the plane step (orthographic)
  double step = 0, fl = 0;
  for (int k = 0; k < 3; ++k) {
    step += (double)cam->V[k] * (double)cam->V[k];
    fl += (double)cam->F[k] * (double)cam->F[k];
  }
  const double foot = cam->kind == 0 ? 2.0 * std::sqrt(step / fl) : 2.0 * std::sqrt(step) * 0x1.0p-28;
  const float fl2 = (float)std::log2(foot * std::ldexp(1.0, coarse_level) + 1e-30);
  const int ntiles = tx * ty;
  hipLaunchKernelGGL(k_features, dim3((ntiles + 3) / 4), dim3(64), 0, (hipStream_t)s, t->view, camera_view(*cam),
                     coarse_level, tx, ty, fl2, feat, zero_stats, zero_slots);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, hipGetErrorString(e));
}
}  // namespace

amr_status amr_lod_features(const amr_tree* t, const amr_camera* cam, int32_t coarse_level, uint16_t* feat,
                            amr_stream s) {
  return launch_features(t, cam, coarse_level, feat, nullptr, nullptr, s);
}

amr_status amr_lod_forward(const amr_lod_model* m, const uint16_t* feat, int64_t n, float* logits, uint16_t* acts,
                           amr_stream s) {
  if (!m || !feat || !logits || n < 0) return fail(AMR_EINVAL, "null argument");
  if (n == 0) return AMR_OK;
  const unsigned blocks = (unsigned)((n + 15) / 16);
  hipLaunchKernelGGL(k_fwd<false>, dim3(blocks), dim3(64 * kFwdWaves), 0, (hipStream_t)s, feat, n, m->Wb, m->P,
                     logits, acts, PlanArgs{});
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, hipGetErrorString(e));
}

amr_status amr_lod_loss(const float* logits, const int8_t* labels, int64_t n, float lambda, float scale,
                        float* dlogits, float* loss_sum, amr_stream s) {
  if (!logits || !labels || !dlogits || n < 0) return fail(AMR_EINVAL, "null argument");
  if (n == 0) return AMR_OK;
  hipLaunchKernelGGL(k_loss, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)s, logits, labels, n,
                     lambda, scale, dlogits, loss_sum);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, hipGetErrorString(e));
}

amr_status amr_lod_backward(amr_lod_model* m, const uint16_t* feat, const uint16_t* acts, const float* dlogits,
                            int64_t n, uint16_t* dz, amr_stream s) {
  if (!m || !feat || !acts || !dlogits || !dz || n < 0) return fail(AMR_EINVAL, "null argument");
  if (n == 0) return AMR_OK;
  hipStream_t st = (hipStream_t)s;
  hipLaunchKernelGGL(k_bwd_data, dim3((unsigned)((n + 15) / 16)), dim3(64), 0, st, m->Wb, acts, dlogits, n, dz);
  const int64_t slice = 1024;
  const unsigned ns = (unsigned)((n + slice - 1) / slice);
  struct Ly {
    const uint16_t* x;
    int in;
    const uint16_t* d;
    int out;
    int w, b;
  } ly[4] = {{feat, kIn, dz, kHid, oW1, oB1},
             {acts, kHid, dz + n * kHid, kHid, oW2, oB2},
             {acts + n * kHid, kHid, dz + 2 * n * kHid, kHid, oW3, oB3},
             {acts + 2 * n * kHid, kHid, dz + 3 * n * kHid, kOut, oW4, oB4}};
  for (const Ly& l : ly)
    hipLaunchKernelGGL(k_wgrad, dim3((l.in / 16) * (l.out / 16), ns), dim3(64), 0, st, l.x, l.in, l.d, l.out, n,
                       slice, m->G + l.w, m->G + l.b);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, hipGetErrorString(e));
}

amr_status amr_lod_zero_grads(amr_lod_model* m, amr_stream s) {
  if (!m) return fail(AMR_EINVAL, "null model");
  hipLaunchKernelGGL(k_zero_f32, dim3((kParams + 255) / 256), dim3(256), 0, (hipStream_t)s, m->G, kParams);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, hipGetErrorString(e));
}

amr_status amr_lod_adam_step(amr_lod_model* m, float lr, amr_stream s) {
  if (!m || !(lr > 0.f)) return fail(AMR_EINVAL, "bad argument");
  const float b1 = 0.9f, b2 = 0.999f;
  m->step += 1;
  // bias corrections 1 - beta^t of the fp32 betas the moment updates use,
  // formed in fp64: in fp32 the difference cancels (1 - 0.999^2 would keep
  // only 4 correct digits)
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)m->step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)m->step));
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, (hipStream_t)s, m->P, m->G, m->M, m->V,
                     m->Wb, kParams, lr, b1, b2, 1e-8f, c1, c2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, hipGetErrorString(e));
}

amr_status amr_lod_labels(const float* const* imgs, int32_t W, int32_t H, float tol, int8_t* labels, amr_stream s) {
  if (!imgs || !labels || W < 1 || H < 1) return fail(AMR_EINVAL, "bad argument");
  ImgPtrs P;
  for (int c = 0; c < kCls; ++c) {
    if (!imgs[c]) return fail(AMR_EINVAL, "null image");
    P.p[c] = imgs[c];
  }
  const int tx = (W + kTile - 1) / kTile, ty = (H + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_labels, dim3(tx * ty), dim3(64), 0, (hipStream_t)s, P, W, H, tx, tx * ty, tol, labels);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, hipGetErrorString(e));
}

// Workspace layout (256-byte aligned parts): 256 reserved bytes, features
// (bf16 [tiles][kIn]), logits (fp32 [tiles][kOut]), tile levels and audit
// flags (int8 [tiles] each), then the two full-depth planes of the audit
// (fp32 [H][W] each: value, and weight for WMEAN).
namespace {
int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }
int64_t ws_slots_offset(int32_t W, int32_t H) {
  const int64_t nt = amr_lod_tiles(W, H);
  const int64_t n16 = (nt + 15) / 16 * 16;
  return align256(256 + n16 * kIn * 2 + n16 * kOut * 4 + 2 * n16 + 64);
}
int64_t ws_planes_offset(int32_t W, int32_t H) {
  return ws_slots_offset(W, H) + (int64_t)kStatSlots * kSlotU64 * 8;
}
}  // namespace

int64_t amr_lod_workspace_bytes(int32_t W, int32_t H) {
  return ws_planes_offset(W, H) + 2 * align256((int64_t)W * H * 4);
}

}  // extern "C"

// Device memory for amr_render_lod_noalloc: a file-scope device array, one
// copy per GPU, loaded with the code object and held until the process
// ends.  Host code never passes the array's name to a kernel (on the host
// it is only a stand-in for the symbol): the device address of each GPU's
// copy comes from hipGetSymbolAddress, fetched once per device with that
// device current, and only that address is used.
static constexpr int64_t kNoAllocScratchBytes = int64_t(40) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// The LOD render on a workspace that the caller checked for size and
// alignment (the two entry points below differ only in where it lives).
amr_status render_lod_on(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_lod_model* m,
                         const amr_render_opts* opts, float* out, float* aux, int8_t* tile_levels,
                         const int8_t* forced_levels, void* workspace, int64_t* stats, amr_stream s) {
  amr_render_opts o = opts ? *opts : amr_render_opts{0, 0, 0, -1};
  const int nf = t->info.nfields;
  if (o.field < 0 || o.field + ((op == AMR_WMEAN && o.los_velocity) ? 2 : 0) >= nf)
    return fail(AMR_EINVAL, "field index out of range");
  if (op == AMR_WMEAN && (o.weight_field < 0 || o.weight_field >= nf)) return fail(AMR_EINVAL, "bad weight field");
  const amr_lod_config& c = m->cfg;
  const int tx = (cam->W + kTile - 1) / kTile, ty = (cam->H + kTile - 1) / kTile, nt = tx * ty;
  const int64_t n16 = ((int64_t)nt + 15) / 16 * 16;
  char* w = (char*)workspace;
  uint16_t* feat = (uint16_t*)(w + 256);
  float* logits = (float*)(w + 256 + n16 * kIn * 2);
  int8_t* lev = (int8_t*)(w + 256 + n16 * kIn * 2 + n16 * kOut * 4);
  uint8_t* aud = (uint8_t*)(lev + n16);
  if (tile_levels) lev = tile_levels;
  unsigned long long* st = (unsigned long long*)stats;
  hipStream_t hs = (hipStream_t)s;
  unsigned long long* slots = (unsigned long long*)(w + ws_slots_offset(cam->W, cam->H));
  amr_status r = launch_features(t, cam, std::min(c.coarse_level, cam->max_level), feat, st, slots, s);
  if (r) return r;
  // network and plan in one launch (k_fwd<true>): level and audit flag per tile
  const PlanArgs pa{c.quantile, c.conf_thresh, cam->max_level, c.audit_frac, (uint64_t)c.audit_seed,
                    forced_levels, lev, aud, slots};
  const unsigned fb = (unsigned)((nt + 15) / 16);
  hipLaunchKernelGGL(k_fwd<true>, dim3(fb), dim3(64 * kFwdWaves), 0, hs, feat, (int64_t)nt, m->Wb, m->P, logits,
                     nullptr, pa);
  RenderArgs a;
  a.t = t->view;
  a.c = camera_view(*cam);
  a.field = o.field;
  a.wfield = o.weight_field;
  a.los = op == AMR_WMEAN ? (o.los_velocity ? 1 : 0) : 0;
  a.max_level = cam->max_level;
  a.out = out;
  a.aux = aux;
  a.packets_x = (cam->W + 7) / 8;
  a.packets_y = (cam->H + 7) / 8;
  const unsigned np = (unsigned)(a.packets_x * a.packets_y);
  float* full_out = (float*)(w + ws_planes_offset(cam->W, cam->H));
  float* full_aux = (float*)((char*)full_out + align256((int64_t)cam->W * cam->H * 4));
  const unsigned rb = (np + kRepairPackets - 1) / kRepairPackets;  // repair blocks
  const int opc = op == AMR_SUM ? kOpSum : op == AMR_MAX ? kOpMax : kOpWMean;
  const bool sw = std_walk(opc, a.t, a.field, a.wfield, a.los, a.max_level);  // walk_span's kStd walk
  if (op == AMR_SUM) {
    if (sw)
      hipLaunchKernelGGL((k_render_tiles<kOpSum, true>), dim3(np), dim3(128), 0, hs, a, lev, aud, tx, full_out,
                         full_aux, st);
    else
      hipLaunchKernelGGL(k_render_tiles<kOpSum>, dim3(np), dim3(128), 0, hs, a, lev, aud, tx, full_out, full_aux,
                         st);
    hipLaunchKernelGGL(k_audit_repair<kOpSum>, dim3(rb), dim3(64), 0, hs, a, lev, aud, tx, c.rel_tol, full_out,
                       full_aux, st, slots);
  } else if (op == AMR_MAX) {
    if (sw)
      hipLaunchKernelGGL((k_render_tiles<kOpMax, true>), dim3(np), dim3(128), 0, hs, a, lev, aud, tx, full_out,
                         full_aux, st);
    else
      hipLaunchKernelGGL(k_render_tiles<kOpMax>, dim3(np), dim3(128), 0, hs, a, lev, aud, tx, full_out, full_aux,
                         st);
    hipLaunchKernelGGL(k_audit_repair<kOpMax>, dim3(rb), dim3(64), 0, hs, a, lev, aud, tx, c.rel_tol, full_out,
                       full_aux, st, slots);
  } else {
    if (sw)
      hipLaunchKernelGGL((k_render_tiles<kOpWMean, true>), dim3(np), dim3(128), 0, hs, a, lev, aud, tx, full_out,
                         full_aux, st);
    else
      hipLaunchKernelGGL(k_render_tiles<kOpWMean>, dim3(np), dim3(128), 0, hs, a, lev, aud, tx, full_out,
                         full_aux, st);
    hipLaunchKernelGGL(k_audit_repair<kOpWMean>, dim3(rb), dim3(64), 0, hs, a, lev, aud, tx, c.rel_tol, full_out,
                       full_aux, st, slots);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, hipGetErrorString(e));
}

amr_status check_lod_args(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_lod_model* m,
                          const float* out, const int64_t* stats) {
  amr_status cs = check_render_common(t, cam);
  if (cs) return cs;
  if (!m || !out || !stats) return fail(AMR_EINVAL, "null argument");
  if (op != AMR_SUM && op != AMR_MAX && op != AMR_WMEAN) return fail(AMR_EINVAL, "bad op");
  if ((uintptr_t)stats & 7) return fail(AMR_EINVAL, "misaligned stats");
  return AMR_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

amr_status scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(AMR_EHIP, std::string("hipGetDevice failed: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(AMR_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(AMR_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return AMR_OK;
}

}  // namespace

extern "C" {

amr_status amr_render_lod(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_lod_model* m,
                          const amr_render_opts* opts, float* out, float* aux, int8_t* tile_levels,
                          const int8_t* forced_levels, void* workspace, int64_t workspace_bytes, int64_t* stats,
                          amr_stream s) {
  amr_status cs = check_lod_args(t, cam, op, m, out, stats);
  if (cs) return cs;
  if (!workspace) return fail(AMR_EINVAL, "null workspace");
  if (workspace_bytes < amr_lod_workspace_bytes(cam->W, cam->H)) return fail(AMR_ECAPACITY, "workspace too small");
  if ((uintptr_t)workspace & 255) return fail(AMR_EINVAL, "misaligned workspace");
  return render_lod_on(t, cam, op, m, opts, out, aux, tile_levels, forced_levels, workspace, stats, s);
}

int64_t amr_lod_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

amr_status amr_render_lod_noalloc(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_lod_model* m,
                                  const amr_render_opts* opts, float* out, float* aux, int8_t* tile_levels,
                                  const int8_t* forced_levels, int64_t* stats, amr_stream s) {
  amr_status cs = check_lod_args(t, cam, op, m, out, stats);
  if (cs) return cs;
  const int64_t need = amr_lod_workspace_bytes(cam->W, cam->H);
  if (need > kNoAllocScratchBytes)
    return fail(AMR_ECAPACITY, "image needs " + std::to_string(need) + " bytes of LOD workspace; the fixed " +
                                   "device scratch of amr_render_lod_noalloc holds " +
                                   std::to_string(kNoAllocScratchBytes));
  void* ws = nullptr;
  cs = scratch_for_current_device(&ws);
  if (cs) return cs;
  return render_lod_on(t, cam, op, m, opts, out, aux, tile_levels, forced_levels, ws, stats, s);
}

}  // extern "C"
