// traverse.h -- per-ray octree traversal core (host + device).
//
// One ray per pixel (Sec. 2.2).  The ray is located in the tree truncated at
// the maximum level (Sec. 2), each cell it meets is visited in order, and a
// visitor accumulates value x chord (sum), the maximum value (maximum
// intensity projection, Sec. 2.1) or a weighted mean.
//
// Geometry is exact.  Positions are integers in units of 2^-28 of the box,
// the ray is r(t) = o + t d with integer o and d (the quantised camera).
// Axes with d_k < 0 are mirrored (x -> 2^28 - x) so every direction
// component is >= 0; the unmirrored cell index along a mirrored axis is the
// bitwise complement of the mirrored one within 28 bits.  Every decision --
// which cell contains the ray just after its entry point, which face it
// leaves through, whether it leaves the box -- is a comparison of two
// parameters (X_a - o_a) / d_a and (X_b - o_b) / d_b made by exact 64-bit
// cross multiplication (|X - o| < 2^31, 0 <= d < 2^30).  Hence the sequence
// of cells along every ray is fully determined, identical on every kernel
// variant and equal to the exact definition.
//
// Stackless restart descent: after leaving a cell at level l through face b,
// the ray's entry point lies in the neighbouring slab, whose prefix at level
// l is known (cell + 1 on every axis tied at the exit time, unchanged on the
// others).  The next cell is found by descending again from the deepest
// complete level (indexed arithmetically by Morton code, no memory read)
// through the first-child array.  Bits finer than level l, needed only when
// the next cell is deeper, are decided one level at a time by comparing the
// entry parameter with the crossing parameter of the midplane.
//
// Chord lengths are computed from the exact integer numerator of the
// parameter difference, scaled by |d| 2^-28 / (d_a d_b): a few fp32 roundings
// per chord at any depth.  Cells at level >= kDeepLevel form this product in
// fp64.
#pragma once
#include <stdint.h>
#include <type_traits>

// Bounds assertions on every cell index, for CPU builds of this core only.
#if defined(AMR_BOUNDS_CHECK)
#include <stdio.h>
#include <stdlib.h>
#define AMR_CHECK_CELL(T, c)                                                  \
  do {                                                                       \
    if ((c) < 0 || (int64_t)(c) >= (T).ncells) {                             \
      fprintf(stderr, "cell index %lld out of range\n", (long long)(c));     \
      abort();                                                               \
    }                                                                        \
  } while (0)
#else
#define AMR_CHECK_CELL(T, c) \
  do {                      \
  } while (0)
#endif

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define AMR_HD __host__ __device__ __forceinline__
#else
#include <math.h>
#define AMR_HD inline
#endif

namespace amr {

constexpr int kFix = 28;
constexpr int32_t kOne = int32_t(1) << kFix;
constexpr int kMaxLevel = 24;
constexpr int kDeepLevel = 18;
constexpr int kMaxArithBase = 10;  // Morton code of the base level fits 30 bits

// Device code sees the tree arrays as global memory, so gathers through
// pointers read from memory (batch image tables) compile to global rather
// than flat loads.  Host code sees plain pointers; the layout is the same.
#if defined(__HIP_DEVICE_COMPILE__)
#define AMR_GLOBAL __attribute__((address_space(1)))
#else
#define AMR_GLOBAL
#endif

struct TreeView {
  const int32_t AMR_GLOBAL* child;  // first-child index per cell, -1 for leaves
  const float AMR_GLOBAL* val;      // [nfields][ncells]
  const uint8_t AMR_GLOBAL* maxdepth;
  int64_t ncells;
  int32_t nfields;
  int32_t base;  // levels 0..base are complete; base <= kMaxArithBase
  int32_t lmax;
  int32_t pad_;
  int32_t off[kMaxLevel + 2];  // first cell index of each level
  // Fields 0..3 interleaved per cell (density and velocity of the usual
  // layout), or null when the tree has fewer than 4 fields: the
  // line-of-sight weighted mean gathers one 16-byte record per cell.
  const struct Cell4 AMR_GLOBAL* packed;
  // First-child index and field 0 of each cell side by side: the fast walk
  // reads one 8-byte record per cell for both the leaf test and the value.
  const struct ChildVal AMR_GLOBAL* cv;
};

struct alignas(16) Cell4 {
  float f0, f1, f2, f3;
};

struct alignas(8) ChildVal {
  int32_t child;
  float v0;
};

struct CameraView {
  int32_t kind, W, H, max_level;
  int64_t O[3], F[3], U[3], V[3];
};

AMR_HD uint32_t spread3(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

AMR_HD uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

AMR_HD int64_t mul64(int32_t a, int32_t b) { return (int64_t)a * (int64_t)b; }

// floor(num / d) for 0 <= num < 2^28 d and 0 < d < 2^31 (quotient below
// 2^28), exactly: the fp64 quotient of the converted operands is within
// 2^-24 of the true one (num's conversion and the division each add a
// relative error of at most 2^-53 to a value below 2^28), so its truncation
// is the quotient or one off, and one integer remainder test corrects it.
// A few dozen instructions instead of a generic 64-bit division.
AMR_HD int32_t div_q28(int64_t num, int32_t d) {
  int32_t q = (int32_t)((double)num / (double)d);
  const int64_t rem = num - mul64(q, d);
  q += rem < 0 ? -1 : (rem >= d ? 1 : 0);
  return q;
}
#if !defined(__HIPCC__)
inline int min(int a, int b) { return a < b ? a : b; }
#endif

AMR_HD void kahan_add(float& s, float& c, float x) {
  float y = x - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

#if defined(__HIPCC__)
#define AMR_UNROLL _Pragma("unroll")
#else
#define AMR_UNROLL
#endif

// Optimisation barrier: the compiler must assume x changes here, so work that
// depends on it is not moved out of the enclosing branch.  Emits nothing.
#if defined(__HIP_DEVICE_COMPILE__)
#define AMR_KEEP_HERE(x) asm volatile("" : "+v"(x))
#else
#define AMR_KEEP_HERE(x) \
  do {                   \
  } while (0)
#endif

// A value the compiler may not rewrite in terms of what it was computed from
// (a pure, instruction-free barrier: unlike AMR_KEEP_HERE it may be moved).
#if defined(__HIP_DEVICE_COMPILE__)
#define AMR_OPAQUE(x) asm("" : "+v"(x))
#else
#define AMR_OPAQUE(x) \
  do {                \
  } while (0)
#endif

// A per-lane condition evaluated here, as a lane mask in scalar registers.
// Without it the compiler re-evaluates a comparison at each later use and
// keeps its (wide) operands live until then.  Emits no instruction.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ inline bool amr_mask_here(bool c) {
  unsigned long long m = __builtin_amdgcn_ballot_w64(c);
  asm("" : "+s"(m));
  return __builtin_amdgcn_inverse_ballot_w64(m);
}
#else
inline bool amr_mask_here(bool c) { return c; }
#endif

// Gathers of one cell record by cell index through a buffer descriptor whose
// stride is the record size: the load unit scales the index and checks it
// against the record count (an index past the end reads zeros), so the walk
// spends no vector instructions on addresses.  The descriptor's last word is
// the hardware's buffer format for gfx9-family chips (32-bit data format).
#if defined(__HIP_DEVICE_COMPILE__)
typedef int32_t amr_i32x2 __attribute__((ext_vector_type(2)));
typedef float amr_f32x4 __attribute__((ext_vector_type(4)));
__device__ amr_i32x2 amr_buf_load_i32x2(__amdgpu_buffer_rsrc_t rsrc, int32_t index, int32_t voffset, int32_t soffset,
                                        int32_t aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v2i32");
__device__ amr_f32x4 amr_buf_load_f32x4(__amdgpu_buffer_rsrc_t rsrc, int32_t index, int32_t voffset, int32_t soffset,
                                        int32_t aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v4f32");
constexpr int32_t kBufFormatWord = 0x00020000;
template <class T>
__device__ inline __amdgpu_buffer_rsrc_t amr_records(const T AMR_GLOBAL* p, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)sizeof(T), (int)(n < 0x7fffffff ? n : 0x7fffffff),
                                           kBufFormatWord);
}
#endif

// Per-ray constants in mirrored coordinates.
struct Ray {
  int32_t o[3];    // mirrored origin
  int32_t d[3];    // |direction|, >= 0
  int32_t flip[3]; // 2^28 - 1 on mirrored axes, else 0
  int64_t d64[3];  // unmirrored direction
  float ulen;      // |d| 2^-28 (fp32)
  float inv_d[3];  // 1 / d_k
  double ulen64;   // |d| 2^-28
  int32_t stop[3]; // the fast walk ends on leaving through plane x_k = stop[k]
};

// Entry point of the current cell: parameter t = (Xa - oa) / da, the
// crossing of plane Xa on axis a; a < 0 when the ray starts inside the box
// (then Xa = oa = 0, da = 1, so t = 0).  p[] holds the integer part of the
// entry point (mirrored), exact on the axes flagged in `exact` and known
// down to level `lam` on the others.
struct Entry {
  int32_t p[3];
  int a;
  // the current cell's entry point has ray parameter en / da (in units of the
  // ray's own parameter scale), entered through a face normal to axis a
  int32_t en, da;
  float inv_da;
  int exact, lam;
};

// Builds the integer ray of pixel (i, j) and clips it to the box.  Returns
// false if the ray spends no positive length inside the box.
AMR_HD bool setup_ray(const CameraView& C, int i, int j, Ray& R, Entry& E) {
  const int64_t ca = 2 * (int64_t)i + 1 - C.W, cb = 2 * (int64_t)j + 1 - C.H;
  int64_t o64[3];
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    if (C.kind == 0) {
      o64[k] = C.O[k];
      R.d64[k] = C.F[k] + ca * C.U[k] + cb * C.V[k];
    } else {
      o64[k] = C.O[k] + ca * C.U[k] + cb * C.V[k];
      R.d64[k] = C.F[k];
    }
  }
  bool miss = false;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    if (R.d64[k] < 0) {
      R.d[k] = (int32_t)(-R.d64[k]);
      R.o[k] = (int32_t)((int64_t)kOne - o64[k]);
      R.flip[k] = kOne - 1;
    } else {
      R.d[k] = (int32_t)R.d64[k];
      R.o[k] = (int32_t)o64[k];
      R.flip[k] = 0;
    }
    if (R.d[k] == 0 && (R.o[k] < 0 || R.o[k] >= kOne)) miss = true;
  }
  // a zero direction spends no positive length anywhere
  if (miss || (R.d[0] | R.d[1] | R.d[2]) == 0) return false;
  // entry parameter: max(0, max over axes of -o_k / d_k), kept as en / ed
  int a = -1;
  int32_t en = 0, ed = 1, oa = 0;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    if (R.d[k] > 0 && R.o[k] < 0) {
      if (a < 0 || mul64(-R.o[k], ed) > mul64(en, R.d[k])) {
        a = k;
        en = -R.o[k];
        ed = R.d[k];
        oa = R.o[k];
      }
    }
  }
  // non-empty iff entry < exit of every slab: en / ed < (2^28 - o_k) / d_k
  AMR_UNROLL
  for (int k = 0; k < 3; ++k)
    if (R.d[k] > 0 && !(mul64(en, R.d[k]) < mul64(kOne - R.o[k], ed))) miss = true;
  if (miss) return false;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    if (a < 0 || R.d[k] == 0) {
      E.p[k] = R.o[k];
    } else if (k == a) {
      E.p[k] = 0;
    } else {
      // floor(x_k) at the entry: (o_k d_a - o_a d_k) / d_a, numerator in [0, 2^28 d_a)
      const int64_t num = mul64(R.o[k], ed) - mul64(oa, R.d[k]);
      E.p[k] = div_q28(num, ed);
    }
  }
  E.a = a;
  E.en = -oa;  // 0 when a < 0
  E.da = ed;   // 1 when a < 0
  E.exact = 7;
  E.lam = kFix;
  // chord scale factors
  const int64_t dd0 = R.d64[0] * R.d64[0] + R.d64[1] * R.d64[1] + R.d64[2] * R.d64[2];
  const float ulen = sqrtf((float)dd0) * 0x1.0p-28f;
  R.ulen = ulen;
  R.ulen64 = sqrt((double)dd0) * 0x1.0p-28;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    R.inv_d[k] = R.d[k] > 0 ? 1.0f / (float)R.d[k] : 0.0f;
  }
  E.inv_da = a < 0 ? 1.0f : 1.0f / (float)ed;
  R.stop[0] = R.stop[1] = R.stop[2] = kOne;
  return true;
}

// int64 -> fp32 as hi * 2^32 + lo in one fused step (identical on host and
// device; at most ~1.5 ulp from the correctly rounded conversion).
AMR_HD float i64_to_f32(int64_t v) {
  const int32_t hi = (int32_t)(v >> 32);
  const uint32_t lo = (uint32_t)(v & 0xffffffffu);
  return fmaf((float)hi, 4294967296.0f, (float)lo);
}

// Chord length of a cell from the exact numerator N of its parameter span:
// N |d| 2^-28 / (d_b d_a), as fp32 products in this fixed order (every walk
// uses this one expression, so that they agree bit for bit).
AMR_HD float chord_f32(int64_t N, float ulen, float inv_db, float inv_da) {
  return i64_to_f32(N) * ulen * inv_db * inv_da;
}

// Ancestor stack for the restart-from-common-ancestor descent: slot l holds
// the first-child index of the current path's cell at level l.
struct NoStack {
  AMR_HD int32_t get(int) const { return 0; }
  AMR_HD void set(int, int32_t) {}
};
struct LocalStack {  // host builds
  int32_t w[kMaxLevel + 1];
  AMR_HD int32_t get(int l) const { return w[l]; }
  AMR_HD void set(int l, int32_t v) { w[l] = v; }
};

// Walks the cells of one ray.  For every cell met, the visitor's
//   fetch(node)        is called as soon as the cell is located, and
//   seg(node, level, len, cm0, cm1, cm2)  once its chord is known
// (cm = mirrored cell coordinates).  Returns the number of cells.
// LCA = false restarts every descent at the complete base level; LCA = true
// restarts at the deepest ancestor shared with the previous cell, whose
// first-child index is kept in the stack S.  Both meet exactly the same cells
// and compute exactly the same chords.
template <bool LCA, class Vis, class Stack>
AMR_HD int32_t walk(const TreeView& T, const Ray& R, Entry& E, int max_level, Vis& vis, Stack& S) {
  const int b0 = T.base < max_level ? T.base : max_level;
  // virtual direction for axes that do not move: their exit never wins
  const int32_t dv0 = R.d[0] > 0 ? R.d[0] : 1, dv1 = R.d[1] > 0 ? R.d[1] : 1, dv2 = R.d[2] > 0 ? R.d[2] : 1;
  const float ulen = R.ulen;
  const float iv0 = R.inv_d[0], iv1 = R.inv_d[1], iv2 = R.inv_d[2];
  int32_t nseg = 0;
  int jr = -1;  // restart level (LCA only): the stack holds levels b0..jr of the entry point's path
  for (;;) {
    // ---- locate the cell containing r(t_entry + 0)
    int lvl;
    int32_t node;
    if (!LCA || jr < b0) {
      lvl = b0;
      const int sb = kFix - b0;
      node = T.off[b0] + (int32_t)morton3((uint32_t)((E.p[0] ^ R.flip[0]) >> sb),
                                          (uint32_t)((E.p[1] ^ R.flip[1]) >> sb),
                                          (uint32_t)((E.p[2] ^ R.flip[2]) >> sb));
    } else {
      lvl = jr + 1;  // bits down to lvl are known: jr < level of the previous cell
      const int s = kFix - lvl;
      const int oct = (((E.p[0] ^ R.flip[0]) >> s) & 1) | ((((E.p[1] ^ R.flip[1]) >> s) & 1) << 1) |
                      ((((E.p[2] ^ R.flip[2]) >> s) & 1) << 2);
      node = S.get(jr) + oct;
    }
    AMR_CHECK_CELL(T, node);
    while (lvl < max_level) {
      const int32_t w = T.child[(uint32_t)node];
      if (w < 0) break;
      if (LCA) S.set(lvl, w);
      ++lvl;
      const int s = kFix - lvl;
      if (lvl > E.lam) {
        // decide bit s of the entry point on the axes not known exactly:
        // x_k(t_e) >= M  <=>  (Xa - o_a) d_k >= (M - o_k) d_a
        AMR_UNROLL
        for (int k = 0; k < 3; ++k) {
          if (E.exact & (1 << k)) continue;
          const int32_t M = E.p[k] + (int32_t(1) << s);
          if (mul64(E.en, R.d[k]) >= mul64(M - R.o[k], E.da)) E.p[k] = M;
        }
        E.lam = lvl;
      }
      const int oct = (((E.p[0] ^ R.flip[0]) >> s) & 1) | ((((E.p[1] ^ R.flip[1]) >> s) & 1) << 1) |
                      ((((E.p[2] ^ R.flip[2]) >> s) & 1) << 2);
      node = w + oct;
      AMR_CHECK_CELL(T, node);
    }
    vis.fetch(node);
    // ---- exit face: smallest (X_k - o_k) / d_k, ties kept (branch-free;
    // plain scalars, so no select is folded into an indexed load)
    const int s = kFix - lvl;
    const int32_t X0 = ((E.p[0] >> s) + 1) << s;
    const int32_t X1 = ((E.p[1] >> s) + 1) << s;
    const int32_t X2 = ((E.p[2] >> s) + 1) << s;
    const int32_t n0 = R.d[0] > 0 ? X0 - R.o[0] : 0x7fffffff;
    const int32_t n1 = R.d[1] > 0 ? X1 - R.o[1] : 0x7fffffff;
    const int32_t n2 = R.d[2] > 0 ? X2 - R.o[2] : 0x7fffffff;
    const int64_t c01 = mul64(n0, dv1) - mul64(n1, dv0);  // sign of t0 - t1
    const bool p1 = c01 > 0;
    const int32_t nA = p1 ? n1 : n0, dA = p1 ? dv1 : dv0;
    const int tieA = c01 == 0 ? 3 : (p1 ? 2 : 1);
    const int64_t c2 = mul64(nA, dv2) - mul64(n2, dA);  // sign of tA - t2
    const bool p2 = c2 > 0;
    const int best = p2 ? 2 : (p1 ? 1 : 0);
    const int tie = p2 ? 4 : (c2 == 0 ? (tieA | 4) : tieA);
    const int32_t nb = p2 ? n2 : nA;
    const int32_t db = p2 ? dv2 : dA;
    const float invb = p2 ? iv2 : (p1 ? iv1 : iv0);
    // ---- chord from the exact numerator of (t_exit - t_entry) d_a d_b
    const int64_t N = mul64(nb, E.da) - mul64(E.en, db);
    float len;
    if (lvl < kDeepLevel)
      len = chord_f32(N, ulen, invb, E.inv_da);
    else
      len = (float)((double)N * R.ulen64 / ((double)E.da * (double)db));
    vis.seg(node, lvl, len, E.p[0] >> s, E.p[1] >> s, E.p[2] >> s);
    ++nseg;
    // ---- leave the box, or enter the neighbour
    const bool out = ((tie & 1) && X0 == kOne) || ((tie & 2) && X1 == kOne) || ((tie & 4) && X2 == kOne);
    if (out) break;
    if (LCA) {
      // deepest level whose cell still contains the new entry point: a tied
      // axis whose level-lvl coordinate ends in t one-bits carries t+1 levels up
      jr = lvl - 1;
      AMR_UNROLL
      for (int k = 0; k < 3; ++k) {
        if (tie & (1 << k)) {
          const uint32_t c = (uint32_t)(E.p[k] >> s);
          const int t1 = __builtin_ctz(~c);
          const int j = lvl - t1 - 1;
          jr = j < jr ? j : jr;
        }
      }
    }
    const int32_t keep = ~((int32_t(1) << s) - 1);
    const int32_t Xs[3] = {X0, X1, X2};
    AMR_UNROLL
    for (int k = 0; k < 3; ++k) {
      if (tie & (1 << k)) {
        E.p[k] = Xs[k];
        E.exact |= 1 << k;
      } else if (R.d[k] > 0) {
        E.p[k] &= keep;
        E.exact &= ~(1 << k);
      }
    }
    E.lam = lvl;
    E.a = best;
    E.en = nb;
    E.da = db;
    E.inv_da = invb;
  }
  return nseg;
}

// Three-input bitwise operations.  On gfx950 the three-input logic
// instruction issues at about 0.6 of the rate of a two-input one, where the
// compiler's own choices (or3, bfi) issue at half rate (as do two two-input
// operations in a row).
#if defined(__HIP_DEVICE_COMPILE__)
__device__ inline uint32_t or3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0xFE); }
// bits of a where m is set, of b elsewhere
__device__ inline uint32_t bitsel(uint32_t m, uint32_t a, uint32_t b) { return __builtin_amdgcn_bitop3_b32(m, a, b, 0xCA); }
#else
inline uint32_t or3(uint32_t a, uint32_t b, uint32_t c) { return a | b | c; }
inline uint32_t bitsel(uint32_t m, uint32_t a, uint32_t b) { return (m & a) | (~m & b); }
#endif

// Octant (bit 0 = x, bit 1 = y, bit 2 = z) of the coordinates' bits at
// position s, s >= 2: each coordinate shifted so that its bit lands in its
// octant position, then bit 0 taken from x, bit 1 from y, bit 2 from z.
AMR_HD uint32_t octant_bits(int32_t x, int32_t y, int32_t z, int s) {
  return bitsel(1u, (uint32_t)x >> s, bitsel(2u, (uint32_t)y >> (s - 1), (uint32_t)z >> (s - 2))) & 7u;
}

// Morton-code step of one complete-level cell along axis k (0, 1, 2) by +1
// when c is set, on a 30-bit code: with the other axes' bits set to one, an
// increment of the whole word carries through them (the bits below k
// included) into the axis' own bits.
AMR_HD uint32_t morton_inc(uint32_t m, int k, bool c) {
  const uint32_t mk = 0x09249249u << k;
  return bitsel(mk, (m | ~mk) + (c ? 1u : 0u), m);
}

// The same walk as walk<false> (identical cells, chords and order), with
// less work per cell:
//  - the Morton index of the complete-level cell is stepped along the axes
//    whose base-level coordinate changes instead of being recomputed;
//  - the first-child index of the current cell's parent stays in a
//    register, so moving to a sibling (about half of all moves) skips the
//    descent from the base level;
//  - child octants are taken from the mirrored coordinates and corrected by
//    one xor with the flipped axes, with no unmirrored copy;
//  - the exit face is decided on lane masks and cross-products compared
//    directly, and the state update needs no selects (bits below the
//    current level are left stale and refined when a deeper cell needs
//    them);
//  - visitors that do not use chord lengths skip their arithmetic.
// kWholeBox: the ray's stop planes are the box faces (R.stop = 2^28 on every
// axis, as setup_ray leaves them), which makes the end test one comparison.
// On return E is no longer the entry state of any cell (and its fields a
// and exact are not kept up to date).
// Visitors that declare kTrackCut = true also learn whether the walk
// stopped its descent at a cell that has children (a cell cut by the level
// limit).  A walk that cut no cell visited exactly the cells, in the same
// order and with the same chords, as a walk of the untruncated tree.
template <class V, class = void>
struct TracksCut {
  static constexpr bool value = false;
};
template <class V>
struct TracksCut<V, decltype((void)V::kTrackCut)> {
  static constexpr bool value = V::kTrackCut;
};
// Visitors that declare kNeedsParams = true also receive, before seg(), the
// ray parameters of the cell's entry and exit as exact numerators with the
// fp32 reciprocals of their denominators (en, 1 / da, nb, 1 / db).
template <class V, class = void>
struct NeedsParams {
  static constexpr bool value = false;
};
template <class V>
struct NeedsParams<V, decltype((void)V::kNeedsParams)> {
  static constexpr bool value = V::kNeedsParams;
};

// kShallow: the caller guarantees max_level < kDeepLevel (no fp64 chords).
// Stk: with a stack other than NoStack (get / set of one int32 per level,
// levels above min(base, max_level)), every descent step records the
// first-child index of the cell it leaves, and a move whose deepest common
// ancestor lies below the base level restarts at that ancestor's child
// instead of at the base level (fewer dependent loads on deep trees; the
// same cells, in the same order, with the same chords).
template <class Vis, bool kWholeBox = false, bool kShallow = false, class Stk = NoStack>
AMR_HD int32_t walk_fast(const TreeView& T, const Ray& R, Entry& E, int max_level, Vis& vis, Stk& stk) {
  constexpr bool kStk = !std::is_same<Stk, NoStack>::value;
  const int b0 = T.base < max_level ? T.base : max_level;
  const int sb = kFix - b0;
  // Direction components, 0 on an axis the ray does not move along: in the
  // cross-multiplied comparisons below such an axis then never exits first
  // (n_j * 0 < n_k * d_j for every moving axis j, as every n > 0), and the
  // refinement of its coordinate bits sees d = 0 as it should.
  const int32_t dv0 = R.d[0], dv1 = R.d[1], dv2 = R.d[2];
  // 1 - o: the exit numerator X - o of a cell is (p | low) + co, one add
  int32_t co0 = 1 - R.o[0], co1 = 1 - R.o[1], co2 = 1 - R.o[2];
  AMR_OPAQUE(co0);
  AMR_OPAQUE(co1);
  AMR_OPAQUE(co2);
  const float ulen = R.ulen;
  const float iv0 = R.inv_d[0], iv1 = R.inv_d[1], iv2 = R.inv_d[2];
  const int32_t f0 = R.flip[0], f1 = R.flip[1], f2 = R.flip[2];
  // The base cell is tracked by the Morton index of its mirrored coordinates,
  // so a step along any axis is an increment; xor with fm (the flipped axes'
  // bits) gives the index of the stored cell.
  // Its low three bits are the flipped axes as an octant mask: the child of a
  // stored cell holding mirrored octant o is child o ^ (fm & 7).
  const uint32_t mask3 = (uint32_t)((uint64_t(1) << (3 * b0)) - 1);
  const uint32_t fm = (f0 ? 0x09249249u : 0u) | (f1 ? 0x12492492u : 0u) | (f2 ? 0x24924924u : 0u);
  uint32_t mb = morton3((uint32_t)(E.p[0] >> sb), (uint32_t)(E.p[1] >> sb), (uint32_t)(E.p[2] >> sb));
  const int32_t offb = T.off[b0];  // first cell of the complete base level
  // first-child index of the current cell's parent: set by every descent
  // step and kept by a sibling step, so it is that of the level lvl - 1 for
  // every cell below the base level
  int32_t pfc = -1;
  int32_t nseg = 0;
  // where the next cell's descent starts: its level and cell (set at the end
  // of each step: the base-level cell, or the previous cell's sibling)
  int lvl = b0;
  int32_t node = offb + (int32_t)((mb ^ fm) & mask3);
#if defined(__HIP_DEVICE_COMPILE__)
  const __amdgpu_buffer_rsrc_t cvr = amr_records(T.cv, T.ncells);
#endif
  for (;;) {
    AMR_CHECK_CELL(T, node);
    float v0;
    for (;;) {
#if defined(__HIP_DEVICE_COMPILE__)
      const amr_i32x2 rec = amr_buf_load_i32x2(cvr, node, 0, 0, 0);
      const int32_t w = rec[0];
      const int32_t vbits = rec[1];
      v0 = __int_as_float(vbits);
#else
      const ChildVal rec = T.cv[(uint32_t)node];
      v0 = rec.v0;
      const int32_t w = rec.child;
#endif
      if (lvl >= max_level || w < 0) {
        if constexpr (TracksCut<Vis>::value) vis.cut_and &= w;  // sign bit clears at a cut
        break;
      }
      pfc = w;
      ++lvl;
      if constexpr (kStk) stk.set(lvl, w);
      const int s = kFix - lvl;
      if (lvl > E.lam) {
        // entry numerator, kept inside this rarely taken branch (hoisted, its
        // three products would run on every cell)
        int32_t en = E.en;
        AMR_KEEP_HERE(en);
        // the coordinates are known down to level lam (their lower bits are
        // left over from earlier cells and cleared here); the bit of each
        // axis at this level is decided exactly from the entry parameter,
        // which for an axis whose stored coordinate is exact (an axis just
        // crossed) gives that coordinate's own bit
        const int32_t known = ~((int32_t(1) << (kFix - E.lam)) - 1);
        const int32_t dvk[3] = {dv0, dv1, dv2};
        const int32_t cok[3] = {co0, co1, co2};
        AMR_UNROLL
        for (int k = 0; k < 3; ++k) {
          const int32_t M = (E.p[k] & known) + (int32_t(1) << s);
          E.p[k] = mul64(en, dvk[k]) >= mul64(M + cok[k] - 1, E.da) ? M : (E.p[k] & known);
        }
        E.lam = lvl;
      }
      node = w + (int32_t)(octant_bits(E.p[0], E.p[1], E.p[2], s) ^ (fm & 7u));
      AMR_CHECK_CELL(T, node);
    }
    vis.fetch0(node, v0);
    const int s = kFix - lvl;
    const int32_t low = (int32_t)((uint32_t)(kOne - 1) >> lvl);  // (1 << s) - 1 by a (full-rate) right shift
    // last coordinate inside the cell (the exit plane is h + 1) and exit numerators
    const int32_t h0 = E.p[0] | low, h1 = E.p[1] | low, h2 = E.p[2] | low;
    const int32_t n0 = h0 + co0, n1 = h1 + co1, n2 = h2 + co2;
    // exit parameters n_k / dv_k compared by cross-multiplication (the
    // products of 31-bit factors compare directly, no difference needed)
    const int64_t P0 = mul64(n0, dv1), P1 = mul64(n1, dv0);
    const bool p1 = P0 > P1, g1 = amr_mask_here(P0 >= P1);
    const int32_t nA = p1 ? n1 : n0, dA = p1 ? dv1 : dv0;
    const int64_t PA = mul64(nA, dv2), P2 = mul64(n2, dA);
    const bool p2 = PA > P2;
    // axes whose exit plane is reached first (several on a tie)
    const bool t2 = PA >= P2;
    const bool t1 = !p2 && g1;
    const bool t0 = !p2 && !p1;
    const int32_t nb = p2 ? n2 : nA;
    const int32_t db = p2 ? dv2 : dA;
    const float invb = p2 ? iv2 : (p1 ? iv1 : iv0);
    float len = 0.0f;
    if (Vis::kNeedsLength) {
      // (the product of the negated entry numerator is the second one's addend)
      const int64_t N = mul64(nb, E.da) + mul64(-E.en, db);
      if (kShallow || max_level < kDeepLevel || lvl < kDeepLevel)
        len = chord_f32(N, ulen, invb, E.inv_da);
      else
        len = (float)((double)N * R.ulen64 / ((double)E.da * (double)db));
    }
    if constexpr (NeedsParams<Vis>::value) vis.params(E.en, E.inv_da, nb, invb);
    vis.seg(node, lvl, len, E.p[0] >> s, E.p[1] >> s, E.p[2] >> s);
    ++nseg;
    // Next cell's coordinates: tied axes enter at their face exactly
    // (X = (p | low) + 1); the others keep the current cell's prefix, their
    // bits below this level left at one (stale from here: refinement
    // recomputes them, for a fixed axis too, so only crossed axes are exact).
    // An axis not crossed stays below its stop plane (no cell straddles one),
    // so the ray ends when a coordinate reaches its stop plane.
    E.p[0] = h0 + (t0 ? 1 : 0);
    E.p[1] = h1 + (t1 ? 1 : 0);
    E.p[2] = h2 + (t2 ? 1 : 0);
    // the rest of the next cell's entry state, set before the end test so
    // that both ways out of this iteration carry the same values (a ray that
    // ends discards them; on return E is not meaningful)
    E.lam = lvl;
    E.en = nb;
    E.da = db;
    E.inv_da = invb;
    if (kWholeBox) {
      if ((uint32_t)(E.p[0] | E.p[1] | E.p[2]) >= (uint32_t)kOne) break;
    } else {
      if (E.p[0] >= R.stop[0] || E.p[1] >= R.stop[1] || E.p[2] >= R.stop[2]) break;
    }
    // restart level, base-cell steps and where the next descent starts
    if (lvl == b0) {
      // a base-level cell (most cells of a typical tree): every tied axis
      // moves the base cell, and the next cell is found from the base level
      // one increment along the exit axis; an edge or corner (several tied
      // axes, rare) moves along every tied axis
      const uint32_t mk = p2 ? 0x24924924u : (p1 ? 0x12492492u : 0x09249249u);
      const uint32_t mb0 = mb;
      mb = bitsel(mk, (mb | ~mk) + 1u, mb);
      if ((t2 && !p2) || (t1 && !p1 && !p2)) {
        mb = morton_inc(mb0, 0, t0);
        mb = morton_inc(mb, 1, t1);
        mb = morton_inc(mb, 2, t2);
      }
      node = offb + (int32_t)((mb ^ fm) & mask3);
    } else {
      // a tied axis whose new coordinate at this level, c + 1, ends in r
      // zero bits (the old c in r one-bits) carries r levels up
      const int span = lvl - b0;
      const int32_t bmask = (int32_t(1) << span) - 1;
      int jr = lvl - 1;
      if (t0) {
        const int32_t c1 = E.p[0] >> s;
        jr = min(jr, lvl - 1 - (int)__builtin_ctz((uint32_t)c1));
        mb = morton_inc(mb, 0, (c1 & bmask) == 0);
      }
      if (t1) {
        const int32_t c1 = E.p[1] >> s;
        jr = min(jr, lvl - 1 - (int)__builtin_ctz((uint32_t)c1));
        mb = morton_inc(mb, 1, (c1 & bmask) == 0);
      }
      if (t2) {
        const int32_t c1 = E.p[2] >> s;
        jr = min(jr, lvl - 1 - (int)__builtin_ctz((uint32_t)c1));
        mb = morton_inc(mb, 2, (c1 & bmask) == 0);
      }
      // the next cell is the sibling of this one when the restart level is
      // that of the cached parent, lvl - 1; else it is found from the base
      // level
      if (jr == lvl - 1) {
        node = pfc + (int32_t)(octant_bits(E.p[0], E.p[1], E.p[2], kFix - 1 - jr) ^ (fm & 7u));
        lvl = jr + 1;
        continue;
      }
      if constexpr (kStk) {
        // the ancestor at level jr is shared (no carry reached the base
        // level, so the base cell is unchanged): restart at its child
        if (jr >= b0) {
          pfc = stk.get(jr + 1);
          node = pfc + (int32_t)(octant_bits(E.p[0], E.p[1], E.p[2], kFix - 1 - jr) ^ (fm & 7u));
          lvl = jr + 1;
          continue;
        }
      }
      node = offb + (int32_t)((mb ^ fm) & mask3);
    }
    lvl = b0;
  }
  return nseg;
}

template <class Vis, bool kWholeBox = false, bool kShallow = false>
AMR_HD int32_t walk_fast(const TreeView& T, const Ray& R, Entry& E, int max_level, Vis& vis) {
  NoStack none;
  return walk_fast<Vis, kWholeBox, kShallow, NoStack>(T, R, E, max_level, vis, none);
}

template <class Vis>
AMR_HD int32_t walk_ray(const TreeView& T, const Ray& R, Entry& E, int max_level, Vis& vis) {
  NoStack S;
  return walk<false>(T, R, E, max_level, vis, S);
}

// ----------------------------------------------------------------- visitors

// kField0: the caller guarantees field0 (no per-cell test).
template <bool kField0 = false>
struct SumVisT {
  static constexpr bool kNeedsLength = true;
  const float AMR_GLOBAL* v;
  bool field0 = false;  // v is field 0: the fast walk hands over the value
  float s = 0.0f, c = 0.0f, x = 0.0f;
  AMR_HD void fetch(int32_t node) { x = v[(uint32_t)node]; }
  AMR_HD void fetch0(int32_t node, float v0) { x = (kField0 || field0) ? v0 : v[(uint32_t)node]; }
  AMR_HD void seg(int32_t, int, float len, int32_t, int32_t, int32_t) { kahan_add(s, c, x * len); }
};
using SumVis = SumVisT<false>;

template <bool kField0 = false>
struct MaxVisT {
  static constexpr bool kNeedsLength = false;
  const float AMR_GLOBAL* v;
  float m;
  bool field0 = false;
  float x = 0.0f;
  AMR_HD void fetch(int32_t node) { x = v[(uint32_t)node]; }
  AMR_HD void fetch0(int32_t node, float v0) { x = (kField0 || field0) ? v0 : v[(uint32_t)node]; }
  AMR_HD void seg(int32_t, int, float, int32_t, int32_t, int32_t) { m = fmaxf(m, x); }
};
using MaxVis = MaxVisT<false>;

// kPackedLos: the caller guarantees the interleaved records (pk) and the
// line-of-sight velocity (los), so neither is tested per cell.
template <bool kPackedLos = false>
struct WMeanVisT {
  static constexpr bool kNeedsLength = true;
  const float AMR_GLOBAL* w;
  const float AMR_GLOBAL* f0;
  const float AMR_GLOBAL* f1;
  const float AMR_GLOBAL* f2;
  const Cell4 AMR_GLOBAL* pk = nullptr;  // weight = field 0, velocity = fields 1..3, interleaved
  int64_t npk = 0;                       // records at pk
  AMR_HD void use_packed(const TreeView& T) {
    pk = T.packed;
    npk = T.ncells;
  }
  float dh[3];
  int los;
  float sw = 0.0f, cw = 0.0f, sf = 0.0f, cf = 0.0f;
  float xw = 0.0f, x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
  AMR_HD void fetch(int32_t node) {
    if (kPackedLos || pk) {
#if defined(__HIP_DEVICE_COMPILE__)
      const amr_f32x4 q = amr_buf_load_f32x4(amr_records(pk, npk), node, 0, 0, 0);
      xw = q[0];
      x0 = q[1];
      x1 = q[2];
      x2 = q[3];
#else
      const Cell4 q = pk[(uint32_t)node];
      xw = q.f0;
      x0 = q.f1;
      x1 = q.f2;
      x2 = q.f3;
#endif
      return;
    }
    xw = w[(uint32_t)node];
    x0 = f0[(uint32_t)node];
    if (los) {
      x1 = f1[(uint32_t)node];
      x2 = f2[(uint32_t)node];
    }
  }
  AMR_HD void fetch0(int32_t node, float) { fetch(node); }
  AMR_HD void seg(int32_t, int, float len, int32_t, int32_t, int32_t) {
    const float wl = xw * len;
    float f = x0;
    // line-of-sight velocity v . d^, as fused multiply-adds (correctly
    // rounded on host and device alike)
    if (kPackedLos || los) f = fmaf(x2, dh[2], fmaf(x1, dh[1], x0 * dh[0]));
    kahan_add(sw, cw, wl);
    kahan_add(sf, cf, wl * f);
  }
};
using WMeanVis = WMeanVisT<false>;

// Whether a wmean render takes the interleaved-record path: weight = field
// 0, line-of-sight velocity of fields 1..3, records built.
AMR_HD bool packed_los(const TreeView& T, int field, int wfield, int los) {
  return los && wfield == 0 && field == 1 && T.packed;
}


struct CountVis {
  static constexpr bool kNeedsLength = false;
  AMR_HD void fetch(int32_t) {}
  AMR_HD void fetch0(int32_t, float) {}
  AMR_HD void seg(int32_t, int, float, int32_t, int32_t, int32_t) {}
};

// Writes (level, ix, iy, iz) of every cell, unmirrored.
struct TraceVis {
  static constexpr bool kNeedsLength = false;
  int32_t* out;
  int32_t flip_bits[3];  // 1 on mirrored axes
  AMR_HD void fetch(int32_t) {}
  AMR_HD void fetch0(int32_t, float) {}
  AMR_HD void seg(int32_t, int lvl, float, int32_t c0, int32_t c1, int32_t c2) {
    const int32_t m = (int32_t(1) << lvl) - 1;
    out[0] = lvl;
    out[1] = flip_bits[0] ? (c0 ^ m) : c0;
    out[2] = flip_bits[1] ? (c1 ^ m) : c1;
    out[3] = flip_bits[2] ? (c2 ^ m) : c2;
    out += 4;
  }
};

// Local resolution of the image along a ray, for the adaptive blur: the
// chord-weighted mean of the cell side in units of the pixel spacing at the
// cell's depth.  A perspective pixel spacing grows with the ray parameter,
// so each cell's side is divided by the parameter at the middle of its
// chord, (en/da + nb/db) / 2; the caller divides the result by the spacing
// at unit parameter (orthographic: the constant spacing).
struct ResAcc {
  int persp = 1;
  float tm = 1.0f;
  float sn = 0.0f, cn = 0.0f, sl = 0.0f, cl = 0.0f;  // Kahan pairs: sum(len side / t), sum(len)
  AMR_HD void res_params(int32_t en, float inv_da, int32_t nb, float inv_db) {
    if (persp) tm = 0.5f * ((float)en * inv_da + (float)nb * inv_db);
  }
  AMR_HD void res_seg(int lvl, float len) {
    const float side = ldexpf(1.0f, -lvl);  // exact
    kahan_add(sn, cn, len * side * rcp(tm));
    kahan_add(sl, cl, len);
  }
  // resolution in units of the spacing at unit parameter; 0 without length
  AMR_HD float res_value(float inv_w0) const {
    const float L = sl - cl;
    return L > 0.0f ? (sn - cn) / L * inv_w0 : 0.0f;
  }
#if defined(__HIP_DEVICE_COMPILE__)
  __device__ static float rcp(float x) { return __builtin_amdgcn_rcpf(x); }  // 1 ulp
#else
  static float rcp(float x) { return 1.0f / x; }
#endif
};

struct ResVis : ResAcc {
  static constexpr bool kNeedsLength = true;
  static constexpr bool kNeedsParams = true;
  AMR_HD void fetch(int32_t) {}
  AMR_HD void fetch0(int32_t, float) {}
  AMR_HD void params(int32_t en, float inv_da, int32_t nb, float inv_db) { res_params(en, inv_da, nb, inv_db); }
  AMR_HD void seg(int32_t, int lvl, float len, int32_t, int32_t, int32_t) { res_seg(lvl, len); }
};

// A projection's visitor V that also accumulates the local resolution, so
// that one walk yields the image and its resolution plane: V sees exactly
// what it sees alone, and the resolution sums exactly what ResVis sums.
template <class V>
struct WithRes : V, ResAcc {
  static constexpr bool kNeedsLength = true;
  static constexpr bool kNeedsParams = true;
  AMR_HD void params(int32_t en, float inv_da, int32_t nb, float inv_db) { res_params(en, inv_da, nb, inv_db); }
  AMR_HD void seg(int32_t node, int lvl, float len, int32_t c0, int32_t c1, int32_t c2) {
    V::seg(node, lvl, len, c0, c1, c2);
    res_seg(lvl, len);
  }
};

// Sets bit `node` of a bitmap for every cell met and counts the bits it
// was first to set (distinct cells over all rays of a launch).
struct MarkVis {
  static constexpr bool kNeedsLength = false;
  uint32_t* bits;
  unsigned long long fresh = 0;
  AMR_HD void fetch(int32_t) {}
  AMR_HD void fetch0(int32_t, float) {}
  AMR_HD void seg(int32_t node, int, float, int32_t, int32_t, int32_t) {
    const uint32_t w = (uint32_t)node >> 5, b = 1u << ((uint32_t)node & 31u);
    if (bits[w] & b) return;  // already marked (plain read: most repeats end here)
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t old = atomicOr(bits + w, b);
#else
    const uint32_t old = bits[w];
    bits[w] = old | b;
#endif
    if (!(old & b)) ++fresh;
  }
};

// ------------------------------------------------------------ one pixel

enum { kOpSum = 0, kOpMax = 1, kOpWMean = 2 };

// The common field layout of an op: sum and max of field 0 (the value the
// fast walk already holds), wmean on the interleaved-record path.
AMR_HD bool std_fields(int op, const TreeView& T, int field, int wfield, int los) {
  return op == kOpWMean ? packed_los(T, field, wfield, los) : field == 0;
}

// Whether a render may use walk_span's kStd walk: the common field layout,
// and for sum and max a maximum level below kDeepLevel.
AMR_HD bool std_walk(int op, const TreeView& T, int field, int wfield, int los, int max_level) {
  return std_fields(op, T, field, wfield, los) && (op == kOpWMean || max_level < kDeepLevel);
}

// The whole per-pixel computation of one projection; out receives the
// pixel value, aux (WMEAN) the weight integral.
// Descent modes: restart at the complete base level (kWalkBase), at the
// common ancestor kept in a stack (kWalkStack), the register-cached form
// (kWalkFast), or that form with an ancestor stack (kWalkFastStack).  All
// meet the same cells with the same chords.
enum { kWalkBase = 0, kWalkStack = 1, kWalkFast = 2, kWalkFastStack = 3 };

template <int MODE, class Vis, class Stack>
AMR_HD int32_t walk_mode(const TreeView& T, const Ray& R, Entry& E, int max_level, Vis& v, Stack& S) {
  if constexpr (MODE == kWalkFast) return walk_fast<Vis, true>(T, R, E, max_level, v);
  if constexpr (MODE == kWalkFastStack) return walk_fast<Vis, true, false, Stack>(T, R, E, max_level, v, S);
  return walk<MODE == kWalkStack>(T, R, E, max_level, v, S);
}

template <int OP, int MODE, class Stack>
AMR_HD void render_pixel(const TreeView& T, const CameraView& C, int field, int wfield, int los, int max_level,
                         int i, int j, float& out, float& aux, Stack& S) {
  Ray R;
  Entry E;
  const bool hit = setup_ray(C, i, j, R, E);
  const int64_t nc = T.ncells;
  if (OP == kOpSum) {
    SumVis v{T.val + (int64_t)field * nc, field == 0};
    if (hit) walk_mode<MODE>(T, R, E, max_level, v, S);
    out = v.s - v.c;
  } else if (OP == kOpMax) {
    MaxVis v{T.val + (int64_t)field * nc, -INFINITY, field == 0};
    if (hit) walk_mode<MODE>(T, R, E, max_level, v, S);
    out = v.m;
  } else {
    WMeanVis v;
    v.w = T.val + (int64_t)wfield * nc;
    v.f0 = T.val + (int64_t)field * nc;
    v.f1 = los ? v.f0 + nc : v.f0;
    v.f2 = los ? v.f0 + 2 * nc : v.f0;
    v.los = los;
    if (packed_los(T, field, wfield, los)) v.use_packed(T);
    v.dh[0] = v.dh[1] = v.dh[2] = 0.0f;
    if (hit) {
      const float n = sqrtf((float)(R.d64[0] * R.d64[0] + R.d64[1] * R.d64[1] + R.d64[2] * R.d64[2]));
      AMR_UNROLL
      for (int k = 0; k < 3; ++k) v.dh[k] = (float)R.d64[k] / n;
      walk_mode<MODE>(T, R, E, max_level, v, S);
    }
    const float W = v.sw - v.cw, Sf = v.sf - v.cf;
    out = W > 0.0f ? Sf / W : 0.0f;
    aux = W;
  }
}

// Number of cells on the ray of pixel (i, j); with cells != NULL they are
// also written (4 int32 each), but only if exactly `cap` of them exist.
// Both passes take walk_fast over the whole ray, the walk the batched and
// single-image renders time, so the sequences and counts are that walk's.
AMR_HD int32_t trace_pixel(const TreeView& T, const CameraView& C, int max_level, int i, int j, int32_t* cells,
                           int64_t cap) {
  Ray R;
  Entry E;
  if (!setup_ray(C, i, j, R, E)) return 0;
  const Entry E0 = E;
  CountVis c;
  const int32_t m = walk_fast<CountVis, true>(T, R, E, max_level, c);
  if (!cells || m != cap) return m;
  TraceVis v;
  v.out = cells;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) v.flip_bits[k] = R.flip[k] ? 1 : 0;
  E = E0;
  walk_fast<TraceVis, true>(T, R, E, max_level, v);
  return m;
}


// ------------------------------------------------------------ split rays
// A long ray can be cut into spans at planes of the base level normal to
// its major axis.  Every cell on the path lies at the base level or deeper,
// so no cell straddles such a plane: the spans partition the ray's cell
// sequence.  A span starts at the exact crossing of its first plane and ends
// on leaving through its last one, so each cell is decided exactly as on the
// unsplit ray.  Spans are walked by different waves and their partial sums
// merged in span order; only the rounding of the sums differs from the
// unsplit walk (the maximum is identical).

// Axis with the largest |d| (lowest index on ties).
AMR_HD int major_axis(const Ray& R) {
  int a = R.d[1] > R.d[0] ? 1 : 0;
  return R.d[2] > (a ? R.d[1] : R.d[0]) ? 2 : a;
}

// Component a of a 3-vector held in registers (selects, not an indexed
// access, so the vector is never spilled to scratch memory).
template <class T>
AMR_HD T pick3(int a, const T (&v)[3]) {
  return a == 2 ? v[2] : (a == 1 ? v[1] : v[0]);
}

// Entry at the crossing of the plane x_a = P (mirrored).  False when the ray
// leaves the box before reaching it.  The caller guarantees that P lies
// beyond the ray's box entry point.
AMR_HD bool plane_entry(const Ray& R, int a, int32_t P, Entry& E) {
  const int32_t da32 = pick3(a, R.d), oa = pick3(a, R.o);
  if (da32 <= 0 || P >= kOne) return false;
  const int64_t da = da32;
  const int64_t dt = (int64_t)P - oa;
  int32_t p[3];
  bool inside = true;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    // x_k at the crossing = (o_k d_a + (P - o_a) d_k) / d_a, in [0, 2^28)
    const int64_t num = (int64_t)R.o[k] * da + dt * (int64_t)R.d[k];
    const bool beyond = num >= (int64_t)kOne * da;  // outside the box (then p is not used)
    if (k != a && beyond) inside = false;
    p[k] = k == a ? P : div_q28(num < 0 || beyond ? 0 : num, da32);
  }
  if (!inside) return false;
  E.p[0] = p[0];
  E.p[1] = p[1];
  E.p[2] = p[2];
  E.a = a;
  E.en = P - oa;
  E.da = da32;
  E.inv_da = pick3(a, R.inv_d);
  E.exact = 7;
  E.lam = kFix;
  return true;
}

// The part of the ray between the base-level slab boundaries lo and hi
// (slab indices along axis a, mirrored frame; lo = INT32_MIN: from the box
// entry, hi = INT32_MAX: to the box exit).  On entry E is the ray's box entry
// (setup_ray); on return E is the span's entry point and R.stop its end
// plane.  False for an empty span.  Boundaries at or before the entry slab's
// lower face are never crossed after the entry, so a span ending there is
// empty and a span starting there starts at the box entry: the spans of any
// increasing boundary sequence partition the ray.
AMR_HD bool span_bounds(Ray& R, Entry& E, int b0, int a, int32_t lo, int32_t hi) {
  const int sb = kFix - b0;
  const int32_t c0 = pick3(a, E.p) >> sb;
  if (hi <= c0) return false;
  if (hi < (int32_t(1) << b0)) {
    const int32_t P = hi << sb;
    R.stop[0] = a == 0 ? P : R.stop[0];
    R.stop[1] = a == 1 ? P : R.stop[1];
    R.stop[2] = a == 2 ? P : R.stop[2];
  }
  if (lo <= c0) return true;
  return plane_entry(R, a, lo << sb, E);
}

// Span w of K: the base-level slabs the ray crosses along its major axis,
// from the slab of its box entry to an estimate of the slab of its exit,
// dealt out in K contiguous runs of (nearly) equal count.  The exit
// estimate only balances the runs: the last non-empty run always continues
// to the box.
AMR_HD bool span_setup(Ray& R, Entry& E, int b0, int K, int w) {
  if (K <= 1) return true;
  const int a = major_axis(R);
  const int32_t da = pick3(a, R.d), oa = pick3(a, R.o);
  if (da <= 0) return w == 0;
  const int sb = kFix - b0;
  const int32_t c0 = pick3(a, E.p) >> sb;
  float te = 3.0e38f;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k)
    if (R.d[k] > 0) te = fminf(te, ((float)kOne - (float)R.o[k]) * R.inv_d[k]);
  const float ae = (float)oa + te * (float)da;
  int32_t c1 = (int32_t)fminf(fmaxf(ae * (1.0f / (float)(1 << sb)), 0.0f), (float)((1 << b0) - 1));
  c1 = c1 < c0 ? c0 : c1;
  const int32_t n = c1 - c0 + 1;
  // run w = slabs [c0 + ceil(w n / K), c0 + ceil((w + 1) n / K)): the first
  // run is never empty and every later one starts past the entry slab
  const int32_t s0 = c0 + (int32_t)(((int64_t)w * n + K - 1) / K);
  const int32_t s1 = c0 + (int32_t)(((int64_t)(w + 1) * n + K - 1) / K);
  if (s0 == s1) return false;
  const int32_t lo = w == 0 ? INT32_MIN : s0;
  const int32_t hi = (w + 1 < K && s1 < c0 + n) ? s1 : INT32_MAX;
  return span_bounds(R, E, b0, a, lo, hi);
}

// The part of the ray inside the cube of level `lc` with integer coordinates
// (cx, cy, cz) (box frame), for walks over one subtree of the tree.  On entry
// E is the ray's box entry (setup_ray); on return E is the entry point into
// the cube and R.stop its far faces, so the walk ends on leaving the cube.
// False when the ray spends no positive length inside it.  Every cell at
// level lc or deeper lies inside the cube or outside it, so when the walk
// starts at level lc or deeper (lc <= min(base, max_level)) the cube's
// cells partition the ray's cells that lie in it, each with the same exact
// decisions as on the whole ray.
// In mirrored coordinates a cube covering cells [lo, hi) of an axis covers
// [2^28 - hi, 2^28 - lo) when that axis is mirrored.  The entry is the
// latest of the box entry and the crossings of the cube's near faces,
// compared exactly; the ray is inside iff the entry point lies in the cube.
AMR_HD bool cube_clip(Ray& R, Entry& E, int lc, int32_t cx, int32_t cy, int32_t cz) {
  const int sc = kFix - lc;
  const int32_t cc[3] = {cx, cy, cz};
  int32_t mlo[3], mhi[3];
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    const int32_t lo = cc[k] << sc, hi = lo + (int32_t(1) << sc);
    mlo[k] = R.flip[k] ? kOne - hi : lo;
    mhi[k] = R.flip[k] ? kOne - lo : hi;
  }
  // latest near-face crossing beyond the box entry (en / da)
  int b = -1;
  int32_t bn = E.en, bd = E.da;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    const int32_t n = mlo[k] - R.o[k];
    if (R.d[k] > 0 && n > 0 && mul64(n, bd) > mul64(bn, R.d[k])) {
      b = k;
      bn = n;
      bd = R.d[k];
    }
  }
  if (b >= 0 && !plane_entry(R, b, mlo[b], E)) return false;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k)
    if (E.p[k] < mlo[k] || E.p[k] >= mhi[k]) return false;
  R.stop[0] = mhi[0];
  R.stop[1] = mhi[1];
  R.stop[2] = mhi[2];
  return true;
}

// Partial accumulators of one span: sum (s0, c0); maximum s0; weighted mean
// (s0, c0) = weight, (s1, c1) = weight x value, each a Kahan pair.
struct Partial {
  float s0, c0, s1, c1;
};

template <int OP>
AMR_HD void partial_init(Partial& P) {
  P.s0 = OP == kOpMax ? -INFINITY : 0.0f;
  P.c0 = P.s1 = P.c1 = 0.0f;
}

// Visitor V that also tracks cuts (TracksCut): cut_and is the bitwise AND of
// the child index of every cell where the descent stopped, negative at a
// leaf, so it stays negative exactly when no cell was cut.
template <class V>
struct CutVis : V {
  static constexpr bool kTrackCut = true;
  int32_t cut_and = -1;
};
template <bool kCut, class V>
using CutIf = typename std::conditional<kCut, CutVis<V>, V>::type;
template <class V>
AMR_HD void take_cut(const V& v, bool* cut) {
  if constexpr (TracksCut<V>::value) *cut = v.cut_and >= 0;
}

// kWholeBox: the span is the whole ray (no stop plane inside the box).
// kCut: *cut receives whether the walk cut a cell (TracksCut).
// kStd: the caller guarantees std_fields(), and for sum and max also
// max_level < kDeepLevel (no per-cell tests of the layout, nor for sum and
// max of the chord precision; measured, the wmean walk is faster with that
// test kept).
// Stk: an ancestor stack for walk_fast (NoStack: none).
template <int OP, bool kWholeBox = false, bool kCut = false, bool kStd = false, class Stk = NoStack>
AMR_HD void walk_span(const TreeView& T, const Ray& R, Entry& E, int max_level, int field, int wfield, int los,
                      Partial& P, bool* cut, Stk& stk) {
  const int64_t nc = T.ncells;
  if (OP == kOpSum) {
    CutIf<kCut, SumVisT<kStd>> v;
    v.v = T.val + (int64_t)field * nc;
    v.field0 = field == 0;
    walk_fast<decltype(v), kWholeBox, kStd, Stk>(T, R, E, max_level, v, stk);
    P.s0 = v.s;
    P.c0 = v.c;
    take_cut(v, cut);
  } else if (OP == kOpMax) {
    CutIf<kCut, MaxVisT<kStd>> v;
    v.v = T.val + (int64_t)field * nc;
    v.m = -INFINITY;
    v.field0 = field == 0;
    walk_fast<decltype(v), kWholeBox, kStd, Stk>(T, R, E, max_level, v, stk);
    P.s0 = v.m;
    take_cut(v, cut);
  } else {
    CutIf<kCut, WMeanVisT<kStd>> v;
    v.w = T.val + (int64_t)wfield * nc;
    v.f0 = T.val + (int64_t)field * nc;
    v.f1 = los ? v.f0 + nc : v.f0;
    v.f2 = los ? v.f0 + 2 * nc : v.f0;
    v.los = los;
    if (kStd || packed_los(T, field, wfield, los)) v.use_packed(T);
    const float n = sqrtf((float)(R.d64[0] * R.d64[0] + R.d64[1] * R.d64[1] + R.d64[2] * R.d64[2]));
    AMR_UNROLL
    for (int k = 0; k < 3; ++k) v.dh[k] = (float)R.d64[k] / n;
    walk_fast<decltype(v), kWholeBox, false, Stk>(T, R, E, max_level, v, stk);
    P.s0 = v.sw;
    P.c0 = v.cw;
    P.s1 = v.sf;
    P.c1 = v.cf;
    take_cut(v, cut);
  }
}

template <int OP, bool kWholeBox = false, bool kCut = false, bool kStd = false>
AMR_HD void walk_span(const TreeView& T, const Ray& R, Entry& E, int max_level, int field, int wfield, int los,
                      Partial& P, bool* cut = nullptr) {
  NoStack none;
  walk_span<OP, kWholeBox, kCut, kStd, NoStack>(T, R, E, max_level, field, wfield, los, P, cut, none);
}

// A per-thread ancestor stack in LDS, laid out [level][thread] (STRIDE
// threads per block) so that a wave's 64 lanes touch 64 consecutive words;
// levels lo + 1 .. max_level.
template <int STRIDE>
struct StridedStack {
  int32_t* base;  // this thread's word of level lo
  int lo;
  AMR_HD int32_t get(int l) const { return base[(l - lo) * STRIDE]; }
  AMR_HD void set(int l, int32_t v) { base[(l - lo) * STRIDE] = v; }
};

// P += Q (Q is the next span along the ray).
template <int OP>
AMR_HD void partial_merge(Partial& P, const Partial& Q) {
  if (OP == kOpMax) {
    P.s0 = fmaxf(P.s0, Q.s0);
    return;
  }
  kahan_add(P.s0, P.c0, Q.s0);
  kahan_add(P.s0, P.c0, -Q.c0);
  if (OP == kOpWMean) {
    kahan_add(P.s1, P.c1, Q.s1);
    kahan_add(P.s1, P.c1, -Q.c1);
  }
}

template <int OP>
AMR_HD void partial_finish(const Partial& P, float& out, float& aux) {
  if (OP == kOpSum) {
    out = P.s0 - P.c0;
  } else if (OP == kOpMax) {
    out = P.s0;
  } else {
    const float W = P.s0 - P.c0, Sf = P.s1 - P.c1;
    out = W > 0.0f ? Sf / W : 0.0f;
    aux = W;
  }
}

}  // namespace amr
