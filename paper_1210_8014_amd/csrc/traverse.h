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

struct TreeView {
  const int32_t* child;  // first-child index per cell, -1 for leaves
  const float* val;      // [nfields][ncells]
  const uint8_t* maxdepth;
  int64_t ncells;
  int32_t nfields;
  int32_t base;  // levels 0..base are complete; base <= kMaxArithBase
  int32_t lmax;
  int32_t pad_;
  int32_t off[kMaxLevel + 2];  // first cell index of each level
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

// Per-ray constants in mirrored coordinates.
struct Ray {
  int32_t o[3];    // mirrored origin
  int32_t d[3];    // |direction|, >= 0
  int32_t flip[3]; // 2^28 - 1 on mirrored axes, else 0
  int64_t d64[3];  // unmirrored direction
  float wk[3];     // |d| 2^-28 / d_k  (chord per unit of parameter numerator)
  float inv_d[3];  // 1 / d_k
  double ulen64;   // |d| 2^-28
};

// Entry point of the current cell: t = (Xa - oa) / da on axis a, or t = 0
// (a < 0) when the ray starts inside the box.  p[] holds the integer part
// of the entry point (mirrored), exactly on the axes flagged in `exact`,
// down to level `lam` on the others.
struct Entry {
  int32_t p[3];
  int a;
  int32_t Xa, oa, da;
  float inv_da;
  int exact, lam;
};

template <class T>
AMR_HD T sel3(const T (&v)[3], int k) {
  return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]);
}

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
  if (miss) return false;
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
      E.p[k] = (int32_t)((uint64_t)num / (uint64_t)(uint32_t)ed);
    }
  }
  E.a = a;
  E.Xa = 0;
  E.oa = oa;
  E.da = ed;
  E.exact = 7;
  E.lam = kFix;
  // chord scale factors
  const int64_t dd0 = R.d64[0] * R.d64[0] + R.d64[1] * R.d64[1] + R.d64[2] * R.d64[2];
  const float ulen = sqrtf((float)dd0) * 0x1.0p-28f;
  R.ulen64 = sqrt((double)dd0) * 0x1.0p-28;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) {
    R.inv_d[k] = R.d[k] > 0 ? 1.0f / (float)R.d[k] : 0.0f;
    R.wk[k] = R.d[k] > 0 ? ulen / (float)R.d[k] : 0.0f;
  }
  E.inv_da = a < 0 ? 0.0f : 1.0f / (float)ed;
  return true;
}

// Walks the cells of one ray.  The visitor sees, for every cell met, its
// index, level, chord length and mirrored cell coordinates:
//   vis.seg(node, level, len, cm0, cm1, cm2)
// It returns the number of cells visited.  max_level truncates the tree.
template <class Vis>
AMR_HD int32_t walk_ray(const TreeView& T, const Ray& R, Entry& E, int max_level, Vis& vis) {
  const int b0 = T.base < max_level ? T.base : max_level;
  int32_t nseg = 0;
  for (;;) {
    // ---- locate the cell containing r(t_entry + 0)
    int lvl = b0;
    const int sb = kFix - b0;
    int32_t node = T.off[b0] + (int32_t)morton3((uint32_t)((E.p[0] ^ R.flip[0]) >> sb),
                                                (uint32_t)((E.p[1] ^ R.flip[1]) >> sb),
                                                (uint32_t)((E.p[2] ^ R.flip[2]) >> sb));
    AMR_CHECK_CELL(T, node);
    while (lvl < max_level) {
      const int32_t w = T.child[node];
      if (w < 0) break;
      ++lvl;
      const int s = kFix - lvl;
      if (lvl > E.lam) {
        // decide bit s of the entry point on the axes not known exactly:
        // x_k(t_e) >= M  <=>  (Xa - o_a) d_k >= (M - o_k) d_a
        AMR_UNROLL
        for (int k = 0; k < 3; ++k) {
          if (E.exact & (1 << k)) continue;
          const int32_t M = E.p[k] + (int32_t(1) << s);
          if (mul64(E.Xa - E.oa, R.d[k]) >= mul64(M - R.o[k], E.da)) E.p[k] = M;
        }
        E.lam = lvl;
      }
      const int oct = (((E.p[0] ^ R.flip[0]) >> s) & 1) | ((((E.p[1] ^ R.flip[1]) >> s) & 1) << 1) |
                      ((((E.p[2] ^ R.flip[2]) >> s) & 1) << 2);
      node = w + oct;
      AMR_CHECK_CELL(T, node);
    }
    // ---- exit face: smallest (X_k - o_k) / d_k over moving axes, ties kept
    const int s = kFix - lvl;
    int32_t X[3];
    int best = -1, tie = 0;
    int32_t nb = 0, db = 1, Xb = 0;
    float wkb = 0.0f, invb = 0.0f;
    AMR_UNROLL
    for (int k = 0; k < 3; ++k) {
      X[k] = ((E.p[k] >> s) + 1) << s;
      if (R.d[k] == 0) continue;
      const int32_t nk = X[k] - R.o[k];
      bool take = best < 0;
      if (!take) {
        const int64_t diff = mul64(nk, db) - mul64(nb, R.d[k]);
        if (diff == 0) tie |= 1 << k;
        take = diff < 0;
      }
      if (take) {
        best = k;
        tie = 1 << k;
        nb = nk;
        db = R.d[k];
        Xb = X[k];
        wkb = R.wk[k];
        invb = R.inv_d[k];
      }
    }
    // ---- chord length from the exact numerator of t_exit - t_entry
    float len;
    if (lvl < kDeepLevel) {
      if (E.a < 0)
        len = (float)nb * wkb;
      else if (E.a == best)
        len = (float)(Xb - E.Xa) * wkb;
      else
        len = (float)(mul64(nb, E.da) - mul64(E.Xa - E.oa, db)) * wkb * E.inv_da;
    } else {
      double l64;
      if (E.a < 0)
        l64 = (double)nb * R.ulen64 / (double)db;
      else if (E.a == best)
        l64 = (double)(Xb - E.Xa) * R.ulen64 / (double)db;
      else
        l64 = (double)(mul64(nb, E.da) - mul64(E.Xa - E.oa, db)) * R.ulen64 / ((double)E.da * (double)db);
      len = (float)l64;
    }
    vis.seg(node, lvl, len, E.p[0] >> s, E.p[1] >> s, E.p[2] >> s);
    ++nseg;
    // ---- leave the box, or enter the neighbour
    bool out = false;
    AMR_UNROLL
    for (int k = 0; k < 3; ++k)
      if ((tie & (1 << k)) && X[k] == kOne) out = true;
    if (out) break;
    const int32_t keep = ~((int32_t(1) << s) - 1);
    AMR_UNROLL
    for (int k = 0; k < 3; ++k) {
      if (tie & (1 << k)) {
        E.p[k] = X[k];
        E.exact |= 1 << k;
      } else if (R.d[k] > 0) {
        E.p[k] &= keep;
        E.exact &= ~(1 << k);
      }
    }
    E.lam = lvl;
    E.a = best;
    E.Xa = Xb;
    E.oa = Xb - nb;
    E.da = db;
    E.inv_da = invb;
  }
  return nseg;
}

// ----------------------------------------------------------------- visitors

struct SumVis {
  const float* v;
  float s = 0.0f, c = 0.0f;
  AMR_HD void seg(int32_t node, int, float len, int32_t, int32_t, int32_t) { kahan_add(s, c, v[node] * len); }
};

struct MaxVis {
  const float* v;
  float m;
  AMR_HD void seg(int32_t node, int, float, int32_t, int32_t, int32_t) { m = fmaxf(m, v[node]); }
};

struct WMeanVis {
  const float* w;
  const float* f0;
  const float* f1;
  const float* f2;
  float dh[3];
  int los;
  float sw = 0.0f, cw = 0.0f, sf = 0.0f, cf = 0.0f;
  AMR_HD void seg(int32_t node, int, float len, int32_t, int32_t, int32_t) {
    const float wl = w[node] * len;
    float f = f0[node];
    if (los) f = f * dh[0] + f1[node] * dh[1] + f2[node] * dh[2];
    kahan_add(sw, cw, wl);
    kahan_add(sf, cf, wl * f);
  }
};

struct CountVis {
  AMR_HD void seg(int32_t, int, float, int32_t, int32_t, int32_t) {}
};

// Writes (level, ix, iy, iz) of every cell, unmirrored.
struct TraceVis {
  int32_t* out;
  int32_t flip_bits[3];  // 1 on mirrored axes
  AMR_HD void seg(int32_t, int lvl, float, int32_t c0, int32_t c1, int32_t c2) {
    const int32_t m = (int32_t(1) << lvl) - 1;
    out[0] = lvl;
    out[1] = flip_bits[0] ? (c0 ^ m) : c0;
    out[2] = flip_bits[1] ? (c1 ^ m) : c1;
    out[3] = flip_bits[2] ? (c2 ^ m) : c2;
    out += 4;
  }
};

// ------------------------------------------------------------ one pixel

enum { kOpSum = 0, kOpMax = 1, kOpWMean = 2 };

// The whole per-pixel computation of one projection; out receives the
// pixel value, aux (WMEAN) the weight integral.
template <int OP>
AMR_HD void render_pixel(const TreeView& T, const CameraView& C, int field, int wfield, int los, int max_level,
                         int i, int j, float& out, float& aux) {
  Ray R;
  Entry E;
  const bool hit = setup_ray(C, i, j, R, E);
  const int64_t nc = T.ncells;
  if (OP == kOpSum) {
    SumVis v{T.val + (int64_t)field * nc};
    if (hit) walk_ray(T, R, E, max_level, v);
    out = v.s - v.c;
  } else if (OP == kOpMax) {
    MaxVis v{T.val + (int64_t)field * nc, -INFINITY};
    if (hit) walk_ray(T, R, E, max_level, v);
    out = v.m;
  } else {
    WMeanVis v;
    v.w = T.val + (int64_t)wfield * nc;
    v.f0 = T.val + (int64_t)field * nc;
    v.f1 = los ? v.f0 + nc : v.f0;
    v.f2 = los ? v.f0 + 2 * nc : v.f0;
    v.los = los;
    v.dh[0] = v.dh[1] = v.dh[2] = 0.0f;
    if (hit) {
      const float n = sqrtf((float)(R.d64[0] * R.d64[0] + R.d64[1] * R.d64[1] + R.d64[2] * R.d64[2]));
      AMR_UNROLL
      for (int k = 0; k < 3; ++k) v.dh[k] = (float)R.d64[k] / n;
      walk_ray(T, R, E, max_level, v);
    }
    const float W = v.sw - v.cw, S = v.sf - v.cf;
    out = W > 0.0f ? S / W : 0.0f;
    aux = W;
  }
}

// Number of cells on the ray of pixel (i, j); with cells != NULL they are
// also written (4 int32 each), but only if exactly `cap` of them exist.
AMR_HD int32_t trace_pixel(const TreeView& T, const CameraView& C, int max_level, int i, int j, int32_t* cells,
                           int64_t cap) {
  Ray R;
  Entry E;
  if (!setup_ray(C, i, j, R, E)) return 0;
  const Entry E0 = E;
  CountVis c;
  const int32_t m = walk_ray(T, R, E, max_level, c);
  if (!cells || m != cap) return m;
  TraceVis v;
  v.out = cells;
  AMR_UNROLL
  for (int k = 0; k < 3; ++k) v.flip_bits[k] = R.flip[k] ? 1 : 0;
  E = E0;
  walk_ray(T, R, E, max_level, v);
  return m;
}

}  // namespace amr
