/*
 * oracle.c -- plain, slow, obviously-correct CPU oracle for per-pixel ray
 * casting through an octree AMR volume.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the GPU library.
 *
 * What it computes (Labadens et al., "Volume Rendering of AMR Simulations"):
 *
 *  - Truncation (Sec. 2, opening paragraph): the camera fixes a maximum level
 *    L; every cell at level L is treated as a leaf, and finer cells are never
 *    read.  A truncated cell carries the restricted value of its subtree
 *    (reading: volume mean for densities, mass-weighted mean for velocities,
 *    computed in fp64 over the 8 children in fixed Morton child order, then
 *    rounded once to fp32).
 *
 *  - Ray casting (Sec. 2.2): one ray per pixel.  The ray starts at the root
 *    and descends the octree top-down; the entry and exit points of the ray
 *    on the faces of each cell it meets are found, and the descent stops at
 *    leaves.  Each leaf's value is multiplied by the length between its entry
 *    and exit points and the contributions are added with no ordering
 *    requirement ("sum").  The maximum-intensity projection mentioned in
 *    Sec. 2.1 is the maximum of the leaf values met ("max").  A mass-weighted
 *    mean of a field along the ray ("wmean") is added over the per-cell
 *    fields the paper lists in Sec. 1 (density, velocity).
 *
 * Exactness: positions are integers in units of 2^-28 of the box, ray
 * directions are integers (the quantised camera record), so every entry and
 * exit parameter is a rational (P - o_k) / d_k, held here as a pair of
 * integers and compared by exact 128-bit cross multiplication.  A cell is on
 * the ray iff the ray spends a positive parameter length inside it (cells
 * are half-open boxes [a, b)); zero-length contacts (edges, corners) are not
 * segments.  Segments are sorted by exact entry parameter.  Chord lengths are
 * formed from an exact 128-bit numerator, then converted to fp64.  Sums use
 * fp64 with Neumaier compensation.
 *
 * Camera: the oracle consumes the integer camera record (origin O, view
 * step F, half-pixel steps U and V), which the tests produce with the
 * oracle's own exact quantiser (camera.py); pixel_ray below turns it into
 * the integer ray of a pixel.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

#define FIX_BITS 28
#define FIX_ONE ((int64_t)1 << FIX_BITS)
#define MAX_LEVEL 24

enum { OC_OK = 0, OC_EINVAL = 1, OC_ETREE = 2, OC_ENOMEM = 3, OC_ECAPACITY = 4 };
enum { OC_SUM = 0, OC_MAX = 1, OC_WMEAN = 2 };

/* ------------------------------------------------------------------ camera */

typedef struct {
  int32_t kind, W, H, max_level;
  int64_t O[3], F[3], U[3], V[3];
} oc_camera;

/* Integer ray of pixel (i, j): through the pixel centre, j = 0 at the bottom. */
static void pixel_ray(const oc_camera* C, int64_t i, int64_t j, int64_t o[3], int64_t dv[3]) {
  int64_t a = 2 * i + 1 - C->W, b = 2 * j + 1 - C->H;
  for (int k = 0; k < 3; ++k) {
    if (C->kind == 0) {
      o[k] = C->O[k];
      dv[k] = C->F[k] + a * C->U[k] + b * C->V[k];
    } else {
      o[k] = C->O[k] + a * C->U[k] + b * C->V[k];
      dv[k] = C->F[k];
    }
  }
}

/* -------------------------------------------------------------------- tree */

typedef struct {
  int32_t level, ix, iy, iz;
  int32_t first_child; /* index of child 0; children 0..7 contiguous; -1 if none */
  int32_t state;       /* 0 = not yet defined, 1 = leaf, 2 = refined */
} oc_node;

typedef struct oc_tree {
  int64_t n, cap;
  oc_node* nodes;
  int32_t nfields, lmax;
  double* v64; /* [nfields][cap] restricted fp64 values */
  float* v32;  /* [nfields][cap] stored fp32 values */
  int32_t* depth; /* deepest leaf level in each node's subtree */
} oc_tree;

static int grow(oc_tree* T, int64_t need) {
  if (need <= T->cap) return 0;
  int64_t nc = T->cap ? T->cap : 1024;
  while (nc < need) nc *= 2;
  oc_node* nn = (oc_node*)realloc(T->nodes, sizeof(oc_node) * nc);
  if (!nn) return -1;
  T->nodes = nn;
  T->cap = nc;
  return 0;
}

void oc_tree_free(oc_tree* T) {
  if (!T) return;
  free(T->nodes);
  free(T->v64);
  free(T->v32);
  free(T->depth);
  free(T);
}

/*
 * Build the oracle's own tree by inserting every leaf from the root.
 * restrict_weight[f] = -1: field f restricts as a volume mean;
 * restrict_weight[f] = w >= 0: field f restricts as a mean weighted by field
 * w (mass-weighted for w = density).
 */
int oc_tree_build(int64_t n, const int32_t* level, const int32_t* ix, const int32_t* iy, const int32_t* iz,
                  const float* fields, int32_t nfields, int64_t field_stride, const int32_t* restrict_weight,
                  oc_tree** out) {
  if (!out || n < 1 || !level || !ix || !iy || !iz || !fields || nfields < 1 || nfields > 16) return OC_EINVAL;
  *out = NULL;
  for (int f = 0; f < nfields; ++f) {
    int w = restrict_weight ? restrict_weight[f] : -1;
    if (w >= nfields || w == f || (w >= 0 && restrict_weight[w] >= 0)) return OC_EINVAL;
  }
  oc_tree* T = (oc_tree*)calloc(1, sizeof(oc_tree));
  if (!T) return OC_ENOMEM;
  T->nfields = nfields;
  int64_t* leaf_of = NULL;
  if (grow(T, 1)) goto nomem;
  T->nodes[0] = (oc_node){0, 0, 0, 0, -1, 0};
  T->n = 1;
  for (int64_t q = 0; q < n; ++q) {
    int32_t l = level[q];
    if (l < 0 || l > MAX_LEVEL) { oc_tree_free(T); return OC_EINVAL; }
    int64_t side = (int64_t)1 << l;
    if (ix[q] < 0 || iy[q] < 0 || iz[q] < 0 || ix[q] >= side || iy[q] >= side || iz[q] >= side) {
      oc_tree_free(T);
      return OC_ETREE;
    }
    for (int f = 0; f < nfields; ++f) {
      float v = fields[(int64_t)f * field_stride + q];
      if (!isfinite(v)) { oc_tree_free(T); return OC_EINVAL; }
    }
    int64_t cur = 0;
    for (int32_t dlev = 0; dlev < l; ++dlev) {
      oc_node* nd = &T->nodes[cur];
      if (nd->state == 1) { oc_tree_free(T); return OC_ETREE; } /* overlaps a coarser leaf */
      if (nd->state == 0) {
        if (grow(T, T->n + 8)) goto nomem;
        nd = &T->nodes[cur];
        nd->state = 2;
        nd->first_child = (int32_t)T->n;
        for (int c = 0; c < 8; ++c) {
          oc_node ch;
          ch.level = dlev + 1;
          ch.ix = 2 * nd->ix + (c & 1);
          ch.iy = 2 * nd->iy + ((c >> 1) & 1);
          ch.iz = 2 * nd->iz + ((c >> 2) & 1);
          ch.first_child = -1;
          ch.state = 0;
          T->nodes[T->n + c] = ch;
        }
        T->n += 8;
        if (T->n >= ((int64_t)1 << 31) - 8) { oc_tree_free(T); return OC_ENOMEM; }
      }
      int sh = l - 1 - dlev;
      int c = ((ix[q] >> sh) & 1) | (((iy[q] >> sh) & 1) << 1) | (((iz[q] >> sh) & 1) << 2);
      cur = T->nodes[cur].first_child + c;
    }
    if (T->nodes[cur].state != 0) { oc_tree_free(T); return OC_ETREE; } /* duplicate or covers finer leaves */
    T->nodes[cur].state = 1;
    T->nodes[cur].first_child = (int32_t)(-2 - q); /* temporarily: which input leaf */
    if (l > T->lmax) T->lmax = l;
  }
  for (int64_t i = 0; i < T->n; ++i)
    if (T->nodes[i].state == 0) { oc_tree_free(T); return OC_ETREE; } /* gap: an octant nobody covers */

  T->v64 = (double*)malloc(sizeof(double) * nfields * T->n);
  T->v32 = (float*)malloc(sizeof(float) * nfields * T->n);
  leaf_of = (int64_t*)malloc(sizeof(int64_t) * T->n);
  if (!T->v64 || !T->v32 || !leaf_of) goto nomem;
  for (int64_t i = 0; i < T->n; ++i) {
    leaf_of[i] = -1;
    if (T->nodes[i].state == 1) {
      leaf_of[i] = -2 - (int64_t)T->nodes[i].first_child;
      T->nodes[i].first_child = -1;
    }
  }
  /* Leaves: fp32 input widened to fp64.  Weighted fields are carried as
   * weight * value ("momentum") while restricting. */
  for (int f = 0; f < nfields; ++f) {
    int w = restrict_weight ? restrict_weight[f] : -1;
    double* vf = T->v64 + (int64_t)f * T->n;
    for (int64_t i = 0; i < T->n; ++i) {
      if (leaf_of[i] < 0) continue;
      double v = (double)fields[(int64_t)f * field_stride + leaf_of[i]];
      if (w >= 0) v *= (double)fields[(int64_t)w * field_stride + leaf_of[i]];
      vf[i] = v;
    }
  }
  /* Restriction, children before parents (children always have larger
   * indices): mean of the 8 children summed in child order 0..7. */
  for (int64_t i = T->n - 1; i >= 0; --i) {
    if (T->nodes[i].state != 2) continue;
    int64_t c0 = T->nodes[i].first_child;
    for (int f = 0; f < nfields; ++f) {
      double* vf = T->v64 + (int64_t)f * T->n;
      double s = 0.0;
      for (int c = 0; c < 8; ++c) s += vf[c0 + c];
      vf[i] = s / 8.0;
    }
  }
  /* Weighted fields: value = (weighted sum) / (restricted weight); at the
   * leaves this is the input value itself, recomputed for uniformity only
   * where the cell is refined. */
  for (int f = 0; f < nfields; ++f) {
    int w = restrict_weight ? restrict_weight[f] : -1;
    if (w < 0) continue;
    double* vf = T->v64 + (int64_t)f * T->n;
    const double* vw = T->v64 + (int64_t)w * T->n;
    for (int64_t i = 0; i < T->n; ++i) {
      if (leaf_of[i] >= 0)
        vf[i] = (double)fields[(int64_t)f * field_stride + leaf_of[i]];
      else
        vf[i] = vw[i] != 0.0 ? vf[i] / vw[i] : 0.0;
    }
  }
  for (int64_t k = 0; k < (int64_t)nfields * T->n; ++k) T->v32[k] = (float)T->v64[k];
  T->depth = (int32_t*)malloc(sizeof(int32_t) * T->n);
  if (!T->depth) goto nomem;
  for (int64_t i = T->n - 1; i >= 0; --i) {
    if (T->nodes[i].state == 1) {
      T->depth[i] = T->nodes[i].level;
    } else {
      int32_t m = 0;
      for (int c = 0; c < 8; ++c)
        if (T->depth[T->nodes[i].first_child + c] > m) m = T->depth[T->nodes[i].first_child + c];
      T->depth[i] = m;
    }
  }
  free(leaf_of);
  *out = T;
  return OC_OK;
nomem:
  free(leaf_of);
  oc_tree_free(T);
  return OC_ENOMEM;
}

int64_t oc_tree_nodes(const oc_tree* T) { return T ? T->n : 0; }
int32_t oc_tree_lmax(const oc_tree* T) { return T ? T->lmax : -1; }

/* Stored fp32 values of the cell (level, ix, iy, iz); OC_EINVAL if the cell
 * is not in the tree. */
int oc_lookup(const oc_tree* T, int32_t l, int32_t x, int32_t y, int32_t z, float* vals, double* vals64) {
  int64_t cur = 0;
  for (int32_t dlev = 0; dlev < l; ++dlev) {
    if (T->nodes[cur].state != 2) return OC_EINVAL;
    int sh = l - 1 - dlev;
    int c = ((x >> sh) & 1) | (((y >> sh) & 1) << 1) | (((z >> sh) & 1) << 2);
    cur = T->nodes[cur].first_child + c;
  }
  for (int f = 0; f < T->nfields; ++f) {
    if (vals) vals[f] = T->v32[(int64_t)f * T->n + cur];
    if (vals64) vals64[f] = T->v64[(int64_t)f * T->n + cur];
  }
  return OC_OK;
}

/* --------------------------------------------------------------- ray cast */

typedef struct {
  int64_t num, den; /* value num / den, den > 0 */
} rat;

static int rat_lt(rat a, rat b) { return (i128)a.num * b.den < (i128)b.num * a.den; }

typedef struct {
  rat t0, t1; /* entry and exit parameters */
  int64_t node;
} seg;

typedef struct {
  seg* s;
  int64_t n, cap;
} segbuf;

static int push(segbuf* B, rat t0, rat t1, int64_t node) {
  if (B->n == B->cap) {
    int64_t nc = B->cap ? 2 * B->cap : 256;
    seg* ns = (seg*)realloc(B->s, sizeof(seg) * nc);
    if (!ns) return -1;
    B->s = ns;
    B->cap = nc;
  }
  B->s[B->n].t0 = t0;
  B->s[B->n].t1 = t1;
  B->s[B->n].node = node;
  B->n++;
  return 0;
}

/* Top-down descent: visit every cell whose box the ray crosses over a
 * positive parameter length, stop at leaves or at the maximum level. */
static int visit(const oc_tree* T, int64_t idx, const int64_t o[3], const int64_t d[3], int32_t L, segbuf* B) {
  const oc_node* nd = &T->nodes[idx];
  int sh = FIX_BITS - nd->level;
  rat enter = {0, 1};
  rat exit_ = {0, 0}; /* den 0: +infinity */
  int32_t cc[3] = {nd->ix, nd->iy, nd->iz};
  for (int k = 0; k < 3; ++k) {
    int64_t lo = (int64_t)cc[k] << sh, hi = ((int64_t)cc[k] + 1) << sh;
    if (d[k] == 0) {
      if (!(lo <= o[k] && o[k] < hi)) return 0;
      continue;
    }
    rat a, b;
    if (d[k] > 0) {
      a.num = lo - o[k]; a.den = d[k];
      b.num = hi - o[k]; b.den = d[k];
    } else {
      a.num = o[k] - hi; a.den = -d[k];
      b.num = o[k] - lo; b.den = -d[k];
    }
    if (rat_lt(enter, a)) enter = a;
    if (exit_.den == 0 || rat_lt(b, exit_)) exit_ = b;
  }
  if (exit_.den == 0) return 0; /* impossible: d != 0 */
  if (!rat_lt(enter, exit_)) return 0;
  if (nd->state == 1 || nd->level >= L) return push(B, enter, exit_, idx);
  for (int c = 0; c < 8; ++c)
    if (visit(T, nd->first_child + c, o, d, L, B)) return -1;
  return 0;
}

static int seg_cmp(const void* pa, const void* pb) {
  const seg* a = (const seg*)pa;
  const seg* b = (const seg*)pb;
  if (rat_lt(a->t0, b->t0)) return -1;
  if (rat_lt(b->t0, a->t0)) return 1;
  return 0;
}

/* Cells of the ray of pixel `pix`, in order of entry. */
static int ray_segments(const oc_tree* T, const oc_camera* C, int64_t pix, segbuf* B, int64_t o[3], int64_t d[3]) {
  B->n = 0;
  pixel_ray(C, pix % C->W, pix / C->W, o, d);
  if (visit(T, 0, o, d, C->max_level, B)) return -1;
  qsort(B->s, (size_t)B->n, sizeof(seg), seg_cmp);
  return 0;
}

/* |d| * 2^-28: length, in box units, of a unit of ray parameter. */
static double unit_length(const int64_t d[3]) {
  i128 dd = (i128)d[0] * d[0] + (i128)d[1] * d[1] + (i128)d[2] * d[2];
  return ldexp((double)sqrtl((long double)dd), -FIX_BITS);
}

/* Chord length in box units: (t1 - t0) |d| 2^-28, numerator exact. */
static double chord(const seg* s, double ulen) {
  i128 num = (i128)s->t1.num * s->t0.den - (i128)s->t0.num * s->t1.den;
  i128 den = (i128)s->t0.den * s->t1.den;
  return (double)num / (double)den * ulen;
}

typedef struct {
  double s, c;
} neum;

static void neum_add(neum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

/*
 * Render a set of pixels (ray_ids = pixel indices j*W + i; NULL = all W*H).
 *   op = OC_SUM:   out_val = sum over cells of v_f * chord
 *   op = OC_MAX:   out_max = max over cells of v_f (-inf when no cell)
 *   op = OC_WMEAN: out_val = sum(w f chord) / sum(w chord) (0 when the
 *                  weight is 0); out_aux = sum(w chord); out_absf =
 *                  sum(w |f| chord) / sum(w chord).  With los != 0, f is
 *                  the line-of-sight velocity (v_field, v_field+1,
 *                  v_field+2) . d / |d|; otherwise f is field v_field.
 *                  out_absf is the scale for error bars: with los it uses
 *                  |v_0 dh_0| + |v_1 dh_1| + |v_2 dh_2| for |f|, the size of
 *                  the terms whose single-precision dot product a renderer
 *                  rounds (the bound for a rounded dot product of n terms is
 *                  about n eps times the sum of their magnitudes);
 *                  out_absdot = sum(w |f| chord) / sum(w chord), the weighted
 *                  mean of |f| itself (equal to out_absf without los).
 * out_count = number of cells on each ray.  Any output may be NULL.
 */
int oc_render(const oc_tree* T, const oc_camera* C, int32_t op, int32_t v_field, int32_t w_field, int32_t los,
              const int64_t* ray_ids, int64_t nrays, double* out_val, float* out_max, double* out_aux,
              double* out_absf, double* out_absdot, int32_t* out_count, int32_t nthreads) {
  if (!T || !C) return OC_EINVAL;
  if (op < 0 || op > 2) return OC_EINVAL;
  if (v_field < 0 || v_field + (los ? 2 : 0) >= T->nfields) return OC_EINVAL;
  if (op == OC_WMEAN && (w_field < 0 || w_field >= T->nfields)) return OC_EINVAL;
  int64_t total = ray_ids ? nrays : (int64_t)C->W * C->H;
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    segbuf B = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < total; ++r) {
      int64_t pix = ray_ids ? ray_ids[r] : r;
      int64_t o[3], d[3];
      if (ray_segments(T, C, pix, &B, o, d)) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      double ulen = unit_length(d);
      const float* vf = T->v32 + (int64_t)v_field * T->n;
      if (out_count) out_count[r] = (int32_t)B.n;
      if (op == OC_SUM) {
        neum acc = {0.0, 0.0};
        for (int64_t k = 0; k < B.n; ++k) neum_add(&acc, (double)vf[B.s[k].node] * chord(&B.s[k], ulen));
        if (out_val) out_val[r] = acc.s + acc.c;
      } else if (op == OC_MAX) {
        float m = -INFINITY;
        for (int64_t k = 0; k < B.n; ++k) {
          float v = vf[B.s[k].node];
          if (v > m) m = v;
        }
        if (out_max) out_max[r] = m;
      } else {
        const float* wf = T->v32 + (int64_t)w_field * T->n;
        double dn = sqrt((double)((i128)d[0] * d[0] + (i128)d[1] * d[1] + (i128)d[2] * d[2]));
        double dh[3] = {(double)d[0] / dn, (double)d[1] / dn, (double)d[2] / dn};
        neum num = {0, 0}, den = {0, 0}, ab = {0, 0}, ad = {0, 0};
        for (int64_t k = 0; k < B.n; ++k) {
          int64_t nd = B.s[k].node;
          double f, fa;
          if (los) {
            const double p0 = (double)T->v32[(int64_t)v_field * T->n + nd] * dh[0];
            const double p1 = (double)T->v32[(int64_t)(v_field + 1) * T->n + nd] * dh[1];
            const double p2 = (double)T->v32[(int64_t)(v_field + 2) * T->n + nd] * dh[2];
            f = p0 + p1 + p2;
            fa = fabs(p0) + fabs(p1) + fabs(p2);
          } else {
            f = (double)vf[nd];
            fa = fabs(f);
          }
          double wl = (double)wf[nd] * chord(&B.s[k], ulen);
          neum_add(&num, wl * f);
          neum_add(&den, wl);
          neum_add(&ab, wl * fa);
          neum_add(&ad, wl * fabs(f));
        }
        double W = den.s + den.c;
        if (out_val) out_val[r] = W != 0.0 ? (num.s + num.c) / W : 0.0;
        if (out_aux) out_aux[r] = W;
        if (out_absf) out_absf[r] = W != 0.0 ? (ab.s + ab.c) / W : 0.0;
        if (out_absdot) out_absdot[r] = W != 0.0 ? (ad.s + ad.c) / W : 0.0;
      }
    }
    free(B.s);
  }
  return err ? OC_ENOMEM : OC_OK;
}

/*
 * Cell sequences of a set of rays, in order along the ray.  For ray r the
 * cells are entries offsets[r] .. offsets[r+1]-1 of:
 *   cells[4 s + 0..3] = level, ix, iy, iz   (unmirrored cell coordinates)
 *   tq[4 s + 0..3]    = entry num, entry den, exit num, exit den (exact
 *                       ray parameters; may be NULL)
 * With cells == NULL only offsets are filled (sizing pass).  Returns
 * OC_ECAPACITY if cap is too small.
 */
int oc_trace(const oc_tree* T, const oc_camera* C, const int64_t* ray_ids, int64_t nrays, int32_t* cells,
             int64_t* tq, int64_t cap, int64_t* offsets, int32_t nthreads) {
  if (!T || !C || !offsets || nrays < 0) return OC_EINVAL;
  int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (nrays > 0 ? nrays : 1));
  if (!cnt) return OC_ENOMEM;
  int rc = oc_render(T, C, OC_MAX, 0, -1, 0, ray_ids, nrays, NULL, NULL, NULL, NULL, NULL, cnt, nthreads);
  if (rc) { free(cnt); return rc; }
  offsets[0] = 0;
  for (int64_t r = 0; r < nrays; ++r) offsets[r + 1] = offsets[r] + cnt[r];
  free(cnt);
  if (!cells) return OC_OK;
  if (offsets[nrays] > cap) return OC_ECAPACITY;
  int err = 0;
#pragma omp parallel
  {
    segbuf B = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrays; ++r) {
      int64_t o[3], d[3];
      if (ray_segments(T, C, ray_ids ? ray_ids[r] : r, &B, o, d)) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      int64_t base = offsets[r];
      for (int64_t k = 0; k < B.n; ++k) {
        const oc_node* nd = &T->nodes[B.s[k].node];
        int32_t* c = cells + 4 * (base + k);
        c[0] = nd->level; c[1] = nd->ix; c[2] = nd->iy; c[3] = nd->iz;
        if (tq) {
          int64_t* q = tq + 4 * (base + k);
          q[0] = B.s[k].t0.num; q[1] = B.s[k].t0.den; q[2] = B.s[k].t1.num; q[3] = B.s[k].t1.den;
        }
      }
    }
    free(B.s);
  }
  return err ? OC_ENOMEM : OC_OK;
}

/*
 * Per-ray statistics used by the learned level of detail, on the tree
 * truncated at C->max_level: for ray r, out[16 r + ...] =
 *   0: sum of v chord, 1: sum of chord, 2: sum of chord log10(v),
 *   3: sum of chord log10(v)^2, 4: 1 if the ray meets the box,
 *   5..14: chord summed by the deepest leaf level below each cell met,
 *          clamped to 7..16 (bin = level - 7),
 *   15: number of cells met.   (v = field `field`, fp32 stored values)
 */
int oc_probe_stats(const oc_tree* T, const oc_camera* C, int32_t field, const int64_t* ray_ids, int64_t nrays,
                   double* out, int32_t nthreads) {
  if (!T || !C || !ray_ids || !out || field < 0 || field >= T->nfields) return OC_EINVAL;
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    segbuf B = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrays; ++r) {
      int64_t o[3], d[3];
      double* q = out + 16 * r;
      for (int k = 0; k < 16; ++k) q[k] = 0.0;
      if (ray_segments(T, C, ray_ids[r], &B, o, d)) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      /* the ray meets the box iff its clip against the root is non-empty */
      segbuf R = {0, 0, 0};
      if (visit(T, 0, o, d, 0, &R) == 0 && R.n > 0) q[4] = 1.0;
      free(R.s);
      double ulen = unit_length(d);
      const float* vf = T->v32 + (int64_t)field * T->n;
      for (int64_t k = 0; k < B.n; ++k) {
        const double l = chord(&B.s[k], ulen);
        const double v = (double)vf[B.s[k].node];
        const double lg = log10(v > 1e-30 ? v : 1e-30);
        q[0] += v * l;
        q[1] += l;
        q[2] += l * lg;
        q[3] += l * lg * lg;
        int b = T->depth[B.s[k].node] - 7;
        if (b < 0) b = 0;
        if (b > 9) b = 9;
        q[5 + b] += l;
      }
      q[15] = (double)B.n;
    }
    free(B.s);
  }
  return err ? OC_ENOMEM : OC_OK;
}

/* The integer ray of a pixel, as the oracle builds it (for the tests). */
void oc_pixel_ray(const oc_camera* C, int64_t i, int64_t j, int64_t* o, int64_t* d) { pixel_ray(C, i, j, o, d); }

/*
 * Slice map (Sec. 3: the "Slicemap" tried on the GPU, a simple tree search):
 * the value of a field on a plane through the volume.  For an orthographic
 * record the point of pixel (i, j) is the origin of its ray, O + aU + bV (in
 * 2^-28 box units); out[r] is the stored fp32 value of field `field` of the
 * cell of the tree truncated at C->max_level that contains the point (cells
 * are half-open, so a point on a face belongs to the cell above it), found by
 * descending from the root one level at a time; NaN for points outside the
 * box.  ray_ids = pixel indices (NULL: all W*H).
 */
int oc_slice(const oc_tree* T, const oc_camera* C, int32_t field, const int64_t* ray_ids, int64_t nrays,
             float* out) {
  if (!T || !C || !out || C->kind != 1 || field < 0 || field >= T->nfields) return OC_EINVAL;
  int64_t total = ray_ids ? nrays : (int64_t)C->W * C->H;
  for (int64_t r = 0; r < total; ++r) {
    int64_t pix = ray_ids ? ray_ids[r] : r;
    int64_t p[3], d[3];
    pixel_ray(C, pix % C->W, pix / C->W, p, d);
    if (p[0] < 0 || p[1] < 0 || p[2] < 0 || p[0] >= FIX_ONE || p[1] >= FIX_ONE || p[2] >= FIX_ONE) {
      out[r] = NAN;
      continue;
    }
    int64_t cur = 0;
    while (T->nodes[cur].state == 2 && T->nodes[cur].level < C->max_level) {
      int sh = FIX_BITS - 1 - T->nodes[cur].level; /* bit of the point that picks the child */
      int c = (int)((p[0] >> sh) & 1) | (int)(((p[1] >> sh) & 1) << 1) | (int)(((p[2] >> sh) & 1) << 2);
      cur = T->nodes[cur].first_child + c;
    }
    out[r] = T->v32[(int64_t)field * T->n + cur];
  }
  return OC_OK;
}

/*
 * Local resolution of the image at each pixel, for the adaptive blur of
 * Sec. 2.2 (the filter size follows the local resolution of the image): the
 * chord-weighted mean, over the cells the pixel's ray meets in the truncated
 * tree, of the cell's side measured in pixels at the cell's depth.  A cell of
 * side 2^-l met between ray parameters t0 and t1 spans 2^-l / w(t) pixels,
 * with the pixel spacing w(t) = 2 |U| t 2^-28 at t = (t0 + t1)/2 for a
 * perspective record (neighbouring pixel rays differ by 2U in direction) and
 * w = 2 |U| 2^-28 for an orthographic one.  out[r] = sum(chord x 2^-l / w) /
 * sum(chord); 0 for rays that miss the box.  fp64 from the exact parameters.
 */
int oc_resolution(const oc_tree* T, const oc_camera* C, const int64_t* ray_ids, int64_t nrays, double* out,
                  int32_t nthreads) {
  if (!T || !C || !out) return OC_EINVAL;
  int64_t total = ray_ids ? nrays : (int64_t)C->W * C->H;
  const double U2 = (double)C->U[0] * (double)C->U[0] + (double)C->U[1] * (double)C->U[1] +
                    (double)C->U[2] * (double)C->U[2];
  const double w0 = 2.0 * sqrt(U2) * ldexp(1.0, -FIX_BITS);
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    segbuf B = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < total; ++r) {
      int64_t o[3], d[3];
      if (ray_segments(T, C, ray_ids ? ray_ids[r] : r, &B, o, d)) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      double ulen = unit_length(d);
      double num = 0.0, den = 0.0;
      for (int64_t k = 0; k < B.n; ++k) {
        const double l = chord(&B.s[k], ulen);
        const double side = ldexp(1.0, -T->nodes[B.s[k].node].level);
        double w = w0;
        if (C->kind == 0) {
          const double t0 = (double)B.s[k].t0.num / (double)B.s[k].t0.den;
          const double t1 = (double)B.s[k].t1.num / (double)B.s[k].t1.den;
          w = w0 * 0.5 * (t0 + t1);
        }
        num += l * side / w;
        den += l;
      }
      out[r] = den > 0.0 ? num / den : 0.0;
    }
    free(B.s);
  }
  return err ? OC_ENOMEM : OC_OK;
}
