// tree.cpp -- linear-octree builder, camera quantisation and the C ABI
// entry points that are not kernels.
//
// Builder (truncation and restriction, Sec. 2 of the paper; layout is this
// library's own):
//   1. validate the leaves (levels 0..24, coordinates in range, finite
//      fields);
//   2. key every leaf by the Morton code of its lowest corner at level 24
//      (72 bits) and sort (LSD radix, skipped when already sorted);
//   3. check that the sorted leaves tile [0, 2^72) contiguously: consecutive
//      aligned dyadic cubes without gap or overlap are exactly the leaf sets
//      of complete octrees;
//   4. emit every cell once, level by level in Morton order: walking the
//      leaves in Morton order, a leaf whose key is aligned to 8^(24-j) is the
//      first leaf below a new level-j ancestor; that ancestor's first child
//      is the next cell emitted at level j+1, so first-child indices come
//      from per-level cursors in a single pass;
//   5. restrict bottom-up in fp64 (children summed in order 0..7, divided by
//      8; weighted fields carried as weight x value), round once to fp32;
//   6. upload child / value / maxdepth arrays.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "internal.h"

namespace amr {

static thread_local std::string g_err = "no error";
static std::atomic<uint64_t> g_serial{1};

void set_error(const std::string& msg) { g_err = msg; }
amr_status fail(amr_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

CameraView camera_view(const amr_camera& c) {
  CameraView v;
  v.kind = c.kind;
  v.W = c.W;
  v.H = c.H;
  v.max_level = c.max_level;
  for (int k = 0; k < 3; ++k) {
    v.O[k] = c.O[k];
    v.F[k] = c.F[k];
    v.U[k] = c.U[k];
    v.V[k] = c.V[k];
  }
  return v;
}

namespace {

typedef unsigned __int128 u128;

inline uint64_t spread21(uint64_t x) {
  // 21-bit integer -> every third bit of a 63-bit word
  x &= 0x1fffffULL;
  x = (x | (x << 32)) & 0x1f00000000ffffULL;
  x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}

// Morton code of a level-l cell normalised to level 24 (72 bits).
inline u128 leaf_key(int l, uint32_t x, uint32_t y, uint32_t z) {
  const int sh = kMaxLevel - l;
  uint64_t X = (uint64_t)x << sh, Y = (uint64_t)y << sh, Z = (uint64_t)z << sh;  // 24-bit
  // low 12 bits of each -> 36-bit code, high 12 bits -> next 36 bits
  uint64_t lo = spread21(X & 0xfff) | (spread21(Y & 0xfff) << 1) | (spread21(Z & 0xfff) << 2);
  uint64_t hi = spread21(X >> 12) | (spread21(Y >> 12) << 1) | (spread21(Z >> 12) << 2);
  return ((u128)hi << 36) | (u128)lo;
}

struct Item {
  uint64_t lo;
  uint32_t hi;
  uint32_t idx;
};

void radix_sort(std::vector<Item>& a) {
  std::vector<Item> b(a.size());
  for (int pass = 0; pass < 9; ++pass) {
    size_t cnt[257] = {0};
    for (const Item& it : a) {
      unsigned byte = pass < 8 ? (unsigned)((it.lo >> (8 * pass)) & 0xff) : (unsigned)(it.hi & 0xff);
      cnt[byte + 1]++;
    }
    bool trivial = false;
    for (int v = 1; v <= 256; ++v)
      if (cnt[v] == a.size()) trivial = true;
    if (trivial) continue;
    for (int v = 0; v < 256; ++v) cnt[v + 1] += cnt[v];
    for (const Item& it : a) {
      unsigned byte = pass < 8 ? (unsigned)((it.lo >> (8 * pass)) & 0xff) : (unsigned)(it.hi & 0xff);
      b[cnt[byte]++] = it;
    }
    a.swap(b);
  }
}

template <class F>
void parallel_for(int64_t n, F&& fn) {
  int nt = (int)std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 64);
  if (n < 65536) nt = 1;
  if (nt == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    int64_t a = n * t / nt, b = n * (t + 1) / nt;
    th.emplace_back([&fn, a, b]() { fn(a, b); });
  }
  for (auto& t : th) t.join();
}

inline int ctz128(u128 k) {
  if (k == 0) return 128;
  uint64_t lo = (uint64_t)k;
  if (lo) return __builtin_ctzll(lo);
  return 64 + __builtin_ctzll((uint64_t)(k >> 64));
}

}  // namespace

}  // namespace amr

using namespace amr;

amr_status amr::check_render_common(const amr_tree* t, const amr_camera* cam) {
  if (!t || !cam) return fail(AMR_EINVAL, "null tree or camera");
  if (t->info.host_only) return fail(AMR_EINVAL, "host_only tree cannot be rendered");
  return check_camera(cam);
}

amr_status amr::check_camera(const amr_camera* cam) {
  if (!cam) return fail(AMR_EINVAL, "null camera");
  if (cam->W < 1 || cam->H < 1 || cam->W > 32768 || cam->H > 32768) return fail(AMR_EINVAL, "bad image size");
  if (cam->max_level < 0 || cam->max_level > kMaxLevel) return fail(AMR_EINVAL, "bad max_level");
  if (cam->kind != 0 && cam->kind != 1) return fail(AMR_EINVAL, "bad camera kind");
  // re-check the integer ranges the kernels rely on (records may be hand-made)
  const int64_t lim = int64_t(1) << 30;
  for (int k = 0; k < 3; ++k) {
    const int64_t span = (int64_t)(cam->W - 1) * std::llabs(cam->U[k]) + (int64_t)(cam->H - 1) * std::llabs(cam->V[k]);
    if (cam->O[k] < -lim || cam->O[k] >= lim) return fail(AMR_EINVAL, "camera origin out of range");
    if (cam->kind == 0) {
      if (std::llabs(cam->F[k]) + span >= lim) return fail(AMR_EINVAL, "camera direction out of range");
    } else {
      if (cam->O[k] - span < -lim || cam->O[k] + span >= lim) return fail(AMR_EINVAL, "camera origin out of range");
      if (std::llabs(cam->F[k]) >= lim) return fail(AMR_EINVAL, "camera direction out of range");
    }
  }
  if (cam->kind == 1 && cam->F[0] == 0 && cam->F[1] == 0 && cam->F[2] == 0)
    return fail(AMR_EINVAL, "zero direction");
  return AMR_OK;
}

extern "C" {

const char* amr_last_error(void) { return g_err.c_str(); }

amr_status amr_build_linear_octree(const amr_leaves* in, const amr_build_opts* opt, amr_stream s, amr_tree** out) {
  (void)s;
  if (!in || !out) return fail(AMR_EINVAL, "null argument");
  *out = nullptr;
  const int64_t n = in->n;
  if (n < 1) return fail(AMR_EINVAL, "no leaves");
  if (!in->level || !in->ix || !in->iy || !in->iz || !in->fields) return fail(AMR_EINVAL, "null leaf array");
  const int nf = in->nfields;
  if (nf < 1 || nf > 8) return fail(AMR_EINVAL, "nfields must be 1..8");
  if (in->field_stride < n) return fail(AMR_EINVAL, "field_stride < n");
  if (in->location != AMR_HOST && in->location != AMR_DEVICE) return fail(AMR_EINVAL, "bad location");
  int32_t rw[8];
  const bool defaults = !opt || opt->use_defaults;
  for (int f = 0; f < nf; ++f) rw[f] = defaults ? (f == 0 ? -1 : 0) : opt->restrict_weight[f];
  if (defaults && nf > 1) rw[0] = -1;
  for (int f = 0; f < nf; ++f) {
    if (rw[f] >= nf || rw[f] < -1 || rw[f] == f || (rw[f] >= 0 && rw[rw[f]] >= 0))
      return fail(AMR_EINVAL, "bad restrict_weight");
  }
  const bool host_only = opt && opt->host_only;

  // host views of the inputs
  std::vector<int32_t> hl, hx, hy, hz;
  std::vector<float> hf;
  const int32_t *L = in->level, *X = in->ix, *Y = in->iy, *Z = in->iz;
  const float* Fv = in->fields;
  if (in->location == AMR_DEVICE) {
    hl.resize(n); hx.resize(n); hy.resize(n); hz.resize(n);
    hf.resize((size_t)nf * in->field_stride);
    int e = dev_download(hl.data(), L, n * 4) | dev_download(hx.data(), X, n * 4) |
            dev_download(hy.data(), Y, n * 4) | dev_download(hz.data(), Z, n * 4) |
            dev_download(hf.data(), Fv, hf.size() * 4);
    if (e) return fail(AMR_EHIP, "download of device leaves failed");
    L = hl.data(); X = hx.data(); Y = hy.data(); Z = hz.data(); Fv = hf.data();
  }
  const int64_t fs = in->field_stride;

  // 1-2. validate, key, sort
  std::vector<Item> items;
  try {
    items.resize(n);
  } catch (...) {
    return fail(AMR_ENOMEM, "host allocation failed");
  }
  std::atomic<int> bad_level{0}, bad_coord{0}, bad_field{0};
  std::atomic<bool> sorted{true};
  parallel_for(n, [&](int64_t a, int64_t b) {
    u128 prev = 0;
    bool have = false;
    for (int64_t q = a; q < b; ++q) {
      int l = L[q];
      if (l < 0 || l > kMaxLevel) { bad_level = 1; continue; }
      int64_t side = int64_t(1) << l;
      if (X[q] < 0 || Y[q] < 0 || Z[q] < 0 || X[q] >= side || Y[q] >= side || Z[q] >= side) {
        bad_coord = 1;
        continue;
      }
      for (int f = 0; f < nf; ++f)
        if (!std::isfinite(Fv[f * fs + q])) bad_field = 1;
      u128 k = leaf_key(l, (uint32_t)X[q], (uint32_t)Y[q], (uint32_t)Z[q]);
      items[q].lo = (uint64_t)k;
      items[q].hi = (uint32_t)(k >> 64);
      items[q].idx = (uint32_t)q;
      if (have && k < prev) sorted = false;
      prev = k;
      have = true;
    }
  });
  if (bad_level) return fail(AMR_EINVAL, "leaf level outside 0..24");
  if (bad_coord) return fail(AMR_ETREE, "leaf coordinate outside 0..2^level-1");
  if (bad_field) return fail(AMR_EINVAL, "NaN or Inf field value");
  if (n > 1 && sorted) {
    // chunk boundaries
    int nt = (int)std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 64);
    if (n < 65536) nt = 1;
    for (int t = 1; t < nt; ++t) {
      int64_t q = n * t / nt;
      u128 a = ((u128)items[q - 1].hi << 64) | items[q - 1].lo, b = ((u128)items[q].hi << 64) | items[q].lo;
      if (b < a) sorted = false;
    }
  }
  if (!sorted) radix_sort(items);

  // 3. tiling check + per-level counts
  int64_t count[kMaxLevel + 1] = {0};
  int lmax = 0, lmin = kMaxLevel;
  {
    u128 pos = 0;
    for (int64_t r = 0; r < n; ++r) {
      const Item& it = items[r];
      const u128 k = ((u128)it.hi << 64) | it.lo;
      const int l = L[it.idx];
      if (k != pos)
        return fail(AMR_ETREE, k > pos ? "leaves leave a gap (incomplete octree)" : "leaves overlap or repeat");
      pos += (u128)1 << (3 * (kMaxLevel - l));
      const int tz = ctz128(k);
      int j0 = k == 0 ? 0 : std::max(0, kMaxLevel - tz / 3);
      for (int j = j0; j < l; ++j) count[j]++;
      count[l]++;
      lmax = std::max(lmax, l);
      lmin = std::min(lmin, l);
    }
    if (pos != ((u128)1 << (3 * kMaxLevel))) return fail(AMR_ETREE, "leaves do not cover the box");
  }
  int64_t off[kMaxLevel + 2];
  off[0] = 0;
  for (int l = 0; l <= kMaxLevel; ++l) off[l + 1] = off[l] + count[l];
  const int64_t ncells = off[kMaxLevel + 1];
  if (ncells >= (int64_t(1) << 31) - 16) return fail(AMR_ENOMEM, "more than 2^31 cells");

  // 4. emit cells level by level
  amr_tree* T = new (std::nothrow) amr_tree();
  if (!T) return fail(AMR_ENOMEM, "host allocation failed");
  std::vector<int32_t> child;
  std::vector<int64_t> leaf_src;  // input leaf of each cell, -1 for refined
  std::vector<double> v64;
  std::vector<uint8_t> md;
  try {
    child.resize(ncells);
    leaf_src.resize(ncells);
    v64.resize((size_t)nf * ncells);
    md.resize(ncells);
  } catch (...) {
    delete T;
    return fail(AMR_ENOMEM, "host allocation failed");
  }
  {
    int64_t cur[kMaxLevel + 2];
    for (int l = 0; l <= kMaxLevel + 1; ++l) cur[l] = off[l];
    for (int64_t r = 0; r < n; ++r) {
      const Item& it = items[r];
      const u128 k = ((u128)it.hi << 64) | it.lo;
      const int l = L[it.idx];
      const int tz = ctz128(k);
      int j0 = k == 0 ? 0 : std::max(0, kMaxLevel - tz / 3);
      for (int j = j0; j < l; ++j) {
        int64_t c = cur[j]++;
        child[c] = (int32_t)cur[j + 1];
        leaf_src[c] = -1;
      }
      int64_t c = cur[l]++;
      child[c] = -1;
      leaf_src[c] = it.idx;
    }
  }
  std::vector<Item>().swap(items);

  // 5. restriction, bottom-up, fp64
  for (int f = 0; f < nf; ++f) {
    double* vf = v64.data() + (size_t)f * ncells;
    const int w = rw[f];
    parallel_for(ncells, [&](int64_t a, int64_t b) {
      for (int64_t c = a; c < b; ++c) {
        if (leaf_src[c] < 0) continue;
        double v = (double)Fv[f * fs + leaf_src[c]];
        if (w >= 0) v *= (double)Fv[w * fs + leaf_src[c]];
        vf[c] = v;
      }
    });
  }
  for (int64_t c = off[kMaxLevel]; c < off[kMaxLevel + 1]; ++c) md[c] = (uint8_t)kMaxLevel;
  for (int l = kMaxLevel - 1; l >= 0; --l) {
    if (count[l] == 0) continue;
    parallel_for(count[l], [&](int64_t a, int64_t b) {
      for (int64_t c = off[l] + a; c < off[l] + b; ++c) {
        const int32_t c0 = child[c];
        if (c0 < 0) {
          md[c] = (uint8_t)l;
          continue;
        }
        uint8_t m = 0;
        for (int k = 0; k < 8; ++k) m = std::max(m, md[c0 + k]);
        md[c] = m;
        for (int f = 0; f < nf; ++f) {
          const double* vf = v64.data() + (size_t)f * ncells;
          double s = 0.0;
          for (int k = 0; k < 8; ++k) s += vf[c0 + k];
          v64[(size_t)f * ncells + c] = s / 8.0;
        }
      }
    });
  }
  std::vector<float> v32((size_t)nf * ncells);
  for (int f = 0; f < nf; ++f) {
    const int w = rw[f];
    const double* vf = v64.data() + (size_t)f * ncells;
    const double* vw = w >= 0 ? v64.data() + (size_t)w * ncells : nullptr;
    float* of = v32.data() + (size_t)f * ncells;
    parallel_for(ncells, [&](int64_t a, int64_t b) {
      for (int64_t c = a; c < b; ++c) {
        double v;
        if (w < 0)
          v = vf[c];
        else if (leaf_src[c] >= 0)
          v = (double)Fv[f * fs + leaf_src[c]];
        else
          v = vw[c] != 0.0 ? vf[c] / vw[c] : 0.0;
        of[c] = (float)v;
      }
    });
  }
  std::vector<double>().swap(v64);
  std::vector<int64_t>().swap(leaf_src);
  std::vector<ChildVal> cv(ncells);
  parallel_for(ncells, [&](int64_t a, int64_t b) {
    for (int64_t c = a; c < b; ++c) cv[c] = ChildVal{child[c], v32[c]};
  });
  std::vector<Cell4> packed;
  if (nf >= 4) {
    packed.resize(ncells);
    parallel_for(ncells, [&](int64_t a, int64_t b) {
      for (int64_t c = a; c < b; ++c)
        packed[c] = Cell4{v32[c], v32[(size_t)ncells + c], v32[2 * (size_t)ncells + c], v32[3 * (size_t)ncells + c]};
    });
  }

  // 6. info + upload
  amr_tree_info_t& I = T->info;
  std::memset(&I, 0, sizeof(I));
  I.ncells = ncells;
  I.nleaves = n;
  I.nfields = nf;
  I.lmax = lmax;
  I.levelmin = lmin;
  I.host_only = host_only ? 1 : 0;
  for (int l = 0; l <= kMaxLevel; ++l) I.cells_per_level[l] = count[l];
  for (int l = 0; l <= kMaxLevel + 1; ++l) I.level_offset[l] = off[l];
  I.device_bytes = host_only ? 0 : ncells * (int64_t)(4 + 4 * nf + 1 + 8) + (int64_t)packed.size() * 16;
  TreeView& V = T->view;
  std::memset(&V, 0, sizeof(V));
  V.ncells = ncells;
  V.nfields = nf;
  V.base = std::min(lmin, kMaxArithBase);
  V.lmax = lmax;
  for (int l = 0; l <= kMaxLevel + 1; ++l) V.off[l] = (int32_t)off[l];
  T->serial = g_serial.fetch_add(1);
  register_tree(T->serial);
  if (host_only) {
    T->h_child.swap(child);
    T->h_val.swap(v32);
    T->h_maxdepth.swap(md);
    T->h_packed.swap(packed);
    T->h_cv.swap(cv);
    V.cv = (const ChildVal AMR_GLOBAL*)T->h_cv.data();
    V.child = (const int32_t AMR_GLOBAL*)T->h_child.data();
    V.val = (const float AMR_GLOBAL*)T->h_val.data();
    V.maxdepth = (const uint8_t AMR_GLOBAL*)T->h_maxdepth.data();
    V.packed = T->h_packed.empty() ? nullptr : (const Cell4 AMR_GLOBAL*)T->h_packed.data();
  } else {
    int e = dev_malloc((void**)&T->d_child, ncells * 4);
    if (!e) e = dev_malloc((void**)&T->d_val, (size_t)nf * ncells * 4);
    if (!e) e = dev_malloc((void**)&T->d_maxdepth, ncells + 64);
    if (!e && !packed.empty()) e = dev_malloc((void**)&T->d_packed, packed.size() * sizeof(Cell4));
    if (!e) e = dev_malloc((void**)&T->d_cv, cv.size() * sizeof(ChildVal));
    if (e) {
      amr_tree_free(T);
      return fail(AMR_ENOMEM, std::string("device allocation failed: ") + dev_error_string(e));
    }
    e = dev_upload(T->d_child, child.data(), ncells * 4);
    if (!e) e = dev_upload(T->d_val, v32.data(), (size_t)nf * ncells * 4);
    if (!e) e = dev_upload(T->d_maxdepth, md.data(), ncells);
    if (!e && !packed.empty()) e = dev_upload(T->d_packed, packed.data(), packed.size() * sizeof(Cell4));
    if (!e) e = dev_upload(T->d_cv, cv.data(), cv.size() * sizeof(ChildVal));
    if (e) {
      amr_tree_free(T);
      return fail(AMR_EHIP, std::string("upload failed: ") + dev_error_string(e));
    }
    V.child = (const int32_t AMR_GLOBAL*)T->d_child;
    V.val = (const float AMR_GLOBAL*)T->d_val;
    V.maxdepth = (const uint8_t AMR_GLOBAL*)T->d_maxdepth;
    V.packed = (const Cell4 AMR_GLOBAL*)T->d_packed;
    V.cv = (const ChildVal AMR_GLOBAL*)T->d_cv;
  }
  *out = T;
  return AMR_OK;
}

void amr_tree_free(amr_tree* t) {
  if (!t) return;
  unregister_tree(t->serial);
  if (t->d_child) dev_free(t->d_child);
  if (t->d_val) dev_free(t->d_val);
  if (t->d_packed) dev_free(t->d_packed);
  if (t->d_cv) dev_free(t->d_cv);
  if (t->d_maxdepth) dev_free(t->d_maxdepth);
  delete t;
}

amr_status amr_tree_info(const amr_tree* t, amr_tree_info_t* info) {
  if (!t || !info) return fail(AMR_EINVAL, "null argument");
  *info = t->info;
  return AMR_OK;
}

amr_status amr_tree_arrays(const amr_tree* t, const int32_t** child, const float** values, const uint8_t** maxdepth) {
  if (!t) return fail(AMR_EINVAL, "null tree");
  if (child) *child = t->view.child;
  if (values) *values = t->view.val;
  if (maxdepth) *maxdepth = t->view.maxdepth;
  return AMR_OK;
}

// Camera quantisation: the exact formula documented in amr.h.  Built with
// -ffp-contract=off so no product or difference is fused.
amr_status amr_set_camera(const amr_camera_desc* d, const amr_tree* t, amr_camera* out) {
  if (!d || !out) return fail(AMR_EINVAL, "null argument");
  if (d->kind != 0 && d->kind != 1) return fail(AMR_EINVAL, "camera kind must be 0 (persp) or 1 (ortho)");
  if (d->W < 1 || d->H < 1 || d->W > 32768 || d->H > 32768) return fail(AMR_EINVAL, "W, H must be 1..32768");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(d->eye[k]) || !std::isfinite(d->target[k]) || !std::isfinite(d->up[k]))
      return fail(AMR_EINVAL, "non-finite camera vector");
  double f[3], fh[3], r[3], rh[3], uh[3];
  for (int k = 0; k < 3; ++k) f[k] = d->target[k] - d->eye[k];
  const double nf = std::sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
  if (!(nf > 0.0) || !std::isfinite(nf)) return fail(AMR_EINVAL, "eye == target");
  for (int k = 0; k < 3; ++k) fh[k] = f[k] / nf;
  r[0] = d->up[1] * fh[2] - d->up[2] * fh[1];
  r[1] = d->up[2] * fh[0] - d->up[0] * fh[2];
  r[2] = d->up[0] * fh[1] - d->up[1] * fh[0];
  const double nr = std::sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
  if (!(nr > 0.0) || !std::isfinite(nr)) return fail(AMR_EINVAL, "up is parallel to the view direction");
  for (int k = 0; k < 3; ++k) rh[k] = r[k] / nr;
  uh[0] = fh[1] * rh[2] - fh[2] * rh[1];
  uh[1] = fh[2] * rh[0] - fh[0] * rh[2];
  uh[2] = fh[0] * rh[1] - fh[1] * rh[0];
  double sc, foot;
  if (d->kind == 0) {
    if (!(d->fov_y > 0.0) || !(d->fov_y < 3.0)) return fail(AMR_EINVAL, "fov_y out of range");
    const double th = std::tan(0.5 * d->fov_y);
    sc = th / (double)d->H;
    foot = 2.0 * nf * th / (double)d->H;
  } else {
    if (!(d->ortho_height > 0.0) || !std::isfinite(d->ortho_height)) return fail(AMR_EINVAL, "ortho_height <= 0");
    sc = d->ortho_height / (2.0 * (double)d->H);
    foot = d->ortho_height / (double)d->H;
  }
  amr_camera c;
  c.kind = d->kind;
  c.W = d->W;
  c.H = d->H;
  auto q = [](double x) { return (int64_t)std::llrint(std::ldexp(x, kFix)); };
  for (int k = 0; k < 3; ++k) {
    c.O[k] = q(d->eye[k]);
    c.F[k] = q(fh[k]);
    c.U[k] = q(rh[k] * sc);
    c.V[k] = q(uh[k] * sc);
  }
  const int64_t lim = int64_t(1) << 30;
  for (int k = 0; k < 3; ++k) {
    const int64_t span = (int64_t)(d->W - 1) * std::llabs(c.U[k]) + (int64_t)(d->H - 1) * std::llabs(c.V[k]);
    if (c.O[k] < -lim || c.O[k] >= lim) return fail(AMR_EINVAL, "eye outside [-4, 4) box");
    if (d->kind == 0) {
      if (std::llabs(c.F[k]) + span >= lim) return fail(AMR_EINVAL, "field of view too wide for the ray range");
    } else {
      if (c.O[k] - span < -lim || c.O[k] + span >= lim) return fail(AMR_EINVAL, "image plane outside [-4, 4) box");
      if (std::llabs(c.F[k]) >= lim) return fail(AMR_EINVAL, "direction out of range");
    }
  }
  int32_t lv;
  if (d->max_level >= 0) {
    if (d->max_level > kMaxLevel) return fail(AMR_EINVAL, "max_level > 24");
    lv = d->max_level;
  } else {
    lv = 0;
    while (lv < 64 && std::ldexp(1.0, -lv) > foot) ++lv;
    lv += d->level_bias;
    lv = std::max(0, std::min(lv, kMaxLevel));
    if (t) lv = std::min(lv, t->info.lmax);
  }
  c.max_level = lv;
  *out = c;
  return AMR_OK;
}

amr_status amr_render(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_render_opts* opts, float* out,
                      float* aux, amr_stream s) {
  amr_status st = check_render_common(t, cam);
  if (st) return st;
  if (!out) return fail(AMR_EINVAL, "null output");
  if (((uintptr_t)out & 3) || ((uintptr_t)aux & 3)) return fail(AMR_EINVAL, "misaligned output");
  if (op != AMR_SUM && op != AMR_MAX && op != AMR_WMEAN) return fail(AMR_EINVAL, "bad op");
  amr_render_opts o = opts ? *opts : amr_render_opts{0, 0, 0, -1};
  const int nf = t->info.nfields;
  if (o.field < 0 || o.field + ((op == AMR_WMEAN && o.los_velocity) ? 2 : 0) >= nf)
    return fail(AMR_EINVAL, "field index out of range");
  if (op == AMR_WMEAN && (o.weight_field < 0 || o.weight_field >= nf)) return fail(AMR_EINVAL, "bad weight field");
  // untuned: the default variant, or for a maximum level 10 or more levels
  // below the complete base level (most moves re-descend several levels) the
  // walk with an ancestor stack, which shortens those re-descents (deep zoom,
  // 11 levels: 34.9 ms against 39.8 ms stackless and 62.8 ms split)
  const int b0 = std::min(t->view.base, cam->max_level);
  int untuned = default_variant();
  if (cam->max_level - b0 >= kDeepSpan)
    for (int k = 0; k < variant_count(); ++k)
      if (std::strcmp(variant_name(k), "p8x8_w4_fastlds") == 0) untuned = k;
  int v = o.variant >= 0 ? o.variant : (t->tuned_variant[op] >= 0 ? t->tuned_variant[op] : untuned);
  if (v >= variant_count()) return fail(AMR_EINVAL, "bad variant");
  RenderArgs a;
  a.t = t->view;
  a.c = camera_view(*cam);
  a.field = o.field;
  a.wfield = o.weight_field;
  a.los = op == AMR_WMEAN ? (o.los_velocity ? 1 : 0) : 0;
  a.max_level = cam->max_level;
  a.out = out;
  a.aux = aux;
  const int pw = variant_packet_width(v), ph = 64 / pw;
  a.packets_x = (cam->W + pw - 1) / pw;
  a.packets_y = (cam->H + ph - 1) / ph;
  int e = launch_render((int)op, v, a, s);
  if (e) return fail(AMR_EHIP, std::string("render launch failed: ") + dev_error_string(e));
  return AMR_OK;
}

int32_t amr_variant_count(void) { return variant_count(); }
int32_t amr_variant_default(void) { return default_variant(); }
const char* amr_variant_name(int32_t v) { return (v >= 0 && v < variant_count()) ? variant_name(v) : "invalid"; }

amr_status amr_count_segments(const amr_tree* t, const amr_camera* cam, int32_t* counts, int64_t* total,
                              amr_stream s) {
  amr_status st = check_render_common(t, cam);
  if (st) return st;
  if (!total) return fail(AMR_EINVAL, "null total");
  if (((uintptr_t)total & 7) || ((uintptr_t)counts & 3)) return fail(AMR_EINVAL, "misaligned output");
  int e = launch_count_all(t->view, camera_view(*cam), counts, total, s);
  if (e) return fail(AMR_EHIP, std::string("count launch failed: ") + dev_error_string(e));
  return AMR_OK;
}

amr_status amr_mark_cells(const amr_tree* t, const amr_camera* cam, uint32_t* bitmap, int64_t* distinct,
                          amr_stream s) {
  amr_status st = check_render_common(t, cam);
  if (st) return st;
  if (!bitmap || !distinct) return fail(AMR_EINVAL, "null argument");
  if (((uintptr_t)bitmap & 3) || ((uintptr_t)distinct & 7)) return fail(AMR_EINVAL, "misaligned output");
  int e = launch_mark(t->view, camera_view(*cam), bitmap, distinct, s);
  if (e) return fail(AMR_EHIP, std::string("mark launch failed: ") + dev_error_string(e));
  return AMR_OK;
}

amr_status amr_trace_rays(const amr_tree* t, const amr_camera* cam, const int64_t* ray_ids, int64_t n,
                          const int64_t* offsets, int32_t* cells, amr_stream s) {
  amr_status st = check_render_common(t, cam);
  if (st) return st;
  if (n < 0 || (n > 0 && (!ray_ids || !offsets || !cells))) return fail(AMR_EINVAL, "null argument");
  if (n == 0) return AMR_OK;
  int e = launch_rays(t->view, camera_view(*cam), ray_ids, n, offsets, cells, nullptr, s);
  if (e) return fail(AMR_EHIP, std::string("trace launch failed: ") + dev_error_string(e));
  return AMR_OK;
}

amr_status amr_count_rays(const amr_tree* t, const amr_camera* cam, const int64_t* ray_ids, int64_t n,
                          int32_t* counts, amr_stream s) {
  amr_status st = check_render_common(t, cam);
  if (st) return st;
  if (n < 0 || (n > 0 && (!ray_ids || !counts))) return fail(AMR_EINVAL, "null argument");
  if (n == 0) return AMR_OK;
  int e = launch_rays(t->view, camera_view(*cam), ray_ids, n, nullptr, nullptr, counts, s);
  if (e) return fail(AMR_EHIP, std::string("count launch failed: ") + dev_error_string(e));
  return AMR_OK;
}

}  // extern "C"
