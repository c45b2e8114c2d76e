// CPU build of the library's per-ray traversal core (traverse.h), for tests
// only: it runs the exact code the HIP kernels run, on host memory, so that
// indexing, termination and exactness are checked on the CPU.  It is not part
// of the product and is never loaded by it.
#include <cstdint>
#include <thread>
#include <vector>

#include "../../paper_1210_8014_amd/csrc/traverse.h"

using namespace amr;

// The (first child, field 0) records the fast walk reads, rebuilt from the
// host arrays for each emulator call (calls come from one thread; the
// worker threads of a call only read them).
static const ChildVal* child_val(const int32_t* child, const float* val, int64_t ncells) {
  static std::vector<ChildVal> cv;
  cv.resize(ncells);
  for (int64_t c = 0; c < ncells; ++c) cv[c] = ChildVal{child[c], val[c]};
  return cv.data();
}

static TreeView make_tree(const int32_t* child, const float* val, int64_t ncells, int32_t nfields, int32_t base,
                          int32_t lmax, const int32_t* off) {
  TreeView T{};
  T.cv = child_val(child, val, ncells);
  T.child = child;
  T.val = val;
  T.maxdepth = nullptr;
  T.ncells = ncells;
  T.nfields = nfields;
  T.base = base;
  T.lmax = lmax;
  for (int l = 0; l < kMaxLevel + 2; ++l) T.off[l] = off[l];
  return T;
}

static CameraView make_cam(const int32_t* k4, const int64_t* ofuv) {
  CameraView C{};
  C.kind = k4[0];
  C.W = k4[1];
  C.H = k4[2];
  C.max_level = k4[3];
  for (int k = 0; k < 3; ++k) {
    C.O[k] = ofuv[k];
    C.F[k] = ofuv[3 + k];
    C.U[k] = ofuv[6 + k];
    C.V[k] = ofuv[9 + k];
  }
  return C;
}

template <class F>
static void par(int64_t n, F fn) {
  int nt = std::max(1u, std::thread::hardware_concurrency());
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([=]() {
      for (int64_t r = n * t / nt; r < n * (t + 1) / nt; ++r) fn(r);
    });
  for (auto& t : th) t.join();
}

extern "C" {

// pix: pixel ids (j*W + i); out/aux/counts indexed like pix.
int emu_render(const int32_t* child, const float* val, int64_t ncells, int32_t nfields, int32_t base, int32_t lmax,
               const int32_t* off, const int32_t* cam4, const int64_t* ofuv, int32_t op, int32_t field,
               int32_t wfield, int32_t los, int32_t max_level, const int64_t* pix, int64_t n, float* out, float* aux,
               int32_t* counts, int32_t lca) {
  const TreeView T = make_tree(child, val, ncells, nfields, base, lmax, off);
  const CameraView C = make_cam(cam4, ofuv);
  par(n, [&](int64_t r) {
    const int i = (int)(pix[r] % C.W), j = (int)(pix[r] / C.W);
    float o = 0.0f, x = 0.0f;
    LocalStack S;
    for (int l = 0; l <= kMaxLevel; ++l) S.w[l] = -7;  // poison: a stale read shows up as a bad index
    if (lca == 1) {
      if (op == 0) render_pixel<kOpSum, kWalkStack>(T, C, field, wfield, los, max_level, i, j, o, x, S);
      else if (op == 1) render_pixel<kOpMax, kWalkStack>(T, C, field, wfield, los, max_level, i, j, o, x, S);
      else render_pixel<kOpWMean, kWalkStack>(T, C, field, wfield, los, max_level, i, j, o, x, S);
    } else if (lca == 3) {
      if (op == 0) render_pixel<kOpSum, kWalkFastStack>(T, C, field, wfield, los, max_level, i, j, o, x, S);
      else if (op == 1) render_pixel<kOpMax, kWalkFastStack>(T, C, field, wfield, los, max_level, i, j, o, x, S);
      else render_pixel<kOpWMean, kWalkFastStack>(T, C, field, wfield, los, max_level, i, j, o, x, S);
    } else if (lca == 2) {
      if (op == 0) render_pixel<kOpSum, kWalkFast>(T, C, field, wfield, los, max_level, i, j, o, x, S);
      else if (op == 1) render_pixel<kOpMax, kWalkFast>(T, C, field, wfield, los, max_level, i, j, o, x, S);
      else render_pixel<kOpWMean, kWalkFast>(T, C, field, wfield, los, max_level, i, j, o, x, S);
    } else {
      if (op == 0) render_pixel<kOpSum, kWalkBase>(T, C, field, wfield, los, max_level, i, j, o, x, S);
      else if (op == 1) render_pixel<kOpMax, kWalkBase>(T, C, field, wfield, los, max_level, i, j, o, x, S);
      else render_pixel<kOpWMean, kWalkBase>(T, C, field, wfield, los, max_level, i, j, o, x, S);
    }
    if (out) out[r] = o;
    if (aux) aux[r] = x;
    if (counts) counts[r] = trace_pixel(T, C, max_level, i, j, nullptr, 0);
  });
  return 0;
}

// offsets[n+1] must hold the prefix sum of the counts.
int emu_trace(const int32_t* child, const float* val, int64_t ncells, int32_t nfields, int32_t base, int32_t lmax,
              const int32_t* off, const int32_t* cam4, const int64_t* ofuv, int32_t max_level, const int64_t* pix,
              int64_t n, const int64_t* offsets, int32_t* cells) {
  const TreeView T = make_tree(child, val, ncells, nfields, base, lmax, off);
  const CameraView C = make_cam(cam4, ofuv);
  par(n, [&](int64_t r) {
    const int i = (int)(pix[r] % C.W), j = (int)(pix[r] / C.W);
    trace_pixel(T, C, max_level, i, j, cells + 4 * offsets[r], offsets[r + 1] - offsets[r]);
  });
  return 0;
}
}

// Split rays: the K spans of each ray walked one after another and merged in
// span order exactly as k_render_split merges its waves.  counts: cells per
// ray summed over the spans.  With cells != NULL, also writes the cells of
// the spans concatenated (offsets from the counts).
// Equal-slab spans (span_setup), K of them.
template <int OP>
static void split_pixel(const TreeView& T, const CameraView& C, int field, int wfield, int los, int max_level, int i,
                        int j, int K, float& o, float& x, int32_t& count, int32_t* cells) {
  const int b0 = T.base < max_level ? T.base : max_level;
  Partial P;
  partial_init<OP>(P);
  count = 0;
  for (int w = 0; w < K; ++w) {
    Partial Q;
    partial_init<OP>(Q);
    Ray R;
    Entry E;
    if (setup_ray(C, i, j, R, E) && span_setup(R, E, b0, K, w)) {
      const Entry E0 = E;
      walk_span<OP>(T, R, E, max_level, field, wfield, los, Q);
      E = E0;
      CountVis cv;
      const int32_t m = walk_fast(T, R, E, max_level, cv);
      if (cells) {
        TraceVis tv;
        tv.out = cells + 4 * (int64_t)count;
        for (int k = 0; k < 3; ++k) tv.flip_bits[k] = R.flip[k] ? 1 : 0;
        E = E0;
        walk_fast(T, R, E, max_level, tv);
      }
      count += m;
    }
    if (w == 0)
      P = Q;
    else
      partial_merge<OP>(P, Q);
  }
  o = 0.0f;
  x = 0.0f;
  partial_finish<OP>(P, o, x);
}

extern "C" int emu_render_split(const int32_t* child, const float* val, int64_t ncells, int32_t nfields, int32_t base,
                                int32_t lmax, const int32_t* off, const int32_t* cam4, const int64_t* ofuv, int32_t op,
                                int32_t field, int32_t wfield, int32_t los, int32_t max_level, const int64_t* pix,
                                int64_t n, float* out, float* aux, int32_t* counts, const int64_t* offsets,
                                int32_t* cells, int32_t K) {
  const TreeView T = make_tree(child, val, ncells, nfields, base, lmax, off);
  const CameraView C = make_cam(cam4, ofuv);
  par(n, [&](int64_t r) {
    const int i = (int)(pix[r] % C.W), j = (int)(pix[r] / C.W);
    float o, x;
    int32_t m;
    int32_t* cc = cells ? cells + 4 * offsets[r] : nullptr;
    if (op == 0) split_pixel<kOpSum>(T, C, field, wfield, los, max_level, i, j, K, o, x, m, cc);
    else if (op == 1) split_pixel<kOpMax>(T, C, field, wfield, los, max_level, i, j, K, o, x, m, cc);
    else split_pixel<kOpWMean>(T, C, field, wfield, los, max_level, i, j, K, o, x, m, cc);
    if (out) out[r] = o;
    if (aux) aux[r] = x;
    if (counts) counts[r] = m;
  });
  return 0;
}

// The learned-LOD tile walk: two spans per ray at level L, recording whether
// any span cut a cell (a cell with children at which the descent stopped).
template <int OP>
static void cut_pixel(const TreeView& T, const CameraView& C, int field, int wfield, int los, int L, int i, int j,
                      float& o, float& x, int32_t& cut) {
  const int b0 = T.base < L ? T.base : L;
  Partial P;
  partial_init<OP>(P);
  bool any = false;
  for (int w = 0; w < 2; ++w) {
    Partial Q;
    partial_init<OP>(Q);
    Ray R;
    Entry E;
    bool c = false;
    if (setup_ray(C, i, j, R, E) && span_setup(R, E, b0, 2, w)) {
      if (w == 1)
        walk_span<OP, true, true>(T, R, E, L, field, wfield, los, Q, &c);
      else
        walk_span<OP, false, true>(T, R, E, L, field, wfield, los, Q, &c);
    }
    any = any || c;
    if (w == 0)
      P = Q;
    else
      partial_merge<OP>(P, Q);
  }
  o = 0.0f;
  x = 0.0f;
  partial_finish<OP>(P, o, x);
  cut = any ? 1 : 0;
}

extern "C" int emu_render_cut(const int32_t* child, const float* val, int64_t ncells, int32_t nfields, int32_t base,
                              int32_t lmax, const int32_t* off, const int32_t* cam4, const int64_t* ofuv, int32_t op,
                              int32_t field, int32_t wfield, int32_t los, int32_t level, const int64_t* pix, int64_t n,
                              float* out, float* aux, int32_t* cut) {
  const TreeView T = make_tree(child, val, ncells, nfields, base, lmax, off);
  const CameraView C = make_cam(cam4, ofuv);
  par(n, [&](int64_t r) {
    const int i = (int)(pix[r] % C.W), j = (int)(pix[r] / C.W);
    float o, x;
    int32_t c;
    if (op == 0) cut_pixel<kOpSum>(T, C, field, wfield, los, level, i, j, o, x, c);
    else if (op == 1) cut_pixel<kOpMax>(T, C, field, wfield, los, level, i, j, o, x, c);
    else cut_pixel<kOpWMean>(T, C, field, wfield, los, level, i, j, o, x, c);
    out[r] = o;
    aux[r] = x;
    cut[r] = c;
  });
  return 0;
}

// The exact quotient helper of the ray set-up, for its own test.
extern "C" void emu_div_q28(const int64_t* num, const int32_t* d, int32_t* q, int64_t n) {
  for (int64_t r = 0; r < n; ++r) q[r] = div_q28(num[r], d[r]);
}

// One chunk of the streamed render (the library's plan arrays: 8-byte
// records with chunk-local first-child indices, fields [nfields][ncells],
// interleaved records or null, local level offsets): every ray of pix is
// clipped to the chunk's cube and its piece walked as the streamed kernel
// walks it, the partial merged into acc (4 floats per ray).  counts[r] is
// increased by the piece's cells; entry[2r..] receives the piece's entry
// parameter (numerator, denominator) or (0, 0) without a piece; with
// offsets, the piece's cells go to cells + 4 offsets[r].
template <int OP, bool kStd>
static void chunk_pixel(const TreeView& T, const CameraView& C, int field, int wfield, int los, int ml, int lc,
                        int cx, int cy, int cz, int i, int j, float* acc, int32_t* count, int64_t* entry,
                        int32_t* cells) {
  Ray R;
  Entry E;
  entry[0] = entry[1] = 0;
  if (!setup_ray(C, i, j, R, E) || !cube_clip(R, E, lc, cx, cy, cz)) return;
  entry[0] = E.en;
  entry[1] = E.da;
  const Entry E0 = E;
  Partial P;
  partial_init<OP>(P);
  walk_span<OP, false, false, kStd>(T, R, E, ml, field, wfield, los, P);
  Partial A{acc[0], acc[1], acc[2], acc[3]};
  partial_merge<OP>(A, P);
  acc[0] = A.s0;
  acc[1] = A.c0;
  acc[2] = A.s1;
  acc[3] = A.c1;
  CountVis cv;
  E = E0;
  *count += walk_fast<CountVis>(T, R, E, ml, cv);
  if (cells) {
    TraceVis tv;
    tv.out = cells;
    for (int k = 0; k < 3; ++k) tv.flip_bits[k] = R.flip[k] ? 1 : 0;
    E = E0;
    walk_fast<TraceVis>(T, R, E, ml, tv);
  }
}

extern "C" int emu_stream_chunk(const int32_t* records, const float* values, const float* packed, int64_t ncells,
                                int32_t nfields, int32_t base, int32_t lmax, const int32_t* off_local, int32_t lc,
                                int32_t cx, int32_t cy, int32_t cz, const int32_t* cam4, const int64_t* ofuv,
                                int32_t op, int32_t field, int32_t wfield, int32_t los, int32_t max_level,
                                const int64_t* pix, int64_t n, float* acc, int32_t* counts, int64_t* entry,
                                const int64_t* offsets, int32_t* cells) {
  TreeView T{};
  T.cv = (const ChildVal*)records;
  T.child = nullptr;
  T.val = values;
  T.ncells = ncells;
  T.nfields = nfields;
  T.base = base;
  T.lmax = lmax;
  for (int l = 0; l < kMaxLevel + 2; ++l) T.off[l] = off_local[l];
  const bool pk = op == kOpWMean && los && wfield == 0 && field == 1 && packed;
  T.packed = pk ? (const Cell4*)packed : nullptr;
  const CameraView C = make_cam(cam4, ofuv);
  const bool sw = std_walk(op, T, field, wfield, los, max_level);
  par(n, [&](int64_t r) {
    const int i = (int)(pix[r] % C.W), j = (int)(pix[r] / C.W);
    float* a = acc + 4 * r;
    int32_t* cc = cells ? cells + 4 * offsets[r] : nullptr;
    int64_t* en = entry + 2 * r;
#define AMR_EMU_CHUNK(OPV, S) \
  chunk_pixel<OPV, S>(T, C, field, wfield, los, max_level, lc, cx, cy, cz, i, j, a, counts + r, en, cc)
    if (op == 0) sw ? AMR_EMU_CHUNK(kOpSum, true) : AMR_EMU_CHUNK(kOpSum, false);
    else if (op == 1) sw ? AMR_EMU_CHUNK(kOpMax, true) : AMR_EMU_CHUNK(kOpMax, false);
    else sw ? AMR_EMU_CHUNK(kOpWMean, true) : AMR_EMU_CHUNK(kOpWMean, false);
#undef AMR_EMU_CHUNK
  });
  return 0;
}

// Final values of streamed partials (acc: 4 floats per ray).
extern "C" void emu_stream_finish(int32_t op, const float* acc, int64_t n, float* out, float* aux) {
  for (int64_t r = 0; r < n; ++r) {
    const Partial P{acc[4 * r], acc[4 * r + 1], acc[4 * r + 2], acc[4 * r + 3]};
    float o = 0.0f, x = 0.0f;
    if (op == 0) partial_finish<kOpSum>(P, o, x);
    else if (op == 1) partial_finish<kOpMax>(P, o, x);
    else partial_finish<kOpWMean>(P, o, x);
    out[r] = o;
    aux[r] = x;
  }
}
