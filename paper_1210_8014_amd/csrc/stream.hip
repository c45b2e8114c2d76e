// stream.hip -- rendering a tree kept in host memory, for trees larger than
// the GPU's memory.  The paper finds that reading the data dominates the
// cost of a render (Sec. 3) and that reading every cell is never required,
// since the camera bounds the depth (Sec. 2); accumulation along a ray may
// take any order (Sec. 2.2).  So the tree is cut into chunks: each chunk is
// the complete subtree under one cell of a level no deeper than the
// tree's complete base level (a cube of the box), stored with chunk-local
// indices in pinned host memory.  A render streams the chunks that the
// camera sees, only their levels down to the camera's maximum level, through
// a few device buffers on a copy stream, while two compute streams take the
// copied chunks in turn, walk every ray's part inside the chunk's cube and
// add it to per-pixel Kahan partials (the maximum for MAX), one plane of
// partials per compute stream, merged at the end.  Each cell lies in exactly one cube
// and is decided exactly as on the whole ray, so MAX is bit-identical to
// the in-memory render and SUM / WMEAN differ from it by rounding only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace amr;

namespace {

struct Chunk {
  int32_t level, ix, iy, iz;
  int64_t first;   // index of the chunk's first cell in the plan's host arrays
  int64_t ncells;  // cells of the subtree at levels >= level
  int64_t level_start[kMaxLevel + 2];  // local index of each level's first cell (levels below `level`: 0)
  int32_t off_local[kMaxLevel + 2];    // levels level..base: local index of Morton code 0 of that level
};

constexpr int64_t kAlign = 256;
constexpr int kMaxBuffers = 8;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <class F>
void parallel_items(int64_t n, F&& fn) {
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(n, std::min(64u, std::max(1u, std::thread::hardware_concurrency()))));
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int64_t i; (i = next.fetch_add(1)) < n;) fn(i);
    });
  for (auto& t : th) t.join();
}

uint32_t compact3(uint32_t x) {
  x &= 0x09249249u;
  x = (x | (x >> 2)) & 0x030C30C3u;
  x = (x | (x >> 4)) & 0x0300F00Fu;
  x = (x | (x >> 8)) & 0x030000FFu;
  x = (x | (x >> 16)) & 0x000003FFu;
  return x;
}

}  // namespace

struct amr_stream_plan {
  amr_tree_info_t info{};
  int32_t base = 0, lmax = 0, nfields = 0;
  int32_t max_chunk_level = 0, min_chunk_level = 0;
  int32_t host_only = 0;
  int64_t cap = 0, total = 0;
  std::vector<Chunk> chunks;
  ChildVal* cv = nullptr;  // [total]
  Cell4* packed = nullptr; // [total] when nfields >= 4
  float* val = nullptr;    // chunk by chunk: [nfields][chunk ncells]
  // device side: nslots buffers of cap cells, used in turn
  int32_t nslots = 0;
  char* slot[kMaxBuffers] = {};
  int64_t slot_bytes = 0, off_packed = 0, off_val = 0;
  hipStream_t copy = nullptr;
  hipStream_t compute2 = nullptr;  // the second compute stream (plane B)
  hipEvent_t started = nullptr, finished2 = nullptr;
  hipEvent_t copied[kMaxBuffers] = {}, consumed[kMaxBuffers] = {};
  bool used[kMaxBuffers] = {};
};

namespace {

void host_free(amr_stream_plan* p, void* q) {
  if (!q) return;
  if (p->host_only)
    std::free(q);
  else
    (void)hipHostFree(q);
}

void* host_alloc(amr_stream_plan* p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (p->host_only) return std::malloc(bytes);
  void* q = nullptr;
  return hipHostMalloc(&q, bytes, hipHostMallocDefault) == hipSuccess ? q : nullptr;
}

void release(amr_stream_plan* p) {
  for (int s = 0; s < kMaxBuffers; ++s) {
    if (p->slot[s]) (void)hipFree(p->slot[s]);
    if (p->copied[s]) (void)hipEventDestroy(p->copied[s]);
    if (p->consumed[s]) (void)hipEventDestroy(p->consumed[s]);
  }
  if (p->started) (void)hipEventDestroy(p->started);
  if (p->finished2) (void)hipEventDestroy(p->finished2);
  if (p->copy) (void)hipStreamDestroy(p->copy);
  if (p->compute2) (void)hipStreamDestroy(p->compute2);
  host_free(p, p->cv);
  host_free(p, p->packed);
  host_free(p, p->val);
  delete p;
}

// Pixel rectangle [i0, i1] x [j0, j1] that holds every pixel whose ray can
// meet the chunk's cube; false when none can.  A point x lies on the ray of
// (a, b) iff x - O = t (F + a U + b V) (perspective, t > 0) or
// x - O = a U + b V + t F (orthographic); solving that 3 x 3 system gives
// (t, a, b) of any point, and the image of a convex set under (a, b) is the
// convex hull of its vertices' images (for a perspective record, where t > 0
// on the whole set).  Perspective: no ray of the image meets the cube before
// t_min = d / (2 Dmax), d the distance from the eye to the cube and Dmax a
// bound on the length of every pixel's direction, since by then a ray is
// closer to the eye than d; so the cube is cut by the plane t = t_min, and
// its part beyond is the convex polytope whose vertices are the corners
// beyond the plane and the crossings of the plane by the cube's edges.  An
// eye inside the cube, or a nearly singular record, gives the whole image.
// The bounds widen by one pixel, far beyond the fp64 rounding, so the
// rectangle is conservative; rays inside it that miss the cube are rejected
// exactly by the kernel.
bool chunk_rect(const amr_camera& cam, const Chunk& c, int32_t r[4]) {
  const int W = cam.W, H = cam.H;
  r[0] = 0;
  r[1] = 0;
  r[2] = W - 1;
  r[3] = H - 1;
  double M[3][3];
  for (int k = 0; k < 3; ++k) {
    const double f = (double)cam.F[k], u = (double)cam.U[k], v = (double)cam.V[k];
    if (cam.kind == 0) {
      M[k][0] = f; M[k][1] = u; M[k][2] = v;
    } else {
      M[k][0] = u; M[k][1] = v; M[k][2] = f;
    }
  }
  double inv[3][3];
  inv[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
  inv[0][1] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
  inv[0][2] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
  inv[1][0] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
  inv[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
  inv[1][2] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
  inv[2][0] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
  inv[2][1] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
  inv[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
  const double det = M[0][0] * inv[0][0] + M[0][1] * inv[1][0] + M[0][2] * inv[2][0];
  double nrm[3];
  for (int col = 0; col < 3; ++col)
    nrm[col] = std::sqrt(M[0][col] * M[0][col] + M[1][col] * M[1][col] + M[2][col] * M[2][col]);
  if (!(std::fabs(det) > 1e-6 * nrm[0] * nrm[1] * nrm[2])) return true;
  const double side = std::ldexp(1.0, kFix - c.level);
  const int32_t cc[3] = {c.ix, c.iy, c.iz};
  double s[8][3];
  for (int corner = 0; corner < 8; ++corner) {
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = (cc[k] + ((corner >> k) & 1)) * side - (double)cam.O[k];
    for (int q = 0; q < 3; ++q) s[corner][q] = (inv[q][0] * d[0] + inv[q][1] * d[1] + inv[q][2] * d[2]) / det;
  }
  double amin = INFINITY, amax = -INFINITY, bmin = INFINITY, bmax = -INFINITY;
  auto take = [&](double a, double b) {
    amin = std::min(amin, a);
    amax = std::max(amax, a);
    bmin = std::min(bmin, b);
    bmax = std::max(bmax, b);
  };
  if (cam.kind == 0) {
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double lo = cc[k] * side, hi = lo + side, o = (double)cam.O[k];
      const double g = o < lo ? lo - o : (o > hi ? o - hi : 0.0);
      d2 += g * g;
    }
    if (!(d2 > 0.0)) return true;  // the eye in the cube or on its surface
    const double dmax = nrm[0] + W * nrm[1] + H * nrm[2];
    const double tmin = 0.5 * std::sqrt(d2) / dmax;
    int nv = 0;
    for (int corner = 0; corner < 8; ++corner) {
      if (s[corner][0] >= tmin) {
        take(s[corner][1] / s[corner][0], s[corner][2] / s[corner][0]);
        ++nv;
      }
      for (int k = 0; k < 3; ++k) {  // the edge to the corner one step up along axis k
        const int other = corner | (1 << k);
        if (other == corner) continue;
        const double t0 = s[corner][0], t1 = s[other][0];
        if ((t0 < tmin) == (t1 < tmin)) continue;
        const double lam = (tmin - t0) / (t1 - t0);
        take((s[corner][1] + lam * (s[other][1] - s[corner][1])) / tmin,
             (s[corner][2] + lam * (s[other][2] - s[corner][2])) / tmin);
        ++nv;
      }
    }
    if (nv == 0) return false;  // the cube lies wholly before t_min: behind the eye
  } else {
    for (int corner = 0; corner < 8; ++corner) take(s[corner][0], s[corner][1]);
  }
  if (!std::isfinite(amin) || !std::isfinite(amax) || !std::isfinite(bmin) || !std::isfinite(bmax)) return true;
  // a = 2i + 1 - W, so i = (a + W - 1) / 2
  const double i0 = std::floor((amin + W - 1) * 0.5) - 1.0, i1 = std::ceil((amax + W - 1) * 0.5) + 1.0;
  const double j0 = std::floor((bmin + H - 1) * 0.5) - 1.0, j1 = std::ceil((bmax + H - 1) * 0.5) + 1.0;
  if (i1 < 0.0 || j1 < 0.0 || i0 > W - 1 || j0 > H - 1) return false;
  r[0] = (int32_t)std::max(0.0, i0);
  r[1] = (int32_t)std::max(0.0, j0);
  r[2] = (int32_t)std::min((double)(W - 1), i1);
  r[3] = (int32_t)std::min((double)(H - 1), j1);
  return true;
}

// ------------------------------------------------------------------ kernels

struct StreamArgs {
  TreeView t;
  CameraView c;
  int32_t field, wfield, los, max_level;
  int32_t lc, cx, cy, cz;
  int32_t i0, j0, rw, rh, px;
  Partial* acc;
};

template <int OP>
__global__ __launch_bounds__(256) void k_stream_init(Partial* acc, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  Partial P;
  partial_init<OP>(P);
  acc[p] = P;
}

// One block of 64 rays (an 8 x 8 packet of the chunk's pixel rectangle):
// each ray is clipped to the chunk's cube and its part there walked and
// added to the pixel's partial.
template <int OP, bool kStd>
__global__ __launch_bounds__(64) void k_stream_chunk(StreamArgs a) {
  extern __shared__ int32_t stack_lds[];  // the walk's ancestor stack
  const int lane = threadIdx.x;
  const int ty = (int)blockIdx.x / a.px, tx = (int)blockIdx.x - ty * a.px;
  const int di = tx * 8 + (lane & 7), dj = ty * 8 + (lane >> 3);
  if (di >= a.rw || dj >= a.rh) return;
  const int i = a.i0 + di, j = a.j0 + dj;
  Ray R;
  Entry E;
  if (!setup_ray(a.c, i, j, R, E)) return;
  if (!cube_clip(R, E, a.lc, a.cx, a.cy, a.cz)) return;
  Partial P;
  partial_init<OP>(P);
  StridedStack<64> S{stack_lds + lane, a.t.base < a.max_level ? a.t.base : a.max_level};
  walk_span<OP, false, false, kStd>(a.t, R, E, a.max_level, a.field, a.wfield, a.los, P, nullptr, S);
  Partial* A = a.acc + (int64_t)j * a.c.W + i;
  Partial Q = *A;
  partial_merge<OP>(Q, P);
  *A = Q;
}

// Plane B (the chunks of the second compute stream) merged into plane A,
// then the pixel's value.
template <int OP>
__global__ __launch_bounds__(256) void k_stream_finish(const Partial* acc, float* out, float* aux, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  Partial A = acc[p];
  partial_merge<OP>(A, acc[n + p]);
  float o = 0.0f, x = 0.0f;
  partial_finish<OP>(A, o, x);
  out[p] = o;
  if (OP == kOpWMean && aux) aux[p] = x;
}

template <int OP, bool kStd>
void launch_chunk(const StreamArgs& a, int blocks, hipStream_t s) {
  const int b0 = a.t.base < a.max_level ? a.t.base : a.max_level;
  const size_t lds = (size_t)(a.max_level - b0 + 1) * 64 * sizeof(int32_t);
  hipLaunchKernelGGL((k_stream_chunk<OP, kStd>), dim3((unsigned)blocks), dim3(64), lds, s, a);
}

}  // namespace

extern "C" {

amr_status amr_stream_plan_create(const amr_tree* t, const amr_stream_opts* opts, amr_stream_plan** out) {
  if (!t || !opts || !out) return fail(AMR_EINVAL, "null argument");
  *out = nullptr;
  if (!t->info.host_only) return fail(AMR_EINVAL, "a stream plan is built from a host_only tree");
  if (opts->max_chunk_cells < 1 || opts->max_chunk_cells >= (int64_t(1) << 31))
    return fail(AMR_EINVAL, "max_chunk_cells must be in 1..2^31-1");
  if (opts->nbuffers != 0 && (opts->nbuffers < 2 || opts->nbuffers > kMaxBuffers))
    return fail(AMR_EINVAL, "nbuffers must be 0 or 2..8");
  const TreeView& V = t->view;
  const int64_t ncells = V.ncells;
  const int nf = V.nfields;
  const int32_t* child = t->h_child.data();
  const float* val = t->h_val.data();
  amr_stream_plan* p = new (std::nothrow) amr_stream_plan();
  if (!p) return fail(AMR_ENOMEM, "host allocation failed");
  p->info = t->info;
  p->base = V.base;
  p->lmax = V.lmax;
  p->nfields = nf;
  p->host_only = opts->host_only ? 1 : 0;
  p->cap = opts->max_chunk_cells;
  p->nslots = opts->nbuffers ? opts->nbuffers : 4;
  int64_t off[kMaxLevel + 2];
  for (int l = 0; l <= kMaxLevel + 1; ++l) off[l] = t->info.level_offset[l];

  // refined cells of each level before each cell: the children of the r-th
  // refined cell of level l are cells off[l+1] + 8r .. + 7 (the builder
  // emits children in the order of their parents)
  std::vector<int32_t> rb;
  int64_t tot[kMaxLevel + 1] = {0};
  try {
    rb.resize(ncells);
  } catch (...) {
    release(p);
    return fail(AMR_ENOMEM, "host allocation failed");
  }
  std::atomic<bool> layout_ok{true};
  parallel_items(kMaxLevel + 1, [&](int64_t l) {
    int32_t r = 0;
    for (int64_t q = off[l]; q < off[l + 1]; ++q) {
      rb[q] = r;
      if (child[q] >= 0) {
        if (child[q] != off[l + 1] + 8 * (int64_t)r) layout_ok = false;
        ++r;
      }
    }
    tot[l] = r;
  });
  if (!layout_ok) {
    release(p);
    return fail(AMR_ETREE, "tree arrays are not in the builder's layout");
  }
  auto rbefore = [&](int l, int64_t q) -> int64_t { return q == off[l + 1] ? tot[l] : rb[q]; };
  // descendant ranges [lo, hi) per level of the cell q at level lc; returns the cell count
  auto ranges = [&](int lc, int64_t q, int64_t* lo, int64_t* hi) -> int64_t {
    int64_t a = q, b = q + 1, n = 0;
    for (int l = 0; l <= kMaxLevel; ++l) lo[l] = hi[l] = 0;
    for (int l = lc; l <= kMaxLevel; ++l) {
      lo[l] = a;
      hi[l] = b;
      n += b - a;
      if (l == kMaxLevel || a == b) break;
      const int64_t a2 = off[l + 1] + 8 * rbefore(l, a), b2 = off[l + 1] + 8 * rbefore(l, b);
      a = a2;
      b = b2;
    }
    return n;
  };

  // partition: cubes in Morton order, split while their subtree exceeds the cap
  struct Cube {
    int32_t level;
    uint32_t code;
  };
  std::vector<Cube> stack{{0, 0u}};
  std::vector<std::array<int64_t, 2 * (kMaxLevel + 1)>> spans;
  while (!stack.empty()) {
    const Cube cu = stack.back();
    stack.pop_back();
    int64_t lo[kMaxLevel + 1], hi[kMaxLevel + 1];
    const int64_t n = ranges(cu.level, off[cu.level] + cu.code, lo, hi);
    if (n <= p->cap) {
      Chunk c{};
      c.level = cu.level;
      c.ix = (int32_t)compact3(cu.code);
      c.iy = (int32_t)compact3(cu.code >> 1);
      c.iz = (int32_t)compact3(cu.code >> 2);
      c.ncells = n;
      c.first = p->total;
      int64_t s = 0;
      for (int l = 0; l <= kMaxLevel; ++l) {
        c.level_start[l] = l < cu.level ? 0 : s;
        if (l >= cu.level) s += hi[l] - lo[l];
      }
      c.level_start[kMaxLevel + 1] = s;
      for (int l = cu.level; l <= V.base; ++l) c.off_local[l] = (int32_t)(off[l] - lo[l] + c.level_start[l]);
      p->total += n;
      p->chunks.push_back(c);
      std::array<int64_t, 2 * (kMaxLevel + 1)> sp;
      for (int l = 0; l <= kMaxLevel; ++l) {
        sp[l] = lo[l];
        sp[kMaxLevel + 1 + l] = hi[l];
      }
      spans.push_back(sp);
    } else if (cu.level < V.base) {
      for (int o = 7; o >= 0; --o) stack.push_back({cu.level + 1, (cu.code << 3) | (uint32_t)o});
    } else {
      release(p);
      return fail(AMR_ECAPACITY, "a subtree under one base-level cell exceeds max_chunk_cells");
    }
  }
  std::vector<int32_t>().swap(rb);
  p->min_chunk_level = kMaxLevel;
  for (const Chunk& c : p->chunks) {
    p->max_chunk_level = std::max(p->max_chunk_level, c.level);
    p->min_chunk_level = std::min(p->min_chunk_level, c.level);
  }

  // host arrays, chunk after chunk, with chunk-local first-child indices
  p->cv = (ChildVal*)host_alloc(p, (size_t)p->total * sizeof(ChildVal));
  p->val = (float*)host_alloc(p, (size_t)p->total * nf * sizeof(float));
  if (nf >= 4) p->packed = (Cell4*)host_alloc(p, (size_t)p->total * sizeof(Cell4));
  if (!p->cv || !p->val || (nf >= 4 && !p->packed)) {
    release(p);
    return fail(AMR_ENOMEM, "host (pinned) allocation failed");
  }
  parallel_items((int64_t)p->chunks.size(), [&](int64_t k) {
    const Chunk& c = p->chunks[k];
    const auto& sp = spans[k];
    ChildVal* cv = p->cv + c.first;
    float* vv = p->val + (size_t)nf * c.first;
    for (int l = c.level; l <= kMaxLevel; ++l) {
      const int64_t lo = sp[l], hi = sp[kMaxLevel + 1 + l];
      if (lo == hi) break;
      const int64_t nlo = l < kMaxLevel ? sp[l + 1] : 0, nls = l < kMaxLevel ? c.level_start[l + 1] : 0;
      for (int64_t q = lo; q < hi; ++q) {
        const int64_t loc = c.level_start[l] + (q - lo);
        const int32_t w = child[q];
        cv[loc] = ChildVal{w >= 0 ? (int32_t)(w - nlo + nls) : -1, val[q]};
        for (int f = 0; f < nf; ++f) vv[(size_t)f * c.ncells + loc] = val[(size_t)f * ncells + q];
        if (p->packed)
          p->packed[c.first + loc] =
              Cell4{val[q], val[(size_t)ncells + q], val[2 * (size_t)ncells + q], val[3 * (size_t)ncells + q]};
      }
    }
  });

  if (!p->host_only) {
    p->off_packed = align_up(p->cap * (int64_t)sizeof(ChildVal));
    p->off_val = p->off_packed + (nf >= 4 ? align_up(p->cap * (int64_t)sizeof(Cell4)) : 0);
    p->slot_bytes = p->off_val + align_up(p->cap * nf * (int64_t)sizeof(float));
    hipError_t e = hipSuccess;
    for (int s = 0; s < p->nslots && e == hipSuccess; ++s) e = hipMalloc((void**)&p->slot[s], (size_t)p->slot_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->compute2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->started, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->finished2, hipEventDisableTiming);
    for (int s = 0; s < p->nslots && e == hipSuccess; ++s) {
      e = hipEventCreateWithFlags(&p->copied[s], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p->consumed[s], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      release(p);
      return fail(AMR_ENOMEM, std::string("device set-up failed: ") + hipGetErrorString(e));
    }
  }
  *out = p;
  return AMR_OK;
}

void amr_stream_plan_free(amr_stream_plan* p) {
  if (!p) return;
  if (!p->host_only) {
    (void)hipStreamSynchronize(p->copy);
    (void)hipStreamSynchronize(p->compute2);
    for (int s = 0; s < p->nslots; ++s)
      if (p->used[s]) (void)hipEventSynchronize(p->consumed[s]);
  }
  release(p);
}

amr_status amr_stream_plan_info(const amr_stream_plan* p, amr_stream_plan_info_t* out) {
  if (!p || !out) return fail(AMR_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->nchunks = (int32_t)p->chunks.size();
  out->min_chunk_level = p->min_chunk_level;
  out->max_chunk_level = p->max_chunk_level;
  out->max_chunk_cells = p->cap;
  for (const Chunk& c : p->chunks) out->largest_chunk = std::max(out->largest_chunk, c.ncells);
  out->cells = p->total;
  out->host_bytes = p->total * (int64_t)(sizeof(ChildVal) + 4 * p->nfields + (p->packed ? sizeof(Cell4) : 0));
  out->device_bytes = p->nslots * p->slot_bytes;
  out->nbuffers = p->nslots;
  return AMR_OK;
}

amr_status amr_stream_chunk(const amr_stream_plan* p, int32_t i, amr_stream_chunk_t* out) {
  if (!p || !out) return fail(AMR_EINVAL, "null argument");
  if (i < 0 || i >= (int32_t)p->chunks.size()) return fail(AMR_EINVAL, "chunk index out of range");
  const Chunk& c = p->chunks[i];
  std::memset(out, 0, sizeof(*out));
  out->level = c.level;
  out->ix = c.ix;
  out->iy = c.iy;
  out->iz = c.iz;
  out->ncells = c.ncells;
  out->first = c.first;
  for (int l = 0; l <= kMaxLevel + 1; ++l) {
    out->level_start[l] = c.level_start[l];
    out->off_local[l] = c.off_local[l];
  }
  out->records = (const int32_t*)(p->cv + c.first);
  out->values = p->val + (size_t)p->nfields * c.first;
  out->packed = p->packed ? (const float*)(p->packed + c.first) : nullptr;
  return AMR_OK;
}

amr_status amr_stream_chunk_rect(const amr_stream_plan* p, int32_t i, const amr_camera* cam, int32_t rect[4]) {
  if (!p || !cam || !rect) return fail(AMR_EINVAL, "null argument");
  if (i < 0 || i >= (int32_t)p->chunks.size()) return fail(AMR_EINVAL, "chunk index out of range");
  amr_status st = check_camera(cam);
  if (st) return st;
  if (!chunk_rect(*cam, p->chunks[i], rect)) {
    rect[0] = rect[1] = 0;
    rect[2] = rect[3] = -1;
  }
  return AMR_OK;
}

int64_t amr_stream_workspace_bytes(int32_t W, int32_t H) {
  if (W < 1 || H < 1) return 0;
  return 2 * (int64_t)W * H * (int64_t)sizeof(Partial);
}

amr_status amr_render_streamed(amr_stream_plan* p, const amr_camera* cam, amr_op op, const amr_render_opts* opts,
                               float* out, float* aux, void* workspace, int64_t workspace_bytes, int64_t* stats,
                               amr_stream s) {
  if (!p) return fail(AMR_EINVAL, "null plan");
  if (p->host_only) return fail(AMR_EINVAL, "a host_only plan cannot render");
  amr_status st = check_camera(cam);
  if (st) return st;
  if (!out || !workspace) return fail(AMR_EINVAL, "null output or workspace");
  if (((uintptr_t)out & 3) || ((uintptr_t)aux & 3) || ((uintptr_t)workspace & 255))
    return fail(AMR_EINVAL, "misaligned buffer");
  if (op != AMR_SUM && op != AMR_MAX && op != AMR_WMEAN) return fail(AMR_EINVAL, "bad op");
  const amr_render_opts o = opts ? *opts : amr_render_opts{0, 0, 0, -1};
  const int nf = p->nfields;
  const int los = op == AMR_WMEAN && o.los_velocity ? 1 : 0;
  if (o.field < 0 || o.field + (los ? 2 : 0) >= nf) return fail(AMR_EINVAL, "field index out of range");
  if (op == AMR_WMEAN && (o.weight_field < 0 || o.weight_field >= nf)) return fail(AMR_EINVAL, "bad weight field");
  if (cam->max_level < p->max_chunk_level)
    return fail(AMR_EINVAL, "max_level is shallower than the plan's deepest chunk level");
  const int64_t npix = (int64_t)cam->W * cam->H;
  if (workspace_bytes < amr_stream_workspace_bytes(cam->W, cam->H)) return fail(AMR_ECAPACITY, "workspace too small");
  hipStream_t hs = (hipStream_t)s;
  Partial* acc = (Partial*)workspace;
  // arrays the op reads: the 8-byte records always; the interleaved records
  // for the line-of-sight wmean of fields (1..3; weight 0); else the fields
  const bool pk = op == AMR_WMEAN && los && o.weight_field == 0 && o.field == 1 && p->packed;
  bool need[8] = {false};
  if (op != AMR_WMEAN) {
    need[o.field] = o.field != 0;
  } else if (!pk) {
    need[o.weight_field] = true;
    need[o.field] = true;
    if (los) need[o.field + 1] = need[o.field + 2] = true;
  }
  const int opi = (int)op;
  const int64_t nb = (npix + 255) / 256, nb2 = (2 * npix + 255) / 256;
  if (opi == kOpSum) hipLaunchKernelGGL(k_stream_init<kOpSum>, dim3((unsigned)nb2), dim3(256), 0, hs, acc, 2 * npix);
  else if (opi == kOpMax) hipLaunchKernelGGL(k_stream_init<kOpMax>, dim3((unsigned)nb2), dim3(256), 0, hs, acc, 2 * npix);
  else hipLaunchKernelGGL(k_stream_init<kOpWMean>, dim3((unsigned)nb2), dim3(256), 0, hs, acc, 2 * npix);
  // the second compute stream starts after the planes are set
  hipError_t e0 = hipEventRecord(p->started, hs);
  if (e0 == hipSuccess) e0 = hipStreamWaitEvent(p->compute2, p->started, 0);
  if (e0 != hipSuccess) return fail(AMR_EHIP, std::string("streamed render failed: ") + hipGetErrorString(e0));
  const int ml = std::min(cam->max_level, p->lmax);
  int64_t bytes = 0, pixels = 0;
  int32_t launched = 0;
  hipError_t e = hipGetLastError();
  for (size_t k = 0; k < p->chunks.size() && e == hipSuccess; ++k) {
    const Chunk& c = p->chunks[k];
    int32_t r[4];
    if (!chunk_rect(*cam, c, r)) continue;
    const int slot = launched % p->nslots;
    // chunks alternate between the caller's stream (plane A) and the plan's
    // second compute stream (plane B), so one chunk's last rays overlap the
    // next chunk's walk; the assignment depends on the chunk order only
    hipStream_t ks = (launched & 1) ? p->compute2 : hs;
    char* buf = p->slot[slot];
    // cells at levels down to the camera's maximum level: a prefix of the chunk
    const int64_t m = c.level_start[ml + 1];
    if (p->used[slot]) e = hipStreamWaitEvent(p->copy, p->consumed[slot], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(buf, p->cv + c.first, (size_t)m * sizeof(ChildVal), hipMemcpyHostToDevice, p->copy);
    bytes += m * (int64_t)sizeof(ChildVal);
    if (e == hipSuccess && pk) {
      e = hipMemcpyAsync(buf + p->off_packed, p->packed + c.first, (size_t)m * sizeof(Cell4), hipMemcpyHostToDevice,
                         p->copy);
      bytes += m * (int64_t)sizeof(Cell4);
    }
    for (int f = 0; f < nf && e == hipSuccess; ++f) {
      if (!need[f]) continue;
      e = hipMemcpyAsync(buf + p->off_val + (size_t)f * c.ncells * 4, p->val + (size_t)nf * c.first + (size_t)f * c.ncells,
                         (size_t)m * 4, hipMemcpyHostToDevice, p->copy);
      bytes += m * 4;
    }
    if (e == hipSuccess) e = hipEventRecord(p->copied[slot], p->copy);
    if (e == hipSuccess) e = hipStreamWaitEvent(ks, p->copied[slot], 0);
    if (e != hipSuccess) break;
    StreamArgs a;
    std::memset(&a, 0, sizeof(a));
    TreeView& T = a.t;
    T.cv = (const ChildVal AMR_GLOBAL*)buf;
    T.packed = pk ? (const Cell4 AMR_GLOBAL*)(buf + p->off_packed) : nullptr;
    T.val = (const float AMR_GLOBAL*)(buf + p->off_val);
    T.ncells = c.ncells;
    T.nfields = nf;
    T.base = p->base;
    T.lmax = p->lmax;
    for (int l = 0; l <= kMaxLevel + 1; ++l) T.off[l] = c.off_local[l];
    a.c = camera_view(*cam);
    a.field = o.field;
    a.wfield = o.weight_field;
    a.los = los;
    a.max_level = cam->max_level;
    a.lc = c.level;
    a.cx = c.ix;
    a.cy = c.iy;
    a.cz = c.iz;
    a.i0 = r[0];
    a.j0 = r[1];
    a.rw = r[2] - r[0] + 1;
    a.rh = r[3] - r[1] + 1;
    a.px = (a.rw + 7) / 8;
    a.acc = acc + ((launched & 1) ? npix : 0);
    const int blocks = a.px * ((a.rh + 7) / 8);
    const bool sw = std_walk(opi, T, o.field, o.weight_field, los, cam->max_level);
    if (opi == kOpSum) sw ? launch_chunk<kOpSum, true>(a, blocks, ks) : launch_chunk<kOpSum, false>(a, blocks, ks);
    else if (opi == kOpMax) sw ? launch_chunk<kOpMax, true>(a, blocks, ks) : launch_chunk<kOpMax, false>(a, blocks, ks);
    else sw ? launch_chunk<kOpWMean, true>(a, blocks, ks) : launch_chunk<kOpWMean, false>(a, blocks, ks);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(p->consumed[slot], ks);
    p->used[slot] = true;
    pixels += (int64_t)a.rw * a.rh;
    ++launched;
  }
  if (e == hipSuccess) e = hipEventRecord(p->finished2, p->compute2);
  if (e == hipSuccess) e = hipStreamWaitEvent(hs, p->finished2, 0);
  if (e == hipSuccess) {
    if (opi == kOpSum) hipLaunchKernelGGL(k_stream_finish<kOpSum>, dim3((unsigned)nb), dim3(256), 0, hs, acc, out, aux, npix);
    else if (opi == kOpMax) hipLaunchKernelGGL(k_stream_finish<kOpMax>, dim3((unsigned)nb), dim3(256), 0, hs, acc, out, aux, npix);
    else hipLaunchKernelGGL(k_stream_finish<kOpWMean>, dim3((unsigned)nb), dim3(256), 0, hs, acc, out, aux, npix);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(AMR_EHIP, std::string("streamed render failed: ") + hipGetErrorString(e));
  if (stats) {
    stats[0] = launched;
    stats[1] = bytes;
    stats[2] = pixels;
  }
  return AMR_OK;
}

}  // extern "C"
