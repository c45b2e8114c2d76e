// batch.hip -- many (tree, camera) images in one persistent launch, and the
// variant autotuner.
//
// The paper renders independent images in parallel and balances them
// dynamically: a master hands work to whichever worker is free (Sec. 3.2),
// which pays off for many independent images (Sec. 3.1).  On the GPU the
// workers are persistent waves and the master is a global atomic counter over
// 64-ray packets of all images: a wave takes the next chunk of packets until
// the counter passes the end.  The grid configurations instead give every
// packet its own block and let the hardware dispatcher hand blocks to free
// CUs in order.  The images of one tree are kept together (so the caches
// hold one tree's working set at a time; trees with the longest rays first)
// and ordered largest first within their tree, so the tail holds small
// pieces.  The launch is captured once into a hipGraph and replayed; the
// per-pixel code is the same as amr_render's, so every image is bit-identical
// to its single-image render with the matching variant (unsplit or split).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <set>
#include <vector>

#include "internal.h"

namespace amr {

namespace {

std::mutex g_live_mu;
std::set<uint64_t>& live_trees() {
  static std::set<uint64_t> s;
  return s;
}

struct BatchImage {
  TreeView t;
  CameraView c;
  float* out;
  float* aux;
  int32_t field, wfield, los, max_level;
  int32_t packets_x, packets_y;
};

// Launch shapes: packet width, descent mode, waves per CU and packets per
// pop of the persistent kernel; or (split > 0) one block per packet over all
// images, dispatched in order by the hardware, each ray walked in `split`
// spans (the same arithmetic as the split single-image variants).
struct BatchConfig {
  int pw, mode, waves_per_cu, chunk, split;
  const char* name;
};
constexpr BatchConfig kBatchConfigs[] = {
    {8, kWalkFast, 16, 2, 0, "p8x8_fast_16w_c2"},   {8, kWalkFast, 8, 2, 0, "p8x8_fast_8w_c2"},
    {8, kWalkFast, 32, 2, 0, "p8x8_fast_32w_c2"},   {8, kWalkFast, 16, 8, 0, "p8x8_fast_16w_c8"},
    {16, kWalkFast, 16, 2, 0, "p16x4_fast_16w_c2"}, {8, kWalkBase, 16, 2, 0, "p8x8_base_16w_c2"},
    {8, kWalkFast, 0, 0, 2, "p8x8_split2_grid"},    {8, kWalkFast, 0, 0, 1, "p8x8_fast_grid"},
};
constexpr int kNumBatchConfigs = sizeof(kBatchConfigs) / sizeof(kBatchConfigs[0]);

template <int OP, int PW, int MODE>
__global__ __launch_bounds__(64) void k_batch(const BatchImage* __restrict__ imgs, const int64_t* __restrict__ begin,
                                              int32_t nimg, int64_t total, unsigned long long* counter, int32_t chunk) {
  constexpr int PH = 64 / PW;
  const int lane = threadIdx.x & 63;
  for (;;) {
    unsigned long long first = 0;
    if (lane == 0) first = atomicAdd(counter, (unsigned long long)chunk);
    first = __shfl(first, 0, 64);
    const int64_t p0 = (int64_t)first;
    if (p0 >= total) break;
    const int64_t p1 = p0 + chunk < total ? p0 + chunk : total;
    for (int64_t p = p0; p < p1; ++p) {
      // image holding packet p: last k with begin[k] <= p (wave-uniform)
      int lo = 0, hi = nimg - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= p) lo = mid; else hi = mid - 1;
      }
      const BatchImage& I = imgs[lo];
      const int64_t q = p - begin[lo];
      const int ty = (int)(q / I.packets_x), tx = (int)(q - (int64_t)ty * I.packets_x);
      const int i = tx * PW + (lane % PW), j = ty * PH + (lane / PW);
      if (i < I.c.W && j < I.c.H) {
        float o = 0.0f, x = 0.0f;
        NoStack S;
        render_pixel<OP, MODE>(I.t, I.c, I.field, I.wfield, I.los, I.max_level, i, j, o, x, S);
        const int64_t pix = (int64_t)j * I.c.W + i;
        I.out[pix] = o;
        if (OP == kOpWMean && I.aux) I.aux[pix] = x;
      }
    }
  }
}

// One block per packet of all images (images largest first, so the long
// pieces start early); K waves walk the K spans of each ray and merge in LDS.
// STD: every image may take walk_span's kStd walk (std_walk).
// STK: the walk keeps an ancestor stack in dynamic LDS (deep batches).
template <int OP, int K, bool STD = false, bool STK = false>
__global__ __launch_bounds__(64 * K) void k_batch_grid(const BatchImage* __restrict__ imgs,
                                                      const int64_t* __restrict__ begin, int32_t nimg) {
  __shared__ float part[(K > 1 ? K - 1 : 1) * 4 * 64];
  extern __shared__ int32_t stack_lds[];  // STK: (levels) x 64K words
  const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
  const int64_t p = blockIdx.x;
  int lo = 0, hi = nimg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= p) lo = mid; else hi = mid - 1;
  }
  const BatchImage& I = imgs[lo];
  const int64_t q = p - begin[lo];
  const int ty = (int)(q / I.packets_x), tx = (int)(q - (int64_t)ty * I.packets_x);
  const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
  const bool in = i < I.c.W && j < I.c.H;
  const int b0 = I.t.base < I.max_level ? I.t.base : I.max_level;
  Partial P;
  partial_init<OP>(P);
  Ray R;
  Entry E;
  if (in && setup_ray(I.c, i, j, R, E) && span_setup(R, E, b0, K, w)) {
    // the last span (the whole ray when K = 1) runs to the box: one-comparison end test
    if constexpr (STK) {
      StridedStack<64 * K> S{stack_lds + threadIdx.x, b0};
      if (K == 1 || w == K - 1)
        walk_span<OP, true, false, STD>(I.t, R, E, I.max_level, I.field, I.wfield, I.los, P, nullptr, S);
      else
        walk_span<OP, false, false, STD>(I.t, R, E, I.max_level, I.field, I.wfield, I.los, P, nullptr, S);
    } else {
      if (K == 1 || w == K - 1)
        walk_span<OP, true, false, STD>(I.t, R, E, I.max_level, I.field, I.wfield, I.los, P);
      else
        walk_span<OP, false, false, STD>(I.t, R, E, I.max_level, I.field, I.wfield, I.los, P);
    }
  }
  if (K > 1) {
    if (w > 0) {
      float* u = part + (w - 1) * 4 * 64 + lane;
      u[0] = P.s0;
      u[64] = P.c0;
      u[128] = P.s1;
      u[192] = P.c1;
    }
    __syncthreads();
    if (w != 0) return;
    for (int v = 1; v < K; ++v) {
      const float* u = part + (v - 1) * 4 * 64 + lane;
      partial_merge<OP>(P, Partial{u[0], u[64], u[128], u[192]});
    }
  }
  if (!in) return;
  float o = 0.0f, x = 0.0f;
  partial_finish<OP>(P, o, x);
  const int64_t pix = (int64_t)j * I.c.W + i;
  I.out[pix] = o;
  if (OP == kOpWMean && I.aux) I.aux[pix] = x;
}

// Longest ray of an image, in cells (for ordering the batch).
__global__ __launch_bounds__(256) void k_longest_ray(TreeView T, CameraView C, int max_level, unsigned* out) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned n = 0;
  if (pix < (int64_t)C.W * C.H) {
    Ray R;
    Entry E;
    if (setup_ray(C, (int)(pix % C.W), (int)(pix / C.W), R, E)) {
      CountVis v;
      n = (unsigned)walk_fast(T, R, E, max_level, v);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned o = (unsigned)__shfl_down((int)n, off, 64);
    n = o > n ? o : n;
  }
  if ((threadIdx.x & 63) == 0 && n) atomicMax(out, n);
}

__global__ void k_zero_counter(unsigned long long* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

template <int OP, bool STD, bool STK>
void launch_grid(int split, int64_t total, int stack_levels, const BatchImage* imgs, const int64_t* begin, int nimg,
                 hipStream_t s) {
  const size_t lds = STK ? (size_t)stack_levels * 64 * split * sizeof(int32_t) : 0;
  if (split == 2)
    hipLaunchKernelGGL((k_batch_grid<OP, 2, STD, STK>), dim3((unsigned)total), dim3(128), lds, s, imgs, begin, nimg);
  else
    hipLaunchKernelGGL((k_batch_grid<OP, 1, STD, STK>), dim3((unsigned)total), dim3(64), lds, s, imgs, begin, nimg);
}

// stack_levels > 0: the deepest image's maximum level lies kDeepSpan or
// more levels below its base level; the grid kernels then keep an ancestor
// stack of that many levels per thread.
template <int OP>
hipError_t launch_batch_op(const BatchConfig& cfg, const BatchImage* imgs, const int64_t* begin, int nimg,
                           int64_t total, unsigned long long* counter, int grid, bool std_layout, int stack_levels,
                           hipStream_t s) {
  if (cfg.split > 0) {
    if (std_layout && stack_levels > 0) launch_grid<OP, true, true>(cfg.split, total, stack_levels, imgs, begin, nimg, s);
    else if (std_layout) launch_grid<OP, true, false>(cfg.split, total, 0, imgs, begin, nimg, s);
    else if (stack_levels > 0) launch_grid<OP, false, true>(cfg.split, total, stack_levels, imgs, begin, nimg, s);
    else launch_grid<OP, false, false>(cfg.split, total, 0, imgs, begin, nimg, s);
  } else if (cfg.pw == 8 && cfg.mode == kWalkFast)
    hipLaunchKernelGGL((k_batch<OP, 8, kWalkFast>), dim3(grid), dim3(64), 0, s, imgs, begin, nimg, total, counter,
                       cfg.chunk);
  else if (cfg.pw == 16 && cfg.mode == kWalkFast)
    hipLaunchKernelGGL((k_batch<OP, 16, kWalkFast>), dim3(grid), dim3(64), 0, s, imgs, begin, nimg, total, counter,
                       cfg.chunk);
  else
    hipLaunchKernelGGL((k_batch<OP, 8, kWalkBase>), dim3(grid), dim3(64), 0, s, imgs, begin, nimg, total, counter,
                       cfg.chunk);
  return hipGetLastError();
}

int num_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

}  // namespace

void register_tree(uint64_t serial) {
  std::lock_guard<std::mutex> g(g_live_mu);
  live_trees().insert(serial);
}
void unregister_tree(uint64_t serial) {
  std::lock_guard<std::mutex> g(g_live_mu);
  live_trees().erase(serial);
}
static bool tree_live(uint64_t serial) {
  std::lock_guard<std::mutex> g(g_live_mu);
  return live_trees().count(serial) != 0;
}

}  // namespace amr

using namespace amr;

struct amr_batch {
  int op = 0;
  int nimg = 0;
  int64_t total_packets = 0;
  int config = -1;
  int grid = 0;
  std::vector<uint64_t> serials;
  std::vector<BatchImage> host_images;  // largest first
  BatchImage* d_imgs = nullptr;
  int64_t* d_begin = nullptr;
  unsigned long long* d_counter = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  // Packet tables for configuration c (its packet width), uploaded.
  hipError_t use_config(int c) {
    const BatchConfig& cfg = kBatchConfigs[c];
    std::vector<BatchImage> v = host_images;
    std::vector<int64_t> begin(nimg + 1, 0);
    for (int k = 0; k < nimg; ++k) {
      v[k].packets_x = (v[k].c.W + cfg.pw - 1) / cfg.pw;
      v[k].packets_y = (v[k].c.H + (64 / cfg.pw) - 1) / (64 / cfg.pw);
      begin[k + 1] = begin[k] + (int64_t)v[k].packets_x * v[k].packets_y;
    }
    hipError_t e = hipMemcpy(d_imgs, v.data(), sizeof(BatchImage) * nimg, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_begin, begin.data(), sizeof(int64_t) * (nimg + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    total_packets = begin[nimg];
    if (cfg.split > 0 && total_packets > 0x7fffffffLL) return hipErrorInvalidValue;  // one block per packet
    config = c;
    grid = cfg.waves_per_cu * num_cus();
    drop_graph();
    return hipSuccess;
  }
  hipError_t enqueue(hipStream_t s) {
    const BatchConfig& cfg = kBatchConfigs[config];
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, d_counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the specialised walk when every image has the op's common field layout
    const int o = op == AMR_SUM ? kOpSum : op == AMR_MAX ? kOpMax : kOpWMean;
    bool sl = true;
    // and the ancestor stack when the deepest image lies kDeepSpan or more
    // levels below its base level
    int span = 0;
    for (const BatchImage& I : host_images) {
      sl = sl && std_walk(o, I.t, I.field, I.wfield, I.los, I.max_level);
      span = std::max(span, I.max_level - std::min(I.t.base, I.max_level));
    }
    const int stack_levels = span >= kDeepSpan ? span + 1 : 0;
    if (op == AMR_SUM)
      return launch_batch_op<kOpSum>(cfg, d_imgs, d_begin, nimg, total_packets, d_counter, grid, sl, stack_levels, s);
    if (op == AMR_MAX)
      return launch_batch_op<kOpMax>(cfg, d_imgs, d_begin, nimg, total_packets, d_counter, grid, sl, stack_levels, s);
    return launch_batch_op<kOpWMean>(cfg, d_imgs, d_begin, nimg, total_packets, d_counter, grid, sl, stack_levels,
                                     s);
  }
  hipError_t capture() {
    drop_graph();
    hipError_t e = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e1 = enqueue(capture_stream);
    hipError_t e2 = hipStreamEndCapture(capture_stream, &graph);
    if (e1 != hipSuccess) return e1;
    if (e2 != hipSuccess) return e2;
    return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  }
  bool stale() const {
    for (uint64_t s : serials)
      if (!tree_live(s)) return true;
    return false;
  }
};

extern "C" {

amr_status amr_batch_create(const amr_tree* const* trees, int32_t ntrees, const amr_camera* cams, int32_t ncams,
                            const int32_t* pairs, int32_t npairs, amr_op op, const amr_render_opts* opts,
                            float* const* outs, float* const* auxs, amr_batch** plan) {
  if (!plan) return fail(AMR_EINVAL, "null plan");
  *plan = nullptr;
  if (!trees || !cams || !pairs || !outs || ntrees < 1 || ncams < 1 || npairs < 1)
    return fail(AMR_EINVAL, "null or empty batch argument");
  if (op != AMR_SUM && op != AMR_MAX && op != AMR_WMEAN) return fail(AMR_EINVAL, "bad op");
  amr_render_opts o = opts ? *opts : amr_render_opts{0, 0, 0, -1};
  std::vector<BatchImage> imgs(npairs);
  std::vector<uint64_t> serials;
  for (int k = 0; k < npairs; ++k) {
    const int ti = pairs[2 * k], ci = pairs[2 * k + 1];
    if (ti < 0 || ti >= ntrees || ci < 0 || ci >= ncams) return fail(AMR_EINVAL, "pair index out of range");
    const amr_tree* t = trees[ti];
    const amr_camera* c = &cams[ci];
    amr_status cs = check_render_common(t, c);
    if (cs) return cs;
    if (!outs[k] || ((uintptr_t)outs[k] & 3) || (auxs && ((uintptr_t)auxs[k] & 3)))
      return fail(AMR_EINVAL, "null or misaligned output");
    const int nf = t->info.nfields;
    if (o.field < 0 || o.field + ((op == AMR_WMEAN && o.los_velocity) ? 2 : 0) >= nf)
      return fail(AMR_EINVAL, "field index out of range");
    if (op == AMR_WMEAN && (o.weight_field < 0 || o.weight_field >= nf)) return fail(AMR_EINVAL, "bad weight field");
    BatchImage& I = imgs[k];
    I.t = t->view;
    I.c = camera_view(*c);
    I.out = outs[k];
    I.aux = auxs ? auxs[k] : nullptr;
    I.field = o.field;
    I.wfield = o.weight_field;
    I.los = (op == AMR_WMEAN && o.los_velocity) ? 1 : 0;
    I.max_level = c->max_level;
    I.packets_x = I.packets_y = 0;
    serials.push_back(t->serial);
  }
  // Order: by tree (below), then images whose longest ray is longest first (a
  // lone wave walking it sets the end of the launch unless it starts early),
  // then larger first.
  std::vector<unsigned> longest(npairs, 0);
  {
    unsigned* d_long = nullptr;
    hipError_t e = hipMalloc((void**)&d_long, sizeof(unsigned) * npairs);
    if (e == hipSuccess) e = hipMemset(d_long, 0, sizeof(unsigned) * npairs);
    for (int k = 0; k < npairs && e == hipSuccess; ++k) {
      const int64_t n = (int64_t)imgs[k].c.W * imgs[k].c.H;
      hipLaunchKernelGGL(k_longest_ray, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, imgs[k].t, imgs[k].c,
                         imgs[k].max_level, d_long + k);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(longest.data(), d_long, sizeof(unsigned) * npairs, hipMemcpyDeviceToHost);
    if (d_long) (void)hipFree(d_long);
    if (e != hipSuccess) return fail(AMR_EHIP, std::string("batch ordering failed: ") + hipGetErrorString(e));
  }
  // images of one tree together (trees in the order of their longest ray),
  // so that the caches hold one tree's working set at a time
  std::vector<unsigned> tree_longest(ntrees, 0);
  for (int k = 0; k < npairs; ++k) tree_longest[pairs[2 * k]] = std::max(tree_longest[pairs[2 * k]], longest[k]);
  std::vector<int> order(npairs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int ta = pairs[2 * a], tb = pairs[2 * b];
    if (ta != tb) {
      if (tree_longest[ta] != tree_longest[tb]) return tree_longest[ta] > tree_longest[tb];
      return ta < tb;
    }
    if (longest[a] != longest[b]) return longest[a] > longest[b];
    return (int64_t)imgs[a].c.W * imgs[a].c.H > (int64_t)imgs[b].c.W * imgs[b].c.H;
  });
  amr_batch* B = new (std::nothrow) amr_batch();
  if (!B) return fail(AMR_ENOMEM, "host allocation failed");
  B->op = op;
  B->nimg = npairs;
  B->serials = serials;
  B->host_images.resize(npairs);
  for (int k = 0; k < npairs; ++k) B->host_images[k] = imgs[order[k]];
  hipError_t e = hipMalloc((void**)&B->d_imgs, sizeof(BatchImage) * npairs);
  if (e == hipSuccess) e = hipMalloc((void**)&B->d_begin, sizeof(int64_t) * (npairs + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&B->d_counter, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipStreamCreate(&B->capture_stream);
  if (e != hipSuccess) {
    amr_batch_free(B);
    return fail(AMR_ENOMEM, std::string("batch allocation failed: ") + hipGetErrorString(e));
  }
  e = B->use_config(0);
  if (e != hipSuccess) {
    amr_batch_free(B);
    return fail(AMR_EHIP, std::string("batch upload failed: ") + hipGetErrorString(e));
  }
  *plan = B;
  return AMR_OK;
}

amr_status amr_render_batch(amr_batch* B, amr_stream s) {
  if (!B) return fail(AMR_EINVAL, "null plan");
  if (B->stale()) return fail(AMR_ESTALE, "a tree of this batch was freed");
  if (!B->exec) {
    hipError_t e = B->capture();
    if (e != hipSuccess) {
      B->drop_graph();
      return fail(AMR_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    }
  }
  hipError_t e = hipGraphLaunch(B->exec, (hipStream_t)s);
  if (e != hipSuccess) return fail(AMR_EHIP, std::string("graph launch failed: ") + hipGetErrorString(e));
  return AMR_OK;
}

int32_t amr_batch_config_count(void) { return kNumBatchConfigs; }
const char* amr_batch_config_name(int32_t c) {
  return (c >= 0 && c < kNumBatchConfigs) ? kBatchConfigs[c].name : "invalid";
}

amr_status amr_batch_set_config(amr_batch* B, int32_t c) {
  if (!B || c < 0 || c >= kNumBatchConfigs) return fail(AMR_EINVAL, "bad plan or configuration");
  hipError_t e = B->use_config(c);
  if (e != hipSuccess) return fail(AMR_EHIP, std::string("batch upload failed: ") + hipGetErrorString(e));
  return AMR_OK;
}

amr_status amr_batch_tune(amr_batch* B, int32_t reps, int32_t* best, float* times_ms) {
  if (!B || reps < 1) return fail(AMR_EINVAL, "bad plan or reps");
  if (B->stale()) return fail(AMR_ESTALE, "a tree of this batch was freed");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(AMR_EHIP, "event creation failed");
  int bi = 0;
  float bt = 3.4e38f;
  amr_status st = AMR_OK;
  for (int c = 0; c < kNumBatchConfigs && st == AMR_OK; ++c) {
    if (B->use_config(c) != hipSuccess) { st = fail(AMR_EHIP, "batch upload failed"); break; }
    float tmin = 3.4e38f;
    for (int r = 0; r < reps + 1; ++r) {  // first launch warms up
      if (hipEventRecord(e0, B->capture_stream) != hipSuccess || B->enqueue(B->capture_stream) != hipSuccess ||
          hipEventRecord(e1, B->capture_stream) != hipSuccess) {
        st = fail(AMR_EHIP, "batch launch failed");
        break;
      }
      float ms = 0.0f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(AMR_EHIP, "batch run failed");
        break;
      }
      if (r > 0 && ms < tmin) tmin = ms;
    }
    if (times_ms) times_ms[c] = tmin;
    if (tmin < bt) { bt = tmin; bi = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != AMR_OK) return st;
  if (B->use_config(bi) != hipSuccess) return fail(AMR_EHIP, "batch upload failed");
  if (best) *best = bi;
  return AMR_OK;
}

int32_t amr_batch_config(const amr_batch* B) { return B ? B->config : -1; }

void amr_batch_free(amr_batch* B) {
  if (!B) return;
  B->drop_graph();
  if (B->capture_stream) (void)hipStreamDestroy(B->capture_stream);
  if (B->d_imgs) (void)hipFree(B->d_imgs);
  if (B->d_begin) (void)hipFree(B->d_begin);
  if (B->d_counter) (void)hipFree(B->d_counter);
  delete B;
}

// Times every single-image variant on this (tree, camera, op) and returns
// the fastest; it becomes the tree's default for the op (variant -1).
amr_status amr_tune(amr_tree* t, const amr_camera* cam, amr_op op, const amr_render_opts* opts, float* out,
                    float* aux, amr_stream s, int32_t reps, int32_t* best, float* times_ms) {
  if (!t || !cam || reps < 1 || op < AMR_SUM || op > AMR_WMEAN) return fail(AMR_EINVAL, "bad argument");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(AMR_EHIP, "event creation failed");
  amr_render_opts o = opts ? *opts : amr_render_opts{0, 0, 0, -1};
  int bi = 0;
  float bt = 3.4e38f;
  amr_status st = AMR_OK;
  for (int v = 0; v < variant_count() && st == AMR_OK; ++v) {
    o.variant = v;
    float tmin = 3.4e38f;
    for (int r = 0; r < reps + 1; ++r) {
      if (hipEventRecord(e0, (hipStream_t)s) != hipSuccess) { st = fail(AMR_EHIP, "event record failed"); break; }
      st = amr_render(t, cam, op, &o, out, aux, s);
      if (st != AMR_OK) break;
      if (hipEventRecord(e1, (hipStream_t)s) != hipSuccess) { st = fail(AMR_EHIP, "event record failed"); break; }
      float ms = 0.0f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(AMR_EHIP, "render failed");
        break;
      }
      if (r > 0 && ms < tmin) tmin = ms;
    }
    if (times_ms) times_ms[v] = tmin;
    if (tmin < bt) { bt = tmin; bi = v; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != AMR_OK) return st;
  t->tuned_variant[op] = bi;
  if (best) *best = bi;
  return AMR_OK;
}

amr_status amr_set_default_variant(amr_tree* t, amr_op op, int32_t v) {
  if (!t || op < AMR_SUM || op > AMR_WMEAN || v < -1 || v >= variant_count()) return fail(AMR_EINVAL, "bad argument");
  t->tuned_variant[op] = v;
  return AMR_OK;
}

}  // extern "C"
