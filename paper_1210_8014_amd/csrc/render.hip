// render.hip -- HIP kernels for gfx950: per-pixel ray casting through the
// linear octree (Sec. 2.2 of the paper: one ray per pixel, top-down to the
// leaves of the tree truncated at the camera's maximum level, value x chord
// summed in any order; Sec. 2.1 names the maximum-intensity projection).
//
// Launch shape: a wave64 owns one 64-ray packet of PW x (64 / PW) adjacent
// pixels, so neighbouring rays walk the same cells and their gathers of the
// first-child and value arrays hit the same cache lines.  A block holds WPB
// waves.  Blocks are dispatched round-robin over the 8 XCDs.  Keeping that
// interleave (consecutive packets on different XCDs at the same time) makes
// all XCDs walk the same region of the tree together, so the memory-side
// Infinity Cache, shared by the XCDs, holds one working set; the optional
// remap that gives each XCD its own band of the image (better reuse in the
// per-XCD L2, 8 working sets at once) measured slower and is kept only as a
// variant.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace amr {

namespace {

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int full = nb - nb % 8;
  if (b >= full) return b;
  return (b % 8) * (full / 8) + b / 8;
}

enum { kRemapNone = 0, kRemapXcd = 1, kRemapCenter = 2 };

// Per-lane ancestor stack in LDS, laid out [level][thread] so the 64 lanes
// of a wave touch 64 consecutive words.
struct LdsStack {
  int32_t* base;
  int stride, lo;
  __device__ int32_t get(int l) const { return base[(l - lo) * stride]; }
  __device__ void set(int l, int32_t v) { base[(l - lo) * stride] = v; }
};

template <int OP, int PW, int WPB, int REMAP, int MODE>
__global__ __launch_bounds__(64 * WPB) void k_render(RenderArgs A) {
  extern __shared__ int32_t lds[];
  constexpr int PH = 64 / PW;
  const int lane = threadIdx.x & 63;
  const int blk = REMAP == kRemapXcd ? xcd_remap((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  int packet = blk * WPB + (int)(threadIdx.x >> 6);
  if (REMAP == kRemapCenter && packet < A.packets_x * A.packets_y)
    packet = center_out(packet, A.packets_x, A.packets_y);
  const int ty = packet / A.packets_x, tx = packet - ty * A.packets_x;
  const int i = tx * PW + (lane % PW), j = ty * PH + (lane / PW);
  if (ty >= A.packets_y || i >= A.c.W || j >= A.c.H) return;
  const int64_t pix = (int64_t)j * A.c.W + i;
  float o = 0.0f, x = 0.0f;
  if (MODE == kWalkStack) {
    LdsStack S{lds + threadIdx.x, (int)blockDim.x, A.t.base < A.max_level ? A.t.base : A.max_level};
    render_pixel<OP, MODE>(A.t, A.c, A.field, A.wfield, A.los, A.max_level, i, j, o, x, S);
  } else if (MODE == kWalkFastStack) {
    const int lo = A.t.base < A.max_level ? A.t.base : A.max_level;
    StridedStack<64 * WPB> S{lds + threadIdx.x, lo};
    render_pixel<OP, MODE>(A.t, A.c, A.field, A.wfield, A.los, A.max_level, i, j, o, x, S);
  } else {
    NoStack S;
    render_pixel<OP, MODE>(A.t, A.c, A.field, A.wfield, A.los, A.max_level, i, j, o, x, S);
  }
  A.out[pix] = o;
  if (OP == kOpWMean && A.aux) A.aux[pix] = x;
}

// Split rays: a block of K waves owns one 8 x 8 packet; wave w walks span w
// of every ray of the packet (span_setup), so the K parts of a long ray run
// concurrently on different waves and the longest rays of an image, which
// bound its time when a lone wave walks them, finish about K times sooner.
// Partial sums meet in LDS and wave 0 merges them in span order.
// STD: the render may take walk_span's kStd walk (std_walk).
template <int OP, int K, int REMAP, bool STD = false>
__global__ __launch_bounds__(64 * K) __attribute__((amdgpu_waves_per_eu(OP == kOpWMean ? 8 : 1))) void k_render_split(
    RenderArgs A) {
  __shared__ float part[(K - 1) * 4 * 64];
  const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
  const int packet =
      REMAP == kRemapCenter ? center_out((int)blockIdx.x, A.packets_x, A.packets_y) : (int)blockIdx.x;
  const int ty = packet / A.packets_x, tx = packet - ty * A.packets_x;
  const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
  const bool in = ty < A.packets_y && i < A.c.W && j < A.c.H;
  const int b0 = A.t.base < A.max_level ? A.t.base : A.max_level;
  Partial P;
  partial_init<OP>(P);
  Ray R;
  Entry E;
  if (in && setup_ray(A.c, i, j, R, E) && span_setup(R, E, b0, K, w)) {
    // the last span always runs to the box (its one-comparison end test)
    if (w == K - 1)
      walk_span<OP, true, false, STD>(A.t, R, E, A.max_level, A.field, A.wfield, A.los, P);
    else
      walk_span<OP, false, false, STD>(A.t, R, E, A.max_level, A.field, A.wfield, A.los, P);
  }
  if (w > 0) {
    float* q = part + (w - 1) * 4 * 64 + lane;
    q[0] = P.s0;
    q[64] = P.c0;
    q[128] = P.s1;
    q[192] = P.c1;
  }
  __syncthreads();
  if (w != 0 || !in) return;
  for (int v = 1; v < K; ++v) {
    const float* q = part + (v - 1) * 4 * 64 + lane;
    const Partial Q{q[0], q[64], q[128], q[192]};
    partial_merge<OP>(P, Q);
  }
  float o = 0.0f, x = 0.0f;
  partial_finish<OP>(P, o, x);
  const int64_t pix = (int64_t)j * A.c.W + i;
  A.out[pix] = o;
  if (OP == kOpWMean && A.aux) A.aux[pix] = x;
}

__global__ void k_zero_i64(int64_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ __launch_bounds__(256) void k_count_all(TreeView T, CameraView C, int32_t* counts,
                                                   unsigned long long* total) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t n = 0;
  if (pix < (int64_t)C.W * C.H) {
    const int i = (int)(pix % C.W), j = (int)(pix / C.W);
    Ray R;
    Entry E;
    if (setup_ray(C, i, j, R, E)) {
      CountVis v;
      n = walk_fast<CountVis, true>(T, R, E, C.max_level, v);  // the benchmarked walk
    }
    if (counts) counts[pix] = n;
  }
  // wave reduction, one atomic per wave
  unsigned long long s = (unsigned long long)n;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(total, s);
}

__global__ __launch_bounds__(256) void k_mark(TreeView T, CameraView C, uint32_t* bits, unsigned long long* fresh) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long f = 0;
  if (pix < (int64_t)C.W * C.H) {
    Ray R;
    Entry E;
    if (setup_ray(C, (int)(pix % C.W), (int)(pix / C.W), R, E)) {
      MarkVis v;
      v.bits = bits;
      walk_fast<MarkVis, true>(T, R, E, C.max_level, v);
      f = v.fresh;
    }
  }
  for (int off = 32; off > 0; off >>= 1) f += __shfl_down(f, off, 64);
  if ((threadIdx.x & 63) == 0 && f) atomicAdd(fresh, f);
}

__global__ __launch_bounds__(256) void k_rays(TreeView T, CameraView C, const int64_t* ray_ids, int64_t n,
                                              const int64_t* offsets, int32_t* cells, int32_t* counts) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t pix = ray_ids[r];
  if (pix < 0 || pix >= (int64_t)C.W * C.H) {
    if (counts) counts[r] = -1;
    return;
  }
  const int i = (int)(pix % C.W), j = (int)(pix / C.W);
  if (cells) {
    trace_pixel(T, C, C.max_level, i, j, cells + 4 * offsets[r], offsets[r + 1] - offsets[r]);
  } else {
    counts[r] = trace_pixel(T, C, C.max_level, i, j, nullptr, 0);
  }
}

// Variant table: packet width, waves per block, XCD remap, descent mode
// (the split variants: waves per block = spans per ray).
struct Variant {
  int pw, wpb;
  int remap;
  int mode;
  const char* name;
};
constexpr Variant kVariants[] = {
    {8, 1, kRemapNone, kWalkFast, "p8x8_w1_fast"},   {8, 2, kRemapNone, kWalkFast, "p8x8_w2_fast"},
    {8, 4, kRemapNone, kWalkFast, "p8x8_w4_fast"},   {16, 4, kRemapNone, kWalkFast, "p16x4_w4_fast"},
    {32, 2, kRemapNone, kWalkFast, "p32x2_w2_fast"}, {8, 1, kRemapNone, kWalkBase, "p8x8_w1_base"},
    {8, 4, kRemapNone, kWalkBase, "p8x8_w4_base"},   {8, 1, kRemapNone, kWalkStack, "p8x8_w1_stack"},
    {8, 4, kRemapXcd, kWalkFast, "p8x8_w4_fast_xcdband"}, {8, 2, kRemapNone, kWalkFast, "p8x8_split2_fast"},
    {8, 4, kRemapNone, kWalkFast, "p8x8_split4_fast"},    {8, 1, kRemapCenter, kWalkFast, "p8x8_w1_fast_center"},
    {8, 2, kRemapCenter, kWalkFast, "p8x8_split2_fast_center"},
    {8, 4, kRemapNone, kWalkFastStack, "p8x8_w4_fastlds"},  {8, 2, kRemapNone, kWalkFastStack, "p8x8_w2_fastlds"},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int OP, int PW, int WPB, int REMAP, int MODE>
hipError_t launch_one(const RenderArgs& a, hipStream_t s) {
  const int64_t packets = (int64_t)a.packets_x * a.packets_y;
  const int64_t blocks = (packets + WPB - 1) / WPB;
  const int b0 = a.t.base < a.max_level ? a.t.base : a.max_level;
  const size_t lds = (MODE == kWalkStack || MODE == kWalkFastStack)
                        ? (size_t)(a.max_level - b0 + 1) * 64 * WPB * sizeof(int32_t)
                        : 0;
  hipLaunchKernelGGL((k_render<OP, PW, WPB, REMAP, MODE>), dim3((unsigned)blocks), dim3(64 * WPB), lds, s, a);
  return hipGetLastError();
}

template <int OP, int K, int REMAP = kRemapNone>
hipError_t launch_split(const RenderArgs& a, hipStream_t s) {
  const int64_t packets = (int64_t)a.packets_x * a.packets_y;
  if (std_walk(OP, a.t, a.field, a.wfield, a.los, a.max_level))
    hipLaunchKernelGGL((k_render_split<OP, K, REMAP, true>), dim3((unsigned)packets), dim3(64 * K), 0, s, a);
  else
    hipLaunchKernelGGL((k_render_split<OP, K, REMAP>), dim3((unsigned)packets), dim3(64 * K), 0, s, a);
  return hipGetLastError();
}

template <int OP>
hipError_t launch_op(int v, const RenderArgs& a, hipStream_t s) {
  switch (v) {
    case 0: return launch_one<OP, 8, 1, kRemapNone, kWalkFast>(a, s);
    case 1: return launch_one<OP, 8, 2, kRemapNone, kWalkFast>(a, s);
    case 2: return launch_one<OP, 8, 4, kRemapNone, kWalkFast>(a, s);
    case 3: return launch_one<OP, 16, 4, kRemapNone, kWalkFast>(a, s);
    case 4: return launch_one<OP, 32, 2, kRemapNone, kWalkFast>(a, s);
    case 5: return launch_one<OP, 8, 1, kRemapNone, kWalkBase>(a, s);
    case 6: return launch_one<OP, 8, 4, kRemapNone, kWalkBase>(a, s);
    case 7: return launch_one<OP, 8, 1, kRemapNone, kWalkStack>(a, s);
    case 8: return launch_one<OP, 8, 4, kRemapXcd, kWalkFast>(a, s);
    case 9: return launch_split<OP, 2>(a, s);
    case 10: return launch_split<OP, 4>(a, s);
    case 11: return launch_one<OP, 8, 1, kRemapCenter, kWalkFast>(a, s);
    case 12: return launch_split<OP, 2, kRemapCenter>(a, s);
    case 13: return launch_one<OP, 8, 4, kRemapNone, kWalkFastStack>(a, s);
    case 14: return launch_one<OP, 8, 2, kRemapNone, kWalkFastStack>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int variant_count() { return kNumVariants; }
// Split in two, packet rows from the middle of the image out: on the
// galaxy-disk views (2048^2, 20M leaves) the edge-on image is bound by its
// longest rays, which cross the middle rows, and runs 1.9x faster than the
// unsplit walk in plain order; face-on and at 45 degrees it costs 10-17%
// (the two span waves of a block finish at different times).
int default_variant() { return 12; }
const char* variant_name(int v) { return kVariants[v].name; }
int variant_packet_width(int v) { return kVariants[v].pw; }

int launch_render(int op, int variant, const RenderArgs& a, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (a.packets_x <= 0 || a.packets_y <= 0) return (int)hipErrorInvalidValue;
  hipError_t e;
  if (op == AMR_SUM)
    e = launch_op<AMR_SUM>(variant, a, s);
  else if (op == AMR_MAX)
    e = launch_op<AMR_MAX>(variant, a, s);
  else
    e = launch_op<AMR_WMEAN>(variant, a, s);
  return (int)e;
}

int launch_count_all(const TreeView& t, const CameraView& c, int32_t* counts, int64_t* total, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, total);
  const int64_t n = (int64_t)c.W * c.H;
  hipLaunchKernelGGL(k_count_all, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, c, counts,
                     (unsigned long long*)total);
  return (int)hipGetLastError();
}

int launch_mark(const TreeView& t, const CameraView& c, uint32_t* bits, int64_t* fresh, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = (int64_t)c.W * c.H;
  hipLaunchKernelGGL(k_mark, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, c, bits,
                     (unsigned long long*)fresh);
  return (int)hipGetLastError();
}

int launch_rays(const TreeView& t, const CameraView& c, const int64_t* ray_ids, int64_t n, const int64_t* offsets,
                int32_t* cells, int32_t* counts, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, c, ray_ids, n, offsets, cells,
                     counts);
  return (int)hipGetLastError();
}

int dev_malloc(void** p, size_t bytes) { return (int)hipMalloc(p, bytes ? bytes : 4); }
int dev_free(void* p) { return (int)hipFree(p); }
int dev_upload(void* dst, const void* src, size_t bytes) {
  return (int)hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
}
int dev_download(void* dst, const void* src, size_t bytes) {
  return (int)hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
}
const char* dev_error_string(int err) { return hipGetErrorString((hipError_t)err); }

}  // namespace amr
