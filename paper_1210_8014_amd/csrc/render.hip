// render.hip -- HIP kernels for gfx950: per-pixel ray casting through the
// linear octree (Sec. 2.2 of the paper: one ray per pixel, top-down to the
// leaves of the tree truncated at the camera's maximum level, value x chord
// summed in any order; Sec. 2.1 names the maximum-intensity projection).
//
// Launch shape: a wave64 owns one 64-ray packet of PW x (64 / PW) adjacent
// pixels, so neighbouring rays walk the same cells and their gathers of the
// first-child and value arrays hit the same cache lines.  A block holds WPB
// waves.  Blocks are dispatched round-robin over the 8 XCDs (each with its
// own L2); the block index is remapped so every XCD renders one contiguous
// band of packets and keeps its part of the tree in its own L2.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace amr {

namespace {

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int full = nb - nb % 8;
  if (b >= full) return b;
  return (b % 8) * (full / 8) + b / 8;
}

template <int OP, int PW, int WPB, bool REMAP>
__global__ __launch_bounds__(64 * WPB) void k_render(RenderArgs A) {
  constexpr int PH = 64 / PW;
  const int lane = threadIdx.x & 63;
  const int blk = REMAP ? xcd_remap((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int packet = blk * WPB + (int)(threadIdx.x >> 6);
  const int ty = packet / A.packets_x, tx = packet - ty * A.packets_x;
  const int i = tx * PW + (lane % PW), j = ty * PH + (lane / PW);
  if (ty >= A.packets_y || i >= A.c.W || j >= A.c.H) return;
  const int64_t pix = (int64_t)j * A.c.W + i;
  float o = 0.0f, x = 0.0f;
  render_pixel<OP>(A.t, A.c, A.field, A.wfield, A.los, A.max_level, i, j, o, x);
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
      n = walk_ray(T, R, E, C.max_level, v);
    }
    if (counts) counts[pix] = n;
  }
  // wave reduction, one atomic per wave
  unsigned long long s = (unsigned long long)n;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(total, s);
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

// Variant table: packet width, waves per block, XCD remap.
struct Variant {
  int pw, wpb;
  bool remap;
  const char* name;
};
constexpr Variant kVariants[] = {
    {8, 4, true, "p8x8_w4_xcd"},  {8, 2, true, "p8x8_w2_xcd"},   {8, 1, true, "p8x8_w1_xcd"},
    {8, 8, true, "p8x8_w8_xcd"},  {16, 4, true, "p16x4_w4_xcd"}, {32, 4, true, "p32x2_w4_xcd"},
    {8, 4, false, "p8x8_w4_linear"},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int OP, int PW, int WPB, bool REMAP>
hipError_t launch_one(const RenderArgs& a, hipStream_t s) {
  const int64_t packets = (int64_t)a.packets_x * a.packets_y;
  const int64_t blocks = (packets + WPB - 1) / WPB;
  hipLaunchKernelGGL((k_render<OP, PW, WPB, REMAP>), dim3((unsigned)blocks), dim3(64 * WPB), 0, s, a);
  return hipGetLastError();
}

template <int OP>
hipError_t launch_op(int v, const RenderArgs& a, hipStream_t s) {
  switch (v) {
    case 0: return launch_one<OP, 8, 4, true>(a, s);
    case 1: return launch_one<OP, 8, 2, true>(a, s);
    case 2: return launch_one<OP, 8, 1, true>(a, s);
    case 3: return launch_one<OP, 8, 8, true>(a, s);
    case 4: return launch_one<OP, 16, 4, true>(a, s);
    case 5: return launch_one<OP, 32, 4, true>(a, s);
    case 6: return launch_one<OP, 8, 4, false>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int variant_count() { return kNumVariants; }
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
