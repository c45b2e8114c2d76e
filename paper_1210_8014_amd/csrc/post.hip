// post.hip -- HIP kernels for gfx950 around the ray caster: the per-pixel
// resolution plane and the adaptive Gaussian post-filter of the image
// (Sec. 2.2: the blur adapts its size to the local resolution of the image,
// hiding the blocks drawn by coarse cells), and slice maps (Sec. 3: the
// "Slicemap" tried on the GPU, a simple tree search for the cell holding
// each point of a plane).
//
// Adaptive filter: sigma(p) = kappa r(p) pixels with r the resolution
// plane.  A ladder of truncated, image-normalised Gaussians of standard
// deviations sigma_k = 0.5 x 2^(k/2), k = 0..10 (radius ceil(3 sigma_k)),
// each exactly separable; the output blends the two levels around sigma(p)
// linearly in log2 sigma (below the first level, with the image itself).
// Pass 1 filters every image row with every level at once from one staging
// of the row in LDS; pass 2 filters the columns of the two levels a pixel
// needs and blends them.  Sums are accumulated in fp64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "internal.h"

namespace amr {
namespace {

constexpr int kBlurLevels = 11;
constexpr int kBlurRmax = 48;  // ceil(3 x 16)
constexpr float kBlurSigma0 = 0.5f;
constexpr int kRowTile = 256;  // pixels of a row per block of pass 1
// ceil(3 sigma_k) of the ladder, sigma_k = 0.5 x 2^(k/2) (checked against the
// computed radii when the ladder is built)
__constant__ constexpr int kBlurMaxRadius[kBlurLevels] = {2, 3, 3, 5, 6, 9, 12, 17, 24, 34, 48};

struct BlurLadder {
  int32_t R[kBlurLevels];
  float w[kBlurLevels][kBlurRmax + 1];  // w[k][d] = exp(-d^2 / (2 sigma_k^2)), d = 0..R[k], 0 beyond
  double total[kBlurLevels];            // sum of w[k][|d|] over d = -R[k]..R[k]: a window inside the image
};

BlurLadder make_ladder() {
  BlurLadder L;
  for (int k = 0; k < kBlurLevels; ++k) {
    const double s = (double)kBlurSigma0 * std::pow(2.0, 0.5 * k);
    L.R[k] = (int32_t)std::ceil(3.0 * s);
    for (int d = 0; d <= kBlurRmax; ++d) L.w[k][d] = d <= L.R[k] ? (float)std::exp(-(double)d * d / (2.0 * s * s)) : 0.f;
    double tail = 0.0;
    for (int d = L.R[k]; d >= 1; --d) tail += (double)L.w[k][d];
    L.total[k] = (double)L.w[k][0] + 2.0 * tail;
  }
  return L;
}

// Weight of level k's taps at distances 0..R inside [0, n) around position x:
// the full window less the taps past either end (none away from the borders).
__device__ inline double window_weight(const BlurLadder& L, int k, int x, int n) {
  double out = 0.0;
  for (int d = x + 1; d <= L.R[k]; ++d) out += (double)L.w[k][d];
  for (int d = n - x; d <= L.R[k]; ++d) out += (double)L.w[k][d];
  return L.total[k] - out;
}

__global__ __launch_bounds__(64) void k_resolution(TreeView T, CameraView C, float inv_w0, float* res, int px) {
  const int lane = threadIdx.x;
  const int ty = (int)blockIdx.x / px, tx = (int)blockIdx.x - ty * px;
  const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
  if (i >= C.W || j >= C.H) return;
  Ray R;
  Entry E;
  float r = 0.0f;
  if (setup_ray(C, i, j, R, E)) {
    ResVis v;
    v.persp = C.kind == 0;
    walk_fast<ResVis, true>(T, R, E, C.max_level, v);
    r = v.res_value(inv_w0);
  }
  res[(int64_t)j * C.W + i] = r;
}

// One walk per ray for both the projection and the resolution plane: the
// visitors of the plain unsplit render (p8x8_w1_fast: one wave per 8 x 8
// packet, whole-ray fast walk) wrapped to also sum the resolution, so that
// out / aux equal that render's and res equals k_resolution's, bit for bit.
template <int OP>
__global__ __launch_bounds__(64) void k_render_res(TreeView T, CameraView C, int field, int wfield, int los,
                                                  float inv_w0, float* out, float* aux, float* res, int px) {
  const int lane = threadIdx.x;
  const int ty = (int)blockIdx.x / px, tx = (int)blockIdx.x - ty * px;
  const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
  if (i >= C.W || j >= C.H) return;
  Ray R;
  Entry E;
  const bool hit = setup_ray(C, i, j, R, E);
  const int64_t nc = T.ncells;
  const int64_t p = (int64_t)j * C.W + i;
  float o, r;
  if (OP == kOpSum) {
    WithRes<SumVis> v;
    v.v = T.val + (int64_t)field * nc;
    v.field0 = field == 0;
    v.persp = C.kind == 0;
    if (hit) walk_fast<WithRes<SumVis>, true>(T, R, E, C.max_level, v);
    o = v.s - v.c;
    r = v.res_value(inv_w0);
  } else if (OP == kOpMax) {
    WithRes<MaxVis> v;
    v.v = T.val + (int64_t)field * nc;
    v.m = -INFINITY;
    v.field0 = field == 0;
    v.persp = C.kind == 0;
    if (hit) walk_fast<WithRes<MaxVis>, true>(T, R, E, C.max_level, v);
    o = v.m;
    r = v.res_value(inv_w0);
  } else {
    WithRes<WMeanVis> v;
    v.w = T.val + (int64_t)wfield * nc;
    v.f0 = T.val + (int64_t)field * nc;
    v.f1 = los ? v.f0 + nc : v.f0;
    v.f2 = los ? v.f0 + 2 * nc : v.f0;
    v.los = los;
    if (packed_los(T, field, wfield, los)) v.use_packed(T);
    v.dh[0] = v.dh[1] = v.dh[2] = 0.0f;
    v.persp = C.kind == 0;
    if (hit) {
      const float n = sqrtf((float)(R.d64[0] * R.d64[0] + R.d64[1] * R.d64[1] + R.d64[2] * R.d64[2]));
      for (int k = 0; k < 3; ++k) v.dh[k] = (float)R.d64[k] / n;
      walk_fast<WithRes<WMeanVis>, true>(T, R, E, C.max_level, v);
    }
    const float W = v.sw - v.cw, Sf = v.sf - v.cf;
    o = W > 0.0f ? Sf / W : 0.0f;
    if (aux) aux[p] = W;
    r = v.res_value(inv_w0);
  }
  out[p] = o;
  res[p] = r;
}

// Pass 1: h_k(x, y) = sum_d w_k(d) I(x + d, y) / sum_d w_k(d) over the taps
// inside the row, for every level k; planes h[k][H][W].  Each distance d is
// visited once: the pair I(x - d) + I(x + d) (zero outside the row, staged
// in LDS) is added, in fp64, to the sum of every level whose window reaches
// d; the weights are the same for every thread.
__global__ __launch_bounds__(kRowTile) void k_blur_rows(const float* __restrict__ img, int W, int H, BlurLadder Lad,
                                                       float* __restrict__ h) {
  __shared__ float row[kRowTile + 2 * kBlurRmax];
  const int y = blockIdx.y, x0 = blockIdx.x * kRowTile, t = threadIdx.x;
  for (int e = t; e < kRowTile + 2 * kBlurRmax; e += kRowTile) {
    const int x = x0 - kBlurRmax + e;
    row[e] = (x >= 0 && x < W) ? img[(int64_t)y * W + x] : 0.0f;
  }
  __syncthreads();
  const int x = x0 + t;
  if (x >= W) return;
  const float* r = row + t + kBlurRmax;
  double acc[kBlurLevels];
  const double c = (double)r[0];
  AMR_UNROLL
  for (int k = 0; k < kBlurLevels; ++k) acc[k] = (double)Lad.w[k][0] * c;
  AMR_UNROLL
  for (int d = 1; d <= kBlurRmax; ++d) {
    const double pair = (double)r[-d] + (double)r[d];
    AMR_UNROLL
    for (int k = 0; k < kBlurLevels; ++k)
      if (d <= kBlurMaxRadius[k]) acc[k] += (double)Lad.w[k][d] * pair;
  }
  const int64_t plane = (int64_t)W * H;
  AMR_UNROLL
  for (int k = 0; k < kBlurLevels; ++k)
    h[k * plane + (int64_t)y * W + x] = (float)(acc[k] / window_weight(Lad, k, x, W));
}

// Pass 2: per pixel, the column filter of the levels around sigma(p) and
// their blend.  Blocks of 64 x 4 pixels: a wave reads 64 consecutive floats
// of a row per tap.
__global__ __launch_bounds__(256) void k_blur_cols(const float* __restrict__ img, const float* __restrict__ res,
                                                  int W, int H, float kappa, BlurLadder Lad,
                                                  const float* __restrict__ h, float* __restrict__ out) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= W || y >= H) return;
  const int64_t p = (int64_t)y * W + x, plane = (int64_t)W * H;
  const float sigma = kappa * res[p];
  const float I = img[p];
  int lo, hi;
  float a;
  if (!(sigma > 0.0f)) {
    out[p] = I;
    return;
  }
  if (sigma < kBlurSigma0) {
    lo = -1;
    hi = 0;
    a = sigma / kBlurSigma0;
  } else {
    const float u = 2.0f * log2f(sigma / kBlurSigma0);
    const int k = (int)floorf(u);
    if (k >= kBlurLevels - 1) {
      lo = hi = kBlurLevels - 1;
      a = 0.0f;
    } else {
      lo = k;
      hi = k + 1;
      a = u - (float)k;
    }
  }
  double b[2];
  for (int q = 0; q < 2; ++q) {
    const int k = q == 0 ? lo : hi;
    if (k < 0) {
      b[q] = (double)I;
      continue;
    }
    if (q == 1 && hi == lo) {
      b[1] = b[0];
      continue;
    }
    // taps at distances 1..R in pairs, those outside the image left out
    const int R = Lad.R[k];
    const float* col = h + k * plane + x;
    double acc = (double)Lad.w[k][0] * (double)col[(int64_t)y * W];
    for (int d = 1; d <= R; ++d) {
      const double up = y - d >= 0 ? (double)col[(int64_t)(y - d) * W] : 0.0;
      const double dn = y + d < H ? (double)col[(int64_t)(y + d) * W] : 0.0;
      acc += (double)Lad.w[k][d] * (up + dn);
    }
    b[q] = acc / window_weight(Lad, k, y, H);
  }
  out[p] = (float)((1.0 - (double)a) * b[0] + (double)a * b[1]);
}

// Slice map: the cell of the truncated tree holding the point O + aU + bV
// of each pixel (orthographic record): located like the walk's descent, from
// the complete base level (Morton index, no memory read) through the
// (first child, field 0) records.  NaN outside the box.
__global__ __launch_bounds__(64) void k_slice(TreeView T, CameraView C, int field, float* out, int px) {
  const int lane = threadIdx.x;
  const int ty = (int)blockIdx.x / px, tx = (int)blockIdx.x - ty * px;
  const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
  if (i >= C.W || j >= C.H) return;
  const int64_t a = 2 * (int64_t)i + 1 - C.W, b = 2 * (int64_t)j + 1 - C.H;
  int64_t p[3];
  bool in = true;
  for (int k = 0; k < 3; ++k) {
    p[k] = C.O[k] + a * C.U[k] + b * C.V[k];
    in = in && p[k] >= 0 && p[k] < kOne;
  }
  float v = __builtin_nanf("");
  if (in) {
    const int L = C.max_level;
    const int b0 = T.base < L ? T.base : L;
    const int sb = kFix - b0;
    int32_t node = T.off[b0] + (int32_t)morton3((uint32_t)(p[0] >> sb), (uint32_t)(p[1] >> sb), (uint32_t)(p[2] >> sb));
    int lvl = b0;
    ChildVal rec = T.cv[(uint32_t)node];
    while (lvl < L && rec.child >= 0) {
      ++lvl;
      const int s = kFix - lvl;
      const int oct = (int)((p[0] >> s) & 1) | (int)(((p[1] >> s) & 1) << 1) | (int)(((p[2] >> s) & 1) << 2);
      node = rec.child + oct;
      rec = T.cv[(uint32_t)node];
    }
    v = field == 0 ? rec.v0 : T.val[(int64_t)field * T.ncells + (uint32_t)node];
  }
  out[(int64_t)j * C.W + i] = v;
}

int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

}  // namespace
}  // namespace amr

using namespace amr;

extern "C" {

// 1 / (pixel spacing at unit ray parameter), from the record's pixel step.
bool inv_spacing(const amr_camera* cam, float* inv_w0) {
  double u2 = 0.0;
  for (int k = 0; k < 3; ++k) u2 += (double)cam->U[k] * (double)cam->U[k];
  if (!(u2 > 0.0)) return false;
  *inv_w0 = (float)(1.0 / (2.0 * std::sqrt(u2) * 0x1.0p-28));
  return true;
}

amr_status amr_render_resolution(const amr_tree* t, const amr_camera* cam, float* res, amr_stream s) {
  amr_status st = check_render_common(t, cam);
  if (st) return st;
  if (!res || ((uintptr_t)res & 3)) return fail(AMR_EINVAL, "null or misaligned output");
  float inv_w0;
  if (!inv_spacing(cam, &inv_w0)) return fail(AMR_EINVAL, "zero pixel step");
  const int px = (cam->W + 7) / 8, py = (cam->H + 7) / 8;
  hipLaunchKernelGGL(k_resolution, dim3((unsigned)(px * py)), dim3(64), 0, (hipStream_t)s, t->view, camera_view(*cam),
                     inv_w0, res, px);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, std::string("resolution launch failed: ") + hipGetErrorString(e));
}

amr_status amr_render_with_resolution(const amr_tree* t, const amr_camera* cam, amr_op op, const amr_render_opts* opts,
                                      float* out, float* aux, float* res, amr_stream s) {
  amr_status st = check_render_common(t, cam);
  if (st) return st;
  if (!out || !res) return fail(AMR_EINVAL, "null output");
  if (((uintptr_t)out & 3) || ((uintptr_t)aux & 3) || ((uintptr_t)res & 3)) return fail(AMR_EINVAL, "misaligned output");
  if (op != AMR_SUM && op != AMR_MAX && op != AMR_WMEAN) return fail(AMR_EINVAL, "bad op");
  const amr_render_opts o = opts ? *opts : amr_render_opts{0, 0, 0, -1};
  const int nf = t->info.nfields;
  const int los = op == AMR_WMEAN && o.los_velocity ? 1 : 0;
  if (o.field < 0 || o.field + (los ? 2 : 0) >= nf) return fail(AMR_EINVAL, "field index out of range");
  if (op == AMR_WMEAN && (o.weight_field < 0 || o.weight_field >= nf)) return fail(AMR_EINVAL, "bad weight field");
  float inv_w0;
  if (!inv_spacing(cam, &inv_w0)) return fail(AMR_EINVAL, "zero pixel step");
  const int px = (cam->W + 7) / 8, py = (cam->H + 7) / 8;
  const dim3 g((unsigned)(px * py));
  hipStream_t hs = (hipStream_t)s;
  const CameraView C = camera_view(*cam);
  if (op == AMR_SUM)
    hipLaunchKernelGGL(k_render_res<kOpSum>, g, dim3(64), 0, hs, t->view, C, o.field, o.weight_field, los, inv_w0,
                       out, aux, res, px);
  else if (op == AMR_MAX)
    hipLaunchKernelGGL(k_render_res<kOpMax>, g, dim3(64), 0, hs, t->view, C, o.field, o.weight_field, los, inv_w0,
                       out, aux, res, px);
  else
    hipLaunchKernelGGL(k_render_res<kOpWMean>, g, dim3(64), 0, hs, t->view, C, o.field, o.weight_field, los, inv_w0,
                       out, aux, res, px);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, std::string("render launch failed: ") + hipGetErrorString(e));
}

int64_t amr_blur_workspace_bytes(int32_t W, int32_t H) {
  if (W < 1 || H < 1) return 0;
  return kBlurLevels * align256((int64_t)W * H * 4);
}

amr_status amr_blur_adaptive(const float* img, const float* res, int32_t W, int32_t H, float kappa, float* out,
                             void* workspace, int64_t workspace_bytes, amr_stream s) {
  if (!img || !res || !out || !workspace) return fail(AMR_EINVAL, "null argument");
  if (W < 1 || H < 1 || W > 32768 || H > 32768) return fail(AMR_EINVAL, "bad image size");
  if (!(kappa >= 0.0f) || !std::isfinite(kappa)) return fail(AMR_EINVAL, "kappa must be finite and >= 0");
  if (((uintptr_t)img & 3) || ((uintptr_t)res & 3) || ((uintptr_t)out & 3) || ((uintptr_t)workspace & 255))
    return fail(AMR_EINVAL, "misaligned buffer");
  if (out == img) return fail(AMR_EINVAL, "out must not alias img");
  if (workspace_bytes < amr_blur_workspace_bytes(W, H)) return fail(AMR_ECAPACITY, "workspace too small");
  static const BlurLadder lad = make_ladder();
  static const bool radii_ok = [] {
    const int host_radius[kBlurLevels] = {2, 3, 3, 5, 6, 9, 12, 17, 24, 34, 48};
    for (int k = 0; k < kBlurLevels; ++k)
      if (lad.R[k] != host_radius[k]) return false;
    return true;
  }();
  if (!radii_ok) return fail(AMR_EINVAL, "blur ladder radii differ from the kernel's table");
  float* h = (float*)workspace;
  hipStream_t hs = (hipStream_t)s;
  hipLaunchKernelGGL(k_blur_rows, dim3((unsigned)((W + kRowTile - 1) / kRowTile), (unsigned)H), dim3(kRowTile), 0, hs,
                     img, W, H, lad, h);
  hipLaunchKernelGGL(k_blur_cols, dim3((unsigned)((W + 63) / 64), (unsigned)((H + 3) / 4)), dim3(256), 0, hs, img, res,
                     W, H, kappa, lad, h, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, std::string("blur launch failed: ") + hipGetErrorString(e));
}

amr_status amr_slice(const amr_tree* t, const amr_camera* cam, int32_t field, float* out, amr_stream s) {
  amr_status st = check_render_common(t, cam);
  if (st) return st;
  if (cam->kind != 1) return fail(AMR_EINVAL, "a slice takes an orthographic record");
  if (field < 0 || field >= t->info.nfields) return fail(AMR_EINVAL, "field index out of range");
  if (!out || ((uintptr_t)out & 3)) return fail(AMR_EINVAL, "null or misaligned output");
  const int px = (cam->W + 7) / 8, py = (cam->H + 7) / 8;
  hipLaunchKernelGGL(k_slice, dim3((unsigned)(px * py)), dim3(64), 0, (hipStream_t)s, t->view, camera_view(*cam), field,
                     out, px);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AMR_OK : fail(AMR_EHIP, std::string("slice launch failed: ") + hipGetErrorString(e));
}

}  // extern "C"
