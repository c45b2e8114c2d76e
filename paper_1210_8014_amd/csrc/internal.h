// internal.h -- library-private declarations shared by the host builder and
// the HIP kernels.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/amr.h"
#include "traverse.h"

struct amr_tree {
  amr::TreeView view;       // device (or host, when host_only) pointers
  amr_tree_info_t info;
  int32_t* d_child = nullptr;
  float* d_val = nullptr;
  uint8_t* d_maxdepth = nullptr;
  // host copies kept only for host_only trees
  std::vector<int32_t> h_child;
  std::vector<float> h_val;
  std::vector<uint8_t> h_maxdepth;
  std::vector<amr::Cell4> h_packed;  // fields 0..3 interleaved (nfields >= 4)
  amr::Cell4* d_packed = nullptr;
  std::vector<amr::ChildVal> h_cv;   // (first child, field 0) per cell
  amr::ChildVal* d_cv = nullptr;
  uint64_t serial = 0;      // unique id (batches detect freed trees)
  int32_t tuned_variant[3] = {-1, -1, -1};  // default kernel variant per op (-1: variant 0)
};

namespace amr {

void set_error(const std::string& msg);
amr_status fail(amr_status st, const std::string& msg);

CameraView camera_view(const amr_camera& c);

// Checks shared by every entry point that walks rays: a renderable tree
// and a camera record inside the integer ranges the kernels rely on (image
// size, maximum level, kind, origin and direction bounds, non-zero
// orthographic direction).  AMR_EINVAL with a message otherwise.
amr_status check_render_common(const amr_tree* t, const amr_camera* cam);
// The camera part of those checks alone.
amr_status check_camera(const amr_camera* cam);

struct RenderArgs {
  TreeView t;
  CameraView c;
  int32_t field, wfield, los, max_level;
  float* out;
  float* aux;
  int32_t packets_x, packets_y;
};

// Packet index of the b-th dispatched packet (b < px * py) when packet rows
// go out from the middle row of the image (middle, one above, one below,
// ...): the rays that cross the most cells usually look through the middle
// of the image, and started first their walks overlap the rest of the image
// instead of finishing alone at its end.
AMR_HD int center_out(int b, int px, int py) {
  const int k = b / px, x = b - k * px;
  const int row = py / 2 + ((k & 1) ? -((k + 1) >> 1) : (k >> 1));
  return row * px + x;
}

// Kernel launchers (render.hip).  Return a hipError_t as int.
int launch_render(int op, int variant, const RenderArgs& a, void* stream);
int launch_count_all(const TreeView& t, const CameraView& c, int32_t* counts, int64_t* total, void* stream);
int launch_mark(const TreeView& t, const CameraView& c, uint32_t* bits, int64_t* fresh, void* stream);
int launch_rays(const TreeView& t, const CameraView& c, const int64_t* ray_ids, int64_t n, const int64_t* offsets,
                int32_t* cells, int32_t* counts, void* stream);
int variant_count();
const char* variant_name(int v);
int variant_packet_width(int v);
int default_variant();  // the variant amr_render uses when none is chosen or tuned
// Trees whose camera maximum level lies this many levels or more below the
// complete base level are walked with an ancestor stack by default (most
// moves re-descend several levels there; the stack shortens them).
constexpr int kDeepSpan = 10;

// Live-tree registry (batch.hip): batches refuse to run on freed trees.
void register_tree(uint64_t serial);
void unregister_tree(uint64_t serial);

// HIP runtime wrappers (render.hip) so the host builder needs no HIP headers.
int dev_malloc(void** p, size_t bytes);
int dev_free(void* p);
int dev_upload(void* dst, const void* src, size_t bytes);
int dev_download(void* dst, const void* src, size_t bytes);
const char* dev_error_string(int err);

}  // namespace amr
