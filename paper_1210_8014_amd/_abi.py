"""ctypes mirror of include/amr.h (structs, enums and signatures)."""
import ctypes

AMR_OK, AMR_EINVAL, AMR_ETREE, AMR_ENOMEM, AMR_EHIP, AMR_ECAPACITY, AMR_ESTALE, AMR_EMODEL = range(8)
STATUS_NAMES = {0: "AMR_OK", 1: "AMR_EINVAL", 2: "AMR_ETREE", 3: "AMR_ENOMEM", 4: "AMR_EHIP", 5: "AMR_ECAPACITY",
                6: "AMR_ESTALE", 7: "AMR_EMODEL"}
AMR_SUM, AMR_MAX, AMR_WMEAN = 0, 1, 2
AMR_HOST, AMR_DEVICE = 0, 1

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class LeavesC(ctypes.Structure):
    _fields_ = [("n", _i64), ("level", _vp), ("ix", _vp), ("iy", _vp), ("iz", _vp), ("fields", _vp),
                ("nfields", _i32), ("location", _i32), ("field_stride", _i64)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("restrict_weight", _i32 * 8), ("use_defaults", _i32), ("host_only", _i32)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("ncells", _i64), ("nleaves", _i64), ("nfields", _i32), ("lmax", _i32), ("levelmin", _i32),
                ("host_only", _i32), ("cells_per_level", _i64 * 25), ("level_offset", _i64 * 26),
                ("device_bytes", _i64)]


class CameraDesc(ctypes.Structure):
    _fields_ = [("kind", _i32), ("W", _i32), ("H", _i32), ("max_level", _i32), ("level_bias", _i32),
                ("pad_", _i32), ("eye", ctypes.c_double * 3), ("target", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("fov_y", ctypes.c_double), ("ortho_height", ctypes.c_double)]


class Camera(ctypes.Structure):
    _fields_ = [("kind", _i32), ("W", _i32), ("H", _i32), ("max_level", _i32), ("O", _i64 * 3), ("F", _i64 * 3),
                ("U", _i64 * 3), ("V", _i64 * 3)]

    def as_dict(self):
        return dict(kind=self.kind, W=self.W, H=self.H, max_level=self.max_level, O=list(self.O), F=list(self.F),
                    U=list(self.U), V=list(self.V))


class RenderOpts(ctypes.Structure):
    _fields_ = [("field", _i32), ("weight_field", _i32), ("los_velocity", _i32), ("variant", _i32)]


class StreamOpts(ctypes.Structure):
    _fields_ = [("max_chunk_cells", _i64), ("host_only", _i32), ("nbuffers", _i32)]


class StreamPlanInfo(ctypes.Structure):
    _fields_ = [("nchunks", _i32), ("min_chunk_level", _i32), ("max_chunk_level", _i32), ("nbuffers", _i32),
                ("max_chunk_cells", _i64), ("largest_chunk", _i64), ("cells", _i64), ("host_bytes", _i64),
                ("device_bytes", _i64)]


class StreamChunk(ctypes.Structure):
    _fields_ = [("level", _i32), ("ix", _i32), ("iy", _i32), ("iz", _i32), ("ncells", _i64), ("first", _i64),
                ("level_start", _i64 * 26), ("off_local", _i32 * 26), ("records", _vp), ("values", _vp),
                ("packed", _vp)]


# name -> (restype, argtypes)
SIGNATURES = {
    "amr_last_error": (ctypes.c_char_p, []),
    "amr_build_linear_octree": (_i32, [ctypes.POINTER(LeavesC), ctypes.POINTER(BuildOpts), _vp,
                                       ctypes.POINTER(_vp)]),
    "amr_tree_free": (None, [_vp]),
    "amr_tree_info": (_i32, [_vp, ctypes.POINTER(TreeInfo)]),
    "amr_tree_arrays": (_i32, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "amr_set_camera": (_i32, [ctypes.POINTER(CameraDesc), _vp, ctypes.POINTER(Camera)]),
    "amr_render": (_i32, [_vp, ctypes.POINTER(Camera), _i32, ctypes.POINTER(RenderOpts), _vp, _vp, _vp]),
    "amr_variant_count": (_i32, []),
    "amr_variant_default": (_i32, []),
    "amr_variant_name": (ctypes.c_char_p, [_i32]),
    "amr_count_segments": (_i32, [_vp, ctypes.POINTER(Camera), _vp, _vp, _vp]),
    "amr_trace_rays": (_i32, [_vp, ctypes.POINTER(Camera), _vp, _i64, _vp, _vp, _vp]),
    "amr_count_rays": (_i32, [_vp, ctypes.POINTER(Camera), _vp, _i64, _vp, _vp]),
    "amr_mark_cells": (_i32, [_vp, ctypes.POINTER(Camera), _vp, _vp, _vp]),
    "amr_render_resolution": (_i32, [_vp, ctypes.POINTER(Camera), _vp, _vp]),
    "amr_render_with_resolution": (_i32, [_vp, ctypes.POINTER(Camera), _i32, ctypes.POINTER(RenderOpts), _vp, _vp, _vp,
                                          _vp]),
    "amr_blur_workspace_bytes": (_i64, [_i32, _i32]),
    "amr_blur_adaptive": (_i32, [_vp, _vp, _i32, _i32, ctypes.c_float, _vp, _vp, _i64, _vp]),
    "amr_slice": (_i32, [_vp, ctypes.POINTER(Camera), _i32, _vp, _vp]),
    "amr_batch_create": (_i32, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(Camera), _i32, ctypes.POINTER(_i32), _i32,
                                _i32, ctypes.POINTER(RenderOpts), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                ctypes.POINTER(_vp)]),
    "amr_render_batch": (_i32, [_vp, _vp]),
    "amr_batch_free": (None, [_vp]),
    "amr_batch_config_count": (_i32, []),
    "amr_batch_config_name": (ctypes.c_char_p, [_i32]),
    "amr_batch_config": (_i32, [_vp]),
    "amr_batch_set_config": (_i32, [_vp, _i32]),
    "amr_batch_tune": (_i32, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float)]),
    "amr_tune": (_i32, [_vp, ctypes.POINTER(Camera), _i32, ctypes.POINTER(RenderOpts), _vp, _vp, _vp, _i32,
                        ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float)]),
    "amr_set_default_variant": (_i32, [_vp, _i32, _i32]),
    "amr_stream_plan_create": (_i32, [_vp, ctypes.POINTER(StreamOpts), ctypes.POINTER(_vp)]),
    "amr_stream_plan_free": (None, [_vp]),
    "amr_stream_plan_info": (_i32, [_vp, ctypes.POINTER(StreamPlanInfo)]),
    "amr_stream_chunk": (_i32, [_vp, _i32, ctypes.POINTER(StreamChunk)]),
    "amr_stream_chunk_rect": (_i32, [_vp, _i32, ctypes.POINTER(Camera), ctypes.POINTER(_i32)]),
    "amr_stream_workspace_bytes": (_i64, [_i32, _i32]),
    "amr_render_streamed": (_i32, [_vp, ctypes.POINTER(Camera), _i32, ctypes.POINTER(RenderOpts), _vp, _vp, _vp,
                                   _i64, ctypes.POINTER(_i64), _vp]),
}


def declare(lib):
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib
