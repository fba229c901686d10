"""ctypes binding of libgaussianpile.so (the C-ABI in include/gaussianpile.h).

Argument marshalling only: every computation runs in the HIP library.  If the
library has not been built, load() raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import math
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgaussianpile.so")
_lib = None

GP_OK, GP_EINVAL, GP_ENOMEM, GP_EHIP, GP_EOVERFLOW, GP_EAGAIN, GP_ECANCELED, GP_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
GP_F32, GP_BF16, GP_F16, GP_Q16, GP_QM = 0, 1, 2, 3, 4
GP_FLAG_EXACT = 1
GP_FLAG_CONV_EXACT = 2
GP_FLAG_FORWARD_ONLY = 4
GP_ADAM_CLAMP_ALPHA, GP_ADAM_ZERO_GRAD = 1, 2
STAGES = ("preprocess", "emit", "sort", "raster_fwd", "raster_bwd", "preprocess_bwd")
STATUS_NAMES = {0: "GP_OK", -1: "GP_EINVAL", -2: "GP_ENOMEM", -3: "GP_EHIP", -4: "GP_EOVERFLOW",
                -5: "GP_EAGAIN", -6: "GP_ECANCELED", -7: "GP_ESTATE"}


class GpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class RenderOpts(C.Structure):
    _fields_ = [("q_cut", C.c_float), ("bbox_sigmas", C.c_float), ("scale_mod", C.c_float),
                ("flags", C.c_uint32)]


class Gaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("attrs", C.c_void_p), ("n", C.c_int64), ("stride", C.c_int64),
                ("mean_dtype", C.c_int32), ("attr_dtype", C.c_int32)]


class Slice(C.Structure):
    _fields_ = [("z", C.c_float), ("sigma_z", C.c_float), ("x0", C.c_float), ("y0", C.c_float),
                ("dx", C.c_float), ("dy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class AdamCfg(C.Structure):
    _fields_ = [("lr", C.c_float * 4), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int32), ("flags", C.c_uint32)]


class VolumeGrid(C.Structure):
    _fields_ = [("x0", C.c_float), ("y0", C.c_float), ("z0", C.c_float), ("dx", C.c_float), ("dy", C.c_float),
                ("dz", C.c_float), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad", C.c_int32)]


def make_grid(grid):
    """VolumeGrid from a dict with nx, ny, nz and optional x0, y0, z0, dx, dy, dz."""
    return VolumeGrid(float(grid.get("x0", 0.0)), float(grid.get("y0", 0.0)), float(grid.get("z0", 0.0)),
                      float(grid.get("dx", 1.0)), float(grid.get("dy", 1.0)), float(grid.get("dz", 1.0)),
                      int(grid["nx"]), int(grid["ny"]), int(grid["nz"]), 0)


class DensifyCfg(C.Structure):
    _fields_ = [("grad_threshold", C.c_float), ("min_alpha", C.c_float), ("max_radius", C.c_float),
                ("split_scale", C.c_float), ("split_factor", C.c_float), ("flags", C.c_uint32)]


class ServerCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_gaussians", C.c_int64), ("max_records", C.c_int64),
                ("max_instances", C.c_int64), ("max_bins", C.c_int32), ("max_batch", C.c_int32),
                ("slots", C.c_int32), ("attr_dtype", C.c_int32), ("use_graphs", C.c_int32),
                ("device", C.c_int32), ("opts", RenderOpts)]


class Request(C.Structure):
    _fields_ = [("volume_id", C.c_int32), ("z", C.c_float), ("sigma_z", C.c_float), ("x0", C.c_float),
                ("y0", C.c_float), ("dx", C.c_float), ("dy", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32)]


class ServeResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("batch_size", C.c_int32), ("batch_id", C.c_int64),
                ("latency_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("retries", C.c_int64), ("resident_bytes", C.c_int64), ("volumes", C.c_int32),
                ("pad", C.c_int32)]


_P = C.c_void_p
_SIGS = {
    "gp_version": (C.c_int32, []),
    "gp_last_error": (C.c_char_p, []),
    "gp_default_opts": (C.c_int32, [C.POINTER(RenderOpts)]),
    "gp_workspace_create": (C.c_int32, [C.POINTER(_P), C.c_int64, C.c_int64]),
    "gp_workspace_destroy": (C.c_int32, [_P]),
    "gp_workspace_check": (C.c_int32, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "gp_render_slices": (C.c_int32, [_P, C.POINTER(Gaussians), C.POINTER(Slice), C.c_int32,
                                     C.POINTER(RenderOpts), _P, _P]),
    "gp_render_backward": (C.c_int32, [_P, C.POINTER(Gaussians), C.POINTER(Slice), C.c_int32,
                                       C.POINTER(RenderOpts), _P, _P, C.c_int64, _P]),
    "gp_render_slices_posed": (C.c_int32, [_P, C.POINTER(Gaussians), C.POINTER(Slice), C.POINTER(C.c_float),
                                           C.c_int32, C.POINTER(RenderOpts), _P, _P]),
    "gp_render_backward_posed": (C.c_int32, [_P, C.POINTER(Gaussians), C.POINTER(Slice), C.POINTER(C.c_float),
                                             C.c_int32, C.POINTER(RenderOpts), _P, _P, C.c_int64, _P]),
    "gp_l1_loss_grad": (C.c_int32, [_P, _P, C.c_int64, C.c_float, _P, _P, _P]),
    "gp_adam_step": (C.c_int32, [_P, _P, _P, _P, C.c_int64, C.c_int64, C.POINTER(AdamCfg), _P]),
    "gp_workspace_set_timing": (C.c_int32, [_P, C.c_int32]),
    "gp_workspace_timings": (C.c_int32, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]),
    "gp_encode": (C.c_int32, [_P, C.c_int64, C.c_int64, _P, C.c_int64, _P, _P, _P]),
    "gp_voxelize": (C.c_int32, [_P, C.POINTER(Gaussians), C.POINTER(VolumeGrid), C.POINTER(RenderOpts), _P, _P]),
    "gp_voxelize_backward": (C.c_int32, [_P, C.POINTER(Gaussians), C.POINTER(VolumeGrid), C.POINTER(RenderOpts),
                                         _P, _P, C.c_int64, _P]),
    "gp_l1_dssim_loss_grad": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_float, _P, _P, _P]),
    "gp_l1_dssim_loss_grad_noalloc": (C.c_int32, [_P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_float, _P, _P, _P]),
    "gp_densify_default_cfg": (C.c_int32, [C.POINTER(DensifyCfg)]),
    "gp_workspace_set_densify_stats": (C.c_int32, [_P, _P, _P, _P, C.c_int64]),
    "gp_densify_prune": (C.c_int32, [_P, _P, _P, C.c_int64, C.c_int64, _P, _P, _P, _P, C.POINTER(DensifyCfg),
                                     _P, _P, _P, C.c_int64, C.POINTER(C.c_int64), _P]),
    "gp_server_default_cfg": (C.c_int32, [C.POINTER(ServerCfg)]),
    "gp_server_create": (C.c_int32, [C.POINTER(_P), C.POINTER(ServerCfg)]),
    "gp_server_add_volume": (C.c_int32, [_P, C.POINTER(Gaussians), C.POINTER(C.c_int32)]),
    "gp_serve_submit": (C.c_int32, [_P, C.POINTER(Request), _P, C.POINTER(C.c_uint64)]),
    "gp_serve_submit_many": (C.c_int32, [_P, C.POINTER(Request), C.POINTER(_P), C.POINTER(C.c_double), C.c_int32,
                                         C.POINTER(C.c_uint64)]),
    "gp_clock_ms": (C.c_double, []),
    "gp_serve_poll": (C.c_int32, [_P, C.c_uint64, C.c_int32, C.POINTER(ServeResult)]),
    "gp_server_stats_get": (C.c_int32, [_P, C.POINTER(ServerStats)]),
    "gp_server_destroy": (C.c_int32, [_P]),
    "gp_debug_export_bins": (C.c_int32, [_P, C.POINTER(C.c_uint64), C.c_int64, C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64), C.c_int64]),
}


def exported_names():
    """Names the binding expects the library to export."""
    return sorted(_SIGS)


def load(path=None):
    """Loads the HIP library (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or _LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2603_20611_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != GP_OK:
        raise GpError(status, load().gp_last_error().decode())
    return status


def make_poses(slices):
    """Host array [n][12] (R_c row-major, t) of the slices' "pose" entries, identity where a
    slice has none; None if no slice has a pose (axial batch)."""
    if not any(s.get("pose") is not None for s in slices):
        return None
    flat = []
    for s in slices:
        p = s.get("pose")
        flat.extend([float(x) for x in (p if p is not None else (1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0))])
    return (C.c_float * len(flat))(*flat)


def default_opts(**kw):
    o = RenderOpts()
    check(load().gp_default_opts(C.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def make_slices(slices):
    arr = (Slice * max(len(slices), 1))()
    for i, s in enumerate(slices):
        arr[i] = Slice(float(s["z"]), float(s["sigma_z"]), float(s.get("x0", 0.0)), float(s.get("y0", 0.0)),
                       float(s.get("dx", 1.0)), float(s.get("dy", 1.0)), int(s["width"]), int(s["height"]))
    return arr


def q_cut_default():
    return float(2.0 * math.log(255.0))
