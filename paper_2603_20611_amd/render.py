"""Torch-facing wrappers of the HIP library: workspaces, the differentiable
renderer (a torch.autograd.Function whose backward is the library's hand-written
adjoint), fused Adam and the L1 loss.  PyTorch provides device memory and the
stream; every step runs in the library's kernels.

Gaussian parameters are a float32 CUDA tensor of shape [11, stride] (rows
mu_x, mu_y, mu_z, l_x, l_y, l_z, q_w, q_x, q_y, q_z, alpha); the first n
columns are the Gaussians.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as B


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Workspace:
    """Library-owned scratch for tile lists.  capacity=(records, instances) fixes the
    buffers (no host synchronisation per render); None sizes them automatically."""

    def __init__(self, capacity=None):
        lib = B.load()
        self._h = C.c_void_p()
        rec, inst = capacity if capacity else (0, 0)
        B.check(lib.gp_workspace_create(C.byref(self._h), int(rec), int(inst)))

    @property
    def handle(self):
        return self._h

    def check(self):
        """(records, instances, bins) of the last render; raises GpError on overflow."""
        r, i, b = C.c_int64(), C.c_int64(), C.c_int64()
        B.check(B.load().gp_workspace_check(self._h, C.byref(r), C.byref(i), C.byref(b)))
        return r.value, i.value, b.value

    def set_timing(self, enable=True, stages=None):
        """Per-stage event timing on (all stages, or the named ones in `stages`) or off."""
        mask = 0
        if enable:
            names = B.STAGES if stages is None else stages
            for name in names:
                mask |= 1 << B.STAGES.index(name)
        B.check(B.load().gp_workspace_set_timing(self._h, mask))

    def timings(self):
        """{stage: (milliseconds summed, launches)} since timing was enabled (synchronises)."""
        n = len(B.STAGES)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        B.check(B.load().gp_workspace_timings(self._h, ms, cnt, n))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(B.STAGES)}

    def set_densify_stats(self, grad_norm=None, count=None, max_radius=None):
        """Accumulate densification statistics in every later backward (None disables).
        grad_norm, max_radius: float32 [n]; count: int32 [n] (all on the device)."""
        self._stats = (grad_norm, count, max_radius)      # keep them alive
        n = grad_norm.numel() if grad_norm is not None else 0
        B.check(B.load().gp_workspace_set_densify_stats(self._h, _ptr(grad_norm), _ptr(count),
                                                         _ptr(max_radius), n))

    def export_bins(self, n_bins, max_keys):
        keys = np.zeros(max(max_keys, 1), np.uint64)
        ranges = np.zeros(2 * max(n_bins, 1), np.int64)
        n = C.c_int64()
        B.check(B.load().gp_debug_export_bins(self._h, keys.ctypes.data_as(C.POINTER(C.c_uint64)), keys.size,
                                              C.byref(n), ranges.ctypes.data_as(C.POINTER(C.c_int64)),
                                              ranges.size))
        return keys[: n.value].astype(np.int64), ranges.reshape(-1, 2)[:n_bins]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            B.load().gp_workspace_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gaussians_struct(params, n=None, attrs=None, attr_dtype=B.GP_F32):
    """gp_gaussians for a [11, stride] float32 tensor (or float32 means [3, stride] plus
    16-bit attrs [8, stride])."""
    if attrs is None:
        assert params.dtype == torch.float32 and params.is_cuda and params.is_contiguous()
        stride = params.shape[1]
        n = stride if n is None else n
        g = B.Gaussians(params.data_ptr(), params.data_ptr() + 3 * stride * 4, n, stride, B.GP_F32, B.GP_F32)
    else:
        stride = params.shape[1]
        assert attrs.shape[1] == stride and attrs.is_contiguous() and params.is_contiguous()
        n = stride if n is None else n
        g = B.Gaussians(params.data_ptr(), attrs.data_ptr(), n, stride, B.GP_F32, attr_dtype)
    return g


def slice_pixels(slices):
    return sum(int(s["width"]) * int(s["height"]) for s in slices)


def render(params, slices, opts=None, ws=None, out=None, n=None, attrs=None, attr_dtype=B.GP_F32):
    """Forward render; returns the packed float32 images (1-D tensor)."""
    lib = B.load()
    ws = ws or Workspace()
    opts = opts or B.default_opts()
    sl = B.make_slices(slices)
    if out is None:
        out = torch.empty(slice_pixels(slices), device=params.device, dtype=torch.float32)
    g = gaussians_struct(params, n, attrs, attr_dtype)
    poses = B.make_poses(slices)
    if poses is None:
        B.check(lib.gp_render_slices(ws.handle, C.byref(g), sl, len(slices), C.byref(opts), _ptr(out), _stream()))
    else:
        B.check(lib.gp_render_slices_posed(ws.handle, C.byref(g), sl, poses, len(slices), C.byref(opts), _ptr(out),
                                           _stream()))
    return out


def render_backward(params, slices, grad_out, ws, opts=None, grad=None, n=None):
    lib = B.load()
    opts = opts or B.default_opts()
    sl = B.make_slices(slices)
    if grad is None:
        grad = torch.zeros_like(params)
    g = gaussians_struct(params, n)
    poses = B.make_poses(slices)
    if poses is None:
        B.check(lib.gp_render_backward(ws.handle, C.byref(g), sl, len(slices), C.byref(opts),
                                       _ptr(grad_out.contiguous()), _ptr(grad), grad.shape[1], _stream()))
    else:
        B.check(lib.gp_render_backward_posed(ws.handle, C.byref(g), sl, poses, len(slices), C.byref(opts),
                                             _ptr(grad_out.contiguous()), _ptr(grad), grad.shape[1], _stream()))
    return grad


class FocusRender(torch.autograd.Function):
    """I = render(params, slices); backward by the library's adjoint (recomputes the
    per-pixel contributions from the forward's tile lists)."""

    @staticmethod
    def forward(ctx, params, slices, opts, ws):
        out = render(params, slices, opts, ws)
        ctx.slices, ctx.opts, ctx.ws = slices, opts, ws
        ctx.save_for_backward(params)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (params,) = ctx.saved_tensors
        grad = render_backward(params, ctx.slices, grad_out, ctx.ws, ctx.opts)
        return grad, None, None, None


def focus_render(params, slices, opts=None, ws=None):
    return FocusRender.apply(params, slices, opts or B.default_opts(), ws or Workspace())


def l1_loss_grad(image, target, grad=None, loss=None, scale=None):
    lib = B.load()
    n = image.numel()
    grad = torch.empty_like(image) if grad is None else grad
    scale = 1.0 / n if scale is None else scale
    B.check(lib.gp_l1_loss_grad(_ptr(image), _ptr(target), n, float(scale), _ptr(grad), _ptr(loss), _stream()))
    return grad


def l1_dssim_loss_grad(image, target, n_slices, width, height, ws, lam=0.2, grad=None, loss=None):
    """dL/dI of L = mean|I - T| + lam (1 - mean SSIM) over [n_slices, height, width] packed slices.
    loss, if given, is a float32 [2] device tensor: += (L1 term, D-SSIM term)."""
    if grad is None:
        grad = torch.empty_like(image)
    B.check(B.load().gp_l1_dssim_loss_grad(ws.handle, _ptr(image), _ptr(target), int(n_slices), int(width),
                                            int(height), float(lam), _ptr(grad), _ptr(loss), _stream()))
    return grad


def l1_dssim_loss_grad_noalloc(image, target, n_slices, width, height, lam=0.2, grad=None, loss=None):
    """As l1_dssim_loss_grad, through the library's allocation-free entry point (its
    scratch is a static device array shared by all calls on the GPU)."""
    if grad is None:
        grad = torch.empty_like(image)
    B.check(B.load().gp_l1_dssim_loss_grad_noalloc(_ptr(image), _ptr(target), int(n_slices), int(width),
                                                    int(height), float(lam), _ptr(grad), _ptr(loss), _stream()))
    return grad


def adam_step(params, grad, m, v, step, lr, betas=(0.9, 0.999), eps=1e-15, n=None, flags=0):
    """lr: (mean, log_scale, quat, alpha) learning rates."""
    lib = B.load()
    cfg = B.AdamCfg((C.c_float * 4)(*[float(x) for x in lr]), betas[0], betas[1], eps, int(step), int(flags))
    stride = params.shape[1]
    n = stride if n is None else n
    B.check(lib.gp_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), n, stride, C.byref(cfg), _stream()))


def densify_cfg(**kw):
    """gp_densify_cfg with the library's defaults, overridden by kw."""
    c = B.DensifyCfg()
    B.check(B.load().gp_densify_default_cfg(C.byref(c)))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def densify_prune(params, m, v, grad_norm, count, max_radius, noise, cfg=None, n=None, capacity=None):
    """Densify and prune; returns (params, m, v, n_new) as new [11, capacity] tensors.

    noise: float32 [6, n] (two 3-vectors per Gaussian for split children)."""
    n = params.shape[1] if n is None else int(n)
    cap = capacity if capacity is not None else 2 * n
    cfg = cfg if cfg is not None else densify_cfg()
    dev = params.device
    po = torch.empty(11, max(cap, 1), device=dev)
    mo = torch.empty_like(po)
    vo = torch.empty_like(po)
    n_out = C.c_int64()
    B.check(B.load().gp_densify_prune(_ptr(params), _ptr(m), _ptr(v), n, params.stride(0), _ptr(grad_norm),
                                      _ptr(count), _ptr(max_radius), _ptr(noise), C.byref(cfg), _ptr(po),
                                      _ptr(mo), _ptr(vo), po.stride(0), C.byref(n_out), _stream()))
    return po, mo, vo, n_out.value


def voxelize(params, grid, ws, opts=None, out=None, n=None, attrs=None, attr_dtype=B.GP_F32):
    """Intensity volume [nz * ny * nx] (flat float32) of the Gaussians on a voxel grid
    (dict with nx, ny, nz and optional x0, y0, z0, dx, dy, dz)."""
    g = B.make_grid(grid)
    opts = opts or B.default_opts()
    if out is None:
        out = torch.empty(g.nx * g.ny * g.nz, device=params.device, dtype=torch.float32)
    gs = gaussians_struct(params, n, attrs, attr_dtype)
    B.check(B.load().gp_voxelize(ws.handle, C.byref(gs), C.byref(g), C.byref(opts), _ptr(out), _stream()))
    return out


def voxelize_backward(params, grid, grad_volume, ws, opts=None, grad=None, n=None, attrs=None,
                      attr_dtype=B.GP_F32):
    """Adds dL/dparams of L = sum grad_volume * V into grad ([11, stride]; created if None)."""
    g = B.make_grid(grid)
    opts = opts or B.default_opts()
    if grad is None:
        grad = torch.zeros_like(params)
    gs = gaussians_struct(params, n, attrs, attr_dtype)
    B.check(B.load().gp_voxelize_backward(ws.handle, C.byref(gs), C.byref(g), C.byref(opts), _ptr(grad_volume),
                                          _ptr(grad), grad.stride(0), _stream()))
    return grad


def encode(params, n=None, stride_out=None):
    """Morton-ordered 14/12-bit codes of a [11, stride] float32 set.

    Returns (codes uint16 [11, stride_out] as int16-typed storage, header float32 [9],
    perm int32 [n]) on the device; codes[:, i] codes Gaussian perm[i]."""
    n = params.shape[1] if n is None else int(n)
    so = max(n, 1) if stride_out is None else int(stride_out)
    codes = torch.empty(11, so, dtype=torch.int16, device=params.device)
    header = torch.zeros(9, dtype=torch.float32, device=params.device)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=params.device)
    B.check(B.load().gp_encode(_ptr(params), n, params.stride(0), _ptr(codes), codes.stride(0), _ptr(perm),
                               _ptr(header), _stream()))
    return codes, header, perm[:n]


def coded_struct(codes, header, n):
    """gp_gaussians of a coded set (GP_QM)."""
    return B.Gaussians(codes.data_ptr(), header.data_ptr(), int(n), codes.shape[1], B.GP_QM, B.GP_QM)


def render_coded(codes, header, n, slices, opts=None, ws=None, out=None):
    """Forward render of a coded set."""
    lib = B.load()
    ws = ws or Workspace()
    opts = opts or B.default_opts()
    sl = B.make_slices(slices)
    if out is None:
        out = torch.empty(slice_pixels(slices), device=codes.device, dtype=torch.float32)
    g = coded_struct(codes, header, n)
    B.check(lib.gp_render_slices(ws.handle, C.byref(g), sl, len(slices), C.byref(opts), _ptr(out), _stream()))
    return out
