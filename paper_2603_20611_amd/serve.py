"""Python handle of the library's slice server (continuous batching of slice
requests over volumes resident in HBM).  Marshalling only; the scheduler,
batching and rendering run in libgaussianpile."""
from __future__ import annotations

import ctypes as C

import torch

from . import binding as B


class Server:
    def __init__(self, **cfg):
        lib = B.load()
        self.cfg = B.ServerCfg()
        B.check(lib.gp_server_default_cfg(C.byref(self.cfg)))
        for k, v in cfg.items():
            if k == "opts":
                self.cfg.opts = v
            else:
                setattr(self.cfg, k, v)
        self._h = C.c_void_p()
        B.check(lib.gp_server_create(C.byref(self._h), C.byref(self.cfg)))

    def add_volume(self, params, n=None):
        """params: float32 CUDA tensor [11, stride]; copied into resident storage."""
        assert params.dtype == torch.float32 and params.is_cuda and params.is_contiguous()
        stride = params.shape[1]
        n = stride if n is None else n
        g = B.Gaussians(params.data_ptr(), params.data_ptr() + 3 * stride * 4, n, stride, B.GP_F32, B.GP_F32)
        vid = C.c_int32()
        B.check(B.load().gp_server_add_volume(self._h, C.byref(g), C.byref(vid)))
        return vid.value

    def submit(self, volume, z, sigma_z, out, width, height, x0=0.0, y0=0.0, dx=1.0, dy=1.0):
        """Queues a slice request; `out` (float32 CUDA, width*height) receives the image."""
        r = B.Request(int(volume), float(z), float(sigma_z), float(x0), float(y0), float(dx), float(dy),
                      int(width), int(height))
        t = C.c_uint64()
        B.check(B.load().gp_serve_submit(self._h, C.byref(r), C.c_void_p(out.data_ptr()), C.byref(t)))
        return t.value

    def submit_many(self, reqs, outs, t_arrival_ms=None):
        """Queues several requests in one call.  reqs: dicts with volume, z, sigma_z, width,
        height and optional x0, y0, dx, dy; outs: float32 CUDA tensors; t_arrival_ms: arrival
        times on the server's clock (clock_ms), or None for now.  Returns the tickets."""
        n = len(reqs)
        arr = (B.Request * max(n, 1))()
        for i, r in enumerate(reqs):
            arr[i] = B.Request(int(r["volume"]), float(r["z"]), float(r["sigma_z"]), float(r.get("x0", 0.0)),
                               float(r.get("y0", 0.0)), float(r.get("dx", 1.0)), float(r.get("dy", 1.0)),
                               int(r["width"]), int(r["height"]))
        ptrs = (C.c_void_p * max(n, 1))(*[o.data_ptr() for o in outs])
        tarr = None if t_arrival_ms is None else (C.c_double * max(n, 1))(*[float(t) for t in t_arrival_ms])
        tickets = (C.c_uint64 * max(n, 1))()
        B.check(B.load().gp_serve_submit_many(self._h, arr, ptrs, tarr, n, tickets))
        return list(tickets[:n])

    @staticmethod
    def clock_ms():
        """The server's clock (milliseconds, steady)."""
        return B.load().gp_clock_ms()

    def poll(self, ticket, timeout_us=-1):
        """Returns a ServeResult, or None while pending (GP_EAGAIN)."""
        res = B.ServeResult()
        st = B.load().gp_serve_poll(self._h, C.c_uint64(ticket), int(timeout_us), C.byref(res))
        if st == B.GP_EAGAIN:
            return None
        B.check(st)
        return res

    def stats(self):
        s = B.ServerStats()
        B.check(B.load().gp_server_stats_get(self._h, C.byref(s)))
        return s

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            B.load().gp_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
