"""Reconstruction loop: fitting a Focus-Gaussian set to a stack of slices.

The loop of Sec. 4.3 ("Optimization"), with the schedule of Sec. 5.1: each
iteration renders a batch of slices, takes the gradient of
L = mean |I - T| + lambda (1 - mean SSIM) (lambda = 0.2), runs the adjoint to
every Gaussian parameter and one Adam step (learning rates 6e-4 for positions,
2e-3 for log-scales, 1e-3 for quaternions, 2e-2 for intensities, decayed
exponentially to 0.1x over the run's nominal 30k iterations; intensities
projected onto alpha >= 0).  Every `densify_every` iterations between
`densify_from` and `densify_until` (Sec. 5.1: 500 to 25,000, every 100) the
statistics the backward accumulated drive the densify / prune pass.

Every step runs in the library's kernels (render, loss, backward, Adam,
densify / prune); this module only keeps the buffers and the schedule.  The
split children's noise is drawn on the device from a seeded generator and
handed to the kernel as input.

Slices of one batch are drawn at random (distinct, in depth order), or as a run
of consecutive slices at a random depth (`consecutive=True`).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import binding as B
from . import render

LR0 = (6e-4, 2e-3, 1e-3, 2e-2)      # positions, log-scales, quaternions, intensities
NOMINAL_ITERS = 30000


class Reconstruction:
    """State of one fit: parameters, Adam moments, gradient, densification
    statistics, the workspace and the target stack (all on the device).

    params: float32 [11, n] (numpy or tensor); target: float32 tensor of the
    stack's slices packed back to back (the slices all share one grid);
    slices: the stack's slice descriptors."""

    def __init__(self, params, target, slices, batch=8, lam=0.2, lr=LR0, total_iters=NOMINAL_ITERS,
                 densify_every=100, densify_from=500, densify_until=25000, grow_room=2.0,
                 consecutive=False, seed=0, densify_cfg=None, opts=None, device="cuda"):
        self.dev = torch.device(device)
        p = torch.as_tensor(params, dtype=torch.float32)
        self.n = int(p.shape[1])
        self.cap = self._round(int(self.n * grow_room) + 64)
        self.params = torch.zeros(11, self.cap, device=self.dev)
        self.params[:, :self.n] = p.to(self.dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.slices = list(slices)
        w0, h0 = int(self.slices[0]["width"]), int(self.slices[0]["height"])
        assert all(int(s["width"]) == w0 and int(s["height"]) == h0 for s in self.slices), "one grid per stack"
        self.W, self.H = w0, h0
        self.target = target.reshape(len(self.slices), self.H, self.W)
        self.batch = int(batch)
        self.lam = float(lam)
        self.lr0 = np.asarray(lr, np.float64)
        self.total_iters = int(total_iters)
        self.densify_every = int(densify_every)
        self.densify_from = int(densify_from)
        self.densify_until = int(densify_until)
        self.consecutive = bool(consecutive)
        self.rng = np.random.default_rng(seed)
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(seed)
        self.dcfg = densify_cfg if densify_cfg is not None else render.densify_cfg()
        self.opts = opts if opts is not None else B.default_opts()
        npix = self.batch * self.H * self.W
        self.img = torch.empty(npix, device=self.dev)
        self.gimg = torch.empty(npix, device=self.dev)
        self.tgt = torch.empty(npix, device=self.dev)
        self.loss = torch.zeros(2, device=self.dev)
        self.it = 0
        self.history = []        # (iteration, mean L1, mean D-SSIM, Gaussians)
        self._loss_from = 0
        self._new_stats()
        self.ws = None
        self._size_workspace()

    @staticmethod
    def _round(n):
        return (n + 63) // 64 * 64

    def _new_stats(self):
        self.st_norm = torch.zeros(self.cap, device=self.dev)
        self.st_count = torch.zeros(self.cap, dtype=torch.int32, device=self.dev)
        self.st_rad = torch.zeros(self.cap, device=self.dev)

    def _size_workspace(self):
        """A fixed-capacity workspace (no host synchronisation per render), sized at
        three times the lists of the deepest-populated batch among a few probes."""
        probe = render.Workspace()
        worst_r = worst_i = 0
        for k in np.linspace(0, len(self.slices) - self.batch, 5).astype(int):
            render.render(self.params, self.slices[k:k + self.batch], self.opts, probe, out=self.img, n=self.n)
            r, i, _ = probe.check()
            worst_r, worst_i = max(worst_r, r), max(worst_i, i)
        del probe
        if self.ws is not None:
            self.ws.close()
        self.ws = render.Workspace(capacity=(3 * worst_r + 65536, 3 * worst_i + 262144))
        self.ws.set_densify_stats(self.st_norm[:self.n], self.st_count[:self.n], self.st_rad[:self.n])

    def _pick(self):
        S = len(self.slices)
        if self.consecutive:
            k0 = int(self.rng.integers(0, S - self.batch + 1))
            return np.arange(k0, k0 + self.batch)
        return np.sort(self.rng.choice(S, self.batch, replace=False))

    def step(self):
        """One iteration (asynchronous: nothing is read back)."""
        idx = self._pick()
        batch = [self.slices[int(k)] for k in idx]
        torch.index_select(self.target, 0, torch.from_numpy(idx).to(self.dev),
                           out=self.tgt.view(self.batch, self.H, self.W))
        render.render(self.params, batch, self.opts, self.ws, out=self.img, n=self.n)
        render.l1_dssim_loss_grad(self.img, self.tgt, self.batch, self.W, self.H, self.ws, lam=self.lam,
                                  grad=self.gimg, loss=self.loss)
        render.render_backward(self.params, batch, self.gimg, self.ws, self.opts, grad=self.grad, n=self.n)
        lr = self.lr0 * 0.1 ** (self.it / self.total_iters)
        render.adam_step(self.params, self.grad, self.m, self.v, self.it + 1, lr, n=self.n,
                         flags=B.GP_ADAM_ZERO_GRAD | B.GP_ADAM_CLAMP_ALPHA)
        self.it += 1
        if (self.densify_every > 0 and self.densify_from <= self.it <= self.densify_until
                and self.it % self.densify_every == 0):
            self.densify()

    def densify(self):
        """Densify / prune from the statistics accumulated since the last pass
        (synchronises: the new count is read back)."""
        self.ws.check()          # every render since the last check fitted its workspace
        noise = torch.randn(6, self.n, device=self.dev, generator=self.gen)
        cap = max(self.cap, self._round(2 * self.n + 64))
        p, m, v, n_new = render.densify_prune(self.params, self.m, self.v, self.st_norm[:self.n],
                                              self.st_count[:self.n], self.st_rad[:self.n], noise,
                                              cfg=self.dcfg, n=self.n, capacity=cap)
        self.params, self.m, self.v = p, m, v
        self.cap = int(p.shape[1])
        self.n = int(n_new)
        self.grad = torch.zeros_like(self.params)
        self._new_stats()
        self._size_workspace()

    def take_loss(self):
        """Mean (L1, D-SSIM) since the last call (synchronises)."""
        l = self.loss.cpu().numpy().astype(np.float64)
        k = max(self.it - self._loss_from, 1)
        self.loss.zero_()
        self._loss_from = self.it
        return float(l[0]) / k, float(l[1]) / k

    def run(self, iters, log_every=100, log=None):
        """iters iterations; records (iteration, L1, D-SSIM, Gaussians) every log_every."""
        for _ in range(iters):
            self.step()
            if log_every and self.it % log_every == 0:
                l1, ds = self.take_loss()
                self.history.append((self.it, l1, ds, self.n))
                if log:
                    log(f"iter {self.it}: L1 {l1:.5f}  D-SSIM {ds:.5f}  Gaussians {self.n}")
        self.ws.check()

    def render_stack(self, chunk=16):
        """The whole stack rendered from the current set (float32 tensor [S, H, W])."""
        out = torch.empty(len(self.slices), self.H, self.W, device=self.dev)
        ws = render.Workspace()
        for k in range(0, len(self.slices), chunk):
            sl = self.slices[k:k + chunk]
            render.render(self.params, sl, self.opts, ws, out=out[k:k + len(sl)].reshape(-1), n=self.n)
        return out

    def psnr(self, reference, peak=None, chunk=16):
        """PSNR (dB) of the rendered stack against `reference` ([S, H, W] or flat),
        with the reference's maximum as the peak unless given."""
        ref = reference.reshape(len(self.slices), self.H, self.W)
        img = self.render_stack(chunk)
        mse = torch.mean((img.double() - ref.double()) ** 2).item()
        pk = float(ref.max().item()) if peak is None else float(peak)
        return 10.0 * math.log10(pk * pk / max(mse, 1e-300))


def timed_iterations(rec, iters):
    """Wall time per iteration of `iters` iterations (device-synchronised)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        rec.step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / iters
