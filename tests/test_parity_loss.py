"""The L1 + D-SSIM slice loss on the GPU against the oracle.

Bars: the gradient within 1e-5 of the oracle's largest gradient magnitude and
the two loss terms within 1e-5 relative (the kernels work in float64 on the
same float32 inputs; the loss terms are summed with float32 atomics).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import ssim as ossim

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[loss] {msg}", flush=True)
    sys.stdout.flush()


def _check(x, y, lam, ws):
    from paper_2603_20611_amd import render as R
    S, H, W = x.shape
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda().reshape(-1)
    yt = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda().reshape(-1)
    loss = torch.zeros(2, device="cuda")
    g = R.l1_dssim_loss_grad(xt, yt, S, W, H, ws, lam=lam, loss=loss)
    torch.cuda.synchronize()
    _, l1, d, eg = ossim.loss(x.astype(np.float32), y.astype(np.float32), lam=lam)
    gg = g.cpu().numpy().reshape(S, H, W)
    err = np.abs(gg - eg).max() / max(np.abs(eg).max(), 1e-30)
    lo = loss.cpu().numpy()
    _say(f"S={S} {W}x{H} lam={lam}: grad err {err:.2e}, l1 {lo[0]:.6g}/{l1:.6g}, dssim {lo[1]:.6g}/{d:.6g}")
    assert err <= 1e-5
    assert lo[0] == pytest.approx(l1, rel=1e-5, abs=1e-7)
    assert lo[1] == pytest.approx(d, rel=1e-5, abs=1e-7)
    return gg


@pytest.mark.parametrize("shape", [(3, 45, 70), (1, 64, 64), (2, 17, 5), (1, 1, 1), (4, 33, 96)])
def test_loss_matches_oracle(gp, shape):
    from paper_2603_20611_amd import render as R
    rng = np.random.default_rng(sum(shape))
    x = rng.uniform(0, 1.5, size=shape)
    y = np.clip(x + rng.normal(0, 0.2, size=shape), 0, None)
    ws = R.Workspace()
    _check(x, y, 0.2, ws)
    ws.close()


def test_rendered_slices_and_smooth_regions(gp):
    from paper_2603_20611_amd import render as R, synth
    _say("rendered slices against a jittered target")
    p, _, tgt = synth.tiny(seed=3)
    slices = synth.axial_slices(3, 64, 64, 1.0, z0=10.5)
    ws = R.Workspace()
    x = R.render(torch.from_numpy(p).cuda(), slices, ws=ws).cpu().numpy().reshape(3, 64, 64)
    y = R.render(torch.from_numpy(tgt).cuda(), slices, ws=ws).cpu().numpy().reshape(3, 64, 64)
    _check(x.astype(np.float64), y.astype(np.float64), 0.2, ws)
    # constant and nearly constant slices: the moment form cancels hardest here
    c = np.full((2, 40, 40), 0.75)
    _check(c + 1e-4 * np.random.default_rng(9).normal(size=c.shape), c, 0.2, ws)
    ws.close()


def test_lambda_zero_is_l1_and_scratch_grows(gp):
    from paper_2603_20611_amd import render as R
    rng = np.random.default_rng(5)
    ws = R.Workspace()
    small = rng.uniform(size=(1, 20, 20))
    _check(small, rng.uniform(size=(1, 20, 20)), 0.0, ws)
    big = rng.uniform(size=(3, 130, 90))          # needs a larger scratch
    g = _check(big, rng.uniform(size=(3, 130, 90)), 0.0, ws)
    assert set(np.unique(np.abs(g) * big.size).round(6)) <= {0.0, 1.0}
    _check(small, rng.uniform(size=(1, 20, 20)), 0.2, ws)   # and a smaller one again
    ws.close()


def test_errors(gp):
    from paper_2603_20611_amd import binding as B, render as R
    ws = R.Workspace()
    x = torch.zeros(16, device="cuda")
    with pytest.raises(B.GpError):
        R.l1_dssim_loss_grad(x, x, 1, 4, 4, ws, lam=-1.0)
    with pytest.raises(B.GpError):
        R.l1_dssim_loss_grad(x, x, -1, 4, 4, ws)
    R.l1_dssim_loss_grad(x, x, 0, 4, 4, ws)   # empty batch: nothing to do
    ws.close()
