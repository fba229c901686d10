"""Densification statistics and densify/prune on the GPU against the oracle.

Bars: record counts bit-exact; gradient-norm statistics within 1e-4 relative
(the gradient bar) and radii within 1e-5; densify/prune decisions identical
(inputs kept away from every threshold so that both sides' binary32 decisions
agree), kept columns and moments bit-exact, split children within 1e-5.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import densify as odens
from paper_2603_20611_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[densify] {msg}", flush=True)
    sys.stdout.flush()


CFG = dict(grad_threshold=5e-5, min_alpha=0.02, max_radius=40.0, split_scale=2.0, split_factor=1.6)


def test_backward_statistics_match_oracle(gp):
    from paper_2603_20611_amd import render as R
    _say("statistics accumulated by the backward")
    extent = (96.0, 80.0, 12.0)
    p = synth.gaussians_microscopy(1500, extent, seed=5)
    slices = synth.axial_slices(3, 96, 80, 1.5, z0=4.0, dz=2.5)
    rng = np.random.default_rng(2)
    weights = [rng.normal(size=(sl["height"], sl["width"])).astype(np.float32) for sl in slices]
    n = p.shape[1]
    pt = torch.from_numpy(p).cuda().contiguous()
    gn = torch.zeros(n, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    rad = torch.zeros(n, device="cuda")
    ws = R.Workspace()
    ws.set_densify_stats(gn, cnt, rad)
    R.render(pt, slices, ws=ws)
    go = torch.from_numpy(np.concatenate([w.reshape(-1) for w in weights])).cuda()
    grad = torch.zeros_like(pt)
    R.render_backward(pt, slices, go, ws, grad=grad)
    torch.cuda.synchronize()
    ws.set_densify_stats()
    e_gn, e_cnt, e_rad = odens.stats(p, slices, weights)
    assert np.array_equal(cnt.cpu().numpy(), e_cnt)
    g = gn.cpu().numpy()
    assert np.abs(g - e_gn).max() <= 1e-4 * np.abs(e_gn).max()
    assert np.abs(rad.cpu().numpy() - e_rad).max() <= 1e-5 * np.abs(e_rad).max()
    ws.close()


def _synthetic_state(n, seed):
    rng = np.random.default_rng(seed)
    p = synth.gaussians_microscopy(n, (64.0, 64.0, 16.0), seed=seed)
    # alphas away from min_alpha, largest scales away from split_scale
    p[10] = np.where(rng.uniform(size=n) < 0.2, 0.01, rng.uniform(0.05, 1.0, n)).astype(np.float32)
    lmax = p[3:6].max(axis=0)
    p[3:6] += np.where(np.abs(np.exp(lmax) - CFG["split_scale"]) < 0.05, 0.1, 0.0).astype(np.float32)
    if n > 10:
        p[0, rng.integers(0, n, 3)] = np.nan
    m = rng.normal(size=(11, n)).astype(np.float32)
    v = rng.uniform(size=(11, n)).astype(np.float32)
    cnt = rng.integers(0, 12, n).astype(np.int32)
    mean = np.where(rng.uniform(size=n) < 0.4, rng.uniform(1e-4, 1e-3, n), rng.uniform(0, 2e-5, n))
    gn = (mean * cnt).astype(np.float32)
    rad = np.where(rng.uniform(size=n) < 0.1, 80.0, rng.uniform(0.5, 30.0, n)).astype(np.float32)
    noise = rng.normal(size=(6, n)).astype(np.float32)
    return p, m, v, gn, cnt, rad, noise


@pytest.mark.parametrize("n", [1, 777, 20000])
def test_densify_prune_matches_oracle(gp, n):
    from paper_2603_20611_amd import render as R
    _say(f"densify/prune n={n}")
    p, m, v, gn, cnt, rad, noise = _synthetic_state(n, seed=n)
    e_p, e_m, e_v, act = odens.densify_prune(p, m, v, gn, cnt, rad, noise, CFG)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    po, mo, vo, n_new = R.densify_prune(cu(p), cu(m), cu(v), cu(gn), cu(cnt), cu(rad), cu(noise),
                                        cfg=R.densify_cfg(**CFG))
    torch.cuda.synchronize()
    assert n_new == e_p.shape[1]
    g_p = po[:, :n_new].cpu().numpy().astype(np.float64)
    g_m = mo[:, :n_new].cpu().numpy().astype(np.float64)
    g_v = vo[:, :n_new].cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(g_m, e_m.astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(g_v, e_v.astype(np.float32).astype(np.float64))
    if n_new:
        err = np.abs(g_p - e_p) / np.maximum(np.abs(e_p), 1.0)
        assert err.max() <= 1e-5
    # columns that are not split children are copied bit for bit
    split_cols = np.repeat(act == odens.SPLIT, np.where(act == odens.DROP, 0, np.where(act == odens.KEEP, 1, 2)))
    np.testing.assert_array_equal(g_p[:, ~split_cols], e_p[:, ~split_cols])


def test_densify_overflow_and_empty(gp):
    from paper_2603_20611_amd import binding as B, render as R
    _say("densify overflow and empty input")
    p, m, v, gn, cnt, rad, noise = _synthetic_state(500, seed=9)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    with pytest.raises(B.GpError) as e:
        R.densify_prune(cu(p), cu(m), cu(v), cu(gn), cu(cnt), cu(rad), cu(noise), cfg=R.densify_cfg(**CFG),
                        capacity=10)
    assert e.value.status == B.GP_EOVERFLOW
    z = torch.zeros(11, 0, device="cuda")
    e1 = torch.zeros(0, device="cuda")
    po, mo, vo, n_new = R.densify_prune(z, z, z, e1, e1.int(), e1, torch.zeros(6, 0, device="cuda"))
    assert n_new == 0
