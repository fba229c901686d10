"""The differentiable voxeliser on the GPU against the oracle.

Bars: tile lists bit-exact; volumes within 1e-5 of the oracle's largest value;
gradients within 1e-4 per parameter block (mu, l, q, alpha).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import voxel as ovox
from paper_2603_20611_amd import synth

pytestmark = pytest.mark.gpu

BLOCKS = {"mean": (0, 3), "log_scale": (3, 6), "quat": (6, 10), "alpha": (10, 11)}


def _say(msg):
    print(f"[voxel] {msg}", flush=True)
    sys.stdout.flush()


def _grid(nx, ny, nz, **kw):
    g = dict(nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, dx=1.0, dy=1.0, dz=1.0)
    g.update(kw)
    return g


def _rel(a, b):
    return float(np.abs(a - b).max()) / max(float(np.abs(b).max()), 1e-30)


def _forward(p, grid, exact=False, check_lists=True):
    from paper_2603_20611_amd import binding as B, render as R
    pt = torch.from_numpy(np.ascontiguousarray(p)).cuda()
    opts = B.default_opts()
    if exact:
        opts.flags = B.GP_FLAG_EXACT
    ws = R.Workspace()
    v = R.voxelize(pt, grid, ws, opts=opts).cpu().numpy().reshape(grid["nz"], grid["ny"], grid["nx"])
    ref = ovox.voxelize(p, grid, exact=exact)
    err = _rel(v, ref)
    if check_lists:
        keys = ovox.lists(p, grid, exact=exact)
        nt = int(np.prod(ovox.grid_tiles(grid)))
        got, ranges = ws.export_bins(nt, keys.size + 16)
        assert np.array_equal(got, keys), "tile lists differ"
    return v, ref, err, ws, pt, opts


@pytest.mark.parametrize("case", ["tiny", "ragged_offset", "exact", "sharp", "wide"])
def test_forward_matches_oracle(gp, case):
    _say(f"forward {case}")
    if case == "tiny":
        p, _, _ = synth.tiny(seed=0)
        grid = _grid(64, 64, 32)
    elif case == "ragged_offset":
        p = synth.gaussians_uniform(1500, (40.0, 30.0, 22.0), np.log(1.2), 0.4, seed=4)
        grid = _grid(37, 29, 19, x0=-1.5, y0=0.75, z0=-0.5, dx=1.1, dy=0.9, dz=1.3)
    elif case == "exact":
        p = synth.gaussians_uniform(60, (24.0, 20.0, 16.0), np.log(1.5), 0.3, seed=5)
        grid = _grid(24, 20, 17)
    elif case == "sharp":
        p = synth.gaussians_uniform(800, (32.0, 32.0, 32.0), np.log(0.3), 0.2, seed=6)
        grid = _grid(32, 32, 32)
    else:
        p = synth.gaussians_microscopy(600, (48.0, 48.0, 24.0), seed=7)
        grid = _grid(48, 48, 24, dz=1.0)
    v, ref, err, ws, _, _ = _forward(p, grid, exact=(case == "exact"))
    _say(f"{case}: rel err {err:.2e}")
    assert err <= 1e-5
    ws.close()


def test_backward_matches_oracle(gp):
    from paper_2603_20611_amd import render as R
    _say("backward")
    p = synth.gaussians_uniform(300, (40.0, 36.0, 24.0), np.log(1.3), 0.3, seed=11)
    grid = _grid(40, 36, 24, x0=0.25, dz=1.2)
    v, ref, err, ws, pt, opts = _forward(p, grid, check_lists=False)
    assert err <= 1e-5
    rng = np.random.default_rng(3)
    w = rng.normal(size=(grid["nz"], grid["ny"], grid["nx"])).astype(np.float32)
    gvol = torch.from_numpy(w).cuda().reshape(-1)
    g = R.voxelize_backward(pt, grid, gvol, ws, opts=opts).cpu().numpy()
    eg = ovox.grad(p, grid, w)
    for name, (r0, r1) in BLOCKS.items():
        e = np.abs(g[r0:r1] - eg[r0:r1]).max() / max(np.abs(eg[r0:r1]).max(), 1e-30)
        _say(f"grad {name}: {e:.2e}")
        assert e <= 1e-4, name
    # deterministic, and it accumulates
    g2 = R.voxelize_backward(pt, grid, gvol, ws, opts=opts, grad=torch.from_numpy(g).cuda()).cpu().numpy()
    np.testing.assert_array_equal(g2, g + g)
    ws.close()


def test_sixteen_bit_attributes(gp):
    from paper_2603_20611_amd import binding as B, render as R
    _say("16-bit attributes")
    p = synth.gaussians_microscopy(500, (40.0, 40.0, 20.0), seed=12)
    grid = _grid(40, 40, 20)
    means = torch.from_numpy(np.ascontiguousarray(p[0:3])).cuda()
    attrs = torch.from_numpy(np.ascontiguousarray(p[3:11].astype(np.float16))).cuda()
    ws = R.Workspace()
    v = R.voxelize(means, grid, ws, attrs=attrs, attr_dtype=B.GP_F16).cpu().numpy().reshape(20, 40, 40)
    q = p.copy()
    q[3:11] = p[3:11].astype(np.float16).astype(np.float32)
    ref = ovox.voxelize(q, grid)
    assert _rel(v, ref) <= 1e-5
    ws.close()


def test_deterministic_empty_and_errors(gp):
    from paper_2603_20611_amd import binding as B, render as R
    p, _, _ = synth.tiny(seed=1)
    grid = _grid(64, 64, 32)
    pt = torch.from_numpy(p).cuda()
    ws = R.Workspace()
    a = R.voxelize(pt, grid, ws).cpu().numpy()
    b = R.voxelize(pt, grid, ws).cpu().numpy()
    assert np.array_equal(a, b)
    # no Gaussians: zeros
    z = R.voxelize(pt[:, :0].contiguous(), _grid(9, 9, 9), ws).cpu().numpy()
    assert not z.any()
    # backward needs the matching voxelisation
    ws2 = R.Workspace()
    with pytest.raises(B.GpError) as e:
        R.voxelize_backward(pt, grid, torch.zeros(64 * 64 * 32, device="cuda"), ws2)
    assert e.value.status == B.GP_ESTATE
    with pytest.raises(B.GpError) as e:
        R.voxelize(pt, dict(nx=4, ny=4, nz=4, dx=0.0), ws2)
    assert e.value.status == B.GP_EINVAL
    # a slice render replaces the voxel lists in the workspace
    sl = synth.axial_slices(1, 32, 32, 1.0)
    R.render(pt, sl, ws=ws)
    with pytest.raises(B.GpError):
        R.voxelize_backward(pt, grid, torch.zeros(64 * 64 * 32, device="cuda"), ws)
    ws.close()
    ws2.close()
