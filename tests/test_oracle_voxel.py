"""Pins of the voxeliser reference against closed forms, brute force and invariants."""
import math

import numpy as np
import pytest
import torch

from oracle import focus, spec32, voxel

F64 = torch.float64


def _grid(nx, ny, nz, x0=0.0, y0=0.0, z0=0.0, dx=1.0, dy=1.0, dz=1.0):
    return dict(nx=nx, ny=ny, nz=nz, x0=x0, y0=y0, z0=z0, dx=dx, dy=dy, dz=dz)


def _random(n, box, seed, ls=(0.0, 0.4)):
    rng = np.random.default_rng(seed)
    p = np.zeros((11, n), np.float32)
    p[0:3] = rng.uniform(0, 1, (3, n)) * np.asarray(box, np.float32)[:, None]
    p[3:6] = rng.normal(ls[0], ls[1], (3, n))
    p[6:10] = rng.normal(size=(4, n))
    p[10] = rng.uniform(0.1, 1.0, n)
    return p


def test_value_at_the_mean_is_alpha():
    p = np.zeros((11, 1), np.float32)
    p[0:3, 0] = (10.5, 6.5, 3.5)           # a voxel centre
    p[3:6, 0] = np.log([1.3, 2.0, 0.7])
    p[6:10, 0] = (0.9, 0.1, -0.3, 0.2)
    p[10, 0] = 0.8
    v = voxel.voxelize(p, _grid(24, 16, 10))
    assert v[3, 6, 10] == pytest.approx(0.8, rel=1e-7)   # float32 parameters
    assert v.max() == v[3, 6, 10]


def test_mass_matches_the_3d_gaussian_integral():
    # sum_v V dV = alpha (2 pi)^(3/2) sqrt(det Sigma) for a Gaussian well inside
    # the grid and wider than a voxel (the voxel sum of a smooth Gaussian is
    # spectrally accurate); exact mode removes the 3-sigma truncation.
    p = np.zeros((11, 1), np.float32)
    p[0:3, 0] = (20.3, 18.7, 16.1)
    l = np.log([2.5, 1.8, 3.0])
    p[3:6, 0] = l
    p[6:10, 0] = (0.7, 0.4, -0.5, 0.3)
    p[10, 0] = 0.6
    g = _grid(40, 36, 32, dx=1.0, dy=1.0, dz=1.0)
    v = voxel.voxelize(p, g, exact=True)
    s = np.exp(l.astype(np.float32).astype(np.float64))
    expect = 0.6 * (2 * np.pi) ** 1.5 * np.prod(s)
    assert v.sum() == pytest.approx(expect, rel=1e-6)


def test_axis_aligned_gaussian_is_separable():
    p = np.zeros((11, 1), np.float32)
    p[0:3, 0] = (7.2, 9.9, 5.4)
    s = np.array([1.5, 2.2, 0.9])
    p[3:6, 0] = np.log(s)
    p[6, 0] = 1.0
    p[10, 0] = 1.0
    g = _grid(16, 20, 12, x0=-1.0, y0=0.5, z0=0.25, dx=0.9, dy=1.1, dz=0.8)
    v = voxel.voxelize(p, g, exact=True)
    ss = np.exp(p[3:6, 0].astype(np.float64))
    mu = p[0:3, 0].astype(np.float64)
    rng = np.random.default_rng(0)
    for _ in range(20):
        i, j, k = rng.integers(0, 16), rng.integers(0, 20), rng.integers(0, 12)
        x = np.array([-1.0 + (i + 0.5) * 0.9, 0.5 + (j + 0.5) * 1.1, 0.25 + (k + 0.5) * 0.8])
        expect = np.exp(-0.5 * np.sum(((x - mu) / ss) ** 2))
        assert v[k, j, i] == pytest.approx(expect, rel=1e-12, abs=1e-300)


def test_brute_force_with_membership():
    p = _random(12, (20, 14, 11), seed=3, ls=(0.0, 0.3))
    g = _grid(20, 14, 11, x0=0.0, y0=0.0, z0=0.0, dx=1.0, dy=1.0, dz=1.0)
    b = voxel.tiles32(p, g)
    v = voxel.voxelize(p, g)
    ntx, nty, ntz = voxel.grid_tiles(g)
    mu, Sigma, alpha = focus.activate(torch.from_numpy(p.astype(np.float64)))
    P = np.linalg.inv(Sigma.numpy())
    ref = np.zeros_like(v)
    for k in range(11):
        for j in range(14):
            for i in range(20):
                x = np.array([i + 0.5, j + 0.5, k + 0.5])
                t = (i // 8, j // 8, k // 8)
                for n in range(12):
                    if not b["member"][n]:
                        continue
                    if all(b["t0"][a][n] <= t[a] <= b["t1"][a][n] for a in range(3)):
                        d = x - mu[n].numpy()
                        ref[k, j, i] += alpha[n].item() * math.exp(-0.5 * d @ P[n] @ d)
    np.testing.assert_allclose(v, ref, rtol=1e-12, atol=1e-300)


def test_tile_boxes_cover_the_three_sigma_box():
    p = _random(300, (60, 50, 40), seed=5)
    g = _grid(60, 50, 40, x0=-2.0, y0=1.0, z0=0.5, dx=1.0, dy=1.0, dz=1.0)
    b = voxel.tiles32(p, g)
    _, Sigma, _ = focus.activate(torch.from_numpy(p.astype(np.float64)))
    S = Sigma.numpy()
    nt = voxel.grid_tiles(g)
    o = (g["x0"], g["y0"], g["z0"])
    checked = 0
    for n in range(300):
        for a in range(3):
            r = 3.0 * math.sqrt(S[n, a, a])
            lo = math.floor((p[a, n] - r - o[a]) / 8.0)
            hi = math.floor((p[a, n] + r - o[a]) / 8.0)
            edge = min(abs((p[a, n] - r - o[a]) / 8.0 - round((p[a, n] - r - o[a]) / 8.0)),
                       abs((p[a, n] + r - o[a]) / 8.0 - round((p[a, n] + r - o[a]) / 8.0)))
            if edge < 1e-4:
                continue            # within rounding of a tile edge
            vis = hi >= 0 and lo <= nt[a] - 1
            if not vis:
                assert not b["member"][n]
                continue
            if b["member"][n]:
                assert b["t0"][a][n] == max(lo, 0) and b["t1"][a][n] == min(hi, nt[a] - 1)
                checked += 1
    assert checked > 500


def test_linearity_and_exact_mode():
    p = _random(40, (24, 24, 24), seed=7)
    g = _grid(24, 24, 24)
    v = voxel.voxelize(p, g)
    v1 = voxel.voxelize(p[:, :17], g)
    v2 = voxel.voxelize(p[:, 17:], g)
    np.testing.assert_allclose(v, v1 + v2, rtol=1e-12, atol=1e-15)
    ve = voxel.voxelize(p, g, exact=True)
    # the 3-sigma truncation only drops tails: exact >= truncated, close in sum
    assert (ve >= v - 1e-15).all()
    assert ve.sum() == pytest.approx(v.sum(), rel=0.05)


def test_gradient_matches_central_differences():
    p = _random(6, (20, 18, 14), seed=9, ls=(0.3, 0.2))
    g = _grid(20, 18, 14)
    rng = np.random.default_rng(1)
    w = rng.normal(size=(14, 18, 20))
    G = voxel.grad(p, g, w)
    keys = voxel.lists(p, g)
    p64 = torch.from_numpy(p.astype(np.float64))

    def L(q):
        return float((voxel.voxelize_t(q, keys, g) * torch.from_numpy(w)).sum())

    h = 1e-6
    for r in range(11):
        for n in (0, 3, 5):
            qp = p64.clone()
            qm = p64.clone()
            qp[r, n] += h
            qm[r, n] -= h
            fd = (L(qp) - L(qm)) / (2 * h)
            assert G[r, n] == pytest.approx(fd, rel=1e-5, abs=1e-8)
    # the quaternion's scale does not change the volume
    q = p64[6:10].numpy()
    assert np.abs(np.sum(G[6:10] * q, axis=0)).max() <= 1e-9 * np.abs(G[6:10]).max()
