"""FP64 reference of the differentiable voxeliser.

TEST INFRASTRUCTURE ONLY: imported by the test-suite alone.  Shares no code
with the HIP path.

The paper's voxeliser (Sec. 4.3, "Differentiable Voxelization") builds an
intensity volume from the world-space Gaussians, before any focus
re-parameterisation: the space is cut into 8 x 8 x 8-voxel tiles, each tile
keeps the Gaussians whose 3-sigma ellipsoid reaches it, and a voxel at x
receives sigma(x) = sum_i g_i(x) over its tile's Gaussians.  Readings:
  * g_i(x) = alpha_i exp(-1/2 (x - mu_i)^T Sigma_i^-1 (x - mu_i)), the
    unnormalised Gaussian with intensity alpha of the forward model;
  * voxel (i, j, k) has centre (x0 + (i + 1/2) dx, y0 + (j + 1/2) dy,
    z0 + (k + 1/2) dz); the volume is stored [nz][ny][nx];
  * "reaches the tile" is the axis-aligned box of the 3-sigma ellipsoid
    (half-widths 3 sqrt(Sigma_aa)), decided in binary32 by the fixed operation
    sequence of `tiles32` so that the lists are reproducible bit for bit;
  * a Gaussian contributes to every voxel of every tile in its box.
Tiles are numbered (tz * nty + ty) * ntx + tx; each tile's list holds its
Gaussians in ascending index order.
"""
import numpy as np
import torch

from oracle import focus, spec32

F64 = torch.float64
f32 = np.float32
VTILE = 8


def grid_tiles(grid):
    return tuple((int(grid[n]) + VTILE - 1) // VTILE for n in ("nx", "ny", "nz"))


def tiles32(params, grid, bbox=spec32.BBOX_DEFAULT, scale_mod=1.0):
    """Binary32 tile box of every Gaussian: dict with 'member' [N] and inclusive
    clamped bounds t0[3][N], t1[3][N] (x, y, z)."""
    act = spec32.activate32(params, scale_mod)
    nt = grid_tiles(grid)
    bbox = f32(bbox)
    eighth = f32(1.0 / VTILE)
    t0, t1 = [], []
    vis = act["ok"].copy()
    with np.errstate(all="ignore"):
        for mu, s, o, d, n in ((act["mux"], act["sxx"], grid["x0"], grid["dx"], nt[0]),
                               (act["muy"], act["syy"], grid["y0"], grid["dy"], nt[1]),
                               (act["muz"], act["szz"], grid["z0"], grid["dz"], nt[2])):
            r = bbox * np.sqrt(s)
            lo = np.floor((((mu - r) - f32(o)) / f32(d)) * eighth)
            hi = np.floor((((mu + r) - f32(o)) / f32(d)) * eighth)
            vis &= (hi >= 0) & (lo <= f32(n - 1))
            t0.append(lo)
            t1.append(hi)
        for a in range(3):
            n = nt[a]
            t0[a] = np.where(vis, np.maximum(t0[a], f32(0)), 0).astype(np.int64)
            t1[a] = np.where(vis, np.minimum(t1[a], f32(n - 1)), -1).astype(np.int64)
    return dict(member=vis, t0=t0, t1=t1)


def lists(params, grid, bbox=spec32.BBOX_DEFAULT, scale_mod=1.0, exact=False):
    """Sorted keys (tile << 32 | gaussian) of all tile-list entries."""
    ntx, nty, ntz = grid_tiles(grid)
    if exact:
        act = spec32.activate32(params, scale_mod)
        idx = np.nonzero(act["ok"])[0].astype(np.int64)
        t = np.arange(ntx * nty * ntz, dtype=np.int64)
        keys = (t[:, None] << 32) + idx[None, :]
        return np.sort(keys.reshape(-1))
    b = tiles32(params, grid, bbox, scale_mod)
    keys = []
    for j in np.nonzero(b["member"])[0]:
        for tz in range(b["t0"][2][j], b["t1"][2][j] + 1):
            for ty in range(b["t0"][1][j], b["t1"][1][j] + 1):
                for tx in range(b["t0"][0][j], b["t1"][0][j] + 1):
                    keys.append((((tz * nty + ty) * ntx + tx) << 32) + int(j))
    return np.sort(np.asarray(keys, dtype=np.int64))


def _centres(grid, ix, iy, iz):
    x = grid["x0"] + (ix.to(F64) + 0.5) * grid["dx"]
    y = grid["y0"] + (iy.to(F64) + 0.5) * grid["dy"]
    z = grid["z0"] + (iz.to(F64) + 0.5) * grid["dz"]
    return torch.stack([x, y, z], -1)


def voxelize_t(p64, keys, grid, scale_mod=1.0):
    """Volume [nz, ny, nx] (float64 tensor, differentiable in p64 [11, N])."""
    nx, ny, nz = int(grid["nx"]), int(grid["ny"]), int(grid["nz"])
    ntx, nty, _ = grid_tiles(grid)
    vol = torch.zeros(nz * ny * nx, dtype=F64)
    if keys.size == 0:
        return vol.reshape(nz, ny, nx) + 0.0 * p64.sum()
    tile = keys >> 32
    gid = keys & 0xFFFFFFFF
    uniq, inv = np.unique(gid, return_inverse=True)
    mu, Sigma, alpha = focus.activate(p64[:, torch.from_numpy(uniq)], scale_mod)
    P = torch.linalg.inv(Sigma)
    inv_t = torch.from_numpy(inv)
    tx = torch.from_numpy(tile % ntx)
    ty = torch.from_numpy((tile // ntx) % nty)
    tz = torch.from_numpy(tile // (ntx * nty))
    o = torch.arange(VTILE)
    lx = o.repeat(VTILE * VTILE)
    ly = o.repeat_interleave(VTILE).repeat(VTILE)
    lz = o.repeat_interleave(VTILE * VTILE)
    ix = tx[:, None] * VTILE + lx[None, :]
    iy = ty[:, None] * VTILE + ly[None, :]
    iz = tz[:, None] * VTILE + lz[None, :]
    inside = (ix < nx) & (iy < ny) & (iz < nz)
    d = _centres(grid, ix, iy, iz) - mu[inv_t][:, None, :]            # [K, 512, 3]
    q = torch.einsum("kva,kab,kvb->kv", d, P[inv_t], d)
    contrib = alpha[inv_t][:, None] * torch.exp(-0.5 * q)
    flat = (iz * ny + iy) * nx + ix
    vol = vol.index_add(0, flat[inside], contrib[inside])
    return vol.reshape(nz, ny, nx)


def voxelize(params, grid, bbox=spec32.BBOX_DEFAULT, scale_mod=1.0, exact=False):
    """Float64 volume [nz, ny, nx] of float32 parameters [11, N]."""
    p64 = focus._as_params64(params)
    keys = lists(np.asarray(params, np.float32), grid, bbox, scale_mod, exact)
    return voxelize_t(p64, keys, grid, scale_mod).numpy()


def grad(params, grid, weights, bbox=spec32.BBOX_DEFAULT, scale_mod=1.0):
    """d/dparams of L = sum_v weights[v] V[v] (float64 [11, N]), membership fixed."""
    p64 = focus._as_params64(params).detach().clone().requires_grad_(True)
    keys = lists(np.asarray(params, np.float32), grid, bbox, scale_mod)
    vol = voxelize_t(p64, keys, grid, scale_mod)
    L = (vol * torch.as_tensor(np.asarray(weights), dtype=F64)).sum()
    if L.requires_grad:
        L.backward()
    g = p64.grad
    return np.zeros(p64.shape) if g is None else g.numpy()
