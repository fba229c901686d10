"""Seeded synthetic workloads (microscopy- and ultrasound-shaped Gaussian sets).

This module only draws random numbers: it holds none of the renderer's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.  The
paper's datasets (TDSC-ABUS ultrasound, light-sheet and confocal microscopy,
Sec. 5.1) are not available; these generators stand in for them with the shapes
and statistics of the workloads the renderer is measured on:

  tiny        2,000 Gaussians, means U([0,64]^2 x [0,32]), log-scales
              N(ln 1.5, 0.3) per axis, unit quaternions uniform on S^3,
              intensities U(0,1); 32 axial slices z = 0.5..31.5 of 64x64 px,
              sigma_z = 1.
  microscopy  hidden set: 70 % filaments (one log-scale N(ln 6, 0.3), two
              N(ln 0.8, 0.2)), 30 % isotropic blobs (N(ln 2, 0.3)), intensities
              LogNormal(-1, 0.5), means uniform in a W x H x Z box; slices
              z = k + 1/2, sigma_z = 2; target noise Poisson(200 I)/200 +
              N(0, 0.01^2).
  ultrasound  hidden set: log-scales N(ln 1.2, 0.4), intensities U(0,1), means
              uniform in 256 x 256 x 400; 400 slices of 256^2, sigma_z = 3;
              target times iid Rayleigh(1) speckle.

Parameters are float32 arrays [11, N] with rows
mu_x, mu_y, mu_z, l_x, l_y, l_z, q_w, q_x, q_y, q_z, alpha.
Slices are dicts with z, sigma_z, x0, y0, dx, dy, width, height.
"""
from __future__ import annotations

import numpy as np

ROWS = ("mu_x", "mu_y", "mu_z", "l_x", "l_y", "l_z", "q_w", "q_x", "q_y", "q_z", "alpha")


def _quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _pack(mu, ls, q, alpha):
    p = np.empty((11, mu.shape[0]), dtype=np.float32)
    p[0:3] = mu.T
    p[3:6] = ls.T
    p[6:10] = q.T
    p[10] = alpha
    return p


def gaussians_uniform(n, box, log_scale_mean, log_scale_std, seed, alpha_range=(0.0, 1.0)):
    """Means uniform in [0,box_x] x [0,box_y] x [0,box_z]; iid normal log-scales."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.0, 1.0, (n, 3)) * np.asarray(box, np.float64)[None, :]
    ls = rng.normal(log_scale_mean, log_scale_std, (n, 3))
    q = _quats(rng, n)
    alpha = rng.uniform(alpha_range[0], alpha_range[1], n)
    return _pack(mu, ls, q, alpha)


def gaussians_microscopy(n, box, seed, filament_frac=0.7):
    """Filaments (one long axis) and isotropic blobs, LogNormal(-1, 0.5) intensities."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.0, 1.0, (n, 3)) * np.asarray(box, np.float64)[None, :]
    fil = rng.uniform(size=n) < filament_frac
    ls = np.empty((n, 3))
    nf = int(fil.sum())
    ls[fil, 0] = rng.normal(np.log(6.0), 0.3, nf)
    ls[fil, 1:] = rng.normal(np.log(0.8), 0.2, (nf, 2))
    ls[~fil, :] = rng.normal(np.log(2.0), 0.3, n - nf)[:, None]
    q = _quats(rng, n)
    alpha = rng.lognormal(-1.0, 0.5, n)
    return _pack(mu, ls, q, alpha)


def axial_slices(n_slices, width, height, sigma_z, z0=0.5, dz=1.0, x0=0.0, y0=0.0,
                 dx=1.0, dy=1.0):
    return [dict(z=z0 + k * dz, sigma_z=sigma_z, x0=x0, y0=y0, dx=dx, dy=dy,
                 width=width, height=height) for k in range(n_slices)]


def jitter_means(params, std, seed):
    rng = np.random.default_rng(seed)
    out = params.copy()
    out[0:3] += rng.normal(0.0, std, out[0:3].shape).astype(np.float32)
    return out


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
def tiny(seed=0):
    """2,000 Gaussians, 32 slices of 64x64, sigma_z = 1 (oracle-sized)."""
    p = gaussians_uniform(2000, (64.0, 64.0, 32.0), np.log(1.5), 0.3, seed)
    slices = axial_slices(32, 64, 64, 1.0)
    target_params = jitter_means(p, 0.5, seed + 1000)
    return p, slices, target_params


def ultrasound_hidden(n=500_000, seed=0):
    return gaussians_uniform(n, (256.0, 256.0, 400.0), np.log(1.2), 0.4, seed)


def ultrasound_slices(n_slices=400, res=256, sigma_z=3.0):
    return axial_slices(n_slices, res, res, sigma_z)


def speckle(shape, seed):
    """iid Rayleigh(scale 1) multiplicative speckle."""
    return np.random.default_rng(seed).rayleigh(1.0, shape).astype(np.float32)


def microscopy_hidden(n=300_000, box=(512.0, 512.0, 128.0), seed=0):
    return gaussians_microscopy(n, box, seed)


def microscopy_learnable(n=200_000, box=(512.0, 512.0, 128.0), seed=1):
    """Random initialisation: means uniform, log-scale ln 1.5, intensities U(0, 0.1)."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.0, 1.0, (n, 3)) * np.asarray(box, np.float64)[None, :]
    ls = np.full((n, 3), np.log(1.5))
    q = _quats(rng, n)
    alpha = rng.uniform(0.0, 0.1, n)
    return _pack(mu, ls, q, alpha)


def photon_noise(image, seed, photons=200.0, read_std=0.01):
    rng = np.random.default_rng(seed)
    lam = np.clip(np.asarray(image, np.float64), 0.0, None) * photons
    return (rng.poisson(lam) / photons + rng.normal(0.0, read_std, lam.shape)).astype(np.float32)


def photon_noise_torch(image, generator, photons=200.0, read_std=0.01):
    """photon_noise on the device (large stacks): Poisson(photons I) / photons +
    N(0, read_std^2), drawn from a seeded torch generator."""
    import torch
    lam = image.clamp(min=0.0) * photons
    out = torch.poisson(lam, generator=generator) / photons
    return out + read_std * torch.randn(out.shape, device=out.device, generator=generator)


def serving_volumes(n_volumes=64, n_min=20_000, n_max=1_000_000, box=(512.0, 512.0, 128.0), seed=3):
    """Resident volumes for the serving workload: sizes log-uniform in [n_min, n_max]."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_volumes)).astype(np.int64)
    return [gaussians_microscopy(int(s), box, seed * 1000 + v) for v, s in enumerate(sizes)]


def serving_requests(n, n_volumes, depth=128.0, extent=512.0, seed=3, rate=2000.0,
                     resolutions=(256, 512, 1024), sigmas=(0.5, 1.0, 2.0, 3.0)):
    """Open-loop Poisson request stream: arrival time (s), volume, z, resolution, sigma_z."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    vol = rng.integers(0, n_volumes, n)
    z = rng.uniform(0.0, depth, n)
    res = rng.choice(np.asarray(resolutions), n)
    sz = rng.choice(np.asarray(sigmas), n)
    return [dict(t=float(t[i]), volume=int(vol[i]), z=float(z[i]), res=int(res[i]),
                 sigma_z=float(sz[i]), dx=extent / float(res[i])) for i in range(n)]
