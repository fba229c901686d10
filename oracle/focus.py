"""FP64 reference of the Focus-Gaussian slice renderer, its gradient, and Adam.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline of the benchmark may import this module.  It shares no code with the
HIP path and is deliberately plain: every per-(Gaussian, slice) quantity is
computed by the paper's literal route with explicit 3x3 matrix inverses, and
every pixel is a direct sum over the members of its tile.

What is followed, step by step:
  * Gaussian parameterisation G = (mu, s, q, alpha), Sigma = R S S^T R^T with
    S = diag(mod * s), R = quatToMatrix(q)  (Sec. 3; supplement, "Derivation
    of Forward rendering process", first three equations);
  * slice camera: mu_c = R_c mu + t, Sigma_c = R_c Sigma R_c^T (supplement,
    "Derivation of Forward rendering process", camera transform), the slice
    being the plane z_c = z of that frame; an axial slice has R_c = I, t = 0
    (so mu_c = mu - z e3 relative to the plane), an oblique slice carries its
    pose (R_c row-major, t) under the key "pose";
  * axial re-parameterisation Sigma_e^-1 = Sigma_c^-1 + e3 e3^T / sigma_z^2,
    mu_e = Sigma_e Sigma_c^-1 mu_c  (Sec. 4.2, Focus Gaussian equation);
  * opacity modulation opacity_r = exp(-1/2 (mu_c^T Sigma_c^-1 mu_c -
    mu_e^T Sigma_e^-1 mu_e))  (Sec. 4.2, opacity modulation equation);
  * screen-space marginal Sigma_2d = Sigma_e[0:2, 0:2], mu_2d = mu_e[0:2]
    (Sec. 4.2, screen-space projection equation);
  * intensity alpha~ = alpha * opacity_r / sqrt(det Sigma_2d)  (Sec. 4.2,
    intensity normalisation equation); with conv_exact=True instead the exact
    value of the convolution integral of Sec. 4.2 (I = integral over t of
    h(t) g_c(x, y, t)), which completing the square in the exponent gives as
    alpha * opacity_r * sqrt(2 pi det Sigma_e / det Sigma_2d);
  * additive rasterisation I(p) = sum_{i in N(p)} alpha~_i exp(-1/2 d^T
    Sigma_2d^-1 d), d = p - mu_2d  (Sec. 4.2, additive rasterisation equation),
    with N(p) the members of p's 16x16 tile from the binary32 specification in
    ``oracle.spec32``;
  * gradient: the exact derivative of the above, obtained by reverse-mode
    automatic differentiation in float64 (the paper's backward pass, Sec. 4.3
    and the supplement's "Derivation of Differentiable Backward Pass",
    computes the same derivative);
  * Adam: Kingma & Ba, Algorithm 1, cited by the paper's implementation details
    (Sec. 5.1), with per-group learning rates.

Limits of the model (Fig. 1 b-d):
  * sigma_z = +inf: the e3 e3^T / sigma_z^2 term vanishes (all-in-focus);
  * sigma_z = 0: the literal route divides by zero; the zero-thickness limit is
    taken instead, Sigma_e -> Sigma_c - Sigma_c e3 e3^T Sigma_c / Sigma_c[2,2]
    and mu_e -> the conditional mean of the Gaussian on the plane, with the
    opacity term as the limit m^2 / Sigma_zz.  This branch is pinned by the
    continuity test against sigma_z = 1e-6 and by point evaluation of g.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import spec32

F64 = torch.float64
TILE = spec32.TILE


# --------------------------------------------------------------------------- #
# Gaussian parameterisation
# --------------------------------------------------------------------------- #
def quat_to_matrix(q):
    """Rotation matrix of unit quaternions q = (w, x, y, z), shape [..., 4] -> [..., 3, 3]."""
    w, x, y, z = q.unbind(-1)
    row0 = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1)
    row1 = torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1)
    row2 = torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)
    return torch.stack([row0, row1, row2], -2)


def activate(params, scale_mod=1.0):
    """params [11, N] float64 -> (mu [N,3], Sigma [N,3,3], alpha [N])."""
    mu = params[0:3].T
    s = torch.exp(params[3:6].T) * scale_mod
    q = params[6:10].T
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    R = quat_to_matrix(q)
    S = torch.diag_embed(s)
    Sigma = R @ S @ S.transpose(-1, -2) @ R.transpose(-1, -2)
    return mu, Sigma, params[10]


# --------------------------------------------------------------------------- #
# Focus Gaussian on one axial slice
# --------------------------------------------------------------------------- #
def focus(mu, Sigma, alpha, z, sigma_z, conv_exact=False, pose=None):
    """Per-Gaussian Focus-Gaussian quantities on the slice z_c = z.

    pose: None (axial, R_c = I, t = 0) or 12 numbers (R_c row-major, t).
    Returns dict with mu2d [n,2], Sigma2d [n,2,2], opacity_r [n], alpha_t [n]
    (and the 3-D mu_e, Sigma_e).
    """
    n = mu.shape[0]
    e3 = torch.tensor([0.0, 0.0, 1.0], dtype=F64)
    if pose is None:
        Rc, t = torch.eye(3, dtype=F64), torch.zeros(3, dtype=F64)
    else:
        pz = torch.as_tensor(np.asarray(pose, dtype=np.float32).astype(np.float64).reshape(-1))
        Rc, t = pz[0:9].reshape(3, 3), pz[9:12]
    # camera frame, measured from the imaging plane z_c = z
    mu_c = mu @ Rc.T + t - float(z) * e3
    Sigma_c = Rc @ Sigma @ Rc.T
    Sc_inv = torch.linalg.inv(Sigma_c)
    sz = float(sigma_z)
    if sz > 0.0:
        inj = 0.0 if math.isinf(sz) else 1.0 / (sz * sz)
        P = Sc_inv + inj * torch.outer(e3, e3)
        Sigma_e = torch.linalg.inv(P)
        mu_e = (Sigma_e @ Sc_inv @ mu_c.unsqueeze(-1)).squeeze(-1)
        q_c = (mu_c.unsqueeze(-2) @ Sc_inv @ mu_c.unsqueeze(-1)).reshape(n)
        q_e = (mu_e.unsqueeze(-2) @ P @ mu_e.unsqueeze(-1)).reshape(n)
        qdiff = q_c - q_e
    else:
        # zero-thickness limit (see module docstring)
        col = Sigma_c[:, :, 2]
        szz = Sigma_c[:, 2, 2]
        Sigma_e = Sigma_c - col.unsqueeze(-1) * col.unsqueeze(-2) / szz[:, None, None]
        mu_e = mu_c - col * (mu_c[:, 2] / szz).unsqueeze(-1)
        qdiff = mu_c[:, 2] * mu_c[:, 2] / szz
    opacity_r = torch.exp(-0.5 * qdiff)
    Sigma2d = Sigma_e[:, 0:2, 0:2]
    mu2d = mu_e[:, 0:2]
    alpha_t = alpha * opacity_r / torch.sqrt(torch.linalg.det(Sigma2d))
    if conv_exact:
        if sz > 0.0:
            alpha_t = alpha_t * torch.sqrt(2.0 * math.pi * torch.linalg.det(Sigma_e))
        else:
            alpha_t = alpha_t * 0.0   # h has zero width: the integral vanishes
    return dict(mu_e=mu_e, Sigma_e=Sigma_e, mu2d=mu2d, Sigma2d=Sigma2d,
                opacity_r=opacity_r, alpha_t=alpha_t, qdiff=qdiff)


# --------------------------------------------------------------------------- #
# Rendering
# --------------------------------------------------------------------------- #
def _as_params64(params):
    if isinstance(params, torch.Tensor):
        return params.to(F64)
    return torch.from_numpy(np.asarray(params, dtype=np.float32).astype(np.float64))


def _pixel_centres(sl, px, py):
    x = sl["x0"] + (px.to(F64) + 0.5) * sl["dx"]
    y = sl["y0"] + (py.to(F64) + 0.5) * sl["dy"]
    return x, y


def slice_instances(params32, sl, q_cut=spec32.Q_CUT_DEFAULT, bbox=spec32.BBOX_DEFAULT,
                    scale_mod=1.0, exact=False):
    """(gaussian index, tile index) of every tile-list entry of one slice, sorted."""
    keys, _ = spec32.bins(params32, [sl], q_cut, bbox, scale_mod, exact)
    return (keys & 0xFFFFFFFF).astype(np.int64), (keys >> 32).astype(np.int64)


def render_slice(params, params32, sl, q_cut=spec32.Q_CUT_DEFAULT, bbox=spec32.BBOX_DEFAULT,
                 scale_mod=1.0, exact=False, instances=None, conv_exact=False):
    """FP64 image [H, W] of one slice.  params: float64 tensor [11, N] (may require grad);
    params32: the same values as float32 numpy (membership is decided on them)."""
    W, H = int(sl["width"]), int(sl["height"])
    ntx = (W + TILE - 1) // TILE
    if instances is None:
        instances = slice_instances(params32, sl, q_cut, bbox, scale_mod, exact)
    gidx, tile = instances
    img = torch.zeros(H * W, dtype=F64)
    if gidx.size == 0:
        return img.reshape(H, W) + 0.0 * params.sum()
    uniq, inv = np.unique(gidx, return_inverse=True)
    u = torch.from_numpy(uniq)
    mu, Sigma, alpha = activate(params[:, u], scale_mod)
    f = focus(mu, Sigma, alpha, sl["z"], sl["sigma_z"], conv_exact, sl.get("pose"))
    inv_t = torch.from_numpy(inv)
    Sinv = torch.linalg.inv(f["Sigma2d"])[inv_t]          # [K,2,2]
    m2 = f["mu2d"][inv_t]                                 # [K,2]
    at = f["alpha_t"][inv_t]                              # [K]
    tx = torch.from_numpy(tile % ntx)
    ty = torch.from_numpy(tile // ntx)
    lx = torch.arange(TILE).repeat(TILE)                  # pixel offsets within a tile
    ly = torch.arange(TILE).repeat_interleave(TILE)
    px = tx[:, None] * TILE + lx[None, :]                 # [K,256]
    py = ty[:, None] * TILE + ly[None, :]
    inside = (px < W) & (py < H)
    X, Y = _pixel_centres(sl, px, py)
    d0 = X - m2[:, 0:1]
    d1 = Y - m2[:, 1:2]
    quad = (Sinv[:, 0, 0, None] * d0 * d0 + (Sinv[:, 0, 1, None] + Sinv[:, 1, 0, None]) * d0 * d1
            + Sinv[:, 1, 1, None] * d1 * d1)
    contrib = at[:, None] * torch.exp(-0.5 * quad)
    flat = (py * W + px)[inside]
    img = img.index_add(0, flat, contrib[inside])
    return img.reshape(H, W)


def render(params, slices, q_cut=spec32.Q_CUT_DEFAULT, bbox=spec32.BBOX_DEFAULT,
           scale_mod=1.0, exact=False, conv_exact=False):
    """List of FP64 images, one per slice.  params: float32 numpy [11, N] or tensor."""
    p64 = _as_params64(params)
    p32 = p64.detach().numpy().astype(np.float32)
    return [render_slice(p64, p32, sl, q_cut, bbox, scale_mod, exact, conv_exact=conv_exact) for sl in slices]


def render_pixels(params, sl, px, py, q_cut=spec32.Q_CUT_DEFAULT, bbox=spec32.BBOX_DEFAULT,
                  scale_mod=1.0, conv_exact=False):
    """FP64 values of selected pixels of one slice, each summed over its tile's list.

    For large workloads: membership is decided for the whole slice (binary32,
    vectorised), then each requested pixel is evaluated on its own."""
    p64 = _as_params64(params)
    p32 = p64.detach().numpy().astype(np.float32)
    W = int(sl["width"])
    ntx = (W + TILE - 1) // TILE
    gidx, tile = slice_instances(p32, sl, q_cut, bbox, scale_mod)
    order = np.argsort(tile, kind="stable")
    gidx, tile = gidx[order], tile[order]
    starts = np.searchsorted(tile, np.arange(tile.max() + 2 if tile.size else 1))
    out = np.zeros(len(px))
    for j, (x, y) in enumerate(zip(px, py)):
        t = (int(y) // TILE) * ntx + int(x) // TILE
        if t + 1 >= len(starts):
            continue
        members = gidx[starts[t]:starts[t + 1]]
        if members.size == 0:
            continue
        mu, Sigma, alpha = activate(p64[:, torch.from_numpy(members)], scale_mod)
        f = focus(mu, Sigma, alpha, sl["z"], sl["sigma_z"], conv_exact, sl.get("pose"))
        X = sl["x0"] + (x + 0.5) * sl["dx"]
        Y = sl["y0"] + (y + 0.5) * sl["dy"]
        d = torch.tensor([X, Y], dtype=F64)[None, :] - f["mu2d"]
        Sinv = torch.linalg.inv(f["Sigma2d"])
        quad = (d.unsqueeze(-2) @ Sinv @ d.unsqueeze(-1)).reshape(-1)
        out[j] = float((f["alpha_t"] * torch.exp(-0.5 * quad)).sum())
    return out


# --------------------------------------------------------------------------- #
# Gradient of a linear functional of the images
# --------------------------------------------------------------------------- #
def grad(params, slices, weights, q_cut=spec32.Q_CUT_DEFAULT, bbox=spec32.BBOX_DEFAULT,
         scale_mod=1.0, exact=False, conv_exact=False):
    """d/dparams of L = sum_k sum_p weights[k][p] * I_k(p), float64 [11, N].

    weights: list of [H, W] arrays (the upstream gradient dL/dI)."""
    p64 = _as_params64(params).detach().clone().requires_grad_(True)
    p32 = p64.detach().numpy().astype(np.float32)
    for sl, w in zip(slices, weights):
        img = render_slice(p64, p32, sl, q_cut, bbox, scale_mod, exact, conv_exact=conv_exact)
        L = (img * torch.as_tensor(np.asarray(w), dtype=F64)).sum()
        if L.requires_grad:
            L.backward()
    g = p64.grad
    return np.zeros(p64.shape) if g is None else g.numpy()


def grad_of_gaussians(params, slices, weights, idx, q_cut=spec32.Q_CUT_DEFAULT,
                      bbox=spec32.BBOX_DEFAULT, scale_mod=1.0):
    """Gradient columns of the Gaussians in idx only (large workloads).

    By linearity of the image in its Gaussians, dL/dtheta_i involves only
    Gaussian i's own contributions, evaluated on the tiles of its lists."""
    p64 = _as_params64(params)
    p32 = p64.detach().numpy().astype(np.float32)
    idx = np.asarray(idx, dtype=np.int64)
    sub = p64[:, torch.from_numpy(idx)].detach().clone().requires_grad_(True)
    for sl, w in zip(slices, weights):
        gidx, tile = slice_instances(p32, sl, q_cut, bbox, scale_mod)
        sel = np.isin(gidx, idx)
        if not sel.any():
            continue
        local = np.searchsorted(np.sort(idx), gidx[sel])
        # map sorted-idx positions back to positions in idx
        order = np.argsort(idx)
        local = order[local]
        img = render_slice(sub, None, sl, instances=(local, tile[sel]), scale_mod=scale_mod)
        L = (img * torch.as_tensor(np.asarray(w), dtype=F64)).sum()
        L.backward()
    g = sub.grad
    return np.zeros(sub.shape) if g is None else g.numpy()


def l1_grad(image, target):
    """dL/dI of L = mean |I - T| with sign(0) = 0 (the L1 term of the loss, Sec. 4.3)."""
    image = np.asarray(image, dtype=np.float64)
    return np.sign(image - np.asarray(target, dtype=np.float64)) / image.size


# --------------------------------------------------------------------------- #
# Adam (Kingma & Ba, Algorithm 1), per-group learning rate
# --------------------------------------------------------------------------- #
GROUP_ROWS = {"mean": (0, 3), "log_scale": (3, 6), "quat": (6, 10), "alpha": (10, 11)}


def adam_step(params, grads, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-15, clamp_alpha=False):
    """One Adam update of [11, N] arrays in float64; lr: dict group -> learning rate.

    clamp_alpha: afterwards project the intensity row onto alpha >= 0 (the
    intensity is used linearly, and a negative one has no physical meaning).
    Returns (params, m, v) as new float64 arrays."""
    p = np.asarray(params, np.float64).copy()
    g = np.asarray(grads, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    for name, (r0, r1) in GROUP_ROWS.items():
        p[r0:r1] -= lr[name] * mhat[r0:r1] / (np.sqrt(vhat[r0:r1]) + eps)
    if clamp_alpha:
        p[10] = np.maximum(p[10], 0.0)
    return p, m, v
