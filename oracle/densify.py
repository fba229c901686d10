"""Reference of the densification statistics and of densify/prune.

TEST INFRASTRUCTURE ONLY: imported by the test-suite alone.  Shares no code
with the HIP path.

The paper states the control in words (Sec. 4.3, "Prune and densification":
Gaussians are densified and pruned according to their footprint radii on the
slices and their intensities; Sec. 5.1 gives the gradient threshold 5e-5 and
the minimum intensity 0.02).  The procedure written out here is the usual
Gaussian-splatting one, which those criteria plug into:

  statistics, per Gaussian j over every slice on which it has a record:
    grad_norm  sum of |dL/dmu_2d| with mu_2d measured in pixels,
    count      number of such slices,
    max_radius largest 3-sigma footprint half-width in pixels,
               bbox * max(sqrt(Sigma_2d[0,0]) / dx, sqrt(Sigma_2d[1,1]) / dy);
  decision (binary32, as the kernels take it):
    drop   non-finite parameters, alpha < min_alpha, max_radius > max_radius;
    grow   grad_norm / count > grad_threshold:
             clone (exact copy, fresh Adam moments) if exp(max l) <= split_scale,
             split otherwise: two children at mu + R diag(s) n_k (n_k given),
             log-scales reduced by ln(split_factor), q and alpha copied;
    keep   otherwise (moments carried over).
The new set lists survivors in Gaussian order, a grown Gaussian's second
output directly after its first.
"""
import numpy as np
import torch

from oracle import focus, spec32

F64 = torch.float64


def stats(params, slices, weights, q_cut=spec32.Q_CUT_DEFAULT, bbox=spec32.BBOX_DEFAULT, scale_mod=1.0):
    """(grad_norm float64 [N], count int64 [N], max_radius float64 [N]) for
    L = sum_k sum_p weights[k][p] I_k(p)."""
    p64 = focus._as_params64(params).detach()
    p32 = p64.numpy().astype(np.float32)
    n = p64.shape[1]
    gnorm = np.zeros(n)
    count = np.zeros(n, np.int64)
    rad = np.zeros(n)
    for sl, w in zip(slices, weights):
        gidx, tile = focus.slice_instances(p32, sl, q_cut, bbox, scale_mod)
        if gidx.size == 0:
            continue
        uniq, inv = np.unique(gidx, return_inverse=True)
        mu, Sigma, alpha = focus.activate(p64[:, torch.from_numpy(uniq)], scale_mod)
        f = focus.focus(mu, Sigma, alpha, sl["z"], sl["sigma_z"])
        m2 = f["mu2d"].detach().clone().requires_grad_(True)
        S2 = f["Sigma2d"].detach()
        at = f["alpha_t"].detach()
        ntx = (int(sl["width"]) + focus.TILE - 1) // focus.TILE
        W, H = int(sl["width"]), int(sl["height"])
        inv_t = torch.from_numpy(inv)
        Sinv = torch.linalg.inv(S2)[inv_t]
        tx = torch.from_numpy(tile % ntx)
        ty = torch.from_numpy(tile // ntx)
        lx = torch.arange(focus.TILE).repeat(focus.TILE)
        ly = torch.arange(focus.TILE).repeat_interleave(focus.TILE)
        px = tx[:, None] * focus.TILE + lx[None, :]
        py = ty[:, None] * focus.TILE + ly[None, :]
        inside = (px < W) & (py < H)
        X = sl["x0"] + (px.to(F64) + 0.5) * sl["dx"]
        Y = sl["y0"] + (py.to(F64) + 0.5) * sl["dy"]
        d0 = X - m2[inv_t, 0:1]
        d1 = Y - m2[inv_t, 1:2]
        quad = (Sinv[:, 0, 0, None] * d0 * d0 + (Sinv[:, 0, 1, None] + Sinv[:, 1, 0, None]) * d0 * d1
                + Sinv[:, 1, 1, None] * d1 * d1)
        contrib = at[inv_t, None] * torch.exp(-0.5 * quad)
        wt = torch.as_tensor(np.asarray(w), dtype=F64).reshape(-1)
        flat = (py * W + px).clamp(max=H * W - 1)
        L = (contrib * wt[flat] * inside).sum()
        L.backward()
        g = m2.grad.numpy()
        gpx = np.hypot(g[:, 0] * sl["dx"], g[:, 1] * sl["dy"])
        gnorm[uniq] += gpx
        count[uniq] += 1
        S = S2.numpy()
        r = bbox * np.maximum(np.sqrt(S[:, 0, 0]) / sl["dx"], np.sqrt(S[:, 1, 1]) / sl["dy"])
        rad[uniq] = np.maximum(rad[uniq], r)
    return gnorm, count, rad


DROP, KEEP, CLONE, SPLIT = 0, 1, 2, 3


def decide(params, grad_norm, count, max_radius, cfg):
    """Action per Gaussian (DROP/KEEP/CLONE/SPLIT), decided in binary32."""
    f = np.float32
    p = np.asarray(params, f)
    gn = np.asarray(grad_norm, f)
    cnt = np.asarray(count, np.int64)
    rad = np.asarray(max_radius, f)
    finite = np.isfinite(p).all(axis=0)
    drop = ~finite | ~(p[10] >= f(cfg["min_alpha"])) | (rad > f(cfg["max_radius"]))
    with np.errstate(all="ignore"):
        mean = np.where(cnt > 0, gn / np.maximum(cnt, 1).astype(f), f(0))
    grow = (cnt > 0) & (mean > f(cfg["grad_threshold"]))
    with np.errstate(all="ignore"):
        big = np.exp(p[3:6].max(axis=0)) > f(cfg["split_scale"])
    act = np.full(p.shape[1], KEEP, np.int64)
    act[grow & ~big] = CLONE
    act[grow & big] = SPLIT
    act[drop] = DROP
    return act


def densify_prune(params, m, v, grad_norm, count, max_radius, noise, cfg):
    """New (params, m, v) as float64 [11, N'] arrays, and the actions."""
    p = np.asarray(params, np.float32).astype(np.float64)
    m = np.asarray(m, np.float64)
    v = np.asarray(v, np.float64)
    noise = np.asarray(noise, np.float64)
    act = decide(params, grad_norm, count, max_radius, cfg)
    cols_p, cols_m, cols_v = [], [], []
    zero = np.zeros(11)
    for j in range(p.shape[1]):
        a = act[j]
        if a == DROP:
            continue
        if a == SPLIT:
            q = p[6:10, j] / np.linalg.norm(p[6:10, j])
            R = focus.quat_to_matrix(torch.from_numpy(q)).numpy()
            s = np.exp(p[3:6, j])
            for k in range(2):
                child = p[:, j].copy()
                child[0:3] = p[0:3, j] + R @ (s * noise[3 * k:3 * k + 3, j])
                child[3:6] = p[3:6, j] - np.log(cfg["split_factor"])
                cols_p.append(child)
                cols_m.append(zero)
                cols_v.append(zero)
            continue
        cols_p.append(p[:, j])
        cols_m.append(m[:, j])
        cols_v.append(v[:, j])
        if a == CLONE:
            cols_p.append(p[:, j])
            cols_m.append(zero)
            cols_v.append(zero)
    if not cols_p:
        e = np.zeros((11, 0))
        return e, e.copy(), e.copy(), act
    return np.stack(cols_p, 1), np.stack(cols_m, 1), np.stack(cols_v, 1), act
