"""FP32 emulation of the tile-membership (binning) specification.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
it exists so that tests, the smoke check and the CPU baseline can decide which
Gaussians belong to which 16x16 tile exactly as a correctly rounded IEEE-754
binary32 machine would.

Why an FP32 emulation inside an FP64 oracle: the paper sums over "the Gaussians
overlapping pixel p" (Sec. 4.2, additive rasterisation equation) and culls
primitives whose opacity modulation falls below a small threshold (Sec. 4.2,
opacity modulation).  Neither the threshold nor the footprint is given, so both
are fixed here as a sequence of binary32 operations (+ - * / sqrt floor, each
correctly rounded, no fused multiply-add).  A pixel receives every member of its
tile's list and nothing else, so membership is part of what the renderer
computes; the image values themselves are computed in FP64 elsewhere
(``oracle.focus``).

Readings of the paper taken here:
  * scale activation s = exp(l) * scale_mod (Sec. 7, S = diag(mod * s); scales are
    stored log-transformed, Sec. 4.3 quantisation);
  * quaternion order (w, x, y, z), normalised before use;
  * axial cull: a (Gaussian, slice) pair is kept iff q_ax = m^2 / D <= q_cut with
    m = mu_z - z, D = sigma_z^2 + Sigma_zz; q_ax equals the Mahalanobis change in
    the opacity-modulation equation, so the cull keeps opacity_r >= exp(-q_cut/2)
    (default q_cut = 2 ln 255, i.e. opacity_r >= 1/255);
  * footprint: the axis-aligned box of the k-sigma ellipse of Sigma_2d (k = 3),
    converted to 16x16 tiles of the slice's pixel grid and clamped to the grid;
  * pixel (px, py) of a slice has centre (x0 + (px + 1/2) dx, y0 + (py + 1/2) dy);
  * oblique slices (the general camera of the supplement's forward derivation,
    mu_c = R_c mu + t, Sigma_c = R_c Sigma R_c^T): a slice may carry a pose
    (R_c row-major, t), and then samples the plane z_c = z of the camera frame.
    In binary32, R' = R_c R_q entry by entry as (R_c[i][0] R_q[0][j] +
    R_c[i][1] R_q[1][j]) + R_c[i][2] R_q[2][j], the covariance and adjugate
    entries are the quadratic forms below with R' in place of R_q, and
    mu_c[i] = ((R_c[i][0] mu_x + R_c[i][1] mu_y) + R_c[i][2] mu_z) + t[i].  The
    identity pose reproduces the axial slice bit for bit.

The exponential needed for s = exp(l) is not correctly rounded on any machine, so
the specification defines its own: Cody-Waite range reduction with the two-part
ln 2 split (C1 = 355/512) followed by the degree-7 Taylor polynomial of e^r on
|r| <= ln2/2, evaluated by Horner's rule with separately rounded multiply and add.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32

# ---- constants of the specification (all exactly representable in binary32) ----
LOG2E = f32(1.4426950408889634)
CW_C1 = f32(0.693359375)                 # 355/512: k * C1 exact for |k| <= 2^14
CW_C2 = f32(-2.12194440054690583e-4)     # ln 2 - C1, rounded to binary32
TAYLOR = [f32(1.0 / 5040.0), f32(1.0 / 720.0), f32(1.0 / 120.0), f32(1.0 / 24.0),
          f32(1.0 / 6.0), f32(0.5), f32(1.0), f32(1.0)]
EXP_LO, EXP_HI = f32(-87.0), f32(88.0)
TILE = 16
Q_CUT_DEFAULT = f32(2.0 * np.log(255.0))
BBOX_DEFAULT = f32(3.0)


def spec_exp(x):
    """e^x in binary32 by Cody-Waite reduction + degree-7 Taylor/Horner (see module doc)."""
    x = np.asarray(x, dtype=f32)
    x = np.minimum(np.maximum(x, EXP_LO), EXP_HI)
    k = np.rint(x * LOG2E)                       # round half to even, binary32
    r = (x - k * CW_C1) - k * CW_C2
    p = np.full_like(x, TAYLOR[0])
    for c in TAYLOR[1:]:
        p = p * r + c                            # two roundings: product, then sum
    ki = k.astype(np.int32)
    two_k = ((ki + 127).astype(np.uint32) << np.uint32(23)).view(f32)
    return (p * two_k).astype(f32)


def _cov32(ls, q, scale_mod):
    s0 = spec_exp(ls[0]) * scale_mod
    s1 = spec_exp(ls[1]) * scale_mod
    s2 = spec_exp(ls[2]) * scale_mod
    qw, qx, qy, qz = q[0], q[1], q[2], q[3]
    n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz
    rn = np.sqrt(n2)
    with np.errstate(divide="ignore", invalid="ignore"):
        w, x, y, z = qw / rn, qx / rn, qy / rn, qz / rn
    two = f32(2.0)
    one = f32(1.0)
    xx, yy, zz = x * x, y * y, z * z
    xy, xz, yz = x * y, x * z, y * z
    wx, wy, wz = w * x, w * y, w * z
    R = [[one - two * (yy + zz), two * (xy - wz), two * (xz + wy)],
         [two * (xy + wz), one - two * (xx + zz), two * (yz - wx)],
         [two * (xz - wy), two * (yz + wx), one - two * (xx + yy)]]
    v0, v1, v2 = s0 * s0, s1 * s1, s2 * s2
    out = _forms(R, v0, v1, v2)
    out.update(n2=n2, R=R, v=(v0, v1, v2))
    return out


def _forms(R, v0, v1, v2):
    """Covariance R diag(v) R^T and adjugate R diag(v1 v2, v0 v2, v0 v1) R^T entries."""
    P0, P1, P2 = v1 * v2, v0 * v2, v0 * v1

    def quad(a, b, w0, w1, w2):
        # sum_j (R[a][j] * R[b][j]) * w_j, summed left to right
        return (((R[a][0] * R[b][0]) * w0 + (R[a][1] * R[b][1]) * w1)
                + (R[a][2] * R[b][2]) * w2)

    return dict(
        sxx=quad(0, 0, v0, v1, v2), sxy=quad(0, 1, v0, v1, v2), sxz=quad(0, 2, v0, v1, v2),
        syy=quad(1, 1, v0, v1, v2), syz=quad(1, 2, v0, v1, v2), szz=quad(2, 2, v0, v1, v2),
        adj00=quad(0, 0, P0, P1, P2), adj01=quad(0, 1, P0, P1, P2),
        adj11=quad(1, 1, P0, P1, P2), adj22=quad(2, 2, P0, P1, P2),
        detS=(v0 * v1) * v2,
    )


def pose32(act, pose):
    """activate32 output seen from a posed slice's camera frame (binary32).

    pose: 12 numbers, R_c row-major then t."""
    pose = np.asarray(pose, dtype=np.float64).astype(f32).reshape(-1)
    Rc = pose[0:9].reshape(3, 3)
    t = pose[9:12]
    R = act["R"]
    Rp = [[(Rc[i][0] * R[0][j] + Rc[i][1] * R[1][j]) + Rc[i][2] * R[2][j] for j in range(3)] for i in range(3)]
    out = dict(act)
    out.update(_forms(Rp, *act["v"]))
    mu = (act["mux"], act["muy"], act["muz"])
    m = [((Rc[i][0] * mu[0] + Rc[i][1] * mu[1]) + Rc[i][2] * mu[2]) + t[i] for i in range(3)]
    out.update(mux=m[0], muy=m[1], muz=m[2], R=Rp)
    return out


def activate32(params, scale_mod=1.0):
    """Per-Gaussian binary32 quantities of the specification.

    params: float32 array [11, N] with rows mu_x, mu_y, mu_z, l_x, l_y, l_z,
    q_w, q_x, q_y, q_z, alpha.  Returns float32 arrays [N] (covariance Sigma and
    its adjugate, both symmetric, as their unique entries) plus the boolean
    'ok': all eleven values finite and |q|^2 > 0.
    """
    p = np.asarray(params, dtype=f32)
    ok = np.all(np.isfinite(p), axis=0)
    d = _cov32(p[3:6], p[6:10], f32(scale_mod))
    ok = ok & (d["n2"] > 0)
    return dict(ok=ok, mux=p[0], muy=p[1], muz=p[2], **d)


def slice_records32(act, sl, q_cut=Q_CUT_DEFAULT, bbox=BBOX_DEFAULT):
    """Binary32 axial test and tile rectangle of every Gaussian on one slice.

    act: output of activate32.  sl: dict with z, sigma_z, x0, y0, dx, dy,
    width, height.  Returns dict with boolean 'member' [N] and int32 tile bounds
    tx0, tx1, ty0, ty1 (inclusive, clamped) valid where member is True.
    """
    z, sz = f32(sl["z"]), f32(sl["sigma_z"])
    x0, y0, dx, dy = f32(sl["x0"]), f32(sl["y0"]), f32(sl["dx"]), f32(sl["dy"])
    ntx = (int(sl["width"]) + TILE - 1) // TILE
    nty = (int(sl["height"]) + TILE - 1) // TILE
    q_cut, bbox = f32(q_cut), f32(bbox)
    one = f32(1.0)
    inv16 = f32(1.0 / TILE)
    with np.errstate(all="ignore"):
        m = act["muz"] - z
        s2 = sz * sz
        D = s2 + act["szz"]
        qax = (m * m) / D
        axial = qax <= q_cut
        invD = one / D
        w = one / (one + act["szz"] / s2)
        A = w * act["sxx"] + act["adj11"] * invD
        C = w * act["syy"] + act["adj00"] * invD
        u = act["sxz"] * invD
        v = act["syz"] * invD
        mx = act["mux"] - u * m
        my = act["muy"] - v * m
        rx = bbox * np.sqrt(A)
        ry = bbox * np.sqrt(C)
        xl = np.floor((((mx - rx) - x0) / dx) * inv16)
        xh = np.floor((((mx + rx) - x0) / dx) * inv16)
        yl = np.floor((((my - ry) - y0) / dy) * inv16)
        yh = np.floor((((my + ry) - y0) / dy) * inv16)
        vis = (xh >= 0) & (xl <= f32(ntx - 1)) & (yh >= 0) & (yl <= f32(nty - 1))
        member = act["ok"] & axial & vis
        tx0 = np.where(member, np.maximum(xl, f32(0)), 0).astype(np.int32)
        tx1 = np.where(member, np.minimum(xh, f32(ntx - 1)), -1).astype(np.int32)
        ty0 = np.where(member, np.maximum(yl, f32(0)), 0).astype(np.int32)
        ty1 = np.where(member, np.minimum(yh, f32(nty - 1)), -1).astype(np.int32)
    return dict(member=member, tx0=tx0, tx1=tx1, ty0=ty0, ty1=ty1, ntx=ntx, nty=nty,
                qax=qax, axial=act["ok"] & axial)


def bins(params, slices, q_cut=Q_CUT_DEFAULT, bbox=BBOX_DEFAULT, scale_mod=1.0, exact=False):
    """Sorted tile lists of a batch of slices (the binning the renderer must reproduce).

    Bins are numbered slice by slice (in the order given), tiles row-major within a
    slice.  Each bin's list holds the indices of its member Gaussians in ascending
    order.  With exact=True every Gaussian whose eleven parameters are finite is a
    member of every tile (no axial cull, no footprint).

    Returns (keys, ranges): keys is an int64 array of (bin << 32 | gaussian) in
    ascending order; ranges is an int64 array [n_bins, 2] of [start, end).
    """
    act = activate32(params, scale_mod)
    keys = []
    nbins = 0
    starts = []
    for sl in slices:
        ntx = (int(sl["width"]) + TILE - 1) // TILE
        nty = (int(sl["height"]) + TILE - 1) // TILE
        if exact:
            idx = np.nonzero(act["ok"])[0]
            for t in range(ntx * nty):
                keys.append(((nbins + t) << 32) + idx.astype(np.int64))
        else:
            r = slice_records32(pose32(act, sl["pose"]) if sl.get("pose") is not None else act, sl, q_cut, bbox)
            idx = np.nonzero(r["member"])[0]
            wx = (r["tx1"][idx] - r["tx0"][idx] + 1).astype(np.int64)
            wy = (r["ty1"][idx] - r["ty0"][idx] + 1).astype(np.int64)
            cnt = wx * wy
            g = np.repeat(idx.astype(np.int64), cnt)
            j = np.arange(int(cnt.sum()), dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
            txs = np.repeat(r["tx0"][idx].astype(np.int64), cnt) + j % np.repeat(wx, cnt)
            tys = np.repeat(r["ty0"][idx].astype(np.int64), cnt) + j // np.repeat(wx, cnt)
            keys.append(((nbins + tys * ntx + txs) << 32) + g)
        starts.append(nbins)
        nbins += ntx * nty
    keys = np.sort(np.concatenate(keys)) if keys else np.zeros(0, np.int64)
    b = keys >> 32
    ranges = np.zeros((nbins, 2), np.int64)
    edges = np.searchsorted(b, np.arange(nbins + 1))
    ranges[:, 0] = edges[:-1]
    ranges[:, 1] = edges[1:]
    return keys, ranges
