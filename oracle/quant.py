"""Reference of the Morton-ordered fixed-point codec of a Gaussian set.

TEST INFRASTRUCTURE ONLY: imported by the test-suite alone.  Shares no code
with the HIP path.

The paper's compression (Sec. 4.3, "Quantization and compression"): Gaussians
are sorted along the Morton (Z-order) curve; positions, normalised to the
scene's bounding box, get 14 bits per axis; intensities are mapped to 12-bit
integers on [0, 1]; log-scales get 12 bits; quaternions are moved to the
positive half-sphere and get 12 bits per component.  (The delta coding and
LZMA stage that follow are a CPU entropy coder, not part of this codec.)

Readings, all decisions taken in binary32 with the operation order below:
  * bounding box lo, hi per axis over the finite means; log-scale range
    [lmin, lmax] over all three axes of the finite log-scales;
  * a value v on [lo, hi] with n levels (2^14 or 2^12) has code
    floor(((v - lo) / (hi - lo)) * (n - 1) + 0.5), clamped to [0, n - 1];
    code 0 if hi == lo; non-finite values get code 0;
  * intensity: normalised to [0, 1] by the largest finite intensity amax
    (the paper's opacities already lie on [0, 1]; the intensities here are
    unbounded), i.e. coded like a value on [0, amax], negatives clamped to 0;
  * quaternion: q / |q|, negated if its w < 0, each component c on [-1, 1]
    coded as floor(((c + 1) * 0.5) * 4095 + 0.5);
  * decoding: lo + code * ((hi - lo) / (n - 1)) (alpha: lo = 0, hi = amax),
    code * (2 / 4095) - 1 for quaternion components;
  * Morton key: bit 3i of the key is bit i of the x code, 3i + 1 of y,
    3i + 2 of z; the order is by key, ties by original index.
Stored: 11 uint16 planes [11][n] in Morton order, the header
(lo_x, lo_y, lo_z, hi_x, hi_y, hi_z, lmin, lmax, amax) and the permutation.
"""
import numpy as np

f32 = np.float32
POS_LEVELS = 1 << 14
ATTR_LEVELS = 1 << 12


def _code(v, lo, hi, levels):
    v = np.asarray(v, f32)
    lo, hi = f32(lo), f32(hi)
    nm1 = f32(levels - 1)
    out = np.zeros(v.shape, np.uint16)
    if not (hi > lo):
        return out
    with np.errstate(all="ignore"):
        u = (v - lo) / (hi - lo)
        c = np.floor(u * nm1 + f32(0.5))
    c = np.where(np.isfinite(c), c, f32(0))
    return np.clip(c, 0, levels - 1).astype(np.uint16)


def _decode(code, lo, hi, levels):
    lo, hi = f32(lo), f32(hi)
    step = (hi - lo) / f32(levels - 1)
    return (lo + np.asarray(code, f32) * step).astype(f32)


def header(params):
    p = np.asarray(params, f32)
    h = np.zeros(9, f32)
    for a in range(3):
        m = p[a][np.isfinite(p[a])]
        h[a], h[3 + a] = (m.min(), m.max()) if m.size else (f32(0), f32(0))
    ls = p[3:6][np.isfinite(p[3:6])]
    h[6], h[7] = (ls.min(), ls.max()) if ls.size else (f32(0), f32(0))
    al = p[10][np.isfinite(p[10])]
    h[8] = max(al.max(), f32(0)) if al.size else f32(0)
    return h


def codes(params, h=None):
    """Codes [11, n] uint16 in the original order, and the header."""
    p = np.asarray(params, f32)
    h = header(p) if h is None else np.asarray(h, f32)
    c = np.zeros((11, p.shape[1]), np.uint16)
    for a in range(3):
        c[a] = _code(p[a], h[a], h[3 + a], POS_LEVELS)
    for a in range(3):
        c[3 + a] = _code(p[3 + a], h[6], h[7], ATTR_LEVELS)
    q = p[6:10]
    with np.errstate(all="ignore"):
        n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]
        qn = q / np.sqrt(n2)
    qn = np.where(qn[0] < 0, -qn, qn)
    for r in range(4):
        with np.errstate(all="ignore"):
            u = (qn[r] + f32(1.0)) * f32(0.5)
            cc = np.floor(u * f32(ATTR_LEVELS - 1) + f32(0.5))
        cc = np.where(np.isfinite(cc), cc, f32(0))
        c[6 + r] = np.clip(cc, 0, ATTR_LEVELS - 1).astype(np.uint16)
    c[10] = _code(np.maximum(p[10], f32(0)), f32(0), h[8], ATTR_LEVELS)
    return c, h


def morton(cx, cy, cz):
    """42-bit Morton keys of 14-bit codes (uint64)."""
    key = np.zeros(np.asarray(cx).shape, np.uint64)
    for i in range(14):
        for a, c in enumerate((cx, cy, cz)):
            bit = (np.asarray(c, np.uint64) >> np.uint64(i)) & np.uint64(1)
            key |= bit << np.uint64(3 * i + a)
    return key


def encode(params):
    """(codes [11, n] uint16 in Morton order, header float32 [9], perm int64 [n])
    with codes[:, i] the codes of Gaussian perm[i]."""
    c, h = codes(params)
    key = morton(c[0], c[1], c[2])
    perm = np.argsort(key, kind="stable")
    return c[:, perm], h, perm


def decode(c, h):
    """Float32 parameters [11, n] of codes in any order."""
    c = np.asarray(c)
    h = np.asarray(h, f32)
    p = np.zeros(c.shape, f32)
    for a in range(3):
        p[a] = _decode(c[a], h[a], h[3 + a], POS_LEVELS)
    for a in range(3):
        p[3 + a] = _decode(c[3 + a], h[6], h[7], ATTR_LEVELS)
    for r in range(4):
        p[6 + r] = (np.asarray(c[6 + r], f32) * (f32(2.0) / f32(ATTR_LEVELS - 1)) - f32(1.0)).astype(f32)
    p[10] = _decode(c[10], f32(0), h[8], ATTR_LEVELS)
    return p
