"""Pins of the Morton fixed-point codec reference."""
import numpy as np
import torch

from oracle import focus, quant

f32 = np.float32


def _params(n, seed):
    rng = np.random.default_rng(seed)
    p = np.zeros((11, n), f32)
    p[0:3] = rng.uniform(0, 1, (3, n)) * np.array([[512.0], [256.0], [128.0]], f32)
    p[3:6] = rng.normal(0.2, 0.5, (3, n))
    p[6:10] = rng.normal(size=(4, n))
    p[10] = rng.uniform(0, 1, n)
    return p


def test_round_trip_within_half_a_step():
    p = _params(5000, 0)
    c, h, perm = quant.encode(p)
    d = quant.decode(c, h)
    q = p[:, perm]
    for a in range(3):
        step = (h[3 + a] - h[a]) / (quant.POS_LEVELS - 1)
        assert np.abs(d[a] - q[a]).max() <= 0.5 * step * (1 + 1e-3) + 1e-4
    step = (h[7] - h[6]) / (quant.ATTR_LEVELS - 1)
    assert np.abs(d[3:6] - q[3:6]).max() <= 0.5 * step * (1 + 1e-3) + 1e-6
    assert np.abs(d[10] - q[10]).max() <= 0.5 * h[8] / 4095 * (1 + 1e-3) + 1e-7


def test_extremes_map_to_end_codes():
    p = _params(100, 1)
    c, h = quant.codes(p)
    for a in range(3):
        assert c[a][np.argmin(p[a])] == 0 and c[a][np.argmax(p[a])] == quant.POS_LEVELS - 1
    ls = p[3:6]
    i = np.unravel_index(np.argmin(ls), ls.shape)
    j = np.unravel_index(np.argmax(ls), ls.shape)
    assert c[3 + i[0], i[1]] == 0 and c[3 + j[0], j[1]] == quant.ATTR_LEVELS - 1


def test_quaternion_half_sphere_keeps_the_rotation():
    p = _params(2000, 2)
    c, h, perm = quant.encode(p)
    d = quant.decode(c, h)
    assert (c[6] >= 2047).all()                     # w >= 0 after the sign flip
    qo = torch.from_numpy(p[6:10, perm].T.astype(np.float64))
    qo = qo / qo.norm(dim=1, keepdim=True)
    qd = torch.from_numpy(d[6:10].T.astype(np.float64))
    qd = qd / qd.norm(dim=1, keepdim=True)
    Ro = focus.quat_to_matrix(qo).numpy()
    Rd = focus.quat_to_matrix(qd).numpy()
    # 12-bit components: rotation error of order 1e-3
    assert np.abs(Ro - Rd).max() < 5e-3


def test_morton_interleave_against_integer_bit_loop():
    rng = np.random.default_rng(3)
    cx, cy, cz = (rng.integers(0, 1 << 14, 200) for _ in range(3))
    k = quant.morton(cx, cy, cz)
    for i in range(200):
        ref = 0
        for b in range(14):
            ref |= ((int(cx[i]) >> b) & 1) << (3 * b)
            ref |= ((int(cy[i]) >> b) & 1) << (3 * b + 1)
            ref |= ((int(cz[i]) >> b) & 1) << (3 * b + 2)
        assert int(k[i]) == ref
    # the unit cube in Z order
    cube = [(x, y, z) for z in (0, 1) for y in (0, 1) for x in (0, 1)]
    keys = quant.morton(*[np.array(v) for v in zip(*cube)])
    assert list(keys) == list(range(8))


def test_order_and_permutation():
    p = _params(3000, 4)
    p[0:3, 100:110] = p[0:3, 100:101]               # ties: same position
    c, h, perm = quant.encode(p)
    assert np.array_equal(np.sort(perm), np.arange(3000))
    k = quant.morton(c[0], c[1], c[2]).astype(np.uint64)
    assert (np.diff(k.astype(np.int64)) >= 0).all()
    tied = [i for i in range(3000) if 100 <= perm[i] < 110]
    assert list(perm[tied]) == sorted(perm[tied])   # ties keep the original order


def test_degenerate_ranges_and_non_finite():
    p = _params(50, 5)
    p[0:3] = 7.0
    p[3:6] = -0.5
    p[1, 3] = np.nan
    c, h = quant.codes(p)
    assert not c[0:6].any()
    d = quant.decode(c, h)
    assert (d[0] == 7.0).all() and (d[3:6] == -0.5).all()
