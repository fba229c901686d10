"""The Morton-ordered 14/12-bit codec on the GPU against the oracle.

Bars: codes, header and order bit-exact (integer work); images of the coded
set within 1e-5 of the oracle on the decoded parameters, tile lists bit-exact.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import focus, quant, spec32
from paper_2603_20611_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[codec] {msg}", flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.abs(a - b).max()) / max(float(np.abs(b).max()), 1e-30)


@pytest.mark.parametrize("case", ["one", "ragged", "microscopy", "degenerate"])
def test_codes_match_oracle(gp, case):
    from paper_2603_20611_amd import render as R
    _say(f"encode {case}")
    if case == "one":
        p = synth.gaussians_uniform(1, (10.0, 10.0, 10.0), 0.0, 0.3, seed=1)
    elif case == "ragged":
        p = synth.gaussians_uniform(777, (64.0, 48.0, 32.0), np.log(1.5), 0.3, seed=2)
        p[0, 5] = np.nan
        p[6:10, 9] = 0.0                    # zero quaternion
        p[10, 11] = 1.7                     # intensity above 1: clamped
    elif case == "microscopy":
        p = synth.gaussians_microscopy(50000, (512.0, 512.0, 128.0), seed=3)
    else:
        p = synth.gaussians_uniform(300, (8.0, 8.0, 8.0), 0.0, 0.2, seed=4)
        p[0:3] = 3.0
    pt = torch.from_numpy(np.ascontiguousarray(p)).cuda()
    codes, header, perm = R.encode(pt)
    torch.cuda.synchronize()
    e_codes, e_header, e_perm = quant.encode(p)
    assert np.array_equal(header.cpu().numpy(), e_header)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), e_perm)
    assert np.array_equal(codes.cpu().numpy().view(np.uint16)[:, :p.shape[1]], e_codes)


def test_coded_render_matches_oracle(gp):
    from paper_2603_20611_amd import render as R
    _say("render of a coded set")
    p = synth.gaussians_microscopy(20000, (128.0, 128.0, 32.0), seed=5)
    pt = torch.from_numpy(p).cuda()
    codes, header, perm = R.encode(pt)
    e_codes, e_header, _ = quant.encode(p)
    d = quant.decode(e_codes, e_header)
    slices = [dict(z=z, sigma_z=s, x0=0.0, y0=0.0, dx=1.0, dy=1.0, width=128, height=112)
              for z, s in ((4.5, 1.0), (16.0, 2.0), (27.25, 0.5))]
    ws = R.Workspace()
    img = R.render_coded(codes, header, p.shape[1], slices, ws=ws).cpu().numpy()
    ref = np.concatenate([x.numpy().reshape(-1) for x in focus.render(d, slices)])
    err = _rel(img, ref)
    _say(f"coded render rel err {err:.2e}")
    assert err <= 1e-5
    keys, _ = spec32.bins(d, slices)
    nb = sum(((s["width"] + 15) // 16) * ((s["height"] + 15) // 16) for s in slices)
    got, _ = ws.export_bins(nb, keys.size + 16)
    assert np.array_equal(got, keys)
    ws.close()


def test_coded_serving_matches_oracle(gp):
    from paper_2603_20611_amd import binding as B, serve
    _say("serving from coded volumes")
    extent = (128.0, 128.0, 32.0)
    vols = [synth.gaussians_microscopy(n, extent, seed=40 + i) for i, n in enumerate([3000, 9000])]
    sv = serve.Server(max_gaussians=1 << 16, max_records=1 << 20, max_instances=4 << 20, max_bins=64 * 64,
                      max_batch=16, slots=2, attr_dtype=B.GP_QM)
    for v in vols:
        sv.add_volume(torch.from_numpy(v).cuda())
    rng = np.random.default_rng(6)
    outs, reqs, tickets = [], [], []
    for _ in range(10):
        r = dict(volume=int(rng.integers(0, 2)), z=float(rng.uniform(0, 32)), sigma_z=float(rng.choice([1.0, 2.0])))
        o = torch.empty(96 * 96, device="cuda")
        outs.append(o)
        reqs.append(r)
        tickets.append(sv.submit(r["volume"], r["z"], r["sigma_z"], o, 96, 96, dx=128 / 96, dy=128 / 96))
    res = [sv.poll(t, timeout_us=30_000_000) for t in tickets]
    torch.cuda.synchronize()
    assert all(x.status == 0 for x in res)
    worst, worst_m = 0.0, 0.0
    for o, r in zip(outs, reqs):
        c, h, _ = quant.encode(vols[r["volume"]])
        d = quant.decode(c, h)
        sl = dict(z=r["z"], sigma_z=r["sigma_z"], x0=0.0, y0=0.0, dx=128 / 96, dy=128 / 96, width=96, height=96)
        ref = focus.render(d, [sl])[0].numpy().reshape(-1)
        worst = max(worst, _rel(o.cpu().numpy(), ref))
        worst_m = max(worst_m, _rel(o.cpu().numpy(), focus.render(vols[r["volume"]], [sl])[0].numpy().reshape(-1)))
    _say(f"coded serving: kernel arithmetic {worst:.2e}, vs float32 masters {worst_m:.2e}")
    assert worst <= 1e-5
    st = sv.stats()
    assert st.volumes == 2
    sv.close()


def test_coded_sets_are_render_only(gp):
    from paper_2603_20611_amd import binding as B, render as R
    import ctypes as C
    p = synth.gaussians_uniform(100, (16.0, 16.0, 16.0), 0.0, 0.2, seed=7)
    pt = torch.from_numpy(p).cuda()
    codes, header, _ = R.encode(pt)
    g = R.coded_struct(codes, header, 100)
    grid = B.make_grid(dict(nx=8, ny=8, nz=8))
    vol = torch.empty(512, device="cuda")
    ws = R.Workspace()
    st = B.load().gp_voxelize(ws.handle, C.byref(g), C.byref(grid), C.byref(B.default_opts()), R._ptr(vol),
                              R._stream())
    assert st == B.GP_EINVAL
    ws.close()
