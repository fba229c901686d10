"""Serving (continuous batching over resident 16-bit volumes) against the oracle (GPU).

Bars: each served image is within 1e-5 (relative to its maximum) of the
oracle evaluated on the dequantised parameters (the kernels' arithmetic), and
for the default 16-bit storage (GP_Q16) within 2e-3 of the oracle on the
float32 masters; a request renders bitwise the same alone and inside a batch.
FP16 and BF16 storage are checked for arithmetic only: on these thin
filaments their quaternion rounding alone exceeds 2e-3.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import focus
from paper_2603_20611_amd import synth

pytestmark = pytest.mark.gpu

EXTENT = (128.0, 128.0, 32.0)


def _say(msg):
    print(f"[serving] {msg}", flush=True)
    sys.stdout.flush()


def _bf16(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32)


def _q16_quat(q):
    """The header's fixed-point rule for unit quaternions, in binary32."""
    f = np.float32
    q = np.asarray(q, f)
    with np.errstate(all="ignore"):
        n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]
        qn = q / np.sqrt(n2)
        qn = np.where((n2 > 0) & np.isfinite(qn), qn, f(0))
    v = np.clip(np.rint(qn * f(32767.0)), -32767, 32767).astype(np.int16)
    return v.astype(f) / f(32767.0)


def _dequant(p, dtype):
    from paper_2603_20611_amd import binding as B
    q = p.copy()
    if dtype == B.GP_F16:
        q[3:11] = p[3:11].astype(np.float16).astype(np.float32)
    elif dtype == B.GP_BF16:
        q[3:11] = _bf16(p[3:11])
    elif dtype == B.GP_Q16:
        q[3:6] = p[3:6].astype(np.float16).astype(np.float32)
        q[10] = p[10].astype(np.float16).astype(np.float32)
        q[6:10] = _q16_quat(p[6:10])
    return q


def _volumes(sizes, seed=40):
    return [synth.gaussians_microscopy(n, EXTENT, seed + i) for i, n in enumerate(sizes)]


def _requests(n, n_vol, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        res = int(rng.choice([64, 96, 128]))
        out.append(dict(volume=int(rng.integers(0, n_vol)), z=float(rng.uniform(0, EXTENT[2])),
                        sigma_z=float(rng.choice([0.5, 1.0, 2.0, 3.0])), width=res, height=res,
                        dx=EXTENT[0] / res, dy=EXTENT[1] / res))
    return out


def _server(vols, **cfg):
    from paper_2603_20611_amd import serve
    base = dict(max_gaussians=1 << 20, max_records=1 << 20, max_instances=4 << 20, max_bins=64 * 64,
                max_batch=32, slots=2)
    base.update(cfg)
    sv = serve.Server(**base)
    ids = [sv.add_volume(torch.from_numpy(v).cuda().contiguous()) for v in vols]
    return sv, ids


def _run(sv, reqs):
    outs, tickets = [], []
    for r in reqs:
        o = torch.empty(r["width"] * r["height"], device="cuda")
        outs.append(o)
        tickets.append(sv.submit(r["volume"], r["z"], r["sigma_z"], o, r["width"], r["height"], dx=r["dx"],
                                 dy=r["dy"]))
    res = [sv.poll(t, timeout_us=30_000_000) for t in tickets]
    torch.cuda.synchronize()
    return [o.cpu().numpy().reshape(r["height"], r["width"]) for o, r in zip(outs, reqs)], res


def _slice(r):
    return dict(z=r["z"], sigma_z=r["sigma_z"], x0=0.0, y0=0.0, dx=r["dx"], dy=r["dy"], width=r["width"],
                height=r["height"])


def _rel(a, b):
    return float(np.abs(a - b).max()) / max(float(np.abs(b).max()), 1e-30)


@pytest.mark.parametrize("dtype_name", ["q16", "f16", "bf16"])
def test_served_images_match_oracle(gp, dtype_name):
    from paper_2603_20611_amd import binding as B
    dtype = {"q16": B.GP_Q16, "f16": B.GP_F16, "bf16": B.GP_BF16}[dtype_name]
    _say(f"served images vs oracle ({dtype_name})")
    vols = _volumes([3000, 8000, 15000, 30000])
    sv, ids = _server(vols, attr_dtype=dtype)
    reqs = _requests(24, len(vols), seed=1)
    imgs, res = _run(sv, reqs)
    assert all(r.status == 0 for r in res)
    assert max(r.batch_size for r in res) > 1
    worst_k, worst_m = 0.0, 0.0
    for img, r in zip(imgs, reqs):
        p = vols[r["volume"]]
        ref_q = focus.render(_dequant(p, dtype), [_slice(r)])[0].numpy()
        worst_k = max(worst_k, _rel(img, ref_q))
        ref_m = focus.render(p, [_slice(r)])[0].numpy()
        worst_m = max(worst_m, _rel(img, ref_m))
    _say(f"{dtype_name}: kernel arithmetic {worst_k:.2e}, vs float32 masters {worst_m:.2e}")
    assert worst_k <= 1e-5
    if dtype == B.GP_Q16:
        assert worst_m <= 2e-3
    st = sv.stats()
    assert st.completed == len(reqs) and st.volumes == 4
    sv.close()


def test_same_alone_and_in_a_batch(gp):
    _say("alone vs in a batch")
    vols = _volumes([5000, 12000, 20000])
    sv, ids = _server(vols)
    reqs = _requests(40, len(vols), seed=2)
    target = reqs[17]
    alone, res_a = _run(sv, [target])
    mix, res_m = _run(sv, reqs)
    assert res_a[0].batch_size == 1 and res_m[17].batch_size > 1
    assert np.array_equal(alone[0], mix[17])
    sv.close()


def test_graph_and_plain_launches_agree(gp):
    _say("graph replay vs plain launches")
    vols = _volumes([6000, 9000])
    reqs = _requests(20, len(vols), seed=3)
    sv_g, _ = _server(vols, use_graphs=1)
    a, _ = _run(sv_g, reqs)
    sv_g.close()
    sv_p, _ = _server(vols, use_graphs=0, max_batch=1, slots=1)
    b, res = _run(sv_p, reqs)
    sv_p.close()
    assert all(r.batch_size == 1 for r in res)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_overflowing_batches_are_rerun_alone(gp):
    """Requests whose lists the admission estimate undercounts about 3x (6,000 small
    Gaussians centred on tile corners of the 256^2 grid, each box on four tiles):
    one alone fits the 30,000-entry capacity, two together do not, so the batches
    the estimate admits overflow, are split, and every request reruns alone and
    matches the oracle."""
    from paper_2603_20611_amd import binding as B
    _say("overflow retry")
    vol = _corner_volume(6000, 256, seed=44)
    rng = np.random.default_rng(45)
    reqs = [dict(volume=0, z=float(rng.uniform(15.0, 17.0)), sigma_z=3.0, width=256, height=256,
                 dx=EXTENT[0] / 256, dy=EXTENT[1] / 256) for _ in range(12)]
    sv, _ = _server([vol], max_instances=30000, max_records=1 << 16, slots=1)
    imgs, res = _run(sv, reqs)
    st = sv.stats()
    assert st.retries > 0
    for img, r, rr in zip(imgs, reqs, res):
        assert rr.status == 0
        ref = focus.render(_dequant(vol, B.GP_Q16), [_slice(r)])[0].numpy()
        assert _rel(img, ref) <= 1e-5
    sv.close()


def test_errors_budget_and_shutdown(gp):
    from paper_2603_20611_amd import binding as B, serve
    _say("errors, budget, shutdown")
    vols = _volumes([4000, 4000])
    per_volume = 4032 * (12 + 16)   # float32 means + 16-bit attributes
    sv = serve.Server(hbm_budget_bytes=per_volume + 100, max_gaussians=1 << 16, max_records=1 << 18,
                      max_instances=1 << 20, max_bins=4096, max_batch=8, slots=2)
    vid = sv.add_volume(torch.from_numpy(vols[0]).cuda())
    with pytest.raises(B.GpError) as e:
        sv.add_volume(torch.from_numpy(vols[1]).cuda())
    assert e.value.status == B.GP_ENOMEM
    out = torch.empty(64 * 64, device="cuda")
    with pytest.raises(B.GpError) as e:
        sv.submit(vid + 5, 1.0, 1.0, out, 64, 64)
    assert e.value.status == B.GP_EINVAL
    with pytest.raises(B.GpError) as e:
        sv.poll(123456, 0)
    assert e.value.status == B.GP_EINVAL
    outs = [torch.empty(128 * 128, device="cuda") for _ in range(60)]
    tickets = [sv.submit(vid, float(i % 30), 1.0, o, 128, 128) for i, o in enumerate(outs)]
    first = sv.poll(tickets[-1], 0)
    assert first is None or first.status == 0
    sv.close()      # cancels what is queued, waits for what runs
    torch.cuda.synchronize()


# --------------------------------------------------------------------------- benchmark configuration
BENCH_SERVER = dict(max_gaussians=64 << 20, max_records=24 << 20, max_instances=48 << 20, max_bins=64 * 4096,
                    max_batch=64, slots=3, use_graphs=1)


def test_bench_config_mixed_grids(gp):
    """The server as the benchmark configures it (262,144-bin batches, captured
    graphs, three slots, GP_Q16 storage) on volumes of the serving workload's
    generator (sizes log-uniform in [20k, 1M], 512 x 512 x 128 extent) and requests
    for 256^2, 512^2 and 1024^2 grids over that extent.  Batches of more than 4,096
    bins over mixed grids take the work-queue raster with a per-bin slice search.
    Sampled pixels of every image (its brightest included) are checked against the
    oracle on the dequantised parameters (1e-5) and on the float32 masters (2e-3),
    and one request rendered alone equals its image in the mix bit for bit."""
    from paper_2603_20611_amd import binding as B, serve
    _say("benchmark server configuration, mixed 256/512/1024 grids")
    vols = synth.serving_volumes(5, 20_000, 1_000_000, (512.0, 512.0, 128.0), seed=5)
    reqs = synth.serving_requests(30, len(vols), depth=128.0, extent=512.0, seed=6)
    sv = serve.Server(**BENCH_SERVER)
    for v in vols:
        sv.add_volume(torch.from_numpy(v).cuda().contiguous())
    outs, tickets = [], []
    for r in reqs:
        o = torch.empty(r["res"] * r["res"], device="cuda")
        outs.append(o)
        tickets.append(sv.submit(r["volume"], r["z"], r["sigma_z"], o, r["res"], r["res"], dx=r["dx"], dy=r["dx"]))
    res = [sv.poll(t, timeout_us=60_000_000) for t in tickets]
    torch.cuda.synchronize()
    assert all(x.status == 0 for x in res)
    # the batches that ran: bins and grids per batch
    by_batch = {}
    for r, x in zip(reqs, res):
        by_batch.setdefault(x.batch_id, []).append(r["res"])
    bins = {b: sum(((g + 15) // 16) ** 2 for g in grids) for b, grids in by_batch.items()}
    mixed_big = [b for b, grids in by_batch.items() if bins[b] > 4096 and len(set(grids)) > 1]
    _say(f"{len(by_batch)} batches, sizes {sorted(len(g) for g in by_batch.values())}, "
         f"{len(mixed_big)} with > 4096 bins over mixed grids")
    assert mixed_big, "no batch took the work-queue raster over mixed grids"
    imgs = [o.cpu().numpy().astype(np.float64).reshape(r["res"], r["res"]) for o, r in zip(outs, reqs)]
    rng = np.random.default_rng(7)
    worst_k, worst_m = 0.0, 0.0
    for img, r in zip(imgs, reqs):
        p = vols[r["volume"]]
        sl = dict(z=r["z"], sigma_z=r["sigma_z"], x0=0.0, y0=0.0, dx=r["dx"], dy=r["dx"], width=r["res"],
                  height=r["res"])
        iy, ix = np.unravel_index(int(np.argmax(img)), img.shape)
        px = np.concatenate([rng.integers(0, r["res"], 24), [ix, r["res"] - 1]])
        py = np.concatenate([rng.integers(0, r["res"], 24), [iy, r["res"] - 1]])
        ref_q = focus.render_pixels(_dequant(p, B.GP_Q16), sl, px, py)
        ref_m = focus.render_pixels(p, sl, px, py)
        got = img[py, px]
        worst_k = max(worst_k, float(np.abs(got - ref_q).max()) / max(abs(float(ref_q[-2])), 1e-30))
        worst_m = max(worst_m, float(np.abs(got - ref_m).max()) / max(abs(float(ref_m[-2])), 1e-30))
    _say(f"kernel arithmetic {worst_k:.2e}, vs float32 masters {worst_m:.2e}")
    assert worst_k <= 1e-5
    assert worst_m <= 2e-3
    # one request of a mixed batch, alone
    j = next(i for i, x in enumerate(res) if x.batch_id in mixed_big)
    r = reqs[j]
    o = torch.empty(r["res"] * r["res"], device="cuda")
    x = sv.poll(sv.submit(r["volume"], r["z"], r["sigma_z"], o, r["res"], r["res"], dx=r["dx"], dy=r["dx"]),
                timeout_us=60_000_000)
    torch.cuda.synchronize()
    assert x.status == 0 and x.batch_size == 1
    assert np.array_equal(o.cpu().numpy().astype(np.float64).reshape(r["res"], r["res"]), imgs[j])
    sv.close()


def test_split_groups_and_oversized_request(gp):
    """Batches sort list entries by the low bits that tell one group's bins apart
    (14 bits in the captured launches), so the server splits a volume's requests
    into groups of at most 16,383 tiles, and launches a batch holding a single
    request of more tiles without the graphs.  Six 1024^2 requests on one volume
    (two groups) in one batch, then one 2560^2 request (25,600 tiles) beside a
    512^2 one: sampled pixels against the oracle on the dequantised parameters
    (1e-5), and each image equal bit for bit to the same request rendered alone."""
    from paper_2603_20611_amd import binding as B, serve
    _say("split groups and an oversized request")
    vols = synth.serving_volumes(2, 60_000, 120_000, (512.0, 512.0, 128.0), seed=15)
    sv = serve.Server(**BENCH_SERVER)
    for v in vols:
        sv.add_volume(torch.from_numpy(v).cuda().contiguous())
    torch.cuda.synchronize()
    reqs = [dict(volume=0, z=20.0 + 15.0 * k, sigma_z=[0.5, 1.0, 2.0][k % 3], width=1024, height=1024, dx=0.5, dy=0.5)
            for k in range(6)]
    # second batch: the oversized request beside a 512^2 one (launched without the graphs)
    reqs += [dict(volume=1, z=64.0, sigma_z=1.0, width=2560, height=2560, dx=0.2, dy=0.2),
             dict(volume=0, z=70.0, sigma_z=3.0, width=512, height=512, dx=1.0, dy=1.0)]
    outs = [torch.empty(r["width"] * r["height"], device="cuda") for r in reqs]
    res = []
    for lo, hi in ((0, 6), (6, 8)):
        tickets = sv.submit_many(reqs[lo:hi], outs[lo:hi])
        res += [sv.poll(t, timeout_us=60_000_000) for t in tickets]
        torch.cuda.synchronize()
    assert all(x.status == 0 for x in res)
    _say(f"batch sizes {[x.batch_size for x in res]}")
    assert res[0].batch_size == 6 and res[6].batch_size == 2, "the requests did not share their batches"
    rng = np.random.default_rng(16)
    worst = 0.0
    for r, o in zip(reqs, outs):
        img = o.cpu().numpy().astype(np.float64).reshape(r["height"], r["width"])
        sl = dict(z=r["z"], sigma_z=r["sigma_z"], x0=0.0, y0=0.0, dx=r["dx"], dy=r["dy"], width=r["width"],
                  height=r["height"])
        iy, ix = np.unravel_index(int(np.argmax(img)), img.shape)
        px = np.concatenate([rng.integers(0, r["width"], 20), [ix]])
        py = np.concatenate([rng.integers(0, r["height"], 20), [iy]])
        ref = focus.render_pixels(_dequant(vols[r["volume"]], B.GP_Q16), sl, px, py)
        worst = max(worst, float(np.abs(img[py, px] - ref).max()) / max(abs(float(ref[-1])), 1e-30))
        alone = torch.empty_like(o)
        x = sv.poll(sv.submit(r["volume"], r["z"], r["sigma_z"], alone, r["width"], r["height"], dx=r["dx"],
                              dy=r["dy"]), timeout_us=60_000_000)
        torch.cuda.synchronize()
        assert x.status == 0 and x.batch_size == 1
        assert torch.equal(alone, o)
    _say(f"kernel arithmetic {worst:.2e}")
    assert worst <= 1e-5
    sv.close()


def test_volumes_added_while_serving(gp):
    """Volumes added from another thread while requests are admitted and launched:
    every request completes and matches the image it renders on a quiet server."""
    import threading
    from paper_2603_20611_amd import serve
    _say("volumes added while serving")
    vols = _volumes([3000, 4000, 5000, 6000, 7000, 8000, 9000, 10000], seed=70)
    sv = serve.Server(max_gaussians=1 << 20, max_records=1 << 20, max_instances=4 << 20, max_bins=64 * 64,
                      max_batch=16, slots=3)
    first = sv.add_volume(torch.from_numpy(vols[0]).cuda().contiguous())
    tens = [torch.from_numpy(v).cuda().contiguous() for v in vols[1:]]
    torch.cuda.synchronize()
    ids = [first]

    def adder():
        for t in tens:
            ids.append(sv.add_volume(t))

    th = threading.Thread(target=adder)
    th.start()
    outs, tickets, used = [], [], []
    rng = np.random.default_rng(71)
    for i in range(200):
        vid = ids[int(rng.integers(0, len(ids)))]     # only volumes already added
        o = torch.empty(64 * 64, device="cuda")
        z = float(rng.uniform(0, EXTENT[2]))
        outs.append(o)
        used.append((vid, z))
        tickets.append(sv.submit(vid, z, 1.0, o, 64, 64, dx=2.0, dy=2.0))
    th.join()
    res = [sv.poll(t, timeout_us=60_000_000) for t in tickets]
    torch.cuda.synchronize()
    assert all(x.status == 0 for x in res)
    assert sv.stats().volumes == len(vols)
    quiet = serve.Server(max_gaussians=1 << 20, max_records=1 << 20, max_instances=4 << 20, max_bins=64 * 64,
                         max_batch=16, slots=3)
    order = {vid: k for k, vid in enumerate(ids)}
    qids = [quiet.add_volume(torch.from_numpy(v).cuda().contiguous()) for v in vols]
    for j in (0, 57, 123, 199):
        vid, z = used[j]
        o = torch.empty(64 * 64, device="cuda")
        x = quiet.poll(quiet.submit(qids[order[vid]], z, 1.0, o, 64, 64, dx=2.0, dy=2.0), timeout_us=30_000_000)
        torch.cuda.synchronize()
        assert x.status == 0 and torch.equal(o, outs[j])
    quiet.close()
    sv.close()


def test_submit_many_and_arrival_stamps(gp):
    """Requests queued in one call render what single submissions render, and a
    request's latency runs from the arrival stamp it was given."""
    from paper_2603_20611_amd import serve
    _say("submit_many, arrival stamps")
    vols = _volumes([5000, 9000], seed=80)
    sv, ids = _server(vols)
    reqs = _requests(12, len(vols), seed=81)
    single, _ = _run(sv, reqs)
    outs = [torch.empty(r["width"] * r["height"], device="cuda") for r in reqs]
    now = serve.Server.clock_ms()
    stamps = [now - 40.0] * len(reqs)
    tickets = sv.submit_many([dict(r, volume=ids[r["volume"]]) for r in reqs], outs, stamps)
    res = [sv.poll(t, timeout_us=30_000_000) for t in tickets]
    torch.cuda.synchronize()
    assert all(x.status == 0 for x in res)
    assert min(x.latency_ms for x in res) >= 40.0
    for o, r, a in zip(outs, reqs, single):
        assert np.array_equal(o.cpu().numpy().reshape(r["height"], r["width"]), a)
    sv.close()


def _corner_volume(n, res, seed):
    """n small isotropic Gaussians centred on tile corners of a res^2 grid over the
    serving extent (each 3-sigma box straddles a corner: 4 tiles, against the 2.2
    of a box of its width at a random offset), in a slab around z = 16."""
    rng = np.random.default_rng(seed)
    t = res // 16
    dx = EXTENT[0] / res
    p = np.zeros((11, n), np.float32)
    p[0] = rng.integers(1, t, n) * 16 * dx
    p[1] = rng.integers(1, t, n) * 16 * dx
    p[2] = rng.uniform(15.5, 16.5, n)
    p[3:6] = np.log(0.16)
    p[6] = 1.0
    p[10] = rng.uniform(0.1, 1.0, n)
    return p


def test_small_bucket_overflow_reruns_in_the_largest(gp):
    """A request whose lists the admission estimate undercounts (1.1 M Gaussians
    centred on tile corners of a 1024^2 grid: 4.4 M entries against an estimate of
    2.4 M) is first replayed in the smallest capacity bucket (4 M entries),
    overflows it, and is replayed in the largest: the image is still the oracle's."""
    from paper_2603_20611_amd import binding as B, serve
    _say("bucket overflow rerun")
    vol = _corner_volume(1_100_000, 1024, seed=82)
    sv = serve.Server(max_gaussians=1 << 22, max_records=1 << 22, max_instances=1 << 24, max_bins=1 << 16,
                      max_batch=8, slots=1)
    sv.add_volume(torch.from_numpy(vol).cuda().contiguous())
    r = dict(volume=0, z=16.0, sigma_z=3.0, width=1024, height=1024, dx=EXTENT[0] / 1024, dy=EXTENT[1] / 1024)
    img, res = _run(sv, [r])
    assert res[0].status == 0
    assert sv.stats().retries >= 1
    rng = np.random.default_rng(83)
    im = img[0].astype(np.float64)
    iy, ix = np.unravel_index(int(np.argmax(im)), im.shape)
    px = np.concatenate([rng.integers(0, 1024, 30), [ix]])
    py = np.concatenate([rng.integers(0, 1024, 30), [iy]])
    ref = focus.render_pixels(_dequant(vol, B.GP_Q16), _slice(r), px, py)
    err = float(np.abs(im[py, px] - ref).max()) / abs(float(ref[-1]))
    _say(f"rerun image: rel err {err:.2e}, retries {sv.stats().retries}")
    assert err <= 1e-5
    sv.close()
