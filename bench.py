"""Benchmark of the Focus-Gaussian slice renderer on one MI355X.

Workload (ultrasound-shaped reconstruction, inputs resident in HBM): 500,000
learnable Gaussians (log-scales N(ln 1.2, 0.4), intensities U(0,1), means
uniform in 256 x 256 x 400), 400 axial slices of 256 x 256 pixels, sigma_z = 3.
The target stack is rendered once from a separate hidden set of 500,000
Gaussians and multiplied by Rayleigh(1) speckle.

Timed phases (each K steps after W warm-up steps, bracketed by a device
synchronisation on both sides):
  forward   one step = the whole 400-slice stack rendered in one launch sequence
            (activation, axial cull, projection, tile-key emission, radix sort,
            additive rasterisation).  `value` = rendered megapixels per second.
  train     one step = one reconstruction iteration on a batch of 8 consecutive
            slices at a random depth: forward, L1 + 0.2 D-SSIM loss gradient, backward,
            fused Adam (learning rates decayed exponentially to 0.1x over
            30,000 iterations).  Reported as fwd_bwd_iter_per_s.

The dominant kernel (additive rasterisation of the forward) is timed with HIP
events recorded by the library on the stream it launches on; its roofline is
the VALU + transcendental issue rate of the chip (4 (pixel, Gaussian) pairs per
clock per SIMD, derived below).  The CPU
oracle is timed on 64 slices of 256 x 256 of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_GAUSS = 500_000
N_SLICES = 400
RES = 256
SIGMA_Z = 3.0
TRAIN_BATCH = 8
LAMBDA_SSIM = 0.2   # weight of the D-SSIM term of the loss
# raster roofline: per (pixel, Gaussian) pair the method needs one exp2 and four
# fp32 VALU operations (offset, two FMAs of the quadratic form, accumulate).
# gfx950 issues 32 fp32 lanes/clk/SIMD (157.3 TFLOP/s fp32 over 1024 SIMDs at
# 2.4 GHz) and transcendentals at a quarter of that rate: 4*2 + 8 = 16 SIMD
# cycles per 64 pairs -> 4 pairs/clk/SIMD.
PEAK_PAIRS_PER_S = 1024 * 2.4e9 * 4.0


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed byte-counter summary,
    or None if the kernel's source has changed since the counters were taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_hbm_bytes.md")):
        for line in open(path):
            f = line.split()
            if len(f) < 5 or f[0] != "traffic" or f[1] != kernel:
                continue
            kv = dict(x.split("=", 1) for x in f[2:])
            src = os.path.join(ROOT, kv["source"])
            if not os.path.exists(src):
                return None
            if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv["sha256_16"]:
                return None
            return int(kv["bytes_per_launch"])
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(params_np, slices):
    """The oracle, as it stands, on 64 slices of the workload."""
    import torch
    from oracle import focus
    sample = slices[N_SLICES // 2 - 32:N_SLICES // 2 + 32]
    t0 = time.perf_counter()
    imgs = focus.render(params_np, sample)
    dt = time.perf_counter() - t0
    del imgs
    px = sum(s["width"] * s["height"] for s in sample)
    return {"value": round(px / dt / 1e6, 4), "unit": "Mpix/s", "cores": int(torch.get_num_threads()),
            "kind": "oracle",
            "sample": f"{len(sample)} consecutive {RES}x{RES} slices (z={sample[0]['z']}..{sample[-1]['z']}) of the "
                      f"{N_GAUSS}-Gaussian workload, float64 oracle, {dt:.1f} s"}


def serving_leg(dev, n_requests, seed=3):
    """Serving workload: 64 resident volumes (log-uniform 20k..1M Gaussians, the
    microscopy generator in a 512x512x128 extent), Poisson requests at 2,000/s
    for slices at z ~ U(0, 128), resolution in {256^2, 512^2, 1024^2}, sigma_z
    in {0.5, 1, 2, 3}.  The batched server (continuous batching, graph replay,
    3 slots) is compared with one launch per request (max_batch 1, 1 slot, no
    graphs) at the same offered load and in a closed loop (all requests queued
    at once: saturation throughput)."""
    import torch
    from paper_2603_20611_amd import serve, synth

    vols = synth.serving_volumes(64, 20_000, 1_000_000, (512.0, 512.0, 128.0), seed=seed)
    reqs = synth.serving_requests(n_requests, len(vols), depth=128.0, extent=512.0, seed=seed, rate=2000.0)
    total_g = sum(v.shape[1] for v in vols)
    log(f"serving: {len(vols)} volumes, {total_g} Gaussians, {len(reqs)} requests")
    outs = [torch.empty(r["res"] * r["res"], device=dev) for r in reqs]
    systems = {
        "batched": dict(max_batch=64, slots=3, use_graphs=1),
        "plain": dict(max_batch=1, slots=1, use_graphs=0),
    }
    result = {"volumes": len(vols), "gaussians": int(total_g), "requests": len(reqs), "offered_req_per_s": 2000.0,
              "attr_storage": "q16 (fp16 log-scales and intensity, int16 unit quaternion)"}
    for name, cfg in systems.items():
        sv = serve.Server(max_gaussians=64 << 20, max_records=24 << 20, max_instances=48 << 20,
                          max_bins=64 * 4096, **cfg)
        for v in vols:
            t = torch.from_numpy(v).to(dev).contiguous()
            sv.add_volume(t)
            del t
        torch.cuda.synchronize()

        def submit(r, o):
            return sv.submit(r["volume"], r["z"], r["sigma_z"], o, r["res"], r["res"], dx=r["dx"], dy=r["dx"])

        # warm-up (graph capture, first launches)
        for r, o in zip(reqs[:8], outs[:8]):
            sv.poll(submit(r, o), -1)
        # open loop at the offered rate
        t0 = time.perf_counter()
        tickets = []
        for r, o in zip(reqs, outs):
            delay = t0 + r["t"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(submit(r, o))
        res = [sv.poll(t, -1) for t in tickets]
        wall = time.perf_counter() - t0
        lat = np.array([x.latency_ms for x in res])
        bs = np.array([x.batch_size for x in res])
        # closed loop: everything queued at once
        t1 = time.perf_counter()
        tickets = [submit(r, o) for r, o in zip(reqs, outs)]
        res2 = [sv.poll(t, -1) for t in tickets]
        wall2 = time.perf_counter() - t1
        lat2 = np.array([x.latency_ms for x in res2])
        ok = all(x.status == 0 for x in res + res2)
        st = sv.stats()
        result[name] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                        "p99_ms": round(float(np.percentile(lat, 99)), 3),
                        "slices_per_s": round(len(reqs) / wall, 1),
                        "mean_batch": round(float(bs.mean()), 2),
                        "saturated_slices_per_s": round(len(reqs) / wall2, 1),
                        "saturated_p50_ms": round(float(np.percentile(lat2, 50)), 3),
                        "saturated_p99_ms": round(float(np.percentile(lat2, 99)), 3),
                        "all_ok": bool(ok), "retries": int(st.retries)}
        log(f"serving {name}: {result[name]}")
        sv.close()
        torch.cuda.synchronize()
    result["saturated_speedup"] = round(result["batched"]["saturated_slices_per_s"]
                                        / result["plain"]["saturated_slices_per_s"], 2)
    return result


def voxel_leg(params, dev, steps=10):
    """Voxeliser on the workload's volume: the learnable Gaussians into 256 x 256 x
    400 unit voxels (the target stack's grid), forward and backward."""
    import torch
    from paper_2603_20611_amd import render
    grid = dict(nx=RES, ny=RES, nz=N_SLICES, x0=0.0, y0=0.0, z0=0.0, dx=1.0, dy=1.0, dz=1.0)
    ws = render.Workspace()
    vol = torch.empty(RES * RES * N_SLICES, device=dev)
    gvol = torch.ones_like(vol)
    grad = torch.zeros_like(params)
    for _ in range(2):
        render.voxelize(params, grid, ws, out=vol)
        render.voxelize_backward(params, grid, gvol, ws, grad=grad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        render.voxelize(params, grid, ws, out=vol)
    torch.cuda.synchronize()
    t_f = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        render.voxelize_backward(params, grid, gvol, ws, grad=grad)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / steps
    return {"grid": [RES, RES, N_SLICES], "forward_ms": round(1e3 * t_f, 4), "fps": round(1.0 / t_f, 1),
            "backward_ms": round(1e3 * t_b, 4)}


def extras_leg(params, slices, dev, steps=5):
    """The rows the forward line does not time, on the same 500k Gaussians: the
    codec (encoding the set, and the 400-slice stack rendered from the coded
    set), an oblique batch (64 slices of 256 x 256 tilted by 30 degrees about x
    through the volume's centre, 1 apart along their normal) and one densify /
    prune pass over the whole set with synthetic statistics."""
    import torch
    from paper_2603_20611_amd import render

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def fixed_ws(draw):
        # as in the forward leg: a workspace sized by one counted render, so
        # that the timed renders run without host synchronisation
        ws_a = render.Workspace()
        draw(ws_a)
        rec, inst, _ = ws_a.check()
        del ws_a
        return render.Workspace(capacity=(int(rec * 1.3) + 4096, int(inst * 1.3) + 16384))

    n = params.shape[1]
    res = {}
    hold = {}
    t_enc = timed(lambda: hold.__setitem__("c", render.encode(params)))
    codes, header, _ = hold["c"]
    img = torch.empty(len(slices) * RES * RES, device=dev)
    ws = fixed_ws(lambda w: render.render_coded(codes, header, n, slices, ws=w, out=img))
    t_qm = timed(lambda: render.render_coded(codes, header, n, slices, ws=ws, out=img))
    res["codec"] = {"encode_ms": round(1e3 * t_enc, 4), "coded_forward_ms": round(1e3 * t_qm, 4),
                    "coded_mpix_per_s": round(len(slices) * RES * RES / t_qm / 1e6, 1), "bytes_per_gaussian": 22}
    c, s_ = np.cos(np.radians(30.0)), np.sin(np.radians(30.0))
    R = np.array([[1.0, 0.0, 0.0], [0.0, c, -s_], [0.0, s_, c]])
    centre = np.array([RES / 2.0, RES / 2.0, N_SLICES / 2.0])
    pose = np.concatenate([R.reshape(-1), -R @ centre]).astype(np.float32)
    obl = [dict(z=float(k) + 0.5, sigma_z=SIGMA_Z, x0=-RES / 2.0, y0=-RES / 2.0, dx=1.0, dy=1.0, width=RES,
                height=RES, pose=pose) for k in range(-32, 32)]
    img_o = torch.empty(len(obl) * RES * RES, device=dev)
    ws_o = fixed_ws(lambda w: render.render(params, obl, ws=w, out=img_o))
    t_ob = timed(lambda: render.render(params, obl, ws=ws_o, out=img_o))
    res["oblique"] = {"slices": len(obl), "tilt_deg": 30.0, "forward_ms": round(1e3 * t_ob, 4),
                      "mpix_per_s": round(len(obl) * RES * RES / t_ob / 1e6, 1)}
    rng = np.random.default_rng(11)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    cnt = torch.from_numpy(rng.integers(0, 12, n).astype(np.int32)).to(dev)
    gn = torch.from_numpy((np.where(rng.uniform(size=n) < 0.1, 2e-4, 1e-5) * cnt.cpu().numpy()).astype(np.float32)).to(dev)
    rad = torch.from_numpy(rng.uniform(0.5, 30.0, n).astype(np.float32)).to(dev)
    noise = torch.from_numpy(rng.normal(size=(6, n)).astype(np.float32)).to(dev)
    t_dp = timed(lambda: hold.__setitem__("d", render.densify_prune(params, m, v, gn, cnt, rad, noise)))
    res["densify_prune"] = {"gaussians_in": n, "gaussians_out": int(hold["d"][3]), "ms": round(1e3 * t_dp, 4)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--train-steps", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this size (calibrates HBM byte counters)")
    ap.add_argument("--forward-only", action="store_true", help="time the forward phase only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not part of this build"}))
        sys.exit(2)

    import torch
    from paper_2603_20611_amd import binding as B, render, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib:
        a = torch.ones(args.copy_probe_mib << 18, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {a.numel() * 4} bytes read and written")
        del a, b
    log("generating workload")
    learn = synth.ultrasound_hidden(N_GAUSS, seed=1)
    hidden = synth.ultrasound_hidden(N_GAUSS, seed=0)
    slices = synth.ultrasound_slices(N_SLICES, RES, SIGMA_Z)
    params = torch.from_numpy(learn).to(dev).contiguous()
    hidden_t = torch.from_numpy(hidden).to(dev).contiguous()

    # target stack: render the hidden set, apply speckle (input data, made once)
    if not args.forward_only:
        ws_t = render.Workspace()
        target = render.render(hidden_t, slices, ws=ws_t)
        target *= torch.from_numpy(synth.speckle(target.numel(), seed=2)).to(dev)
        del ws_t
    del hidden_t
    torch.cuda.synchronize()

    # size a fixed workspace from one counted render, then render without host syncs
    ws_a = render.Workspace()
    out = torch.empty(N_SLICES * RES * RES, device=dev)
    render.render(params, slices, ws=ws_a, out=out)
    rec, inst, bins = ws_a.check()
    del ws_a
    ws = render.Workspace(capacity=(int(rec * 1.3) + 4096, int(inst * 1.3) + 16384))
    log(f"records={rec} instances={inst} bins={bins}")

    # ---------------- forward phase
    for _ in range(args.warmup):
        render.render(params, slices, ws=ws, out=out)
    torch.cuda.synchronize()
    ws.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        render.render(params, slices, ws=ws, out=out)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    st = ws.timings()
    ws.set_timing(False)
    ws.check()
    fwd_ms = 1e3 * t_fwd / args.steps
    mpix = N_SLICES * RES * RES * args.steps / t_fwd / 1e6
    raster_ms = st["raster_fwd"][0] / max(st["raster_fwd"][1], 1)
    pairs = 256.0 * inst
    achieved = pairs / (raster_ms * 1e-3)
    log(f"forward: {fwd_ms:.3f} ms/step, {mpix:.0f} Mpix/s; stages (ms/launch): "
        + ", ".join(f"{k}={v[0] / max(v[1], 1):.3f}" for k, v in st.items() if v[1]))

    if args.forward_only:
        print(json.dumps({"forward_ms": round(fwd_ms, 4), "mpix_per_s": round(mpix, 1),
                          "stage_ms": {k: round(v_[0] / max(v_[1], 1), 4) for k, v_ in st.items() if v_[1]},
                          "records": rec, "instances": inst}), flush=True)
        return

    # ---------------- training phase
    n_train = args.train_steps or max(args.steps * 5, 50)
    grad = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    img = torch.empty(TRAIN_BATCH * RES * RES, device=dev)
    gimg = torch.empty_like(img)
    loss = torch.zeros(2, device=dev)
    rng = np.random.default_rng(7)
    starts = rng.integers(0, N_SLICES - TRAIN_BATCH + 1, size=n_train + args.warmup)
    batches = [slices[int(k):int(k) + TRAIN_BATCH] for k in starts]
    opts = B.default_opts()
    ws_tr = render.Workspace(capacity=(int(rec * TRAIN_BATCH / N_SLICES * 3) + 65536,
                                       int(inst * TRAIN_BATCH / N_SLICES * 3) + 262144))
    lr0 = np.array([6e-4, 2e-3, 1e-3, 2e-2])
    total_iters = 30000

    def train_step(it, batch, k0):
        render.render(params, batch, opts, ws_tr, out=img)
        tgt = target[k0 * RES * RES:(k0 + TRAIN_BATCH) * RES * RES]
        render.l1_dssim_loss_grad(img, tgt, TRAIN_BATCH, RES, RES, ws_tr, lam=LAMBDA_SSIM, grad=gimg, loss=loss)
        render.render_backward(params, batch, gimg, ws_tr, opts, grad=grad)
        lr = lr0 * 0.1 ** (it / total_iters)
        render.adam_step(params, grad, m, v, it + 1, lr, flags=B.GP_ADAM_ZERO_GRAD | B.GP_ADAM_CLAMP_ALPHA)

    for i in range(args.warmup):
        train_step(i, batches[i], int(starts[i]))
    torch.cuda.synchronize()
    ws_tr.set_timing(True)
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + n_train):
        train_step(i, batches[i], int(starts[i]))
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t0
    st_tr = ws_tr.timings()
    ws_tr.check()
    it_s = n_train / t_tr
    log(f"train: {1e3 * t_tr / n_train:.3f} ms/iter ({it_s:.0f} it/s); stages (ms/launch): "
        + ", ".join(f"{k}={v_[0] / max(v_[1], 1):.3f}" for k, v_ in st_tr.items() if v_[1]))

    result = {
        "metric": "Mpix/s fwd & fwd+bwd iter/s @500k Gaussians; serving p50/p99 ms vs plain",
        "value": round(mpix, 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fwd_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ultrasound-shaped reconstruction: 500k Gaussians, 400 axial slices of 256x256, "
                               "sigma_z=3, whole stack per forward step",
                   "gaussians": N_GAUSS, "slices": N_SLICES, "resolution": RES, "sigma_z": SIGMA_Z,
                   "train_batch_slices": TRAIN_BATCH},
        "fwd_bwd_iter_per_s": round(it_s, 1),
        "fwd_bwd_ms_per_iter": round(1e3 * t_tr / n_train, 4),
        "train_steps": n_train,
        "stage_ms": {k: round(v_[0] / max(v_[1], 1), 4) for k, v_ in st.items() if v_[1]},
        "train_stage_ms": {k: round(v_[0] / max(v_[1], 1), 4) for k, v_ in st_tr.items() if v_[1]},
        "records": rec, "instances": inst, "pairs_per_step": int(pairs),
        "roofline": {"bound": "alu", "kernel": "k_raster_fwd", "achieved": round(achieved / 1e9, 1),
                     "peak": round(PEAK_PAIRS_PER_S / 1e9, 1), "unit": "Gpair/s",
                     "frac": round(achieved / PEAK_PAIRS_PER_S, 4), "traffic": measured_traffic("k_raster_fwd"),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel_ms": round(raster_ms, 4)},
    }
    log("voxeliser")
    result["voxelize"] = voxel_leg(params, dev)
    log(f"voxelize: {result['voxelize']}")
    log("codec, oblique batch, densify / prune")
    result.update(extras_leg(params, slices, dev))
    log(f"codec: {result['codec']}; oblique: {result['oblique']}; densify_prune: {result['densify_prune']}")
    if not args.no_serving:
        result["serving"] = serving_leg(dev, args.serving_requests)
    if not args.no_cpu:
        log("timing the CPU oracle on 64 slices")
        result["cpu_baseline"] = cpu_baseline(learn, slices)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
