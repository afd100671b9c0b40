#!/usr/bin/env python3
"""Throughput of the QFCA score path on one MI355X.

Workload: one 256 x 256 feature map with C = 256 float32 channels (seeded
Gaussian random-field texture with three anomalies), PCA residual with k = 32
components, B = 32 bins, T = 15 windows, sigma_s = 1.

One step = one image through quantisation (PCA residual projection + bins)
and the score map (window histograms, Algorithm 1, association, channel mean,
blur), with the image's model fitted beforehand on the same image (the
zero-shot fit latency is reported separately as fit_ms).  Inputs are resident
in device memory when the timed region starts.

Prints one JSON line.  --gpus above 1 is refused: this benchmark measures one
GPU.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak figures of the MI355X used as roofline denominators.
HBM_PEAK_GBS = 8000.0
# 32-bit vector ALU lane-operations per second: 256 CUs x 64 lanes x 2.4 GHz
# (packed FP32 is not used).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic vector operations per (pixel, channel, bin) of the score kernel:
# window cumulative count by separable running sums (4), the closed-form
# transport numerator from two neighbouring counts and the reference tables
# (10), the per-bin error I / P (4) and the separable box association (4).
SCORE_OPS_PER_PCB = 22
METRIC = "score Mpixel/s at 256\u00b2\u00d7256ch (FP32 vs BF16-batched); p50/p99 latency"


# HBM traffic of the score kernel on this workload comes from rocprofv3 byte
# counters (FETCH_SIZE and WRITE_SIZE, scaled by what they read for an
# elementwise kernel of known size), recorded in this summary together with a
# hash of the sources the counters were taken on; it is reported only while
# the sources are unchanged.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_score_t15_256x256_C256_B32.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2510_15602_amd", "csrc", f)
                  for f in ("qfca_tiles.h", "qfca_score.hip", "qfca_api.cpp")]


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """Bytes per launch (read + write) of k_score_t<15> on the 256x256 x 256
    workload, or None if no summary matches the current kernel sources."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"traffic: sources_sha256=([0-9a-f]+) read_bytes=(\d+) write_bytes=(\d+)", text)
    if not m or m.group(1) != kernel_sources_sha256():
        return None
    return int(m.group(2)) + int(m.group(3))


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--seed", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-steps", type=int, default=50)
    ap.add_argument("--batch-images", type=int, default=64,
                    help="images in the uneven BF16 batch measured beside the single-image path (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the open-loop Poisson serving run (0: skip)")
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--serve-max-batch", type=int, default=64)
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="after the run, run an elementwise kernel twice over a MIB-sized float32 buffer so "
                         "that hardware byte counters of the run can be scaled by a copy of known size")
    return ap.parse_args()


def batched_leg(args, q, torch, np, dev):
    """64 images with sides drawn from {128,192,256,384,512}, C=256, k=32,
    B=32, T=15, BF16 projection: one graph replay of the persistent
    quantise-histogram-score kernel per step, every image's model fitted on
    the image beforehand (untimed)."""
    import qfca_synth
    imgs, p = qfca_synth.workload_batch_torch(n=args.batch_images, device=dev)
    ctx = q.Context(0)
    prm = q.Params.make(C=p["C"], k=p["k"], B=p["B"], T=p["T"], q_lo=p["q_lo"], q_hi=p["q_hi"],
                        sigma_s=p["sigma_s"], proj_prec=q.QFCA_PREC_BF16)
    prm32 = q.Params.make(C=p["C"], k=p["k"], B=p["B"], T=p["T"], q_lo=p["q_lo"], q_hi=p["q_hi"],
                          sigma_s=p["sigma_s"], proj_prec=q.QFCA_PREC_FP32)
    jobs, fit_ms, px = [], [], 0
    for X, _, _ in imgs:
        C, H, W = X.shape
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m = q.qfca_fit_pca(ctx, prm, X)
        torch.cuda.synchronize()
        fit_ms.append((time.perf_counter() - t0) * 1e3)
        jobs.append((m, X, torch.empty((H, W), device=dev), torch.empty((C, H, W), dtype=torch.uint8, device=dev)))
        px += H * W
    tile = None
    if not args.no_autotune:
        ws, hb, tms = q.qfca_autotune(ctx, jobs)
        tile = {"Ws": ws, "Hb": hb, "ms": round(tms, 3)}
    for _ in range(args.batch_warmup):
        q.qfca_score_batch(ctx, jobs)
    torch.cuda.synchronize()
    ctx.profile_read("score")
    ctx.profile(True, kernels=["score"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        q.qfca_score_batch(ctx, jobs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    ev_ms, ev_n = ctx.profile_read("score")
    if q.qfca_batch_error(ctx) != 0:
        raise RuntimeError("batched kernel reported a failed dependency wait")
    ms = (t1 - t0) * 1e3 / args.batch_steps
    # BF16 against the FP32 projection with the same model: bin flips and
    # score-map error (outside the timed region)
    flips = 0
    err = 0.0
    for (m, X, score, bins) in jobs:
        m32 = q.qfca_model_create(ctx, prm32, m.read("mu"), m.read("V"), m.read("edges"), m.read("delta"),
                                  m.read("cR"))
        b32, _ = q.qfca_quantize(ctx, m32, X)
        s32 = q.qfca_score_map(ctx, m32, b32).score
        flips += int((b32 != bins).sum().item())
        err = max(err, float(((score - s32).abs().max() / s32.abs().max().clamp_min(1e-30)).item()))
        m32.close()
    sides = sorted({int(j[1].shape[1]) for j in jobs})
    return {
        "value": round(px / (ms * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_step": round(ms, 3),
        "graph_ms": round(ev_ms / max(ev_n, 1), 3), "images": len(jobs), "pixels": px,
        "steps": args.batch_steps, "warmup": args.batch_warmup, "dtype": "bf16-proj/f32",
        "workload": f"{len(jobs)} images, sides from {sides}, C={p['C']} float32, PCA residual k={p['k']} "
                    f"(BF16 MFMA, FP32 accumulation), B={p['B']}, T={p['T']}, one persistent kernel per step "
                    f"under a HIP graph",
        "tile": tile, "fit_ms_median": round(float(np.median(fit_ms)), 3),
        "bf16_flip_rate_vs_fp32": flips / (px * p["C"]),
        "bf16_max_score_rel_err_vs_fp32": err,
    }


def serving_leg(args, q, torch, np, dev, tile=None):
    """Open-loop Poisson arrivals of single images (sides 128/256/512, C=256,
    BF16 projection) against 8 resident class models, through the
    continuous-batching server.  Latency = completion - scheduled arrival."""
    import qfca_synth
    C, k, B, T = 256, 32, 32, 15
    ctx = q.Context(0)
    prm = q.Params.make(C=C, k=k, B=B, T=T, proj_prec=q.QFCA_PREC_BF16)
    classes = range(8)
    models = []
    for c in classes:  # exemplar: an anomaly-free 256x256 texture of the class
        X, _, _ = qfca_synth.make_texture_torch(C, 256, 256, 400 + c, dev, class_seed=400 + c)
        models.append(q.qfca_fit_pca(ctx, prm, X))
        del X
    sides = (128, 256, 512)
    pool = {}  # (class, side, variant) -> features of a request image with anomalies
    for c in classes:
        for sd in sides:
            for v in range(2):
                X, _, _ = qfca_synth.make_texture_torch(
                    C, sd, sd, 10000 + 100 * c + 10 * sd // 128 + v, dev, class_seed=400 + c,
                    anomalies=[("shift", 8, max(8, sd // 8)), ("scale", 8, max(8, sd // 8))])
                pool[(c, sd, v)] = X
    torch.cuda.synchronize()
    srv = q.Server(0, hbm_budget=int(args.serve_budget_gib * (1 << 30)), max_inflight=args.serve_slots,
                   max_batch=args.serve_max_batch, Ws=tile["Ws"] if tile else 0, Hb=tile["Hb"] if tile else 0)

    def run(duration, seed):
        sched = qfca_synth.poisson_arrivals(args.serve_rate, duration, seed=seed, sides=sides, n_classes=8)
        outs = [torch.empty((sd, sd), device=dev) for (_, sd, _) in sched]
        torch.cuda.synchronize()
        t0 = q.qfca_clock() + 0.05
        arrive, px, done = {}, {}, []
        for i, (ta, sd, c) in enumerate(sched):
            due = t0 + ta
            while True:
                now = q.qfca_clock()
                if now >= due:
                    break
                if due - now > 0.002:
                    time.sleep(0.001)
                    done += srv.poll()
            tk = srv.submit(models[c], pool[(c, sd, i & 1)], outs[i])
            arrive[tk] = due
            px[tk] = sd * sd
        srv.drain()
        done += srv.poll()
        lat = np.array([c["t_done"] - arrive[c["ticket"]] for c in done])
        bs = np.array([c["batch_size"] for c in done])
        t_end = max(c["t_done"] for c in done)
        return sched, lat, bs, sum(px.values()), t_end - t0, [c["status"] for c in done]

    run(args.serve_warmup, seed=5)  # graph captures and first-touch costs
    st0 = srv.stats()
    sched, lat, bs, pxs, wall, status = run(args.serve_seconds, seed=4)
    st = srv.stats()
    srv.close()
    for m in models:
        m.close()
    if any(s != 0 for s in status):
        raise RuntimeError("a served request failed")
    busy = st["device_busy_s"] - st0["device_busy_s"]
    return {
        "workload": f"Poisson arrivals at {args.serve_rate:g} req/s for {args.serve_seconds:g} s, sides "
                    f"{list(sides)}, C={C}, k={k} (BF16 projection), B={B}, T={T}, 8 resident class models "
                    f"fitted on anomaly-free 256x256 exemplars",
        "requests": len(sched), "offered_mpx_s": round(pxs / args.serve_seconds / 1e6, 3),
        "throughput_mpx_s": round(pxs / wall / 1e6, 3), "throughput_req_s": round(len(sched) / wall, 2),
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 3),
                       "mean": round(1e3 * float(lat.mean()), 3), "max": round(1e3 * float(lat.max()), 3)},
        "mean_batch": round(float(bs.mean()), 2), "launches": st["launches"] - st0["launches"],
        "device_busy_frac": round(busy / wall, 4) if wall > 0 else None,
        "overlapped_launches": st["overlapped"] - st0["overlapped"],
        "max_inflight_seen": st["max_inflight_seen"], "deferred_memory": st["deferred_memory"] - st0["deferred_memory"],
        "hbm_budget_gib": args.serve_budget_gib, "arena_peak_gib": round(st["arena_peak"] / 2 ** 30, 3),
        "slots": args.serve_slots, "max_batch": args.serve_max_batch,
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (images shard across GPUs with no exchange; there is no "
              "multi-GPU run): use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2510_15602_amd as q
    import qfca_synth

    ts, p = qfca_synth.workload_256(args.seed)
    tex = ts[0]
    C, H, W = tex.X.shape
    dev = torch.device("cuda:0")
    X = torch.from_numpy(tex.X).to(dev)
    ctx = q.Context(0)
    prec = q.QFCA_PREC_BF16 if args.prec == "bf16" else q.QFCA_PREC_FP32
    prm = q.Params.make(C=C, k=p["k"], B=p["B"], T=p["T"], q_lo=p["q_lo"], q_hi=p["q_hi"],
                        sigma_s=p["sigma_s"], proj_prec=prec)

    # zero-shot fit latency (not part of the step)
    fit_ms = []
    model = None
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m = q.qfca_fit_pca(ctx, prm, X)
        torch.cuda.synchronize()
        fit_ms.append((time.perf_counter() - t0) * 1e3)
        if model is not None:
            model.close()
        model = m

    bins = torch.empty((C, H, W), dtype=torch.uint8, device=dev)
    out = q.ScoreMaps(torch.empty((H, W), dtype=torch.float32, device=dev))

    def step():
        q.qfca_quantize(ctx, model, X, bins=bins)
        q.qfca_score_map(ctx, model, bins, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k in q.KERNELS:
        ctx.profile_read(k)
    # HIP events around the dominant kernel only inside the timed region (the
    # roofline's duration); the other kernels are timed in a pass after it
    ctx.profile(True, kernels=["score"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    kt = {"score": ctx.profile_read("score")}
    ctx.profile(True)
    for _ in range(min(args.steps, 20)):
        step()
    torch.cuda.synchronize()
    ctx.profile(False)
    for k in q.KERNELS:
        v = ctx.profile_read(k)
        if k != "score":
            kt[k] = v
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = H * W / (ms_per_step * 1e-3) / 1e6

    # per-image latency (each step synchronised), outside the timed region
    lat = []
    for _ in range(args.latency_steps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)

    score_ms = kt["score"][0] / max(kt["score"][1], 1)
    proj_ms = kt["proj"][0] / max(kt["proj"][1], 1)
    score_ops = float(H) * W * C * p["B"] * SCORE_OPS_PER_PCB
    achieved = score_ops / (score_ms * 1e-3) / 1e12
    proj_bytes = float(H) * W * (4 * C + C)
    default_workload = (H, W, C, p["B"], p["T"]) == (256, 256, 256, 32, 15)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": measured_traffic() if default_workload else None, "traffic_unit": "bytes/launch",
                "kernel": "k_score", "avg_ms": round(score_ms, 4),
                "ops_per_launch": score_ops}
    kernels = {
        k: {"avg_ms": round(v[0] / max(v[1], 1), 4), "launches": v[1]} for k, v in kt.items()}
    kernels["proj"]["hbm_gbs"] = round(proj_bytes / (proj_ms * 1e-3) / 1e9, 1)
    kernels["proj"]["hbm_frac"] = round(proj_bytes / (proj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        om, _, _ = oracle.fit(tex.X, p["k"], p["B"], p["T"], p["q_lo"], p["q_hi"])
        t0 = time.perf_counter()
        R = oracle.residual(tex.X, om.mu, om.V)
        ob = oracle.quantize(R, p["B"], om.edges)
        oracle.score(ob, p["T"], p["B"], om.cR, om.delta, p["sigma_s"])
        dt = time.perf_counter() - t0
        cpu = {"value": round(H * W / dt / 1e6, 5), "unit": "Mpixel/s", "cores": oracle.num_threads(),
               "kind": "oracle", "seconds": round(dt, 3),
               "sample": f"the full {H}x{W} image, C={C}: FP64 residual, quantisation and score "
                         f"(window counts, literal Alg. 1, direct association, direct blur)"}

    batched = None
    if args.batch_images > 0:
        batched = batched_leg(args, q, torch, np, dev)
        torch.cuda.empty_cache()
    serving = None
    if args.serve_seconds > 0:
        serving = serving_leg(args, q, torch, np, dev, tile=batched["tile"] if batched else None)
        torch.cuda.empty_cache()

    res = {
        "metric": METRIC,
        "path": "FP32 projection" if prec == 0 else "BF16 projection",
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == 0 else "bf16-proj/f32",
        "data": "synthetic",
        "config": {"workload": "256x256 feature map, C=256 float32, PCA residual k=32, B=32, T=15, "
                               "sigma_s=1, 1 image per step, model fitted on the image",
                   "H": H, "W": W, "C": C, "k": p["k"], "B": p["B"], "T": p["T"],
                   "seed": args.seed},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "fit_ms": round(float(np.median(fit_ms)), 3),
        "zero_shot_ms": round(float(np.median(fit_ms)) + float(np.percentile(lat, 50)), 3),
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "batched_bf16": batched,
        "serving_bf16": serving,
    }
    print(json.dumps(res), flush=True)
    if args.calib_copy:
        # an elementwise kernel that reads and writes MIB MiB each
        n = args.calib_copy * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
