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
import json
import os
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


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--seed", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-steps", type=int, default=50)
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-sized float32 buffer twice (device to device) so that "
                         "hardware byte counters of the run can be scaled by a copy of known size")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures a single GPU; run it with --gpus 1 (multi-GPU runs are not part of "
              "this build).", file=sys.stderr)
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
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    kt = {k: ctx.profile_read(k) for k in q.KERNELS}
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
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
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

    res = {
        "metric": "score Mpixel/s at 256x256x256ch (FP32 plain path)" if prec == 0 else
                  "score Mpixel/s at 256x256x256ch (BF16 projection)",
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
    }
    print(json.dumps(res), flush=True)
    if args.calib_copy:
        n = args.calib_copy * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
