"""Benchmark of the PI^2-RH hot path on one MI355X.

A step is one receding-horizon iteration of the whole path on device-resident
inputs: sampled rollouts through the LWPR model (pi_rollout_cost), the
path-integral update (pi_update) and the plan shift (pi_rh_shift).

Workload: the quadrotor configuration -- K = 2048 rollouts, horizon T = 100,
M = 1 sampled sub-rollout, 6 LWPR outputs x 256 local models over d = 16
inputs with R = 4 PLS projections, 20 cylinder obstacles, FP32.

Prints one JSON line: whole-job rollout-steps/s, per-iteration and update
latency percentiles, the roofline of the rollout kernel (algorithmic FLOP per
launch over its mean HIP-event duration; HBM bytes per launch from the
committed rocprofv3 counter summary while the kernel sources are unchanged)
and the FP64 oracle's rate on the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LWPR rollout steps/s + PI^2 update p50/p99 latency; fwd+adjoint & batched vs plain"
PEAK_FP32_MFMA = 157.3e12      # MI355X dense FP32 matrix peak, FLOP/s
PEAK_HBM = 8.0e12              # bytes/s
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "rollout_pair_kernel.quad_k2048_t100.traffic.txt")


def flops_per_sample_step(model):
    """Algorithmic work of one sample-step: every local model of every output
    costs d^2 + 3d + 1 (kernel distance with symmetric D) + 2d + 1 (affine
    local prediction) + 6 (mixture accumulation) = d^2 + 5d + 8 flop."""
    d = model.d
    return model.Ltot * (d * d + 5 * d + 8)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def cpu_baseline(prob, model, n_rollouts=0):
    """The FP64 oracle's rollout rate on rollouts 0..n-1 of the workload (all of
    them by default: the whole rollout stage, a few seconds on 16 cores)."""
    import oracle
    n_rollouts = n_rollouts or prob.K
    t0 = time.perf_counter()
    oracle.rollout_cost(prob, model, k_range=(0, n_rollouts))
    dt = time.perf_counter() - t0
    what = ("all %d rollouts" % prob.K) if n_rollouts == prob.K else ("rollouts k=0..%d" % (n_rollouts - 1))
    return {"value": n_rollouts * max(prob.M, 1) * prob.T / dt, "unit": "rollout-steps/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "FP64 oracle, %s of the workload x %d steps (the rollout stage), %.1f s wall"
                      % (what, prob.T, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rollouts", type=int, default=0, help="oracle sample (0 = all K rollouts)")
    ap.add_argument("--tile-samples", type=int, default=0)
    ap.add_argument("--tile-waves", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy a 512 MiB buffer once (a plain copy kernel of "
                         "known size for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rollouts would shard by k with one small all-reduce per update)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1503_00330_amd as pi
    import synth

    torch.cuda.set_device(0)
    prob, model, _ = synth.config(1)
    dp = pi.DeviceProblem(prob, tile_samples=args.tile_samples, tile_waves=args.tile_waves)
    # the model is fixed over the receding-horizon loop: fold it once
    dm = pi.DeviceModel(model).fold()
    cost = torch.empty((prob.K, prob.T), dtype=torch.float32, device="cuda")
    x0_init, u_init = dp.x0.clone(), dp.u_nom.clone()
    # reserve every workspace before timing
    pi.rollout_cost(dp, dm, out=cost)
    pi.update(dp, cost)
    pi.rh_shift(dp, dm)
    torch.cuda.synchronize()
    dp.x0.copy_(x0_init)
    dp.u_nom.copy_(u_init)
    dp.iter.zero_()

    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(record):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record(stream)
        pi.rollout_cost(dp, dm, out=cost)
        e1.record(stream)
        pi.update(dp, cost)
        e2.record(stream)
        pi.rh_shift(dp, dm)
        e3.record(stream)
        if record is not None:
            record.append((e0, e1, e2, e3))

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    roll_ms = [a.elapsed_time(b) for a, b, c, d in evs]
    upd_ms = [b.elapsed_time(c) for a, b, c, d in evs]
    it_ms = [a.elapsed_time(d) for a, b, c, d in evs]
    ms_per_step = wall * 1e3 / args.steps
    ssteps = prob.K * max(prob.M, 1) * prob.T
    value = ssteps * args.steps / wall

    flop = flops_per_sample_step(model) * ssteps
    roll_mean_s = float(np.mean(roll_ms)) * 1e-3
    achieved = flop / roll_mean_s
    plan = pi.rollout_describe(dp, dm)
    from paper_1503_00330_amd.profiling import traffic_from_summary
    traffic = traffic_from_summary(TRAFFIC_SUMMARY) if plan["kernel"] == "rollout_pair_kernel" else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "quadrotor PI2-RH iteration (rollout+update+shift): K=2048 rollouts, "
                               "T=100, M=1, LWPR d=16, 6 outputs x 256 local models, R=4, "
                               "20 obstacles, FP32",
                   "K": prob.K, "T": prob.T, "M": prob.M, "d": model.d, "n_out": model.n_out,
                   "L_per_output": int(model.L_off[1]), "R": model.R},
        "latency_ms": {"iteration_p50": percentile(it_ms, 50), "iteration_p99": percentile(it_ms, 99),
                       "update_p50": percentile(upd_ms, 50), "update_p99": percentile(upd_ms, 99),
                       "rollout_mean": float(np.mean(roll_ms))},
        "roofline": {"bound": "mfma", "kernel": plan["kernel"],
                     "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_MFMA, "traffic": traffic,
                     "flop_per_launch": flop, "flop_per_sample_step": flops_per_sample_step(model),
                     "launch": {k: plan[k] for k in ("tile_samples", "tile_waves", "tile_split")}},
    }
    if args.calibrate_copy:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, model, args.cpu_rollouts)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
