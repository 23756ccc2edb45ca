"""Benchmark of the PI^2-RH hot path on one MI355X.

A step is one receding-horizon control step of the whole path on
device-resident inputs: sampled rollouts through the LWPR model
(pi_rollout_cost), the path-integral update (pi_update) and the plant step with
the plan shift (pi_rh_shift), each replayed from a HIP graph captured once.

Workload (the largest single-GPU one): the 12-state quadrotor with K = 65536
rollouts, horizon T = 200, M = 1 sampled sub-rollout, 6 LWPR outputs x 1024
local models over d = 16 inputs with R = 4 PLS projections, 20 cylinder
obstacles, FP32, warm-started over the receding-horizon loop.

Prints one JSON line: whole-job rollout-steps/s, per-control-step, rollout and
update latency percentiles, the roofline of the rollout kernel (algorithmic
FLOP per launch over its mean HIP-event duration inside the timed loop; HBM
bytes per launch from the committed rocprofv3 counter summary while the kernel
sources are unchanged), the FP64 oracle's rate on a bounded sample of the same
workload on the host cores, and secondary figures: the 2048-rollout quadrotor
iteration, 64 batched controllers against 64 plain ones, and the fused
forward + adjoint against the forward alone.
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
PEAK_BF16_MFMA = 2.5e15        # MI355X dense bf16 (and fp16) matrix peak, FLOP/s
# the pieces forms of the d = 16 contraction: matrix dtype and piece products per block
PIECES = {"mfma-bf16x3": ("bf16x3", 6), "mfma-f16x2": ("f16x2", 3)}
PEAK_HBM = 8.0e12              # bytes/s
TRAFFIC_SUMMARY = {
    "rollout_mfma_kernel": os.path.join(ROOT, "profiles", "rollout_mfma_kernel.quad_k65536_t200.traffic.txt"),
    "rollout_pair_kernel": os.path.join(ROOT, "profiles", "rollout_pair_kernel.quad_k2048_t100.traffic.txt"),
}


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def flops_per_sample_step(model):
    """Algorithmic work of one sample-step: every local model of every output
    costs d^2 + 3d + 1 (kernel distance with symmetric D) + 2d + 1 (affine
    local prediction) + 6 (mixture accumulation) = d^2 + 5d + 8 flop."""
    d = model.d
    return model.Ltot * (d * d + 5 * d + 8)


def pieces_flops_per_launch(model, n_samples, T, products):
    """Matrix-core work a pieces form of the contraction executes: per 16-row
    tile of samples, 16-model tile and step, 6 blocks of 32 features x the
    form's piece products (6 for bf16x3, 3 for f16x2), each a 16x16x32 product
    of 2*16*16*32 flop (the padded feature layout and the piece products it
    takes to reach float32 accuracy, not algorithmic work)."""
    n_model_tiles = sum((int(model.L_off[i + 1]) - int(model.L_off[i]) + 15) // 16 for i in range(model.n_out))
    return ((n_samples + 15) // 16) * n_model_tiles * T * 6 * products * (2 * 16 * 16 * 32)


def roofline(model, plan, n_samples, T, flop, seconds, traffic, autotuned):
    """The rollout kernel's roofline entry: algorithmic FLOP over the measured
    duration against the peak of the matrix instructions it runs (float32, or
    bf16 / fp16 for the pieces forms, which also report their executed matrix
    rate and the float32-equivalent fraction)."""
    achieved = flop / seconds
    pieces = PIECES.get(plan["variant"])
    peak = PEAK_BF16_MFMA if pieces else PEAK_FP32_MFMA
    r = {"bound": "mfma", "kernel": plan["kernel"], "mfma_dtype": pieces[0] if pieces else "f32",
         "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
         "traffic": traffic, "flop_per_launch": flop, "flop_per_sample_step": flops_per_sample_step(model),
         "sample_steps_per_launch": n_samples * T,
         "launch": dict({k: plan[k] for k in ("variant", "tile_samples", "tile_waves", "tile_split")},
                        autotuned=autotuned)}
    if pieces:
        ex = pieces_flops_per_launch(model, n_samples, T, pieces[1])
        r.update({"executed_flop_per_launch": ex, "executed": ex / seconds / 1e12,
                  "executed_frac": ex / seconds / PEAK_BF16_MFMA,
                  "fp32_equivalent_peak": PEAK_FP32_MFMA / 1e12,
                  "fp32_equivalent_frac": achieved / PEAK_FP32_MFMA})
    return r


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, model, n_rollouts):
    """The FP64 oracle's rollout rate on rollouts 0..n-1 of the workload.
    Rollouts are independent and equally expensive (counter-based noise), so
    the rate of a prefix is the rate of the whole stage."""
    import oracle
    n_rollouts = min(n_rollouts, prob.K)
    t0 = time.perf_counter()
    oracle.rollout_cost(prob, model, k_range=(0, n_rollouts))
    dt = time.perf_counter() - t0
    return {"value": n_rollouts * max(prob.M, 1) * prob.T / dt, "unit": "rollout-steps/s",
            "cores": oracle.max_threads(), "cpu": cpu_model(), "kind": "oracle",
            "sample": "FP64 oracle, rollouts k=0..%d of the %d x %d-step workload (the rollout "
                      "stage, %d of %d rollouts), %.1f s wall" % (n_rollouts - 1, prob.K, prob.T,
                                                                 n_rollouts, prob.K, dt)}


def capture(fn):
    """One HIP graph of fn()'s launches, recorded on a side stream."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    return g


def events_ms(pairs):
    return [a.elapsed_time(b) for a, b in pairs]


# ------------------------------------------------------------- secondary keys

def extra_config1(steps):
    """The 2048-rollout, 100-step quadrotor iteration (rollout + update + shift),
    eager launches, launch shape from the autotuner: small enough to leave
    compute units idle with one tile per workgroup, so pairs of workgroups
    share a tile."""
    import torch
    import paper_1503_00330_amd as pi
    import synth
    from paper_1503_00330_amd import tune
    prob, model, _ = synth.config(1)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model).fold()
    tune.ensure(dp, dm)
    cost = torch.empty((prob.K, prob.T), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(rec):
        e = [ev() for _ in range(3)]
        e[0].record(stream)
        pi.rollout_cost(dp, dm, out=cost)
        e[1].record(stream)
        pi.update(dp, cost)
        pi.rh_shift(dp, dm)
        e[2].record(stream)
        rec.append(e)
    junk = []
    for _ in range(3):
        step(junk)
    torch.cuda.synchronize()
    rec = []
    for _ in range(steps):
        step(rec)
    torch.cuda.synchronize()
    roll = [a.elapsed_time(b) for a, b, c in rec]
    it = [a.elapsed_time(c) for a, b, c in rec]
    flop = flops_per_sample_step(model) * prob.K * prob.T
    plan = pi.rollout_describe(dp, dm)
    rl = roofline(model, plan, prob.K * max(prob.M, 1), prob.T, flop, float(np.mean(roll)) * 1e-3, None, True)
    return {"workload": "quadrotor K=2048 T=100 M=1, 6 x 256 models, eager iteration",
            "rollout_steps_per_s": prob.K * prob.T / (float(np.mean(it)) * 1e-3),
            "iteration_ms_p50": percentile(it, 50), "iteration_ms_p99": percentile(it, 99),
            "rollout_ms_mean": float(np.mean(roll)), "kernel": plan["kernel"], "launch": rl["launch"],
            "rollout_frac_fp32_peak": flop / (float(np.mean(roll)) * 1e-3) / PEAK_FP32_MFMA,
            "roofline": {k: v for k, v in rl.items() if k not in ("traffic", "launch", "kernel")}}


def extra_batched(reps):
    """64 quadrotor controllers with uneven K, L, T and obstacles (autotuned
    tiles): batched rollouts and one batched control step against 64 plain
    ones on the same stream."""
    import bench_extra
    r = bench_extra.w_batched(argparse.Namespace(steps=reps, tile_samples=0))
    return r


def extra_adjoint(reps):
    """Fused forward + adjoint against the forward alone, K = 8192, T = 400."""
    import bench_extra
    return bench_extra.w_adjoint(argparse.Namespace(steps=reps))


# ---------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rollouts", type=int, default=1024, help="oracle sample: rollouts 0..n-1")
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--extras", default="config1,batched_vs_plain,adjoint_vs_forward",
                    help="comma-separated secondary workloads to run")
    ap.add_argument("--no-tune", action="store_true", help="library default launch shapes (no autotuner)")
    ap.add_argument("--eager", action="store_true",
                    help="launch the control steps directly instead of replaying graphs "
                         "(the same kernels; for profilers that count per dispatch)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy a 512 MiB buffer once (a plain copy kernel of "
                         "known size for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (rollouts "
              "would shard by k with one small all-reduce per update)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1503_00330_amd as pi
    import synth

    torch.cuda.set_device(0)
    prob, model, _ = synth.config(2)
    dp = pi.DeviceProblem(prob)
    dm = pi.DeviceModel(model).fold()      # the model is fixed over the loop: fold once
    if not args.no_tune:
        # the rollout launch shape from the autotuner (tuned now unless cached)
        from paper_1503_00330_amd import tune
        tune.ensure(dp, dm)
        log("launch tuned: %s" % (pi.rollout_describe(dp, dm),))
    cost = torch.empty((prob.K, prob.T), dtype=torch.float32, device="cuda")
    saved = (dp.x0.clone(), dp.u_nom.clone(), dp.iter.clone())
    # one eager control step reserves every workspace and runs the library's
    # per-device checks before capture
    pi.rollout_cost(dp, dm, out=cost)
    pi.update(dp, cost)
    pi.rh_shift(dp, dm)
    torch.cuda.synchronize()
    if args.eager:
        run_roll = lambda: pi.rollout_cost(dp, dm, out=cost)
        run_upd = lambda: pi.update(dp, cost)
        run_shift = lambda: pi.rh_shift(dp, dm)
    else:
        run_roll = capture(lambda: pi.rollout_cost(dp, dm, out=cost)).replay
        run_upd = capture(lambda: pi.update(dp, cost)).replay
        run_shift = capture(lambda: pi.rh_shift(dp, dm)).replay
        log("graphs captured")
    for t, s in zip((dp.x0, dp.u_nom, dp.iter), saved):
        t.copy_(s)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(record):
        e = [ev() for _ in range(4)]
        e[0].record(stream)
        run_roll()
        e[1].record(stream)
        run_upd()
        e[2].record(stream)
        run_shift()
        e[3].record(stream)
        record.append(e)

    junk = []
    for _ in range(args.warmup):
        step(junk)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log("timed loop: %d control steps in %.2f s" % (args.steps, wall))

    roll_ms = [a.elapsed_time(b) for a, b, c, d in evs]
    upd_ms = [b.elapsed_time(c) for a, b, c, d in evs]
    it_ms = [a.elapsed_time(d) for a, b, c, d in evs]
    ms_per_step = wall * 1e3 / args.steps
    ssteps = prob.K * max(prob.M, 1) * prob.T
    value = ssteps * args.steps / wall

    flop = flops_per_sample_step(model) * ssteps
    roll_mean_s = float(np.mean(roll_ms)) * 1e-3
    plan = pi.rollout_describe(dp, dm)
    from paper_1503_00330_amd.profiling import launch_tag, traffic_from_summary
    summ = TRAFFIC_SUMMARY.get(plan["kernel"])
    traffic = traffic_from_summary(summ, launch_tag(plan)) if summ else None
    pieces = PIECES.get(plan["variant"])
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
        "config": {"workload": "quadrotor PI2-RH receding-horizon control step (rollout + update + "
                               "plant step and shift, each a HIP graph replay), warm-started: "
                               "K=65536 rollouts, T=200, M=1, LWPR d=16, 6 outputs x 1024 local "
                               "models, R=4, 20 obstacles, FP32",
                   "K": prob.K, "T": prob.T, "M": prob.M, "d": model.d, "n_out": model.n_out,
                   "L_per_output": int(model.L_off[1]), "R": model.R, "graph": not args.eager,
                   "mfma": {"bf16x3": "bf16x3: float32 mixture products as six bf16 piece products, "
                                      "float32 accumulation",
                            "f16x2": "f16x2: float32 mixture products of power-of-two scaled values as "
                                     "three fp16 piece products, float32 accumulation"}.get(
                                pieces[0] if pieces else None, "f32")},
        "latency_ms": {"control_step_p50": percentile(it_ms, 50),
                       "control_step_p99": percentile(it_ms, 99),
                       "rollout_p50": percentile(roll_ms, 50), "rollout_p99": percentile(roll_ms, 99),
                       "update_p50": percentile(upd_ms, 50), "update_p99": percentile(upd_ms, 99),
                       "rollout_mean": float(np.mean(roll_ms))},
        "roofline": roofline(model, plan, prob.K * max(prob.M, 1), prob.T, flop, roll_mean_s, traffic,
                             not args.no_tune),
    }
    if args.calibrate_copy:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    del run_roll, run_upd, run_shift, cost
    if not args.no_extras:
        wanted = set(args.extras.split(","))
        for key, fn, n in (("config1", extra_config1, 20), ("batched_vs_plain", extra_batched, 2),
                           ("adjoint_vs_forward", extra_adjoint, 3)):
            if key not in wanted:
                continue
            try:
                out[key] = fn(n)
            except Exception as exc:   # a secondary figure never hides the headline
                out[key] = {"error": "%s: %s" % (type(exc).__name__, exc)}
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            log("secondary workload %s done" % key)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, model, args.cpu_rollouts)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
