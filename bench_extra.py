"""Measurements of the other workloads of the PI^2-RH hot path (one JSON line each).

  --workload cfg0      point mass, FP64, K=256, T=20: per-iteration latency p50/p99
                       (eager and HIP-graph replay)
  --workload rh-graph  quadrotor, 6 x 1024 local models, K=65536, T=200: receding-
                       horizon loop, one control step per HIP-graph replay;
                       per-iteration latency p50/p99 and pi_update alone
  --workload batched   64 quadrotor problems with uneven K, L, T and obstacles in one
                       persistent launch vs 64 sequential plain launches
  --workload adjoint   quadrotor, K=8192, T=400, checkpoints every 20: fused forward +
                       adjoint (pi_rollout_adjoint) vs the forward rollout alone
  --workload paper     the paper's model (hybrid quadrotor, d = 4, 15/15/24 local
                       models) at its GPU timing shapes (1000 rollouts x 50 steps,
                       M sub-rollouts), the largest K per 20 ms iteration, and
                       whole control steps at the rollout and iteration counts
                       of the paper's Table 2
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

PEAK_FP32 = 157.3e12
PEAK_FP64 = 78.6e12


def flops_per_sample_step(model):
    d = model.d
    return model.Ltot * (d * d + 5 * d + 8)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def timed(fn, n, stream):
    import torch
    out = []
    for _ in range(n):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        out.append((a, b))
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in out]


def w_cfg0(args):
    import torch
    import paper_1503_00330_amd as pi
    from paper_1503_00330_amd.rh import RHController
    import synth
    prob, model, _ = synth.config(0)
    res = {}
    for graph in (False, True):
        dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
        c = RHController(dp, dm, iterations=1, graph=graph)
        for _ in range(5):
            c.step()
        torch.cuda.synchronize()
        ms = timed(c.step, args.steps, torch.cuda.current_stream())
        res["graph" if graph else "eager"] = {"p50_us": pct(ms, 50) * 1e3, "p99_us": pct(ms, 99) * 1e3}
    ss = prob.K * prob.T
    return {"workload": "point mass FP64 PI2-RH iteration K=256 T=20 d=6 2x16 models",
            "latency": res, "rollout_steps_per_s_graph": ss / (res["graph"]["p50_us"] * 1e-6),
            "dtype": "f64"}


def w_rh_graph(args):
    import torch
    import paper_1503_00330_amd as pi
    from paper_1503_00330_amd.rh import RHController
    import synth
    prob, model, extra = synth.config(2)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    c = RHController(dp, dm, iterations=1, graph=True)
    c.capture()
    steps = args.steps or extra["rh_steps"]
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        c.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = timed(c.step, steps, stream)
    wall = time.perf_counter() - t0
    cost = torch.empty((prob.K, prob.T), dtype=torch.float32, device="cuda")
    pi.rollout_cost(dp, dm, out=cost)
    upd = timed(lambda: pi.update(dp, cost), 10, stream)
    roll = timed(lambda: pi.rollout_cost(dp, dm, out=cost), 2, stream)
    ss = prob.K * prob.T
    flop = flops_per_sample_step(model) * ss
    return {"workload": "quadrotor RH loop, HIP graph per control step: K=65536 T=200 d=16 "
                        "6x1024 models R=4 M=1",
            "steps": steps, "iteration_ms_p50": pct(ms, 50), "iteration_ms_p99": pct(ms, 99),
            "update_ms_p50": pct(upd, 50), "update_ms_p99": pct(upd, 99),
            "rollout_ms": float(np.mean(roll)), "rollout_steps_per_s": ss / (float(np.mean(roll)) * 1e-3),
            "rollout_tflops": flop / (float(np.mean(roll)) * 1e-3) / 1e12,
            "rollout_frac_fp32_peak": flop / (float(np.mean(roll)) * 1e-3) / PEAK_FP32,
            "wall_s": wall, "dtype": "f32"}


def w_batched(args):
    """64 independent controllers with uneven K, L, T and obstacles.  Tiles
    are picked by the autotuner (uniform tile shape over the batch; cached).
    Reported: the batched rollouts against 64 plain rollout launches, each
    problem in the fastest of the library's default launches of the three
    contractions (`speedup`), and with the batch's own tile shape and
    contraction (`speedup_same_tiles`: bitwise the same costs), and one batched
    control step (rollouts, updates, plant steps and shifts; one HIP graph)
    against 64 plain control steps with the batch's tiles (one HIP graph of
    all 64), with the bitwise check that both leave every problem's state the
    same."""
    import torch
    import paper_1503_00330_amd as pi
    from paper_1503_00330_amd import tune
    import synth
    batch = synth.batched_config()
    dms = [pi.DeviceModel(m).fold() for _, m in batch]
    dps = [pi.DeviceProblem(p, tile_samples=args.tile_samples, tile_split=1) for p, _ in batch]
    if not args.tile_samples:
        tiles = tune.ensure_batch(dps, dms)
    else:
        tiles = (args.tile_samples, 4, dps[0].variant)
    for dp in dps:               # plain launches with the batch's tile and waves
        dp.tile_waves = tiles[1]
    stream = torch.cuda.current_stream()
    start = [(d.x0.clone(), d.u_nom.clone(), d.iter.clone()) for d in dps]

    def restore():
        for d, (x, u, it) in zip(dps, start):
            d.x0.copy_(x), d.u_nom.copy_(u), d.iter.copy_(it)

    br = pi.BatchedRollout(dps, dms)
    br.run()
    costs = [torch.empty((p.K, p.T), dtype=torch.float32, device="cuda") for p in dps]

    def seq():
        for dp, dm, c in zip(dps, dms, costs):
            pi.rollout_cost(dp, dm, out=c)
    seq()
    torch.cuda.synchronize()
    tb = timed(br.run, args.steps or 3, stream)
    ts = timed(seq, args.steps or 3, stream)
    same_cost = all(torch.equal(a, c) for a, c in zip(br.costs, costs))
    # the plain baseline a caller would run: each problem on its own in the
    # fastest of the library's default launches of the three contractions
    # (float32 products or bf16 pieces: 16 rollouts per tile, workgroup pairs
    # when the tiles leave compute units idle; fp16 pieces: the 128-rollout
    # shared tile), timed problem by problem
    forms = (pi.PI_VARIANT_MFMA, pi.PI_VARIANT_MFMA_BF16X3, pi.PI_VARIANT_MFMA_F16X2)
    best, picks = [], {}
    for (p, _), dm, c in zip(batch, dms, costs):
        t_form = {}
        for v in forms:
            dp1 = pi.DeviceProblem(p, variant=v)
            pi.rollout_cost(dp1, dm, out=c)
            t_form[v] = float(np.median(timed(lambda: pi.rollout_cost(dp1, dm, out=c), args.steps or 3, stream)))
        v = min(t_form, key=t_form.get)
        best.append(t_form[v])
        picks[v] = picks.get(v, 0) + 1
    td = [sum(best)]

    def seq_step():
        for dp, dm, c in zip(dps, dms, costs):
            pi.rollout_cost(dp, dm, out=c)
            pi.update(dp, c)
            pi.rh_shift(dp, dm)
    seq_step()              # reserves the workspaces before capture
    torch.cuda.synchronize()
    restore()
    g_seq = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g_seq, stream=side):
            seq_step()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    restore()
    br.capture()
    torch.cuda.synchronize()
    reps = args.steps or 3
    tcb = timed(br.graph.replay, reps, stream)
    after_b = [(d.x0.clone(), d.u_nom.clone(), d.iter.clone()) for d in dps]
    restore()
    tcs = timed(g_seq.replay, reps, stream)
    after_s = [(d.x0.clone(), d.u_nom.clone(), d.iter.clone()) for d in dps]
    same_step = all(torch.equal(x, y) for a, b in zip(after_b, after_s) for x, y in zip(a, b))
    restore()
    flop = sum(flops_per_sample_step(m) * p.K * p.T for p, m in batch)
    ss = sum(p.K * p.T for p, _ in batch)
    mb = float(np.median(tb))
    return {"workload": "64 quadrotor problems, K in 512..16384, L in 64..1024 per output, "
                        "T in 50..200, 10..40 obstacles",
            "tiles": {"tile_samples": tiles[0], "tile_waves": tiles[1],
                      "mfma": {pi.PI_VARIANT_MFMA_BF16X3: "bf16x3", pi.PI_VARIANT_MFMA_F16X2: "f16x2"}.get(
                          tiles[2], "f32"),
                      "autotuned": not args.tile_samples},
            "batched_ms": mb,
            "sequential_default_ms": float(np.median(td)),
            "sequential_default_forms": {{pi.PI_VARIANT_MFMA: "f32", pi.PI_VARIANT_MFMA_BF16X3: "bf16x3",
                                          pi.PI_VARIANT_MFMA_F16X2: "f16x2"}[v]: n for v, n in picks.items()},
            "speedup": float(np.median(td) / mb),
            "sequential_same_tiles_ms": float(np.median(ts)),
            "speedup_same_tiles": float(np.median(ts) / mb),
            "control_step_batched_ms": float(np.median(tcb)),
            "control_step_sequential_same_tiles_ms": float(np.median(tcs)),
            "control_step_speedup_same_tiles": float(np.median(tcs) / np.median(tcb)),
            "batched_rollout_steps_per_s": ss / (mb * 1e-3),
            "batched_tflops": flop / (mb * 1e-3) / 1e12,
            "batched_frac_fp32_peak": flop / (mb * 1e-3) / PEAK_FP32,   # float32-equivalent for the pieces forms
            "bitwise_equal_to_plain": bool(same_cost), "control_step_bitwise_equal": bool(same_step),
            "dtype": "f32"}


def w_adjoint(args):
    import torch
    import paper_1503_00330_amd as pi
    import synth
    prob, model, extra = synth.config(4, obs_kind=synth.OBS_SMOOTH)
    dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model)
    stream = torch.cuda.current_stream()
    cost = torch.empty((prob.K, prob.T), dtype=torch.float32, device="cuda")
    pi.rollout_cost(dp, dm, out=cost)
    pi.rollout_adjoint(dp, dm, ckpt_every=extra["ckpt"])
    torch.cuda.synchronize()
    tf = timed(lambda: pi.rollout_cost(dp, dm, out=cost), args.steps or 3, stream)
    ta = timed(lambda: pi.rollout_adjoint(dp, dm, ckpt_every=extra["ckpt"]), args.steps or 3, stream)
    # the whole horizon as one segment: traced by the forward itself, no
    # recompute, the workspace of every step
    pi.rollout_adjoint(dp, dm, ckpt_every=prob.T)
    tw = timed(lambda: pi.rollout_adjoint(dp, dm, ckpt_every=prob.T), args.steps or 3, stream)
    # the forward and the segment recomputes in the two-piece fp16 contraction
    # (the reverse sweep and the parameter pass stay float32), against the
    # plain forward in the same contraction
    dph = pi.DeviceProblem(prob, variant=pi.PI_VARIANT_MFMA_F16X2)
    pi.rollout_cost(dph, dm, out=cost)
    pi.rollout_adjoint(dph, dm, ckpt_every=extra["ckpt"])
    torch.cuda.synchronize()
    tfh = timed(lambda: pi.rollout_cost(dph, dm, out=cost), args.steps or 3, stream)
    tah = timed(lambda: pi.rollout_adjoint(dph, dm, ckpt_every=extra["ckpt"]), args.steps or 3, stream)
    ss = prob.K * prob.T
    d = model.d
    f_fwd = flops_per_sample_step(model) * ss
    f_adj = model.Ltot * (3 * d * d + 9 * d + 15) * ss
    import ctypes
    ps, ms = dp.struct(), dm.struct()
    ws_bytes = int(pi.load().pi_adjoint_workspace_bytes(ctypes.byref(ps), ctypes.byref(ms), extra["ckpt"]))
    ws_whole = int(pi.load().pi_adjoint_workspace_bytes(ctypes.byref(ps), ctypes.byref(ms), prob.T))
    return {"workload": "quadrotor adjoint K=8192 T=400 d=16 6x256 models, checkpoints every 20, "
                        "smooth obstacles",
            "ckpt_every": extra["ckpt"], "workspace_bytes": ws_bytes,
            "executed_forward_passes": 2,
            "whole_horizon_segment": {"fused_forward_adjoint_ms": float(np.median(tw)), "workspace_bytes": ws_whole,
                                      "ratio": float(np.median(tw) / np.median(tf))},
            "forward_ms": float(np.median(tf)), "fused_forward_adjoint_ms": float(np.median(ta)),
            "ratio": float(np.median(ta) / np.median(tf)),
            "forward_rollout_steps_per_s": ss / (float(np.median(tf)) * 1e-3),
            "fused_rollout_steps_per_s": ss / (float(np.median(ta)) * 1e-3),
            "forward_tflops": f_fwd / (float(np.median(tf)) * 1e-3) / 1e12,
            "fused_algorithmic_tflops": (f_fwd + f_adj) / (float(np.median(ta)) * 1e-3) / 1e12,
            "f16x2_forward": {"forward_ms": float(np.median(tfh)), "fused_forward_adjoint_ms": float(np.median(tah)),
                              "ratio": float(np.median(tah) / np.median(tfh)),
                              "fused_vs_float32_fused": float(np.median(tah) / np.median(ta))},
            "dtype": "f32"}


def w_paper(args):
    """The paper's timing shapes on its own model structure (Sec. 4, 4.1): the
    hybrid quadrotor with three LWPR models of (angles, thrust), 15/15/24 local
    models; one iteration = rollouts + update.  Also the largest K whose
    iteration fits in 20 ms, per M (a real-time budget of the kind the paper's
    controller runs under)."""
    import torch
    import paper_1503_00330_amd as pi
    import synth
    stream = torch.cuda.current_stream()

    def iteration_ms(M, K, reps):
        prob, model = synth.paper_shape(M=M, K=K)
        dp, dm = pi.DeviceProblem(prob), pi.DeviceModel(model).fold()
        cost = torch.empty((prob.K, prob.T), dtype=torch.float32, device="cuda")

        def it():
            pi.rollout_cost(dp, dm, out=cost)
            pi.update(dp, cost)
        it()
        torch.cuda.synchronize()
        return timed(it, reps, stream)

    rows = []
    for M in (0, 1, 4, 8, 16, 32):
        ms = iteration_ms(M, 1000, args.steps or 20)
        # largest K (multiple of 1000) with p50 iteration <= 20 ms, by doubling then bisection
        lo, hi = 1000, 2000
        while float(np.percentile(iteration_ms(M, hi, 5), 50)) <= 20.0 and hi < 1 << 24:
            lo, hi = hi, hi * 2
        while hi - lo > max(1000, lo // 50):
            mid = (lo + hi) // 2
            if float(np.percentile(iteration_ms(M, mid, 5), 50)) <= 20.0:
                lo = mid
            else:
                hi = mid
        rows.append({"M": M, "iteration_ms_p50": pct(ms, 50), "iteration_ms_p99": pct(ms, 99),
                     "sub_rollout_steps_per_s": 1000 * max(M, 1) * 50 / (pct(ms, 50) * 1e-3),
                     "max_K_in_20ms": lo})
    # Table 2's settings (rollouts, iterations per control step) for the
    # sub-rollout counts: one whole control step (iterations x (rollouts +
    # update), then the plant step and shift) replayed as a HIP graph
    from paper_1503_00330_amd.rh import RHController
    table2 = []
    for M, K, iters in ((1, 1000, 2), (4, 1000, 2), (8, 1000, 1), (16, 970, 1), (32, 950, 1)):
        prob, model = synth.paper_shape(M=M, K=K)
        ctl = RHController(pi.DeviceProblem(prob), pi.DeviceModel(model), iterations=iters, graph=True)
        for _ in range(3):
            ctl.step()
        torch.cuda.synchronize()
        ms = timed(ctl.step, args.steps or 20, stream)
        table2.append({"M": M, "K": K, "iterations": iters, "control_step_ms_p50": pct(ms, 50),
                       "control_step_ms_p99": pct(ms, 99)})
    return {"workload": "paper's model and timing shapes: hybrid quadrotor, LWPR (phi, theta, psi, F) -> "
                        "(x'', y'', z''), 15/15/24 local models, R = 2, 1000 rollouts x 50 steps, "
                        "M sub-rollouts (M = 0: mean prediction only); iteration = rollouts + update",
            "rows": rows, "table2_control_steps": table2, "dtype": "f32",
            "paper_reference": "GTX 780 Ti: 6.5 ms (M = 0) and 18 ms (M = 32) per iteration (Sec. 4)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True,
                    choices=["cfg0", "rh-graph", "batched", "adjoint", "paper"])
    ap.add_argument("--steps", type=int, default=0)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tile-samples", type=int, default=0)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    fn = {"cfg0": w_cfg0, "rh-graph": w_rh_graph, "batched": w_batched, "adjoint": w_adjoint,
          "paper": w_paper}[args.workload]
    if args.workload == "cfg0" and not args.steps:
        args.steps = 200
    out = fn(args)
    out["bench"] = args.workload
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
