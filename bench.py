"""Benchmark of the whole-body MPPI hot path on one MI355X.

One step = one closed-loop control step of the box-pushing workload (K = 4096 samples,
horizon H = 60 at dt = 0.01 s, 8 knots per joint, the quadruped and a free 2 kg box on
flat ground; by default 2000 timed steps as 10 episodes of 200 steps from seeds 0-9):
Philox sampling, the fused rollout of all samples (the lane-split kernel, 16 lanes per
sample, FP32 step arithmetic), the Eq. 1 / Eq. 2 update with first-control extraction
and shift, and one plant step with the chosen control -- all on the GPU, inputs resident
in HBM.  Prints one JSON line.

Metric: rollout-steps/s (K * H per control step) and the p50/p99 control-step latency
(HIP events around each step on the library's stream).  The roofline object reports the
rollout kernel's algorithmic FLOP rate (flops per rollout-step counted from the step's
formulation, times K * H, over its event-timed duration) against the MI355X vector peak
of the step's arithmetic type.  cpu_baseline times the FP64 CPU oracle on a bounded
sample of the same workload on this host's cores.  learned_vs_plain runs a bounded
version of the learned-proposal comparison (train on GPU closed loops, then plain MPPI
at several K against the proposal at K/4 on the same seeds).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2409_10469_amd.roofline import PEAK_TFLOPS, flops_per_rollout_step  # noqa: E402
from paper_2409_10469_amd.timing import DeviceEvent  # noqa: E402

SCENE_NAMES = {0: "flat ground", 1: "heightfield 64x64", 2: "flat ground + static box (climb)",
               3: "flat ground + free box (push)"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("mppi_device.h", "mppi_kernels.hip", "rollout16.hip"):
        h.update(open(os.path.join(ROOT, "paper_2409_10469_amd", "csrc", f), "rb").read())
    h.update(open(os.path.join(ROOT, "paper_2409_10469_amd", "build.py"), "rb").read())  # compile flags
    return h.hexdigest()[:16]


def _kernel_tag(lanes: int) -> str:
    return "rollout16" if lanes == 16 else "rollout"


def _kernel_name(scene: int, arith: str, lanes: int) -> str:
    r = "double" if arith == "fp64" else "float"
    s = "float" if arith == "fp32" else "double"
    return f"rollout16_kernel<{scene}, {r}, {s}>" if lanes == 16 else f"rollout_kernel<{scene}, {r}>"


def _dtype(arith: str) -> str:
    return {"fp64": "f64", "fp32": "f32", "mixed": "f32+f64"}[arith]


def traffic_from_profile(workload: str, arith: str, lanes: int = 16):
    """Counter-measured HBM bytes per rollout launch, if the committed counter summary
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{_kernel_tag(lanes)}_{workload}_{arith}_hbm.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def hbm_rate(bytes_per_launch, kernel_ms):
    """HBM bytes of the rollout launch (counters, copy-calibrated) over its live duration."""
    if bytes_per_launch is None:
        return None
    gbs = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    return {"achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
            "bytes_per_launch": bytes_per_launch}


def counter_rate(flops_per_launch, kernel_ms, peak):
    if flops_per_launch is None:
        return None
    tf = flops_per_launch / (kernel_ms * 1e-3) / 1e12
    return {"achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak, "flops_per_launch": flops_per_launch,
            "source": "VALU instruction counters, 64 x (ADD + MUL + 2 FMA + TRANS)"}


def counter_flops_from_profile(workload: str, arith: str, lanes: int = 16):
    """Counter FLOPs per rollout launch (64 x (ADD + MUL + 2 FMA + TRANS) from the VALU
    instruction counters), if the committed summary was taken on the current source."""
    path = os.path.join(ROOT, "profiles", f"{_kernel_tag(lanes)}_{workload}_{arith}_flops.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("counter_flops_per_launch")


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(orc, workload, p, seed, seconds, threads):
    """Closed-loop control steps of the oracle for about `seconds`: rollout-steps/s, steps."""
    from paper_2409_10469_amd import workloads as W
    x = W.initial_state(seed, workload["scene"])
    mu = W.stance_knots(p["nk"])
    steps, t0 = 0, time.perf_counter()
    while True:
        u0, mu, _, _ = orc.mppi_step(p, steps, x, mu, nthreads=threads)
        x, _, _ = orc.step(x, u0, p["kp"], p["kd"], p["dt"])
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return steps * p["K"] * p["H"] / el, steps, el


def cpu_baseline(workload, seed, seconds):
    """The FP64 oracle on this host: all cores (OpenMP over samples) for `seconds`, one
    thread for a third of that; the paper's CPU rate is quoted beside it as context."""
    from oracle import oracle as O
    from paper_2409_10469_amd import workloads as W
    md = W.model_dict(workload, seed)
    p = W.params_dict(workload, seed)
    orc = O.Oracle(md)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    rate, steps, el = _oracle_rate(orc, workload, p, seed, seconds, threads)
    rate1, steps1, el1 = _oracle_rate(orc, workload, p, seed, seconds / 3, 1)
    return {"value": rate, "unit": "rollout-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} closed-loop control steps of {workload['name']} (K={p['K']}, H={p['H']}) "
                      f"in {el:.1f} s, FP64 oracle, OpenMP over samples",
            "single_thread": {"value": rate1, "unit": "rollout-steps/s",
                              "sample": f"{steps1} control steps in {el1:.1f} s on one thread"},
            "ms_per_update": el / steps * 1e3, "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "paper_reference": {"value": 1.2e5, "unit": "rollout-steps/s",
                                "derived_from": "100 Hz control with 30 samples x 40 steps (Sec. IV-A), a lower bound",
                                "hardware": "Intel i9-12900KS, multi-threaded MuJoCo rollouts",
                                "note": "different simulator and contact model; context, not a target"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed control steps")
    ap.add_argument("--episode-steps", type=int, default=200,
                    help="control steps per closed-loop episode (a new seed every episode)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="box_push",
                    help="box_push (default), heightfield_walk, flat_walk, box_climb, batched_serving, "
                         "proposal_training, ablations or tracking")
    ap.add_argument("--arith", default="fp32", choices=["fp64", "fp32", "mixed"],
                    help="step arithmetic: fp64, fp32, or mixed (FP32 geometry, FP64 implicit system; lane-split "
                         "kernel, single-controller workloads)")
    ap.add_argument("--lanes", type=int, default=16, choices=[4, 16],
                    help="rollout kernel: 16 lanes per sample (lane-split, default) or 4 (one lane per leg)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the bounded learned-proposal comparison of the default run")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--pairs", type=int, default=1_000_000, help="proposal_training: closed-loop pairs")
    ap.add_argument("--epochs", type=int, default=8, help="proposal_training: Adam epochs")
    ap.add_argument("--eval-seeds", type=int, default=10, help="proposal_training: evaluation episodes")
    ap.add_argument("--eval-steps", type=int, default=200, help="proposal_training: steps per evaluation episode")
    ap.add_argument("--eval-instances", type=int, default=256,
                    help="proposal_training: instances of the batched-serving evaluation")
    ap.add_argument("--batch-tuning", default=None, metavar="BPC,ORDER,MODE",
                    help="batched_serving: fixed tuning instead of the autotuner (blocks per CU, tile order "
                         "0 admission / 1 longest first, launch mode 0 per scene / 1 one kernel for every scene)")
    ap.add_argument("--budget-mib", type=int, default=256,
                    help="batched_serving: the HBM budget that admits instances (MiB); 256 (default) admits every "
                         "request, about 256 live; 64 binds admission")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the multi-GPU sharding is a design only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2409_10469_amd import binding as B
    from paper_2409_10469_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.arith == "mixed" and args.workload in ("batched_serving", "proposal_training", "tracking"):
        print(json.dumps({"error": "mixed arithmetic runs in single controllers only (the lane-split rollout)"}))
        sys.exit(2)
    if args.workload == "batched_serving":
        return bench_serving(args)
    if args.workload == "proposal_training":
        return bench_proposal(args)
    if args.workload == "tracking":
        return bench_tracking(args)
    if args.workload == "ablations":
        return bench_ablation(args)
    wl = W.WORKLOADS[args.workload]
    md = W.model_dict(wl, args.seed)
    p = W.params_dict(wl, args.seed, arith=args.arith, lanes=args.lanes)
    model = B.Model(md)
    K, H, nk = p["K"], p["H"], p["nk"]
    stream = torch.cuda.current_stream()
    # closed-loop episodes of `episode_steps` control steps on one terrain, each from its
    # own seeded initial state with its own controller (own Philox key); controllers and
    # buffers are made before the timed region
    n_ep = max(1, -(-args.steps // args.episode_steps))
    seeds = [args.seed + e for e in range(n_ep)]
    ctls = [B.Controller(model, dict(p, seed=sd)) for sd in seeds]
    x0s = [torch.tensor(W.initial_state(sd, wl["scene"]), dtype=torch.float32, device="cuda") for sd in seeds]
    stance = torch.tensor(W.stance_knots(nk), dtype=torch.float32, device="cuda")
    x = [torch.empty(model.nx, dtype=torch.float32, device="cuda") for _ in range(2)]
    costs = torch.empty(K, dtype=torch.float32, device="cuda")
    u0 = torch.empty(12, dtype=torch.float32, device="cuda")
    cur = {"ctl": ctls[0], "i": 0}

    def start_episode(e):
        cur["ctl"] = ctls[e]
        cur["ctl"].set_nominal(stance)
        cur["ctl"].set_step(0)
        x[0].copy_(x0s[e])
        cur["i"] = 0

    def control_step(ev_start=None, ev_roll=None, ev_end=None, weights=None):
        i, ctl = cur["i"], cur["ctl"]
        xi, xo = x[i % 2], x[(i + 1) % 2]
        if ev_start:
            ev_start.record(stream)
        ctl.rollout_batch(xi, costs=costs)
        if ev_roll:
            ev_roll.record(stream)
        ctl.update_shift(costs, u0, weights=weights)
        model.sim_step_into(xi.view(1, -1), u0.view(1, -1), p["kp"], p["kd"], p["dt"], xo.view(1, -1),
                            arith=args.arith)
        if ev_end:
            ev_end.record(stream)
        cur["i"] = i + 1

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    start_episode(0)
    for _ in range(args.warmup):
        control_step()
    torch.cuda.synchronize()
    # Stream events (device-scope release, see timing.py); each record costs the stream a
    # few microseconds, so a step records one at its start, its latency running to the
    # next step's start (to an event of its own at the end of an episode, so that the
    # next episode's reset is not counted), and every ROLL_EVERY-th step one more after
    # its rollout for the rollout kernel's duration
    ROLL_EVERY = 4
    last = lambda k: (k + 1) % args.episode_steps == 0 or k == args.steps - 1  # noqa: E731
    ev_start = [DeviceEvent() for _ in range(args.steps)]
    ev_roll = {k: DeviceEvent() for k in range(0, args.steps, ROLL_EVERY)}
    ev_end = {k: DeviceEvent() for k in range(args.steps) if last(k)}
    wbuf = torch.empty((args.steps, K), dtype=torch.float32, device="cuda")  # each step's Eq. 1 weights
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k % args.episode_steps == 0:
            start_episode(k // args.episode_steps)
        control_step(ev_start[k], ev_roll.get(k), ev_end.get(k), wbuf[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = np.array([ev_start[k].elapsed_time(ev_end[k] if k in ev_end else ev_start[k + 1])
                        for k in range(args.steps)])
    roll_ms = np.array([ev_start[k].elapsed_time(e) for k, e in sorted(ev_roll.items())])
    status = max(c.sync_status() for c in ctls)
    w64 = wbuf.double()
    ess = (w64.sum(1) ** 2 / (w64 ** 2).sum(1)).cpu().numpy()  # effective sample size per step
    xf = x[cur["i"] % 2].cpu().numpy()

    value = K * H * args.steps / elapsed
    flops = flops_per_rollout_step(wl["scene"], nk) * K * H
    achieved = flops / (roll_ms.mean() * 1e-3) / 1e12
    # mixed arithmetic is priced against the FP32 peak, the higher of the two it uses
    peak = PEAK_TFLOPS["fp32" if args.arith == "mixed" else args.arith]
    out = {
        "metric": "rollout-steps/sec + p99 MPPI step latency; learned-proposal vs plain at equal cost",
        "value": value,
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": _dtype(args.arith),
        "data": "synthetic",
        "config": {"workload": wl["name"], "K": K, "H": H, "dt": p["dt"], "n_knots": nk,
                   "scene": SCENE_NAMES[wl["scene"]], "closed_loop": True, "state": "f32",
                   "step_arithmetic": args.arith, "rollout_lanes_per_sample": args.lanes,
                   "episodes": n_ep, "episode_steps": args.episode_steps, "seeds": [seeds[0], seeds[-1]]},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "mean": float(step_ms.mean())},
        "rollout_kernel_ms": float(roll_ms.mean()),
        "timing": f"stream events: every step's start (latency to the next start, or to an event of its own at an "
                  f"episode's end), and the rollout's end on every {ROLL_EVERY}th step ({roll_ms.size} launches)",
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic_from_profile(wl["name"], args.arith, args.lanes),
                     "flops_per_rollout_step": flops_per_rollout_step(wl["scene"], nk),
                     "kernel": _kernel_name(wl["scene"], args.arith, args.lanes)},
        "counter_flops": counter_rate(counter_flops_from_profile(wl["name"], args.arith, args.lanes), roll_ms.mean(),
                                      peak),
        "hbm_gbs": hbm_rate(traffic_from_profile(wl["name"], args.arith, args.lanes), roll_ms.mean()),
        "ess": {"mean": float(np.mean(ess)), "median": float(np.median(ess)), "min": float(np.min(ess)),
                "of_K": K},
        "final_state_finite": bool(np.isfinite(xf).all()),
        "update_status": int(status),
    }
    if not args.no_learned:
        out["learned_vs_plain"] = learned_vs_plain(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.seed, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def learned_vs_plain(args):
    """Bounded learned-proposal comparison (the full one is --workload proposal_training):
    2e5 closed-loop pairs from the flat and heightfield walks, 6 Adam epochs, then the
    heightfield walk (v_ref 0.5, 5 held-out seeds x 100 steps) with plain MPPI at K in
    {256, 512, 1024, 2048, 4096} against the proposal at 256 samples with plain MPPI at
    K = 1024 as the fallback (cost gate, best-sample gate, best-sample gate with both sets
    rolled out in one launch on every step) and ungated."""
    from paper_2409_10469_amd import binding as B
    from paper_2409_10469_amd import proposal as PR
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    data = PR.generate(n_pairs=200_000, episode_steps=200, instances=256, seed=args.seed, log=log)
    tr, ho = PR.split(data, holdout=0.05, seed=args.seed)
    pol = B.Policy(max_batch=4096, seed=args.seed)
    pol.set_normalization(*PR.normalization(data, tr))
    PR.train(pol, data, tr, epochs=6, batch=4096, lr=1e-3, seed=args.seed, held=ho, log=log)
    ev = PR.evaluate(pol, K_plain=(256, 512, 1024, 2048, 4096), K_learned=1024, seeds=range(100, 105), steps=100,
                     log=log)
    res = {"task": "heightfield walk, v_ref 0.5, closed loop", "seeds": ev["seeds"], "steps": ev["steps"],
           "training": "2e5 pairs, 6 epochs", "seconds": time.perf_counter() - t0,
           "plain": {str(k): {"episode_cost": v["mean"], "ci95": v["ci95"], "samples_per_step": k,
                              "latency_p50_ms": v["latency_ms"]["p50"], "latency_p99_ms": v["latency_ms"]["p99"]}
                     for k, v in ev["plain"].items()}}
    for g in ("cost", "best", "best-concurrent", "none"):
        e = ev["learned_" + g]
        res["learned_gate_" + g.replace("-", "_")] = {
            "episode_cost": e["mean"], "ci95": e["ci95"], "k_prop": e["k_prop"],
            "samples_per_step": e["samples_per_step"], "acceptance": e["acceptance"],
            "latency_p50_ms": e["latency_ms"]["p50"], "latency_p99_ms": e["latency_ms"]["p99"],
            "smallest_plain_K_matching": e["smallest_plain_K_matching"], "sample_ratio": e["sample_ratio"]}
    return res


def bench_serving(args):
    """256 MPPI instances (mixed tasks, K log-uniform in [256, 4096], H uniform in
    [20, 80]) under a seeded Poisson stream admitted by an HBM budget (256 MiB by default)."""
    import numpy as np
    from paper_2409_10469_amd.serving import ServingSim
    sim = ServingSim(seed=args.seed, arith=args.arith, budget_bytes=args.budget_mib << 20)
    sim.prefill(256)
    fixed = None
    if args.batch_tuning:
        fixed = [int(v) for v in args.batch_tuning.split(",")]
        if len(fixed) != 3:
            raise SystemExit("--batch-tuning takes BPC,ORDER,MODE")
        sim.batch.set_tuning(fixed[0], fixed[1])
        sim.batch.set_launch_mode(fixed[2])
    r = sim.run(args.steps, warmup=args.warmup, autotune=fixed is None)
    lat = r["latency_ms"]
    value = r["rollout_steps"] / r["elapsed"]
    achieved = r["flops"] / (lat.sum() * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.arith]
    qd = r["queue_delay"]
    out = {
        "metric": "rollout-steps/sec + p99 MPPI step latency",
        "value": value, "unit": "rollout-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["elapsed"] / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": _dtype(args.arith), "data": "synthetic",
        "config": {"workload": "batched_serving", "target_instances": 256, "K": "log-uniform [256, 4096]",
                   "H": "uniform [20, 80]", "tasks": "flat, heightfield, box climb, box push",
                   "arrivals": "Poisson, lifetime 200 steps", "hbm_budget_mib": args.budget_mib, "state": "f32",
                   "step_arithmetic": args.arith},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "host_admission_ms": {"p50": float(np.percentile(r["host_ms"], 50)),
                              "p99": float(np.percentile(r["host_ms"], 99))},
        "live_instances": {"mean": float(r["live"].mean()), "min": int(r["live"].min()), "max": int(r["live"].max())},
        "queueing_delay_steps": {"mean": float(qd.mean()) if qd.size else 0.0,
                                 "p99": float(np.percentile(qd, 99)) if qd.size else 0.0},
        "autotune": {"blocks_per_cu": r["tune"][0], "order": "longest_first" if r["tune"][1] else "admission",
                     "launch": "one kernel for every scene" if r["tune"][3] else "one kernel per scene",
                     "ms": r["tune"][2]} if r["tune"] else None,
        "fixed_tuning": {"blocks_per_cu": fixed[0], "order": "longest_first" if fixed[1] else "admission",
                         "launch": "one kernel for every scene" if fixed[2] else "one kernel per scene"}
        if fixed else None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None},
        "budget": r["stats"],
    }
    print(json.dumps(out), flush=True)


def mlp_train_flops_per_pair():
    """Algorithmic flops of one training pair: forward and weight-gradient products over
    every layer, input-gradient products over layers 1..4 (2 flops per multiply-add)."""
    dims = (40, 512, 512, 512, 512, 144)
    layers = list(zip(dims[:-1], dims[1:]))
    fwd = sum(2 * a * b for a, b in layers)
    return 2 * fwd + sum(2 * a * b for a, b in layers[1:])


def bench_proposal(args):
    """Learned-proposal training: closed-loop pairs from the flat and heightfield walks
    generated on the GPU, then Adam epochs on the Gaussian NLL (batch 4096)."""
    import numpy as np
    import torch
    from paper_2409_10469_amd import binding as B
    from paper_2409_10469_amd import proposal as PR
    log = lambda m: print(m, flush=True)
    t0 = time.perf_counter()
    data = PR.generate(n_pairs=args.pairs, episode_steps=200, instances=256, seed=args.seed, arith=args.arith, log=log)
    gen_s = time.perf_counter() - t0
    tr, ho = PR.split(data, holdout=0.05, seed=args.seed)
    pol = B.Policy(max_batch=4096, seed=args.seed)
    pol.set_normalization(*PR.normalization(data, tr))
    nll0 = PR.nll(pol, data, ho)
    hist = PR.train(pol, data, tr, epochs=args.epochs, batch=4096, lr=1e-3, seed=args.seed, held=ho, log=log)
    # timed train steps for the roofline (events on the policy's stream)
    stream = torch.cuda.current_stream()
    idx = tr[:4096].contiguous()
    loss = torch.empty(1, device="cuda")
    for _ in range(5):
        pol.train_step(data["X"], data["Y"], index=idx, B=4096, lr=0.0, loss=loss)
    e0, e1 = DeviceEvent(), DeviceEvent()
    n_t = 50
    e0.record(stream)
    for _ in range(n_t):
        pol.train_step(data["X"], data["Y"], index=idx, B=4096, lr=0.0, loss=loss)
    e1.record(stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / n_t
    fl = mlp_train_flops_per_pair() * 4096
    achieved = fl / (step_ms * 1e-3) / 1e12
    pairs_s = 4096 / (step_ms * 1e-3)
    ev = PR.evaluate(pol, seeds=range(100, 100 + args.eval_seeds), steps=args.eval_steps, arith=args.arith, log=log)
    evb = PR.evaluate_batched(pol, n_inst=args.eval_instances, steps=args.eval_steps, arith=args.arith, log=log)
    train_s = sum(h[2] for h in hist)
    train_steps = sum(h[3] for h in hist)
    st = data["stats"]
    out = {
        "metric": "learned-proposal training pairs/sec", "value": pairs_s, "unit": "pairs/s", "n_gpus": 1,
        "steps": n_t, "warmup": 5, "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (fp32 accumulate, fp32 Adam)", "data": "synthetic (GPU closed loops)",
        "config": {"workload": "proposal_training", "network": "40-512x4-144 SiLU", "batch": 4096,
                   "pairs": int(data["X"].shape[0]), "held_out_pairs": int(ho.numel()), "epochs": args.epochs,
                   "sources": "flat_walk (K=64,H=25,4 knots -> 6) + heightfield_walk (K=1024,H=50,6 knots)",
                   "rollout_arithmetic": args.arith},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None, "flops_per_pair": mlp_train_flops_per_pair(),
                     "scope": "whole train step (13 GEMMs, loss, reduction, Adam)"},
        "held_out_nll": {"untrained": nll0, "per_epoch": [h[1] for h in hist]},
        "train_nll_per_epoch": [h[0] for h in hist],
        "equal_cost_evaluation": {
            "task": "heightfield walk, v_ref 0.5, closed loop", "seeds": ev["seeds"], "steps": ev["steps"],
            "plain_episode_cost": {str(k): v["mean"] for k, v in ev["plain"].items()},
            "plain_episode_cost_ci95": {str(k): v["ci95"] for k, v in ev["plain"].items()},
            "plain_step_latency_ms": {str(k): v["latency_ms"] for k, v in ev["plain"].items()},
            "learned": {g: {"episode_cost": ev["learned_" + g]["mean"], "k_prop": ev["learned_" + g]["k_prop"],
                            "fallback_K": ev["learned_" + g]["K_fallback"],
                            "acceptance": ev["learned_" + g]["acceptance"],
                            "samples_per_step": ev["learned_" + g]["samples_per_step"],
                            "step_latency_ms": ev["learned_" + g]["latency_ms"],
                            "episode_cost_ci95": ev["learned_" + g]["ci95"],
                            "smallest_plain_K_matching": ev["learned_" + g]["smallest_plain_K_matching"],
                            "sample_ratio": ev["learned_" + g]["sample_ratio"]}
                        for g in ("cost", "best", "best-concurrent", "none")},
            "gates": "cost: the proposal's K/4 samples are rolled out, then the plain step's K samples only when "
                     "the proposal's centre costs more than the nominal (fallback); best: the same with the least "
                     "cost over the proposal's samples other than the nominal; best-concurrent: the best-sample "
                     "gate with both sample sets rolled out in one launch on every step; none: always the K/4 "
                     "proposal samples alone, nominal kept as sample 1"},
        "batched_equal_cost": evb,
        "epoch_seconds": train_s / max(len(hist), 1), "train_steps": train_steps,
        "generation": {"seconds": gen_s, "batch_seconds": st["seconds"], "episodes": st["episodes"],
                       "falls": st["falls"], "control_steps": st["control_steps"],
                       "rollout_steps_per_s": st["rollout_steps"] / max(st["seconds"], 1e-9)},
    }
    print(json.dumps(out), flush=True)


def bench_ablation(args):
    """The ablations of the plain method: closed-loop episodes with the cubic, linear and
    zeroth-order knot interpolation (same seeds, samples and horizon), then one-at-a-time
    sweeps of lambda, H, K and the control rate on the heightfield walk."""
    from paper_2409_10469_amd import ablations as AB
    log = lambda m: print(m, flush=True)
    t0 = time.perf_counter()
    res = AB.sampling_ablation(seeds=range(args.seed, args.seed + args.eval_seeds), steps=args.eval_steps,
                               arith=args.arith, log=log)
    sweeps = AB.hyperparameter_sweeps(seeds=range(args.seed, args.seed + args.eval_seeds), steps=args.eval_steps,
                                      arith=args.arith, log=log)
    sweeps["rate_hz_dt4ms"] = AB.control_rate_sweep(seeds=range(args.seed, args.seed + args.eval_seeds),
                                                    arith=args.arith, log=log)
    walk = res["heightfield_walk_6_knots"]["bases"]
    out = {"metric": "closed-loop episode cost of the plain method's ablations", "value": walk["cubic"]["mean"],
           "unit": "episode cost (heightfield walk, cubic)", "n_gpus": 1, "steps": args.eval_steps,
           "warmup": 0, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": _dtype(args.arith), "data": "synthetic",
           "config": {"workload": "ablations", "seeds": [args.seed, args.seed + args.eval_seeds - 1],
                      "episode_steps": args.eval_steps},
           "tasks": res, "sweeps": sweeps, "seconds": time.perf_counter() - t0}
    print(json.dumps(out), flush=True)


def bench_tracking(args):
    """Eq. 3 / Eq. 4 (the tracking cost) against the running cost in closed loop: walking on
    flat ground and on the heightfield with the standing and the trotting joint reference,
    the box push with the l1 box term, and the control-step latency the cost kernel adds
    at the heightfield launch shape (K 1024, H 50)."""
    import numpy as np
    import torch
    from paper_2409_10469_amd import ablations as AB
    from paper_2409_10469_amd import binding as Bd
    from paper_2409_10469_amd import workloads as W
    log = lambda m: print(m, flush=True)
    t0 = time.perf_counter()
    seeds = range(args.seed, args.seed + args.eval_seeds)
    walk = AB.tracking_ablation(seeds=seeds, steps=300, arith=args.arith, log=log)
    push = AB.push_ablation(seeds=seeds, steps=400, arith=args.arith, log=log)
    # latency of a control step with each cost (events on the controller's stream)
    wl = W.TERRAIN_WALK
    model = Bd.Model(W.model_dict(wl, 0))
    lat = {}
    for name in ("running", "tracking"):
        p = dict(W.params_dict(wl, 0), arith=args.arith, cost=name)
        ctl = Bd.Controller(model, p)
        if name == "tracking":
            ctl.set_tracking_cost(W.tracking_cost())
        x = torch.tensor(W.initial_state(0, wl["scene"]), dtype=torch.float32, device="cuda")
        u0 = torch.empty(12, dtype=torch.float32, device="cuda")
        ctl.set_nominal(torch.tensor(W.stance_knots(p["nk"]), dtype=torch.float32, device="cuda"))
        for _ in range(10):
            ctl.step(x, u0)
        ev = [(DeviceEvent(), DeviceEvent()) for _ in range(200)]
        for a, b in ev:
            a.record()
            ctl.step(x, u0)
            b.record()
        torch.cuda.synchronize()
        v = [a.elapsed_time(b) for a, b in ev]
        lat[name] = dict(p50=float(np.percentile(v, 50)), p99=float(np.percentile(v, 99)))
        log(f"  control step with the {name} cost: p50 {lat[name]['p50']:.3f} ms, p99 {lat[name]['p99']:.3f} ms")
    trot = walk["heightfield"]["eq3_trot"]
    out = {"metric": "closed-loop forward-velocity error with the Eq. 3 trotting reference (heightfield)",
           "value": trot["v_err"], "unit": "m/s", "n_gpus": 1, "steps": 300, "warmup": 0,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": _dtype(args.arith), "data": "synthetic",
           "config": {"workload": "tracking", "seeds": [args.seed, args.seed + args.eval_seeds - 1],
                      "walk_steps": 300, "push_steps": 400, "controller": "K 1024, H 50, dt 0.01, 6 knots (walk); "
                      "K 4096, H 60, 8 knots (push)"},
           "walk": walk, "push": push, "step_latency_ms": lat, "seconds": time.perf_counter() - t0}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
