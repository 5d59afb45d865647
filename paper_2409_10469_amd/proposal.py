"""Learned sampling proposal: training data from GPU closed loops and training.

Data.  Closed loops of the flat-ground walk (64 samples, 25 steps of 0.02 s, 4 knots)
and the heightfield walk (1024 samples, 50 steps of 0.01 s, 6 knots) run as instances
of a Batch; each instance draws its forward-velocity command from U[0, 0.8] m/s (the
lateral and yaw-rate commands are 0) and records, every control step, the state the step
started from and the step's updated, unshifted knots.  Each record becomes one pair
  input  = state with base x, y relative to the episode origin, then the command (40)
  target = updated knots at 6 knots per joint (72); the 4-knot plans are resampled to 6
           knots at the same fractions of their 0.5 s horizon (both horizons are 0.5 s).
Rows from the step at which an episode's base drops below 0.12 m (a fall) or turns
non-finite, onwards, are dropped.  Episodes are split into training and held-out sets
by episode.

Training.  Gaussian negative log-likelihood with Adam (lr 1e-3, batch 4096), inputs and
targets standardised with the training set's per-feature mean and std.  Every product,
loss, gradient and update runs in the library's kernels; this module generates the
index permutations and evaluates held-out loss.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding as B
from . import workloads as W
from .timing import DeviceEvent

CONFIGS = (W.FLAT_WALK, W.TERRAIN_WALK)
V_RANGE = (0.0, 0.8)
FALL_Z = 0.12


def generate(n_pairs=1_000_000, episode_steps=200, instances=256, seed=0, arith="fp64", budget=1 << 30,
             log=print):
    """Closed-loop pairs from both configs, half each.  Returns dict of float32 device
    tensors X (N x 40), Y (N x 72) and int32 episode ids, plus bookkeeping."""
    import torch
    rng = np.random.default_rng([seed, 77])
    Xs, Ys, Es = [], [], []
    ep_id = 0
    stats = dict(episodes=0, falls=0, control_steps=0, rollout_steps=0, seconds=0.0)
    stream = torch.cuda.current_stream()
    for ci, wl in enumerate(CONFIGS):
        target = n_pairs // len(CONFIGS) + (n_pairs % len(CONFIGS) if ci == 0 else 0)
        got = 0
        nk, K, H = wl["nk"], wl["K"], wl["H"]
        nx, D = 37, 12 * nk
        batch = B.Batch(max_instances=instances, budget_bytes=budget, max_horizon=H,
                        max_hf_cells=W.HF_N * W.HF_N, arith=arith)
        model = B.Model(W.model_dict(wl, 0))
        slot = batch.add_model(model)
        while got < target:
            n_inst = min(instances, math.ceil((target - got) / episode_steps))
            recs, meta = [], []
            # one record per instance, consecutive, as the pairs kernel reads them
            rec_all = torch.empty((n_inst, episode_steps, nx + D), dtype=torch.float32, device="cuda")
            for k in range(n_inst):
                s = int(rng.integers(1 << 30))
                v = float(rng.uniform(*V_RANGE))
                origin = tuple(rng.uniform(-0.5, 0.5, 2)) if wl["scene"] == W.SCENE_HEIGHTFIELD else (0.0, 0.0)
                p = W.params_dict(wl, s, v_ref=v, instance=ep_id + k, arith=arith)
                x0 = W.initial_state(s, wl["scene"], origin=origin)
                i = batch.admit(slot, p, x0, W.stance_knots(nk))
                if i is None:
                    raise RuntimeError("instance does not fit in the generation budget")
                rec = rec_all[k]
                batch.record(i, rec)
                recs.append((i, rec))
                meta.append((v, origin))
            t0 = time.perf_counter()
            for _ in range(episode_steps):
                batch.step()
            stream.synchronize()
            stats["seconds"] += time.perf_counter() - t0
            stats["control_steps"] += n_inst * episode_steps
            stats["rollout_steps"] += n_inst * episode_steps * K * H
            for i, _ in recs:
                batch.record(i, None)
                batch.remove(i)
            # fall cut, features and 6-knot targets in the library's pairs kernel
            oc = torch.tensor([[o[0], o[1], v] for v, o in meta], dtype=torch.float32, device="cuda")
            feat, tgt, count = B.policy_pairs(rec_all, oc, nk, FALL_Z, stream=stream)
            for k, n_ok in enumerate(count.cpu().tolist()):
                if n_ok < episode_steps:
                    stats["falls"] += 1
                if n_ok == 0:
                    continue
                Xs.append(feat[k, :n_ok])
                Ys.append(tgt[k, :n_ok])
                Es.append(torch.full((n_ok,), ep_id, dtype=torch.int32, device="cuda"))
                got += n_ok
                ep_id += 1
                stats["episodes"] += 1
            log(f"  {wl['name']}: {got}/{target} pairs, {stats['episodes']} episodes, {stats['falls']} falls")
        del batch
    X = torch.cat(Xs)[:n_pairs].contiguous()
    Y = torch.cat(Ys)[:n_pairs].contiguous()
    E = torch.cat(Es)[:n_pairs].contiguous()
    return dict(X=X, Y=Y, episode=E, stats=stats)


def split(data, holdout=0.05, seed=0):
    """Training / held-out row indices by episode."""
    import torch
    E = data["episode"].cpu().numpy()
    eps = np.unique(E)
    rng = np.random.default_rng([seed, 78])
    held = set(rng.choice(eps, max(1, int(len(eps) * holdout)), replace=False).tolist())
    mask = np.array([e in held for e in E])
    tr = torch.as_tensor(np.nonzero(~mask)[0].astype(np.int32), device="cuda")
    ho = torch.as_tensor(np.nonzero(mask)[0].astype(np.int32), device="cuda")
    return tr, ho


def normalization(data, rows, floor=1e-3):
    X, Y = data["X"][rows.long()], data["Y"][rows.long()]
    im, isd = X.mean(0), X.std(0).clamp_min(floor)
    om, osd = Y.mean(0), Y.std(0).clamp_min(floor)
    return [t.double().cpu().numpy() for t in (im, isd, om, osd)]


def nll(policy, data, rows, chunk=4096):
    """Held-out Gaussian NLL (mean over rows and outputs): the library's loss over chunks
    of at most max_batch rows, weighted by their row counts."""
    tot, n = 0.0, 0
    chunk = min(chunk, policy.max_batch)
    for a in range(0, rows.numel(), chunk):
        r = rows[a:a + chunk].contiguous()
        tot += float(policy.nll(data["X"], data["Y"], index=r).item()) * r.numel()
        n += r.numel()
    return tot / n


def train(policy, data, rows, epochs=10, batch=4096, lr=1e-3, seed=0, held=None, log=print):
    """Adam on the Gaussian NLL.  Returns per-epoch (train loss, held-out NLL, seconds)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    n = rows.numel()
    for ep in range(epochs):
        perm = rows[torch.randperm(n, generator=g, device="cuda")].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc = torch.zeros(1, dtype=torch.float32, device="cuda")
        steps = 0
        for a in range(0, n - batch + 1, batch):
            policy.train_step(data["X"], data["Y"], index=perm[a:a + batch], B=batch, lr=lr, loss=loss)
            acc += loss
            steps += 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tl = float(acc.item()) / max(steps, 1)
        hl = nll(policy, data, held) if held is not None else float("nan")
        hist.append((tl, hl, dt, steps))
        log(f"  epoch {ep}: train NLL {tl:.4f}  held-out NLL {hl:.4f}  {dt:.2f} s ({steps} steps)")
    return hist


def _stage_cost_torch(x, tau, p):
    """Running cost of the walking task at state x after a plant step with torques tau."""
    z, qx, qy, vx = x[2], x[4], x[5], x[19]
    rzz = 1.0 - 2.0 * (qx * qx + qy * qy)
    return (p["w_h"] * (z - p["h_ref"]) ** 2 + p["w_o"] * (1.0 - rzz * rzz) + p["w_v"] * (vx - p["v_ref"]) ** 2
            + p["w_tau"] * (tau * tau).sum())


def episode(model, p, seed, steps, policy=None, k_prop=0, arith="fp64", gate="cost", lat=None):
    """One closed-loop episode of a walking task (the model's scene, walking cost of p)
    from the seeded stance; returns the
    episode cost sum dt * l, the final state and the proposal counters.  With a list
    `lat`, appends each control step's latency in ms: stream events around the step, so
    the time runs from the moment the plant state is on the device to the first control
    (with a gate: the proposal's rollout, the plain one where it runs, and the gated update)."""
    import torch
    from . import binding as Bd
    ctl = Bd.Controller(model, dict(p, seed=seed, arith=arith))
    x0 = W.initial_state(seed, model.scene)
    x = torch.tensor(x0, dtype=torch.float32, device="cuda")
    xn = torch.empty_like(x)
    tau = torch.empty(12, dtype=torch.float32, device="cuda")
    u0 = torch.empty(12, dtype=torch.float32, device="cuda")
    ctl.set_nominal(torch.tensor(W.stance_knots(p["nk"]), dtype=torch.float32, device="cuda"))
    if policy is not None:
        ctl.set_proposal(policy, k_prop=k_prop, cmd=(p["v_ref"], 0.0, 0.0), origin=(float(x0[0]), float(x0[1])),
                         gate=gate)
    cost = torch.zeros((), dtype=torch.float64, device="cuda")
    ev = []
    for _ in range(steps):
        if lat is not None:
            e0, e1 = DeviceEvent(), DeviceEvent()
            e0.record()
        ctl.step(x, u0)
        if lat is not None:
            e1.record()
            ev.append((e0, e1))
        model.sim_step_into(x.view(1, -1), u0.view(1, -1), p["kp"], p["kd"], p["dt"], xn.view(1, -1),
                            tau_out=tau.view(1, -1), arith=arith)
        cost += p["dt"] * _stage_cost_torch(xn.double(), tau.double(), p)
        x, xn = xn, x
    acc, n = ctl.proposal_stats() if policy is not None else (0, 0)
    if lat is not None:
        torch.cuda.synchronize()
        lat.extend(a.elapsed_time(b) for a, b in ev)
    return float(cost.item()), x.cpu().numpy(), acc, n


def evaluate(policy, K_plain=(64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384), K_learned=1024, ratio=4,
             seeds=range(100, 110),
             steps=200, v_ref=0.5, arith="fp64", log=print):
    """Plain MPPI at each K against the learned proposal with K_learned / ratio samples
    (K_learned on fallback steps) over the same seeds; episode costs, fallback rate and the
    average samples per step."""
    from . import binding as Bd
    wl = W.TERRAIN_WALK
    model = Bd.Model(W.model_dict(wl, 0))
    p = W.params_dict(wl, 0, v_ref=v_ref)
    def pct(v):
        return dict(p50=float(np.percentile(v, 50)), p99=float(np.percentile(v, 99)), mean=float(np.mean(v)))

    def ci95(v):  # normal-approximation interval of the mean over the seeds
        v = np.asarray(v, dtype=np.float64)
        h = 1.96 * v.std(ddof=1) / np.sqrt(v.size) if v.size > 1 else float("nan")
        return [float(v.mean() - h), float(v.mean() + h)]

    out = {"plain": {}, "seeds": list(seeds), "steps": steps, "v_ref": v_ref}
    for K in K_plain:
        lat = []
        costs = [episode(model, dict(p, K=K), s, steps, arith=arith, lat=lat)[0] for s in seeds]
        out["plain"][K] = dict(mean=float(np.mean(costs)), ci95=ci95(costs), costs=costs, samples_per_step=K,
                               latency_ms=pct(lat))
        log(f"  plain K={K}: episode cost {np.mean(costs):.3f}, step latency p50 {np.percentile(lat, 50):.3f} "
            f"p99 {np.percentile(lat, 99):.3f} ms")
    kp = K_learned // ratio
    for gate in ("cost", "best", "best-concurrent", "none"):
        lat = []
        res = [episode(model, dict(p, K=K_learned), s, steps, policy=policy, k_prop=kp, arith=arith, gate=gate,
                       lat=lat) for s in seeds]
        costs = [r[0] for r in res]
        acc = sum(r[2] for r in res)
        n = sum(r[3] for r in res)
        # a gated step on the lane-split rollout rolls out the proposal and, only when the
        # gate falls back, the plain step's K samples; the concurrent gate both on every
        # step (in one launch); the ungated step the proposal only
        if gate == "none":
            samples = float(kp)
        elif gate.endswith("-concurrent"):
            samples = float(kp + K_learned)
        else:
            samples = float(kp + (1.0 - acc / max(n, 1)) * K_learned)
        out["learned_" + gate] = dict(mean=float(np.mean(costs)), ci95=ci95(costs), costs=costs, k_prop=kp,
                                      K_fallback=K_learned,
                                      accepted=acc, steps=n, acceptance=acc / max(n, 1), samples_per_step=samples,
                                      latency_ms=pct(lat))
        # the smallest plain K whose mean episode cost is not above the learned controller's
        match = [K for K in K_plain if out["plain"][K]["mean"] <= np.mean(costs)]
        out["learned_" + gate]["smallest_plain_K_matching"] = min(match) if match else None
        out["learned_" + gate]["sample_ratio"] = (min(match) / samples if match else
                                                  "> %g" % (max(K_plain) / samples))
        log(f"  learned K/{ratio}={kp}, gate {gate}: episode cost {np.mean(costs):.3f}, "
            f"acceptance {acc / max(n, 1):.2f}, {samples:.0f} samples/step, step latency p50 "
            f"{np.percentile(lat, 50):.3f} p99 {np.percentile(lat, 99):.3f} ms")
    return out


def evaluate_batched(policy, n_inst=256, K_plain=(256, 1024), k_prop=256, steps=200, seed0=100, v_ref=0.5,
                     arith="fp64", budget=1 << 30, log=print):
    """Batched serving of n_inst heightfield walks (initial states from seeds seed0, ...)
    in one batch per controller: plain MPPI at each K in K_plain and the learned proposal
    with k_prop samples (ungated, the shifted nominal kept as sample 1).  The batch's
    tuning is chosen by the autotuner on a separate batch of the same instances, so the
    evaluated closed loops start from their initial states.  Per controller: the mean
    episode cost (the batch's running cost, sum of dt * l), the fraction of instances
    whose base ended below the fall height, the latency of each whole batch step (stream
    events around it, including the proposal's features, network pass and head), and
    rollout-steps/s over the steps."""
    import torch
    from . import binding as Bd
    wl = W.TERRAIN_WALK
    model = Bd.Model(W.model_dict(wl, 0))
    nk, H = wl["nk"], wl["H"]

    def make(K, learned):
        batch = Bd.Batch(max_instances=n_inst, budget_bytes=budget, max_horizon=H, max_hf_cells=W.HF_N * W.HF_N,
                         arith=arith)
        slot = batch.add_model(model)
        ids = []
        for k in range(n_inst):
            s = seed0 + k
            p = dict(W.params_dict(wl, s, v_ref=v_ref, instance=k, arith=arith), K=K)
            x0 = W.initial_state(s, W.SCENE_HEIGHTFIELD)
            i = batch.admit(slot, p, x0, W.stance_knots(nk))
            if i is None:
                raise RuntimeError("the batch does not fit in the evaluation budget")
            if learned:
                batch.set_proposal(i, policy, cmd=(v_ref, 0.0, 0.0), origin=(float(x0[0]), float(x0[1])))
            ids.append(i)
        return batch, ids

    out = {"task": "heightfield walk, v_ref %.2f, closed loop" % v_ref, "instances": n_inst, "steps": steps,
           "seeds": [seed0, seed0 + n_inst - 1], "controllers": {}}
    runs = [("plain_K%d" % K, K, False) for K in K_plain] + [("learned_K%d" % k_prop, k_prop, True)]
    for name, K, learned in runs:
        tb, _ = make(K, learned)
        tb.autotune(steps=3)
        bpc, order, mode = tb.tuning()
        del tb
        batch, ids = make(K, learned)
        batch.set_tuning(bpc, order)
        batch.set_launch_mode(mode)
        ev = []
        t0 = time.perf_counter()
        for _ in range(steps):
            e0, e1 = DeviceEvent(), DeviceEvent()
            e0.record()
            batch.step()
            e1.record()
            ev.append((e0, e1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        reads = [batch.read(i, 37, nk) for i in ids]
        costs = np.array([r[3] for r in reads], dtype=np.float64)
        falls = int(sum(1 for r in reads if not (r[0][2] > FALL_Z)))
        out["controllers"][name] = dict(
            samples_per_step=K, proposal=learned, episode_cost=float(np.mean(costs)),
            episode_cost_median=float(np.median(costs)), falls=falls,
            latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                            mean=float(lat.mean())),
            rollout_steps_per_s=n_inst * K * H * steps / wall,
            tuning=dict(blocks_per_cu=bpc, order=order, launch_mode=mode))
        log(f"  batched {name}: episode cost {np.mean(costs):.3f}, falls {falls}/{n_inst}, step latency p50 "
            f"{np.percentile(lat, 50):.3f} p99 {np.percentile(lat, 99):.3f} ms")
        del batch
    return out

