"""Closed-loop ablations of the plain method on the synthetic tasks (the paper's Sec. IV
studies): the knot interpolation (sampling representation), and sweeps of the
temperature lambda, the horizon H, the number of samples K and the control rate.

Every setting runs the same seeded episodes (initial states and Philox keys) through the
GPU controller and the GPU plant; the score is the episode cost sum dt * l of the task's
running cost, averaged over the seeds with a normal-approximation 95% interval.
"""
from __future__ import annotations

import numpy as np

from . import binding as B
from . import workloads as W
from .proposal import FALL_Z, _stage_cost_torch, episode

BASES = {"cubic": 0, "linear": 1, "zeroth_order": 2, "direct": 3}


def _summary(costs, falls):
    v = np.asarray(costs, dtype=np.float64)
    h = 1.96 * v.std(ddof=1) / np.sqrt(v.size) if v.size > 1 else float("nan")
    return dict(mean=float(v.mean()), ci95=[float(v.mean() - h), float(v.mean() + h)], falls=int(falls),
                costs=[float(c) for c in v])


def sampling_ablation(seeds=range(10), steps=200, arith="fp64", log=print):
    """Episode cost with each sampling representation on three tasks: the heightfield walk
    with 6 and with 4 knots per joint, and the climb onto the 0.3 m box with the base
    height target raised by the box height.  Same seeds, samples and horizon for every
    representation; direct sampling draws one value per control step (H per joint) with
    the same sigma."""
    tasks = [
        ("heightfield_walk_6_knots", W.TERRAIN_WALK, {}),
        ("heightfield_walk_4_knots", W.TERRAIN_WALK, {"nk": 4}),
        ("box_climb_6_knots", W.BOX_CLIMB, {"h_ref": W.WALK_COST["h_ref"] + 2 * W.CLIMB_BOX_HALF[2]}),
    ]
    out = {}
    for name, wl, over in tasks:
        model = B.Model(W.model_dict(wl, 0))
        res = {}
        for bname, basis in BASES.items():
            costs, falls = [], 0
            for sd in seeds:
                p = dict(W.params_dict(wl, sd, **over), basis=basis)
                if basis == 3:  # direct: one value per control step (lane-split rollout)
                    p.update(nk=p["H"], lanes=16)
                c, xf, _, _ = episode(model, p, sd, steps, arith=arith)
                costs.append(c)
                falls += int(not (xf[2] > FALL_Z))
            res[bname] = _summary(costs, falls)
            log(f"  {name} {bname}: episode cost {res[bname]['mean']:.3f}, falls {falls}/{len(costs)}")
        order = sorted(res, key=lambda b: res[b]["mean"])
        out[name] = dict(K=wl["K"], H=wl["H"], nk=over.get("nk", wl["nk"]), bases=res, ranking=order)
    return out


def episode_held(model, p, seed, steps, hold, arith="fp64", trace=None):
    """A closed-loop episode in which the controller replans every `hold` plant steps.
    Between replans the plant follows the last plan: each step applies the first knot of
    the plan and advances it by the warm-start shift (the interpolant one step later); the
    advanced plan is the nominal of the next replan.  With a list `trace`, appends per
    plant step (t, replanned, state, nominal before the step, applied control) as host
    arrays."""
    import torch
    ctl = B.Controller(model, dict(p, seed=seed, arith=arith))
    S = torch.as_tensor(ctl.basis_matrices()[1], device="cuda")
    nk = p["nk"]
    x = torch.tensor(W.initial_state(seed, model.scene), dtype=torch.float32, device="cuda")
    xn = torch.empty_like(x)
    tau = torch.empty(12, dtype=torch.float32, device="cuda")
    u0 = torch.empty(12, dtype=torch.float32, device="cuda")
    ctl.set_nominal(torch.tensor(W.stance_knots(nk), dtype=torch.float32, device="cuda"))
    cost = torch.zeros((), dtype=torch.float64, device="cuda")
    plan = None
    for t in range(steps):
        replan = t % hold == 0
        if trace is not None:
            before = (ctl.get_nominal() if plan is None else plan.reshape(-1)).cpu().numpy().copy()
            xs = x.cpu().numpy().copy()
        if replan:
            if plan is not None:
                ctl.set_nominal(plan.reshape(-1).contiguous())
            ctl.step(x, u0)
            plan = ctl.get_nominal().view(12, nk)  # already advanced by one step
        else:
            u0.copy_(plan[:, 0])
            plan = plan @ S.T
        if trace is not None:
            trace.append((t, replan, xs, before, u0.cpu().numpy().copy()))
        model.sim_step_into(x.view(1, -1), u0.view(1, -1), p["kp"], p["kd"], p["dt"], xn.view(1, -1),
                            tau_out=tau.view(1, -1), arith=arith)
        cost += p["dt"] * _stage_cost_torch(xn.double(), tau.double(), p)
        x, xn = xn, x
    return float(cost.item()), x.cpu().numpy()


RATE_FINE = dict(dt=0.004, H=125, holds=[1, 2, 3, 4, 5, 10, 20, 25], seconds=2.0)


def control_rate_sweep(seeds=range(10), arith="fp64", fine=RATE_FINE, log=print):
    """The control rate up to 250 Hz (Sec. IV-E sweeps 10-250 Hz): the heightfield walk with
    plant and controller at dt = 4 ms (horizon 125 steps = 0.5 s, as the 50 x 10 ms
    default), replanning every `hold` plant steps -- 250, 125, 83.3, 62.5, 50, 25, 12.5 and
    10 Hz -- over episodes of the same 2 s as the default sweeps."""
    wl = W.TERRAIN_WALK
    model = B.Model(W.model_dict(wl, 0))
    steps = int(round(fine["seconds"] / fine["dt"]))
    res = {}
    for hold in fine["holds"]:
        rate = 1.0 / (fine["dt"] * hold)
        costs, falls = [], 0
        for sd in seeds:
            p = dict(W.params_dict(wl, sd), dt=fine["dt"], H=fine["H"])
            c, xf = episode_held(model, p, sd, steps, hold, arith=arith)
            costs.append(c)
            falls += int(not (xf[2] > FALL_Z))
        res["%.4g" % rate] = dict(_summary(costs, falls), hold=hold)
        log(f"  rate {rate:.4g} Hz (dt 4 ms, hold {hold}): episode cost {res['%.4g' % rate]['mean']:.3f}, "
            f"falls {falls}/{len(costs)}")
    best = min(res, key=lambda k: res[k]["mean"])
    return dict(values=res, best=best, dt=fine["dt"], H=fine["H"], episode_seconds=fine["seconds"])


SWEEPS = {
    "lam": [0.005, 0.01, 0.02, 0.05, 0.1, 0.2, 0.3],
    "H": [5, 10, 20, 30, 40, 50, 75, 100],
    "K": [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096],
    "rate_hz": [100, 50, 25, 12.5, 10],
}


def hyperparameter_sweeps(seeds=range(10), steps=200, arith="fp64", sweeps=None, log=print):
    """One-at-a-time sweeps around the heightfield walk (K 1024, H 50, dt 0.01, 6 knots,
    lambda 0.05): the temperature, the horizon in steps (knots stay evenly spread over it),
    the samples, and the control rate (replanning every 100 / rate plant steps)."""
    wl = W.TERRAIN_WALK
    model = B.Model(W.model_dict(wl, 0))
    out = {}
    for axis, values in (sweeps or SWEEPS).items():
        res = {}
        for v in values:
            costs, falls = [], 0
            for sd in seeds:
                p = W.params_dict(wl, sd)
                if axis == "rate_hz":
                    hold = int(round(1.0 / (p["dt"] * v)))
                    c, xf = episode_held(model, p, sd, steps, hold, arith=arith)
                else:
                    p[axis] = type(p[axis])(v)
                    c, xf, _, _ = episode(model, p, sd, steps, arith=arith)
                costs.append(c)
                falls += int(not (xf[2] > FALL_Z))
            res[str(v)] = _summary(costs, falls)
            log(f"  {axis} = {v}: episode cost {res[str(v)]['mean']:.3f}, falls {falls}/{len(costs)}")
        best = min(res, key=lambda k: res[k]["mean"])
        out[axis] = dict(values=res, best=best)
    return out


# ---- Eq. 3 / Eq. 4 tracking cost (Sec. IV-B, IV-D) --------------------------------
def _walk_metrics(xs, v_cmd, dt):
    """Task-level scores of a walking episode from its plant states (steps x nx): whether it
    fell (base below the fall height at any step), the mean forward velocity over the second
    half, its error from the command, the lateral drift and the mean height and tilt."""
    z = xs[:, 2]
    half = xs[xs.shape[0] // 2:]
    vx = float(half[:, 19].mean())
    tilt = np.degrees(np.arccos(np.clip(1 - 2 * (xs[:, 4] ** 2 + xs[:, 5] ** 2), -1, 1)))
    return dict(fell=bool((z < FALL_Z).any()), vx=vx, v_err=abs(vx - v_cmd[0]), y_drift=float(abs(xs[-1, 1] - xs[0, 1])),
                distance=float(xs[-1, 0] - xs[0, 0]), z_mean=float(z.mean()), tilt_mean_deg=float(tilt.mean()))


def episode_tracking(model, p, track, seed, steps, arith="fp64", push_goal=None):
    """A closed-loop episode whose controller uses the Eq. 3 / Eq. 4 cost (track: the
    tracking-cost dict; its p_ref0 is moved to the episode's start).  The controller's step
    counter is the gait clock.  With push_goal (box scene), every control step re-aims the
    robot's position reference at the box centre and its commanded velocity along the
    box-to-goal direction (the paper places the robot's goal at the box centre).  Returns
    the plant states (steps x nx, host)."""
    import torch
    ctl = B.Controller(model, dict(p, seed=seed, arith=arith, cost="tracking"))
    x0 = W.initial_state(seed, model.scene)
    c = dict(track, p_ref0=(float(x0[0]), float(x0[1]), track["p_ref0"][2]))
    ctl.set_tracking_cost(c)
    x = torch.tensor(x0, dtype=torch.float32, device="cuda")
    xn = torch.empty_like(x)
    u0 = torch.empty(12, dtype=torch.float32, device="cuda")
    ctl.set_nominal(torch.tensor(W.stance_knots(p["nk"]), dtype=torch.float32, device="cuda"))
    xs = torch.empty((steps, x.numel()), dtype=torch.float32, device="cuda")
    for t in range(steps):
        if push_goal is not None:
            bxy = x[W.NX:W.NX + 2].cpu().numpy().astype(np.float64)
            d = np.asarray(push_goal) - bxy
            v = track["push_speed"] * d / max(np.linalg.norm(d), 1e-6)
            tnow = t * p["dt"]
            c = dict(c, v_cmd=(float(v[0]), float(v[1])),
                     p_ref0=(float(bxy[0] - v[0] * tnow), float(bxy[1] - v[1] * tnow), track["p_ref0"][2]))
            ctl.set_tracking_cost(c)
        ctl.step(x, u0)
        model.sim_step_into(x.view(1, -1), u0.view(1, -1), p["kp"], p["kd"], p["dt"], xn.view(1, -1), arith=arith)
        xs[t].copy_(xn)
        x, xn = xn, x
    return xs.cpu().numpy().astype(np.float64)


def episode_running(model, p, seed, steps, arith="fp64"):
    """The same closed loop with the running cost (the plain default), plant states back."""
    import torch
    ctl = B.Controller(model, dict(p, seed=seed, arith=arith))
    x = torch.tensor(W.initial_state(seed, model.scene), dtype=torch.float32, device="cuda")
    xn = torch.empty_like(x)
    u0 = torch.empty(12, dtype=torch.float32, device="cuda")
    ctl.set_nominal(torch.tensor(W.stance_knots(p["nk"]), dtype=torch.float32, device="cuda"))
    xs = torch.empty((steps, x.numel()), dtype=torch.float32, device="cuda")
    for t in range(steps):
        ctl.step(x, u0)
        model.sim_step_into(x.view(1, -1), u0.view(1, -1), p["kp"], p["kd"], p["dt"], xn.view(1, -1), arith=arith)
        xs[t].copy_(xn)
        x, xn = xn, x
    return xs.cpu().numpy().astype(np.float64)


def _agg(rows):
    keys = [k for k in rows[0] if k != "fell"]
    out = {k: float(np.mean([r[k] for r in rows])) for k in keys}
    out["falls"] = int(sum(r["fell"] for r in rows))
    out["episodes"] = len(rows)
    return out


def tracking_ablation(seeds=range(10), steps=300, arith="fp64", v_cmd=(0.5, 0.0), track_over=None, log=print):
    """Walking with three costs on flat ground and on the heightfield (controller of the
    heightfield walk: K 1024, H 50, dt 0.01, 6 knots): the running cost, Eq. 3 with a
    time-invariant standing joint reference, and Eq. 3 with the Raibert trotting reference.
    Scores are task-level (falls, forward velocity and its error, drift, height, tilt), the
    same for every cost."""
    out = {}
    for scene_name, wl, scene in (("flat", W.TERRAIN_WALK, W.SCENE_FLAT), ("heightfield", W.TERRAIN_WALK,
                                                                           W.SCENE_HEIGHTFIELD)):
        md = W.model_dict(wl, 0) if scene == W.SCENE_HEIGHTFIELD else W.model_dict(W.FLAT_WALK, 0)
        model = B.Model(md)
        res = {}
        for name in ("running", "eq3_stand", "eq3_trot"):
            rows = []
            for sd in seeds:
                p = W.params_dict(wl, sd, v_ref=v_cmd[0])
                if name == "running":
                    xs = episode_running(model, p, sd, steps, arith=arith)
                else:
                    c = W.tracking_cost(gait=1 if name == "eq3_trot" else 0, v_cmd=v_cmd, **(track_over or {}))
                    xs = episode_tracking(model, p, c, sd, steps, arith=arith)
                rows.append(_walk_metrics(xs, v_cmd, p["dt"]))
            res[name] = _agg(rows)
            r = res[name]
            log(f"  {scene_name} {name}: falls {r['falls']}/{r['episodes']}, vx {r['vx']:.3f} (err {r['v_err']:.3f}), "
                f"drift {r['y_drift']:.3f}, z {r['z_mean']:.3f}, tilt {r['tilt_mean_deg']:.1f} deg")
        out[scene_name] = res
    return out


PUSH_TRACK = dict(box_w=10.0)  # with the base-position weight raised to 10 in xy (push_ablation)


def push_ablation(seeds=range(10), steps=400, arith="fp64", push_speed=0.3, track_over=None, log=print):
    """Box push (controller of the box-push workload: K 4096, H 60, 8 knots): the running
    cost with squared distances against Eq. 3 + Eq. 4 (trot reference aimed at the box,
    l1 box-to-goal term with weight 10, base-position weight 10 in xy).  Scores: the box's
    final distance to its goal, the closest it came, and success as the box coming within
    0.3 m of the goal (the paper's criterion)."""
    wl = W.BOX_PUSH
    if track_over is None:
        q = list(W.tracking_cost()["Q"])
        q[0] = q[1] = 10.0
        track_over = dict(PUSH_TRACK, Q=q)
    res = {}
    for name in ("running_squared", "eq3_eq4_l1"):
        rows = []
        for sd in seeds:
            model = B.Model(W.model_dict(wl, sd))
            p = W.params_dict(wl, sd)
            goal = np.asarray(p["goal"])
            if name == "running_squared":
                xs = episode_running(model, p, sd, steps, arith=arith)
            else:
                c = dict(W.tracking_cost(gait=1, box_goal_xy=tuple(goal), **(track_over or {})), push_speed=push_speed)
                xs = episode_tracking(model, p, c, sd, steps, arith=arith, push_goal=goal)
            d = np.linalg.norm(xs[:, W.NX:W.NX + 2] - goal[None], axis=1)
            rows.append(dict(final_distance=float(d[-1]), closest=float(d.min()), success=bool(d.min() <= 0.3),
                             fell=bool((xs[:, 2] < FALL_Z).any())))
        r = dict(final_distance=float(np.mean([x["final_distance"] for x in rows])),
                 closest=float(np.mean([x["closest"] for x in rows])), successes=int(sum(x["success"] for x in rows)),
                 falls=int(sum(x["fell"] for x in rows)), episodes=len(rows))
        res[name] = r
        log(f"  push {name}: success {r['successes']}/{r['episodes']}, final distance {r['final_distance']:.3f}, "
            f"closest {r['closest']:.3f}, falls {r['falls']}")
    return res
