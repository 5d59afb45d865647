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

BASES = {"cubic": 0, "linear": 1, "zeroth_order": 2}


def _summary(costs, falls):
    v = np.asarray(costs, dtype=np.float64)
    h = 1.96 * v.std(ddof=1) / np.sqrt(v.size) if v.size > 1 else float("nan")
    return dict(mean=float(v.mean()), ci95=[float(v.mean() - h), float(v.mean() + h)], falls=int(falls),
                costs=[float(c) for c in v])


def sampling_ablation(seeds=range(10), steps=200, arith="fp64", log=print):
    """Episode cost with each knot interpolation on three tasks: the heightfield walk with
    6 and with 4 knots per joint, and the climb onto the 0.3 m box with the base height
    target raised by the box height.  Same seeds, samples and horizon for every basis."""
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
                c, xf, _, _ = episode(model, p, sd, steps, arith=arith)
                costs.append(c)
                falls += int(not (xf[2] > FALL_Z))
            res[bname] = _summary(costs, falls)
            log(f"  {name} {bname}: episode cost {res[bname]['mean']:.3f}, falls {falls}/{len(costs)}")
        order = sorted(res, key=lambda b: res[b]["mean"])
        out[name] = dict(K=wl["K"], H=wl["H"], nk=over.get("nk", wl["nk"]), bases=res, ranking=order)
    return out


def episode_held(model, p, seed, steps, hold, arith="fp64"):
    """A closed-loop episode in which the controller replans every `hold` plant steps.
    Between replans the plant follows the last plan: each step applies the first knot of
    the plan and advances it by the warm-start shift (the interpolant one step later); the
    advanced plan is the nominal of the next replan."""
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
        if t % hold == 0:
            if plan is not None:
                ctl.set_nominal(plan.reshape(-1).contiguous())
            ctl.step(x, u0)
            plan = ctl.get_nominal().view(12, nk)  # already advanced by one step
        else:
            u0.copy_(plan[:, 0])
            plan = plan @ S.T
        model.sim_step_into(x.view(1, -1), u0.view(1, -1), p["kp"], p["kd"], p["dt"], xn.view(1, -1),
                            tau_out=tau.view(1, -1), arith=arith)
        cost += p["dt"] * _stage_cost_torch(xn.double(), tau.double(), p)
        x, xn = xn, x
    return float(cost.item()), x.cpu().numpy()


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
