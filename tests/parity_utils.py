"""Shared helpers for GPU-vs-oracle parity tests."""
from __future__ import annotations

import numpy as np

from paper_2409_10469_amd import workloads as W

# state blocks compared separately (robot): p, quat, q_joint, v_world, omega_body, qd_joint
BLOCKS = [(0, 3), (3, 7), (7, 19), (19, 22), (22, 25), (25, 37)]
BOX_BLOCKS = [(37, 40), (40, 44), (44, 47), (47, 50)]

STEP_TOL = 1e-5      # per-step state error, relative per block
COST_TOL = 1e-4      # rollout cost over <= 10 steps, relative
KNOT_TOL = 1e-3      # updated knots, absolute [rad]


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def round_model(d: dict) -> dict:
    """Both sides consume the same FP32-representable model."""
    out = {}
    for k, v in d.items():
        if k == "hf":
            out[k] = f32(v)
        elif isinstance(v, (float, np.floating)):
            out[k] = float(np.float32(v))
        elif isinstance(v, (tuple, list)) and v and isinstance(v[0], (float, np.floating, int)):
            out[k] = tuple(float(np.float32(x)) for x in v)
        else:
            out[k] = v
    return out


def round_params(p: dict) -> dict:
    out = dict(p)
    for k in ("dt", "sigma", "lam", "kp", "kd", "w_h", "h_ref", "w_o", "w_v", "v_ref", "w_tau", "w_reach", "w_box"):
        out[k] = float(np.float32(p[k]))
    out["goal"] = tuple(float(np.float32(g)) for g in p.get("goal", (0.0, 0.0)))
    return out


def step_error(x_gpu, x_ora, box=False):
    """max over blocks of |dx|_inf / max(|x_ora|_inf, 1), one value per row."""
    x_gpu, x_ora = np.atleast_2d(x_gpu), np.atleast_2d(x_ora)
    errs = []
    for a, b in BLOCKS + (BOX_BLOCKS if box else []):
        d = np.abs(x_gpu[:, a:b] - x_ora[:, a:b]).max(1)
        s = np.maximum(np.abs(x_ora[:, a:b]).max(1), 1.0)
        errs.append(d / s)
    return np.max(np.stack(errs, 1), 1)


def random_walk_states(orc, seeds, steps, dt, kp=40.0, kd=1.0, scale=0.3, scene=W.SCENE_FLAT):
    """States along oracle trajectories driven by random joint targets around the stance."""
    states, targets = [], []
    for s in seeds:
        rng = np.random.default_rng(1000 + s)
        x = f32(W.initial_state(s, scene))
        base = np.tile(W.STANCE_JOINTS, 4)
        u = base + rng.uniform(-scale, scale, 12)
        for k in range(steps):
            if k % 5 == 0:
                u = base + rng.uniform(-scale, scale, 12)
            uu = f32(u)
            states.append(x.copy())
            targets.append(uu.copy())
            xn, _, rc = orc.step(x, uu, kp, kd, dt)
            if rc or not np.isfinite(xn).all():
                break
            x = f32(xn)
    return np.array(states), np.array(targets)


def box_contact_states(n, seed=0):
    """Robot at stance with random velocities and a free box pressed against its front:
    trunk corners inside the box, feet against its faces, box corners into the trunk."""
    rng = np.random.default_rng(seed)
    xs = []
    for i in range(n):
        x = W.initial_state(seed * 1000 + i, W.SCENE_FREE_BOX)
        x[19:37] = rng.normal(size=18) * np.r_[0.3, 0.3, 0.2, 1, 1, 1, np.full(12, 2.0)]
        yaw = rng.uniform(-0.9, 0.9)
        x[37:40] = (rng.uniform(0.33, 0.42), rng.uniform(-0.12, 0.12), W.FREE_BOX_HALF[2] + rng.uniform(-0.004, 0.02))
        x[40:44] = (np.cos(yaw / 2), 0.0, 0.0, np.sin(yaw / 2))
        x[44:50] = rng.normal(size=6) * np.r_[0.3, 0.3, 0.1, 0.5, 0.5, 0.5]
        xs.append(f32(x))
    return np.array(xs)
