"""Shared helpers for GPU-vs-oracle parity tests."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W

# state blocks compared separately (robot): p, quat, q_joint, v_world, omega_body, qd_joint
BLOCKS = [(0, 3), (3, 7), (7, 19), (19, 22), (22, 25), (25, 37)]
BOX_BLOCKS = [(37, 40), (40, 44), (44, 47), (47, 50)]

STEP_TOL = 1e-5      # per-step state error, relative per block (FP64 step)
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


U32 = 2.0 ** -24


def fp32_step_bound(orc, x, u, kp, kd, dt):
    """Per-state bound on the FP32 step's error, derived before any GPU result: the step
    solves (M + dt D) dv = dt f for the robot (18x18) and the free box (6x6).  An FP32
    Cholesky-type solve is backward stable, so the computed dv satisfies a system whose
    matrix and right side are perturbed by about (n + 1) u of their magnitude (u = 2^-24;
    the assembly in FP32 adds as many roundings again), which moves dv by at most
    kappa_2(A) * 2 (n + 1) u |dv| (kappa_2 from the oracle's FP64 system).  Every block is
    compared relative to max(|block|, 1) >= 1, the velocities are v + dv and the positions
    take dt (< 1) times the velocity error, so that is a bound on the block errors.
    Returns the larger of it and the FP64 step's 1e-5."""
    A, r, _ = orc.step_system(x, u, kp, kd, dt)
    ev = np.linalg.eigvalsh(A)
    bound = 2 * 19 * (ev[-1] / ev[0]) * U32 * np.abs(np.linalg.solve(A, r)).max()
    if len(x) == W.NX_BOX:
        Ab, rb, _ = orc.step_system_box(x, u, kp, kd, dt)
        evb = np.linalg.eigvalsh(Ab)
        bound = max(bound, 2 * 7 * (evb[-1] / evb[0]) * U32 * np.abs(np.linalg.solve(Ab, rb)).max())
    return max(STEP_TOL, bound)


ULP_FACTOR = 8   # FP32 roundings between the state and a contact depth or joint frame


def ulp_sensitivity(orc, x, u, kp, kd, dt):
    """The oracle's own one-ulp sensitivity of the step, block-relative like step_error:
    sum over the inputs (state and joint targets) of |x+(in + ulp) - x+(in - ulp)| / 2,
    each input moved by one FP32 ulp, central differences in FP64."""
    x = np.asarray(x, np.float64)
    u = np.asarray(u, np.float64)
    base, _, _ = orc.step(x, u, kp, kd, dt)
    acc = np.zeros_like(base)
    for vec, is_x in ((x, True), (u, False)):
        for i in range(len(vec)):
            h = float(np.spacing(np.float32(vec[i]))) if vec[i] != 0 else float(np.spacing(np.float32(1e-30)))
            a, b = vec.copy(), vec.copy()
            a[i] += h
            b[i] -= h
            xa = orc.step(a, u, kp, kd, dt)[0] if is_x else orc.step(x, a, kp, kd, dt)[0]
            xb = orc.step(b, u, kp, kd, dt)[0] if is_x else orc.step(x, b, kp, kd, dt)[0]
            acc += np.abs(xa - xb) / 2
    blocks = BLOCKS + (BOX_BLOCKS if len(x) == W.NX_BOX else [])
    return max(acc[a:b].max() / max(np.abs(base[a:b]).max(), 1.0) for a, b in blocks)


def mixed_step_bound(orc, x, u, kp, kd, dt):
    """Per-state bound of the step with FP32 kinematics and contact geometry and the FP64
    implicit system, derived before any GPU result: the FP32 part rounds each contact
    depth, lever arm and joint frame a few times (quaternion to rotation, rotation times
    offset, translation, one trigonometric call), which acts as a perturbation of the
    inputs by at most ULP_FACTOR ulps; the FP64 system adds nothing at this scale.  So
    ULP_FACTOR times the oracle's one-ulp sensitivity, or the FP64 step's 1e-5 if larger."""
    return max(STEP_TOL, ULP_FACTOR * ulp_sensitivity(orc, x, u, kp, kd, dt))


def r16_knot_sensitivity(p, step, mu, costs):
    """First-order change of the updated knots when every cost moves by the cost
    tolerance: sum_n (w_n / lambda) |L_n| COST_TOL |theta_n - mu'|, max over knots."""
    w, _ = O.weights(costs, p["lam"])
    theta = mu + p["sigma"] * O.sample_eps(p, step)
    theta[0] = mu
    mup = w @ theta
    ok = np.isfinite(costs)
    return float((w[ok, None] * np.abs(costs[ok, None]) * np.abs(theta[ok] - mup)).sum(0).max() / p["lam"] * COST_TOL)
