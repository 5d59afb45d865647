"""Seeded synthetic workloads for whole-body MPPI on a quadruped.

This module only *describes* inputs: the robot and scene constants, the MPPI
hyperparameters of each workload, and seeded generators for the data both the GPU
library and the CPU oracle consume (initial states, the heightfield array, the box
placement, explicit noise for parity runs).  It holds none of the method's
arithmetic: no dynamics, no sampling transform, no cost, no update.

The paper's robot model, terrains and per-task hyperparameters are not published in
the text (the model is a Unitree Go1 in MuJoCo, Sec. IV-A); these synthetic stand-ins
have the same structure: an 18-DoF floating-base quadruped with three revolute joints
per leg, flat or uneven terrain, a box to climb or push, horizons of a few tenths of a
second at dt = 0.01-0.02 s, and tens to thousands of samples.
"""
from __future__ import annotations

import math

import numpy as np

NX = 37          # robot state: p(3) quat(4) q(12) v_w(3) w_b(3) qd(12)
NX_BOX = 50      # plus free box: p(3) quat(4) v_w(3) w_b(3)
NQ = 19
NU = 12

SCENE_FLAT, SCENE_HEIGHTFIELD, SCENE_STATIC_BOX, SCENE_FREE_BOX = 0, 1, 2, 3

# Synthetic quadruped: trunk box, hips at (+-hip_x, +-hip_y, 0), abduction (x), flexion
# (y), knee (y); thigh and calf uniform rods; massless hip links and foot spheres.
ROBOT = dict(
    trunk_size=(0.38, 0.094, 0.114), trunk_mass=5.2,
    hip_x=0.188, hip_y=0.047,
    thigh_len=0.213, thigh_mass=1.0,
    calf_len=0.213, calf_mass=0.2,
    foot_r=0.02, gravity=9.81,
    k=2.0e4, c=5.0e2, mu=0.8, vs=0.01,
)

STANCE_JOINTS = (0.0, 0.9, -1.8)   # per leg (abduction, flexion, knee) [rad]

# Cost weights shared by the walking tasks: height, uprightness, forward velocity, torque.
WALK_COST = dict(w_h=100.0, h_ref=0.27, w_o=10.0, w_v=1.0, v_ref=0.5, w_tau=1.0e-3,
                 w_reach=0.0, w_box=0.0, goal=(0.0, 0.0))
PUSH_COST = dict(w_h=100.0, h_ref=0.27, w_o=10.0, w_v=0.0, v_ref=0.0, w_tau=1.0e-3,
                 w_reach=1.0, w_box=2.0, goal=(0.0, 0.0))

FLAT_WALK = dict(name="flat_walk", scene=SCENE_FLAT, K=64, H=25, dt=0.02, nk=4, sigma=0.3, lam=0.1,
                 kp=40.0, kd=1.0, cost=WALK_COST, updates=1)
TERRAIN_WALK = dict(name="heightfield_walk", scene=SCENE_HEIGHTFIELD, K=1024, H=50, dt=0.01, nk=6, sigma=0.25,
                    lam=0.05, kp=40.0, kd=1.0, cost=WALK_COST, updates=200)
BOX_PUSH = dict(name="box_push", scene=SCENE_FREE_BOX, K=4096, H=60, dt=0.01, nk=8, sigma=0.25, lam=0.05,
                kp=40.0, kd=1.0, cost=PUSH_COST, updates=1)
BOX_CLIMB = dict(name="box_climb", scene=SCENE_STATIC_BOX, K=1024, H=50, dt=0.01, nk=6, sigma=0.25, lam=0.05,
                 kp=40.0, kd=1.0, cost=WALK_COST, updates=1)

WORKLOADS = {w["name"]: w for w in (FLAT_WALK, TERRAIN_WALK, BOX_PUSH, BOX_CLIMB)}

HF_N = 64
HF_CELL = 0.05
HF_AMPLITUDE = 0.02
FREE_BOX_HALF = (0.2, 0.2, 0.15)
FREE_BOX_MASS = 2.0
CLIMB_BOX_HALF = (0.5, 0.5, 0.15)   # 1.0 x 1.0 x 0.3 m
CLIMB_BOX_AHEAD = 0.6


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def stance_height(robot=ROBOT) -> float:
    """Base height at which the four feet of the stance pose carry the weight."""
    leg_drop = (robot["thigh_len"] + robot["calf_len"]) * math.cos(STANCE_JOINTS[1])
    total = robot["trunk_mass"] + 4 * (robot["thigh_mass"] + robot["calf_mass"])
    return leg_drop + robot["foot_r"] - total * robot["gravity"] / (4 * robot["k"])


def initial_state(seed: int, scene: int = SCENE_FLAT, jitter: float = 0.05, origin=(0.0, 0.0)) -> np.ndarray:
    """Stance at rest with seeded uniform joint offsets in [-jitter, jitter]."""
    nx = NX_BOX if scene == SCENE_FREE_BOX else NX
    x = np.zeros(nx)
    x[0], x[1] = origin
    x[2] = stance_height()
    x[3] = 1.0
    x[7:19] = np.tile(STANCE_JOINTS, 4) + _rng(seed, 1).uniform(-jitter, jitter, 12)
    if scene == SCENE_FREE_BOX:
        x[NX + 0] = 1.0
        x[NX + 2] = FREE_BOX_HALF[2] - FREE_BOX_MASS * ROBOT["gravity"] / (4 * ROBOT["k"])
        x[NX + 3] = 1.0
    return x


def box_goal(seed: int, box_xy=(1.0, 0.0), distance: float = 1.5) -> tuple:
    """Box goal 1.5 m from the box at a seeded angle in [-pi/2, pi/2] around +x."""
    ang = _rng(seed, 3).uniform(-math.pi / 2, math.pi / 2)
    return (box_xy[0] + distance * math.cos(ang), box_xy[1] + distance * math.sin(ang))


def heightfield(seed: int, n: int = HF_N, cell: float = HF_CELL, amplitude: float = HF_AMPLITUDE,
                centre=(0.0, 0.0)):
    """Sum of 8 seeded plane waves on an n x n grid (row = y), scaled so max|h| = amplitude.

    Returns (heights[n, n] float64, x0, y0) with the grid centred on `centre`.
    """
    r = _rng(seed, 2)
    lam = r.uniform(0.2, 1.6, 8)
    direction = r.uniform(0, 2 * math.pi, 8)
    phase = r.uniform(0, 2 * math.pi, 8)
    x0 = centre[0] - 0.5 * (n - 1) * cell
    y0 = centre[1] - 0.5 * (n - 1) * cell
    xs = x0 + cell * np.arange(n)
    ys = y0 + cell * np.arange(n)
    X, Y = np.meshgrid(xs, ys)          # X[iy, ix]
    h = np.zeros((n, n))
    for i in range(8):
        kx = 2 * math.pi / lam[i] * math.cos(direction[i])
        ky = 2 * math.pi / lam[i] * math.sin(direction[i])
        h += np.sin(kx * X + ky * Y + phase[i])
    h *= amplitude / np.abs(h).max()
    return h, x0, y0


def stance_knots(nk: int) -> np.ndarray:
    """Nominal plan holding the stance: 12 joints x nk knots (joint-major)."""
    return np.repeat(np.tile(STANCE_JOINTS, 4)[:, None], nk, axis=1).reshape(-1)


def explicit_noise(seed: int, K: int, nk: int) -> np.ndarray:
    """Standard-normal noise K x 12nk for runs that pass noise in explicitly."""
    return _rng(seed, 4).standard_normal((K, 12 * nk))


def scene_extras(workload: dict, seed: int) -> dict:
    """Scene data for a workload: heightfield, static box or free box and goal."""
    sc = workload["scene"]
    out = dict(scene=sc)
    if sc == SCENE_HEIGHTFIELD:
        h, x0, y0 = heightfield(seed)
        out.update(hf=h, hf_x0=x0, hf_y0=y0, hf_cell=HF_CELL)
    elif sc == SCENE_STATIC_BOX:
        out.update(sbox_center=(CLIMB_BOX_AHEAD + CLIMB_BOX_HALF[0], 0.0, CLIMB_BOX_HALF[2]),
                   sbox_half=CLIMB_BOX_HALF)
    elif sc == SCENE_FREE_BOX:
        out.update(box_half=FREE_BOX_HALF, box_mass=FREE_BOX_MASS, goal=box_goal(seed))
    return out


def tracking_cost(gait: int = 1, v_cmd=(0.5, 0.0), origin=(0.0, 0.0), box_goal_xy=None, **override) -> dict:
    """Parameters of the Eq. 3 / Eq. 4 tracking cost (shared keys for the library and the
    oracle).  Q is diagonal over the state error [p(3), attitude(3), q(12), v(3), w(3),
    qd(12)], R over the joint targets.  gait 1 trots (period 0.4 s, half stance, 8 cm
    foot lift); gait 0 holds the standing pose."""
    Q = ([1.0, 1.0, 100.0] + [10.0, 10.0, 1.0] + [0.1] * 12 + [1.0, 1.0, 0.1] + [0.1, 0.1, 0.1] + [1.0e-3] * 12)
    c = dict(Q=Q, R=[0.5] * 12, p_ref0=(origin[0], origin[1], WALK_COST["h_ref"]), v_cmd=tuple(v_cmd),
             period=0.4, duty=0.5, swing_height=0.08, stand_height=WALK_COST["h_ref"] - ROBOT["foot_r"],
             raibert_k=0.1, box_w=0.0, box_goal=(0.0, 0.0), gait=int(gait))
    if box_goal_xy is not None:
        c.update(box_w=2.0, box_goal=tuple(box_goal_xy))
    c.update(override)
    return c


def model_dict(workload: dict, seed: int, **override) -> dict:
    """Robot plus scene description as one flat dict (keys shared by both sides)."""
    d = dict(ROBOT)
    d.update(scene_extras(workload, seed))
    d.update(override)
    return d


def params_dict(workload: dict, seed: int, **override) -> dict:
    p = dict(K=workload["K"], H=workload["H"], nk=workload["nk"], dt=workload["dt"], sigma=workload["sigma"],
             lam=workload["lam"], kp=workload["kp"], kd=workload["kd"], seed=int(seed), instance=0)
    p.update(workload["cost"])
    if workload["scene"] == SCENE_FREE_BOX:
        p["goal"] = box_goal(seed)
    p.update(override)
    return p
