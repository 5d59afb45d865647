"""ctypes front end of the FP64 oracle (oracle/mppi_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline
leg of the benchmark.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mppi_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

NX, NX_BOX, NQ, NV = 37, 50, 19, 18


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable x86-64-v3, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC,
                               os.path.join(HERE, "mlp_oracle.c"), os.path.join(HERE, "tracking_oracle.c"), "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Model(C.Structure):
    _fields_ = [
        ("trunk_size", C.c_double * 3), ("trunk_mass", C.c_double),
        ("hip_x", C.c_double), ("hip_y", C.c_double),
        ("thigh_len", C.c_double), ("thigh_mass", C.c_double),
        ("calf_len", C.c_double), ("calf_mass", C.c_double),
        ("foot_r", C.c_double), ("gravity", C.c_double),
        ("k", C.c_double), ("c", C.c_double), ("mu", C.c_double), ("vs", C.c_double),
        ("scene", C.c_int32), ("hf_nx", C.c_int32), ("hf_ny", C.c_int32), ("pad0", C.c_int32),
        ("hf_cell", C.c_double), ("hf_x0", C.c_double), ("hf_y0", C.c_double),
        ("hf", C.POINTER(C.c_double)),
        ("sbox_center", C.c_double * 3), ("sbox_half", C.c_double * 3),
        ("box_half", C.c_double * 3), ("box_mass", C.c_double),
    ]


class Params(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("H", C.c_int32), ("nk", C.c_int32), ("basis", C.c_int32),
        ("dt", C.c_double), ("sigma", C.c_double), ("lam", C.c_double), ("kp", C.c_double), ("kd", C.c_double),
        ("w_h", C.c_double), ("h_ref", C.c_double), ("w_o", C.c_double), ("w_v", C.c_double),
        ("v_ref", C.c_double), ("w_tau", C.c_double), ("w_reach", C.c_double), ("w_box", C.c_double),
        ("goal", C.c_double * 2),
        ("seed", C.c_uint64), ("instance", C.c_uint32), ("pad1", C.c_uint32),
    ]


class Tracking(C.Structure):
    """Eq. 3 / Eq. 4 tracking-cost parameters (orc_tracking)."""
    _fields_ = [
        ("Q", C.c_double * 36), ("R", C.c_double * 12), ("p_ref0", C.c_double * 3), ("v_cmd", C.c_double * 2),
        ("period", C.c_double), ("duty", C.c_double), ("swing_height", C.c_double), ("stand_height", C.c_double),
        ("raibert_k", C.c_double), ("box_w", C.c_double), ("box_goal", C.c_double * 2),
        ("gait", C.c_int32), ("pad", C.c_int32),
    ]


def tracking(c: dict) -> Tracking:
    """Build an orc_tracking from a dict with the same keys (arrays for Q, R, p_ref0,
    v_cmd, box_goal)."""
    s = Tracking()
    s.Q[:] = [float(v) for v in c["Q"]]
    s.R[:] = [float(v) for v in c["R"]]
    s.p_ref0[:] = [float(v) for v in c["p_ref0"]]
    s.v_cmd[:] = [float(v) for v in c["v_cmd"]]
    for key in ("period", "duty", "swing_height", "stand_height", "raibert_k", "box_w"):
        setattr(s, key, float(c[key]))
    s.box_goal[:] = [float(v) for v in c.get("box_goal", (0.0, 0.0))]
    s.gait = int(c["gait"])
    return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        u32p = C.POINTER(C.c_uint32)
        mp, pp, tp = C.POINTER(Model), C.POINTER(Params), C.POINTER(Tracking)
        sig = {
            "orc_nx": (C.c_int, [mp]),
            "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
            "orc_sample_eps": (None, [pp, C.c_uint32, dp]),
            "orc_philox_raw": (None, [pp, C.c_uint32, u32p]),
            "orc_spline_basis": (None, [C.c_int, C.c_int, C.c_double, dp]),
            "orc_basis_matrix": (None, [C.c_int, C.c_int, C.c_int, C.c_double, dp]),
            "orc_shift_matrix_b": (None, [C.c_int, C.c_int, C.c_int, C.c_double, dp]),
            "orc_interp_eval": (None, [C.c_int, C.c_int, C.c_double, dp, C.c_double, dp]),
            "orc_spline_eval": (None, [C.c_int, C.c_double, dp, C.c_double, dp]),
            "orc_shift_matrix": (None, [C.c_int, C.c_int, C.c_double, dp]),
            "orc_fk": (None, [mp, dp, dp, dp, dp]),
            "orc_foot_positions": (None, [mp, dp, dp]),
            "orc_mass_matrix": (None, [mp, dp, dp]),
            "orc_bias": (None, [mp, dp, dp, dp]),
            "orc_kinetic_energy": (C.c_double, [mp, dp, dp]),
            "orc_kinetic_energy_fd": (C.c_double, [mp, dp, dp, C.c_double]),
            "orc_potential_energy": (C.c_double, [mp, dp]),
            "orc_momentum": (None, [mp, dp, dp, dp, dp]),
            "orc_retract": (None, [dp, dp, C.c_double, dp]),
            "orc_accel": (None, [mp, dp, dp, dp, dp]),
            "orc_rk4": (None, [mp, dp, dp, dp, C.c_double, C.c_int, C.c_int, dp, C.c_double]),
            "orc_step": (C.c_int, [mp, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp]),
            "orc_contact_total": (None, [mp, dp, dp, dp, C.POINTER(C.c_int)]),
            "orc_step_system": (C.c_int, [mp, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp]),
            "orc_step_system_box": (C.c_int, [mp, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp]),
            "orc_terrain": (C.c_int, [mp, dp, C.c_double, dp, dp]),
            "orc_sphere_box": (C.c_int, [dp, C.c_double, dp, dp, dp, dp, dp]),
            "orc_point_box": (C.c_int, [dp, dp, dp, dp, dp, dp]),
            "orc_contact_law": (C.c_int, [mp, C.c_double, dp, dp, dp, dp]),
            "orc_stage_cost": (C.c_double, [mp, pp, dp, dp]),
            "orc_rollout": (C.c_double, [mp, pp, dp, dp, dp]),
            "orc_rollout_batch": (None, [mp, pp, dp, dp, dp, dp, dp, C.c_int]),
            "orc_weights": (C.c_int, [C.c_int, C.c_double, dp, dp]),
            "orc_update": (C.c_int, [pp, dp, dp, dp, dp, dp]),
            "orc_shift": (None, [pp, dp, dp, dp]),
            "orc_mppi_step": (C.c_int, [mp, pp, C.c_uint32, dp, dp, dp, dp, C.c_int]),
            "orc_mppi_step_proposal": (C.c_int, [mp, pp, C.c_uint32, dp, dp, dp, dp, C.c_int, C.c_int, dp, dp, dp,
                                                 C.POINTER(C.c_int), C.c_int]),
            "orc_leg_ik": (None, [mp, dp, dp]),
            "orc_gait_foot": (None, [tp, C.c_int, C.c_double, dp, dp, dp]),
            "orc_gait_reference": (None, [mp, tp, C.c_double, dp, dp]),
            "orc_tracking_stage": (C.c_double, [mp, tp, C.c_double, dp, dp, dp, dp]),
            "orc_tracking_cost": (C.c_double, [mp, pp, tp, C.c_uint32, dp, dp]),
            "orc_rollout_tracking": (C.c_double, [mp, pp, tp, C.c_uint32, dp, dp, dp]),
            "orc_mppi_step_tracking": (C.c_int, [mp, pp, tp, C.c_uint32, dp, dp, dp, dp, C.c_int]),
            "orc_policy_features": (None, [dp, dp, dp, dp, dp, dp]),
            "orc_policy_head": (None, [dp, dp, dp, C.c_int, C.c_double, dp, dp]),
            "orc_mlp_n_params": (C.c_int, []),
            "orc_mlp_forward": (None, [dp, C.c_int, dp, dp, C.c_int]),
            "orc_mlp_loss": (C.c_double, [dp, C.c_int, dp, dp, C.c_int]),
            "orc_mlp_grad": (C.c_double, [dp, C.c_int, dp, dp, dp, C.c_int]),
            "orc_adam": (None, [dp, dp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


class Oracle:
    """One robot+scene model with convenience wrappers returning numpy arrays."""

    def __init__(self, model: dict):
        self.model_dict = dict(model)
        m = Model()
        for key in ("trunk_mass", "hip_x", "hip_y", "thigh_len", "thigh_mass", "calf_len", "calf_mass", "foot_r",
                    "gravity", "k", "c", "mu", "vs"):
            setattr(m, key, float(model[key]))
        m.trunk_size[:] = [float(v) for v in model["trunk_size"]]
        m.scene = int(model.get("scene", 0))
        self._hf = None
        if "hf" in model:
            hf = _f64(model["hf"])
            self._hf = hf
            m.hf_ny, m.hf_nx = hf.shape
            m.hf_cell, m.hf_x0, m.hf_y0 = float(model["hf_cell"]), float(model["hf_x0"]), float(model["hf_y0"])
            m.hf = _dp(hf)
        m.sbox_center[:] = [float(v) for v in model.get("sbox_center", (0, 0, 0))]
        m.sbox_half[:] = [float(v) for v in model.get("sbox_half", (0, 0, 0))]
        m.box_half[:] = [float(v) for v in model.get("box_half", (0, 0, 0))]
        m.box_mass = float(model.get("box_mass", 0.0))
        self.m = m
        self.L = lib()
        self.nx = self.L.orc_nx(C.byref(m))

    # ---- parameters ----------------------------------------------------
    @staticmethod
    def params(p: dict) -> Params:
        s = Params()
        s.K, s.H, s.nk = int(p["K"]), int(p["H"]), int(p["nk"])
        for key in ("dt", "sigma", "lam", "kp", "kd", "w_h", "h_ref", "w_o", "w_v", "v_ref", "w_tau", "w_reach",
                    "w_box"):
            setattr(s, key, float(p[key]))
        s.goal[:] = [float(v) for v in p.get("goal", (0.0, 0.0))]
        s.seed = int(p.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
        s.instance = int(p.get("instance", 0))
        s.basis = int(p.get("basis", 0))
        return s

    # ---- rigid body ----------------------------------------------------
    def fk(self, q):
        q = _f64(q, NQ)
        R, pos, com = np.zeros((13, 3, 3)), np.zeros((13, 3)), np.zeros((13, 3))
        self.L.orc_fk(C.byref(self.m), _dp(q), _dp(R), _dp(pos), _dp(com))
        return R, pos, com

    def feet(self, q):
        q = _f64(q, NQ)
        out = np.zeros((4, 3))
        self.L.orc_foot_positions(C.byref(self.m), _dp(q), _dp(out))
        return out

    def mass_matrix(self, q):
        q = _f64(q, NQ)
        M = np.zeros((NV, NV))
        self.L.orc_mass_matrix(C.byref(self.m), _dp(q), _dp(M))
        return M

    def bias(self, q, v):
        q, v = _f64(q, NQ), _f64(v, NV)
        b = np.zeros(NV)
        self.L.orc_bias(C.byref(self.m), _dp(q), _dp(v), _dp(b))
        return b

    def kinetic_energy(self, q, v):
        return self.L.orc_kinetic_energy(C.byref(self.m), _dp(_f64(q, NQ)), _dp(_f64(v, NV)))

    def kinetic_energy_fd(self, q, v, eps=1e-5):
        return self.L.orc_kinetic_energy_fd(C.byref(self.m), _dp(_f64(q, NQ)), _dp(_f64(v, NV)), eps)

    def potential_energy(self, q):
        return self.L.orc_potential_energy(C.byref(self.m), _dp(_f64(q, NQ)))

    def momentum(self, q, v):
        P, Lo = np.zeros(3), np.zeros(3)
        self.L.orc_momentum(C.byref(self.m), _dp(_f64(q, NQ)), _dp(_f64(v, NV)), _dp(P), _dp(Lo))
        return P, Lo

    def retract(self, q, v, t):
        out = np.zeros(NQ)
        self.L.orc_retract(_dp(_f64(q, NQ)), _dp(_f64(v, NV)), float(t), _dp(out))
        return out

    def accel(self, q, v, tau_gen):
        out = np.zeros(NV)
        self.L.orc_accel(C.byref(self.m), _dp(_f64(q, NQ)), _dp(_f64(v, NV)), _dp(_f64(tau_gen, NV)), _dp(out))
        return out

    def rk4(self, q, v, dt, nsteps, tau_gen=None, spring_target=None, kp=0.0):
        q, v = _f64(q, NQ).copy(), _f64(v, NV).copy()
        tg = _f64(tau_gen, NV) if tau_gen is not None else None
        st = _f64(spring_target, 12) if spring_target is not None else np.zeros(12)
        self.L.orc_rk4(C.byref(self.m), _dp(q), _dp(v), _dp(tg), float(dt), int(nsteps),
                       int(spring_target is not None), _dp(st), float(kp))
        return q, v

    # ---- discrete dynamics, cost --------------------------------------
    def step(self, x, u, kp, kd, dt):
        x = _f64(x, self.nx)
        xo, tau = np.zeros(self.nx), np.zeros(12)
        rc = self.L.orc_step(C.byref(self.m), _dp(x), _dp(_f64(u, 12)), float(kp), float(kd), float(dt), _dp(xo),
                             _dp(tau))
        return xo, tau, rc

    def step_system(self, x, u, kp, kd, dt):
        A, r = np.zeros((NV, NV)), np.zeros(NV)
        n = self.L.orc_step_system(C.byref(self.m), _dp(_f64(x, self.nx)), _dp(_f64(u, 12)), float(kp), float(kd),
                                   float(dt), _dp(A), _dp(r))
        return A, r, n

    def contact_total(self, x):
        Fr, Fb, n = np.zeros(3), np.zeros(3), C.c_int(0)
        self.L.orc_contact_total(C.byref(self.m), _dp(_f64(x, self.nx)), _dp(Fr), _dp(Fb), C.byref(n))
        return Fr, Fb, n.value

    def step_system_box(self, x, u, kp, kd, dt):
        """The free box's 6x6 system of the step (scene 3): A_b, rhs_b, active contacts."""
        A, r = np.zeros((6, 6)), np.zeros(6)
        n = self.L.orc_step_system_box(C.byref(self.m), _dp(_f64(x, self.nx)), _dp(_f64(u, 12)), float(kp),
                                       float(kd), float(dt), _dp(A), _dp(r))
        return A, r, n

    def terrain(self, c, r):
        d, n = C.c_double(0), np.zeros(3)
        hit = self.L.orc_terrain(C.byref(self.m), _dp(_f64(c, 3)), float(r), C.byref(d), _dp(n))
        return bool(hit), d.value, n

    def contact_law(self, delta, n, vrel):
        F, D = np.zeros(3), np.zeros((3, 3))
        hit = self.L.orc_contact_law(C.byref(self.m), float(delta), _dp(_f64(n, 3)), _dp(_f64(vrel, 3)), _dp(F),
                                     _dp(D))
        return bool(hit), F, D

    def stage_cost(self, p: dict, x, tau):
        ps = self.params(p)
        return self.L.orc_stage_cost(C.byref(self.m), C.byref(ps), _dp(_f64(x, self.nx)), _dp(_f64(tau, 12)))

    def rollout(self, p: dict, x0, theta, traj=False):
        ps = self.params(p)
        tr = np.zeros((p["H"] + 1, self.nx)) if traj else None
        L = self.L.orc_rollout(C.byref(self.m), C.byref(ps), _dp(_f64(x0, self.nx)), _dp(_f64(theta, 12 * p["nk"])),
                               _dp(tr))
        return (L, tr) if traj else L

    def rollout_batch(self, p: dict, x0, mu, eps, traj=False, nthreads=0):
        ps = self.params(p)
        K, D = p["K"], 12 * p["nk"]
        costs = np.zeros(K)
        tr = np.zeros((K, p["H"] + 1, self.nx)) if traj else None
        self.L.orc_rollout_batch(C.byref(self.m), C.byref(ps), _dp(_f64(x0, self.nx)), _dp(_f64(mu, D)),
                                 _dp(_f64(eps, K * D)), _dp(costs), _dp(tr), int(nthreads))
        return (costs, tr) if traj else costs

    def mppi_step(self, p: dict, step: int, x0, mu, nthreads=0):
        ps = self.params(p)
        mu = _f64(mu, 12 * p["nk"]).copy()
        u0, costs = np.zeros(12), np.zeros(p["K"])
        rc = self.L.orc_mppi_step(C.byref(self.m), C.byref(ps), int(step), _dp(_f64(x0, self.nx)), _dp(mu), _dp(u0),
                                  _dp(costs), int(nthreads))
        return u0, mu, costs, rc

    def mppi_step_proposal(self, p: dict, step: int, x0, mu, center, sd, Kp, gate=0, nthreads=0):
        """Learned-proposal step; returns (u0, shifted nominal, proposal costs (Kp),
        fallback costs (K, zeros when accepted), accepted, status)."""
        ps = self.params(p)
        D = 12 * p["nk"]
        mu = _f64(mu, D).copy()
        u0, cp, cf = np.zeros(12), np.zeros(Kp), np.zeros(p["K"])
        acc = C.c_int(0)
        rc = self.L.orc_mppi_step_proposal(C.byref(self.m), C.byref(ps), int(step), _dp(_f64(x0, self.nx)), _dp(mu),
                                           _dp(_f64(center, D)), _dp(_f64(sd, D)), int(Kp), int(gate), _dp(u0), _dp(cp),
                                           _dp(cf), C.byref(acc), int(nthreads))
        return u0, mu, cp, cf, bool(acc.value), rc

    # ---- Eq. 3 / Eq. 4 tracking cost -------------------------------------
    def leg_ik(self, p_hip):
        q = np.zeros(3)
        self.L.orc_leg_ik(C.byref(self.m), _dp(_f64(p_hip, 3)), _dp(q))
        return q

    def gait_reference(self, c: dict, t: float, x0):
        u = np.zeros(12)
        self.L.orc_gait_reference(C.byref(self.m), C.byref(tracking(c)), float(t), _dp(_f64(x0, self.nx)), _dp(u))
        return u

    def tracking_stage(self, c: dict, t_x, x, q_ref, u, u_ref):
        return self.L.orc_tracking_stage(C.byref(self.m), C.byref(tracking(c)), float(t_x), _dp(_f64(x, self.nx)),
                                         _dp(_f64(q_ref, 12)), _dp(_f64(u, 12)), _dp(_f64(u_ref, 12)))

    def tracking_cost(self, p: dict, c: dict, step: int, traj, u):
        """Cost of a trajectory ((H+1) x nx) under controls (H x 12) at control step `step`."""
        H = p["H"]
        return self.L.orc_tracking_cost(C.byref(self.m), C.byref(self.params(p)), C.byref(tracking(c)), int(step),
                                        _dp(_f64(traj, (H + 1) * self.nx)), _dp(_f64(u, 12 * H)))

    def rollout_tracking(self, p: dict, c: dict, step: int, x0, theta, traj=False):
        tr = np.zeros((p["H"] + 1, self.nx)) if traj else None
        L = self.L.orc_rollout_tracking(C.byref(self.m), C.byref(self.params(p)), C.byref(tracking(c)), int(step),
                                        _dp(_f64(x0, self.nx)), _dp(_f64(theta, 12 * p["nk"])), _dp(tr))
        return (L, tr) if traj else L

    def mppi_step_tracking(self, p: dict, c: dict, step: int, x0, mu, nthreads=0):
        mu = _f64(mu, 12 * p["nk"]).copy()
        u0, costs = np.zeros(12), np.zeros(p["K"])
        rc = self.L.orc_mppi_step_tracking(C.byref(self.m), C.byref(self.params(p)), C.byref(tracking(c)),
                                           int(step), _dp(_f64(x0, self.nx)), _dp(mu), _dp(u0), _dp(costs),
                                           int(nthreads))
        return u0, mu, costs, rc


def gait_foot(c: dict, leg: int, t: float, v_h, cmd_h):
    out = np.zeros(3)
    lib().orc_gait_foot(C.byref(tracking(c)), int(leg), float(t), _dp(_f64(v_h, 2)), _dp(_f64(cmd_h, 2)), _dp(out))
    return out


# ---- model-free pieces ---------------------------------------------------
def sphere_box(c, r, p, quat, h):
    """Sphere (centre c, radius r) against an oriented box: (hit, depth, normal box -> sphere)."""
    d, n = C.c_double(0), np.zeros(3)
    hit = lib().orc_sphere_box(_dp(_f64(c, 3)), float(r), _dp(_f64(p, 3)), _dp(_f64(quat, 4)), _dp(_f64(h, 3)),
                               C.byref(d), _dp(n))
    return bool(hit), d.value, n


def point_box(x, p, quat, h):
    """Point strictly inside an oriented box: (hit, depth of the shallowest face, its outward normal)."""
    d, n = C.c_double(0), np.zeros(3)
    hit = lib().orc_point_box(_dp(_f64(x, 3)), _dp(_f64(p, 3)), _dp(_f64(quat, 4)), _dp(_f64(h, 3)), C.byref(d),
                              _dp(n))
    return bool(hit), d.value, n


def philox(ctr, key):
    L = lib()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    u32p = C.POINTER(C.c_uint32)
    L.orc_philox4x32_10(c.ctypes.data_as(u32p), k.ctypes.data_as(u32p), o.ctypes.data_as(u32p))
    return o


def sample_eps(p: dict, step: int):
    ps = Oracle.params(p)
    out = np.zeros((p["K"], 12 * p["nk"]))
    lib().orc_sample_eps(C.byref(ps), int(step), _dp(out))
    return out


def philox_raw(p: dict, step: int):
    ps = Oracle.params(p)
    nb = (12 * p["nk"] + 3) // 4
    out = np.zeros((p["K"], 4 * nb), dtype=np.uint32)
    lib().orc_philox_raw(C.byref(ps), int(step), out.ctypes.data_as(C.POINTER(C.c_uint32)))
    return out


def spline_basis(nk, H, dt):
    B = np.zeros((H, nk))
    lib().orc_spline_basis(int(nk), int(H), float(dt), _dp(B))
    return B


def basis_matrix(basis, nk, H, dt):
    """H x nk matrix of the knot interpolation (0 cubic, 1 linear, 2 zeroth order) at k dt."""
    B = np.zeros((H, nk))
    lib().orc_basis_matrix(int(basis), int(nk), int(H), float(dt), _dp(B))
    return B


def shift_matrix_b(basis, nk, H, dt):
    S = np.zeros((nk, nk))
    lib().orc_shift_matrix_b(int(basis), int(nk), int(H), float(dt), _dp(S))
    return S


def interp_eval(basis, knots, T, t):
    k = _f64(knots)
    out = np.zeros(1)
    lib().orc_interp_eval(int(basis), int(k.size), float(T), _dp(k), float(t), _dp(out))
    return out[0]


def spline_eval(knots, T, t):
    k = _f64(knots)
    out = np.zeros(1)
    lib().orc_spline_eval(int(k.size), float(T), _dp(k), float(t), _dp(out))
    return out[0]


def shift_matrix(nk, H, dt):
    S = np.zeros((nk, nk))
    lib().orc_shift_matrix(int(nk), int(H), float(dt), _dp(S))
    return S


def weights(costs, lam):
    c = _f64(costs)
    w = np.zeros(c.size)
    rc = lib().orc_weights(int(c.size), float(lam), _dp(c), _dp(w))
    return w, rc


def update(p: dict, costs, mu, eps):
    ps = Oracle.params(p)
    K, D = p["K"], 12 * p["nk"]
    out, w = np.zeros(D), np.zeros(K)
    rc = lib().orc_update(C.byref(ps), _dp(_f64(costs, K)), _dp(_f64(mu, D)), _dp(_f64(eps, K * D)), _dp(out), _dp(w))
    return out, w, rc


def shift(p: dict, mu_prime):
    ps = Oracle.params(p)
    D = 12 * p["nk"]
    mu, u0 = np.zeros(D), np.zeros(12)
    lib().orc_shift(C.byref(ps), _dp(_f64(mu_prime, D)), _dp(mu), _dp(u0))
    return mu, u0


# ---- learned proposal (MLP) ----------------------------------------------------
MLP_DIMS = (40, 512, 512, 512, 512, 144)


def mlp_n_params():
    return lib().orc_mlp_n_params()


def mlp_forward(P, X, bf16=False):
    X = _f64(X)
    B = X.shape[0]
    out = np.zeros((B, 144))
    lib().orc_mlp_forward(_dp(_f64(P)), B, _dp(X), _dp(out), int(bf16))
    return out


def mlp_loss(P, X, Y, bf16=False):
    X, Y = _f64(X), _f64(Y)
    return lib().orc_mlp_loss(_dp(_f64(P)), X.shape[0], _dp(X), _dp(Y), int(bf16))


def mlp_grad(P, X, Y, bf16=False):
    X, Y = _f64(X), _f64(Y)
    G = np.zeros(mlp_n_params())
    L = lib().orc_mlp_grad(_dp(_f64(P)), X.shape[0], _dp(X), _dp(Y), _dp(G), int(bf16))
    return L, G


def adam(P, m, v, G, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    P, m, v = _f64(P).copy(), _f64(m).copy(), _f64(v).copy()
    lib().orc_adam(_dp(P), _dp(m), _dp(v), _dp(_f64(G)), P.size, int(t), lr, b1, b2, eps)
    return P, m, v


def policy_features(x, cmd, origin, in_mean, in_std):
    f = np.zeros(40)
    lib().orc_policy_features(_dp(_f64(x, 37)), _dp(_f64(cmd, 3)), _dp(_f64(origin, 2)), _dp(_f64(in_mean, 40)),
                              _dp(_f64(in_std, 40)), _dp(f))
    return f


def policy_head(out, out_mean, out_std, nk, sigma_max):
    c, sd = np.zeros(12 * nk), np.zeros(12 * nk)
    lib().orc_policy_head(_dp(_f64(out, 144)), _dp(_f64(out_mean, 72)), _dp(_f64(out_std, 72)), int(nk),
                          float(sigma_max), _dp(c), _dp(sd))
    return c, sd


def mlp_layer_views(P):
    """(W, b) views of each layer of a flat parameter vector."""
    out, off = [], 0
    for fi, fo in zip(MLP_DIMS[:-1], MLP_DIMS[1:]):
        W = P[off:off + fi * fo].reshape(fi, fo)
        b = P[off + fi * fo:off + fi * fo + fo]
        out.append((W, b))
        off += fi * fo + fo
    return out
