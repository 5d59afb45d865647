"""Thin ctypes binding of the C ABI in include/mppi.h.

Argument marshalling only: every step of the hot path runs in the HIP kernels of
libmppi.so.  PyTorch supplies device memory (the workspace and the caller's buffers)
and the stream.  There is no CPU fallback: if the library is missing or the GPU is
absent the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmppi.so")

OK, WARN_ALL_NONFINITE, EINVAL, ENOMEM, EHIP, ESTATE = 0, 1, -1, -2, -3, -6
ARITH = {"fp64": 0, "fp32": 1, "mixed": 2}
# proposal gates (include/mppi_policy.h); "-concurrent": one launch rolls out the proposal and the
# plain fallback on every step
GATE = {"cost": 0, "none": 1, "best": 2, "cost-concurrent": 4, "best-concurrent": 6}


class MppiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mppi status {status}: {msg}")
        self.status = status


class ModelDesc(C.Structure):
    _fields_ = [
        ("trunk_size", C.c_float * 3), ("trunk_mass", C.c_float),
        ("hip_x", C.c_float), ("hip_y", C.c_float),
        ("thigh_len", C.c_float), ("thigh_mass", C.c_float),
        ("calf_len", C.c_float), ("calf_mass", C.c_float),
        ("foot_r", C.c_float), ("gravity", C.c_float),
        ("contact_k", C.c_float), ("contact_c", C.c_float), ("friction_mu", C.c_float), ("slip_velocity", C.c_float),
        ("scene", C.c_int32), ("hf_nx", C.c_int32), ("hf_ny", C.c_int32),
        ("hf_cell", C.c_float), ("hf_x0", C.c_float), ("hf_y0", C.c_float),
        ("heightfield", C.POINTER(C.c_float)),
        ("sbox_center", C.c_float * 3), ("sbox_half", C.c_float * 3),
        ("box_half", C.c_float * 3), ("box_mass", C.c_float),
    ]


class Params(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("H", C.c_int32), ("n_knots", C.c_int32),
        ("dt", C.c_float), ("sigma", C.c_float), ("lam", C.c_float), ("kp", C.c_float), ("kd", C.c_float),
        ("w_height", C.c_float), ("h_ref", C.c_float), ("w_upright", C.c_float), ("w_vel", C.c_float),
        ("v_ref", C.c_float), ("w_torque", C.c_float), ("w_reach", C.c_float), ("w_box", C.c_float),
        ("goal", C.c_float * 2),
        ("seed", C.c_uint64), ("instance", C.c_uint32), ("arith", C.c_int32), ("basis", C.c_int32),
        ("cost", C.c_int32), ("lanes", C.c_int32),
    ]


class TrackingCost(C.Structure):
    """mppi_tracking_cost: Eq. 3 / Eq. 4 weights, references and gait constants."""
    _fields_ = [
        ("Q", C.c_float * 36), ("R", C.c_float * 12), ("p_ref0", C.c_float * 3), ("v_cmd", C.c_float * 2),
        ("period", C.c_float), ("duty", C.c_float), ("swing_height", C.c_float), ("stand_height", C.c_float),
        ("raibert_gain", C.c_float), ("box_weight", C.c_float), ("box_goal", C.c_float * 2),
        ("gait", C.c_int32), ("reserved", C.c_int32),
    ]


COST = {"running": 0, "tracking": 1}


_lib = None


def lib():
    """Load libmppi.so (built by paper_2409_10469_amd.build); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built (run __graft_entry__.build())")
        # torch ships its own HIP runtime under the same soname; loading torch first makes
        # the library bind to that one, so the process has a single runtime for the
        # workspace, the streams and the kernels
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, fp, u32p = C.c_void_p, C.c_void_p, C.c_void_p
        sig = {
            "mppi_model_create": (C.c_int, [C.POINTER(ModelDesc), C.POINTER(C.c_void_p)]),
            "mppi_model_destroy": (None, [vp]),
            "mppi_model_nx": (C.c_int, [vp]),
            "mppi_create": (C.c_int, [vp, C.POINTER(Params), C.POINTER(C.c_void_p)]),
            "mppi_step_static": (C.c_int, [vp, vp, vp, vp, vp]),
            "mppi_destroy": (None, [vp]),
            "mppi_workspace_bytes": (C.c_size_t, [vp]),
            "mppi_get_basis": (C.c_int, [vp, vp, vp]),
            "mppi_bind": (C.c_int, [vp, vp, C.c_size_t, vp]),
            "mppi_set_nominal": (C.c_int, [vp, fp]),
            "mppi_get_nominal": (C.c_int, [vp, fp]),
            "mppi_set_step": (C.c_int, [vp, C.c_uint32]),
            "mppi_get_step": (C.c_uint32, [vp]),
            "mppi_sample": (C.c_int, [vp, fp, u32p]),
            "mppi_rollout_batch": (C.c_int, [vp, fp, fp, fp, fp]),
            "mppi_update": (C.c_int, [vp, fp, fp, fp, fp]),
            "mppi_step": (C.c_int, [vp, fp, fp]),
            "mppi_update_shift": (C.c_int, [vp, fp, fp, fp]),
            "mppi_sync_status": (C.c_int, [vp]),
            "mppi_set_tracking_cost": (C.c_int, [vp, C.POINTER(TrackingCost)]),
            "mppi_sim_step": (C.c_int, [vp, C.c_int, C.c_int, fp, fp, C.c_float, C.c_float, C.c_float, fp, fp, fp,
                                        vp]),
            "mppi_status_str": (C.c_char_p, [C.c_int]),
            "mppi_last_error": (C.c_char_p, [vp]),
            "mppi_step_proposal": (C.c_int, [vp, fp, fp, fp, C.c_int, C.c_int, fp]),
            "mppi_set_proposal": (C.c_int, [vp, vp, C.c_int, C.c_int, vp, vp]),
            "mppi_proposal_stats": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "mppi_policy_n_params": (C.c_int, []),
            "mppi_policy_create": (C.c_int, [C.c_char_p, C.c_uint64, C.c_int, C.POINTER(C.c_void_p)]),
            "mppi_policy_destroy": (None, [vp]),
            "mppi_policy_workspace_bytes": (C.c_size_t, [vp]),
            "mppi_policy_bind": (C.c_int, [vp, vp, C.c_size_t, vp]),
            "mppi_policy_set_normalization": (C.c_int, [vp, vp, vp, vp, vp]),
            "mppi_policy_get_params": (C.c_int, [vp, fp]),
            "mppi_policy_get_normalization": (C.c_int, [vp, vp, vp, vp, vp]),
            "mppi_policy_set_params": (C.c_int, [vp, fp]),
            "mppi_policy_forward": (C.c_int, [vp, fp, C.c_int, fp]),
            "mppi_policy_grad": (C.c_int, [vp, fp, fp, vp, C.c_int, fp, fp]),
            "mppi_policy_nll": (C.c_int, [vp, fp, fp, vp, C.c_int, fp]),
            "mppi_policy_pairs": (C.c_int, [C.c_int, C.c_int, C.c_int, fp, fp, C.c_float, fp, fp, vp, vp]),
            "mppi_policy_adam": (C.c_int, [vp, fp, C.c_float]),
            "mppi_policy_train_step": (C.c_int, [vp, fp, fp, vp, C.c_int, C.c_float, fp]),
            "mppi_policy_steps": (C.c_int, [vp]),
            "mppi_policy_save": (C.c_int, [vp, C.c_char_p]),
            "mppi_policy_head": (C.c_int, [vp, fp, C.c_int, C.c_float, fp, fp]),
            "mppi_policy_last_error": (C.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status < 0:
        msg = lib().mppi_last_error(ctx).decode()
        raise MppiError(status, msg)
    return status


def _ptr(t):
    if t is None:
        return None
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous(), "device tensors only"
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def model_desc(d: dict) -> tuple:
    """Build the C model description from a workload dict; returns (desc, keepalive)."""
    m = ModelDesc()
    m.trunk_size[:] = [float(v) for v in d["trunk_size"]]
    for k_py, k_c in (("trunk_mass", "trunk_mass"), ("hip_x", "hip_x"), ("hip_y", "hip_y"),
                      ("thigh_len", "thigh_len"), ("thigh_mass", "thigh_mass"), ("calf_len", "calf_len"),
                      ("calf_mass", "calf_mass"), ("foot_r", "foot_r"), ("gravity", "gravity"),
                      ("k", "contact_k"), ("c", "contact_c"), ("mu", "friction_mu"), ("vs", "slip_velocity")):
        setattr(m, k_c, float(d[k_py]))
    m.scene = int(d.get("scene", 0))
    keep = None
    if "hf" in d:
        hf = np.ascontiguousarray(d["hf"], dtype=np.float32)
        keep = hf
        m.hf_ny, m.hf_nx = hf.shape
        m.hf_cell, m.hf_x0, m.hf_y0 = float(d["hf_cell"]), float(d["hf_x0"]), float(d["hf_y0"])
        m.heightfield = hf.ctypes.data_as(C.POINTER(C.c_float))
    m.sbox_center[:] = [float(v) for v in d.get("sbox_center", (0, 0, 0))]
    m.sbox_half[:] = [float(v) for v in d.get("sbox_half", (0, 0, 0))]
    m.box_half[:] = [float(v) for v in d.get("box_half", (0, 0, 0))]
    m.box_mass = float(d.get("box_mass", 0.0))
    return m, keep


def params_struct(p: dict) -> Params:
    s = Params()
    s.K, s.H, s.n_knots = int(p["K"]), int(p["H"]), int(p["nk"])
    s.dt, s.sigma, s.lam, s.kp, s.kd = (float(p[k]) for k in ("dt", "sigma", "lam", "kp", "kd"))
    s.w_height, s.h_ref, s.w_upright = float(p["w_h"]), float(p["h_ref"]), float(p["w_o"])
    s.w_vel, s.v_ref, s.w_torque = float(p["w_v"]), float(p["v_ref"]), float(p["w_tau"])
    s.w_reach, s.w_box = float(p["w_reach"]), float(p["w_box"])
    s.goal[:] = [float(v) for v in p.get("goal", (0.0, 0.0))]
    s.seed = int(p.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    s.instance = int(p.get("instance", 0))
    s.arith = ARITH[p.get("arith", "fp64")]
    s.basis = int(p.get("basis", 0))  # 0 cubic, 1 linear, 2 zeroth order
    s.cost = COST[p.get("cost", "running")]
    s.lanes = int(p.get("lanes", 0))  # 0 default, 4 quad kernel, 16 lane-split kernel
    return s


def tracking_struct(c: dict) -> TrackingCost:
    """Marshal a tracking-cost dict (keys as in workloads.tracking_cost) into the C struct."""
    s = TrackingCost()
    s.Q[:] = [float(v) for v in c["Q"]]
    s.R[:] = [float(v) for v in c["R"]]
    s.p_ref0[:] = [float(v) for v in c["p_ref0"]]
    s.v_cmd[:] = [float(v) for v in c["v_cmd"]]
    s.period, s.duty = float(c["period"]), float(c["duty"])
    s.swing_height, s.stand_height = float(c["swing_height"]), float(c["stand_height"])
    s.raibert_gain, s.box_weight = float(c["raibert_k"]), float(c["box_w"])
    s.box_goal[:] = [float(v) for v in c.get("box_goal", (0.0, 0.0))]
    s.gait = int(c["gait"])
    s.reserved = int(c.get("reserved", 0))
    return s


class Model:
    def __init__(self, d: dict):
        desc, keep = model_desc(d)
        h = C.c_void_p()
        _check(lib().mppi_model_create(C.byref(desc), C.byref(h)))
        self.h = h
        self.nx = lib().mppi_model_nx(h)
        self.scene = desc.scene
        self._hf_host = keep
        self._hf_dev = None

    def hf_device(self):
        import torch
        if self._hf_host is None:
            return None
        if self._hf_dev is None:
            self._hf_dev = torch.from_numpy(self._hf_host).cuda()
        return self._hf_dev

    def sim_step(self, x, u, kp, kd, dt, tau_out=None, stream=None, arith="fp64"):
        """One dynamics step of n states x (n x nx) with joint targets u (n x 12)."""
        import torch
        n = x.shape[0]
        xo = torch.empty_like(x)
        _check(lib().mppi_sim_step(self.h, ARITH[arith], n, _ptr(x), _ptr(u), kp, kd, dt, _ptr(xo), _ptr(tau_out),
                                   _ptr(self.hf_device()), _stream(stream)))
        return xo

    def sim_step_into(self, x, u, kp, kd, dt, out, tau_out=None, stream=None, arith="fp64"):
        """As sim_step, writing into the preallocated `out` (n x nx)."""
        _check(lib().mppi_sim_step(self.h, ARITH[arith], x.shape[0], _ptr(x), _ptr(u), kp, kd, dt, _ptr(out),
                                   _ptr(tau_out), _ptr(self.hf_device()), _stream(stream)))
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mppi_model_destroy(self.h)
            self.h = None


class Controller:
    """One MPPI instance bound to a torch-allocated device workspace."""

    def __init__(self, model: Model, p: dict, stream=None, bind=True):
        import torch
        self.model = model
        self.p = dict(p)
        ps = params_struct(p)
        h = C.c_void_p()
        _check(lib().mppi_create(model.h, C.byref(ps), C.byref(h)))
        self.h = h
        self.K, self.H, self.nk = int(p["K"]), int(p["H"]), int(p["nk"])
        self.D = 12 * self.nk
        self.stream = stream
        if not bind:  # for mppi_step_static, which needs an unbound controller
            self.ws = None
            return
        nbytes = lib().mppi_workspace_bytes(h)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off:off + nbytes]
        self.stream = stream
        _check(lib().mppi_bind(h, C.c_void_p(self.ws_view.data_ptr()), nbytes, _stream(stream)), h)

    def _s(self, status):
        return _check(status, self.h)

    def set_nominal(self, knots):
        self._s(lib().mppi_set_nominal(self.h, _ptr(knots)))

    def get_nominal(self):
        import torch
        out = torch.empty(self.D, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_get_nominal(self.h, _ptr(out)))
        return out

    def set_step(self, step):
        self._s(lib().mppi_set_step(self.h, int(step)))

    def basis_matrices(self):
        """Host copies of the interpolation matrix B (H x nk) and the shift S (nk x nk)."""
        Bm = np.zeros((self.p["H"], self.p["nk"]))
        Sm = np.zeros((self.p["nk"], self.p["nk"]), dtype=np.float32)
        self._s(lib().mppi_get_basis(self.h, Bm.ctypes.data_as(C.c_void_p), Sm.ctypes.data_as(C.c_void_p)))
        return Bm, Sm

    @property
    def step_counter(self):
        return lib().mppi_get_step(self.h)

    def sample(self, raw=False):
        import torch
        eps = torch.empty((self.K, self.D), dtype=torch.float32, device="cuda")
        nb = (self.D + 3) // 4
        r = torch.empty((self.K, 4 * nb), dtype=torch.int32, device="cuda") if raw else None
        self._s(lib().mppi_sample(self.h, _ptr(eps), _ptr(r)))
        return (eps, r) if raw else eps

    def rollout_batch(self, x0, eps=None, traj=False, costs=None):
        import torch
        costs = costs if costs is not None else torch.empty(self.K, dtype=torch.float32, device="cuda")
        tr = torch.empty((self.K, self.H + 1, self.model.nx), dtype=torch.float32, device="cuda") if traj else None
        self._s(lib().mppi_rollout_batch(self.h, _ptr(x0), _ptr(eps), _ptr(costs), _ptr(tr)))
        return (costs, tr) if traj else costs

    def update(self, costs, eps=None, weights=False):
        import torch
        out = torch.empty(self.D, dtype=torch.float32, device="cuda")
        w = torch.empty(self.K, dtype=torch.float32, device="cuda") if weights else None
        self._s(lib().mppi_update(self.h, _ptr(costs), _ptr(eps), _ptr(out), _ptr(w)))
        return (out, w) if weights else out

    def step_static(self, x0, nominal, u0=None):
        """mppi_step_static: one plain control step of an unbound controller in the
        library's static device scratch; `nominal` (device) is updated in place."""
        import torch
        if u0 is None:
            u0 = torch.empty(12, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_step_static(self.h, _ptr(x0), _ptr(nominal), _ptr(u0), _stream(self.stream)))
        return u0

    def step(self, x0, u0=None):
        import torch
        u0 = u0 if u0 is not None else torch.empty(12, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_step(self.h, _ptr(x0), _ptr(u0)))
        return u0

    def update_shift(self, costs, u0=None, weights=None):
        import torch
        u0 = u0 if u0 is not None else torch.empty(12, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_update_shift(self.h, _ptr(costs), _ptr(u0), _ptr(weights)))
        return u0

    def sync_status(self):
        return self._s(lib().mppi_sync_status(self.h))

    def set_tracking_cost(self, c: dict):
        """Eq. 3 / Eq. 4 cost parameters (controller created with cost="tracking")."""
        self._s(lib().mppi_set_tracking_cost(self.h, C.byref(tracking_struct(c))))

    def step_proposal(self, x0, center, sd, k_prop, u0=None, gate="cost"):
        """One control step sampling k_prop knots around an explicit proposal (mean, std).
        gate "cost": the update keeps the proposal only if its centre costs no more than the
        nominal, and runs the plain step's K samples otherwise (decided on the device);
        "best": the same with the proposal's least sample cost other than the nominal's;
        "cost-concurrent" / "best-concurrent": the same gates with both sample sets rolled
        out in one launch on every step; "none": the proposal's samples alone."""
        import torch
        u0 = u0 if u0 is not None else torch.empty(12, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_step_proposal(self.h, _ptr(x0), _ptr(center), _ptr(sd), int(k_prop), GATE[gate],
                                         _ptr(u0)))
        return u0

    def set_proposal(self, policy, k_prop=0, cmd=(0.0, 0.0, 0.0), origin=(0.0, 0.0), gate="cost"):
        """Route later step() calls through the learned proposal (policy None: plain MPPI)."""
        c = np.ascontiguousarray(cmd, dtype=np.float32)
        o = np.ascontiguousarray(origin, dtype=np.float32)
        self._s(lib().mppi_set_proposal(self.h, policy.h if policy is not None else None, int(k_prop), GATE[gate],
                                        c.ctypes.data_as(C.c_void_p), o.ctypes.data_as(C.c_void_p)))
        self._policy = policy  # keep alive while in use

    def proposal_stats(self):
        """(accepted, proposal steps): device counters, read with a synchronisation."""
        a, n = C.c_int(), C.c_int()
        self._s(lib().mppi_proposal_stats(self.h, C.byref(a), C.byref(n)))
        return a.value, n.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mppi_destroy(self.h)
            self.h = None


N_POLICY_PARAMS = 882832


def policy_pairs(records, origin_cmd, n_knots, fall_z, stream=None):
    """mppi_policy_pairs: training pairs of closed-loop records (device tensor
    n_rec x steps x (37 + 12 n_knots)) with origins and commands (n_rec x 3).  Returns
    features (n_rec x steps x 40), targets (n_rec x steps x 72) and the pair count of each
    record (device tensors; rows past a record's count are not written)."""
    import torch
    n_rec, steps, w = records.shape
    assert w == 37 + 12 * n_knots and tuple(origin_cmd.shape) == (n_rec, 3)
    feat = torch.empty((n_rec, steps, 40), dtype=torch.float32, device="cuda")
    tgt = torch.empty((n_rec, steps, 72), dtype=torch.float32, device="cuda")
    count = torch.empty(n_rec, dtype=torch.int32, device="cuda")
    status = lib().mppi_policy_pairs(n_rec, steps, n_knots, _ptr(records), _ptr(origin_cmd), float(fall_z),
                                     _ptr(feat), _ptr(tgt), _ptr(count), _stream(stream))
    if status < 0:
        raise MppiError(status, lib().mppi_policy_last_error(None).decode())
    return feat, tgt, count


class Policy:
    """Learned proposal network (include/mppi_policy.h) on a torch-allocated workspace."""

    def __init__(self, max_batch=4096, seed=0, ckpt=None, stream=None):
        import torch
        L = lib()
        h = C.c_void_p()
        rc = L.mppi_policy_create(ckpt.encode() if ckpt else None, int(seed) & 0xFFFFFFFFFFFFFFFF, int(max_batch),
                                  C.byref(h))
        if rc < 0:
            raise MppiError(rc, L.mppi_policy_last_error(None).decode())
        self.h = h
        self.max_batch = int(max_batch)
        nbytes = L.mppi_policy_workspace_bytes(h)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off:off + nbytes]
        self.stream = stream
        self._s(L.mppi_policy_bind(h, C.c_void_p(self.ws_view.data_ptr()), nbytes, _stream(stream)))
        self._norm = self.get_normalization()

    def _s(self, status):
        if status < 0:
            raise MppiError(status, lib().mppi_policy_last_error(self.h).decode())
        return status

    def set_normalization(self, in_mean, in_std, out_mean, out_std):
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (in_mean, in_std, out_mean, out_std)]
        assert [a.size for a in arrs] == [40, 40, 72, 72]
        self._s(lib().mppi_policy_set_normalization(self.h, *[a.ctypes.data_as(C.c_void_p) for a in arrs]))
        self._norm = tuple(a.astype(np.float64) for a in arrs)

    def get_normalization(self):
        arrs = [np.zeros(n, np.float32) for n in (40, 40, 72, 72)]
        self._s(lib().mppi_policy_get_normalization(self.h, *[a.ctypes.data_as(C.c_void_p) for a in arrs]))
        return tuple(a.astype(np.float64) for a in arrs)

    def get_params(self):
        import torch
        out = torch.empty(N_POLICY_PARAMS, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_policy_get_params(self.h, _ptr(out)))
        return out

    def set_params(self, P):
        self._s(lib().mppi_policy_set_params(self.h, _ptr(P)))

    def forward(self, X):
        import torch
        out = torch.empty((X.shape[0], 144), dtype=torch.float32, device="cuda")
        self._s(lib().mppi_policy_forward(self.h, _ptr(X), int(X.shape[0]), _ptr(out)))
        return out

    def grad(self, X, Y, index=None, B=None):
        """Loss and gradient over rows index[:B] of X and Y (int32 device indices, each a
        valid row; they are not checked on the host) or the first B rows."""
        import torch
        assert index is None or index.dtype == torch.int32
        B = int(B if B is not None else (index.shape[0] if index is not None else X.shape[0]))
        G = torch.empty(N_POLICY_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_policy_grad(self.h, _ptr(X), _ptr(Y), _ptr(index), B, _ptr(G), _ptr(loss)))
        return loss, G

    def nll(self, X, Y, index=None, B=None):
        """The loss alone (mppi_policy_nll) over rows index[:B] of X and Y (as grad): a
        device tensor of one float."""
        import torch
        assert index is None or index.dtype == torch.int32
        B = int(B if B is not None else (index.shape[0] if index is not None else X.shape[0]))
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_policy_nll(self.h, _ptr(X), _ptr(Y), _ptr(index), B, _ptr(loss)))
        return loss

    def adam(self, G, lr):
        self._s(lib().mppi_policy_adam(self.h, _ptr(G), float(lr)))

    def train_step(self, X, Y, index=None, B=None, lr=1e-3, loss=None):
        """Gradient then Adam over rows index[:B] of X and Y (as grad)."""
        import torch
        assert index is None or index.dtype == torch.int32
        B = int(B if B is not None else (index.shape[0] if index is not None else X.shape[0]))
        loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_policy_train_step(self.h, _ptr(X), _ptr(Y), _ptr(index), B, float(lr), _ptr(loss)))
        return loss

    @property
    def steps(self):
        return lib().mppi_policy_steps(self.h)

    def save(self, path):
        self._s(lib().mppi_policy_save(self.h, str(path).encode()))

    def head(self, out_row, nk, sigma_max):
        import torch
        c = torch.empty(12 * nk, dtype=torch.float32, device="cuda")
        sd = torch.empty(12 * nk, dtype=torch.float32, device="cuda")
        self._s(lib().mppi_policy_head(self.h, _ptr(out_row), int(nk), float(sigma_max), _ptr(c), _ptr(sd)))
        return c, sd

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mppi_policy_destroy(self.h)
            self.h = None


class Batch:
    """Batched serving of many MPPI instances (one graph launch per control step)."""

    def __init__(self, max_instances, budget_bytes, max_horizon=80, max_hf_cells=4096, arith="fp64", stream=None):
        import torch
        L = lib()
        if not hasattr(L, "_batch_sigs"):
            vp = C.c_void_p
            sig = {
                "mppi_batch_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
                "mppi_batch_destroy": (None, [vp]),
                "mppi_batch_control_bytes": (C.c_size_t, [C.c_int, C.c_int]),
                "mppi_batch_bind": (C.c_int, [vp, vp, C.c_size_t, vp]),
                "mppi_batch_add_model": (C.c_int, [vp, vp, C.POINTER(C.c_int)]),
                "mppi_batch_admit": (C.c_int, [vp, C.c_int, C.POINTER(Params), vp, vp, C.POINTER(C.c_int)]),
                "mppi_batch_remove": (C.c_int, [vp, C.c_int]),
                "mppi_batch_step": (C.c_int, [vp]),
                "mppi_batch_record": (C.c_int, [vp, C.c_int, vp, C.c_int]),
                "mppi_batch_set_tuning": (C.c_int, [vp, C.c_int, C.c_int]),
                "mppi_batch_set_launch_mode": (C.c_int, [vp, C.c_int]),
                "mppi_batch_get_tuning": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
                "mppi_batch_autotune": (C.c_int, [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                                  C.POINTER(C.c_float)]),
                "mppi_batch_read": (C.c_int, [vp, C.c_int, vp, vp, vp, vp, vp]),
                "mppi_batch_stats": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_size_t),
                                               C.POINTER(C.c_size_t)]),
                "mppi_batch_last_error": (C.c_char_p, [vp]),
                "mppi_batch_set_proposal": (C.c_int, [vp, C.c_int, vp, vp, vp]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            L._batch_sigs = True
        self.L = L
        h = C.c_void_p()
        self._chk(L.mppi_batch_create(max_instances, max_horizon, max_hf_cells, ARITH[arith], C.byref(h)))
        self.h = h
        ctrl = L.mppi_batch_control_bytes(max_instances, ARITH[arith])
        total = ctrl + int(budget_bytes)
        self.ws = torch.empty(total + 256, dtype=torch.uint8, device="cuda")
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off:off + total]
        self.models = []
        self._chk(L.mppi_batch_bind(h, C.c_void_p(self.ws_view.data_ptr()), total, _stream(stream)))

    def _chk(self, status):
        if status < 0:
            raise MppiError(status, self.L.mppi_batch_last_error(getattr(self, "h", None)).decode())
        return status

    def add_model(self, model: "Model") -> int:
        slot = C.c_int()
        self._chk(self.L.mppi_batch_add_model(self.h, model.h, C.byref(slot)))
        self.models.append(model)
        return slot.value

    def admit(self, slot: int, p: dict, x0, mu):
        """Returns the instance id, or None if it does not fit in the budget."""
        ps = params_struct(p)
        x0 = np.ascontiguousarray(x0, dtype=np.float32)
        mu = np.ascontiguousarray(mu, dtype=np.float32)
        i = C.c_int()
        rc = self.L.mppi_batch_admit(self.h, slot, C.byref(ps), x0.ctypes.data_as(C.c_void_p),
                                     mu.ctypes.data_as(C.c_void_p), C.byref(i))
        if rc == -5:
            return None
        self._chk(rc)
        return i.value

    def remove(self, i):
        self._chk(self.L.mppi_batch_remove(self.h, int(i)))
        getattr(self, "_records", {}).pop(i, None)
        getattr(self, "_policies", {}).pop(i, None)

    def step(self):
        self._chk(self.L.mppi_batch_step(self.h))

    def record(self, i, rec=None):
        """Record [x_s, mu'_s] of instance i into the device tensor rec (cap x (nx + 12 nk),
        float32) from the next step on; rec None stops.  The tensor is kept alive here."""
        if rec is not None:
            assert rec.dtype.is_floating_point and rec.element_size() == 4 and rec.dim() == 2
        self._chk(self.L.mppi_batch_record(self.h, int(i), _ptr(rec), int(rec.shape[0]) if rec is not None else 0))
        self._records = getattr(self, "_records", {})
        if rec is None:
            self._records.pop(i, None)
        else:
            self._records[i] = rec

    def set_proposal(self, i, policy=None, cmd=(0.0, 0.0, 0.0), origin=(0.0, 0.0)):
        """Instance i takes its K samples from the policy (ungated), or plain samples again
        with policy None.  Every proposal instance shares one policy; it is kept alive here."""
        c = np.ascontiguousarray(cmd, dtype=np.float32)
        o = np.ascontiguousarray(origin, dtype=np.float32)
        assert c.shape == (3,) and o.shape == (2,)
        self._chk(self.L.mppi_batch_set_proposal(self.h, int(i), policy.h if policy is not None else None,
                                                 c.ctypes.data_as(C.c_void_p), o.ctypes.data_as(C.c_void_p)))
        self._policies = getattr(self, "_policies", {})
        if policy is None:
            self._policies.pop(i, None)
        else:
            self._policies[i] = policy

    def set_tuning(self, blocks_per_cu, order):
        self._chk(self.L.mppi_batch_set_tuning(self.h, blocks_per_cu, order))

    def set_launch_mode(self, mode):
        """0: one persistent kernel per scene; 1: one kernel over a queue of every scene's tiles."""
        self._chk(self.L.mppi_batch_set_launch_mode(self.h, int(mode)))

    def tuning(self):
        """(blocks_per_cu, order, launch mode) now in effect."""
        bb, bo, bm = C.c_int(), C.c_int(), C.c_int()
        self._chk(self.L.mppi_batch_get_tuning(self.h, C.byref(bb), C.byref(bo), C.byref(bm)))
        return bb.value, bo.value, bm.value

    def autotune(self, steps=3):
        """Times the 16 candidate tunings (the launch mode too) and keeps the fastest;
        returns (blocks_per_cu, order, ms per step); tuning() also gives the mode."""
        bb, bo, ms = C.c_int(), C.c_int(), C.c_float()
        self._chk(self.L.mppi_batch_autotune(self.h, steps, C.byref(bb), C.byref(bo), C.byref(ms)))
        return bb.value, bo.value, ms.value

    def read(self, i, nx, nk):
        x, u0, mu = np.zeros(nx, np.float32), np.zeros(12, np.float32), np.zeros(12 * nk, np.float32)
        acc, step = np.zeros(1, np.float32), np.zeros(1, np.uint32)
        vp = lambda a: a.ctypes.data_as(C.c_void_p)
        self._chk(self.L.mppi_batch_read(self.h, int(i), vp(x), vp(u0), vp(mu), vp(acc), vp(step)))
        return x, u0, mu, float(acc[0]), int(step[0])

    def stats(self):
        n, t, u, pool = C.c_int(), C.c_int(), C.c_size_t(), C.c_size_t()
        self._chk(self.L.mppi_batch_stats(self.h, C.byref(n), C.byref(t), C.byref(u), C.byref(pool)))
        return dict(live=n.value, tiles=t.value, bytes_used=u.value, bytes_pool=pool.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mppi_batch_destroy(self.h)
            self.h = None
