"""The C-ABI library loads and exports every entry point its header declares; host-side
validation rejects bad descriptions without touching a GPU (CPU only)."""
import ctypes as C
import os
import re

import pytest

from paper_2409_10469_amd import binding as B
from paper_2409_10469_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


def _declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(mppi_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = C.CDLL(B.LIB_PATH)
    names = _declared()
    assert len(names) >= 50
    for n in names:
        assert hasattr(L, n), n


def test_policy_host_validation_and_checkpoint_errors(tmp_path):
    L = B.lib()
    assert L.mppi_policy_n_params() == B.N_POLICY_PARAMS
    h = C.c_void_p()
    assert L.mppi_policy_create(None, 0, 0, C.byref(h)) == B.EINVAL and not h.value
    assert L.mppi_policy_create(None, 0, 70000, C.byref(h)) == B.EINVAL
    assert L.mppi_policy_create(str(tmp_path / "missing").encode(), 0, 16, C.byref(h)) == B.EINVAL
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"MPPIPOL1" + b"\0" * 64)
    assert L.mppi_policy_create(str(bad).encode(), 0, 16, C.byref(h)) == B.EINVAL
    assert L.mppi_policy_create(None, 7, 256, C.byref(h)) == B.OK and h.value
    # calls that need a bound workspace refuse without one
    assert L.mppi_policy_forward(h, None, 1, None) == B.ESTATE
    assert L.mppi_policy_save(h, b"x") == B.ESTATE
    one = (C.c_float * 72)(*([1.0] * 72))
    zero = (C.c_float * 72)()
    assert L.mppi_policy_set_normalization(h, one, zero, one, one) == B.EINVAL  # zero input std
    assert L.mppi_policy_set_normalization(h, zero, one, zero, one) == B.OK
    assert L.mppi_policy_workspace_bytes(h) > 4 * 4 * B.N_POLICY_PARAMS
    L.mppi_policy_destroy(h)


def _model_handle(**over):
    d = W.model_dict(W.FLAT_WALK, 0)
    d.update(over)
    desc, keep = B.model_desc(d)
    h = C.c_void_p()
    rc = B.lib().mppi_model_create(C.byref(desc), C.byref(h))
    return rc, h


@pytest.mark.parametrize("over", [dict(trunk_mass=0.0), dict(k=-1.0), dict(scene=7), dict(calf_len=float("nan"))])
def test_model_validation(over):
    rc, h = _model_handle(**over)
    assert rc == B.EINVAL and not h.value
    assert B.lib().mppi_last_error(None)


def test_heightfield_validation():
    import numpy as np
    d = W.model_dict(W.TERRAIN_WALK, 0)
    d["hf"] = np.zeros((200, 200))  # larger than the LDS-staged maximum
    desc, keep = B.model_desc(d)
    h = C.c_void_p()
    assert B.lib().mppi_model_create(C.byref(desc), C.byref(h)) == B.EINVAL


@pytest.mark.parametrize("over", [dict(K=0), dict(H=0), dict(H=1000), dict(nk=1), dict(nk=9), dict(dt=0.0),
                                  dict(lam=0.0), dict(sigma=-1.0), dict(kd=-1.0), dict(basis=3), dict(basis=-1)])
def test_params_validation(over):
    rc, mh = _model_handle()
    assert rc == 0
    p = W.params_dict(W.FLAT_WALK, 0)
    p.update(over)
    ps = B.params_struct(p)
    h = C.c_void_p()
    assert B.lib().mppi_create(mh, C.byref(ps), C.byref(h)) == B.EINVAL
    assert not h.value
    B.lib().mppi_model_destroy(mh)


def test_workspace_size_and_unbound_calls():
    rc, mh = _model_handle()
    p = W.params_dict(W.FLAT_WALK, 0)
    ps = B.params_struct(p)
    h = C.c_void_p()
    assert B.lib().mppi_create(mh, C.byref(ps), C.byref(h)) == 0
    nbytes = B.lib().mppi_workspace_bytes(h)
    D, K = 12 * p["nk"], p["K"]
    assert nbytes >= 4 * (D * K + 2 * K + D + p["H"] * p["nk"])
    # launching calls before a workspace is bound fail without launching
    assert B.lib().mppi_step(h, C.c_void_p(256), C.c_void_p(512)) == B.ESTATE
    assert B.lib().mppi_rollout_batch(h, C.c_void_p(256), None, C.c_void_p(512), None) == B.ESTATE
    # misaligned or short workspaces are refused before any copy
    assert B.lib().mppi_bind(h, C.c_void_p(4096 + 4), nbytes, None) == B.EINVAL
    assert B.lib().mppi_bind(h, C.c_void_p(4096), nbytes - 1, None) == B.ENOMEM
    assert B.lib().mppi_set_step(h, 5) == 0 and B.lib().mppi_get_step(h) == 5
    B.lib().mppi_destroy(h)
    B.lib().mppi_model_destroy(mh)


def test_box_scene_validation():
    rc, h = _model_handle(scene=W.SCENE_FREE_BOX, box_half=(0.2, 0.2, 0.15), box_mass=2.0)
    assert rc == 0 and B.lib().mppi_model_nx(h) == 50
    B.lib().mppi_model_destroy(h)
    rc, h = _model_handle(scene=W.SCENE_FREE_BOX, box_half=(0.2, 0.2, 0.15), box_mass=0.0)
    assert rc == B.EINVAL
    rc, h = _model_handle(scene=W.SCENE_STATIC_BOX, sbox_center=(1.1, 0, 0.15), sbox_half=(0.5, 0.5, 0.15))
    assert rc == 0 and B.lib().mppi_model_nx(h) == 37
    B.lib().mppi_model_destroy(h)
    rc, h = _model_handle(scene=W.SCENE_STATIC_BOX, sbox_center=(1.1, 0, 0.15), sbox_half=(0.5, -0.5, 0.15))
    assert rc == B.EINVAL


def test_batch_create_validation():
    L = B.lib()
    vp = C.c_void_p
    L.mppi_batch_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(vp)]
    L.mppi_batch_control_bytes.restype = C.c_size_t
    L.mppi_batch_control_bytes.argtypes = [C.c_int, C.c_int]
    h = vp()
    assert L.mppi_batch_create(0, 80, 4096, 0, C.byref(h)) == B.EINVAL
    assert L.mppi_batch_create(16, 0, 4096, 0, C.byref(h)) == B.EINVAL
    assert L.mppi_batch_create(16, 80, 4096, 5, C.byref(h)) == B.EINVAL
    assert L.mppi_batch_create(16, 256, 14336, 0, C.byref(h)) == B.EINVAL  # LDS stage over 64 KiB
    assert L.mppi_batch_control_bytes(16, 0) > 16 * 256


def test_proposal_calls_reject_a_null_context():
    L = B.lib()
    assert L.mppi_step_proposal(None, None, None, None, 16, 0, None) == B.EINVAL
    assert L.mppi_set_proposal(None, None, 16, 0, None, None) == B.EINVAL
    assert L.mppi_proposal_stats(None, None, None) == B.EINVAL
    assert L.mppi_batch_set_proposal(None, 0, None, None, None) == B.EINVAL


@pytest.mark.parametrize("basis", [0, 1, 2])
@pytest.mark.parametrize("nk,H,dt", [(2, 10, 0.02), (4, 25, 0.02), (6, 50, 0.01), (8, 60, 0.01), (5, 80, 0.01)])
def test_library_basis_and_shift_equal_the_oracle(basis, nk, H, dt):
    """The controller's host-built interpolation and shift matrices against the oracle's,
    from the same FP32 dt (so knot-time steps of the zeroth-order hold are decided alike)."""
    import numpy as np
    from oracle import oracle as O
    rc, mh = _model_handle()
    p = W.params_dict(W.FLAT_WALK, 0, K=8, H=H, nk=nk)
    p["basis"], p["dt"] = basis, float(np.float32(dt))
    ps = B.params_struct(p)
    h = C.c_void_p()
    assert B.lib().mppi_create(mh, C.byref(ps), C.byref(h)) == 0
    Bm = np.zeros((H, nk))
    Sm = np.zeros((nk, nk), dtype=np.float32)
    assert B.lib().mppi_get_basis(h, Bm.ctypes.data_as(C.c_void_p), Sm.ctypes.data_as(C.c_void_p)) == 0
    np.testing.assert_allclose(Bm, O.basis_matrix(basis, nk, H, p["dt"]), atol=1e-12)
    np.testing.assert_allclose(Sm, O.shift_matrix_b(basis, nk, H, p["dt"]), atol=1e-6)
    assert B.lib().mppi_get_basis(None, None, None) == B.EINVAL
    B.lib().mppi_destroy(h)
    B.lib().mppi_model_destroy(mh)


def test_tracking_workspace_holds_the_trajectories():
    rc, mh = _model_handle()
    p = W.params_dict(W.FLAT_WALK, 0)
    sizes = []
    for extra in ({}, dict(cost="tracking")):
        ps = B.params_struct(dict(p, **extra))
        h = C.c_void_p()
        assert B.lib().mppi_create(mh, C.byref(ps), C.byref(h)) == 0
        sizes.append(B.lib().mppi_workspace_bytes(h))
        B.lib().mppi_destroy(h)
    assert sizes[1] - sizes[0] >= 4 * p["K"] * (p["H"] + 1) * 37
    ps = B.params_struct(p)
    ps.cost = 2
    h = C.c_void_p()
    assert B.lib().mppi_create(mh, C.byref(ps), C.byref(h)) == B.EINVAL
    B.lib().mppi_model_destroy(mh)


@pytest.mark.parametrize("bad", [dict(duty=1.0), dict(duty=0.0), dict(period=0.0), dict(stand_height=0.0),
                                 dict(swing_height=-0.01), dict(box_w=-1.0), dict(gait=2), dict(reserved=1),
                                 dict(Q=[1.0] * 35 + [-1.0]), dict(R=[float("nan")] + [1.0] * 11),
                                 dict(v_cmd=(float("inf"), 0.0))])
def test_tracking_cost_validation(bad):
    rc, mh = _model_handle()
    p = W.params_dict(W.FLAT_WALK, 0, cost="tracking")
    ps = B.params_struct(p)
    h = C.c_void_p()
    assert B.lib().mppi_create(mh, C.byref(ps), C.byref(h)) == 0
    good = W.tracking_cost()
    assert B.lib().mppi_set_tracking_cost(h, C.byref(B.tracking_struct(good))) == 0
    assert B.lib().mppi_set_tracking_cost(h, C.byref(B.tracking_struct(dict(good, **bad)))) == B.EINVAL
    # unbound: the rollout refuses before launching
    assert B.lib().mppi_rollout_batch(h, C.c_void_p(256), None, C.c_void_p(512), None) == B.ESTATE
    B.lib().mppi_destroy(h)
    # a running-cost controller refuses tracking parameters
    ps = B.params_struct(W.params_dict(W.FLAT_WALK, 0))
    assert B.lib().mppi_create(mh, C.byref(ps), C.byref(h)) == 0
    assert B.lib().mppi_set_tracking_cost(h, C.byref(B.tracking_struct(good))) == B.EINVAL
    B.lib().mppi_destroy(h)
    B.lib().mppi_model_destroy(mh)
