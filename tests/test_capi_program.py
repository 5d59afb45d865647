"""A plain C program against the C ABI (tests/capi/closed_loop.c): it compiles and links
with gcc against libmppi.so and the HIP runtime alone (CPU), and on the GPU its closed
loop equals, bit for bit, the same calls made through the Python binding."""
import os
import subprocess

import numpy as np
import pytest

from paper_2409_10469_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2409_10469_amd")
SRC = os.path.join(ROOT, "tests", "capi", "closed_loop.c")


def _build(out):
    if not os.path.exists(os.path.join(PKG, "libmppi.so")):
        pytest.skip("libmppi.so is not built")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), SRC, "-L" + PKG, "-lmppi", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath," + PKG + ":/opt/rocm/lib", "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return str(out)


def test_c_program_compiles_against_the_abi(tmp_path):
    exe = _build(tmp_path / "closed_loop")
    assert os.access(exe, os.X_OK)


def _input(wl, seed, steps):
    R = W.ROBOT
    p = W.params_dict(wl, seed, K=128, H=20, instance=5)
    model = [*R["trunk_size"], R["trunk_mass"], R["hip_x"], R["hip_y"], R["thigh_len"], R["thigh_mass"],
             R["calf_len"], R["calf_mass"], R["foot_r"], R["gravity"], R["k"], R["c"], R["mu"], R["vs"]]
    params = [p["K"], p["H"], p["nk"], p["dt"], p["sigma"], p["lam"], p["kp"], p["kd"], p["w_h"], p["h_ref"], p["w_o"],
              p["w_v"], p["v_ref"], p["w_tau"], p["seed"], p["instance"]]
    x0 = np.float32(W.initial_state(seed))
    mu = np.float32(W.stance_knots(p["nk"]))
    text = "\n".join([" ".join(repr(float(np.float32(v))) for v in model),
                      " ".join(repr(float(v)) if isinstance(v, float) else str(v) for v in params), str(steps),
                      " ".join(repr(float(v)) for v in x0), " ".join(repr(float(v)) for v in mu)])
    return text, p, x0, mu


@pytest.mark.gpu
def test_c_program_closed_loop_equals_the_binding(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10469_amd import binding as B
    exe = _build(tmp_path / "closed_loop")
    wl, seed, steps = W.FLAT_WALK, 3, 15
    text, p, x0, mu = _input(wl, seed, steps)
    (tmp_path / "in.txt").write_text(text)
    r = subprocess.run([exe, str(tmp_path / "in.txt")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    vals = np.array([float(v) for v in r.stdout.split()], dtype=np.float32)
    cx, cu = vals[:37], vals[37:49]
    # the same calls through the binding
    p = dict(p, dt=float(np.float32(p["dt"])))
    model = B.Model(W.model_dict(wl, 0))
    ctl = B.Controller(model, p)
    ctl.set_nominal(torch.tensor(mu, device="cuda"))
    x = torch.tensor(x0, device="cuda")
    xn = torch.empty_like(x)
    u0 = torch.empty(12, dtype=torch.float32, device="cuda")
    for _ in range(steps):
        ctl.step(x, u0)
        model.sim_step_into(x.view(1, -1), u0.view(1, -1), p["kp"], p["kd"], p["dt"], xn.view(1, -1))
        x, xn = xn, x
    np.testing.assert_array_equal(cx, x.cpu().numpy())
    np.testing.assert_array_equal(cu, u0.cpu().numpy())
