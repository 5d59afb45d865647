"""The ablation harness on the GPU: replanning at a lower control rate, and the
consistency of its settings with the plain closed loop."""
import numpy as np
import pytest

from paper_2409_10469_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10469_amd import binding
    binding.lib()
    return binding


def test_replanning_every_step_is_the_plain_closed_loop(B):
    from paper_2409_10469_amd import ablations as AB
    from paper_2409_10469_amd import proposal as PR
    wl = W.TERRAIN_WALK
    model = B.Model(W.model_dict(wl, 0))
    p = W.params_dict(wl, 3, K=128)
    c1, x1, _, _ = PR.episode(model, p, 3, 30)
    c2, x2 = AB.episode_held(model, p, 3, 30, hold=1)
    assert c1 == c2 and np.array_equal(x1, x2)


@pytest.mark.parametrize("basis", [0, 1, 2])
def test_held_plan_follows_the_oracle_shift_chain(B, basis):
    """Replanning every 4 plant steps with each knot interpolation: a replan's first
    control and nominal equal the oracle's Algorithm 1 step from the same state, nominal
    and Philox step, and the held steps apply the first knot of S^j mu' -- the oracle's
    shift matrix applied j times to the replan's update."""
    from oracle import oracle as O
    from paper_2409_10469_amd import ablations as AB
    from tests.parity_utils import KNOT_TOL, round_model, round_params
    wl = W.TERRAIN_WALK
    md = round_model(W.model_dict(wl, 0))
    model = B.Model(md)
    p = round_params(dict(W.params_dict(wl, 1, K=64), basis=basis))
    trace = []
    c, x = AB.episode_held(model, p, 1, 16, hold=4, trace=trace)
    assert np.isfinite(c) and np.isfinite(x).all()
    orc = O.Oracle(md)
    S = O.shift_matrix_b(basis, p["nk"], p["H"], p["dt"])
    replans = 0
    for t, replan, xs, before, u in trace:
        if replan:
            ou0, omu, _, rc = orc.mppi_step(dict(p, seed=1), replans, xs.astype(np.float64),
                                           before.astype(np.float64))
            assert rc == 0
            assert np.abs(u - ou0).max() <= KNOT_TOL, (t, basis)
            plan = omu.reshape(12, p["nk"])  # S mu'
            replans += 1
            j = 1
        else:
            # held step j after the replan applies the first knot of S^j mu'
            assert np.abs(u - plan[:, 0]).max() <= KNOT_TOL, (t, basis, j)
            plan = plan @ S.T
            j += 1
    assert replans == 4
    if basis == 2:  # the zeroth-order hold's shift is the identity: the replan's u0 is held
        np.testing.assert_array_equal(S, np.eye(p["nk"]))


def test_fine_control_rate_sweep_runs_at_250_hz(B):
    """The 4 ms plant and controller: replanning every step (250 Hz) is the plain closed
    loop at dt = 4 ms, and a short sweep returns finite costs for every rate."""
    from paper_2409_10469_amd import ablations as AB
    from paper_2409_10469_amd import proposal as PR
    wl = W.TERRAIN_WALK
    model = B.Model(W.model_dict(wl, 0))
    p = dict(W.params_dict(wl, 2, K=128), dt=0.004, H=125)
    c1, x1, _, _ = PR.episode(model, p, 2, 40)
    c2, x2 = AB.episode_held(model, p, 2, 40, hold=1)
    assert c1 == c2 and np.array_equal(x1, x2)
    res = AB.control_rate_sweep(seeds=range(1), fine=dict(AB.RATE_FINE, holds=[1, 2, 25], seconds=0.2),
                                log=lambda *a: None)
    assert set(res["values"]) == {"250", "125", "10"}
    assert all(np.isfinite(v["mean"]) for v in res["values"].values())
