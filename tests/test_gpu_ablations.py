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
def test_held_plan_follows_the_shifted_knots(B, basis):
    """Between replans the applied controls are the first knots of the plan advanced by
    the shift: with the zeroth-order hold (shift = identity) they stay the replan's u0."""
    from paper_2409_10469_amd import ablations as AB
    wl = W.TERRAIN_WALK
    model = B.Model(W.model_dict(wl, 0))
    p = dict(W.params_dict(wl, 1, K=64), basis=basis)
    c, x = AB.episode_held(model, p, 1, 24, hold=4)
    assert np.isfinite(c) and np.isfinite(x).all()
    ctl = B.Controller(model, p)
    _, S = ctl.basis_matrices()
    if basis == 2:
        np.testing.assert_array_equal(S, np.eye(p["nk"], dtype=np.float32))
