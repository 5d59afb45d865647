"""The control step that allocates nothing (mppi_step_static), through the C ABI: two
calls in a row on unbound controllers -- the box push at its full shape (K=4096, H=60),
then a smaller heightfield walk (K=512, H=30) -- equal, bit for bit, the step of the same
controller bound to its own workspace (mppi_step): same kernels on the same inputs."""
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


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).cuda().contiguous()


def test_static_step_equals_the_bound_step_twice_second_smaller(B):
    for wl, over, step in ((W.BOX_PUSH, {}, 3), (W.TERRAIN_WALK, dict(K=512, H=30), 7)):
        print("case:", wl["name"], over, flush=True)
        md = W.model_dict(wl, 0)
        p = W.params_dict(wl, 0, arith="fp32", **over)
        model = B.Model(md)
        bound = B.Controller(model, p)
        static = B.Controller(model, p, bind=False)
        x0 = _dev(W.initial_state(1, wl["scene"]))
        mu = _dev(W.stance_knots(p["nk"]) + np.random.default_rng(step).uniform(-0.05, 0.05, 12 * p["nk"]))
        bound.set_nominal(mu)
        bound.set_step(step)
        u_ref = bound.step(x0).cpu().numpy()
        nom_ref = bound.get_nominal().cpu().numpy()
        assert bound.sync_status() == 0
        nominal = mu.clone()
        static.set_step(step)
        u = static.step_static(x0, nominal)
        torch.cuda.synchronize()
        assert static.step_counter == step + 1
        assert np.array_equal(u.cpu().numpy(), u_ref)
        assert np.array_equal(nominal.cpu().numpy(), nom_ref)


def test_static_step_rejects_a_bound_controller_and_oversized_workspaces(B):
    md = W.model_dict(W.FLAT_WALK, 0)
    model = B.Model(md)
    p = W.params_dict(W.FLAT_WALK, 0)
    x0 = _dev(W.initial_state(0))
    nominal = _dev(W.stance_knots(p["nk"]))
    with pytest.raises(B.MppiError):
        B.Controller(model, p).step_static(x0, nominal)
    big = B.Controller(model, dict(p, K=1 << 16, H=60, nk=60, basis=3, dt=0.01), bind=False)
    with pytest.raises(B.MppiError, match="static scratch"):
        big.step_static(x0, nominal)
