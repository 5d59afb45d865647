"""GPU parity of the lane-split rollout (16 lanes per sample) against the FP64 oracle,
through the C ABI, at the quad kernel's bars:
  per-step state error <= 1e-5 relative per block (FP64 step) from the GPU's own states;
  rollout costs within 1e-4 relative over 10-step horizons;
  updated knots within 1e-3;
and its costs equal to the quad kernel's up to summation order.  The other arithmetics
are held to bounds derived from the oracle before any GPU result:
  MIXED (FP32 kinematics and contact geometry, FP64 implicit system): 8 times the
    oracle's one-ulp input sensitivity of the step (parity_utils.mixed_step_bound);
  FP32 (everything in FP32): the backward-stable solve bound kappa_2(A) 2 (n + 1) u |dv|
    of the step's implicit systems (parity_utils.fp32_step_bound).
Per-step states are compared from identical FP32 inputs; the costs of FP32-state
trajectories are checked as sums of the oracle's stage costs of the GPU's own states."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W
from tests.parity_utils import (COST_TOL, KNOT_TOL, STEP_TOL, box_contact_states, f32, fp32_step_bound,
                                mixed_step_bound, r16_knot_sensitivity, random_walk_states, round_model,
                                round_params, step_error)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10469_amd import binding
    binding.lib()
    return binding


def _setup(B, workload, seed=0, **pover):
    md = round_model(W.model_dict(workload, seed))
    p = round_params(W.params_dict(workload, seed, **pover))
    p.setdefault("lanes", 16)
    orc = O.Oracle(md)
    model = B.Model(md)
    ctl = B.Controller(model, p)
    return md, p, orc, model, ctl


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).cuda().contiguous()


def _say(*a):
    print("case:", *a, flush=True)


@pytest.mark.parametrize("workload,K", [(W.FLAT_WALK, 64), (W.FLAT_WALK, 50), (W.TERRAIN_WALK, 48),
                                        (W.BOX_CLIMB, 33), (W.BOX_PUSH, 21)])
def test_split_rollout_costs_10_steps(B, workload, K):
    _say("split 10-step costs", workload["name"], K)
    md, p, orc, model, ctl = _setup(B, workload, K=K, H=10, lanes=16)
    x0 = f32(W.initial_state(3, workload["scene"]))
    if workload["scene"] == W.SCENE_FREE_BOX:
        x0 = box_contact_states(1, seed=5)[0]
    mu = f32(W.stance_knots(p["nk"]) + np.random.default_rng(2).uniform(-0.1, 0.1, 12 * p["nk"]))
    eps = f32(W.explicit_noise(5, K, p["nk"]))
    ctl.set_nominal(_dev(mu))
    costs, traj = ctl.rollout_batch(_dev(x0), eps=_dev(eps), traj=True)
    got = costs.cpu().numpy().astype(np.float64)
    want = orc.rollout_batch(p, x0, mu, eps)
    assert np.isfinite(want).all()
    rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-6)
    assert rel.max() <= COST_TOL, (rel.max(), int(rel.argmax()))
    tr = traj.cpu().numpy().astype(np.float64)
    assert np.array_equal(tr[:, 0], np.broadcast_to(x0, tr[:, 0].shape))


def _chain(orc, p, mu, eps, tr, costs, samples, box=False, every=1):
    Bm = O.spline_basis(p["nk"], p["H"], p["dt"])
    for n in samples:
        theta = mu + (p["sigma"] * eps[n] if n else 0.0)
        U = Bm @ theta.reshape(12, p["nk"]).T
        L = 0.0
        for k in range(p["H"]):
            if not np.isfinite(tr[n, k + 1]).all():
                break
            xn, tau, _ = orc.step(tr[n, k], U[k], p["kp"], p["kd"], p["dt"])
            if k % every == 0:
                assert step_error(tr[n, k + 1], xn, box=box).max() <= STEP_TOL, (n, k)
            L += p["dt"] * orc.stage_cost(p, tr[n, k + 1], tau)
        else:
            if every == 1:
                assert abs(costs[n] - L) <= COST_TOL * max(abs(L), 1e-6), n


def test_split_heightfield_full_size_chain(B):
    """The heightfield walk at its launch shape (K=1024, H=50): sampled samples are chains
    of oracle steps taken from the GPU's own states, and their costs sum those steps."""
    _say("split heightfield K=1024 H=50 chain")
    md, p, orc, model, ctl = _setup(B, W.TERRAIN_WALK)
    x0 = f32(W.initial_state(1, W.SCENE_HEIGHTFIELD))
    mu = f32(W.stance_knots(p["nk"]))
    ctl.set_nominal(_dev(mu))
    costs, traj = ctl.rollout_batch(_dev(x0), traj=True)
    eps = ctl.sample().cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    tr = traj.cpu().numpy().astype(np.float64)
    c = costs.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    _chain(orc, p, mu, eps, tr, c, [0, 1, p["K"] - 1] + list(rng.integers(0, p["K"], 5)))


def test_split_box_push_full_size_chain(B):
    """The pushing workload at the benchmark's launch shape (K=4096, H=60, 8 knots) with
    the box within reach: sampled samples, every third step, against the oracle."""
    _say("split box push K=4096 H=60 chain")
    md, p, orc, model, ctl = _setup(B, W.BOX_PUSH)
    x0 = f32(W.initial_state(0, W.SCENE_FREE_BOX))
    x0[37] = 0.45
    mu = f32(W.stance_knots(p["nk"]))
    ctl.set_nominal(_dev(mu))
    costs, traj = ctl.rollout_batch(_dev(x0), traj=True)
    eps = ctl.sample().cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    tr = traj.cpu().numpy().astype(np.float64)
    c = costs.cpu().numpy()
    assert np.isfinite(c).mean() > 0.9
    samples = [0, 1, p["K"] - 1, int(np.argmin(c))] + list(np.random.default_rng(1).integers(0, p["K"], 3))
    _chain(orc, p, mu, eps, tr, c, samples, box=True, every=3)


def test_split_costs_equal_the_quad_kernel(B):
    """Same step, same arithmetic, same Philox noise: the costs equal the quad kernel's up
    to summation order.  (The noise the rollout stores feeds the update, which the full
    control steps below check against the oracle.)"""
    _say("split and quad agreement")
    md, p, orc, model, ctl = _setup(B, W.TERRAIN_WALK, K=300, H=20)
    q = B.Controller(model, dict(p, lanes=4))
    x0 = _dev(W.initial_state(2, W.SCENE_HEIGHTFIELD))
    mu = _dev(W.stance_knots(p["nk"]))
    ctl.set_nominal(mu)
    q.set_nominal(mu)
    a = ctl.rollout_batch(x0).cpu().numpy().astype(np.float64)
    b = q.rollout_batch(x0).cpu().numpy().astype(np.float64)
    rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-6)
    assert rel.max() <= COST_TOL


def test_split_mppi_step_matches_oracle(B):
    _say("split flat-walk control steps")
    md, p, orc, model, ctl = _setup(B, W.FLAT_WALK)
    for seed in range(3):
        x0 = f32(W.initial_state(seed))
        mu = f32(W.stance_knots(4))
        ctl.set_nominal(_dev(mu))
        ctl.set_step(seed)
        u0 = ctl.step(_dev(x0))
        nominal = ctl.get_nominal().cpu().numpy()
        assert ctl.sync_status() == 0
        ou0, omu, _, _ = orc.mppi_step(p, seed, x0, mu)
        assert np.abs(u0.cpu().numpy() - ou0).max() <= KNOT_TOL, seed
        assert np.abs(nominal - omu).max() <= KNOT_TOL, seed


def test_split_box_push_control_step_matches_oracle(B):
    """One full control step of the pushing workload at K=4096, H=60 (the update then runs
    four passes over the costs) against the oracle's Algorithm 1."""
    _say("split box push K=4096 control step")
    md, p, orc, model, ctl = _setup(B, W.BOX_PUSH)
    x0 = f32(W.initial_state(0, W.SCENE_FREE_BOX))
    mu = f32(W.stance_knots(p["nk"]))
    ctl.set_nominal(_dev(mu))
    ctl.set_step(0)
    u0 = ctl.step(_dev(x0)).cpu().numpy()
    nominal = ctl.get_nominal().cpu().numpy()
    assert ctl.sync_status() == 0
    ou0, omu, ocosts, rc = orc.mppi_step(p, 0, x0, mu)
    assert rc == 0
    assert r16_knot_sensitivity(p, 0, mu, ocosts) <= KNOT_TOL  # the comparison is robust to cost errors
    assert np.abs(u0 - ou0).max() <= KNOT_TOL
    assert np.abs(nominal - omu).max() <= KNOT_TOL


@pytest.mark.parametrize("K,H,nk", [(1, 5, 4), (5, 1, 2), (7, 3, 3), (13, 80, 8)])
def test_split_edges(B, K, H, nk):
    """Ragged workgroups (K not a multiple of 4), a one-step horizon, two knots, the
    longest horizon and most knots the workloads use."""
    _say("split edges", K, H, nk)
    md, p, orc, model, ctl = _setup(B, W.FLAT_WALK, K=K, H=H, nk=nk, dt=0.01)
    x0 = f32(W.initial_state(4))
    mu = f32(W.stance_knots(nk))
    eps = f32(W.explicit_noise(1, K, nk) * 0.3)
    ctl.set_nominal(_dev(mu))
    costs, traj = ctl.rollout_batch(_dev(x0), eps=_dev(eps), traj=True)
    tr = traj.cpu().numpy().astype(np.float64)
    c = costs.cpu().numpy().astype(np.float64)
    Bm = O.spline_basis(nk, H, p["dt"])
    for n in range(K):
        theta = mu + (p["sigma"] * eps[n] if n else 0.0)
        U = Bm @ theta.reshape(12, nk).T
        for k in range(min(H, 12)):
            xn, _, _ = orc.step(tr[n, k], U[k], p["kp"], p["kd"], p["dt"])
            assert step_error(tr[n, k + 1], xn).max() <= STEP_TOL, (n, k)


def test_split_runs_are_bitwise_deterministic(B):
    _say("split determinism")
    md, p, orc, model, ctl = _setup(B, W.BOX_PUSH, K=256, H=20)
    x0 = _dev(box_contact_states(1, seed=2)[0])
    a = ctl.rollout_batch(x0).cpu().numpy()
    b = ctl.rollout_batch(x0).cpu().numpy()
    assert np.array_equal(a, b)


def _one_step_split(B, model, p, xs, us, arith):
    """One rollout step per state on the lane-split kernel: K = 1, H = 1, constant knots
    equal to the joint targets (every basis reproduces constants)."""
    ctl = B.Controller(model, dict(p, K=1, H=1, nk=2, sigma=0.0, arith=arith, lanes=16))
    eps = _dev(np.zeros((1, 24)))
    out = []
    for x, u in zip(xs, us):
        ctl.set_nominal(_dev(np.repeat(u, 2)))
        _, traj = ctl.rollout_batch(_dev(x), eps=eps, traj=True)
        out.append(traj[0, 1].cpu().numpy().astype(np.float64))
    return np.array(out)


def _states(orc, workload, p):
    if workload["scene"] == W.SCENE_FREE_BOX:
        xs = box_contact_states(60, seed=1)
        us = f32(np.tile(W.STANCE_JOINTS, 4) + np.random.default_rng(3).uniform(-0.3, 0.3, (len(xs), 12)))
        return xs, us
    return random_walk_states(orc, seeds=range(3), steps=40, dt=p["dt"], scene=workload["scene"])


@pytest.mark.parametrize("workload", [W.FLAT_WALK, W.TERRAIN_WALK, W.BOX_PUSH])
def test_split_fp64_one_step_parity(B, workload):
    _say("split fp64 one-step", workload["name"])
    md, p, orc, model, ctl = _setup(B, workload)
    xs, us = _states(orc, workload, p)
    got = _one_step_split(B, model, p, xs, us, "fp64")
    want = np.array([orc.step(x, u, p["kp"], p["kd"], p["dt"])[0] for x, u in zip(xs, us)])
    err = step_error(got, want, box=workload["scene"] == W.SCENE_FREE_BOX)
    assert err.max() <= STEP_TOL, (err.max(), int(err.argmax()))


@pytest.mark.parametrize("workload", [W.FLAT_WALK, W.TERRAIN_WALK, W.BOX_PUSH])
def test_split_mixed_one_step_within_ulp_sensitivity(B, workload):
    _say("split mixed one-step", workload["name"])
    md, p, orc, model, ctl = _setup(B, workload)
    xs, us = _states(orc, workload, p)
    got = _one_step_split(B, model, p, xs, us, "mixed")
    want = np.array([orc.step(x, u, p["kp"], p["kd"], p["dt"])[0] for x, u in zip(xs, us)])
    err = step_error(got, want, box=workload["scene"] == W.SCENE_FREE_BOX)
    bound = np.array([mixed_step_bound(orc, x, u, p["kp"], p["kd"], p["dt"]) for x, u in zip(xs, us)])
    print("mixed step error: max %.2e median %.2e; bound min %.2e median %.2e; worst error / bound %.2f"
          % (err.max(), np.median(err), bound.min(), np.median(bound), (err / bound).max()))
    assert (err <= bound).all(), (int((err / bound).argmax()), (err / bound).max())


@pytest.mark.parametrize("workload", [W.FLAT_WALK, W.TERRAIN_WALK, W.BOX_PUSH])
def test_split_fp32_one_step_within_conditioning_bound(B, workload):
    _say("split fp32 one-step", workload["name"])
    md, p, orc, model, ctl = _setup(B, workload)
    xs, us = _states(orc, workload, p)
    got = _one_step_split(B, model, p, xs, us, "fp32")
    want = np.array([orc.step(x, u, p["kp"], p["kd"], p["dt"])[0] for x, u in zip(xs, us)])
    err = step_error(got, want, box=workload["scene"] == W.SCENE_FREE_BOX)
    bound = np.array([fp32_step_bound(orc, x, u, p["kp"], p["kd"], p["dt"]) for x, u in zip(xs, us)])
    print("fp32 step error: max %.2e median %.2e; worst error / bound %.3f" % (err.max(), np.median(err),
                                                                               (err / bound).max()))
    assert (err <= bound).all()


@pytest.mark.parametrize("arith", ["mixed", "fp32"])
def test_split_box_push_chain_costs_sum_oracle_stage_costs(B, arith):
    """Full box-push shape (K=4096, H=60) with the faster arithmetics: sampled samples'
    costs equal the sum of the oracle's stage costs of the GPU's own states within
    COST_TOL, and every third step is within the arithmetic's per-step bound."""
    _say("split box push chain", arith)
    md, p, orc, model, ctl = _setup(B, W.BOX_PUSH, arith=arith)
    x0 = f32(W.initial_state(0, W.SCENE_FREE_BOX))
    x0[37] = 0.45
    mu = f32(W.stance_knots(p["nk"]))
    ctl.set_nominal(_dev(mu))
    costs, traj = ctl.rollout_batch(_dev(x0), traj=True)
    eps = ctl.sample().cpu().numpy().astype(np.float64)
    tr = traj.cpu().numpy().astype(np.float64)
    c = costs.cpu().numpy().astype(np.float64)
    Bm = O.spline_basis(p["nk"], p["H"], p["dt"])
    bound = mixed_step_bound if arith == "mixed" else fp32_step_bound
    rng = np.random.default_rng(4)
    for n in [0, p["K"] - 1, int(np.argmin(c))] + list(rng.integers(0, p["K"], 2)):
        theta = mu + (p["sigma"] * eps[n] if n else 0.0)
        U = Bm @ theta.reshape(12, p["nk"]).T
        L = 0.0
        for k in range(p["H"]):
            xk = tr[n, k]
            tau = p["kp"] * (U[k] - xk[7:19]) - p["kd"] * xk[25:37]
            L += p["dt"] * orc.stage_cost(p, tr[n, k + 1], tau)
            if k % 6 == 0:
                xn, _, _ = orc.step(xk, U[k], p["kp"], p["kd"], p["dt"])
                e = step_error(tr[n, k + 1], xn, box=True).max()
                assert e <= bound(orc, xk, U[k], p["kp"], p["kd"], p["dt"]), (n, k, e)
        assert abs(c[n] - L) <= COST_TOL * max(abs(L), 1e-6), (n, c[n], L)


# ---------------------------------------------------------------------------- direct sampling
@pytest.mark.parametrize("workload,K,H", [(W.FLAT_WALK, 50, 10), (W.BOX_PUSH, 21, 10)])
def test_split_direct_rollout_costs_10_steps(B, workload, K, H):
    """Direct per-step sampling (basis 3, one value per step): 10-step costs against the
    oracle's direct rollouts on the same noise."""
    _say("split direct costs", workload["name"], K, H)
    md, p, orc, model, ctl = _setup(B, workload, K=K, H=H, nk=H, basis=3)
    x0 = f32(W.initial_state(3, workload["scene"]))
    if workload["scene"] == W.SCENE_FREE_BOX:
        x0 = box_contact_states(1, seed=5)[0]
    mu = f32(W.stance_knots(H) + np.random.default_rng(2).uniform(-0.1, 0.1, 12 * H))
    eps = f32(W.explicit_noise(5, K, H))
    ctl.set_nominal(_dev(mu))
    got = ctl.rollout_batch(_dev(x0), eps=_dev(eps)).cpu().numpy().astype(np.float64)
    want = orc.rollout_batch(p, x0, mu, eps)
    rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-6)
    assert rel.max() <= COST_TOL, (rel.max(), int(rel.argmax()))


@pytest.mark.parametrize("K,H", [(256, 50), (1025, 60)])
def test_split_direct_mppi_step_matches_oracle(B, K, H):
    """Full control steps with direct sampling on the heightfield (Philox noise drawn in
    the step loop, 12 H values updated over knot chunks): first control and shifted plan
    against the oracle's Algorithm 1."""
    _say("split direct control steps", K, H)
    md, p, orc, model, ctl = _setup(B, W.TERRAIN_WALK, K=K, H=H, nk=H, basis=3)
    for seed in range(2):
        x0 = f32(W.initial_state(seed, W.SCENE_HEIGHTFIELD))
        mu = f32(W.stance_knots(H))
        ctl.set_nominal(_dev(mu))
        ctl.set_step(seed)
        u0 = ctl.step(_dev(x0)).cpu().numpy()
        nominal = ctl.get_nominal().cpu().numpy()
        assert ctl.sync_status() == 0
        ou0, omu, ocosts, rc = orc.mppi_step(p, seed, x0, mu)
        assert rc == 0
        assert r16_knot_sensitivity(p, seed, mu, ocosts) <= KNOT_TOL
        assert np.abs(u0 - ou0).max() <= KNOT_TOL, seed
        assert np.abs(nominal - omu).max() <= KNOT_TOL, seed


def test_update_over_knot_chunks_matches_oracle(B):
    """The update with 60 values per joint (eight chunks of the knot loop) against the
    oracle's Eq. 1 / Eq. 2 on identical costs and noise."""
    _say("update knot chunks")
    md, p, orc, model, ctl = _setup(B, W.FLAT_WALK, K=700, H=60, nk=60, basis=3, dt=0.01)
    rng = np.random.default_rng(9)
    mu = f32(W.stance_knots(60) + rng.uniform(-0.2, 0.2, 720))
    eps = f32(rng.standard_normal((700, 720)))
    costs = f32(rng.uniform(0.5, 2.5, 700))
    ctl.set_nominal(_dev(mu))
    knots, w = ctl.update(_dev(costs), eps=_dev(eps), weights=True)
    want, ww, rc = O.update(p, costs, mu, eps)
    assert rc == 0
    assert np.abs(knots.cpu().numpy() - want).max() <= 1e-5
    np.testing.assert_allclose(w.cpu().numpy(), ww, rtol=1e-4, atol=1e-7)
