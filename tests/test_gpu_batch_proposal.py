"""Batched serving with the learned proposal, on the GPU: instances whose samples come from
the policy (ungated) against the single-instance controller with the same policy and
gate, and against the oracle's chain (features, BF16-operand forward, head, proposal
step, plant step).

The batch step, proposal launches included, is one captured graph: the test replays it
four times and checks every replay.

Tolerances: against the controller 1e-5 absolute on the first control and the nominal
and STEP_TOL on the plant state (the same kernels up to the rollout's launch shape);
against the oracle KNOT_TOL and STEP_TOL, as for the plain batch.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W
from tests.parity_utils import KNOT_TOL, STEP_TOL, f32, round_model, round_params, step_error

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
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda().contiguous()


def _policy(B, max_batch=8, seed=5):
    pol = B.Policy(max_batch=max_batch, seed=seed)
    rng = np.random.default_rng(6)
    norm = (rng.normal(size=40) * 0.1, rng.uniform(0.5, 2.0, 40), np.repeat(np.tile(W.STANCE_JOINTS, 4), 6),
            np.full(72, 0.05))
    pol.set_normalization(*norm)
    return pol, [f32(v) for v in norm]


# (workload, K, H, nk, seed, instance id, proposal command or None for plain sampling)
SPECS = [
    (W.TERRAIN_WALK, 64, 30, 6, 1, 7, (0.5, 0.0, 0.0)),
    (W.FLAT_WALK, 48, 20, 4, 2, 9, (0.3, 0.1, -0.2)),
    (W.FLAT_WALK, 32, 20, 4, 3, 10, None),
]


@pytest.mark.parametrize("mode", [0, 1])  # per-scene kernels, one kernel for every scene
def test_batched_proposal_matches_controller_and_oracle(B, mode):
    pol, (im, isd, om, osd) = _policy(B)
    batch = B.Batch(max_instances=8, budget_bytes=64 << 20, max_horizon=80, max_hf_cells=4096)
    batch.set_launch_mode(mode)
    models, mds, slots = {}, {}, {}
    for wl in (W.FLAT_WALK, W.TERRAIN_WALK):
        mds[wl["name"]] = round_model(W.model_dict(wl, 0))
        models[wl["name"]] = B.Model(mds[wl["name"]])
        slots[wl["name"]] = batch.add_model(models[wl["name"]])
    ids, refs = [], []
    for wl, K, H, nk, seed, inst, cmd in SPECS:
        p = round_params(W.params_dict(wl, seed, K=K, H=H, nk=nk, instance=inst))
        x0 = f32(W.initial_state(seed, wl["scene"]))
        mu = f32(W.stance_knots(nk) + np.random.default_rng(seed).uniform(-0.05, 0.05, 12 * nk))
        i = batch.admit(slots[wl["name"]], p, x0, mu)
        origin = (float(x0[0]) - 0.1, float(x0[1]) + 0.2)
        if cmd is not None:
            batch.set_proposal(i, pol, cmd=cmd, origin=origin)
        ids.append(i)
        refs.append([wl, p, cmd, origin, x0, mu])
    # four graph replays, with eager controller steps and synchronisations between them;
    # before the third the policy's weights change in place, which the captured network
    # pass must pick up (it reads the weights, it did not copy them)
    for step in range(4):
        if step == 2:
            P = pol.get_params()
            pol.set_params(P * 1.01 + 1e-3)
            torch.cuda.synchronize()
        batch.step()
        torch.cuda.synchronize()
        for i, ref in zip(ids, refs):
            wl, p, cmd, origin, x0, mu = ref
            name = wl["name"]
            model, orc = models[name], O.Oracle(mds[name])
            bx, bu0, bmu, acc, bstep = batch.read(i, model.nx, p["nk"])
            assert bstep == step + 1
            # the single-instance controller with the same policy, ungated
            ctl = B.Controller(model, p)
            ctl.set_nominal(_dev(mu))
            ctl.set_step(step)
            if cmd is not None:
                ctl.set_proposal(pol, k_prop=p["K"], cmd=cmd, origin=origin, gate="none")
            u0 = ctl.step(_dev(x0))
            nominal = ctl.get_nominal().cpu().numpy()
            x1 = model.sim_step(_dev(x0[None]), u0[None].contiguous(), p["kp"], p["kd"], p["dt"]).cpu().numpy()[0]
            assert np.abs(bu0 - u0.cpu().numpy()).max() <= 1e-5, (name, step)
            assert np.abs(bmu - nominal).max() <= 1e-5, (name, step)
            assert step_error(bx.astype(np.float64), x1.astype(np.float64)).max() <= STEP_TOL, (name, step)
            # the oracle's chain
            if cmd is not None:
                feat = O.policy_features(x0, f32(cmd), f32(origin), im, isd)
                out = O.mlp_forward(pol.get_params().cpu().numpy().astype(np.float64), feat[None], bf16=True)[0]
                c, sd = O.policy_head(out, om, osd, p["nk"], p["sigma"])
                ou0, onom, _, _, oacc, _ = orc.mppi_step_proposal(p, step, x0, mu, f32(c), f32(sd), p["K"], gate=1)
                assert oacc
            else:
                ou0, onom, _, _ = orc.mppi_step(p, step, x0, mu)
            assert np.abs(bu0 - ou0).max() <= KNOT_TOL, (name, step)
            assert np.abs(bmu - onom).max() <= KNOT_TOL, (name, step)
            ox, _, _ = orc.step(x0, f32(bu0), p["kp"], p["kd"], p["dt"])
            assert step_error(bx.astype(np.float64), ox).max() <= STEP_TOL, (name, step)
            ref[4], ref[5] = f32(bx), f32(bmu)  # both paths continue from the batch's state


def test_batched_proposal_switches_back_to_plain_sampling(B):
    pol, _ = _policy(B)
    batch = B.Batch(max_instances=4, budget_bytes=16 << 20, max_horizon=40, max_hf_cells=0)
    wl = W.FLAT_WALK
    md = round_model(W.model_dict(wl, 0))
    model = B.Model(md)
    slot = batch.add_model(model)
    p = round_params(W.params_dict(wl, 4, K=40, H=15, nk=4, instance=3))
    x0, mu = f32(W.initial_state(4)), f32(W.stance_knots(4))
    i = batch.admit(slot, p, x0, mu)
    batch.set_proposal(i, pol, cmd=(0.4, 0.0, 0.0), origin=(0.0, 0.0))
    batch.step()
    batch.set_proposal(i, None)
    batch.step()
    bx, bu0, bmu, _, bstep = batch.read(i, model.nx, 4)
    assert bstep == 2
    # the state and nominal after the (deterministic) first step, from a second batch that
    # stops there; the first batch's second step must be the plain step from them
    batch2 = B.Batch(max_instances=4, budget_bytes=16 << 20, max_horizon=40, max_hf_cells=0)
    j = batch2.admit(batch2.add_model(model), p, x0, mu)
    batch2.set_proposal(j, pol, cmd=(0.4, 0.0, 0.0), origin=(0.0, 0.0))
    batch2.step()
    x_1, _, mu_1, _, _ = batch2.read(j, model.nx, 4)
    ou0, onom, _, _ = O.Oracle(md).mppi_step(p, 1, f32(x_1), f32(mu_1))
    assert np.abs(bu0 - ou0).max() <= KNOT_TOL
    assert np.abs(bmu - onom).max() <= KNOT_TOL


def test_batched_proposal_rejects_what_it_cannot_serve(B):
    pol, _ = _policy(B, max_batch=1)
    batch = B.Batch(max_instances=4, budget_bytes=16 << 20, max_horizon=40, max_hf_cells=0)
    flat = B.Model(round_model(W.model_dict(W.FLAT_WALK, 0)))
    push = B.Model(round_model(W.model_dict(W.BOX_PUSH, 0)))
    s_flat, s_push = batch.add_model(flat), batch.add_model(push)
    p = round_params(W.params_dict(W.FLAT_WALK, 0, K=16, H=10, nk=4))
    pp = round_params(W.params_dict(W.BOX_PUSH, 0, K=16, H=10, nk=4))
    a = batch.admit(s_flat, p, f32(W.initial_state(0)), f32(W.stance_knots(4)))
    b = batch.admit(s_flat, dict(p, instance=1), f32(W.initial_state(1)), f32(W.stance_knots(4)))
    c = batch.admit(s_push, pp, f32(W.initial_state(0, W.SCENE_FREE_BOX)), f32(W.stance_knots(4)))
    with pytest.raises(B.MppiError):
        batch.set_proposal(c, pol)  # 50-float state
    other, _ = _policy(B, max_batch=4, seed=9)
    batch.set_proposal(a, pol)
    with pytest.raises(B.MppiError):
        batch.set_proposal(b, other)  # one policy per batch
    batch.set_proposal(b, pol)
    with pytest.raises(B.MppiError):
        batch.step()  # two proposal instances, max_batch 1
    batch.set_proposal(b, None)
    batch.step()
    torch.cuda.synchronize()
