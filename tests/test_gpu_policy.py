"""GPU parity of the learned proposal against the oracle: the BF16 MFMA network (forward,
gradient, Adam), the head, checkpoints, the proposal control step (built on the plain
explicit-noise rollout and update kernels) and the learned step end to end.  The two
tests of an earlier implementation of the step, which ran a modified rollout kernel
that faulted the GPU, stay skipped with the reason.

Tolerances (relative L2 over the compared array unless stated):
  forward vs the BF16-operand oracle       <= 1e-3  (same operand roundings; FP32 vs FP64
                                                      sums can flip a rare bf16 rounding)
  gradient vs the BF16-operand oracle      <= 1e-2  per weight matrix and per bias vector,
                                                      both max |diff| / max |ref| and relative
                                                      L2 (the backward rounds dz to bf16 too,
                                                      so flips compound)
  gradient vs the exact FP64 oracle        <= 2e-2, cosine >= 0.999
  Adam vs FP64 Adam on the same gradient   per element: FP32 rounding of the master weight
                                           each step plus 1e-6 of the step size
  head                                     <= 1e-5
  proposal step: costs COST_TOL, knots and first control KNOT_TOL (as the plain step).
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W
from tests.parity_utils import KNOT_TOL, f32, round_model, round_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10469_amd import binding
    binding.lib()
    return binding


def _dev(a, dtype=np.float32):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).cuda().contiguous()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def _params(pol):
    return pol.get_params().cpu().numpy().astype(np.float64)


def _tensor_slices():
    """(name, slice) of every weight matrix and every bias vector in the flat vector."""
    out, off = [], 0
    for l, (fi, fo) in enumerate(zip(O.MLP_DIMS[:-1], O.MLP_DIMS[1:])):
        out.append((f"W{l}", slice(off, off + fi * fo)))
        out.append((f"b{l}", slice(off + fi * fo, off + fi * fo + fo)))
        off += fi * fo + fo
    return out


def _per_tensor(G, R, tol):
    """Each weight matrix and each bias vector on its own: max |G - R| <= tol max |R| and
    relative L2 <= tol (a bias gradient is too small a share of its layer's norm to be
    checked through the layer)."""
    for name, sl in _tensor_slices():
        worst = np.abs(G[sl] - R[sl]).max() / max(np.abs(R[sl]).max(), 1e-30)
        assert worst <= tol, (name, worst)
        assert _rel(G[sl], R[sl]) <= tol, (name, _rel(G[sl], R[sl]))


# ---------------------------------------------------------------------------- forward
@pytest.mark.parametrize("Bsz", [1, 100, 256])
def test_forward_matches_bf16_oracle(B, Bsz):
    pol = B.Policy(max_batch=512, seed=11)
    P = _params(pol)
    X = np.random.default_rng(Bsz).normal(size=(Bsz, 40)).astype(np.float32)
    out = pol.forward(_dev(X)).cpu().numpy()
    ref = O.mlp_forward(P, f32(X), bf16=True)
    exact = O.mlp_forward(P, f32(X))
    assert np.isfinite(out).all()
    assert _rel(out, ref) <= 1e-3, _rel(out, ref)
    assert _rel(out, exact) <= 2e-2


def test_forward_standardises_inputs(B):
    pol = B.Policy(max_batch=64, seed=3)
    rng = np.random.default_rng(5)
    mean, std = rng.normal(size=40).astype(np.float32), rng.uniform(0.5, 3, 40).astype(np.float32)
    pol.set_normalization(mean, std, np.zeros(72), np.ones(72))
    X = (rng.normal(size=(37, 40)) * std + mean).astype(np.float32)
    out = pol.forward(_dev(X)).cpu().numpy()
    ref = O.mlp_forward(_params(pol), (f32(X) - f32(mean)) / f32(std), bf16=True)
    assert _rel(out, ref) <= 1e-3


# ---------------------------------------------------------------------------- gradient
@pytest.mark.parametrize("Bsz,gather", [(64, False), (200, True)])
def test_gradient_matches_oracle(B, Bsz, gather):
    pol = B.Policy(max_batch=256, seed=21)
    P = _params(pol)
    rng = np.random.default_rng(Bsz)
    N = 300 if gather else Bsz
    Xall = rng.normal(size=(N, 40)).astype(np.float32)
    Yall = rng.normal(size=(N, 72)).astype(np.float32)
    idx = rng.permutation(N)[:Bsz].astype(np.int32) if gather else None
    loss, G = pol.grad(_dev(Xall), _dev(Yall), _dev(idx, np.int32) if gather else None, B=Bsz)
    G = G.cpu().numpy().astype(np.float64)
    rows = idx if gather else np.arange(Bsz)
    X, Y = f32(Xall[rows]), f32(Yall[rows])
    Lb, Gb = O.mlp_grad(P, X, Y, bf16=True)
    Le, Ge = O.mlp_grad(P, X, Y)
    assert abs(float(loss.item()) - Lb) <= 1e-3 * abs(Lb)
    _per_tensor(G, Gb, 1e-2)
    assert _rel(G, Ge) <= 2e-2
    assert G @ Ge / (np.linalg.norm(G) * np.linalg.norm(Ge)) >= 0.999


def test_gradient_with_batch_splits_matches_oracle(B):
    """Batch 1024 (gathered rows): the weight gradients reduce 8 batch splits and the bias
    gradients 16 to 32 per-tile column partials, as in the training launches."""
    pol = B.Policy(max_batch=1024, seed=31)
    P = _params(pol)
    rng = np.random.default_rng(77)
    N, Bsz = 1500, 1024
    Xall = rng.normal(size=(N, 40)).astype(np.float32)
    Yall = rng.normal(size=(N, 72)).astype(np.float32)
    idx = rng.permutation(N)[:Bsz].astype(np.int32)
    loss, G = pol.grad(_dev(Xall), _dev(Yall), _dev(idx, np.int32), B=Bsz)
    G = G.cpu().numpy().astype(np.float64)
    Lb, Gb = O.mlp_grad(P, f32(Xall[idx]), f32(Yall[idx]), bf16=True)
    assert abs(float(loss.item()) - Lb) <= 1e-3 * abs(Lb)
    _per_tensor(G, Gb, 1e-2)


def test_gradient_is_deterministic(B):
    pol = B.Policy(max_batch=256, seed=2)
    rng = np.random.default_rng(0)
    X, Y = _dev(rng.normal(size=(256, 40))), _dev(rng.normal(size=(256, 72)))
    l1, g1 = pol.grad(X, Y)
    l2, g2 = pol.grad(X, Y)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_train_step_equals_gradient_then_adam(B):
    """The fused training step (reduction and Adam in one pass) against the separate
    gradient and Adam calls: same loss, same parameters, bit for bit."""
    rng = np.random.default_rng(3)
    N, Bsz = 700, 512
    X, Y = _dev(rng.normal(size=(N, 40))), _dev(rng.normal(size=(N, 72)))
    idx = _dev(rng.permutation(N)[:Bsz], np.int32)
    a, b = B.Policy(max_batch=Bsz, seed=12), B.Policy(max_batch=Bsz, seed=12)
    for _ in range(2):
        la = a.train_step(X, Y, index=idx, B=Bsz, lr=1e-3)
        lb, g = b.grad(X, Y, idx, B=Bsz)
        b.adam(g, 1e-3)
        assert torch.equal(la, lb)
        assert torch.equal(a.get_params(), b.get_params())
    out_a, out_b = a.forward(X[:64]), b.forward(X[:64])
    assert torch.equal(out_a, out_b)  # the BF16 shadows agree too


# ---------------------------------------------------------------------------- Adam
def test_adam_two_steps_match_oracle_and_refresh_bf16_weights(B):
    pol = B.Policy(max_batch=64, seed=4)
    P0 = _params(pol)
    rng = np.random.default_rng(9)
    n = P0.size
    G1 = (rng.normal(size=n) * 1e-2).astype(np.float32)
    G2 = (rng.normal(size=n) * 1e-2).astype(np.float32)
    pol.adam(_dev(G1), 1e-3)
    pol.adam(_dev(G2), 1e-3)
    assert pol.steps == 2
    P = _params(pol)
    m, v = np.zeros(n), np.zeros(n)
    Po, m, v = O.adam(P0, m, v, f32(G1), 1)
    Po, m, v = O.adam(Po, m, v, f32(G2), 2)
    # FP32 master weights: each step rounds p to FP32 (half an ulp, 2^-24 relative), and
    # the update lr m^/(sqrt(v^)+eps) carries FP32 arithmetic error (~1e-6 of lr)
    assert np.all(np.abs(P - Po) <= 2 * 2.0 ** -24 * np.abs(Po) + 2 * 1e-6 * 1e-3)
    # the products read the refreshed BF16 copies of the updated weights
    X = rng.normal(size=(16, 40)).astype(np.float32)
    out = pol.forward(_dev(X)).cpu().numpy()
    assert _rel(out, O.mlp_forward(P, f32(X), bf16=True)) <= 1e-3


def test_train_step_reduces_loss_and_checkpoint_round_trip(B, tmp_path):
    pol = B.Policy(max_batch=128, seed=8)
    rng = np.random.default_rng(1)
    norm = (rng.normal(size=40), rng.uniform(0.5, 2, 40), rng.normal(size=72), rng.uniform(0.5, 2, 72))
    pol.set_normalization(*norm)
    X = _dev(rng.normal(size=(128, 40)))
    W0 = rng.normal(size=(40, 72)) * 0.3
    Y = _dev(np.tanh(rng.normal(size=(128, 40)) @ W0))
    losses = [float(pol.train_step(X, Y, lr=1e-3).item()) for _ in range(30)]
    assert losses[-1] < 0.8 * losses[0], losses
    path = tmp_path / "pol.ckpt"
    pol.save(path)
    pol2 = B.Policy(max_batch=128, ckpt=str(path))
    assert pol2.steps == pol.steps == 30
    for a, b in zip(pol2.get_normalization(), norm):
        np.testing.assert_array_equal(a, np.float32(b))
    assert torch.equal(pol2.get_params(), pol.get_params())
    # identical next step from the restored moments
    l1 = pol.train_step(X, Y, lr=1e-3)
    l2 = pol2.train_step(X, Y, lr=1e-3)
    assert torch.equal(l1, l2) and torch.equal(pol2.get_params(), pol.get_params())


# ---------------------------------------------------------------------------- head
@pytest.mark.parametrize("nk", [4, 6, 8])
def test_head_matches_oracle(B, nk):
    pol = B.Policy(max_batch=1, seed=0)
    rng = np.random.default_rng(nk)
    om, os_ = rng.normal(size=72).astype(np.float32), rng.uniform(0.05, 0.5, 72).astype(np.float32)
    pol.set_normalization(np.zeros(40), np.ones(40), om, os_)
    out = rng.normal(size=144).astype(np.float32)
    c, sd = pol.head(_dev(out), nk, 0.25)
    oc, osd = O.policy_head(f32(out), f32(om), f32(os_), nk, float(np.float32(0.25)))
    assert np.abs(c.cpu().numpy() - oc).max() <= 1e-5 * max(1.0, np.abs(oc).max())
    assert np.abs(sd.cpu().numpy() - osd).max() <= 1e-5 * np.abs(osd).max()


# ---------------------------------------------------------------------------- proposal step
def _ctl(B, K=64, H=10, lanes=0, **extra):
    wl = W.FLAT_WALK
    md = round_model(W.model_dict(wl, 0))
    p = round_params(W.params_dict(wl, 3, K=K, H=H, lanes=lanes, **extra))
    return md, p, O.Oracle(md), B.Controller(B.Model(md), p)


FAULTED = ("records the first implementation of the proposal step, which passed the per-knot std, the "
           "sample-1 override and the gate as new arguments of the quad rollout kernel; that build faulted the GPU "
           "(memory aperture violation in rollout_kernel<0, double>) on its first run and no cause was shown, so "
           "the change was taken out; the step now runs on the unchanged kernels "
           "(test_proposal_step_on_plain_kernels_matches_oracle)")


@pytest.mark.skip(reason=FAULTED)
@pytest.mark.parametrize("accept", [True, False])
def test_step_proposal_matches_oracle(B, accept):
    md, p, orc, ctl = _ctl(B)
    D = 12 * p["nk"]
    rng = np.random.default_rng(2)
    mu = f32(W.stance_knots(p["nk"]))
    x0 = f32(W.initial_state(3))
    if accept:   # nominal perturbed badly, proposal near the stance
        nominal = f32(mu + 0.5)
        center = f32(mu + 0.02 * rng.normal(size=D))
    else:        # proposal far worse than the nominal
        nominal = mu
        center = f32(mu + 0.8)
    sd = f32(rng.uniform(0.05, 0.2, D))
    Kp = 16
    ctl.set_nominal(_dev(nominal))
    ctl.set_step(5)
    u0 = ctl.step_proposal(_dev(x0), _dev(center), _dev(sd), Kp).cpu().numpy()
    nom = ctl.get_nominal().cpu().numpy()
    acc, steps = ctl.proposal_stats()
    ou0, onom, cp, cf, oacc, rc = orc.mppi_step_proposal(p, 5, x0, nominal, center, sd, Kp)
    assert oacc == accept and acc == int(accept) and steps == 1
    assert ctl.sync_status() == 0 and ctl.step_counter == 6
    assert np.abs(u0 - ou0).max() <= KNOT_TOL
    assert np.abs(nom - onom).max() <= KNOT_TOL


@pytest.mark.skip(reason=FAULTED)
def test_learned_step_matches_oracle_chain(B):
    """mppi_step through the policy: features, BF16 forward, head and proposal step against
    the oracle's features, BF16-operand forward, head and proposal step."""
    md, p, orc, ctl = _ctl(B, K=64, H=10)
    pol = B.Policy(max_batch=1, seed=5)
    rng = np.random.default_rng(6)
    im, isd = rng.normal(size=40) * 0.1, rng.uniform(0.5, 2.0, 40)
    om = np.repeat(np.tile(W.STANCE_JOINTS, 4), 6)   # joint-major: 6 knots per joint
    osd = np.full(72, 0.05)
    pol.set_normalization(im, isd, om, osd)
    cmd, origin = (0.5, 0.0, 0.0), (0.1, -0.2)
    ctl.set_proposal(pol, k_prop=16, cmd=cmd, origin=origin)
    x0 = f32(W.initial_state(2))
    mu = f32(W.stance_knots(p["nk"]))
    ctl.set_nominal(_dev(mu))
    ctl.set_step(0)
    u0 = ctl.step(_dev(x0)).cpu().numpy()
    nom = ctl.get_nominal().cpu().numpy()
    acc, steps = ctl.proposal_stats()
    feat = O.policy_features(x0, f32(cmd), f32(origin), f32(im), f32(isd))
    out = O.mlp_forward(_params(pol), feat[None], bf16=True)[0]
    c, sd = O.policy_head(out, f32(om), f32(osd), p["nk"], p["sigma"])
    ou0, onom, cp, cf, oacc, rc = orc.mppi_step_proposal(p, 0, x0, mu, f32(c), f32(sd), 16)
    assert steps == 1 and acc == int(oacc)
    assert np.abs(u0 - ou0).max() <= KNOT_TOL
    assert np.abs(nom - onom).max() <= KNOT_TOL
    ctl.set_proposal(None)
    ctl.step(_dev(x0))
    assert ctl.proposal_stats()[1] == 1  # plain steps are not counted


def test_nll_is_the_gradient_steps_loss_and_the_formula(B):
    """mppi_policy_nll: bit for bit the loss mppi_policy_grad reports for the same rows
    (same forward, loss kernel and summation order), and the Gaussian NLL of the network's
    own outputs computed here in FP64."""
    pol = B.Policy(max_batch=512, seed=4)
    rng = np.random.default_rng(12)
    norm = (rng.normal(size=40) * 0.1, rng.uniform(0.5, 2.0, 40), rng.normal(size=72) * 0.2,
            rng.uniform(0.05, 0.3, 72))
    pol.set_normalization(*norm)
    X = torch.as_tensor(rng.normal(size=(700, 40)), dtype=torch.float32).cuda()
    Y = torch.as_tensor(rng.normal(size=(700, 72)) * 0.2, dtype=torch.float32).cuda()
    for idx in (None, torch.as_tensor(rng.choice(700, 333, replace=False).astype(np.int32)).cuda()):
        B_ = 500 if idx is None else None
        loss = pol.nll(X, Y, index=idx, B=B_).item()
        lg, _ = pol.grad(X, Y, index=idx, B=B_)
        assert np.float32(loss).tobytes() == np.float32(lg.item()).tobytes(), (loss, lg.item())
        rows = np.arange(500) if idx is None else idx.cpu().numpy()
        out = pol.forward(X[torch.as_tensor(rows).long().cuda()].contiguous()).cpu().numpy().astype(np.float64)
        y = (Y.cpu().numpy()[rows].astype(np.float64) - norm[2].astype(np.float32)) / norm[3].astype(np.float32)
        m, s = out[:, :72], out[:, 72:]
        want = np.mean(0.5 * (y - m) ** 2 * np.exp(-2 * s) + s)
        assert abs(loss - want) <= 1e-5 * max(1.0, abs(want)), (loss, want)


@pytest.mark.parametrize("nk", [4, 6, 3])
def test_pairs_from_records_match_a_reference(B, nk):
    """mppi_policy_pairs against a reference written here: the fall cut (first row not
    finite or not above the fall height), features (state minus origin, command) bit for
    bit, and 6-knot targets against the oracle's not-a-knot spline evaluated at the six
    fractions of the horizon (FP32 sums: 1e-5)."""
    rng = np.random.default_rng(nk)
    n_rec, steps, W_ = 6, 30, 37 + 12 * nk
    rec = rng.normal(size=(n_rec, steps, W_)).astype(np.float32)
    rec[:, :, 2] = rng.uniform(0.2, 0.3, (n_rec, steps))
    fall = 0.12
    rec[1, 7, 2] = 0.05                 # falls at row 7
    rec[2, 0, 37 + 5] = np.nan          # a knot not finite at row 0: no pair
    rec[3, 29, 20] = np.inf             # the last row not finite
    rec[4, 12, 2] = np.float32(fall)    # at the fall height (not above): cut
    rec[5, 3, 2] = np.nan               # a non-finite height
    want_n = [30, 7, 0, 29, 12, 3]
    oc = np.c_[rng.uniform(-0.5, 0.5, (n_rec, 2)), rng.uniform(0, 0.8, n_rec)].astype(np.float32)
    feat, tgt, count = B.policy_pairs(torch.as_tensor(rec).cuda(), torch.as_tensor(oc).cuda(), nk, fall)
    torch.cuda.synchronize()
    assert count.cpu().tolist() == want_n
    feat, tgt = feat.cpu().numpy(), tgt.cpu().numpy()
    for r in range(n_rec):
        n = want_n[r]
        f = np.zeros((n, 40), np.float32)
        f[:, :37] = rec[r, :n, :37]
        f[:, 0] -= oc[r, 0]
        f[:, 1] -= oc[r, 1]
        f[:, 37] = oc[r, 2]
        assert np.array_equal(feat[r, :n], f), r
        for k in range(n):
            kn = rec[r, k, 37:].reshape(12, nk).astype(np.float64)
            ref = np.array([[O.spline_eval(kn[j], 1.0, i / 5) for i in range(6)] for j in range(12)]).reshape(72)
            assert np.abs(tgt[r, k] - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()), (r, k)


def test_pairs_edges(B):
    """One-row records, a single record, eight knots, and a record whose first row has
    fallen: counts 1, 1 and 0; one record of one row; targets at eight knots against the
    oracle's spline."""
    rng = np.random.default_rng(99)
    nk = 8
    rec = rng.normal(size=(3, 1, 37 + 12 * nk)).astype(np.float32)
    rec[:, :, 2] = 0.25
    rec[2, 0, 2] = 0.01
    oc = np.zeros((3, 3), np.float32)
    feat, tgt, count = B.policy_pairs(torch.as_tensor(rec).cuda(), torch.as_tensor(oc).cuda(), nk, 0.12)
    assert count.cpu().tolist() == [1, 1, 0]
    t = tgt.cpu().numpy()
    for r in range(2):
        kn = rec[r, 0, 37:].reshape(12, nk).astype(np.float64)
        ref = np.array([[O.spline_eval(kn[j], 1.0, i / 5) for i in range(6)] for j in range(12)]).reshape(72)
        assert np.abs(t[r, 0] - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    one = torch.as_tensor(rec[:1]).cuda()
    _, _, c1 = B.policy_pairs(one, torch.zeros((1, 3), device="cuda"), nk, 0.12)
    assert c1.cpu().tolist() == [1]
    with pytest.raises(B.MppiError):
        B.policy_pairs(one, torch.zeros((1, 3), device="cuda"), nk, float("nan"))


def test_training_pipeline_on_closed_loop_data(B):
    """Pairs from GPU closed loops of both walking configs, then a few Adam epochs: the
    held-out NLL falls well below the untrained network's."""
    from paper_2409_10469_amd import proposal as PR
    data = PR.generate(n_pairs=16000, episode_steps=40, instances=64, seed=3, log=lambda *a: None)
    X, Y = data["X"], data["Y"]
    assert X.shape == (16000, 40) and Y.shape == (16000, 72)
    assert torch.isfinite(X).all() and torch.isfinite(Y).all()
    assert (X[:, 2] > PR.FALL_Z).all()
    v = X[:, 37].cpu().numpy()
    assert v.min() >= 0.0 and v.max() <= 0.8 and (X[:, 38:] == 0).all()
    tr, ho = PR.split(data, holdout=0.1, seed=0)
    assert tr.numel() + ho.numel() == 16000 and ho.numel() > 0
    pol = B.Policy(max_batch=1024, seed=1)
    pol.set_normalization(*PR.normalization(data, tr))
    before = PR.nll(pol, data, ho)
    hist = PR.train(pol, data, tr, epochs=4, batch=1024, lr=1e-3, seed=0, held=ho, log=lambda *a: None)
    after = hist[-1][1]
    assert np.isfinite(after) and after < before - 0.5, (before, after)


# ---------------------------------------------------------------------------- proposal step
@pytest.mark.parametrize("lanes", [4, 16])
@pytest.mark.parametrize("accept,gate", [(True, "cost"), (False, "cost"), (False, "none"), (True, "best"),
                                         (False, "best"), (True, "best-concurrent"), (False, "best-concurrent"),
                                         (False, "cost-concurrent")])
def test_proposal_step_on_plain_kernels_matches_oracle(B, accept, gate, lanes):
    """The proposal step in both branches of each gate, and ungated, against the oracle's
    proposal step; with the lane-split rollout the plain fallback is rolled out only when
    the gate rejects unless the concurrent flag asks for both rollouts side by side, with
    the quad rollout always beside the proposal."""
    md, p, orc, ctl = _ctl(B, lanes=lanes)
    D = 12 * p["nk"]
    rng = np.random.default_rng(2)
    mu = f32(W.stance_knots(p["nk"]))
    x0 = f32(W.initial_state(3))
    if accept:   # nominal perturbed badly, proposal near the stance
        nominal = f32(mu + 0.5)
        center = f32(mu + 0.02 * rng.normal(size=D))
    else:        # proposal far worse than the nominal
        nominal = mu
        center = f32(mu + 0.8)
    sd = f32(rng.uniform(0.05, 0.2, D))
    Kp = 16
    ctl.set_nominal(_dev(nominal))
    ctl.set_step(5)
    u0 = ctl.step_proposal(_dev(x0), _dev(center), _dev(sd), Kp, gate=gate).cpu().numpy()
    nom = ctl.get_nominal().cpu().numpy()
    acc, steps = ctl.proposal_stats()
    ou0, onom, cp, cf, oacc, rc = orc.mppi_step_proposal(p, 5, x0, nominal, center, sd, Kp,
                                                         gate={"cost": 0, "none": 1, "best": 2}[gate.split("-")[0]])
    taken = accept or gate == "none"
    assert oacc == taken and acc == int(taken) and steps == 1
    assert ctl.sync_status() == (0 if taken else 2) and ctl.step_counter == 6  # 2: MPPI_WARN_FALLBACK
    assert np.abs(u0 - ou0).max() <= KNOT_TOL
    assert np.abs(nom - onom).max() <= KNOT_TOL


@pytest.mark.parametrize("accept", [True, False])
def test_gated_step_is_bitwise_the_chosen_branch(B, accept):
    """The cost gate is decided on the device after both rollouts ran side by side (the
    proposal's on an internal stream): an accepted gated step equals the ungated step bit
    for bit, a rejected one equals the plain step bit for bit, and a second gated step
    repeats the first exactly."""
    md, p, orc, ctl = _ctl(B)
    D = 12 * p["nk"]
    rng = np.random.default_rng(2)
    mu = f32(W.stance_knots(p["nk"]))
    x0 = _dev(W.initial_state(3))
    if accept:
        nominal = f32(mu + 0.5)
        center = f32(mu + 0.02 * rng.normal(size=D))
    else:
        nominal = mu
        center = f32(mu + 0.8)
    sd = _dev(rng.uniform(0.05, 0.2, D))
    c = _dev(center)
    runs = []
    for mode in ("cost", "cost", "ref"):
        ctl.set_nominal(_dev(nominal))
        ctl.set_step(5)
        if mode == "ref":
            u0 = ctl.step_proposal(x0, c, sd, 16, gate="none") if accept else ctl.step(x0)
        else:
            u0 = ctl.step_proposal(x0, c, sd, 16, gate="cost")
        runs.append((u0.cpu().numpy(), ctl.get_nominal().cpu().numpy()))
    acc, steps = ctl.proposal_stats()
    assert steps == (3 if accept else 2) and acc == (3 if accept else 0)
    for u, n in runs[1:]:
        assert np.array_equal(u, runs[0][0]) and np.array_equal(n, runs[0][1])


@pytest.mark.parametrize("lanes", [4, 16])
@pytest.mark.parametrize("accept", [True, False])
@pytest.mark.parametrize("gate", ["cost", "best"])
def test_concurrent_gate_matches_the_sequential_gate(B, accept, gate, lanes):
    """The concurrent flag rolls out the proposal and the plain samples in one launch on
    every step, centred on the nominal: the plain samples mu + sigma eps_n (the product
    rounded once in FP32), the proposal's mu + ((c - mu) + e_n) (the offset rounded once).
    The gate decides as the sequential gate does and every step agrees with it within that
    rounding; the nominal's own sample (theta_1 = mu) is exact, so the cost gate's
    comparison differs only in the centre's cost.  Two steps in a row; counters, status
    and step count equal."""
    md, p, orc, ctl = _ctl(B, lanes=lanes)
    D = 12 * p["nk"]
    rng = np.random.default_rng(7)
    mu = f32(W.stance_knots(p["nk"]))
    x0 = _dev(W.initial_state(3))
    if accept:
        nominal = f32(mu + 0.5)
        center = f32(mu + 0.02 * rng.normal(size=D))
    else:
        nominal = mu
        center = f32(mu + 0.8)
    sd, c = _dev(rng.uniform(0.05, 0.2, D)), _dev(center)
    runs = []
    for g in (gate, gate + "-concurrent"):
        ctl.set_nominal(_dev(nominal))
        ctl.set_step(5)
        out = []
        for _ in range(2):
            a0, n0 = ctl.proposal_stats()
            u0 = ctl.step_proposal(x0, c, sd, 16, gate=g)
            a1, n1 = ctl.proposal_stats()
            assert n1 == n0 + 1
            out.append((u0.cpu().numpy(), ctl.get_nominal().cpu().numpy(), ctl.sync_status(), a1 - a0))
        runs.append((out, ctl.step_counter))
    (o1, s1), (o2, s2) = runs
    assert s1 == s2
    assert o1[0][3] == int(accept)  # the first step takes the branch the inputs were made for
    for (u1, m1, st1, acc1), (u2, m2, st2, acc2) in zip(o1, o2):
        assert st1 == st2 and acc1 == acc2
        assert np.abs(u1 - u2).max() <= KNOT_TOL and np.abs(m1 - m2).max() <= KNOT_TOL


@pytest.mark.parametrize("variant", ["direct basis", "mixed arithmetic"])
@pytest.mark.parametrize("accept", [True, False])
def test_concurrent_gate_with_direct_basis_and_mixed_arithmetic(B, variant, accept):
    """The concurrent best-sample gate on the lane-split rollout with one value per control
    step (nk = H, noise drawn in the step loop) and with the mixed arithmetic: the oracle's
    proposal step within the knot bar, and the sequential gate's decision."""
    extra = dict(basis=3, nk=10) if variant == "direct basis" else dict(arith="mixed")
    md, p, orc, ctl = _ctl(B, H=10, lanes=16, **extra)
    D = 12 * p["nk"]
    rng = np.random.default_rng(4)
    mu = f32(W.stance_knots(p["nk"]))
    x0 = f32(W.initial_state(3))
    if accept:
        nominal = f32(mu + 0.5)
        center = f32(mu + 0.02 * rng.normal(size=D))
    else:
        nominal = mu
        center = f32(mu + 0.8)
    sd = f32(rng.uniform(0.05, 0.2, D))
    out = {}
    for g in ("best", "best-concurrent"):
        ctl.set_nominal(_dev(nominal))
        ctl.set_step(5)
        a0, _ = ctl.proposal_stats()
        u0 = ctl.step_proposal(_dev(x0), _dev(center), _dev(sd), 16, gate=g).cpu().numpy()
        out[g] = (u0, ctl.get_nominal().cpu().numpy(), ctl.proposal_stats()[0] - a0, ctl.sync_status())
    ou0, onom, cp, cf, oacc, rc = orc.mppi_step_proposal(p, 5, x0, nominal, center, sd, 16, gate=2)
    assert oacc == accept
    for g, (u0, nom, acc, st) in out.items():
        assert acc == int(accept) and st == (0 if accept else 2), g
        assert np.abs(u0 - ou0).max() <= KNOT_TOL and np.abs(nom - onom).max() <= KNOT_TOL, g


@pytest.mark.parametrize("lanes", [4, 16])
@pytest.mark.parametrize("gate", ["cost-concurrent", "best-concurrent"])
def test_concurrent_gate_falls_back_cleanly_from_a_corrupted_proposal(B, gate, lanes):
    """The one launch of the concurrent gate is centred on the nominal, so a proposal whose
    centre is not finite, or absurdly far off, spoils only its own samples: the gate
    rejects it and the step is the plain step within the FP32 rounding of the plain
    offsets, the acceptance counter unchanged."""
    md, p, orc, ctl = _ctl(B, K=64, H=10, lanes=lanes)
    D = 12 * p["nk"]
    x0 = f32(W.initial_state(5))
    mu = f32(W.stance_knots(p["nk"]))
    sd = np.full(D, 0.1, np.float32)
    ref = B.Controller(B.Model(md), p)
    for bad in (np.nan, 1.0e30):
        center = mu.copy()
        center[3] = bad
        for c in (ctl, ref):
            c.set_nominal(_dev(mu))
            c.set_step(2)
        a0, n0 = ctl.proposal_stats()
        u0 = ctl.step_proposal(_dev(x0), _dev(center), _dev(sd), 16, gate=gate).cpu().numpy()
        a1, n1 = ctl.proposal_stats()
        assert (a1 - a0, n1 - n0) == (0, 1)
        assert ctl.sync_status() == 2  # MPPI_WARN_FALLBACK
        ur = ref.step(_dev(x0)).cpu().numpy()
        assert np.all(np.isfinite(u0))
        assert np.abs(u0 - ur).max() <= KNOT_TOL
        assert np.abs(ctl.get_nominal().cpu().numpy() - ref.get_nominal().cpu().numpy()).max() <= KNOT_TOL


def test_concurrent_flag_rejected_without_a_gate(B):
    """The concurrent flag names a way to roll out the fallback: with gate none there is
    none, and the step is refused before any work."""
    md, p, orc, ctl = _ctl(B, lanes=16)
    D = 12 * p["nk"]
    mu = _dev(W.stance_knots(p["nk"]))
    x0 = _dev(W.initial_state(3))
    sd = _dev(np.full(D, 0.1))
    u0 = _dev(np.zeros(12))
    rc = B.lib().mppi_step_proposal(ctl.h, B._ptr(x0), B._ptr(mu), B._ptr(sd), 16, 1 | 4, B._ptr(u0))
    assert rc == -1


def test_learned_step_on_plain_kernels_matches_oracle_chain(B):
    """mppi_step through the policy: features, BF16 forward, head and proposal step against
    the oracle's features, BF16-operand forward, head and proposal step."""
    md, p, orc, ctl = _ctl(B, K=64, H=10)
    pol = B.Policy(max_batch=1, seed=5)
    rng = np.random.default_rng(6)
    im, isd = rng.normal(size=40) * 0.1, rng.uniform(0.5, 2.0, 40)
    om = np.repeat(np.tile(W.STANCE_JOINTS, 4), 6)   # joint-major: 6 knots per joint
    osd = np.full(72, 0.05)
    pol.set_normalization(im, isd, om, osd)
    cmd, origin = (0.5, 0.0, 0.0), (0.1, -0.2)
    ctl.set_proposal(pol, k_prop=16, cmd=cmd, origin=origin)
    x0 = f32(W.initial_state(2))
    mu = f32(W.stance_knots(p["nk"]))
    ctl.set_nominal(_dev(mu))
    ctl.set_step(0)
    u0 = ctl.step(_dev(x0)).cpu().numpy()
    nom = ctl.get_nominal().cpu().numpy()
    acc, steps = ctl.proposal_stats()
    feat = O.policy_features(x0, f32(cmd), f32(origin), f32(im), f32(isd))
    out = O.mlp_forward(_params(pol), feat[None], bf16=True)[0]
    c, sd = O.policy_head(out, f32(om), f32(osd), p["nk"], p["sigma"])
    ou0, onom, cp, cf, oacc, rc = orc.mppi_step_proposal(p, 0, x0, mu, f32(c), f32(sd), 16)
    assert steps == 1 and acc == int(oacc)
    assert np.abs(u0 - ou0).max() <= KNOT_TOL
    assert np.abs(nom - onom).max() <= KNOT_TOL
    ctl.set_proposal(None)
    ctl.step(_dev(x0))
    assert ctl.proposal_stats()[1] == 1  # plain steps are not counted


def test_trained_proposal_gains_over_plain_and_untrained_at_equal_samples(B):
    """What the trained network gains: closed-loop heightfield walks (3 seeds x 100 steps,
    v_ref 0.5) with the K/4 = 256-sample proposal (ungated, nominal kept as sample 1)
    against plain MPPI with the same 256 samples and against the untrained network; then
    in batched serving, where fewer samples also shorten the step."""
    from paper_2409_10469_amd import proposal as PR
    data = PR.generate(n_pairs=200000, episode_steps=100, instances=256, seed=11, log=lambda *a: None)
    tr, ho = PR.split(data, holdout=0.05, seed=0)
    norm = PR.normalization(data, tr)
    trained = B.Policy(max_batch=4096, seed=1)
    trained.set_normalization(*norm)
    PR.train(trained, data, tr, epochs=4, batch=4096, lr=1e-3, seed=0, held=None, log=lambda *a: None)
    untrained = B.Policy(max_batch=1, seed=1)
    untrained.set_normalization(*norm)
    wl = W.TERRAIN_WALK
    model = B.Model(W.model_dict(wl, 0))
    p = W.params_dict(wl, 0, v_ref=0.5)
    seeds, steps = (100, 101, 102), 100
    plain = np.mean([PR.episode(model, dict(p, K=256), s, steps)[0] for s in seeds])
    learned = np.mean([PR.episode(model, dict(p, K=1024), s, steps, policy=trained, k_prop=256, gate="none")[0]
                       for s in seeds])
    naive = np.mean([PR.episode(model, dict(p, K=1024), s, steps, policy=untrained, k_prop=256, gate="none")[0]
                     for s in seeds])
    assert np.isfinite([plain, learned, naive]).all()
    assert learned < 0.8 * plain, (learned, plain)
    assert learned < naive, (learned, naive)
    # batched serving (64 instances in one batch): the learned proposal at 256 samples
    # against plain MPPI at 256 samples (cost) and at 1024 samples (step latency)
    evb = PR.evaluate_batched(trained, n_inst=64, K_plain=(256, 1024), k_prop=256, steps=100, log=lambda *a: None)
    c = evb["controllers"]
    assert c["learned_K256"]["episode_cost"] < 0.8 * c["plain_K256"]["episode_cost"], c
    assert c["learned_K256"]["latency_ms"]["p99"] < c["plain_K1024"]["latency_ms"]["p99"], c
    # with plain MPPI kept as the fallback (best-sample gate, K = 1024 on a fallback):
    # the K/4 proposal reaches plain MPPI's cost at K with fewer samples rolled out per
    # step, counting every fallback's K samples
    lat_p, lat_l = [], []
    seeds = tuple(range(100, 106))
    plain_k = [PR.episode(model, dict(p, K=1024), s, steps, lat=lat_p)[0] for s in seeds]
    res = [PR.episode(model, dict(p, K=1024), s, steps, policy=trained, k_prop=256, gate="best", lat=lat_l)
           for s in seeds]
    learned_g = [r[0] for r in res]
    acc, n = sum(r[2] for r in res), sum(r[3] for r in res)
    samples = 256 + (1.0 - acc / n) * 1024
    half = lambda v: 1.96 * np.std(v, ddof=1) / np.sqrt(len(v))
    print("gated learned %.3f +- %.3f at %.0f samples/step (acceptance %.2f); plain K=1024 %.3f +- %.3f; "
          "p99 %.3f vs %.3f ms" % (np.mean(learned_g), half(learned_g), samples, acc / n, np.mean(plain_k),
                                   half(plain_k), np.percentile(lat_l, 99), np.percentile(lat_p, 99)))
    assert np.mean(learned_g) + half(learned_g) < np.mean(plain_k), (learned_g, plain_k)
    assert samples < 0.75 * 1024, samples


def test_corrupted_proposal_falls_back_to_the_plain_step(B):
    """A non-finite proposal centre fails the cost gate: the step is the plain step, bit
    for bit, and the acceptance counter does not move."""
    md, p, orc, ctl = _ctl(B, K=64, H=10)
    D = 12 * p["nk"]
    x0 = f32(W.initial_state(5))
    mu = f32(W.stance_knots(p["nk"]))
    center = mu.copy()
    center[3] = np.nan
    sd = np.full(D, 0.1, np.float32)
    ctl.set_nominal(_dev(mu))
    ctl.set_step(2)
    u0 = ctl.step_proposal(_dev(x0), _dev(center), _dev(sd), 16, gate="cost").cpu().numpy()
    nominal = ctl.get_nominal().cpu().numpy()
    acc, steps = ctl.proposal_stats()
    assert (acc, steps) == (0, 1)
    ref = B.Controller(B.Model(md), p)
    ref.set_nominal(_dev(mu))
    ref.set_step(2)
    assert np.array_equal(u0, ref.step(_dev(x0)).cpu().numpy())
    assert np.array_equal(nominal, ref.get_nominal().cpu().numpy())
    assert ctl.step_counter == ref.step_counter == 3
