"""Pins of the oracle's learned-proposal pieces (CPU): the network head (de-standardise,
resample 6 -> nk knots, clamp), the input features, and the proposal step's two branches
(the accepted update against per-sample rollouts and a brute-force softmax, the fallback
against the plain step)."""
import math

import numpy as np

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W


def test_head_identity_resample_and_destandardise():
    rng = np.random.default_rng(0)
    out = rng.normal(size=144) * 0.3
    mean, std = rng.normal(size=72), rng.uniform(0.5, 2.0, 72)
    c, sd = O.policy_head(out, mean, std, 6, 10.0)
    np.testing.assert_allclose(c, out[:72] * std + mean, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(sd, np.exp(out[72:]) * std, rtol=1e-14)


def test_head_resample_reproduces_cubics_and_clamps():
    # a cubic in normalised time is reproduced exactly by the not-a-knot spline, so the
    # resampled knots are the cubic at the new knot times
    cub = lambda t, j: 0.1 * j + 0.5 * t - 1.2 * t ** 2 + 0.7 * t ** 3
    out = np.zeros(144)
    for j in range(12):
        out[j * 6:(j + 1) * 6] = [cub(k / 5, j) for k in range(6)]
    out[72:] = 5.0                     # far above any clamp
    out[72:78] = -50.0                 # far below
    for nk in (2, 3, 4, 5, 7, 8):
        c, sd = O.policy_head(out, np.zeros(72), np.ones(72), nk, 0.3)
        want = np.array([cub(i / (nk - 1), j) for j in range(12) for i in range(nk)])
        np.testing.assert_allclose(c, want, atol=1e-13)
        np.testing.assert_allclose(sd[:nk], 0.02, rtol=1e-14)
        np.testing.assert_allclose(sd[nk:], 0.3, rtol=1e-14)


def test_features():
    x = np.arange(37.0)
    f = O.policy_features(x, [0.5, 0.1, -0.2], [10.0, -3.0], np.zeros(40), np.full(40, 2.0))
    want = np.concatenate([[0 - 10.0, 1 + 3.0], x[2:], [0.5, 0.1, -0.2]]) / 2.0
    np.testing.assert_array_equal(f, want)


def _setup(K=12, H=8):
    wl = W.FLAT_WALK
    o = O.Oracle(W.model_dict(wl, 0))
    p = W.params_dict(wl, 5, K=K, H=H)
    x0 = W.initial_state(5, wl["scene"])
    mu = W.stance_knots(p["nk"])
    return o, p, x0, mu


def test_proposal_accepted_branch_is_weighted_mean_of_its_samples():
    o, p, x0, mu = _setup()
    D = 12 * p["nk"]
    rng = np.random.default_rng(1)
    center = mu + 0.02 * rng.normal(size=D)
    sd = rng.uniform(0.05, 0.2, D)
    Kp = 7
    # make the proposal mean the better of the two: the nominal is perturbed badly
    bad_mu = mu + 0.6
    u0, nom, cp, cf, acc, rc = o.mppi_step_proposal(p, 3, x0, bad_mu, center, sd, Kp)
    assert acc and rc == 0 and not cf.any()
    eps = O.sample_eps(dict(p, K=Kp), 3)
    thetas = [center, bad_mu] + [center + sd * eps[n] for n in range(2, Kp)]
    L = np.array([o.rollout(p, x0, th) for th in thetas])
    np.testing.assert_allclose(cp, L, rtol=1e-13)
    assert L[0] <= L[1]
    w = np.exp(-(L - L.min()) / p["lam"])
    w /= w.sum()
    mup = sum(wi * th for wi, th in zip(w, thetas))
    want_nom, want_u0 = O.shift(p, mup)
    np.testing.assert_allclose(nom, want_nom, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(u0, want_u0, rtol=1e-12, atol=1e-14)


def test_proposal_fallback_is_the_plain_step():
    o, p, x0, mu = _setup()
    D = 12 * p["nk"]
    center = mu + 0.8          # far worse than the nominal
    sd = np.full(D, 0.1)
    u0, nom, cp, cf, acc, rc = o.mppi_step_proposal(p, 2, x0, mu, center, sd, 5)
    assert not acc
    assert cp[0] > cp[1]
    u0p, nomp, costsp, rcp = o.mppi_step(p, 2, x0, mu)
    np.testing.assert_array_equal(u0, u0p)
    np.testing.assert_array_equal(nom, nomp)
    np.testing.assert_array_equal(cf, costsp)
    assert rc == rcp


def test_proposal_nonfinite_mean_falls_back():
    o, p, x0, mu = _setup()
    D = 12 * p["nk"]
    center = np.full(D, np.nan)
    u0, nom, cp, cf, acc, rc = o.mppi_step_proposal(p, 0, x0, mu, center, np.full(D, 0.1), 4)
    assert not acc and math.isinf(cp[0])
    u0p, nomp, _, _ = o.mppi_step(p, 0, x0, mu)
    np.testing.assert_array_equal(nom, nomp)


def test_ungated_proposal_takes_the_proposal_samples():
    """gate 1: the weighted mean of the proposal samples even when the centre is worse."""
    o, p, x0, mu = _setup()
    D = 12 * p["nk"]
    center = mu + 0.8
    sd = np.full(D, 0.1)
    Kp = 6
    u0, nom, cp, cf, acc, rc = o.mppi_step_proposal(p, 1, x0, mu, center, sd, Kp, gate=1)
    assert acc and cp[0] > cp[1] and not cf.any()
    eps = O.sample_eps(dict(p, K=Kp), 1)
    thetas = [center, mu] + [center + sd * eps[n] for n in range(2, Kp)]
    L = np.array([o.rollout(p, x0, th) for th in thetas])
    w = np.exp(-(L - L.min()) / p["lam"])
    w /= w.sum()
    want_nom, want_u0 = O.shift(p, sum(wi * th for wi, th in zip(w, thetas)))
    np.testing.assert_allclose(nom, want_nom, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(u0, want_u0, rtol=1e-12, atol=1e-14)


def test_best_sample_gate_decides_on_the_least_proposal_cost():
    """gate 2: the proposal is taken when its least cost over the samples other than the
    nominal (sample 1) is not above the nominal's -- checked against per-sample rollouts --
    and the step is then the weighted mean of the proposal samples, else the plain step."""
    o, p, x0, mu = _setup()
    D = 12 * p["nk"]
    Kp = 6
    seen = set()
    for k, off in enumerate((0.02, 0.15, 0.3, 0.6, 0.9)):
        rng = np.random.default_rng(20 + k)
        center = mu + off * rng.choice([-1.0, 1.0], D)
        sd = np.full(D, 0.08)
        u0, nom, cp, cf, acc, rc = o.mppi_step_proposal(p, 4, x0, mu, center, sd, Kp, gate=2)
        eps = O.sample_eps(dict(p, K=Kp), 4)
        thetas = [center, mu] + [center + sd * eps[n] for n in range(2, Kp)]
        L = np.array([o.rollout(p, x0, th) for th in thetas])
        np.testing.assert_allclose(cp, L, rtol=1e-13)
        want_acc = bool(np.delete(L, 1).min() <= L[1])
        assert acc == want_acc
        seen.add(acc)
        if acc:
            w = np.exp(-(L - L.min()) / p["lam"])
            w /= w.sum()
            want_nom, want_u0 = O.shift(p, sum(wi * th for wi, th in zip(w, thetas)))
        else:
            want_u0, want_nom, _, _ = o.mppi_step(p, 4, x0, mu)
        np.testing.assert_allclose(nom, want_nom, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(u0, want_u0, rtol=1e-12, atol=1e-14)
    assert seen == {True, False}  # both branches exercised
