"""Pins of the oracle's composite functions against their separately pinned parts (CPU
only):
  * the implicit system of one step (Sec. III-A dynamics, linearly implicit in
    velocity) against the mass matrix, the bias and the PD law;
  * the step against the solve of that system and the base retraction;
  * a rollout (Algorithm 1 inner loop) against a chain of steps with the interpolated
    joint targets and the running cost;
  * a batch of rollouts against per-sample rollouts of theta = mu + sigma eps;
  * one MPPI step (Algorithm 1) against sampling, rollouts, the Eq. 1 / Eq. 2 update and
    the shift.
A wrong index, a dropped term or a misplaced time step in a composite fails here even
when each part is right.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W

NQ, NV = 19, 18
KP, KD = 40.0, 1.0


def _air_state(seed):
    """The robot high above the ground (no contact) with random velocities."""
    rng = np.random.default_rng(seed)
    x = W.initial_state(seed)
    x[2] = 5.0
    q = rng.normal(size=4)
    x[3:7] = q / np.linalg.norm(q)
    x[19:37] = rng.normal(size=18) * 0.5
    return x


def test_step_system_without_contact_is_mass_matrix_bias_and_pd():
    m = O.Oracle(W.model_dict(W.FLAT_WALK, 0))
    rng = np.random.default_rng(1)
    x = _air_state(1)
    u = np.tile(W.STANCE_JOINTS, 4) + rng.normal(size=12) * 0.2
    dt = 0.02
    A, r, n = m.step_system(x, u, KP, KD, dt)
    assert n == 0
    q, v = x[:NQ], x[NQ:]
    E = np.zeros((NV, NV))
    E[6:, 6:] = KD * np.eye(12)
    np.testing.assert_allclose(A, m.mass_matrix(q) + dt * E, rtol=1e-12, atol=1e-14)
    f = -m.bias(q, v)
    f[6:] += KP * (u - q[7:]) - KD * v[6:]
    np.testing.assert_allclose(r, dt * f, rtol=1e-12, atol=1e-14)


def test_step_system_in_contact_adds_symmetric_psd_damping():
    m = O.Oracle(W.model_dict(W.FLAT_WALK, 0))
    x = W.initial_state(2)  # standing: the feet touch the ground
    x[19:37] = np.random.default_rng(2).normal(size=18) * 0.1
    u = np.tile(W.STANCE_JOINTS, 4)
    dt = 0.02
    A, _, n = m.step_system(x, u, KP, KD, dt)
    assert n > 0
    np.testing.assert_allclose(A, A.T, atol=1e-9 * np.abs(A).max())
    E = np.zeros((NV, NV))
    E[6:, 6:] = KD * np.eye(12)
    C = A - m.mass_matrix(x[:NQ]) - dt * E  # dt times the contact damping
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() >= -1e-9 * np.abs(C).max()
    assert np.abs(C).max() > 0


@pytest.mark.parametrize("scene_state", ["air", "standing"])
def test_step_is_the_solve_and_the_base_retraction(scene_state):
    m = O.Oracle(W.model_dict(W.FLAT_WALK, 0))
    x = _air_state(3) if scene_state == "air" else W.initial_state(3)
    u = np.tile(W.STANCE_JOINTS, 4) + np.random.default_rng(3).normal(size=12) * 0.1
    dt = 0.02
    A, r, _ = m.step_system(x, u, KP, KD, dt)
    v1 = x[NQ:] + np.linalg.solve(A, r)
    q1 = m.retract(x[:NQ], v1, dt)
    q1[3:7] /= np.linalg.norm(q1[3:7])  # the step renormalises the quaternion
    xo, tau, rc = m.step(x, u, KP, KD, dt)
    assert rc == 0
    np.testing.assert_allclose(xo[NQ:], v1, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(xo[:NQ], q1, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(tau, KP * (u - x[7:NQ]) - KD * x[NQ + 6:], rtol=1e-14)


@pytest.mark.parametrize("basis", [0, 1, 2])
def test_rollout_is_a_chain_of_steps_with_interpolated_targets(basis):
    wl = W.TERRAIN_WALK
    m = O.Oracle(W.model_dict(wl, 0))
    p = W.params_dict(wl, 0, H=12, nk=4, basis=basis)
    x0 = W.initial_state(4, wl["scene"])
    theta = W.stance_knots(4) + np.random.default_rng(4).normal(size=48) * 0.1
    L, traj = m.rollout(p, x0, theta, traj=True)
    Bm = O.basis_matrix(basis, 4, p["H"], p["dt"])
    x, want = x0.copy(), 0.0
    for k in range(p["H"]):
        u = theta.reshape(12, 4) @ Bm[k]  # joint targets of step k
        x, tau, rc = m.step(x, u, p["kp"], p["kd"], p["dt"])
        assert rc == 0
        want += p["dt"] * m.stage_cost(p, x, tau)  # cost at the post-step state
        # the targets' summation order differs from the oracle's loop: last-bit
        # differences, amplified by the contact stiffness
        np.testing.assert_allclose(traj[k + 1], x, rtol=1e-10, atol=1e-11)
    assert L == pytest.approx(want, rel=1e-10)


def test_rollout_batch_is_per_sample_rollouts():
    wl = W.FLAT_WALK
    m = O.Oracle(W.model_dict(wl, 0))
    p = W.params_dict(wl, 0, K=5, H=6)
    D = 12 * p["nk"]
    x0 = W.initial_state(5)
    mu = W.stance_knots(p["nk"]) + np.random.default_rng(5).normal(size=D) * 0.05
    eps = np.random.default_rng(6).normal(size=(p["K"], D))
    costs = m.rollout_batch(p, x0, mu, eps)
    for n in range(p["K"]):
        theta = mu + (p["sigma"] * eps[n] if n else 0.0)  # sample 0 is the nominal
        assert costs[n] == pytest.approx(m.rollout(p, x0, theta), rel=1e-13)


def test_mppi_step_is_sample_rollouts_update_and_shift():
    wl = W.FLAT_WALK
    m = O.Oracle(W.model_dict(wl, 0))
    p = W.params_dict(wl, 123, K=9, H=8, instance=4)
    D = 12 * p["nk"]
    x0 = W.initial_state(6)
    mu = W.stance_knots(p["nk"]) + np.random.default_rng(7).normal(size=D) * 0.05
    step = 3
    u0, mu_new, costs, rc = m.mppi_step(p, step, x0, mu)
    eps = O.sample_eps(p, step)  # the step's own Philox counters
    want_costs = m.rollout_batch(p, x0, mu, eps)
    np.testing.assert_allclose(costs, want_costs, rtol=1e-13)
    mup, _, _ = O.update(p, want_costs, mu, eps)
    want_mu, want_u0 = O.shift(p, mup)
    np.testing.assert_allclose(u0, want_u0, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(mu_new, want_mu, rtol=1e-12, atol=1e-14)
