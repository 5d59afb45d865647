"""Pins of the oracle's rigid-body terms (CPU only).

The whole-body simulator of Sec. III-A is replaced by floating-base rigid-body dynamics.
Its mass matrix and bias forces are pinned against quantities computed independently:
finite differences of the kinetic energy built from forward kinematics, finite
differences of the potential energy, Christoffel symbols of the mass matrix, energy
conservation and momentum conservation under RK4 integration, and closed forms.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W

NV = 18


def _model(**kw):
    d = W.model_dict(W.FLAT_WALK, 0)
    d.update(kw)
    return O.Oracle(d)


def _random_config(rng, z=0.3):
    q = np.zeros(19)
    q[:3] = rng.uniform(-0.5, 0.5, 3)
    q[2] = z
    quat = rng.normal(size=4)
    q[3:7] = quat / np.linalg.norm(quat)
    q[7:19] = np.tile(W.STANCE_JOINTS, 4) + rng.uniform(-0.6, 0.6, 12)
    return q


def test_fk_closed_forms():
    m = _model()
    q = np.zeros(19)
    q[3] = 1.0
    q[:3] = (0.1, -0.2, 0.5)
    r = W.ROBOT
    L = r["thigh_len"] + r["calf_len"]
    for leg, (sx, sy) in enumerate([(1, 1), (1, -1), (-1, 1), (-1, -1)]):
        want = np.array([0.1 + sx * r["hip_x"], -0.2 + sy * r["hip_y"], 0.5 - L])
        np.testing.assert_allclose(m.feet(q)[leg], want, atol=1e-12)
    q[7:19] = np.tile(W.STANCE_JOINTS, 4)
    feet = m.feet(q)
    for leg, (sx, sy) in enumerate([(1, 1), (1, -1), (-1, 1), (-1, -1)]):
        want = np.array([0.1 + sx * r["hip_x"], -0.2 + sy * r["hip_y"], 0.5 - L * math.cos(0.9)])
        np.testing.assert_allclose(feet[leg], want, atol=1e-12)


def test_fk_abduction_rotates_about_x():
    m = _model()
    q = np.zeros(19)
    q[3] = 1.0
    q[7] = 0.3  # FL abduction
    r = W.ROBOT
    L = r["thigh_len"] + r["calf_len"]
    want = np.array([r["hip_x"], r["hip_y"] + L * math.sin(0.3), -L * math.cos(0.3)])
    np.testing.assert_allclose(m.feet(q)[0], want, atol=1e-12)


def test_mass_matrix_closed_form_blocks():
    m = _model()
    rng = np.random.default_rng(0)
    for _ in range(5):
        q = _random_config(rng)
        M = m.mass_matrix(q)
        np.testing.assert_allclose(M, M.T, atol=1e-13)
        assert np.linalg.eigvalsh(M).min() > 0
        np.testing.assert_allclose(M[:3, :3], 10.0 * np.eye(3), atol=1e-12)
        R, _, com = m.fk(q)
        masses = np.array([W.ROBOT["trunk_mass"]] + [0.0, W.ROBOT["thigh_mass"], W.ROBOT["calf_mass"]] * 4)
        c = (masses[:, None] * com).sum(0) / masses.sum() - q[:3]
        skew = np.array([[0, -c[2], c[1]], [c[2], 0, -c[0]], [-c[1], c[0], 0]])
        # linear momentum per unit body-frame angular velocity: (R e_k) x (c - p) * m
        np.testing.assert_allclose(M[:3, 3:6], -10.0 * skew @ R[0], atol=1e-12)


def test_mass_matrix_from_kinetic_energy_fd():
    """M_ij by polarisation of T(v) = 1/2 sum m|c_dot|^2 + 1/2 w^T I w, where the body
    velocities come from central differences of forward kinematics."""
    m = _model()
    rng = np.random.default_rng(1)
    for _ in range(3):
        q = _random_config(rng)
        M = m.mass_matrix(q)
        Mfd = np.zeros((NV, NV))
        E = np.eye(NV)
        Tii = [m.kinetic_energy_fd(q, E[i], 1e-5) for i in range(NV)]
        for i in range(NV):
            Mfd[i, i] = 2 * Tii[i]
            for j in range(i + 1, NV):
                Mfd[i, j] = Mfd[j, i] = m.kinetic_energy_fd(q, E[i] + E[j], 1e-5) - Tii[i] - Tii[j]
        np.testing.assert_allclose(M, Mfd, rtol=0, atol=1e-7 * np.abs(M).max())


def test_gravity_is_gradient_of_potential():
    m = _model()
    rng = np.random.default_rng(2)
    for _ in range(3):
        q = _random_config(rng)
        g = m.bias(q, np.zeros(NV))
        h = 1e-6
        gfd = np.array([(m.potential_energy(m.retract(q, e, h)) - m.potential_energy(m.retract(q, e, -h))) / (2 * h)
                        for e in np.eye(NV)])
        np.testing.assert_allclose(g, gfd, rtol=0, atol=1e-6 * np.abs(g).max())


def test_joint_coriolis_from_christoffel_symbols():
    """With the base at rest, the joint rows of b - g equal the Christoffel form
    sum_jk (dM_ij/dq_k - 1/2 dM_jk/dq_i) v_j v_k (joint coordinates are true coordinates)."""
    m = _model(gravity=0.0)
    rng = np.random.default_rng(3)
    q = _random_config(rng)
    v = np.zeros(NV)
    v[6:] = rng.normal(size=12)
    h = 1e-6
    dM = np.zeros((NV, NV, NV))  # dM[:, :, k] = dM/dq_k (joints only)
    for k in range(6, NV):
        e = np.zeros(NV)
        e[k] = 1
        dM[:, :, k] = (m.mass_matrix(m.retract(q, e, h)) - m.mass_matrix(m.retract(q, e, -h))) / (2 * h)
    want = np.zeros(NV)
    for i in range(6, NV):
        want[i] = np.einsum("jk,j,k->", dM[i, :, :], v, v) - 0.5 * np.einsum("jk,j,k->", dM[:, :, i], v, v)
    b = m.bias(q, v)
    np.testing.assert_allclose(b[6:], want[6:], rtol=0, atol=1e-6 * np.abs(b[6:]).max())


def _airborne_state(rng):
    q = _random_config(rng, z=3.0)
    v = rng.normal(size=NV) * 0.8
    return q, v


def test_energy_conserved_without_contact_and_damping():
    """T + V_gravity + V_springs is conserved by the continuous dynamics (RK4, dt=1e-4, 1 s)."""
    kp = 40.0
    m = _model()
    rng = np.random.default_rng(4)
    q, v = _airborne_state(rng)
    target = np.tile(W.STANCE_JOINTS, 4)

    def energy(q, v):
        return (m.kinetic_energy(q, v) + m.potential_energy(q) + 0.5 * kp * np.sum((target - q[7:]) ** 2))

    E0 = energy(q, v)
    q1, v1 = m.rk4(q, v, 1e-4, 10000, spring_target=target, kp=kp)
    assert abs(energy(q1, v1) - E0) < 1e-9 * abs(E0)


def test_momentum_conserved_in_free_flight():
    kp = 40.0
    m = _model(gravity=0.0)
    rng = np.random.default_rng(5)
    q, v = _airborne_state(rng)
    target = np.tile(W.STANCE_JOINTS, 4)
    P0, L0 = m.momentum(q, v)
    # instantaneous: momentum rate is zero at the accelerations the dynamics produce
    tau = np.zeros(NV)
    tau[6:] = kp * (target - q[7:])
    a = m.accel(q, v, tau)
    h = 1e-6
    Pp, Lp = m.momentum(m.retract(q, v, h), v + h * a)
    Pm, Lm = m.momentum(m.retract(q, v, -h), v - h * a)
    assert np.abs((Pp - Pm) / (2 * h)).max() < 1e-6
    assert np.abs((Lp - Lm) / (2 * h)).max() < 1e-6
    q1, v1 = m.rk4(q, v, 1e-4, 5000, spring_target=target, kp=kp)
    P1, L1 = m.momentum(q1, v1)
    np.testing.assert_allclose(P1, P0, atol=1e-10 * max(1, np.abs(P0).max()))
    np.testing.assert_allclose(L1, L0, atol=1e-9 * max(1, np.abs(L0).max()))


def test_free_fall_of_whole_robot():
    """With no contact and no joint torque the centre of mass falls at g."""
    m = _model()
    rng = np.random.default_rng(6)
    q, v = _airborne_state(rng)
    a = m.accel(q, v, np.zeros(NV))
    P0, _ = m.momentum(q, v)
    h = 1e-6
    Pp, _ = m.momentum(m.retract(q, v, h), v + h * a)
    Pm, _ = m.momentum(m.retract(q, v, -h), v - h * a)
    np.testing.assert_allclose((Pp - Pm) / (2 * h), [0, 0, -10.0 * 9.81], atol=1e-5)
