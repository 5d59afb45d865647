"""Pins of the oracle's tracking cost (Eq. 3 with a trotting gait reference, Eq. 4 box
term), CPU only:
  * leg inverse kinematics against the oracle's pinned forward kinematics (round trip
    over the workspace, the standing pose, clamping along the foot direction);
  * the gait's foot path: continuity at every phase boundary, diagonal pairs in phase
    and half a period apart, apex height at mid-swing, a stance foot at rest in the
    world while the base moves at the commanded velocity, the Raibert foothold shift;
  * joint references = IK of the foot path; invariance under a yaw rotation of the
    base together with its velocity and the command;
  * the stage: zero on the reference, each weight alone against an independently built
    deviation (a rotation by a known angle for the attitude), the l1 box term;
  * composites: trajectory cost = sum of stages with interpolated controls at the
    right times; rollout = dynamics trajectory + cost; MPPI step = sampling, rollouts,
    Eq. 1 / Eq. 2 update and shift.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W

NQ = 19
L1 = W.ROBOT["thigh_len"]
L2 = W.ROBOT["calf_len"]
HIPS = np.array([[W.ROBOT["hip_x"], W.ROBOT["hip_y"], 0.0], [W.ROBOT["hip_x"], -W.ROBOT["hip_y"], 0.0],
                 [-W.ROBOT["hip_x"], W.ROBOT["hip_y"], 0.0], [-W.ROBOT["hip_x"], -W.ROBOT["hip_y"], 0.0]])


@pytest.fixture(scope="module")
def orc():
    return O.Oracle(W.model_dict(W.FLAT_WALK, 0))


def _q_at_origin(joints):
    q = np.zeros(NQ)
    q[3] = 1.0
    q[7:] = joints
    return q


def _feet_rel(orc, joints):
    """Foot centres relative to their hips, trunk at the origin, identity attitude."""
    return orc.feet(_q_at_origin(joints)) - HIPS


def _quat_axis_angle(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * a])


def test_ik_round_trip_through_forward_kinematics(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        # points well inside the reach: distance in [0.1, 0.4] m, below the hip
        d = rng.uniform(0.1, 0.4)
        v = rng.normal(size=3)
        v[2] = -abs(v[2]) - 0.5
        p = d * v / np.linalg.norm(v)
        q = orc.leg_ik(p)
        assert -math.pi <= q[2] <= 0.0  # knee bent backwards
        rel = _feet_rel(orc, np.tile(q, 4))
        for leg in range(4):  # the same joint angles put every foot at p from its hip
            np.testing.assert_allclose(rel[leg], p, atol=1e-12)


def test_ik_of_the_foot_under_the_hip_is_the_standing_pose(orc):
    h = (L1 + L2) * math.cos(0.9)
    np.testing.assert_allclose(orc.leg_ik([0.0, 0.0, -h]), W.STANCE_JOINTS, atol=1e-12)


def test_ik_clamps_reach_along_the_foot_direction(orc):
    far = np.array([0.3, 0.1, -0.5])
    q = orc.leg_ik(far)
    rel = _feet_rel(orc, np.tile(q, 4))[0]
    assert np.linalg.norm(rel) == pytest.approx(0.999 * (L1 + L2), rel=1e-12)
    np.testing.assert_allclose(rel / np.linalg.norm(rel), far / np.linalg.norm(far), atol=1e-12)


def _trot(**kw):
    return W.tracking_cost(gait=1, **kw)


def test_foot_path_is_continuous_at_every_phase_boundary():
    c = _trot()
    T, duty = c["period"], c["duty"]
    cmd = np.array([0.5, 0.1])
    v = np.array([0.3, -0.05])
    for leg in range(4):
        off = 0.0 if leg in (0, 3) else 0.5
        for phase in (duty, 1.0):  # stance -> swing, swing -> next stance
            t = (phase - off) * T + 3 * T  # a later period, any leg
            a = O.gait_foot(c, leg, t - 1e-9, v, cmd)
            b = O.gait_foot(c, leg, t + 1e-9, v, cmd)
            np.testing.assert_allclose(a, b, atol=1e-6)


def test_diagonal_pairs_move_together_and_half_a_period_apart():
    c = _trot()
    T = c["period"]
    cmd, v = np.array([0.4, 0.0]), np.array([0.45, 0.02])
    for t in np.linspace(0.0, 2 * T, 37):
        f = [O.gait_foot(c, leg, t, v, cmd) for leg in range(4)]
        np.testing.assert_array_equal(f[0], f[3])
        np.testing.assert_array_equal(f[1], f[2])
        np.testing.assert_allclose(f[1], O.gait_foot(c, 0, t + T / 2, v, cmd), atol=1e-12)


def test_swing_apex_and_stance_height():
    c = _trot()
    T, duty = c["period"], c["duty"]
    cmd = np.array([0.5, 0.0])
    mid_swing = (duty + (1 - duty) / 2) * T
    f = O.gait_foot(c, 0, mid_swing, cmd, cmd)
    assert f[2] == pytest.approx(-c["stand_height"] + c["swing_height"], abs=1e-12)
    assert f[0] == pytest.approx(0.0, abs=1e-12)  # halfway between lift-off and touchdown
    for t in np.linspace(0, duty * T, 9)[:-1]:
        assert O.gait_foot(c, 0, t, cmd, cmd)[2] == pytest.approx(-c["stand_height"], abs=1e-15)


def test_stance_foot_rests_in_the_world_when_the_base_moves_at_the_command():
    c = _trot()
    T, duty = c["period"], c["duty"]
    cmd = np.array([0.6, -0.2])
    ts = np.linspace(0.0, duty * T, 11)[:-1]
    world = [O.gait_foot(c, 0, t, cmd, cmd)[:2] + cmd * t for t in ts]  # hip moves at cmd
    np.testing.assert_allclose(np.ptp(np.array(world), axis=0), 0.0, atol=1e-12)
    # the stride is centred under the hip (Raibert neutral point at zero velocity error)
    touchdown = O.gait_foot(c, 0, 0.0, cmd, cmd)[:2]
    liftoff = O.gait_foot(c, 0, duty * T - 1e-12, cmd, cmd)[:2]
    np.testing.assert_allclose(touchdown + liftoff, 0.0, atol=1e-9)


def test_raibert_foothold_moves_with_the_velocity_error():
    c = _trot()
    cmd = np.array([0.5, 0.0])
    base = O.gait_foot(c, 0, 0.0, cmd, cmd)
    err = np.array([0.2, -0.1])
    moved = O.gait_foot(c, 0, 0.0, cmd + err, cmd)
    np.testing.assert_allclose(moved[:2] - base[:2], c["raibert_k"] * err, atol=1e-12)


def test_joint_reference_is_ik_of_the_foot_path(orc):
    c = _trot()
    x0 = W.initial_state(3)
    x0[19:21] = (0.3, 0.05)
    for t in (0.0, 0.07, 0.26, 0.41):
        u = orc.gait_reference(c, t, x0)
        rel = _feet_rel(orc, u)
        for leg in range(4):
            want = O.gait_foot(c, leg, t, x0[19:21], np.array(c["v_cmd"]))
            np.testing.assert_allclose(rel[leg], want, atol=1e-12)


def test_standing_gait_is_the_standing_pose_at_all_times(orc):
    c = W.tracking_cost(gait=0, stand_height=(L1 + L2) * math.cos(0.9))
    x0 = W.initial_state(4)
    for t in (0.0, 0.13, 1.7):
        np.testing.assert_allclose(orc.gait_reference(c, t, x0), np.tile(W.STANCE_JOINTS, 4), atol=1e-12)


def test_joint_reference_is_invariant_under_a_yaw_of_base_velocity_and_command(orc):
    psi = 0.7
    Rz = np.array([[math.cos(psi), -math.sin(psi)], [math.sin(psi), math.cos(psi)]])
    c = _trot(v_cmd=(0.5, 0.1))
    x0 = W.initial_state(5)
    x0[19:21] = (0.35, -0.05)
    x1 = x0.copy()
    x1[3:7] = _quat_axis_angle([0, 0, 1], psi)
    x1[19:21] = Rz @ x0[19:21]
    c1 = dict(c, v_cmd=tuple(Rz @ np.array(c["v_cmd"])))
    for t in (0.05, 0.3):
        np.testing.assert_allclose(orc.gait_reference(c1, t, x1), orc.gait_reference(c, t, x0), atol=1e-12)


def _reference_state(orc, c, t, q_ref):
    x = np.zeros(orc.nx)
    x[0:2] = np.array(c["p_ref0"][:2]) + np.array(c["v_cmd"]) * t
    x[2] = c["p_ref0"][2]
    x[3] = 1.0
    x[7:19] = q_ref
    x[19:21] = c["v_cmd"]
    return x


def test_stage_is_zero_on_the_reference_and_each_weight_alone(orc):
    c = _trot(v_cmd=(0.4, -0.1), origin=(0.3, -0.2))
    rng = np.random.default_rng(6)
    t = 0.37
    q_ref = np.tile(W.STANCE_JOINTS, 4) + rng.normal(size=12) * 0.1
    u_ref = q_ref + rng.normal(size=12) * 0.05
    x = _reference_state(orc, c, t, q_ref)
    assert orc.tracking_stage(c, t, x, q_ref, u_ref, u_ref) <= 1e-30  # rounding of p_ref(t) only
    Q, R = np.array(c["Q"]), np.array(c["R"])

    def one(xm, u=u_ref):
        return orc.tracking_stage(c, t, xm, q_ref, u, u_ref)

    d = 0.013
    for i, idx in ((0, 0), (1, 1), (2, 2)):  # base position
        xm = x.copy()
        xm[idx] += d
        assert one(xm) == pytest.approx(Q[i] * d * d, rel=1e-9)
    for j in range(12):  # joints, joint velocities
        xm = x.copy()
        xm[7 + j] += d
        assert one(xm) == pytest.approx(Q[6 + j] * d * d, rel=1e-9)
        xm = x.copy()
        xm[25 + j] += d
        assert one(xm) == pytest.approx(Q[24 + j] * d * d, rel=1e-9)
    for i in range(3):  # base linear and angular velocity
        xm = x.copy()
        xm[19 + i] += d
        assert one(xm) == pytest.approx(Q[18 + i] * d * d, rel=1e-9)
        xm = x.copy()
        xm[22 + i] += d
        assert one(xm) == pytest.approx(Q[21 + i] * d * d, rel=1e-9)
    for j in range(12):  # controls
        u = u_ref.copy()
        u[j] += d
        assert one(x, u) == pytest.approx(R[j] * d * d, rel=1e-9)
    # attitude: a rotation by angle a about each axis costs Q (2 sin(a/2))^2, for q and -q
    for i, axis in enumerate(np.eye(3)):
        for a in (0.05, 0.4):
            xm = x.copy()
            xm[3:7] = _quat_axis_angle(axis, a)
            want = Q[3 + i] * (2 * math.sin(a / 2)) ** 2
            assert one(xm) == pytest.approx(want, rel=1e-9)
            xm[3:7] = -xm[3:7]
            assert one(xm) == pytest.approx(want, rel=1e-9)


def test_box_term_is_the_weighted_l1_distance():
    orc = O.Oracle(W.model_dict(W.BOX_PUSH, 0))
    c = _trot(box_goal_xy=(2.0, -0.5))
    t = 0.2
    q_ref = np.tile(W.STANCE_JOINTS, 4)
    x = _reference_state(orc, c, t, q_ref)
    for bx, by in ((2.0, -0.5), (1.3, 0.2), (2.4, -1.1)):
        x[37:39] = (bx, by)
        want = c["box_w"] * (abs(2.0 - bx) + abs(-0.5 - by))
        assert orc.tracking_stage(c, t, x, q_ref, q_ref, q_ref) == pytest.approx(want, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("basis", [0, 1])
def test_trajectory_cost_is_the_sum_of_stages_at_the_right_times(orc, basis):
    wl = W.FLAT_WALK
    p = W.params_dict(wl, 0, H=9, nk=4, basis=basis)
    c = _trot()
    x0 = W.initial_state(7)
    theta = W.stance_knots(4) + np.random.default_rng(7).normal(size=48) * 0.1
    step = 13
    L, traj = orc.rollout_tracking(p, c, step, x0, theta, traj=True)
    _, traj_dyn = orc.rollout(p, x0, theta, traj=True)
    np.testing.assert_array_equal(traj, traj_dyn)  # same dynamics as the plain rollout
    Bm = O.basis_matrix(basis, 4, p["H"], p["dt"])
    u = np.array([theta.reshape(12, 4) @ Bm[k] for k in range(p["H"])])
    assert orc.tracking_cost(p, c, step, traj, u) == L
    want = 0.0
    for k in range(p["H"]):
        tk, tx = (step + k) * p["dt"], (step + k + 1) * p["dt"]
        want += p["dt"] * orc.tracking_stage(c, tx, traj[k + 1], orc.gait_reference(c, tx, x0), u[k],
                                             orc.gait_reference(c, tk, x0))
    assert L == pytest.approx(want, rel=1e-12)


def test_mppi_step_with_tracking_is_sample_rollouts_update_and_shift(orc):
    p = W.params_dict(W.FLAT_WALK, 321, K=7, H=8, instance=2)
    c = _trot()
    D = 12 * p["nk"]
    x0 = W.initial_state(8)
    mu = W.stance_knots(p["nk"]) + np.random.default_rng(8).normal(size=D) * 0.05
    step = 5
    u0, mu_new, costs, rc = orc.mppi_step_tracking(p, c, step, x0, mu)
    assert rc == 0
    eps = O.sample_eps(p, step)
    want = [orc.rollout_tracking(p, c, step, x0, mu + (p["sigma"] * eps[n] if n else 0.0)) for n in range(p["K"])]
    np.testing.assert_allclose(costs, want, rtol=1e-13)
    mup, _, _ = O.update(p, np.array(want), mu, eps)
    want_mu, want_u0 = O.shift(p, mup)
    np.testing.assert_allclose(mu_new, want_mu, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(u0, want_u0, rtol=1e-12, atol=1e-14)
