"""Pins of the oracle's box and terrain contact geometry (CPU only).

The box-climb (Sec. IV-C) and box-push (Sec. IV-D) scenes rest on three geometric
primitives: a foot sphere against an oriented box (closest point), a point inside an
oriented box (shallowest face) and the heightfield below a point (bilinear).  Each is
pinned here by geometry that does not use the oracle's own formulas:
  * a sphere beside a face, an edge or a corner of a rotated box has its closest box
    point on that face, edge or corner, so depth and normal follow from the local offset;
  * the closest point of random outside points agrees with a brute-force search over a
    dense sample of the solid box;
  * inside the box, the shallowest face is the one with the least distance to go;
  * a bilinear heightfield h = a x y is reproduced exactly by bilinear interpolation, so
    height, slope and normal have closed forms, and a wrong corner weight fails;
  * every robot-box pair applies equal and opposite forces (Newton's third law);
  * a contact that separates faster than k delta / c pulls (no clamp on the normal law,
    the reading of Sec. III-A's soft contact taken here) and then has no friction.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_10469_amd import workloads as W

HALF = np.array([0.2, 0.15, 0.1])
CENTRE = np.array([0.3, -0.2, 0.5])


def _rot(axis, ang):
    """Rodrigues rotation matrix and the matching unit quaternion (w, x, y, z)."""
    u = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    R = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    q = np.r_[math.cos(ang / 2), math.sin(ang / 2) * u]
    return R, q


POSES = [_rot((0, 0, 1), 0.0), _rot((0, 0, 1), 0.7), _rot((1, 2, -0.5), 1.9)]


@pytest.mark.parametrize("pose", range(len(POSES)))
def test_sphere_beside_a_face(pose):
    R, q = POSES[pose]
    r = 0.05
    for axis in range(3):
        for sgn in (1, -1):
            for gap in (0.01, 0.03, 0.049):
                loc = np.array([0.3, -0.4, 0.2]) * HALF  # inside the face's extent
                loc[axis] = sgn * (HALF[axis] + gap)
                hit, d, n = O.sphere_box(CENTRE + R @ loc, r, CENTRE, q, HALF)
                e = np.zeros(3)
                e[axis] = sgn
                assert hit
                assert abs(d - (r - gap)) < 1e-12
                np.testing.assert_allclose(n, R @ e, atol=1e-12)
            loc[axis] = sgn * (HALF[axis] + r + 1e-6)  # just out of reach
            assert not O.sphere_box(CENTRE + R @ loc, r, CENTRE, q, HALF)[0]


@pytest.mark.parametrize("pose", range(len(POSES)))
def test_sphere_beside_edges_and_corners(pose):
    R, q = POSES[pose]
    r = 0.05
    rng = np.random.default_rng(pose)
    for _ in range(40):
        sg = rng.choice([-1.0, 1.0], 3)
        off = rng.uniform(0.005, 0.025, 3)
        free = rng.integers(0, 4)  # 0..2: an edge along that axis; 3: a corner
        loc = sg * (HALF + off)
        corner = sg * HALF
        if free < 3:
            loc[free] = rng.uniform(-0.8, 0.8) * HALF[free]
            corner[free] = loc[free]
        e = loc - corner  # closest point is the edge or corner point
        dist = np.linalg.norm(e)
        hit, d, n = O.sphere_box(CENTRE + R @ loc, r, CENTRE, q, HALF)
        assert hit == (dist < r)
        if hit:
            assert abs(d - (r - dist)) < 1e-12
            np.testing.assert_allclose(n, R @ (e / dist), atol=1e-12)


def test_sphere_closest_point_agrees_with_brute_force():
    """Outside the box, r - depth is the distance to the nearest point of the solid box,
    found here by searching a dense grid of the box (spacing 2 mm)."""
    R, q = POSES[2]
    g = [np.linspace(-h, h, int(round(2 * h / 0.002)) + 1) for h in HALF]
    pts = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
    surf = pts[(np.abs(np.abs(pts) - HALF) < 1e-12).any(1)]  # the nearest point of a solid box is on its surface
    rng = np.random.default_rng(5)
    r = 0.3
    checked = 0
    for _ in range(60):
        loc = rng.uniform(-1.0, 1.0, 3) * (HALF + 0.2)
        if (np.abs(loc) <= HALF).all():
            continue
        brute = np.sqrt(((surf - loc) ** 2).sum(1)).min()
        hit, d, n = O.sphere_box(CENTRE + R @ loc, r, CENTRE, q, HALF)
        assert hit == (brute < r - 2e-3) or abs(brute - r) < 2e-3
        if hit:
            assert abs((r - d) - brute) < 2e-3  # within the grid spacing
            if brute > 0.05:  # far enough that the grid's 1.5 mm offset turns the direction < 0.03 rad
                j = np.sqrt(((surf - loc) ** 2).sum(1)).argmin()
                want = R @ ((loc - surf[j]) / np.linalg.norm(loc - surf[j]))
                assert np.dot(n, want) > 0.999  # the normal points from the nearest surface point
            checked += 1
    assert checked > 20


@pytest.mark.parametrize("pose", range(len(POSES)))
def test_centre_inside_takes_the_shallowest_face(pose):
    R, q = POSES[pose]
    r = 0.02
    rng = np.random.default_rng(10 + pose)
    for _ in range(60):
        loc = rng.uniform(-0.97, 0.97, 3) * HALF
        togo = HALF - np.abs(loc)
        i = int(np.argmin(togo))
        e = np.zeros(3)
        e[i] = 1.0 if loc[i] >= 0 else -1.0
        hit, d, n = O.sphere_box(CENTRE + R @ loc, r, CENTRE, q, HALF)
        assert hit
        assert abs(d - (r + togo[i])) < 1e-12
        np.testing.assert_allclose(n, R @ e, atol=1e-12)
        hit, d, n = O.point_box(CENTRE + R @ loc, CENTRE, q, HALF)
        assert hit
        assert abs(d - togo[i]) < 1e-12
        np.testing.assert_allclose(n, R @ e, atol=1e-12)


def test_point_outside_or_on_the_surface_is_no_contact():
    R, q = POSES[1]
    rng = np.random.default_rng(3)
    outside = 0
    for _ in range(80):
        loc = rng.uniform(-2, 2, 3) * HALF
        if (np.abs(loc) < HALF).all():
            continue
        outside += 1
        assert not O.point_box(CENTRE + R @ loc, CENTRE, q, HALF)[0]
    assert outside > 40
    # exactly on a face (identity pose so the point is representable): strictly inside only
    assert not O.point_box(CENTRE + np.array([HALF[0], 0.0, 0.0]), CENTRE, (1, 0, 0, 0), HALF)[0]


# ------------------------------------------------------------------ pairs of bodies
def _airborne_robot_and_box(box_centre, yaw=0.0, seed=0):
    """Robot high in the air (no ground contact) with a floating box (no ground contact)."""
    rng = np.random.default_rng(seed)
    x = W.initial_state(seed, W.SCENE_FREE_BOX)
    x[0:3] = (0.0, 0.0, 5.0)
    x[19:37] = rng.normal(size=18) * np.r_[0.3, 0.3, 0.3, 1, 1, 1, np.full(12, 2.0)]
    x[37:40] = box_centre
    x[40:44] = (math.cos(yaw / 2), 0, 0, math.sin(yaw / 2))
    x[44:50] = rng.normal(size=6) * 0.4
    return x


@pytest.mark.parametrize("seed", range(4))
def test_robot_box_forces_are_equal_and_opposite(seed):
    m = O.Oracle(W.model_dict(W.BOX_PUSH, 0))
    th = 0.5 * np.array(W.ROBOT["trunk_size"])
    bh = np.array(W.FREE_BOX_HALF)
    # the trunk's (+x, +y, +z) corner 1-3 cm inside the box's (-x, -y, -z) corner: a trunk
    # corner in the box and a box corner in the trunk
    centre = np.array([th[0], th[1], 5.0 + th[2]]) + bh - np.array([0.01, 0.02, 0.03])
    x = _airborne_robot_and_box(centre, seed=seed)
    Fr, Fb, n = m.contact_total(x)
    assert n == 2
    assert np.linalg.norm(Fr) > 1.0
    np.testing.assert_allclose(Fr, -Fb, atol=1e-12 * np.linalg.norm(Fr))
    # a foot sphere inside the box's lower face
    feet = m.feet(x[:19]).reshape(4, 3)
    centre = feet[0] + np.array([0.0, 0.0, bh[2] + 0.01])
    x = _airborne_robot_and_box(centre, seed=seed)
    Fr, Fb, n = m.contact_total(x)
    assert n >= 1 and np.linalg.norm(Fr) > 1.0
    np.testing.assert_allclose(Fr, -Fb, atol=1e-12 * np.linalg.norm(Fr))


def test_box_corner_in_the_trunk_pushes_along_the_trunk_face():
    """A box balanced on one corner that dips 4 mm into the tilted trunk's top face: the
    only contact; at rest the box is pushed out along the trunk's top-face normal with
    the spring force k delta, the trunk the other way."""
    m = O.Oracle(W.model_dict(W.BOX_PUSH, 0))
    th = 0.5 * np.array(W.ROBOT["trunk_size"])
    bh = np.array(W.FREE_BOX_HALF)
    x = _airborne_robot_and_box(np.zeros(3))
    x[19:37] = 0.0
    Rt, qt = _rot((0.3, 0.2, 1.0), 0.4)
    x[3:7] = qt
    top = Rt @ np.array([0, 0, 1.0])
    depth = 0.004
    corner = x[0:3] + Rt @ np.array([0.0, 0.0, th[2] - depth])
    d = -np.ones(3) / math.sqrt(3)  # the box's (-,-,-) corner direction, turned to point along -top
    ax = np.cross(d, -top)
    Rb, qb = _rot(ax, math.acos(np.clip(d @ -top, -1, 1)))
    np.testing.assert_allclose(Rb @ d, -top, atol=1e-12)
    x[37:40] = corner + Rb @ bh
    x[40:44] = qb
    x[44:50] = 0.0
    Fr, Fb, n = m.contact_total(x)
    assert n == 1
    np.testing.assert_allclose(Fb, W.ROBOT["k"] * depth * top, atol=1e-9)
    np.testing.assert_allclose(Fr, -Fb, atol=1e-12)


# ------------------------------------------------------------------ the normal law
def test_separating_contact_pulls_and_has_no_friction():
    """A level box lifting off at 0.5 m/s with a small overlap: k delta - c v_n < 0, so
    every corner pulls (no clamp), and the Coulomb term scales with max(F_n, 0) = 0."""
    m = O.Oracle(W.model_dict(W.BOX_PUSH, 0))
    k, c = W.ROBOT["k"], W.ROBOT["c"]
    hit, F, D = m.contact_law(1e-3, (0, 0, 1.0), (0.3, -0.2, 0.5))
    assert hit
    np.testing.assert_allclose(F, [0, 0, k * 1e-3 - c * 0.5], atol=1e-12)  # pulls, no tangential part
    np.testing.assert_allclose(D, c * np.diag([0, 0, 1.0]), atol=1e-12)
    hz, mb, G = W.FREE_BOX_HALF[2], W.FREE_BOX_MASS, W.ROBOT["gravity"]
    z, v, dt = hz - 2e-4, 0.5, 0.01
    x = W.initial_state(0, W.SCENE_FREE_BOX, jitter=0.0)
    x[0], x[2] = -20.0, 50.0
    x[37:40] = (1.0, 0.0, z)
    x[44:50] = 0.0
    x[46] = v
    x[44] = 0.2  # sliding too: no friction while pulling
    Fr, Fb, n = m.contact_total(x)
    assert n == 4
    np.testing.assert_allclose(Fb, [0, 0, 4 * (k * (hz - z) - c * v)], atol=1e-9)
    assert Fb[2] < 0
    xn, _, rc = m.step(x, np.zeros(12), 0.0, 0.0, dt)
    vn = v + dt * (4 * k * (hz - z) - 4 * c * v - mb * G) / (mb + 4 * c * dt)
    assert rc == 0
    assert abs(xn[46] - vn) < 1e-12 and abs(xn[39] - (z + dt * vn)) < 1e-13
    assert abs(xn[44] - 0.2) < 1e-12  # no tangential force, no tangential damping


# ------------------------------------------------------------------ heightfield
def _bilinear_model(a):
    d = W.model_dict(W.TERRAIN_WALK, 0)
    n = d["hf"].shape[0]
    xs = d["hf_x0"] + d["hf_cell"] * np.arange(n)
    ys = d["hf_y0"] + d["hf_cell"] * np.arange(n)
    d["hf"] = a * np.outer(ys, xs)  # hf[iy, ix] = a x y
    return O.Oracle(d), d


def test_bilinear_heightfield_is_exact_for_h_equals_axy():
    a = 0.4
    m, d = _bilinear_model(a)
    rng = np.random.default_rng(2)
    span = 0.5 * (d["hf"].shape[0] - 1) * d["hf_cell"]
    r = 0.02
    for _ in range(50):
        px, py = rng.uniform(-0.9, 0.9, 2) * span
        h = a * px * py
        z = h + rng.uniform(-0.015, 0.015)
        hit, delta, n = m.terrain((px, py, z), r)
        g = np.array([a * py, a * px])
        want_n = np.r_[-g, 1.0] / math.sqrt(1 + g @ g)
        np.testing.assert_allclose(n, want_n, atol=1e-12)
        assert abs(delta - (h + r - z) * want_n[2]) < 1e-12
        assert hit == (h + r - z > 0)


def test_heightfield_clamps_outside_the_grid():
    a = 0.4
    m, d = _bilinear_model(a)
    n = d["hf"].shape[0]
    xmax = d["hf_x0"] + (n - 1) * d["hf_cell"]
    py = 0.3
    hit, delta, nrm = m.terrain((xmax + 0.5, py, 0.0), 0.0)
    h = a * xmax * py  # the edge value, and no slope along x out there
    want_n = np.array([0.0, -a * xmax, 1.0]) / math.sqrt(1 + (a * xmax) ** 2)
    np.testing.assert_allclose(nrm, want_n, atol=1e-12)
    assert abs(delta - h * want_n[2]) < 1e-12


def test_step_systems_reproduce_the_step():
    """The exported robot and box systems of a step are the ones the step solves: their
    solutions are the step's velocity changes (the FP32 error bound is derived from them)."""
    m = O.Oracle(W.model_dict(W.BOX_PUSH, 0))
    from tests.parity_utils import box_contact_states
    u = np.tile(W.STANCE_JOINTS, 4)
    for x in box_contact_states(5, seed=4):
        xn, _, rc = m.step(x, u, 40.0, 1.0, 0.01)
        A, r, n = m.step_system(x, u, 40.0, 1.0, 0.01)
        np.testing.assert_allclose(x[19:37] + np.linalg.solve(A, r), xn[19:37], rtol=0, atol=1e-12)
        Ab, rb, nb = m.step_system_box(x, u, 40.0, 1.0, 0.01)
        np.testing.assert_allclose(x[44:50] + np.linalg.solve(Ab, rb), xn[44:50], rtol=0, atol=1e-12)
