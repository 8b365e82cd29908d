"""The comparison helper on the CPU: results that differ from the oracle's only
by another reading of an ambiguous sample pass as resolved; a wrong loss or
gradient fails; the readings the oracle takes change nothing else."""
import numpy as np
import pytest

import oracle as O
from paper_2306_08132_amd import synth as S
from tests import parity_check as P


@pytest.fixture(scope="module")
def tiny():
    hand, grid, q = S.config_workload("tiny")
    return O.Hand(hand.rounded()), O.Obj(grid), q.astype(np.float32).astype(np.float64)


def test_step_ex_without_flips_is_the_step(tiny):
    H, ob, q = tiny
    for K in (1, 3):
        op = O.Params(r_dil=0.005, K=K)
        a = O.step(H, ob, op, q[:16])
        b = O.step_ex(H, ob, op, q[:16], kink_d=P.KINK_D, kink_face=P.KINK_FACE, max_amb=8)
        assert np.array_equal(a["loss"], b["loss"]) and np.array_equal(a["grad"], b["grad"])


def test_other_readings_are_resolved_and_mistakes_fail(tiny):
    H, ob, q = tiny
    op = O.Params(r_dil=0.005)
    ref = O.step_ex(H, ob, op, q, kink_d=P.KINK_D, kink_face=P.KINK_FACE, max_amb=64)
    amb = [b for b in range(q.shape[0]) if P.units_of(ref["amb"][b])]
    assert len(amb) >= 3
    # a "GPU" result that took the other reading of each such candidate's most ambiguous unit
    flips = []
    for b in amb:
        flips += [(b, *f) for f in P.units_of(ref["amb"][b])[0][1]]
    alt = O.step_ex(H, ob, op, q, flips=flips)
    moved = [b for b in amb if np.abs(alt["grad"][b] - ref["grad"][b]).max() > 1e-3 * np.abs(ref["grad"][b]).max()]
    rep = P.compare(alt["loss"].astype(np.float32), alt["grad"].astype(np.float32), H, ob, op, q, label="planted",
                    say=lambda *a: None)
    P.assert_ok(rep)
    assert rep["resolved"] >= len(moved) and rep["failed"] == 0
    # a wrong gradient on one candidate is not resolved
    g = alt["grad"].copy()
    g[5] *= 1.01
    rep = P.compare(alt["loss"], g, H, ob, op, q, say=lambda *a: None)
    assert rep["status"][5] == 3
    with pytest.raises(AssertionError):
        P.assert_ok(rep)
    # nor a wrong loss
    lo = alt["loss"].copy()
    lo[7] += 1e-3 * max(abs(lo[7]), 1.0)
    rep = P.compare(lo, None, H, ob, op, q, say=lambda *a: None)
    assert rep["status"][7] == 3


def test_shared_coordinates_flip_together():
    amb = [(2, 0, 9, 1, 1e-5, 0), (3, 0, 9, 1, 1e-5, 0), (0, 0, 9, 1, 3e-5, 0), (4, 2, 9, 1, 2e-5, 1),
           (5, 0, 11, 0, 1e-8, 1)]
    units = P.units_of(amb)
    # the d-branch unit (smallest margin), the x-face shared by tests 2..6 at k = 0,
    # test 4's face at k = 2, and test 0's own x coordinate
    assert [len(u[1]) for u in units] == [1, 5, 1, 1]
    assert units[1][1] == [(m, 0, 9, 1) for m in (2, 3, 4, 5, 6)]


def test_conditioning_sets_aside_only_what_it_explains(tiny):
    """With several iterations and conditioning measured, a wrong loss or
    gradient fails however many ambiguous decisions the candidate holds: a
    candidate is set aside only when the movement of the FP64 result under
    FP32-resolution changes of q covers its error."""
    H, ob, q = tiny
    op = O.Params(r_dil=0.005, K=3)
    ref = O.step(H, ob, op, q[:12])
    lo, g = ref["loss"].copy(), ref["grad"].copy()
    lo[3] *= 1.0 + 1e-2
    g[4] *= 1.05
    rep = P.compare(lo, g, H, ob, op, q[:12], conditioning=True, max_units=1, say=lambda *a: None)
    assert rep["status"][3] == 3 and rep["status"][4] == 3
    assert rep["lcond"][3] < 1e-3 and rep["gcond"][4] < 1e-2
    assert np.all(rep["status"][[b for b in range(12) if b not in (3, 4)]] == 0)


def test_grid_boundary_face_reading(oracle_lib):
    """A sample on the grid box's own face (u = 0 along y) with z beyond the
    box is read inside (the trilinear y-slope plus the direction to the clamped
    point) or, as the other reading of that face, clamped along y (no y part).
    An affine grid phi = 0.5 x + 0.25 y - 0.125 z + 1/16 has slope (0.5, 0.25,
    -0.125), so the +x test's normal is g = (0.5, 0.25, 1) or g' = (0.5, 0, 1);
    nothing penetrates and w_pen = 0, so the x-gradient of the loss changes by
    the leak term of that sample alone,
      w_s / (7 dt) alpha (e . g') g'_x / w' - (same with g),
    w = |g|^2 + |r x g|^2 / (I/m). The oracle reports the face and the other
    reading reproduces this number."""
    from tests.helpers import dyadic_plane_grid, point_hand
    grid = dyadic_plane_grid()
    Im = 0.25
    ob = O.Obj(grid, inertia_over_mass=Im)
    p = np.array([0.3, -1.0, 1.5])  # y on the box's face, z half a unit above the box
    H = O.Hand(point_hand([p]))
    op = O.Params(r_dil=0.0, w_pen=0.0, alpha_leak=0.3)
    q = np.zeros((1, 6))
    dv = op.dt * op.v0
    ref = O.step_ex(H, ob, op, q, kink_d=P.KINK_D, kink_face=P.KINK_FACE, max_amb=64)
    assert (0, 0, 0, 2) in [tuple(int(x) for x in a[:4]) for a in ref["amb"][0]]
    alt = O.step_ex(H, ob, op, q, flips=[(0, 0, 0, 0, 2)])
    r = p - dv * np.array([1.0, 0.0, 0.0])
    phi, g, _ = O.sample(ob, r[None])
    assert np.allclose(g[0], [0.5, 0.25, 1.0], rtol=0, atol=1e-12)

    def term(gv):
        u = np.cross(r, gv)
        w = gv @ gv + (u @ u) / Im
        return gv[0] * op.alpha_leak * gv[0] / w

    want = op.w_stable / (7 * op.dt) * (term(np.array([0.5, 0.0, 1.0])) - term(np.array([0.5, 0.25, 1.0])))
    got = alt["grad"][0, 0] - ref["grad"][0, 0]
    assert abs(want) > 1e-3
    assert got == pytest.approx(want, rel=1e-9)
    assert np.array_equal(alt["loss"], ref["loss"])


def quadratic_dyadic_grid(n=33, lo=-1.0, h=1.0 / 16):
    """Vertex values 0.5 x^2 + 0.25 y - 0.125 z + 1/16, exact in FP32: the
    trilinear x-slope jumps across every x cell face."""
    from paper_2306_08132_amd.synth import Grid
    g = Grid(n=n, lo=np.full(3, lo), h=h, values=np.empty(0, np.float32), prims=[], bound_radius=0.0)
    X = g.vertex_positions()
    vals = 0.5 * X[:, 0] ** 2 + 0.25 * X[:, 1] - 0.125 * X[:, 2] + 0.0625
    assert np.array_equal(vals.astype(np.float32).astype(np.float64), vals)
    g.values = vals.astype(np.float32)
    return g


def two_sided(ob, p, op, what, nudges):
    """The oracle reports a sample of kind `what` at p; the default and the
    other reading of the reported samples are the step at p + nudges[0] and
    p + nudges[1], in some order."""
    from tests.helpers import point_hand
    H = O.Hand(point_hand([p]))
    q = np.zeros((1, 6))
    ref = O.step_ex(H, ob, op, q, kink_d=P.KINK_D, kink_face=P.KINK_FACE, max_amb=64)
    amb = [tuple(int(x) for x in a[:4]) for a in ref["amb"][0] if int(a[3]) == what]
    assert amb
    alt = O.step_ex(H, ob, op, q, flips=[(0, *f) for f in amb])
    lo = O.step(O.Hand(point_hand([p + nudges[0]])), ob, op, q)
    hi = O.step(O.Hand(point_hand([p + nudges[1]])), ob, op, q)

    def close(a, b):
        g = max(np.abs(a["grad"]).max(), np.abs(b["grad"]).max())
        return (abs(a["loss"][0] - b["loss"][0]) <= 1e-6 * abs(b["loss"][0])
                and np.abs(a["grad"] - b["grad"]).max() <= 1e-5 * g)

    assert not close(lo, hi)
    assert (close(ref, lo) and close(alt, hi)) or (close(ref, hi) and close(alt, lo))
    return amb


def test_cell_face_reading_is_the_other_side(oracle_lib):
    """A point on an interior x cell face of a grid whose x-slope jumps
    there, inside the dilated surface: reading the other cell is the step
    1e-10 m to the other side (the rest test and the y and z tests share the
    face)."""
    ob = O.Obj(quadratic_dyadic_grid(), inertia_over_mass=0.25)
    p = np.array([0.25, 0.125, -0.5])  # u_x = 20: the face between cells 19 and 20
    phi = 0.5 * p[0] ** 2 + 0.25 * p[1] - 0.125 * p[2] + 0.0625
    amb = two_sided(ob, p, O.Params(r_dil=phi + 0.01), 1,
                    (np.array([-1e-10, 0.0, 0.0]), np.array([1e-10, 0.0, 0.0])))
    assert {a[0] for a in amb} == {2, 3, 4, 5, 6}


def test_activation_reading_is_the_other_side(oracle_lib):
    """A sample at the activation d = -eps exactly (eps the contact tolerance)
    on an affine grid: reading it active or not is the step with the point
    moved 1e-10 m along the gradient to either side."""
    from tests.helpers import dyadic_plane_grid
    ob = O.Obj(dyadic_plane_grid(), inertia_over_mass=0.25)
    p = np.array([0.25, 0.125, -0.5])
    phi = 0.5 * p[0] + 0.25 * p[1] - 0.125 * p[2] + 0.0625
    op = O.Params()
    eps = 5e-3 * op.dt * op.v0
    op.r_dil = phi + eps  # the rest test's d = phi - r_dil = -eps
    g = np.array([0.5, 0.25, -0.125])
    two_sided(ob, p, op, 0, (-1e-10 * g / np.linalg.norm(g), 1e-10 * g / np.linalg.norm(g)))
