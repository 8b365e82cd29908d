"""Closed-form pins of two oracle parts that GPU parity cannot check (both
sides follow the same reading):

* the penetration loss L_pen = 1/2 sum_i C_i^2 with C_i = max(0, -(phi(p_i) -
  r_dil)) at the object's rest pose (Sec. III-C constraint, Sec. III-B
  dilation; the loss term is the build's reading), value and gradient, on a
  tilted plane where every velocity test's displacement would change the
  depths;
* the Phong point of Sec. III-B (read as Phong tessellation's blend
  p = (1 - alpha) r* + alpha sum_b w_b psi_b(r*)) on an octahedron with radial
  vertex normals, where it has the closed form p_i = w_i + alpha w_i (1 - w_i),
  and its convergence to the sphere under refinement.

No GPU needed."""
import numpy as np
import pytest

import oracle as O
from paper_2306_08132_amd import synth as S
from tests.helpers import point_hand


# ---------------------------------------------------------------------------
# L_pen
# ---------------------------------------------------------------------------
def _tilted_plane():
    n = np.array([1.0, 0.5, 2.0])
    n /= np.linalg.norm(n)
    return n, 0.003  # phi(r) = n . r - 0.003


def _pen_hand(n, c, depths):
    """Contacts at the given depths below the plane n . r = c (negative depth:
    above it), spread along the plane so the lever arms differ."""
    rng = np.random.default_rng(3)
    t1 = np.cross(n, [0.0, 0.0, 1.0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    pts = []
    for d in depths:
        a, b = rng.uniform(-0.03, 0.03, size=2)
        pts.append((c - d) * n + a * t1 + b * t2)
    return np.array(pts)


@pytest.mark.parametrize("r_dil", [0.0, 0.0025])
def test_lpen_closed_form_on_a_plane(oracle_lib, r_dil):
    """terms[1] = 1/2 sum (delta_i + r)^2 over the contacts with delta_i + r > 0,
    exactly; with only w_pen set, the loss gradient is sum_i d_i n . dp_i/dq:
    -sum (delta_i + r) n along the wrist translations and sum d_i n . (e x p_i)
    about the wrist's z, y and x axes at q = 0. A dropped 1/2 doubles the value;
    sampling at a test's displaced pose instead of the rest pose moves every
    depth by up to dt v0 |n_j| (0.44 mm here)."""
    n, c = _tilted_plane()
    depths = np.array([0.004, 0.0012, 0.0002, -0.0005, -0.004, 0.007])
    pts = _pen_hand(n, c, depths)
    hand = O.Hand(point_hand(pts))
    ob = O.Obj(kind=O.OBJ_PLANE, normal=n, offset=c, inertia_over_mass=2e-4)
    P = O.Params(r_dil=r_dil, w_stable=0.0, w_pen=1.0, w_range=0.0, w_limit=0.0)
    q = np.zeros(6)
    out = O.step(hand, ob, P, q[None])
    pen = np.maximum(depths + r_dil, 0.0)
    want = 0.5 * np.sum(pen * pen)
    assert out["terms"][0, 1] == pytest.approx(want, rel=1e-13, abs=1e-20)
    assert out["loss"][0] == pytest.approx(want, rel=1e-13, abs=1e-20)
    d = -pen  # d_i where the contact penetrates
    g = out["grad"][0]
    np.testing.assert_allclose(g[:3], np.sum(d) * n, rtol=1e-11, atol=1e-16)
    for j, axis in zip((3, 4, 5), np.eye(3)[[2, 1, 0]]):
        want_j = np.sum(d * (np.cross(axis, pts) @ n))
        assert g[j] == pytest.approx(want_j, rel=1e-10, abs=1e-16), j
    # the displaced poses of the six moving tests would change the value
    dv = P.dt * P.v0
    for m_dir in np.concatenate([np.eye(3), -np.eye(3)]):
        moved = np.maximum(depths + r_dil + dv * (m_dir @ n), 0.0)
        assert abs(0.5 * np.sum(moved * moved) - want) > 1e-3 * want


def test_lpen_ignores_contacts_outside_the_dilated_surface(oracle_lib):
    """Contacts above the plane by more than r_dil add nothing to L_pen, and
    L_pen grows from zero as r_dil passes their height."""
    n, c = _tilted_plane()
    pts = _pen_hand(n, c, [-0.002, -0.003])
    hand = O.Hand(point_hand(pts))
    ob = O.Obj(kind=O.OBJ_PLANE, normal=n, offset=c, inertia_over_mass=2e-4)
    vals = []
    for r in (0.0, 0.0019, 0.0025, 0.004):
        P = O.Params(r_dil=r, w_stable=0.0, w_pen=1.0, w_range=0.0, w_limit=0.0)
        vals.append(O.step(hand, ob, P, np.zeros((1, 6)))["terms"][0, 1])
    assert vals[0] == 0.0 and vals[1] == 0.0
    assert vals[2] == pytest.approx(0.5 * 0.0005 ** 2, rel=1e-12)
    assert vals[3] == pytest.approx(0.5 * (0.002 ** 2 + 0.001 ** 2), rel=1e-12)


# ---------------------------------------------------------------------------
# Phong point
# ---------------------------------------------------------------------------
def octahedron():
    """Vertices +-e_x, +-e_y, +-e_z with radial unit normals; faces
    counter-clockwise seen from outside."""
    V = np.concatenate([np.eye(3), -np.eye(3)])
    faces = []
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                a = 0 if sx > 0 else 3
                b = 1 if sy > 0 else 4
                c = 2 if sz > 0 else 5
                faces.append((a, b, c) if sx * sy * sz > 0 else (a, c, b))
    return S.TriMesh(V, np.array(faces, np.int32), V.copy())


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("w", [(0.5, 0.3, 0.2), (0.15, 0.6, 0.25)])
def test_phong_point_closed_form_on_an_octahedron(alpha, w):
    """On the face (e_x, e_y, e_z) a flat closest point r* has coordinates equal
    to its barycentric weights w; vertex b's tangent plane is x . e_b = 1, so
    psi_b(r*) = r* + (1 - w_b) e_b and the Phong point is
    p_i = w_i + alpha w_i (1 - w_i). Points off the face along its normal (outside
    and inside) have rho = +-|r - p|. Swapping alpha and 1 - alpha, or giving a
    vertex's weight to another vertex's plane, breaks the equality."""
    m = octahedron()
    M = O.Mesh(m.vertices, m.faces, m.normals, alpha)
    w = np.asarray(w)
    rstar = w.copy()
    p = w + alpha * w * (1.0 - w)
    nf = np.ones(3) / np.sqrt(3.0)
    for s in (0.2, 0.02, -0.05):
        r = rstar + s * nf
        out = O.mesh_sdf(M, r[None])
        np.testing.assert_allclose(out["closest"][0], rstar, atol=1e-15)
        want = np.sign(s) * np.linalg.norm(r - p)
        assert out["rho"][0] == pytest.approx(want, rel=1e-12, abs=1e-15), (s, out["rho"][0], want)
        np.testing.assert_allclose(out["grad"][0], (r - p) / want, rtol=1e-10, atol=1e-14)
    # the slips this pins: alpha swapped, weights on the wrong vertices
    alt = [w + (1.0 - alpha) * w * (1.0 - w), w + alpha * np.roll(w, 1) * (1.0 - w)]
    r = rstar + 0.2 * nf
    got = O.mesh_sdf(M, r[None])["rho"][0]
    for pa in alt:
        if not np.allclose(pa, p):
            assert abs(np.linalg.norm(r - pa) - got) > 1e-4


@pytest.mark.parametrize("alpha", [0.0, 0.5, 0.75, 1.0])
def test_phong_surface_converges_to_the_sphere(alpha):
    """Icospheres of 2..5 subdivisions with their exact radial normals: the
    largest error of rho against the unit sphere's distance |r| - 1, over points
    within 5% of the surface, falls at least at second order in the edge length
    (each subdivision halves the edges)."""
    rng = np.random.default_rng(7)
    d = rng.normal(size=(1000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = d * rng.uniform(0.95, 1.05, size=(1000, 1))
    exact = np.linalg.norm(r, axis=1) - 1.0
    errs = []
    for lev in range(2, 6):
        m = S.icosphere(lev)
        out = O.mesh_sdf(O.Mesh(m.vertices, m.faces, m.normals, alpha), r)
        errs.append(np.abs(out["rho"] - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders >= 1.8), (alpha, errs, orders)
    assert errs[-1] < 2e-3


@pytest.mark.parametrize("f", [0.5, 2.0, 40.0])
def test_contact_tolerance_on_a_plane(oracle_lib, f):
    """The activation threshold d < -eps, eps = 5e-3 dt v0 (contact
    tolerance), on one contact and the plane x = offset seen by the +x test
    (rotation frozen by a huge inertia): the test moves the object by dt v0
    along +x, so the contact ends at d = -f eps. Below the tolerance (f = 0.5)
    nothing happens; beyond it the correction removes all of it (x1 = x0 -
    f eps along x, d = 0). A second iteration starts from a resolved contact
    (d = 0 up to rounding), which is not active: the pose stays, and the
    derivative of the final pose along the hand's x is that of the first
    iteration, exactly 1 (the constraint moves the object with the hand)."""
    dv = 1e-3
    eps = 5e-3 * dv
    off = -dv + f * eps
    ob = O.Obj(kind=O.OBJ_PLANE, normal=np.array([1.0, 0.0, 0.0]), offset=off, inertia_over_mass=1e6)
    hand = O.Hand(point_hand([[0.0, 0.0, 0.0]]))
    for K in (1, 2):
        P = O.Params(K=K, r_dil=0.0, alpha_leak=0.0, dt=dv, v0=1.0)
        tr = O.trace(hand, ob, P, np.zeros(6))
        x = tr["poses"][0, :, 0]  # +x test: x before each iteration and after the last
        lam = tr["samples"][0, :, 0, 5]
        assert x[0] == pytest.approx(dv, abs=1e-18)
        if f < 1.0:
            assert np.all(lam == 0.0) and np.all(x == x[0])
        else:
            assert x[1] == pytest.approx(dv - f * eps, abs=1e-15 * dv)
            assert lam[0] != 0.0 and np.all(lam[1:] == 0.0)
            assert np.all(x[1:] == x[1])
    # the loss gradient along the wrist's x: with the contact active the +x
    # test's final |x| = dv - f eps + (q_x) moves with q_x (derivative 1 over M dt
    # in L_stable); below the tolerance it does not depend on q_x
    P = O.Params(K=2, r_dil=0.0, alpha_leak=0.0, dt=dv, v0=1.0, w_pen=0.0, w_range=0.0, w_limit=0.0)
    g = O.step(hand, ob, P, np.zeros((1, 6)))["grad"][0]
    expect = (1.0 / (7 * dv)) if f > 1.0 else 0.0
    assert g[0] == pytest.approx(expect, rel=1e-9, abs=1e-9)
