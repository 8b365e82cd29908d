"""Pins of the oracle's grid SDF sampler (trilinear grid of Sec. III-A, with
the analytic gradient and the out-of-box extension) against closed forms, and
of its seven-query central-difference normal (the finite differencing that
Sec. III-A contrasts with, an oracle option for comparison)."""
import numpy as np
import pytest

from paper_2306_08132_amd import synth as S
from tests.helpers import dyadic_plane_grid


def test_exact_at_vertices(oracle_lib):
    O = oracle_lib
    g = S.make_grid(S.make_object("ellipsoids", seed=3), 24)
    ob = O.Obj(g)
    P = g.vertex_positions()
    idx = np.random.default_rng(0).choice(P.shape[0], 2000, replace=False)
    phi, _, _ = O.sample(ob, P[idx])
    np.testing.assert_allclose(phi, g.values[idx].astype(np.float64), atol=1e-15, rtol=0)
    # the last vertex along each axis (u = N-1 lies in cell N-2 with f = 1)
    last = (g.n - 1) * (1 + g.n + g.n * g.n)
    phi, _, _ = O.sample(ob, P[[last, 0]])
    np.testing.assert_allclose(phi, g.values[[last, 0]], atol=1e-15, rtol=0)


def test_affine_field_reproduced_exactly(oracle_lib):
    """Trilinear interpolation reproduces an affine field: value and gradient."""
    O = oracle_lib
    coef, off = np.array([0.5, 0.25, -0.125]), 0.0625
    g = dyadic_plane_grid(coef=coef, off=off)
    ob = O.Obj(g)
    rng = np.random.default_rng(1)
    r = g.lo + rng.random((5000, 3)) * g.h * (g.n - 1)
    phi, grad, _ = O.sample(ob, r)
    np.testing.assert_allclose(phi, r @ coef + off, atol=1e-14, rtol=0)
    np.testing.assert_allclose(grad, np.broadcast_to(coef, grad.shape), atol=1e-13, rtol=0)


def test_sphere_within_trilinear_error_bound(oracle_lib):
    """|phi - (|r| - R)| <= h^2/8 * sum_j max |d2 phi / dx_j^2| (+ FP32 storage)."""
    O = oracle_lib
    R = 0.04
    g = S.make_grid(S.make_object("sphere", seed=0, radius=R), 64)
    ob = O.Obj(g)
    rng = np.random.default_rng(2)
    d = rng.normal(size=(20000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = rng.uniform(0.5 * R, 1.4 * R, size=(20000, 1))
    r = d * rad
    phi, grad, _ = O.sample(ob, r)
    exact = np.linalg.norm(r, axis=1) - R
    # d2/dx_j2 of |r| is (1 - x_j^2/|r|^2)/|r| <= 1/|r|; take the cell's nearest radius
    rmin = np.linalg.norm(r, axis=1) - np.sqrt(3) * g.h
    bound = g.h ** 2 / 8 * 3.0 / rmin + 1e-8
    assert np.all(np.abs(phi - exact) <= bound)
    # gradient: unit normal up to O(h) interpolation error
    nrm = r / np.linalg.norm(r, axis=1, keepdims=True)
    assert np.max(np.linalg.norm(grad - nrm, axis=1)) < 3 * g.h / rmin.min()


def test_box_exact_in_affine_regions(oracle_lib):
    """An axis-aligned box SDF is affine wherever one face is nearest; cells
    whose 8 corners share that face reproduce it exactly."""
    O = oracle_lib
    from paper_2306_08132_amd.synth import Grid
    half = np.array([0.25, 0.375, 0.5])
    g = Grid(n=33, lo=np.full(3, -1.0), h=1.0 / 16, values=np.empty(0, np.float32), prims=[],
             bound_radius=0)
    P = g.vertex_positions()
    vals = S.box_sdf(P, np.zeros(3), np.eye(3), half)
    g.values = vals.astype(np.float32)
    ob = O.Obj(g)
    rng = np.random.default_rng(3)
    r = g.lo + rng.random((20000, 3)) * 2.0

    def region(x):  # which face is nearest / active, as an integer label
        q = np.abs(x) - half
        inside = np.all(q <= 0, axis=-1)
        lab_in = np.argmax(q, axis=-1) * 2 + (np.take_along_axis(x, np.argmax(q, -1)[:, None], 1)[:, 0] > 0)
        outmask = (q > 0)
        lab_out = 10 + (outmask * np.array([1, 2, 4])).sum(-1) * 8 + ((x > 0) * np.array([1, 2, 4])).sum(-1)
        return np.where(inside, lab_in, lab_out), outmask.sum(-1)

    u = (r - g.lo) / g.h
    c = np.minimum(np.floor(u), g.n - 2)
    labs = []
    for corner in np.array(np.meshgrid([0, 1], [0, 1], [0, 1], indexing="ij")).reshape(3, -1).T:
        labs.append(region(g.lo + (c + corner) * g.h)[0])
    labs = np.stack(labs, 1)
    lab_r, nout = region(r)
    same = np.all(labs == lab_r[:, None], axis=1) & (nout <= 1)
    assert same.sum() > 1000
    phi, grad, _ = O.sample(ob, r[same])
    exact = S.box_sdf(r[same], np.zeros(3), np.eye(3), half)
    np.testing.assert_allclose(phi, exact, atol=1e-14, rtol=0)


def test_outside_box_continuous_and_not_below_true_distance(oracle_lib):
    O = oracle_lib
    R = 0.04
    g = S.make_grid(S.make_object("sphere", seed=0, radius=R), 32)
    ob = O.Obj(g)
    rng = np.random.default_rng(4)
    side = g.h * (g.n - 1)
    # continuity across each face of the box
    for ax in range(3):
        for sgn in (0.0, 1.0):
            r = g.lo + rng.random((500, 3)) * side
            r[:, ax] = g.lo[ax] + sgn * side
            eps = 1e-9
            r_in, r_out = r.copy(), r.copy()
            r_in[:, ax] += (-eps if sgn else eps)
            r_out[:, ax] += (eps if sgn else -eps)
            a, _, _ = O.sample(ob, r_in)
            b, _, _ = O.sample(ob, r_out)
            assert np.max(np.abs(a - b)) < 1e-7
    # far outside: phi >= |r| - R up to the trilinear error at the box boundary
    r = rng.normal(size=(4000, 3))
    r = r / np.linalg.norm(r, axis=1, keepdims=True) * rng.uniform(0.07, 0.3, size=(4000, 1))
    phi, grad, _ = O.sample(ob, r)
    inb = np.all(np.abs(r) <= side / 2, axis=1)
    out = ~inb
    assert out.sum() > 1000
    assert np.all(phi[out] >= np.linalg.norm(r[out], axis=1) - R - g.h ** 2 / 8 * 3 / 0.04)


def test_hessian_is_derivative_of_gradient(oracle_lib):
    """The Hessian (dual numbers) agrees with central differences of the
    gradient away from cell faces, and its diagonal is zero inside the box."""
    O = oracle_lib
    g = S.make_grid(S.make_object("ellipsoids", seed=5), 20)
    ob = O.Obj(g)
    rng = np.random.default_rng(6)
    r = g.lo + (rng.random((3000, 3)) * 1.2 - 0.1) * g.h * (g.n - 1)
    phi, grad, H, margin = O.sample(ob, r, hess=True)
    keep = margin > 1e-3
    eps = 1e-7
    for a in range(3):
        rp, rm = r.copy(), r.copy()
        rp[:, a] += eps
        rm[:, a] -= eps
        _, gp, _ = O.sample(ob, rp)
        _, gm, _ = O.sample(ob, rm)
        fd = (gp - gm) / (2 * eps)
        np.testing.assert_allclose(H[keep, :, a], fd[keep], atol=1e-4 * np.abs(H).max())
    inside = np.all((r > g.lo) & (r < g.lo + g.h * (g.n - 1)), axis=1)
    assert np.all(np.abs(np.einsum("nii->ni", H[inside])) == 0.0)
    np.testing.assert_allclose(H, np.swapaxes(H, 1, 2), atol=1e-12 * np.abs(H).max())


def test_inertia_from_vertex_count(oracle_lib):
    """I/m = 2/5 R_eq^2 with V = h^3 #(phi < 0): a sphere recovers its radius."""
    O = oracle_lib
    R = 0.04
    g = S.make_grid(S.make_object("sphere", seed=0, radius=R), 96)
    Im = O.Obj(g).inertia_over_mass()
    assert abs(Im / (0.4 * R * R) - 1.0) < 0.01
    # exact count: k negative vertices
    g2 = S.make_grid(S.make_object("sphere", seed=0, radius=R), 16)
    vals = np.ones_like(g2.values)
    vals[:37] = -1.0
    g2.values = vals
    Req = (3 * 37 * g2.h ** 3 / (4 * np.pi)) ** (1 / 3)
    assert O.Obj(g2).inertia_over_mass() == pytest.approx(0.4 * Req ** 2, rel=1e-14)


def _quadratic_grid(n=33, lo=-0.5, h=1.0 / 32):
    """Grid of |r|^2 - 1/16 on dyadic vertices, whose values FP32 holds exactly."""
    from paper_2306_08132_amd.synth import Grid
    g = Grid(n=n, lo=np.full(3, lo), h=h, values=np.empty(0, np.float32), prims=[], bound_radius=0.0)
    P = g.vertex_positions()
    vals = (P * P).sum(axis=1) - 1.0 / 16
    assert np.array_equal(vals.astype(np.float32).astype(np.float64), vals)
    g.values = vals.astype(np.float32)
    return g


def test_central_difference_normal_closed_forms(oracle_lib):
    """The seven-query normal (Sec. III-A's finite differencing, an oracle
    option for comparison) against closed forms. On an affine field it equals
    the field's gradient, like the analytic one. On |r|^2 the trilinear blend
    is piecewise linear along each axis with knots at the vertices, and its
    central difference over +-h is exactly 2r at every point whose offsets
    stay in the box, while the analytic gradient of the blend is constant
    within a cell (the sum of the cell's two vertex coordinates); the value
    is the same blend either way."""
    O = oracle_lib
    rng = np.random.default_rng(7)
    coef = np.array([0.5, 0.25, -0.125])
    ga = dyadic_plane_grid(coef=coef, off=0.0625)
    ra = ga.lo + ga.h + rng.random((3000, 3)) * ga.h * (ga.n - 3)
    _, gfd, _ = O.sample(O.Obj(ga, fd_normal=True), ra)
    np.testing.assert_allclose(gfd, np.broadcast_to(coef, gfd.shape), atol=1e-13, rtol=0)
    gq = _quadratic_grid()
    rq = gq.lo + gq.h + rng.random((3000, 3)) * gq.h * (gq.n - 3)
    phi_fd, n_fd, _ = O.sample(O.Obj(gq, fd_normal=True), rq)
    phi_an, n_an, _ = O.sample(O.Obj(gq), rq)
    np.testing.assert_allclose(n_fd, 2.0 * rq, atol=1e-12, rtol=0)
    np.testing.assert_array_equal(phi_fd, phi_an)
    cell = np.floor((rq - gq.lo) / gq.h)
    np.testing.assert_allclose(n_an, 2.0 * (gq.lo + cell * gq.h) + gq.h, atol=1e-12, rtol=0)
    assert np.abs(n_an - n_fd).max() > 0.5 * gq.h  # the two normals differ inside a cell


def test_central_difference_normal_gradient_and_accuracy(oracle_lib):
    """With the seven-query normal the dual gradient of the loss still equals
    central differences of the loss outside kinks. On a sphere's grid the
    seven-query normal is second-order accurate and the analytic gradient of
    the trilinear blend first-order (constant along an axis within a cell),
    so near the surface the former lies closer to the exact normal r/|r|."""
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=8)
    H = O.Hand(hand)
    ob = O.Obj(grid, fd_normal=True)
    P = O.Params(alpha_leak=0.0)
    g = O.step(H, ob, P, q)["grad"]
    fd, ex = O.fd_grad(H, ob, P, q, h=1e-6)
    assert ex.mean() < 0.6
    tol = 1e-5 * np.abs(g).max(axis=1, keepdims=True)
    bad = (np.abs(fd - g) > tol) & ~ex
    assert not bad.any(), np.argwhere(bad)[:5]
    sph = S.make_grid(S.make_object("sphere", seed=0), 64)
    rng = np.random.default_rng(11)
    d = rng.normal(size=(4000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    radius = float(sph.prims[0][2])  # the grid holds |r| - radius about the origin
    pts = d * (radius + rng.uniform(-0.5, 0.5, (4000, 1)) * sph.h * 4)
    _, n_an, _ = O.sample(O.Obj(sph), pts)
    _, n_fd, _ = O.sample(O.Obj(sph, fd_normal=True), pts)
    e_an = np.linalg.norm(n_an - d, axis=1)
    e_fd = np.linalg.norm(n_fd - d, axis=1)
    assert np.median(e_fd) < 0.5 * np.median(e_an), (np.median(e_fd), np.median(e_an))
