"""Pins of the oracle's mesh Phong signed distance (Sec. III-B) against what
geometry fixes: the closest point of a triangle against dense sampling of it,
a box mesh against the exact box SDF (distance and sign, inside and outside),
the winding number against inside/outside of a sphere, the flat gradient
against central differences, flat faces unchanged by the Phong blend, the
Phong surface closer to a sphere than the flat mesh, and the gradient
pointing towards increasing distance (the sign reading of the stated
gradient). No GPU needed."""
import numpy as np
import pytest

import oracle as O
from paper_2306_08132_amd import synth as S


def omesh(m, alpha):
    return O.Mesh(m.vertices, m.faces, m.normals, alpha)


def test_closest_point_on_triangle_minimizes():
    rng = np.random.default_rng(0)
    u, v = np.meshgrid(np.linspace(0, 1, 301), np.linspace(0, 1, 301))
    keep = u + v <= 1.0
    u, v = u[keep], v[keep]
    for _ in range(30):
        a, b, c = rng.normal(size=(3, 3))
        r = rng.normal(size=3) * 2.0
        x, bary = O.closest_on_triangle(a, b, c, r)
        assert np.all(bary >= -1e-12) and abs(bary.sum() - 1.0) < 1e-12
        assert np.allclose(x, bary[0] * a + bary[1] * b + bary[2] * c, atol=1e-12)
        samples = a + u[:, None] * (b - a) + v[:, None] * (c - a)
        dmin = np.linalg.norm(samples - r, axis=1).min()
        d = np.linalg.norm(x - r)
        assert d <= dmin + 1e-12
        # the dense grid's spacing bounds how far it can miss the minimum
        assert dmin - d <= np.linalg.norm(np.stack([b - a, c - a]), axis=1).max() / 300 + 1e-12


@pytest.mark.parametrize("splits", [1, 3])
def test_box_mesh_is_the_exact_box_sdf(splits):
    half = np.array([0.02, 0.03, 0.015])
    m = S.mesh_box(half, splits=splits)
    rng = np.random.default_rng(splits)
    r = rng.uniform(-0.05, 0.05, size=(3000, 3))
    r[:1000] *= 0.25  # plenty of inside points
    out = O.mesh_sdf(omesh(m, 0.0), r)
    exact = S.box_sdf(r, np.zeros(3), np.eye(3), half)
    assert np.abs(out["rho"] - exact).max() < 1e-15
    assert (exact < 0).sum() > 500


def test_winding_number_inside_outside():
    m = S.icosphere(2)
    M = omesh(m, 0.0)
    rng = np.random.default_rng(1)
    for _ in range(40):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        assert O.winding_number(M, d * rng.uniform(0.0, 0.9)) == pytest.approx(1.0, abs=1e-9)
        assert O.winding_number(M, d * rng.uniform(1.1, 3.0)) == pytest.approx(0.0, abs=1e-9)


def test_flat_gradient_is_central_difference():
    m = S.mesh_ellipsoid([0.03, 0.02, 0.04], subdivisions=2)
    M = omesh(m, 0.0)
    rng = np.random.default_rng(2)
    r = rng.uniform(-0.06, 0.06, size=(400, 3))
    out = O.mesh_sdf(M, r)
    h = 1e-7
    fd = np.zeros_like(r)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd[:, j] = (O.mesh_sdf(M, r + e)["rho"] - O.mesh_sdf(M, r - e)["rho"]) / (2 * h)
    ok = out["gap"] > 1e-4  # away from points equidistant from two parts of the surface
    assert ok.sum() > 150
    assert np.abs(fd[ok] - out["grad"][ok]).max() < 1e-6


def test_phong_keeps_flat_faces():
    """Where a face's three vertex normals equal its own normal, every vertex
    tangent plane is the face's plane and the curved point is the flat one."""
    half = np.array([0.02, 0.03, 0.015])
    m = S.mesh_box(half, splits=4)
    rng = np.random.default_rng(3)
    r = rng.uniform(-0.05, 0.05, size=(3000, 3))
    flat = O.mesh_sdf(omesh(m, 0.0), r)
    curved = O.mesh_sdf(omesh(m, 1.0), r)
    fn = np.cross(m.vertices[m.faces[:, 1]] - m.vertices[m.faces[:, 0]],
                  m.vertices[m.faces[:, 2]] - m.vertices[m.faces[:, 0]])
    fn /= np.linalg.norm(fn, axis=1, keepdims=True)
    planar = np.all(np.abs((m.normals[m.faces] * fn[:, None, :]).sum(axis=2) - 1.0) < 1e-12, axis=1)
    sel = planar[flat["face"]]
    assert sel.sum() > 200
    assert np.abs(curved["rho"][sel] - flat["rho"][sel]).max() < 1e-15
    # elsewhere the blend moves the surface
    assert np.abs(curved["rho"][~sel] - flat["rho"][~sel]).max() > 1e-5


def test_phong_is_closer_to_the_sphere():
    m = S.icosphere(2)
    rng = np.random.default_rng(4)
    d = rng.normal(size=(2000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = d * rng.uniform(0.9, 1.1, size=(2000, 1))
    exact = np.linalg.norm(r, axis=1) - 1.0
    e_flat = np.abs(O.mesh_sdf(omesh(m, 0.0), r)["rho"] - exact).mean()
    e_phong = np.abs(O.mesh_sdf(omesh(m, 0.75), r)["rho"] - exact).mean()
    assert e_phong < 0.75 * e_flat


def test_gradient_points_to_increasing_distance():
    """The stated gradient (r - p) / rho: a small step along it increases rho,
    inside and outside."""
    m = S.mesh_ellipsoid([0.03, 0.02, 0.04], subdivisions=2)
    M = omesh(m, 0.75)
    rng = np.random.default_rng(5)
    r = rng.uniform(-0.05, 0.05, size=(600, 3))
    r[:300] *= 0.4  # inside points
    out = O.mesh_sdf(M, r)
    ok = (out["gap"] > 1e-4) & (np.abs(out["rho"]) > 1e-4)
    step = O.mesh_sdf(M, r + 1e-6 * out["grad"])["rho"]
    assert ok.sum() > 200 and (out["rho"][ok] < 0).sum() > 50
    assert np.all(step[ok] > out["rho"][ok])
    assert np.allclose(np.linalg.norm(out["grad"], axis=1), 1.0, atol=1e-12)
