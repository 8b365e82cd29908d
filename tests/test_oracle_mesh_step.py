"""Pins of the oracle's grasp step on a mesh object (Sec. III-B's Phong signed
distance inside Sec. III-C's constraint): the step's sampler against the mesh
query routine; on a flat face the step is the step on that face's plane, bit
for bit up to rounding; the dual gradient against central differences of the
loss; and the leaky rule's hand-point part along the stated normal (the
gradient the paper states), in closed form. No GPU needed."""
import numpy as np
import pytest

import oracle as O
from paper_2306_08132_amd import synth as S
from tests.helpers import SIM_DIRS, point_hand


def octahedron(scale):
    """Vertices +-scale e_i with radial unit normals; faces counter-clockwise
    seen from outside."""
    V = np.concatenate([np.eye(3), -np.eye(3)])
    faces = []
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                a = 0 if sx > 0 else 3
                b = 1 if sy > 0 else 4
                c = 2 if sz > 0 else 5
                faces.append((a, b, c) if sx * sy * sz > 0 else (a, c, b))
    return S.TriMesh(scale * V, np.array(faces, np.int32), V.copy())


def sphere_mesh(radius, lev=2):
    m = S.icosphere(lev)
    return S.TriMesh(radius * m.vertices, m.faces, m.normals)


def mesh_obj(m, alpha, Im):
    M = O.Mesh(m.vertices, m.faces, m.normals, alpha)
    return M, O.Obj(mesh=M, inertia_over_mass=Im)


def test_step_sampler_is_the_mesh_query(oracle_lib):
    """Value and stated normal of the step's sampler (region-wise formula in
    the step's scalar type) against the mesh query routine, around a
    2-subdivision icosphere of 4 cm at alpha = 0.5."""
    m = sphere_mesh(0.04)
    M, ob = mesh_obj(m, 0.5, 1e-3)
    rng = np.random.default_rng(3)
    d = rng.normal(size=(400, 3))
    r = d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(0.02, 0.06, size=(400, 1))
    phi, g, _ = O.sample(ob, r)
    ref = O.mesh_sdf(M, r)
    np.testing.assert_allclose(phi, ref["rho"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(g, ref["grad"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("K", [1, 3])
def test_flat_face_step_is_the_plane_step(oracle_lib, K):
    """alpha = 0 and every sample's closest point inside the face (e_x, e_y,
    e_z) of a 5 cm octahedron: the mesh's distance there is the face plane's,
    x + y + z = 5 cm, so loss and gradient equal the step on that plane."""
    s = 0.05
    m = octahedron(s)
    Im = 4e-4
    _, ob = mesh_obj(m, 0.0, Im)
    n = np.ones(3) / np.sqrt(3.0)
    plane = O.Obj(kind=O.OBJ_PLANE, normal=n, offset=s / np.sqrt(3.0), inertia_over_mass=Im)
    c = np.full(3, s / 3.0)
    t1 = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    t2 = np.cross(n, t1)
    rng = np.random.default_rng(5)
    pts = [c + 0.006 * (a * t1 + b * t2) + depth * n
           for a, b, depth in zip(rng.uniform(-1, 1, 10), rng.uniform(-1, 1, 10), rng.uniform(-2e-3, 1.5e-3, 10))]
    hand = O.Hand(point_hand(pts))
    q = rng.normal(size=(6, 6)) * np.array([1e-3, 1e-3, 1e-3, 0.01, 0.01, 0.01])
    P = O.Params(K=K, r_dil=0.0005)
    a, b = O.step(hand, ob, P, q), O.step(hand, plane, P, q)
    np.testing.assert_allclose(a["loss"], b["loss"], rtol=1e-10)
    scale = np.abs(b["grad"]).max(axis=1, keepdims=True)
    np.testing.assert_allclose(a["grad"], b["grad"], rtol=0, atol=1e-9 * scale.max())
    assert np.abs(b["grad"]).max() > 0.0


@pytest.mark.parametrize("K", [1, 3])
def test_mesh_step_gradient_is_central_differences(oracle_lib, K):
    """Exact gradient (alpha_leak = 0) of the step on a Phong icosphere
    (alpha = 0.5) against FP64 central differences of the loss, outside
    kinks (face, region and sign changes are part of the discrete-state
    signature)."""
    m = sphere_mesh(0.04)
    _, ob = mesh_obj(m, 0.5, 0.4 * 0.04 ** 2)
    rng = np.random.default_rng(11)
    d = rng.normal(size=(12, 3))
    pts = d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(0.0375, 0.0405, size=(12, 1))
    hand = O.Hand(point_hand(pts))
    q = rng.normal(size=(6, 6)) * np.array([1e-3, 1e-3, 1e-3, 0.01, 0.01, 0.01])
    P = O.Params(K=K, alpha_leak=0.0, r_dil=0.001)
    g = O.step(hand, ob, P, q)["grad"]
    fd, ex = O.fd_grad(hand, ob, P, q, h=1e-7)
    ok = ~ex
    assert ok.mean() > 0.6
    scale = np.abs(fd).max(axis=1, keepdims=True)
    assert np.all(np.abs(g - fd)[ok] <= 2e-5 * np.broadcast_to(scale, g.shape)[ok])


def test_leak_takes_the_stated_normal(oracle_lib):
    """One contact 4 mm outside a Phong icosphere (alpha = 0.75), so no test
    penetrates: every correction is zero in value and the loss gradient along
    the wrist's x comes from the leak alone. With dC = -alpha dd_hand and
    dd_hand = g . dp, g the stated normal (r - p) / rho (the gradient the
    paper states, as the trilinear gradient is on a grid), the +-axis tests
    give
      dL/dq_x = w_s / (7 dt) sum_m (e_m . g_m) alpha g_m,x / w_m,
    w_m = |g_m|^2 + |a_m x g_m|^2 / (I/m). The exact gradient of rho (central
    differences of the mesh query) in place of g gives a different number."""
    m = sphere_mesh(0.04, lev=1)
    Im = 0.4 * 0.04 ** 2
    M, ob = mesh_obj(m, 0.75, Im)
    p = np.array([0.017, 0.029, 0.031])
    p *= (0.04 + 0.004) / np.linalg.norm(p)
    hand = O.Hand(point_hand([p]))
    al = 0.3
    P = O.Params(alpha_leak=al, r_dil=0.0, w_pen=0.0)
    dv = P.dt * P.v0
    got = O.step(hand, ob, P, np.zeros((1, 6)))["grad"][0, 0]
    want, exact = 0.0, 0.0
    h = 1e-7
    for e in SIM_DIRS[:6]:
        r = p - dv * np.asarray(e)  # the object moved by dv e: the hand point in its frame
        out = O.mesh_sdf(M, r[None])
        assert out["rho"][0] > 1e-3
        gm = out["grad"][0]
        grad = np.array([(O.mesh_sdf(M, (r + h * u)[None])["rho"][0] - O.mesh_sdf(M, (r - h * u)[None])["rho"][0])
                         / (2 * h) for u in np.eye(3)])
        u = np.cross(r, gm)
        w = gm @ gm + (u @ u) / Im
        want += (np.asarray(e) @ gm) * al * gm[0] / w
        exact += (np.asarray(e) @ gm) * al * grad[0] / w
    want *= P.w_stable / (7 * P.dt)
    exact *= P.w_stable / (7 * P.dt)
    assert got == pytest.approx(want, rel=1e-9)
    assert abs(exact - want) > 1e-3 * abs(want)
