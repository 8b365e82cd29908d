"""Pins of the oracle's grasp step (Sec. III-C PBD step, Sec. IV-A losses and
optimizer) against closed forms, invariants, an Eq. (1) evaluation with a
finite-difference constraint Jacobian, and finite differences of the loss."""
import numpy as np
import pytest

from paper_2306_08132_amd import synth as S
from tests.helpers import SIM_DIRS, point_hand, rotvec_matrix

R_SPH = 0.04


def sphere_obj(O, center=(0.0, 0.0, 0.0), R=R_SPH):
    return O.Obj(kind=O.OBJ_SPHERE, center=center, radius=R, inertia_over_mass=0.4 * R * R)


def plane_obj(O, normal=(0.0, 0.0, 1.0), offset=0.0, Im=1e-3):
    return O.Obj(kind=O.OBJ_PLANE, normal=normal, offset=offset, inertia_over_mass=Im)


def q_wrist(t=(0.0, 0.0, 0.0)):
    q = np.zeros(6)
    q[:3] = t
    return q


# ---------------------------------------------------------------------------
# numpy evaluation of Eq. (1) with a numerical constraint Jacobian
# ---------------------------------------------------------------------------
def _phi_np(kind, r, center=None, R=None, normal=None, offset=None):
    if kind == "sphere":
        return np.linalg.norm(r - center) - R
    return float(np.dot(r, normal) - offset)


def eq1_correction(points, x, theta, Im, r_dil, phi):
    """Average over the active (C > 0) constraints of -M^-1 J^T (J M^-1 J^T)^-1 C
    (Eq. (1)), where C(x, R) = max(0, -(phi(R^T (p - x)) - r_dil)) and J is
    taken by central differences over x and over a world-frame rotation
    exp([e]x) R. The average is the parallel stand-in for the paper's
    Gauss-Seidel step over the constraints."""
    R0 = rotvec_matrix(theta)
    Minv = np.diag([1, 1, 1, 1 / Im, 1 / Im, 1 / Im])
    total = np.zeros(6)

    def C(p, dx, de):
        R = rotvec_matrix(de) @ R0
        return max(0.0, -(phi(R.T @ (p - (x + dx))) - r_dil))

    eps = 1e-7
    n_active = 0
    for p in points:
        c0 = C(p, np.zeros(3), np.zeros(3))
        if c0 <= 0.0:
            continue
        n_active += 1
        J = np.zeros(6)
        for a in range(3):
            e = np.zeros(3)
            e[a] = eps
            J[a] = (C(p, e, np.zeros(3)) - C(p, -e, np.zeros(3))) / (2 * eps)
            J[3 + a] = (C(p, np.zeros(3), e) - C(p, np.zeros(3), -e)) / (2 * eps)
        total += -Minv @ J * c0 / (J @ Minv @ J)
    return total / max(n_active, 1)


@pytest.mark.parametrize("K", [1, 3])
@pytest.mark.parametrize("shape", ["sphere", "plane"])
def test_correction_is_eq1_with_numerical_jacobian(oracle_lib, K, shape):
    O = oracle_lib
    rng = np.random.default_rng(11)
    if shape == "sphere":
        c = np.array([0.01, -0.005, 0.002])
        ob = sphere_obj(O, center=c)
        Im = 0.4 * R_SPH ** 2
        phi = lambda r: _phi_np("sphere", r, center=c, R=R_SPH)
        d = rng.normal(size=(6, 3))
        pts = c + d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(0.03, 0.045, size=(6, 1))
    else:
        n = np.array([0.3, -0.2, 1.0])
        n /= np.linalg.norm(n)
        Im = 2e-4
        ob = plane_obj(O, normal=n, offset=0.004, Im=Im)
        phi = lambda r: _phi_np("plane", r, normal=n, offset=0.004)
        pts = rng.normal(size=(5, 3)) * 0.02
    hand = O.Hand(point_hand(pts))
    P = O.Params(K=K, omega=0.7, r_dil=0.002)
    tr = O.trace(hand, ob, P, q_wrist())
    poses = tr["poses"]
    for m in range(7):
        np.testing.assert_allclose(poses[m, 0, :3], P.dt * P.v0 * SIM_DIRS[m], atol=1e-18)
        np.testing.assert_array_equal(poses[m, 0, 3:], 0.0)
        for k in range(K):
            x, th = poses[m, k, :3], poses[m, k, 3:]
            want = P.omega * eq1_correction(pts, x, th, Im, P.r_dil, phi)
            got = poses[m, k + 1] - poses[m, k]
            np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-12)


def test_rotated_object_frame_samples(oracle_lib):
    """After a rotating iteration, samples use r = R(theta)^T (p - x) and
    g = R(theta) grad(phi)(r), with R the rotation-vector exponential."""
    O = oracle_lib
    c = np.array([0.012, 0.0, -0.004])
    ob = sphere_obj(O, center=c)
    rng = np.random.default_rng(12)
    d = rng.normal(size=(8, 3))
    pts = c + d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(0.025, 0.045, size=(8, 1))
    P = O.Params(K=3, r_dil=0.001)
    tr = O.trace(O.Hand(point_hand(pts)), ob, P, q_wrist())
    assert np.abs(tr["poses"][:, 1:, 3:]).max() > 1e-3  # the object did rotate
    for m in range(7):
        for k in range(3):
            x, th = tr["poses"][m, k, :3], tr["poses"][m, k, 3:]
            R = rotvec_matrix(th)
            r = (pts - x) @ R  # rows: R^T (p - x)
            dist = np.linalg.norm(r - c, axis=1)
            np.testing.assert_allclose(tr["samples"][m, k, :, 0], dist - R_SPH - P.r_dil, atol=1e-15)
            g = ((r - c) / dist[:, None]) @ R.T
            np.testing.assert_allclose(tr["samples"][m, k, :, 1:4], g, atol=1e-14)


def test_linear_constraint_resolved_in_one_iteration(oracle_lib):
    """One contact below a plane with its lever arm along the normal:
    dx = -C n, dtheta = 0, and the next iteration sees C = 0 exactly."""
    O = oracle_lib
    delta = 0.003
    ob = plane_obj(O, normal=(0, 0, 1), offset=0.0)
    P = O.Params(K=2)
    tr = O.trace(O.Hand(point_hand([[0.0, 0.0, -delta]])), ob, P, q_wrist())
    for m in (4, 5, 6):  # lever arm stays along z for the z and rest tests
        x0 = tr["poses"][m, 0, :3]
        C = delta + x0[2]
        np.testing.assert_allclose(tr["poses"][m, 1, :3] - x0, [0, 0, -C], atol=1e-18)
        np.testing.assert_array_equal(tr["poses"][m, 1, 3:], 0.0)
        assert abs(tr["samples"][m, 1, 0, 0]) <= 1e-18
        assert tr["samples"][m, 1, 0, 5] == 0.0 or abs(tr["samples"][m, 1, 0, 5]) < 1e-18


def test_aligned_contacts_resolve_once(oracle_lib):
    """Three contacts at the same depth below a plane, lever arms along the
    normal: the averaged update is the single-contact one (-C n), not three
    times it, and the next iteration sees no penetration."""
    O = oracle_lib
    delta = 0.002
    ob = plane_obj(O, normal=(0, 0, 1), offset=0.0)
    P = O.Params(K=2)
    pts = [[0.0, 0.0, -delta], [0.0, 0.0, -delta], [0.0, 0.0, -delta]]
    tr = O.trace(O.Hand(point_hand(pts)), ob, P, q_wrist())
    for m in (4, 5, 6):
        x0 = tr["poses"][m, 0, :3]
        C = delta + x0[2]
        np.testing.assert_allclose(tr["poses"][m, 1, :3] - x0, [0, 0, -C], atol=1e-18)
        assert np.all(np.abs(tr["samples"][m, 1, :, 0]) <= 1e-18)


def test_many_iterations_stay_bounded(oracle_lib):
    """Sixteen projection iterations on a grid with many penetrating contacts:
    the averaged iteration keeps the poses bounded (the summed form overshoots
    by the contact count each iteration), and the leak confined to hand
    points keeps the gradient within a small factor of the one-iteration
    gradient (leaking along the pose chain compounds it to ~1e25)."""
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=6)
    P = O.Params(K=16, r_dil=0.01)
    r = O.step(O.Hand(hand.rounded()), O.Obj(grid), P, q)
    assert np.isfinite(r["loss"]).all() and np.isfinite(r["grad"]).all()
    assert np.abs(r["grad"]).max() < 1e7
    tr = O.trace(O.Hand(hand.rounded()), O.Obj(grid), P, q[0])
    assert np.abs(tr["poses"]).max() < 0.1  # metres / radians


def test_nonpenetrating_contacts_contribute_exactly_zero(oracle_lib):
    """A sample corrects the pose (lambda < 0) exactly when it penetrates
    beyond the contact tolerance, d < -5e-3 dt v0; every other sample,
    including those between -eps and 0, contributes exactly zero."""
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=8)
    H, ob = O.Hand(hand), O.Obj(grid)
    P = O.Params()
    eps = 5e-3 * P.dt * P.v0
    seen_band = 0
    for b in range(8):
        for r_dil in (0.0, 0.004):
            P.r_dil = r_dil
            tr = O.trace(H, ob, P, q[b])
            s = tr["samples"]
            assert np.all(s[..., 5][s[..., 0] >= -eps] == 0.0)
            assert np.all(s[..., 5][s[..., 0] < -eps] < 0.0)
            seen_band += int(((s[..., 0] < 0.0) & (s[..., 0] >= -eps)).sum())
    assert seen_band > 0


def test_no_contact_gives_free_flight(oracle_lib):
    """Hand far from the object: no correction, v+ = v0 in six tests, so
    L_stable = 6 v0 / 7 and L_pen = 0."""
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=4)
    q = q.copy()
    q[:, :3] *= 10.0  # 1 m away, outside the grid box
    H, ob = O.Hand(hand), O.Obj(grid)
    for v0 in (1.0, 0.25):
        P = O.Params(v0=v0)
        out = O.step(H, ob, P, q, grad=False)
        np.testing.assert_allclose(out["terms"][:, 0], 6 * v0 / 7, rtol=1e-15)
        np.testing.assert_array_equal(out["terms"][:, 1], 0.0)
        tr = O.trace(H, ob, P, q[0])
        np.testing.assert_array_equal(tr["poses"][:, 1], tr["poses"][:, 0])


def test_antipodal_contacts_cancel(oracle_lib):
    """Equal penetrations at +-a: in the rest test the summed correction is 0."""
    O = oracle_lib
    rng = np.random.default_rng(13)
    d = rng.normal(size=(5, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    depth = rng.uniform(0.001, 0.004, size=(5, 1))
    half = d * (R_SPH - depth)
    pts = np.concatenate([half, -half])
    P = O.Params()
    tr = O.trace(O.Hand(point_hand(pts)), sphere_obj(O), P, q_wrist())
    np.testing.assert_allclose(tr["poses"][6, 1], 0.0, atol=1e-15)
    lam = tr["samples"][6, 0, :, 5]
    assert np.all(lam < 0)
    # on a grid symmetric about the origin the cancellation holds to rounding
    g = S.make_grid(S.make_object("sphere", seed=0, radius=R_SPH), 65)
    tr = O.trace(O.Hand(point_hand(pts)), O.Obj(g), P, q_wrist())
    s = tr["samples"][6, 0]
    scale = np.abs(s[:, 5, None] * s[:, 1:4]).sum()
    assert np.abs(tr["poses"][6, 1, :3]).max() <= 1e-6 * scale


def test_dilation_equals_grown_sphere(oracle_lib):
    O = oracle_lib
    hand, _, q = S.config_workload("tiny", B=3)
    H = O.Hand(hand)
    r = 0.006
    a = O.step(H, sphere_obj(O, R=R_SPH), O.Params(r_dil=r), q, grad=False)
    ob2 = O.Obj(kind=O.OBJ_SPHERE, radius=R_SPH + r, inertia_over_mass=0.4 * R_SPH ** 2)
    b = O.step(H, ob2, O.Params(r_dil=0.0), q, grad=False)
    np.testing.assert_allclose(a["loss"], b["loss"], rtol=1e-12)


def test_joint_loss_special_values(oracle_lib):
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=1)
    H, ob = O.Hand(hand), O.Obj(grid)
    mid = 0.5 * (hand.q_low + hand.q_up)
    base = q[0].copy()
    base[:3] *= 10.0
    base[6:] = mid[6:]
    t = O.step(H, ob, O.Params(), base, grad=False)["terms"][0]
    assert t[2] == 0.0 and t[3] == 0.0
    j = 8
    span = hand.q_up[j] - mid[j]
    for delta, lim in [(0.3 * span, 0.0), (span + 0.05, 0.05), (-span - 0.02, 0.02)]:
        qq = base.copy()
        qq[j] = mid[j] + delta
        t = O.step(H, ob, O.Params(), qq, grad=False)["terms"][0]
        assert t[2] == pytest.approx(abs(delta), rel=1e-12)
        assert t[3] == pytest.approx(lim, rel=1e-9, abs=1e-15)
    # wrist entries never enter the joint losses
    qq = base.copy()
    qq[3:6] += 5.0
    t = O.step(H, ob, O.Params(), qq, grad=False)["terms"][0]
    assert t[2] == 0.0 and t[3] == 0.0


def test_leaky_gradient_zero_without_leak_and_linear_in_alpha(oracle_lib):
    """With no penetration anywhere, the exact gradient of L_stable is 0 and
    the leaky gradient is linear in alpha (Sec. III-C, leaky gradient)."""
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=3)
    q = q.copy()
    q[:, :3] *= 3.0  # 30 cm away: nothing touches
    H, ob = O.Hand(hand), O.Obj(grid)
    base = dict(w_range=0.0, w_limit=0.0)
    g0 = O.step(H, ob, O.Params(alpha_leak=0.0, **base), q)["grad"]
    g1 = O.step(H, ob, O.Params(alpha_leak=1.0, **base), q)["grad"]
    ga = O.step(H, ob, O.Params(alpha_leak=0.1, **base), q)["grad"]
    np.testing.assert_array_equal(g0, 0.0)
    assert np.abs(g1).max() > 0
    np.testing.assert_allclose(ga, 0.1 * g1, rtol=1e-12, atol=1e-12 * np.abs(g1).max())


def test_leak_is_affine_in_alpha_over_iterations(oracle_lib):
    """With several projection iterations and penetrating contacts, the
    gradient is affine in alpha: the leak acts on hand points only and its
    tangent then travels through the exact iteration map. (Leaking along the
    object-pose chain too would add alpha^2, alpha^3, ... terms.)"""
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=3)
    H, ob = O.Hand(hand), O.Obj(grid)
    g = {a: O.step(H, ob, O.Params(K=3, r_dil=0.01, alpha_leak=a), q)["grad"] for a in (0.0, 0.1, 0.2, 0.4)}
    d1 = g[0.1] - g[0.0]
    assert np.abs(d1).max() > 1e-6 * np.abs(g[0.0]).max()  # the leak matters here
    scale = np.abs(g[0.4]).max()
    np.testing.assert_allclose(g[0.2] - g[0.0], 2.0 * d1, atol=1e-9 * scale)
    np.testing.assert_allclose(g[0.4] - g[0.0], 4.0 * d1, atol=1e-9 * scale)


@pytest.mark.parametrize("h", [1e-4, 1e-6])
def test_gradient_matches_finite_differences_on_sphere(oracle_lib, h):
    O = oracle_lib
    hand, _, q = S.config_workload("tiny", B=12)
    H, ob = O.Hand(hand), sphere_obj(O)
    P = O.Params(alpha_leak=0.0, K=1)
    g = O.step(H, ob, P, q)["grad"]
    fd, ex = O.fd_grad(H, ob, P, q, h=h)
    assert ex.mean() < 0.5
    tol = (2e-4 if h == 1e-4 else 1e-6) * np.abs(g).max(axis=1, keepdims=True)
    bad = (np.abs(fd - g) > tol) & ~ex
    assert not bad.any(), np.argwhere(bad)[:5]


def test_gradient_matches_finite_differences_on_grid(oracle_lib):
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=12)
    H, ob = O.Hand(hand), O.Obj(grid)
    for K in (1, 3):
        P = O.Params(alpha_leak=0.0, K=K)
        g = O.step(H, ob, P, q)["grad"]
        fd, ex = O.fd_grad(H, ob, P, q, h=1e-6)
        assert ex.mean() < 0.6
        tol = 1e-5 * np.abs(g).max(axis=1, keepdims=True)
        bad = (np.abs(fd - g) > tol) & ~ex
        assert not bad.any(), np.argwhere(bad)[:5]


def test_adam_first_step_and_constant_gradient(oracle_lib):
    O = oracle_lib
    q, m, v, g = S.adam_state(4, 10, seed=2)
    lr, eps = 1e-3, 1e-8
    q1, m1, v1 = O.adam(q, np.zeros_like(m), np.zeros_like(v), g, 1, lr=lr, eps=eps)
    np.testing.assert_allclose(q1 - q, -lr * g / (np.abs(g) + eps), rtol=1e-12)
    # constant gradient: bias correction makes every step -lr g / (|g| + eps)
    qq, mm, vv = q.copy(), np.zeros_like(m), np.zeros_like(v)
    for t in range(1, 21):
        qq, mm, vv = O.adam(qq, mm, vv, g, t, lr=lr, eps=eps)
    np.testing.assert_allclose(qq - q, -20 * lr * g / (np.abs(g) + eps), rtol=1e-9)


def test_rank_is_stable_sort(oracle_lib):
    O = oracle_lib
    r = O.rank(np.array([3.0, 1.0, 2.0, 1.0, 0.0, 2.0]))
    assert r.tolist() == [4, 1, 3, 2, 5, 0]


def test_optimize_is_steps_then_adam_with_linear_dilation(oracle_lib):
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=6)
    H, ob = O.Hand(hand), O.Obj(grid)
    T, r0 = 4, 0.01
    out = O.optimize(H, ob, O.Params(), q, T=T, r0=r0, history=True)
    qq = q.copy()
    m = np.zeros_like(qq)
    v = np.zeros_like(qq)
    for t in range(T):
        st = O.step(H, ob, O.Params(r_dil=r0 * (1 - t / (T - 1))), qq)
        np.testing.assert_array_equal(st["loss"], out["history"][t])
        qq, m, v = O.adam(qq, m, v, st["grad"], t + 1)
    np.testing.assert_array_equal(qq, out["q"])
    fin = O.step(H, ob, O.Params(r_dil=0.0), qq, grad=False)
    np.testing.assert_array_equal(fin["loss"], out["loss"])
    assert out["rank"].tolist() == np.argsort(fin["loss"], kind="stable").tolist()
