"""Pins of the oracle's Coulomb friction (Sec. III-C cites a friction model
without stating it; the reading is positional friction in position-based
dynamics: each active contact's tangential displacement over the step is
removed up to mu C). Closed forms on an inclined plane: a contact sticks
when the test velocity lies within the friction cone (tan(beta) <= mu) and
slides, slowed by mu C, beyond it; the friction correction is tangential;
mu = 0 is the frictionless step bit for bit; the dual gradient equals central
differences of the loss and stays affine in the leak factor. No GPU needed."""
import numpy as np
import pytest

import oracle as O
from paper_2306_08132_amd import synth as S
from tests.helpers import SIM_DIRS, point_hand


def plane(normal, Im=1e6):
    n = np.asarray(normal, float)
    n /= np.linalg.norm(n)
    return n, O.Obj(kind=O.OBJ_PLANE, normal=n, offset=0.0, inertia_over_mass=Im)


@pytest.mark.parametrize("mu", [0.0, 0.3, 0.5, 0.9])
def test_inclined_plane_sticks_inside_the_cone_and_slides_outside(oracle_lib, mu):
    """One contact at the object's centre, on a plane through it whose normal
    makes beta = 20 degrees with +x and 70 degrees with +y. A test moving the
    object by x0 = dt v0 e penetrates by C = |x0| cos(beta) and slides by
    |x0| sin(beta) along the plane: the normal correction removes C, friction
    removes min(|x0| sin(beta), mu C) of the slide. So the object ends at rest
    when tan(beta) <= mu and keeps |x0| (sin(beta) - mu cos(beta)) of its
    tangential motion otherwise (rotation frozen by a huge inertia)."""
    beta = np.deg2rad(20.0)
    n, ob = plane([np.cos(beta), np.sin(beta), 0.0])
    hand = O.Hand(point_hand([[0.0, 0.0, 0.0]]))
    P = O.Params(mu=mu, r_dil=0.0)
    tr = O.trace(hand, ob, P, np.zeros(6))
    dv = P.dt * P.v0
    for m, e in enumerate(SIM_DIRS[:6]):
        x0 = dv * e
        x1 = tr["poses"][m, 1, :3]
        cb = float(e @ n)
        if cb <= 0.0:  # the object moves away from the contact: nothing happens
            np.testing.assert_allclose(x1, x0, atol=1e-18)
            continue
        sb = np.sqrt(max(1.0 - cb * cb, 0.0))
        t = (x0 - (x0 @ n) * n)
        t = t / np.linalg.norm(t)
        slide = max(dv * sb - mu * dv * cb, 0.0)
        np.testing.assert_allclose(x1, slide * t, atol=1e-12 * dv)
        stuck = sb / cb <= mu
        assert (np.linalg.norm(x1) < 1e-10 * dv) == stuck, (m, mu, sb / cb)
        # the correction beyond the normal one is tangential
        corr = x1 - x0 + (dv * cb) * n
        assert abs(corr @ n) <= 1e-12 * dv


def test_zero_friction_is_the_frictionless_step(oracle_lib):
    hand, grid, q = S.config_workload("tiny", B=12)
    H, ob = O.Hand(hand.rounded()), O.Obj(grid)
    a = O.step(H, ob, O.Params(r_dil=0.005), q)
    b = O.step(H, ob, O.Params(r_dil=0.005, mu=0.0), q)
    assert np.array_equal(a["loss"], b["loss"]) and np.array_equal(a["grad"], b["grad"])
    c = O.step(H, ob, O.Params(r_dil=0.005, mu=0.5), q)
    assert np.abs(c["loss"] - a["loss"]).max() > 1e-3


@pytest.mark.parametrize("K", [1, 3])
def test_friction_gradient_is_central_differences(oracle_lib, K):
    """Exact gradient (alpha = 0) against FP64 central differences of the loss
    on an analytic sphere, outside kinks (the static/kinetic switch, contact
    changes and the rest flagged by the oracle's discrete-state signature)."""
    rng = np.random.default_rng(21)
    d = rng.normal(size=(12, 3))
    pts = d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(0.038, 0.041, size=(12, 1))
    hand = O.Hand(point_hand(pts))
    ob = O.Obj(kind=O.OBJ_SPHERE, center=(0.002, -0.001, 0.0), radius=0.04, inertia_over_mass=0.4 * 0.04 ** 2)
    q = rng.normal(size=(6, 6)) * np.array([2e-3, 2e-3, 2e-3, 0.02, 0.02, 0.02])
    P = O.Params(mu=0.6, K=K, alpha_leak=0.0, r_dil=0.001)
    g = O.step(hand, ob, P, q)["grad"]
    fd, ex = O.fd_grad(hand, ob, P, q, h=1e-7)
    ok = ~ex
    assert ok.mean() > 0.7
    scale = np.abs(fd).max(axis=1, keepdims=True)
    assert np.all(np.abs(g - fd)[ok] <= 2e-5 * np.broadcast_to(scale, g.shape)[ok])


def test_friction_gradient_on_a_grid_and_leak_linearity(oracle_lib):
    """On the small workload's grid with friction: the dual gradient against
    central differences (alpha = 0, kink-excluded), and the leaky gradient
    affine in alpha (grad(0.1) = grad(0) + 0.1 (grad(1) - grad(0)))."""
    hand, grid, q = S.config_workload("tiny", B=6)
    H, ob = O.Hand(hand.rounded()), O.Obj(grid)
    P0 = O.Params(mu=0.5, alpha_leak=0.0, r_dil=0.004)
    g0 = O.step(H, ob, P0, q)["grad"]
    fd, ex = O.fd_grad(H, ob, P0, q, h=1e-7)
    ok = ~ex
    assert ok.mean() > 0.5
    scale = np.abs(fd).max(axis=1, keepdims=True)
    assert np.all(np.abs(g0 - fd)[ok] <= 1e-4 * np.broadcast_to(scale, g0.shape)[ok])
    g1 = O.step(H, ob, O.Params(mu=0.5, alpha_leak=1.0, r_dil=0.004), q)["grad"]
    gl = O.step(H, ob, O.Params(mu=0.5, alpha_leak=0.1, r_dil=0.004), q)["grad"]
    np.testing.assert_allclose(gl, g0 + 0.1 * (g1 - g0), rtol=1e-9, atol=1e-9 * np.abs(g1).max())


@pytest.mark.parametrize("beta_mrad, stuck", [(0.0, False), (0.5, False), (2.0, True)])
def test_friction_floor(oracle_lib, beta_mrad, stuck):
    """A slide up to 1e-3 dt v0 has no direction and gets no friction: on a
    plane tilted by beta from the +x test's direction, the +x test slides by
    dt v0 sin(beta). At beta = 0 and 0.5 mrad (slides 0 and 5e-4 dt v0) the
    object keeps its slide, as without friction; at 2 mrad (2e-3 dt v0, far
    inside the cone for mu = 0.5) it sticks."""
    beta = beta_mrad * 1e-3
    n, ob = plane([np.cos(beta), np.sin(beta), 0.0])
    hand = O.Hand(point_hand([[0.0, 0.0, 0.0]]))
    P = O.Params(mu=0.5, r_dil=0.0)
    x1 = O.trace(hand, ob, P, np.zeros(6))["poses"][0, 1, :3]
    x0 = P.dt * P.v0 * np.array([1.0, 0.0, 0.0])
    free = x0 - (x0 @ n) * n
    if stuck:
        assert np.linalg.norm(x1) < 1e-12 * P.dt * P.v0
    else:
        np.testing.assert_allclose(x1, free, atol=1e-15 * P.dt * P.v0)
        x1f = O.trace(hand, ob, O.Params(mu=0.0, r_dil=0.0), np.zeros(6))["poses"][0, 1, :3]
        assert np.array_equal(x1, x1f)
