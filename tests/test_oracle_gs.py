"""Pins of the oracle's literal Gauss-Seidel projection (Sec. III-C: the
constraint updates of Eq. (1) applied one after another). On a plane with
the object's rotation frozen (huge inertia), every update is a translation
along the normal, so a sweep ends with the deepest penetration resolved
exactly, x = x0 + min_i d_i n, whatever the order, while the averaged form
moves by the mean of the active d_i. With a single penetrating contact both
forms take the same step. The dual-number gradient of the sweep equals FP64
central differences (h = 1e-7) outside kinks, on a sphere and on a grid,
K = 1 and 2.
No GPU needed."""
import numpy as np
import pytest

from paper_2306_08132_amd import synth as S

GS = 1


def plane(O, normal, offset, Im=1e12):
    return O.Obj(kind=O.OBJ_PLANE, normal=normal, offset=offset, inertia_over_mass=Im)


def test_gs_on_a_plane_resolves_the_deepest(oracle_lib):
    O = oracle_lib
    hand, _, q = S.config_workload("tiny", B=4)
    H = O.Hand(hand)
    rng = np.random.default_rng(3)
    for b in range(4):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        p = O.fk(H, q[b])[0]
        h = p @ n
        off = np.quantile(h, 0.2)  # a fifth of the contacts below the plane
        ob = plane(O, n, off)
        for proj in (0, GS):
            P = O.Params(projection=proj, r_dil=0.001)
            tr = O.trace(H, ob, P, q[b], samples=False)
            for m in range(7):
                x0 = tr["poses"][m, 0, :3]
                d = (p - x0) @ n - off - P.r_dil
                act = d < 0
                assert act.sum() > 10
                want = x0 + (d.min() if proj == GS else d[act].mean()) * n
                np.testing.assert_allclose(tr["poses"][m, 1, :3], want, rtol=0, atol=1e-12)
                assert np.abs(tr["poses"][m, 1, 3:]).max() < 1e-9  # rotation frozen


def test_one_penetrating_contact_gives_the_same_step(oracle_lib):
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=16, n_contacts=32)
    H = O.Hand(hand)
    p = O.fk(H, q)
    rng = np.random.default_rng(4)
    used = 0
    for b in range(16):
        for _ in range(20):
            n = rng.normal(size=3)
            n /= np.linalg.norm(n)
            order = np.sort(p[b] @ n)
            if order[1] - order[0] >= 0.003:  # the next contact stays clear in every test (1 mm moves)
                break
        else:
            continue
        used += 1
        off = order[0] + 0.0002  # only the lowest contact lies below, by 0.2 mm
        ob = plane(O, n, off, Im=4e-4)
        a = O.step(H, ob, O.Params(projection=0), q[b:b + 1])
        g = O.step(H, ob, O.Params(projection=GS), q[b:b + 1])
        np.testing.assert_allclose(g["loss"], a["loss"], rtol=1e-13)
        # the leak moves the pose tangent after each sample in the sweep, so
        # only the value is order-free; the gradients differ by leak terms
        assert np.all(np.isfinite(g["grad"]))
    assert used >= 4


def sphere_obj(O):
    return O.Obj(kind=O.OBJ_SPHERE, center=(0.0, 0.0, 0.0), radius=0.04, inertia_over_mass=0.4 * 0.04 ** 2)


@pytest.mark.parametrize("K", [1, 2])
def test_gs_gradient_matches_finite_differences(oracle_lib, K):
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=10)
    H = O.Hand(hand)
    # h = 1e-7: at 1e-6 the grid's cell boundaries already bend the differences
    # of both projection forms by up to 1e-4 of the gradient
    for ob, h, rel in ((sphere_obj(O), 1e-7, 2e-6), (O.Obj(grid), 1e-7, 2e-6)):
        P = O.Params(projection=GS, alpha_leak=0.0, K=K)
        g = O.step(H, ob, P, q)["grad"]
        fd, ex = O.fd_grad(H, ob, P, q, h=h)
        assert ex.mean() < 0.6
        tol = rel * np.abs(g).max(axis=1, keepdims=True)
        bad = (np.abs(fd - g) > tol) & ~ex
        assert not bad.any(), np.argwhere(bad)[:5]


def test_gs_differs_from_the_averaged_form(oracle_lib):
    """With several penetrating contacts and a finite inertia the two forms
    give different losses (the sweep is not the averaged step)."""
    O = oracle_lib
    hand, grid, q = S.config_workload("tiny", B=8)
    H, ob = O.Hand(hand), O.Obj(grid)
    a = O.step(H, ob, O.Params(projection=0), q, grad=False)["loss"]
    g = O.step(H, ob, O.Params(projection=GS), q, grad=False)["loss"]
    assert np.abs(a - g).max() > 1e-3 * np.abs(a).max()
