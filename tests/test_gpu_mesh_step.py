"""GPU parity of the grasp step on a mesh object (Sec. III-B's Phong signed
distance inside Sec. III-C's constraint; `grasp_step_fused_mesh`) against the
FP64 oracle's step on the same mesh: loss and gradient of every candidate
(tests/parity_check.py), one and three projection iterations, with and without
dilation and leak. The kernel queries the mesh's hierarchy at every sample and
differentiates through the closest point (face interior, edge or vertex) and
the Phong point by hand; the oracle takes the same quantities with dual
numbers. A sample within FP32 resolution of the flat surface may take either
sign (reported by the oracle and tried both ways); the closest feature can
also tie at FP32 resolution (a gradient-only difference), which the
conditioning measure covers with several iterations."""
import numpy as np
import pytest
import torch

import oracle as O
import parity_check as P
from paper_2306_08132_amd import synth as S

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2306_08132_amd.api import Context
    c = Context(0, arena_bytes=1 << 30)
    yield c
    c.close()


def prm_pair(**kw):
    from paper_2306_08132_amd.api import StepParams
    sp = StepParams(**kw)
    op = O.Params()
    for k in vars(op):
        v = getattr(sp, k)
        setattr(op, k, float(np.float32(v)) if isinstance(v, float) else v)
    return sp, op


def mesh_pair(ctx, m, alpha, Im):
    """The mesh on the device and the oracle's view of the FP32 values the
    device holds."""
    mf = S.TriMesh(f32(m.vertices), m.faces, f32(m.normals))
    dm = ctx.mesh(mf, float(np.float32(alpha)))
    M = O.Mesh(mf.vertices, mf.faces, mf.normals, float(np.float32(alpha)))
    return dm, M, O.Obj(mesh=M, inertia_over_mass=float(np.float32(Im)))


def gpu_step(ctx, h, dm, sp, Im, q):
    qd = torch.tensor(q, dtype=torch.float32, device=DEV)
    m, v = torch.zeros_like(qd), torch.zeros_like(qd)
    loss = torch.empty(q.shape[0], device=DEV)
    dq = torch.empty_like(qd)
    ctx.step_fused_mesh(h, dm, sp, qd, m, v, 1, inertia_over_mass=float(np.float32(Im)), loss=loss, dq=dq)
    torch.cuda.synchronize()
    return loss.cpu().numpy(), dq.cpu().numpy(), qd


@pytest.mark.parametrize("K", [1, 3])
def test_mesh_step_parity_tiny(ctx, K):
    hand, _, q = S.config_workload("tiny")
    Im = 0.4 * 0.04 ** 2
    m = S.mesh_ellipsoid((0.045, 0.035, 0.04), subdivisions=2)
    dm, _, ob = mesh_pair(ctx, m, 0.75, Im)
    h = ctx.hand(hand)
    H = O.Hand(hand.rounded())
    q32 = f32(q)
    for kw in (dict(r_dil=0.005), dict(r_dil=0.0, alpha_leak=0.0)):
        sp, op = prm_pair(K=K, **kw)
        loss, dq, _ = gpu_step(ctx, h, dm, sp, Im, q)
        rep = P.compare(loss, dq, H, ob, op, q32, conditioning=True, max_units=8, label=f"mesh K={K} {kw}",
                        say=say)
        P.assert_ok(rep, max_set_aside=0.0)
    h.destroy()
    dm.unload()


def test_mesh_step_parity_ragged_box(ctx):
    """Ragged contact counts on a box mesh (flat faces, sharp edges and
    corners: every region kind), flat (alpha = 0) and curved (alpha = 1)."""
    box = S.mesh_box((0.03, 0.025, 0.035), splits=2)
    Im = 0.4 * 0.03 ** 2
    for F, J, n, B in [(3, 3, 65, 6), (4, 4, 1000, 8)]:
        hand = S.make_hand(F, J, n, seed=F + n)
        q = S.make_candidates(hand, B, seed=n, shell_radius=0.045 + 0.06)
        h = ctx.hand(hand)
        H = O.Hand(hand.rounded())
        for alpha in (0.0, 1.0):
            dm, _, ob = mesh_pair(ctx, box, alpha, Im)
            sp, op = prm_pair(r_dil=0.01)
            loss, dq, _ = gpu_step(ctx, h, dm, sp, Im, q)
            rep = P.compare(loss, dq, H, ob, op, f32(q), conditioning=True, max_units=8,
                            label=f"mesh box alpha={alpha} {F}x{J} Nc={n}", say=say)
            P.assert_ok(rep, max_set_aside=0.0)
            dm.unload()
        h.destroy()


def test_mesh_step_adam_and_refusals(ctx):
    """The fused mesh step's Adam update is the oracle's Adam on the step's
    own gradient; Gauss-Seidel, friction and a non-finite I/m are refused."""
    from paper_2306_08132_amd._lib import GraspError
    from paper_2306_08132_amd.api import StepParams
    hand, _, q = S.config_workload("tiny", B=16)
    Im = 0.4 * 0.04 ** 2
    m = S.mesh_ellipsoid((0.045, 0.035, 0.04), subdivisions=2)
    dm, _, _ = mesh_pair(ctx, m, 0.75, Im)
    h = ctx.hand(hand)
    sp = StepParams(r_dil=0.005)
    loss, dq, qd = gpu_step(ctx, h, dm, sp, Im, q)
    lr, b1, b2, eps = (float(np.float32(x)) for x in (1e-3, 0.9, 0.999, 1e-8))
    qa, _, _ = O.adam(f32(q), np.zeros_like(q), np.zeros_like(q), dq.astype(np.float64), 1, lr=lr, b1=b1, b2=b2,
                      eps=eps)
    np.testing.assert_allclose(qd.cpu().numpy(), qa, rtol=0, atol=1e-6 * (np.abs(qa).max() + lr))
    qt = torch.tensor(q, dtype=torch.float32, device=DEV)
    z = torch.zeros_like(qt)
    for bad, kw in ((StepParams(projection=1), {}), (StepParams(mu=0.5), {}),
                    (StepParams(), {"inertia_over_mass": float("nan")})):
        with pytest.raises(GraspError):
            ctx.step_fused_mesh(h, dm, bad, qt, z, z.clone(), 1, **kw)
    h.destroy()
    dm.unload()


def test_mesh_step_sample_exact_gradient(ctx):
    """The sample the mesh step takes (grasp_debug_mesh_step_sample): rho and
    the stated normal against the oracle's mesh query, and the exact gradient
    of rho (through the closest point and the Phong point) against central
    differences of the oracle's rho, near the surface of a Phong ellipsoid
    (alpha = 0.75) where the closest feature is well determined (the oracle's
    medial gap above 1e-4 m, flat distance below 1 cm)."""
    m = S.mesh_ellipsoid((0.045, 0.035, 0.04), subdivisions=2)
    dm, M, _ = mesh_pair(ctx, m, 0.75, 1e-3)
    rng = np.random.default_rng(2)
    d = rng.normal(size=(4000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = f32(d * np.array([0.045, 0.035, 0.04]) * rng.uniform(0.8, 1.2, size=(4000, 1)))
    out = dm.step_sample(torch.tensor(r, dtype=torch.float32, device=DEV)).cpu().numpy().astype(np.float64)
    ref = O.mesh_sdf(M, r)
    ok = (ref["gap"] > 1e-4) & (ref["dist_flat"] < 1e-2) & (ref["dist_flat"] > 1e-5)
    assert ok.mean() > 0.5
    np.testing.assert_allclose(out[ok, 0], ref["rho"][ok], rtol=0, atol=2e-6)
    np.testing.assert_allclose(out[ok, 1:4], ref["grad"][ok], rtol=0, atol=2e-4)
    h = 1e-7
    fd = np.stack([(O.mesh_sdf(M, r + h * u)["rho"] - O.mesh_sdf(M, r - h * u)["rho"]) / (2 * h) for u in np.eye(3)],
                  axis=1)
    err = np.abs(out[:, 4:7] - fd).max(axis=1)
    say(f"exact gradient of rho: {int(ok.sum())} points, max err {err[ok].max():.2e}, "
        f"regions {np.bincount(out[ok, 7].astype(int), minlength=3)}")
    assert np.all(err[ok] < 2e-3)
    # it differs from the stated normal where alpha moves the Phong point with r
    assert np.abs(out[ok, 4:7] - out[ok, 1:4]).max() > 1e-2
    dm.unload()


def test_face_cache_is_the_walk(ctx):
    """The one-iteration mesh step records each sample's nearest face in the
    forward and the adjoint reuses it; captured into a graph it walks the
    hierarchy again instead (a later step may move the context's buffer).
    Both give the same bits: the same face at the same point. Replayed twice
    with eager work in between."""
    from paper_2306_08132_amd.api import StepParams
    hand, _, q = S.config_workload("tiny")
    Im = float(np.float32(0.4 * 0.04 ** 2))
    dm, _, _ = mesh_pair(ctx, S.mesh_ellipsoid((0.045, 0.035, 0.04), subdivisions=2), 0.75, Im)
    h = ctx.hand(hand)
    sp = StepParams(r_dil=0.005)
    qa = torch.tensor(q, dtype=torch.float32, device=DEV)
    la, ga = torch.empty(q.shape[0], device=DEV), torch.empty_like(qa)
    ctx.step_fused_mesh(h, dm, sp, qa, torch.zeros_like(qa), torch.zeros_like(qa), 1, inertia_over_mass=Im,
                        loss=la, dq=ga)
    torch.cuda.synchronize()
    qb = torch.tensor(q, dtype=torch.float32, device=DEV)
    mb, vb = torch.zeros_like(qb), torch.zeros_like(qb)
    lb, gb = torch.empty_like(la), torch.empty_like(ga)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.step_fused_mesh(h, dm, sp, qb, mb, vb, 1, inertia_over_mass=Im, loss=lb, dq=gb, stream=s)
    q0 = torch.tensor(q, dtype=torch.float32, device=DEV)
    for _ in range(2):
        qb.copy_(q0)
        mb.zero_()
        vb.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (qb * 2).sum().item()
        assert torch.equal(la, lb) and torch.equal(ga, gb) and torch.equal(qa, qb)
    h.destroy()
    dm.unload()
