"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs. Tolerances: relative 1e-5 on SDF samples and contact
positions, 1e-4 on losses, 1e-3 on gradients; exact on contact-to-link
indexing; rankings equal up to swaps inside near-tied groups. Every
candidate is checked: a sample within FP32 resolution of d = 0 or of a cell
face may take either reading (tests/parity_check.py), and a candidate is
only set aside (at most 1%) when it has more such samples than are
enumerated. Where the FP64 gradient itself moves by more than a quarter of
the tolerance under FP32-resolution changes of q (|v| near zero after
several projection iterations), the gradient tolerance is four times that
movement, capped at 1e-2, for a stated share of the candidates."""
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


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2306_08132_amd.api import Context
    c = Context(0, arena_bytes=1 << 30)
    yield c
    c.close()


def f32(x):
    """A parameter as the GPU receives it (FP32), widened for the oracle."""
    return float(np.float32(x)) if isinstance(x, float) else x


def prm_pair(**kw):
    """(GPU params, oracle params) holding the same FP32 values."""
    from paper_2306_08132_amd.api import StepParams
    sp = StepParams(**kw)
    op = O.Params()
    for k in vars(op):
        setattr(op, k, f32(getattr(sp, k)))
    return sp, op


@pytest.fixture(scope="module")
def tiny():
    hand, grid, q = S.config_workload("tiny")
    return hand, grid, q


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=DEV)


def ohand(hand):
    return O.Hand(hand.rounded())


@pytest.mark.parametrize("fj", [(3, 3, 512, 0), (4, 4, 1000, 1), (5, 4, 4096, 2), (2, 3, 70, 3)])
def test_contact_links_exact(ctx, fj):
    F, J, n, s = fj
    say("contact links", fj)
    hand = S.make_hand(F, J, n, seed=s)
    h = ctx.hand(hand)
    assert np.array_equal(h.contact_links(), hand.contact_link)


LAYOUTS = {"yzquads": 1, "zpairs": 2}


@pytest.mark.parametrize("layout", ["yzquads", "zpairs"])
@pytest.mark.parametrize("which", ["sphere64", "ellipsoids48", "mixed33"])
def test_sdf_sampler_parity(ctx, which, layout):
    say("sampler", which, layout)
    if which == "sphere64":
        g = S.make_grid(S.make_object("sphere", seed=0), 64)
    elif which == "ellipsoids48":
        g = S.make_grid(S.make_object("ellipsoids", seed=2), 48)
    else:
        g = S.make_grid(S.make_object("mixed", seed=3, n_prims=5), 33)
    sd = ctx.sdf(g, layout=LAYOUTS[layout])
    r = S.random_points(g, 20000, seed=7).astype(np.float32)
    out, H = ctx.debug_sdf_sample(sd, dev(r), hess=True)
    torch.cuda.synchronize()
    out, H = out.cpu().numpy().astype(np.float64), H.cpu().numpy().astype(np.float64).reshape(-1, 3, 3)
    phi, grad, Ho, margin = O.sample(O.Obj(g), r.astype(np.float64), hess=True)
    tol_phi = 1e-5 * np.maximum(np.abs(phi), g.h)
    assert np.all(np.abs(out[:, 0] - phi) <= tol_phi), np.max(np.abs(out[:, 0] - phi) / tol_phi)
    ok = margin > 1e-4  # away from cell faces and the box boundary
    gn = np.linalg.norm(grad, axis=1)
    err = np.abs(out[:, 1:] - grad).max(axis=1)
    assert np.all(err[ok] <= 1e-5 * np.maximum(gn[ok], 1.0)), np.max(err[ok])
    scale = np.maximum(np.abs(Ho).reshape(-1, 9).max(axis=1), 1.0 / g.h)
    herr = np.abs(H - Ho).reshape(-1, 9).max(axis=1)
    assert np.all(herr[ok] <= 1e-4 * scale[ok]), np.max(herr[ok] / scale[ok])
    say("  gradients not compared (within 1e-4 cell units of a face, where the gradient jumps):", (~ok).mean())
    assert (~ok).mean() <= 0.01
    assert inertia_close(ctx, sd, g)


def inertia_close(ctx, sd, g):
    return abs(sd.inertia_over_mass() - O.Obj(g).inertia_over_mass()) <= 1e-6 * O.Obj(g).inertia_over_mass()


def test_fk_and_trace_parity(ctx, tiny):
    hand, grid, q = tiny
    say("fk/trace tiny")
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    sp, op = prm_pair(r_dil=0.004)
    tr = ctx.debug_trace(h, sd, sp, dev(q[:16]))
    torch.cuda.synchronize()
    Hh, ob = ohand(hand), O.Obj(grid)
    q32 = q[:16].astype(np.float32).astype(np.float64)
    p_or = O.fk(Hh, q32)
    p = tr["p"].cpu().numpy()
    scale = np.maximum(np.abs(p_or).max(axis=(1, 2)), 0.01)
    assert np.all(np.abs(p - p_or).max(axis=(1, 2)) <= 1e-5 * scale)
    for b in range(4):
        t = O.trace(Hh, ob, op, q32[b])
        s_gpu = tr["samples"][b].cpu().numpy()
        d_gpu, d_or = s_gpu[..., 0], t["samples"][..., 0]
        assert np.all(np.abs(d_gpu - d_or) <= 1e-5 * np.maximum(np.abs(d_or), grid.h))
        # non-penetrating samples contribute exactly zero
        assert np.all(s_gpu[..., 5][d_gpu >= 0] == 0.0)
        # pose components are sums over contacts that can cancel: the tolerance
        # scales with the sum of the summands' magnitudes
        pg = tr["poses"][b].cpu().numpy()
        lam = np.abs(t["samples"][:, 0, :, 5])                      # [7][Nc]
        gn = np.linalg.norm(t["samples"][:, 0, :, 1:4], axis=-1)
        an = np.linalg.norm(p_or[b][None] - t["poses"][:, 0, None, :3], axis=-1)
        Im = ob.inertia_over_mass()
        lin = (lam * gn).sum(1)[:, None] + np.abs(t["poses"][:, 0, :3]).max()
        ang = (lam * gn * an).sum(1)[:, None] / Im
        err = np.abs(pg - t["poses"])[:, 1]
        assert np.all(err[:, :3] <= 1e-5 * lin + 1e-9) and np.all(err[:, 3:] <= 1e-5 * ang + 1e-9)


def compare_step(ctx, hand, grid, q, sp, op, label, layout=0, conditioning=False, max_set_aside=0.01):
    """Split forward and backward at q against the oracle (tests/parity_check:
    every candidate checked, ambiguous samples under either FP32 reading).
    conditioning: with several projection iterations rounding early in the
    trajectory can move later active sets; a candidate that misses is held
    to four times the movement of the FP64 loss and gradient under
    FP32-resolution changes of q (the gradient's capped at 1e-2), set aside
    only where that movement covers its error and exceeds the cap (at most
    max_set_aside of the candidates), and fails otherwise."""
    h, sd = ctx.hand(hand), ctx.sdf(grid, layout=layout)
    B = q.shape[0]
    qd = dev(q)
    loss = torch.empty(B, device=DEV)
    terms = torch.empty((B, 4), device=DEV)
    nb = ctx.workspace_bytes(h, sd, sp, B)
    ws = torch.empty(max(nb, 4), dtype=torch.uint8, device=DEV)
    ctx.step_fwd(h, sd, sp, qd, loss, terms, ws=ws)
    dq = torch.empty_like(qd)
    ctx.step_bwd(h, sd, sp, qd, dq, ws=ws)
    torch.cuda.synchronize()
    loss, terms, dq = loss.cpu().numpy(), terms.cpu().numpy(), dq.cpu().numpy()
    q32 = q.astype(np.float32).astype(np.float64)
    rep = P.compare(loss, dq, ohand(hand), O.Obj(grid), op, q32, conditioning=conditioning, label=label, say=say)
    P.assert_ok(rep, max_set_aside=max_set_aside)
    return loss, dq, rep["ref"]


def test_step_parity_tiny(ctx, tiny):
    hand, grid, q = tiny
    sp, op = prm_pair(r_dil=0.005)
    compare_step(ctx, hand, grid, q, sp, op, "tiny r=5mm")
    sp, op = prm_pair(r_dil=0.0, alpha_leak=0.0)
    compare_step(ctx, hand, grid, q, sp, op, "tiny exact")


def test_step_parity_ragged_and_small(ctx):
    """Contact counts off the 64-lane chunk size, one-link hand, tiny grid."""
    for F, J, n, N, B in [(3, 3, 65, 16, 5), (4, 4, 1000, 40, 9), (5, 4, 777, 33, 7)]:
        hand = S.make_hand(F, J, n, seed=F + n)
        grid = S.make_grid(S.make_object("ellipsoids", seed=n), N)
        q = S.make_candidates(hand, B, seed=n, shell_radius=grid.bound_radius + 0.06)
        sp, op = prm_pair(r_dil=0.003)
        compare_step(ctx, hand, grid, q, sp, op, f"ragged {F}x{J} Nc={n}")


def test_step_parity_iterations(ctx, tiny):
    """K > 1 projection iterations, with and without pose checkpoints."""
    hand, grid, q = tiny
    outs = []
    for K, ck in [(4, 1), (4, 2), (4, 4)]:
        sp, op = prm_pair(K=K, ckpt_every=ck, r_dil=0.004)
        loss, dq, _ = compare_step(ctx, hand, grid, q[:24], sp, op, f"K={K} ckpt={ck}", conditioning=True,
                                   max_set_aside=0.0)
        outs.append((loss, dq))
    for loss, dq in outs[1:]:
        assert np.array_equal(loss, outs[0][0]) and np.array_equal(dq, outs[0][1])


def test_save_recompute_and_fused_identical(ctx, tiny):
    from paper_2306_08132_amd.api import MODE_RECOMPUTE, MODE_SAVE
    hand, grid, q = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    B = 32
    res = {}
    for mode in (MODE_SAVE, MODE_RECOMPUTE):
        sp, _ = prm_pair(r_dil=0.004, mode=mode)
        qd = dev(q[:B])
        loss = torch.empty(B, device=DEV)
        ws = None
        if mode == MODE_SAVE:
            ws = torch.empty(ctx.workspace_bytes(h, sd, sp, B), dtype=torch.uint8, device=DEV)
        ctx.step_fwd(h, sd, sp, qd, loss, ws=ws)
        dq = torch.empty_like(qd)
        ctx.step_bwd(h, sd, sp, qd, dq, ws=ws)
        res[mode] = (loss.cpu().numpy(), dq.cpu().numpy())
    assert np.array_equal(res[MODE_SAVE][0], res[MODE_RECOMPUTE][0])
    assert np.array_equal(res[MODE_SAVE][1], res[MODE_RECOMPUTE][1])
    # fused forward + backward + Adam equals the separate calls bit for bit
    sp, _ = prm_pair(r_dil=0.004)
    qf = dev(q[:B])
    m = torch.zeros_like(qf)
    v = torch.zeros_like(qf)
    lf = torch.empty(B, device=DEV)
    dqf = torch.empty_like(qf)
    ctx.step_fused(h, sd, sp, qf, m, v, 1, loss=lf, dq=dqf)
    qs = dev(q[:B])
    ms, vs = torch.zeros_like(qs), torch.zeros_like(qs)
    g = torch.tensor(res[MODE_SAVE][1], device=DEV)
    ctx.adam(qs, ms, vs, g, 1)
    torch.cuda.synchronize()
    assert np.array_equal(lf.cpu().numpy(), res[MODE_SAVE][0])
    assert np.array_equal(dqf.cpu().numpy(), res[MODE_SAVE][1])
    assert torch.equal(qf, qs) and torch.equal(m, ms) and torch.equal(v, vs)


def test_adam_parity(ctx):
    q, m, v, g = S.adam_state(64, 22, seed=5)
    for t in (1, 7, 300):
        qd, md, vd, gd = (dev(a) for a in (q, m, v, g))
        ctx.adam(qd, md, vd, gd, t)
        torch.cuda.synchronize()
        r = O.adam(*(a.astype(np.float32).astype(np.float64) for a in (q, m, v, g)), t,
                   lr=f32(1e-3), b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
        for got, want in zip((qd, md, vd), r):
            np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-6, atol=1e-7)


def test_autograd_function(ctx, tiny):
    from paper_2306_08132_amd.api import GraspStep
    hand, grid, q = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    sp, op = prm_pair(r_dil=0.004)
    qd = dev(q[:8]).requires_grad_(True)
    w = torch.linspace(0.5, 2.0, 8, device=DEV)
    (GraspStep.apply(qd, ctx, h, sd, sp) * w).sum().backward()
    ref = O.step(ohand(hand), O.Obj(grid), op, q[:8].astype(np.float32).astype(np.float64))
    want = ref["grad"] * w.cpu().numpy()[:, None]
    err = np.abs(qd.grad.cpu().numpy() - want).max(axis=1) / np.abs(want).max(axis=1)
    assert np.all(err <= 1e-3)


def test_gradient_matches_finite_differences(ctx, tiny):
    """The GPU adjoint against FP64 central differences of the oracle loss
    (exact gradient, alpha = 0), outside kinks."""
    hand, grid, q = tiny
    sp, op = prm_pair(alpha_leak=0.0, r_dil=0.004)
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    B = 8
    qd = dev(q[:B])
    loss = torch.empty(B, device=DEV)
    dq = torch.empty_like(qd)
    ctx.step_fwd(h, sd, sp, qd, loss)
    ctx.step_bwd(h, sd, sp, qd, dq)
    torch.cuda.synchronize()
    fd, ex = O.fd_grad(ohand(hand), O.Obj(grid), op, q[:B].astype(np.float32).astype(np.float64), h=1e-6)
    g = dq.cpu().numpy()
    scale = np.abs(fd).max(axis=1, keepdims=True)
    bad = (np.abs(g - fd) > 1e-3 * scale) & ~ex
    say("fd excluded fraction", ex.mean())
    assert not bad.any()


def test_nonfinite_input_stays_in_bounds(ctx, tiny):
    """A NaN/Inf coordinate (wrist or finger) gives a NaN loss, never a bad access."""
    hand, grid, q = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    sp, _ = prm_pair()
    qq = q[:4].copy()
    qq[0, 0] = np.nan
    qq[1, 7] = np.inf
    qq[2, 3] = -np.inf
    loss = torch.empty(4, device=DEV)
    qd = dev(qq)
    ctx.step_fwd(h, sd, sp, qd, loss)
    dq = torch.empty_like(qd)
    ctx.step_bwd(h, sd, sp, qd, dq)
    torch.cuda.synchronize()
    l = loss.cpu().numpy()
    assert not np.isfinite(l[:3]).any() and np.isfinite(l[3])


def test_full_size_diff_sampled(ctx):
    """Full differentiable-step workload (4096 candidates, 2048 contacts,
    128^3): the fused launch as benchmarked, 48 sampled candidates against
    the oracle (every one checked, ambiguous samples under either reading)."""
    hand, grid, q = S.config_workload("diff")
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    sp, op = prm_pair(r_dil=0.005)
    B = q.shape[0]
    qd = dev(q)
    m, v = torch.zeros_like(qd), torch.zeros_like(qd)
    loss = torch.empty(B, device=DEV)
    dq = torch.empty_like(qd)
    ctx.step_fused(h, sd, sp, qd, m, v, 1, loss=loss, dq=dq)
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(B, 48, replace=False)
    rep = P.compare(loss.cpu().numpy()[idx], dq.cpu().numpy()[idx], ohand(hand), O.Obj(grid), op,
                    q[idx].astype(np.float32).astype(np.float64), label="diff full (48 sampled)", say=say)
    P.assert_ok(rep)


def test_every_tile_bit_identical(ctx, tiny):
    """Launch tiles change speed only: every tile gives the same bits."""
    hand, grid, q = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    res = []
    for K in (1, 2):
        sp, _ = prm_pair(r_dil=0.004, K=K)
        B = 40
        for wpb in (1, 2, 4):
            for occ in (1, 2, 3, 4, 5, 6):
                ctx.set_tile(h, sd, sp, B, wpb, occ)
                qd = dev(q[:B])
                m, v = torch.zeros_like(qd), torch.zeros_like(qd)
                loss = torch.empty(B, device=DEV)
                dq = torch.empty_like(qd)
                ctx.step_fused(h, sd, sp, qd, m, v, 1, loss=loss, dq=dq)
                res.append((K, loss.cpu().numpy(), dq.cpu().numpy(), qd.cpu().numpy()))
        (best, ms) = ctx.tune(h, sd, sp, dev(q[:B]), reps=1)
        say("K", K, "tuned tile", best, ms)
    for K in (1, 2):
        rk = [r for r in res if r[0] == K]
        for r in rk[1:]:
            assert all(np.array_equal(x, y) for x, y in zip(r[1:], rk[0][1:]))


def test_locality_order_changes_nothing(ctx, tiny):
    """Launches of at least 256 candidates run them in a locality order (by
    wrist direction, XCD-contiguous); the bits equal those of unordered
    launches of the same candidates in slices of 100."""
    hand, grid, _ = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    B = 600
    q = S.make_candidates(hand, B, seed=77, shell_radius=grid.bound_radius + 0.06)
    for K in (1, 2):
        sp, _ = prm_pair(r_dil=0.004, K=K)
        outs = []
        for sl in ((0, B),) + tuple((i, i + 100) for i in range(0, B, 100)):
            n = sl[1] - sl[0]
            qd = dev(q[sl[0]:sl[1]])
            m, v = torch.zeros_like(qd), torch.zeros_like(qd)
            loss = torch.empty(n, device=DEV)
            dq = torch.empty_like(qd)
            ctx.step_fused(h, sd, sp, qd, m, v, 1, loss=loss, dq=dq)
            outs.append((loss.cpu().numpy(), dq.cpu().numpy(), qd.cpu().numpy()))
        whole = outs[0]
        parts = [np.concatenate([o[k] for o in outs[1:]]) for k in range(3)]
        say("K", K, "ordered vs sliced max |diff| loss", float(np.nanmax(np.abs(whole[0] - parts[0]))))
        assert all(np.array_equal(a, b) for a, b in zip(whole, parts))


def test_gather_layouts_bit_identical(ctx, tiny):
    """yz-quads and z-pairs hold the same corner values: every step
    (K = 1 and K = 2, fused and split) and every sample agree bit for bit;
    the yz-quad path also meets the oracle on its own."""
    hand, grid, q = tiny
    h = ctx.hand(hand)
    sds = {name: ctx.sdf(grid, layout=code) for name, code in LAYOUTS.items()}
    r = dev(S.random_points(grid, 4096, seed=9).astype(np.float32))
    samples = {name: ctx.debug_sdf_sample(sd, r, hess=True) for name, sd in sds.items()}
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(samples["yzquads"], samples["zpairs"]))
    for K in (1, 2):
        sp, _ = prm_pair(r_dil=0.004, K=K)
        outs = {}
        for name, sd in sds.items():
            qd = dev(q)
            m, v = torch.zeros_like(qd), torch.zeros_like(qd)
            loss = torch.empty(q.shape[0], device=DEV)
            dq = torch.empty_like(qd)
            ctx.step_fused(h, sd, sp, qd, m, v, 1, loss=loss, dq=dq)
            outs[name] = (loss.cpu().numpy(), dq.cpu().numpy(), qd.cpu().numpy())
        say("layouts K", K, "max |loss diff|", float(np.abs(outs["yzquads"][0] - outs["zpairs"][0]).max()))
        assert all(np.array_equal(a, b) for a, b in zip(outs["yzquads"], outs["zpairs"]))
    sp, op = prm_pair(r_dil=0.005)
    compare_step(ctx, hand, grid, q, sp, op, "tiny r=5mm, yz-quads", layout=LAYOUTS["yzquads"])


def test_plain_form_parity(ctx, tiny):
    """The unfused per-job form against the oracle, and against the fused
    step (same formulas, different summation order)."""
    hand, grid, q = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    sp, op = prm_pair(r_dil=0.005)
    B = q.shape[0]
    ws = ctx.plain_workspace(h, sd, sp, B)
    qp = dev(q)
    m, v = torch.zeros_like(qp), torch.zeros_like(qp)
    loss = torch.empty(B, device=DEV)
    ctx.plain_step(h, sd, sp, qp, m, v, 1, ws, loss=loss)
    qf = dev(q)
    mf, vf = torch.zeros_like(qf), torch.zeros_like(qf)
    lf = torch.empty(B, device=DEV)
    dqf = torch.empty_like(qf)
    ctx.step_fused(h, sd, sp, qf, mf, vf, 1, loss=lf, dq=dqf)
    torch.cuda.synchronize()
    lp = loss.cpu().numpy()
    # m after one step is (1 - b1) dq: the plain gradient against the oracle
    dq_plain = m.cpu().numpy() / np.float32(1 - np.float32(0.9))
    rep = P.compare(lp, dq_plain, ohand(hand), O.Obj(grid), op, q.astype(np.float32).astype(np.float64),
                    label="plain form", say=say)
    P.assert_ok(rep)
    # Adam's first step is -lr sign(g): the update direction where |g| is not tiny
    g = rep["ref"]["grad"]
    big = np.abs(g) > 1e-3 * np.abs(g).max(axis=1, keepdims=True)
    upd = (qp.cpu().numpy() - q.astype(np.float32))
    ok = big & (rep["status"] == 0)[:, None]
    assert np.all(np.sign(upd[ok]) == -np.sign(g[ok]))
    assert np.allclose(lp, lf.cpu().numpy(), rtol=1e-5, atol=1e-6)


def _fused(ctx, h, sd, sp, q, stream=None):
    qd = dev(q)
    m, v = torch.zeros_like(qd), torch.zeros_like(qd)
    loss = torch.empty(q.shape[0], device=DEV)
    dq = torch.empty_like(qd)
    ctx.step_fused(h, sd, sp, qd, m, v, 1, loss=loss, dq=dq, stream=stream)
    return qd, m, v, loss, dq


def test_two_streams_share_the_order_buffer(ctx, tiny):
    """Ordered launches from two streams at once (they share the context's
    order buffer, each waiting on the device for the other) give the bits of
    the same launches run one after another."""
    hand, grid, _ = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    sp, _ = prm_pair(r_dil=0.004)
    qa = S.make_candidates(hand, 700, seed=81, shell_radius=grid.bound_radius + 0.06)
    qb = S.make_candidates(hand, 900, seed=82, shell_radius=grid.bound_radius + 0.06)
    ref = [_fused(ctx, h, sd, sp, q) for q in (qa, qb)]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for rep in range(3):
        o1 = _fused(ctx, h, sd, sp, qa, stream=s1)
        o2 = _fused(ctx, h, sd, sp, qb, stream=s2)
        torch.cuda.synchronize()
        outs.append((o1, o2))
    for o1, o2 in outs:
        assert all(torch.equal(a, b) for a, b in zip(o1, ref[0]))
        assert all(torch.equal(a, b) for a, b in zip(o2, ref[1]))


def test_step_captured_in_a_graph(ctx, tiny):
    """A fused step captured into a HIP graph (the order kernel stays out of
    captures) and replayed several times, with eager work in between, matches
    eager steps bit for bit on every replay."""
    hand, grid, _ = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    sp, _ = prm_pair(r_dil=0.004)
    q0 = S.make_candidates(hand, 400, seed=83, shell_radius=grid.bound_radius + 0.06)
    # eager reference: three consecutive steps
    qe = dev(q0)
    me, ve = torch.zeros_like(qe), torch.zeros_like(qe)
    le = torch.empty(q0.shape[0], device=DEV)
    ref = []
    for t in range(3):
        ctx.step_fused(h, sd, sp, qe, me, ve, t + 1, loss=le)
        torch.cuda.synchronize()
        ref.append((qe.clone(), le.clone()))
    # graph: capture one step at t = 1 on fresh state, replay it as steps 1..3
    # (the Adam step index is baked into the capture, so compare step 1 of each
    # replay from the same starting state)
    qg = dev(q0)
    mg, vg = torch.zeros_like(qg), torch.zeros_like(qg)
    lg = torch.empty(q0.shape[0], device=DEV)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        ctx.step_fused(h, sd, sp, qg, mg, vg, 1, loss=lg, stream=s)
    for rep in range(3):
        qg.copy_(dev(q0)); mg.zero_(); vg.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (qg * 2).sum().item()  # eager work between replays
        assert torch.equal(qg, ref[0][0]) and torch.equal(lg, ref[0][1]), rep


@pytest.mark.parametrize("case", ["k1", "k1-wide-tests", "k1-outside", "k3", "k3-outside"])
@pytest.mark.parametrize("layout", ["yzquads", "zpairs"])
def test_culled_forward_matches_full_pass(ctx, tiny, case, layout):
    """The untraced forward pass skips groups of samples whose block bound
    proves them clear of the surface; the traced pass evaluates every sample.
    Pose trajectories and active-constraint counts agree bit for bit, the
    penetration energy agrees with the traced samples, and some groups are
    skipped. Cases: one bound per contact (K = 1, dv below the cell size),
    per-sample bounds (dv above it, and K > 1 with rotating tests), and hands
    partly outside the grid box (distance term of the bound)."""
    hand, grid, q = tiny
    q = np.array(q[:48], dtype=np.float64)
    if case.endswith("outside"):
        q[:, 0] += 0.05  # wrist 5 cm along x: part of the hand leaves the 12 cm box
    K = 3 if case.startswith("k3") else 1
    dt = 2.5e-3 if case == "k1-wide-tests" else 1e-3  # dv = dt v0 above / below the 1.9 mm cell
    assert (dt > grid.h) == (case == "k1-wide-tests")
    say("culled vs full", case, layout)
    h, sd = ctx.hand(hand), ctx.sdf(grid, layout=LAYOUTS[layout])
    sp, _ = prm_pair(r_dil=0.006, K=K, ckpt_every=1, dt=dt)
    qd = dev(q)
    B = q.shape[0]
    ws = torch.zeros(ctx.workspace_bytes(h, sd, sp, B) // 4, dtype=torch.float32, device=DEV)
    loss = torch.empty(B, device=DEV)
    terms = torch.empty((B, 4), device=DEV)
    ctx.step_fwd(h, sd, sp, qd, loss, terms=terms, ws=ws)
    tr = ctx.debug_trace(h, sd, sp, qd, p_world=False)
    live, total = ctx.debug_forward_groups(h, sd, sp, qd)
    torch.cuda.synchronize()
    npose = B * 7 * (K + 1) * 6
    poses = ws[:npose].view(B, K + 1, 7, 6).transpose(1, 2)  # checkpoints are slot-major per candidate
    assert torch.equal(poses, tr["poses"]), float((poses - tr["poses"]).abs().max())
    counts = ws[npose:npose + B * K * 7].view(B, K, 7).cpu().numpy()
    sm = tr["samples"].cpu().numpy()  # [B][7][K][Nc][6]: d, g, w, lambda
    assert np.array_equal(counts, (sm[..., 5] != 0).sum(axis=-1).transpose(0, 2, 1))
    d0 = sm[:, 6, 0, :, 0].astype(np.float64)
    lpen = 0.5 * np.where(d0 < 0, d0 * d0, 0.0).sum(axis=1)
    got = terms[:, 1].cpu().numpy().astype(np.float64)
    assert np.allclose(got, lpen, rtol=1e-5, atol=1e-12), np.abs(got - lpen).max()
    passes = K  # forward passes of a fused step with a checkpoint every iteration
    assert total == B * passes * -(-hand.n_contacts // 9)
    say("  live groups", live, "of", total)
    assert 0 < live < total


def test_stored_oracle_values(ctx, tiny):
    """The HIP path against the oracle values stored under tests/golden (written
    by make_oracle_tiny.py), with no oracle run: loss within 1e-4, gradient
    within 1e-3 of its largest component, for one and three iterations."""
    from test_golden import load_oracle_tiny
    hand, grid, _ = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    for K, r_dil, rows in load_oracle_tiny():
        sp, _ = prm_pair(r_dil=r_dil, K=K)
        q = np.stack([r[1] for r in rows])
        B = q.shape[0]
        qd = dev(q)
        loss = torch.empty(B, device=DEV)
        terms = torch.empty((B, 4), device=DEV)
        ws = torch.empty(max(ctx.workspace_bytes(h, sd, sp, B), 4), dtype=torch.uint8, device=DEV)
        ctx.step_fwd(h, sd, sp, qd, loss, terms, ws=ws)
        dq = torch.empty_like(qd)
        ctx.step_bwd(h, sd, sp, qd, dq, ws=ws)
        torch.cuda.synchronize()
        loss, dq = loss.cpu().numpy().astype(np.float64), dq.cpu().numpy().astype(np.float64)
        want_loss = np.array([r[2] for r in rows])
        want_grad = np.stack([r[4] for r in rows])
        lerr = np.abs(loss - want_loss) / np.maximum(np.abs(want_loss), sp.w_stable * sp.v0)
        gerr = np.abs(dq - want_grad).max(axis=1) / np.abs(want_grad).max(axis=1)
        say(f"stored oracle values K={K}: B={B} loss rel err {lerr.max():.2e}, grad rel err {gerr.max():.2e}")
        assert np.all(lerr <= 1e-4), lerr
        assert np.all(gerr <= 1e-3), gerr


def test_trajectory_teacher_forced(ctx, tiny):
    """100 fused steps on the small workload (64 candidates, 512 contacts,
    64^3 grid) along the dilation schedule from 1 cm, every step checked from
    the GPU's own state: loss and gradient of every candidate against the
    oracle at that q (samples within FP32 resolution of d = 0 or of a cell
    face under either reading), and the Adam update against the oracle's Adam
    fed the GPU's gradient and moments (1e-6 relative to the operands'
    magnitudes). The free-running trajectories (each side on its own state,
    final loss at zero dilation) are reported, not asserted: FP32 and FP64
    states drift apart over many steps."""
    from paper_2306_08132_amd.api import StepParams
    hand, grid, q0 = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    H, ob = ohand(hand), O.Obj(grid)
    B, T, r0 = q0.shape[0], 100, 0.01
    qd = dev(q0)
    m, v = torch.zeros_like(qd), torch.zeros_like(qd)
    loss = torch.empty(B, device=DEV)
    dq = torch.empty_like(qd)
    worst_l = worst_g = 0.0
    resolved, set_aside = [], []
    for t in range(T):
        r = float(np.float32(r0)) * (1.0 - min(t, T - 1) / (T - 1))
        sp, op = prm_pair(r_dil=r)
        q_prev, m_prev, v_prev = (x.cpu().numpy().astype(np.float64) for x in (qd, m, v))
        ctx.step_fused(h, sd, sp, qd, m, v, t + 1, loss=loss, dq=dq)
        torch.cuda.synchronize()
        lg, gg = loss.cpu().numpy(), dq.cpu().numpy()
        rep = P.compare(lg, gg, H, ob, op, q_prev, conditioning=True, label=f"step {t}", say=lambda *a: None)
        P.assert_ok(rep, max_set_aside=2.0 / B)
        if rep["resolved"] or rep["conditioned"] or rep["set_aside"]:
            say(f"  step {t}: resolved {rep['resolved']}, within conditioning {rep['conditioned']} "
                f"(largest {rep['max_cond']:.1e}), set aside {rep['set_aside']}")
        resolved.append(rep["resolved"] / B)
        set_aside.append(rep["set_aside"] / B)
        worst_l = max(worst_l, rep["max_lerr"])
        worst_g = max(worst_g, rep["max_gerr"])
        lr, b1, b2, eps = f32(1e-3), f32(0.9), f32(0.999), f32(1e-8)
        g64 = gg.astype(np.float64)
        qa, ma, va = O.adam(q_prev, m_prev, v_prev, g64, t + 1, lr=lr, b1=b1, b2=b2, eps=eps)
        # 1e-6 relative to the operands: b1 m and (1 - b1) g may cancel, and
        # the rounding of m carries through the bias correction into q
        sm = b1 * np.abs(m_prev) + (1.0 - b1) * np.abs(g64)
        sv = b2 * v_prev + (1.0 - b2) * g64 * g64
        vhat = va / (1.0 - b2 ** (t + 1))
        sq = np.abs(q_prev) + lr * (sm / (1.0 - b1 ** (t + 1))) / (np.sqrt(vhat) + eps)
        for name, got, want, scale in (("q", qd, qa, sq), ("m", m, ma, sm), ("v", v, va, sv)):
            err = np.abs(got.cpu().numpy() - want)
            assert np.all(err <= 1e-6 * scale + 1e-7), (t, name, np.argmax(err - 1e-6 * scale), err.max())
    say(f"trajectory: {T} steps, B={B}: worst loss rel err {worst_l:.2e}, worst grad rel err {worst_g:.2e}; "
        f"candidates resolved by an FP32 reading: mean {np.mean(resolved):.4f} max {np.max(resolved):.4f}; "
        f"set aside: mean {np.mean(set_aside):.4f} max {np.max(set_aside):.4f}")
    assert np.mean(set_aside) <= 0.01
    # free running: the GPU's final loss at zero dilation against the oracle's own optimisation
    fin = torch.empty(B, device=DEV)
    ctx.step_fwd(h, sd, StepParams(r_dil=0.0), qd, fin)
    torch.cuda.synchronize()
    _, op0 = prm_pair()
    own = O.optimize(H, ob, op0, q0.astype(np.float32).astype(np.float64), T=T, r0=f32(r0), lr=f32(1e-3),
                     b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
    rel = np.abs(fin.cpu().numpy() - own["loss"]) / np.maximum(np.abs(own["loss"]), op0.w_stable * op0.v0)
    say(f"trajectory free-running: final loss rel diff median {np.median(rel):.2e}, max {rel.max():.2e}; "
        f"median final loss GPU {np.median(fin.cpu().numpy()):.4f}, oracle {np.median(own['loss']):.4f}")


def test_auto_mode_recomputes_when_the_workspace_exceeds_the_budget(ctx, tiny):
    """GraspStep in AUTO mode keeps pose checkpoints only when the workspace
    fits its budget; with a budget of 0 bytes the backward recomputes FK and
    the samples, and the gradient is bit-identical to SAVE's."""
    from paper_2306_08132_amd.api import MODE_AUTO, MODE_SAVE, GraspStep, StepParams
    hand, grid, q = tiny
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    grads = {}
    for name, mode, budget in (("save", MODE_SAVE, None), ("auto-fits", MODE_AUTO, 1 << 30),
                               ("auto-recompute", MODE_AUTO, 0)):
        sp = StepParams(r_dil=0.004, K=4, ckpt_every=2, mode=mode)
        qd = dev(q[:32]).requires_grad_(True)
        GraspStep.apply(qd, ctx, h, sd, sp, budget).sum().backward()
        torch.cuda.synchronize()
        grads[name] = qd.grad.cpu().numpy()
    assert ctx.workspace_bytes(h, sd, StepParams(K=4, ckpt_every=2), 32) > 0
    assert np.array_equal(grads["save"], grads["auto-fits"])
    assert np.array_equal(grads["save"], grads["auto-recompute"])


@pytest.mark.parametrize("which", ["tiny", "diff"])
def test_ranking_matches_oracle(ctx, which):
    """Candidates ranked by the GPU's loss at zero dilation (the served form's
    final ranking: stable sort of the FP32 losses) against the oracle's
    stable sort of its FP64 losses at the same q: the same permutation up to
    swaps inside groups of near-tied losses (|dL| <= 2e-4 max |L|)."""
    from paper_2306_08132_amd.api import StepParams
    if which == "tiny":
        hand, grid, q = S.config_workload("tiny")
        idx = np.arange(q.shape[0])
    else:
        hand, grid, q = S.config_workload("diff")
        idx = np.random.default_rng(4).choice(q.shape[0], 96, replace=False)
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    qs = q[idx]
    loss = torch.empty(len(idx), device=DEV)
    ctx.step_fwd(h, sd, StepParams(r_dil=0.0), dev(qs), loss)
    torch.cuda.synchronize()
    lg = loss.cpu().numpy()
    rank_gpu = np.argsort(lg, kind="stable")
    _, op = prm_pair(r_dil=0.0)
    ref = O.step(ohand(hand), O.Obj(grid), op, qs.astype(np.float32).astype(np.float64), grad=False)
    P.assert_rank_matches(rank_gpu, ref["loss"], label=f"ranking {which}", say=say)
