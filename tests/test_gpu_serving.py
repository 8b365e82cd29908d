"""GPU: the serving loop. A job's results are the same alone and in a mix
of overlapping jobs (bit-exact), cancelled and non-finite jobs end without
disturbing the others, jobs that can never fit are refused, a job with an
evaluation set retires with its metrics and top 10, and a Gauss-Seidel job
equals its fused steps launched directly."""
import time

import numpy as np
import pytest
import torch

from paper_2306_08132_amd import synth as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup(gpu):
    from paper_2306_08132_amd.api import Context
    ctx = Context(0, arena_bytes=512 << 20)
    ctx.serve_config(capacity=4096, max_jobs=16)
    objs = []
    for k, (F, J, nc, N, B) in enumerate([(3, 3, 256, 24, 40), (4, 4, 512, 32, 64), (5, 4, 700, 28, 24)]):
        hand = S.make_hand(F, J, nc, seed=40 + k)
        grid = S.make_grid(S.make_object("ellipsoids", seed=50 + k, n_range=(2, 3)), N)
        q = S.make_candidates(hand, B, seed=60 + k, shell_radius=grid.bound_radius + 0.06).astype(np.float32)
        objs.append((ctx.hand(hand), ctx.sdf(grid), q))
    yield ctx, objs
    ctx.close()


def wait(ctx, jid, B, nd, timeout=120.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        r = ctx.poll(jid, B, nd)
        if r is not None:
            return r
        time.sleep(0.005)
    raise TimeoutError(f"job {jid} did not finish")


def test_alone_equals_in_mix(setup):
    ctx, objs = setup
    h, sd, q = objs[1]
    say("serving: job alone")
    a = ctx.submit(h, sd, q, T=8)
    alone = wait(ctx, a, q.shape[0], h.n_dof)
    assert alone["status"] == 0 and alone["steps"] == 8
    say("serving: job in a mix of overlapping jobs")
    ids = []
    ids.append((ctx.submit(objs[0][0], objs[0][1], objs[0][2], T=12), objs[0]))
    time.sleep(0.01)
    mid = ctx.submit(h, sd, q, T=8)
    time.sleep(0.005)
    ids.append((ctx.submit(objs[2][0], objs[2][1], objs[2][2], T=5), objs[2]))
    mixed = wait(ctx, mid, q.shape[0], h.n_dof)
    for jid, (hh, _, qq) in ids:
        assert wait(ctx, jid, qq.shape[0], hh.n_dof)["status"] == 0
    for k in ("q", "loss", "terms", "rank"):
        assert np.array_equal(alone[k], mixed[k]), k
    assert mixed["t_submit"] <= mixed["t_admit"] <= mixed["t_done"]
    # ranking: stable sort of the final losses
    assert mixed["rank"].tolist() == np.argsort(mixed["loss"], kind="stable").tolist()


def test_final_loss_is_forward_at_zero_dilation(setup):
    from paper_2306_08132_amd.api import StepParams
    ctx, objs = setup
    h, sd, q = objs[0]
    r = wait(ctx, ctx.submit(h, sd, q, T=3), q.shape[0], h.n_dof)
    qd = torch.tensor(r["q"], device="cuda:0")
    loss = torch.empty(q.shape[0], device="cuda:0")
    ctx.step_fwd(h, sd, StepParams(r_dil=0.0), qd, loss)
    torch.cuda.synchronize()
    assert np.array_equal(loss.cpu().numpy(), r["loss"])


def test_cancel_and_nonfinite_leave_others_intact(setup):
    ctx, objs = setup
    h0, sd0, q0 = objs[0]
    h2, sd2, q2 = objs[2]
    ref = wait(ctx, ctx.submit(h2, sd2, q2, T=6), q2.shape[0], h2.n_dof)
    bad = q0.copy()
    bad[3, 0] = np.nan
    j_bad = ctx.submit(h0, sd0, bad, T=20)
    j_long = ctx.submit(h0, sd0, q0, T=10000)
    j_ok = ctx.submit(h2, sd2, q2, T=6)
    time.sleep(0.05)
    ctx.cancel(j_long)
    rb = wait(ctx, j_bad, q0.shape[0], h0.n_dof)
    rl = wait(ctx, j_long, q0.shape[0], h0.n_dof)
    ro = wait(ctx, j_ok, q2.shape[0], h2.n_dof)
    same = np.array_equal(ro["q"], ref["q"])
    say("statuses", rb["status"], rb["steps"], rl["status"], rl["steps"], ro["status"], ro["steps"], "same", same,
        "max diff", float(np.abs(ro["q"] - ref["q"]).max()))
    assert rb["status"] == -6 and rb["steps"] == 1
    assert rl["status"] == -7
    assert ro["status"] == 0 and same


def test_refusals(setup):
    from paper_2306_08132_amd.api import GraspError
    ctx, objs = setup
    h, sd, q = objs[0]
    big = np.zeros((5000, h.n_dof), np.float32)  # more than the 4096-candidate capacity
    with pytest.raises(GraspError):
        ctx.submit(h, sd, big, T=2)
    with pytest.raises(GraspError):
        ctx.poll(123456789, 1, h.n_dof)
    st = ctx.serve_stats()
    assert st["steps"] > 0 and st["contact_evals"] > 0


def test_job_with_evaluation(setup):
    """A job that names an evaluation set retires with the metrics of every
    candidate at its final configuration and the top 10 by final loss: the
    same bits as evaluating and selecting on the job's returned q and loss."""
    from paper_2306_08132_amd._lib import GraspError
    ctx, _ = setup
    dev = "cuda:0"
    hand = S.make_hand(3, 3, 256, seed=70)
    grid = S.make_grid(S.make_object("ellipsoids", seed=71, n_range=(2, 3)), 32)
    q = S.make_candidates(hand, 48, seed=72, shell_radius=grid.bound_radius + 0.04).astype(np.float32)
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    ev = ctx.eval_points(h, S.make_eval_points(hand, 700, 500, seed=73))
    thr = [0.002, 0.005, 0.009]
    say("serving: job with evaluation")
    jid = ctx.submit(h, sd, q, T=6, eval_points=ev, thresholds=thr, top_k=10)
    with pytest.raises(GraspError, match="live job"):
        ev.unload()  # the job still needs it
    t0 = time.time()
    r = None
    while r is None and time.time() - t0 < 120.0:
        r = ctx.poll(jid, q.shape[0], h.n_dof, n_metrics=4, top_k=10)
        time.sleep(0.005)
    assert r is not None and r["status"] == 0
    met = ctx.evaluate(ev, sd, torch.as_tensor(r["q"], device=dev), thr)
    top, mean = ctx.select_top(torch.as_tensor(r["loss"], device=dev), 10, metrics=met)
    assert np.array_equal(r["metrics"], met.cpu().numpy())
    assert np.array_equal(r["top"], top.cpu().numpy()) and np.array_equal(r["top_mean"], mean.cpu().numpy())
    assert np.array_equal(r["top"], r["rank"][:10])
    assert (r["metrics"][:, 2] > 0).any()
    other = S.make_hand(3, 3, 128, seed=74)
    ho = ctx.hand(other)
    qo = S.make_candidates(other, 4, seed=75, shell_radius=0.1).astype(np.float32)
    with pytest.raises(GraspError, match="another hand"):
        ctx.submit(ho, sd, qo, T=2, eval_points=ev, thresholds=thr)
    with pytest.raises(GraspError, match="evaluation set"):
        ctx.submit(h, sd, q, T=2, top_k=3)
    with pytest.raises(GraspError, match="top_k"):
        ctx.submit(h, sd, q, T=2, eval_points=ev, thresholds=thr, top_k=65)
    ev.unload()
    ho.destroy()


def test_gauss_seidel_job(setup):
    """A served job with the Gauss-Seidel projection, running beside an
    averaged job, gives the same bits as its fused steps launched directly on
    the same dilation schedule followed by the forward at zero dilation."""
    from paper_2306_08132_amd.api import StepParams
    from paper_2306_08132_amd._lib import PROJECTION_GAUSS_SEIDEL as GS
    ctx, objs = setup
    dev = "cuda:0"
    h, sd, q = objs[1]
    T, r0 = 6, 0.01
    say("serving: Gauss-Seidel job beside an averaged job")
    other = ctx.submit(objs[0][0], objs[0][1], objs[0][2], T=9)
    jid = ctx.submit(h, sd, q, T=T, r0=r0, prm=StepParams(projection=GS))
    r = wait(ctx, jid, q.shape[0], h.n_dof)
    assert r["status"] == 0 and r["steps"] == T
    assert wait(ctx, other, objs[0][2].shape[0], objs[0][0].n_dof)["status"] == 0
    say("serving: the same Gauss-Seidel steps launched directly")
    qd = torch.as_tensor(q, device=dev).clone()
    m, v = torch.zeros_like(qd), torch.zeros_like(qd)
    loss = torch.empty(q.shape[0], device=dev)
    terms = torch.empty(q.shape[0], 4, device=dev)
    for t in range(T):
        r_dil = float(np.float32(r0)) * (1.0 - min(t, T - 1) / (T - 1))
        ctx.step_fused(h, sd, StepParams(projection=GS, r_dil=r_dil), qd, m, v, t + 1, loss=loss)
    ctx.step_fwd(h, sd, StepParams(projection=GS, r_dil=0.0), qd, loss, terms)
    torch.cuda.synchronize()
    assert np.array_equal(r["q"], qd.cpu().numpy())
    assert np.array_equal(r["loss"], loss.cpu().numpy())
    assert np.array_equal(r["terms"], terms.cpu().numpy())
    assert not np.array_equal(r["q"], q)  # the job moved its candidates


def test_gauss_seidel_job_reserves_its_start_poses(gpu):
    """A Gauss-Seidel job's footprint holds its sweep start-pose table (168 K
    bytes per candidate and 64-contact chunk): in a 16 MiB arena a job of 4096
    candidates, 8 chunks and K = 4 (22 MB of start poses) can never fit and is
    refused at submission, while the same job with the averaged projection
    is admitted and runs."""
    from paper_2306_08132_amd.api import Context, GraspError, StepParams
    from paper_2306_08132_amd._lib import PROJECTION_GAUSS_SEIDEL as GS
    ctx = Context(0, arena_bytes=16 << 20)
    try:
        ctx.serve_config(capacity=4096, max_jobs=4)
        hand = S.make_hand(3, 3, 512, seed=80)
        grid = S.make_grid(S.make_object("ellipsoids", seed=81, n_range=(2, 3)), 24)
        q = S.make_candidates(hand, 4096, seed=82, shell_radius=grid.bound_radius + 0.06).astype(np.float32)
        h, sd = ctx.hand(hand), ctx.sdf(grid)
        say("serving: a Gauss-Seidel job larger than the arena is refused")
        with pytest.raises(GraspError, match="never fit"):
            ctx.submit(h, sd, q, T=2, prm=StepParams(projection=GS, K=4))
        r = wait(ctx, ctx.submit(h, sd, q, T=2, prm=StepParams(K=4)), q.shape[0], h.n_dof)
        assert r["status"] == 0 and r["steps"] == 2
    finally:
        ctx.close()
