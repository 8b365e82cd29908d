"""GPU: the batched form. Every job's results must be bit-identical to its
own fused single-job steps, alone or mixed with other jobs, and with the
launch replayed from a hipGraph or issued eagerly."""
import numpy as np
import pytest
import torch

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


@pytest.fixture(scope="module")
def objects(ctx):
    """Four jobs' geometry: different hands, grid resolutions and sizes (the
    last one large enough to run in the candidate locality order)."""
    out = []
    for k, (F, J, nc, N, B) in enumerate([(3, 3, 300, 24, 7), (4, 4, 700, 40, 13), (5, 4, 1000, 33, 5),
                                          (3, 3, 300, 24, 300)]):
        hand = S.make_hand(F, J, nc, seed=10 + k)
        grid = S.make_grid(S.make_object("mixed", seed=20 + k, n_prims=3), N)
        q = S.make_candidates(hand, B, seed=30 + k, shell_radius=grid.bound_radius + 0.06)
        out.append((ctx.hand(hand), ctx.sdf(grid), q))
    return out


def r0f():
    return float(np.float32(0.01))


def make_jobs(objects, idx, K=1):
    from paper_2306_08132_amd.api import BatchJob, StepParams
    jobs = []
    for i in idx:
        h, sd, q = objects[i]
        jobs.append(BatchJob(h, sd, StepParams(K=K), torch.tensor(q, dtype=torch.float32, device=DEV), T=6,
                             r0=r0f()))
    return jobs


def run_single(ctx, objects, i, steps, K=1):
    """Reference: the same job advanced by grasp_step_fused, one launch per step."""
    from paper_2306_08132_amd.api import StepParams
    h, sd, q0 = objects[i]
    q = torch.tensor(q0, dtype=torch.float32, device=DEV)
    m, v = torch.zeros_like(q), torch.zeros_like(q)
    loss = torch.empty(q.shape[0], device=DEV)
    T = 6
    for t in range(steps):
        r = float(np.float32(np.float64(np.float32(r0f())) * (1.0 - min(t, T - 1) / (T - 1))))
        ctx.step_fused(h, sd, StepParams(K=K, r_dil=r), q, m, v, t + 1, loss=loss)
    torch.cuda.synchronize()
    return q.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), loss.cpu().numpy()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_single_job_steps(ctx, objects, use_graph):
    from paper_2306_08132_amd.api import Batch
    say("batch vs single, graph =", use_graph)
    stream = torch.cuda.Stream()
    b = Batch(ctx, capacity=64, max_jobs=8, use_graph=use_graph)
    jobs = make_jobs(objects, [0, 1, 2])
    with torch.cuda.stream(stream):
        for s in range(3):
            b.step(jobs, stream=stream)
            # eager work between replays
            _ = (jobs[0].q * 2).sum().item()
    stream.synchronize()
    for i, j in enumerate(jobs):
        q, m, v, loss = run_single(ctx, objects, i, 3)
        assert np.array_equal(j.q.cpu().numpy(), q)
        assert np.array_equal(j.m.cpu().numpy(), m) and np.array_equal(j.v.cpu().numpy(), v)
        assert np.array_equal(j.loss.cpu().numpy(), loss)
        assert j.t == 3
    b.close()


def test_batch_with_ordered_job(ctx, objects):
    """A job of 300 candidates runs in its locality order inside the batch
    and in single-job launches; both equal bit for bit."""
    from paper_2306_08132_amd.api import Batch
    stream = torch.cuda.Stream()
    b = Batch(ctx, capacity=512, max_jobs=4, use_graph=True)
    jobs = make_jobs(objects, [3, 1])
    with torch.cuda.stream(stream):
        for s in range(3):
            b.step(jobs, stream=stream)
    stream.synchronize()
    for j, i in zip(jobs, [3, 1]):
        q, m, v, loss = run_single(ctx, objects, i, 3)
        say("ordered job", i, "max |dq|", float(np.abs(j.q.cpu().numpy() - q).max()))
        assert np.array_equal(j.q.cpu().numpy(), q) and np.array_equal(j.loss.cpu().numpy(), loss)
    b.close()


def test_job_alone_equals_job_in_mix(ctx, objects):
    from paper_2306_08132_amd.api import Batch
    stream = torch.cuda.Stream()
    alone = make_jobs(objects, [1])
    mix = make_jobs(objects, [2, 1, 0])
    b1 = Batch(ctx, capacity=64, max_jobs=8)
    b2 = Batch(ctx, capacity=64, max_jobs=8)
    with torch.cuda.stream(stream):
        for s in range(4):
            b1.step(alone, stream=stream)
            b2.step(mix, stream=stream)
    stream.synchronize()
    assert np.array_equal(alone[0].q.cpu().numpy(), mix[1].q.cpu().numpy())
    assert np.array_equal(alone[0].loss.cpu().numpy(), mix[1].loss.cpu().numpy())
    b1.close()
    b2.close()


def test_batch_mixed_iterations_and_tiles(ctx, objects):
    """Jobs with K = 1 and K = 2 in one step (two launches), every tile identical."""
    from paper_2306_08132_amd.api import Batch, BatchJob, StepParams
    res = []
    for wpb, occ in [(4, 1), (1, 3), (2, 2)]:
        stream = torch.cuda.Stream()
        b = Batch(ctx, capacity=64, max_jobs=8)
        b.set_tile(wpb, occ)
        jobs = make_jobs(objects, [0, 2]) + make_jobs(objects, [1], K=2)
        with torch.cuda.stream(stream):
            for s in range(2):
                b.step(jobs, stream=stream)
        stream.synchronize()
        res.append([j.q.cpu().numpy() for j in jobs])
        b.close()
    for r in res[1:]:
        assert all(np.array_equal(x, y) for x, y in zip(r, res[0]))
    q, _, _, _ = run_single(ctx, objects, 1, 2, K=2)
    assert np.array_equal(res[0][2], q)


def test_batch_capacity_and_bad_jobs_rejected(ctx, objects):
    from paper_2306_08132_amd.api import Batch, GraspError
    b = Batch(ctx, capacity=10, max_jobs=2)
    with pytest.raises(GraspError):
        b.step(make_jobs(objects, [0, 1]))      # 20 candidates > capacity 10
    with pytest.raises(GraspError):
        b.step(make_jobs(objects, [0, 2, 2]))   # 3 jobs > max_jobs 2
    b.close()
