"""GPU: grasp_step_fused_static, the fused step for callers that cannot
allocate (its candidate order in the library's fixed device array), through
the C ABI against grasp_step_fused on the same inputs: loss, terms, dq and
the updated q, m, v bit for bit, on two calls in a row, the second with
fewer candidates (the array keeps the first call's order beyond them), for
one and for four projection iterations; a call too large for the array is
refused; a captured graph of it replays to the eager result."""
import numpy as np
import pytest
import torch

from paper_2306_08132_amd import synth as S

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def setup(gpu):
    from paper_2306_08132_amd.api import Context
    ctx = Context(0, arena_bytes=256 << 20)
    hand, grid, q = S.config_workload("tiny", B=900)
    yield ctx, ctx.hand(hand), ctx.sdf(grid), q
    ctx.close()


def run(ctx, h, sd, sp, q, static, stream=None):
    qd = torch.tensor(q, dtype=torch.float32, device=DEV)
    m = torch.full_like(qd, 1e-3)
    v = torch.full_like(qd, 1e-6)
    B = q.shape[0]
    loss = torch.empty(B, device=DEV)
    terms = torch.empty((B, 4), device=DEV)
    dq = torch.empty_like(qd)
    f = ctx.step_fused_static if static else ctx.step_fused
    f(h, sd, sp, qd, m, v, 3, loss=loss, terms=terms, dq=dq, stream=stream)
    torch.cuda.synchronize()
    return qd, m, v, loss, terms, dq


@pytest.mark.parametrize("K", [1, 4])
def test_static_step_equals_fused_step(setup, K):
    from paper_2306_08132_amd.api import StepParams
    ctx, h, sd, q = setup
    sp = StepParams(r_dil=0.004, K=K, ckpt_every=2 if K > 1 else 1)
    for B in (900, 300):  # both run the candidate order; the second call is smaller
        want = run(ctx, h, sd, sp, q[:B], static=False)
        got = run(ctx, h, sd, sp, q[:B], static=True)
        for name, a, b in zip(("q", "m", "v", "loss", "terms", "dq"), got, want):
            assert torch.equal(a, b), (K, B, name, float((a - b).abs().max()))
        print(f"static vs fused, K={K}, B={B}: identical", flush=True)


def test_static_step_limits(setup):
    from paper_2306_08132_amd._lib import GraspError
    from paper_2306_08132_amd.api import StepParams
    ctx, h, sd, q = setup
    big = np.zeros((262145, h.n_dof), np.float32)
    qd = torch.tensor(big, device=DEV)
    with pytest.raises(GraspError, match="262144"):
        ctx.step_fused_static(h, sd, StepParams(), qd, torch.zeros_like(qd), torch.zeros_like(qd), 1)
    small = torch.tensor(q[:8], dtype=torch.float32, device=DEV)
    with pytest.raises(GraspError, match="Gauss-Seidel"):
        ctx.step_fused_static(h, sd, StepParams(projection=1), small, torch.zeros_like(small),
                              torch.zeros_like(small), 1)


def test_static_step_in_a_graph(setup):
    """Captured with its order kernel, replayed three times with eager work in
    between: every replay equals the eager call."""
    from paper_2306_08132_amd.api import StepParams
    ctx, h, sd, q = setup
    sp = StepParams(r_dil=0.004)
    want = run(ctx, h, sd, sp, q[:600], static=True)
    qd = torch.tensor(q[:600], dtype=torch.float32, device=DEV)
    m, v = torch.full_like(qd, 1e-3), torch.full_like(qd, 1e-6)
    loss = torch.empty(600, device=DEV)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        ctx.step_fused_static(h, sd, sp, qd, m, v, 3, loss=loss, stream=s)
    q0 = torch.tensor(q[:600], dtype=torch.float32, device=DEV)
    for _ in range(3):
        qd.copy_(q0)
        m.fill_(1e-3)
        v.fill_(1e-6)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (qd * 2).sum().item()
        assert torch.equal(qd, want[0]) and torch.equal(loss, want[3])
