"""Stored fixtures under tests/golden/: the step parameters the paper states
(checked against every default: the C library's, the Python binding's and the
oracle's), and FP64 oracle values for the tiny workload written by
make_oracle_tiny.py (the oracle must keep reproducing them; the HIP path is
compared with them in test_gpu_parity.py). No GPU needed."""
import ctypes as C
import inspect
import os

import numpy as np
import pytest

import oracle as O
from paper_2306_08132_amd import synth as S

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_parameters():
    out = {}
    for line in open(os.path.join(GOLDEN, "paper_parameters.txt")):
        if line.strip() and not line.startswith("#"):
            name, value = line.split()[:2]
            out[name] = value
    return out


def load_oracle_tiny():
    """[(K, r_dil, [(index, q, loss, terms, grad), ...]), ...]"""
    cases, cur = [], None
    lines = [l.split() for l in open(os.path.join(GOLDEN, "oracle_tiny.txt")) if l.strip() and l[0] != "#"]
    i = 0
    while i < len(lines):
        head = lines[i]
        assert head[0] == "case"
        cur = (int(head[1]), float(np.float32(float(head[2]))), [])  # an FP32 value
        n = int(head[3])
        i += 1
        for _ in range(n):
            idx = int(lines[i][1])
            q = np.array(lines[i + 1][1:], float).astype(np.float32).astype(np.float64)  # FP32 values
            loss = float(lines[i + 2][1])
            terms = np.array(lines[i + 3][1:], float)
            grad = np.array(lines[i + 4][1:], float)
            cur[2].append((idx, q, loss, terms, grad))
            i += 5
        cases.append(cur)
    return cases


def test_paper_parameters_are_every_default():
    from paper_2306_08132_amd import _lib
    P = paper_parameters()
    assert int(P["tests"]) == O.M_SIMS == len(P["test_velocity"].split(","))
    assert int(P["time_steps"]) == 1 == O.Params().K
    dt, alpha, lr = float(P["dt"]), float(P["leak_alpha"]), float(P["learning_rate"])
    # the oracle and the Python binding
    assert (O.Params().dt, O.Params().alpha_leak) == (dt, alpha)
    assert (_lib.StepParams().dt, _lib.StepParams().alpha_leak, _lib.StepParams().K) == (dt, alpha, 1)
    assert inspect.signature(O.adam).parameters["lr"].default == lr
    from paper_2306_08132_amd.api import Context
    assert inspect.signature(Context.step_fused).parameters["lr"].default == lr
    # the C library (host code only)
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgrasp.so not built")
    p = _lib.StepParamsC()
    _lib.Library.get().grasp_default_params(C.byref(p))
    assert (p.dt, p.alpha_leak, p.K) == (C.c_float(dt).value, C.c_float(alpha).value, 1)


def test_test_velocities_are_the_paper_set():
    """Before the first iteration each test's object sits at dt v0 along its
    initial velocity: the set is +-x, +-y, +-z and rest."""
    P = paper_parameters()
    hand, grid, q = S.config_workload("tiny")
    prm = O.Params()
    tr = O.trace(O.Hand(hand.rounded()), O.Obj(grid), prm, q[0], samples=False)
    x0 = tr["poses"][:, 0, :]
    assert np.all(x0[:, 3:] == 0.0)
    axis = {"x": 0, "y": 1, "z": 2}
    want = set()
    for v in P["test_velocity"].split(","):
        d = np.zeros(3)
        if v != "0":
            d[axis[v[1]]] = 1.0 if v[0] == "+" else -1.0
        want.add(tuple(d * prm.dt * prm.v0))
    got = {tuple(r) for r in x0[:, :3]}
    assert got == want


def test_oracle_reproduces_stored_values():
    hand, grid, q = S.config_workload("tiny")
    H, ob = O.Hand(hand.rounded()), O.Obj(grid)
    q32 = np.asarray(q, np.float32).astype(np.float64)
    for K, r_dil, rows in load_oracle_tiny():
        assert len(rows) >= 4
        prm = O.Params()
        for k in vars(prm):
            v = getattr(prm, k)
            setattr(prm, k, float(np.float32(v)) if isinstance(v, float) else v)
        prm.K, prm.r_dil = K, r_dil
        idx = np.array([r[0] for r in rows])
        qs = np.stack([r[1] for r in rows])
        assert np.array_equal(qs, q32[idx])  # stored inputs are the generator's
        ref = O.step(H, ob, prm, qs, grad=True)
        for j, (_, _, loss, terms, grad) in enumerate(rows):
            assert ref["loss"][j] == pytest.approx(loss, rel=1e-12, abs=1e-15)
            assert np.allclose(ref["terms"][j], terms, rtol=1e-12, atol=1e-15)
            assert np.allclose(ref["grad"][j], grad, rtol=1e-10, atol=1e-10 * np.abs(grad).max())
