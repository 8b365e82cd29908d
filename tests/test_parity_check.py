"""The comparison helper on the CPU: results that differ from the oracle's only
by another reading of an ambiguous sample pass as resolved; a wrong loss or
gradient fails; the readings the oracle takes change nothing else."""
import numpy as np
import pytest

import oracle as O
from paper_2306_08132_amd import synth as S
from tests import parity_check as P


@pytest.fixture(scope="module")
def tiny():
    hand, grid, q = S.config_workload("tiny")
    return O.Hand(hand.rounded()), O.Obj(grid), q.astype(np.float32).astype(np.float64)


def test_step_ex_without_flips_is_the_step(tiny):
    H, ob, q = tiny
    for K in (1, 3):
        op = O.Params(r_dil=0.005, K=K)
        a = O.step(H, ob, op, q[:16])
        b = O.step_ex(H, ob, op, q[:16], kink_d=P.KINK_D, kink_face=P.KINK_FACE, max_amb=8)
        assert np.array_equal(a["loss"], b["loss"]) and np.array_equal(a["grad"], b["grad"])


def test_other_readings_are_resolved_and_mistakes_fail(tiny):
    H, ob, q = tiny
    op = O.Params(r_dil=0.005)
    ref = O.step_ex(H, ob, op, q, kink_d=P.KINK_D, kink_face=P.KINK_FACE, max_amb=64)
    amb = [b for b in range(q.shape[0]) if P.units_of(ref["amb"][b])]
    assert len(amb) >= 3
    # a "GPU" result that took the other reading of each such candidate's most ambiguous unit
    flips = []
    for b in amb:
        flips += [(b, *f) for f in P.units_of(ref["amb"][b])[0][1]]
    alt = O.step_ex(H, ob, op, q, flips=flips)
    moved = [b for b in amb if np.abs(alt["grad"][b] - ref["grad"][b]).max() > 1e-3 * np.abs(ref["grad"][b]).max()]
    rep = P.compare(alt["loss"].astype(np.float32), alt["grad"].astype(np.float32), H, ob, op, q, label="planted",
                    say=lambda *a: None)
    P.assert_ok(rep)
    assert rep["resolved"] >= len(moved) and rep["failed"] == 0
    # a wrong gradient on one candidate is not resolved
    g = alt["grad"].copy()
    g[5] *= 1.01
    rep = P.compare(alt["loss"], g, H, ob, op, q, say=lambda *a: None)
    assert rep["status"][5] == 3
    with pytest.raises(AssertionError):
        P.assert_ok(rep)
    # nor a wrong loss
    lo = alt["loss"].copy()
    lo[7] += 1e-3 * max(abs(lo[7]), 1.0)
    rep = P.compare(lo, None, H, ob, op, q, say=lambda *a: None)
    assert rep["status"][7] == 3


def test_shared_coordinates_flip_together():
    amb = [(2, 0, 9, 1, 1e-5, 0), (3, 0, 9, 1, 1e-5, 0), (0, 0, 9, 1, 3e-5, 0), (4, 2, 9, 1, 2e-5, 1),
           (5, 0, 11, 0, 1e-8, 1)]
    units = P.units_of(amb)
    # the d-branch unit (smallest margin), the x-face shared by tests 2..6 at k = 0,
    # test 4's face at k = 2, and test 0's own x coordinate
    assert [len(u[1]) for u in units] == [1, 5, 1, 1]
    assert units[1][1] == [(m, 0, 9, 1) for m in (2, 3, 4, 5, 6)]


def test_conditioning_sets_aside_only_what_it_explains(tiny):
    """With several iterations and conditioning measured, a wrong loss or
    gradient fails however many ambiguous decisions the candidate holds: a
    candidate is set aside only when the movement of the FP64 result under
    FP32-resolution changes of q covers its error."""
    H, ob, q = tiny
    op = O.Params(r_dil=0.005, K=3)
    ref = O.step(H, ob, op, q[:12])
    lo, g = ref["loss"].copy(), ref["grad"].copy()
    lo[3] *= 1.0 + 1e-2
    g[4] *= 1.05
    rep = P.compare(lo, g, H, ob, op, q[:12], conditioning=True, max_units=1, say=lambda *a: None)
    assert rep["status"][3] == 3 and rep["status"][4] == 3
    assert rep["lcond"][3] < 1e-3 and rep["gcond"][4] < 1e-2
    assert np.all(rep["status"][[b for b in range(12) if b not in (3, 4)]] == 0)
