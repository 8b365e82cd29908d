"""Pins of the oracle's readings of FP32-ambiguous mesh samples (the step on a
mesh object, Sec. III-B's Phong distance in Sec. III-C's constraint): where a
discrete choice of the query is decided at a tie (the side of the flat surface,
which of two equidistant surface points, the region of the closest point), the
oracle reports the sample, and taking the other reading gives the step's
result at the hand point moved by 1e-10 m to the other side of the tie, while
the default reading gives it on its own side. The ties are exact: a box mesh
with dyadic half extents and dyadic points. No GPU needed."""
import numpy as np
import pytest

import oracle as O
from paper_2306_08132_amd import synth as S
from tests import parity_check as P
from tests.helpers import point_hand

HALF = np.array([0.03125, 0.0234375, 0.0390625])  # 1/32, 3/128, 5/128 m
DELTA = 1e-10


def box(alpha):
    m = S.mesh_box(HALF, splits=1)
    M = O.Mesh(m.vertices, m.faces, m.normals, alpha)
    return O.Obj(mesh=M, inertia_over_mass=0.4 * 0.03 ** 2)


def run(ob, p, op, flips=()):
    H = O.Hand(point_hand([p]))
    return O.step_ex(H, ob, op, np.zeros((1, 6)), flips=[(0, *f) for f in flips], kink_d=P.KINK_D,
                     kink_face=P.KINK_FACE, max_amb=64)


def close(a, b):
    g = max(np.abs(a["grad"]).max(), np.abs(b["grad"]).max())
    return (abs(a["loss"][0] - b["loss"][0]) <= 1e-6 * abs(b["loss"][0])
            and np.abs(a["grad"] - b["grad"]).max() <= 1e-5 * g)


def check(ob, p, op, what, nudges):
    ref = run(ob, p, op)
    amb = [tuple(int(x) for x in a[:4]) for a in ref["amb"][0] if int(a[3]) == what]
    assert amb, f"no ambiguity of kind {what} reported"
    alt = run(ob, p, op, flips=amb)
    lo, hi = run(ob, p + nudges[0], op), run(ob, p + nudges[1], op)
    # the two sides of the tie differ, and the two readings are the two sides
    assert not close(lo, hi)
    assert (close(ref, lo) and close(alt, hi)) or (close(ref, hi) and close(alt, lo))
    return amb


def test_medial_tie_between_two_faces(oracle_lib):
    """Inside the box, 1/256 m from both the +x and the +y face (Phong alpha
    0.5): the closest point is on either face; the rest test and the two z
    tests keep the tie."""
    t = 1.0 / 256
    p = np.array([HALF[0] - t, HALF[1] - t, 0.001953125])
    amb = check(box(0.5), p, O.Params(r_dil=0.002), 7,
                (np.array([DELTA, 0.0, 0.0]), np.array([0.0, DELTA, 0.0])))
    assert {a[0] for a in amb} == {4, 5, 6}


def test_region_border_of_the_closest_point(oracle_lib):
    """Outside the +x face at 1/512 m, level with the box edge y = half_y
    (flat faces, alpha = 0), inside the dilation: the closest point lies on
    the border of the face's interior and its edge, where the normal's
    derivative changes (zero on the interior, a rotation about the edge
    beyond it)."""
    t = 1.0 / 512
    p = np.array([HALF[0] + t, HALF[1], 0.001953125])
    check(box(0.0), p, O.Params(r_dil=0.004), 8,
          (np.array([0.0, -DELTA, 0.0]), np.array([0.0, DELTA, 0.0])))


def test_side_of_the_flat_surface(oracle_lib):
    """On the +z face of the box (Phong alpha 0.5, corner vertex normals
    averaged over the faces they touch, so the Phong point lies off the flat
    face): the flat mesh's sign decides rho's sign, and rho jumps by twice the
    Phong offset across the face."""
    p = np.array([0.0078125, 0.00390625, HALF[2]])
    check(box(0.5), p, O.Params(r_dil=0.004), 6,
          (np.array([0.0, 0.0, -DELTA]), np.array([0.0, 0.0, DELTA])))
