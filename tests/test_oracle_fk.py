"""Pins of the oracle's forward kinematics (Sec. III-C, p = FK(q)) against
geometry fixed independently of it: the generator's rest pose, rigid-body
invariants and closed-form rotations (scipy)."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2306_08132_amd import synth as S

HANDS = [(3, 3, 300, 0), (4, 4, 500, 1), (5, 4, 700, 2)]


@pytest.fixture(scope="module", params=HANDS, ids=lambda p: f"{p[0]}x{p[1]}")
def hand(request):
    F, J, n, s = request.param
    return S.make_hand(F, J, n, seed=s)


def _subtree(parent, l):
    out = {l}
    for k in range(len(parent)):
        a = k
        while a >= 0:
            if a == l:
                out.add(k)
                break
            a = parent[a]
    return out


def test_rest_pose_equals_generator_positions(oracle_lib, hand):
    O = oracle_lib
    p = O.fk(O.Hand(hand), np.zeros(hand.n_dof))[0]
    np.testing.assert_allclose(p, hand.contact_rest_world, atol=1e-15, rtol=0)


def test_rigid_link_invariance(oracle_lib, hand):
    O = oracle_lib
    H = O.Hand(hand)
    q = S.make_candidates(hand, 5, seed=7, shell_radius=0.1)
    p = O.fk(H, q)
    c = hand.contact_rest_world
    for l in range(hand.n_links):
        idx = np.nonzero(hand.contact_link == l)[0][:12]
        d0 = np.linalg.norm(c[idx, None] - c[None, idx], axis=-1)
        for b in range(q.shape[0]):
            pb = p[b, idx]
            d = np.linalg.norm(pb[:, None] - pb[None, :], axis=-1)
            np.testing.assert_allclose(d, d0, atol=1e-12, rtol=0)


def test_joint_origin_distances_invariant(oracle_lib, hand):
    """Distance between a joint origin and its parent's joint origin is fixed."""
    O = oracle_lib
    H = O.Hand(hand)
    q = S.make_candidates(hand, 4, seed=3, shell_radius=0.1)
    _, T = O.fk(H, q, frames=True)
    o = T[..., [3, 7, 11]]
    for l in range(1, hand.n_links):
        pa = hand.parent[l]
        d0 = np.linalg.norm(hand.link_rest_o[l] - hand.link_rest_o[pa])
        np.testing.assert_allclose(np.linalg.norm(o[:, l] - o[:, pa], axis=-1), d0, atol=1e-12)


@pytest.mark.parametrize("beta", [0.3, -0.7, 1.4])
def test_single_joint_rotation_closed_form(oracle_lib, hand, beta):
    """Turning one joint rotates exactly its subtree about the world joint axis
    through the joint origin; a point on the axis stays fixed."""
    O = oracle_lib
    H = O.Hand(hand)
    for l in range(1, hand.n_links):
        q = np.zeros(hand.n_dof)
        q[5 + l] = beta
        p = O.fk(H, q)[0]
        Rw = Rotation.from_rotvec(hand.joint_world_axis[l] * beta).as_matrix()
        o = hand.link_rest_o[l]
        sub = np.isin(hand.contact_link, sorted(_subtree(hand.parent, l)))
        c = hand.contact_rest_world
        expect = np.where(sub[:, None], (c - o) @ Rw.T + o, c)
        np.testing.assert_allclose(p, expect, atol=1e-14)


def test_wrist_is_translation_then_zyx_euler(oracle_lib, hand):
    O = oracle_lib
    H = O.Hand(hand)
    rng = np.random.default_rng(5)
    for _ in range(4):
        q = np.zeros(hand.n_dof)
        q[:3] = rng.normal(size=3) * 0.1
        q[3:6] = rng.uniform(-3, 3, size=3)
        p = O.fk(H, q)[0]
        R = Rotation.from_euler("ZYX", q[3:6]).as_matrix()
        np.testing.assert_allclose(p, hand.contact_rest_world @ R.T + q[:3], atol=1e-14)
