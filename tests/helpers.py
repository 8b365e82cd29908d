"""Shared test helpers: small hand-built hands and objects (input construction only)."""
from types import SimpleNamespace

import numpy as np

EYE34 = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).reshape(12)


def point_hand(points):
    """A palm-only hand (6 DOF) whose contacts sit at the given palm-frame points."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    return SimpleNamespace(
        parent=np.array([-1], np.int32), joint_origin=EYE34[None, :].copy(),
        joint_axis=np.array([[0.0, 0.0, 1.0]]), q_low=np.zeros(6), q_up=np.zeros(6),
        contact_local=pts, contact_link=np.zeros(len(pts), np.int32))


def rotvec_matrix(theta):
    from scipy.spatial.transform import Rotation
    return Rotation.from_rotvec(np.asarray(theta, dtype=np.float64)).as_matrix()


def dyadic_plane_grid(n=33, lo=-1.0, h=1.0 / 16, coef=(0.5, 0.25, -0.125), off=0.0625):
    """Grid of an affine field whose vertex values are exact in FP32."""
    from paper_2306_08132_amd.synth import Grid
    g = Grid(n=n, lo=np.full(3, lo), h=h, values=np.empty(0, np.float32), prims=[], bound_radius=0.0)
    P = g.vertex_positions()
    vals = P @ np.asarray(coef) + off
    assert np.array_equal(vals.astype(np.float32).astype(np.float64), vals)
    g.values = vals.astype(np.float32)
    return g


SIM_DIRS = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [0, 0, 0]],
                    dtype=np.float64)
