"""GPU parity of the mesh object (Sec. III-B) against the FP64 oracle: the
Phong signed distance from the BVH query kernel (value, sign and stated
gradient), grids filled from a mesh on the device against grids the oracle
fills from the same mesh, a grasp step on such a grid against the oracle's
step on its own grid, and the loader's refusals. Tolerances: value within
1e-5 of max(|rho|, edge length) plus the oracle's medial gap (a point nearly
equidistant from two parts of the surface may pick either in FP32); exact
sign where the point lies more than 1e-6 m from the flat mesh; gradient
within 1e-5 where the gap exceeds 1e-5 m, |rho| > 1 mm and the value is
well determined. Where the flat distances of several faces lie within FP32
resolution of the best, FP32 may pick any of them; the oracle reports how far
apart their Phong distances lie (the spread), which is added to the value
tolerance. The stated
distance takes its sign from the flat mesh and its size from the Phong point,
so it jumps by twice the Phong offset across the flat surface: within 1e-6 m
of it FP32 may take either side, and there the value may differ by 2 |rho|."""
import numpy as np
import pytest
import torch

import oracle as O
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


def f32mesh(m):
    """The mesh as the GPU receives it (FP32 coordinates and normals)."""
    return S.TriMesh(m.vertices.astype(np.float32).astype(np.float64), m.faces,
                     m.normals.astype(np.float32).astype(np.float64))


def edge_length(m):
    v = m.vertices[m.faces]
    return float(np.linalg.norm(v[:, 1] - v[:, 0], axis=1).mean())


def points_around(m, n, seed):
    rng = np.random.default_rng(seed)
    R = m.bound_radius()
    r = rng.uniform(-1.6 * R, 1.6 * R, size=(n, 3))
    r[: n // 3] *= 0.5  # inside points
    d = rng.normal(size=(n // 3, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # points within a few millimetres of the surface
    r[n // 3: 2 * (n // 3)] = m.vertices[rng.integers(0, m.vertices.shape[0], n // 3)] + d * 3e-3
    return r.astype(np.float32)


def compare_samples(ctx, m, alpha, r, label):
    m = f32mesh(m)
    gm = ctx.mesh(m, alpha)
    out = gm.sample(torch.as_tensor(r, device=DEV)).cpu().numpy().astype(np.float64)
    ref = O.mesh_sdf(O.Mesh(m.vertices, m.faces, m.normals, float(np.float32(alpha))), r.astype(np.float64))
    rho, g = out[:, 0], out[:, 1:]
    scale = np.maximum(np.abs(ref["rho"]), edge_length(m))
    err = np.abs(rho - ref["rho"])
    near = ref["dist_flat"] < 1e-6
    tol = 1e-5 * scale + ref["gap"] + ref["spread"] + np.where(near, 2.0 * np.abs(ref["rho"]), 0.0)
    say(f"{label}: n={len(r)} max rho err {err.max():.2e}, off the flat surface {err[~near].max():.2e} "
        f"(rel {(err[~near] / scale[~near]).max():.2e}), medial {np.mean(ref['gap'] < 1e-5):.3f}, "
        f"on the flat surface {near.sum()}")
    assert np.all(err <= tol), (np.argmax(err - tol), (err - tol).max())
    assert near.mean() < 0.01
    firm = ~near & (np.abs(ref["rho"]) > 1e-6)
    assert np.array_equal(np.sign(rho[firm]), np.sign(ref["rho"][firm]))
    ok = (ref["gap"] > 1e-5) & (np.abs(ref["rho"]) > 1e-3) & (ref["spread"] < 1e-7 * np.abs(ref["rho"]))
    gerr = np.abs(g[ok] - ref["grad"][ok]).max()
    say(f"  grad err {gerr:.2e} over {ok.sum()} points")
    assert ok.sum() > len(r) // 8
    assert gerr <= 1e-5
    gm.unload()


@pytest.mark.parametrize("alpha", [0.0, 0.75])
def test_ellipsoid_mesh_samples(ctx, alpha):
    m = S.mesh_ellipsoid([0.03, 0.02, 0.045], rotation=S.Rotation.from_euler("xyz", [0.3, -0.5, 1.1]).as_matrix(),
                         center=(0.004, -0.002, 0.001), subdivisions=3)
    compare_samples(ctx, m, alpha, points_around(m, 3000, 1), f"ellipsoid mesh alpha={alpha}")


def test_box_mesh_samples(ctx):
    m = S.mesh_box([0.02, 0.035, 0.015], splits=3)
    compare_samples(ctx, m, 0.5, points_around(m, 3000, 2), "split box mesh alpha=0.5")


def test_fine_mesh_samples(ctx):
    m = S.random_mesh_object(seed=7, subdivisions=5)  # 20480 faces: a deeper hierarchy
    compare_samples(ctx, m, 0.75, points_around(m, 600, 3), "fine ellipsoid mesh")


def test_nonfinite_point_gives_nan(ctx):
    m = f32mesh(S.icosphere(1))
    gm = ctx.mesh(m, 0.5)
    r = torch.tensor([[np.nan, 0.0, 0.0], [0.0, np.inf, 0.0], [2.0, 0.0, 0.0]], dtype=torch.float32, device=DEV)
    out = gm.sample(r).cpu().numpy()
    assert np.all(np.isnan(out[:2])) and np.all(np.isfinite(out[2]))
    gm.unload()


def test_invalid_meshes_are_refused(ctx):
    from paper_2306_08132_amd._lib import GraspError
    m = S.icosphere(1)
    open_mesh = S.TriMesh(m.vertices, m.faces[:-1], m.normals)
    flipped = S.TriMesh(m.vertices, m.faces[:, ::-1].copy(), m.normals)
    bad_index = S.TriMesh(m.vertices, np.where(m.faces == 3, 10_000, m.faces), m.normals)
    for mesh, what in ((open_mesh, "closed"), (flipped, "volume"), (bad_index, "range")):
        with pytest.raises(GraspError) as e:
            ctx.mesh(mesh, 0.5)
        assert what in str(e.value)
    with pytest.raises(GraspError):
        ctx.mesh(m, 1.5)


def oracle_grid(m, alpha, n, lo, h):
    """The grid the oracle fills from the same mesh (FP64, stored FP32)."""
    i = np.arange(n, dtype=np.float64)
    z, y, x = np.meshgrid(lo[2] + i * h, lo[1] + i * h, lo[0] + i * h, indexing="ij")
    p = np.stack([x, y, z], axis=-1).reshape(-1, 3)
    out = O.mesh_sdf(O.Mesh(m.vertices, m.faces, m.normals, alpha), p)
    g = S.Grid(n, np.asarray(lo, float), h, out["rho"].astype(np.float32), [], m.bound_radius())
    return g, out["dist_flat"], out["gap"] + out["spread"]


def test_grid_from_mesh_and_step(ctx):
    """A grid filled on the device from a mesh holds the oracle's values; a
    grasp step on it matches the oracle's step on the oracle's grid."""
    from paper_2306_08132_amd.api import StepParams
    m = f32mesh(S.mesh_ellipsoid([0.035, 0.025, 0.03], subdivisions=3))
    alpha = float(np.float32(0.75))
    n = 50  # 4^3 bricks of the fill with a ragged edge
    lo = np.float32([-0.06, -0.06, -0.06]).astype(np.float64)
    h = float(np.float32(0.12 / (n - 1)))
    gm = ctx.mesh(m, alpha)
    sd = gm.grid(n, lo, h, inertia_over_mass=4e-4)
    g_or, flat, gap = oracle_grid(m, alpha, n, lo, h)
    # read the device grid back only to compare it; the oracle never sees it
    r = torch.as_tensor(g_or.vertex_positions().astype(np.float32), device=DEV)
    got = ctx.debug_sdf_sample(sd, r).cpu().numpy()[:, 0].astype(np.float64)
    want = g_or.values.astype(np.float64)
    err = np.abs(got - want)
    near = flat < 1e-6
    say(f"grid from mesh: max err {err.max():.2e}, off the flat surface {err[~near].max():.2e}, "
        f"on it {near.sum()} of {near.size}")
    assert np.all(err <= 1e-5 * np.maximum(np.abs(want), h) + gap + np.where(near, 2.0 * np.abs(want), 0.0))
    # the fill walks the hierarchy once per 4^3 brick of vertices, the point
    # query once per point: at the vertices they agree up to the grid's own
    # interpolation rounding and faces tied within FP32 (either sign on the
    # flat surface)
    lane = gm.sample(r).cpu().numpy()[:, 0].astype(np.float64)
    dl = np.abs(got - lane)
    say(f"fill against the point query: max diff {dl.max():.2e}, bit-equal {np.mean(dl == 0):.4f}")
    assert np.all(dl <= 4e-6 * np.maximum(np.abs(lane), h) + np.where(near, 2.0 * np.abs(lane), 0.0))
    # a step on each side's own grid
    hand, _, q = S.config_workload("tiny")
    hd = ctx.hand(hand)
    sp = StepParams(r_dil=float(np.float32(0.005)))
    op = O.Params()
    for k in vars(op):
        setattr(op, k, float(np.float32(getattr(sp, k))) if isinstance(getattr(op, k), float) else getattr(op, k))
    qd = torch.as_tensor(np.asarray(q, np.float32), device=DEV)
    loss = torch.empty(q.shape[0], device=DEV)
    ctx.step_fwd(hd, sd, sp, qd, loss)
    torch.cuda.synchronize()
    ref = O.step(O.Hand(hand.rounded()), O.Obj(g_or, inertia_over_mass=float(np.float32(4e-4))), op,
                 np.asarray(q, np.float32).astype(np.float64), grad=False, margins=True)
    lerr = np.abs(loss.cpu().numpy() - ref["loss"]) / np.maximum(np.abs(ref["loss"]), op.w_stable * op.v0)
    # the two grids differ by up to the value tolerance above: a sample that
    # close to d = 0 may be active on one side only, and the averaged
    # correction then changes by a whole constraint
    flagged = ref["min_abs_d"] < 2.0 * err.max() + 1e-7
    say(f"step on the mesh grid: max loss rel err {lerr[~flagged].max():.2e}, flagged {flagged.sum()} "
        f"(their errs {np.round(lerr[flagged], 4).tolist()})")
    assert np.all(lerr[~flagged] <= 1e-4)
    assert flagged.mean() <= 0.2
    sd.unload()
    gm.unload()
