"""Seeded synthetic inputs for the grasp step: hands, object SDF grids, candidate
poses and job streams.

This module is input generation only. It builds geometry (capsule hands, exact
signed distances of primitives, initial poses) and holds none of the grasp
method's arithmetic: no forward kinematics of a configuration, no grid
sampling, no contact projection, loss, gradient or optimizer step. Both the
HIP path and the FP64 oracle are fed from here; neither is imported here.

The paper's hands (Barrett, Allegro, Shadow) and objects (YCB, EGAD) are not
available, so these generators stand in for them at their scale: objects of a
few centimetres, 3/4/5-finger hands with capsule links, and candidates batched
per object (Sec. V, Sec. IV-A).

Conventions shared with the library interface:
  * link 0 is the palm; ``parent[l] < l``; ``n_dof = 6 + (n_links - 1)``.
  * ``joint_origin[l]`` is a row-major 3x4 rigid transform from the parent link
    frame to joint ``l`` at q = 0; ``joint_axis[l]`` is a unit vector in that
    joint frame. The wrist is Trans(q0..q2) * Rz(q3) * Ry(q4) * Rx(q5).
  * SDF grids are vertex-centred: vertex (ix, iy, iz) lies at lo + (ix, iy, iz) h,
    and its value sits at index (iz * N + iy) * N + ix (x fastest).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial.transform import Rotation

CM = 0.01  # metres per centimetre

__all__ = [
    "Hand", "Grid", "make_hand", "make_object", "make_grid", "make_candidates",
    "sphere_sdf", "box_sdf", "ellipsoid_sdf", "plane_sdf", "random_points",
    "make_job_stream", "config_workload", "adam_state",
]


# ----------------------------------------------------------------------------
# hands
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Hand:
    """An articulated hand: link tree, joint frames and limits, contact points.

    All arrays are float64 / int32; ``as_f32`` gives the FP32 copy the GPU
    library receives, and ``rounded`` the same values widened back to float64.
    """
    parent: np.ndarray          # [L] int32
    joint_origin: np.ndarray    # [L][12] float64 (row-major 3x4)
    joint_axis: np.ndarray      # [L][3] float64, unit, joint frame
    q_low: np.ndarray           # [n_dof]
    q_up: np.ndarray            # [n_dof]
    contact_local: np.ndarray   # [Nc][3] in the frame of contact_link[i]
    contact_link: np.ndarray    # [Nc] int32
    # geometry kept for tests (not part of the interface)
    contact_rest_world: np.ndarray   # [Nc][3] world position at q = 0
    link_rest_R: np.ndarray          # [L][3][3] world rotation of link frames at q = 0
    link_rest_o: np.ndarray          # [L][3] world origin of link frames at q = 0
    joint_world_axis: np.ndarray     # [L][3] joint axes in the world at q = 0
    n_fingers: int = 0
    joints_per_finger: int = 0
    capsules: np.ndarray | None = None  # [L][7] world capsule of each link at q = 0: a, b, radius

    @property
    def n_links(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_dof(self) -> int:
        return 6 + self.n_links - 1

    @property
    def n_contacts(self) -> int:
        return int(self.contact_link.shape[0])

    def rounded(self) -> "Hand":
        """The same hand with every float rounded to FP32 and widened back."""
        f = lambda a: a.astype(np.float32).astype(np.float64)
        return dataclasses.replace(
            self, joint_origin=f(self.joint_origin), joint_axis=f(self.joint_axis),
            q_low=f(self.q_low), q_up=f(self.q_up), contact_local=f(self.contact_local))


def _capsule_points(rng, a, b, radius, n):
    """n points on the surface of the capsule with segment a->b, stratified by
    area along the axis (cap, cylinder, cap) with a uniform azimuth."""
    axis = b - a
    length = float(np.linalg.norm(axis))
    z = axis / length
    # orthonormal frame around z
    tmp = np.array([1.0, 0.0, 0.0]) if abs(z[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    x = np.cross(z, tmp)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    cap = 2.0 * math.pi * radius * radius
    cyl = 2.0 * math.pi * radius * length
    total = 2.0 * cap + cyl
    s = (np.arange(n) + rng.random(n)) / n * total
    az = rng.random(n) * 2.0 * math.pi
    radial = np.cos(az)[:, None] * x + np.sin(az)[:, None] * y
    out = np.empty((n, 3))
    m0 = s < cap
    m2 = s >= cap + cyl
    m1 = ~(m0 | m2)
    # cap at a: area from the pole grows as 2 pi r^2 (1 - cos psi)
    cpsi = 1.0 - s[m0] / (2.0 * math.pi * radius * radius)
    spsi = np.sqrt(np.clip(1.0 - cpsi * cpsi, 0.0, None))
    out[m0] = a + radius * (-cpsi[:, None] * z + spsi[:, None] * radial[m0])
    zz = (s[m1] - cap) / (2.0 * math.pi * radius)
    out[m1] = a + zz[:, None] * z + radius * radial[m1]
    cpsi = 1.0 - (s[m2] - cap - cyl) / (2.0 * math.pi * radius * radius)
    spsi = np.sqrt(np.clip(1.0 - cpsi * cpsi, 0.0, None))
    out[m2] = b + radius * (cpsi[:, None] * z + spsi[:, None] * radial[m2])
    return out


def _split_counts(weights, total):
    """Largest-remainder split of ``total`` items proportional to ``weights``,
    every part at least 1."""
    w = np.asarray(weights, dtype=np.float64)
    raw = w / w.sum() * (total - len(w))
    base = np.floor(raw).astype(np.int64)
    rem = total - len(w) - base.sum()
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    return base + 1


def make_hand(n_fingers: int, joints_per_finger: int, n_contacts: int, seed: int,
              shuffle: bool = True, random_link_frames: bool = True) -> Hand:
    """A capsule hand (Sec. III-C's hand model, synthetic stand-in).

    Palm: link 0, capsule of radius 1.5 cm around a 4 cm segment on local x.
    Fingers mount on a 3 cm ring around the palm's +z approach axis at angles
    2 pi f / F, at the palm's front (z = 1.5 cm), and extend along +z.
    Each finger has ``joints_per_finger`` links, capsules of length U[2, 5] cm
    and radius 0.8 cm. With 3 joints all are flexion joints (limits
    [-10, 90] deg); with 4 the first is an abduction joint ([-20, 20] deg).
    Link frames get a random rest orientation so that the joint origins carry
    real rotations. Contacts are spread over all links in proportion to
    capsule area; with ``shuffle`` their caller order is random.
    """
    rng = np.random.default_rng(seed)
    F, J = n_fingers, joints_per_finger
    L = 1 + F * J
    parent = np.zeros(L, np.int32)
    parent[0] = -1
    rest_R = np.zeros((L, 3, 3))
    rest_o = np.zeros((L, 3))
    waxis = np.zeros((L, 3))
    rest_R[0] = np.eye(3)
    caps = [(np.array([-2.0 * CM, 0.0, 0.0]), np.array([2.0 * CM, 0.0, 0.0]), 1.5 * CM)]
    lim_lo = [0.0] * 6
    lim_up = [0.0] * 6
    flex_lo, flex_up = math.radians(-10.0), math.radians(90.0)
    abd_lo, abd_up = math.radians(-20.0), math.radians(20.0)
    zhat = np.array([0.0, 0.0, 1.0])
    for f in range(F):
        ang = 2.0 * math.pi * f / F
        radial = np.array([math.cos(ang), math.sin(ang), 0.0])
        flex_axis = np.array([math.sin(ang), -math.cos(ang), 0.0])  # + curls inward
        base = 3.0 * CM * radial + 1.5 * CM * zhat
        lens = rng.uniform(2.0 * CM, 5.0 * CM, size=J)
        o = base.copy()
        for s in range(J):
            l = 1 + f * J + s
            parent[l] = 0 if s == 0 else l - 1
            rest_o[l] = o
            if random_link_frames:
                rest_R[l] = Rotation.random(random_state=rng.integers(1 << 31)).as_matrix()
            else:
                rest_R[l] = np.eye(3)
            abduct = (J >= 4 and s == 0)
            waxis[l] = radial if abduct else flex_axis
            lim_lo.append(abd_lo if abduct else flex_lo)
            lim_up.append(abd_up if abduct else flex_up)
            caps.append((o.copy(), o + lens[s] * zhat, 0.8 * CM))
            o = o + lens[s] * zhat
    joint_origin = np.zeros((L, 12))
    joint_axis = np.zeros((L, 3))
    for l in range(1, L):
        p = parent[l]
        Rrel = rest_R[p].T @ rest_R[l]
        trel = rest_R[p].T @ (rest_o[l] - rest_o[p])
        joint_origin[l] = np.concatenate([Rrel, trel[:, None]], axis=1).reshape(12)
        joint_axis[l] = rest_R[l].T @ waxis[l]
    joint_origin[0] = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).reshape(12)
    # contacts, proportional to capsule area
    areas = [2 * math.pi * r * np.linalg.norm(b - a) + 4 * math.pi * r * r for a, b, r in caps]
    counts = _split_counts(areas, n_contacts)
    pts, links = [], []
    for l, ((a, b, r), n) in enumerate(zip(caps, counts)):
        pts.append(_capsule_points(rng, a, b, r, int(n)))
        links.append(np.full(int(n), l, np.int32))
    world = np.concatenate(pts)
    link = np.concatenate(links)
    if shuffle:
        perm = rng.permutation(n_contacts)
        world, link = world[perm], link[perm]
    local = np.einsum("nji,nj->ni", rest_R[link], world - rest_o[link])
    return Hand(parent=parent, joint_origin=joint_origin, joint_axis=joint_axis,
                q_low=np.array(lim_lo), q_up=np.array(lim_up), contact_local=local,
                contact_link=link.astype(np.int32), contact_rest_world=world,
                link_rest_R=rest_R, link_rest_o=rest_o, joint_world_axis=waxis,
                n_fingers=F, joints_per_finger=J,
                capsules=np.array([np.concatenate([a, b, [r]]) for a, b, r in caps]))


@dataclasses.dataclass
class EvalPoints:
    """Weighted samples of a hand's surface and volume for the evaluation
    metrics: surface samples carry the area they stand for (m^2), volume
    samples the volume (m^3); coordinates in the frame of their link."""
    surface_link: np.ndarray    # [Ns] int32
    surface_local: np.ndarray   # [Ns][3]
    surface_area: np.ndarray    # [Ns]
    volume_link: np.ndarray     # [Nv] int32
    volume_local: np.ndarray    # [Nv][3]
    volume_weight: np.ndarray   # [Nv]
    surface_rest: np.ndarray    # [Ns][3] world positions at q = 0 (for tests)
    volume_rest: np.ndarray     # [Nv][3]

    def as_f32(self) -> "EvalPoints":
        f = lambda a: a.astype(np.float32).astype(np.float64)
        return dataclasses.replace(self, surface_local=f(self.surface_local), surface_area=f(self.surface_area),
                                   volume_local=f(self.volume_local), volume_weight=f(self.volume_weight))


def _segment_distance(p, a, b):
    ab = b - a
    t = np.clip(((p - a) @ ab) / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(p - (a + t[:, None] * ab), axis=1)


def _cap_height(v, radius):
    """Height h in [0, r] of the spherical cap of volume v (pi h^2 (3r - h) / 3,
    increasing in h), by bisection."""
    lo = np.zeros_like(v)
    hi = np.full_like(v, radius)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        below = math.pi * mid * mid * (3.0 * radius - mid) / 3.0 < v
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


def _capsule_volume_points(rng, a, b, radius, n):
    """n points inside the capsule a->b, stratified by volume along the axis
    (cap, cylinder, cap), uniform over the disc at each axial position."""
    axis = b - a
    length = float(np.linalg.norm(axis))
    z = axis / length
    tmp = np.array([1.0, 0.0, 0.0]) if abs(z[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    x = np.cross(z, tmp)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    cap = 2.0 * math.pi * radius ** 3 / 3.0
    cyl = math.pi * radius * radius * length
    total = 2.0 * cap + cyl
    v = (np.arange(n) + rng.random(n)) / n * total
    t = np.empty(n)  # axial coordinate from a
    m0 = v < cap
    m2 = v >= cap + cyl
    m1 = ~(m0 | m2)
    t[m0] = -radius + _cap_height(v[m0], radius)
    t[m1] = (v[m1] - cap) / (math.pi * radius * radius)
    t[m2] = length + radius - _cap_height(total - v[m2], radius)
    off = np.clip(np.where(t < 0.0, -t, np.where(t > length, t - length, 0.0)), 0.0, radius)
    disc = np.sqrt(radius * radius - off * off)
    s = disc * np.sqrt(rng.random(n))
    az = rng.random(n) * 2.0 * math.pi
    return a + t[:, None] * z + (s * np.cos(az))[:, None] * x + (s * np.sin(az))[:, None] * y


def make_eval_points(hand: Hand, n_surface: int, n_volume: int, seed: int) -> EvalPoints:
    """Surface and volume samples of the capsule hand for contact area and
    intersection volume (Sec. V-A metrics).

    Each link's capsule gets a share of the samples proportional to its area
    (volume), stratified along its axis; a sample weighs the capsule's area
    (volume) over its share. A surface sample strictly inside another link's
    capsule, and a volume sample strictly inside a lower-numbered link's
    capsule, is dropped, so the weights cover the union of the capsules at
    q = 0 once (collinear links of a straight finger form one capsule)."""
    rng = np.random.default_rng(seed)
    caps = [(c[0:3], c[3:6], float(c[6])) for c in hand.capsules]
    L = len(caps)
    areas = [2 * math.pi * r * np.linalg.norm(b - a) + 4 * math.pi * r * r for a, b, r in caps]
    vols = [math.pi * r * r * np.linalg.norm(b - a) + 4.0 * math.pi * r ** 3 / 3.0 for a, b, r in caps]
    ns = _split_counts(areas, n_surface)
    nv = _split_counts(vols, n_volume) if n_volume > 0 else np.zeros(L, np.int64)
    out = {}
    for kind, counts, size, gen in (("surface", ns, areas, _capsule_points), ("volume", nv, vols, _capsule_volume_points)):
        pts, links, wts = [], [], []
        for l, ((a, b, r), n) in enumerate(zip(caps, counts)):
            if n == 0:
                continue
            p = gen(rng, a, b, r, int(n))
            others = [k for k in range(L) if k != l] if kind == "surface" else list(range(l))
            keep = np.ones(len(p), bool)
            for k in others:
                keep &= _segment_distance(p, caps[k][0], caps[k][1]) >= caps[k][2]
            pts.append(p[keep])
            links.append(np.full(int(keep.sum()), l, np.int32))
            wts.append(np.full(int(keep.sum()), size[l] / n))
        world = np.concatenate(pts) if pts else np.zeros((0, 3))
        link = np.concatenate(links) if links else np.zeros(0, np.int32)
        w = np.concatenate(wts) if wts else np.zeros(0)
        local = np.einsum("nji,nj->ni", hand.link_rest_R[link], world - hand.link_rest_o[link])
        out[kind] = (link, local, w, world)
    s, v = out["surface"], out["volume"]
    return EvalPoints(surface_link=s[0], surface_local=s[1], surface_area=s[2], volume_link=v[0],
                      volume_local=v[1], volume_weight=v[2], surface_rest=s[3], volume_rest=v[3])


# ----------------------------------------------------------------------------
# exact signed distances of primitives (float64), used to fill the grids
# ----------------------------------------------------------------------------
def sphere_sdf(p, center, radius):
    return np.linalg.norm(p - np.asarray(center), axis=-1) - radius


def plane_sdf(p, normal, offset):
    n = np.asarray(normal, dtype=np.float64)
    return p @ (n / np.linalg.norm(n)) - offset


def box_sdf(p, center, rotation, half):
    """Exact SDF of an oriented box; ``rotation`` maps box frame -> world."""
    y = (p - np.asarray(center)) @ np.asarray(rotation)
    q = np.abs(y) - np.asarray(half)
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
    inside = np.minimum(q.max(axis=-1), 0.0)
    return outside + inside


def ellipsoid_sdf(p, center, rotation, semi, iters: int = 16):
    """Exact signed distance to an oriented ellipsoid.

    The closest point follows the classical Lagrange-multiplier reduction to a
    1-D root (Eberly, "Distance from a Point to an Ellipse, an Ellipsoid, or a
    Hyperellipsoid"): in the first octant of the ellipsoid frame the closest
    point is x_i = e_i^2 y_i / (t + e_i^2) with t the unique root of
    F(t) = sum_i (e_i y_i / (t + e_i^2))^2 - 1 on t > -min(e)^2. F is convex and
    decreasing there, so Newton's method started left of the root (where F >= 0)
    increases monotonically to it; a bisection bracket guards the steps.
    """
    e = np.asarray(semi, dtype=np.float64)
    y = np.abs((p - np.asarray(center)) @ np.asarray(rotation))
    y = np.where(y == 0.0, 1e-30, y)
    e2 = e * e
    ey = e * y
    # every t_i = e_i y_i - e_i^2 makes term i equal to 1, so F(t_i) >= 0
    lo = np.max(ey - e2, axis=-1)
    lo = np.maximum(lo, -e2.min() + 1e-300)
    hi = np.maximum(np.sqrt((ey * ey).sum(axis=-1)), lo)
    t = lo.copy()
    for _ in range(iters):
        den = t[..., None] + e2
        rat = ey / den
        Fv = (rat * rat).sum(axis=-1) - 1.0
        dF = -2.0 * (rat * rat / den).sum(axis=-1)
        step = np.where(dF < 0.0, -Fv / dF, 0.0)
        tn = t + step
        # keep inside the bracket [lo, hi]; Newton from the left never passes the root
        lo = np.where(Fv >= 0.0, t, lo)
        hi = np.where(Fv < 0.0, t, hi)
        bad = ~((tn >= lo) & (tn <= hi))
        t_new = np.where(bad, 0.5 * (lo + hi), tn)
        if np.array_equal(t_new, t):
            break
        t = t_new
    x = e2 * y / (t[..., None] + e2)
    dist = np.linalg.norm(x - y, axis=-1)
    inside = ((y / e) ** 2).sum(axis=-1) < 1.0
    return np.where(inside, -dist, dist)


# ----------------------------------------------------------------------------
# objects and grids
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Grid:
    n: int
    lo: np.ndarray        # [3] float64
    h: float
    values: np.ndarray    # [N*N*N] float32, x fastest
    prims: list           # primitive descriptions (for analytic checks)
    bound_radius: float   # max over primitives of |centre| + largest semi-axis

    def vertex_positions(self):
        i = np.arange(self.n) * self.h
        z, y, x = np.meshgrid(i + self.lo[2], i + self.lo[1], i + self.lo[0], indexing="ij")
        return np.stack([x, y, z], axis=-1).reshape(-1, 3)


def make_object(kind: str, seed: int, n_prims: int | None = None,
                n_range=(3, 6), radius: float = 4.0 * CM) -> list:
    """Primitive list for an object.

    kind = "sphere": one sphere of ``radius`` at the origin.
    kind = "ellipsoids": a union of n ellipsoids, semi-axes U[1.5, 5] cm,
    uniform SO(3) orientation, centres U[-2, 2] cm per axis.
    kind = "mixed": the same, each primitive an ellipsoid or a box (half
    extents U[1.5, 5] cm) with equal probability.
    """
    rng = np.random.default_rng(seed)
    if kind == "sphere":
        return [("sphere", np.zeros(3), radius)]
    if n_prims is None:
        n_prims = int(rng.integers(n_range[0], n_range[1] + 1))
    prims = []
    for _ in range(n_prims):
        semi = rng.uniform(1.5 * CM, 5.0 * CM, size=3)
        rot = Rotation.random(random_state=rng.integers(1 << 31)).as_matrix()
        centre = rng.uniform(-2.0 * CM, 2.0 * CM, size=3)
        is_box = kind == "mixed" and rng.random() < 0.5
        prims.append(("box" if is_box else "ellipsoid", centre, rot, semi))
    return prims


def object_sdf(prims, p):
    """Union (minimum) of the primitives' exact signed distances at points p."""
    out = None
    for pr in prims:
        if pr[0] == "sphere":
            d = sphere_sdf(p, pr[1], pr[2])
        elif pr[0] == "box":
            d = box_sdf(p, pr[1], pr[2], pr[3])
        elif pr[0] == "ellipsoid":
            d = ellipsoid_sdf(p, pr[1], pr[2], pr[3])
        elif pr[0] == "plane":
            d = plane_sdf(p, pr[1], pr[2])
        else:
            raise ValueError(pr[0])
        out = d if out is None else np.minimum(out, d)
    return out


def bound_radius(prims) -> float:
    r = 0.0
    for pr in prims:
        if pr[0] == "sphere":
            r = max(r, float(np.linalg.norm(pr[1])) + pr[2])
        elif pr[0] in ("box", "ellipsoid"):
            ext = float(np.max(pr[3])) * (math.sqrt(3.0) if pr[0] == "box" else 1.0)
            r = max(r, float(np.linalg.norm(pr[1])) + ext)
    return r


def make_grid(prims, n: int, margin: float = 2.0 * CM, side: float | None = None,
              lo=None, chunk: int = 1 << 17, device: str | None = None) -> Grid:
    """FP32 vertex-centred SDF grid of the union of ``prims``.

    The cube is centred on the origin with side 2 (R_bound + margin), where
    R_bound is the largest |centre| + semi-axis; a 4 cm sphere gives 12 cm.
    With ``device`` (a torch device) the same FP64 distances are evaluated
    with torch there, which large grids need to be built in seconds.
    """
    rb = bound_radius(prims)
    if side is None:
        side = 2.0 * (rb + margin)
    lo = np.full(3, -0.5 * side) if lo is None else np.asarray(lo, np.float64)
    h = side / (n - 1)
    g = Grid(n=n, lo=lo, h=h, values=np.empty(0, np.float32), prims=prims, bound_radius=rb)
    if device is not None:
        g.values = _grid_values_torch(prims, n, lo, h, device)
        return g
    pos = g.vertex_positions()
    vals = np.empty(pos.shape[0], np.float64)
    for s in range(0, pos.shape[0], chunk):
        vals[s:s + chunk] = object_sdf(prims, pos[s:s + chunk])
    g.values = vals.astype(np.float32)
    return g


def _grid_values_torch(prims, n, lo, h, device, chunk=1 << 22):
    """Vertex values of the union in FP64 with torch (same formulas as the
    numpy path: exact sphere/box distances, ellipsoid by the Newton root)."""
    import torch
    i = torch.arange(n, dtype=torch.float64, device=device) * h
    out = torch.empty(n ** 3, dtype=torch.float64, device=device)
    z, y, x = torch.meshgrid(i + lo[2], i + lo[1], i + lo[0], indexing="ij")
    P = torch.stack([x, y, z], dim=-1).reshape(-1, 3)
    del x, y, z
    for s in range(0, P.shape[0], chunk):
        p = P[s:s + chunk]
        best = None
        for pr in prims:
            if pr[0] == "sphere":
                d = torch.linalg.norm(p - torch.as_tensor(pr[1], device=device), dim=-1) - pr[2]
            elif pr[0] == "box":
                yb = (p - torch.as_tensor(pr[1], device=device)) @ torch.as_tensor(pr[2], device=device)
                q = yb.abs() - torch.as_tensor(pr[3], device=device)
                d = torch.linalg.norm(q.clamp(min=0.0), dim=-1) + q.max(dim=-1).values.clamp(max=0.0)
            else:
                d = _ellipsoid_torch(p, pr[1], pr[2], pr[3], device)
            best = d if best is None else torch.minimum(best, d)
        out[s:s + chunk] = best
    return out.to(torch.float32).cpu().numpy()


def _ellipsoid_torch(p, center, rotation, semi, device, iters=16):
    import torch
    e = torch.as_tensor(semi, dtype=torch.float64, device=device)
    y = ((p - torch.as_tensor(center, device=device)) @ torch.as_tensor(rotation, device=device)).abs()
    y = torch.where(y == 0.0, torch.full_like(y, 1e-30), y)
    e2 = e * e
    ey = e * y
    lo = (ey - e2).max(dim=-1).values
    lo = torch.clamp(lo, min=float(-e2.min()) + 1e-300)
    hi = torch.maximum(torch.sqrt((ey * ey).sum(dim=-1)), lo)
    t = lo.clone()
    for _ in range(iters):
        den = t[:, None] + e2
        rat = ey / den
        Fv = (rat * rat).sum(dim=-1) - 1.0
        dF = -2.0 * (rat * rat / den).sum(dim=-1)
        step = torch.where(dF < 0.0, -Fv / dF, torch.zeros_like(Fv))
        tn = t + step
        lo = torch.where(Fv >= 0.0, t, lo)
        hi = torch.where(Fv < 0.0, t, hi)
        bad = ~((tn >= lo) & (tn <= hi))
        t = torch.where(bad, 0.5 * (lo + hi), tn)
    x = e2 * y / (t[:, None] + e2)
    dist = torch.linalg.norm(x - y, dim=-1)
    inside = ((y / e) ** 2).sum(dim=-1) < 1.0
    return torch.where(inside, -dist, dist)


def random_points(grid: Grid, n: int, seed: int, outside_frac: float = 0.25):
    """Query points for sampler checks: most inside the grid box, some around it."""
    rng = np.random.default_rng(seed)
    side = grid.h * (grid.n - 1)
    n_out = int(n * outside_frac)
    inside = grid.lo + rng.random((n - n_out, 3)) * side
    around = grid.lo - 0.5 * side + rng.random((n_out, 3)) * 2.0 * side
    return np.concatenate([inside, around])


# ----------------------------------------------------------------------------
# candidates (stand-in for approach sampling) and optimizer state
# ----------------------------------------------------------------------------
def make_candidates(hand: Hand, B: int, seed: int, shell_radius: float) -> np.ndarray:
    """Initial configurations q [B][n_dof] (float64).

    The paper samples initial poses with the approach-sampling procedure of its
    prior work (Sec. IV-A), which is not given. Stand-in: the wrist lies
    uniformly on a sphere of ``shell_radius`` around the object, the palm's +z
    axis points at the object centre, the roll about that axis is U[0, 2 pi),
    and finger joints are uniform within their limits. The wrist orientation
    is stored as ZYX Euler angles, R = Rz(q3) Ry(q4) Rx(q5).
    """
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(B, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pos = d * shell_radius
    z = -d
    ref = np.where(np.abs(z[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    x = np.cross(ref, z)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    roll = rng.uniform(0.0, 2.0 * math.pi, size=B)
    c, s = np.cos(roll)[:, None], np.sin(roll)[:, None]
    xr = c * x + s * y
    yr = -s * x + c * y
    R = np.stack([xr, yr, z], axis=2)  # columns = palm axes in the world
    eul = Rotation.from_matrix(R).as_euler("ZYX")
    q = np.zeros((B, hand.n_dof))
    q[:, 0:3] = pos
    q[:, 3:6] = eul
    lo, up = hand.q_low[6:], hand.q_up[6:]
    q[:, 6:] = lo + rng.random((B, hand.n_dof - 6)) * (up - lo)
    return q


def adam_state(B: int, n_dof: int, seed: int, scale: float = 1.0):
    """Random (q, m, v, g) for optimizer-step checks; v > 0."""
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(B, n_dof)) * scale
    m = rng.normal(size=(B, n_dof)) * 0.1
    v = rng.random((B, n_dof)) * 0.01
    g = rng.normal(size=(B, n_dof))
    return q, m, v, g


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------
def config_workload(name: str, seed: int | None = None, B: int | None = None,
                    n: int | None = None, n_contacts: int | None = None, device: str | None = None):
    """(hand, grid, q0) for a named workload, optionally shrunk for tests.

    tiny  : 3 fingers x 3 joints (15 DOF), 512 contacts, 4 cm sphere, 64^3 grid
            over a 12 cm cube, 64 candidates on a 10 cm shell, seed 0.
    diff  : 4 fingers x 4 joints (22 DOF), 2048 contacts, union of 3-6
            ellipsoids on a 128^3 grid, 4096 candidates, seed 1.
    large : 5 fingers x 4 joints (26 DOF), 8192 contacts, union of 8
            ellipsoids/boxes on a 256^3 grid, 65536 candidates, seed 4.
    """
    if name == "tiny":
        s = 0 if seed is None else seed
        hand = make_hand(3, 3, n_contacts or 512, seed=s)
        prims = make_object("sphere", seed=s)
        grid = make_grid(prims, n or 64)
        q = make_candidates(hand, B or 64, seed=s + 100, shell_radius=grid.bound_radius + 6.0 * CM)
    elif name == "diff":
        s = 1 if seed is None else seed
        hand = make_hand(4, 4, n_contacts or 2048, seed=s)
        prims = make_object("ellipsoids", seed=s, n_range=(3, 6))
        grid = make_grid(prims, n or 128, device=device)
        q = make_candidates(hand, B or 4096, seed=s + 100, shell_radius=grid.bound_radius + 6.0 * CM)
    elif name == "large":
        s = 4 if seed is None else seed
        hand = make_hand(5, 4, n_contacts or 8192, seed=s)
        prims = make_object("mixed", seed=s, n_prims=8)
        grid = make_grid(prims, n or 256, device=device)
        q = make_candidates(hand, B or 65536, seed=s + 100, shell_radius=grid.bound_radius + 6.0 * CM)
    else:
        raise ValueError(name)
    return hand, grid, q


def config_eval_points(name: str, hand: Hand) -> EvalPoints:
    """The evaluation samples of a named workload's hand: tiny 1024 + 1024,
    diff 4096 + 4096, large 8192 + 8192 surface + volume samples."""
    n, seed = {"tiny": (1024, 20), "diff": (4096, 21), "large": (8192, 24)}[name]
    return make_eval_points(hand, n, n, seed=seed)


def make_job_stream(n_jobs: int, rate: float, seed: int, B_range=(256, 8192),
                    res_choices=(64, 96, 128, 192, 256), steps: int = 300):
    """Poisson arrivals (mean ``rate`` jobs/s) of grasp jobs with random hands
    and composite-primitive objects. Returns a list of dicts (no geometry is
    built here; callers build hands/grids from the recorded seeds)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
    jobs = []
    for j in range(n_jobs):
        jobs.append(dict(
            arrival=float(t[j]),
            fingers=int(rng.integers(3, 6)),
            joints=4 if rng.random() < 0.5 else 3,
            n_contacts=int(rng.choice([1024, 2048, 4096])),
            res=int(rng.choice(res_choices)),
            B=int(rng.integers(B_range[0], B_range[1] + 1)),
            obj_seed=int(rng.integers(1 << 30)),
            hand_seed=int(rng.integers(1 << 30)),
            steps=steps,
        ))
    return jobs


# ----------------------------------------------------------------------------
# triangle meshes (the mesh object of Sec. III-B)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class TriMesh:
    """A closed triangle mesh, faces counter-clockwise seen from outside,
    with unit vertex normals for the Phong surface."""
    vertices: np.ndarray  # [V][3] float64
    faces: np.ndarray     # [F][3] int32
    normals: np.ndarray   # [V][3] float64

    def bound_radius(self) -> float:
        return float(np.linalg.norm(self.vertices, axis=1).max())


def icosphere(subdivisions: int) -> TriMesh:
    """Unit sphere: an icosahedron whose faces are split in four
    ``subdivisions`` times, new vertices pushed onto the sphere; normals are
    the exact radial directions."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, float) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
             (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdivisions):
        mid = {}

        def midpoint(i, j):
            key = (min(i, j), max(i, j))
            if key not in mid:
                p = verts[i] + verts[j]
                verts.append(p / np.linalg.norm(p))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts)
    return TriMesh(V, np.array(faces, np.int32), V.copy())


def mesh_ellipsoid(semi, rotation=None, center=(0.0, 0.0, 0.0), subdivisions: int = 3) -> TriMesh:
    """An ellipsoid (semi-axes along the rotation's columns) from a scaled
    icosphere; vertex normals are the exact surface normals there."""
    s = icosphere(subdivisions)
    e = np.asarray(semi, float)
    R = np.eye(3) if rotation is None else np.asarray(rotation, float)
    local = s.vertices * e
    n = s.vertices / e  # gradient of sum (x_i / e_i)^2 at the surface point, up to a factor
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return TriMesh(local @ R.T + np.asarray(center, float), s.faces, n @ R.T)


def mesh_box(half, splits: int = 1, center=(0.0, 0.0, 0.0)) -> TriMesh:
    """An axis-aligned box whose six faces are each split into splits x splits
    squares (two triangles each). Vertices inside a face get that face's
    normal; vertices on box edges and corners the normalized mean of the
    normals of the faces they touch."""
    h = np.asarray(half, float)
    verts, index = [], {}

    def vid(p):
        key = tuple(np.round(p, 12))
        if key not in index:
            index[key] = len(verts)
            verts.append(np.array(p, float))
        return index[key]

    faces = []
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            u, w = (axis + 1) % 3, (axis + 2) % 3
            grid = {}
            for a in range(splits + 1):
                for b in range(splits + 1):
                    p = np.zeros(3)
                    p[axis] = sgn * h[axis]
                    p[u] = -h[u] + 2.0 * h[u] * a / splits
                    p[w] = -h[w] + 2.0 * h[w] * b / splits
                    grid[a, b] = vid(p)
            for a in range(splits):
                for b in range(splits):
                    q00, q10, q01, q11 = grid[a, b], grid[a + 1, b], grid[a, b + 1], grid[a + 1, b + 1]
                    # (u, w, axis) is right-handed: u x w = axis direction, so
                    # counter-clockwise in (u, w) faces +axis
                    if sgn > 0:
                        faces += [(q00, q10, q11), (q00, q11, q01)]
                    else:
                        faces += [(q00, q11, q10), (q00, q01, q11)]
    V = np.array(verts)
    N = np.zeros_like(V)
    for i, p in enumerate(V):
        for axis in range(3):
            if abs(abs(p[axis]) - h[axis]) < 1e-12 * h.max():
                N[i, axis] += np.sign(p[axis])
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    return TriMesh(V + np.asarray(center, float), np.array(faces, np.int32), N)


def random_mesh_object(seed: int, n_prims: int = 1, subdivisions: int = 3) -> TriMesh:
    """An ellipsoid mesh of the sizes the grid objects use (semi-axes
    U[1.5, 5] cm, uniform orientation); n_prims > 1 is not a closed union and
    is refused."""
    if n_prims != 1:
        raise ValueError("mesh objects are single closed surfaces")
    rng = np.random.default_rng(seed)
    semi = rng.uniform(1.5 * CM, 5.0 * CM, size=3)
    rot = Rotation.random(random_state=rng.integers(1 << 31)).as_matrix()
    return mesh_ellipsoid(semi, rot, (0.0, 0.0, 0.0), subdivisions)
