"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY. The oracle is the plain reference the GPU grasp
step is checked against. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does. It shares no
code with the GPU library and imports nothing from it.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = [os.path.join(_HERE, "oracle.cpp"), os.path.join(_HERE, "mesh.cpp")]

OBJ_GRID, OBJ_SPHERE, OBJ_PLANE, OBJ_BOX, OBJ_MESH = 0, 1, 2, 3, 4
M_SIMS = 7


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with g++ (C++17, OpenMP)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB_PATH + ".tmp"] + SRC
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Hand(C.Structure):
    _fields_ = [("n_links", C.c_int), ("parent", C.POINTER(C.c_int)),
                ("joint_origin", C.POINTER(C.c_double)), ("joint_axis", C.POINTER(C.c_double)),
                ("q_low", C.POINTER(C.c_double)), ("q_up", C.POINTER(C.c_double)),
                ("n_contacts", C.c_int), ("contact_local", C.POINTER(C.c_double)),
                ("contact_link", C.POINTER(C.c_int))]


class _Obj(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int), ("lo", C.c_double * 3), ("h", C.c_double),
                ("values", C.POINTER(C.c_float)), ("center", C.c_double * 3), ("radius", C.c_double),
                ("half", C.c_double * 3), ("normal", C.c_double * 3), ("offset", C.c_double),
                ("inertia_over_mass", C.c_double), ("fd_normal", C.c_int), ("mesh", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("v0", C.c_double), ("K", C.c_int), ("omega", C.c_double),
                ("r_dil", C.c_double), ("alpha_leak", C.c_double), ("w_stable", C.c_double),
                ("w_pen", C.c_double), ("w_range", C.c_double), ("w_limit", C.c_double),
                ("w_min", C.c_double), ("projection", C.c_int), ("mu", C.c_double)]


@dataclasses.dataclass
class Params:
    """Step parameters (Sec. III-C, Sec. IV-A; unstated values are readings)."""
    dt: float = 1e-3
    v0: float = 1.0
    K: int = 1
    omega: float = 1.0
    r_dil: float = 0.0
    alpha_leak: float = 0.1
    w_stable: float = 1.0
    w_pen: float = 1e4
    w_range: float = 1e-2
    w_limit: float = 1.0
    w_min: float = 1e-8
    projection: int = 0  # 0 averaged corrections, 1 Gauss-Seidel sweep
    mu: float = 0.0      # Coulomb friction coefficient (0: frictionless)

    def _c(self):
        return _Params(self.dt, self.v0, self.K, self.omega, self.r_dil, self.alpha_leak,
                       self.w_stable, self.w_pen, self.w_range, self.w_limit, self.w_min, int(self.projection),
                       float(self.mu))


_lib = None


class _Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int), ("vertices", C.POINTER(C.c_double)), ("normals", C.POINTER(C.c_double)),
                ("n_faces", C.c_int), ("faces", C.POINTER(C.c_int)), ("alpha", C.c_double)]


class Mesh:
    """A closed triangle mesh (outward faces) with unit vertex normals for the
    Phong surface (Sec. III-B), held in FP64 for the oracle."""

    def __init__(self, vertices, faces, normals, alpha: float):
        self.vertices = np.ascontiguousarray(vertices, np.float64).reshape(-1, 3)
        self.faces = np.ascontiguousarray(faces, np.int32).reshape(-1, 3)
        self.normals = np.ascontiguousarray(normals, np.float64).reshape(-1, 3)
        self.alpha = float(alpha)
        self.c = _Mesh(self.vertices.shape[0], _ptr(self.vertices), _ptr(self.normals), self.faces.shape[0],
                       _ptr(self.faces, C.c_int), self.alpha)


def mesh_sdf(mesh: Mesh, r):
    """Phong signed distance and the paper's gradient at points r [n][3], with
    the flat closest point, its face, the flat distance, the medial gap and
    the spread of Phong distances over faces tied at FP32 resolution."""
    r = np.ascontiguousarray(r, np.float64).reshape(-1, 3)
    n = r.shape[0]
    rho, grad, cl = np.zeros(n), np.zeros((n, 3)), np.zeros((n, 3))
    face, flat, gap, spread = np.zeros(n, np.int32), np.zeros(n), np.zeros(n), np.zeros(n)
    _check(lib().oracle_mesh_sdf(C.byref(mesh.c), n, _ptr(r), _ptr(rho), _ptr(grad), _ptr(cl), _ptr(face, C.c_int),
                                 _ptr(flat), _ptr(gap), _ptr(spread)), "oracle_mesh_sdf")
    return {"rho": rho, "grad": grad, "closest": cl, "face": face, "dist_flat": flat, "gap": gap, "spread": spread}


def winding_number(mesh: Mesh, r) -> float:
    r = np.ascontiguousarray(r, np.float64).reshape(3)
    return lib().oracle_winding_number(C.byref(mesh.c), _ptr(r))


def closest_on_triangle(a, b, c, r):
    a, b, c, r = (np.ascontiguousarray(x, np.float64).reshape(3) for x in (a, b, c, r))
    out, bary = np.zeros(3), np.zeros(3)
    _check(lib().oracle_closest_on_triangle(_ptr(a), _ptr(b), _ptr(c), _ptr(r), _ptr(out), _ptr(bary)),
           "oracle_closest_on_triangle")
    return out, bary


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        hp, op, pp = C.POINTER(_Hand), C.POINTER(_Obj), C.POINTER(_Params)
        L.oracle_fk.argtypes = [hp, C.c_int, dp, dp, dp]
        L.oracle_sample.argtypes = [op, C.c_int, dp, dp, dp, dp, dp]
        L.oracle_inertia_over_mass.argtypes = [op]
        L.oracle_inertia_over_mass.restype = C.c_double
        L.oracle_step.argtypes = [hp, op, pp, C.c_int, dp, dp, dp, dp, dp, C.c_int]
        L.oracle_trace.argtypes = [hp, op, pp, dp, dp, dp, dp]
        L.oracle_step_ex.argtypes = [hp, op, pp, C.c_int, dp, dp, dp, dp, C.c_int, ip, C.POINTER(_Flip),
                                     C.c_double, C.c_double, C.c_int, C.POINTER(_Amb), ip, C.c_int]
        L.oracle_fd_grad.argtypes = [hp, op, pp, C.c_int, dp, C.c_double, dp, ip, C.c_int]
        L.oracle_adam.argtypes = [C.c_int, dp, dp, dp, dp, C.c_int, C.c_double, C.c_double,
                                  C.c_double, C.c_double]
        L.oracle_rank.argtypes = [C.c_int, dp, ip]
        L.oracle_evaluate.argtypes = [hp, op, C.c_int, dp, C.POINTER(_Eval), C.c_int, dp, C.c_double, dp, dp,
                                      C.c_int]
        L.oracle_select_top.argtypes = [C.c_int, dp, C.c_int, C.c_int, C.c_int, dp, ip, dp]
        mp = C.POINTER(_Mesh)
        L.oracle_mesh_sdf.argtypes = [mp, C.c_int, dp, dp, dp, dp, ip, dp, dp, dp]
        L.oracle_winding_number.argtypes = [mp, dp]
        L.oracle_winding_number.restype = C.c_double
        L.oracle_closest_on_triangle.argtypes = [dp, dp, dp, dp, dp, dp]
        L.oracle_optimize.argtypes = [hp, op, pp, C.c_int, dp, C.c_int, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, ip, dp,
                                      C.c_int]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


class Hand:
    """Oracle view of a hand (any object with the synth.Hand fields)."""

    def __init__(self, h):
        self.parent = np.ascontiguousarray(h.parent, dtype=np.int32)
        self.joint_origin = _d(h.joint_origin)
        self.joint_axis = _d(h.joint_axis)
        self.q_low = _d(h.q_low)
        self.q_up = _d(h.q_up)
        self.contact_local = _d(h.contact_local)
        self.contact_link = np.ascontiguousarray(h.contact_link, dtype=np.int32)
        self.n_links = int(self.parent.shape[0])
        self.n_dof = 6 + self.n_links - 1
        self.n_contacts = int(self.contact_link.shape[0])
        self.c = _Hand(self.n_links, _ptr(self.parent, C.c_int), _ptr(self.joint_origin),
                       _ptr(self.joint_axis), _ptr(self.q_low), _ptr(self.q_up), self.n_contacts,
                       _ptr(self.contact_local), _ptr(self.contact_link, C.c_int))


class Obj:
    """Oracle view of an object: a grid (synth.Grid) or an analytic shape."""

    def __init__(self, grid=None, kind=OBJ_GRID, center=(0, 0, 0), radius=0.0, half=(0, 0, 0),
                 normal=(0, 0, 1), offset=0.0, inertia_over_mass=0.0, fd_normal=False, mesh=None):
        self.values = None
        self.mesh = mesh  # a Mesh: the Phong signed distance (inertia_over_mass must be given)
        c = _Obj()
        c.kind = OBJ_MESH if mesh is not None else kind
        if mesh is not None:
            c.mesh = C.cast(C.pointer(mesh.c), C.c_void_p)
        if grid is not None:
            self.values = np.ascontiguousarray(grid.values, dtype=np.float32)
            c.kind = OBJ_GRID
            c.n = int(grid.n)
            c.lo = (C.c_double * 3)(*[float(x) for x in grid.lo])
            c.h = float(grid.h)
            c.values = _ptr(self.values, C.c_float)
        c.center = (C.c_double * 3)(*center)
        c.radius = radius
        c.half = (C.c_double * 3)(*half)
        n = np.asarray(normal, dtype=np.float64)
        n = n / np.linalg.norm(n)
        c.normal = (C.c_double * 3)(*n)
        c.offset = offset
        c.inertia_over_mass = inertia_over_mass
        c.fd_normal = int(bool(fd_normal))  # grid: central-difference normal (seven queries)
        self.c = c

    def inertia_over_mass(self) -> float:
        return float(lib().oracle_inertia_over_mass(C.byref(self.c)))


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} failed with code {rc}")


def fk(hand: Hand, q, frames: bool = False):
    q = _d(q).reshape(-1, hand.n_dof)
    B = q.shape[0]
    p = np.zeros((B, hand.n_contacts, 3))
    T = np.zeros((B, hand.n_links, 12)) if frames else None
    _check(lib().oracle_fk(C.byref(hand.c), B, _ptr(q), _ptr(p), _ptr(T)), "oracle_fk")
    return (p, T) if frames else p


def sample(obj: Obj, r, hess: bool = False):
    r = _d(r).reshape(-1, 3)
    n = r.shape[0]
    phi = np.zeros(n)
    g = np.zeros((n, 3))
    H = np.zeros((n, 3, 3)) if hess else None
    margin = np.zeros(n)
    _check(lib().oracle_sample(C.byref(obj.c), n, _ptr(r), _ptr(phi), _ptr(g), _ptr(H), _ptr(margin)),
           "oracle_sample")
    return (phi, g, H, margin) if hess else (phi, g, margin)


def step(hand: Hand, obj: Obj, prm: Params, q, grad: bool = True, margins: bool = False,
         threads: int = 0):
    q = _d(q).reshape(-1, hand.n_dof)
    B = q.shape[0]
    loss = np.zeros(B)
    terms = np.zeros((B, 4))
    g = np.zeros((B, hand.n_dof)) if grad else None
    mg = np.zeros((B, 3)) if margins else None
    pc = prm._c()
    _check(lib().oracle_step(C.byref(hand.c), C.byref(obj.c), C.byref(pc), B, _ptr(q), _ptr(loss),
                             _ptr(terms), _ptr(g), _ptr(mg), threads), "oracle_step")
    out = {"loss": loss, "terms": terms}
    if grad:
        out["grad"] = g
    if margins:
        out["min_abs_d"] = mg[:, 0]
        out["min_face"] = mg[:, 1]
        out["min_face_all"] = mg[:, 2]
    return out


class _Flip(C.Structure):
    _fields_ = [("m", C.c_int), ("k", C.c_int), ("i", C.c_int), ("what", C.c_int)]


class _Amb(C.Structure):
    _fields_ = [("m", C.c_int), ("k", C.c_int), ("i", C.c_int), ("what", C.c_int), ("margin", C.c_double),
                ("penetrating", C.c_int)]


def step_ex(hand: Hand, obj: Obj, prm: Params, q, flips=(), kink_d: float = -1.0, kink_face: float = -1.0,
            max_amb: int = 0, grad: bool = True, threads: int = 0):
    """oracle_step with readings of ambiguous samples and their report.
    flips: (b, m, k, i, what) tuples, what 0 = the other side of d = 0, 1..3 =
    the other cell along x, y, z, 4 = the other side of the friction cone,
    5 = the other side of the friction floor. With max_amb > 0, "amb" lists
    per candidate the first max_amb samples (m, k, i, what, margin,
    penetrating) within kink_d of d = 0, of mu C or of the friction floor, or
    kink_face cell units of a cell face, and "n_amb" their full counts."""
    q = _d(q).reshape(-1, hand.n_dof)
    B = q.shape[0]
    loss = np.zeros(B)
    terms = np.zeros((B, 4))
    g = np.zeros((B, hand.n_dof)) if grad else None
    nf = len(flips)
    fb = np.array([f[0] for f in flips], np.int32) if nf else None
    farr = (_Flip * max(nf, 1))(*[_Flip(int(f[1]), int(f[2]), int(f[3]), int(f[4])) for f in flips])
    amb = (_Amb * max(B * max_amb, 1))()
    namb = np.zeros(B, np.int32)
    pc = prm._c()
    _check(lib().oracle_step_ex(C.byref(hand.c), C.byref(obj.c), C.byref(pc), B, _ptr(q), _ptr(loss), _ptr(terms),
                                _ptr(g), nf, _ptr(fb, C.c_int), farr, float(kink_d), float(kink_face), int(max_amb),
                                amb if max_amb > 0 else None, _ptr(namb, C.c_int), threads), "oracle_step_ex")
    out = {"loss": loss, "terms": terms, "n_amb": namb}
    if grad:
        out["grad"] = g
    if max_amb > 0:
        out["amb"] = [[(a.m, a.k, a.i, a.what, a.margin, a.penetrating)
                       for a in amb[b * max_amb:b * max_amb + min(int(namb[b]), max_amb)]] for b in range(B)]
    return out


def trace(hand: Hand, obj: Obj, prm: Params, q, samples: bool = True):
    q = _d(q).reshape(hand.n_dof)
    poses = np.zeros((M_SIMS, prm.K + 1, 6))
    smp = np.zeros((M_SIMS, prm.K, hand.n_contacts, 6)) if samples else None
    p = np.zeros((hand.n_contacts, 3))
    pc = prm._c()
    _check(lib().oracle_trace(C.byref(hand.c), C.byref(obj.c), C.byref(pc), _ptr(q), _ptr(poses),
                              _ptr(smp), _ptr(p)), "oracle_trace")
    return {"poses": poses, "samples": smp, "p": p}


def fd_grad(hand: Hand, obj: Obj, prm: Params, q, h: float = 1e-4, threads: int = 0):
    q = _d(q).reshape(-1, hand.n_dof)
    B = q.shape[0]
    g = np.zeros((B, hand.n_dof))
    ex = np.zeros((B, hand.n_dof), np.int32)
    pc = prm._c()
    _check(lib().oracle_fd_grad(C.byref(hand.c), C.byref(obj.c), C.byref(pc), B, _ptr(q), h, _ptr(g),
                                _ptr(ex, C.c_int), threads), "oracle_fd_grad")
    return g, ex.astype(bool)


def adam(q, m, v, g, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    q, m, v, g = (_d(a).copy() for a in (q, m, v, g))
    _check(lib().oracle_adam(q.size, _ptr(q), _ptr(m), _ptr(v), _ptr(g), t, lr, b1, b2, eps), "oracle_adam")
    return q, m, v


def rank(loss):
    loss = _d(loss)
    r = np.zeros(loss.shape[0], np.int32)
    _check(lib().oracle_rank(loss.shape[0], _ptr(loss), _ptr(r, C.c_int)), "oracle_rank")
    return r


class _Eval(C.Structure):
    _fields_ = [("n_surface", C.c_int), ("surface_link", C.POINTER(C.c_int)),
                ("surface_local", C.POINTER(C.c_double)), ("surface_area", C.POINTER(C.c_double)),
                ("n_volume", C.c_int), ("volume_link", C.POINTER(C.c_int)),
                ("volume_local", C.POINTER(C.c_double)), ("volume_weight", C.POINTER(C.c_double))]


class EvalPoints:
    """Oracle view of weighted hand samples (any object with the
    synth.EvalPoints fields)."""

    def __init__(self, e):
        self.sl = np.ascontiguousarray(e.surface_link, dtype=np.int32)
        self.sp = _d(e.surface_local).reshape(-1, 3)
        self.sa = _d(e.surface_area)
        self.vl = np.ascontiguousarray(e.volume_link, dtype=np.int32)
        self.vp = _d(e.volume_local).reshape(-1, 3)
        self.vw = _d(e.volume_weight)
        self.c = _Eval(self.sl.shape[0], _ptr(self.sl, C.c_int), _ptr(self.sp), _ptr(self.sa),
                       self.vl.shape[0], _ptr(self.vl, C.c_int), _ptr(self.vp), _ptr(self.vw))


def evaluate(hand: Hand, obj: Obj, q, ev: EvalPoints, thresholds, delta: float = 0.0, threads: int = 0):
    """Contact area at each threshold and intersection volume [B][T + 1], and
    the weight of samples within delta of each threshold [B][T + 1]."""
    q = _d(q).reshape(-1, hand.n_dof)
    thr = _d(thresholds).reshape(-1)
    B, M = q.shape[0], thr.shape[0] + 1
    out, slack = np.zeros((B, M)), np.zeros((B, M))
    _check(lib().oracle_evaluate(C.byref(hand.c), C.byref(obj.c), B, _ptr(q), C.byref(ev.c), thr.shape[0],
                                 _ptr(thr), delta, _ptr(out), _ptr(slack), threads), "oracle_evaluate")
    return out, slack


def evaluate_mesh(hand, mesh: Mesh, q, ev, thresholds):
    """Contact area at each threshold and intersection volume [B][T + 1]
    against a mesh object's Phong signed distance (Sec. III-B, Sec. V-A),
    from the same weighted samples: placed by the oracle's forward kinematics
    (each sample set as the contact set of the hand) and queried through
    mesh_sdf. Also the per-sample query outputs [B][N] of both sets ("surface",
    "volume": rho, gap, spread, dist_flat) for tolerances. A configuration
    with a non-finite coordinate gets NaN."""
    import types
    q = _d(q).reshape(-1, 6 + len(hand.parent) - 1)
    thr = _d(thresholds).reshape(-1)
    B = q.shape[0]
    out = np.zeros((B, thr.shape[0] + 1))
    per = {}
    for kind, link, local, w in (("surface", ev.surface_link, ev.surface_local, ev.surface_area),
                                 ("volume", ev.volume_link, ev.volume_local, ev.volume_weight)):
        w = _d(w)
        n = w.shape[0]
        if n == 0:
            per[kind] = {k: np.zeros((B, 0)) for k in ("rho", "gap", "spread", "dist_flat")}
            continue
        view = types.SimpleNamespace(parent=hand.parent, joint_origin=hand.joint_origin, joint_axis=hand.joint_axis,
                                     q_low=hand.q_low, q_up=hand.q_up, contact_local=local, contact_link=link)
        p = fk(Hand(view), np.nan_to_num(q))
        res = mesh_sdf(mesh, p.reshape(-1, 3))
        per[kind] = {k: res[k].reshape(B, n) for k in ("rho", "gap", "spread", "dist_flat")}
        rho = per[kind]["rho"]
        if kind == "surface":
            for t, tau in enumerate(thr):
                out[:, t] = ((rho < tau) * w).sum(axis=1)
        else:
            out[:, -1] = ((rho < 0.0) * w).sum(axis=1)
    out[~np.isfinite(q).all(axis=1)] = np.nan
    return out, per


def select_top(key, k: int, higher_is_better: bool = False, metrics=None):
    """Indices of the k best keys (NaN last, ties by index) and the mean of
    metrics [B][M] over them."""
    key = _d(key).reshape(-1)
    B = key.shape[0]
    met = _d(np.zeros((B, 0)) if metrics is None else metrics).reshape(B, -1)
    top = np.zeros(k, np.int32)
    mean = np.zeros(met.shape[1])
    _check(lib().oracle_select_top(B, _ptr(key), int(higher_is_better), k, met.shape[1], _ptr(met),
                                   _ptr(top, C.c_int), _ptr(mean)), "oracle_select_top")
    return top, mean


def optimize(hand: Hand, obj: Obj, prm: Params, q0, T: int, r0: float = 0.01, lr=1e-3, b1=0.9,
             b2=0.999, eps=1e-8, use_gd=False, history=False, threads: int = 0):
    q = _d(q0).reshape(-1, hand.n_dof).copy()
    B = q.shape[0]
    fl = np.zeros(B)
    ft = np.zeros((B, 4))
    rk = np.zeros(B, np.int32)
    hist = np.zeros((T, B)) if history else None
    pc = prm._c()
    _check(lib().oracle_optimize(C.byref(hand.c), C.byref(obj.c), C.byref(pc), B, _ptr(q), T, r0, lr, b1,
                                 b2, eps, int(use_gd), _ptr(fl), _ptr(ft), _ptr(rk, C.c_int), _ptr(hist),
                                 threads), "oracle_optimize")
    out = {"q": q, "loss": fl, "terms": ft, "rank": rk}
    if history:
        out["history"] = hist
    return out
