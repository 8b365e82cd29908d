"""Python front end of the grasp library: contexts, resident hands and SDF
grids, the step calls on torch tensors, and a torch.autograd.Function.

PyTorch supplies device memory and streams only; every computation runs in
the HIP kernels of libgrasp.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import (BatchJobC, EvalDescC, HandDesc, JobDescC, JobResultC, Library, MeshDescC, MeshGridDescC, SdfDesc,
                   ServeStatsC, StepParams,
                   TileC, GRASP_EAGAIN, MODE_AUTO, MODE_RECOMPUTE, MODE_SAVE, GraspError)

__all__ = ["Context", "Hand", "Sdf", "StepParams", "GraspStep", "GraspError", "Batch", "BatchJob",
           "MODE_AUTO", "MODE_SAVE", "MODE_RECOMPUTE"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Context:
    """A grasp context on one GPU; its arena is a torch uint8 tensor."""

    def __init__(self, device: int = 0, arena_bytes: int = 1 << 30, arena: torch.Tensor | None = None):
        self.lib = Library.get()
        self.device = device
        if arena is None:
            arena = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        self.arena = arena
        h = C.c_void_p()
        self.lib.call("grasp_init", device, C.c_void_p(arena.data_ptr()), arena.numel(), C.byref(h))
        self.h = h
        self._ws = None

    def close(self):
        if self.h:
            self.lib.grasp_shutdown(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- resident objects ---------------------------------------------------
    def hand(self, hand) -> "Hand":
        return Hand(self, hand)

    def sdf(self, grid, inertia_over_mass: float = 0.0, layout: int = 0) -> "Sdf":
        return Sdf(self, grid, inertia_over_mass, layout)

    def mesh(self, mesh, alpha: float, normals: bool = True) -> "Mesh":
        return Mesh(self, mesh, alpha, normals)

    def eval_points(self, hand: "Hand", points) -> "EvalPoints":
        return EvalPoints(self, hand, points)

    # -- post-synthesis evaluation (Sec. V-A metrics) -------------------------
    def evaluate(self, ev: "EvalPoints", sdf, q, thresholds, out=None, stream=None):
        """[B][T + 1]: contact area at each threshold (m), then intersection volume."""
        thr = np.ascontiguousarray(thresholds, np.float32).reshape(-1)
        if out is None:
            out = torch.empty((q.shape[0], thr.shape[0] + 1), dtype=torch.float32, device=q.device)
        self.lib.call("grasp_evaluate", self.h, ev.id, sdf.id, q.shape[0], _ptr(q), thr.shape[0],
                      thr.ctypes.data_as(C.POINTER(C.c_float)), _ptr(out), _stream(stream))
        return out

    def evaluate_mesh(self, ev: "EvalPoints", mesh: "Mesh", q, thresholds, out=None, stream=None):
        """As evaluate, against a mesh object's Phong signed distance."""
        thr = np.ascontiguousarray(thresholds, np.float32).reshape(-1)
        if out is None:
            out = torch.empty((q.shape[0], thr.shape[0] + 1), dtype=torch.float32, device=q.device)
        self.lib.call("grasp_evaluate_mesh", self.h, ev.id, mesh.id, q.shape[0], _ptr(q), thr.shape[0],
                      thr.ctypes.data_as(C.POINTER(C.c_float)), _ptr(out), _stream(stream))
        return out

    def select_top(self, key, k: int, higher_is_better: bool = False, metrics=None, stream=None):
        """(indices [k] best first, mean of metrics [B][M] over them or None)."""
        top = torch.empty(k, dtype=torch.int32, device=key.device)
        M = 0 if metrics is None else metrics.shape[1]
        mean = torch.empty(M, dtype=torch.float32, device=key.device) if M else None
        self.lib.call("grasp_select_top", self.h, key.shape[0], _ptr(key), int(higher_is_better), k, M,
                      _ptr(metrics) if M else None, _ptr(top), _ptr(mean), _stream(stream))
        return top, mean

    # -- steps -----------------------------------------------------------------
    def workspace_bytes(self, hand, sdf, prm: StepParams, B: int) -> int:
        out = C.c_size_t()
        pc = prm.c()
        self.lib.call("grasp_step_workspace_bytes", self.h, hand.id, sdf.id, C.byref(pc), B, C.byref(out))
        return out.value

    def step_fwd(self, hand, sdf, prm: StepParams, q, loss, terms=None, ws=None, stream=None):
        pc = prm.c()
        nbytes = 0 if ws is None else ws.numel() * ws.element_size()
        self.lib.call("grasp_step_fwd", self.h, hand.id, sdf.id, C.byref(pc), q.shape[0], _ptr(q), _ptr(loss),
                      _ptr(terms), _ptr(ws), nbytes, _stream(stream))

    def step_bwd(self, hand, sdf, prm: StepParams, q, dq, dloss=None, ws=None, stream=None):
        pc = prm.c()
        nbytes = 0 if ws is None else ws.numel() * ws.element_size()
        self.lib.call("grasp_step_bwd", self.h, hand.id, sdf.id, C.byref(pc), q.shape[0], _ptr(q), _ptr(dloss),
                      _ptr(dq), _ptr(ws), nbytes, _stream(stream))

    def adam(self, q, m, v, g, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.lib.call("grasp_adam_step", self.h, q.numel(), _ptr(q), _ptr(m), _ptr(v), _ptr(g), t, lr, b1, b2, eps,
                      _stream(stream))

    def step_fused(self, hand, sdf, prm: StepParams, q, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8,
                   loss=None, terms=None, dq=None, stream=None):
        pc = prm.c()
        self.lib.call("grasp_step_fused", self.h, hand.id, sdf.id, C.byref(pc), q.shape[0], _ptr(q), _ptr(m),
                      _ptr(v), t, lr, b1, b2, eps, _ptr(loss), _ptr(terms), _ptr(dq), _stream(stream))

    def step_fused_mesh(self, hand, mesh, prm: StepParams, q, m, v, t: int, inertia_over_mass: float = 0.0, lr=1e-3,
                        b1=0.9, b2=0.999, eps=1e-8, loss=None, terms=None, dq=None, stream=None):
        """grasp_step_fused_mesh: the fused step with the mesh's Phong signed
        distance sampled at every contact (inertia_over_mass <= 0: from the
        mesh's volume)."""
        pc = prm.c()
        self.lib.call("grasp_step_fused_mesh", self.h, hand.id, mesh.id, C.byref(pc), float(inertia_over_mass),
                      q.shape[0], _ptr(q), _ptr(m), _ptr(v), t, lr, b1, b2, eps, _ptr(loss), _ptr(terms), _ptr(dq),
                      _stream(stream))

    def step_fused_static(self, hand, sdf, prm: StepParams, q, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8,
                          loss=None, terms=None, dq=None, stream=None):
        """grasp_step_fused_static: the fused step with no allocation (its
        candidate order in the library's fixed device array; B <= 262144)."""
        pc = prm.c()
        self.lib.call("grasp_step_fused_static", self.h, hand.id, sdf.id, C.byref(pc), q.shape[0], _ptr(q),
                      _ptr(m), _ptr(v), t, lr, b1, b2, eps, _ptr(loss), _ptr(terms), _ptr(dq), _stream(stream))

    def plain_workspace_bytes(self, hand, sdf, prm: StepParams, B: int) -> int:
        out = C.c_size_t()
        pc = prm.c()
        self.lib.call("grasp_plain_workspace_bytes", self.h, hand.id, sdf.id, C.byref(pc), B, C.byref(out))
        return out.value

    def plain_workspace(self, hand, sdf, prm: StepParams, B: int) -> torch.Tensor:
        return torch.empty(self.plain_workspace_bytes(hand, sdf, prm, B), dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    def plain_step(self, hand, sdf, prm: StepParams, q, m, v, t: int, ws, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8,
                   loss=None, terms=None, stream=None):
        """The unfused per-job form: loss at q, then Adam on q, m, v in place."""
        pc = prm.c()
        self.lib.call("grasp_plain_step", self.h, hand.id, sdf.id, C.byref(pc), q.shape[0], _ptr(q), _ptr(m),
                      _ptr(v), t, lr, b1, b2, eps, _ptr(loss), _ptr(terms), _ptr(ws), ws.numel(), _stream(stream))

    def tune(self, hand, sdf, prm: StepParams, q, reps: int = 3):
        """Times every launch tile on a copy of q; returns ((wpb, occ), ms per step)."""
        pc = prm.c()
        best = TileC()
        ms = C.c_float()
        self.lib.call("grasp_tune", self.h, hand.id, sdf.id, C.byref(pc), q.shape[0], _ptr(q), reps, C.byref(best),
                      C.byref(ms))
        return (best.waves_per_block, best.min_waves_per_simd), ms.value

    def set_tile(self, hand, sdf, prm: StepParams, B: int, wpb: int, occ: int):
        pc = prm.c()
        t = TileC(wpb, occ)
        self.lib.call("grasp_set_tile", self.h, hand.id, sdf.id, C.byref(pc), B, C.byref(t))

    # -- serving ---------------------------------------------------------------
    def serve_config(self, capacity: int = 65536, max_jobs: int = 256):
        self.lib.call("grasp_serve_config", self.h, capacity, max_jobs)

    def submit(self, hand, sdf, q0, T: int, r0: float = 0.01, prm: StepParams | None = None, lr=1e-3, b1=0.9,
               b2=0.999, eps=1e-8, eval_points=None, thresholds=(), top_k: int = 0, record_history: bool = False) -> int:
        """Queues a grasp job (host q0 [B][n_dof]); returns its id. With an
        evaluation set the job retires with its metrics at the given
        thresholds and, with top_k, the best candidates and their means.
        record_history keeps q before and the loss at every step."""
        q0 = _f32(q0)
        prm = prm or StepParams()
        thr = [float(x) for x in thresholds]
        d = JobDescC(hand.id, sdf.id, q0.shape[0], q0.ctypes.data, T, r0, prm.c(), lr, b1, b2, eps,
                     eval_points.id if eval_points is not None else 0, len(thr),
                     (C.c_float * 8)(*(thr + [0.0] * (8 - len(thr)))[:8]), top_k, int(record_history))
        out = C.c_uint64()
        self.lib.call("grasp_submit", self.h, C.byref(d), C.byref(out))
        return out.value

    def poll(self, job: int, B: int, n_dof: int, n_metrics: int = 0, top_k: int = 0, T: int = 0):
        """None while the job runs; then a dict of its results (status, q, loss, terms, rank, times, and
        for jobs with an evaluation set: metrics [B][n_metrics], top [top_k], top_mean [n_metrics]; with
        T > 0, for a job that recorded its history, hist_q [steps][B][n_dof] and hist_loss [steps][B])."""
        q = np.zeros((B, n_dof), np.float32)
        loss = np.zeros(B, np.float32)
        terms = np.zeros((B, 4), np.float32)
        rank = np.zeros(B, np.int32)
        met = np.zeros((B, n_metrics), np.float32) if n_metrics else None
        top = np.zeros(top_k, np.int32) if top_k else None
        mean = np.zeros(n_metrics, np.float32) if top_k else None
        hq = np.zeros((T, B, n_dof), np.float32) if T else None
        hl = np.zeros((T, B), np.float32) if T else None
        ptr = lambda a: None if a is None else a.ctypes.data
        r = JobResultC(0, q.ctypes.data, loss.ctypes.data, terms.ctypes.data, rank.ctypes.data, 0, 0, 0, 0,
                       ptr(met), ptr(top), ptr(mean), ptr(hq), ptr(hl))
        code = self.lib.grasp_poll(self.h, job, C.byref(r))
        if code == GRASP_EAGAIN:
            return None
        if code not in (0, -6, -7):
            self.lib.check(code, "grasp_poll")
        return {"status": r.status, "q": q, "loss": loss, "terms": terms, "rank": rank, "t_submit": r.t_submit,
                "t_admit": r.t_admit, "t_done": r.t_done, "steps": r.steps, "metrics": met, "top": top,
                "top_mean": mean, "hist_q": None if hq is None else hq[:r.steps],
                "hist_loss": None if hl is None else hl[:r.steps]}

    def cancel(self, job: int):
        self.lib.call("grasp_cancel", self.h, job)

    def serve_stats(self) -> dict:
        st = ServeStatsC()
        self.lib.call("grasp_serve_stats_get", self.h, C.byref(st))
        return {"steps": st.steps, "contact_evals": st.contact_evals, "queued": st.queued,
                "resident": st.resident, "finished": st.finished}

    def debug_sdf_sample(self, sdf, r, hess: bool = False, stream=None):
        n = r.shape[0]
        out = torch.empty((n, 4), dtype=torch.float32, device=r.device)
        H = torch.empty((n, 9), dtype=torch.float32, device=r.device) if hess else None
        self.lib.call("grasp_debug_sdf_sample", self.h, sdf.id, n, _ptr(r), _ptr(out), _ptr(H), _stream(stream))
        return (out, H) if hess else out

    def debug_trace(self, hand, sdf, prm: StepParams, q, p_world=True, poses=True, samples=True, stream=None):
        B, dev = q.shape[0], q.device
        pw = torch.empty((B, hand.n_contacts, 3), dtype=torch.float32, device=dev) if p_world else None
        ps = torch.empty((B, 7, prm.K + 1, 6), dtype=torch.float32, device=dev) if poses else None
        sm = torch.empty((B, 7, prm.K, hand.n_contacts, 6), dtype=torch.float32, device=dev) if samples else None
        pc = prm.c()
        self.lib.call("grasp_debug_trace", self.h, hand.id, sdf.id, C.byref(pc), B, _ptr(q), _ptr(pw), _ptr(ps),
                      _ptr(sm), _stream(stream))
        return {"p": pw, "poses": ps, "samples": sm}

    def debug_trace_mesh(self, hand, mesh, prm: StepParams, q, inertia_over_mass: float = 0.0, stream=None):
        """The mesh step's forward with its trace (as debug_trace)."""
        B, dev = q.shape[0], q.device
        pw = torch.empty((B, hand.n_contacts, 3), dtype=torch.float32, device=dev)
        ps = torch.empty((B, 7, prm.K + 1, 6), dtype=torch.float32, device=dev)
        sm = torch.empty((B, 7, prm.K, hand.n_contacts, 6), dtype=torch.float32, device=dev)
        pc = prm.c()
        self.lib.call("grasp_debug_trace_mesh", self.h, hand.id, mesh.id, C.byref(pc), float(inertia_over_mass), B,
                      _ptr(q), _ptr(pw), _ptr(ps), _ptr(sm), _stream(stream))
        return {"p": pw, "poses": ps, "samples": sm}

    def debug_forward_groups(self, hand, sdf, prm: StepParams, q, stream=None):
        """(groups gathered, groups) over the forward passes of one fused step at q."""
        cnt = torch.zeros(2, dtype=torch.int64, device=q.device)
        pc = prm.c()
        self.lib.call("grasp_debug_forward_groups", self.h, hand.id, sdf.id, C.byref(pc), q.shape[0], _ptr(q),
                      _ptr(cnt), _stream(stream))
        g = cnt.cpu()
        return int(g[0]), int(g[1])


class Hand:
    """A hand resident in a context (grasp_create_hand)."""

    def __init__(self, ctx: Context, hand):
        self.ctx = ctx
        parent = _i32(hand.parent)
        origin = _f32(hand.joint_origin)
        axis = _f32(hand.joint_axis)
        lo, up = _f32(hand.q_low), _f32(hand.q_up)
        cl, lk = _f32(hand.contact_local), _i32(hand.contact_link)
        fp, ip = C.POINTER(C.c_float), C.POINTER(C.c_int32)
        d = HandDesc(parent.shape[0], parent.ctypes.data_as(ip), origin.ctypes.data_as(fp),
                     axis.ctypes.data_as(fp), lo.ctypes.data_as(fp), up.ctypes.data_as(fp), lk.shape[0],
                     cl.ctypes.data_as(fp), lk.ctypes.data_as(ip))
        hid = C.c_uint64()
        ctx.lib.call("grasp_create_hand", ctx.h, C.byref(d), C.byref(hid))
        self.id = hid.value
        self.n_links = int(parent.shape[0])
        self.n_dof = 6 + self.n_links - 1
        self.n_contacts = int(lk.shape[0])

    def contact_links(self) -> np.ndarray:
        out = np.zeros(self.n_contacts, np.int32)
        self.ctx.lib.call("grasp_hand_contact_links", self.ctx.h, self.id, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out

    def destroy(self):
        self.ctx.lib.call("grasp_destroy_hand", self.ctx.h, self.id)


class Sdf:
    """An SDF grid resident in a context (grasp_load_sdf)."""

    def __init__(self, ctx: Context, grid, inertia_over_mass: float = 0.0, layout: int = 0):
        self.ctx = ctx
        vals = _f32(grid.values)
        d = SdfDesc(int(grid.n), (C.c_float * 3)(*[float(x) for x in grid.lo]), float(grid.h),
                    vals.ctypes.data_as(C.POINTER(C.c_float)), float(inertia_over_mass), int(layout))
        sid = C.c_uint64()
        ctx.lib.call("grasp_load_sdf", ctx.h, C.byref(d), C.byref(sid))
        self.id = sid.value
        self.n = int(grid.n)

    @classmethod
    def resident(cls, ctx: Context, sid: int, n: int) -> "Sdf":
        """A grid the library already holds (e.g. built from a mesh)."""
        s = cls.__new__(cls)
        s.ctx, s.id, s.n = ctx, sid, n
        return s

    def inertia_over_mass(self) -> float:
        out = C.c_float()
        self.ctx.lib.call("grasp_sdf_inertia", self.ctx.h, self.id, C.byref(out))
        return out.value

    def unload(self):
        self.ctx.lib.call("grasp_unload_sdf", self.ctx.h, self.id)


class Mesh:
    """A closed triangle mesh resident in a context (grasp_load_mesh): its
    Phong signed distance (Sec. III-B) on the device."""

    def __init__(self, ctx: Context, mesh, alpha: float, normals: bool = True):
        self.ctx = ctx
        self._v = _f32(mesh.vertices)
        self._n = _f32(mesh.normals) if normals else None
        self._f = np.ascontiguousarray(mesh.faces, np.int32)
        fp = C.POINTER(C.c_float)
        d = MeshDescC(self._v.shape[0], self._v.ctypes.data_as(fp),
                      self._n.ctypes.data_as(fp) if self._n is not None else None, self._f.shape[0],
                      self._f.ctypes.data_as(C.POINTER(C.c_int32)), float(alpha))
        mid = C.c_uint64()
        ctx.lib.call("grasp_load_mesh", ctx.h, C.byref(d), C.byref(mid))
        self.id = mid.value

    def sample(self, r, stream=None):
        """(rho, grad rho) [n][4] at device points r [n][3]."""
        out = torch.empty((r.shape[0], 4), dtype=torch.float32, device=r.device)
        self.ctx.lib.call("grasp_mesh_sample", self.ctx.h, self.id, r.shape[0], _ptr(r), _ptr(out), _stream(stream))
        return out

    def step_sample(self, r, stream=None):
        """(rho, stated normal, exact gradient of rho, region) [n][8] at device
        points r [n][3]: the sample the mesh step takes."""
        out = torch.empty((r.shape[0], 8), dtype=torch.float32, device=r.device)
        self.ctx.lib.call("grasp_debug_mesh_step_sample", self.ctx.h, self.id, r.shape[0], _ptr(r), _ptr(out),
                          _stream(stream))
        return out

    def grid(self, n: int, lo, h: float, layout: int = 0, inertia_over_mass: float = 0.0) -> "Sdf":
        """An SDF grid of the Phong distance sampled on the device at n^3 vertices."""
        d = MeshGridDescC(int(n), (C.c_float * 3)(*[float(x) for x in lo]), float(h), float(inertia_over_mass),
                          int(layout))
        sid = C.c_uint64()
        self.ctx.lib.call("grasp_load_sdf_from_mesh", self.ctx.h, self.id, C.byref(d), C.byref(sid))
        return Sdf.resident(self.ctx, sid.value, int(n))

    def unload(self):
        self.ctx.lib.call("grasp_unload_mesh", self.ctx.h, self.id)


class EvalPoints:
    """A hand's weighted surface and volume samples resident in a context
    (grasp_load_eval_points)."""

    def __init__(self, ctx: Context, hand: Hand, points):
        self.ctx = ctx
        sl, sp, sa = _i32(points.surface_link), _f32(points.surface_local), _f32(points.surface_area)
        vl, vp, vw = _i32(points.volume_link), _f32(points.volume_local), _f32(points.volume_weight)
        fp, ip = C.POINTER(C.c_float), C.POINTER(C.c_int32)
        d = EvalDescC(sl.shape[0], sl.ctypes.data_as(ip), sp.ctypes.data_as(fp), sa.ctypes.data_as(fp),
                      vl.shape[0], vl.ctypes.data_as(ip), vp.ctypes.data_as(fp), vw.ctypes.data_as(fp))
        eid = C.c_uint64()
        ctx.lib.call("grasp_load_eval_points", ctx.h, hand.id, C.byref(d), C.byref(eid))
        self.id = eid.value

    def unload(self):
        self.ctx.lib.call("grasp_unload_eval_points", self.ctx.h, self.id)


class GraspStep(torch.autograd.Function):
    """loss = GraspStep.apply(q, ctx, hand, sdf, params[, ws_budget]): the grasp
    loss of each candidate (grasp_step_fwd); backward is the hand-written
    adjoint (grasp_step_bwd). In SAVE mode a workspace tensor carries the pose
    checkpoints from forward to backward; RECOMPUTE needs none and the
    backward recomputes FK and the samples. AUTO saves only when the workspace
    fits ws_budget bytes (default: half of the device's free memory), so a
    batch too large for memory recomputes instead of failing."""

    @staticmethod
    def forward(fctx, q, ctx: Context, hand: Hand, sdf: Sdf, prm: StepParams, ws_budget=None):
        q = q.detach().contiguous()
        if q.dtype != torch.float32 or q.dim() != 2 or q.shape[1] != hand.n_dof:
            raise ValueError("q must be float32 [B][n_dof]")
        B = q.shape[0]
        loss = torch.empty(B, dtype=torch.float32, device=q.device)
        ws = None
        if prm.mode != MODE_RECOMPUTE:
            nb = ctx.workspace_bytes(hand, sdf, prm, B)
            if prm.mode == MODE_AUTO:
                budget = ws_budget if ws_budget is not None else torch.cuda.mem_get_info(q.device)[0] // 2
                if nb > budget:
                    nb = -1  # recompute in the backward
            if nb >= 0:
                ws = torch.empty(max(nb, 4), dtype=torch.uint8, device=q.device)
        ctx.step_fwd(hand, sdf, prm, q, loss, ws=ws)
        fctx.save_for_backward(q)
        fctx.extra = (ctx, hand, sdf, prm, ws)
        return loss

    @staticmethod
    def backward(fctx, dloss):
        (q,) = fctx.saved_tensors
        ctx, hand, sdf, prm, ws = fctx.extra
        dq = torch.empty_like(q)
        ctx.step_bwd(hand, sdf, prm, q, dq, dloss=dloss.contiguous().to(torch.float32), ws=ws)
        return dq, None, None, None, None, None


class BatchJob:
    """One job of a batched step: its resident hand and grid, parameters,
    device tensors q, m, v (updated in place) and schedule position."""

    def __init__(self, hand: Hand, sdf: Sdf, prm: StepParams, q, m=None, v=None, loss=None, terms=None,
                 t: int = 0, T: int = 300, r0: float = 0.01, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, dq=None):
        self.hand, self.sdf, self.prm = hand, sdf, prm
        self.q = q
        self.m = torch.zeros_like(q) if m is None else m
        self.v = torch.zeros_like(q) if v is None else v
        self.loss = torch.empty(q.shape[0], dtype=torch.float32, device=q.device) if loss is None else loss
        self.terms = terms
        self.dq = dq
        self.t, self.T, self.r0 = t, T, r0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def c(self) -> BatchJobC:
        return BatchJobC(self.hand.id, self.sdf.id, self.prm.c(), self.q.shape[0], self.q.data_ptr(),
                         self.m.data_ptr(), self.v.data_ptr(), self.loss.data_ptr(),
                         None if self.terms is None else self.terms.data_ptr(),
                         None if self.dq is None else self.dq.data_ptr(), self.t, self.T, self.r0,
                         self.lr, self.b1, self.b2, self.eps)


class Batch:
    """grasp_batch: one launch per optimizer step over many jobs."""

    def __init__(self, ctx: Context, capacity: int, max_jobs: int = 64, use_graph: bool = True):
        self.ctx = ctx
        h = C.c_void_p()
        ctx.lib.call("grasp_batch_create", ctx.h, capacity, max_jobs, int(use_graph), C.byref(h))
        self.h = h

    def set_tile(self, wpb: int, occ: int):
        t = TileC(wpb, occ)
        self.ctx.lib.call("grasp_batch_set_tile", self.h, C.byref(t))

    def step(self, jobs, stream=None):
        arr = (BatchJobC * len(jobs))(*[j.c() for j in jobs])
        self.ctx.lib.call("grasp_batch_step", self.h, C.cast(arr, C.c_void_p), len(jobs), _stream(stream))
        for j, c in zip(jobs, arr):
            j.t = c.t

    def flags(self, n: int) -> np.ndarray:
        out = np.zeros(n, np.int32)
        self.ctx.lib.call("grasp_batch_flags", self.h, n, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out

    def close(self):
        if self.h:
            self.ctx.lib.grasp_batch_destroy(self.h)
            self.h = None
