"""ctypes binding of libgrasp.so (the C ABI in include/grasp.h).

Argument marshalling only: every step of the grasp path runs in the HIP
library. If the library is missing this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrasp.so")

GRASP_OK, GRASP_EINVAL, GRASP_ENOMEM, GRASP_EDEVICE = 0, -1, -2, -3
GRASP_EBUSY, GRASP_EAGAIN, GRASP_ENONFINITE, GRASP_ECANCELED = -4, -5, -6, -7
MODE_AUTO, MODE_SAVE, MODE_RECOMPUTE = 0, 1, 2
PROJECTION_AVERAGED, PROJECTION_GAUSS_SEIDEL = 0, 1
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EBUSY", -5: "EAGAIN",
                -6: "ENONFINITE", -7: "ECANCELED"}


class GraspError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class HandDesc(C.Structure):
    _fields_ = [("n_links", C.c_int32), ("parent", C.POINTER(C.c_int32)),
                ("joint_origin", C.POINTER(C.c_float)), ("joint_axis", C.POINTER(C.c_float)),
                ("q_low", C.POINTER(C.c_float)), ("q_up", C.POINTER(C.c_float)),
                ("n_contacts", C.c_int32), ("contact_local", C.POINTER(C.c_float)),
                ("contact_link", C.POINTER(C.c_int32))]


class SdfDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("lo", C.c_float * 3), ("h", C.c_float),
                ("values", C.POINTER(C.c_float)), ("inertia_over_mass", C.c_float), ("layout", C.c_int32)]


LAYOUT_AUTO, LAYOUT_YZQUADS, LAYOUT_ZPAIRS = 0, 1, 2


class MeshDescC(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("vertices", C.POINTER(C.c_float)), ("normals", C.POINTER(C.c_float)),
                ("n_faces", C.c_int32), ("faces", C.POINTER(C.c_int32)), ("alpha", C.c_float)]


class MeshGridDescC(C.Structure):
    _fields_ = [("n", C.c_int32), ("lo", C.c_float * 3), ("h", C.c_float), ("inertia_over_mass", C.c_float),
                ("layout", C.c_int32)]


class EvalDescC(C.Structure):
    _fields_ = [("n_surface", C.c_int32), ("surface_link", C.POINTER(C.c_int32)),
                ("surface_local", C.POINTER(C.c_float)), ("surface_area", C.POINTER(C.c_float)),
                ("n_volume", C.c_int32), ("volume_link", C.POINTER(C.c_int32)),
                ("volume_local", C.POINTER(C.c_float)), ("volume_weight", C.POINTER(C.c_float))]


MAX_THRESHOLDS, MAX_TOP = 8, 64


class TileC(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("min_waves_per_simd", C.c_int32)]


class StepParamsC(C.Structure):
    _fields_ = [("dt", C.c_float), ("v0", C.c_float), ("K", C.c_int32), ("ckpt_every", C.c_int32),
                ("omega", C.c_float), ("r_dil", C.c_float), ("alpha_leak", C.c_float),
                ("w_stable", C.c_float), ("w_pen", C.c_float), ("w_range", C.c_float),
                ("w_limit", C.c_float), ("w_min", C.c_float), ("mode", C.c_int32), ("projection", C.c_int32),
                ("mu", C.c_float)]


class BatchJobC(C.Structure):
    _fields_ = [("hand", C.c_uint64), ("sdf", C.c_uint64), ("p", StepParamsC), ("B", C.c_int32),
                ("q", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p), ("loss", C.c_void_p),
                ("terms", C.c_void_p), ("dq", C.c_void_p), ("t", C.c_int32), ("T", C.c_int32),
                ("r0", C.c_float), ("lr", C.c_float), ("b1", C.c_float), ("b2", C.c_float), ("eps", C.c_float)]


class JobDescC(C.Structure):
    _fields_ = [("hand", C.c_uint64), ("sdf", C.c_uint64), ("B", C.c_int32), ("q0", C.c_void_p),
                ("T", C.c_int32), ("r0", C.c_float), ("p", StepParamsC), ("lr", C.c_float), ("b1", C.c_float),
                ("b2", C.c_float), ("eps", C.c_float), ("eval", C.c_uint64), ("n_thr", C.c_int32),
                ("thresholds", C.c_float * 8), ("top_k", C.c_int32), ("record_history", C.c_int32)]


class JobResultC(C.Structure):
    _fields_ = [("status", C.c_int32), ("q", C.c_void_p), ("loss", C.c_void_p), ("terms", C.c_void_p),
                ("rank", C.c_void_p), ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("steps", C.c_int32), ("metrics", C.c_void_p), ("top", C.c_void_p), ("top_mean", C.c_void_p),
                ("hist_q", C.c_void_p), ("hist_loss", C.c_void_p)]


class ServeStatsC(C.Structure):
    _fields_ = [("steps", C.c_int64), ("contact_evals", C.c_int64), ("queued", C.c_int32),
                ("resident", C.c_int32), ("finished", C.c_int32)]


@dataclasses.dataclass
class StepParams:
    """Mirror of grasp_step_params (defaults of grasp_default_params)."""
    dt: float = 1e-3
    v0: float = 1.0
    K: int = 1
    ckpt_every: int = 1
    omega: float = 1.0
    r_dil: float = 0.0
    alpha_leak: float = 0.1
    w_stable: float = 1.0
    w_pen: float = 1e4
    w_range: float = 1e-2
    w_limit: float = 1.0
    w_min: float = 1e-8
    mode: int = MODE_AUTO
    projection: int = 0  # PROJECTION_AVERAGED or PROJECTION_GAUSS_SEIDEL
    mu: float = 0.0      # Coulomb friction coefficient (0: frictionless)

    def c(self) -> StepParamsC:
        return StepParamsC(self.dt, self.v0, self.K, self.ckpt_every, self.omega, self.r_dil,
                           self.alpha_leak, self.w_stable, self.w_pen, self.w_range, self.w_limit,
                           self.w_min, self.mode, self.projection, self.mu)


# (name, restype, argtypes) of every exported entry point in include/grasp.h
_VP, _SZ, _I32, _U64, _F = C.c_void_p, C.c_size_t, C.c_int32, C.c_uint64, C.c_float
_FP, _IP = C.POINTER(C.c_float), C.POINTER(C.c_int32)
SIGNATURES = [
    ("grasp_init", _I32, [C.c_int, _VP, _SZ, C.POINTER(_VP)]),
    ("grasp_shutdown", None, [_VP]),
    ("grasp_last_error", C.c_char_p, []),
    ("grasp_create_hand", _I32, [_VP, C.POINTER(HandDesc), C.POINTER(_U64)]),
    ("grasp_destroy_hand", _I32, [_VP, _U64]),
    ("grasp_hand_contact_links", _I32, [_VP, _U64, _IP]),
    ("grasp_load_sdf", _I32, [_VP, C.POINTER(SdfDesc), C.POINTER(_U64)]),
    ("grasp_load_mesh", _I32, [_VP, C.POINTER(MeshDescC), C.POINTER(_U64)]),
    ("grasp_unload_mesh", _I32, [_VP, _U64]),
    ("grasp_mesh_sample", _I32, [_VP, _U64, _I32, _VP, _VP, _VP]),
    ("grasp_debug_mesh_step_sample", _I32, [_VP, _U64, _I32, _VP, _VP, _VP]),
    ("grasp_load_sdf_from_mesh", _I32, [_VP, _U64, C.POINTER(MeshGridDescC), C.POINTER(_U64)]),
    ("grasp_unload_sdf", _I32, [_VP, _U64]),
    ("grasp_load_eval_points", _I32, [_VP, _U64, C.POINTER(EvalDescC), C.POINTER(_U64)]),
    ("grasp_unload_eval_points", _I32, [_VP, _U64]),
    ("grasp_evaluate", _I32, [_VP, _U64, _U64, _I32, _VP, _I32, _FP, _VP, _VP]),
    ("grasp_evaluate_mesh", _I32, [_VP, _U64, _U64, _I32, _VP, _I32, _FP, _VP, _VP]),
    ("grasp_select_top", _I32, [_VP, _I32, _VP, _I32, _I32, _I32, _VP, _VP, _VP, _VP]),
    ("grasp_sdf_inertia", _I32, [_VP, _U64, _FP]),
    ("grasp_default_params", None, [C.POINTER(StepParamsC)]),
    ("grasp_step_workspace_bytes", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, C.POINTER(_SZ)]),
    ("grasp_step_fwd", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, _VP, _VP, _VP, _VP, _SZ, _VP]),
    ("grasp_step_bwd", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, _VP, _VP, _VP, _VP, _SZ, _VP]),
    ("grasp_adam_step", _I32, [_VP, _I32, _VP, _VP, _VP, _VP, _I32, _F, _F, _F, _F, _VP]),
    ("grasp_step_fused", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, _VP, _VP, _VP, _I32, _F, _F, _F,
                                _F, _VP, _VP, _VP, _VP]),
    ("grasp_step_fused_static", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, _VP, _VP, _VP, _I32, _F, _F, _F,
                                _F, _VP, _VP, _VP, _VP]),
    ("grasp_step_fused_mesh", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _F, _I32, _VP, _VP, _VP, _I32, _F, _F,
                                      _F, _F, _VP, _VP, _VP, _VP]),
    ("grasp_debug_trace_mesh", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _F, _I32, _VP, _VP, _VP, _VP, _VP]),
    ("grasp_plain_workspace_bytes", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, C.POINTER(_SZ)]),
    ("grasp_plain_step", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, _VP, _VP, _VP, _I32, _F, _F, _F, _F,
                                _VP, _VP, _VP, _SZ, _VP]),
    ("grasp_tune", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, _VP, _I32, C.POINTER(TileC), _FP]),
    ("grasp_set_tile", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, C.POINTER(TileC)]),
    ("grasp_batch_create", _I32, [_VP, _I32, _I32, _I32, C.POINTER(_VP)]),
    ("grasp_batch_destroy", _I32, [_VP]),
    ("grasp_batch_set_tile", _I32, [_VP, C.POINTER(TileC)]),
    ("grasp_batch_step", _I32, [_VP, _VP, _I32, _VP]),
    ("grasp_batch_flags", _I32, [_VP, _I32, _IP]),
    ("grasp_serve_config", _I32, [_VP, _I32, _I32]),
    ("grasp_submit", _I32, [_VP, C.POINTER(JobDescC), C.POINTER(_U64)]),
    ("grasp_poll", _I32, [_VP, _U64, C.POINTER(JobResultC)]),
    ("grasp_cancel", _I32, [_VP, _U64]),
    ("grasp_serve_stats_get", _I32, [_VP, C.POINTER(ServeStatsC)]),
    ("grasp_debug_sdf_sample", _I32, [_VP, _U64, _I32, _VP, _VP, _VP, _VP]),
    ("grasp_debug_trace", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, _VP, _VP, _VP, _VP, _VP]),
    ("grasp_debug_forward_groups", _I32, [_VP, _U64, _U64, C.POINTER(StepParamsC), _I32, _VP, _VP, _VP]),
]


class Library:
    """The loaded libgrasp.so with typed entry points."""
    _inst = None

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise RuntimeError(f"libgrasp.so not built at {path}; run paper_2306_08132_amd.build.build()")
        self.path = path
        self.dll = C.CDLL(path)
        for name, res, args in SIGNATURES:
            f = getattr(self.dll, name)
            f.restype = res
            f.argtypes = args

    @classmethod
    def get(cls) -> "Library":
        if cls._inst is None:
            cls._inst = cls()
        return cls._inst

    def __getattr__(self, name):
        return getattr(self.dll, name)

    def check(self, code: int, where: str):
        if code != GRASP_OK:
            msg = self.dll.grasp_last_error()
            raise GraspError(code, where, msg.decode() if msg else "")
        return code

    def call(self, name: str, *args):
        return self.check(getattr(self.dll, name)(*args), name)
