"""ctypes binding of the C ABI in include/flash.h (argument marshalling only).

Every step of the simulation runs inside the HIP library; this module only
converts numpy arrays to the C structures and back.  The library must be
built (paper_2604_17513_amd/build.py); importing the binding without it
raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

from . import scenes

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflash_mi355x.so")

FLASH_OK = 0
FLASH_ERR_INVALID_ARG = 1
FLASH_ERR_OUT_OF_MEMORY = 2
FLASH_ERR_DEVICE = 3
FLASH_ERR_CAPACITY = 4
FLASH_ERR_NOT_CONVERGED = 5
FLASH_ERR_NONFINITE = 6
FLASH_ERR_UNSUPPORTED = 7
FLASH_FP32, FLASH_FP64 = 0, 1
FLASH_WS_ZERO, FLASH_WS_PREV, FLASH_WS_LEARNED = 0, 1, 2
FLASH_METRIC_EXACT, FLASH_METRIC_LIGHTWEIGHT = 0, 1
MAX_OBSTACLES = 4
MAX_GRIPPERS = 2

EXPORTED = [
    "flash_create_batch", "flash_destroy_batch", "flash_set_state", "flash_get_state",
    "flash_set_state_device", "flash_get_state_device",
    "flash_set_obstacles", "flash_get_obstacles", "flash_set_grippers", "flash_step", "flash_synchronize",
    "flash_contacts", "flash_residual", "flash_residual_history", "flash_stats", "flash_set_kernel_timing",
    "flash_kernel_times", "flash_kernel_name", "flash_phase_times", "flash_schedule_info", "flash_ws_load",
    "flash_ws_record", "flash_ws_history", "flash_checkpoint_size", "flash_save_checkpoint",
    "flash_load_checkpoint", "flash_renderer_create", "flash_renderer_destroy", "flash_render",
    "flash_ws_collect", "flash_mlp_create", "flash_mlp_destroy", "flash_mlp_set_params", "flash_mlp_get_params",
    "flash_mlp_get_params_bf16", "flash_mlp_set_norm", "flash_mlp_get_norm", "flash_mlp_fit_norm",
    "flash_mlp_forward", "flash_mlp_grad", "flash_mlp_grad_noalloc", "flash_mlp_train", "flash_mlp_eval",
    "flash_last_error",
    "flash_version",
]
MLP_FEATURES, MLP_HIDDEN, MLP_OUTPUTS, MLP_PARAMS, MLP_NORM = 16, 128, 3, 35587, 35


class flash_env_desc(C.Structure):
    _fields_ = [("elem", C.c_int32), ("n_vertices", C.c_int32), ("n_elements", C.c_int32),
                ("reserved", C.c_int32), ("rest_x", C.POINTER(C.c_double)),
                ("elements", C.POINTER(C.c_int32)), ("density", C.c_double), ("thickness", C.c_double),
                ("young", C.c_double), ("poisson", C.c_double), ("bending", C.c_double), ("mu", C.c_double)]


class flash_obstacle(C.Structure):
    _fields_ = [("kind", C.c_int32), ("move_steps", C.c_int32), ("center", C.c_double * 3),
                ("rot", C.c_double * 9), ("size", C.c_double * 3), ("lin_vel", C.c_double * 3)]


class flash_gripper(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("lin_vel", C.c_double * 3), ("radius", C.c_double),
                ("move_steps", C.c_int32), ("grasp", C.c_int32)]


class flash_params(C.Structure):
    _fields_ = [("h", C.c_double), ("gravity", C.c_double * 3), ("lg_iterations", C.c_int32),
                ("max_inner_iterations", C.c_int32), ("ncp_tol", C.c_double), ("contact_margin", C.c_double),
                ("max_force", C.c_double), ("precision", C.c_int32), ("warm_start", C.c_int32),
                ("use_graph", C.c_int32), ("max_contacts_per_env", C.c_int32), ("inner_tol", C.c_double),
                ("contact_fp32", C.c_int32), ("fixed_schedule", C.c_int32),
                ("stream_groups", C.c_int32), ("fused_lg", C.c_int32), ("contact_metric", C.c_int32),
                ("global_contact_solve", C.c_int32), ("twin_chunk", C.c_int32)]


class flash_contact(C.Structure):
    _fields_ = [("env", C.c_int32), ("vertex", C.c_int32), ("obstacle", C.c_int32), ("mode", C.c_int32),
                ("normal", C.c_double * 3), ("tangent1", C.c_double * 3), ("gap", C.c_double),
                ("impulse", C.c_double * 3), ("lambda_", C.c_double * 3)]


class flash_env_stats(C.Structure):
    _fields_ = [("inner_iterations", C.c_int32), ("refactorizations", C.c_int32), ("contacts", C.c_int32),
                ("fp64_polar", C.c_int32), ("flags", C.c_int32), ("ws_state", C.c_int32),
                ("residual", C.c_double)]


class flash_camera(C.Structure):
    _fields_ = [("position", C.c_double * 3), ("rot", C.c_double * 9), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class FlashError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"flash status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH}; build it with paper_2604_17513_amd/build.py")
        # torch brings its own HIP runtime; loading it first makes this library bind to the same
        # one (a second runtime in the process would leave torch without a device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, I32, D = C.c_void_p, C.c_int32, C.POINTER(C.c_double)
        L.flash_create_batch.argtypes = [C.POINTER(flash_env_desc), I32, C.POINTER(flash_params), P, C.POINTER(P)]
        L.flash_destroy_batch.argtypes = [P]
        L.flash_set_state.argtypes = [P, I32, D, D]
        L.flash_get_state.argtypes = [P, I32, D, D]
        L.flash_set_state_device.argtypes = [P, I32, P, P, I32]
        L.flash_get_state_device.argtypes = [P, I32, P, P, I32]
        L.flash_set_obstacles.argtypes = [P, I32, C.POINTER(flash_obstacle), I32]
        L.flash_get_obstacles.argtypes = [P, I32, C.POINTER(flash_obstacle), I32, C.POINTER(I32)]
        L.flash_set_grippers.argtypes = [P, I32, C.POINTER(flash_gripper), I32]
        L.flash_step.argtypes = [P, I32]
        L.flash_checkpoint_size.argtypes = [P, C.POINTER(C.c_size_t)]
        L.flash_save_checkpoint.argtypes = [P, P, C.c_size_t, C.POINTER(C.c_size_t)]
        L.flash_load_checkpoint.argtypes = [P, P, C.c_size_t]
        L.flash_synchronize.argtypes = [P]
        L.flash_renderer_create.argtypes = [C.POINTER(flash_env_desc), I32, P, C.POINTER(P)]
        L.flash_renderer_destroy.argtypes = [P]
        L.flash_render.argtypes = [P, P, C.c_int64, C.POINTER(flash_obstacle), C.POINTER(I32),
                                   C.POINTER(flash_camera), I32, I32, P, P, P]
        L.flash_contacts.argtypes = [P, I32, C.POINTER(flash_contact), I32, C.POINTER(I32)]
        L.flash_residual.argtypes = [P, D, D, C.POINTER(I32)]
        L.flash_stats.argtypes = [P, C.POINTER(flash_env_stats)]
        L.flash_residual_history.argtypes = [P, D, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                             C.POINTER(C.c_int64), I32]
        L.flash_set_kernel_timing.argtypes = [P, I32]
        L.flash_kernel_times.argtypes = [P, D, C.POINTER(C.c_int64), I32, C.POINTER(I32)]
        L.flash_kernel_name.argtypes = [I32]
        L.flash_kernel_name.restype = C.c_char_p
        L.flash_phase_times.argtypes = [P, D]
        L.flash_schedule_info.argtypes = [P, C.POINTER(I32), D]
        F32, I64 = C.POINTER(C.c_float), C.c_int64
        L.flash_ws_load.argtypes = [P, C.POINTER(C.c_uint16), C.c_size_t, F32]
        L.flash_ws_record.argtypes = [P, I32]
        L.flash_ws_history.argtypes = [P, C.POINTER(I64), C.POINTER(I64), I32]
        L.flash_ws_collect.argtypes = [P, P, P, I64, C.POINTER(I64)]
        L.flash_mlp_create.argtypes = [I64, C.c_uint64, P, C.POINTER(P)]
        L.flash_mlp_destroy.argtypes = [P]
        L.flash_mlp_set_params.argtypes = [P, F32, I64]
        L.flash_mlp_get_params.argtypes = [P, F32, I64]
        L.flash_mlp_get_params_bf16.argtypes = [P, C.POINTER(C.c_uint16), I64]
        L.flash_mlp_set_norm.argtypes = [P, F32]
        L.flash_mlp_get_norm.argtypes = [P, F32]
        L.flash_mlp_fit_norm.argtypes = [P, P, P, I64]
        L.flash_mlp_forward.argtypes = [P, P, I64, P]
        L.flash_mlp_grad.argtypes = [P, P, P, I64, F32, F32]
        L.flash_mlp_grad_noalloc.argtypes = [P, P, P, I64, P, P, P]
        L.flash_mlp_train.argtypes = [P, P, P, I64, I32, I32, C.c_float, C.c_uint64, F32]
        L.flash_mlp_eval.argtypes = [P, P, P, I64, F32]
        L.flash_last_error.restype = C.c_char_p
        L.flash_version.restype = C.c_char_p
        for name in EXPORTED:
            fn = getattr(L, name)
            if name not in ("flash_kernel_name", "flash_last_error", "flash_version"):
                fn.restype = C.c_int
        _lib = L
    return _lib


def _check(st: int, allow=()):
    if st != FLASH_OK and st not in allow:
        raise FlashError(st, lib().flash_last_error().decode())
    return st


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def params_struct(p: scenes.Params, precision: int = FLASH_FP32, warm_start: int = FLASH_WS_PREV,
                  use_graph: bool = False, max_contacts: int = 0, inner_tol: float = 0.0,
                  fixed_schedule: bool = False, contact_fp32: bool = False,
                  stream_groups: int = 0, fused_lg: bool = False, contact_metric: int = 0,
                  global_contact_solve: int = 0, twin_chunk: int = 0) -> flash_params:
    s = flash_params()
    s.h = p.h
    for k in range(3):
        s.gravity[k] = p.gravity[k]
    s.lg_iterations = p.lg_iterations
    s.max_inner_iterations = p.max_inner_iterations
    s.ncp_tol = p.ncp_tol
    s.contact_margin = p.contact_margin
    s.max_force = p.max_force
    s.precision = precision
    s.warm_start = warm_start
    s.use_graph = 1 if use_graph else 0
    s.max_contacts_per_env = max_contacts
    s.inner_tol = inner_tol
    s.fixed_schedule = 1 if fixed_schedule else 0
    s.contact_fp32 = 1 if contact_fp32 else 0
    s.stream_groups = int(stream_groups)
    s.fused_lg = 1 if fused_lg else 0
    s.contact_metric = int(contact_metric)
    s.global_contact_solve = int(global_contact_solve)
    s.twin_chunk = int(twin_chunk)
    return s


def gripper_struct(g: scenes.Gripper) -> flash_gripper:
    s = flash_gripper()
    for k in range(3):
        s.center[k] = g.center[k]
        s.lin_vel[k] = g.lin_vel[k]
    s.radius = g.radius
    s.move_steps = g.move_steps
    s.grasp = 1 if g.grasp else 0
    return s


def obstacle_struct(o: scenes.Obstacle) -> flash_obstacle:
    s = flash_obstacle()
    s.kind = o.kind
    s.move_steps = o.move_steps
    for k in range(3):
        s.center[k] = o.center[k]
        s.size[k] = o.size[k]
        s.lin_vel[k] = o.lin_vel[k]
    R = np.asarray(o.rot, dtype=np.float64).reshape(3, 3)
    for k in range(9):
        s.rot[k] = R.reshape(-1)[k]
    return s


def env_descs(envs: Sequence[scenes.EnvDesc]):
    """flash_env_desc array for envs, and the numpy arrays it points into (keep them alive)."""
    keep = []
    descs = (flash_env_desc * len(envs))()
    for i, e in enumerate(envs):
        rest = np.ascontiguousarray(e.rest_x, dtype=np.float64)
        el = np.ascontiguousarray(e.elements, dtype=np.int32)
        keep += [rest, el]
        d = descs[i]
        d.elem = e.elem
        d.n_vertices = e.n_vertices
        d.n_elements = e.n_elements
        d.rest_x = _dptr(rest)
        d.elements = el.ctypes.data_as(C.POINTER(C.c_int32))
        d.density, d.thickness, d.young = e.density, e.thickness, e.young
        d.poisson, d.bending, d.mu = e.poisson, e.bending, e.mu
    return descs, keep


class Batch:
    """A batch of environments living on the GPU (wraps flash_create_batch)."""

    def __init__(self, envs: Sequence[scenes.EnvDesc], params: scenes.Params, precision: int = FLASH_FP32,
                 warm_start: int = FLASH_WS_PREV, use_graph: bool = False, max_contacts: int = 0,
                 stream: Optional[int] = None, inner_tol: float = 0.0, fixed_schedule: bool = False,
                 contact_fp32: bool = False, stream_groups: int = 0, fused_lg: bool = False,
                 contact_metric: int = 0, global_contact_solve: int = 0, twin_chunk: int = 0):
        L = lib()
        self.n_envs = len(envs)
        self.params = params
        self.nv = [e.n_vertices for e in envs]
        descs, self._keep = env_descs(envs)
        self._p = params_struct(params, precision, warm_start, use_graph, max_contacts, inner_tol, fixed_schedule,
                                contact_fp32, stream_groups, fused_lg, contact_metric, global_contact_solve,
                                twin_chunk)
        h = C.c_void_p()
        _check(L.flash_create_batch(descs, self.n_envs, C.byref(self._p), C.c_void_p(stream or 0), C.byref(h)))
        self._h = h
        self._keep = []

    # -- lifecycle -----------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().flash_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state -----------------------------------------------------------------------
    def set_state(self, x, v=None, env: int = -1):
        xa = np.ascontiguousarray(np.concatenate(x) if isinstance(x, (list, tuple)) else x, dtype=np.float64)
        va = None
        if v is not None:
            va = np.ascontiguousarray(np.concatenate(v) if isinstance(v, (list, tuple)) else v, dtype=np.float64)
        _check(lib().flash_set_state(self._h, env, _dptr(xa), _dptr(va) if va is not None else None))

    def get_state(self, env: int = -1):
        n = sum(self.nv) if env < 0 else self.nv[env]
        x = np.empty((n, 3))
        v = np.empty((n, 3))
        _check(lib().flash_get_state(self._h, env, _dptr(x), _dptr(v)))
        return x, v

    def set_state_device(self, x_dev, v_dev=None, env: int = -1):
        """State from device arrays [3][n] (float32 or float64 tensors, component-major); asynchronous."""
        es = _elem_size(x_dev)
        if v_dev is not None and _elem_size(v_dev) != es:
            raise ValueError("x and v must share one element type")
        _check(lib().flash_set_state_device(self._h, env, C.c_void_p(_devptr(x_dev)),
                                            C.c_void_p(_devptr(v_dev)) if v_dev is not None else None, es))

    def get_state_device(self, x_dev, v_dev=None, env: int = -1):
        """State into device arrays [3][n] (float32 or float64 tensors); asynchronous."""
        ref = x_dev if x_dev is not None else v_dev
        es = _elem_size(ref)
        _check(lib().flash_get_state_device(self._h, env,
                                            C.c_void_p(_devptr(x_dev)) if x_dev is not None else None,
                                            C.c_void_p(_devptr(v_dev)) if v_dev is not None else None, es))

    def split(self, a: np.ndarray) -> List[np.ndarray]:
        return np.split(a, np.cumsum(self.nv)[:-1])

    def set_obstacles(self, obstacles, env: int = -1):
        if env < 0:
            n = len(obstacles[0])
            arr = (flash_obstacle * (self.n_envs * n))()
            for e, lst in enumerate(obstacles):
                assert len(lst) == n
                for q, o in enumerate(lst):
                    arr[e * n + q] = obstacle_struct(o)
        else:
            n = len(obstacles)
            arr = (flash_obstacle * max(n, 1))()
            for q, o in enumerate(obstacles):
                arr[q] = obstacle_struct(o)
        _check(lib().flash_set_obstacles(self._h, env, arr, n))

    def set_grippers(self, grippers, env: int = -1):
        """grippers: per-env lists of scenes.Gripper (env = -1, equal lengths) or one env's list."""
        if env < 0:
            n = len(grippers[0])
            arr = (flash_gripper * max(self.n_envs * n, 1))()
            for e, lst in enumerate(grippers):
                assert len(lst) == n
                for q, g in enumerate(lst):
                    arr[e * n + q] = gripper_struct(g)
        else:
            n = len(grippers)
            arr = (flash_gripper * max(n, 1))()
            for q, g in enumerate(grippers):
                arr[q] = gripper_struct(g)
        _check(lib().flash_set_grippers(self._h, env, arr, n))

    def get_obstacles(self, env: int):
        arr = (flash_obstacle * MAX_OBSTACLES)()
        n = C.c_int32()
        _check(lib().flash_get_obstacles(self._h, env, arr, MAX_OBSTACLES, C.byref(n)))
        out = []
        for q in range(n.value):
            s = arr[q]
            out.append(scenes.Obstacle(s.kind, np.array(s.center[:]), np.array(s.rot[:]).reshape(3, 3),
                                       np.array(s.size[:]), np.array(s.lin_vel[:]), s.move_steps))
        return out

    # -- stepping --------------------------------------------------------------------
    def step(self, n: int = 1):
        _check(lib().flash_step(self._h, n))

    def synchronize(self):
        _check(lib().flash_synchronize(self._h))

    # -- queries -----------------------------------------------------------------------
    def contacts(self, env: int = -1):
        n = C.c_int32()
        _check(lib().flash_contacts(self._h, env, None, 0, C.byref(n)), allow=(FLASH_ERR_CAPACITY,))
        cap = max(n.value, 1)
        arr = (flash_contact * cap)()
        _check(lib().flash_contacts(self._h, env, arr, cap, C.byref(n)))
        k = n.value
        out = {
            "env": np.array([arr[i].env for i in range(k)], dtype=np.int64),
            "vertex": np.array([arr[i].vertex for i in range(k)], dtype=np.int64),
            "obstacle": np.array([arr[i].obstacle for i in range(k)], dtype=np.int64),
            "mode": np.array([arr[i].mode for i in range(k)], dtype=np.int64),
            "normal": np.array([arr[i].normal[:] for i in range(k)]).reshape(k, 3),
            "tangent1": np.array([arr[i].tangent1[:] for i in range(k)]).reshape(k, 3),
            "gap": np.array([arr[i].gap for i in range(k)]),
            "impulse": np.array([arr[i].impulse[:] for i in range(k)]).reshape(k, 3),
            "lambda": np.array([arr[i].lambda_[:] for i in range(k)]).reshape(k, 3),
        }
        return out

    def residual(self):
        per = np.empty(self.n_envs)
        mx = C.c_double()
        its = np.empty(self.n_envs, dtype=np.int32)
        st = lib().flash_residual(self._h, _dptr(per), C.byref(mx), its.ctypes.data_as(C.POINTER(C.c_int32)))
        _check(st, allow=(FLASH_ERR_NOT_CONVERGED, FLASH_ERR_NONFINITE, FLASH_ERR_CAPACITY))
        return per, mx.value, its, st

    def residual_history(self, reset: bool = True, full: bool = False):
        """(worst residual, failed env-steps: above ncp_tol or contacts dropped beyond the capacity)
        since the last reset; with full=True also (Newton iterations, env-steps)."""
        mx = C.c_double()
        over, newton, steps = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().flash_residual_history(self._h, C.byref(mx), C.byref(over), C.byref(newton), C.byref(steps),
                                            1 if reset else 0))
        if full:
            return mx.value, over.value, newton.value, steps.value
        return mx.value, over.value

    def stats(self):
        arr = (flash_env_stats * self.n_envs)()
        _check(lib().flash_stats(self._h, arr))
        return [dict(inner_iterations=s.inner_iterations, refactorizations=s.refactorizations,
                     contacts=s.contacts, fp64_polar=s.fp64_polar, flags=s.flags, ws_state=s.ws_state,
                     residual=s.residual)
                for s in arr]

    def set_kernel_timing(self, mask):
        """mask: True (every kernel class), False (off) or a bitmask of kernel classes."""
        if mask is True:
            mask = 0xFFFF
        elif mask is False:
            mask = 0
        _check(lib().flash_set_kernel_timing(self._h, int(mask)))

    def schedule_info(self):
        """(columns per tile, rows in flight per wave, work items, tuned, candidate ms per apply launch)."""
        info = np.zeros(5, dtype=np.int32)
        ms = np.zeros(6)
        _check(lib().flash_schedule_info(self._h, info.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(ms)))
        return dict(tile_cols=int(info[0]), unroll=int(info[1]), work_items=int(info[2]), tuned=bool(info[3]),
                    stream_groups=int(info[4]), candidate_ms=ms.tolist())

    def phase_times(self):
        out = np.zeros(16)
        _check(lib().flash_phase_times(self._h, _dptr(out)))
        names = ["setup", "residual", "base_inverse", "rhs", "cap_build", "cap_lu", "direction", "line_search",
                 "n_factor", "n_reuse", "n_ls_fail", "n_unconverged", "cap_rows_mean", "cap_rows_max",
                 "newton", "solves"]
        return dict(zip(names, out.tolist()))

    def kernel_times(self):
        ms = np.zeros(16)
        cnt = np.zeros(16, dtype=np.int64)
        n = C.c_int32()
        _check(lib().flash_kernel_times(self._h, _dptr(ms), cnt.ctypes.data_as(C.POINTER(C.c_int64)), 16,
                                        C.byref(n)))
        return {lib().flash_kernel_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(n.value)}


    # -- learned warm start ----------------------------------------------------------
    def ws_load(self, weights_bf16: np.ndarray, norm: np.ndarray):
        w = np.ascontiguousarray(weights_bf16, dtype=np.uint16)
        nm = np.ascontiguousarray(norm, dtype=np.float32)
        _check(lib().flash_ws_load(self._h, w.ctypes.data_as(C.POINTER(C.c_uint16)), w.size, _fptr(nm)))

    def ws_history(self, reset: bool = True):
        """(env-steps started from the prediction, env-steps restarted from the plain start) since the last reset."""
        a, r = C.c_int64(), C.c_int64()
        _check(lib().flash_ws_history(self._h, C.byref(a), C.byref(r), 1 if reset else 0))
        return a.value, r.value

    def save_checkpoint(self) -> bytes:
        """Everything the next step reads besides the model and the network weights, as bytes."""
        n = C.c_size_t()
        _check(lib().flash_checkpoint_size(self._h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().flash_save_checkpoint(self._h, C.cast(buf, C.c_void_p), n.value, C.byref(n)))
        return buf.raw[:n.value]

    def load_checkpoint(self, blob: bytes):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(lib().flash_load_checkpoint(self._h, C.cast(buf, C.c_void_p), len(blob)))

    def ws_record(self, on: bool = True):
        _check(lib().flash_ws_record(self._h, 1 if on else 0))

    def ws_collect(self, feat_dev, lab_dev, capacity: int, n: int) -> int:
        """Appends the last step's (feature, label) rows at row n of device arrays; returns the new count."""
        cnt = C.c_int64(n)
        _check(lib().flash_ws_collect(self._h, C.c_void_p(_devptr(feat_dev)), C.c_void_p(_devptr(lab_dev)),
                                      int(capacity), C.byref(cnt)))
        return cnt.value


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _elem_size(x) -> int:
    """Bytes per element of a device tensor (4 or 8)."""
    return int(x.element_size())


def _devptr(x) -> int:
    """Device address of a tensor-like object (anything with data_ptr()) or an int."""
    return int(x.data_ptr()) if hasattr(x, "data_ptr") else int(x)


class Mlp:
    """The warm-start network trainer (wraps flash_mlp_*); data arguments are device arrays."""

    def __init__(self, max_rows: int, seed: int = 0, stream: Optional[int] = None):
        h = C.c_void_p()
        _check(lib().flash_mlp_create(int(max_rows), int(seed), C.c_void_p(stream or 0), C.byref(h)))
        self._h = h
        self.max_rows = max_rows

    def close(self):
        if getattr(self, "_h", None):
            lib().flash_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, w: np.ndarray):
        a = np.ascontiguousarray(w, dtype=np.float32)
        _check(lib().flash_mlp_set_params(self._h, _fptr(a), a.size))

    def params(self) -> np.ndarray:
        a = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(lib().flash_mlp_get_params(self._h, _fptr(a), a.size))
        return a

    def params_bf16(self) -> np.ndarray:
        a = np.empty(MLP_PARAMS, dtype=np.uint16)
        _check(lib().flash_mlp_get_params_bf16(self._h, a.ctypes.data_as(C.POINTER(C.c_uint16)), a.size))
        return a

    def set_norm(self, norm: np.ndarray):
        a = np.ascontiguousarray(norm, dtype=np.float32)
        _check(lib().flash_mlp_set_norm(self._h, _fptr(a)))

    def norm(self) -> np.ndarray:
        a = np.empty(MLP_NORM, dtype=np.float32)
        _check(lib().flash_mlp_get_norm(self._h, _fptr(a)))
        return a

    def fit_norm(self, feat_dev, lab_dev, n: int):
        _check(lib().flash_mlp_fit_norm(self._h, C.c_void_p(_devptr(feat_dev)), C.c_void_p(_devptr(lab_dev)), int(n)))

    def forward(self, x_dev, n: int, y_dev):
        _check(lib().flash_mlp_forward(self._h, C.c_void_p(_devptr(x_dev)), int(n), C.c_void_p(_devptr(y_dev))))

    def grad(self, x_dev, target_dev, n: int):
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        _check(lib().flash_mlp_grad(self._h, C.c_void_p(_devptr(x_dev)), C.c_void_p(_devptr(target_dev)), int(n),
                                    _fptr(g), _fptr(loss)))
        return g, float(loss[0])

    def train(self, feat_dev, lab_dev, n: int, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
        losses = np.zeros(epochs, dtype=np.float32)
        _check(lib().flash_mlp_train(self._h, C.c_void_p(_devptr(feat_dev)), C.c_void_p(_devptr(lab_dev)), int(n),
                                     int(epochs), int(batch), float(lr), int(seed), _fptr(losses)))
        return losses

    def eval(self, feat_dev, lab_dev, n: int) -> float:
        loss = np.zeros(1, dtype=np.float32)
        _check(lib().flash_mlp_eval(self._h, C.c_void_p(_devptr(feat_dev)), C.c_void_p(_devptr(lab_dev)), int(n),
                                    _fptr(loss)))
        return float(loss[0])


def mlp_grad_noalloc(params_dev, x_dev, target_dev, n: int, grad_dev, loss_dev=None, stream: int = 0):
    """flash_mlp_grad_noalloc: loss and gradient into device arrays, no allocation, asynchronous."""
    _check(lib().flash_mlp_grad_noalloc(C.c_void_p(_devptr(params_dev)), C.c_void_p(_devptr(x_dev)),
                                        C.c_void_p(_devptr(target_dev)), int(n), C.c_void_p(_devptr(grad_dev)),
                                        C.c_void_p(_devptr(loss_dev)) if loss_dev is not None else None,
                                        C.c_void_p(stream)))


def camera_struct(cam) -> flash_camera:
    """cam: dict with position (3,), rot (3, 3) camera-to-world (columns: image right, image down,
    optical axis), fx, fy, cx, cy in pixels."""
    s = flash_camera()
    R = np.asarray(cam["rot"], dtype=np.float64).reshape(-1)
    for k in range(3):
        s.position[k] = float(cam["position"][k])
    for k in range(9):
        s.rot[k] = float(R[k])
    s.fx, s.fy, s.cx, s.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    return s


class Renderer:
    """Batched depth ray casting of the envs' surfaces (wraps flash_renderer_create / flash_render)."""

    def __init__(self, envs: Sequence[scenes.EnvDesc], stream: Optional[int] = None):
        self.n_envs = len(envs)
        self.nv = [e.n_vertices for e in envs]
        descs, keep = env_descs(envs)
        h = C.c_void_p()
        _check(lib().flash_renderer_create(descs, self.n_envs, C.c_void_p(stream or 0), C.byref(h)))
        self._h = h

    def render(self, x_dev, cams, width: int, height: int, obstacles=None, depth=True, instance=True,
               points=False):
        """x_dev: torch float32 CUDA tensor [3, ld] of all envs' vertex positions (ld >= total
        vertices); cams: per-env camera dicts; obstacles: per-env lists of scenes.Obstacle (or None).
        Returns a dict of torch CUDA tensors: depth [n_envs, height, width] (float32), instance
        (int32) and points [n_envs, height, width, 3] (float32), each when asked for."""
        import torch
        assert x_dev.dtype == torch.float32 and x_dev.is_cuda and x_dev.dim() == 2 and x_dev.shape[0] == 3
        x_dev = x_dev.contiguous()
        n = self.n_envs
        cam_arr = (flash_camera * n)()
        for e in range(n):
            cam_arr[e] = camera_struct(cams[e])
        ob_arr = (flash_obstacle * (n * MAX_OBSTACLES))()
        nob = (C.c_int32 * n)()
        if obstacles is not None:
            for e, lst in enumerate(obstacles):
                nob[e] = len(lst)        # the library rejects counts above MAX_OBSTACLES
                for q, o in enumerate(lst[:MAX_OBSTACLES]):
                    ob_arr[e * MAX_OBSTACLES + q] = obstacle_struct(o)
        dev = x_dev.device
        out = {}
        if depth:
            out["depth"] = torch.empty((n, height, width), dtype=torch.float32, device=dev)
        if instance:
            out["instance"] = torch.empty((n, height, width), dtype=torch.int32, device=dev)
        if points:
            out["points"] = torch.empty((n, height, width, 3), dtype=torch.float32, device=dev)
        ptr = lambda k: C.c_void_p(out[k].data_ptr() if k in out else 0)  # noqa: E731
        torch.cuda.synchronize(dev)
        _check(lib().flash_render(self._h, C.c_void_p(x_dev.data_ptr()), int(x_dev.stride(0)), ob_arr, nob,
                                  cam_arr, int(width), int(height), ptr("depth"), ptr("instance"), ptr("points")))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().flash_renderer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_scene(sc: scenes.Scene, precision: int = FLASH_FP32, warm_start: int = FLASH_WS_PREV,
               use_graph: bool = False, max_contacts: int = 0, inner_tol: float = 0.0,
               fixed_schedule: bool = False, contact_fp32: bool = False, stream_groups: int = 0,
               fused_lg: bool = False, contact_metric: int = 0, global_contact_solve: int = 0,
               twin_chunk: int = 0) -> Batch:
    """Creates a batch for a scene and uploads its initial state and obstacles."""
    b = Batch(sc.envs, sc.params, precision, warm_start, use_graph, max_contacts, inner_tol=inner_tol,
              fixed_schedule=fixed_schedule, contact_fp32=contact_fp32, stream_groups=stream_groups,
              fused_lg=fused_lg, contact_metric=contact_metric, global_contact_solve=global_contact_solve,
              twin_chunk=twin_chunk)
    b.set_state(sc.x0, sc.v0)
    n_obs = {len(o) for o in sc.obstacles}
    if len(n_obs) == 1:
        b.set_obstacles(sc.obstacles)
    else:
        for e, lst in enumerate(sc.obstacles):
            b.set_obstacles(lst, env=e)
    if sc.grippers:
        n_g = {len(g) for g in sc.grippers}
        if len(n_g) == 1:
            b.set_grippers(sc.grippers)
        else:
            for e, lst in enumerate(sc.grippers):
                b.set_grippers(lst, env=e)
    return b
