"""Python binding of libsqrtba.so and libsqrtba64.so (ctypes).  Argument marshalling only.

Every numerical step runs in the libraries' HIP kernels; this module converts
numpy arrays to the C ABIs of include/sqrtba.h (FP32) and include/sqrtba64.h
(FP64, ``Context(precision=64)``), raises SqrtBAError on a non-zero status, and
uses PyTorch only for device memory (the workspace) and the HIP stream.  It
fails loudly when a library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsqrtba.so")
LIB64_PATH = os.path.join(_HERE, "libsqrtba64.so")

OK, E_INVALID, E_OOM, E_HIP, E_STATE, E_NONFINITE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_OOM", -3: "E_HIP", -4: "E_STATE", -5: "E_NONFINITE",
                -6: "E_UNSUPPORTED"}
PCG_STATUS = {0: "converged", 1: "max_iters", 2: "breakdown", 3: "zero_rhs", 4: "inactive"}
LM_STATUS = {0: "max_iters", 1: "func_tol", 2: "lambda_max", 3: "nonfinite"}
MAX_OBS_PER_LANDMARK = 512


class SqrtBAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [
        ("lambda0", C.c_double), ("lambda_min", C.c_double), ("lambda_max", C.c_double),
        ("accept_ratio", C.c_double), ("max_lm_iters", C.c_int32), ("func_tol", C.c_double),
        ("pcg_max_iters", C.c_int32), ("pcg_rel_tol", C.c_double), ("pcg_check_every", C.c_int32),
        ("use_graph", C.c_int32), ("pcg_forcing_eta", C.c_double), ("landmark_blocks", C.c_int32),
        ("huber_delta", C.c_double), ("pcg_test_kernel", C.c_int32),
    ]


class LMReport(C.Structure):
    _fields_ = [
        ("initial_cost", C.c_double), ("final_cost", C.c_double), ("iterations", C.c_int32),
        ("accepted", C.c_int32), ("total_pcg_iters", C.c_int32), ("status", C.c_int32),
        ("solve_seconds", C.c_double), ("time_to_tol", C.c_double),
    ]


class LMRecord(C.Structure):
    _fields_ = [
        ("iter", C.c_int32), ("accepted", C.c_int32), ("pcg_iters", C.c_int32), ("pcg_status", C.c_int32),
        ("lambda_", C.c_double), ("cost", C.c_double), ("new_cost", C.c_double),
        ("model_decrease", C.c_double), ("rel_res", C.c_double), ("t_seconds", C.c_double),
    ]


STAGES = ["linearize", "marginalize", "damp", "precond", "matvec", "pcg_vector", "backsub", "update"]


class Tuning(C.Structure):
    _fields_ = [("rows_min_k", C.c_int32), ("huge_rows", C.c_int32), ("huge_side", C.c_int32),
                ("large_separate", C.c_int32), ("small_rows", C.c_int32), ("persist_wgs", C.c_int32),
                ("stream_loads", C.c_int32)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class TuningTrial(C.Structure):
    _fields_ = [("shape", Tuning), ("ms", C.c_double)]


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8), ("bytes", C.c_double * 8),
                ("units", C.c_int64 * 8)]


_lib = None
_lib64 = None

P = C.c_void_p
I32, I64, U64 = C.c_int32, C.c_int64, C.c_uint64
PD, PF, PI32, PI64, PU8 = (C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_int32),
                           C.POINTER(C.c_int64), C.POINTER(C.c_uint8))

_SIGS = {
    "sqrtba_version": (I32, []),
    "sqrtba_default_options": (None, [C.POINTER(Options)]),
    "sqrtba_create": (I32, [C.POINTER(P), C.POINTER(Options), P]),
    "sqrtba_set_options": (I32, [P, C.POINTER(Options)]),
    "sqrtba_destroy": (None, [P]),
    "sqrtba_last_error": (C.c_char_p, [P]),
    "sqrtba_set_problems": (I32, [P, I32, PI64, PI64]),
    "sqrtba_set_cameras": (I32, [P, I64, PF]),
    "sqrtba_set_landmarks": (I32, [P, I64, PF]),
    "sqrtba_set_observations": (I32, [P, I64, PI32, PI32, PF]),
    "sqrtba_set_cameras_device": (I32, [P, I64, P]),
    "sqrtba_set_landmarks_device": (I32, [P, I64, P]),
    "sqrtba_set_observations_device": (I32, [P, I64, P, P, P]),
    "sqrtba_workspace_bytes": (I32, [P, C.POINTER(U64)]),
    "sqrtba_bind_workspace": (I32, [P, P, U64]),
    "sqrtba_set_active": (I32, [P, PU8]),
    "sqrtba_linearize": (I32, [P, PD]),
    "sqrtba_marginalize": (I32, [P]),
    "sqrtba_damp": (I32, [P, PD]),
    "sqrtba_solve": (I32, [P, PI32, PD, PI32]),
    "sqrtba_back_substitute": (I32, [P, PD]),
    "sqrtba_update": (I32, [P, PD]),
    "sqrtba_commit": (I32, [P, PU8]),
    "sqrtba_lm_solve": (I32, [P, C.POINTER(LMReport)]),
    "sqrtba_lm_solve_tracked": (I32, [P, PD, C.POINTER(LMReport)]),
    "sqrtba_get_lm_history": (I32, [P, I32, C.POINTER(LMRecord), I32, PI32]),
    "sqrtba_get_cameras": (I32, [P, PF]),
    "sqrtba_get_landmarks": (I32, [P, PF]),
    "sqrtba_get_cameras_device": (I32, [P, P]),
    "sqrtba_get_landmarks_device": (I32, [P, P]),
    "sqrtba_debug_bookkeeping": (I32, [P, PI64, PI64, PI64, PU8, PU8]),
    "sqrtba_debug_linearization": (I32, [P, PF, PF, PF]),
    "sqrtba_debug_scales": (I32, [P, PF, PF]),
    "sqrtba_debug_rcs_matvec": (I32, [P, I32, PF, PF]),
    "sqrtba_debug_rhs": (I32, [P, PF]),
    "sqrtba_rcs_matvec_noalloc": (I32, [P, P, P]),
    "sqrtba_debug_precond": (I32, [P, PF]),
    "sqrtba_debug_block": (I32, [P, I64, PI32, PF, PF]),
    "sqrtba_debug_solution": (I32, [P, PF, PF]),
    "sqrtba_debug_set_pose_increment": (I32, [P, PF]),
    "sqrtba_profile_enable": (I32, [P, I32]),
    "sqrtba_profile_get": (I32, [P, C.POINTER(Profile)]),
    "sqrtba_save_state": (I32, [P]),
    "sqrtba_restore_state": (I32, [P]),
    "sqrtba_mlp_num_params": (I32, []),
    "sqrtba_mlp_init": (I32, [P, U64]),
    "sqrtba_mlp_set_params": (I32, [P, PF]),
    "sqrtba_mlp_get_params": (I32, [P, PF]),
    "sqrtba_set_preconditioner": (I32, [P, I32]),
    "sqrtba_pcg_trace": (I32, [P, I32, I32]),
    "sqrtba_trace_size": (I32, [P, PI32, PI32]),
    "sqrtba_mlp_train": (I32, [P, I32, I32, C.c_double, U64, PD]),
    "sqrtba_mlp_eval": (I32, [P, I32, PF, PF, PF, PF, PD, PF]),
    "sqrtba_learned_stats": (I32, [P, PI64, PI64, PI64]),
    "sqrtba_debug_features": (I32, [P, PF, PF]),
    "sqrtba_debug_learned_precond": (I32, [P, PF]),
    "sqrtba_get_tuning": (I32, [P, C.POINTER(Tuning)]),
    "sqrtba_set_tuning": (I32, [P, C.POINTER(Tuning)]),
    "sqrtba_autotune": (I32, [P, I32, C.POINTER(Tuning), C.POINTER(TuningTrial), I32, PI32]),
    "sqrtba_time_product": (I32, [P, I32, PD, PD]),
}
EXPORTED = tuple(_SIGS)

# The FP64 library exports every call except the learned preconditioner's, under the
# prefix sqrtba64_, with double in place of float arrays.
FP32_ONLY = ("sqrtba_mlp_num_params", "sqrtba_mlp_init", "sqrtba_mlp_set_params", "sqrtba_mlp_get_params",
             "sqrtba_set_preconditioner", "sqrtba_pcg_trace", "sqrtba_trace_size", "sqrtba_mlp_train",
             "sqrtba_mlp_eval", "sqrtba_learned_stats", "sqrtba_debug_features", "sqrtba_debug_learned_precond")
_SIGS64 = {"sqrtba64_" + name[len("sqrtba_"):]: (res, [PD if a is PF else a for a in args])
           for name, (res, args) in _SIGS.items() if name not in FP32_ONLY}
EXPORTED64 = tuple(_SIGS64)


def _load(path, sigs):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2103_01843_amd.build` "
                          "(the HIP library is required; there is no fallback)")
    h = C.CDLL(path)
    for name, (res, args) in sigs.items():
        f = getattr(h, name)
        f.restype = res
        f.argtypes = args
    return h


def lib(precision: int = 32):
    """The loaded FP32 (or FP64) library; raises ImportError if it has not been built."""
    global _lib, _lib64
    if precision == 64:
        if _lib64 is None:
            _lib64 = _load(LIB64_PATH, _SIGS64)
        return _lib64
    if precision != 32:
        raise ValueError("precision is 32 or 64")
    if _lib is None:
        _lib = _load(LIB_PATH, _SIGS)
    return _lib


class _Api:
    """The entry points of one library by their unprefixed names (linearize, solve, ...)."""

    def __init__(self, precision: int):
        self._h = lib(precision)
        self._prefix = "sqrtba64_" if precision == 64 else "sqrtba_"

    def __getattr__(self, name):
        if self._prefix == "sqrtba64_" and "sqrtba_" + name in FP32_ONLY:
            raise SqrtBAError(E_UNSUPPORTED, f"{name}: the learned preconditioner is FP32 only")
        return getattr(self._h, self._prefix + name)


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _arr(x, dtype, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x), dtype=dtype)
    if shape is not None:
        a = a.reshape(shape)
    return a


def default_options(**kw) -> Options:
    o = Options()
    lib().sqrtba_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


@dataclass
class Report:
    initial_cost: float
    final_cost: float
    iterations: int
    accepted: int
    total_pcg_iters: int
    status: str
    solve_seconds: float
    time_to_tol: float


class Context:
    """One sqrtba context (one or a batch of problems) on the current HIP device."""

    def __init__(self, options: Optional[Options] = None, stream=None, precision: int = 32, **kw):
        self._api = _Api(precision)
        self.precision = precision
        self._rt = np.float64 if precision == 64 else np.float32  # element type of the state arrays
        self._rc = C.c_double if precision == 64 else C.c_float
        if options is None:
            options = default_options(**kw)
        elif kw:
            raise TypeError("pass either options or keyword options")
        self.options = options
        handle = None
        if stream is not None:
            handle = int(getattr(stream, "cuda_stream", stream))
        self._h = P()
        st = self._api.create(C.byref(self._h), C.byref(options), P(handle) if handle else None)
        if st != OK:
            raise SqrtBAError(st, "create failed")
        self.n_problems = 1
        self.n_cams = 0
        self.n_points = 0
        self._workspace = None

    def set_options(self, **kw):
        """Change options of this context (validated by the library), e.g. pcg_forcing_eta=0.1."""
        opt = Options()
        C.memmove(C.byref(opt), C.byref(self.options), C.sizeof(Options))
        for k, v in kw.items():
            if k not in dict(Options._fields_):
                raise TypeError(f"unknown option {k}")
            setattr(opt, k, v)
        self._check(self._api.set_options(self._h, C.byref(opt)))
        self.options = opt

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            self._api.destroy(self._h)
            self._h = None
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st: int):
        if st != OK:
            msg = self._api.last_error(self._h)
            raise SqrtBAError(st, msg.decode() if msg else "")

    # -- problem definition
    def set_problems(self, cam_off: Sequence[int], pt_off: Sequence[int]):
        co, po = _arr(cam_off, np.int64), _arr(pt_off, np.int64)
        self._check(self._api.set_problems(self._h, len(co) - 1, _ptr(co, C.c_int64), _ptr(po, C.c_int64)))
        self.n_problems = len(co) - 1

    def set_cameras(self, params):
        a = _arr(params, self._rt)
        self._check(self._api.set_cameras(self._h, a.size // 9 if a.size else 0, _ptr(a, self._rc)))
        self.n_cams = a.size // 9

    def set_landmarks(self, xyz):
        a = _arr(xyz, self._rt)
        self._check(self._api.set_landmarks(self._h, a.size // 3 if a.size else 0, _ptr(a, self._rc)))
        self.n_points = a.size // 3

    def set_observations(self, cam, pt, uv):
        c, p, u = _arr(cam, np.int32), _arr(pt, np.int32), _arr(uv, self._rt)
        if c.shape != p.shape or u.size != 2 * c.size:
            raise ValueError("observation arrays have inconsistent shapes")
        self._check(self._api.set_observations(self._h, c.size, _ptr(c, C.c_int32), _ptr(p, C.c_int32),
                                                  _ptr(u, self._rc)))

    def load(self, cameras, points, obs_cam, obs_pt, obs_uv, cam_off=None, pt_off=None):
        if cam_off is not None:
            self.set_problems(cam_off, pt_off)
        self.set_cameras(cameras)
        self.set_landmarks(points)
        self.set_observations(obs_cam, obs_pt, obs_uv)
        return self

    # -- the same from device-resident arrays (e.g. CUDA tensors); the library copies them
    def _device(self, t, dtype, n, what):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.dtype == dtype
                and t.numel() == n):
            raise ValueError(f"{what}: need a contiguous CUDA tensor of {n} {dtype} elements")
        return P(t.data_ptr())

    def _tdtype(self):
        import torch
        return torch.float64 if self.precision == 64 else torch.float32

    def set_cameras_device(self, params):
        n = params.numel() // 9
        self._check(self._api.set_cameras_device(self._h, n, self._device(params, self._tdtype(), 9 * n, "cameras")))
        self.n_cams = n

    def set_landmarks_device(self, xyz):
        n = xyz.numel() // 3
        self._check(self._api.set_landmarks_device(self._h, n, self._device(xyz, self._tdtype(), 3 * n, "landmarks")))
        self.n_points = n

    def set_observations_device(self, cam, pt, uv):
        import torch
        n = cam.numel()
        self._check(self._api.set_observations_device(
            self._h, n, self._device(cam, torch.int32, n, "observation cameras"),
            self._device(pt, torch.int32, n, "observation landmarks"),
            self._device(uv, self._tdtype(), 2 * n, "observation pixels")))

    def load_device(self, cameras, points, obs_cam, obs_pt, obs_uv, cam_off=None, pt_off=None):
        """load() from CUDA tensors (offsets, if any, stay host sequences)."""
        if cam_off is not None:
            self.set_problems(cam_off, pt_off)
        self.set_cameras_device(cameras)
        self.set_landmarks_device(points)
        self.set_observations_device(obs_cam, obs_pt, obs_uv)
        return self

    def get_cameras_device(self, out):
        self._check(self._api.get_cameras_device(self._h, self._device(out, self._tdtype(), 9 * self.n_cams, "out")))
        return out

    def get_landmarks_device(self, out):
        self._check(self._api.get_landmarks_device(self._h, self._device(out, self._tdtype(), 3 * self.n_points,
                                                                          "out")))
        return out

    def workspace_bytes(self) -> int:
        n = C.c_uint64()
        self._check(self._api.workspace_bytes(self._h, C.byref(n)))
        return int(n.value)

    def bind_torch_workspace(self, device="cuda"):
        """Allocate the device workspace with PyTorch and hand it to the library."""
        import torch
        nbytes = self.workspace_bytes()
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        addr = ws.data_ptr()
        off = (-addr) % 256
        self._check(self._api.bind_workspace(self._h, P(addr + off), nbytes))
        self._workspace = ws
        return ws

    def set_active(self, mask):
        m = _arr(mask, np.uint8)
        self._check(self._api.set_active(self._h, _ptr(m, C.c_uint8)))

    # -- the LM step
    def linearize(self) -> np.ndarray:
        out = np.zeros(self.n_problems)
        self._check(self._api.linearize(self._h, _ptr(out, C.c_double)))
        return out

    def marginalize(self):
        self._check(self._api.marginalize(self._h))

    def damp(self, lam):
        l = _arr(np.broadcast_to(np.asarray(lam, dtype=np.float64), (self.n_problems,)), np.float64)
        self._check(self._api.damp(self._h, _ptr(l, C.c_double)))

    def solve(self):
        it = np.zeros(self.n_problems, np.int32)
        rel = np.zeros(self.n_problems)
        st = np.zeros(self.n_problems, np.int32)
        self._check(self._api.solve(self._h, _ptr(it, C.c_int32), _ptr(rel, C.c_double), _ptr(st, C.c_int32)))
        return it, rel, st

    def back_substitute(self) -> np.ndarray:
        out = np.zeros(self.n_problems)
        self._check(self._api.back_substitute(self._h, _ptr(out, C.c_double)))
        return out

    def update(self) -> np.ndarray:
        out = np.zeros(self.n_problems)
        self._check(self._api.update(self._h, _ptr(out, C.c_double)))
        return out

    def commit(self, accept):
        a = _arr(np.broadcast_to(np.asarray(accept, dtype=np.uint8), (self.n_problems,)), np.uint8)
        self._check(self._api.commit(self._h, _ptr(a, C.c_uint8)))

    def lm_solve(self, tol_cost=None) -> List[Report]:
        reps = (LMReport * self.n_problems)()
        if tol_cost is None:
            self._check(self._api.lm_solve(self._h, reps))
        else:
            t = _arr(np.broadcast_to(np.asarray(tol_cost, dtype=np.float64), (self.n_problems,)), np.float64)
            self._check(self._api.lm_solve_tracked(self._h, _ptr(t, C.c_double), reps))
        return [Report(r.initial_cost, r.final_cost, r.iterations, r.accepted, r.total_pcg_iters,
                       LM_STATUS.get(r.status, str(r.status)), r.solve_seconds, r.time_to_tol) for r in reps]

    def history(self, problem: int = 0) -> List[dict]:
        n = C.c_int32()
        self._check(self._api.get_lm_history(self._h, problem, None, 0, C.byref(n)))
        recs = (LMRecord * max(1, n.value))()
        self._check(self._api.get_lm_history(self._h, problem, recs, n.value, C.byref(n)))
        return [{"iter": r.iter, "accepted": bool(r.accepted), "pcg_iters": r.pcg_iters,
                 "pcg_status": PCG_STATUS.get(r.pcg_status, r.pcg_status), "lambda": r.lambda_, "cost": r.cost,
                 "new_cost": r.new_cost, "pred": r.model_decrease, "rel_res": r.rel_res, "t": r.t_seconds}
                for r in recs[: n.value]]

    def get_cameras(self) -> np.ndarray:
        out = np.zeros((self.n_cams, 9), self._rt)
        self._check(self._api.get_cameras(self._h, _ptr(out, self._rc)))
        return out

    def get_landmarks(self) -> np.ndarray:
        out = np.zeros((self.n_points, 3), self._rt)
        self._check(self._api.get_landmarks(self._h, _ptr(out, self._rc)))
        return out

    # -- learned preconditioner
    def mlp_init(self, seed: int = 0):
        self._check(self._api.mlp_init(self._h, seed))

    def mlp_set_params(self, params):
        a = _arr(params, np.float32)
        if a.size != self._api.mlp_num_params():
            raise ValueError("wrong parameter count")
        self._check(self._api.mlp_set_params(self._h, _ptr(a, C.c_float)))

    def mlp_get_params(self) -> np.ndarray:
        out = np.zeros(self._api.mlp_num_params(), np.float32)
        self._check(self._api.mlp_get_params(self._h, _ptr(out, C.c_float)))
        return out

    def set_preconditioner(self, mode: str):
        self._check(self._api.set_preconditioner(self._h, {"block_jacobi": 0, "learned": 1}[mode]))

    def pcg_trace(self, max_solves: int, iters_per_solve: int):
        self._check(self._api.pcg_trace(self._h, max_solves, iters_per_solve))

    def trace_size(self):
        a, b = C.c_int32(), C.c_int32()
        self._check(self._api.trace_size(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def mlp_train(self, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0) -> np.ndarray:
        out = np.zeros(max(steps, 1))
        self._check(self._api.mlp_train(self._h, steps, batch, lr, seed, _ptr(out, C.c_double)))
        return out[:steps]

    def mlp_eval(self, feats, lfac, p, q):
        f, l, pp, qq = (_arr(a, np.float32) for a in (feats, lfac, p, q))
        n = f.shape[0]
        loss = C.c_double()
        grad = np.zeros(self._api.mlp_num_params(), np.float32)
        self._check(self._api.mlp_eval(self._h, n, _ptr(f, C.c_float), _ptr(l, C.c_float), _ptr(pp, C.c_float),
                                          _ptr(qq, C.c_float), C.byref(loss), _ptr(grad, C.c_float)))
        return loss.value, grad

    def learned_stats(self) -> dict:
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self._api.learned_stats(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return {"learned_solves": a.value, "fallbacks": b.value, "wasted_iters": c.value}

    def debug_features(self):
        f = np.zeros((self.n_cams, 64), np.float32)
        l = np.zeros((self.n_cams, 45), np.float32)
        self._check(self._api.debug_features(self._h, _ptr(f, C.c_float), _ptr(l, C.c_float)))
        return f, l

    def debug_learned_precond(self) -> np.ndarray:
        out = np.zeros((self.n_cams, 9, 9), np.float32)
        self._check(self._api.debug_learned_precond(self._h, _ptr(out, C.c_float)))
        return out

    # -- measurement and snapshots
    def profile_enable(self, on: bool = True):
        self._check(self._api.profile_enable(self._h, 1 if on else 0))

    def profile(self) -> dict:
        pr = Profile()
        self._check(self._api.profile_get(self._h, C.byref(pr)))
        return {name: {"ms": pr.ms[i], "launches": int(pr.launches[i]), "bytes": pr.bytes[i],
                       "units": int(pr.units[i])} for i, name in enumerate(STAGES)}

    # -- launch shapes of the product
    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(self._api.get_tuning(self._h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **shape):
        t = Tuning(**{**self.get_tuning(), **shape})
        self._check(self._api.set_tuning(self._h, C.byref(t)))

    def autotune(self, reps: int = 10):
        """Pick the fastest product launch shapes on this problem; returns
        (chosen shapes, [(shapes, ms per product), ...] of every candidate)."""
        best = Tuning()
        trials = (TuningTrial * 32)()
        n = C.c_int32()
        self._check(self._api.autotune(self._h, reps, C.byref(best), trials, 32, C.byref(n)))
        return best.as_dict(), [(trials[i].shape.as_dict(), trials[i].ms) for i in range(min(n.value, 32))]

    def time_product(self, reps: int = 50):
        """(mean ms per product over reps back-to-back launches, algorithmic bytes per product)."""
        ms, by = C.c_double(), C.c_double()
        self._check(self._api.time_product(self._h, reps, C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def save_state(self):
        self._check(self._api.save_state(self._h))

    def restore_state(self):
        self._check(self._api.restore_state(self._h))

    # -- inspection exports
    def debug_bookkeeping(self) -> dict:
        n = C.c_int64()
        self._check(self._api.debug_bookkeeping(self._h, C.byref(n), None, None, None, None))
        perm = np.zeros(n.value, np.int64)
        lm_off = np.zeros(self.n_points + 1, np.int64)
        la = np.zeros(self.n_points, np.uint8)
        ca = np.zeros(self.n_cams, np.uint8)
        self._check(self._api.debug_bookkeeping(self._h, C.byref(n), _ptr(perm, C.c_int64),
                                                   _ptr(lm_off, C.c_int64), _ptr(la, C.c_uint8),
                                                   _ptr(ca, C.c_uint8)))
        return {"obs_perm": perm, "lm_off": lm_off, "lm_active": la.astype(bool), "cam_active": ca.astype(bool)}

    def debug_linearization(self):
        n = len(self.debug_bookkeeping()["obs_perm"])
        r = np.zeros((n, 2), self._rt)
        Jp = np.zeros((n, 2, 9), self._rt)
        Jl = np.zeros((n, 2, 3), self._rt)
        self._check(self._api.debug_linearization(self._h, _ptr(r, self._rc), _ptr(Jp, self._rc),
                                                     _ptr(Jl, self._rc)))
        return r, Jp, Jl

    def debug_scales(self):
        sc = np.zeros((self.n_cams, 9), self._rt)
        sp = np.zeros((self.n_points, 3), self._rt)
        self._check(self._api.debug_scales(self._h, _ptr(sc, self._rc), _ptr(sp, self._rc)))
        return sc, sp

    def debug_rcs_matvec(self, V) -> np.ndarray:
        V = _arr(V, self._rt)
        V2 = V.reshape(-1, 9 * self.n_cams)
        out = np.zeros_like(V2)
        self._check(self._api.debug_rcs_matvec(self._h, V2.shape[0], _ptr(V2, self._rc), _ptr(out, self._rc)))
        return out.reshape(V.shape)

    def rcs_matvec_noalloc(self, v, out):
        """out = (B^T B + lambda I) v for CUDA tensors v, out of 9 n_cams elements, on the
        context's stream without synchronizing or allocating (static scratch)."""
        n = 9 * self.n_cams
        self._check(self._api.rcs_matvec_noalloc(self._h, self._device(v, self._tdtype(), n, "v"),
                                                 self._device(out, self._tdtype(), n, "out")))
        return out

    def debug_rhs(self) -> np.ndarray:
        out = np.zeros(9 * self.n_cams, self._rt)
        self._check(self._api.debug_rhs(self._h, _ptr(out, self._rc)))
        return out

    def debug_precond(self) -> np.ndarray:
        out = np.zeros((self.n_cams, 9, 9), self._rt)
        self._check(self._api.debug_precond(self._h, _ptr(out, self._rc)))
        return out

    def debug_block(self, pt: int):
        k = C.c_int32()
        self._check(self._api.debug_block(self._h, pt, C.byref(k), None, None))
        if k.value == 0:
            return 0, None, None
        kk = k.value
        out = np.zeros((2 * kk + 3, 9 * kk + 4), self._rt)
        fac = np.zeros(24, self._rt)
        self._check(self._api.debug_block(self._h, pt, C.byref(k), _ptr(out, self._rc), _ptr(fac, self._rc)))
        return kk, out, fac

    def debug_solution(self):
        dxp = np.zeros(9 * self.n_cams, self._rt)
        dxl = np.zeros((self.n_points, 3), self._rt)
        self._check(self._api.debug_solution(self._h, _ptr(dxp, self._rc), _ptr(dxl, self._rc)))
        return dxp, dxl

    def debug_set_pose_increment(self, dxp):
        a = _arr(dxp, self._rt)
        self._check(self._api.debug_set_pose_increment(self._h, _ptr(a, self._rc)))
