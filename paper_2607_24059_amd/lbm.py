"""ctypes binding of liblbm.so (include/lbm.h): argument marshalling only.

Every function below has the name and the argument order of the C entry
point it wraps.  The library must be built in-tree first
(``python -m paper_2607_24059_amd.build``); there is no fallback path: if the
shared library is missing, loading raises.

`Engine` is a small convenience owner: it allocates the device workspace
with torch (torch is used for device memory and the stream only) and keeps
the context pointer.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_EUNSTABLE, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = range(7)
STORAGE = {"f32": 0, "f16_dev": 1, "bf16_dev": 2, "f16_dev_r32": 3, "bf16_dev_r32": 4,
           "f32_raw": 5, "f64": 6, "f16_neq": 7, "f32_moments": 8}
LBM_WARN_LOWFREQ = 0x1


class lbm_params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("storage", C.c_int32),
        ("n", C.c_int64 * 3),
        ("dx", C.c_double),
        ("dt", C.c_double),
        ("nu", C.c_double),
        ("omega_rho", C.c_double),
        ("omega_q", C.c_double),
        ("alpha_rho", C.c_double),
        ("gamma", C.c_double),
        ("rho_ref", C.c_double),
    ]


class lbm_diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64),
        ("time", C.c_double),
        ("mass", C.c_double),
        ("mom", C.c_double * 3),
        ("kinetic", C.c_double),
        ("enstrophy", C.c_double),
        ("div_l2", C.c_double),
        ("max_u", C.c_double),
        ("rho_min", C.c_double),
        ("rho_max", C.c_double),
        ("nonfinite", C.c_int64),
        ("flags", C.c_uint32),
    ]


class lbm_walls(C.Structure):
    _fields_ = [("rho_out", C.c_double), ("u_bottom", C.c_double), ("u_top", C.c_double),
                ("correction", C.c_int32)]


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {lbm_strerror(status)} (status {status})")
        self.status = status


_lib = None

# name -> (restype, argtypes) of every exported entry point
SIGNATURES = {
    "lbm_check_params": (C.c_int, [C.POINTER(lbm_params), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_uint32)]),
    "lbm_workspace_bytes": (C.c_size_t, [C.POINTER(lbm_params)]),
    "lbm_init": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(lbm_params), C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_size_t, C.c_void_p]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_set_fusion": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_fusion": (C.c_int32, [C.c_void_p]),
    "lbm_set_walls": (C.c_int, [C.c_void_p, C.POINTER(lbm_walls), C.c_void_p]),
    "lbm_moments": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_moments_device": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_diagnostics": (C.c_int, [C.c_void_p, C.POINTER(lbm_diag)]),
    "lbm_diagnostics_noalloc": (C.c_int, [C.c_void_p, C.POINTER(lbm_diag)]),
    "lbm_state_bytes": (C.c_size_t, [C.c_void_p]),
    "lbm_save_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lbm_load_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lbm_step_count": (C.c_int64, [C.c_void_p]),
    "lbm_destroy": (None, [C.c_void_p]),
    "lbm_strerror": (C.c_char_p, [C.c_int]),
    "lbm_copy_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
}


def lib():
    """Load liblbm.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2607_24059_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ok(status: int, where: str) -> None:
    if status != LBM_OK:
        raise LbmError(status, where)


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    if not (a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]):
        raise TypeError("host arrays must be C-contiguous float64")
    return a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------- #
# one function per C entry point                                              #
# --------------------------------------------------------------------------- #

def make_params(dim, n, dx, dt, nu, omega_rho=6 / 5, omega_q=23 / 20, alpha_rho=3 / 40,
                gamma=1.0, rho_ref=1.0, storage="f32") -> lbm_params:
    n = list(n) + [1] * (3 - len(n))
    return lbm_params(int(dim), STORAGE[storage] if isinstance(storage, str) else int(storage),
                      (C.c_int64 * 3)(*[int(v) for v in n]), float(dx), float(dt), float(nu),
                      float(omega_rho), float(omega_q), float(alpha_rho), float(gamma), float(rho_ref))


def lbm_check_params(p: lbm_params):
    mu, aq, fl = C.c_double(), C.c_double(), C.c_uint32()
    st = lib().lbm_check_params(C.byref(p), C.byref(mu), C.byref(aq), C.byref(fl))
    return st, mu.value, aq.value, fl.value


def lbm_workspace_bytes(p: lbm_params) -> int:
    return int(lib().lbm_workspace_bytes(C.byref(p)))


def lbm_init(p: lbm_params, u0: np.ndarray, rho0: np.ndarray | None, workspace_ptr: int,
             ws_bytes: int, stream_ptr: int) -> int:
    ctx = C.c_void_p()
    st = lib().lbm_init(C.byref(ctx), C.byref(p), _ptr(u0), _ptr(rho0), C.c_void_p(workspace_ptr),
                        C.c_size_t(ws_bytes), C.c_void_p(stream_ptr))
    _ok(st, "lbm_init")
    return ctx.value


def lbm_step(ctx: int, nsteps: int) -> None:
    _ok(lib().lbm_step(C.c_void_p(ctx), C.c_int64(nsteps)), "lbm_step")


def lbm_set_fusion(ctx: int, steps_per_launch: int) -> None:
    _ok(lib().lbm_set_fusion(C.c_void_p(ctx), int(steps_per_launch)), "lbm_set_fusion")


def lbm_fusion(ctx: int) -> int:
    return int(lib().lbm_fusion(C.c_void_p(ctx)))


def lbm_set_walls(ctx: int, walls: lbm_walls | None, u_in: np.ndarray | None) -> None:
    if walls is None:
        _ok(lib().lbm_set_walls(C.c_void_p(ctx), None, None), "lbm_set_walls")
        return
    u = np.ascontiguousarray(u_in, dtype=np.float64)
    _ok(lib().lbm_set_walls(C.c_void_p(ctx), C.byref(walls), u.ctypes.data_as(C.c_void_p)), "lbm_set_walls")


def lbm_moments(ctx: int, rho: np.ndarray, q: np.ndarray | None) -> None:
    _ok(lib().lbm_moments(C.c_void_p(ctx), _ptr(rho), _ptr(q)), "lbm_moments")


def lbm_moments_device(ctx: int, out_ptr: int) -> None:
    _ok(lib().lbm_moments_device(C.c_void_p(ctx), C.c_void_p(out_ptr)), "lbm_moments_device")


def lbm_diagnostics(ctx: int) -> tuple[int, lbm_diag]:
    d = lbm_diag()
    st = lib().lbm_diagnostics(C.c_void_p(ctx), C.byref(d))
    if st not in (LBM_OK, LBM_ENONFINITE):
        raise LbmError(st, "lbm_diagnostics")
    return st, d


def lbm_diagnostics_noalloc(ctx: int) -> tuple[int, lbm_diag]:
    d = lbm_diag()
    st = lib().lbm_diagnostics_noalloc(C.c_void_p(ctx), C.byref(d))
    if st not in (LBM_OK, LBM_ENONFINITE):
        raise LbmError(st, "lbm_diagnostics_noalloc")
    return st, d


def lbm_state_bytes(ctx: int) -> int:
    return int(lib().lbm_state_bytes(C.c_void_p(ctx)))


def lbm_save_state(ctx: int, buf: np.ndarray) -> None:
    _ok(lib().lbm_save_state(C.c_void_p(ctx), buf.ctypes.data_as(C.c_void_p), C.c_size_t(buf.nbytes)),
        "lbm_save_state")


def lbm_load_state(ctx: int, buf: np.ndarray) -> None:
    _ok(lib().lbm_load_state(C.c_void_p(ctx), buf.ctypes.data_as(C.c_void_p), C.c_size_t(buf.nbytes)),
        "lbm_load_state")


def lbm_step_count(ctx: int) -> int:
    return int(lib().lbm_step_count(C.c_void_p(ctx)))


def lbm_destroy(ctx: int) -> None:
    lib().lbm_destroy(C.c_void_p(ctx))


def lbm_strerror(status: int) -> str:
    return lib().lbm_strerror(int(status)).decode()


def lbm_copy_probe(dst_ptr: int, src_ptr: int, nbytes: int, stream_ptr: int) -> None:
    _ok(lib().lbm_copy_probe(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), C.c_size_t(nbytes),
                             C.c_void_p(stream_ptr)), "lbm_copy_probe")


def diag_dict(d: lbm_diag, dim: int) -> dict:
    return {
        "step": d.step, "time": d.time, "mass": d.mass, "mom": list(d.mom)[:dim],
        "kinetic": d.kinetic, "enstrophy": d.enstrophy, "div_l2": d.div_l2, "max_u": d.max_u,
        "rho_min": d.rho_min, "rho_max": d.rho_max, "nonfinite": d.nonfinite, "flags": d.flags,
    }


# --------------------------------------------------------------------------- #
# convenience owner                                                           #
# --------------------------------------------------------------------------- #

@dataclass
class Engine:
    """One run on the current torch device and stream."""

    params: lbm_params
    ctx: int
    workspace: object  # torch uint8 tensor holding all device memory
    stream: object

    @classmethod
    def create(cls, params: lbm_params, u0: np.ndarray, rho0: np.ndarray | None = None,
               stream=None) -> "Engine":
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the engine needs a GPU")
        nbytes = lbm_workspace_bytes(params)
        if nbytes == 0:
            st, *_ = lbm_check_params(params)
            raise LbmError(st if st != LBM_OK else LBM_EINVAL, "lbm_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        stream = stream if stream is not None else torch.cuda.current_stream()
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        rho0 = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.float64)
        ctx = lbm_init(params, u0, rho0, ws.data_ptr(), nbytes, stream.cuda_stream)
        return cls(params, ctx, ws, stream)

    @property
    def dim(self) -> int:
        return self.params.dim

    @property
    def shape(self):
        n = list(self.params.n)
        return (n[1], n[0]) if self.dim == 2 else (n[2], n[1], n[0])

    def step(self, n: int) -> None:
        lbm_step(self.ctx, n)

    def set_walls(self, u_in, rho_out: float, u_bottom: float = 0.0, u_top: float = 0.0,
                  correction: bool = False) -> None:
        """Channel boundaries (inlet velocity u_in [2][ny], outlet density, walls);
        u_in=None restores periodic boundaries."""
        if u_in is None:
            lbm_set_walls(self.ctx, None, None)
        else:
            lbm_set_walls(self.ctx, lbm_walls(float(rho_out), float(u_bottom), float(u_top), int(bool(correction))),
                          u_in)

    def set_fusion(self, steps_per_launch: int) -> None:
        lbm_set_fusion(self.ctx, steps_per_launch)

    def fusion(self) -> int:
        return lbm_fusion(self.ctx)

    def moments(self):
        rho = np.empty(self.shape)
        q = np.empty((self.dim,) + self.shape)
        lbm_moments(self.ctx, rho, q)
        return rho, q

    def moments_device(self, out) -> None:
        lbm_moments_device(self.ctx, out.data_ptr())

    def diagnostics(self) -> dict:
        st, d = lbm_diagnostics(self.ctx)
        out = diag_dict(d, self.dim)
        out["status"] = st
        return out

    def save_state(self) -> np.ndarray:
        buf = np.empty(lbm_state_bytes(self.ctx), dtype=np.uint8)
        lbm_save_state(self.ctx, buf)
        return buf

    def load_state(self, buf: np.ndarray) -> None:
        lbm_load_state(self.ctx, buf)

    @property
    def steps(self) -> int:
        return lbm_step_count(self.ctx)

    def close(self) -> None:
        if self.ctx:
            lbm_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
