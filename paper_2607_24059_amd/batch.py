"""ctypes binding of the batched engine (include/lbm_batch.h): marshalling only.

`Batch` owns a torch device workspace and the batch handle.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from .lbm import STORAGE, LbmError, _ok, lib

LBM_OK = 0


class lbm_run_spec(C.Structure):
    _fields_ = [
        ("n", C.c_int64 * 3),
        ("dx", C.c_double),
        ("dt", C.c_double),
        ("nu", C.c_double),
        ("omega_rho", C.c_double),
        ("omega_q", C.c_double),
        ("alpha_rho", C.c_double),
        ("rho_ref", C.c_double),
    ]


SIGNATURES = {
    "lbm_batch_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(lbm_run_spec)]),
    "lbm_batch_init": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_int32,
                                 C.POINTER(lbm_run_spec), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                 C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_int32)]),
    "lbm_batch_autotune": (C.c_int, [C.c_void_p, C.c_char_p]),
    "lbm_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_batch_moments": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "lbm_batch_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64)]),
    "lbm_batch_tile_width": (C.c_int32, [C.c_void_p, C.c_int32]),
    "lbm_batch_grid": (C.c_int32, [C.c_void_p]),
    "lbm_batch_fused_grid": (C.c_int32, [C.c_void_p]),
    "lbm_batch_fused_tile": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbm_batch_set_fused_shape": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_batch_set_fused_grid": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_batch_set_fusion": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_batch_fusion": (C.c_int32, [C.c_void_p]),
    "lbm_batch_destroy": (None, [C.c_void_p]),
}

_bound = False


def blib():
    global _bound
    L = lib()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def make_run(n, dx, dt, nu, omega_rho=6 / 5, omega_q=23 / 20, alpha_rho=3 / 40, rho_ref=1.0):
    n = list(n) + [1] * (3 - len(n))
    return lbm_run_spec((C.c_int64 * 3)(*[int(v) for v in n]), float(dx), float(dt), float(nu),
                        float(omega_rho), float(omega_q), float(alpha_rho), float(rho_ref))


def _spec_array(runs):
    arr = (lbm_run_spec * len(runs))()
    for i, r in enumerate(runs):
        arr[i] = r
    return arr


def lbm_batch_workspace_bytes(dim: int, storage, runs) -> int:
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    return int(blib().lbm_batch_workspace_bytes(dim, st, len(runs), _spec_array(runs)))


def lbm_batch_init(dim, storage, runs, u0s, rho0s, workspace_ptr, ws_bytes, stream_ptr) -> int:
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    n = len(runs)
    for a in u0s:
        if not (a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]):
            raise TypeError("u0 arrays must be C-contiguous float64")
    uptr = (C.c_void_p * n)(*[a.ctypes.data for a in u0s])
    rptr = None
    if rho0s is not None:
        rptr = (C.c_void_p * n)(*[(a.ctypes.data if a is not None else None) for a in rho0s])
    bad = C.c_int32(-1)
    h = C.c_void_p()
    s = blib().lbm_batch_init(C.byref(h), dim, st, n, _spec_array(runs), uptr, rptr,
                              C.c_void_p(workspace_ptr), C.c_size_t(ws_bytes), C.c_void_p(stream_ptr),
                              C.byref(bad))
    if s != LBM_OK:
        raise LbmError(s, f"lbm_batch_init (run {bad.value})")
    return h.value


def lbm_batch_autotune(h: int, cache_path: str | None) -> None:
    _ok(blib().lbm_batch_autotune(C.c_void_p(h), cache_path.encode() if cache_path else None),
        "lbm_batch_autotune")


def lbm_batch_step(h: int, nsteps: int) -> None:
    _ok(blib().lbm_batch_step(C.c_void_p(h), C.c_int64(nsteps)), "lbm_batch_step")


def lbm_batch_moments(h: int, run: int, rho: np.ndarray, q: np.ndarray | None) -> None:
    _ok(blib().lbm_batch_moments(C.c_void_p(h), run, rho.ctypes.data_as(C.c_void_p),
                                 None if q is None else q.ctypes.data_as(C.c_void_p)), "lbm_batch_moments")


def lbm_batch_info(h: int):
    cells, tiles, steps = C.c_int64(), C.c_int64(), C.c_int64()
    _ok(blib().lbm_batch_info(C.c_void_p(h), C.byref(cells), C.byref(tiles), C.byref(steps)), "lbm_batch_info")
    return cells.value, tiles.value, steps.value


def lbm_batch_tile_width(h: int, run: int) -> int:
    return int(blib().lbm_batch_tile_width(C.c_void_p(h), run))


def lbm_batch_grid(h: int) -> int:
    return int(blib().lbm_batch_grid(C.c_void_p(h)))


def lbm_batch_fused_grid(h: int) -> int:
    return int(blib().lbm_batch_fused_grid(C.c_void_p(h)))


def lbm_batch_fused_tile(h: int, run: int) -> tuple[int, int]:
    tx, ty = C.c_int32(), C.c_int32()
    _ok(blib().lbm_batch_fused_tile(C.c_void_p(h), run, C.byref(tx), C.byref(ty)), "lbm_batch_fused_tile")
    return tx.value, ty.value


def lbm_batch_set_fused_shape(h: int, shape: int) -> None:
    _ok(blib().lbm_batch_set_fused_shape(C.c_void_p(h), int(shape)), "lbm_batch_set_fused_shape")


def lbm_batch_set_fused_grid(h: int, blocks_per_cu: int) -> None:
    _ok(blib().lbm_batch_set_fused_grid(C.c_void_p(h), int(blocks_per_cu)), "lbm_batch_set_fused_grid")


def lbm_batch_set_fusion(h: int, steps_per_launch: int) -> None:
    _ok(blib().lbm_batch_set_fusion(C.c_void_p(h), steps_per_launch), "lbm_batch_set_fusion")


def lbm_batch_fusion(h: int) -> int:
    return int(blib().lbm_batch_fusion(C.c_void_p(h)))


def lbm_batch_destroy(h: int) -> None:
    blib().lbm_batch_destroy(C.c_void_p(h))


@dataclass
class Batch:
    dim: int
    runs: list
    handle: int
    workspace: object
    stream: object

    @classmethod
    def create(cls, dim, storage, runs, u0s, rho0s=None, stream=None) -> "Batch":
        import torch
        nbytes = lbm_batch_workspace_bytes(dim, storage, runs)
        if nbytes == 0:
            from .lbm import lbm_check_params, make_params
            for i, r in enumerate(runs):
                p = make_params(dim, tuple(r.n)[:dim], r.dx, r.dt, r.nu, r.omega_rho, r.omega_q,
                                r.alpha_rho, rho_ref=r.rho_ref, storage=storage)
                st, *_ = lbm_check_params(p)
                if st != LBM_OK:
                    raise LbmError(st, f"lbm_batch_workspace_bytes (run {i})")
            raise LbmError(1, "lbm_batch_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        stream = stream if stream is not None else torch.cuda.current_stream()
        u0s = [np.ascontiguousarray(u, dtype=np.float64) for u in u0s]
        h = lbm_batch_init(dim, storage, runs, u0s, rho0s, ws.data_ptr(), nbytes, stream.cuda_stream)
        return cls(dim, list(runs), h, ws, stream)

    def autotune(self, cache_path: str | None = None) -> None:
        lbm_batch_autotune(self.handle, cache_path)

    def step(self, n: int) -> None:
        lbm_batch_step(self.handle, n)

    def shape(self, r: int):
        n = list(self.runs[r].n)
        return (n[1], n[0]) if self.dim == 2 else (n[2], n[1], n[0])

    def moments(self, r: int):
        shp = self.shape(r)
        rho = np.empty(shp)
        q = np.empty((self.dim,) + shp)
        lbm_batch_moments(self.handle, r, rho, q)
        return rho, q

    def info(self):
        return lbm_batch_info(self.handle)

    def grid(self) -> int:
        return lbm_batch_grid(self.handle)

    def fused_grid(self) -> int:
        return lbm_batch_fused_grid(self.handle)

    def set_fusion(self, steps_per_launch: int) -> None:
        lbm_batch_set_fusion(self.handle, steps_per_launch)

    def fusion(self) -> int:
        return lbm_batch_fusion(self.handle)

    def tile_width(self, r: int) -> int:
        return lbm_batch_tile_width(self.handle, r)

    def fused_tile(self, r: int) -> tuple[int, int]:
        return lbm_batch_fused_tile(self.handle, r)

    def set_fused_shape(self, shape: int) -> None:
        lbm_batch_set_fused_shape(self.handle, shape)

    def set_fused_grid(self, blocks_per_cu: int) -> None:
        lbm_batch_set_fused_grid(self.handle, blocks_per_cu)

    def close(self) -> None:
        if self.handle:
            lbm_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
