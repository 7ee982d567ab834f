"""ctypes binding of the batched linear-spectrum kernels (include/lbm_spectrum.h):
argument marshalling only.

The C entry points take device arrays; `matrix` and `eigenvalues` below copy
host inputs to the device with torch, call the entry point on torch's current
stream and copy the results back.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from .lbm import _ok, lib


class lbm_lin_state(C.Structure):
    _fields_ = [
        ("mu", C.c_double),
        ("dx", C.c_double),
        ("omega_rho", C.c_double),
        ("omega_q", C.c_double),
        ("alpha_rho", C.c_double),
        ("alpha_q", C.c_double),
        ("rho_bar", C.c_double),
        ("q_bar", C.c_double * 3),
        ("dp_drho", C.c_double),
    ]


SIGNATURES = {
    "lbm_spectrum_order": (C.c_int32, [C.c_int32]),
    "lbm_spectrum_matrix": (C.c_int, [C.c_int32, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
    "lbm_spectrum_eigs": (C.c_int, [C.c_int32, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}

_bound = False


def slib():
    global _bound
    L = lib()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def make_state(mu, dx=1e-6, omega_rho=1.0, omega_q=1.0, alpha_rho=0.25, alpha_q=0.0, rho_bar=1.0,
               q_bar=(0.0, 0.0, 0.0), dp_drho=1.0) -> lbm_lin_state:
    q = list(q_bar) + [0.0] * (3 - len(q_bar))
    return lbm_lin_state(float(mu), float(dx), float(omega_rho), float(omega_q), float(alpha_rho),
                         float(alpha_q), float(rho_bar), (C.c_double * 3)(*[float(v) for v in q]),
                         float(dp_drho))


def lbm_spectrum_order(dim: int) -> int:
    return int(slib().lbm_spectrum_order(dim))


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _states_dev(states):
    import torch
    arr = (lbm_lin_state * len(states))(*states)
    raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
    return torch.from_numpy(raw).cuda()


def _inputs(dim, states, theta, state_of_point):
    theta = np.asarray(theta, dtype=np.float64).reshape(-1, dim)
    npts = theta.shape[0]
    st = _states_dev(states)
    th = _dev(theta, np.float64)
    idx = None if state_of_point is None else _dev(np.asarray(state_of_point).reshape(npts), np.int32)
    return npts, st, th, idx


def matrix(dim: int, states, theta, state_of_point=None) -> np.ndarray:
    """E(theta) of each point as complex [npts][n][n]."""
    import torch
    npts, st, th, idx = _inputs(dim, states, theta, state_of_point)
    n = lbm_spectrum_order(dim)
    out = torch.empty((npts, n, n, 2), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    _ok(slib().lbm_spectrum_matrix(dim, npts, st.data_ptr(), len(states),
                                   None if idx is None else idx.data_ptr(), th.data_ptr(), out.data_ptr(),
                                   s.cuda_stream), "lbm_spectrum_matrix")
    e = out.cpu().numpy()
    return e[..., 0] + 1j * e[..., 1]


class Problem:
    """Device inputs and outputs of one lbm_spectrum_eigs call; `launch`
    enqueues the call on a stream, `results` copies the outputs back."""

    def __init__(self, dim: int, states, theta, state_of_point=None):
        import torch
        self.dim = dim
        self.nstates = len(states)
        self.npts, self.st, self.th, self.idx = _inputs(dim, states, theta, state_of_point)
        n = lbm_spectrum_order(dim)
        self.eig = torch.empty((self.npts, n, 2), dtype=torch.float64, device="cuda")
        self.rad = torch.empty(self.npts, dtype=torch.float64, device="cuda")
        self.info = torch.empty(self.npts, dtype=torch.int32, device="cuda")
        self.flops = torch.empty(self.npts, dtype=torch.float64, device="cuda")

    def launch(self, stream=None) -> None:
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _ok(slib().lbm_spectrum_eigs(self.dim, self.npts, self.st.data_ptr(), self.nstates,
                                     None if self.idx is None else self.idx.data_ptr(), self.th.data_ptr(),
                                     self.eig.data_ptr(), self.rad.data_ptr(), self.info.data_ptr(),
                                     self.flops.data_ptr(), s.cuda_stream), "lbm_spectrum_eigs")

    def results(self) -> dict:
        e = self.eig.cpu().numpy()
        return {"eig": e[..., 0] + 1j * e[..., 1], "radius": self.rad.cpu().numpy(),
                "info": self.info.cpu().numpy(), "flops": self.flops.cpu().numpy()}


def eigenvalues(dim: int, states, theta, state_of_point=None):
    """Eigenvalues (complex [npts][n]), spectral radius [npts], QR sweeps or
    failure code [npts] and counted flops [npts] of every point."""
    pb = Problem(dim, states, theta, state_of_point)
    pb.launch()
    return pb.results()
