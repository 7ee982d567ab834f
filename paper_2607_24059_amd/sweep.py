"""Parameter sweeps of the Taylor-Green test (Section 5.1, Fig. 2 and Fig. 3)
as one batch of independent runs on the GPU.

The test: the Taylor-Green vortex u = (sin x cos y, -cos x sin y) e^{-2 nu t}
on the torus [0, 2 pi]^2 with 75 cells per direction, mu = dx^2/dt = 8, run
to t = 1, error = absolute discrete L2 norm of u_x - u_x,exact,
sqrt(dx^2 sum e^2).  The density starts well prepared, rho = 1 + dx^2 Phi with
the vortex's pressure Phi (the truncated density-pressure relation of
Section 3).  The paper does not give the viscosity of these runs; nu = 0.01
is used.

* Fig. 2: the (omega_rho, alpha_rho) plane with omega_q = 1 (relaxation
  scheme for the momentum sets), alpha_q set by nu.
* Fig. 3: omega_q (= omega_qx = omega_qy) varied for three
  (omega_rho, alpha_rho) pairs on one isoline of alpha_rho (1/omega_rho - 1/2),
  the density diffusivity of the modified equations (Section 3).

Every run advances in one batch (include/lbm_batch.h): one persistent launch
per five time steps for all runs together.  The error of each run is evaluated
from its FP64 moments.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

import inputs

from . import batch

# (omega_rho, alpha_rho) pairs of Section 5.1 (one isoline of the density diffusivity)
PAIRS = ((1.0, 1.0 / 20.0), (6.0 / 5.0, 3.0 / 40.0), (3.0 / 2.0, 3.0 / 20.0))


@dataclass(frozen=True)
class TaylorGreen:
    n: int = 75
    nu: float = 0.01
    mu: float = 8.0
    t_final: float = 1.0
    prepared: bool = True

    @property
    def dx(self) -> float:
        return 2.0 * math.pi / self.n

    @property
    def dt(self) -> float:
        return self.dx * self.dx / self.mu

    def steps(self) -> int:
        return int(round(self.t_final / self.dt))

    def initial(self):
        u0 = inputs.taylor_green(self.n)
        rho0 = None
        if self.prepared:
            rho0 = inputs.well_prepared_density(inputs.taylor_green_pressure(self.n), self.dx)
        return u0, rho0

    def error(self, rho: np.ndarray, q: np.ndarray, u0: np.ndarray, steps: int) -> float:
        """Absolute discrete L2 error on u_x at t = steps dt."""
        decay = math.exp(-2.0 * self.nu * steps * self.dt)
        e = q[0] / rho - u0[0] * decay
        return float(math.sqrt(self.dx ** 2 * float(np.sum(e * e))))


def figure2_points(omega_rho=None, alpha_rho=None):
    """(omega_rho, alpha_rho, omega_q = 1) over a grid of the density parameters."""
    if omega_rho is None:
        omega_rho = np.round(np.arange(1.0, 1.96, 0.05), 4)
    if alpha_rho is None:
        alpha_rho = np.round(np.arange(0.01, 0.2501, 0.01), 5)
    return [(float(w), float(a), 1.0) for a in alpha_rho for w in omega_rho]


def figure3_points(omega_q=None, pairs=PAIRS):
    """(omega_rho, alpha_rho, omega_q) for each pair and each omega_q."""
    if omega_q is None:
        omega_q = np.round(np.arange(1.0, 1.6001, 0.025), 4)
    return [(float(wr), float(ar), float(wq)) for wr, ar in pairs for wq in omega_q]


@dataclass
class SweepResult:
    points: list
    errors: np.ndarray    # per run; inf where the run did not stay finite
    steps: int
    cells: int            # cells over all runs
    seconds: float        # wall time of the batched time stepping (synchronised)

    @property
    def glups(self) -> float:
        return self.cells * self.steps / self.seconds / 1e9

    def grid(self, nw: int, na: int, start: int = 0) -> np.ndarray:
        """Errors of a figure2_points sweep of nw x na runs placed at run
        `start` of the batch, as [alpha index][omega index]."""
        return self.errors[start:start + nw * na].reshape(na, nw)


def run(points, tg: TaylorGreen = TaylorGreen(), storage: str = "f32", fuse: int | None = None,
        autotune: bool = False, keep_moments: bool = False):
    """Advance one run per (omega_rho, alpha_rho, omega_q) point in one batch
    to t_final and return the errors on u_x (and, with keep_moments, the
    moments of every run)."""
    import torch

    u0, rho0 = tg.initial()
    specs = [batch.make_run((tg.n, tg.n), tg.dx, tg.dt, tg.nu, omega_rho=wr, omega_q=wq, alpha_rho=ar)
             for wr, ar, wq in points]
    b = batch.Batch.create(2, storage, specs, [u0] * len(specs), None if rho0 is None else [rho0] * len(specs))
    try:
        if autotune:
            b.autotune()
        if fuse is not None:
            b.set_fusion(fuse)
        steps = tg.steps()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        seconds = time.perf_counter() - t0
        errors = np.empty(len(points))
        moments = []
        for r in range(len(points)):
            rho, q = b.moments(r)
            e = tg.error(rho, q, u0, steps) if np.all(np.isfinite(q)) and np.all(rho > 0) else math.inf
            errors[r] = e if math.isfinite(e) else math.inf
            if keep_moments:
                moments.append((rho, q))
        cells, _, _ = b.info()
    finally:
        b.close()
    res = SweepResult(list(points), errors, steps, int(cells), seconds)
    return (res, moments) if keep_moments else res
