"""The allocation-free diagnostics entry point (lbm_diagnostics_noalloc)
against lbm_diagnostics, through the C ABI.

Both run the same kernels in the same fixed reduction order, so every field
must be equal bit for bit.  Two calls in a row, the second on a smaller grid
(fewer partials than the first left in the shared static scratch), then a
third on the first grid again; the small case is also checked against the
oracle's definitions on the same moments.
"""

import ctypes as C

import numpy as np
import pytest

import inputs
from oracle import diagnostics as odiag
from oracle import scheme

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_24059_amd import lbm  # noqa: E402

FIELDS = ("step", "time", "mass", "kinetic", "enstrophy", "div_l2", "max_u", "rho_min", "rho_max",
          "nonfinite", "flags")


def _engine(dim, n, steps, nu=0.02):
    p = scheme.params_for_grid(dim, n, nu)
    u0 = inputs.taylor_green(n) if dim == 2 else inputs.abc_flow(n, 0.25, 0.25, 0.25)
    prm = lbm.make_params(dim, (n,) * dim, p.dx, p.dt, p.nu, p.omega_rho, p.omega_q, p.alpha_rho)
    eng = lbm.Engine.create(prm, u0)
    eng.step(steps)
    return eng, p


def _same(a: lbm.lbm_diag, b: lbm.lbm_diag):
    for f in FIELDS:
        assert getattr(a, f) == getattr(b, f), f
    assert list(a.mom) == list(b.mom)


def test_noalloc_diagnostics_equal_two_calls_shrinking():
    print("[no-alloc] 2D 2048^2 (the largest partial count), then 2D 48^2, then 3D 20^3", flush=True)
    big, _ = _engine(2, 2048, 6)
    st_ref, ref = lbm.lbm_diagnostics(big.ctx)
    st, got = lbm.lbm_diagnostics_noalloc(big.ctx)
    assert st == st_ref == lbm.LBM_OK
    _same(got, ref)

    small, p = _engine(2, 48, 30)
    st_ref, ref = lbm.lbm_diagnostics(small.ctx)
    st, got = lbm.lbm_diagnostics_noalloc(small.ctx)
    assert st == st_ref == lbm.LBM_OK
    _same(got, ref)
    rho, q = small.moments()
    o = odiag.from_moments(rho, q, p.dx)
    for key in ("mass", "kinetic", "enstrophy", "div_l2", "max_u", "rho_min", "rho_max"):
        assert getattr(got, key) == pytest.approx(o[key], rel=1e-12, abs=1e-300), key
    small.close()

    s3, _ = _engine(3, 20, 10)
    st_ref, ref = lbm.lbm_diagnostics(s3.ctx)
    st, got = lbm.lbm_diagnostics_noalloc(s3.ctx)
    assert st == st_ref == lbm.LBM_OK
    _same(got, ref)
    s3.close()

    # the first context again, after smaller calls left their partials behind
    st, got = lbm.lbm_diagnostics_noalloc(big.ctx)
    st_ref, ref = lbm.lbm_diagnostics(big.ctx)
    _same(got, ref)
    big.close()


def test_noalloc_diagnostics_reports_nonfinite():
    n = 16
    eng, _ = _engine(2, n, 0)
    blob = eng.save_state()
    f = blob[:-8].view(np.float32)
    f[5] = np.nan
    eng.load_state(blob)
    st, d = lbm.lbm_diagnostics_noalloc(eng.ctx)
    assert st == lbm.LBM_ENONFINITE and d.nonfinite == 1
    eng.close()


def test_noalloc_diagnostics_rejects_null():
    assert lbm.lib().lbm_diagnostics_noalloc(None, None) == lbm.LBM_EINVAL
    eng, _ = _engine(2, 16, 0)
    assert lbm.lib().lbm_diagnostics_noalloc(C.c_void_p(eng.ctx), None) == lbm.LBM_EINVAL
    eng.close()
