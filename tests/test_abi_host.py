"""Host-only checks of the C ABI: the library loads, exports every symbol the
headers declare, and validates parameters without touching a GPU."""

import ctypes as C
import glob
import math
import os
import re

import pytest

from paper_2607_24059_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(lbm\w*)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    names = _declared_functions()
    assert "lbm_init" in names and "lbm_step" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    """The Python binding carries one signature per declared entry point."""
    import paper_2607_24059_amd.lbm as B
    sigs = set(B.SIGNATURES)
    for extra in ("batch", "closure", "cnn", "spectrum"):
        mod = getattr(__import__("paper_2607_24059_amd", fromlist=[extra]), extra, None)
        if mod is not None and hasattr(mod, "SIGNATURES"):
            sigs |= set(mod.SIGNATURES)
    assert set(_declared_functions()) <= sigs


def _params(**kw):
    base = dict(dim=2, n=(64, 64), dx=0.1, dt=0.1 ** 2 / 8, nu=0.01)
    base.update(kw)
    return lbm.make_params(**base)


def test_check_params_derives_mu_and_alpha():
    st, mu, aq, fl = lbm.lbm_check_params(_params())
    assert st == lbm.LBM_OK
    assert mu == pytest.approx(8.0, rel=1e-14)
    # nu = 2 mu alpha_q (1/omega_q - 1/2)
    assert 2 * mu * aq * (1 / (23 / 20) - 0.5) == pytest.approx(0.01, rel=1e-14)
    assert fl == 0


@pytest.mark.parametrize("kw,status", [
    (dict(omega_q=2.0), lbm.LBM_EUNSTABLE),
    (dict(omega_rho=0.0), lbm.LBM_EUNSTABLE),
    (dict(alpha_rho=0.26), lbm.LBM_EUNSTABLE),
    (dict(dim=3, n=(8, 8, 8), alpha_rho=0.17), lbm.LBM_EUNSTABLE),
    (dict(nu=100.0), lbm.LBM_EUNSTABLE),         # alpha_q beyond 1/4
    (dict(dx=0.0), lbm.LBM_EINVAL),
    (dict(dt=-1.0), lbm.LBM_EINVAL),
    (dict(gamma=1.4), lbm.LBM_EINVAL),
    (dict(n=(64, 64, 2)), lbm.LBM_EINVAL),       # 2D needs nz = 1
    (dict(n=(0, 64)), lbm.LBM_EINVAL),
    (dict(storage=9), lbm.LBM_EINVAL),
    (dict(rho_ref=0.0), lbm.LBM_EINVAL),
])
def test_check_params_rejects(kw, status):
    st, *_ = lbm.lbm_check_params(_params(**kw))
    assert st == status
    assert lbm.lbm_workspace_bytes(_params(**kw)) == 0


def test_low_frequency_warning_flag():
    """mu^2 (alpha_rho + alpha_q) < 1 raises the warning bit."""
    st, mu, aq, fl = lbm.lbm_check_params(_params(dt=0.1 ** 2 / 1.5, alpha_rho=0.05))
    assert st == lbm.LBM_OK and fl & lbm.LBM_WARN_LOWFREQ


def test_workspace_bytes_cover_both_buffers():
    for storage, per in (("f32", 4 * 15), ("f16_dev", 2 * 15), ("f16_dev_r32", 4 * 3 + 2 * 12),
                         ("f64", 8 * 15), ("f16_neq", 4 * 3 + 2 * 12),
                         ("f32_moments", 4 * 3)):
        omegas = dict(omega_rho=1.0, omega_q=1.0) if storage == "f32_moments" else {}
        nb = lbm.lbm_workspace_bytes(_params(storage=storage, n=(4096, 4096), **omegas))
        staging = 24 if 2 * per < 2 * 24 and per < 24 else 0   # FP64 staging region if a buffer is smaller
        assert nb >= (2 * per + staging) * 4096 * 4096
        assert nb < (2 * per + staging) * 4096 * 4096 * 1.01 + (16 << 20)   # + diagnostics scratch
    nb3 = lbm.lbm_workspace_bytes(_params(dim=3, n=(256, 256, 256)))
    assert nb3 >= 2 * 28 * 4 * 256 ** 3


def test_batch_has_no_fp64_mode():
    """The FP64 reference storage is single-run only: the batch sizes it as invalid."""
    from paper_2607_24059_amd import batch
    spec = batch.make_run((64, 64, 1), 2 * math.pi / 64, (2 * math.pi / 64) ** 2 / 8, 1e-3)
    assert batch.lbm_batch_workspace_bytes(2, lbm.STORAGE["f64"], [spec]) == 0
    assert batch.lbm_batch_workspace_bytes(2, lbm.STORAGE["f32"], [spec]) > 0


def test_moment_storage_only_for_the_relaxation_scheme():
    st, *_ = lbm.lbm_check_params(_params(storage="f32_moments"))
    assert st == lbm.LBM_EINVAL
    st, *_ = lbm.lbm_check_params(_params(storage="f32_moments", omega_rho=1.0, omega_q=1.0))
    assert st == lbm.LBM_OK


def test_strerror():
    assert lbm.lbm_strerror(lbm.LBM_OK) == "ok"
    assert "workspace" in lbm.lbm_strerror(lbm.LBM_ENOMEM)


def test_spectrum_host_validation():
    """lbm_spectrum_* reject bad arguments on the host, before any launch."""
    from paper_2607_24059_amd import spectrum as S
    L = S.slib()
    assert S.lbm_spectrum_order(2) == 15 and S.lbm_spectrum_order(3) == 28
    assert S.lbm_spectrum_order(1) == 0 and S.lbm_spectrum_order(4) == 0
    fake = 0x1000                                   # never dereferenced: every call fails validation
    assert L.lbm_spectrum_eigs(4, 1, fake, 1, None, fake, fake, None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_spectrum_eigs(2, -1, fake, 1, None, fake, fake, None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_spectrum_eigs(2, 1, fake, 0, None, fake, fake, None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_spectrum_eigs(2, 1, None, 1, None, fake, fake, None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_spectrum_eigs(2, 1, fake, 1, None, None, fake, None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_spectrum_eigs(2, 1, fake, 1, None, fake, None, None, None, None, None) == lbm.LBM_EINVAL
    assert L.lbm_spectrum_matrix(3, 1, fake, 1, None, fake, None, None) == lbm.LBM_EINVAL
    assert L.lbm_spectrum_matrix(2, 1, fake, 1, None, None, fake, None) == lbm.LBM_EINVAL
    # no points: nothing to launch
    assert L.lbm_spectrum_eigs(2, 0, fake, 1, None, fake, fake, None, None, None, None) == lbm.LBM_OK
    assert L.lbm_spectrum_matrix(3, 0, fake, 1, None, fake, fake, None) == lbm.LBM_OK
    assert C.sizeof(S.lbm_lin_state) == 11 * 8
