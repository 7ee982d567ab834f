"""Host logic of the closure driver (no GPU): the equal-error speedup."""

import math

import pytest

from paper_2607_24059_amd import closure as cl

LEVELS = (256, 512, 1024)
ERR = {"256": 4e-5, "512": 1e-5, "1024": 3e-5}   # FP32 rounding lifts the finest level
TIME = {"256": 0.9, "512": 4.6, "1024": 70.0}


def test_interpolated_between_levels():
    r = cl.equal_error_speedup(LEVELS, ERR, TIME, 2e-5, 1.0)
    assert r["note"] == "interpolated"
    assert r["N_star"] == pytest.approx(256 * math.sqrt(2), rel=1e-12)        # second order: e ~ N^-2
    assert r["speedup"] == pytest.approx(0.9 * math.sqrt(4.6 / 0.9), rel=1e-12)


def test_no_extrapolation_past_the_rounding_floor():
    """Below the 512 error (the 1024 level, rounding-limited, has a larger
    one) there is no equal-error point: the curve is not extended."""
    r = cl.equal_error_speedup(LEVELS, ERR, TIME, 5e-6, 2.0)
    assert math.isnan(r["N_star"]) and math.isnan(r["speedup"])
    assert "without extrapolation" in r["note"]
    # a target below a nearly flat last segment is refused the same way
    flat = {"256": 4e-5, "512": 1.06e-5, "1024": 1.03e-5}
    assert math.isnan(cl.equal_error_speedup(LEVELS, flat, TIME, 7.3e-6, 3.0)["N_star"])
    # interpolation on the last segment is kept
    r = cl.equal_error_speedup(LEVELS, flat, TIME, 1.05e-5, 3.0)
    assert r["note"] == "interpolated" and 512 < r["N_star"] < 1024


def test_no_equal_error_point():
    r = cl.equal_error_speedup(LEVELS, ERR, TIME, 5e-5, 3.0)
    assert math.isnan(r["N_star"]) and math.isnan(r["speedup"])


def test_last_decreasing_level():
    assert cl.last_decreasing_level(LEVELS, ERR) == 512
    assert cl.last_decreasing_level(LEVELS, {"256": 4e-5, "512": 1e-5, "1024": 3e-6}) == 1024
    assert cl.last_decreasing_level(LEVELS, {"256": 4e-5, "512": 5e-5, "1024": 3e-6}) == 256


def test_restriction_binding_checks_the_buffer_sizes():
    """The restriction writes 3 (nfx/r)(nfy/r) values: a level that does not
    divide the fine grid, or an output buffer of another size, is refused
    before any device call."""
    torch = pytest.importorskip("torch")
    fine = torch.empty(3 * 2048 * 2048)
    with pytest.raises(ValueError):
        cl.lbm_restrict(fine, 2048, 2048, 2048 // 768, 1.0, torch.empty(3 * 768 * 768), None)
    with pytest.raises(ValueError):
        cl.lbm_restrict(fine, 2048, 2048, 3, 1.0, torch.empty(3 * 682 * 682), None)
