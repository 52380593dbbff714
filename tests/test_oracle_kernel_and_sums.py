"""Pins of the oracle's smoothing kernel and exact summation (CPU only).

The kernel is pinned by what the paper and the mathematics fix: unit
integral (Remark on kernel properties), compact support at r_c = 3h, the
smoothness of the quintic spline at q = 1, 2, and a derivative that matches
finite differences of W.  The exact summation is pinned against Python's
math.fsum, an independent correctly-rounded summation routine.
"""
import math

import numpy as np
import pytest
from scipy import integrate

pytestmark = pytest.mark.filterwarnings("ignore")


def _integral(oracle, dim, h):
    W = lambda r: oracle.kernel_W(dim, h, r)
    pts = [h, 2 * h]
    if dim == 1:
        f = lambda r: 2.0 * W(r)
    elif dim == 2:
        f = lambda r: 2.0 * math.pi * r * W(r)
    else:
        f = lambda r: 4.0 * math.pi * r * r * W(r)
    val = 0.0
    edges = [0.0, h, 2 * h, 3 * h]
    for a, b in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=200)
        val += v
    return val


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("h", [1.0, 0.025, 0.2])
def test_kernel_normalised(oracle_lib, dim, h):
    assert abs(_integral(oracle_lib, dim, h) - 1.0) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_support_and_sign(oracle_lib, dim):
    h = 0.1
    o = oracle_lib
    assert o.kernel_W(dim, h, 3 * h) == 0.0
    assert o.kernel_dW(dim, h, 3 * h) == 0.0
    assert o.kernel_W(dim, h, 3.5 * h) == 0.0
    rs = np.linspace(1e-6, 3 * h * 0.999, 500)
    w = np.array([o.kernel_W(dim, h, r) for r in rs])
    dw = np.array([o.kernel_dW(dim, h, r) for r in rs])
    assert np.all(w > 0)
    assert np.all(dw < 0)          # monotonically decreasing (Remark on kernel properties)
    assert np.all(np.diff(w) < 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_derivative_matches_finite_differences(oracle_lib, dim):
    h = 0.3
    o = oracle_lib
    for q in [0.05, 0.4, 0.99, 1.01, 1.5, 1.99, 2.01, 2.6, 2.95]:
        r = q * h
        e = 1e-6 * h
        fd = (o.kernel_W(dim, h, r + e) - o.kernel_W(dim, h, r - e)) / (2 * e)
        an = o.kernel_dW(dim, h, r)
        assert abs(fd - an) <= 1e-7 * abs(an) + 1e-9 * abs(o.kernel_W(dim, h, 0.0)) / h


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_smooth_at_breakpoints(oracle_lib, dim):
    h = 1.0
    o = oracle_lib
    for q in [1.0, 2.0]:
        e = 1e-9
        for f in (o.kernel_W, o.kernel_dW):
            lo, hi = f(dim, h, q - e), f(dim, h, q + e)
            assert abs(lo - hi) < 1e-6 * max(abs(lo), 1e-12)


def test_kernel_peak_value(oracle_lib):
    # W(0) h^d = 66 sigma_d, with sigma_d from the unit integral; the values
    # follow from exact integration of the quintic spline.
    assert abs(oracle_lib.kernel_W(2, 1.0, 0.0) - 0.3076551620) < 1e-9
    assert abs(oracle_lib.kernel_W(3, 1.0, 0.0) - 0.1750704374) < 1e-9


def test_fsum_matches_math_fsum(oracle_lib):
    rng = np.random.default_rng(7)
    for trial in range(50):
        n = int(rng.integers(1, 3000))
        v = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
        v = np.concatenate([v, -v[: n // 2] * (1 + 1e-15)])
        rng.shuffle(v)
        assert oracle_lib.fsum(v) == math.fsum(v)


def test_fsum_hard_cases(oracle_lib):
    cases = [
        [1e100, 1.0, -1e100, 1e-100, 1e50, -1.0, -1e50],
        [1.0, 1e-16, 1e-16],               # exact sum needs more than a double
        [2.0 ** 53, 1.0, 1.0 / 2 ** 40],   # round up through the half-way correction
        [0.1] * 10,
        [],
    ]
    for c in cases:
        assert oracle_lib.fsum(np.array(c, dtype=np.float64)) == math.fsum(c)
