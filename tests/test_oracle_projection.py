"""Pins for oracle.projection: 1D Gaussian cell integrals (eq. galten_int)."""
import mpmath
import numpy as np
import pytest

from oracle.projection import gauss_cell_integral, gauss_cell_integral_dpos

mpmath.mp.dps = 40


def _mp_cell(t, y0, y1):
    t, y0, y1 = mpmath.mpf(t), mpmath.mpf(y0), mpmath.mpf(y1)
    if t == 0:
        return y1 - y0
    c = mpmath.sqrt(mpmath.pi) / (2 * t)
    if y0 >= 0:
        return c * (mpmath.erfc(t * y0) - mpmath.erfc(t * y1))
    if y1 <= 0:
        return c * (mpmath.erfc(-t * y1) - mpmath.erfc(-t * y0))
    return c * (mpmath.erf(t * y1) - mpmath.erf(t * y0))


def _mp_dpos(t, y0, y1):
    t, y0, y1 = mpmath.mpf(t), mpmath.mpf(y0), mpmath.mpf(y1)
    return mpmath.exp(-(t * y0) ** 2) - mpmath.exp(-(t * y1) ** 2)


def _cases(seed=7, m=400):
    rng = np.random.default_rng(seed)
    t = 10.0 ** rng.uniform(-6, 3, m)
    h = 10.0 ** rng.uniform(-3, 0.5, m)
    # cell positions spread over many Gaussian widths and many cells
    y0 = rng.choice([-1, 1], m) * 10.0 ** rng.uniform(-4, 4, m) - rng.uniform(0, 1, m) * h
    return t, y0, y0 + h


def test_against_mpmath_random_and_ill_conditioned():
    t, y0, y1 = _cases()
    got = gauss_cell_integral(t, y0, y1)
    for i in range(t.size):
        ref = _mp_cell(t[i], y0[i], y1[i])
        if ref < mpmath.mpf("1e-300"):
            assert got[i] < 1e-290
            continue
        rel = abs((mpmath.mpf(got[i]) - ref) / ref)
        # exp(-u^2) amplifies the rounding of u = t*y by 2u^2 (inherent
        # conditioning of the entry with respect to its FP64 inputs)
        umin = min(abs(t[i] * y0[i]), abs(t[i] * y1[i])) if y0[i] * y1[i] > 0 else 0.0
        assert rel < 4e-15 * (1.0 + 2.0 * umin * umin), (t[i], y0[i], y1[i], float(rel))


def test_flat_gaussian_far_cells():
    # t*h tiny and the cell far out: erf difference would lose ~1e-12
    t = np.full(50, 5.9e-5)
    y0 = np.linspace(100.0, 8000.0, 50)
    got = gauss_cell_integral(t, y0, y0 + 1.0)
    for i in range(50):
        ref = _mp_cell(t[i], y0[i], y0[i] + 1.0)
        assert abs((mpmath.mpf(got[i]) - ref) / ref) < 2e-15


def test_zero_t_is_width():
    y0 = np.array([-3.0, 0.0, 2.5])
    assert np.array_equal(gauss_cell_integral(0.0, y0, y0 + 0.25), np.full(3, 0.25))


def test_mirror_symmetry():
    t, y0, y1 = _cases(8, 200)
    a = gauss_cell_integral(t, y0, y1)
    b = gauss_cell_integral(t, -y1, -y0)
    assert np.allclose(a, b, rtol=4e-15, atol=0)


def test_telescoping_partition():
    # the cells of a partition add up to the integral over the union
    for t in (1e-3, 0.3, 2.0, 40.0):
        e = np.linspace(-7.3, 11.1, 301)
        parts = gauss_cell_integral(t, e[:-1], e[1:])
        whole = _mp_cell(t, e[0], e[-1])
        assert abs((mpmath.mpf(float(np.sum(parts))) - whole) / whole) < 1e-14


def test_derivative_against_mpmath_and_fd():
    t, y0, y1 = _cases(9, 200)
    got = gauss_cell_integral_dpos(t, y0, y1)
    for i in range(t.size):
        ref = _mp_dpos(t[i], y0[i], y1[i])
        scale = max(abs(ref), mpmath.mpf("1e-300"))
        umin = min(abs(t[i] * y0[i]), abs(t[i] * y1[i]))
        assert abs(mpmath.mpf(got[i]) - ref) / scale < 4e-15 * (1.0 + 2.0 * umin * umin)
    # d/da of the integral over [x0 - a, x1 - a]: moving a right moves the cell left
    rng = np.random.default_rng(3)
    t = 10.0 ** rng.uniform(-2, 1, 50)
    y0 = rng.uniform(-3, 3, 50)
    y1 = y0 + rng.uniform(0.05, 0.5, 50)
    eps = 1e-6
    fd = (gauss_cell_integral(t, y0 - eps, y1 - eps) - gauss_cell_integral(t, y0 + eps, y1 + eps)) / (2 * eps)
    assert np.allclose(gauss_cell_integral_dpos(t, y0, y1), fd, rtol=1e-7, atol=1e-9)
