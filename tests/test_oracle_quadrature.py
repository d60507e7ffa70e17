"""Pins for oracle.quadrature: the sinc rules for 1/r (eqs. laplace, sinc_Newt, hM)."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle.quadrature import rule_u, rule_s, gaussian_sum, _CalibrationProblem, calibration_cells
from oracle.prism import exact_galerkin_entries
from oracle.projection import gauss_cell_integral
from workloads import rule_s_params


def test_rule_u_poisson_closed_form():
    # (h/sqrt(pi)) sum_{k in Z} exp(-k^2 h^2 r^2) = (1/r) sum_{m in Z} exp(-pi^2 m^2/(h r)^2)
    # (Poisson summation / Jacobi theta); rule U is that sum cut at |k| <= M.
    for M, C0 in ((20, 1.0), (35, 2.0), (8, 0.5)):
        t, w = rule_u(M, C0)
        hM = C0 * np.log(M) / M
        assert t.size == 2 * M + 1 and np.allclose(np.diff(t), hM, rtol=1e-12)
        r = np.linspace(0.3, 12.0, 60)
        m = np.arange(1, 40)
        theta = (1.0 + 2.0 * np.exp(-np.pi ** 2 * np.outer(1.0 / (hM * r) ** 2, m ** 2)).sum(1)) / r
        k = np.arange(M + 1, M + 4000)
        tail = 2.0 * hM / np.sqrt(np.pi) * np.exp(-np.outer(r * r, (k * hM) ** 2)).sum(1)
        assert np.allclose(gaussian_sum(t, w, r), theta - tail, rtol=1e-13, atol=0)


def test_rule_s_substitution_integral():
    # with t = s sinh(u): 1/r = (s/sqrt(pi)) * integral over R of cosh(u) exp(-s^2 sinh(u)^2 r^2) du
    s = 0.7
    for r in (0.05, 1.0, 13.0):
        f = lambda u: s / np.sqrt(np.pi) * np.cosh(u) * np.exp(-(s * np.sinh(u) * r) ** 2)
        U = np.arcsinh(40.0 / (s * r))   # the integrand is below exp(-1600) beyond
        v, _ = quad(f, -U, U, epsabs=0, epsrel=1e-13, limit=400)
        assert abs(v * r - 1.0) < 1e-12
    # the folded sinc rule converges to it (exponentially in M)
    for r in (0.05, 1.0, 13.0):
        t, w = rule_s(400, 2.0, s)
        t2, w2 = rule_s(400, 1.5, s)
        assert abs(gaussian_sum(t, w, r) * r - 1.0) < 1e-12
        assert abs(gaussian_sum(t2, w2, r) * r - 1.0) < 1e-12


def test_rule_s_folding_matches_unfolded_sum():
    M, C0, s = 30, 3.0, 0.01
    t, w = rule_s(M, C0, s)
    hM = C0 * np.log(M) / M
    k = np.arange(-M, M + 1)
    tu = s * np.sinh(k * hM)
    wu = s * hM * np.cosh(k * hM) / np.sqrt(np.pi)
    r = np.logspace(-2, 3, 40)
    assert np.allclose(gaussian_sum(t, w, r), gaussian_sum(tu, wu, r), rtol=1e-14)


@pytest.mark.parametrize("M,X", [(47, 4096), (59, 16384), (29, 256)])
def test_calibrated_rule_against_exact_tensor(M, X):
    C0, s = rule_s_params(M, X)
    t, w = rule_s(M, C0, s)
    stored = [r for r in __import__("workloads.configs", fromlist=["_table"])._table()
              if r["M"] == M and r["X"] == X][0]["max_rel_err"]
    prob = _CalibrationProblem(X)
    assert prob.max_rel_error(t, w) <= stored * 1.0001
    # out of sample: other random cells and a charge off the node
    rng = np.random.default_rng(99)
    cells = rng.integers(-X, X, size=(300, 3))
    for shift in ((0.0, 0.0, 0.0), (0.3, 0.7, 0.5)):
        ex = exact_galerkin_entries(cells, 1.0, shift)
        b = [gauss_cell_integral(t[:, None], (cells[None, :, l] - shift[l]),
                                 (cells[None, :, l] + 1.0 - shift[l])) for l in range(3)]
        approx = (b[0] * b[1] * b[2]).T @ w
        assert np.max(np.abs(approx - ex) / ex) < 5 * stored


def test_rule_s_accuracy_band_against_inverse_r():
    C0, s = rule_s_params(47, 4096)
    t, w = rule_s(47, C0, s)
    r = np.logspace(np.log10(0.5), np.log10(4096 * np.sqrt(3)), 400)
    assert np.max(np.abs(gaussian_sum(t, w, r) * r - 1.0)) < 2e-6
