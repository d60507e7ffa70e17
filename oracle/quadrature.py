"""Sinc quadratures for 1/r = pi^{-1/2} * integral over R of exp(-t^2 r^2) dt.

Test infrastructure only (see ``oracle/__init__``).

Rule U (Sec. 2.1, eqs. sinc_Newt and hM), as printed: nodes t_k = k h_M for
k = -M..M and h_M = C0 log(M)/M. The printed weight g_k = h_M omits the
pi^{-1/2} of eq. laplace; without it the sum tends to sqrt(pi)/r, so the weight
used is h_M/sqrt(pi) (reading G1). R = 2M+1 terms.

Rule S: the same sinc rule after the substitution t = s sinh(u), the standard
form of the exponentially convergent quadrature the section cites, folded over
+-k because the integrand is even (the "R <= M+1" count of eq. Newt_canTens):
t_q = s sinh(q h_M), q = 0..M, w_0 = s h_M/sqrt(pi),
w_q = 2 s h_M cosh(q h_M)/sqrt(pi). The scale s and C0 are fixed per grid by
``calibrate_rule_s`` against the exact Galerkin tensor (reading G2).

Pins (tests/test_oracle_quadrature.py): rule U against its Poisson-summation
closed form; rule S against scipy's adaptive integral of the substituted
integrand and against 1/r in its accuracy band; calibrated rules against the
exact tensor of ``oracle.prism``.
"""
import numpy as np

from .projection import gauss_cell_integral
from .prism import exact_galerkin_entries

_SQRT_PI = np.sqrt(np.pi)


def rule_u(M, C0=1.0):
    """Uniform sinc rule (eqs. sinc_Newt, hM). Returns (t, w), 2M+1 terms."""
    hM = C0 * np.log(M) / M
    k = np.arange(-M, M + 1, dtype=np.float64)
    return k * hM, np.full(2 * M + 1, hM / _SQRT_PI)


def rule_s(M, C0, s):
    """sinh-mapped, folded sinc rule. Returns (t, w), M+1 terms."""
    hM = C0 * np.log(M) / M
    q = np.arange(0, M + 1, dtype=np.float64)
    t = s * np.sinh(q * hM)
    w = 2.0 * s * hM * np.cosh(q * hM) / _SQRT_PI
    w[0] = s * hM / _SQRT_PI
    return t, w


def gaussian_sum(t, w, r):
    """sum_k w_k exp(-t_k^2 r^2): the quadrature's approximation of 1/r."""
    r = np.asarray(r, np.float64)
    return np.exp(-np.multiply.outer(r * r, t * t)) @ w


# --------------------------------------------------------------------------
# Rule-S calibration (reading G2): grid units (h = 1), charge on a node.
# --------------------------------------------------------------------------

def calibration_cells(X, seed=0):
    """Sample cells i >= 0 of the master grid [-X, X)^3 (by symmetry
    b_{-1-i} = b_i only i >= 0 is needed): the near-singular block, the axes
    and diagonals at log-spaced distances, the far corner and seeded random
    cells."""
    near = np.array(np.meshgrid(*(np.arange(4),) * 3, indexing="ij")).reshape(3, -1).T
    m = np.unique(np.round(np.logspace(0.5, np.log10(X - 1), 24)).astype(int))
    z = np.zeros_like(m)
    lines = np.concatenate([np.stack([m, z, z], 1), np.stack([m, m, z], 1),
                            np.stack([m, m, m], 1), np.stack([m, 1 + z, z], 1)])
    rng = np.random.default_rng(seed)
    rnd = rng.integers(0, X, size=(160, 3))
    far = np.array([[X - 1, X - 1, X - 1], [X - 1, 0, 0]])
    return np.unique(np.concatenate([near, lines, rnd, far]), axis=0)


class _CalibrationProblem:
    def __init__(self, X, seed=0):
        self.cells = calibration_cells(X, seed)
        self.exact = exact_galerkin_entries(self.cells, 1.0)
        self.coords, self.inv = np.unique(self.cells, return_inverse=True)
        self.inv = self.inv.reshape(self.cells.shape)

    def max_rel_error(self, t, w):
        b = gauss_cell_integral(t[:, None], self.coords[None, :], self.coords[None, :] + 1.0)
        approx = (b[:, self.inv[:, 0]] * b[:, self.inv[:, 1]] * b[:, self.inv[:, 2]]).T @ w
        return float(np.max(np.abs(approx - self.exact) / self.exact))


def calibrate_rule_s(M, X, n_coarse=18, n_fine=9):
    """(C0, s) minimising the entrywise maximum relative error of P_R against
    the exact tensor over ``calibration_cells(X)``, in grid units.

    Deterministic grid search: a coarse grid over C0 in [1.5, 8] and
    log10(s*X) in [-2, 1], then a finer grid around the best point.
    Returns (C0, s, max_rel_error).
    """
    prob = _CalibrationProblem(X)
    best = (np.inf, None, None)
    c_lo, c_hi = 1.5, 8.0
    l_lo, l_hi = -2.0, 1.0
    for n_grid in (n_coarse, n_fine, n_fine):
        cs = np.linspace(c_lo, c_hi, n_grid)
        ls = np.linspace(l_lo, l_hi, n_grid)
        for C0 in cs:
            for lg in ls:
                s = 10.0 ** lg / X
                err = prob.max_rel_error(*rule_s(M, C0, s))
                if err < best[0]:
                    best = (err, C0, lg)
        dc = (c_hi - c_lo) / (n_grid - 1)
        dl = (l_hi - l_lo) / (n_grid - 1)
        c_lo, c_hi = best[1] - dc, best[1] + dc
        l_lo, l_hi = best[2] - dl, best[2] + dl
    return float(best[1]), float(10.0 ** best[2] / X), float(best[0])
