"""Pins for the canonical-format checker used at full size and for the far-cell
offsets of the direct sum (oracle.canonical, oracle.lattice).

* ``sample_columns`` is the only checker of full-size GPU results (sampled
  entries of the headline, periodic and batch workloads, eq. CP_form). It is
  pinned against brute force in exact integer arithmetic (a dropped coefficient,
  a transposed or swapped axis, a wrong column pick changes the integers), and
  against the full ``reconstruct`` (einsum) and ``sample`` on random factors.
* The direct sum evaluates the offset of cell g from image k as
  (g - k n) h - (a + b/2) rather than x_g - (a + b k) (equal in exact
  arithmetic); far along a long lattice the second form loses about
  log10(L n) digits. The entries are checked against 50-digit mpmath sums of
  the cell integrals over every image on a lattice of 64 x 128 cells.
"""
import itertools

import mpmath
import numpy as np

from oracle.canonical import reconstruct, sample, sample_columns
from oracle.lattice import Geometry, factor_entries, direct_factors
from oracle.quadrature import rule_s
from workloads import rule_s_params


def test_sample_columns_exact_integer_brute_force():
    rng = np.random.default_rng(31)
    K, lens = 7, (5, 4, 6)
    F = [rng.integers(-9, 10, (K, n)) for n in lens]
    coef = rng.integers(-5, 6, K)
    picks = [np.array([4, 0, 2]), np.array([3, 1]), np.array([5, 0, 3, 1])]
    cols = [F[l][:, picks[l]].astype(np.float64) for l in range(3)]
    sel = np.array(list(itertools.product(range(3), range(2), range(4))))
    sel = sel[rng.permutation(len(sel))]
    got = sample_columns(cols, coef.astype(np.float64), sel)
    for s, (a, b, c) in enumerate(sel):
        i, j, k = picks[0][a], picks[1][b], picks[2][c]
        exact = sum(int(coef[r]) * int(F[0][r, i]) * int(F[1][r, j]) * int(F[2][r, k])
                    for r in range(K))
        assert got[s] == exact, (s, (i, j, k), got[s], exact)


def test_sample_columns_equals_full_reconstruction():
    rng = np.random.default_rng(32)
    K, lens = 23, (11, 9, 13)
    F = [rng.standard_normal((K, n)) for n in lens]
    coef = rng.standard_normal(K)
    full = reconstruct(F, coef)
    picks = [np.sort(rng.choice(n, 4, replace=False)) for n in lens]
    cols = [F[l][:, picks[l]] for l in range(3)]
    sel = np.array(list(itertools.product(range(4), range(4), range(4))))
    got = np.asarray(sample_columns(cols, coef, sel), np.float64)
    idx = np.stack([picks[l][sel[:, l]] for l in range(3)], 1)
    ref = full[idx[:, 0], idx[:, 1], idx[:, 2]]
    scale = np.abs(reconstruct([np.abs(f) for f in F], np.abs(coef))).max()
    assert np.max(np.abs(got - ref)) < 1e-14 * scale
    assert np.array_equal(np.asarray(sample(F, coef, idx)), np.asarray(sample_columns(cols, coef, sel)))


def _cell_sum_mp(t, a, b, n, g, images):
    """sum over images k of the integral of exp(-t^2 (x - a - b k)^2) over
    cell g = [-b/2 + g b/n, -b/2 + (g+1) b/n], at the working precision of
    mpmath: t, a, b are taken as their exact binary values and the cell size
    is the exact b/n (not its FP64 rounding)."""
    t, a, b = mpmath.mpf(t), mpmath.mpf(a), mpmath.mpf(b)
    h = b / n
    x0 = -b / 2 + g * h
    x1 = x0 + h
    acc = mpmath.mpf(0)
    for k in images:
        c = a + b * k
        u0, u1 = t * (x0 - c), t * (x1 - c)
        if u0 >= 0:
            d = mpmath.erfc(u0) - mpmath.erfc(u1)
        elif u1 <= 0:
            d = mpmath.erfc(-u1) - mpmath.erfc(-u0)
        else:
            d = mpmath.erf(u1) - mpmath.erf(u0)
        acc += mpmath.sqrt(mpmath.pi) / (2 * t) * d
    return acc


def test_far_cells_against_mpmath():
    # b/n = 1/12 is not a binary fraction, so cell edges far along the
    # lattice carry rounding; 64 unit cells of 120 cells (7680 cells). The
    # rewritten offset keeps every row within 1e-14 of its maximum here, where
    # x_g - (a + b k) was off by up to 9e-13.
    b, n, L = 10.0, 120, (64, 1, 1)
    geom = Geometry(b, n, L, False)
    C0, s = rule_s_params(47, L[0] * n)
    t, _ = rule_s(47, C0, s * n / b)
    qs = [3, 20, 27, 30, 33, 36, 40, 47]         # wide ... narrow terms
    a = 1.2345678901234567                       # off-grid charge, node 74 of each cell
    g = np.concatenate([np.arange(7600, 7680, 7), np.arange(63 * n + 71, 63 * n + 78),
                        np.arange(3800, 3850, 5), np.arange(31 * n + 71, 31 * n + 78),
                        np.arange(0, 40, 6), np.arange(71, 78)])
    got = factor_entries(geom, t[qs], np.array([[a, 0.0, 0.0]]), 0, g)
    with mpmath.workdps(50):
        ref = np.array([[float(_cell_sum_mp(t[q], a, b, n, int(gg), range(L[0]))) for gg in g]
                        for q in qs])
    rowmax = np.max(np.abs(ref), axis=1)
    assert np.all(rowmax > 0)
    err = np.max(np.abs(got - ref), axis=1)
    assert np.all(err <= 5e-14 * rowmax), err / rowmax
    # the full direct sum gives the same entries
    Fd, _ = direct_factors(geom, t[qs], np.ones(len(qs)), np.array([[a, 0.0, 0.0]]), np.ones(1))
    assert np.max(np.abs(Fd[0][:, g] - got)) <= 1e-15 * np.max(rowmax)
