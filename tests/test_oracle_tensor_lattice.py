"""Pins for the oracle's non-equidistant tensor lattices (Sec. 3.1, remark
after eq. EwaldTensorM0): lattice points at arbitrary per-axis coordinates
s_l[k] (units of the cell h), the sum over all image triples split into
per-axis sums.

  * equidistant coordinates s_l[k] = n k reduce to the box lattice (the
    independently pinned direct sum of Theorem 3.1's setting);
  * the direct per-axis sum equals a 3D brute force over every image triple
    (on-grid and off-grid coordinates, off-grid charges, mixed signs);
  * coordinates that are whole numbers of cells: equal to the master-window
    route (the paper's windows with irregular shifts);
  * cell averages match point charges away from the charges;
  * derivative factors match central differences.
"""
import numpy as np

from oracle.lattice import (Geometry, TensorLattice, direct_factors, tensor_lattice_factors,
                            tensor_lattice_assembled, tensor_lattice_brute_force,
                            tensor_lattice_entries)
from oracle.canonical import reconstruct, sample
from oracle.quadrature import rule_s
from workloads import rule_s_params


def _quad(M, n, b, X=256):
    C0, s = rule_s_params(M, X)
    return rule_s(M, C0, s * n / b)


def _rows_close(a, b, rtol):
    scale = np.maximum(np.max(np.abs(b), axis=1), 1e-300)
    return np.all(np.max(np.abs(a - b), axis=1) <= rtol * scale)


def test_equidistant_coordinates_are_the_box_lattice():
    b, n, L = 10.0, 8, (3, 2, 4)
    rng = np.random.default_rng(21)
    t, w = _quad(29, n, b)
    pos = -0.5 * b + rng.uniform(0, 1, (3, 3)) * b
    Z = np.array([1.0, -2.0, 1.0])
    tl = TensorLattice(b, n, tuple(L[l] * n for l in range(3)),
                       tuple(float(n) * np.arange(L[l]) for l in range(3)))
    Ft, ct = tensor_lattice_factors(tl, t, w, pos, Z)
    Fd, cd = direct_factors(Geometry(b, n, L), t, w, pos, Z)
    assert np.array_equal(ct, cd)
    for l in range(3):
        assert _rows_close(Ft[l], Fd[l], 1e-13), l


def _irregular(rng, b, n, L, on_grid):
    """Per-axis coordinates (cells): a seeded irregular spacing between 0.6 n
    and 1.4 n cells."""
    s = []
    for Ll in L:
        gaps = rng.uniform(0.6, 1.4, Ll - 1) * n
        c = np.concatenate([[0.0], np.cumsum(gaps)])
        s.append(np.rint(c) if on_grid else c)
    N = tuple(int(np.ceil(s[l][-1] + n)) for l in range(3))
    return tuple(s), N


def test_direct_equals_brute_force_and_master_windows():
    b, n, L = 6.0, 6, (3, 2, 3)
    rng = np.random.default_rng(22)
    t, w = _quad(29, n, b)
    pos = -0.5 * b + rng.uniform(0, 1, (2, 3)) * b
    Z = np.array([2.0, -1.0])
    for on_grid in (True, False):
        s, N = _irregular(rng, b, n, L, on_grid)
        tl = TensorLattice(b, n, N, s)
        F, c = tensor_lattice_factors(tl, t, w, pos, Z)
        P = reconstruct(F, c)
        Pb = tensor_lattice_brute_force(tl, t, w, pos, Z)
        scale = np.max(np.abs(reconstruct(F, np.abs(c))))
        assert np.max(np.abs(P - Pb)) < 1e-13 * scale, on_grid
        if on_grid:
            Fa, ca = tensor_lattice_assembled(tl, t, w, pos, Z)
            for l in range(3):
                assert _rows_close(Fa[l], F[l], 1e-13), l
    # an axis with a single lattice point and one with coinciding points
    s = (np.array([0.0]), np.array([0.0, 0.0, 2.5 * n]), np.array([0.3 * n, 1.9 * n]))
    N = (n, int(np.ceil(3.5 * n)), int(np.ceil(2.9 * n)))
    tl = TensorLattice(b, n, N, s)
    F, c = tensor_lattice_factors(tl, t, w, pos, Z)
    Pb = tensor_lattice_brute_force(tl, t, w, pos, Z)
    scale = np.max(np.abs(reconstruct(F, np.abs(c))))
    assert np.max(np.abs(reconstruct(F, c) - Pb)) < 1e-13 * scale


def test_point_charges_away_from_the_charges():
    b, n = 10.0, 16
    rng = np.random.default_rng(23)
    t, w = _quad(47, n, b)
    s, N = _irregular(rng, b, n, (3, 2, 2), False)
    tl = TensorLattice(b, n, N, s)
    pos = -0.5 * b + rng.uniform(0.2, 0.8, (2, 3)) * b
    Z = np.array([1.0, -1.0])
    F, c = tensor_lattice_factors(tl, t, w, pos, Z)
    h = tl.h
    idx = np.stack([rng.integers(0, N[l], 3000) for l in range(3)], 1)
    centres = -0.5 * b + (idx + 0.5) * h
    imgs = np.array(np.meshgrid(s[0], s[1], s[2], indexing="ij")).reshape(3, -1).T
    charges = (pos[:, None, :] + h * imgs[None]).reshape(-1, 3)
    q = np.repeat(Z, imgs.shape[0])
    d = np.linalg.norm(centres[:, None, :] - charges[None], axis=-1)
    keep = d.min(axis=1) > 5 * h
    ref = np.sum(q[None, :] / d[keep], axis=1)
    v = np.asarray(sample(F, c, idx[keep]), np.float64) / h ** 3
    vabs = np.asarray(sample(F, np.abs(c), idx[keep]), np.float64) / h ** 3
    assert keep.sum() > 1000
    assert np.max(np.abs(v - ref) / vabs) < 2e-4


def test_derivative_factors_are_central_differences():
    b, n = 6.0, 6
    rng = np.random.default_rng(24)
    t, w = _quad(29, n, b)
    s, N = _irregular(rng, b, n, (2, 3, 2), False)
    tl = TensorLattice(b, n, N, s)
    pos = -0.5 * b + rng.uniform(0.1, 0.9, (1, 3)) * b
    dF, _ = tensor_lattice_factors(tl, t, w, pos, [1.0], derivative=True)
    step = 1e-6 * b
    for l in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[0, l] += step
        pm[0, l] -= step
        Fp, _ = tensor_lattice_factors(tl, t, w, pp, [1.0])
        Fm, _ = tensor_lattice_factors(tl, t, w, pm, [1.0])
        fd = (Fp[l] - Fm[l]) / (2 * step)
        scale = np.max(np.abs(dF[l]))
        assert np.max(np.abs(fd - dF[l])) < 1e-6 * scale, l


def test_sampled_columns_match_full_factors():
    b, n = 6.0, 6
    rng = np.random.default_rng(25)
    t, w = _quad(29, n, b)
    s, N = _irregular(rng, b, n, (3, 2, 2), False)
    tl = TensorLattice(b, n, N, s)
    pos = -0.5 * b + rng.uniform(0, 1, (2, 3)) * b
    for deriv in (False, True):
        F, _ = tensor_lattice_factors(tl, t, w, pos, [1.0, -1.0], derivative=deriv)
        for l in range(3):
            g = np.sort(rng.choice(N[l], 5, replace=False))
            # the same definition on fewer columns (vectorised sums may round
            # differently in the last bit)
            got = tensor_lattice_entries(tl, t, pos, l, g, deriv)
            assert np.max(np.abs(got - F[l][:, g])) <= 1e-15 * np.max(np.abs(F[l]))
