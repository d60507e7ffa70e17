"""Pins for oracle.lattice / oracle.canonical: assembled lattice sums.

T1  assembled (Theorem 3.1, Lemma 3.2) = direct (every image projected at its
    own position) = 3D brute force over shifted full master tensors, to
    rounding (the paper reports ~1e-14 for a 16x16x2 cluster, Fig. 3.4).
T7  symmetry and linearity; T8 special cases; T10 physics (point charges);
T9  growth of non-neutral sums with L (Sec. 3.2).
"""
import json
import os

import numpy as np
import pytest

from oracle.lattice import (Geometry, direct_factors, assembled_factors, brute_force_tensor,
                            factor_entries, point_charge_potential)
from oracle.canonical import reconstruct, sample, scalar_product, hadamard, concatenate
from oracle.quadrature import rule_u, rule_s
from workloads import rule_s_params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _quad_s(M, n, b, X):
    C0, s = rule_s_params(M, X)
    return rule_s(M, C0, s * n / b)


def _unsigned(F, coef, R):
    return np.abs(coef)


@pytest.mark.parametrize("periodic,L,n,M0", [
    (False, (3, 2, 3), 8, 2),
    (False, (1, 1, 1), 10, 3),
    (True, (3, 3, 3), 8, 2),
    (True, (4, 3, 2), 6, 3),
])
def test_assembled_equals_direct_equals_brute_force(periodic, L, n, M0):
    rng = np.random.default_rng(11)
    b = 10.0
    geom = Geometry(b, n, L, periodic)
    t, w = _quad_s(29, n, b, 256)
    pos = -0.5 * b + rng.uniform(0, 1, (M0, 3)) * b
    Z = rng.choice([-2.0, -1.0, 1.0, 2.0], M0)
    Fd, cd = direct_factors(geom, t, w, pos, Z)
    Fa, ca = assembled_factors(geom, t, w, pos, Z)
    for l in range(3):
        assert np.allclose(Fa[l], Fd[l], rtol=1e-13, atol=1e-13 * np.abs(Fd[l]).max())
    P_bf = brute_force_tensor(geom, t, w, pos, Z)
    P_a = reconstruct(Fa, ca)
    scale = np.abs(reconstruct(Fa, np.abs(ca))).max()
    assert np.max(np.abs(P_a - P_bf)) < 1e-13 * scale
    assert np.max(np.abs(reconstruct(Fd, cd) - P_bf)) < 1e-13 * scale


def test_paper_cluster_assembled_vs_direct():
    # Sec. 3.1, Fig. 3.4: 16x16x2 lattice of unit charges, assembled vs direct
    # canonical sum agree to ~1e-14 (absolute, on potentials of order 10-100)
    with open(os.path.join(GOLDEN, "fig3_4_cluster.json")) as f:
        g = json.load(f)
    geom = Geometry(g["b"], g["n"], tuple(g["L"]), False)
    t, w = rule_u(g["M"], 1.0)
    pos = np.zeros((1, 3))
    Fd, cd = direct_factors(geom, t, w, pos, [1.0])
    Fa, ca = assembled_factors(geom, t, w, pos, [1.0])
    h3 = geom.h ** 3
    rng = np.random.default_rng(5)
    idx = np.stack([rng.integers(0, geom.N(l), 4000) for l in range(3)], 1)
    vd = np.asarray(sample(Fd, cd, idx), np.float64) / h3
    va = np.asarray(sample(Fa, ca, idx), np.float64) / h3
    assert np.max(np.abs(vd - va)) <= g["abs_diff_bound"]
    assert np.max(np.abs(vd)) > 1.0


def test_single_node_atom_is_one_master_window():
    # L = 1, one charge on a node: every axis vector is a window of the same
    # master (eq. sub_tens), so the three factors coincide (p1 = p2 = p3,
    # eq. Newt_canTens) and the rank is R
    b, n = 8.0, 12
    geom = Geometry(b, n, (1, 1, 1))
    t, w = rule_u(12, 1.0)
    pos = np.array([[-0.5 * b + 5 * b / n] * 3])
    F, c = direct_factors(geom, t, w, pos, [1.0])
    assert F[0].shape == (t.size, n)
    assert np.array_equal(F[0], F[1]) and np.array_equal(F[1], F[2])
    # window: cell g sees the charge at node 5, so column g equals the master at g - 5
    x = np.arange(-n, n, dtype=float)
    from oracle.projection import gauss_cell_integral
    m = gauss_cell_integral(t[:, None], (x * geom.h)[None], ((x + 1) * geom.h)[None])
    assert np.allclose(F[0], m[:, np.arange(n) - 5 + n], rtol=1e-15)


def test_symmetry_and_linearity():
    b, n, L = 10.0, 8, (3, 3, 3)
    geom = Geometry(b, n, L)
    t, w = _quad_s(29, n, b, 256)
    # one charge at the centre node of the unit cell: the lattice sum is
    # symmetric under axis permutations and the mirror of the box
    pos = np.zeros((1, 3))
    F, c = assembled_factors(geom, t, w, pos, [1.0])
    assert np.allclose(F[0], F[1], rtol=1e-15) and np.allclose(F[1], F[2], rtol=1e-15)
    P = reconstruct(F, c)
    assert np.allclose(P, P[::-1, :, :], rtol=1e-13)
    assert np.allclose(P, P.transpose(1, 2, 0), rtol=1e-13)
    # linearity in Z and superposition of atoms
    rng = np.random.default_rng(2)
    pos2 = -0.5 * b + rng.uniform(0, 1, (2, 3)) * b
    Fa, ca = assembled_factors(geom, t, w, pos2, [1.5, -0.5])
    F1, c1 = assembled_factors(geom, t, w, pos2[:1], [1.0])
    F2, c2 = assembled_factors(geom, t, w, pos2[1:], [1.0])
    P12 = reconstruct(Fa, ca)
    assert np.allclose(P12, 1.5 * reconstruct(F1, c1) - 0.5 * reconstruct(F2, c2),
                       rtol=0, atol=1e-13 * np.abs(P12).max())
    # the concatenated canonical sum (eq. conc) is the same tensor
    Fc, cc = concatenate(F1, 1.5 * c1, F2, -0.5 * c2)
    assert np.allclose(reconstruct(Fc, cc), P12, rtol=0, atol=1e-13 * np.abs(P12).max())


def test_potential_matches_point_charges_away_from_charges():
    # cell averages of the lattice potential vs sum of Z/|x - a| at the cell
    # centre; a cube's average of a harmonic function differs from the centre
    # value only at fourth order in h/distance
    b, n, L = 10.0, 20, (2, 2, 2)
    geom = Geometry(b, n, L)
    t, w = _quad_s(47, n, b, 256)
    rng = np.random.default_rng(4)
    pos = -0.5 * b + rng.uniform(0.2, 0.8, (2, 3)) * b
    Z = np.array([1.0, -1.0])
    F, c = assembled_factors(geom, t, w, pos, Z)
    idx = np.stack([rng.integers(0, geom.N(l), 3000) for l in range(3)], 1)
    h = geom.h
    centres = -0.5 * b + (idx + 0.5) * h
    K = np.array(np.meshgrid(*(np.arange(2),) * 3, indexing="ij")).reshape(3, -1).T * b
    dist = np.min(np.linalg.norm(centres[:, None, None, :] - (pos[None, :, None, :] + K[None, None]), axis=-1), axis=(1, 2))
    keep = dist > 5 * h
    v = np.asarray(sample(F, c, idx[keep]), np.float64) / h ** 3
    ref = point_charge_potential(geom, pos, Z, centres[keep])
    vabs = np.asarray(sample(F, np.abs(c), idx[keep]), np.float64) / h ** 3
    assert np.max(np.abs(v - ref) / vabs) < 2e-4


def test_growth_with_L_of_non_neutral_sums():
    # centre value of L x 1 x 1, L x L x 1 and L x L x L sums of unit charges:
    # growth ~ log L, ~ L and ~ L^2 (Sec. 3.2); the successive increments
    # p_2L - p_L tend to a constant, double, quadruple respectively
    b, n = 4.0, 4
    t, w = _quad_s(41, n, b, 256)
    def centre_value(L):
        geom = Geometry(b, n, L)
        F, c = assembled_factors(geom, t, w, np.zeros((1, 3)), [1.0])
        idx = np.array([[geom.N(l) // 2 for l in range(3)]])
        return float(sample(F, c, idx)[0]) / geom.h ** 3
    for shape, ratio in (((1, 0, 0), 1.0), ((1, 1, 0), 2.0), ((1, 1, 1), 4.0)):
        Ls = [8, 16, 32]
        p = [centre_value(tuple(Lv if s else 1 for s in shape)) for Lv in Ls]
        r = (p[2] - p[1]) / (p[1] - p[0])
        assert abs(r - ratio) < 0.15 * ratio, (shape, r)


def test_factor_entries_match_full_factors():
    b, n, L = 10.0, 8, (4, 2, 3)
    geom = Geometry(b, n, L)
    t, w = _quad_s(35, n, b, 256)
    rng = np.random.default_rng(8)
    pos = -0.5 * b + rng.uniform(0, 1, (3, 3)) * b
    F, _ = direct_factors(geom, t, w, pos, [1, 1, 1])
    for l in range(3):
        g = rng.integers(0, geom.N(l), 7)
        assert np.allclose(factor_entries(geom, t, pos, l, g), F[l][:, g], rtol=1e-15, atol=0)


def test_scalar_and_hadamard_products_against_full_tensors():
    rng = np.random.default_rng(6)
    FA = [rng.normal(size=(5, m)) for m in (4, 6, 3)]
    FB = [rng.normal(size=(3, m)) for m in (4, 6, 3)]
    ca, cb = rng.normal(size=5), rng.normal(size=3)
    A, B = reconstruct(FA, ca), reconstruct(FB, cb)
    assert np.isclose(scalar_product(FA, ca, FB, cb), np.sum(A * B), rtol=1e-13)
    Fh, ch = hadamard(FA, ca, FB, cb)
    assert np.allclose(reconstruct(Fh, ch), A * B, rtol=1e-12, atol=1e-12)
