"""Pins for oracle.physics: energy (eq. scal), forces, Richardson (Sec. 3.2)."""
import numpy as np
import pytest

from oracle.lattice import Geometry, direct_factors, assembled_factors
from oracle.canonical import reconstruct
from oracle.physics import (energy, forces_adjoint, forces_adjoint_atoms, forces_fd,
                            richardson_linear, richardson_quadratic, nuclear_matrix)
from workloads import small_box, small_periodic, make_basis
from oracle.quadrature import rule_s, rule_u


def _tw(sysm):
    q = sysm.quad
    return rule_u(q["M"], q["C0"]) if q["rule"] == "U" else rule_s(q["M"], q["C0"], q["s"])


def _geom(sysm):
    return Geometry(sysm.b, sysm.n, sysm.L, sysm.periodic)


@pytest.mark.parametrize("maker,seed", [(small_box, 21), (small_periodic, 22)])
def test_energy_equals_full_grid_sum(maker, seed):
    sysm = maker(seed, n=8, M0=3) if maker is small_box else maker(seed, n=8, L=(3, 3, 3), M0=3)
    t, w = _tw(sysm)
    geom = _geom(sysm)
    E = energy(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d)
    F, c = direct_factors(geom, t, w, sysm.pos, sysm.Z)
    P = reconstruct(F, c)
    rho = reconstruct(sysm.density.D, sysm.density.d)
    ref = np.sum(P * rho)
    Eabs = np.sum(reconstruct(F, np.abs(c)) * rho)
    assert abs(E - ref) < 1e-13 * Eabs


def test_derivative_factors_match_finite_differences():
    sysm = small_box(31, n=8, L=(3, 2, 2), M0=2)
    t, w = _tw(sysm)
    geom = _geom(sysm)
    dF, _ = direct_factors(geom, t, w, sysm.pos, sysm.Z, derivative=True)
    dA, _ = assembled_factors(geom, t, w, sysm.pos, sysm.Z, derivative=True)
    eps = 1e-6
    for l in range(3):
        pp, pm = sysm.pos.copy(), sysm.pos.copy()
        pp[:, l] += eps
        pm[:, l] -= eps
        Fp, _ = direct_factors(geom, t, w, pp, sysm.Z)
        Fm, _ = direct_factors(geom, t, w, pm, sysm.Z)
        fd = (Fp[l] - Fm[l]) / (2 * eps)
        assert np.allclose(dF[l], fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max())
        assert np.allclose(dA[l], dF[l], rtol=1e-12, atol=1e-14 * np.abs(dF[l]).max())


@pytest.mark.parametrize("maker,seed", [(small_box, 41), (small_periodic, 42)])
def test_forces_adjoint_against_finite_differences(maker, seed):
    sysm = maker(seed, n=8, M0=3) if maker is small_box else maker(seed, n=8, L=(3, 3, 3), M0=3)
    t, w = _tw(sysm)
    geom = _geom(sysm)
    Fa = forces_adjoint(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d)
    Ffd = forces_fd(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d, 1e-4 * sysm.b)
    assert np.max(np.abs(Fa - Ffd)) < 1e-6 * np.max(np.abs(Fa))


def test_richardson_exact_on_model_sequences():
    p, c = 0.731, 2.9
    for L in (4, 8, 16):
        assert np.isclose(richardson_linear(p + c * L, p + c * 2 * L), p, rtol=1e-14)
        assert np.isclose(richardson_quadratic(p + c * L * L, p + c * 4 * L * L), p, rtol=1e-14)


def test_neutral_periodic_sum_converges_in_L():
    # a neutral cell with zero dipole (a charge pair placed symmetrically about
    # the cell centre has a dipole; two opposite pairs cancel it): p_L settles
    b, n = 6.0, 6
    pos = np.array([[-1.5, 0.0, 0.0], [1.5, 0.0, 0.0], [0.0, -1.5, 0.0], [0.0, 1.5, 0.0]])
    Z = np.array([1.0, 1.0, -1.0, -1.0])
    t, w = rule_s(41, 3.7, 2.7e-3 * n / b)
    vals = []
    for L in (5, 9, 17):
        geom = Geometry(b, n, (L, L, L), True)
        F, c = assembled_factors(geom, t, w, pos, Z)
        vals.append(float(reconstruct(F, c, (1, 1, 1), (1, 1, 1))[0, 0, 0]) / geom.h ** 3)
    assert abs(vals[2] - vals[1]) < 0.5 * abs(vals[1] - vals[0])


def test_forces_of_selected_atoms_match_full_adjoint():
    sysm = small_box(51, n=8, M0=4)
    t, w = _tw(sysm)
    geom = _geom(sysm)
    full = forces_adjoint(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d)
    part = forces_adjoint_atoms(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d, [2, 0])
    assert np.allclose(part, full[[2, 0]], rtol=1e-13, atol=1e-15 * np.abs(full).max())


def test_nuclear_matrix_against_full_grid():
    # v_km = sum_i G_k(i) G_m(i) P_i on a tiny full grid (eq. nuc_pot)
    sysm = small_box(61, n=8, L=(2, 2, 2), M0=2)
    t, w = _tw(sysm)
    geom = _geom(sysm)
    F, c = direct_factors(geom, t, w, sysm.pos, sysm.Z)
    g = make_basis(sysm, 5)
    V = nuclear_matrix(F, c, g)
    P = reconstruct(F, c)
    G = [np.einsum("i,j,k->ijk", g[0][k], g[1][k], g[2][k]) for k in range(5)]
    ref = np.array([[np.sum(G[k] * G[m] * P) for m in range(5)] for k in range(5)])
    Vabs = nuclear_matrix(F, np.abs(c), g)
    assert np.max(np.abs(V - ref)) < 1e-13 * np.max(np.abs(Vabs))
    assert np.allclose(V, V.T, rtol=0, atol=1e-14 * np.max(np.abs(Vabs)))


def test_richardson_on_periodic_sums_of_a_dipole_free_cell():
    # the regularised sum of a neutral, dipole-free cell changes little
    # between L and 2L, and the linear formula is exact when p_L is linear
    b, n = 6.0, 6
    pos = np.array([[-1.5, 0.0, 0.0], [1.5, 0.0, 0.0], [0.0, -1.5, 0.0], [0.0, 1.5, 0.0]])
    Z = np.array([1.0, 1.0, -1.0, -1.0])
    t, w = rule_s(41, 3.7, 2.7e-3 * n / b)
    vals = {}
    for L in (4, 8):
        geom = Geometry(b, n, (L, L, L), True)
        F, c = assembled_factors(geom, t, w, pos, Z)
        vals[L] = reconstruct(F, c) / geom.h ** 3
    lin = richardson_linear(vals[4], vals[8])
    assert lin.shape == (n, n, n)
    assert np.max(np.abs(lin - vals[8])) < np.max(np.abs(vals[8] - vals[4])) * 2 + 1e-12
