"""Pins for oracle.physics: energy (eq. scal), forces, Richardson (Sec. 3.2)."""
import numpy as np
import pytest

from oracle.lattice import Geometry, direct_factors, assembled_factors
from oracle.canonical import reconstruct
from oracle.physics import (energy, forces_adjoint, forces_adjoint_atoms, forces_fd,
                            richardson_linear, richardson_quadratic)
from workloads import small_box, small_periodic
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
