"""Pins for oracle.prism: exact Galerkin entries p_i (eq. galten)."""
import numpy as np
import pytest
from scipy.integrate import tplquad

from oracle.prism import newton_box_integral, _closed_form, _gauss_legendre, exact_galerkin_entries


def _cubature(lo, hi):
    f = lambda z, y, x: 1.0 / np.sqrt(x * x + y * y + z * z)
    v, _ = tplquad(f, lo[0], hi[0], lo[1], hi[1], lo[2], hi[2], epsabs=1e-14, epsrel=1e-13)
    return v


@pytest.mark.parametrize("lo,hi", [
    ((0, 0, 0), (1, 1, 1)),            # singular corner cell
    ((1, -1, 2), (2, 0, 3)),
    ((-3, 2, -1), (-2, 3, 0)),
    ((0.2, 0.3, 0.1), (0.9, 1.4, 0.6)),
    ((-0.7, 0.0, 0.5), (0.3, 0.2, 1.5)),  # crosses a coordinate plane
    ((4, 5, -6), (5, 6, -5)),
])
def test_closed_form_against_cubature(lo, hi):
    got = newton_box_integral(np.array(lo, float), np.array(hi, float))
    ref = _cubature(lo, hi)
    assert abs(got - ref) / ref < 2e-12


def test_cell_containing_the_charge():
    # [-1/2, 1/2]^3 is eight corner cubes of edge 1/2; p scales like edge^2
    corner = newton_box_integral(np.zeros(3), np.ones(3))
    centred = newton_box_integral(np.full(3, -0.5), np.full(3, 0.5))
    assert abs(centred - 8 * 0.25 * corner) < 1e-14 * centred
    assert abs(corner - _cubature((0, 0, 0), (1, 1, 1))) < 1e-13


def test_closed_form_and_gauss_legendre_overlap():
    rng = np.random.default_rng(0)
    for _ in range(20):
        c = rng.normal(size=3)
        c = c / np.linalg.norm(c) * rng.uniform(3, 5)
        lo = np.floor(c)[None]
        a = _closed_form(lo, lo + 1)
        b = _gauss_legendre(lo, lo + 1)
        assert abs(a - b) / b < 1e-13


def test_multipole_limit():
    # a cube has no dipole (about its centre) and no quadrupole moment, so
    # p = volume/|c| (1 + O(|c|^-4)) far away
    for d in (40.0, 80.0, 160.0):
        c = np.array([d, 0.3 * d, -0.6 * d])
        lo = (c - 0.5)[None]
        p = newton_box_integral(lo, lo + 1.0)
        rel = abs(p * np.linalg.norm(c) - 1.0)
        assert rel < 1.0 / np.linalg.norm(c) ** 4


def test_exact_entries_shift_and_scale():
    cells = np.array([[0, 0, 0], [3, -2, 1], [-1, -1, -1]])
    h = 0.37
    a = exact_galerkin_entries(cells, h, shift=(0.25, 0.5, 0.75))
    lo = (cells - np.array([0.25, 0.5, 0.75])) * h
    assert np.allclose(a, newton_box_integral(lo, lo + h), rtol=1e-15)
    # p scales like h^2
    assert np.allclose(exact_galerkin_entries(cells, 2 * h), 4 * exact_galerkin_entries(cells, h), rtol=1e-13)
