"""Energy, forces and Richardson extrapolation on top of the lattice sums.

Test infrastructure only (see ``oracle/__init__``).

Energy: E = <P, rho>, the canonical scalar product (Appendix, eq. scal) of the
raw Galerkin lattice tensor P with a charge density rho sampled at cell
midpoints and held in canonical form (D, d) (Sec. 2.2, Example 2.1: sampling at
midpoints, eq. nuc_pot). Since P's entries are cell integrals of the potential,
E approximates the integral of rho times the potential.

Forces: F_{nu,l} = -dE/da_{nu,l}. Moving atom nu moves all its lattice images,
and only the axis-l vectors of atom nu depend on a_{nu,l}, so
  dE/da_{nu,l} = Z_nu sum_q w_q sum_s d_s G'_l[nu q, s] prod_{l' != l} G_{l'}[nu q, s]
with G_l = F_l D_l^T and G'_l the same Gram of the derivative vectors. The
finite-difference route re-evaluates E at displaced positions and shares
nothing with this formula but the energy itself.

Richardson (Sec. 3.2): for sums growing linearly in L, 2 p_L - p_{2L}; for
quadratic growth, (4 p_L - p_{2L})/3.

Nuclear-potential operator matrix (Sec. 2.2, Example 2.1, eq. nuc_pot): for
separable basis functions G_k = g_k^(1) (x) g_k^(2) (x) g_k^(3) sampled at cell
midpoints, v_km = <G_k (.) G_m, P> with the Hadamard product of eq. had and the
scalar product of eq. scal.
"""
import numpy as np

from .lattice import direct_factors
from .canonical import scalar_product, hadamard


def energy(geom, t, w, pos, Z, D, d, factors=None):
    """E = <P, rho> (eq. scal)."""
    if factors is None:
        factors = direct_factors(geom, t, w, pos, Z)
    F, coef = factors
    return scalar_product(F, coef, D, d)


def forces_adjoint(geom, t, w, pos, Z, D, d):
    """F[nu, l] = -dE/da_{nu,l} from value and derivative Grams."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    M0, R = pos.shape[0], len(t)
    F, _ = direct_factors(geom, t, w, pos, Z)
    dF, _ = direct_factors(geom, t, w, pos, Z, derivative=True)
    G = [F[l] @ D[l].T for l in range(3)]
    dG = [dF[l] @ D[l].T for l in range(3)]
    coef = (np.asarray(Z, np.float64)[:, None] * np.asarray(w)[None, :]).ravel()
    out = np.zeros((M0, 3))
    for l in range(3):
        prod = dG[l].copy()
        for m in range(3):
            if m != l:
                prod = prod * G[m]
        per_r = coef * (prod @ np.asarray(d))
        out[:, l] = -per_r.reshape(M0, R).sum(axis=1)
    return out


def forces_adjoint_atoms(geom, t, w, pos, Z, D, d, atoms):
    """Rows ``atoms`` of ``forces_adjoint``, computing only those atoms'
    vectors (the force on atom nu involves atom nu's Grams only)."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    Z = np.asarray(Z, np.float64)
    out = np.zeros((len(atoms), 3))
    for i, nu in enumerate(atoms):
        out[i] = forces_adjoint(geom, t, w, pos[nu:nu + 1], Z[nu:nu + 1], D, d)[0]
    return out


def forces_fd(geom, t, w, pos, Z, D, d, step):
    """Central finite differences of the oracle energy (step in length units)."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    out = np.zeros_like(pos)
    for nu in range(pos.shape[0]):
        for l in range(3):
            pp = pos.copy()
            pm = pos.copy()
            pp[nu, l] += step
            pm[nu, l] -= step
            out[nu, l] = -(energy(geom, t, w, pp, Z, D, d) - energy(geom, t, w, pm, Z, D, d)) / (2 * step)
    return out


def richardson_linear(pL, p2L):
    """Regularised value for a sum growing like c L: 2 p_L - p_2L."""
    return 2.0 * np.asarray(pL) - np.asarray(p2L)


def richardson_quadratic(pL, p2L):
    """Regularised value for a sum growing like c L^2: (4 p_L - p_2L)/3."""
    return (4.0 * np.asarray(pL) - np.asarray(p2L)) / 3.0


def nuclear_matrix(F, coef, g):
    """v_km = <G_k (.) G_m, P> (eq. nuc_pot): G_k (.) G_m is the rank-one
    canonical tensor with vectors g_k^(l) (.) g_m^(l) (eq. had), and the scalar
    product with the canonical P follows eq. scal. g[l]: (N_b, N_l)."""
    Nb = g[0].shape[0]
    V = np.zeros((Nb, Nb))
    for k in range(Nb):
        for m in range(Nb):
            Hk = [(g[l][k] * g[l][m])[None, :] for l in range(3)]
            V[k, m] = scalar_product(F, coef, Hk, np.ones(1))
    return V
