"""Canonical-format operations (Appendix: eqs. CP_form, scal, had, conc).

Test infrastructure only (see ``oracle/__init__``).

A canonical tensor is (F, coef): F[l] has shape (K, n_l), one row per rank-one
term, and A = sum_r coef[r] F[0][r] (x) F[1][r] (x) F[2][r] (eq. CP_form).
"""
import numpy as np


def reconstruct(F, coef, origin=(0, 0, 0), extent=None):
    """Full sub-box A[o0:o0+e0, o1:o1+e1, o2:o2+e2] by a plain einsum."""
    if extent is None:
        extent = tuple(F[l].shape[1] - origin[l] for l in range(3))
    s = [slice(origin[l], origin[l] + extent[l]) for l in range(3)]
    return np.einsum("r,ri,rj,rk->ijk", coef, F[0][:, s[0]], F[1][:, s[1]], F[2][:, s[2]])


def sample(F, coef, idx):
    """Entries A[i, j, k] for index triples idx (shape (m, 3)) in extended
    precision (np.longdouble products and sums)."""
    idx = np.asarray(idx)
    c = np.asarray(coef, np.longdouble)
    a = np.asarray(F[0][:, idx[:, 0]], np.longdouble)
    b = np.asarray(F[1][:, idx[:, 1]], np.longdouble)
    d = np.asarray(F[2][:, idx[:, 2]], np.longdouble)
    return np.sum(c[:, None] * a * b * d, axis=0)


def sample_columns(cols, coef, sel):
    """Entries from factor columns only: cols[l] has shape (K, m_l) holding the
    factor columns at the distinct indices of axis l, and sel (m, 3) picks one
    column per axis for each requested entry. Extended precision."""
    sel = np.asarray(sel)
    c = np.asarray(coef, np.longdouble)
    a = np.asarray(cols[0], np.longdouble)[:, sel[:, 0]]
    b = np.asarray(cols[1], np.longdouble)[:, sel[:, 1]]
    d = np.asarray(cols[2], np.longdouble)[:, sel[:, 2]]
    return np.sum(c[:, None] * a * b * d, axis=0)


def scalar_product(FA, ca, FB, cb):
    """<A, B> = sum_i sum_j c_i c_j prod_l <a_i^(l), b_j^(l)>  (eq. scal)."""
    G = np.ones((len(ca), len(cb)))
    for l in range(3):
        G = G * (FA[l] @ FB[l].T)
    return float(np.asarray(ca) @ G @ np.asarray(cb))


def hadamard(FA, ca, FB, cb):
    """A (.) B in canonical form: rank Ra*Rb, 1D pointwise products (eq. had)."""
    F = [np.einsum("in,jn->ijn", FA[l], FB[l]).reshape(-1, FA[l].shape[1]) for l in range(3)]
    return F, np.outer(ca, cb).ravel()


def concatenate(FA, ca, FB, cb):
    """A + B by concatenating factor matrices: rank Ra+Rb (eq. conc)."""
    return [np.concatenate([FA[l], FB[l]]) for l in range(3)], np.concatenate([ca, cb])
