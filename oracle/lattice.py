"""Lattice sums of Newton kernels in canonical format (Sec. 2.2, Sec. 3).

Test infrastructure only (see ``oracle/__init__``).

Geometry (Sec. 2.1 and Sec. 3.1, eq. N0grid): unit cell [-b/2, b/2]^3 with n
cells of size h = b/n per edge. Box case: the lattice cells are shifted by b*k,
k_l = 0..L_l-1, the grid covers B_l = [-b/2, b/2 + (L_l-1) b] with N_l = L_l n
cells, cell g spanning [-b/2 + g h, -b/2 + (g+1) h] (reading G10: image indices
start at 0). Periodic case (Sec. 3.2, eq. EwaldSumP): the potential is wanted
on the reference cell only (N_l = n) and the images are k in {-p..p} for odd
L = 2p+1, and {-L/2 .. L/2-1} for even L (reading G8).

Charges sit anywhere in the unit cell (reading G6): the cell integrals are taken
at the continuous positions a_nu + b k, which reduces to the paper's
node-centred windows when a_nu is a grid node. The offset of cell g from image
k is evaluated as (g - k n) h - (a_nu + b/2), which equals
(-b/2 + g h) - (a_nu + b k) because b = n h, but does not subtract two
coordinates of lattice size (that would cost log10(L n) digits far out). The
cell width is passed as h itself rather than formed as the difference of the
two rounded edges, which matters where a wide Gaussian is nearly flat across
the cell (Sec. 2.1: cells of size h).

The canonical rank index is r = nu*R + q (atom-major); coef[r] = Z_nu w_q is kept
apart from the vectors (reading G4, eq. CP_form).

Two independent routes are given, and T1 requires them to agree to rounding:
  * ``direct_factors``: every image projected at its own position and the
    images summed per vector (the direct sum, eqs. core_tens / EwaldSumE).
  * ``assembled_factors``: one master vector per (atom, axis, q) on a doubled
    grid (eq. master_pot) and windows of it summed over the lattice shifts
    (Theorem 3.1 / eq. EwaldTensorM0, Lemma 3.2).
``brute_force_tensor`` sums the shifted full 3D master tensors over all L^3
images (tiny grids only) as the reference for both.

Non-equidistant tensor lattices (Sec. 3.1, remark after eq. EwaldTensorM0):
``tensor_lattice_factors`` (direct sum at arbitrary per-axis lattice
coordinates), ``tensor_lattice_assembled`` (master windows, for coordinates
that are whole numbers of cells) and ``tensor_lattice_brute_force`` (3D sum
over every image triple). Pinned against each other, against
``direct_factors`` for equidistant coordinates, and against point charges.
"""
from dataclasses import dataclass

import numpy as np

from .projection import gauss_cell_integral, gauss_cell_integral_dpos


@dataclass(frozen=True)
class Geometry:
    b: float
    n: int
    L: tuple
    periodic: bool = False

    @property
    def h(self):
        return self.b / self.n

    def N(self, l):
        return self.n if self.periodic else self.L[l] * self.n

    def edges(self, l):
        """Cell edges x_0..x_N of axis l."""
        return -0.5 * self.b + self.h * np.arange(self.N(l) + 1, dtype=np.float64)

    def images(self, l):
        L = self.L[l]
        if not self.periodic:
            return np.arange(L)
        if L % 2 == 1:
            p = L // 2
            return np.arange(-p, p + 1)
        return np.arange(-(L // 2), L // 2)


def direct_factors(geom, t, w, pos, Z, derivative=False):
    """Direct canonical sum: factors F[l] of shape (M0*R, N_l) and coef.

    F[l][nu*R+q, g] = sum_k b_g(t_q; a_{nu,l} + b k), each image's cell integral
    taken at its own continuous position. With ``derivative`` the entries are
    the derivatives with respect to a_{nu,l} of the same sums (all images move
    with the atom).
    """
    t = np.asarray(t, np.float64)
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    M0, R = pos.shape[0], t.size
    cell = gauss_cell_integral_dpos if derivative else gauss_cell_integral
    F = []
    for l in range(3):
        g = np.arange(geom.N(l))
        out = np.zeros((M0 * R, geom.N(l)))
        for nu in range(M0):
            acc = np.zeros((R, geom.N(l)))
            a = pos[nu, l] + 0.5 * geom.b
            for k in geom.images(l):
                y0 = (g - k * geom.n) * geom.h - a
                y1 = (g + 1 - k * geom.n) * geom.h - a
                acc += cell(t[:, None], y0[None, :], y1[None, :], geom.h)
            out[nu * R:(nu + 1) * R] = acc
        F.append(out)
    coef = (np.asarray(Z, np.float64)[:, None] * np.asarray(w, np.float64)[None, :]).ravel()
    return F, coef


def node_and_offset(geom, a):
    """p = floor((a + b/2)/h) and delta = (a + b/2)/h - p (position in cells)."""
    s = (np.asarray(a, np.float64) + 0.5 * geom.b) / geom.h
    p = np.floor(s)
    return p.astype(np.int64), s - p


def master_extent(geom, l):
    """Half-width X (in cells) of the master grid of axis l: master index
    j in [-X, X) covers every cell offset g - p - k n that a sum needs."""
    ks = geom.images(l)
    lo = -(geom.n - 1) - ks.max() * geom.n          # g=0, p=n-1, largest k
    hi = (geom.N(l) - 1) - ks.min() * geom.n + 1     # g=N-1, p=0, smallest k
    return int(max(-lo, hi))


def master_vectors(geom, t, delta, X, derivative=False):
    """Master vectors (eq. master_pot) for a charge ``delta`` cells right of a
    node: m[q, j + X] = integral over [(j - delta) h, (j + 1 - delta) h] of
    exp(-t_q^2 y^2) dy, for j in [-X, X)."""
    j = np.arange(-X, X, dtype=np.float64)
    cell = gauss_cell_integral_dpos if derivative else gauss_cell_integral
    return cell(np.asarray(t)[:, None], ((j - delta) * geom.h)[None, :],
                ((j + 1.0 - delta) * geom.h)[None, :], geom.h)


def assembled_factors(geom, t, w, pos, Z, derivative=False):
    """Assembled canonical vectors (Theorem 3.1, eq. EwaldTensorM0; Lemma 3.2).

    v[g] = sum_k m[g - p - k n] over the lattice shifts, where m is the master
    vector of the atom's sub-cell offset on a grid twice the size of the
    summation domain.
    """
    t = np.asarray(t, np.float64)
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    M0, R = pos.shape[0], t.size
    F = []
    for l in range(3):
        X = master_extent(geom, l)
        g = np.arange(geom.N(l))
        out = np.zeros((M0 * R, geom.N(l)))
        for nu in range(M0):
            p, d = node_and_offset(geom, pos[nu, l])
            m = master_vectors(geom, t, d, X, derivative)
            acc = np.zeros((R, geom.N(l)))
            for k in geom.images(l):
                acc += m[:, g - p - k * geom.n + X]
            out[nu * R:(nu + 1) * R] = acc
        F.append(out)
    coef = (np.asarray(Z, np.float64)[:, None] * np.asarray(w, np.float64)[None, :]).ravel()
    return F, coef


def brute_force_tensor(geom, t, w, pos, Z):
    """Raw Galerkin tensor P of the lattice by 3D brute force (tiny grids).

    For each atom the full 3D rank-R master tensor on the doubled grid is
    formed once, and its 3D windows for all L1*L2*L3 images are added with
    weight Z_nu (eqs. sub_tens, core_tens, EwaldSumE/EwaldSumP).
    """
    t = np.asarray(t, np.float64)
    w = np.asarray(w, np.float64)
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    shape = tuple(geom.N(l) for l in range(3))
    P = np.zeros(shape)
    X = [master_extent(geom, l) for l in range(3)]
    for nu in range(pos.shape[0]):
        pd = [node_and_offset(geom, pos[nu, l]) for l in range(3)]
        m = [master_vectors(geom, t, pd[l][1], X[l]) for l in range(3)]
        master3d = np.einsum("q,qi,qj,qk->ijk", w, m[0], m[1], m[2])
        for k0 in geom.images(0):
            s0 = np.arange(shape[0]) - pd[0][0] - k0 * geom.n + X[0]
            for k1 in geom.images(1):
                s1 = np.arange(shape[1]) - pd[1][0] - k1 * geom.n + X[1]
                for k2 in geom.images(2):
                    s2 = np.arange(shape[2]) - pd[2][0] - k2 * geom.n + X[2]
                    P += Z[nu] * master3d[np.ix_(s0, s1, s2)]
    return P


def factor_entries(geom, t, pos, l, g, derivative=False):
    """Entries F[l][:, g] of the direct factors for selected cells g only
    (used to sample full-size configurations). Returns shape (M0*R, len(g))."""
    t = np.asarray(t, np.float64)
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    g = np.asarray(g)
    cell = gauss_cell_integral_dpos if derivative else gauss_cell_integral
    out = np.zeros((pos.shape[0] * t.size, g.size))
    for nu in range(pos.shape[0]):
        acc = np.zeros((t.size, g.size))
        a = pos[nu, l] + 0.5 * geom.b
        for k in geom.images(l):
            y0 = (g - k * geom.n) * geom.h - a
            y1 = (g + 1 - k * geom.n) * geom.h - a
            acc += cell(t[:, None], y0[None, :], y1[None, :], geom.h)
        out[nu * t.size:(nu + 1) * t.size] = acc
    return out


def point_charge_potential(geom, pos, Z, points):
    """sum over atoms and images of Z/|x - a| at physical points (shape (m,3))."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    points = np.asarray(points, np.float64)
    K = np.array(np.meshgrid(geom.images(0), geom.images(1), geom.images(2),
                             indexing="ij")).reshape(3, -1).T * geom.b
    out = np.zeros(points.shape[0])
    for nu in range(pos.shape[0]):
        d = points[:, None, :] - (pos[nu] + K)[None, :, :]
        out += Z[nu] * np.sum(1.0 / np.linalg.norm(d, axis=-1), axis=1)
    return out


# ---------------------------------------------------------------------------
# Non-equidistant tensor lattices (Sec. 3.1, the remark after eq.
# EwaldTensorM0: the summation stays valid when the L1 x L2 x L3 lattice is a
# tensor product of arbitrary 1D point sets).
#
# The lattice point k = (k0, k1, k2) shifts every unit-cell charge by
# h (s_0[k0], s_1[k1], s_2[k2]); s_l holds L_l coordinates along axis l in
# units of the grid cell h = b/n, not necessarily whole numbers (equidistant
# box: s_l[k] = n k). Axis l has N_l cells, cell g spanning
# [-b/2 + g h, -b/2 + (g+1) h]. The cell offset from an image is formed as
# (g - s_l[k]) h - (a + b/2): the lattice-size difference g - s_l[k] first,
# so that its rounding error scales with the distance from the image, as in
# the box lattice's (g - k n) h - (a + b/2).
# Because the shift is a tensor product, the 3D sum over all image triples
# splits into per-axis sums (the argument of Theorem 3.1 with the windows
# replaced by arbitrary shifts), so the rank stays M0 * R.
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class TensorLattice:
    b: float
    n: int
    N: tuple       # grid cells per axis
    s: tuple       # three 1D arrays of lattice coordinates (units of h)

    @property
    def h(self):
        return self.b / self.n


def tensor_lattice_factors(tl, t, w, pos, Z, derivative=False):
    """Direct sum over the lattice coordinates of every axis:
    F[l][nu*R+q, g] = sum_k b_g(t_q; a_{nu,l} + h s_l[k]), each image's cell
    integral at its own continuous position. With ``derivative`` the entries
    are the derivatives with respect to a_{nu,l} (all images move with the
    atom)."""
    t = np.asarray(t, np.float64)
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    M0, R = pos.shape[0], t.size
    cell = gauss_cell_integral_dpos if derivative else gauss_cell_integral
    F = []
    for l in range(3):
        g = np.arange(tl.N[l], dtype=np.float64)
        out = np.zeros((M0 * R, tl.N[l]))
        for nu in range(M0):
            acc = np.zeros((R, tl.N[l]))
            a = pos[nu, l] + 0.5 * tl.b
            for sk in np.asarray(tl.s[l], np.float64):
                y0 = (g - sk) * tl.h - a
                y1 = (g + 1.0 - sk) * tl.h - a
                acc += cell(t[:, None], y0[None, :], y1[None, :], tl.h)
            out[nu * R:(nu + 1) * R] = acc
        F.append(out)
    coef = (np.asarray(Z, np.float64)[:, None] * np.asarray(w, np.float64)[None, :]).ravel()
    return F, coef


def tensor_lattice_entries(tl, t, pos, l, g, derivative=False):
    """Columns g of ``tensor_lattice_factors``' factor F[l] only (to sample
    full-size lattices). Returns shape (M0*R, len(g))."""
    t = np.asarray(t, np.float64)
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    g = np.asarray(g, np.float64)
    cell = gauss_cell_integral_dpos if derivative else gauss_cell_integral
    out = np.zeros((pos.shape[0] * t.size, g.size))
    for nu in range(pos.shape[0]):
        acc = np.zeros((t.size, g.size))
        a = pos[nu, l] + 0.5 * tl.b
        for sk in np.asarray(tl.s[l], np.float64):
            acc += cell(t[:, None], ((g - sk) * tl.h - a)[None, :],
                        ((g + 1.0 - sk) * tl.h - a)[None, :], tl.h)
        out[nu * t.size:(nu + 1) * t.size] = acc
    return out


def tensor_lattice_assembled(tl, t, w, pos, Z):
    """The same sum by the paper's route when every lattice coordinate is a
    whole number of cells (s_l[k] = m_k): one master vector per (atom, axis)
    on a doubled grid (eq. master_pot) and, per lattice coordinate, its window
    shifted by m_k cells, added pointwise (Theorem 3.1 with irregular
    shifts)."""
    t = np.asarray(t, np.float64)
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    M0, R = pos.shape[0], t.size
    geom = Geometry(tl.b, tl.n, (1, 1, 1))
    F = []
    for l in range(3):
        m_cells = np.rint(np.asarray(tl.s[l], np.float64)).astype(np.int64)
        if not np.array_equal(m_cells, np.asarray(tl.s[l], np.float64)):
            raise ValueError("lattice coordinates must be whole numbers of cells")
        g = np.arange(tl.N[l])
        X = int(tl.N[l] + tl.n + np.max(np.abs(m_cells)) + 2)
        out = np.zeros((M0 * R, tl.N[l]))
        for nu in range(M0):
            p, d = node_and_offset(geom, pos[nu, l])
            mv = master_vectors(geom, t, d, X)
            acc = np.zeros((R, tl.N[l]))
            for mk in m_cells:
                acc += mv[:, g - p - mk + X]
            out[nu * R:(nu + 1) * R] = acc
        F.append(out)
    coef = (np.asarray(Z, np.float64)[:, None] * np.asarray(w, np.float64)[None, :]).ravel()
    return F, coef


def tensor_lattice_brute_force(tl, t, w, pos, Z):
    """Raw Galerkin tensor of the lattice by 3D brute force (tiny grids): for
    every atom and every image triple (k0, k1, k2), the rank-R tensor
    sum_q w_q (x)_l b(t_q; a_l + h s_l[k_l]) of that single image, formed in
    3D and added with weight Z_nu (eqs. core_tens, EwaldSumE)."""
    t = np.asarray(t, np.float64)
    w = np.asarray(w, np.float64)
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    P = np.zeros(tuple(tl.N))
    edges = [-0.5 * tl.b + tl.h * np.arange(tl.N[l] + 1, dtype=np.float64) for l in range(3)]
    for nu in range(pos.shape[0]):
        for s0 in tl.s[0]:
            for s1 in tl.s[1]:
                for s2 in tl.s[2]:
                    c = pos[nu] + tl.h * np.array([s0, s1, s2])
                    v = [gauss_cell_integral(t[:, None], (edges[l][:-1] - c[l])[None, :],
                                             (edges[l][1:] - c[l])[None, :])
                         for l in range(3)]
                    P += Z[nu] * np.einsum("q,qi,qj,qk->ijk", w, v[0], v[1], v[2])
    return P
