"""Exact entries of the Galerkin Newton tensor P (Sec. 2.1, eq. galten).

Test infrastructure only (see ``oracle/__init__``).

p_i = integral over cell i of 1/|x| dx. For a rectangular cell this is the
classical closed-form Newtonian potential of a uniform box at the origin: with
r = |(x, y, z)|,

    F = xy ln(z+r) + yz ln(x+r) + zx ln(y+r)
        - x^2/2 atan(yz/(xr)) - y^2/2 atan(zx/(yr)) - z^2/2 atan(xy/(zr)),

whose mixed third derivative is 1/r, summed with alternating signs over the
eight corners. The formula is used in the positive octant only (a cell that
crosses a coordinate plane is folded into two pieces there, since 1/|x| is even
in each coordinate), so no logarithm sees a cancelling argument.

Away from the origin the eight-corner sum cancels like (distance/size)^3; cells
whose centre lies at least ``FAR`` cell sizes away use an 8x8x8 Gauss-Legendre
product rule instead, on which the smooth integrand is exact to rounding.

Pins (tests/test_oracle_prism.py): scipy cubature on near cells including the
singular ones, agreement of the two formulas where both hold, and the
multipole limit (a cube has no quadrupole moment, so p = vol/|c| + O(|c|^-5)).
"""
import numpy as np

FAR = 3.0
_GX, _GW = np.polynomial.legendre.leggauss(8)


def _xlog(c, arg):
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(c == 0.0, 0.0, c * np.log(np.where(c == 0.0, 1.0, arg)))


def _sqatan(s, num, den):
    # s^2/2 * atan(num/den), with the s = 0 limit 0 and den = 0 -> pi/2 sign.
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.arctan2(num, den)
    return np.where(s == 0.0, 0.0, 0.5 * s * s * a)


def _corner(x, y, z):
    r = np.sqrt(x * x + y * y + z * z)
    return (_xlog(x * y, z + r) + _xlog(y * z, x + r) + _xlog(z * x, y + r)
            - _sqatan(x, y * z, x * r) - _sqatan(y, z * x, y * r)
            - _sqatan(z, x * y, z * r))


def _octant_box(x0, x1, y0, y1, z0, z1):
    """Integral of 1/|x| over [x0,x1]x[y0,y1]x[z0,z1] with all bounds >= 0."""
    tot = 0.0
    for xs, sx in ((x1, 1.0), (x0, -1.0)):
        for ys, sy in ((y1, 1.0), (y0, -1.0)):
            for zs, sz in ((z1, 1.0), (z0, -1.0)):
                tot = tot + sx * sy * sz * _corner(xs, ys, zs)
    return tot


def _fold(lo, hi):
    """Pieces of [lo, hi] folded into [0, inf): list of (a, b, mask)."""
    p1a = np.where(lo >= 0, lo, np.where(hi <= 0, -hi, 0.0))
    p1b = np.where(lo >= 0, hi, np.where(hi <= 0, -lo, hi))
    p2a = np.zeros_like(lo)
    p2b = np.where((lo < 0) & (hi > 0), -lo, 0.0)
    return [(p1a, p1b), (p2a, p2b)]


def _closed_form(lo, hi):
    pieces = [_fold(lo[..., d], hi[..., d]) for d in range(3)]
    tot = np.zeros(lo.shape[:-1])
    for ax, bx in pieces[0]:
        for ay, by in pieces[1]:
            for az, bz in pieces[2]:
                live = (bx > ax) & (by > ay) & (bz > az)
                v = _octant_box(ax, bx, ay, by, az, bz)
                tot = tot + np.where(live, v, 0.0)
    return tot


def _gauss_legendre(lo, hi):
    half = 0.5 * (hi - lo)
    mid = 0.5 * (hi + lo)
    pts = [mid[..., d, None] + half[..., d, None] * _GX for d in range(3)]
    X = pts[0][..., :, None, None]
    Y = pts[1][..., None, :, None]
    Z = pts[2][..., None, None, :]
    W = _GW[:, None, None] * _GW[None, :, None] * _GW[None, None, :]
    f = W / np.sqrt(X * X + Y * Y + Z * Z)
    return f.sum(axis=(-3, -2, -1)) * half[..., 0] * half[..., 1] * half[..., 2]


def newton_box_integral(lo, hi):
    """Integral of 1/|x| over boxes [lo, hi] (arrays of shape (..., 3))."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    size = np.max(hi - lo, axis=-1)
    centre = np.linalg.norm(0.5 * (lo + hi), axis=-1)
    far = centre >= FAR * size
    out = np.empty(lo.shape[:-1])
    if np.any(far):
        out[far] = _gauss_legendre(lo[far], hi[far])
    if np.any(~far):
        out[~far] = _closed_form(lo[~far], hi[~far])
    return out


def exact_galerkin_entries(cells, h, shift=(0.0, 0.0, 0.0)):
    """p_i for integer cells i (shape (m, 3)) of a grid of size h.

    Cell i spans [(i - shift) h, (i + 1 - shift) h] in each coordinate, i.e. the
    charge sits ``shift`` cells to the right of the node that opens cell 0.
    """
    cells = np.asarray(cells, np.float64)
    s = np.asarray(shift, np.float64)
    return newton_box_integral((cells - s) * h, (cells + 1.0 - s) * h)
