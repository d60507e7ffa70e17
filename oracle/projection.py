"""1D Gaussian cell integrals (Sec. 2.1, eqs. C_nD_0 and galten_int).

Test infrastructure only (see ``oracle/__init__``).

The canonical vectors of the Newton kernel are, entry by entry,

    b_i(t) = integral over cell i of exp(-t^2 x^2) dx              (eq. galten_int)

for a piecewise-constant basis function psi_i (the indicator of cell i). Here
the cell is given directly by its two edges y0 < y1, measured from the charge.

Method (plain definition, written out):
  * t = 0: the integral is the cell width.
  * Otherwise, with u = t*y, the integral is sqrt(pi)/(2t) times a difference of
    error functions. The difference is taken on the side where it does not
    cancel: erfc on each tail, erf across the origin (a sum of two positive
    terms there).
  * When the two erfc values are so close that their difference would lose more
    than two bits (condition number erfc(a)/(erfc(a)-erfc(b)) > 4), the
    integrand is nearly constant across the cell and a 20-point Gauss-Legendre
    rule on the cell is used instead; it is exact to rounding there.

Pins (tests/test_oracle_projection.py): mpmath at 40 digits on random and
ill-conditioned cells, the telescoping identity over a partition, t=0, mirror
symmetry, and central differences for the derivative.
"""
import numpy as np
from scipy.special import erf, erfc

_SQRT_PI = np.sqrt(np.pi)
_GL_X, _GL_W = np.polynomial.legendre.leggauss(20)
_COND_MAX = 4.0


def _gauss_legendre_cell(t, y0, y1, width):
    half = 0.5 * width
    mid = 0.5 * (y1 + y0)
    y = mid[..., None] + half[..., None] * _GL_X
    f = np.exp(-(t[..., None] * y) ** 2)
    return half * (f @ _GL_W)


def gauss_cell_integral(t, y0, y1, width=None):
    """Integral of exp(-t^2 y^2) over [y0, y1] (eq. galten_int), broadcasting.

    t >= 0 and y0 < y1 are required. FP64 throughout. ``width``: the cell
    width y1 - y0 when the caller knows it exactly (the grid's h); far from the
    charge the difference of the two rounded edges loses log10(|y|/h) digits,
    which matters where the integrand is nearly flat (the t = 0 and
    Gauss-Legendre branches).
    """
    if width is None:
        width = np.asarray(y1, np.float64) - np.asarray(y0, np.float64)
    t, y0, y1, width = np.broadcast_arrays(np.asarray(t, np.float64),
                                           np.asarray(y0, np.float64),
                                           np.asarray(y1, np.float64),
                                           np.asarray(width, np.float64))
    out = np.empty(t.shape, np.float64)
    zero_t = t == 0.0
    out[zero_t] = width[zero_t]
    nz = ~zero_t
    tt, a0, a1, wd = t[nz], y0[nz], y1[nz], width[nz]
    u0, u1 = tt * a0, tt * a1
    right = u0 >= 0.0
    left = u1 <= 0.0
    mid = ~(right | left)
    big = np.empty_like(u0)       # larger erfc (or the whole value across 0)
    diff = np.empty_like(u0)
    big[right] = erfc(u0[right])
    diff[right] = big[right] - erfc(u1[right])
    big[left] = erfc(-u1[left])
    diff[left] = big[left] - erfc(-u0[left])
    diff[mid] = erf(u1[mid]) + erf(-u0[mid])
    big[mid] = diff[mid]
    val = (_SQRT_PI / (2.0 * tt)) * diff
    # erfc underflow on both edges: the true value is below the FP64 range.
    underflow = big == 0.0
    val[underflow] = 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        cond = np.where(underflow, 1.0, big / diff)
    ill = ~(cond <= _COND_MAX)
    if np.any(ill):
        val[ill] = _gauss_legendre_cell(tt[ill], a0[ill], a1[ill], wd[ill])
    out[nz] = val
    return out


def gauss_cell_integral_dpos(t, y0, y1, width=None):
    """Derivative of the cell integral with respect to the charge position a.

    With y = x - a the cell is [x0 - a, x1 - a] = [y0, y1], so
    d/da = exp(-t^2 y0^2) - exp(-t^2 y1^2). It is evaluated as the larger
    exponential times -expm1 of the exponent difference, which does not cancel.
    ``width`` as in ``gauss_cell_integral``.
    """
    if width is None:
        width = np.asarray(y1, np.float64) - np.asarray(y0, np.float64)
    t, y0, y1, width = np.broadcast_arrays(np.asarray(t, np.float64),
                                           np.asarray(y0, np.float64),
                                           np.asarray(y1, np.float64),
                                           np.asarray(width, np.float64))
    t2 = t * t
    # y1^2 - y0^2 = (y1 - y0)(y1 + y0)
    dsq = width * (y1 + y0)
    near0 = np.abs(y0) <= np.abs(y1)
    out = np.empty(t.shape, np.float64)
    # |y0| <= |y1|: e0 - e1 = e0 * (1 - exp(-t^2 dsq)) = -e0 * expm1(-t^2 dsq)
    a = near0
    out[a] = -np.exp(-t2[a] * y0[a] * y0[a]) * np.expm1(-t2[a] * dsq[a])
    # otherwise:   e0 - e1 = e1 * (exp(t^2 dsq) - 1) = e1 * expm1(t^2 dsq), dsq < 0
    b = ~near0
    out[b] = np.exp(-t2[b] * y1[b] * y1[b]) * np.expm1(t2[b] * dsq[b])
    return out
