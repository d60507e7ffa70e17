"""The number of Hermite-series terms the cell integrals keep (flat cells of
the kernel vectors, Sec. 2.1): the thresholds on c = tau/2 in the device
header must cut the series only where the dropped terms are negligible.

The series is exp(-a^2) sum_m H_2m(a) c^2m / (2m+1)!, the mean of exp(-u^2)
over [a - c, a + c]; a cell takes it when tau <= 0.35 and |a| tau <= 0.25.
Here the kept and the full (40-term) sums are formed in extended precision
with the Hermite recurrence, over a grid of (a, c) covering that domain up to
each threshold, and the dropped part must stay below 1e-16 (the cell values
are at most 1 in these units, and the parity gate on the factors is 1e-12 of
each row's maximum). CPU only; the thresholds are read from the source."""
import math
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1405_2270_amd", "csrc", "ls_common.hpp")


def thresholds():
    src = open(HDR).read()
    m = re.search(r"const int mt = (.*?);", src, re.S)
    assert m, "term-count expression not found"
    pairs = re.findall(r"c < ([0-9.eE+-]+) \? (\d+)", m.group(1))
    last = re.search(r": (\d+)\s*$", m.group(1).strip())
    assert pairs and last
    return [(float(t), int(n)) for t, n in pairs], int(last.group(1))


def series(a, c, terms):
    """exp(-a^2) times the first `terms` terms (m = 0 .. terms-1), longdouble."""
    a = np.longdouble(a)
    c2 = np.longdouble(c) ** 2
    hkm1, hk = np.longdouble(1), 2 * np.abs(a)   # H_0, H_1 at |a|
    s = np.longdouble(1)
    cp = np.longdouble(1)
    fact = np.longdouble(1)                      # (2m+1)!
    for m in range(1, terms):
        h2 = 2 * np.abs(a) * hk - 2 * (2 * m - 1) * hkm1
        h3 = 2 * np.abs(a) * h2 - 2 * (2 * m) * hk
        hkm1, hk = h2, h3
        cp *= c2
        fact *= (2 * m) * (2 * m + 1)
        s += h2 * cp / fact
    return np.exp(-a * a) * s


def test_series_matches_the_integral_it_expands():
    # pin the expansion itself: mean of exp(-u^2) over [a-c, a+c] by erf
    for a, c in [(0.0, 0.1), (0.7, 0.05), (2.5, 0.02), (-1.3, 0.15)]:
        exact = math.sqrt(math.pi) / (4 * c) * (math.erf(a + c) - math.erf(a - c))
        assert abs(float(series(a, c, 40)) - exact) < 1e-14


def test_kept_terms_bound_the_dropped_part():
    table, last = thresholds()
    assert last == 8
    edges = [0.0] + [t for t, _ in table] + [0.175]
    counts = [n for _, n in table] + [last]
    worst = 0.0
    for lo, hi, n in zip(edges[:-1], edges[1:], counts):
        for c in np.linspace(max(lo, 1e-7), hi * (1 - 1e-12), 7):
            tau = 2 * c
            amax = min(0.25 / tau, 27.0)             # the series domain; beyond 27 exp(-a^2) = 0
            for a in np.linspace(0.0, amax, 41):
                err = abs(float(series(a, c, 40) - series(a, c, n)))
                worst = max(worst, err)
                assert err < 1e-16, (c, a, n, err)
    assert worst > 0.0
