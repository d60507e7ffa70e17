"""The library's erfc (the cell integrals' edge values, ls_erfc_fit.hpp).

Pinned against 40-digit mpmath erfc: the header's polynomial, evaluated in
double precision step by step as the device does, stays within 2e-15
relative error on [0, 26.5] (erfc a normal double there); the header is what
its generator writes (no hand edits)."""
import os
import re

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1405_2270_amd", "csrc")
HDR = os.path.join(CSRC, "ls_erfc_fit.hpp")


def _parse():
    src = open(HDR).read()
    body = src[src.index("constexpr double c["):src.index("};")]
    coef = [float(v) for v in re.findall(r"[-+]?\d+\.\d+(?:e[-+]?\d+)?", body.split("=", 1)[1])]
    A, B = [float(v) for v in re.search(r"fma\(([-\d.e]+), t, ([-\d.e]+)\)", src).groups()]
    return coef, A, B


def _fit(u, coef, A, B):
    # the device steps in double; the FMA remainder of u*u taken exactly
    t = 4.0 / (4.0 + u)
    x = A * t + B
    p = coef[-1]
    for c in coef[-2::-1]:
        p = p * x + c
    hi = u * u
    lo = float(mp.mpf(u) * mp.mpf(u) - mp.mpf(hi))
    e = float(mp.exp(-mp.mpf(hi)))  # exp correctly rounded
    return (e - e * lo) * (t * p)


def test_header_is_generated():
    import importlib.util
    spec = importlib.util.spec_from_file_location("gen_erfc_fit", os.path.join(CSRC, "gen_erfc_fit.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    A, B, mono = gen.coefficients()
    assert gen.render(A, B, mono) == open(HDR).read()


def test_accuracy_against_mpmath():
    mp.mp.dps = 40
    coef, A, B = _parse()
    assert len(coef) == 23
    rng = np.random.default_rng(5)
    us = np.concatenate([np.linspace(0.0, 26.5, 1200), rng.uniform(0.0, 26.5, 1200),
                         rng.uniform(0.0, 0.5, 300), [0.0, 1e-300, 1e-8, 26.5]])
    worst = 0.0
    for u in us:
        u = float(u)
        ref = mp.erfc(mp.mpf(u))
        worst = max(worst, float(abs(mp.mpf(_fit(u, coef, A, B)) / ref - 1)))
    assert worst < 2e-15, worst


def test_planted_coefficient_error_is_caught():
    # a single coefficient off by one part in 1e-12 breaks the bound
    mp.mp.dps = 40
    coef, A, B = _parse()
    bad = list(coef)
    bad[7] *= 1 + 1e-12
    errs = [float(abs(mp.mpf(_fit(u, bad, A, B)) / mp.erfc(mp.mpf(u)) - 1))
            for u in np.linspace(0.0, 26.5, 300)]
    assert max(errs) > 2e-15
