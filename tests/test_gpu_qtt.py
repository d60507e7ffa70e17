"""Quantics-TT compression (Sec. 4, eq. EwaldTensorQTT) through the C ABI
against the oracle's TT-SVD: ranks equal (integers, bit-exact), the expanded
vectors equal the oracle's expansion to 1e-12 of the vector's largest entry,
and the TT-SVD error bound ||x - x_QTT|| <= eps ||x||."""
import numpy as np
import pytest
import torch

from oracle.qtt import tt_svd, tt_full
from oracle.lattice import Geometry, direct_factors, factor_entries
from oracle.quadrature import rule_s
from workloads import small_box, config2

pytestmark = pytest.mark.gpu
dev = torch.device("cuda:0")


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _check(L, X, eps, expect_ok=True):
    X = np.atleast_2d(np.asarray(X, np.float64))
    cores, ranks, status = L.qtt_compress(_t(X), eps)
    Y = L.qtt_expand(cores, ranks, status, X.shape[1]).cpu().numpy()
    ranks, status = ranks.cpu().numpy(), status.cpu().numpy()
    worst = 0.0
    for v in range(X.shape[0]):
        assert status[v] == 1, (v, status[v])
        oc, orr = tt_svd(X[v], eps)
        assert list(ranks[v]) == orr, (v, list(ranks[v]), orr)
        xo = tt_full(oc)[:X.shape[1]]
        scale = np.max(np.abs(X[v]))
        if scale == 0.0:
            assert np.all(Y[v] == 0.0)
            continue
        err = np.max(np.abs(Y[v] - xo)) / scale
        worst = max(worst, err)
        assert err < 1e-12, (v, err)
        assert np.linalg.norm(Y[v] - X[v]) <= eps * np.linalg.norm(X[v]) * (1 + 1e-9) + 1e-13 * np.linalg.norm(X[v])
    return ranks, worst


@pytest.mark.parametrize("d", [2, 5, 8, 10])
def test_random_vectors_exact(d):
    import paper_1405_2270_amd as L
    rng = np.random.default_rng(40 + d)
    _check(L, rng.standard_normal((3, 1 << d)), 0.0)


def test_closed_form_ranks():
    import paper_1405_2270_amd as L
    i = np.arange(4096, dtype=np.float64)
    u = i / 4096
    X = [0.999 ** i, np.sin(0.0137 * i + 0.4)] + [
        np.polynomial.polynomial.polyval(u, np.arange(1, m + 2, dtype=np.float64)) for m in (1, 2, 3)]
    ranks, _ = _check(L, np.array(X), 1e-13)
    assert [int(r.max()) for r in ranks] == [1, 2, 2, 3, 4]


def test_padding_and_zero_vector():
    import paper_1405_2270_amd as L
    rng = np.random.default_rng(44)
    X = np.zeros((3, 100))
    X[0] = np.linspace(1.0, 2.0, 100)
    X[1] = rng.standard_normal(100)
    _check(L, X, 1e-10)


@pytest.mark.parametrize("eps", [1e-4, 1e-8, 1e-12])
def test_assembled_vectors_small_lattice(eps):
    import paper_1405_2270_amd as L
    s = small_box(45, n=16, L=(8, 4, 16), M0=2)
    q = s.quad
    t, w = rule_s(q["M"], q["C0"], q["s"])
    F, _ = direct_factors(Geometry(s.b, s.n, s.L), t, w, s.pos, s.Z)
    for l in range(3):
        _check(L, F[l], eps)


def test_failures_are_reported():
    import paper_1405_2270_amd as L
    rng = np.random.default_rng(46)
    X = _t(rng.standard_normal((2, 4096)))
    cores, ranks, status = L.qtt_compress(X, 0.0)       # generic ranks reach 64
    assert status.cpu().tolist() == [-1, -1]
    Y = L.qtt_expand(cores, ranks, status, 4096)
    assert torch.isnan(Y).all()
    cores, ranks, status = L.qtt_compress(_t(rng.standard_normal((1, 256))), 0.0, cap=40)
    assert status.cpu().tolist() == [-2]


def test_rank_limits_of_the_two_launches():
    # one matrix whose vectors end in different launches: rank 1 (first
    # launch, ranks up to 8), a sum of 8 cosines of rank 16 (each cosine has
    # rank 2; redone by the second launch, ranks up to 32) and a random vector
    # beyond rank 32 (refused)
    import paper_1405_2270_amd as L
    i = np.arange(4096, dtype=np.float64)
    waves = sum(np.cos(wk * i + 0.3 * k) for k, wk in enumerate(np.linspace(0.013, 2.9, 8)))
    X = np.array([0.999 ** i, waves])
    ranks, _ = _check(L, X, 1e-12)
    assert int(ranks[0].max()) == 1 and int(ranks[1].max()) == 16
    rng = np.random.default_rng(47)
    Xg = _t(np.vstack([X, rng.standard_normal((1, 4096))]))
    cores, ranks, status = L.qtt_compress(Xg, 1e-12)
    assert status.cpu().tolist() == [1, 1, -1]


@pytest.mark.slow
def test_headline_factor_rows_sampled():
    # the assembled vectors of the headline workload (N = 4096): 48 rows per
    # axis, every rank term of two atoms, at eps = 1e-6
    import paper_1405_2270_amd as L
    s = config2()
    q = s.quad
    t, w = rule_s(q["M"], q["C0"], q["s"])
    geom = Geometry(s.b, s.n, s.L)
    for l in range(3):
        F = factor_entries(geom, t, s.pos[:2], l, np.arange(4096))
        ranks, worst = _check(L, F, 1e-6)
        print(f"axis {l}: max QTT rank {ranks.max()}, worst expansion difference {worst:.2e}")
