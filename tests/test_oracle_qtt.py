"""Pins for oracle.qtt (Sec. 4; Appendix: TT format and quantics folding)."""
import numpy as np
import pytest

from oracle.qtt import tt_svd, tt_full, tt_storage, qtt_digits


@pytest.mark.parametrize("d", [2, 5, 8, 10])
def test_exact_at_eps_zero_with_generic_ranks(d):
    rng = np.random.default_rng(d)
    x = rng.standard_normal(1 << d)
    cores, ranks = tt_svd(x, 0.0)
    assert ranks == [min(1 << k, 1 << (d - k)) for k in range(d + 1)]
    assert np.max(np.abs(tt_full(cores) - x)) < 1e-13 * np.max(np.abs(x))
    assert tt_storage(ranks) == sum(c.size for c in cores)


def test_closed_form_ranks_of_the_appendix():
    # exponentials: rank 1; sampled sine and cosine: rank 2; polynomials of
    # degree m: rank m + 1 (for every unfolding with enough digits)
    d = 12
    i = np.arange(1 << d, dtype=np.float64)
    _, r = tt_svd(0.999 ** i, 1e-13)
    assert max(r) == 1
    _, r = tt_svd(np.sin(0.0137 * i + 0.4), 1e-13)
    assert max(r) == 2
    u = i / (1 << d)
    for m in (1, 2, 3, 4):
        p = np.polynomial.polynomial.polyval(u, np.arange(1, m + 2, dtype=np.float64))
        _, r = tt_svd(p, 1e-13)
        assert max(r) == m + 1, (m, r)


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_error_bound_and_monotone_ranks(eps):
    rng = np.random.default_rng(3)
    d = 11
    i = np.arange(1 << d)
    # a sum of Gaussians of several widths and centres (the canonical vectors'
    # shape), plus a little noise so that the ranks depend on eps
    x = sum(np.exp(-((i - c) / w) ** 2) for c, w in zip(rng.uniform(0, 1 << d, 6),
                                                         rng.uniform(3, 300, 6)))
    x = x + 1e-7 * rng.standard_normal(x.size)
    cores, ranks = tt_svd(x, eps)
    assert np.linalg.norm(tt_full(cores) - x) <= eps * np.linalg.norm(x) * (1 + 1e-12)
    _, ranks2 = tt_svd(x, eps * 10)
    assert all(a <= b for a, b in zip(ranks2, ranks))


def test_block_lemma_repeated_blocks():
    # Lemma 4.3: a vector of 2^L2 copies of a block x0 (length 2^L1): with the
    # most significant digits first, the copies are the leading L2 digits, on
    # which the vector is constant: ranks 1 there, then the block's own ranks
    rng = np.random.default_rng(5)
    L1, L2 = 6, 4
    x0 = np.exp(-((np.arange(1 << L1) - 20.0) / 7.0) ** 2) + 0.1 * rng.standard_normal(1 << L1)
    x = np.tile(x0, 1 << L2)
    _, r0 = tt_svd(x0, 1e-12)
    _, r = tt_svd(x, 1e-12)
    assert r[:L2 + 1] == [1] * (L2 + 1)
    assert r[L2:] == r0


def test_zero_padding_and_digits():
    assert qtt_digits(1) == 2 and qtt_digits(4) == 2 and qtt_digits(5) == 3 and qtt_digits(4096) == 12
    x = np.linspace(1.0, 2.0, 100)
    cores, ranks = tt_svd(x, 0.0)
    v = tt_full(cores)
    assert v.size == 128 and np.max(np.abs(v[:100] - x)) < 1e-14 * 2 and np.all(np.abs(v[100:]) < 1e-14)


def test_truncation_rank_is_minimal():
    # x = a + eta b with a of QTT rank 1 (an exponential) and b a random unit
    # vector: by Eckart-Young every unfolding has a rank-1 approximation within
    # eta, so a threshold delta = 1.2 eta must give rank 1 everywhere, while a
    # threshold below the discarded norms (about eta / sqrt(2) at the first
    # unfolding) must keep rank 2 there
    rng = np.random.default_rng(9)
    d = 10
    a = 0.997 ** np.arange(1 << d)
    b = rng.standard_normal(1 << d)
    b /= np.linalg.norm(b)
    eta = 1e-4 * np.linalg.norm(a)
    x = a + eta * b
    scale = np.sqrt(d - 1) / np.linalg.norm(x)
    _, r = tt_svd(x, 1.2 * eta * scale)
    assert r == [1] * (d + 1)
    _, r = tt_svd(x, 0.5 * eta * scale)
    assert r[1] == 2
