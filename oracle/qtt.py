"""Quantics-TT (QTT) compression of assembled canonical vectors (Sec. 4,
eq. EwaldTensorQTT; Appendix, the TT format eq. tt and the quantics folding).

Test infrastructure only (see ``oracle/__init__``).

A vector of length N = 2^d is folded into a 2 x 2 x ... x 2 tensor of order d
and written in the tensor-train format (eq. tt): entry i is the product of d
matrices G_k[:, j_k, :] of sizes r_{k-1} x r_k (r_0 = r_d = 1), where the
j_k are the binary digits of i. The QTT ranks are the r_k.

Readings (the paper gives the format but not the compression algorithm):
  * digit order: j_1 is the most significant bit (the row-major folding
    x.reshape(2, ..., 2)); the paper's coding takes the least significant bit
    first. Each unfolding separates the same digits in both orders, so the
    exact ranks are the same sequence reversed; only the order of the
    truncation sweep differs.
  * algorithm: the TT-SVD of Oseledets (SIAM J. Sci. Comput. 33, 2011):
    left to right, the unfolding with rows (alpha_{k-1}, j_k) is decomposed
    by the SVD, the left singular vectors of the kept singular values form
    core k, and S V^T, refolded, goes on to step k+1.
  * truncation: at every step the smallest rank r whose discarded singular
    values have Euclidean norm <= delta = eps ||x||_2 / sqrt(d - 1), so that
    ||x - x_QTT||_2 <= eps ||x||_2 (the theorem behind TT-SVD). eps = 0 keeps
    every non-zero singular value (r >= 1 always).
  * N not a power of two: zero padding to the next power of two (d >= 2).

Pins (tests/test_oracle_qtt.py): exact reconstruction at eps = 0 with the
generic ranks min(2^k, 2^(d-k)); the closed-form QTT ranks the Appendix
states (1 for exponentials, 2 for sampled trigonometric functions, m + 1 for
polynomials of degree m); the error bound; the block lemma (Lemma 4.3: a
vector made of repeated copies of a block has the block's ranks).
"""
import numpy as np


def qtt_digits(N):
    """d with 2^d >= N, d >= 2."""
    d = 2
    while (1 << d) < N:
        d += 1
    return d


def tt_svd(x, eps):
    """QTT cores [G_1 .. G_d] (G_k of shape (r_{k-1}, 2, r_k)) and the ranks
    [r_0 .. r_d] of the vector x (zero-padded to a power of two)."""
    x = np.asarray(x, np.float64).ravel()
    d = qtt_digits(x.size)
    xp = np.zeros(1 << d)
    xp[:x.size] = x
    delta = eps * np.linalg.norm(xp) / np.sqrt(d - 1)
    cores, ranks = [], [1]
    C = xp.reshape(2, -1)              # rows j_1, columns the other digits
    r = 1
    for _ in range(d - 1):
        U, S, Vt = np.linalg.svd(C, full_matrices=False)
        # tail[i] = || S[i:] ||_2
        tail = np.sqrt(np.cumsum((S ** 2)[::-1]))[::-1]
        rk = S.size
        for i in range(1, S.size):
            if tail[i] <= delta:
                rk = i
                break
        cores.append(U[:, :rk].reshape(r, 2, rk))
        C = (S[:rk, None] * Vt[:rk]).reshape(rk * 2, -1)
        r = rk
        ranks.append(rk)
    cores.append(C.reshape(r, 2, 1))
    ranks.append(1)
    return cores, ranks


def tt_full(cores):
    """The vector of length 2^d that QTT cores represent (eq. tt)."""
    v = np.ones((1, 1))
    for G in cores:
        r0, q, r1 = G.shape
        v = (v @ G.reshape(r0, q * r1)).reshape(-1, r1)
    return v.ravel()


def tt_storage(ranks):
    """Numbers stored by the QTT cores: sum_k 2 r_{k-1} r_k."""
    return int(sum(2 * ranks[k] * ranks[k + 1] for k in range(len(ranks) - 1)))
