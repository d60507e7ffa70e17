"""FP16x3 rank order and chunk skipping (Appendix, eq. CP_form).

The preparation of LS_F16X3 puts the ranks in decreasing max|f0[r]| and marks,
per plane i of axis 0, the 32-rank chunks with a nonzero FP16 term there; the
persistent tiles skip the others. Checked here: the order and the marks
against their definition, recomputed on the host from the device factors
(exact: the same FP64 products), the reported work, and the reconstruction
with skipped chunks against the oracle, every FP16x3 tile, on a box where a
third of the planes skip the narrow terms' chunk.
"""
import numpy as np
import pytest
import torch

from oracle.canonical import reconstruct as o_reconstruct
from oracle.lattice import Geometry, direct_factors
from oracle.quadrature import rule_s
from workloads import small_box
from _gates import gate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_2270_amd as L
    return L


def _floor_log2(m):
    # floor(log2 m) for m > 0, exactly (0 for a zero row, as the library)
    f, e = np.frexp(m)
    return np.where(m > 0, e - 1, 0).astype(np.float64)


def _setup(L):
    sysm = small_box(151, n=32, L=(3, 2, 2), M0=2)
    q = sysm.quad
    t, w = rule_s(q["M"], q["C0"], q["s"])
    qt = L.quadrature("S", q["M"], q["C0"], q["s"])
    dev = torch.device("cuda:0")
    T = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    spec = L.LatticeSpec(sysm.b, sysm.n, sysm.L, False)
    F, coef = L.assemble(spec, qt, T(sysm.pos), T(sysm.Z), None)
    return sysm, t, w, F, coef


def test_order_marks_and_work(L):
    sysm, t, w, F, coef = _setup(L)
    ws = L.reconstruct_prepare(F, coef, "f16x3")
    N = [f.shape[1] for f in F]
    boxes = [(0, 0, 0, N[0], N[1], N[2]), (5, 3, 7, 40, 17, 9)]
    plan = L.reconstruct_f16_plan(F, coef, boxes, ws)
    f = [x.cpu().numpy() for x in F]
    c = coef.cpu().numpy()
    K = c.size
    m0, m1, m2 = (np.abs(x).max(axis=1) for x in f)
    # the order: decreasing max|f0[r]|, ties by index
    perm = np.lexsort((np.arange(K), -m0))
    assert np.array_equal(plan["perm"], perm)
    # the scales and the marks, as the header defines them
    e1, e2 = _floor_log2(m1), _floor_log2(m2)
    bound = np.abs(c) * m0 * m2 * 2.0 ** (e1 - 13)
    g = 13 - _floor_log2(np.array([bound.max()]))[0]
    c32 = c * 2.0 ** (g - 13 + e1) * 2.0 ** e2
    nz = np.abs(c32[perm][:, None] * f[0][perm]) > 2.0 ** -27
    nch = (K + 31) // 32
    want = np.zeros(N[0], np.uint32)
    for ch in range(nch):
        want |= np.where(nz[32 * ch:32 * ch + 32].any(axis=0), np.uint32(1 << ch), np.uint32(0))
    assert np.array_equal(plan["masks"], want)
    # some planes skip the chunk of the narrowest terms
    assert 0 < int((want == 1).sum()) < N[0]
    runs = np.array([bin(int(m)).count("1") if m else 1 for m in want])
    cv = sum(int(runs[b[0]:b[0] + b[3]].sum()) * b[4] * b[5] for b in boxes)
    assert plan["chunk_values"] == cv < nch * sum(b[3] * b[4] * b[5] for b in boxes)


def test_skipping_tiles_against_oracle(L):
    sysm, t, w, F, coef = _setup(L)
    Fo, co = direct_factors(Geometry(sysm.b, sysm.n, sysm.L, False), t, w, sysm.pos, sysm.Z)
    h3 = sysm.h ** 3
    N = [f.shape[1] for f in F]
    boxes = [(0, 0, 0, N[0], N[1], N[2]), (5, 3, 7, 40, 17, 9)]
    refs = [(o_reconstruct(Fo, co, b[:3], b[3:]) / h3, o_reconstruct(Fo, np.abs(co), b[:3], b[3:]) / h3)
            for b in boxes]
    first = None
    for tile in range(1, L.reconstruct_tiles("f16x3") + 1):
        outs = L.reconstruct(F, coef, boxes, 1.0 / h3, "f16x3", tile)
        torch.cuda.synchronize()
        for b, out, (ref, ref_abs) in zip(boxes, outs, refs):
            got = out.double().cpu().numpy()
            rel_mag = np.abs(got - ref).max() / np.abs(ref_abs).max()
            assert rel_mag < gate("f16x3", coef.numel()), (tile, b, rel_mag)
        if tile in (1, 2, 4):
            # the 16x16 tiles that stage f2 from its FP32 copy agree bit for bit
            cat = torch.cat([o.reshape(-1) for o in outs])
            if first is None:
                first = cat.clone()
            else:
                assert torch.equal(cat, first), tile


def test_many_ranks_keep_their_order(L):
    # K > 1024: the given order, no chunk skipped; the result against the
    # oracle's einsum on random factors
    rng = np.random.default_rng(1405)
    K, N = 1100, (20, 36, 70)
    Fh = [rng.standard_normal((K, n)) for n in N]
    ch = rng.standard_normal(K)
    dev = torch.device("cuda:0")
    F = [torch.as_tensor(f, device=dev) for f in Fh]
    coef = torch.as_tensor(ch, device=dev)
    boxes = [(0, 0, 0, N[0], N[1], N[2]), (3, 5, 9, 11, 17, 33)]
    ws = L.reconstruct_prepare(F, coef, "f16x3")
    plan = L.reconstruct_f16_plan(F, coef, boxes, ws)
    nch = (K + 31) // 32
    assert np.array_equal(plan["perm"], np.arange(K))
    assert np.all(plan["masks"] == np.uint32(0xFFFFFFFF))
    assert plan["chunk_values"] == nch * sum(b[3] * b[4] * b[5] for b in boxes)
    outs = L.reconstruct(F, coef, boxes, 1.0, "f16x3", 0, ws)
    torch.cuda.synchronize()
    for b, out in zip(boxes, outs):
        ref = o_reconstruct(Fh, ch, b[:3], b[3:])
        ref_abs = o_reconstruct([np.abs(f) for f in Fh], np.abs(ch), b[:3], b[3:])
        rel_mag = np.abs(out.double().cpu().numpy() - ref).max() / np.abs(ref_abs).max()
        assert rel_mag < gate("f16x3", K), (b, rel_mag)
