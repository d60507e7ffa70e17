"""Split-precision reconstruction kernels at full size (lattice of the 4096^3
grid, K = 384, 256^3 boxes).

BF16x6: the per-tile kernels (16x16 shape: tiles 10 and 12; 32x32 shape: 11
and 13) and the persistent stream kernels (14 and 16 with the 16x16 shape, 15
with the 32x32 one) issue the same MFMAs in the same order for every output
element, so within a shape their results must agree bit for bit. FP16x3: the
stream kernel with 128-column tiles (1), with 64-column tiles (2) and with
every wave loading the rank factors (4) must agree bit for bit, and so must
the 32x32 kernels with 64- and 128-column tiles (3, 8) and the two 16x16
kernels that read f2 in FP64 (5, 7). The boxes cover both store
paths of the stream kernel (tiles inside the box, unmasked; tiles cut by the
box edge in rows or columns, masked; columns cut inside a 128-column tile),
box offsets that are not a multiple of 4 and rows that are not 16-byte
aligned, and several boxes per launch, so that a workgroup's stream crosses
from one box to the next. The stream kernels (BF16x6, and FP16x3 with both
MFMA shapes, both tile widths and both f2 sources) are also checked against
the oracle at sampled points of a 256^3 box and of a box with a cut column
tile."""
import numpy as np
import pytest
import torch

from oracle.lattice import Geometry, factor_entries
from oracle.canonical import sample_columns
from oracle.quadrature import rule_s
from workloads import config2
from _gates import gate

pytestmark = pytest.mark.gpu

dev = torch.device("cuda:0")


@pytest.fixture(scope="module")
def setup():
    import paper_1405_2270_amd as L
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    s = config2()
    q = s.quad
    qt = L.quadrature("S", q["M"], q["C0"], q["s"])
    spec = L.LatticeSpec(s.b, s.n, tuple(s.L), False)
    pos = torch.as_tensor(s.pos, dtype=torch.float64, device=dev)
    Z = torch.as_tensor(s.Z, dtype=torch.float64, device=dev)
    F, coef = L.assemble(spec, qt, pos, Z, L.kernel_vectors(spec, qt, pos))
    torch.cuda.synchronize()
    return L, s, F, coef


def _boxes(s):
    o = [int(v) for v in s.boxes[0][:3]]
    return [
        (*o, 256, 256, 256),  # tiles inside the box
        (*o, 2, 256, 132),    # last column tile cut at 132
        (*o, 1, 255, 3),      # rows and columns cut; 765 values, so the next offsets are odd
        (*o, 2, 256, 128),    # whole tiles at an odd offset
        (*o, 3, 256, 130),    # e2 = 130: rows not 16-byte aligned
    ]


@pytest.mark.parametrize("precision,ref_tile,tiles", [("bf16x6", 10, (12, 14, 16)), ("bf16x6", 11, (13, 15)),
                                                       ("f16x3", 1, (2, 4)), ("f16x3", 3, (8,)),
                                                       ("f16x3", 5, (7,))])
def test_tiles_agree_bitwise(setup, precision, ref_tile, tiles):
    L, s, F, coef = setup
    boxes = _boxes(s)
    scale = 1.0 / (s.b / (s.n)) ** 3
    ref = L.reconstruct(F, coef, boxes, scale, precision, ref_tile)
    torch.cuda.synchronize()
    for tile in tiles:
        got = L.reconstruct(F, coef, boxes, scale, precision, tile)
        torch.cuda.synchronize()
        for b, (x, y) in enumerate(zip(got, ref)):
            assert x.shape == y.shape
            same = torch.equal(x, y)
            if not same:
                d = (x - y).abs()
                print("tile", tile, "box", boxes[b], "max diff", float(d.max()),
                      "at", np.unravel_index(int(d.argmax()), tuple(x.shape)))
            assert same, (precision, tile, boxes[b])
        del got


@pytest.mark.parametrize("precision,tile", [("bf16x6", 14), ("f16x3", 1), ("f16x3", 2), ("f16x3", 3),
                                            ("f16x3", 5), ("f16x3", 6), ("f16x3", 8)])
def test_stream_matches_oracle_sampled(setup, precision, tile):
    L, s, F, coef = setup
    q = s.quad
    t, w = rule_s(q["M"], q["C0"], q["s"])
    geom = Geometry(s.b, s.n, tuple(s.L), False)
    h3 = (s.b / s.n) ** 3
    rng = np.random.default_rng(11)
    boxes = _boxes(s)
    outs = L.reconstruct(F, coef, boxes, 1.0 / h3, precision, tile)
    coef_o = (s.Z[:, None] * w[None, :]).ravel()
    for b, V in zip(boxes[:2], outs[:2]):
        sel_local = [np.sort(rng.choice(b[3 + l], min(5, b[3 + l]), replace=False)) for l in range(3)]
        cols = [factor_entries(geom, t, s.pos, l, b[l] + sel_local[l]) for l in range(3)]
        n0, n1, n2 = (len(x) for x in sel_local)
        sel = np.array(np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")).reshape(3, -1).T
        ref = np.asarray(sample_columns(cols, coef_o, sel), np.float64) / h3
        ref_abs = np.asarray(sample_columns(cols, np.abs(coef_o), sel), np.float64) / h3
        got = V[sel_local[0][sel[:, 0]], sel_local[1][sel[:, 1]], sel_local[2][sel[:, 2]]]
        err = np.max(np.abs(got.double().cpu().numpy() - ref))
        assert err / np.max(np.abs(ref_abs)) < 1e-6, (precision, tile, b, err)


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x6", "f16x3"])
def test_autotune_choice_is_kept_per_shape_class(setup, precision):
    # ls_reconstruct_autotune times every tile on the call and caches the
    # fastest under the call's shape class; tile 0 then runs it (bit for bit
    # the explicit tile), other extents stay untuned, offsets do not matter
    L, s, F, coef = setup
    boxes = _boxes(s)[1:]
    scale = 1.0 / (s.b / s.n) ** 3
    dtype = torch.float64 if precision == "f64" else torch.float32
    n = sum(b[3] * b[4] * b[5] for b in boxes)
    assert L.reconstruct_tuned_tile(F, coef, boxes, precision) == (0, 0.0)
    out = torch.full((n,), float("nan"), dtype=dtype, device=dev)
    tile, ms = L.reconstruct_autotune(F, coef, boxes, out, scale, precision, reps=2)
    torch.cuda.synchronize()
    print(f"autotune {precision}: tile {tile}, {ms:.4f} ms")
    assert 1 <= tile <= L.reconstruct_tiles(precision) and ms > 0
    t2, ms2 = L.reconstruct_tuned_tile(F, coef, boxes, precision)
    assert t2 == tile and abs(ms2 - ms) <= 1e-6 * ms
    a = L.reconstruct(F, coef, boxes, scale, precision, 0)
    b = L.reconstruct(F, coef, boxes, scale, precision, tile)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b))
    # the autotuner's output is the reconstruction (the last tile it ran),
    # within the precision's gate (rel_mag against the FP64 path)
    ref = torch.cat([x.reshape(-1) for x in L.reconstruct(F, coef, boxes, scale, "f64")])
    mag = torch.cat([x.reshape(-1) for x in L.reconstruct(F, coef.abs(), boxes, scale, "f64")])
    err = float((out.double() - ref).abs().max() / mag.abs().max())
    assert err < gate(precision, coef.numel()), err
    other = [b[:5] + (b[5] - 1,) for b in boxes]
    assert L.reconstruct_tuned_tile(F, coef, other, precision)[0] == 0
    moved = [(b[0] + 1,) + b[1:] for b in boxes]
    assert L.reconstruct_tuned_tile(F, coef, moved, precision)[0] == tile
