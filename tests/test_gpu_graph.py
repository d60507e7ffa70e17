"""The device step (kernel vectors -> assembly -> energy -> reconstruction)
captured in a HIP graph and replayed: every replay must reproduce the eager
results bit for bit, with unrelated eager work on the device between replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import small_box


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_2270_amd as lib
    return lib


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision,tile", [("f64", 0), ("f32", 0), ("bf16x6", 0), ("bf16x6", 10), ("bf16x6", 14), ("f16x3", 0)])
def test_graph_replay_matches_eager(L, precision, tile):
    s = small_box(140590, n=32, L=(4, 3, 4), M0=4, nbox=2)
    q = s.quad
    spec = L.LatticeSpec(s.b, s.n, s.L, False)
    qt = L.quadrature(q["rule"], q["M"], q["C0"], q["s"])
    pos, Z = _t(s.pos), _t(s.Z)
    D = [_t(x) for x in s.density.D]
    d = _t(s.density.d)
    boxes = [tuple(int(v) for v in b) for b in s.boxes]
    boxes.append((0, 0, 0, s.N(0), min(s.N(1), 256), s.N(2)))
    nv = sum(b[3] * b[4] * b[5] for b in boxes)
    dt = torch.float64 if precision == "f64" else torch.float32
    K = s.K
    ews = torch.empty(L.api.lib().ls_energy_workspace(K, 8), dtype=torch.uint8, device="cuda")
    rws = torch.empty(3 * ((K + 31) // 32) * s.N(1) * 64, dtype=torch.uint8, device="cuda")
    out = torch.empty(nv, dtype=dt, device="cuda")

    def step():
        m = L.kernel_vectors(spec, qt, pos)
        F, coef = L.assemble(spec, qt, pos, Z, m)
        E = L.energy(F, coef, D, d, "f64", ews)
        L.reconstruct_into(F, coef, boxes, out, 1.0, precision, tile, rws)
        return F, coef, E

    F, coef, E = step()
    torch.cuda.synchronize()
    ref_out, ref_E = out.clone(), E.clone()
    ref_F = [f.clone() for f in F]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gF, gc, gE = step()

    other = small_box(140591, n=16, L=(3, 3, 3), M0=2, nbox=1)
    for rep in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out), (precision, rep)
        assert torch.equal(gE, ref_E), (precision, rep)
        for a, b in zip(gF, ref_F):
            assert torch.equal(a, b), (precision, rep)
        # unrelated eager work between replays
        so = other.quad
        sp = L.LatticeSpec(other.b, other.n, other.L, False)
        qo = L.quadrature(so["rule"], so["M"], so["C0"], so["s"])
        Fo, co = L.assemble(sp, qo, _t(other.pos), _t(other.Z))
        L.reconstruct(Fo, co, [tuple(int(v) for v in other.boxes[0])], 1.0, precision)
        torch.cuda.synchronize()
