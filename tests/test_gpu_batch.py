"""Batched systems in one persistent launch against the FP64 oracle.

Each system's energy (FP64 throughout) and its reconstructed sub-box (FP64,
FP32, split-bf16x3, split-bf16x6 or scaled FP16x3 reconstruction) are compared
with the oracle; graph
replays must be bitwise identical; every tile variant and the autotuned one
must give the same results (FP64 and FP32 tiles sum in the same order: equal
to 1e-12; the split tiles use two MFMA shapes: each within the oracle gate)."""
import numpy as np
import pytest
import torch

from oracle.lattice import Geometry, direct_factors, factor_entries
from oracle.canonical import reconstruct as o_reconstruct, sample_columns
from oracle.physics import energy as o_energy
from oracle.quadrature import rule_s
from workloads import small_box, config4
from _gates import gate

pytestmark = pytest.mark.gpu
dev = torch.device("cuda:0")


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _systems():
    out = []
    specs = [dict(seed=201, n=8, L=(3, 3, 3), M0=2, box="cell"),
             dict(seed=202, n=12, L=(2, 4, 3), M0=3, box="ragged"),
             dict(seed=203, n=6, L=(5, 2, 2), M0=1, box="cell", neutral=False),
             dict(seed=204, n=16, L=(2, 2, 2), M0=4, box="ragged"),
             dict(seed=205, n=10, L=(4, 4, 1), M0=2, box="cell")]
    for sp in specs:
        s = small_box(sp["seed"], n=sp["n"], L=sp["L"], M0=sp["M0"], neutral=sp.get("neutral", True))
        rng = np.random.default_rng(sp["seed"])
        if sp["box"] == "cell":
            o = [(s.L[l] // 2) * s.n for l in range(3)]
            e = [s.n] * 3
        else:
            e = [int(rng.integers(1, s.n + 1)) for _ in range(3)]
            o = [int(rng.integers(0, s.L[l] * s.n - e[l] + 1)) for l in range(3)]
        out.append((s, tuple(o) + tuple(e)))
    return out


def _batch(L, systems, precision):
    items = []
    for s, box in systems:
        q = s.quad
        items.append(dict(lat=L.LatticeSpec(s.b, s.n, s.L, False),
                          quad=L.quadrature("S", q["M"], q["C0"], q["s"]),
                          pos=_t(s.pos), Z=_t(s.Z), D=[_t(x) for x in s.density.D],
                          d=_t(s.density.d), box=box))
    return L.Batch(items, precision)


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x6", "bf16x3", "f16x3"])
def test_batch_against_oracle(precision):
    import paper_1405_2270_amd as L
    systems = _systems()
    B = _batch(L, systems, precision)
    B.run(tile=2)
    sec, err = B.report()
    assert err == 0 and np.all(sec > 0)
    first = [o.double().cpu().numpy().copy() for o in B.out]
    E1 = [float(e.cpu()) for e in B.E]
    refs, Ks = [], []
    for i, (s, box) in enumerate(systems):
        q = s.quad
        t, w = rule_s(q["M"], q["C0"], q["s"])
        geom = Geometry(s.b, s.n, s.L, False)
        Eo = o_energy(geom, t, w, s.pos, s.Z, s.density.D, s.density.d)
        Eabs = o_energy(geom, t, w, s.pos, np.abs(s.Z), s.density.D, s.density.d)
        assert abs(E1[i] - Eo) / abs(Eabs) < 1e-12, (i, E1[i], Eo)
        Fo, co = direct_factors(geom, t, w, s.pos, s.Z)
        ref = o_reconstruct(Fo, co, box[:3], box[3:]) / s.h ** 3
        ref_abs = o_reconstruct(Fo, np.abs(co), box[:3], box[3:]) / s.h ** 3
        refs.append((ref, np.max(np.abs(ref_abs))))
        Ks.append(len(co))
        err_v = np.max(np.abs(first[i] - ref)) / np.max(np.abs(ref_abs))
        print(f"batch {precision} system {i}: rel_mag {err_v:.3e}")
        assert err_v < gate(precision, len(co)), (i, err_v)
    # graph replay: bitwise identical
    B.run(tile=2)
    torch.cuda.synchronize()
    for i in range(len(systems)):
        assert np.array_equal(B.out[i].double().cpu().numpy(), first[i])
        assert float(B.E[i].cpu()) == E1[i]
    # every tile variant and the autotuned one give the same values
    for tile in range(1, L.api.lib().ls_batch_tiles() + 1):
        B.run(tile=tile)
        torch.cuda.synchronize()
        for i in range(len(systems)):
            a = B.out[i].double().cpu().numpy()
            if precision in ("f64", "f32"):
                assert np.max(np.abs(a - first[i])) <= 1e-12 * np.max(np.abs(first[i])) + 1e-300
            else:
                ref, scale = refs[i]
                assert np.max(np.abs(a - ref)) / scale < gate(precision, Ks[i]), (tile, i)
    best, ms = B.autotune()
    assert 1 <= best <= L.api.lib().ls_batch_tiles() and ms > 0
    B.run()
    sec, err = B.report()
    assert err == 0
    B.close()


def test_batch_rejects_bad_systems():
    import paper_1405_2270_amd as L
    from paper_1405_2270_amd._lib import LatsumError
    (s, box), = _systems()[:1]
    bad = (0, 0, 0, s.n + 1, 2, 2)   # extent beyond one unit cell
    with pytest.raises(LatsumError):
        _batch(L, [(s, bad)], "f64")
    # an unknown precision code is refused by the library
    from paper_1405_2270_amd import _lib
    _lib.PRECISIONS["unknown"] = 9
    try:
        with pytest.raises(LatsumError):
            _batch(L, [(s, box)], "unknown")
    finally:
        del _lib.PRECISIONS["unknown"]


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x6", "f16x3"])
def test_config4_smallest_systems_against_oracle(precision):
    # the batched workload's own systems: the six cheapest (oracle cost) in a
    # batch with six mid-size ones; sampled sub-box values and energies
    import paper_1405_2270_amd as L
    systems = config4()
    cost = [s.K * s.N(0) * s.L[0] for s in systems]
    order = np.argsort(cost)
    pick = list(order[:6]) + list(order[200:206])
    chosen = [(systems[i], tuple(int(v) for v in systems[i].boxes[0])) for i in pick]
    B = _batch(L, chosen, precision)
    B.run()
    sec, err = B.report()
    assert err == 0
    rng = np.random.default_rng(9)
    for k, (s, box) in enumerate(chosen[:6]):
        q = s.quad
        t, w = rule_s(q["M"], q["C0"], q["s"])
        geom = Geometry(s.b, s.n, s.L, False)
        Eo = o_energy(geom, t, w, s.pos, s.Z, s.density.D, s.density.d)
        Eabs = o_energy(geom, t, w, s.pos, np.abs(s.Z), s.density.D, s.density.d)
        assert abs(float(B.E[k].cpu()) - Eo) / abs(Eabs) < 1e-12
        sel_local = [np.sort(rng.choice(box[3 + l], 5, replace=False)) for l in range(3)]
        cols = [factor_entries(geom, t, s.pos, l, box[l] + sel_local[l]) for l in range(3)]
        sel = np.array(np.meshgrid(np.arange(5), np.arange(5), np.arange(5), indexing="ij")).reshape(3, -1).T
        coef = (s.Z[:, None] * w[None, :]).ravel()
        ref = np.asarray(sample_columns(cols, coef, sel), np.float64) / s.h ** 3
        ref_abs = np.asarray(sample_columns(cols, np.abs(coef), sel), np.float64) / s.h ** 3
        got = B.out[k][sel_local[0][sel[:, 0]], sel_local[1][sel[:, 1]], sel_local[2][sel[:, 2]]]
        err_v = np.max(np.abs(got.double().cpu().numpy() - ref)) / np.max(np.abs(ref_abs))
        print(f"config4 {precision} system {pick[k]}: rel_mag {err_v:.3e}")
        assert err_v < gate(precision, len(coef))
    B.close()


def test_autotune_cache_by_shape_class(tmp_path):
    # the autotuned tile is cached under the batch's shape class: a second
    # batch of the same shapes (other positions and charges) starts with it,
    # a batch of other shapes does not; the cache file is written and read
    import paper_1405_2270_amd as L
    path = str(tmp_path / "tune.txt")
    L.batch_cache_file(path)
    systems = _systems()
    B = _batch(L, systems, "f32")
    assert B.tuned_tile() == (0, 0.0)
    best, ms = B.autotune()
    assert B.tuned_tile()[0] == best
    B.close()
    moved = []
    for s, box in systems:
        s2 = small_box(s.seed + 1000, n=s.n, L=s.L, M0=s.M0)
        moved.append((s2, box))
    B2 = _batch(L, moved, "f32")
    assert B2.tuned_tile()[0] == best
    B2.run()  # tile 0: the cached one
    sec, err = B2.report()
    assert err == 0
    B2.close()
    B3 = _batch(L, systems[:3], "f32")
    assert B3.tuned_tile() == (0, 0.0)
    B3.close()
    lines = open(path).read().split()
    assert len(lines) == 4 and int(lines[2]) == best
    # a fresh process state: reloaded from the file
    L.batch_cache_file(None)
    B4 = _batch(L, systems, "f32")
    assert B4.tuned_tile() == (0, 0.0)
    B4.close()
    L.batch_cache_file(path)
    B5 = _batch(L, systems, "f32")
    assert B5.tuned_tile()[0] == best
    B5.close()
    L.batch_cache_file(None)
