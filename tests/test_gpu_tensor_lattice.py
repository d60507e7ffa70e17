"""Non-equidistant tensor lattices (Sec. 3.1, remark after eq.
EwaldTensorM0) through the C ABI against the oracle: value and derivative
factors (row-wise 1e-12), reconstruction (FP64 1e-12, FP16x3 1e-6 rel_mag),
energy (1e-12), the equidistant case against the box assembly, and the
full-size non-equidistant workload at sampled columns and points."""
import numpy as np
import pytest
import torch

from oracle.lattice import (Geometry, TensorLattice, direct_factors, tensor_lattice_factors,
                            tensor_lattice_entries)
from oracle.canonical import reconstruct as o_reconstruct, sample_columns, scalar_product
from oracle.quadrature import rule_s
from workloads import small_tensor, small_box, config_tensor, make_density

pytestmark = pytest.mark.gpu
dev = torch.device("cuda:0")


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _rows_close(a, b, rtol, rowscale=None):
    rowmax = np.max(np.abs(b), axis=1) if rowscale is None else np.asarray(rowscale)
    scale = np.maximum(rowmax, 1e-12 * np.max(rowmax))
    err = np.max(np.abs(a - b), axis=1)
    if np.any(err > rtol * scale):
        r = int(np.argmax(err / scale))
        print(f"worst row {r}: err/scale {err[r] / scale[r]:.3e}")
        return False
    return True


def _specs(L, sysm):
    q = sysm.quad
    t, w = rule_s(q["M"], q["C0"], q["s"])
    qt = L.quadrature("S", q["M"], q["C0"], q["s"])
    s = sysm.extra["s"]
    tl = L.TensorLatticeSpec(sysm.b, sysm.n, sysm.extra["N"], [_t(x) for x in s])
    otl = TensorLattice(sysm.b, sysm.n, sysm.extra["N"], s)
    return t, w, qt, tl, otl


def _coincident():
    s = small_tensor(405, n=10, L=(1, 3, 2), M0=2)
    n = s.n
    s.extra["s"] = (np.array([0.0]), np.array([0.0, 0.0, 25.5]), np.array([3.25, 19.0]))
    s.extra["N"] = (n, int(np.ceil(25.5)) + n, 19 + n)
    s.density = make_density(s.b, n, s.L, False, np.random.default_rng(405), N=s.extra["N"])
    return s


CASES = [
    ("offgrid", lambda: small_tensor(401, n=12, L=(3, 2, 4), M0=3)),
    ("ongrid", lambda: small_tensor(402, n=10, L=(4, 3, 2), M0=2, on_grid=True)),
    ("single_and_repeated", _coincident),
    ("wide_jitter", lambda: small_tensor(403, n=8, L=(5, 1, 3), M0=4, jitter=0.45)),
]


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
def test_tensor_lattice_against_oracle(name, maker):
    import paper_1405_2270_amd as L
    sysm = maker()
    t, w, qt, tl, otl = _specs(L, sysm)
    pos, Z = _t(sysm.pos), _t(sysm.Z)
    F, coef = L.assemble_tensor(tl, qt, pos, Z)
    dF, _ = L.assemble_tensor(tl, qt, pos, None, derivative=True)
    torch.cuda.synchronize()
    Fo, co = tensor_lattice_factors(otl, t, w, sysm.pos, sysm.Z)
    dFo, _ = tensor_lattice_factors(otl, t, w, sysm.pos, sysm.Z, derivative=True)
    assert np.allclose(coef.cpu().numpy(), co, rtol=1e-15, atol=0)
    for l in range(3):
        assert _rows_close(F[l].cpu().numpy(), Fo[l], 1e-12), (name, "value", l)
        assert _rows_close(dF[l].cpu().numpy(), dFo[l], 1e-12), (name, "derivative", l)
    h3 = sysm.h ** 3
    full = (0, 0, 0) + tuple(sysm.extra["N"])
    ref = o_reconstruct(Fo, co) / h3
    ref_abs = np.max(np.abs(o_reconstruct(Fo, np.abs(co)))) / h3
    for precision, gate in (("f64", 1e-12), ("f16x3", 1e-6), ("f32", 1e-6)):
        V = L.reconstruct(F, coef, [full], 1.0 / h3, precision)[0]
        err = np.max(np.abs(V.double().cpu().numpy() - ref)) / ref_abs
        assert err < gate, (name, precision, err)
    D = [_t(x) for x in sysm.density.D]
    E = float(L.energy(F, coef, D, _t(sysm.density.d), "f64").cpu())
    Eo = scalar_product(Fo, co, sysm.density.D, sysm.density.d)
    Eabs = scalar_product(Fo, np.abs(co), sysm.density.D, sysm.density.d)
    assert abs(E - Eo) / abs(Eabs) < 1e-12, (name, E, Eo)


def test_equidistant_coordinates_match_box_assembly():
    import paper_1405_2270_amd as L
    sysm = small_box(406, n=12, L=(3, 2, 4), M0=3)
    q = sysm.quad
    qt = L.quadrature("S", q["M"], q["C0"], q["s"])
    spec = L.LatticeSpec(sysm.b, sysm.n, sysm.L, False)
    pos, Z = _t(sysm.pos), _t(sysm.Z)
    Fb, cb = L.assemble(spec, qt, pos, Z, L.kernel_vectors(spec, qt, pos))
    s = [_t(float(sysm.n) * np.arange(sysm.L[l])) for l in range(3)]
    tl = L.TensorLatticeSpec(sysm.b, sysm.n, tuple(sysm.N(l) for l in range(3)), s)
    Ft, ct = L.assemble_tensor(tl, qt, pos, Z)
    torch.cuda.synchronize()
    assert torch.equal(cb, ct)
    t, w = rule_s(q["M"], q["C0"], q["s"])
    Fo, _ = direct_factors(Geometry(sysm.b, sysm.n, sysm.L), t, w, sysm.pos, sysm.Z)
    for l in range(3):
        assert _rows_close(Ft[l].cpu().numpy(), Fb[l].cpu().numpy(), 1e-12), l
        assert _rows_close(Ft[l].cpu().numpy(), Fo[l], 1e-12), l


def test_invalid_tensor_lattice_raises():
    import paper_1405_2270_amd as L
    from paper_1405_2270_amd._lib import LatsumError
    sysm = small_tensor(407, n=8, L=(2, 2, 2), M0=1)
    t, w, qt, tl, otl = _specs(L, sysm)
    bad = L.TensorLatticeSpec(sysm.b, sysm.n, (0, 8, 8), tl.s)
    with pytest.raises(LatsumError):
        L.assemble_tensor(bad, qt, _t(sysm.pos), _t(sysm.Z))


@pytest.mark.slow
def test_config_tensor_sampled():
    # non-equidistant workload at full size: sampled factor columns and
    # potential values at sampled points of two 256^3 boxes
    import paper_1405_2270_amd as L
    sysm = config_tensor()
    t, w, qt, tl, otl = _specs(L, sysm)
    F, coef = L.assemble_tensor(tl, qt, _t(sysm.pos), _t(sysm.Z))
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    h3 = sysm.h ** 3
    coef_o = (sysm.Z[:, None] * w[None, :]).ravel()
    for b in [tuple(int(v) for v in x) for x in sysm.boxes[:2]]:
        sel_local = [np.sort(rng.choice(b[3 + l], 6, replace=False)) for l in range(3)]
        cols = [tensor_lattice_entries(otl, t, sysm.pos, l, b[l] + sel_local[l]) for l in range(3)]
        for l in range(3):
            got = F[l][:, b[l] + sel_local[l]].cpu().numpy()
            assert _rows_close(got, cols[l], 1e-12, F[l].abs().max(dim=1).values.cpu().numpy())
        sel = np.array(np.meshgrid(np.arange(6), np.arange(6), np.arange(6),
                                   indexing="ij")).reshape(3, -1).T
        ref = np.asarray(sample_columns(cols, coef_o, sel), np.float64) / h3
        ref_abs = np.asarray(sample_columns(cols, np.abs(coef_o), sel), np.float64) / h3
        for precision, gate in (("f64", 1e-12), ("f16x3", 1e-6)):
            V = L.reconstruct(F, coef, [b], 1.0 / h3, precision)[0]
            got = V[sel_local[0][sel[:, 0]], sel_local[1][sel[:, 1]], sel_local[2][sel[:, 2]]]
            err = np.max(np.abs(got.double().cpu().numpy() - ref)) / np.max(np.abs(ref_abs))
            print(f"config_tensor box {b[:3]} {precision}: rel_mag {err:.3e}")
            assert err < gate, (precision, err)
            del V
            torch.cuda.empty_cache()
