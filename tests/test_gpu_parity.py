"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Error measures (both stated for every potential/energy check):
  rel_inf = max|x - x_o| / max|x_o|
  rel_mag = max|x - x_o| / max|x_o^{|Z|}|, the oracle rerun with |Z_nu|, which
            is the scale rounding errors follow when charges cancel.
Gates: FP64 path 1e-12 (rel_mag, and rel_inf where charges do not cancel;
factor and master rows 1e-12 of each row's maximum; forces normwise),
mixed FP32 / split-bf16x6 / scaled FP16x3 1e-6 (rel_mag), split-bf16x3 its
own arithmetic bound (about 5e-5: it does not meet 1e-6, see _gates.py),
forces 1e-5 normwise for the FP32 Grams.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle.lattice import Geometry, direct_factors, master_vectors, node_and_offset, factor_entries
from oracle.canonical import reconstruct as o_reconstruct, sample_columns
from oracle.physics import energy as o_energy, forces_adjoint, forces_adjoint_atoms
from oracle.quadrature import rule_u, rule_s
from workloads import small_box, small_periodic, config1, config2, config3, config5

pytestmark = pytest.mark.gpu

dev = torch.device("cuda:0")


@pytest.fixture(scope="module")
def L():
    import paper_1405_2270_amd as lib
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return lib


def _quads(sysm, L):
    q = sysm.quad
    if q["rule"] == "U":
        t, w = rule_u(q["M"], q["C0"])
        qt = L.quadrature("U", q["M"], q["C0"])
    else:
        t, w = rule_s(q["M"], q["C0"], q["s"])
        qt = L.quadrature("S", q["M"], q["C0"], q["s"])
    return t, w, qt


def _spec(sysm, L):
    return L.LatticeSpec(sysm.b, sysm.n, tuple(sysm.L), sysm.periodic)


def _geom(sysm):
    return Geometry(sysm.b, sysm.n, tuple(sysm.L), sysm.periodic)


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _gpu_factors(L, sysm, qt, fused=False):
    spec = _spec(sysm, L)
    pos, Z = _t(sysm.pos), _t(sysm.Z)
    masters = None if (fused or sysm.periodic) else L.kernel_vectors(spec, qt, pos)
    F, coef = L.assemble(spec, qt, pos, Z, masters)
    torch.cuda.synchronize()
    return F, coef


def _close_rows(a, b, rtol, rowscale=None):
    """Row-wise normwise agreement: max_j |a_rj - b_rj| <= rtol * scale_r with
    scale_r = max(max_j |b_rj|, 1e-12 * max |b|), where max_j runs over the
    whole vector when only some of its entries are compared (``rowscale``:
    the vector maxima). Elementwise relative checks
    would be limited by input conditioning: in a Gaussian tail exp(-u^2)
    turns the rounding of the cell offset (~eps * n cells, from the position
    given in FP64) into a relative error of 2u * du on either side."""
    rowmax = np.max(np.abs(b), axis=1) if rowscale is None else np.asarray(rowscale)
    scale = np.maximum(rowmax, 1e-12 * np.max(rowmax))
    err = np.max(np.abs(a - b), axis=1)
    bad = err > rtol * scale
    if np.any(bad):
        r = int(np.argmax(err / scale))
        j = int(np.argmax(np.abs(a[r] - b[r])))
        print(f"worst: row {r} col {j}: {a[r, j]!r} vs {b[r, j]!r} "
              f"(err/scale {err[r] / scale[r]:.3e}, row max {rowmax[r]:.3e})")
        return False
    return True


SMALL = [
    ("box_offgrid", lambda: small_box(101, n=12, L=(3, 2, 4), M0=3)),
    ("box_ongrid_U", lambda: small_box(102, n=10, L=(2, 3, 2), M0=2, rule="U", M=12, on_grid=True)),
    ("box_single", lambda: small_box(103, n=9, L=(1, 1, 1), M0=1, neutral=False)),
    ("box_L17", lambda: small_box(104, n=6, L=(17, 3, 9), M0=2)),
    ("periodic_odd", lambda: small_periodic(105, n=12, L=(5, 5, 3), M0=4)),
    ("periodic_even", lambda: small_periodic(106, n=10, L=(4, 6, 2), M0=3)),
]


@pytest.mark.parametrize("name,maker", SMALL, ids=[s[0] for s in SMALL])
def test_quadrature_and_masters(L, name, maker):
    sysm = maker()
    t, w, qt = _quads(sysm, L)
    assert np.allclose(qt.t, t, rtol=1e-15, atol=0) and np.allclose(qt.w, w, rtol=1e-15, atol=0)
    if sysm.periodic:
        return
    spec = _spec(sysm, L)
    geom = _geom(sysm)
    X = L.master_halfwidth(spec)
    for deriv in (False, True):
        m = L.kernel_vectors(spec, qt, _t(sysm.pos), derivative=deriv).cpu().numpy()
        for nu in range(sysm.M0):
            for l in range(3):
                _, d = node_and_offset(geom, sysm.pos[nu, l])
                ref = master_vectors(geom, t, d, X, derivative=deriv)
                assert _close_rows(m[nu * 3 + l], ref, 1e-12), (name, deriv, nu, l)


# the periodic cell has no stored-masters path (its cells are generated in
# registers), so only the fused assembly applies there
ASM_CASES = [(name, maker, fused) for name, maker in SMALL for fused in (False, True)
             if fused or not name.startswith("periodic")]


@pytest.mark.parametrize("name,maker,fused", ASM_CASES,
                         ids=[f"{c[0]}-{'fused' if c[2] else 'masters'}" for c in ASM_CASES])
def test_assembled_factors(L, name, maker, fused):
    sysm = maker()
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt, fused)
    Fo, co = direct_factors(_geom(sysm), t, w, sysm.pos, sysm.Z)
    for l in range(3):
        assert _close_rows(F[l].cpu().numpy(), Fo[l], 1e-12), (name, l)
    assert np.allclose(coef.cpu().numpy(), co, rtol=1e-15, atol=0)


@pytest.mark.parametrize("name,maker", SMALL, ids=[s[0] for s in SMALL])
def test_derivative_factors(L, name, maker):
    sysm = maker()
    t, w, qt = _quads(sysm, L)
    spec = _spec(sysm, L)
    pos = _t(sysm.pos)
    Fo, _ = direct_factors(_geom(sysm), t, w, sysm.pos, sysm.Z, derivative=True)
    variants = [None] if sysm.periodic else [None, L.kernel_vectors(spec, qt, pos, derivative=True)]
    for masters in variants:
        F, _ = L.assemble(spec, qt, pos, None, masters, derivative=True)
        for l in range(3):
            a, b = F[l].cpu().numpy(), Fo[l]
            assert _close_rows(a, b, 1e-12), (name, l)


# box lattices whose widest axis selects each instantiation of the stored-
# masters assembly: up to 8, 16, 32 and 64 images per residue window, and the
# direct kernel beyond 64 (Theorem 3.1, eq. EwaldTensorM0)
WIDTHS = [
    ("L12", lambda: small_box(121, n=5, L=(12, 2, 3), M0=2)),
    ("L40", lambda: small_box(122, n=4, L=(2, 40, 2), M0=2)),
    ("L64", lambda: small_box(123, n=3, L=(3, 2, 64), M0=2)),
    ("L70", lambda: small_box(124, n=3, L=(70, 2, 3), M0=2)),
]


@pytest.mark.parametrize("name,maker", WIDTHS, ids=[s[0] for s in WIDTHS])
@pytest.mark.parametrize("deriv", [False, True], ids=["value", "derivative"])
def test_assembly_lattice_widths(L, name, maker, deriv):
    sysm = maker()
    t, w, qt = _quads(sysm, L)
    spec = _spec(sysm, L)
    pos = _t(sysm.pos)
    Fo, co = direct_factors(_geom(sysm), t, w, sysm.pos, sysm.Z, derivative=deriv)
    masters = L.kernel_vectors(spec, qt, pos, derivative=deriv)
    F, coef = L.assemble(spec, qt, pos, None if deriv else _t(sysm.Z), masters, derivative=deriv)
    torch.cuda.synchronize()
    for l in range(3):
        assert _close_rows(F[l].cpu().numpy(), Fo[l], 1e-12), (name, deriv, l)
    if not deriv:
        assert np.allclose(coef.cpu().numpy(), co, rtol=1e-15, atol=0)
        h3 = sysm.h ** 3
        full = (0, 0, 0, F[0].shape[1], F[1].shape[1], F[2].shape[1])
        V = L.reconstruct(F, coef, [full], 1.0 / h3, "f64")[0].cpu().numpy()
        ref = o_reconstruct(Fo, co) / h3
        ref_abs = o_reconstruct(Fo, np.abs(co)) / h3
        assert _errors(V, ref, ref_abs)[1] < 1e-12, name


def _errors(got, ref, ref_abs):
    err = np.max(np.abs(got - ref))
    return err / np.max(np.abs(ref)), err / np.max(np.abs(ref_abs))


from _gates import gate as _gate  # noqa: E402


@pytest.mark.parametrize("name,maker", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x6", "bf16x3", "f16x3"])
def test_reconstruct(L, name, maker, precision):
    sysm = maker()
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    Fo, co = direct_factors(_geom(sysm), t, w, sysm.pos, sysm.Z)
    h3 = sysm.h ** 3
    boxes = [tuple(b) for b in sysm.boxes]
    full = (0, 0, 0, F[0].shape[1], F[1].shape[1], F[2].shape[1])
    boxes.append(full)
    tiles = [0] + list(range(1, L.reconstruct_tiles(precision) + 1))
    for tile in tiles:
        outs = L.reconstruct(F, coef, boxes, 1.0 / h3, precision, tile)
        torch.cuda.synchronize()
        for b, out in zip(boxes, outs):
            ref = o_reconstruct(Fo, co, b[:3], b[3:]) / h3
            ref_abs = o_reconstruct(Fo, np.abs(co), b[:3], b[3:]) / h3
            rel_inf, rel_mag = _errors(out.double().cpu().numpy(), ref, ref_abs)
            assert rel_mag < _gate(precision, coef.numel()), (name, precision, tile, b, rel_inf, rel_mag)
            if precision == "f64" and np.all(sysm.Z > 0):
                assert rel_inf < 1e-12


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x6", "bf16x3", "f16x3"])
def test_reconstruct_tiles_over_several_i(L, precision):
    # boxes whose 43 or more values of j put a 128-row tile's rows in up to
    # four values of i (the tiles' per-i rank factors), one with 42 (five
    # values: each element loads its own f0), and the whole grid, every tile
    # id against the oracle (Appendix, eq. CP_form)
    sysm = small_box(141, n=12, L=(3, 5, 2), M0=3)
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    Fo, co = direct_factors(_geom(sysm), t, w, sysm.pos, sysm.Z)
    h3 = sysm.h ** 3
    N = [f.shape[1] for f in F]
    boxes = [(0, 0, 0, N[0], N[1], N[2]), (2, 7, 3, 5, 43, 20), (0, 3, 0, 3, 42, N[2]), (1, 1, 1, 4, 59, 7)]
    for tile in range(L.reconstruct_tiles(precision) + 1):
        outs = L.reconstruct(F, coef, boxes, 1.0 / h3, precision, tile)
        torch.cuda.synchronize()
        for b, out in zip(boxes, outs):
            ref = o_reconstruct(Fo, co, b[:3], b[3:]) / h3
            ref_abs = o_reconstruct(Fo, np.abs(co), b[:3], b[3:]) / h3
            rel_inf, rel_mag = _errors(out.double().cpu().numpy(), ref, ref_abs)
            assert rel_mag < _gate(precision, coef.numel()), (precision, tile, b, rel_inf, rel_mag)


@pytest.mark.parametrize("precision", ["f64", "bf16x6", "bf16x3", "f16x3"])
def test_prepared_matches_reconstruct(L, precision):
    # the preparation as a call of its own (on another stream, joined by an
    # event), then two prepared calls on different boxes: bit for bit the
    # results of ls_reconstruct, every tile of the precision
    sysm = small_box(131, n=12, L=(5, 4, 6), M0=3)
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    N = [f.shape[1] for f in F]
    boxes_a = [(0, 0, 0, N[0], N[1], N[2]), (3, 5, 7, 20, 30, 41)]
    boxes_b = [(1, 2, 3, 17, 9, 65)]
    for tile in range(L.reconstruct_tiles(precision) + 1):
        refs = [L.reconstruct(F, coef, bx, 1.0, precision, tile) for bx in (boxes_a, boxes_b)]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ws = L.reconstruct_prepare(F, coef, precision)
        torch.cuda.current_stream().wait_stream(side)
        for bx, ref in zip((boxes_a, boxes_b), refs):
            n = sum(b[3] * b[4] * b[5] for b in bx)
            out = torch.empty(n, dtype=ref[0].dtype, device=dev)
            L.reconstruct_into(F, coef, bx, out, 1.0, precision, tile, ws, prepared=True)
            torch.cuda.synchronize()
            assert torch.equal(out, torch.cat([r.reshape(-1) for r in ref])), (precision, tile, bx)


@pytest.mark.parametrize("name,maker", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_energy(L, name, maker, precision):
    sysm = maker()
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    D = [_t(x) for x in sysm.density.D]
    d = _t(sysm.density.d)
    E = float(L.energy(F, coef, D, d, precision).cpu())
    geom = _geom(sysm)
    Eo = o_energy(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d)
    Eabs = o_energy(geom, t, w, sysm.pos, np.abs(sysm.Z), sysm.density.D, sysm.density.d)
    gate = 1e-12 if precision == "f64" else 1e-6
    assert abs(E - Eo) / abs(Eabs) < gate, (name, E, Eo, Eabs)


@pytest.mark.parametrize("name,maker", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_forces_and_energy_by_adjoint(L, name, maker, precision):
    sysm = maker()
    t, w, qt = _quads(sysm, L)
    spec = _spec(sysm, L)
    D = [_t(x) for x in sysm.density.D]
    d = _t(sysm.density.d)
    Fg, Eg = L.forces(spec, qt, _t(sysm.pos), _t(sysm.Z), D, d, precision)
    geom = _geom(sysm)
    Fo = forces_adjoint(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d)
    Eo = o_energy(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d)
    Eabs = o_energy(geom, t, w, sysm.pos, np.abs(sysm.Z), sysm.density.D, sysm.density.d)
    gate = 1e-12 if precision == "f64" else 1e-5
    err = np.max(np.abs(Fg.cpu().numpy() - Fo)) / np.max(np.abs(Fo))
    assert err < gate, (name, precision, err)
    assert abs(float(Eg.cpu()) - Eo) / abs(Eabs) < (1e-12 if precision == "f64" else 1e-6)


def test_autograd_matches_finite_differences(L):
    sysm = small_box(111, n=10, L=(3, 3, 3), M0=3)
    t, w, qt = _quads(sysm, L)
    spec = _spec(sysm, L)
    D = [_t(x) for x in sysm.density.D]
    d = _t(sysm.density.d)
    pos = _t(sysm.pos).requires_grad_(True)
    E = L.lattice_energy(pos, _t(sysm.Z), D, d, spec, qt, "f64")
    E.backward()
    g = pos.grad.cpu().numpy()
    step = 1e-4 * sysm.b
    fd = np.zeros_like(g)
    for nu in range(sysm.M0):
        for l in range(3):
            pp, pm = sysm.pos.copy(), sysm.pos.copy()
            pp[nu, l] += step
            pm[nu, l] -= step
            Ep = float(L.forces(spec, qt, _t(pp), _t(sysm.Z), D, d, "f64")[1].cpu())
            Em = float(L.forces(spec, qt, _t(pm), _t(sysm.Z), D, d, "f64")[1].cpu())
            fd[nu, l] = (Ep - Em) / (2 * step)
    assert np.max(np.abs(g - fd)) < 1e-6 * np.max(np.abs(fd))


def test_reproducible_bitwise(L):
    sysm = small_box(121, n=12, L=(4, 4, 4), M0=4)
    t, w, qt = _quads(sysm, L)
    outs = []
    for _ in range(2):
        F, coef = _gpu_factors(L, sysm, qt)
        V = L.reconstruct(F, coef, [(0, 0, 0, 48, 48, 48)], 1.0, "f64")[0]
        E = L.energy(F, coef, [_t(x) for x in sysm.density.D], _t(sysm.density.d), "f64")
        outs.append((F[0].cpu().numpy(), V.cpu().numpy(), float(E.cpu())))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_invalid_arguments_raise(L):
    from paper_1405_2270_amd._lib import LatsumError
    sysm = small_box(131, n=8, L=(2, 2, 2), M0=2)
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    with pytest.raises(LatsumError):
        L.reconstruct(F, coef, [(0, 0, 10, 8, 8, 8)], 1.0, "f64")   # outside the factors
    with pytest.raises(LatsumError):
        L.reconstruct(F, coef, [(0, 0, 0, 0, 8, 8)], 1.0, "f64")    # empty extent
    with pytest.raises(LatsumError):
        L.reconstruct(F, coef, [(0, 0, 0, 4, 4, 4)], 1.0, "f64", tile=99)
    with pytest.raises(LatsumError):
        L.energy(F, coef, [_t(x) for x in sysm.density.D], _t(sysm.density.d), "bf16x3")
    bad = L.LatticeSpec(sysm.b, 0, (2, 2, 2))
    with pytest.raises(LatsumError):
        L.kernel_vectors(bad, qt, _t(sysm.pos))
    # the periodic cell generates every cell integral in registers: the library
    # refuses stored masters for it (a buffer of the right size, so that the
    # binding's own size check passes and the refusal is the library's)
    per = L.LatticeSpec(sysm.b, 8, (2, 2, 2), True)
    nm = sysm.pos.shape[0] * 3 * qt.R * 2 * L.master_halfwidth(per)
    with pytest.raises(LatsumError):
        L.assemble(per, qt, _t(sysm.pos), _t(sysm.Z),
                   torch.zeros(nm, dtype=torch.float64, device=dev))
    # the preparation as a call of its own: a short workspace, and an unknown
    # precision code, are refused before any launch; FP64 needs none
    from paper_1405_2270_amd import _lib
    lib = L.api.lib()
    canon = L.api._canon(F, coef)
    short = torch.empty(16, dtype=torch.uint8, device=dev)
    assert lib.ls_reconstruct_prepare(ctypes.byref(canon), _lib.PRECISIONS["f16x3"],
                                      ctypes.c_void_p(short.data_ptr()), 16, None) == -4
    assert lib.ls_reconstruct_prepare(ctypes.byref(canon), 9, None, 0, None) == -1
    assert lib.ls_reconstruct_prepare(ctypes.byref(canon), _lib.PRECISIONS["f64"], None, 0, None) == 0
    with pytest.raises(ValueError):
        L.reconstruct_into(F, coef, [(0, 0, 0, 4, 4, 4)], torch.empty(64, device=dev), 1.0,
                           "f16x3", 0, short, prepared=True)


def test_positions_outside_the_cell_stay_exact(L):
    # a charge at the upper cell edge or slightly outside: the node index is
    # clamped, the geometry is not
    b, n = 10.0, 8
    pos = np.array([[0.5 * b, -0.5 * b, 0.3], [0.5 * b + 0.7, 0.1, -0.5 * b - 0.2]])
    Z = np.array([1.0, -1.0])
    t, w = rule_s(29, 3.4, 2.45e-3 * n / b)
    qt = L.quadrature("S", 29, 3.4, 2.45e-3 * n / b)
    spec = L.LatticeSpec(b, n, (3, 3, 3))
    F, coef = L.assemble(spec, qt, _t(pos), _t(Z), L.kernel_vectors(spec, qt, _t(pos)))
    Fo, _ = direct_factors(Geometry(b, n, (3, 3, 3)), t, w, pos, Z)
    for l in range(3):
        assert _close_rows(F[l].cpu().numpy(), Fo[l], 1e-12)


def test_config1_full_potential(L):
    # small benchmark case: full 128^3 potential of 8 unit charges (L = 2)
    sysm = config1()
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    Fo, co = direct_factors(_geom(sysm), t, w, sysm.pos, sysm.Z)
    h3 = sysm.h ** 3
    ref = o_reconstruct(Fo, co) / h3
    for precision in ("f64", "f32", "bf16x6"):
        V = L.reconstruct(F, coef, [tuple(sysm.boxes[0])], 1.0 / h3, precision)[0]
        rel_inf, _ = _errors(V.double().cpu().numpy(), ref, ref)
        assert rel_inf < _gate(precision, coef.numel()), (precision, rel_inf)


@pytest.mark.slow
def test_config2_sampled(L):
    # headline workload at full size: factors sampled column by column against
    # the oracle, and potential values at sampled points of two 256^3 boxes
    sysm = config2()
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    geom = _geom(sysm)
    rng = np.random.default_rng(7)
    boxes = [tuple(b) for b in sysm.boxes[:2]]
    h3 = sysm.h ** 3
    for bi, b in enumerate(boxes):
        sel_local = [np.sort(rng.choice(b[3 + l], 6, replace=False)) for l in range(3)]
        cols = [factor_entries(geom, t, sysm.pos, l, b[l] + sel_local[l]) for l in range(3)]
        for l in range(3):
            got = F[l][:, b[l] + sel_local[l]].cpu().numpy()
            assert _close_rows(got, cols[l], 1e-12, F[l].abs().max(dim=1).values.cpu().numpy())
        sel = np.array(np.meshgrid(np.arange(6), np.arange(6), np.arange(6), indexing="ij")).reshape(3, -1).T
        coef_o = (sysm.Z[:, None] * w[None, :]).ravel()
        ref = np.asarray(sample_columns(cols, coef_o, sel), np.float64) / h3
        ref_abs = np.asarray(sample_columns(cols, np.abs(coef_o), sel), np.float64) / h3
        for precision in ("f64", "f32", "bf16x6", "bf16x3", "f16x3"):
            V = L.reconstruct(F, coef, [b], 1.0 / h3, precision)[0]
            got = V[sel_local[0][sel[:, 0]], sel_local[1][sel[:, 1]], sel_local[2][sel[:, 2]]]
            rel_inf, rel_mag = _errors(got.double().cpu().numpy(), ref, ref_abs)
            print(f"config2 box {bi} {precision}: rel_inf {rel_inf:.3e} rel_mag {rel_mag:.3e}")
            assert rel_mag < _gate(precision, coef.numel()), (precision, rel_inf, rel_mag)
            del V
            torch.cuda.empty_cache()


def test_config2_energy_grams_and_repeat(L):
    # energy at full size (K = 384, N = 4096, 48 workgroups in the final sum):
    # the Grams left in the workspace and E against a float64 evaluation of
    # the same definition (eq. scal) from the same factors, and two calls
    # bitwise equal (the final sum runs in workgroup order)
    sysm = config2()
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    D = [_t(x) for x in sysm.density.D]
    d = _t(sysm.density.d)
    K, Krho = int(coef.numel()), int(d.numel())
    ws = torch.empty(L.api.lib().ls_energy_workspace(K, Krho), dtype=torch.uint8, device=dev)
    E1 = float(L.energy(F, coef, D, d, "f64", ws).cpu())
    G = ws[:3 * K * Krho * 8].view(torch.float64).view(3, K, Krho).cpu().numpy()
    E2 = float(L.energy(F, coef, D, d, "f64", ws).cpu())
    assert E1 == E2
    Fh = [f.cpu().numpy() for f in F]
    Dh = [np.asarray(x, np.float64) for x in sysm.density.D]
    Gr = np.stack([Fh[l] @ Dh[l].T for l in range(3)])
    assert np.max(np.abs(G - Gr)) <= 1e-12 * np.max(np.abs(Gr))
    c, dd = coef.cpu().numpy(), np.asarray(sysm.density.d, np.float64)
    terms = c[:, None] * dd[None, :] * Gr[0] * Gr[1] * Gr[2]
    assert abs(E1 - terms.sum()) <= 1e-12 * np.abs(terms).sum(), (E1, terms.sum())


@pytest.mark.slow
def test_config3_periodic_sampled(L):
    # periodic workload at full size: factor columns and sampled cell values
    sysm = config3()
    t, w, qt = _quads(sysm, L)
    F, coef = _gpu_factors(L, sysm, qt)
    geom = _geom(sysm)
    rng = np.random.default_rng(11)
    sel_local = [np.sort(rng.choice(sysm.n, 5, replace=False)) for l in range(3)]
    cols = [factor_entries(geom, t, sysm.pos, l, sel_local[l]) for l in range(3)]
    for l in range(3):
        assert _close_rows(F[l][:, sel_local[l]].cpu().numpy(), cols[l], 1e-12,
                           F[l].abs().max(dim=1).values.cpu().numpy())
    sel = np.array(np.meshgrid(np.arange(5), np.arange(5), np.arange(5), indexing="ij")).reshape(3, -1).T
    coef_o = (sysm.Z[:, None] * w[None, :]).ravel()
    h3 = sysm.h ** 3
    ref = np.asarray(sample_columns(cols, coef_o, sel), np.float64) / h3
    ref_abs = np.asarray(sample_columns(cols, np.abs(coef_o), sel), np.float64) / h3
    for precision in ("f64", "f32", "bf16x6", "bf16x3", "f16x3"):
        V = L.reconstruct(F, coef, [tuple(sysm.boxes[0])], 1.0 / h3, precision)[0]
        got = V[sel_local[0][sel[:, 0]], sel_local[1][sel[:, 1]], sel_local[2][sel[:, 2]]]
        rel_inf, rel_mag = _errors(got.double().cpu().numpy(), ref, ref_abs)
        print(f"config3 {precision}: rel_inf {rel_inf:.3e} rel_mag {rel_mag:.3e}")
        assert rel_mag < _gate(precision, coef.numel()), (precision, rel_inf, rel_mag)
        del V
        torch.cuda.empty_cache()


@pytest.mark.slow
def test_config5_forces_sampled(L):
    # forces workload at full size: oracle adjoint on sampled atoms, and the
    # GPU FP64 energy's central differences (step 1e-4 b) on the same atoms
    sysm = config5()
    t, w, qt = _quads(sysm, L)
    spec = _spec(sysm, L)
    D = [_t(x) for x in sysm.density.D]
    d = _t(sysm.density.d)
    F64, E64 = L.forces(spec, qt, _t(sysm.pos), _t(sysm.Z), D, d, "f64")
    F32, _ = L.forces(spec, qt, _t(sysm.pos), _t(sysm.Z), D, d, "f32")
    F64 = F64.cpu().numpy()
    F32 = F32.cpu().numpy()
    atoms = [0, 17, 42]
    geom = _geom(sysm)
    Fo = forces_adjoint_atoms(geom, t, w, sysm.pos, sysm.Z, sysm.density.D, sysm.density.d, atoms)
    scale = np.max(np.abs(Fo))
    e64 = np.max(np.abs(F64[atoms] - Fo)) / scale
    e32 = np.max(np.abs(F32[atoms] - Fo)) / scale
    print(f"config5 forces vs oracle adjoint: f64 {e64:.3e} f32 {e32:.3e}")
    assert e64 < 1e-12 and e32 < 1e-5, (e64, e32)
    step = sysm.extra["fd_step"]
    for nu in atoms:
        for l in range(3):
            pp, pm = sysm.pos.copy(), sysm.pos.copy()
            pp[nu, l] += step
            pm[nu, l] -= step
            Ep = float(L.forces(spec, qt, _t(pp), _t(sysm.Z), D, d, "f64")[1].cpu())
            Em = float(L.forces(spec, qt, _t(pm), _t(sysm.Z), D, d, "f64")[1].cpu())
            fd = -(Ep - Em) / (2 * step)
            assert abs(fd - F64[nu, l]) < 1e-5 * np.max(np.abs(F64)), (nu, l, fd, F64[nu, l])


@pytest.mark.parametrize("f2_shift", [0, 50])
def test_f16x3_wide_dynamic_range(L, f2_shift):
    # random factors whose rank rows span 10^-9 .. 10^9 per axis and
    # coefficients 10^-5 .. 10^5 of both signs (rank products over 10^40 apart,
    # far beyond the FP16 range, results still inside FP32): the per-rank
    # power-of-two scaling must keep every FP16 term finite and the result
    # within the mixed-precision gate of the FP64 path (itself checked
    # against the oracle above); boxes with ragged edges and one single cell.
    # f2_shift = 50 moves the f2 rows of alternate ranks to 10^50 and 10^-50
    # times their size (outside FP32) and the coefficients by the inverse, so
    # the tiles that stage f2 from an FP32 copy must scale it per rank too.
    rng = np.random.default_rng(61)
    K, lens = 100, (37, 290, 70)
    F = [torch.as_tensor(rng.random((K, n)) * 10.0 ** rng.uniform(-9, 9, (K, 1)), device=dev)
         for n in lens]
    coef = torch.as_tensor(rng.choice([-1.0, 1.0], K) * 10.0 ** rng.uniform(-5, 5, K), device=dev)
    if f2_shift:
        sh = torch.as_tensor(np.where(np.arange(K) % 2 == 0, 10.0, 0.1) ** f2_shift, device=dev)
        F[2] = F[2] * sh[:, None]
        coef = coef / sh
    boxes = [(3, 17, 5, 30, 270, 61), (0, 0, 0, 1, 1, 1)]
    ref = L.reconstruct(F, coef, boxes, 1.0, "f64")
    ref_abs = L.reconstruct([f.abs() for f in F], coef.abs(), boxes, 1.0, "f64")
    for tile in range(L.reconstruct_tiles("f16x3") + 1):
        got = L.reconstruct(F, coef, boxes, 1.0, "f16x3", tile)
        for b, (g, r, ra) in enumerate(zip(got, ref, ref_abs)):
            assert torch.isfinite(g).all(), (tile, b)
            err = float((g.double() - r).abs().max()) / float(ra.abs().max())
            assert err < 1e-6, (tile, b, err)


FUSED_CASES = [c for c in SMALL + WIDTHS if not c[0].startswith("periodic")]


@pytest.mark.parametrize("name,maker", FUSED_CASES, ids=[c[0] for c in FUSED_CASES])
@pytest.mark.parametrize("deriv", [False, True], ids=["value", "derivative"])
def test_fused_box_assembly_equals_stored_masters(L, name, maker, deriv):
    # kernel vectors generated inside the assembly (LDS window) give the
    # stored-masters assembly's factors bit for bit (L > 64 takes the
    # per-entry route and is compared with the oracle elsewhere); the row
    # maxima written beside them are the rows' maxima exactly
    sysm = maker()
    t, w, qt = _quads(sysm, L)
    spec = _spec(sysm, L)
    pos = _t(sysm.pos)
    Z = None if deriv else _t(sysm.Z)
    Fm, cm = L.assemble(spec, qt, pos, Z, L.kernel_vectors(spec, qt, pos, derivative=deriv),
                        derivative=deriv)
    K = Fm[0].shape[0]
    Ff = [torch.empty_like(f) for f in Fm]
    cf = None if deriv else torch.empty_like(cm)
    rmax = torch.full((3, K), -1.0, dtype=torch.float64, device=dev)
    L.assemble_into(spec, qt, pos, Z, None, Ff, cf, derivative=deriv, rowmax=rmax)
    torch.cuda.synchronize()
    for l in range(3):
        if max(sysm.L) <= 64:
            assert torch.equal(Ff[l], Fm[l]), (name, deriv, l)
        assert torch.equal(rmax[l], Ff[l].abs().max(dim=1).values), (name, deriv, l)
    if not deriv:
        assert torch.equal(cf, cm)


def test_row_maxima_on_every_assembly_route(L):
    # stored masters and the periodic cell compute the maxima after the
    # assembly; the FP16x3 reconstruction with them equals the one that
    # finds them itself, bit for bit
    for sysm in (small_box(131, n=10, L=(3, 2, 4), M0=3), small_periodic(132, n=12, L=(5, 3, 5), M0=3)):
        t, w, qt = _quads(sysm, L)
        spec = _spec(sysm, L)
        pos, Z = _t(sysm.pos), _t(sysm.Z)
        masters = None if sysm.periodic else L.kernel_vectors(spec, qt, pos)
        F, coef = L.assemble(spec, qt, pos, Z, masters)
        rmax = torch.empty((3, coef.numel()), dtype=torch.float64, device=dev)
        F2 = [torch.empty_like(f) for f in F]
        c2 = torch.empty_like(coef)
        L.assemble_into(spec, qt, pos, Z, masters, F2, c2, rowmax=rmax)
        torch.cuda.synchronize()
        for l in range(3):
            assert torch.equal(F2[l], F[l])
            assert torch.equal(rmax[l], F[l].abs().max(dim=1).values)
        box = [(0, 0, 0) + tuple(int(f.shape[1]) for f in F)]
        V1 = L.reconstruct(F, coef, box, 1.0, "f16x3")[0]
        V2 = L.reconstruct(F, coef, box, 1.0, "f16x3", rowmax=rmax)[0]
        torch.cuda.synchronize()
        assert torch.equal(V1, V2)


def test_config2_fused_assembly_bitwise(L):
    # the headline workload: fused kernel vectors + assembly equal the
    # stored-masters route bit for bit at full size
    sysm = config2()
    t, w, qt = _quads(sysm, L)
    spec = _spec(sysm, L)
    pos, Z = _t(sysm.pos), _t(sysm.Z)
    Fm, cm = L.assemble(spec, qt, pos, Z, L.kernel_vectors(spec, qt, pos))
    Ff = [torch.empty_like(f) for f in Fm]
    cf = torch.empty_like(cm)
    rmax = torch.empty((3, cm.numel()), dtype=torch.float64, device=dev)
    L.assemble_into(spec, qt, pos, Z, None, Ff, cf, rowmax=rmax)
    torch.cuda.synchronize()
    for l in range(3):
        assert torch.equal(Ff[l], Fm[l]), l
        assert torch.equal(rmax[l], Fm[l].abs().max(dim=1).values), l


@pytest.mark.slow
def test_config2_full_factors_and_energy_against_oracle(L):
    # the headline workload at full size against the oracle's direct sum:
    # every factor row of the step's fused assembly (1e-12 of each row's
    # maximum) and the energy <P, rho> (eq. scal) for FP64 (1e-12) and FP32
    # Grams (1e-6), rel_mag with the |Z| energy
    from oracle.canonical import scalar_product
    sysm = config2()
    t, w, qt = _quads(sysm, L)
    spec = _spec(sysm, L)
    Fo, co = direct_factors(_geom(sysm), t, w, sysm.pos, sysm.Z)
    rm = torch.empty((3, len(co)), dtype=torch.float64, device=dev)
    F, coef = L.assemble(spec, qt, _t(sysm.pos), _t(sysm.Z), None, rowmax=rm)
    torch.cuda.synchronize()
    for l in range(3):
        assert _close_rows(F[l].cpu().numpy(), Fo[l], 1e-12), l
    D = [_t(x) for x in sysm.density.D]
    d = _t(sysm.density.d)
    Eo = scalar_product(Fo, co, sysm.density.D, sysm.density.d)
    Eabs = scalar_product(Fo, np.abs(co), sysm.density.D, sysm.density.d)
    for precision, gate in (("f64", 1e-12), ("f32", 1e-6)):
        E = float(L.energy(F, coef, D, d, precision).cpu())
        err = abs(E - Eo) / abs(Eabs)
        print(f"config2 energy {precision}: rel_mag {err:.3e} (E {E!r}, oracle {Eo!r})")
        assert err < gate, (precision, err)
