"""ls_forces_noalloc (fixed device scratch, no workspace argument) against
ls_forces with a caller workspace, through the C ABI: two calls in a row, the
second on a smaller problem, each bit for bit equal to ls_forces on the same
inputs (the same kernels in the same order), and checked against the oracle
adjoint; an oversized problem is refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

from oracle.lattice import Geometry
from oracle.physics import forces_adjoint
from oracle.quadrature import rule_s
from workloads import small_box

pytestmark = pytest.mark.gpu
dev = torch.device("cuda:0")


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _args(L, s):
    q = s.quad
    qt = L.quadrature("S", q["M"], q["C0"], q["s"])
    spec = L.LatticeSpec(s.b, s.n, tuple(s.L), False)
    pos, Z = _t(s.pos), _t(s.Z)
    D = [_t(x) for x in s.density.D]
    d = _t(s.density.d)
    return qt, spec, pos, Z, D, d


def _call_both(L, s, precision):
    from paper_1405_2270_amd import _lib
    lib = L.api.lib()
    qt, spec, pos, Z, D, d = _args(L, s)
    M0 = pos.shape[0]
    lat, quad, rho = spec.c(), qt.c(), L.api._canon(D, d, "density")
    prec = _lib.PRECISIONS[precision]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    need = int(lib.ls_forces_workspace(ctypes.byref(lat), M0, qt.R, len(D[0])))
    assert 0 < need <= _NOALLOC_BYTES
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    F_ref = torch.full((M0, 3), np.nan, dtype=torch.float64, device=dev)
    E_ref = torch.full((), np.nan, dtype=torch.float64, device=dev)
    st = lib.ls_forces(ctypes.byref(lat), ctypes.byref(quad), M0, ctypes.c_void_p(pos.data_ptr()),
                       ctypes.c_void_p(Z.data_ptr()), ctypes.byref(rho), prec,
                       ctypes.c_void_p(F_ref.data_ptr()), ctypes.c_void_p(E_ref.data_ptr()),
                       ctypes.c_void_p(ws.data_ptr()), need, stream)
    assert st == 0, lib.ls_last_error()
    F = torch.full((M0, 3), np.nan, dtype=torch.float64, device=dev)
    E = torch.full((), np.nan, dtype=torch.float64, device=dev)
    st = lib.ls_forces_noalloc(ctypes.byref(lat), ctypes.byref(quad), M0,
                               ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(Z.data_ptr()),
                               ctypes.byref(rho), prec, ctypes.c_void_p(F.data_ptr()),
                               ctypes.c_void_p(E.data_ptr()), stream)
    assert st == 0, lib.ls_last_error()
    torch.cuda.synchronize()
    return F.cpu().numpy(), float(E.cpu()), F_ref.cpu().numpy(), float(E_ref.cpu()), qt


_NOALLOC_BYTES = 8 << 20


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_forces_match_workspace_forces(precision):
    import paper_1405_2270_amd as L
    assert torch.cuda.is_available()
    # the larger problem first, then a smaller one: the second call must not
    # see anything the first left in the shared scratch
    for s in (small_box(711, n=12, L=(4, 3, 5), M0=6), small_box(712, n=8, L=(2, 2, 3), M0=2)):
        F, E, F_ref, E_ref, qt = _call_both(L, s, precision)
        assert np.all(np.isfinite(F)) and np.isfinite(E)
        assert np.array_equal(F, F_ref) and E == E_ref, (precision, s.L, np.max(np.abs(F - F_ref)))
        q = s.quad
        t, w = rule_s(q["M"], q["C0"], q["s"])
        Fo = forces_adjoint(Geometry(s.b, s.n, tuple(s.L), False), t, w, s.pos, s.Z,
                            s.density.D, s.density.d)
        err = np.max(np.abs(F - Fo)) / np.max(np.abs(Fo))
        assert err < (1e-12 if precision == "f64" else 1e-5), (precision, err)


def test_noalloc_refuses_oversized_problem():
    import paper_1405_2270_amd as L
    from paper_1405_2270_amd import _lib
    lib = L.api.lib()
    s = small_box(713, n=8, L=(2, 2, 2), M0=2)
    qt, spec, pos, Z, D, d = _args(L, s)
    lat, quad, rho = spec.c(), qt.c(), L.api._canon(D, d, "density")
    M0_big = 4000  # Grams alone: 2 * 3 * 4000 * R * 8 * 8 bytes, far above 8 MiB
    assert lib.ls_forces_workspace(ctypes.byref(lat), M0_big, qt.R, len(D[0])) > _NOALLOC_BYTES
    F = torch.empty((M0_big, 3), dtype=torch.float64, device=dev)
    st = lib.ls_forces_noalloc(ctypes.byref(lat), ctypes.byref(quad), M0_big,
                               ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(Z.data_ptr()),
                               ctypes.byref(rho), _lib.PRECISIONS["f64"],
                               ctypes.c_void_p(F.data_ptr()), None,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.LS_EWORKSPACE
    assert b"scratch" in lib.ls_last_error()
