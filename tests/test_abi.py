"""The C ABI without a GPU: the library loads, exports every declared entry
point, its host-side steps match the oracle, and invalid calls fail before
anything is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.quadrature import rule_u, rule_s
from oracle.lattice import Geometry, master_extent

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "latsum.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1405_2270_amd import _lib
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    from paper_1405_2270_amd import _lib
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.EXPORTS, name
    assert lib.ls_version().startswith(b"latsum")


@pytest.mark.parametrize("M,C0", [(20, 1.0), (7, 2.5), (59, 4.4)])
def test_quadrature_matches_oracle(M, C0):
    import paper_1405_2270_amd as L
    q = L.quadrature("U", M, C0)
    t, w = rule_u(M, C0)
    assert q.R == 2 * M + 1
    assert np.allclose(q.t, t, rtol=1e-15, atol=1e-15) and np.allclose(q.w, w, rtol=1e-15, atol=0)
    q = L.quadrature("S", M, C0, 3.3e-3)
    t, w = rule_s(M, C0, 3.3e-3)
    assert q.R == M + 1
    assert np.allclose(q.t, t, rtol=4e-16, atol=0) and np.allclose(q.w, w, rtol=4e-16, atol=0)


@pytest.mark.parametrize("n,L,periodic", [(8, (3, 2, 5), False), (16, (5, 5, 5), True),
                                          (10, (4, 6, 2), True), (7, (1, 1, 1), False)])
def test_master_halfwidth_covers_oracle_extent(n, L, periodic):
    import paper_1405_2270_amd as lib
    X = lib.master_halfwidth(lib.LatticeSpec(10.0, n, L, periodic))
    g = Geometry(10.0, n, L, periodic)
    assert X == max(master_extent(g, l) for l in range(3))


def test_invalid_host_arguments(lib):
    from paper_1405_2270_amd import _lib
    t = np.zeros(3)
    R = ctypes.c_int32(0)
    st = lib.ls_quadrature(0, 20, 1.0, 1.0, t.ctypes.data_as(_lib.c_double_p),
                           t.ctypes.data_as(_lib.c_double_p), 3, ctypes.byref(R))
    assert st == _lib.LS_EINVAL and b"capacity" in lib.ls_last_error()
    st = lib.ls_quadrature(1, 1, 1.0, 1.0, t.ctypes.data_as(_lib.c_double_p),
                           t.ctypes.data_as(_lib.c_double_p), 3, ctypes.byref(R))
    assert st == _lib.LS_EINVAL
    X = ctypes.c_int32(0)
    bad = _lib.Lattice(0, (ctypes.c_int32 * 3)(1, 1, 1), 10.0, 0)
    assert lib.ls_master_halfwidth(ctypes.byref(bad), ctypes.byref(X)) == _lib.LS_EINVAL
    # null descriptors: rejected on the host, nothing launched
    assert lib.ls_reconstruct(None, None, 1, 1.0, 0, 0, None, None, 0, None) == _lib.LS_EINVAL
    assert lib.ls_energy(None, None, 0, None, None, 0, None) == _lib.LS_EINVAL
    assert lib.ls_assemble(None, None, 1, None, None, None, 0, 0, None, None, None, None,
                           None, None) == _lib.LS_EINVAL
    # Richardson sums: periodic lattices only, order 1 or 2 (nothing launched)
    t2, w2 = np.array([1.0, 2.0]), np.array([0.5, 0.5])
    quad = _lib.Quad(2, t2.ctypes.data_as(_lib.c_double_p), w2.ctypes.data_as(_lib.c_double_p))
    box = _lib.Lattice(8, (ctypes.c_int32 * 3)(3, 3, 3), 10.0, 0)
    per = _lib.Lattice(8, (ctypes.c_int32 * 3)(3, 3, 3), 10.0, 1)
    dummy = ctypes.c_void_p(16)
    for lat, order, needle in ((box, 1, b"periodic"), (per, 3, b"order"), (per, 0, b"order")):
        st = lib.ls_richardson(ctypes.byref(lat), ctypes.byref(quad), 1, dummy, dummy, order,
                               dummy, dummy, dummy, dummy, None)
        assert st == _lib.LS_EINVAL and needle in lib.ls_last_error(), (order, lib.ls_last_error())
    # the no-allocation forces refuse a problem beyond their fixed scratch on
    # the host, before any device query
    rho = _lib.Canon(8, (ctypes.c_int32 * 3)(24, 24, 24), (ctypes.c_void_p * 3)(16, 16, 16), 16)
    st = lib.ls_forces_noalloc(ctypes.byref(box), ctypes.byref(quad), 20000, dummy, dummy,
                               ctypes.byref(rho), 0, dummy, None, None)
    assert st == _lib.LS_EWORKSPACE and b"scratch" in lib.ls_last_error()
    # workspaces must be 256-byte aligned (their kernels issue 16-byte loads):
    # a large enough but misaligned one is refused on the host
    misaligned = ctypes.c_void_p(4096 + 8)
    st = lib.ls_forces(ctypes.byref(box), ctypes.byref(quad), 1, dummy, dummy, ctypes.byref(rho), 0,
                       dummy, None, misaligned, 1 << 40, None)
    assert st == _lib.LS_EINVAL and b"aligned" in lib.ls_last_error(), lib.ls_last_error()
    P = _lib.Canon(4, (ctypes.c_int32 * 3)(24, 24, 24), (ctypes.c_void_p * 3)(16, 16, 16), 16)
    st = lib.ls_energy(ctypes.byref(P), ctypes.byref(rho), 0, dummy, misaligned, 1 << 40, None)
    assert st == _lib.LS_EINVAL and b"aligned" in lib.ls_last_error(), lib.ls_last_error()
    st = lib.ls_reconstruct_prepare(ctypes.byref(P), 4, misaligned, 1 << 40, None)
    assert st == _lib.LS_EINVAL and b"aligned" in lib.ls_last_error(), lib.ls_last_error()
    # the reconstruction autotuner refuses a bad repetition count on the host;
    # its cache answers "not tuned" for a class never timed (host only)
    B1 = (_lib.Box * 1)(_lib.Box((ctypes.c_int32 * 3)(0, 0, 0), (ctypes.c_int32 * 3)(4, 4, 4)))
    tile, ms = ctypes.c_int32(-1), ctypes.c_double(-1.0)
    for reps in (0, 1001):
        st = lib.ls_reconstruct_autotune(ctypes.byref(P), B1, 1, 1.0, 4, dummy, dummy, 1 << 40, reps,
                                         None, ctypes.byref(tile), ctypes.byref(ms))
        assert st == _lib.LS_EINVAL and b"reps" in lib.ls_last_error(), lib.ls_last_error()
        assert tile.value == 0 and ms.value == 0.0
    st = lib.ls_reconstruct_autotune(ctypes.byref(P), B1, 1, 1.0, 4, dummy, dummy, 1 << 40, 3,
                                     None, None, None)
    assert st == _lib.LS_EINVAL
    for prec in range(5):
        st = lib.ls_reconstruct_tuned_tile(ctypes.byref(P), B1, 1, prec, dummy, 1 << 40,
                                           ctypes.byref(tile), ctypes.byref(ms))
        assert st == _lib.LS_OK and tile.value == 0 and ms.value == 0.0
    assert lib.ls_reconstruct_tuned_tile(ctypes.byref(P), B1, 1, 7, None, 0, ctypes.byref(tile),
                                         None) == _lib.LS_EINVAL
    assert lib.ls_reconstruct_tuned_tile(ctypes.byref(P), B1, 0, 0, None, 0, ctypes.byref(tile),
                                         None) == _lib.LS_EINVAL
    # the FP16x3 plan query checks its boxes and workspace on the host before
    # any copy; the FP16x3 workspace also holds the rank order (K words) and
    # one chunk mask per plane of axis 0
    cv = ctypes.c_int64(-1)
    B9 = (_lib.Box * 1)(_lib.Box((ctypes.c_int32 * 3)(0, 0, 21), (ctypes.c_int32 * 3)(4, 4, 4)))
    assert lib.ls_reconstruct_f16_plan(ctypes.byref(P), B9, 1, dummy, 1 << 40, None, None,
                                       ctypes.byref(cv)) == _lib.LS_EINVAL
    assert lib.ls_reconstruct_f16_plan(ctypes.byref(P), B1, 0, dummy, 1 << 40, None, None,
                                       ctypes.byref(cv)) == _lib.LS_EINVAL
    need = lib.ls_reconstruct_workspace(ctypes.byref(P), 4)
    assert lib.ls_reconstruct_f16_plan(ctypes.byref(P), B1, 1, dummy, need - 1, None, None,
                                       ctypes.byref(cv)) == _lib.LS_EWORKSPACE
    assert lib.ls_reconstruct_f16_plan(ctypes.byref(P), B1, 1, None, need, None, None,
                                       ctypes.byref(cv)) == _lib.LS_EWORKSPACE
    assert cv.value == -1
    P2 = _lib.Canon(4, (ctypes.c_int32 * 3)(1024, 24, 24), (ctypes.c_void_p * 3)(16, 16, 16), 16)
    assert lib.ls_reconstruct_workspace(ctypes.byref(P2), 4) >= need + 1000 * 4 - 256
    # a batch system whose factor columns the kernel's 32-bit buffer offsets
    # cannot address (M0 R >= 2^20 ranks) is refused on the host, by index
    tq, wq = np.linspace(0.1, 2.0, 60), np.full(60, 0.01)
    quad60 = _lib.Quad(60, tq.ctypes.data_as(_lib.c_double_p), wq.ctypes.data_as(_lib.c_double_p))
    rho8 = _lib.Canon(8, (ctypes.c_int32 * 3)(24, 24, 24), (ctypes.c_void_p * 3)(16, 16, 16), 16)
    sysd = (_lib.System * 1)()
    sysd[0] = _lib.System(box, quad60, 20000, 16, 16, rho8,
                          _lib.Box((ctypes.c_int32 * 3)(0, 0, 0), (ctypes.c_int32 * 3)(4, 4, 4)), 16, 16)
    handle, nws = ctypes.c_void_p(), ctypes.c_size_t(0)
    st = lib.ls_batch_create(sysd, 1, 4, ctypes.byref(handle), ctypes.byref(nws))
    assert st == _lib.LS_EINVAL and b"system 0" in lib.ls_last_error() and b"2 GB" in lib.ls_last_error(), \
        lib.ls_last_error()
    assert lib.ls_reconstruct_tiles(0) >= 1 and lib.ls_reconstruct_tiles(9) == 0
    assert lib.ls_reconstruct_tiles(4) == 8 and lib.ls_reconstruct_workspace(None, 4) == 0
    assert lib.ls_reconstruct_workspace(None, 2) == 0
    assert lib.ls_energy_workspace(10, 8) >= 3 * 10 * 8 * 8
