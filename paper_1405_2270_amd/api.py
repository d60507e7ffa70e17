"""Python surface of the latsum library: marshals torch tensors into the C ABI.

PyTorch supplies device memory and the current stream; every arithmetic step
runs in the HIP library. Inputs must be CUDA (HIP) tensors of dtype float64 and
contiguous; outputs are allocated here with torch and filled by the library.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import Lattice, Quad, Canon, Box, System, TensorLattice, check, lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev_f64(x, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    return x


def _pos_tensor(pos):
    pos = _dev_f64(pos, "pos")
    if pos.dim() != 2 or pos.shape[1] != 3 or pos.shape[0] < 1:
        raise ValueError("pos must have shape [M0][3] with M0 >= 1")
    return pos


def _charges(Z, M0):
    Z = _dev_f64(Z, "Z")
    if Z.numel() != M0:
        raise ValueError(f"Z must hold {M0} charges (got {Z.numel()})")
    return Z


@dataclass(frozen=True)
class LatticeSpec:
    """Grid and lattice: unit cell edge b, n cells per edge, L images per axis."""
    b: float
    n: int
    L: tuple
    periodic: bool = False

    @property
    def h(self):
        return self.b / self.n

    def N(self, l):
        return self.n if self.periodic else self.L[l] * self.n

    def c(self):
        return Lattice(self.n, (ctypes.c_int32 * 3)(*self.L), self.b, int(self.periodic))


class TensorLatticeSpec:
    """Non-equidistant tensor lattice: unit cell edge b, n cells per edge
    (h = b/n), N[l] grid cells per axis and the lattice coordinates s[l] of
    each axis in units of h (three 1D float64 device tensors)."""

    def __init__(self, b, n, N, s):
        self.b, self.n, self.N = float(b), int(n), tuple(int(v) for v in N)
        if len(self.N) != 3 or len(s) != 3:
            raise ValueError("three axes are required")
        self.s = tuple(_dev_f64(x, f"s[{l}]").reshape(-1) for l, x in enumerate(s))
        for l, x in enumerate(self.s):
            if not x.is_contiguous() or x.numel() < 1:
                raise ValueError(f"s[{l}] must be a non-empty contiguous vector")

    @property
    def h(self):
        return self.b / self.n

    def c(self):
        return TensorLattice(self.n, self.b, (ctypes.c_int32 * 3)(*self.N),
                             (ctypes.c_int32 * 3)(*[x.numel() for x in self.s]),
                             (ctypes.c_void_p * 3)(*[x.data_ptr() for x in self.s]))


class QuadTable:
    """Quadrature nodes/weights held on the host (FP64) for the C ABI."""

    def __init__(self, t, w):
        self.t = np.ascontiguousarray(t, np.float64)
        self.w = np.ascontiguousarray(w, np.float64)
        self.R = int(self.t.size)

    def c(self):
        return Quad(self.R, self.t.ctypes.data_as(_lib.c_double_p),
                    self.w.ctypes.data_as(_lib.c_double_p))


def quadrature(rule, M, C0=1.0, s=1.0):
    """Sinc quadrature table computed by the library (``rule`` 'U' or 'S')."""
    code = {"U": _lib.LS_RULE_U, "S": _lib.LS_RULE_S}[rule]
    cap = 2 * M + 1
    t = np.zeros(cap)
    w = np.zeros(cap)
    R = ctypes.c_int32(0)
    check("ls_quadrature", lib().ls_quadrature(code, M, C0, s, t.ctypes.data_as(_lib.c_double_p),
                                               w.ctypes.data_as(_lib.c_double_p), cap,
                                               ctypes.byref(R)))
    return QuadTable(t[:R.value], w[:R.value])


def master_halfwidth(lat):
    X = ctypes.c_int32(0)
    check("ls_master_halfwidth", lib().ls_master_halfwidth(ctypes.byref(lat.c()), ctypes.byref(X)))
    return X.value


def kernel_vectors(lat, quad, pos, derivative=False):
    """Master vectors [M0*3][R][2X] (FP64) for every atom and axis."""
    pos = _pos_tensor(pos)
    X = master_halfwidth(lat)
    out = torch.empty((pos.shape[0] * 3, quad.R, 2 * X), dtype=torch.float64, device=pos.device)
    return kernel_vectors_into(lat, quad, pos, out, derivative)


def kernel_vectors_into(lat, quad, pos, out, derivative=False):
    """As ``kernel_vectors`` but into a caller-provided tensor of M0*3*R*2X doubles."""
    pos = _pos_tensor(pos)
    M0 = pos.shape[0]
    X = master_halfwidth(lat)
    out = _dev_f64(out, "masters")
    if out.numel() != M0 * 3 * quad.R * 2 * X or not out.is_contiguous():
        raise ValueError(f"masters must be contiguous with M0*3*R*2X = {M0 * 3 * quad.R * 2 * X} values")
    check("ls_kernel_vectors", lib().ls_kernel_vectors(ctypes.byref(lat.c()), ctypes.byref(quad.c()),
                                                       M0, _ptr(pos), X, int(derivative), _ptr(out),
                                                       _stream()))
    return out


def assemble(lat, quad, pos, Z, masters=None, derivative=False, rowmax=None):
    """Assembled canonical factors [f0, f1, f2] ([K][N_l] FP64 each) and coef [K]
    (``masters`` None: the box lattice's kernel vectors generated inside the
    assembly where its window fits, else every cell integral in registers)."""
    pos = _pos_tensor(pos)
    M0 = pos.shape[0]
    K = M0 * quad.R
    dev = pos.device
    F = [torch.empty((K, lat.N(l)), dtype=torch.float64, device=dev) for l in range(3)]
    coef = None if derivative else torch.empty(K, dtype=torch.float64, device=dev)
    return assemble_into(lat, quad, pos, Z, masters, F, coef, derivative, rowmax)


def assemble_tensor(tl, quad, pos, Z, derivative=False):
    """Assembled factors of a non-equidistant tensor lattice (``TensorLatticeSpec``):
    [f0, f1, f2] ([K][N_l] FP64 each) and coef [K] (None for derivatives)."""
    pos = _pos_tensor(pos)
    M0 = pos.shape[0]
    K = M0 * quad.R
    dev = pos.device
    for x in tl.s:
        if x.device != dev:
            raise ValueError("lattice coordinates and positions must be on one device")
    F = [torch.empty((K, tl.N[l]), dtype=torch.float64, device=dev) for l in range(3)]
    coef = None if derivative else torch.empty(K, dtype=torch.float64, device=dev)
    return assemble_tensor_into(tl, quad, pos, Z, F, coef, derivative)


def assemble_tensor_into(tl, quad, pos, Z, F, coef, derivative=False):
    """As ``assemble_tensor`` but into caller-provided factors F and coef."""
    pos = _pos_tensor(pos)
    M0 = pos.shape[0]
    K = M0 * quad.R
    for l in range(3):
        f = _dev_f64(F[l], "factor")
        if tuple(f.shape) != (K, tl.N[l]) or not f.is_contiguous():
            raise ValueError(f"factor {l} must be contiguous with shape {(K, tl.N[l])}")
    if not derivative:
        Z = _charges(Z, M0)
        coef = _dev_f64(coef, "coef")
        if coef.numel() != K:
            raise ValueError("coef must have K entries")
    check("ls_assemble_tensor", lib().ls_assemble_tensor(
        ctypes.byref(tl.c()), ctypes.byref(quad.c()), M0, _ptr(pos),
        _ptr(None if derivative else Z), int(derivative), _ptr(F[0]), _ptr(F[1]), _ptr(F[2]),
        _ptr(coef), _stream()))
    return F, coef


def assemble_into(lat, quad, pos, Z, masters, F, coef, derivative=False, rowmax=None):
    """As ``assemble`` but into caller-provided factors F and coef; ``rowmax``
    (a [3][K] float64 device tensor, optional) receives max_g |f_l[r][g]|."""
    pos = _pos_tensor(pos)
    M0 = pos.shape[0]
    K = M0 * quad.R
    for l in range(3):
        f = _dev_f64(F[l], "factor")
        if tuple(f.shape) != (K, lat.N(l)):
            raise ValueError(f"factor {l} must have shape {(K, lat.N(l))}")
    if not derivative:
        Z = _charges(Z, M0)
        coef = _dev_f64(coef, "coef")
        if coef.numel() != K:
            raise ValueError("coef must have K entries")
    X = master_halfwidth(lat)
    if masters is not None:
        masters = _dev_f64(masters, "masters")
        if masters.numel() != M0 * 3 * quad.R * 2 * X:
            raise ValueError(f"masters must hold M0*3*R*2X = {M0 * 3 * quad.R * 2 * X} values")
    if rowmax is not None:
        rowmax = _dev_f64(rowmax, "rowmax")
        if rowmax.numel() != 3 * K or not rowmax.is_contiguous():
            raise ValueError(f"rowmax must be contiguous with 3*K = {3 * K} values")
    check("ls_assemble", lib().ls_assemble(ctypes.byref(lat.c()), ctypes.byref(quad.c()), M0,
                                           _ptr(pos), _ptr(None if derivative else Z),
                                           _ptr(masters), X, int(derivative), _ptr(F[0]),
                                           _ptr(F[1]), _ptr(F[2]), _ptr(None if derivative else coef),
                                           _ptr(rowmax), _stream()))
    return F, coef


def _canon(F, coef, name="factor", rowmax=None):
    """Canonical-tensor descriptor of three device factor matrices [K][len_l]
    and their coefficients [K], all contiguous float64 on one device
    (``rowmax``: optional [3][K] row maxima of the factors, as ``assemble``
    writes them)."""
    if len(F) != 3:
        raise ValueError(f"{name}: three factor matrices are required")
    for l, f in enumerate(F):
        _dev_f64(f, f"{name}[{l}]")
        if f.dim() != 2:
            raise ValueError(f"{name}[{l}] must be a matrix [K][len]")
    K = int(F[0].shape[0])
    if any(int(f.shape[0]) != K for f in F):
        raise ValueError(f"{name}: the factor matrices must have the same number of rows")
    coef = _dev_f64(coef, f"{name} coefficients")
    if coef.numel() != K:
        raise ValueError(f"{name}: {K} coefficients are required (got {coef.numel()})")
    if any(x.device != F[0].device for x in (F[1], F[2], coef)):
        raise ValueError(f"{name}: all tensors must be on one device")
    if rowmax is not None:
        rowmax = _dev_f64(rowmax, f"{name} row maxima")
        if rowmax.numel() != 3 * K or not rowmax.is_contiguous() or rowmax.device != F[0].device:
            raise ValueError(f"{name}: row maxima must be a contiguous [3][K] tensor on the device")
    return Canon(K, (ctypes.c_int32 * 3)(*[int(f.shape[1]) for f in F]),
                 (ctypes.c_void_p * 3)(*[f.data_ptr() for f in F]), coef.data_ptr(),
                 rowmax.data_ptr() if rowmax is not None else None)


def _out_tensor(out, dtype, numel, device, name="out"):
    """A caller-provided output must be a contiguous device tensor of the
    precision's element type with room for ``numel`` elements (the library
    writes through the raw pointer)."""
    if not isinstance(out, torch.Tensor) or not out.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if out.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} for this precision (got {out.dtype})")
    if not out.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if out.device != device:
        raise ValueError(f"{name} must be on {device}")
    if out.numel() < numel:
        raise ValueError(f"{name} holds {out.numel()} elements, {numel} are required")
    return out


def _ws_tensor(ws, device, name="workspace"):
    if ws is None:
        return None
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or not ws.is_contiguous():
        raise TypeError(f"{name} must be a contiguous device tensor")
    if ws.device != device:
        raise ValueError(f"{name} must be on {device}")
    return ws


def _recon_ws(canon, prec, device, ws):
    need = int(lib().ls_reconstruct_workspace(ctypes.byref(canon), prec))
    if need == 0:
        return None, 0
    ws = _ws_tensor(ws, device)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    return ws, ws.numel() * ws.element_size()


def reconstruct(F, coef, boxes, scale=1.0, precision="f64", tile=0, ws=None, rowmax=None):
    """Sub-boxes of the canonical tensor. ``boxes``: iterable of
    (o0, o1, o2, e0, e1, e2). Returns one tensor [e0][e1][e2] per box
    (views of a single allocation). ``ws``: optional uint8 device workspace
    (split-bf16 precisions; allocated here when missing or short). ``rowmax``:
    the factors' row maxima from ``assemble`` (optional, FP16x3 uses them)."""
    _canon(F, coef, rowmax=rowmax)
    boxes = [tuple(int(v) for v in b) for b in boxes]
    prec = _lib.PRECISIONS[precision]
    dtype = torch.float64 if prec == _lib.LS_F64 else torch.float32
    sizes = [b[3] * b[4] * b[5] for b in boxes]
    flat = torch.empty(sum(sizes), dtype=dtype, device=F[0].device)
    reconstruct_into(F, coef, boxes, flat, scale, precision, tile, ws, rowmax=rowmax)
    out, off = [], 0
    for b, s in zip(boxes, sizes):
        out.append(flat[off:off + s].view(b[3], b[4], b[5]))
        off += s
    return out


def reconstruct_into(F, coef, boxes, out, scale=1.0, precision="f64", tile=0, ws=None,
                     prepared=False, rowmax=None):
    """As ``reconstruct`` but into a caller-provided flat tensor. ``prepared``:
    ``ws`` already holds the preparation of these factors for this precision
    (``reconstruct_prepare``, or an earlier call with the same ``ws``)."""
    boxes = [tuple(int(v) for v in b) for b in boxes]
    if any(len(b) != 6 for b in boxes):
        raise ValueError("a box is (o0, o1, o2, e0, e1, e2)")
    prec = _lib.PRECISIONS[precision]
    canon = _canon(F, coef, rowmax=rowmax)
    dtype = torch.float64 if prec == _lib.LS_F64 else torch.float32
    _out_tensor(out, dtype, sum(max(b[3], 0) * max(b[4], 0) * max(b[5], 0) for b in boxes),
                F[0].device)
    need = int(lib().ls_reconstruct_workspace(ctypes.byref(canon), prec))
    ws = _ws_tensor(ws, F[0].device)
    if prepared and need > 0 and (ws is None or ws.numel() * ws.element_size() < need):
        raise ValueError("prepared=True needs the prepared workspace (%d bytes)" % need)
    ws, nws = _recon_ws(canon, prec, F[0].device, ws)
    cb = (Box * len(boxes))(*[Box((ctypes.c_int32 * 3)(*b[:3]), (ctypes.c_int32 * 3)(*b[3:]))
                              for b in boxes])
    name = "ls_reconstruct_prepared" if prepared else "ls_reconstruct"
    check(name, getattr(lib(), name)(ctypes.byref(canon), cb, len(boxes), float(scale), prec,
                                     int(tile), _ptr(out), _ptr(ws), nws, _stream()))
    return out


def reconstruct_prepare(F, coef, precision, ws=None, rowmax=None):
    """The workspace preparation of ``reconstruct`` for these factors and this
    precision, as a call of its own (enqueued on the current stream). Returns
    the workspace (allocated when ``ws`` is None or too small; None when the
    precision needs none)."""
    prec = _lib.PRECISIONS[precision]
    canon = _canon(F, coef, rowmax=rowmax)
    ws, nws = _recon_ws(canon, prec, F[0].device, ws)
    check("ls_reconstruct_prepare", lib().ls_reconstruct_prepare(ctypes.byref(canon), prec, _ptr(ws),
                                                                 nws, _stream()))
    return ws


def reconstruct_tiles(precision):
    return int(lib().ls_reconstruct_tiles(_lib.PRECISIONS[precision]))


def _boxes_c(boxes):
    boxes = [tuple(int(v) for v in b) for b in boxes]
    if not boxes or any(len(b) != 6 for b in boxes):
        raise ValueError("boxes: one or more (o0, o1, o2, e0, e1, e2)")
    cb = (Box * len(boxes))(*[Box((ctypes.c_int32 * 3)(*b[:3]), (ctypes.c_int32 * 3)(*b[3:]))
                              for b in boxes])
    return boxes, cb


def reconstruct_autotune(F, coef, boxes, out, scale=1.0, precision="f64", ws=None, rowmax=None,
                         reps=3):
    """Times every tile of ``precision`` on this call (``ls_reconstruct_autotune``,
    synchronous) into the caller's flat ``out``; later calls of the same shape
    class with tile 0 take the fastest. Returns (tile, ms per call)."""
    boxes, cb = _boxes_c(boxes)
    prec = _lib.PRECISIONS[precision]
    canon = _canon(F, coef, rowmax=rowmax)
    dtype = torch.float64 if prec == _lib.LS_F64 else torch.float32
    _out_tensor(out, dtype, sum(max(b[3], 0) * max(b[4], 0) * max(b[5], 0) for b in boxes),
                F[0].device)
    ws, nws = _recon_ws(canon, prec, F[0].device, _ws_tensor(ws, F[0].device))
    t, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    check("ls_reconstruct_autotune",
          lib().ls_reconstruct_autotune(ctypes.byref(canon), cb, len(boxes), float(scale), prec,
                                        _ptr(out), _ptr(ws), nws, int(reps), _stream(),
                                        ctypes.byref(t), ctypes.byref(ms)))
    return int(t.value), float(ms.value)


def reconstruct_tuned_tile(F, coef, boxes, precision="f64", ws_bytes=None):
    """(tile, ms) the autotuner chose for this shape class, (0, 0.0) if none.
    ``ws_bytes``: the workspace the calls pass (None: as ``reconstruct``
    allocates it)."""
    boxes, cb = _boxes_c(boxes)
    prec = _lib.PRECISIONS[precision]
    canon = _canon(F, coef)
    need = int(lib().ls_reconstruct_workspace(ctypes.byref(canon), prec))
    nws = need if ws_bytes is None else int(ws_bytes)
    t, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    check("ls_reconstruct_tuned_tile",
          lib().ls_reconstruct_tuned_tile(ctypes.byref(canon), cb, len(boxes), prec,
                                          ctypes.c_void_p(1 if nws > 0 else 0), nws,
                                          ctypes.byref(t), ctypes.byref(ms)))
    return int(t.value), float(ms.value)



def reconstruct_f16_plan(F, coef, boxes, ws):
    """The FP16x3 preparation held in ``ws`` (made by ``reconstruct_prepare``
    on the same factors) and the work of reconstructing ``boxes`` from it:
    dict with ``perm`` (int32, slot s -> the caller's rank), ``masks``
    (uint32 per plane of axis 0, bit c: rank chunk c runs there) and
    ``chunk_values`` (sum over the boxes' values of the chunks their plane
    runs). Synchronizes the device."""
    import numpy as np
    boxes, cb = _boxes_c(boxes)
    canon = _canon(F, coef)
    ws = _ws_tensor(ws, F[0].device)
    if ws is None:
        raise ValueError("the workspace of reconstruct_prepare is required")
    torch.cuda.synchronize(F[0].device)
    K, n0 = int(F[0].shape[0]), int(F[0].shape[1])
    perm = np.zeros(K, np.int32)
    masks = np.zeros(n0, np.uint32)
    cv = ctypes.c_int64(0)
    check("ls_reconstruct_f16_plan",
          lib().ls_reconstruct_f16_plan(ctypes.byref(canon), cb, len(boxes), _ptr(ws),
                                        ws.numel() * ws.element_size(),
                                        perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                        ctypes.byref(cv)))
    return {"perm": perm, "masks": masks, "chunk_values": int(cv.value)}

def energy(F, coef, D, d, precision="f64", ws=None):
    """E = <P, rho> (eq. scal) as a device scalar tensor."""
    cP, cR = _canon(F, coef), _canon(D, d, "density")
    K, Krho = int(F[0].shape[0]), int(D[0].shape[0])
    need = int(lib().ls_energy_workspace(K, Krho))
    ws = _ws_tensor(ws, F[0].device)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=F[0].device)
    E = torch.empty((), dtype=torch.float64, device=F[0].device)
    check("ls_energy", lib().ls_energy(ctypes.byref(cP), ctypes.byref(cR),
                                       _lib.PRECISIONS[precision], _ptr(E), _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream()))
    return E


def forces(lat, quad, pos, Z, D, d, precision="f64", ws=None):
    """(F [M0][3], E) with F = -dE/dpos, by the adjoint of the assembled sums."""
    pos = _pos_tensor(pos)
    M0 = pos.shape[0]
    Z = _charges(Z, M0)
    cR = _canon(D, d, "density")
    need = int(lib().ls_forces_workspace(ctypes.byref(lat.c()), M0, quad.R, int(D[0].shape[0])))
    ws = _ws_tensor(ws, pos.device)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=pos.device)
    F = torch.empty((M0, 3), dtype=torch.float64, device=pos.device)
    E = torch.empty((), dtype=torch.float64, device=pos.device)
    check("ls_forces", lib().ls_forces(ctypes.byref(lat.c()), ctypes.byref(quad.c()), M0, _ptr(pos),
                                       _ptr(Z), ctypes.byref(cR),
                                       _lib.PRECISIONS[precision], _ptr(F), _ptr(E), _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream()))
    return F, E


def qtt_compress(X, eps, cap=None):
    """Quantics-TT compression of the rows of X ([nvec][len] float64 device,
    e.g. an assembled factor matrix): (cores [nvec][cap] float64, ranks
    [nvec][d+1] int32, status [nvec] int32); see ls_qtt_compress."""
    X = _dev_f64(X, "X")
    if X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous [nvec][len] matrix")
    nvec, length = int(X.shape[0]), int(X.shape[1])
    d = int(lib().ls_qtt_digits(length))
    if cap is None:
        cap = 8192
    cores = torch.empty((nvec, cap), dtype=torch.float64, device=X.device)
    ranks = torch.empty((nvec, d + 1), dtype=torch.int32, device=X.device)
    status = torch.empty(nvec, dtype=torch.int32, device=X.device)
    check("ls_qtt_compress", lib().ls_qtt_compress(_ptr(X), nvec, length, length, float(eps), int(cap),
                                                   _ptr(cores), _ptr(ranks), _ptr(status), _stream()))
    return cores, ranks, status


def qtt_expand(cores, ranks, status, length):
    """The vectors [nvec][length] that QTT cores represent (NaN rows where the
    compression failed)."""
    for name, t, dt in (("cores", cores, torch.float64), ("ranks", ranks, torch.int32),
                        ("status", status, torch.int32)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {dt} device tensor")
    nvec, cap = int(cores.shape[0]), int(cores.shape[1])
    d = int(lib().ls_qtt_digits(int(length)))
    if tuple(ranks.shape) != (nvec, d + 1) or status.numel() != nvec:
        raise ValueError("ranks must be [nvec][d+1] and status [nvec]")
    Y = torch.empty((nvec, int(length)), dtype=torch.float64, device=cores.device)
    check("ls_qtt_expand", lib().ls_qtt_expand(_ptr(cores), _ptr(ranks), _ptr(status), nvec,
                                               int(length), cap, _ptr(Y), int(length), _stream()))
    return Y


def combine(FA, ca, alpha, FB, cb, beta):
    """alpha A + beta B as one canonical tensor (eq. conc): factors [A; B]."""
    cA, cB = _canon(FA, ca, "A"), _canon(FB, cb, "B")
    Kt = int(FA[0].shape[0] + FB[0].shape[0])
    dev = FA[0].device
    F = [torch.empty((Kt, int(FA[l].shape[1])), dtype=torch.float64, device=dev) for l in range(3)]
    coef = torch.empty(Kt, dtype=torch.float64, device=dev)
    check("ls_canon_combine", lib().ls_canon_combine(ctypes.byref(cA), float(alpha),
                                                     ctypes.byref(cB), float(beta),
                                                     _ptr(F[0]), _ptr(F[1]), _ptr(F[2]), _ptr(coef),
                                                     _stream()))
    return F, coef


def richardson(lat, quad, pos, Z, order="linear"):
    """Richardson-regularised periodic sum on the reference cell (Sec. 3.2):
    the assembled periodic tensors at L and 2L combined as 2 P_L - P_2L
    (``linear``) or (4 P_L - P_2L)/3 (``quadratic``), in canonical form."""
    if order not in ("linear", "quadratic"):
        raise ValueError("order must be 'linear' or 'quadratic'")
    pos = _pos_tensor(pos)
    M0 = pos.shape[0]
    Z = _charges(Z, M0)
    K2 = 2 * M0 * quad.R
    dev = pos.device
    F = [torch.empty((K2, lat.n), dtype=torch.float64, device=dev) for _ in range(3)]
    coef = torch.empty(K2, dtype=torch.float64, device=dev)
    check("ls_richardson", lib().ls_richardson(ctypes.byref(lat.c()), ctypes.byref(quad.c()), M0,
                                               _ptr(pos), _ptr(Z), 1 if order == "linear" else 2,
                                               _ptr(F[0]), _ptr(F[1]), _ptr(F[2]), _ptr(coef),
                                               _stream()))
    return F, coef


def nuclear_matrix(F, coef, g, ws=None):
    """V[k][m] = <G_k (.) G_m, P> (eq. nuc_pot) for rank-one basis functions
    with samples g[l] (device [Nb][N_l])."""
    cP = _canon(F, coef)
    K, Nb = int(F[0].shape[0]), int(g[0].shape[0])
    for l, x in enumerate(g):
        _dev_f64(x, f"basis samples [{l}]")
        if tuple(x.shape) != (Nb, int(F[l].shape[1])):
            raise ValueError(f"basis samples [{l}] must have shape {(Nb, int(F[l].shape[1]))}")
    need = int(lib().ls_nuclear_workspace(K, Nb))
    ws = _ws_tensor(ws, F[0].device)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=F[0].device)
    V = torch.empty((Nb, Nb), dtype=torch.float64, device=F[0].device)
    check("ls_nuclear_matrix", lib().ls_nuclear_matrix(ctypes.byref(cP), Nb, _ptr(g[0]),
                                                       _ptr(g[1]), _ptr(g[2]), _ptr(V), _ptr(ws),
                                                       ws.numel() * ws.element_size(), _stream()))
    return V


class LatticeEnergy(torch.autograd.Function):
    """E(pos) = <P(pos), rho> with the hand-written adjoint as its gradient.

    forward(pos, Z, D0, D1, D2, d, lat, quad, precision) -> E (0-d tensor).
    The forward pass runs ls_forces, which yields E and -dE/dpos together;
    backward returns grad_E * dE/dpos for ``pos`` and None elsewhere.
    """

    @staticmethod
    def forward(ctx, pos, Z, D0, D1, D2, d, lat, quad, precision):
        F, E = forces(lat, quad, pos.detach().contiguous(), Z, [D0, D1, D2], d, precision)
        ctx.save_for_backward(F)
        return E

    @staticmethod
    def backward(ctx, gE):
        (F,) = ctx.saved_tensors
        return (-F * gE, None, None, None, None, None, None, None, None)


def lattice_energy(pos, Z, D, d, lat, quad, precision="f64"):
    return LatticeEnergy.apply(pos, Z, D[0], D[1], D[2], d, lat, quad, precision)


class Batch:
    """Many box lattice systems in one persistent launch (graph replay).

    ``systems``: list of dicts with keys lat (LatticeSpec), quad (QuadTable),
    pos, Z (device float64), D (three device tensors [R_rho][N_l]), d (device
    [R_rho]) and box (o0, o1, o2, e0, e1, e2), extent at most one unit cell per
    axis. Outputs: ``self.out[i]`` ([e0][e1][e2] cell averages) and
    ``self.E[i]`` (energy), both device tensors filled by ``run``.
    """

    def __init__(self, systems, precision="f32"):
        self.precision = precision
        prec = _lib.PRECISIONS[precision]
        dtype = torch.float64 if prec == _lib.LS_F64 else torch.float32
        dev = systems[0]["pos"].device
        self._keep = []
        self.out, self.E = [], []
        arr = (System * len(systems))()
        for i, sy in enumerate(systems):
            b = [int(v) for v in sy["box"]]
            out = torch.empty((b[3], b[4], b[5]), dtype=dtype, device=dev)
            E = torch.empty((), dtype=torch.float64, device=dev)
            self.out.append(out)
            self.E.append(E)
            q = sy["quad"]
            self._keep.append((q, sy["pos"], sy["Z"], sy["D"], sy["d"]))
            arr[i].lat = sy["lat"].c()
            arr[i].quad = q.c()
            arr[i].M0 = int(sy["pos"].shape[0])
            pos_i = _pos_tensor(sy["pos"])
            arr[i].pos = pos_i.data_ptr()
            arr[i].Z = _charges(sy["Z"], int(pos_i.shape[0])).data_ptr()
            arr[i].rho = _canon(sy["D"], sy["d"])
            arr[i].box = Box((ctypes.c_int32 * 3)(*b[:3]), (ctypes.c_int32 * 3)(*b[3:]))
            arr[i].out = out.data_ptr()
            arr[i].E = E.data_ptr()
        self._handle = ctypes.c_void_p(0)
        ws = ctypes.c_size_t(0)
        check("ls_batch_create", lib().ls_batch_create(arr, len(systems), prec,
                                                       ctypes.byref(self._handle), ctypes.byref(ws)))
        self.ws = torch.empty(int(ws.value), dtype=torch.uint8, device=dev)
        self.count = len(systems)

    def run(self, tile=0):
        check("ls_batch_run", lib().ls_batch_run(self._handle, _ptr(self.ws), self.ws.numel(),
                                                 int(tile), _stream()))

    def autotune(self):
        t = ctypes.c_int32(0)
        ms = ctypes.c_double(0.0)
        check("ls_batch_autotune", lib().ls_batch_autotune(self._handle, _ptr(self.ws), self.ws.numel(),
                                                           _stream(), ctypes.byref(t), ctypes.byref(ms)))
        return t.value, ms.value

    def tuned_tile(self):
        """(tile, ms) of this batch's shape class in the autotune cache ((0, 0.0)
        if it has none)."""
        t = ctypes.c_int32(0)
        ms = ctypes.c_double(0.0)
        check("ls_batch_tuned_tile", lib().ls_batch_tuned_tile(self._handle, ctypes.byref(t),
                                                               ctypes.byref(ms)))
        return t.value, ms.value

    def report(self, phases=False):
        """(per-system seconds, error flag) of the last completed run; with
        ``phases`` also the spans of the folding, vector and tile phases."""
        torch.cuda.synchronize()
        sec = np.zeros(self.count)
        ph = np.zeros(3)
        err = ctypes.c_int32(0)
        check("ls_batch_report", lib().ls_batch_report(self._handle, _ptr(self.ws),
                                                       sec.ctypes.data_as(_lib.c_double_p),
                                                       ph.ctypes.data_as(_lib.c_double_p),
                                                       ctypes.byref(err)))
        if phases:
            return sec, int(err.value), ph
        return sec, int(err.value)

    def close(self):
        if self._handle:
            torch.cuda.synchronize()
            lib().ls_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_cache_file(path):
    """Name the autotune cache file of the batches (None: in-process only):
    loads its entries and writes new ones there."""
    check("ls_batch_cache_file", lib().ls_batch_cache_file(
        None if path is None else os.fsencode(path)))


def probe_copy(src, dst):
    """Plain device copy of src into dst (reference kernel for the HBM roofline)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    check("ls_probe_copy", lib().ls_probe_copy(_ptr(src), _ptr(dst), nbytes, _stream()))


def probe_mfma(precision, blocks, iters, out, shape=0):
    """MFMA issue loop (reference kernel for the matrix-core roofline); returns
    the floating-point operations of the launch. out: float32, blocks*256.
    shape 0: 16x16 instructions, 1: 32x32."""
    if out.dtype != torch.float32 or out.numel() < blocks * 256:
        raise ValueError("out must be float32 with blocks*256 elements")
    flops = ctypes.c_double(0.0)
    check("ls_probe_mfma", lib().ls_probe_mfma(_lib.PRECISIONS[precision], int(shape), int(blocks),
                                               int(iters), _ptr(out), ctypes.byref(flops),
                                               _stream()))
    return flops.value
