"""ctypes binding of liblatsum.so (argument marshalling only).

The library is loaded from this package directory; there is no fallback: if
it is missing or fails to load, every call raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblatsum.so")

LS_OK, LS_EINVAL, LS_EHIP, LS_EUNSUPPORTED, LS_EWORKSPACE = 0, -1, -2, -3, -4
LS_F64, LS_F32, LS_BF16X3, LS_BF16X6, LS_F16X3 = 0, 1, 2, 3, 4
LS_RULE_U, LS_RULE_S = 0, 1

PRECISIONS = {"f64": LS_F64, "f32": LS_F32, "bf16x3": LS_BF16X3, "bf16x6": LS_BF16X6,
              "f16x3": LS_F16X3}

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)


class Lattice(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("L", ctypes.c_int32 * 3), ("b", ctypes.c_double),
                ("periodic", ctypes.c_int32)]


class Quad(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("t", c_double_p), ("w", c_double_p)]


class Canon(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("len", ctypes.c_int32 * 3),
                ("f", ctypes.c_void_p * 3), ("coef", ctypes.c_void_p), ("rowmax", ctypes.c_void_p)]


class TensorLattice(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("b", ctypes.c_double), ("N", ctypes.c_int32 * 3),
                ("L", ctypes.c_int32 * 3), ("s", ctypes.c_void_p * 3)]


class Box(ctypes.Structure):
    _fields_ = [("o", ctypes.c_int32 * 3), ("e", ctypes.c_int32 * 3)]


class System(ctypes.Structure):
    _fields_ = [("lat", Lattice), ("quad", Quad), ("M0", ctypes.c_int32),
                ("pos", ctypes.c_void_p), ("Z", ctypes.c_void_p), ("rho", Canon), ("box", Box),
                ("out", ctypes.c_void_p), ("E", ctypes.c_void_p)]


class LatsumError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


_LIB = None

_SIGNATURES = {
    "ls_version": (ctypes.c_char_p, []),
    "ls_last_error": (ctypes.c_char_p, []),
    "ls_quadrature": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     c_double_p, c_double_p, ctypes.c_int32, c_int32_p]),
    "ls_master_halfwidth": (ctypes.c_int, [ctypes.POINTER(Lattice), c_int32_p]),
    "ls_kernel_vectors": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.POINTER(Quad), ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "ls_assemble": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.POINTER(Quad), ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ls_assemble_tensor": (ctypes.c_int, [ctypes.POINTER(TensorLattice), ctypes.POINTER(Quad),
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ls_reconstruct": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.POINTER(Box), ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p]),
    "ls_reconstruct_prepared": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.POINTER(Box), ctypes.c_int32,
                                               ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                               ctypes.c_void_p]),
    "ls_reconstruct_prepare": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_size_t, ctypes.c_void_p]),
    "ls_reconstruct_workspace": (ctypes.c_size_t, [ctypes.POINTER(Canon), ctypes.c_int32]),
    "ls_reconstruct_tiles": (ctypes.c_int32, [ctypes.c_int32]),
    "ls_reconstruct_autotune": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.POINTER(Box), ctypes.c_int32,
                                               ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_double)]),
    "ls_reconstruct_tuned_tile": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.POINTER(Box), ctypes.c_int32,
                                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                                 ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_double)]),
    "ls_reconstruct_f16_plan": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.POINTER(Box), ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_size_t, c_int32_p,
                                               ctypes.POINTER(ctypes.c_uint32),
                                               ctypes.POINTER(ctypes.c_int64)]),
    "ls_energy_workspace": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "ls_energy": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.POINTER(Canon), ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "ls_forces_workspace": (ctypes.c_size_t, [ctypes.POINTER(Lattice), ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32]),
    "ls_forces": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.POINTER(Quad), ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Canon),
                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_size_t, ctypes.c_void_p]),
    "ls_forces_noalloc": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.POINTER(Quad), ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Canon),
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "ls_richardson": (ctypes.c_int, [ctypes.POINTER(Lattice), ctypes.POINTER(Quad), ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "ls_canon_combine": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.c_double, ctypes.POINTER(Canon),
                                        ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ls_qtt_digits": (ctypes.c_int32, [ctypes.c_int32]),
    "ls_qtt_compress": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ls_qtt_expand": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p]),
    "ls_nuclear_workspace": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "ls_nuclear_matrix": (ctypes.c_int, [ctypes.POINTER(Canon), ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "ls_batch_create": (ctypes.c_int, [ctypes.POINTER(System), ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_size_t)]),
    "ls_batch_tiles": (ctypes.c_int32, []),
    "ls_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                    ctypes.c_void_p]),
    "ls_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p, c_int32_p, c_double_p]),
    "ls_batch_cache_file": (ctypes.c_int, [ctypes.c_char_p]),
    "ls_batch_tuned_tile": (ctypes.c_int, [ctypes.c_void_p, c_int32_p, c_double_p]),
    "ls_batch_report": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, c_double_p, c_double_p,
                                       c_int32_p]),
    "ls_batch_destroy": (None, [ctypes.c_void_p]),
    "ls_probe_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p]),
    "ls_probe_mfma": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_void_p, c_double_p, ctypes.c_void_p]),
}

EXPORTS = tuple(_SIGNATURES)


def lib():
    """The loaded library (raises if liblatsum.so is missing)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1405_2270_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = handle
    return _LIB


def check(fn_name, status):
    if status != LS_OK:
        msg = lib().ls_last_error().decode(errors="replace")
        raise LatsumError(fn_name, status, msg)
