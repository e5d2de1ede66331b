"""ctypes binding of libtetmf.so (argument marshalling only).

The library must have been built for gfx950 (paper_2404_08371_amd.build);
loading fails loudly when it is missing -- there is no fallback path.
"""
import ctypes
import os
import sys

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtetmf.so")
_LIB = None

c_i64p = ctypes.POINTER(ctypes.c_int64)
c_dp = ctypes.POINTER(ctypes.c_double)
c_u8p = ctypes.POINTER(ctypes.c_uint8)
c_vp = ctypes.c_void_p
c_int = ctypes.c_int
c_i64 = ctypes.c_int64

# (name, restype, argtypes); the order matches include/tetmf.h
SIGNATURES = [
    ("tmf_version", ctypes.c_char_p, []),
    ("tmf_last_error", ctypes.c_char_p, []),
    ("tmf_status_string", ctypes.c_char_p, [c_int]),
    ("tmf_mesh_create", c_int, [c_dp, c_i64, c_i64p, c_i64, c_int, c_int, ctypes.POINTER(c_vp)]),
    ("tmf_mesh_destroy", None, [c_vp]),
    ("tmf_mesh_layout", c_int, [c_vp, c_int, c_i64p, c_i64p]),
    ("tmf_mesh_dof_info", c_int, [c_vp, c_int, c_i64p, c_dp, c_u8p, c_u8p]),
    ("tmf_op_create", c_int, [c_vp, c_int, c_int, c_int, c_dp, c_dp, c_int, ctypes.POINTER(c_vp)]),
    ("tmf_op_destroy", None, [c_vp]),
    ("tmf_op_info", c_int, [c_vp, c_i64p, c_i64p, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    ("tmf_apply", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("tmf_apply_adjoint", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("tmf_apply_timed", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("tmf_apply_noalloc", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("tmf_apply_local", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("tmf_interface_sum", c_int, [c_vp, c_vp, c_vp]),
    ("tmf_diagonal", c_int, [c_vp, c_vp, c_vp, c_vp]),
    ("tmf_op_store_matrices", c_int, [c_vp, c_vp, c_vp]),
    ("tmf_apply_stored", c_int, [c_vp, c_vp, c_vp, c_vp]),
    ("tmf_op_num_tiles", c_int, [c_vp, ctypes.POINTER(c_int)]),
    ("tmf_op_tile_shape", c_int, [c_vp, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                  ctypes.POINTER(c_int)]),
    ("tmf_op_set_tile", c_int, [c_vp, c_int]),
    ("tmf_op_get_tile", c_int, [c_vp, ctypes.POINTER(c_int)]),
    ("tmf_op_autotune", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(c_int),
                                ctypes.POINTER(ctypes.c_float)]),
    ("tmf_op_tune", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_int, ctypes.c_char_p, ctypes.POINTER(c_int),
                            ctypes.POINTER(ctypes.c_float)]),
    ("tmf_batch_create", c_int, [ctypes.POINTER(c_vp), c_int, ctypes.POINTER(c_vp)]),
    ("tmf_batch_destroy", None, [c_vp]),
    ("tmf_batch_info", c_int, [c_vp, ctypes.POINTER(c_int), c_i64p]),
    ("tmf_batch_apply", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("tmf_batch_apply_timed", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("tmf_batch_diagonal", c_int, [c_vp, c_vp, c_vp, c_vp]),
    ("tmf_batch_set_tile", c_int, [c_vp, c_int]),
    ("tmf_batch_autotune", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(c_int),
                                   ctypes.POINTER(ctypes.c_float)]),
    ("tmf_batch_tune", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_int, ctypes.c_char_p, ctypes.POINTER(c_int),
                               ctypes.POINTER(ctypes.c_float)]),
    ("tmf_ir_create", c_int, [c_vp, c_vp, c_vp, ctypes.POINTER(c_vp)]),
    ("tmf_ir_destroy", None, [c_vp]),
    ("tmf_ir_solve", c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(ctypes.c_double), c_vp]),
]

OPTIONAL = set()


class TetmfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("tetmf error %d (%s): %s" % (status, STATUS.get(status, "?"), msg))
        self.status = status


STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "device error",
          -4: "unsupported", -5: "not converged"}


def path():
    return _PATH


def lib():
    global _LIB
    if _LIB is None:
        # PyTorch ships its own HIP runtime with the same SONAME; loading it
        # first makes the library bind to that single runtime instance, so
        # torch streams, events and allocations are valid handles for it.
        import torch  # noqa: F401
        if not os.path.exists(_PATH):
            raise RuntimeError("libtetmf.so is not built (%s); run `python -m paper_2404_08371_amd.build`"
                               % _PATH)
        L = ctypes.CDLL(_PATH)
        for name, res, args in SIGNATURES:
            if name in OPTIONAL and not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(status):
    if status != 0:
        msg = lib().tmf_last_error().decode(errors="replace")
        raise TetmfError(status, msg)
    return status


def release(handle, destroy_name):
    """Destroy a library handle; skipped while the interpreter shuts down
    (the HIP runtime and this module's globals may already be gone)."""
    try:
        if handle is None or not handle.value or sys.is_finalizing() or _LIB is None:
            return
        getattr(_LIB, destroy_name)(handle)
    except (AttributeError, TypeError, ImportError):
        pass
