"""ctypes binding of libmera.so (include/mera.h).

Argument marshalling only: every numerical step runs in the HIP library.  The
library is loaded from this package directory (or from the path in the environment
variable MERA_LIBRARY, e.g. the sanitizer build); if it is missing, loading it raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MERA_LIBRARY") or os.path.join(HERE, "libmera.so")

MERA_OK, MERA_EINVAL, MERA_ESHAPE, MERA_EWORKSPACE, MERA_EDEVICE, MERA_ENUMERIC, MERA_ENOTCONV = range(7)
MERA_LEFT, MERA_RIGHT, MERA_AVG = 0, 1, 2
MERA_FP64, MERA_FP32, MERA_BF16X3 = 0, 1, 2
(MERA_OP_ASCEND, MERA_OP_DESCEND, MERA_OP_ENV_U, MERA_OP_ENV_W, MERA_OP_POLAR,
 MERA_OP_FIXED_POINT, MERA_OP_ENERGY, MERA_OP_TREE_ASCEND, MERA_OP_TREE_DESCEND,
 MERA_OP_TREE_ENV_W, MERA_OP_POLAR_NEAR) = range(11)

EXPORTED = (
    "mera_ascend", "mera_descend", "mera_env_u", "mera_env_w", "mera_polar_update",
    "mera_fixed_point_rho", "mera_energy", "mera_tfim_hamiltonian", "mera_workspace_bytes",
    "mera_strerror", "mera_last_error", "mera_flops", "mera_profile_begin", "mera_profile_end",
    "mera_workspace_bytes_min", "mera_mfma_peak", "mera_contract", "mera_schedule_plan",
    "mera_descend_noalloc", "mera_tree_descend", "mera_tree_ascend", "mera_tree_env_w",
    "mera_polar_update_near",
)


class MeraLayer(ctypes.Structure):
    _fields_ = [("din", ctypes.c_int32), ("dout", ctypes.c_int32),
                ("u_d", ctypes.c_void_p), ("w_d", ctypes.c_void_p)]


class MeraProfileEntry(ctypes.Structure):
    _fields_ = [("step", ctypes.c_char * 48), ("arith", ctypes.c_int32), ("op", ctypes.c_int32),
                ("flops", ctypes.c_double), ("ms", ctypes.c_double)]


class MeraError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libmera.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1906_12030_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    lp = ctypes.POINTER(MeraLayer)
    lib.mera_ascend.argtypes = [lp, vp, vp, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    lib.mera_descend.argtypes = [lp, vp, vp, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    lib.mera_descend_noalloc.argtypes = [lp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    for name in ("mera_tree_descend", "mera_tree_ascend"):
        getattr(lib, name).argtypes = [i32, i32, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, sz, vp]
        getattr(lib, name).restype = ctypes.c_int
    lib.mera_tree_env_w.argtypes = [i32, i32, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    lib.mera_tree_env_w.restype = ctypes.c_int
    lib.mera_descend_noalloc.restype = ctypes.c_int
    lib.mera_env_u.argtypes = [lp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    lib.mera_env_w.argtypes = [lp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    lib.mera_polar_update.argtypes = [vp, i64, i64, vp, vp, vp, sz, vp]
    lib.mera_polar_update_near.argtypes = [vp, vp, i64, i64, dbl, vp, vp, vp, sz, vp]
    lib.mera_fixed_point_rho.argtypes = [lp, vp, i32, dbl, ctypes.c_int, vp, vp, sz, vp]
    lib.mera_energy.argtypes = [vp, vp, i64, vp, vp]
    lib.mera_tfim_hamiltonian.argtypes = [dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.mera_workspace_bytes.argtypes = [ctypes.c_int, i32, i32, ctypes.c_int, ctypes.c_int]
    lib.mera_workspace_bytes.restype = sz
    lib.mera_workspace_bytes_min.argtypes = [ctypes.c_int, i32, i32, ctypes.c_int, ctypes.c_int]
    lib.mera_workspace_bytes_min.restype = sz
    lib.mera_flops.argtypes = [ctypes.c_int, i32, i32, ctypes.c_int]
    lib.mera_flops.restype = dbl
    lib.mera_strerror.argtypes = [ctypes.c_int]
    lib.mera_strerror.restype = ctypes.c_char_p
    lib.mera_last_error.argtypes = []
    lib.mera_last_error.restype = ctypes.c_char_p
    lib.mera_contract.argtypes = [ctypes.c_char_p, vp, ctypes.c_char_p, vp, ctypes.c_char_p, vp,
                                  ctypes.c_char_p, ctypes.POINTER(i64), dbl, dbl, ctypes.c_int, vp, sz, vp]
    lib.mera_contract.restype = ctypes.c_int
    lib.mera_mfma_peak.argtypes = [ctypes.c_int, vp, sz, ctypes.POINTER(dbl)]
    lib.mera_mfma_peak.restype = ctypes.c_int
    lib.mera_schedule_plan.argtypes = [ctypes.c_int, i32, i32, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, sz,
                                       ctypes.POINTER(sz)]
    lib.mera_schedule_plan.restype = ctypes.c_int
    lib.mera_profile_begin.argtypes = []
    lib.mera_profile_begin.restype = ctypes.c_int
    lib.mera_profile_end.argtypes = [ctypes.POINTER(MeraProfileEntry), i32, ctypes.POINTER(i32)]
    lib.mera_profile_end.restype = ctypes.c_int
    for name in ("mera_ascend", "mera_descend", "mera_env_u", "mera_env_w", "mera_polar_update",
                 "mera_polar_update_near", "mera_fixed_point_rho", "mera_energy",
                 "mera_tfim_hamiltonian"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != MERA_OK:
        lib = load()
        detail = lib.mera_strerror(status).decode()
        last = lib.mera_last_error().decode()
        raise MeraError(status, where, f"{detail} ({last})" if last else detail)


def mera_descend_noalloc(layer, rho_in_d, rho_out_d, placement, precision, stream):
    return load().mera_descend_noalloc(ctypes.byref(layer), rho_in_d, rho_out_d, placement, precision, stream)


def mera_tree_descend(din, dout, w_d, rho_in_d, rho_out_d, placement, precision, ws_d, ws_bytes, stream):
    return load().mera_tree_descend(din, dout, w_d, rho_in_d, rho_out_d, placement, precision, ws_d, ws_bytes,
                                    stream)


def mera_tree_ascend(din, dout, w_d, h_in_d, h_out_d, placement, precision, ws_d, ws_bytes, stream):
    return load().mera_tree_ascend(din, dout, w_d, h_in_d, h_out_d, placement, precision, ws_d, ws_bytes, stream)


def mera_tree_env_w(din, dout, w_d, h_d, rho_d, env_d, placement, precision, ws_d, ws_bytes, stream):
    return load().mera_tree_env_w(din, dout, w_d, h_d, rho_d, env_d, placement, precision, ws_d, ws_bytes,
                                  stream)


def mera_ascend(layer, h_in_d, h_out_d, placement, precision, ws_d, ws_bytes, stream):
    return load().mera_ascend(ctypes.byref(layer), h_in_d, h_out_d, placement, precision, ws_d, ws_bytes, stream)


def mera_descend(layer, rho_in_d, rho_out_d, placement, precision, ws_d, ws_bytes, stream):
    return load().mera_descend(ctypes.byref(layer), rho_in_d, rho_out_d, placement, precision, ws_d, ws_bytes, stream)


def mera_env_u(layer, h_d, rho_d, env_d, placement, precision, ws_d, ws_bytes, stream):
    return load().mera_env_u(ctypes.byref(layer), h_d, rho_d, env_d, placement, precision, ws_d, ws_bytes, stream)


def mera_env_w(layer, h_d, rho_d, env_d, placement, precision, ws_d, ws_bytes, stream):
    return load().mera_env_w(ctypes.byref(layer), h_d, rho_d, env_d, placement, precision, ws_d, ws_bytes, stream)


def mera_polar_update(env_d, rows, cols, out_d, sv_d, ws_d, ws_bytes, stream):
    return load().mera_polar_update(env_d, rows, cols, out_d, sv_d, ws_d, ws_bytes, stream)


def mera_polar_update_near(env_d, prev_d, rows, cols, tie, out_d, sv_d, ws_d, ws_bytes, stream):
    return load().mera_polar_update_near(env_d, prev_d, rows, cols, tie, out_d, sv_d, ws_d, ws_bytes,
                                         stream)


def mera_fixed_point_rho(layer, rho_d, iters, tol, precision, resid_d, ws_d, ws_bytes, stream):
    return load().mera_fixed_point_rho(ctypes.byref(layer), rho_d, iters, float(tol), precision, resid_d,
                                       ws_d, ws_bytes, stream)


def mera_energy(h_d, rho_d, n, e_d, stream):
    return load().mera_energy(h_d, rho_d, n, e_d, stream)


def mera_tfim_hamiltonian(field):
    h = (ctypes.c_double * 64)()
    c = ctypes.c_double(0.0)
    st = load().mera_tfim_hamiltonian(field, h, ctypes.byref(c))
    return st, list(h), c.value


def mera_workspace_bytes(op, din, dout, precision, placement):
    return int(load().mera_workspace_bytes(op, din, dout, precision, placement))


def mera_workspace_bytes_min(op, din, dout, precision, placement):
    return int(load().mera_workspace_bytes_min(op, din, dout, precision, placement))


def mera_flops(op, din, dout, placement):
    return float(load().mera_flops(op, din, dout, placement))


def mera_contract(la, a_ptr, lb, b_ptr, lc, c_ptr, labels, sizes, alpha, beta, precision, ws, ws_bytes, stream):
    arr = (ctypes.c_int64 * len(sizes))(*sizes)
    return load().mera_contract(la.encode(), a_ptr, lb.encode(), b_ptr, lc.encode(), c_ptr, labels.encode(),
                                arr, alpha, beta, precision, ws, ws_bytes, stream)


def mera_mfma_peak(kind, scratch_ptr, scratch_bytes):
    """(status, TFLOP/s) of the matrix-core microbenchmark (0 bf16, 1 f32, 2 f64)."""
    t = ctypes.c_double(0.0)
    st = load().mera_mfma_peak(kind, scratch_ptr, scratch_bytes, ctypes.byref(t))
    return st, float(t.value)


def mera_profile_begin():
    return load().mera_profile_begin()


def mera_profile_end(max_entries=200000):
    buf = (MeraProfileEntry * max_entries)()
    n = ctypes.c_int32(0)
    st = load().mera_profile_end(buf, max_entries, ctypes.byref(n))
    return st, [(buf[i].step.decode(), int(buf[i].arith), float(buf[i].flops), float(buf[i].ms),
                 int(buf[i].op)) for i in range(n.value)]


def mera_schedule_plan(op, din, dout, precision, placement):
    """(status, [lines]) of the contraction schedule with the kernel chosen for each step."""
    need = ctypes.c_size_t(0)
    lib = load()
    st = lib.mera_schedule_plan(op, din, dout, precision, placement, None, 0, ctypes.byref(need))
    if st != MERA_OK:
        return st, []
    buf = ctypes.create_string_buffer(need.value)
    st = lib.mera_schedule_plan(op, din, dout, precision, placement, buf, need.value, None)
    return st, [ln for ln in buf.value.decode().split("\n") if ln]
