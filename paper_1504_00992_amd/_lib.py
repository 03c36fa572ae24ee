"""ctypes binding of libtebd_rrsvd.so (argument marshalling only).

Every entry point of include/tebd_rrsvd.h is exposed under the same name.
The functions here only turn torch tensors into device pointers and the
current torch stream into a hipStream_t; all arithmetic of the bond update
runs in the library's HIP kernels.  If the library is missing or cannot be
loaded, every call raises: there is no CPU fallback.
"""
import ctypes
import os

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libtebd_rrsvd.so")

TEBD_OK = 0
TEBD_ERR_ARG = 1
TEBD_ERR_SHAPE = 2
TEBD_ERR_WORKSPACE = 3
TEBD_ERR_DEVICE = 4

DEV_NONFINITE = 1
DEV_QR_FALLBACK = 2
DEV_JACOBI_NOCONV = 4
DEV_LAMBDA_FLOOR = 8
DEV_CHI_BOUND = 16
DEV_BAD_STATE = 32
DEV_RANK_RETRY = 64

EXPORTED = ("tebd_last_error", "tebd_version", "tebd_workspace_size", "rrsvd_truncate",
            "tebd_bond_update", "tebd_sweep", "tebd_adjoint_workspace_size", "tebd_tape_size", "tebd_sweep_record",
            "tebd_sweep_adjoint", "tebd_profile_enable", "tebd_profile_read", "tebd_size_class",
            "rrsvd_truncate_noalloc", "tebd_tune_set", "tebd_tune_get")


class TebdParams(ctypes.Structure):
    _fields_ = [("chi_max", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("trunc_eps", ctypes.c_double),
                ("lambda_floor", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("stream_id", ctypes.c_uint32), ("adaptive", ctypes.c_int32)]


class TebdMps(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int32), ("n_sites", ctypes.c_int32),
                ("d_max", ctypes.c_int32), ("chi_max", ctypes.c_int32),
                ("d", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
                ("lambda_", ctypes.c_void_p), ("chi", ctypes.c_void_p)]


class TebdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"tebd status {status}: {message}")
        self.status = status


_lib = None


def load():
    """Load the shared library once; raise if it is absent or broken."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1504_00992_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    pp = ctypes.POINTER(ctypes.c_void_p)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    lib.tebd_last_error.restype = ctypes.c_char_p
    lib.tebd_last_error.argtypes = []
    lib.tebd_version.restype = ctypes.c_char_p
    lib.tebd_version.argtypes = []
    lib.tebd_workspace_size.restype = ctypes.c_int
    lib.tebd_workspace_size.argtypes = [ctypes.POINTER(TebdMps), i64, pi64, pi64,
                                        ctypes.POINTER(TebdParams), ctypes.POINTER(sz)]
    lib.rrsvd_truncate.restype = ctypes.c_int
    lib.rrsvd_truncate.argtypes = [i64, pi64, pi64, pp, pi64, pp, ctypes.POINTER(TebdParams),
                                   pp, i64, pp, pp, i64, vp, vp, vp, vp, sz, vp]
    lib.rrsvd_truncate_noalloc.restype = ctypes.c_int
    lib.rrsvd_truncate_noalloc.argtypes = [i64, pi64, pi64, pp, pi64, pp,
                                           ctypes.POINTER(TebdParams), pp, i64, pp, pp, i64, vp,
                                           vp, vp, vp]
    lib.tebd_bond_update.restype = ctypes.c_int
    lib.tebd_bond_update.argtypes = [ctypes.POINTER(TebdMps), i32, i32, vp,
                                     ctypes.POINTER(TebdParams), vp, vp, vp, sz, vp]
    lib.tebd_sweep.restype = ctypes.c_int
    lib.tebd_sweep.argtypes = [ctypes.POINTER(TebdMps), vp, i64, i32, ctypes.POINTER(TebdParams),
                               vp, vp, vp, sz, vp]
    lib.tebd_adjoint_workspace_size.restype = ctypes.c_int
    lib.tebd_adjoint_workspace_size.argtypes = [ctypes.POINTER(TebdMps), ctypes.POINTER(TebdParams),
                                                ctypes.POINTER(sz)]
    lib.tebd_tape_size.restype = ctypes.c_int
    lib.tebd_tape_size.argtypes = [ctypes.POINTER(TebdMps), ctypes.POINTER(TebdParams),
                                   ctypes.POINTER(sz)]
    lib.tebd_sweep_record.restype = ctypes.c_int
    lib.tebd_sweep_record.argtypes = [ctypes.POINTER(TebdMps), vp, i64, i32,
                                      ctypes.POINTER(TebdParams), vp, vp, vp, sz, vp, sz, vp]
    lib.tebd_sweep_adjoint.restype = ctypes.c_int
    lib.tebd_sweep_adjoint.argtypes = [ctypes.POINTER(TebdMps), vp, i64, i32,
                                       ctypes.POINTER(TebdParams), vp, sz, vp, vp, vp, vp, vp, sz,
                                       vp]
    lib.tebd_profile_enable.restype = ctypes.c_int
    lib.tebd_profile_enable.argtypes = [i32]
    lib.tebd_profile_read.restype = ctypes.c_int
    lib.tebd_profile_read.argtypes = [i32, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.tebd_size_class.restype = ctypes.c_int32
    lib.tebd_size_class.argtypes = [i32, i32, i32]
    lib.tebd_tune_set.restype = ctypes.c_int
    lib.tebd_tune_set.argtypes = [i32, i32, i32, i32]
    lib.tebd_tune_get.restype = ctypes.c_int32
    lib.tebd_tune_get.argtypes = [i32, i32, i32]
    _lib = lib
    return lib


def check(status):
    if status != TEBD_OK:
        raise TebdError(status, load().tebd_last_error().decode())
    return status


def params(chi_max, p=10, q=2, trunc_eps=1e-10, lambda_floor=1e-14, seed=1504, stream_id=0,
           precision=0, adaptive=0):
    return TebdParams(int(chi_max), int(p), int(q), int(precision), float(trunc_eps),
                      float(lambda_floor), int(seed), int(stream_id) & 0xFFFFFFFF, int(adaptive))


def _i64_array(values):
    arr = (ctypes.c_int64 * len(values))(*[int(v) for v in values])
    return arr


def _ptr_array(values):
    return (ctypes.c_void_p * len(values))(*[int(v) if v is not None else None for v in values])


def tebd_last_error():
    return load().tebd_last_error().decode()


def tebd_version():
    return load().tebd_version().decode()


def tebd_workspace_size(prm, mps=None, m=None, n=None):
    """Raw call: bytes of workspace (mps: TebdMps or None; m, n: int lists)."""
    lib = load()
    out = ctypes.c_size_t(0)
    if mps is not None:
        check(lib.tebd_workspace_size(ctypes.byref(mps), 0, None, None, ctypes.byref(prm),
                                      ctypes.byref(out)))
    else:
        check(lib.tebd_workspace_size(None, len(m), _i64_array(m), _i64_array(n),
                                      ctypes.byref(prm), ctypes.byref(out)))
    return out.value


def rrsvd_truncate(m, n, a_ptrs, lda, omega_ptrs, prm, u_ptrs, ldu, s_ptrs, vh_ptrs, ldvh,
                   chi_kept_ptr, disc_ptr, status_ptr, ws_ptr, ws_bytes, stream):
    """Raw call with integer device addresses (lists for per-problem pointers)."""
    lib = load()
    batch = len(m)
    om = _ptr_array(omega_ptrs) if omega_ptrs is not None else None
    return lib.rrsvd_truncate(batch, _i64_array(m), _i64_array(n), _ptr_array(a_ptrs),
                              _i64_array(lda), om, ctypes.byref(prm), _ptr_array(u_ptrs), int(ldu),
                              _ptr_array(s_ptrs), _ptr_array(vh_ptrs), int(ldvh), chi_kept_ptr,
                              disc_ptr, status_ptr, ws_ptr, int(ws_bytes), stream)


def rrsvd_truncate_noalloc(m, n, a_ptrs, lda, omega_ptrs, prm, u_ptrs, ldu, s_ptrs, vh_ptrs,
                           ldvh, chi_kept_ptr, disc_ptr, status_ptr, stream):
    """Raw call of the no-allocation variant (static scratch, no workspace)."""
    lib = load()
    om = _ptr_array(omega_ptrs) if omega_ptrs is not None else None
    return lib.rrsvd_truncate_noalloc(len(m), _i64_array(m), _i64_array(n), _ptr_array(a_ptrs),
                                      _i64_array(lda), om, ctypes.byref(prm), _ptr_array(u_ptrs),
                                      int(ldu), _ptr_array(s_ptrs), _ptr_array(vh_ptrs),
                                      int(ldvh), chi_kept_ptr, disc_ptr, status_ptr, stream)


def tebd_bond_update(mps, chain, bond, gate_ptr, prm, disc_ptr, status_ptr, ws_ptr, ws_bytes,
                     stream):
    lib = load()
    return lib.tebd_bond_update(ctypes.byref(mps), int(chain), int(bond), gate_ptr,
                                ctypes.byref(prm), disc_ptr, status_ptr, ws_ptr, int(ws_bytes),
                                stream)


def tebd_sweep(mps, gates_ptr, gate_chain_stride, parity, prm, disc_ptr, status_ptr, ws_ptr,
               ws_bytes, stream):
    lib = load()
    return lib.tebd_sweep(ctypes.byref(mps), gates_ptr, int(gate_chain_stride), int(parity),
                          ctypes.byref(prm), disc_ptr, status_ptr, ws_ptr, int(ws_bytes), stream)


def tebd_adjoint_workspace_size(mps, prm):
    out = ctypes.c_size_t(0)
    check(load().tebd_adjoint_workspace_size(ctypes.byref(mps), ctypes.byref(prm),
                                             ctypes.byref(out)))
    return out.value


def tebd_tape_size(mps, prm):
    out = ctypes.c_size_t(0)
    check(load().tebd_tape_size(ctypes.byref(mps), ctypes.byref(prm), ctypes.byref(out)))
    return out.value


def tebd_sweep_record(mps, gates_ptr, gate_chain_stride, parity, prm, disc_ptr, status_ptr,
                      tape_ptr, tape_bytes, ws_ptr, ws_bytes, stream):
    return load().tebd_sweep_record(ctypes.byref(mps), gates_ptr, int(gate_chain_stride),
                                    int(parity), ctypes.byref(prm), disc_ptr, status_ptr, tape_ptr,
                                    int(tape_bytes), ws_ptr, int(ws_bytes), stream)


def tebd_sweep_adjoint(mps_in, gates_ptr, gate_chain_stride, parity, prm, tape_ptr, tape_bytes,
                       gamma_bar_ptr, lambda_bar_ptr, gate_bar_ptr, status_ptr, ws_ptr, ws_bytes,
                       stream):
    return load().tebd_sweep_adjoint(ctypes.byref(mps_in), gates_ptr, int(gate_chain_stride),
                                     int(parity), ctypes.byref(prm), tape_ptr, int(tape_bytes),
                                     gamma_bar_ptr, lambda_bar_ptr, gate_bar_ptr, status_ptr,
                                     ws_ptr, int(ws_bytes), stream)


def tebd_profile_enable(on):
    check(load().tebd_profile_enable(1 if on else 0))


def tebd_tune_set(precision, max_rows, width, variant):
    """Set one autotune-cache entry (tile variant of the sketch products)."""
    return int(load().tebd_tune_set(int(precision), int(max_rows), int(width), int(variant)))


def tebd_tune_get(precision, max_rows, width):
    return int(load().tebd_tune_get(int(precision), int(max_rows), int(width)))


def tebd_size_class(factorization, rows, l):
    """Size class (kernel) of a QR (factorization 0) or small SVD (1)."""
    return int(load().tebd_size_class(int(factorization), int(rows), int(l)))


def tebd_profile_read(capacity=96):
    """{kind: (milliseconds, launches)} recorded since profiling was enabled."""
    lib = load()
    names = (ctypes.c_char_p * capacity)()
    ms = (ctypes.c_double * capacity)()
    launches = (ctypes.c_int64 * capacity)()
    count = ctypes.c_int32(0)
    check(lib.tebd_profile_read(capacity, names, ms, launches, ctypes.byref(count)))
    return {names[i].decode(): (ms[i], int(launches[i])) for i in range(count.value)}
