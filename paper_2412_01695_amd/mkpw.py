"""ctypes binding of libmkpw.so (the C-ABI declared in include/mkpw.h).

Argument marshalling only: each ``pw_*`` function here calls the C function of
the same name; device arrays are passed as raw pointers (torch tensors on
the GPU, or integers), host arrays as numpy buffers.  Every status other
than PW_OK raises ``PwError`` carrying the library's message, except
PW_ENOCONV from the solvers, which is returned so the caller can read the
per-system flags.  The library must have been built
(``python -m paper_2412_01695_amd.build``); importing this module without it
raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MKPW_LIB selects another build of the same library (e.g. an instrumented one)
LIB_PATH = os.environ.get("MKPW_LIB") or os.path.join(_HERE, "libmkpw.so")

PW_OK, PW_EINVAL, PW_ENOMEM, PW_EDEVICE, PW_ENOCONV, PW_ESTATE = 0, -1, -2, -3, -4, -5
PW_FP64, PW_MIXED = 0, 1
STATUS_NAMES = {0: "PW_OK", -1: "PW_EINVAL", -2: "PW_ENOMEM", -3: "PW_EDEVICE", -4: "PW_ENOCONV",
                -5: "PW_ESTATE"}

EXPORTS = ["pw_create", "pw_destroy", "pw_last_error", "pw_set_option", "pw_get_option", "pw_set_lattice", "pw_set_cutoff",
           "pw_set_kpoints", "pw_get_miller", "pw_set_vloc", "pw_set_projectors", "pw_set_qij", "pw_init_guess",
           "pw_h_psi", "pw_s_psi", "pw_davidson", "pw_dfpt_cg", "pw_dfpt_rhs", "pw_drho"]

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2412_01695_amd.build`")

# PyTorch ships its own HIP/HSA runtime with the same SONAME (libamdhip64.so.7)
# as the system ROCm the library is linked against.  Loading the library first
# would map both runtimes into the process, and device memory and streams from
# torch would then be used through a second, independent runtime.  Importing
# torch first makes the library bind to the runtime torch already loaded.
try:
    import torch as _torch  # noqa: F401
except ImportError:  # host-only use without torch: the system runtime is the only one
    _torch = None
_lib = C.CDLL(LIB_PATH)

_vp, _i, _d, _i64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
_pd, _pi = C.POINTER(C.c_double), C.POINTER(C.c_int32)
_sig = {
    "pw_create": (_i, [C.POINTER(_vp), _i, _vp]),
    "pw_destroy": (None, [_vp]),
    "pw_last_error": (C.c_char_p, [_vp]),
    "pw_set_option": (_i, [_vp, C.c_char_p, _i64]),
    "pw_get_option": (_i, [_vp, C.c_char_p, C.POINTER(_i64)]),
    "pw_set_lattice": (_i, [_vp, _pd]),
    "pw_set_cutoff": (_i, [_vp, _d, _pi]),
    "pw_set_kpoints": (_i, [_vp, _i, _pd, _pi, _pi]),
    "pw_get_miller": (_i, [_vp, _i, _pi]),
    "pw_set_vloc": (_i, [_vp, _pd]),
    "pw_set_projectors": (_i, [_vp, _i, _vp, _vp]),
    "pw_set_qij": (_i, [_vp, _vp]),
    "pw_init_guess": (_i, [_vp, _i, C.c_uint64, _vp]),
    "pw_h_psi": (_i, [_vp, _i, _i, _vp, _vp]),
    "pw_s_psi": (_i, [_vp, _i, _i, _vp, _vp]),
    "pw_davidson": (_i, [_vp, _i, _i, _vp, _pd, _d, _i, _pi, _pi]),
    "pw_dfpt_cg": (_i, [_vp, _i, _i, _vp, _pd, _pd, _i, _vp, _vp, _d, _i, _pi]),
    "pw_dfpt_rhs": (_i, [_vp, _vp, _i, _vp, _vp, _vp, _vp]),
    "pw_drho": (_i, [_vp, _vp, _i, _pd, _vp, _vp, _vp]),
}
for _n, (_r, _a) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _r
    _f.argtypes = _a


class PwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(x):
    """Device pointer of a torch tensor / int, or host pointer of a numpy array."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take a pointer of {type(x)}")


def _dbl(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_pd)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_pi)


def _check(ctx, st, allow_noconv=False):
    if st == PW_OK or (allow_noconv and st == PW_ENOCONV):
        return st
    msg = _lib.pw_last_error(ctx).decode(errors="replace") if ctx else ""
    raise PwError(st, msg)


def pw_create(hip_device: int = 0, hip_stream=None):
    h = _vp()
    st = _lib.pw_create(C.byref(h), int(hip_device), _vp(hip_stream) if hip_stream else None)
    if st != PW_OK:
        raise PwError(st, "pw_create failed")
    return h


def pw_destroy(ctx):
    _lib.pw_destroy(ctx)


def pw_last_error(ctx) -> str:
    return _lib.pw_last_error(ctx).decode(errors="replace")


def pw_set_option(ctx, key: str, value: int):
    return _check(ctx, _lib.pw_set_option(ctx, key.encode(), int(value)))


def pw_get_option(ctx, key: str) -> int:
    v = C.c_int64(0)
    _check(ctx, _lib.pw_get_option(ctx, key.encode(), C.byref(v)))
    return int(v.value)


def pw_set_lattice(ctx, a):
    a, p = _dbl(np.asarray(a).reshape(9))
    return _check(ctx, _lib.pw_set_lattice(ctx, p))


def pw_set_cutoff(ctx, ecut_ry: float, fft=(0, 0, 0)):
    f, p = _i32(np.asarray(fft).reshape(3))
    return _check(ctx, _lib.pw_set_cutoff(ctx, float(ecut_ry), p))


def pw_set_kpoints(ctx, k_cart):
    k, p = _dbl(np.asarray(k_cart).reshape(-1, 3))
    nk = k.shape[0]
    npw = np.zeros(nk, dtype=np.int32)
    npwx = np.zeros(1, dtype=np.int32)
    _check(ctx, _lib.pw_set_kpoints(ctx, nk, p, npw.ctypes.data_as(_pi), npwx.ctypes.data_as(_pi)))
    return npw, int(npwx[0])


def pw_get_miller(ctx, ik: int, npw: int):
    m = np.zeros((npw, 3), dtype=np.int32)
    _check(ctx, _lib.pw_get_miller(ctx, int(ik), m.ctypes.data_as(_pi)))
    return m


def pw_get_miller_all(ctx, npw):
    """Every k's Miller list, concatenated (sum(npw), 3)."""
    m = np.zeros((int(np.sum(npw)), 3), dtype=np.int32)
    _check(ctx, _lib.pw_get_miller(ctx, -1, m.ctypes.data_as(_pi)))
    return m


def pw_init_guess(ctx, nbnd: int, seed: int, psi):
    return _check(ctx, _lib.pw_init_guess(ctx, int(nbnd), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(psi)))


def pw_set_vloc(ctx, v_r):
    v, p = _dbl(v_r)
    return _check(ctx, _lib.pw_set_vloc(ctx, p))


def pw_set_projectors(ctx, beta, dij):
    """beta: host complex128 (nk, nproj, npwx); dij: host complex128 (nproj, nproj)."""
    beta = np.ascontiguousarray(beta, dtype=np.complex128)
    dij = np.ascontiguousarray(dij, dtype=np.complex128)
    nproj = beta.shape[1] if beta.ndim == 3 else 0
    return _check(ctx, _lib.pw_set_projectors(ctx, nproj, beta.ctypes.data if nproj else None,
                                              dij.ctypes.data if nproj else None))


def pw_set_qij(ctx, qij):
    """qij: host complex128 (nproj, nproj), or None to remove the overlap."""
    if qij is None:
        return _check(ctx, _lib.pw_set_qij(ctx, None))
    q = np.ascontiguousarray(qij, dtype=np.complex128)
    return _check(ctx, _lib.pw_set_qij(ctx, q.ctypes.data))


def pw_h_psi(ctx, prec: int, nbnd: int, psi, hpsi):
    return _check(ctx, _lib.pw_h_psi(ctx, int(prec), int(nbnd), _ptr(psi), _ptr(hpsi)))


def pw_s_psi(ctx, prec: int, nbnd: int, psi, spsi):
    return _check(ctx, _lib.pw_s_psi(ctx, int(prec), int(nbnd), _ptr(psi), _ptr(spsi)))


def pw_davidson(ctx, prec: int, nbnd: int, psi, nk: int, tol_ry: float, max_iter: int):
    """Returns (status, eig (nk, nbnd) Ha, iters (nk), converged (nk))."""
    eig = np.zeros((nk, nbnd), dtype=np.float64)
    iters = np.zeros(nk, dtype=np.int32)
    conv = np.zeros(nk, dtype=np.int32)
    st = _lib.pw_davidson(ctx, int(prec), int(nbnd), _ptr(psi), eig.ctypes.data_as(_pd), float(tol_ry),
                          int(max_iter), iters.ctypes.data_as(_pi), conv.ctypes.data_as(_pi))
    _check(ctx, st, allow_noconv=True)
    return st, eig, iters, conv


def pw_dfpt_cg(ctx, prec: int, nocc: int, psi_occ, eps_ha, alpha_ha, nrhs: int, rhs, dpsi, thr: float,
               max_iter: int):
    """Returns (status, iters (nk*nrhs))."""
    eps, pe = _dbl(eps_ha)
    alpha, pa = _dbl(alpha_ha)
    iters = np.zeros(eps.size, dtype=np.int32)
    st = _lib.pw_dfpt_cg(ctx, int(prec), int(nocc), _ptr(psi_occ), pe, pa, int(nrhs), _ptr(rhs), _ptr(dpsi),
                         float(thr), int(max_iter), iters.ctypes.data_as(_pi))
    _check(ctx, st, allow_noconv=True)
    return st, iters


def pw_dfpt_rhs(ctx_kq, ctx_k, nocc: int, dv_r, psi_k, psi_occ_kq, rhs):
    """dv_r: host complex (N1, N2, N3); device arrays as torch tensors or pointers."""
    dv = np.ascontiguousarray(dv_r, dtype=np.complex128)
    return _check(ctx_kq, _lib.pw_dfpt_rhs(ctx_kq, ctx_k, int(nocc), dv.ctypes.data, _ptr(psi_k), _ptr(psi_occ_kq),
                                           _ptr(rhs)))


def pw_drho(ctx_kq, ctx_k, nbnd: int, wk, psi_k, dpsi_kq, drho_r):
    w, pw = _dbl(wk)
    return _check(ctx_kq, _lib.pw_drho(ctx_kq, ctx_k, int(nbnd), pw, _ptr(psi_k), _ptr(dpsi_kq), _ptr(drho_r)))
