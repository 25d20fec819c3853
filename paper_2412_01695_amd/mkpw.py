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
           "pw_h_psi", "pw_h_psi_noalloc", "pw_s_psi", "pw_davidson", "pw_dfpt_cg", "pw_dfpt_rhs", "pw_drho"]

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
    "pw_h_psi_noalloc": (_i, [_vp, _i, _i, _vp, _vp]),
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


def _dims(ctx):
    """The context's sizes as the library reports them (nk, npwx, nproj, mesh)."""
    g = lambda k: pw_get_option(ctx, k)
    return {"nk": g("nk"), "npwx": g("npwx"), "nproj": g("nproj"), "fft": (g("fft1"), g("fft2"), g("fft3"))}


_C128, _C64 = "complex128", "complex64"


def _dev(x, name, shape, dtype):
    """Check a device array before its pointer crosses the ABI: a torch tensor
    must live on the GPU, be contiguous and have exactly this dtype and shape.
    A bare integer is taken as a raw device pointer that the caller vouches
    for (nothing can be checked)."""
    if isinstance(x, int):
        return x
    if not hasattr(x, "data_ptr"):
        raise TypeError(f"{name}: expected a device tensor or a raw pointer, got {type(x).__name__}")
    if getattr(x, "device", None) is None or x.device.type != "cuda":
        raise ValueError(f"{name}: must be a GPU tensor (got device {getattr(x, 'device', None)})")
    if str(x.dtype).replace("torch.", "") != dtype:
        raise ValueError(f"{name}: dtype must be {dtype}, got {str(x.dtype).replace('torch.', '')}")
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name}: shape must be {tuple(shape)}, got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return x.data_ptr()


def _host(a, name, shape, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.size != int(np.prod(shape)):
        raise ValueError(f"{name}: expected {int(np.prod(shape))} values {tuple(shape)}, got {a.size}")
    return a


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
    _npw_of.pop(getattr(ctx, "value", None), None)
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
    _npw_of.pop(ctx.value, None)  # the basis is reset
    a, p = _dbl(np.asarray(a).reshape(9))
    return _check(ctx, _lib.pw_set_lattice(ctx, p))


def pw_set_cutoff(ctx, ecut_ry: float, fft=(0, 0, 0)):
    f, p = _i32(np.asarray(fft).reshape(3))
    return _check(ctx, _lib.pw_set_cutoff(ctx, float(ecut_ry), p))


# npw per k-point of each context whose k-points were set through this module
# (keyed by the context's address), so that the Miller read-backs are sized by
# what the library will write, not by what the caller says
_npw_of = {}


def pw_set_kpoints(ctx, k_cart):
    k, p = _dbl(np.asarray(k_cart).reshape(-1, 3))
    nk = k.shape[0]
    npw = np.zeros(nk, dtype=np.int32)
    npwx = np.zeros(1, dtype=np.int32)
    _npw_of.pop(ctx.value, None)
    _check(ctx, _lib.pw_set_kpoints(ctx, nk, p, npw.ctypes.data_as(_pi), npwx.ctypes.data_as(_pi)))
    _npw_of[ctx.value] = npw.copy()
    return npw, int(npwx[0])


def _known_npw(ctx):
    npw = _npw_of.get(ctx.value)
    if npw is None or npw.size != _dims(ctx)["nk"]:
        raise ValueError("the context's k-points were not set through this binding; their basis sizes are unknown")
    return npw


def pw_get_miller(ctx, ik: int, npw: int | None = None):
    """Miller indices (npw[ik], 3) of k-point ik; npw, if given, must match."""
    known = _known_npw(ctx)
    if not 0 <= int(ik) < known.size:
        raise ValueError(f"ik = {ik} outside [0, {known.size})")
    if npw is not None and int(npw) != int(known[ik]):
        raise ValueError(f"npw = {npw} but k-point {ik} has {int(known[ik])} plane waves")
    m = np.zeros((int(known[ik]), 3), dtype=np.int32)
    _check(ctx, _lib.pw_get_miller(ctx, int(ik), m.ctypes.data_as(_pi)))
    return m


def pw_get_miller_all(ctx, npw=None):
    """Every k's Miller list, concatenated (sum(npw), 3); npw, if given, must match."""
    known = _known_npw(ctx)
    if npw is not None and not np.array_equal(np.asarray(npw), known):
        raise ValueError("npw does not match the context's basis sizes")
    m = np.zeros((int(np.sum(known)), 3), dtype=np.int32)
    _check(ctx, _lib.pw_get_miller(ctx, -1, m.ctypes.data_as(_pi)))
    return m


def _rows(ctx, nvec):
    d = _dims(ctx)
    return (d["nk"], int(nvec), d["npwx"])


def _wf(prec):
    return _C128 if int(prec) == PW_FP64 else _C64


def pw_init_guess(ctx, nbnd: int, seed: int, psi):
    """psi: device complex128 (nk, nbnd, npwx)."""
    p = _dev(psi, "psi", _rows(ctx, nbnd), _C128)
    return _check(ctx, _lib.pw_init_guess(ctx, int(nbnd), int(seed) & 0xFFFFFFFFFFFFFFFF, p))


def pw_set_vloc(ctx, v_r):
    """v_r: host real (N1, N2, N3), Ha."""
    v, p = _dbl(_host(v_r, "v_r", _dims(ctx)["fft"], np.float64))
    return _check(ctx, _lib.pw_set_vloc(ctx, p))


def pw_set_projectors(ctx, beta, dij):
    """beta: host complex128 (nk, nproj, npwx); dij: host complex128 (nproj, nproj)."""
    beta = np.ascontiguousarray(beta, dtype=np.complex128)
    dij = np.ascontiguousarray(dij, dtype=np.complex128)
    nproj = beta.shape[1] if beta.ndim == 3 else 0
    if nproj:
        d = _dims(ctx)
        if beta.shape != (d["nk"], nproj, d["npwx"]):
            raise ValueError(f"beta: shape must be ({d['nk']}, nproj, {d['npwx']}), got {beta.shape}")
        if dij.shape != (nproj, nproj):
            raise ValueError(f"dij: shape must be ({nproj}, {nproj}), got {dij.shape}")
    return _check(ctx, _lib.pw_set_projectors(ctx, nproj, beta.ctypes.data if nproj else None,
                                              dij.ctypes.data if nproj else None))


def pw_set_qij(ctx, qij):
    """qij: host complex128 (nproj, nproj), or None to remove the overlap."""
    if qij is None:
        return _check(ctx, _lib.pw_set_qij(ctx, None))
    n = _dims(ctx)["nproj"]
    q = np.ascontiguousarray(qij, dtype=np.complex128)
    if n:  # without projectors the library refuses the call (PW_ESTATE) before reading q
        q = _host(q, "qij", (n, n), np.complex128)
    return _check(ctx, _lib.pw_set_qij(ctx, q.ctypes.data))


def pw_h_psi(ctx, prec: int, nbnd: int, psi, hpsi):
    """psi, hpsi: device (nk, nbnd, npwx), complex128 (PW_FP64) or complex64 (PW_MIXED)."""
    shape, dt = _rows(ctx, nbnd), _wf(prec)
    p, h = _dev(psi, "psi", shape, dt), _dev(hpsi, "hpsi", shape, dt)
    return _check(ctx, _lib.pw_h_psi(ctx, int(prec), int(nbnd), p, h))


def pw_h_psi_noalloc(ctx, prec: int, nbnd: int, psi, hpsi):
    """pw_h_psi without any device allocation (fixed staging array per GPU)."""
    shape, dt = _rows(ctx, nbnd), _wf(prec)
    p, h = _dev(psi, "psi", shape, dt), _dev(hpsi, "hpsi", shape, dt)
    return _check(ctx, _lib.pw_h_psi_noalloc(ctx, int(prec), int(nbnd), p, h))


def pw_s_psi(ctx, prec: int, nbnd: int, psi, spsi):
    """psi, spsi: device (nk, nbnd, npwx), complex128 (PW_FP64) or complex64 (PW_MIXED)."""
    shape, dt = _rows(ctx, nbnd), _wf(prec)
    p, s = _dev(psi, "psi", shape, dt), _dev(spsi, "spsi", shape, dt)
    return _check(ctx, _lib.pw_s_psi(ctx, int(prec), int(nbnd), p, s))


def pw_davidson(ctx, prec: int, nbnd: int, psi, nk: int | None, tol_ry: float, max_iter: int):
    """psi: device complex128 (nk, nbnd, npwx), guess in, eigenvectors out.
    nk, if given, must be the context's k-point count.
    Returns (status, eig (nk, nbnd) Ha, iters (nk), converged (nk))."""
    shape = _rows(ctx, nbnd)
    if nk is not None and int(nk) != shape[0]:
        raise ValueError(f"nk = {nk} but the context holds {shape[0]} k-points")
    nk = shape[0]
    p = _dev(psi, "psi", shape, _C128)
    eig = np.zeros((nk, nbnd), dtype=np.float64)
    iters = np.zeros(nk, dtype=np.int32)
    conv = np.zeros(nk, dtype=np.int32)
    st = _lib.pw_davidson(ctx, int(prec), int(nbnd), p, eig.ctypes.data_as(_pd), float(tol_ry),
                          int(max_iter), iters.ctypes.data_as(_pi), conv.ctypes.data_as(_pi))
    _check(ctx, st, allow_noconv=True)
    return st, eig, iters, conv


def pw_dfpt_cg(ctx, prec: int, nocc: int, psi_occ, eps_ha, alpha_ha, nrhs: int, rhs, dpsi, thr: float,
               max_iter: int):
    """psi_occ: device complex128 (nk, nocc, npwx); eps_ha: host (nk, nrhs);
    alpha_ha: host (nk); rhs, dpsi: device complex128 (nk, nrhs, npwx).
    Returns (status, iters (nk*nrhs))."""
    nk = _dims(ctx)["nk"]
    eps, pe = _dbl(_host(eps_ha, "eps_ha", (nk, nrhs), np.float64))
    alpha, pa = _dbl(_host(alpha_ha, "alpha_ha", (nk,), np.float64))
    pu = _dev(psi_occ, "psi_occ", _rows(ctx, nocc), _C128)
    pr = _dev(rhs, "rhs", _rows(ctx, nrhs), _C128)
    px = _dev(dpsi, "dpsi", _rows(ctx, nrhs), _C128)
    iters = np.zeros(nk * int(nrhs), dtype=np.int32)
    st = _lib.pw_dfpt_cg(ctx, int(prec), int(nocc), pu, pe, pa, int(nrhs), pr, px, float(thr), int(max_iter),
                         iters.ctypes.data_as(_pi))
    _check(ctx, st, allow_noconv=True)
    return st, iters


def pw_dfpt_rhs(ctx_kq, ctx_k, nocc: int, dv_r, psi_k, psi_occ_kq, rhs):
    """dv_r: host complex (N1, N2, N3); psi_k: device complex128 (nk, nocc,
    npwx_k); psi_occ_kq, rhs: device complex128 (nk, nocc, npwx_kq)."""
    dv = _host(dv_r, "dv_r", _dims(ctx_kq)["fft"], np.complex128)
    pk = _dev(psi_k, "psi_k", _rows(ctx_k, nocc), _C128)
    pq = _dev(psi_occ_kq, "psi_occ_kq", _rows(ctx_kq, nocc), _C128)
    pr = _dev(rhs, "rhs", _rows(ctx_kq, nocc), _C128)
    return _check(ctx_kq, _lib.pw_dfpt_rhs(ctx_kq, ctx_k, int(nocc), dv.ctypes.data, pk, pq, pr))


def pw_drho(ctx_kq, ctx_k, nbnd: int, wk, psi_k, dpsi_kq, drho_r):
    """wk: host (nk); psi_k: device complex128 (nk, nbnd, npwx_k); dpsi_kq:
    device complex128 (nk, nbnd, npwx_kq); drho_r: device complex128 (N1, N2, N3)."""
    d = _dims(ctx_kq)
    w, pw = _dbl(_host(wk, "wk", (d["nk"],), np.float64))
    pk = _dev(psi_k, "psi_k", _rows(ctx_k, nbnd), _C128)
    pq = _dev(dpsi_kq, "dpsi_kq", _rows(ctx_kq, nbnd), _C128)
    pd = _dev(drho_r, "drho_r", d["fft"], _C128)
    return _check(ctx_kq, _lib.pw_drho(ctx_kq, ctx_k, int(nbnd), pw, pk, pq, pd))
