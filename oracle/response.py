"""Linear response at a wavevector q (oracle; test infrastructure only).

Sec. 2.3: the perturbed wavefunctions live on the k+q spheres, so the
perturbing potential takes a function of the k sphere to the k+q sphere, and
the induced density of Eq. drho pairs a function of the k sphere with one of
the k+q sphere on the real-space mesh.

* ``dv_cross_matrix``: the plain definition of the local perturbation between
  the two spheres, L[G', G] = dV~[(m_G' - m_G) mod N] with dV~ the forward
  transform of the lattice-periodic part dV(r) of the perturbation (Eq.
  fwFFT); dV u = L u.
* ``dv_psi_realspace``: the same by the steps of Sec. 2.2.2 and Sec. 4 --
  scatter u_k onto the mesh, inverse transform, multiply by dV(r), forward
  transform, gather on the k+q sphere.
* ``dfpt_rhs_q``: -(1 - S P_v^{k+q}) dV u_k (Eq. linear_system with dS = 0,
  P_v^{k+q} from the S-orthonormal occupied states at k+q).
* ``drho``: Eq. drho without the augmentation term,
  drho(r) = 4 sum_k w_k sum_nu conj(u_k nu(r)) du_k nu(r),
  with u(r) = sum_G u(G) exp(2 pi i m_G . l / N) (the inverse transform of
  Sec. 4, no normalisation) and du the solution of the linear system on the
  k+q sphere (already in the conduction manifold, so P_c du = du).
"""
from __future__ import annotations

import numpy as np

from . import basis, dft


def dv_cross_matrix(miller_out: np.ndarray, miller_in: np.ndarray, fft, dvt: np.ndarray) -> np.ndarray:
    """L[G', G] = dV~[(m_G' - m_G) mod N] for G' on the output sphere, G on the input one."""
    d = miller_out[:, None, :] - miller_in[None, :, :]
    d = np.mod(d, np.asarray(fft, dtype=np.int64))
    return dvt[d[..., 0], d[..., 1], d[..., 2]]


def dv_psi_realspace(miller_out, miller_in, fft, dv_r, u_in) -> np.ndarray:
    """dV u for (nbnd, npw_in) rows through the real-space mesh, (nbnd, npw_out)."""
    gi = basis.grid_index(miller_in, fft)
    go = basis.grid_index(miller_out, fft)
    out = np.empty((u_in.shape[0], miller_out.shape[0]), dtype=np.complex128)
    for b in range(u_in.shape[0]):
        box = np.zeros(tuple(fft), dtype=np.complex128)
        box[gi[:, 0], gi[:, 1], gi[:, 2]] = u_in[b]
        c = dft.forward(np.asarray(dv_r) * dft.inverse(box))
        out[b] = c[go[:, 0], go[:, 1], go[:, 2]]
    return out


def dfpt_rhs_q(dvu_kq: np.ndarray, u_occ_kq: np.ndarray, s_kq: np.ndarray | None = None) -> np.ndarray:
    """rhs_nu = -(1 - S P_v) dV u_nu for dvu_kq given as (npw_kq, nocc) columns."""
    su = u_occ_kq if s_kq is None else s_kq @ u_occ_kq
    return -(dvu_kq - su @ (u_occ_kq.conj().T @ dvu_kq))


def to_mesh(miller: np.ndarray, fft, rows: np.ndarray) -> np.ndarray:
    """Rows (nbnd, npw) of plane-wave coefficients -> (nbnd, N1, N2, N3) real-space values."""
    g = basis.grid_index(miller, fft)
    out = np.empty((rows.shape[0],) + tuple(fft), dtype=np.complex128)
    for b in range(rows.shape[0]):
        box = np.zeros(tuple(fft), dtype=np.complex128)
        box[g[:, 0], g[:, 1], g[:, 2]] = rows[b]
        out[b] = dft.inverse(box)
    return out


def drho(fft, weights, miller_k, u_k, miller_kq, du_kq) -> np.ndarray:
    """Eq. drho (no augmentation term) on the mesh: 4 sum_k w_k sum_nu conj(u(r)) du(r).

    miller_k[i], u_k[i] (nocc, npw_k) and miller_kq[i], du_kq[i] (nocc, npw_kq) per k-point i."""
    out = np.zeros(tuple(fft), dtype=np.complex128)
    for w, mk, uk, mq, dq in zip(weights, miller_k, u_k, miller_kq, du_kq):
        a = to_mesh(mk, fft, uk)
        b = to_mesh(mq, fft, dq)
        out += 4.0 * w * np.sum(a.conj() * b, axis=0)
    return out
