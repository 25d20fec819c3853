"""Kohn-Sham Hamiltonian and overlap on the plane-wave basis (oracle; test
infrastructure only).

Sec. 2.2: H = kinetic + local + nonlocal.
  kinetic   C'(G) = (1/2)|k+G|^2 C(G)                         (Sec. 2.2.1)
  local     C -> inverse FFT -> multiply by V(r) -> forward FFT
            with the 1/N_r factor on the forward transform      (Sec. 2.2.2)
  nonlocal  lambda_n = sum_G beta_n(k+G)^* C(G)                (Eq. lambdah)
            gamma_m  = sum_n D_mn lambda_n                      (Eq. gamma)
            V_NL C   = sum_m gamma_m beta_m(k+G)                (Eq. finalnl)

Two independent routes are provided:
  * ``dense_h`` writes the matrix out.  Substituting the two transforms of
    Sec. 4 into the local step gives sum_G' V~[(m_G - m_G') mod N] C(G') with
    V~ = forward transform of V(r); the nonlocal step is the rank-nproj
    matrix beta D beta^H.  H|psi> is then H_k psi.
  * ``h_psi_realspace`` follows the steps above literally for each band,
    with the naive separable DFT of ``oracle.dft``.
Both agree for any mesh on which G -> m mod N is one-to-one.

Sec. 2.2 (overlap) and Sec. 2.2.3: S = 1 + sum_mn q_mn |beta_m><beta_n|,
applied from the same projections as the nonlocal term
  delta_m = sum_n q_mn lambda_n                                  (Eq. delta_eq)
  S C     = C + sum_m delta_m beta_m(k+G)                         (Eq. finals)
``overlap_matrix`` writes S_k out; ``s_psi_projections`` follows the two
equations literally.  With no q the overlap is the identity.
"""
from __future__ import annotations

import numpy as np

from . import basis, dft


def vtilde(v_r: np.ndarray) -> np.ndarray:
    """Fourier coefficients of the real-space potential, Eq. fwFFT."""
    return dft.forward(np.asarray(v_r, dtype=np.float64))


def local_matrix(miller: np.ndarray, fft, vt: np.ndarray) -> np.ndarray:
    """L[G, G'] = V~[(m_G - m_G') mod N]."""
    d = miller[:, None, :] - miller[None, :, :]
    n = np.asarray(fft, dtype=np.int64)
    d = np.mod(d, n)
    return vt[d[..., 0], d[..., 1], d[..., 2]]


def nonlocal_matrix(beta: np.ndarray, dij: np.ndarray) -> np.ndarray:
    """N[G, G'] = sum_mn beta_m(G) D_mn beta_n(G')^*  (beta is (nproj, npw))."""
    return beta.T @ dij @ beta.conj()


def overlap_matrix(beta: np.ndarray, qij) -> np.ndarray:
    """S[G, G'] = delta_GG' + sum_mn beta_m(G) q_mn beta_n(G')^*  (identity when qij is None)."""
    npw = beta.shape[1]
    s = np.eye(npw, dtype=np.complex128)
    if qij is not None:
        s += beta.T @ np.asarray(qij, dtype=np.complex128) @ beta.conj()
    return s


def s_psi_projections(beta: np.ndarray, qij, psi: np.ndarray) -> np.ndarray:
    """S|psi> for (nbnd, npw) rows by Eqs. lambdah, delta_eq and finals."""
    if qij is None:
        return np.array(psi, dtype=np.complex128)
    lam = beta.conj() @ psi.T                      # Eq. lambdah   (nproj, nbnd)
    dlt = np.asarray(qij) @ lam                    # Eq. delta_eq
    return psi + (beta.T @ dlt).T                  # Eq. finals


def dense_h(kin: np.ndarray, miller: np.ndarray, fft, vt: np.ndarray, beta: np.ndarray,
            dij: np.ndarray) -> np.ndarray:
    """H_k as an (npw, npw) complex128 matrix."""
    h = local_matrix(miller, fft, vt) + nonlocal_matrix(beta, dij)
    h[np.diag_indices_from(h)] += kin
    return h


def h_psi_dense(h: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """H|psi> for psi given as (nbnd, npw) rows."""
    return (h @ psi.T).T


def h_psi_realspace(kin, miller, fft, v_r, beta, dij, psi) -> np.ndarray:
    """H|psi> band by band through the real-space mesh (Sec. 2.2.2, Sec. 4)."""
    g = basis.grid_index(miller, fft)
    out = np.empty_like(psi, dtype=np.complex128)
    lam = beta.conj() @ psi.T          # (nproj, nbnd)  Eq. lambdah
    gam = dij @ lam                    # Eq. gamma
    vnl = (beta.T @ gam).T             # Eq. finalnl
    for b in range(psi.shape[0]):
        box = np.zeros(tuple(fft), dtype=np.complex128)
        box[g[:, 0], g[:, 1], g[:, 2]] = psi[b]
        u = dft.inverse(box)
        u = np.asarray(v_r) * u
        c = dft.forward(u)
        out[b] = c[g[:, 0], g[:, 1], g[:, 2]] + kin * psi[b] + vnl[b]
    return out


class KPoint:
    """Everything the oracle needs at one k: basis, kinetic, projectors, H_k."""

    def __init__(self, cfg, ik: int, vt: np.ndarray, beta_fn, dij=None, qij=None):
        self.ik = ik
        self.k = np.asarray(cfg.kpts[ik], dtype=np.float64)
        self.miller, q2 = basis.sphere(cfg.lat, self.k, cfg.ecut_ry)
        self.kin = basis.kinetic(q2)
        self.npw = self.miller.shape[0]
        self.beta = beta_fn(cfg, ik, self.miller)
        self.dij = cfg.dij if dij is None else dij
        self.h = dense_h(self.kin, self.miller, cfg.fft, vt, self.beta, self.dij)
        self.qij = getattr(cfg, "qij", None) if qij is None else qij
        self._s = None

    @property
    def s(self) -> np.ndarray:
        """S_k as an (npw, npw) complex128 matrix (built on first use)."""
        if self._s is None:
            self._s = overlap_matrix(self.beta, self.qij)
        return self._s


def h_psi(cfg, v_r, beta_fn, psi_by_k):
    """Plain-definition H|psi> over a list of k-points: build H_k, multiply.

    ``psi_by_k[ik]`` is (nbnd, npw_k) in the oracle's plane-wave order.
    Returns a list of arrays of the same shapes."""
    vt = vtilde(v_r)
    out = []
    for ik, psi in enumerate(psi_by_k):
        kp = KPoint(cfg, ik, vt, beta_fn)
        out.append(h_psi_dense(kp.h, psi))
    return out
