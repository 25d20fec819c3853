"""Eigenpairs and linear solves for one k-point (oracle; test infrastructure only).

* ``lowest_eigpairs``: the plain definition of what Davidson returns, the
  lowest nbnd eigenpairs of H_k psi = eps S_k psi (Eq. ks; S = I when no
  overlap is given), by dense (generalized) diagonalisation.
* ``davidson``: the block-Davidson steps of Sec. 2.1 in the paper's order,
  used to compare iteration behaviour (parity targets stay the dense values).
* ``pcg``: the preconditioned conjugate gradient of Sec. 2.4 (Eqs. ax1,
  row2, row3, row4, updated, ax2, lambda, updatex, updater, updatedold).
* ``dfpt_*``: the DFPT linear system of Eq. linear_system at q = 0 with
  the valence projector of Eq. projector,
      (H - eps_nu S + alpha S P_v S) x = rhs,    P_v = sum_mu |u_mu><u_mu|
  (S-orthonormal u), its right-hand side -(1 - S P_v) dV u_nu (dS = 0),
  the shift alpha and the preconditioner of Sec. 2.4, and its exact
  solution.  Without an overlap S = I.

Readings where the paper is silent (units, stopping rules, alpha, the
complex inner product of the CG) are the project's and are listed with the
design notes; each is stated again at the function that uses it.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def lowest_eigpairs(h: np.ndarray, nbnd: int, s: np.ndarray | None = None):
    """Lowest nbnd eigenvalues (Ha) and eigenvectors (npw, nbnd) of Hermitian h,
    or of the pencil (h, s) with s Hermitian positive definite (eigenvectors
    then S-orthonormal)."""
    if s is None:
        w, v = np.linalg.eigh(h)
    else:
        w, v = scipy.linalg.eigh(h, s)
    return w[:nbnd], v[:, :nbnd]


def _reduced_eig(ht, st, nbnd, rcond=1e-9):
    """Lowest nbnd solutions of (H~ - eps S~) v = 0 (Sec. 2.1, reduced problem).

    Solved through the eigenvectors of S~, dropping directions whose overlap
    eigenvalue is below rcond * max (a nearly dependent correction vector
    carries no new information); v is S~-orthonormal."""
    s, u = np.linalg.eigh(st)
    keep = s > rcond * s[-1]
    x = u[:, keep] / np.sqrt(s[keep])[None, :]
    w, y = np.linalg.eigh(x.conj().T @ ht @ x)
    return w[:nbnd], x @ y[:, :nbnd]


def _orthonormal_complement(basis, corr, s, drop=1e-10):
    """Normalised correction vectors (Sec. 2.1, normalisation step), made
    S-orthogonal to the current basis and to each other first (two passes of
    Gram-Schmidt in the S inner product) so the reduced overlap stays well
    conditioned; a vector with nothing left after the projection is dropped."""
    def snorm(c):
        return float(np.sqrt(np.real(np.vdot(c, s @ c))))

    out = []
    for j in range(corr.shape[1]):
        c = corr[:, j].copy()
        n0 = snorm(c)
        for _ in range(2):
            c -= basis @ (basis.conj().T @ (s @ c))
            for o in out:
                c -= o * np.vdot(o, s @ c)
        n = snorm(c)
        if n > drop * n0:
            out.append(c / n)
    return np.array(out).T if out else np.zeros((corr.shape[0], 0), dtype=corr.dtype)


def davidson(h: np.ndarray, psi0: np.ndarray, nbnd: int, eps_th: float, max_iter: int = 200,
             max_basis_factor: int = 4, res_tol: float | None = None, s: np.ndarray | None = None):
    """Sec. 2.1 Davidson for one k, for H psi = eps S psi (S = I when s is None).

    psi0: (nbnd, npw) starting vectors.  H_diag and S_diag are the exact
    diagonals of h and s.  A correction is added for every band whose
    eigenvalue moved by more than eps_th (and, when ``res_tol`` is given,
    whose residual norm |(H - eps S) phi| is still above it); when the basis
    would exceed max_basis_factor * nbnd vectors the basis restarts from the
    current Ritz vectors.  Returns (eigenvalues, vectors (nbnd, npw),
    iterations); the vectors are S-orthonormal."""
    sm = np.eye(h.shape[0], dtype=np.complex128) if s is None else s
    hdiag = np.real(np.diag(h))
    sdiag = np.real(np.diag(sm))
    basis = np.array(psi0, dtype=np.complex128).T          # (npw, nbase)
    hb = h @ basis
    sb = sm @ basis
    ht = basis.conj().T @ hb
    st = basis.conj().T @ sb
    eps, v = _reduced_eig(ht, st, nbnd)
    phi, hphi, sphi = basis @ v, hb @ v, sb @ v
    todo = np.ones(nbnd, dtype=bool)
    it = 0
    for it in range(1, max_iter + 1):
        idx = np.nonzero(todo)[0]
        if idx.size == 0:
            break
        # correction vectors (H_diag - eps S_diag)^-1 (H - eps S) phi
        res = hphi[:, idx] - sphi[:, idx] * eps[idx][None, :]
        den = hdiag[:, None] - eps[idx][None, :] * sdiag[:, None]
        den = np.where(np.abs(den) < 1e-2, np.where(den < 0, -1e-2, 1e-2), den)
        corr = res / den
        if basis.shape[1] + idx.size > max_basis_factor * nbnd:
            basis, hb, sb = phi.copy(), hphi.copy(), sphi.copy()
        corr = _orthonormal_complement(basis, corr, sm)
        if corr.shape[1] == 0:
            break
        basis = np.concatenate([basis, corr], axis=1)
        hb = np.concatenate([hb, h @ corr], axis=1)
        sb = np.concatenate([sb, sm @ corr], axis=1)
        # extended reduced Hamiltonian and overlap, then the reduced problem
        ht = basis.conj().T @ hb
        st = basis.conj().T @ sb
        new_eps, v = _reduced_eig(0.5 * (ht + ht.conj().T), 0.5 * (st + st.conj().T), nbnd)
        phi, hphi, sphi = basis @ v, hb @ v, sb @ v
        todo = np.abs(new_eps - eps) > eps_th
        if res_tol is not None:
            rn = np.linalg.norm(hphi - sphi * new_eps[None, :], axis=0)
            todo |= rn > res_tol
        eps = new_eps
    # final Rayleigh-Ritz on the nbnd Ritz vectors alone, with H and S applied
    # afresh: a well-conditioned reduced problem, so the returned eigenvalues
    # carry no round-off from nearly dependent basis vectors
    hphi = h @ phi
    sphi = sm @ phi
    eps, v = _reduced_eig(phi.conj().T @ hphi, phi.conj().T @ sphi, nbnd)
    return eps, (phi @ v).T, it


def pcg(apply_a, apply_minv, b: np.ndarray, x0: np.ndarray, thr: float, max_iter: int = 1000):
    """Sec. 2.4 preconditioned CG for one system A x = b.

    Complex vectors: rho = Re(d^H r) and lambda = -Re(d^H r) / Re(d^H t)
    (A Hermitian and M real make the imaginary parts round-off).  The gamma
    step (Eqs. row4, updated) runs from the second iteration on; the loop
    stops as soon as |rho| < thr.  Returns (x, iterations, rho)."""
    x = np.array(x0, dtype=np.complex128)
    r = apply_a(x) - b                                   # Eq. ax1
    d_old = None
    rho_old = None
    rho = np.inf
    for it in range(1, max_iter + 1):
        d = apply_minv(r)                                # Eq. row2
        rho = float(np.real(np.vdot(d, r)))              # Eq. row3
        if abs(rho) < thr:
            return x, it - 1, rho
        if it > 1:
            gamma = rho / rho_old                        # Eq. row4
            d = d + gamma * d_old                        # Eq. updated
        t = apply_a(d)                                   # Eq. ax2
        lam = -float(np.real(np.vdot(d, r))) / float(np.real(np.vdot(d, t)))  # Eq. lambda
        x = x + lam * d                                  # Eq. updatex
        r = r + lam * t                                  # Eq. updater
        d_old = d                                        # Eq. updatedold
        rho_old = rho
    return x, max_iter, rho


def dfpt_alpha(eps_occ: np.ndarray) -> float:
    """alpha = max(2 (eps_max - eps_min) over the occupied bands, 0.1 Ha), so that
    alpha + eps_mu - eps_nu > 0 for all occupied mu, nu."""
    return float(max(2.0 * (np.max(eps_occ) - np.min(eps_occ)), 0.1))


def dfpt_matrix(h: np.ndarray, u_occ: np.ndarray, eps_nu: float, alpha: float,
                s: np.ndarray | None = None) -> np.ndarray:
    """A = H - eps_nu S + alpha sum_mu S|u_mu><u_mu|S  (Eq. projector; u_occ is
    (npw, nocc), S-orthonormal; S = I when s is None)."""
    if s is None:
        return h - eps_nu * np.eye(h.shape[0]) + alpha * (u_occ @ u_occ.conj().T)
    su = s @ u_occ
    return h - eps_nu * s + alpha * (su @ su.conj().T)


def dfpt_rhs(dv_mat: np.ndarray, u_occ: np.ndarray, s: np.ndarray | None = None) -> np.ndarray:
    """rhs_nu = -(1 - S P_v) dV u_nu restricted to the sphere, all nu: (npw, nocc)
    (the conduction projector of Eq. linear_system applied on the left, with
    dS = 0; S = I when s is None)."""
    y = dv_mat @ u_occ
    su = u_occ if s is None else s @ u_occ
    y = y - su @ (u_occ.conj().T @ y)
    return -y


def dfpt_precond(kin: np.ndarray, u_nu: np.ndarray) -> np.ndarray:
    """Sec. 2.4 diagonal preconditioner in Ha: M_GG = max(1, (|k+G|^2/2) / T_nu),
    T_nu = <u_nu| -grad^2/2 |u_nu>."""
    t = float(np.sum(kin * np.abs(u_nu) ** 2))
    return np.maximum(1.0, kin / t)


def dfpt_solve_exact(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """The unique x = A^-1 b (plain definition)."""
    return np.linalg.solve(a, b)
