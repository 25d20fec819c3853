"""Pins for the oracle's solvers (Sec. 2.1 Davidson, Sec. 2.3 Eq. linear_system and
Eq. projector, Sec. 2.4 preconditioned CG).

Davidson must land on the dense eigenvalues; the CG must land on the exact
solution, which is checked two independent ways (LU solve and the
eigenbasis closed form x = sum_i v_i (v_i^H b) / (lambda_i - eps + alpha[i<=nocc]))."""
import numpy as np
import pytest

from oracle import hamiltonian as ham, solvers
from paper_2412_01695_amd import synth

from helpers import beta_fn


@pytest.fixture(scope="module")
def c1k():
    cfg = synth.make_config(1)
    v = synth.vloc_grid(cfg)
    vt = ham.vtilde(v)
    return cfg, v, [ham.KPoint(cfg, ik, vt, beta_fn) for ik in range(cfg.nk)]


def test_davidson_reaches_dense_eigenvalues(c1k):
    cfg, _, kps = c1k
    tol_ha = 0.5e-10          # 1e-10 Ry
    for kp in kps:
        psi0 = synth.psi_guess(cfg, kp.ik, kp.miller)
        w, vecs, it = solvers.davidson(kp.h, psi0, cfg.nbnd, eps_th=0.1 * tol_ha, res_tol=1e-6)
        ref, _ = solvers.lowest_eigpairs(kp.h, cfg.nbnd)
        assert np.max(np.abs(w - ref)) < tol_ha
        r = kp.h @ vecs.T - vecs.T * w[None, :]
        assert np.max(np.linalg.norm(r, axis=0)) < 1e-5
        np.testing.assert_allclose(vecs.conj() @ vecs.T, np.eye(cfg.nbnd), atol=1e-10)
        assert 1 <= it < 200


def test_davidson_restart_path(c1k):
    # a basis that may only hold 2 nbnd vectors forces restarts; the answer is unchanged
    cfg, _, kps = c1k
    kp = kps[2]
    psi0 = synth.psi_guess(cfg, kp.ik, kp.miller)
    w, _, _ = solvers.davidson(kp.h, psi0, cfg.nbnd, eps_th=1e-12, res_tol=1e-6, max_basis_factor=2)
    ref, _ = solvers.lowest_eigpairs(kp.h, cfg.nbnd)
    assert np.max(np.abs(w - ref)) < 1e-10


def _dfpt_system(cfg, v, kp, nocc):
    w, u = solvers.lowest_eigpairs(kp.h, nocc)
    alpha = solvers.dfpt_alpha(w)
    dv = synth.dv_grid(cfg)
    dvm = ham.local_matrix(kp.miller, cfg.fft, ham.vtilde(dv))
    rhs = solvers.dfpt_rhs(dvm, u)
    return w, u, alpha, rhs


def test_dfpt_cg_matches_exact_solution(c1k):
    cfg, v, kps = c1k
    nocc = 5                  # a gap follows band 5 at every C1 k-point (no split multiplet)
    for kp in kps:
        w, u, alpha, rhs = _dfpt_system(cfg, v, kp, nocc)
        evals, evecs = np.linalg.eigh(kp.h)
        for nu in range(nocc):
            a = solvers.dfpt_matrix(kp.h, u, w[nu], alpha)
            b = rhs[:, nu]
            x_lu = solvers.dfpt_solve_exact(a, b)
            # eigenbasis closed form (u are exactly the lowest eigenvectors)
            shift = np.where(np.arange(evals.size) < nocc, alpha, 0.0)
            x_cf = evecs @ ((evecs.conj().T @ b) / (evals - w[nu] + shift))
            np.testing.assert_allclose(x_lu, x_cf, atol=1e-10 * np.linalg.norm(x_cf))
            m = solvers.dfpt_precond(kp.kin, u[:, nu])
            x, it, rho = solvers.pcg(lambda y: a @ y, lambda y: y / m, b, np.zeros_like(b), thr=1e-24)
            assert it < 1000 and abs(rho) < 1e-24
            assert np.linalg.norm(a @ x - b) <= 1e-9 * np.linalg.norm(b)
            np.testing.assert_allclose(x, x_cf, atol=1e-8 * np.linalg.norm(x_cf))


def test_dfpt_rhs_is_orthogonal_to_valence(c1k):
    cfg, v, kps = c1k
    w, u, alpha, rhs = _dfpt_system(cfg, v, kps[1], 5)
    assert np.max(np.abs(u.conj().T @ rhs)) < 1e-14
    assert alpha > 0 and np.all(alpha + w[:, None] - w[None, :] > 0)


def test_pcg_on_a_small_spd_system():
    # Hermitian positive definite system with a known answer
    rng = np.random.default_rng(5)
    n = 30
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.linspace(0.5, 20.0, n)
    a = (q * lam) @ q.conj().T
    x_true = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    b = a @ x_true
    x, it, rho = solvers.pcg(lambda y: a @ y, lambda y: y, b, np.zeros(n, complex), thr=1e-26)
    np.testing.assert_allclose(x, x_true, atol=1e-10)
    assert it <= 2 * n
    # one step from the exact answer stops immediately
    x2, it2, _ = solvers.pcg(lambda y: a @ y, lambda y: y, b, x_true, thr=1e-20)
    assert it2 == 0


def test_dfpt_precond_single_plane_wave_closed_form(c1k):
    # u = one plane wave G0 (any phase): T_nu = |k+G0|^2 / 2, so the Sec. 2.4
    # preconditioner is M_GG = max(1, |k+G|^2 / |k+G0|^2), a ratio of squared
    # wavevectors that no factor 1/2 survives in
    cfg, _, kps = c1k
    for kp in kps[1:]:
        q2 = np.sum(synth.q_vectors(cfg, kp.ik, kp.miller) ** 2, axis=1)
        for j in (0, kp.npw // 3, kp.npw - 1):
            if q2[j] == 0.0:
                continue
            u = np.zeros(kp.npw, complex)
            u[j] = np.exp(0.7j)
            m = solvers.dfpt_precond(kp.kin, u)
            np.testing.assert_allclose(m, np.maximum(1.0, q2 / q2[j]), rtol=1e-14)


def test_dfpt_precond_two_plane_waves_closed_form(c1k):
    # |u(Ga)|^2 = 1/4, |u(Gb)|^2 = 3/4: T_nu = (|k+Ga|^2 + 3 |k+Gb|^2) / 8, and
    # every G with |k+G|^2 / 2 <= T_nu gets M_GG = 1
    cfg, _, kps = c1k
    kp = kps[2]
    q2 = np.sum(synth.q_vectors(cfg, kp.ik, kp.miller) ** 2, axis=1)
    a, b = 5, kp.npw - 7
    u = np.zeros(kp.npw, complex)
    u[a] = 0.5 * np.exp(-0.3j)
    u[b] = np.sqrt(0.75) * 1j
    t = (q2[a] + 3.0 * q2[b]) / 8.0
    m = solvers.dfpt_precond(kp.kin, u)
    np.testing.assert_allclose(m, np.maximum(1.0, 0.5 * q2 / t), rtol=1e-14)
    assert np.all(m[0.5 * q2 <= t] == 1.0) and np.all(m[0.5 * q2 > t * (1 + 1e-12)] > 1.0)
