"""Pins for the oracle's overlap operator S = 1 + sum q_mn |beta_m><beta_n|
(Sec. 2.2, Eqs. delta_eq and finals) and for the generalized problems built on
it: the Davidson of Sec. 2.1 for H psi = eps S psi and the DFPT system
(H - eps S + alpha S P_v S) x = rhs of Eqs. linear_system and projector.

Each pin is fixed by the mathematics rather than by re-typing the oracle:
  * the Woodbury closed form of S^-1 built from beta and q alone (fixes the
    orientation of q, the conjugation of beta and the sign of the term);
  * a rank-one overlap on free electrons, whose generalized eigenvalues are
    the roots of a scalar secular equation found here by bisection;
  * a constant potential c together with D + c q shifts every generalized
    eigenvalue by exactly c (H + c S);
  * q = 0 gives the standard problem back;
  * the DFPT solution in closed form in the generalized eigenbasis."""
import numpy as np
import pytest

from oracle import hamiltonian as ham, solvers
from paper_2412_01695_amd import synth

from helpers import beta_fn, zero_beta_fn


def _hermitian_q(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return a @ a.conj().T / n + 0.5 * np.eye(n)


@pytest.fixture(scope="module")
def c1s():
    cfg = synth.with_overlap(synth.make_config(1))
    v = synth.vloc_grid(cfg)
    vt = ham.vtilde(v)
    return cfg, v, [ham.KPoint(cfg, ik, vt, beta_fn) for ik in range(cfg.nk)]


def test_overlap_inverse_by_woodbury():
    # S = 1 + B q B^H with B = beta^T:  S^-1 = 1 - B (q^-1 + B^H B)^-1 B^H
    cfg = synth.make_config(1)
    q = _hermitian_q(cfg.nproj, 3)
    kp = ham.KPoint(cfg, 3, ham.vtilde(np.zeros(cfg.fft)), beta_fn, qij=q)
    b = kp.beta.T
    sinv = np.eye(kp.npw) - b @ np.linalg.solve(np.linalg.inv(q) + b.conj().T @ b, b.conj().T)
    np.testing.assert_allclose(kp.s @ sinv, np.eye(kp.npw), atol=1e-12)
    # both oracle routes of S|psi>
    psi = synth.psi_guess(cfg, 3, kp.miller)
    np.testing.assert_allclose(ham.s_psi_projections(kp.beta, q, psi), (kp.s @ psi.T).T, atol=1e-14)


def test_rank_one_overlap_secular_equation():
    # V = 0, D = 0, one projector with q = s0:  T x = eps (1 + s0 b b^H) x.  With distinct
    # kinetic energies t_G and every b_G != 0 each eigenvalue is a root of
    #   f(eps) = 1 - eps s0 sum_G |b_G|^2 / (t_G - eps),
    # one in (0, t_min) and one between each pair of consecutive t_G.
    cfg = synth.make_config(1)
    tp = 2.0 * np.pi / synth.A_FCC
    c = synth.Config("generic-k", cfg.lat, cfg.ecut_ry, cfg.fft, tp * np.array([[0.11, 0.23, 0.37]]), 6,
                     cfg.tau, cfg.projectors[:1], np.zeros((1, 1), complex), cfg.seed)
    s0 = 40.0
    kp = ham.KPoint(c, 0, ham.vtilde(np.zeros(c.fft)), beta_fn, qij=np.array([[s0]], complex))
    t = kp.kin
    w_b = np.abs(kp.beta[0]) ** 2
    order = np.argsort(t)
    t, w_b = t[order], w_b[order]
    assert np.min(np.diff(t)) > 1e-9 and np.min(w_b) > 0
    # the secular function is monotone decreasing between its poles
    f = lambda e: 1.0 - e * s0 * np.sum(w_b / (t - e))  # noqa: E731

    def bisect(lo, hi):
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if f(mid) > 0:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    nb = 6
    roots = [bisect(0.0, t[0] * (1 - 1e-15))]
    for i in range(nb - 1):
        gap = t[i + 1] - t[i]
        roots.append(bisect(t[i] + 1e-15 * gap, t[i + 1] - 1e-15 * gap))
    w, v = solvers.lowest_eigpairs(kp.h, nb, kp.s)
    np.testing.assert_allclose(w, roots, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v.conj().T @ kp.s @ v, np.eye(nb), atol=1e-12)


def test_constant_potential_plus_cq_shifts_spectrum(c1s):
    cfg, v, kps = c1s
    c = 0.37
    vt1 = ham.vtilde(v + c)
    for kp in kps[:2]:
        k1 = ham.KPoint(cfg, kp.ik, vt1, beta_fn, dij=cfg.dij + c * cfg.qij)
        w0, _ = solvers.lowest_eigpairs(kp.h, cfg.nbnd, kp.s)
        w1, _ = solvers.lowest_eigpairs(k1.h, cfg.nbnd, k1.s)
        np.testing.assert_allclose(w1 - w0, c, atol=1e-12)


def test_zero_q_is_the_standard_problem(c1s):
    cfg, v, _ = c1s
    vt = ham.vtilde(v)
    kp = ham.KPoint(cfg, 1, vt, beta_fn, qij=np.zeros((cfg.nproj, cfg.nproj), complex))
    np.testing.assert_array_equal(kp.s, np.eye(kp.npw))
    w0, _ = solvers.lowest_eigpairs(kp.h, cfg.nbnd)
    w1, _ = solvers.lowest_eigpairs(kp.h, cfg.nbnd, kp.s)
    np.testing.assert_allclose(w1, w0, atol=1e-13)
    kz = ham.KPoint(synth.make_config(1), 1, vt, zero_beta_fn)
    np.testing.assert_array_equal(kz.s, np.eye(kz.npw))


def test_generalized_davidson_reaches_dense_eigenvalues(c1s):
    cfg, _, kps = c1s
    tol_ha = 0.5e-10
    for kp in kps:
        psi0 = synth.psi_guess(cfg, kp.ik, kp.miller)
        w, vecs, it = solvers.davidson(kp.h, psi0, cfg.nbnd, eps_th=0.1 * tol_ha, res_tol=1e-6, s=kp.s)
        ref, _ = solvers.lowest_eigpairs(kp.h, cfg.nbnd, kp.s)
        assert np.max(np.abs(w - ref)) < tol_ha
        r = kp.h @ vecs.T - (kp.s @ vecs.T) * w[None, :]
        assert np.max(np.linalg.norm(r, axis=0)) < 1e-5
        np.testing.assert_allclose(vecs.conj() @ kp.s @ vecs.T, np.eye(cfg.nbnd), atol=1e-10)
        assert 1 <= it < 200


def test_dfpt_with_overlap_closed_form(c1s):
    # in the S-orthonormal generalized eigenbasis V (V^H S V = 1, V^H H V = Lambda):
    #   V^H A V = Lambda - eps + alpha [i < nocc]  =>  x = V (Lambda - eps + alpha P)^-1 V^H b
    cfg, v, kps = c1s
    nocc = 5
    dv = synth.dv_grid(cfg)
    for kp in kps[:2]:
        evals, evecs = solvers.lowest_eigpairs(kp.h, kp.npw, kp.s)
        u = evecs[:, :nocc]
        w = evals[:nocc]
        alpha = solvers.dfpt_alpha(w)
        dvm = ham.local_matrix(kp.miller, cfg.fft, ham.vtilde(dv))
        rhs = solvers.dfpt_rhs(dvm, u, kp.s)
        # the right-hand side has no valence component: U^H rhs = 0
        assert np.max(np.abs(u.conj().T @ rhs)) < 1e-13 * np.max(np.abs(rhs))
        shift = np.where(np.arange(evals.size) < nocc, alpha, 0.0)
        for nu in range(nocc):
            a = solvers.dfpt_matrix(kp.h, u, w[nu], alpha, kp.s)
            b = rhs[:, nu]
            x_cf = evecs @ ((evecs.conj().T @ b) / (evals - w[nu] + shift))
            x_lu = solvers.dfpt_solve_exact(a, b)
            np.testing.assert_allclose(x_lu, x_cf, atol=1e-10 * np.linalg.norm(x_cf))
            m = solvers.dfpt_precond(kp.kin, u[:, nu])
            x, it, rho = solvers.pcg(lambda y: a @ y, lambda y: y / m, b, np.zeros_like(b), thr=1e-24)
            assert it < 1000
            np.testing.assert_allclose(x, x_cf, atol=1e-8 * np.linalg.norm(x_cf))
