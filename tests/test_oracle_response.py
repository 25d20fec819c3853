"""Pins for the oracle's linear response at q != 0 (Sec. 2.3, Eqs. linear_system
and drho): the perturbation taken from the k sphere to the k+q sphere, the
right-hand side, and the induced density.

Fixed by the mathematics rather than by re-typing the oracle:
  * a perturbation with a single complex Fourier component m0 couples exactly
    the pairs with m_G' - m_G = m0 (mod N), with weight one (fixes the sign and
    the order of the index difference and the transform normalisation);
  * a constant perturbation c returns c u on the Miller indices the two
    spheres share and zero elsewhere;
  * two single plane waves give drho(r) = 4 w exp(2 pi i (m2 - m1) . l / N)
    (fixes which factor is conjugated and the factor 4 w);
  * the mesh average of drho is 4 sum w sum_nu sum_G conj(u(G)) du(G) over the
    shared Miller indices (orthogonality of plane waves on the mesh);
  * at q = 0 with du = u the density is real, non-negative and averages to
    4 sum w nocc;
  * the right-hand side has no component along the occupied k+q states."""
import numpy as np
import pytest

from oracle import basis, dft, hamiltonian as ham, response, solvers
from paper_2412_01695_amd import synth

from helpers import beta_fn


@pytest.fixture(scope="module")
def c1q():
    cfg = synth.make_config(1)
    cq = synth.shifted(cfg, synth.q_paper())
    return cfg, cq


def _spheres(cfg, cq, ik):
    mk, _ = basis.sphere(cfg.lat, cfg.kpts[ik], cfg.ecut_ry)
    mq, _ = basis.sphere(cq.lat, cq.kpts[ik], cq.ecut_ry)
    return mk, mq


def test_cross_matrix_equals_realspace_route(c1q):
    cfg, cq = c1q
    dv = synth.dv_complex_grid(cfg)
    dvt = dft.forward(dv)
    for ik in range(cfg.nk):
        mk, mq = _spheres(cfg, cq, ik)
        u = synth.psi_guess(cfg, ik, mk, nbnd=3)
        a = (response.dv_cross_matrix(mq, mk, cfg.fft, dvt) @ u.T).T
        b = response.dv_psi_realspace(mq, mk, cfg.fft, dv, u)
        np.testing.assert_allclose(a, b, atol=1e-13 * np.max(np.abs(a)))


def test_single_fourier_component_perturbation(c1q):
    cfg, cq = c1q
    n = np.array(cfg.fft)
    m0 = np.array([2, -1, 1])
    l = np.array(np.meshgrid(*[np.arange(x) for x in n], indexing="ij"))
    dv = np.exp(2j * np.pi * sum(l[i] * m0[i] / n[i] for i in range(3)))
    dvt = dft.forward(dv)
    mk, mq = _spheres(cfg, cq, 3)
    lm = response.dv_cross_matrix(mq, mk, cfg.fft, dvt)
    want = np.all(np.mod(mq[:, None, :] - mk[None, :, :] - m0, n) == 0, axis=2).astype(float)
    assert want.sum() > 10
    np.testing.assert_allclose(lm, want, atol=1e-13)


def test_constant_perturbation(c1q):
    cfg, cq = c1q
    c = 0.37 - 0.21j
    mk, mq = _spheres(cfg, cq, 2)
    u = synth.psi_guess(cfg, 2, mk, nbnd=2)
    out = response.dv_psi_realspace(mq, mk, cfg.fft, np.full(cfg.fft, c), u)
    keyk = {tuple(r): i for i, r in enumerate(mk)}
    want = np.zeros_like(out)
    for j, r in enumerate(mq):
        if tuple(r) in keyk:
            want[:, j] = c * u[:, keyk[tuple(r)]]
    assert 0 < np.count_nonzero(want[0]) < mq.shape[0]
    np.testing.assert_allclose(out, want, atol=1e-14)


def test_drho_of_two_plane_waves():
    cfg = synth.make_config(1)
    n = np.array(cfg.fft)
    m1, m2 = np.array([[1, 0, -1]]), np.array([[-2, 1, 0]])
    w = 0.3
    d = response.drho(cfg.fft, [w], [m1], [np.ones((1, 1))], [m2], [np.ones((1, 1))])
    l = np.array(np.meshgrid(*[np.arange(x) for x in n], indexing="ij"))
    want = 4 * w * np.exp(2j * np.pi * sum(l[i] * (m2[0, i] - m1[0, i]) / n[i] for i in range(3)))
    np.testing.assert_allclose(d, want, atol=1e-13)


def test_drho_mean_is_the_shared_overlap(c1q):
    cfg, cq = c1q
    ws = np.full(cfg.nk, 1.0 / cfg.nk)
    mks, mqs, us, dus = [], [], [], []
    want = 0.0
    for ik in range(cfg.nk):
        mk, mq = _spheres(cfg, cq, ik)
        u = synth.psi_guess(cfg, ik, mk, nbnd=3)
        du = synth.random_vectors(5, ik, mq, 3)
        mks.append(mk), mqs.append(mq), us.append(u), dus.append(du)
        keyq = {tuple(r): j for j, r in enumerate(mq)}
        for i, r in enumerate(mk):
            if tuple(r) in keyq:
                want += 4 * ws[ik] * np.sum(u[:, i].conj() * du[:, keyq[tuple(r)]])
    d = response.drho(cfg.fft, ws, mks, us, mqs, dus)
    np.testing.assert_allclose(d.mean(), want, atol=1e-12 * abs(want))


def test_drho_at_q0_is_a_density():
    cfg = synth.make_config(1)
    ws = np.full(cfg.nk, 0.25)
    mks, us = [], []
    for ik in range(cfg.nk):
        mk, _ = basis.sphere(cfg.lat, cfg.kpts[ik], cfg.ecut_ry)
        mks.append(mk)
        us.append(synth.psi_guess(cfg, ik, mk, nbnd=4))
    d = response.drho(cfg.fft, ws, mks, us, mks, us)
    assert np.max(np.abs(d.imag)) < 1e-14 * np.max(np.abs(d.real))
    assert d.real.min() >= 0
    np.testing.assert_allclose(d.real.mean(), 4 * np.sum(ws) * 4, rtol=1e-13)


def test_rhs_has_no_valence_component_at_kq(c1q):
    cfg, cq = c1q
    cq = synth.with_overlap(cq)
    dvt = dft.forward(synth.dv_complex_grid(cfg))
    vt = ham.vtilde(synth.vloc_grid(cfg))
    ik = 1
    mk, _ = basis.sphere(cfg.lat, cfg.kpts[ik], cfg.ecut_ry)
    kq = ham.KPoint(cq, ik, vt, beta_fn)
    _, uq = solvers.lowest_eigpairs(kq.h, 5, kq.s)
    u = synth.psi_guess(cfg, ik, mk, nbnd=5)
    dvu = response.dv_cross_matrix(kq.miller, mk, cfg.fft, dvt) @ u.T
    rhs = response.dfpt_rhs_q(dvu, uq, kq.s)
    assert np.max(np.abs(uq.conj().T @ rhs)) < 1e-13 * np.max(np.abs(rhs))
