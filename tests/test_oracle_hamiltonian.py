"""Pins for the oracle's Hamiltonian (Sec. 2.2; Eqs. lambdah, gamma, finalnl; Sec. 4).

Each pin is fixed by the mathematics rather than by re-typing the oracle:
free electrons, a constant potential, a single complex Fourier component
of V (fixes the sign and the order of the index difference), the rank and
action of the nonlocal term on orthonormal projectors (fixes conjugation and
the orientation of D), hermiticity, the two independent oracle routes,
time reversal and the cubic point group."""
import itertools
import math

import numpy as np
import pytest

from oracle import basis, dft, hamiltonian as ham, solvers
from paper_2412_01695_amd import synth

from helpers import beta_fn, zero_beta_fn


@pytest.fixture(scope="module")
def c1():
    cfg = synth.make_config(1)
    return cfg, synth.vloc_grid(cfg)


def test_free_electron_eigenvalues_exact(c1):
    cfg, _ = c1
    vt = ham.vtilde(np.zeros(cfg.fft))
    for ik in range(cfg.nk):
        kp = ham.KPoint(cfg, ik, vt, zero_beta_fn)
        w, _ = solvers.lowest_eigpairs(kp.h, cfg.nbnd)
        np.testing.assert_allclose(w, np.sort(kp.kin)[:cfg.nbnd], atol=1e-14)
        psi = synth.psi_guess(cfg, ik, kp.miller)
        np.testing.assert_allclose(ham.h_psi_dense(kp.h, psi), kp.kin[None, :] * psi, atol=1e-15)


def test_free_electron_gamma_spectrum_closed_form():
    # k = 0, V = 0, D = 0: eigenvalues are (1/2)|G|^2 = (1/2)(2pi/a)^2 (h^2+k^2+l^2) with the
    # bcc shell degeneracies of tests/golden/bcc_shells.txt
    import os
    cfg = synth.make_config(1)
    c = synth.Config(cfg.name, cfg.lat, cfg.ecut_ry, cfg.fft, np.zeros((1, 3)), 15, cfg.tau,
                     cfg.projectors, cfg.dij, cfg.seed)
    kp = ham.KPoint(c, 0, ham.vtilde(np.zeros(c.fft)), zero_beta_fn)
    unit = 0.5 * (2 * math.pi / synth.A_FCC) ** 2
    rows = [tuple(map(int, ln.split())) for ln in open(os.path.join(os.path.dirname(__file__), "golden",
            "bcc_shells.txt")) if ln.strip() and not ln.startswith("#")]
    ref = np.concatenate([np.full(n, s * unit) for s, n in rows])
    w = np.linalg.eigvalsh(kp.h)
    assert w.size <= ref.size
    np.testing.assert_allclose(w, ref[:w.size], atol=1e-13)


def test_constant_potential_shifts_spectrum(c1):
    cfg, v = c1
    c = -0.37
    vt0 = ham.vtilde(v)
    vt1 = ham.vtilde(v + c)
    for ik in range(cfg.nk):
        h0 = ham.KPoint(cfg, ik, vt0, beta_fn).h
        h1 = ham.KPoint(cfg, ik, vt1, beta_fn).h
        np.testing.assert_allclose(h1 - h0, c * np.eye(h0.shape[0]), atol=1e-13)
        np.testing.assert_allclose(np.linalg.eigvalsh(h1), np.linalg.eigvalsh(h0) + c, atol=1e-12)


def test_single_complex_fourier_component():
    # V(r) = cos(t) + 2 sin(t), t = 2pi l.m0/N  =>  V~[m0] = 1/2 - i, V~[-m0] = 1/2 + i
    cfg = synth.make_config(1)
    n = cfg.fft
    m0 = np.array([1, -2, 1])
    l = np.array(np.meshgrid(*[np.arange(x) for x in n], indexing="ij"))
    t = 2 * math.pi * sum(l[i] * m0[i] / n[i] for i in range(3))
    vt = ham.vtilde(np.cos(t) + 2 * np.sin(t))
    kp = ham.KPoint(cfg, 2, vt, zero_beta_fn)
    off = kp.h - np.diag(kp.kin)
    d = kp.miller[:, None, :] - kp.miller[None, :, :]
    plus = np.all(d == m0, axis=-1)
    minus = np.all(d == -m0, axis=-1)
    assert plus.sum() > 0
    np.testing.assert_allclose(off[plus], 0.5 - 1j, atol=1e-14)
    np.testing.assert_allclose(off[minus], 0.5 + 1j, atol=1e-14)
    np.testing.assert_allclose(off[~(plus | minus)], 0.0, atol=1e-14)


def test_nonlocal_on_orthonormal_projectors():
    # with orthonormal projector columns B, H_nl B = B D for any Hermitian D
    rng = np.random.default_rng(3)
    npw, npj = 40, 5
    q, _ = np.linalg.qr(rng.standard_normal((npw, npj)) + 1j * rng.standard_normal((npw, npj)))
    a = rng.standard_normal((npj, npj)) + 1j * rng.standard_normal((npj, npj))
    d = a + a.conj().T
    hnl = ham.nonlocal_matrix(q.T, d)
    np.testing.assert_allclose(hnl @ q, q @ d, atol=1e-13)
    assert np.linalg.matrix_rank(hnl, tol=1e-10) == npj
    # a vector orthogonal to every projector is annihilated
    x = rng.standard_normal(npw) + 1j * rng.standard_normal(npw)
    x -= q @ (q.conj().T @ x)
    np.testing.assert_allclose(hnl @ x, 0.0, atol=1e-13)


@pytest.mark.parametrize("cid", [1, 2])
def test_hermitian(cid):
    cfg = synth.make_config(cid)
    vt = ham.vtilde(synth.vloc_grid(cfg))
    rng = np.random.default_rng(4)
    for ik in (0, cfg.nk - 1):
        kp = ham.KPoint(cfg, ik, vt, beta_fn)
        assert np.max(np.abs(kp.h - kp.h.conj().T)) < 1e-15
        phi = rng.standard_normal(kp.npw) + 1j * rng.standard_normal(kp.npw)
        psi = rng.standard_normal(kp.npw) + 1j * rng.standard_normal(kp.npw)
        phi /= np.linalg.norm(phi)
        psi /= np.linalg.norm(psi)
        a = np.vdot(phi, kp.h @ psi)
        b = np.vdot(psi, kp.h @ phi)
        assert abs(a - b.conjugate()) < 1e-13


def test_dense_route_equals_realspace_route(c1):
    cfg, v = c1
    vt = ham.vtilde(v)
    for ik in range(cfg.nk):
        kp = ham.KPoint(cfg, ik, vt, beta_fn)
        psi = synth.psi_guess(cfg, ik, kp.miller)
        a = ham.h_psi_dense(kp.h, psi)
        b = ham.h_psi_realspace(kp.kin, kp.miller, cfg.fft, v, kp.beta, cfg.dij, psi)
        np.testing.assert_allclose(a, b, atol=1e-13)


def test_realspace_route_on_a_larger_mesh(c1):
    # the local term does not depend on the mesh once it is one-to-one on the sphere
    cfg, _ = c1
    ik = 3
    m, q2 = basis.sphere(cfg.lat, cfg.kpts[ik], cfg.ecut_ry)
    beta = beta_fn(cfg, ik, m)
    psi = synth.psi_guess(cfg, ik, m)
    out = []
    for n in (cfg.fft, (20, 20, 20)):
        c = synth.Config(cfg.name, cfg.lat, cfg.ecut_ry, n, cfg.kpts, cfg.nbnd, cfg.tau, cfg.projectors,
                         cfg.dij, cfg.seed)
        # V with only a few Fourier components, all representable on both meshes
        v_small = np.real(dft.inverse(_few_components(n)))
        out.append(ham.h_psi_realspace(basis.kinetic(q2), m, n, v_small, beta, cfg.dij, psi))
    np.testing.assert_allclose(out[0], out[1], atol=1e-13)


def _few_components(n):
    ft = np.zeros(n, dtype=np.complex128)
    for (i, j, k), val in {(0, 0, 0): -0.2, (1, 0, 0): 0.05, (-1, 0, 0): 0.05, (1, 1, -1): 0.03 - 0.01j,
                           (-1, -1, 1): 0.03 + 0.01j}.items():
        ft[i % n[0], j % n[1], k % n[2]] = val
    return ft


def test_time_reversal_eigenvalues(c1):
    cfg, v = c1
    vt = ham.vtilde(v)
    for ik in (1, 3):
        kp = ham.KPoint(cfg, ik, vt, beta_fn)
        cm = synth.Config(cfg.name, cfg.lat, cfg.ecut_ry, cfg.fft, -cfg.kpts, cfg.nbnd, cfg.tau,
                          cfg.projectors, cfg.dij, cfg.seed)
        km = ham.KPoint(cm, ik, vt, beta_fn)
        np.testing.assert_allclose(np.linalg.eigvalsh(kp.h), np.linalg.eigvalsh(km.h), atol=1e-12)


def test_cubic_symmetry_eigenvalues(c1):
    cfg, v = c1
    vt = ham.vtilde(v)
    k = cfg.kpts[3]                  # general k point: no symmetry of its own
    ref = None
    for perm in itertools.permutations(range(3)):
        for sg in ((1, 1, 1), (-1, 1, -1), (1, -1, -1), (-1, -1, 1)):
            kr = np.array([sg[i] * k[perm[i]] for i in range(3)])
            c = synth.Config(cfg.name, cfg.lat, cfg.ecut_ry, cfg.fft, kr[None, :], cfg.nbnd, cfg.tau,
                             cfg.projectors, cfg.dij, cfg.seed)
            w = np.linalg.eigvalsh(ham.KPoint(c, 0, vt, beta_fn).h)[:cfg.nbnd]
            if ref is None:
                ref = w
            np.testing.assert_allclose(w, ref, atol=1e-11)


def test_atom_translation_by_lattice_vector(c1):
    cfg, _ = c1
    c2 = synth.Config(cfg.name, cfg.lat, cfg.ecut_ry, cfg.fft, cfg.kpts, cfg.nbnd,
                      cfg.tau + cfg.lat[0] - 2 * cfg.lat[2], cfg.projectors, cfg.dij, cfg.seed)
    v1, v2 = synth.vloc_grid(cfg), synth.vloc_grid(c2)
    np.testing.assert_allclose(v1, v2, atol=1e-12)
    h1 = ham.KPoint(cfg, 3, ham.vtilde(v1), beta_fn).h
    h2 = ham.KPoint(c2, 3, ham.vtilde(v2), beta_fn).h
    np.testing.assert_allclose(h1, h2, atol=1e-12)
