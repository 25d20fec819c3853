"""Edge cases and the largest workload through the C-ABI on the GPU.

One k-point and one band through every entry point; the full 1728-k x 24-band
launch at 36^3 (the largest mesh and basis) checked on sampled k-points in FP64
and mixed precision; a perturbation on k-lists whose spheres differ in size."""
import numpy as np
import pytest

from oracle import dft, hamiltonian as ham, response, solvers
from paper_2412_01695_amd import synth

from gpu_util import to_dev, torch_cuda
from helpers import beta_fn, miller_map

pytestmark = pytest.mark.gpu


def _system(cfg, **kw):
    torch = torch_cuda()
    from paper_2412_01695_amd.system import System
    return torch, System(cfg, 0, **kw)


def _oracle_rows(s, ik, rows, kp):
    perm = miller_map(s.miller[ik], kp.miller)
    out = np.zeros((rows.shape[0], kp.npw), complex)
    out[:, perm] = rows[:, :s.npw[ik]]
    return out, perm


def test_one_k_one_band_everywhere():
    from paper_2412_01695_amd import mkpw
    cfg0 = synth.with_overlap(synth.make_config(1))
    cfg = synth.subset(cfg0, [2])
    cfg.nbnd = 1
    torch, s = _system(cfg)
    vt = ham.vtilde(s.vloc)
    kp = ham.KPoint(cfg, 0, vt, beta_fn)
    psi = s.psi_guess(1)
    po, perm = _oracle_rows(s, 0, psi[0], kp)
    for fn, mat in ((mkpw.pw_h_psi, kp.h), (mkpw.pw_s_psi, kp.s)):
        d = to_dev(torch, psi)
        out = torch.full_like(d, float("nan"))
        torch.cuda.synchronize()
        fn(s.ctx, 0, 1, d, out)
        torch.cuda.synchronize()
        ref = (mat @ po.T).T[:, perm]
        got = out.cpu().numpy()[0, :, :s.npw[0]]
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    d = to_dev(torch, psi)
    st, eig, iters, conv = mkpw.pw_davidson(s.ctx, 0, 1, d, 1, 1e-10, 300)
    torch.cuda.synchronize()
    w, u = solvers.lowest_eigpairs(kp.h, 1, kp.s)
    assert st == 0 and abs(eig[0, 0] - w[0]) < 0.5e-10
    # CG with one system
    alpha = np.array([0.5])
    dv = synth.dv_grid(cfg)
    rhs_o = solvers.dfpt_rhs(ham.local_matrix(kp.miller, cfg.fft, ham.vtilde(dv)), u, kp.s)
    rhs = np.zeros((1, 1, s.npwx), complex)
    rhs[0, 0, :s.npw[0]] = rhs_o[perm, 0]
    ul = np.zeros((1, 1, s.npwx), complex)
    ul[0, 0, :s.npw[0]] = u[perm, 0]
    x = torch.zeros((1, 1, s.npwx), dtype=torch.complex128, device="cuda")
    drhs, du = to_dev(torch, rhs), to_dev(torch, ul)
    torch.cuda.synchronize()
    st, it = mkpw.pw_dfpt_cg(s.ctx, 0, 1, du, w[:1].reshape(1, 1).copy(), alpha, 1, drhs, x, 1e-26, 500)
    torch.cuda.synchronize()
    xo = solvers.dfpt_solve_exact(solvers.dfpt_matrix(kp.h, u, w[0], 0.5, kp.s), rhs_o[:, 0])
    got = x.cpu().numpy()[0, 0, :s.npw[0]]
    assert st == 0 and np.max(np.abs(got - xo[perm])) <= 1e-9 * np.max(np.abs(xo))


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 2e-6)])
def test_largest_workload_full_batch_sampled(prec, tol):
    # 1728 k x 24 bands at 36^3, npw up to 489: the largest launch of the library's workloads
    from paper_2412_01695_amd import mkpw
    cfg = synth.make_config(4)
    torch, s = _system(cfg)
    psi = s.psi_guess()
    dt = torch.complex128 if prec == 0 else torch.complex64
    d = to_dev(torch, psi, dt)
    h = torch.full_like(d, float("nan"))
    torch.cuda.synchronize()
    mkpw.pw_h_psi(s.ctx, prec, cfg.nbnd, d, h)
    torch.cuda.synchronize()
    hv = h.cpu().numpy().astype(np.complex128)
    vt = ham.vtilde(s.vloc)
    ks = list(range(0, cfg.nk, 199)) + [cfg.nk - 1]
    worst, scale = 0.0, 0.0
    for ik in ks:
        kp = ham.KPoint(cfg, ik, vt, beta_fn)
        po, perm = _oracle_rows(s, ik, psi[ik], kp)
        ref = ham.h_psi_dense(kp.h, po)[:, perm]
        worst = max(worst, np.max(np.abs(hv[ik, :, :s.npw[ik]] - ref)))
        scale = max(scale, np.max(np.abs(ref)))
        assert np.all(hv[ik, :, s.npw[ik]:] == 0)
    print("1728-k full batch prec", prec, "rel err", worst / scale)
    assert worst <= tol * scale


def test_perturbation_between_unequal_spheres():
    # k and k+q lists whose spheres have different sizes at every k (q off the lattice)
    from paper_2412_01695_amd import mkpw
    cfg = synth.make_config(1)
    torch = torch_cuda()
    from paper_2412_01695_amd.system import System
    sk = System(cfg, 0)
    sq = System(synth.shifted(cfg, synth.q_paper() * 1.7), 0)
    assert np.any(sk.npw != sq.npw)
    nocc = 3
    dv = synth.dv_complex_grid(cfg)
    dvt = dft.forward(dv)
    vt = ham.vtilde(sk.vloc)
    uk = sk.psi_guess(nocc)
    uq = np.zeros((cfg.nk, nocc, sq.npwx), complex)
    ref = np.zeros_like(uq)
    for ik in range(cfg.nk):
        kk = ham.KPoint(cfg, ik, vt, beta_fn)
        kq = ham.KPoint(sq.cfg, ik, vt, beta_fn)
        _, u = solvers.lowest_eigpairs(kq.h, nocc)
        pq = miller_map(sq.miller[ik], kq.miller)
        uq[ik, :, :sq.npw[ik]] = u.T[:, pq]
        uko, _ = _oracle_rows(sk, ik, uk[ik], kk)
        r = response.dfpt_rhs_q(response.dv_cross_matrix(kq.miller, kk.miller, cfg.fft, dvt) @ uko.T, u)
        ref[ik, :, :sq.npw[ik]] = r.T[:, pq]
    out = torch.full((cfg.nk, nocc, sq.npwx), float("nan"), dtype=torch.complex128, device="cuda")
    a, b = to_dev(torch, uk), to_dev(torch, uq)
    torch.cuda.synchronize()
    mkpw.pw_dfpt_rhs(sq.ctx, sk.ctx, nocc, dv, a, b, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_mismatched_contexts_are_refused():
    from paper_2412_01695_amd import mkpw
    torch = torch_cuda()
    from paper_2412_01695_amd.system import System
    s1 = System(synth.make_config(1), 0)
    s2 = System(synth.make_config(2), 0)
    with pytest.raises(mkpw.PwError) as e:
        mkpw.pw_drho(s1.ctx, s2.ctx, 1, np.ones(s1.nk), 0, 0, 0)
    assert e.value.status == mkpw.PW_EINVAL
