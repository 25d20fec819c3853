"""The overlap operator S and the generalized solvers through the C-ABI on the GPU,
against the FP64 oracle.

S|psi>: element by element within 1e-13 (FP64) / 2e-6 (complex64) of the
largest |S psi|; a copy of psi without an overlap.
Davidson for H psi = eps S psi: eigenvalues within 1e-10 Ry of the dense
generalized diagonalisation (FP64), 1e-6 Ry after the refinement of the
mixed solve; the returned vectors S-orthonormal, residuals |H psi - eps S psi|
small.
CG for (H - eps S + alpha S P_v S) x = rhs: within 1e-9 (relative) of the
oracle's exact solve, with the oracle's S-orthonormal eigenvectors as the
valence states on both sides."""
import numpy as np
import pytest

from oracle import hamiltonian as ham, solvers
from paper_2412_01695_amd import synth

from gpu_util import to_dev, torch_cuda
from helpers import beta_fn, miller_map

pytestmark = pytest.mark.gpu

TOL64 = 1e-13
TOL32 = 2e-6
TOL_FP64_HA = 0.5e-10
TOL_MIXED_HA = 0.5e-6


def _system(cfg, **kw):
    torch = torch_cuda()
    from paper_2412_01695_amd.system import System
    return torch, System(cfg, 0, **kw)


def _kpoints(cfg, s, ks):
    vt = ham.vtilde(s.vloc)
    return {ik: ham.KPoint(cfg, ik, vt, beta_fn) for ik in ks}


def _apply_s(torch, s, psi, prec):
    from paper_2412_01695_amd import mkpw
    dt = torch.complex128 if prec == mkpw.PW_FP64 else torch.complex64
    d = to_dev(torch, psi, dt)
    out = torch.full_like(d, float("nan"))
    torch.cuda.synchronize()  # torch's fill runs on its own stream, the library on the context's
    mkpw.pw_s_psi(s.ctx, prec, psi.shape[1], d, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("cid,step", [(1, 1), (2, 21), (4, 97)])
def test_s_psi_matches_oracle(cid, step):
    cfg = synth.with_overlap(synth.subset(synth.make_config(cid), np.arange(0, synth.make_config(cid).nk, step)))
    torch, s = _system(cfg)
    psi = s.psi_guess()
    kps = _kpoints(cfg, s, range(cfg.nk))
    ref = {}
    for ik, kp in kps.items():
        perm = miller_map(s.miller[ik], kp.miller)
        po = np.zeros((psi.shape[1], kp.npw), complex)
        po[:, perm] = psi[ik, :, :s.npw[ik]]
        ref[ik] = (kp.s @ po.T).T[:, perm]
    scale = max(np.max(np.abs(r)) for r in ref.values())
    for prec, tol in ((0, TOL64), (1, TOL32)):
        out = _apply_s(torch, s, psi, prec)
        worst = 0.0
        for ik, r in ref.items():
            n = s.npw[ik]
            worst = max(worst, np.max(np.abs(out[ik, :, :n] - r)))
            assert np.all(out[ik, :, n:] == 0)
        print(cfg.name, prec, "S psi rel err", worst / scale)
        assert worst <= tol * scale
    # the overlap term is not negligible on these inputs
    assert max(np.max(np.abs(r - psi[ik, :, :s.npw[ik]])) for ik, r in ref.items()) > 1e-2 * scale


def test_s_psi_without_overlap_and_in_place():
    from paper_2412_01695_amd import mkpw
    cfg = synth.with_overlap(synth.make_config(1))
    torch, s = _system(cfg)
    psi = s.psi_guess()
    with_q = _apply_s(torch, s, psi, 0)
    # in place gives the same result as out of place
    d = to_dev(torch, psi)
    mkpw.pw_s_psi(s.ctx, 0, cfg.nbnd, d, d)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), with_q)
    mkpw.pw_set_qij(s.ctx, None)
    assert np.array_equal(_apply_s(torch, s, psi, 0), psi)


def _check_general(torch, s, psi, eig, tol_res):
    from paper_2412_01695_amd import mkpw
    h = torch.empty_like(psi)
    sp = torch.empty_like(psi)
    torch.cuda.synchronize()
    mkpw.pw_h_psi(s.ctx, mkpw.PW_FP64, eig.shape[1], psi, h)
    mkpw.pw_s_psi(s.ctx, mkpw.PW_FP64, eig.shape[1], psi, sp)
    torch.cuda.synchronize()
    p, hp, spp = psi.cpu().numpy(), h.cpu().numpy(), sp.cpu().numpy()
    for ik in range(s.nk):
        n = s.npw[ik]
        g = p[ik, :, :n].conj() @ spp[ik, :, :n].T
        assert np.max(np.abs(g - np.eye(g.shape[0]))) < 1e-12
        r = hp[ik, :, :n] - eig[ik][:, None] * spp[ik, :, :n]
        assert np.max(np.linalg.norm(r, axis=1)) < tol_res
        assert np.all(p[ik, :, n:] == 0)


@pytest.mark.parametrize("cid,step", [(1, 1), (2, 16)])
def test_generalized_davidson(cid, step):
    from paper_2412_01695_amd import mkpw
    cfg0 = synth.make_config(cid)
    cfg = synth.with_overlap(synth.subset(cfg0, np.arange(0, cfg0.nk, step)))
    torch, s = _system(cfg)
    kps = _kpoints(cfg, s, range(cfg.nk))
    ref = {ik: solvers.lowest_eigpairs(kp.h, cfg.nbnd, kp.s)[0] for ik, kp in kps.items()}
    std = {ik: np.linalg.eigvalsh(kp.h)[:cfg.nbnd] for ik, kp in kps.items()}
    for prec, tol_ry, tol_ha, tol_res in ((0, 1e-10, TOL_FP64_HA, 1e-5), (1, 1e-6, TOL_MIXED_HA, 2e-3)):
        psi = to_dev(torch, s.psi_guess())
        st, eig, iters, conv = mkpw.pw_davidson(s.ctx, prec, cfg.nbnd, psi, s.nk, tol_ry, 300)
        torch.cuda.synchronize()
        assert st == 0 and conv.all()
        err = max(np.max(np.abs(eig[ik] - ref[ik])) for ik in ref)
        shift = max(np.max(np.abs(std[ik] - ref[ik])) for ik in ref)
        print(cfg.name, "prec", prec, "max |eig err| Ha", err, "S moves eigenvalues by", shift,
              "iters", iters.min(), iters.max())
        assert err < tol_ha and shift > 1e-3
        _check_general(torch, s, psi, eig, tol_res)


def _dfpt_case_s(cfg, s, nocc):
    """Oracle S-orthonormal eigenvectors as u, eps, alpha, rhs per k, in library
    order, and the exact solutions."""
    kps = _kpoints(cfg, s, range(cfg.nk))
    dvt = ham.vtilde(synth.dv_grid(cfg))
    u_l = np.zeros((cfg.nk, nocc, s.npwx), complex)
    rhs_l = np.zeros((cfg.nk, nocc, s.npwx), complex)
    eps = np.zeros((cfg.nk, nocc))
    alpha = np.zeros(cfg.nk)
    x_ref = []
    for ik, kp in kps.items():
        w, u = solvers.lowest_eigpairs(kp.h, nocc, kp.s)
        a = solvers.dfpt_alpha(w)
        rhs = solvers.dfpt_rhs(ham.local_matrix(kp.miller, cfg.fft, dvt), u, kp.s)
        perm = miller_map(s.miller[ik], kp.miller)
        n = s.npw[ik]
        u_l[ik, :, :n] = u.T[:, perm]
        rhs_l[ik, :, :n] = rhs.T[:, perm]
        eps[ik] = w
        alpha[ik] = a
        x_ref.append(np.array([solvers.dfpt_solve_exact(solvers.dfpt_matrix(kp.h, u, w[nu], a, kp.s),
                                                        rhs[:, nu])[perm] for nu in range(nocc)]))
    return u_l, rhs_l, eps, alpha, x_ref


@pytest.mark.parametrize("cid,step,nocc", [(1, 1, 5), (3, 128, 16)])
def test_cg_with_overlap(cid, step, nocc):
    from paper_2412_01695_amd import mkpw
    cfg0 = synth.make_config(cid)
    cfg = synth.with_overlap(synth.subset(cfg0, np.arange(0, cfg0.nk, step)))
    torch, s = _system(cfg)
    u, rhs, eps, alpha, x_ref = _dfpt_case_s(cfg, s, nocc)
    du, drhs = to_dev(torch, u), to_dev(torch, rhs)
    for prec in (0, 1):
        dx = torch.zeros_like(drhs)
        torch.cuda.synchronize()
        st, iters = mkpw.pw_dfpt_cg(s.ctx, prec, nocc, du, eps, alpha, nocc, drhs, dx, 1e-24, 1000)
        torch.cuda.synchronize()
        assert st == 0
        x = dx.cpu().numpy()
        worst = 0.0
        for ik in range(cfg.nk):
            n = s.npw[ik]
            for nu in range(nocc):
                ref = x_ref[ik][nu]
                worst = max(worst, np.linalg.norm(x[ik, nu, :n] - ref) / np.linalg.norm(ref))
            assert np.all(x[ik, :, n:] == 0)
        print(cfg.name, "CG prec", prec, "worst rel err", worst, "iters", iters.min(), iters.max())
        assert worst < 1e-9
