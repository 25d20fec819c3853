"""pw_h_psi_noalloc (the H|psi> entry point that allocates nothing) against
pw_h_psi through the C-ABI: two calls in a row, the second on a smaller
input (fewer k-points, fewer bands, a smaller mesh), in FP64 and in mixed
precision, each within the H|psi> parity bars (FP64 1e-13, complex64 2e-6 of
the largest element)."""
import numpy as np
import pytest

from paper_2412_01695_amd import synth

from gpu_util import to_dev, torch_cuda

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 2e-6}


def _both(torch, mkpw, s, prec, psi):
    dt = torch.complex128 if prec == 0 else torch.complex64
    d = to_dev(torch, psi, dt)
    h_ref = torch.full_like(d, float("nan"))
    h_new = torch.full_like(d, float("nan"))
    torch.cuda.synchronize()
    held = mkpw.pw_get_option(s.ctx, "device_bytes")
    mkpw.pw_h_psi_noalloc(s.ctx, prec, psi.shape[1], d, h_new)   # first, on a fresh context
    torch.cuda.synchronize()
    assert mkpw.pw_get_option(s.ctx, "device_bytes") == held    # it allocated nothing
    mkpw.pw_h_psi(s.ctx, prec, psi.shape[1], d, h_ref)
    torch.cuda.synchronize()
    return h_ref.cpu().numpy(), h_new.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_h_psi_twice(prec):
    torch = torch_cuda()
    from paper_2412_01695_amd import mkpw
    from paper_2412_01695_amd.system import System
    big = synth.subset(synth.make_config(2), np.arange(0, 512, 3))          # 171 k x 20 bands, 24^3
    small = synth.make_config(1)                                             # 4 k x 8 bands, 15^3
    for cfg in (big, small):
        s = System(cfg, 0)
        try:
            psi = s.psi_guess()
            ref, new = _both(torch, mkpw, s, prec, psi)
            assert np.all(np.isfinite(new))
            scale = np.max(np.abs(ref))
            err = np.max(np.abs(new - ref))
            print(cfg.name, "prec", prec, "max |noalloc - h_psi| / max", err / scale)
            assert err <= TOL[prec] * scale
            for ik in range(cfg.nk):
                assert np.all(new[ik, :, s.npw[ik]:] == 0)
            # a second no-alloc call on the same context leaves its memory unchanged
            d = to_dev(torch, psi, torch.complex128 if prec == 0 else torch.complex64)
            h2 = torch.empty_like(d)
            held = mkpw.pw_get_option(s.ctx, "device_bytes")
            torch.cuda.synchronize()
            mkpw.pw_h_psi_noalloc(s.ctx, prec, cfg.nbnd, d, h2)
            torch.cuda.synchronize()
            assert mkpw.pw_get_option(s.ctx, "device_bytes") == held
            assert np.array_equal(h2.cpu().numpy(), new)
        finally:
            s.close()
