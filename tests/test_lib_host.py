"""Host-side checks of the C-ABI library (no GPU needed).

The library loads, exports every function declared in include/mkpw.h, and
a host-only context (hip_device = -1) builds the same plane-wave spheres as
the oracle and rejects invalid input with the documented status codes."""
import os
import re

import numpy as np
import pytest

from oracle import basis
from paper_2412_01695_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mk():
    from paper_2412_01695_amd import mkpw
    return mkpw


def test_exports_match_header(mk):
    hdr = open(os.path.join(ROOT, "include", "mkpw.h")).read()
    declared = sorted(set(re.findall(r"^\s*(?:pw_status|void|const char\*)\s+(pw_\w+)\(", hdr, re.M)))
    assert declared == sorted(mk.EXPORTS)
    import ctypes
    lib = ctypes.CDLL(mk.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name)


def _host_ctx(mk, cfg):
    ctx = mk.pw_create(-1, None)
    mk.pw_set_lattice(ctx, cfg.lat)
    mk.pw_set_cutoff(ctx, cfg.ecut_ry, cfg.fft)
    return ctx


@pytest.mark.parametrize("cid", [1, 2, 3, 4])
def test_miller_sets_match_oracle(mk, cid):
    cfg = synth.make_config(cid)
    ctx = _host_ctx(mk, cfg)
    try:
        npw, npwx = mk.pw_set_kpoints(ctx, cfg.kpts)
        assert npwx % 64 == 0 and npwx >= npw.max() and npwx - npw.max() < 64
        for ik in range(0, cfg.nk, max(1, cfg.nk // 40)):
            m = mk.pw_get_miller(ctx, ik, npw[ik])
            mo, q2 = basis.sphere(cfg.lat, cfg.kpts[ik], cfg.ecut_ry)
            assert npw[ik] == mo.shape[0]
            assert {tuple(x) for x in m} == {tuple(x) for x in mo}
            # library order: ascending |k+G|^2
            q = synth.q_vectors(cfg, ik, m)
            qq = np.einsum("ij,ij->i", q, q)
            assert np.all(np.diff(qq) >= -1e-12)
            # no plane wave within 1e-9 of the cutoff (no ambiguous membership)
            assert np.min(np.abs(q2 - cfg.ecut_ry)) > 1e-9
    finally:
        mk.pw_destroy(ctx)


def test_auto_fft_rule(mk):
    cfg = synth.make_config(2)
    ctx = mk.pw_create(-1, None)
    mk.pw_set_lattice(ctx, cfg.lat)
    mk.pw_set_cutoff(ctx, 30.0, (0, 0, 0))
    npw, npwx = mk.pw_set_kpoints(ctx, cfg.kpts[:4])
    assert npw.min() > 0
    mk.pw_destroy(ctx)


def test_error_paths(mk):
    cfg = synth.make_config(1)
    ctx = mk.pw_create(-1, None)
    with pytest.raises(mk.PwError) as e:
        mk.pw_set_cutoff(ctx, 15.0, (15, 15, 15))
    assert e.value.status == mk.PW_ESTATE
    with pytest.raises(mk.PwError) as e:
        mk.pw_set_lattice(ctx, np.zeros(9))
    assert e.value.status == mk.PW_EINVAL
    mk.pw_set_lattice(ctx, cfg.lat)
    with pytest.raises(mk.PwError) as e:
        mk.pw_set_option(ctx, "no_such_option", 1)
    assert e.value.status == mk.PW_EINVAL
    # a mesh too small for the sphere
    mk.pw_set_cutoff(ctx, 15.0, (6, 6, 6))
    with pytest.raises(mk.PwError) as e:
        mk.pw_set_kpoints(ctx, cfg.kpts)
    assert e.value.status == mk.PW_EINVAL and "too small" in str(e.value)
    mk.pw_set_cutoff(ctx, 15.0, (15, 15, 15))
    npw, npwx = mk.pw_set_kpoints(ctx, cfg.kpts)
    # non-Hermitian D
    beta = np.zeros((cfg.nk, 4, npwx), dtype=np.complex128)
    d = cfg.dij.copy()
    d[0, 1] = 0.3
    with pytest.raises(mk.PwError) as e:
        mk.pw_set_projectors(ctx, beta, d)
    assert e.value.status == mk.PW_EINVAL
    mk.pw_set_projectors(ctx, beta, cfg.dij)
    # a host-only context runs no device work
    with pytest.raises(mk.PwError) as e:
        mk.pw_h_psi(ctx, mk.PW_FP64, 4, 0, 0)
    assert e.value.status == mk.PW_ESTATE
    # non-finite potential
    v = np.zeros(cfg.fft)
    v[1, 2, 3] = np.nan
    with pytest.raises(mk.PwError) as e:
        mk.pw_set_vloc(ctx, v)
    assert e.value.status == mk.PW_EINVAL
    mk.pw_destroy(ctx)


def test_overlap_coefficients(mk):
    # q needs projectors first, must be Hermitian, and goes away with new projectors or NULL
    cfg = synth.make_config(1)
    ctx = _host_ctx(mk, cfg)
    try:
        npw, npwx = mk.pw_set_kpoints(ctx, cfg.kpts)
        q = synth.q_model(cfg)
        with pytest.raises(mk.PwError) as e:
            mk.pw_set_qij(ctx, q)
        assert e.value.status == mk.PW_ESTATE
        beta = np.zeros((cfg.nk, cfg.nproj, npwx), dtype=np.complex128)
        mk.pw_set_projectors(ctx, beta, cfg.dij)
        assert mk.pw_get_option(ctx, "overlap") == 0
        bad = q.copy()
        bad[0, 1] = 0.2 + 0.1j
        with pytest.raises(mk.PwError) as e:
            mk.pw_set_qij(ctx, bad)
        assert e.value.status == mk.PW_EINVAL and "Hermitian" in str(e.value)
        bad = q.copy()
        bad[2, 2] = np.inf
        with pytest.raises(mk.PwError) as e:
            mk.pw_set_qij(ctx, bad)
        assert e.value.status == mk.PW_EINVAL
        herm = q.copy()
        herm[0, 1], herm[1, 0] = 0.2 + 0.1j, 0.2 - 0.1j
        mk.pw_set_qij(ctx, herm)
        assert mk.pw_get_option(ctx, "overlap") == 1
        mk.pw_set_qij(ctx, None)
        assert mk.pw_get_option(ctx, "overlap") == 0
        mk.pw_set_qij(ctx, q)
        mk.pw_set_projectors(ctx, beta, cfg.dij)     # new projectors drop q
        assert mk.pw_get_option(ctx, "overlap") == 0
        mk.pw_set_qij(ctx, q)
        mk.pw_set_kpoints(ctx, cfg.kpts)              # so do new k-points
        assert mk.pw_get_option(ctx, "overlap") == 0
        with pytest.raises(mk.PwError) as e:
            mk.pw_s_psi(ctx, mk.PW_FP64, 4, 0, 0)
        assert e.value.status == mk.PW_ESTATE
    finally:
        mk.pw_destroy(ctx)


def test_shape_options(mk):
    # the H|psi> launch-shape options: accepted values round-trip, others are refused
    ctx = mk.pw_create(-1, None)
    for key, good, bad in (("hpsi_variant", (0, 1, 2, 3, 4, 5), (-1, 6)), ("hpsi_threads", (0, 256, 512, 1024), (128, 300)),
                           ("hpsi_slab", (0, 1, 36), (-1, 513)), ("tune_log", (0, 1), ()),
                           ("cg_switch_digits", (2, 10, 20), (1, 21)), ("dav_nconv", (0, 8, 1024), (-1, 1025)),
                           ("mixed_switch_rtol_e7", (100, 2000, 100000), (99, 100001))):
        for v in good:
            mk.pw_set_option(ctx, key, v)
            assert mk.pw_get_option(ctx, key) == v
        for v in bad:
            with pytest.raises(mk.PwError) as e:
                mk.pw_set_option(ctx, key, v)
            assert e.value.status == mk.PW_EINVAL
    ctx2 = mk.pw_create(-1, None)
    assert mk.pw_get_option(ctx2, "mixed_switch_rtol_e7") == 2000  # default: residual 2e-4
    mk.pw_destroy(ctx2)
    for key in ("hpsi_variant_tuned", "hpsi_slab_tuned", "hpsi_threads_tuned"):
        assert mk.pw_get_option(ctx, key) == 0  # nothing launched yet
    mk.pw_destroy(ctx)


def test_single_hip_runtime_whatever_the_import_order():
    # the binding must bind the library to torch's HIP runtime even when it is
    # imported before torch; two runtimes in one process crash on first use
    import subprocess
    import sys
    code = ("import paper_2412_01695_amd.mkpw, torch; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


class _FakeDev:
    """Stands in for a device tensor in the binding's argument checks (its
    pointer is never used: the host-only context refuses device work)."""

    def __init__(self, shape, dtype, contiguous=True, device="cuda"):
        self.shape, self.dtype, self._c = tuple(shape), "torch." + dtype, contiguous
        self.device = type("D", (), {"type": device})()

    def data_ptr(self):
        return 0

    def is_contiguous(self):
        return self._c


def test_binding_checks_device_arrays_against_the_context(mk):
    cfg = synth.make_config(1)
    ctx = _host_ctx(mk, cfg)
    try:
        npw, npwx = mk.pw_set_kpoints(ctx, cfg.kpts)
        assert mk.pw_get_option(ctx, "nk") == cfg.nk and mk.pw_get_option(ctx, "npwx") == npwx
        assert [mk.pw_get_option(ctx, f"fft{i}") for i in (1, 2, 3)] == list(cfg.fft)
        good = (cfg.nk, 8, npwx)
        bad_cases = [
            ((cfg.nk - 1, 8, npwx), "complex128", True, "cuda"),   # too few k-points
            ((cfg.nk, 8, npwx - 64), "complex128", True, "cuda"),  # short rows
            (good, "complex64", True, "cuda"),                     # complex64 on the FP64 path
            (good, "complex128", False, "cuda"),                   # a strided view
            (good, "complex128", True, "cpu"),                     # host memory
        ]
        for shape, dt, contig, dev in bad_cases:
            with pytest.raises(ValueError):
                mk.pw_h_psi(ctx, mk.PW_FP64, 8, _FakeDev(shape, dt, contig, dev), _FakeDev(good, "complex128"))
        with pytest.raises(ValueError):  # complex128 on the mixed path
            mk.pw_h_psi(ctx, mk.PW_MIXED, 8, _FakeDev(good, "complex128"), _FakeDev(good, "complex128"))
        with pytest.raises(ValueError):  # nk that is not the context's
            mk.pw_davidson(ctx, mk.PW_FP64, 8, _FakeDev(good, "complex128"), cfg.nk + 1, 1e-10, 10)
        with pytest.raises(ValueError):  # eps with the wrong number of systems
            mk.pw_dfpt_cg(ctx, mk.PW_FP64, 8, _FakeDev(good, "complex128"), np.zeros((cfg.nk, 7)), np.ones(cfg.nk),
                          8, _FakeDev(good, "complex128"), _FakeDev(good, "complex128"), 1e-20, 10)
        with pytest.raises(ValueError):  # projector rows of the wrong length
            mk.pw_set_projectors(ctx, np.zeros((cfg.nk, 4, npwx - 1), complex), np.eye(4))
        with pytest.raises(ValueError):  # Miller count that is not the k-point's
            mk.pw_get_miller(ctx, 0, int(npw[0]) - 1)
        # arrays that pass the checks reach the library, which refuses device work here
        for prec, dt in ((mk.PW_FP64, "complex128"), (mk.PW_MIXED, "complex64")):
            with pytest.raises(mk.PwError) as e:
                mk.pw_h_psi(ctx, prec, 8, _FakeDev(good, dt), _FakeDev(good, dt))
            assert e.value.status == mk.PW_ESTATE
    finally:
        mk.pw_destroy(ctx)
