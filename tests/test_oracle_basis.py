"""Pins for the oracle's plane-wave sphere (Sec. 2.2.1 sphere inequality, Sec. 4 G mesh).

The reciprocal lattice of fcc is bcc: G = (2pi/a)(h,k,l) with h,k,l all even
or all odd.  Counting those triples by brute force (a parametrisation that
does not use the b_i vectors at all) and the textbook shell table in
tests/golden/bcc_shells.txt both fix the number of plane waves at k = 0."""
import math
import os

import numpy as np
import pytest

from oracle import basis
from paper_2412_01695_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bcc_shells.txt")


def _bcc_count(n2max, strict=True):
    r = int(math.isqrt(int(n2max))) + 2
    c = 0
    for h in range(-r, r + 1):
        for k in range(-r, r + 1):
            for l in range(-r, r + 1):
                if (h % 2 == k % 2 == l % 2):
                    s = h * h + k * k + l * l
                    if (s < n2max) if strict else (s <= n2max):
                        c += 1
    return c


def test_golden_shells_match_brute_force():
    rows = [tuple(map(int, ln.split())) for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    cum = 0
    for s, n in rows:
        assert _bcc_count(s, strict=False) - _bcc_count(s, strict=True) == n
        cum += n
        assert _bcc_count(s, strict=False) == cum


@pytest.mark.parametrize("n2", [0.5, 3.5, 4.5, 11.5, 20.5, 36.5])
def test_gamma_sphere_counts_bcc_shells(n2):
    lat = synth.fcc_lattice()
    unit = (2 * math.pi / synth.A_FCC) ** 2
    m, q2 = basis.sphere(lat, np.zeros(3), n2 * unit)
    assert m.shape[0] == _bcc_count(n2)


def test_cutoff_is_strict():
    # a cutoff exactly on the |G|^2 = 3 (2pi/a)^2 shell excludes that shell
    lat = synth.fcc_lattice()
    unit = (2 * math.pi / synth.A_FCC) ** 2
    m, q2 = basis.sphere(lat, np.zeros(3), 3.0 * unit * (1 - 1e-15))
    assert m.shape[0] == 1
    m, q2 = basis.sphere(lat, np.zeros(3), 3.0 * unit * (1 + 1e-12))
    assert m.shape[0] == 9


def test_sphere_contents_and_order():
    cfg = synth.make_config(1)
    b = basis.reciprocal(cfg.lat)
    np.testing.assert_allclose(cfg.lat @ b.T, 2 * math.pi * np.eye(3), atol=1e-13)
    for ik in range(cfg.nk):
        m, q2 = basis.sphere(cfg.lat, cfg.kpts[ik], cfg.ecut_ry)
        q = cfg.kpts[ik] + m @ b
        np.testing.assert_allclose(np.einsum("ij,ij->i", q, q), q2, rtol=1e-14)
        assert np.all(q2 < cfg.ecut_ry)
        assert np.all(np.diff(q2) >= 0)
        # brute force over a generous box: nothing inside the sphere is missing
        r = np.arange(-12, 13)
        mm = np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T
        qq = cfg.kpts[ik] + mm @ b
        assert int(np.sum(np.einsum("ij,ij->i", qq, qq) < cfg.ecut_ry)) == m.shape[0]
        assert len({tuple(x) for x in m}) == m.shape[0]


@pytest.mark.parametrize("cid", [1, 2, 3, 4])
def test_configs_injective_on_their_mesh(cid):
    cfg = synth.make_config(cid)
    for ik in range(0, cfg.nk, max(1, cfg.nk // 16)):
        m, _ = basis.sphere(cfg.lat, cfg.kpts[ik], cfg.ecut_ry)
        assert basis.is_injective(m, cfg.fft)


def test_time_reversal_sphere():
    # the sphere at -k is the negated sphere at k
    cfg = synth.make_config(1)
    k = cfg.kpts[3]
    m1, q1 = basis.sphere(cfg.lat, k, cfg.ecut_ry)
    m2, q2 = basis.sphere(cfg.lat, -k, cfg.ecut_ry)
    assert {tuple(x) for x in m1} == {tuple(-x) for x in m2}
