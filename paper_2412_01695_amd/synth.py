"""Seeded synthetic inputs shared by the library harness and the oracle tests.

This module only *defines inputs*: the crystal (fcc lattice, atoms), the
k-point lists, the local potential sampled on the real-space grid, the
analytic projector functions, the D coefficients, the initial wavefunction
guesses and the DFPT perturbing potential.  It holds none of the method's
arithmetic (no plane-wave sphere, no Fourier transform of a wavefunction,
no Hamiltonian, no solver).  Both sides call it on their own plane-wave
lists (Miller indices), and every value it returns depends only on the seed
and on the Miller index / Cartesian vector it is asked about, never on the
order of the list it is given.

Units: lengths in bohr, energies in Hartree, cutoffs in Ry
(the sphere is |k+G|^2 < ecut_Ry in bohr^-2).

The five workloads are small-cell metals sampled on dense k meshes, the
situation the many-k method targets (paper, Introduction and Sec. 5.1); the
paper's own bcc-W PAW system cannot be reproduced here (no pseudopotential
data), so Gaussian model potentials stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

A_FCC = 7.6  # bohr


def fcc_lattice(a: float = A_FCC) -> np.ndarray:
    """Rows a1, a2, a3 of the fcc primitive cell (bohr)."""
    h = 0.5 * a
    return np.array([[0.0, h, h], [h, 0.0, h], [h, h, 0.0]], dtype=np.float64)


def reciprocal_rows(lat: np.ndarray) -> np.ndarray:
    """Rows b1, b2, b3 with a_i . b_j = 2 pi delta_ij (needed to place k-points)."""
    return 2.0 * math.pi * np.linalg.inv(lat).T


def mp_grid(n1: int, n2: int, n3: int, lat: np.ndarray) -> np.ndarray:
    """Monkhorst-Pack mesh u_r = (2r - n - 1)/(2n), r = 1..n, no symmetry
    reduction, r1 outermost; returns Cartesian k (nk, 3) in bohr^-1."""
    b = reciprocal_rows(lat)
    u = [np.array([(2 * r - n - 1) / (2.0 * n) for r in range(1, n + 1)]) for n in (n1, n2, n3)]
    f = np.array(np.meshgrid(u[0], u[1], u[2], indexing="ij")).reshape(3, -1).T
    return f @ b


@dataclass
class Projector:
    atom: int        # index into Config.tau
    rc: float        # Gaussian radius (bohr)
    l: int           # 0 = s, 1 = p
    alpha: int = -1  # Cartesian component for p (0, 1, 2)


@dataclass
class Config:
    name: str
    lat: np.ndarray
    ecut_ry: float
    fft: tuple
    kpts: np.ndarray             # (nk, 3) Cartesian bohr^-1
    nbnd: int
    tau: np.ndarray              # (nat, 3) Cartesian bohr
    projectors: list
    dij: np.ndarray              # (nproj, nproj) complex Hermitian, Ha
    seed: int
    extra: dict = field(default_factory=dict)
    qij: np.ndarray | None = None  # (nproj, nproj) complex Hermitian overlap coefficients; None: S = 1

    @property
    def omega(self) -> float:
        return float(abs(np.linalg.det(self.lat)))

    @property
    def nk(self) -> int:
        return int(self.kpts.shape[0])

    @property
    def nproj(self) -> int:
        return len(self.projectors)


def _sp_projectors(atoms, rcs):
    out = []
    for ia in atoms:
        for rc in rcs:
            out.append(Projector(ia, rc, 0))
            for al in range(3):
                out.append(Projector(ia, rc, 1, al))
    return out


def _d_one_channel(nat: int) -> np.ndarray:
    d = np.zeros((4 * nat, 4 * nat), dtype=np.complex128)
    for ia in range(nat):
        o = 4 * ia
        d[o, o] = 0.5
        for al in range(3):
            d[o + 1 + al, o + 1 + al] = -0.2
    return d


def _d_two_channel() -> np.ndarray:
    # order: s(rc1), p(rc1) x3, s(rc2), p(rc2) x3 ; couples channels of the same (l, m)
    d = np.zeros((8, 8), dtype=np.complex128)
    d[0, 0], d[0, 4], d[4, 0], d[4, 4] = 0.5, 0.1, 0.1, 0.3
    for al in range(3):
        i, j = 1 + al, 5 + al
        d[i, i], d[i, j], d[j, i], d[j, j] = -0.2, 0.05, 0.05, -0.1
    return d


def q_model(cfg: Config) -> np.ndarray:
    """Model overlap coefficients q_pq (Ha-free, Hermitian, positive definite)
    with the block structure of D: per atom, q = 16 on s and 12 on each p of
    a single channel; with two radial channels the same (l, m) are coupled,
    s [[16, 4], [4, 10]] and p [[12, 3], [3, 8]].  With these values the
    projector term of S is of order 0.1 - 0.5, like an augmentation charge."""
    n = cfg.nproj
    q = np.zeros((n, n), dtype=np.complex128)
    by_atom = {}
    for i, pr in enumerate(cfg.projectors):
        by_atom.setdefault(pr.atom, []).append(i)
    for idx in by_atom.values():
        rcs = sorted({cfg.projectors[i].rc for i in idx})
        for i in idx:
            pi = cfg.projectors[i]
            for j in idx:
                pj = cfg.projectors[j]
                if pi.l != pj.l or pi.alpha != pj.alpha:
                    continue
                ci, cj = rcs.index(pi.rc), rcs.index(pj.rc)
                blk = ((16.0, 4.0), (4.0, 10.0)) if pi.l == 0 else ((12.0, 3.0), (3.0, 8.0))
                q[i, j] = blk[ci][cj]
    return q


def with_overlap(cfg: Config, qij=None) -> Config:
    """The same workload with the overlap S = 1 + sum_pq |beta_p> q_pq <beta_q|
    (`q_model` unless `qij` is given)."""
    c = Config(cfg.name + "-uspp", cfg.lat, cfg.ecut_ry, cfg.fft, cfg.kpts, cfg.nbnd, cfg.tau,
               cfg.projectors, cfg.dij, cfg.seed, dict(cfg.extra))
    c.qij = q_model(cfg) if qij is None else np.asarray(qij, dtype=np.complex128)
    return c


def q_paper() -> np.ndarray:
    """The phonon wavevector of the paper's benchmark, (2 pi / a)(-1/8, -1/4, 3/8), here
    in units of this cell's a (Cartesian bohr^-1)."""
    return (2.0 * math.pi / A_FCC) * np.array([-0.125, -0.25, 0.375])


def shifted(cfg: Config, q_cart) -> Config:
    """The same workload with every k-point moved by q (the k+q list of a response
    calculation at wavevector q)."""
    c = Config(cfg.name + "-kq", cfg.lat, cfg.ecut_ry, cfg.fft, cfg.kpts + np.asarray(q_cart)[None, :],
               cfg.nbnd, cfg.tau, cfg.projectors, cfg.dij, cfg.seed, dict(cfg.extra), cfg.qij)
    return c


def dv_complex_grid(cfg: Config, seed: int = 11) -> np.ndarray:
    """A complex lattice-periodic perturbation (the periodic part of a potential at
    q != 0 need not be real): sum over 0 < |G|^2 <= 4 (2 pi/a)^2 of
    c_G exp(iG.r) / (1 + |G|^2), c_G = exp(i phi_G), phi ~ U[0, 2 pi) from `seed`."""
    g2max = 4.0 * (2.0 * math.pi / A_FCC) ** 2
    m, g = _lattice_vectors_in_sphere(cfg.lat, g2max)
    keep = np.any(m != 0, axis=1)
    m, g = m[keep], g[keep]
    phi = np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, size=m.shape[0])
    amp = 1.0 / (1.0 + np.einsum("ij,ij->i", g, g))
    fr = _grid_frac(cfg.fft)
    out = np.zeros(fr.shape[0], dtype=np.complex128)
    for j in range(m.shape[0]):
        out += amp[j] * np.exp(1j * (phi[j] + 2.0 * math.pi * (fr @ m[j])))
    return out.reshape(cfg.fft)


def make_config(cid: int) -> Config:
    """The four batch workloads (ids 1..4); id 5 is the serving stream (`serving_requests`)."""
    lat = fcc_lattice()
    tp = 2.0 * math.pi / A_FCC
    one_atom = np.zeros((1, 3))
    two_atoms = np.array([[0.0, 0.0, 0.0], [0.25 * A_FCC] * 3])
    if cid == 1:
        k = tp * np.array([[0, 0, 0], [0.25, 0, 0], [0.25, 0.25, 0.25], [-0.125, -0.25, 0.375]])
        return Config("fcc1-ecut15-fft15-4k", lat, 15.0, (15, 15, 15), k, 8, one_atom,
                      _sp_projectors([0], [1.0]), _d_one_channel(1), 1696)
    if cid == 2:
        return Config("fcc1-ecut30-fft24-512k", lat, 30.0, (24, 24, 24), mp_grid(8, 8, 8, lat), 20,
                      one_atom, _sp_projectors([0], [1.0, 1.6]), _d_two_channel(), 1697)
    if cid == 3:
        return Config("fcc2-ecut30-fft30-2048k", lat, 30.0, (30, 30, 30), mp_grid(16, 16, 8, lat), 16,
                      two_atoms, _sp_projectors([0, 1], [1.0]), _d_one_channel(2), 1698,
                      extra={"nocc": 16, "nrhs": 16, "dv_seed": 7})
    if cid == 4:
        return Config("fcc1-ecut40-fft36-1728k", lat, 40.0, (36, 36, 36), mp_grid(12, 12, 12, lat), 24,
                      one_atom, _sp_projectors([0], [1.0]), _d_one_channel(1), 1699)
    raise ValueError(f"unknown config id {cid}")


def gapped(cfg: Config, scale: float = 32.0, nocc: int = 8) -> Config:
    """The same workload with a local potential `scale` times deeper, which
    opens a gap above band `nocc` over the whole Brillouin zone (an insulator):
    for the two-atom cell, scale 32 leaves about 0.3 Ha between bands 8 and 9
    over the k and k+q lists at the paper's q, so that the DFPT systems at
    q != 0 are positive definite on the conduction states.  `nb_solve` is the
    band count for the eigensolver: nocc + 4, the three above the first empty
    band being buffer bands (at some k bands 9 and 10, or 12 and 13, come
    within 0.002 Ha, which slows the convergence of the top band of a block)."""
    c = Config(cfg.name.replace("fcc2", f"fcc2x{scale:g}") + f"-nocc{nocc}", cfg.lat, cfg.ecut_ry, cfg.fft,
               cfg.kpts, cfg.nbnd, cfg.tau, cfg.projectors, cfg.dij, cfg.seed,
               dict(cfg.extra, vloc_scale=float(scale), nocc=nocc, nrhs=nocc, nb_solve=nocc + 4), cfg.qij)
    return c


def subset(cfg: Config, ks) -> Config:
    """Same crystal and cutoff on a subset of the k-list (indices `ks`)."""
    ks = np.asarray(ks, dtype=np.int64)
    c = Config(cfg.name + f"-sub{len(ks)}", cfg.lat, cfg.ecut_ry, cfg.fft, cfg.kpts[ks].copy(),
               cfg.nbnd, cfg.tau, cfg.projectors, cfg.dij, cfg.seed, dict(cfg.extra), cfg.qij)
    c.extra["k_index"] = ks
    return c


# ----------------------------------------------------------------------------- real-space fields

def _grid_frac(fft):
    n1, n2, n3 = fft
    l = np.array(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3,
                             indexing="ij")).reshape(3, -1).T
    return l  # (Nr, 3) fractional coordinates, C order (l3 fastest)


def _lattice_vectors_in_sphere(lat, g2max):
    b = reciprocal_rows(lat)
    mmax = [int(math.ceil(math.sqrt(g2max) * np.linalg.norm(lat[i]) / (2 * math.pi))) + 1 for i in range(3)]
    r = [np.arange(-m, m + 1) for m in mmax]
    m = np.array(np.meshgrid(*r, indexing="ij")).reshape(3, -1).T
    g = m @ b
    keep = np.einsum("ij,ij->i", g, g) <= g2max
    m, g = m[keep], g[keep]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0]))
    return m[order], g[order]


def _cos_sum(fft, lat, mill, coef_re, coef_im, shift_frac):
    """f(r_l) = sum_j Re[(coef_re + i coef_im)_j exp(i 2pi m_j . (l/N - shift))], chunked."""
    fr = _grid_frac(fft)
    out = np.zeros(fr.shape[0])
    for s in range(0, mill.shape[0], 256):
        ph = 2.0 * math.pi * ((fr[None, :, :] - shift_frac[None, None, :]) * mill[s:s + 256, None, :]).sum(-1)
        out += (coef_re[s:s + 256, None] * np.cos(ph) - coef_im[s:s + 256, None] * np.sin(ph)).sum(0)
    return out.reshape(fft)


def vloc_grid(cfg: Config) -> np.ndarray:
    """V_loc(r) on the FFT grid, real, Ha, C order (N1, N2, N3).

    Model potential V(G) = -3 exp(-|G|^2/2) / Omega per atom, summed over the
    reciprocal lattice vectors with |G|^2 <= 4 ecut (the density cutoff) and
    placed at each atom with the structure factor exp(-i G.tau)."""
    m, g = _lattice_vectors_in_sphere(cfg.lat, 4.0 * cfg.ecut_ry)
    depth = 3.0 * float(cfg.extra.get("vloc_scale", 1.0))
    vg = -depth * np.exp(-0.5 * np.einsum("ij,ij->i", g, g)) / cfg.omega
    out = np.zeros(cfg.fft)
    inv_lat = np.linalg.inv(cfg.lat)
    for t in cfg.tau:
        out += _cos_sum(cfg.fft, cfg.lat, m, vg, np.zeros_like(vg), t @ inv_lat)
    return out


def dv_grid(cfg: Config, seed: int = 7) -> np.ndarray:
    """Smooth random-phase perturbing potential dV(r) (real, Ha):
    Re sum_{0<|G|^2<=4(2pi/a)^2} exp(i phi_G)/(1+|G|^2) exp(iG.r), phi ~ U[0, 2pi)
    drawn in Miller-lexicographic order from `seed`."""
    g2max = 4.0 * (2.0 * math.pi / A_FCC) ** 2
    m, g = _lattice_vectors_in_sphere(cfg.lat, g2max)
    keep = np.any(m != 0, axis=1)
    m, g = m[keep], g[keep]
    phi = np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, size=m.shape[0])
    amp = 1.0 / (1.0 + np.einsum("ij,ij->i", g, g))
    return _cos_sum(cfg.fft, cfg.lat, m, amp * np.cos(phi), amp * np.sin(phi), np.zeros(3))


# ----------------------------------------------------------------------------- G-space inputs

def q_vectors(cfg: Config, ik: int, miller: np.ndarray) -> np.ndarray:
    """Cartesian k+G for the given Miller indices (npw, 3)."""
    return cfg.kpts[ik][None, :] + np.asarray(miller, dtype=np.float64) @ reciprocal_rows(cfg.lat)


def beta_values(cfg: Config, q: np.ndarray) -> np.ndarray:
    """Projector functions beta_p(q) for q = k+G (nproj, npw) complex128.

    s:   Omega^-1/2 exp(-q^2 rc^2/2) exp(-i q.tau)
    p_a: Omega^-1/2 (-i) q_a rc exp(-q^2 rc^2/2) exp(-i q.tau)
    (the (-i)^l factor keeps beta(r) real)."""
    q = np.asarray(q, dtype=np.float64)
    q2 = np.einsum("ij,ij->i", q, q)
    out = np.empty((len(cfg.projectors), q.shape[0]), dtype=np.complex128)
    radial, phase = {}, {}
    for p, pr in enumerate(cfg.projectors):
        if pr.rc not in radial:
            radial[pr.rc] = np.exp(-0.5 * q2 * pr.rc * pr.rc) / math.sqrt(cfg.omega)
        if pr.atom not in phase:
            t = cfg.tau[pr.atom]
            phase[pr.atom] = None if not np.any(t) else np.exp(-1j * (q @ t))
        f = radial[pr.rc] if pr.l == 0 else (-1j * pr.rc) * q[:, pr.alpha] * radial[pr.rc]
        out[p] = f if phase[pr.atom] is None else f * phase[pr.atom]
    return out


_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x):
    """SplitMix64 finaliser (Steele, Lea & Flood 2014; constants as published by
    Vigna) applied elementwise to uint64 arrays (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _normal_pairs(seed, ik, band, miller):
    """Two independent N(0, 1) draws per (seed, k, band, Miller index), from a
    counter-based hash: the value at a plane wave does not depend on which other
    plane waves, k-points or bands are drawn, nor on their order."""
    m = np.asarray(miller, dtype=np.int64)
    key = _splitmix64(np.uint64(seed) * np.ones(1, np.uint64))
    key = _splitmix64(key ^ np.asarray(ik, dtype=np.uint64))
    key = _splitmix64(key[..., None] ^ np.asarray(band, dtype=np.uint64)[None, :])   # (..., nbnd)
    packed = ((m[..., 0] + 512) << 20) | ((m[..., 1] + 512) << 10) | (m[..., 2] + 512)
    h1 = _splitmix64(key[..., :, None] ^ packed.astype(np.uint64)[..., None, :])
    h2 = _splitmix64(h1)
    u1 = 1.0 - (h1 >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)   # (0, 1]
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)         # [0, 1)
    r = np.sqrt(-2.0 * np.log(u1))                                                      # Box-Muller
    return r * np.cos(2.0 * math.pi * u2), r * np.sin(2.0 * math.pi * u2)


def psi_guess(cfg: Config, ik: int, miller: np.ndarray, nbnd: int | None = None,
              seed: int | None = None) -> np.ndarray:
    """Initial wavefunctions (nbnd, npw) complex128, normalised per band.

    psi(G) = (x + i y) / (1 + |k+G|^2/2), x, y ~ N(0, 1) drawn by a
    counter-based hash of (seed, k index, band, Miller index), so the value
    at a plane wave does not depend on the order of `miller`."""
    nbnd = cfg.nbnd if nbnd is None else nbnd
    seed = cfg.seed if seed is None else seed
    miller = np.asarray(miller)
    x, y = _normal_pairs(seed, np.uint64(ik), np.arange(nbnd, dtype=np.uint64), miller)
    z = (x + 1j * y).reshape(nbnd, miller.shape[0])
    q = q_vectors(cfg, ik, miller)
    z /= (1.0 + 0.5 * np.einsum("ij,ij->i", q, q))[None, :]
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    return z


def psi_guess_all(cfg: Config, miller_by_k, npwx: int, nbnd: int | None = None,
                  seed: int | None = None) -> np.ndarray:
    """`psi_guess` for every k at once, in the (nk, nbnd, npwx) layout (zero padding)."""
    nbnd = cfg.nbnd if nbnd is None else nbnd
    seed = cfg.seed if seed is None else seed
    nk = len(miller_by_k)
    npw = np.array([m.shape[0] for m in miller_by_k])
    mm = np.zeros((nk, npwx, 3), dtype=np.int64)
    valid = np.arange(npwx)[None, :] < npw[:, None]
    for ik, m in enumerate(miller_by_k):
        mm[ik, :npw[ik]] = m
    x, y = _normal_pairs(seed, np.arange(nk, dtype=np.uint64), np.arange(nbnd, dtype=np.uint64), mm)
    z = (x + 1j * y) * valid[:, None, :]
    q = cfg.kpts[:, None, :] + mm.astype(np.float64) @ reciprocal_rows(cfg.lat)
    z /= (1.0 + 0.5 * np.einsum("kgi,kgi->kg", q, q))[:, None, :]
    z /= np.linalg.norm(z, axis=2, keepdims=True)
    return z


def random_vectors(seed: int, ik: int, miller: np.ndarray, nvec: int) -> np.ndarray:
    """Plain complex Gaussian vectors (nvec, npw), order-independent like `psi_guess`."""
    miller = np.asarray(miller)
    order = np.lexsort((miller[:, 2], miller[:, 1], miller[:, 0]))
    rng = np.random.default_rng([seed, 977, ik])
    x = rng.standard_normal((nvec, miller.shape[0])) + 1j * rng.standard_normal((nvec, miller.shape[0]))
    z = np.empty_like(x)
    z[:, order] = x
    return z


# ----------------------------------------------------------------------------- serving stream

def fft_rule(lat: np.ndarray, ecut_ry: float) -> tuple:
    """Smallest 2,3,5-smooth N_i >= 2 floor(2 k_c |a_i| / 2pi) + 1 with k_c = sqrt(ecut)."""
    kc = math.sqrt(ecut_ry)

    def smooth(n):
        while True:
            m = n
            for p in (2, 3, 5):
                while m % p == 0:
                    m //= p
            if m == 1:
                return n
            n += 1

    return tuple(smooth(2 * int(math.floor(2 * kc * np.linalg.norm(lat[i]) / (2 * math.pi))) + 1)
                 for i in range(3))


def serving_requests(n: int = 1000, rate: float = 20.0, seed: int = 2024):
    """Poisson stream of Davidson solve requests: arrival times (s) and configs.

    nk ~ U{16..1024}, ecut ~ U[20, 45] Ry, nbnd ~ U{8..32}, nat ~ U{1, 2};
    k-points uniform in the reciprocal cell; request r uses seed 1695 + r."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    reqs = []
    lat = fcc_lattice()
    b = reciprocal_rows(lat)
    for r in range(n):
        nk = int(rng.integers(16, 1025))
        ecut = float(rng.uniform(20.0, 45.0))
        nbnd = int(rng.integers(8, 33))
        nat = int(rng.integers(1, 3))
        kr = np.random.default_rng([1695 + r, 1])
        kf = kr.uniform(-0.5, 0.5, size=(nk, 3))
        tau = np.zeros((1, 3)) if nat == 1 else np.array([[0.0, 0.0, 0.0], [0.25 * A_FCC] * 3])
        cfg = Config(f"req{r}", lat, ecut, fft_rule(lat, ecut), kf @ b, nbnd, tau,
                     _sp_projectors(list(range(nat)), [1.0]), _d_one_channel(nat), 1695 + r)
        reqs.append((float(t[r]), cfg))
    return reqs
