"""Plane-wave basis per k-point (oracle; test infrastructure only).

Sec. 2.2.1 (sphere inequality): the wavefunction at k is expanded on the
reciprocal-lattice vectors G with (1/2)|k+G|^2 < E_cut.  With E_cut quoted in
Ry and energies in Ha this is |k+G|^2 < ecut_Ry (bohr^-2), strict.

Sec. 4 (G mesh): G = m1 b1 + m2 b2 + m3 b3 with integer Miller indices; a
negative m is stored on the FFT mesh at m mod N.

The order of the plane waves inside one k is a convention of this project
(the paper does not fix it): ascending |k+G|^2, ties broken by (m1, m2, m3)
lexicographically.  Tests compare by Miller index, never by position.
"""
from __future__ import annotations

import math

import numpy as np


def reciprocal(lat: np.ndarray) -> np.ndarray:
    """b_j rows with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(np.asarray(lat, dtype=np.float64)).T


def sphere(lat: np.ndarray, k: np.ndarray, ecut_ry: float):
    """Miller indices (npw, 3) int64 and |k+G|^2 (npw,) of the basis at k."""
    b = reciprocal(lat)
    kc = math.sqrt(ecut_ry)
    # |m_i| <= |k+G| |a_i| / 2pi + |k . a_i| / 2pi  (since m_i = (k+G).a_i/2pi - k.a_i/2pi)
    lim = []
    for i in range(3):
        ai = np.asarray(lat[i], dtype=np.float64)
        c = np.dot(k, ai) / (2 * math.pi)
        r = kc * np.linalg.norm(ai) / (2 * math.pi)
        lim.append((int(math.floor(-c - r)) - 1, int(math.ceil(-c + r)) + 1))
    rng = [np.arange(lo, hi + 1) for lo, hi in lim]
    m = np.array(np.meshgrid(*rng, indexing="ij")).reshape(3, -1).T
    q = np.asarray(k)[None, :] + m @ b
    q2 = np.einsum("ij,ij->i", q, q)
    keep = q2 < ecut_ry
    m, q2 = m[keep], q2[keep]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], q2))
    return m[order].astype(np.int64), q2[order]


def kinetic(q2: np.ndarray) -> np.ndarray:
    """Sec. 2.2.1 (kinetic coefficient): C' = (1/2)|k+G|^2 C, in Ha."""
    return 0.5 * q2


def grid_index(miller: np.ndarray, fft) -> np.ndarray:
    """(m1 mod N1, m2 mod N2, m3 mod N3) for each plane wave."""
    n = np.asarray(fft, dtype=np.int64)
    return np.mod(miller, n[None, :])


def is_injective(miller: np.ndarray, fft) -> bool:
    """True when no two plane waves land on the same FFT-mesh point."""
    g = grid_index(miller, fft)
    lin = (g[:, 0] * fft[1] + g[:, 1]) * fft[2] + g[:, 2]
    return np.unique(lin).size == lin.size
