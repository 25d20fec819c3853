"""Separable 3D discrete Fourier transform, written out (oracle; test infrastructure only).

Sec. 4 defines the transform pair on the N1 x N2 x N3 mesh:
  inverse  f(l) = sum_m  f~(m) exp(+i 2pi l.m/N)       (no normalisation)
  forward  f~(m) = (1/N_r) sum_l f(l) exp(-i 2pi l.m/N)  (Eq. fwFFT)
and evaluates the inverse as three 1D passes: over m3 (Eq. zfft), then m2
(Eq. yfft), then m1 (Eq. xfft).  Here each 1D pass is the plain O(N^2) sum,
applied as a matrix product with the DFT matrix of that axis (the paper
notes these sums cost N_i^2 and are replaced by FFTs on the device; the
oracle keeps the plain sums).

Arrays are C ordered (l1, l2, l3) with l3 fastest.
"""
from __future__ import annotations

import math

import numpy as np


def dft_matrix(n: int, sign: int) -> np.ndarray:
    """W[l, m] = exp(sign * i 2pi l m / n)  (l m reduced mod n before the angle)."""
    lm = np.mod(np.outer(np.arange(n), np.arange(n)), n)
    ang = sign * 2.0 * math.pi * lm / n
    return np.cos(ang) + 1j * np.sin(ang)


def _pass(f: np.ndarray, axis: int, sign: int) -> np.ndarray:
    w = dft_matrix(f.shape[axis], sign)
    g = np.moveaxis(f, axis, -1)
    g = g @ w.T            # out[..., l] = sum_m in[..., m] W[l, m]
    return np.moveaxis(g, -1, axis)


def inverse(ft: np.ndarray) -> np.ndarray:
    """Reciprocal -> real space: z pass (Eq. zfft), y pass (Eq. yfft), x pass (Eq. xfft)."""
    f = np.asarray(ft, dtype=np.complex128)
    f = _pass(f, 2, +1)
    f = _pass(f, 1, +1)
    f = _pass(f, 0, +1)
    return f


def forward(f: np.ndarray) -> np.ndarray:
    """Real -> reciprocal space with the 1/N_r factor (Eq. fwFFT)."""
    g = np.asarray(f, dtype=np.complex128)
    g = _pass(g, 0, -1)
    g = _pass(g, 1, -1)
    g = _pass(g, 2, -1)
    return g / g.size
