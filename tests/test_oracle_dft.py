"""Pins for the oracle's separable DFT (Sec. 4, Eqs. zfft, yfft, xfft, fwFFT).

Closed forms (delta <-> single plane wave), the inverse/forward pair being
the identity (1/N_r on the forward side only), Parseval, separability, and
agreement with numpy.fft as an independent library."""
import math

import numpy as np
import pytest

from oracle import dft

SHAPES = [(3, 4, 5), (15, 15, 15), (6, 10, 9)]


@pytest.mark.parametrize("shape", SHAPES)
def test_inverse_of_delta_is_plane_wave(shape):
    m0 = (1, shape[1] - 2, 3 % shape[2])
    ft = np.zeros(shape, dtype=np.complex128)
    ft[m0] = 1.0
    f = dft.inverse(ft)
    l = np.array(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"))
    ph = 2 * math.pi * sum(l[i] * m0[i] / shape[i] for i in range(3))
    np.testing.assert_allclose(f, np.exp(1j * ph), atol=1e-13)


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_of_plane_wave_is_unit_delta(shape):
    m0 = (shape[0] - 1, 2, 1)
    l = np.array(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"))
    ph = 2 * math.pi * sum(l[i] * m0[i] / shape[i] for i in range(3))
    ft = dft.forward(np.exp(1j * ph))
    ref = np.zeros(shape)
    ref[m0] = 1.0
    np.testing.assert_allclose(ft, ref, atol=1e-13)


@pytest.mark.parametrize("shape", SHAPES)
def test_roundtrip_and_parseval(shape):
    rng = np.random.default_rng(0)
    ft = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    f = dft.inverse(ft)
    np.testing.assert_allclose(dft.forward(f), ft, atol=1e-12)
    n = np.prod(shape)
    assert abs(np.sum(np.abs(f) ** 2) - n * np.sum(np.abs(ft) ** 2)) < 1e-9 * n * np.sum(np.abs(ft) ** 2)


@pytest.mark.parametrize("shape", SHAPES)
def test_matches_numpy_fft(shape):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    n = np.prod(shape)
    np.testing.assert_allclose(dft.inverse(x), n * np.fft.ifftn(x), atol=1e-11)
    np.testing.assert_allclose(dft.forward(x), np.fft.fftn(x) / n, atol=1e-13)


def test_separable_axis_by_axis():
    # a product of 1D functions transforms into the product of 1D transforms
    rng = np.random.default_rng(2)
    shape = (5, 6, 4)
    a = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in shape]
    ft = a[0][:, None, None] * a[1][None, :, None] * a[2][None, None, :]
    one = [n * np.fft.ifft(v) for v, n in zip(a, shape)]
    ref = one[0][:, None, None] * one[1][None, :, None] * one[2][None, None, :]
    np.testing.assert_allclose(dft.inverse(ft), ref, atol=1e-12)


def test_dft_matrix_unitary_up_to_n():
    for n in (7, 15, 24, 36):
        w = dft.dft_matrix(n, +1)
        np.testing.assert_allclose(w @ w.conj().T, n * np.eye(n), atol=1e-11)
        np.testing.assert_allclose(dft.dft_matrix(n, -1), w.conj(), atol=1e-15)
