"""Pins of the oracle's real-field transforms: the half spectrum (columns
0..nx/2 of the 2D transform of a real field) and its inverse, defined on the
Hermitian part of the input (the symmetry X[-b][-a] = conj(X[b][a]) of the
transform of real data, Sec. II.B).

Fixed independently of the oracle: numpy.fft.rfft2 and irfft2 (a separate
implementation; numpy's inverse also reads only the Hermitian part of the
a = 0 and a = nx/2 columns), a cosine mode's two-spike half spectrum, the
round trip, and the projection being idempotent; odd sides, whose half
spectrum has no self-conjugate column besides a = 0, included."""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("ny,nx", [(4, 2), (2, 8), (16, 16), (32, 8), (8, 64), (5, 3), (6, 15), (7, 7),
                                   (12, 9), (3, 10)])
def test_rfft2d_matches_numpy_and_round_trips(ny, nx):
    x = np.random.default_rng(nx * 31 + ny).standard_normal((ny, nx))
    X = oracle.rfft2d(x)
    assert X.shape == (ny, nx // 2 + 1)
    assert np.abs(X - np.fft.rfft2(x)).max() <= 1e-13 * max(1.0, np.abs(X).max())
    assert np.abs(oracle.irfft2d(X, nx) - x).max() <= 1e-14 * nx * ny


def test_half_spectrum_of_a_cosine_mode():
    ny, nx, m, n = 16, 32, 3, 5
    j, k = np.meshgrid(np.arange(nx), np.arange(ny))
    x = np.cos(2 * math.pi * (m * j / nx + n * k / ny))
    X = oracle.rfft2d(x)
    ref = np.zeros_like(X)
    ref[n, m] = nx * ny / 2          # the +(m, n) exponential
    # -(m, n) lands at column nx - m > nx/2, outside the half spectrum
    assert np.abs(X - ref).max() <= 1e-12 * nx * ny


@pytest.mark.parametrize("ny,nx", [(8, 8), (6, 4), (16, 2), (5, 5), (6, 9), (9, 6), (4, 1), (1, 7)])
def test_inverse_of_a_non_hermitian_half_spectrum_matches_numpy(ny, nx):
    rng = np.random.default_rng(7 + nx + ny)
    X = rng.standard_normal((ny, nx // 2 + 1)) + 1j * rng.standard_normal((ny, nx // 2 + 1))
    got = oracle.irfft2d(X, nx)
    assert np.abs(got - np.fft.irfft2(X, s=(ny, nx))).max() <= 1e-14 * nx * ny
    # the projection onto the Hermitian part is idempotent
    full = oracle.hermitian_extension(X, nx)
    again = oracle.hermitian_extension(full[:, : nx // 2 + 1], nx)
    assert np.abs(full - again).max() <= 1e-15 * np.abs(full).max()


def test_odd_side_extension_by_hand():
    """nx = 3, ny = 1: the half spectrum [X0, X1] extends to
    [Re X0, X1, conj(X1)] (only a = 0 maps to itself)."""
    X = np.array([[2.0 + 3.0j, 1.0 - 4.0j]])
    full = oracle.hermitian_extension(X, 3)
    assert np.array_equal(full, np.array([[2.0 + 0.0j, 1.0 - 4.0j, 1.0 + 4.0j]]))
    # and the inverse is the real field of that spectrum, by the DFT sum
    x = oracle.irfft2d(X, 3)
    j = np.arange(3)
    ref = (2.0 + 2 * ((1.0 - 4.0j) * np.exp(2j * math.pi * j / 3)).real) / 3
    assert np.abs(x[0] - ref).max() <= 1e-15
