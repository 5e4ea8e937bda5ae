"""Pins of the oracle's transforms and solves on lengths that are not powers
of two (the extension beyond the N = 2^m of Sec. II.D: the DFT sum of
Eq. (DFT) for any N, and the solves of Sec. III on such grids).

Fixed independently of the oracle: numpy.fft (a separate implementation of
the same sums), a shifted delta whose transform is a pure phase, the
inverse, Parseval, and single Fourier modes whose solutions are closed
forms."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

SIZES_1D = [1, 3, 5, 6, 7, 9, 10, 12, 15, 21, 35, 100, 105]


@pytest.mark.parametrize("n", SIZES_1D)
def test_fft1d_matches_numpy_on_any_length(n):
    x = W.random_field((n,), seed=n)
    ref = np.fft.fft(x)
    assert np.abs(oracle.fft1d(x) - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert np.abs(oracle.ifft1d(oracle.fft1d(x)) - x).max() <= 1e-14 * n


@pytest.mark.parametrize("n,j0", [(7, 3), (15, 11), (30, 29)])
def test_fft1d_of_a_shifted_delta_is_a_pure_phase(n, j0):
    x = np.zeros(n, dtype=np.complex128)
    x[j0] = 1.0
    k = np.arange(n)
    ref = np.exp(-2j * math.pi * ((j0 * k) % n) / n)
    assert np.abs(oracle.fft1d(x) - ref).max() <= 4e-15


@pytest.mark.parametrize("shape", [(20, 12), (30, 96), (5, 7), (3, 1), (48, 64), (49, 25)])
def test_fft2d_matches_numpy_and_inverts(shape):
    x = W.random_field(shape, seed=sum(shape))
    X = oracle.fft2d(x, threads=4)
    assert oracle.rel_l2(X, np.fft.fft2(x)) <= 1e-14
    assert oracle.rel_l2(oracle.ifft2d(X, threads=4), x) <= 1e-14
    # Parseval: sum |x|^2 = sum |X|^2 / P
    assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(X) ** 2) / x.size) <= 1e-12 * np.sum(np.abs(x) ** 2)


def _mode(nx, ny, lx, ly, m, n):
    X, Y = np.meshgrid(W.grid(nx, lx), W.grid(ny, ly))
    th = 2 * math.pi * (m * X / lx + n * Y / ly)
    k2 = (2 * math.pi) ** 2 * ((m / lx) ** 2 + (n / ly) ** 2)
    return np.cos(th), np.sin(th), k2


@pytest.mark.parametrize("nx,ny,m,n", [(24, 30, 2, -3), (35, 21, 5, 1), (15, 9, -7, 4), (12, 10, 0, 5)])
def test_solves_on_single_modes_of_odd_and_even_grids(nx, ny, m, n):
    lx, ly = 1.5, 0.8
    cm, sm, k2 = _mode(nx, ny, lx, ly, m, n)
    u = oracle.solve_poisson(2.0 * cm + 0.3, lx, ly)   # the constant is the mean, dropped
    assert np.abs(u - (-2.0 / k2) * cm).max() <= 1e-12 * 2.0 / k2
    kappa, t, c = 0.02, 0.4, 0.9
    d = oracle.solve_diffusion(cm, lx, ly, kappa, t)
    assert np.abs(d - math.exp(-kappa * k2 * t) * cm).max() <= 1e-13
    w = c * math.sqrt(k2)
    uu, vv = oracle.solve_wave(cm, sm, lx, ly, c, t, want_v=True)
    assert np.abs(uu - (math.cos(w * t) * cm + math.sin(w * t) / w * sm)).max() <= 1e-12
    assert np.abs(vv - (-w * math.sin(w * t) * cm + math.cos(w * t) * sm)).max() <= 1e-11 * max(1.0, w)


def test_poisson_on_an_odd_grid_satisfies_the_discrete_equation():
    """Residual check: the spectral Laplacian of u equals s minus its mean."""
    nx, ny, lx, ly = 45, 27, 2.0, 1.2
    s = W.random_field((ny, nx), seed=5).real.astype(np.complex128)
    u = oracle.solve_poisson(s, lx, ly)
    kx = 2 * math.pi * np.fft.fftfreq(nx, d=lx / nx)
    ky = 2 * math.pi * np.fft.fftfreq(ny, d=ly / ny)
    KX, KY = np.meshgrid(kx, ky)
    lap = np.fft.ifft2(-(KX ** 2 + KY ** 2) * np.fft.fft2(u))
    assert np.abs(lap - (s - s.mean())).max() <= 1e-11 * np.abs(s).max()
