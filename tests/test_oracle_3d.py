"""Pins of the oracle's 3D transforms and solves (the n-dimensional extension
of Sec. II.D; the solves of Sec. III on a 3D periodic box).

Fixed independently of the oracle: the 3D DFT summed by brute force on tiny
grids, numpy.fft.fftn on larger ones, the inverse and Parseval, and single
Fourier modes in closed form for the three solves."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _brute_dft3(x):
    nz, ny, nx = x.shape
    out = np.zeros_like(x, dtype=np.complex128)
    j, k, l = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="xy")
    for c in range(nz):
        for b in range(ny):
            for a in range(nx):
                ph = np.exp(-2j * math.pi * (a * np.arange(nx)[None, None, :] / nx
                                             + b * np.arange(ny)[None, :, None] / ny
                                             + c * np.arange(nz)[:, None, None] / nz))
                out[c, b, a] = np.sum(x * ph)
    return out


@pytest.mark.parametrize("shape", [(2, 4, 8), (4, 2, 2), (8, 8, 4), (1, 2, 16)])
def test_fft3d_matches_the_brute_force_dft(shape):
    x = W.random_field(shape, seed=sum(shape))
    ref = _brute_dft3(x)
    assert np.abs(oracle.fft3d(x) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fft3d_matches_numpy_and_inverts():
    x = W.random_field((16, 32, 8), seed=3)
    X = oracle.fft3d(x, threads=4)
    assert oracle.rel_l2(X, np.fft.fftn(x)) <= 1e-14
    assert oracle.rel_l2(oracle.ifft3d(X, threads=4), x) <= 1e-14
    # Parseval: sum |x|^2 = sum |X|^2 / P
    assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(X) ** 2) / x.size) <= 1e-12 * np.sum(np.abs(x) ** 2)


def _mode(nx, ny, nz, lx, ly, lz, m):
    x, y, z = W.grid(nx, lx), W.grid(ny, ly), W.grid(nz, lz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    th = 2 * math.pi * (m[0] * X / lx + m[1] * Y / ly + m[2] * Z / lz)
    k2 = (2 * math.pi) ** 2 * ((m[0] / lx) ** 2 + (m[1] / ly) ** 2 + (m[2] / lz) ** 2)
    return np.cos(th), k2


@pytest.mark.parametrize("m", [(1, 0, 0), (2, -1, 3), (0, 0, 1)])
def test_3d_solves_on_single_modes(m):
    nx, ny, nz, lx, ly, lz = 16, 8, 32, 1.0, 2.0, 0.5
    mode, k2 = _mode(nx, ny, nz, lx, ly, lz, m)
    s = 3.0 * mode + 0.7   # the constant is the mean, dropped by Poisson
    u = oracle.solve3d(s, lx, ly, lz, 0)
    assert np.abs(u - (-3.0 / k2) * mode).max() <= 1e-12 * 3.0 / k2
    kappa, t, c = 0.01, 0.3, 0.8
    d = oracle.solve3d(mode, lx, ly, lz, 1, kappa, t)
    assert np.abs(d - math.exp(-kappa * k2 * t) * mode).max() <= 1e-13
    w = oracle.solve3d(mode, lx, ly, lz, 2, c, t)
    assert np.abs(w - math.cos(c * math.sqrt(k2) * t) * mode).max() <= 1e-13


def test_3d_reduces_to_2d_when_nz_is_one():
    f = W.random_field((1, 16, 32), seed=9)
    assert oracle.rel_l2(oracle.fft3d(f)[0], oracle.fft2d(f[0])) <= 1e-15
    assert oracle.rel_l2(oracle.solve3d(f, 1.0, 2.0, 1.0, 0)[0], oracle.solve_poisson(f[0], 1.0, 2.0)) <= 1e-14
