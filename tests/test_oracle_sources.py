"""Pins of the oracle's time-independent-source solves (Sec. III.B, III.C).

Each pin is fixed by the mathematics, not by the oracle's own formulas:
single real Fourier modes against the forced-oscillator and forced-decay
closed forms evaluated pointwise, constant fields against the k = 0 ODE, the
differential equation itself checked by finite differences in time on random
fields (spectra from numpy's FFT, not the oracle's), the initial conditions,
the source-free limit, and the long-time limit of diffusion against the
oracle's Poisson solve."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _grid(nx, ny, lx, ly):
    X, Y = np.meshgrid(W.grid(nx, lx), W.grid(ny, ly))
    return X, Y


@pytest.mark.parametrize("m,n", [(1, 0), (2, -3), (0, 1)])
def test_wave_source_single_mode_matches_the_forced_oscillator(m, n):
    nx, ny, lx, ly, c = 32, 16, 1.5, 2.0, 0.7
    a, b, sig = 0.8, -0.3, 2.5
    X, Y = _grid(nx, ny, lx, ly)
    th = 2 * math.pi * (m * X / lx + n * Y / ly)
    w = c * 2 * math.pi * math.hypot(m / lx, n / ly)
    f, g, s = a * np.cos(th), b * np.sin(th), sig * np.cos(th)
    for t in (0.0, 0.37, 2.9):
        u, v = oracle.solve_wave_source(f, g, s, lx, ly, c, t, want_v=True)
        # u'' + w^2 u = sig cos(th) with u(0) = a cos(th), u'(0) = b sin(th)
        ref_u = ((a - sig / w ** 2) * math.cos(w * t) + sig / w ** 2) * np.cos(th) + b / w * math.sin(w * t) * np.sin(th)
        ref_v = -w * (a - sig / w ** 2) * math.sin(w * t) * np.cos(th) + b * math.cos(w * t) * np.sin(th)
        assert np.abs(u - ref_u).max() <= 1e-13
        assert np.abs(v - ref_v).max() <= 1e-13


@pytest.mark.parametrize("m,n", [(1, 1), (3, 0)])
def test_diffusion_source_single_mode_matches_forced_decay(m, n):
    nx, ny, lx, ly, kappa = 16, 32, 2.0, 1.0, 0.05
    a, sig = 1.3, -0.6
    X, Y = _grid(nx, ny, lx, ly)
    th = 2 * math.pi * (m * X / lx + n * Y / ly)
    q = kappa * (2 * math.pi) ** 2 * ((m / lx) ** 2 + (n / ly) ** 2)
    for t in (0.0, 0.2, 5.0):
        u = oracle.solve_diffusion_source(a * np.cos(th), sig * np.cos(th), lx, ly, kappa, t)
        ref = (a * math.exp(-q * t) + sig * (1 - math.exp(-q * t)) / q) * np.cos(th)
        assert np.abs(u - ref).max() <= 1e-13


def test_constant_fields_follow_the_k0_equations():
    nx = ny = 8
    f0, g0, s0, t = 0.4, -1.1, 3.0, 1.7
    one = np.ones((ny, nx))
    u, v = oracle.solve_wave_source(f0 * one, g0 * one, s0 * one, 1.0, 1.0, 1.0, t, want_v=True)
    assert np.allclose(u, f0 + g0 * t + s0 * t * t / 2, rtol=0, atol=1e-13)
    assert np.allclose(v, g0 + s0 * t, rtol=0, atol=1e-13)
    ud = oracle.solve_diffusion_source(f0 * one, s0 * one, 1.0, 1.0, 0.3, t)
    assert np.allclose(ud, f0 + s0 * t, rtol=0, atol=1e-13)


def test_wave_source_satisfies_the_equation_in_time():
    """Per Fourier mode: (U(t+h) - 2U(t) + U(t-h))/h^2 = -w^2 U(t) + S to
    O(h^2), with spectra taken by numpy's FFT.  Dropping the constant
    particular solution s^/w^2 breaks this by |S|."""
    nx, ny, lx, ly, c, t, h = 16, 16, 1.0, 1.0, 0.9, 0.6, 1e-4
    f = W.random_field((ny, nx), seed=1)
    g = W.random_field((ny, nx), seed=2)
    s = W.random_field((ny, nx), seed=3)
    u = {d: oracle.solve_wave_source(f, g, s, lx, ly, c, t + d * h)[0] for d in (-1, 0, 1)}
    U = {d: np.fft.fft2(u[d]) for d in u}
    S = np.fft.fft2(s)
    kx = oracle.signed_wavenumbers(nx, lx)
    ky = oracle.signed_wavenumbers(ny, ly)
    w2 = c * c * (ky[:, None] ** 2 + kx[None, :] ** 2)
    lhs = (U[1] - 2 * U[0] + U[-1]) / h ** 2
    rhs = -w2 * U[0] + S
    # per mode: truncation h^2 w^2/12 relative, rounding eps |U|/h^2
    assert (np.abs(lhs - rhs) <= 1e-5 * (np.abs(w2 * U[0]) + np.abs(S))).all()
    # initial conditions and the velocity as the time derivative
    u0, v0 = oracle.solve_wave_source(f, g, s, lx, ly, c, 0.0, want_v=True)
    assert np.abs(u0 - f).max() <= 1e-12 and np.abs(v0 - g).max() <= 1e-12
    _, v = oracle.solve_wave_source(f, g, s, lx, ly, c, t, want_v=True)
    assert np.abs((u[1] - u[-1]) / (2 * h) - v).max() <= 1e-4 * np.abs(v).max()


def test_diffusion_source_satisfies_the_equation_in_time():
    nx, ny, lx, ly, kappa, t, h = 16, 8, 2.0, 1.0, 0.02, 0.4, 1e-4
    f = W.random_field((ny, nx), seed=4)
    s = W.random_field((ny, nx), seed=5)
    U = {d: np.fft.fft2(oracle.solve_diffusion_source(f, s, lx, ly, kappa, t + d * h)) for d in (-1, 0, 1)}
    S = np.fft.fft2(s)
    kx = oracle.signed_wavenumbers(nx, lx)
    ky = oracle.signed_wavenumbers(ny, ly)
    q = kappa * (ky[:, None] ** 2 + kx[None, :] ** 2)
    lhs = (U[1] - U[-1]) / (2 * h)
    rhs = -q * U[0] + S
    assert np.abs(lhs - rhs).max() <= 1e-6 * (np.abs(q * U[0]).max() + np.abs(S).max())
    assert np.abs(oracle.solve_diffusion_source(f, s, lx, ly, kappa, 0.0) - f).max() <= 1e-12


def test_zero_source_reduces_to_the_source_free_solves():
    nx, ny, lx, ly = 32, 16, 1.0, 3.0
    f = W.random_field((ny, nx), seed=6)
    g = W.random_field((ny, nx), seed=7)
    z = np.zeros((ny, nx), dtype=np.complex128)
    u, v = oracle.solve_wave_source(f, g, z, lx, ly, 1.3, 0.77, want_v=True)
    ru, rv = oracle.solve_wave(f, g, lx, ly, 1.3, 0.77, want_v=True)
    assert oracle.rel_l2(u, ru) <= 1e-14 and oracle.rel_l2(v, rv) <= 1e-14
    ud = oracle.solve_diffusion_source(f, z, lx, ly, 0.1, 0.3)
    assert oracle.rel_l2(ud, oracle.solve_diffusion(f, lx, ly, 0.1, 0.3)) <= 1e-14


def test_diffusion_source_tends_to_the_poisson_equilibrium():
    """For large t the nonzero modes settle where kappa lap(u) + s - mean(s) = 0,
    i.e. u - mean(u) = -poisson(s)/kappa, while the mean grows as mean(s) t."""
    nx, ny, lx, ly, kappa, t = 16, 16, 1.0, 1.0, 0.5, 40.0
    f = W.random_field((ny, nx), seed=8)
    s = W.random_field((ny, nx), seed=9)
    u = oracle.solve_diffusion_source(f, s, lx, ly, kappa, t)
    eq = -oracle.solve_poisson(s, lx, ly) / kappa
    assert oracle.rel_l2(u - u.mean(), eq) <= 1e-12
    assert abs(u.mean() - (f.mean() + s.mean() * t)) <= 1e-12 * abs(s.mean() * t)
