"""Pins of the oracle's Poisson, diffusion and wave solves (CPU only).

Closed forms written out from the PDE, not from the oracle:
  * Poisson (Sec. III.A): each Fourier mode a cos(theta) + b sin(theta),
    theta = 2 pi (m x/lx + n y/ly), has the zero-mean solution
    -(a cos theta + b sin theta) / ((2 pi m/lx)^2 + (2 pi n/ly)^2).
  * Diffusion (Sec. III.B): a Gaussian of variance s0^2 spreads to variance
    s0^2 + 2 kappa t with amplitude s0^2/(s0^2 + 2 kappa t) (2D heat kernel);
    on the periodic box the solution is the sum over periodic images.
  * Wave (Sec. III.C): the standing mode sin(2 pi p x) sin(2 pi q y) oscillates
    as cos(w t), w = 2 pi c sqrt(p^2 + q^2); its energy is 17 pi^2 for (3, 5).
plus invariants: mean conservation (Sec. III.B, III.C), energy conservation,
diffusion semigroup, time reversibility of the wave propagator.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

THREADS = oracle.default_threads()


def _poisson_closed_form(ms: W.ModeSum) -> np.ndarray:
    x = W.grid(ms.nx, ms.lx)
    y = W.grid(ms.ny, ms.ly)
    X, Y = np.meshgrid(x, y)
    u = np.zeros_like(X)
    for m, n, a, b in zip(ms.m, ms.n, ms.a, ms.b):
        th = 2 * math.pi * (m * X / ms.lx + n * Y / ms.ly)
        k2 = (2 * math.pi * m / ms.lx) ** 2 + (2 * math.pi * n / ms.ly) ** 2
        u -= (a * np.cos(th) + b * np.sin(th)) / k2
    if ms.sine_amp != 0:
        u += np.sin(2 * math.pi * X / ms.lx) * np.sin(2 * math.pi * Y / ms.ly)
    return u


def test_poisson_config1_closed_form(closed_forms):
    ms = W.poisson_source(64, 64, seed=1)
    assert ms.sine_amp == pytest.approx(closed_forms["poisson_sine_amp"], rel=1e-15)
    u = oracle.solve_poisson(ms.field, 1.0, 1.0)
    ref = _poisson_closed_form(ms)
    assert oracle.rel_l2(u, ref) <= 1e-13
    assert abs(np.mean(u)) <= 1e-15
    assert np.max(np.abs(u.imag)) <= 1e-14


@pytest.mark.parametrize("nx,ny,lx,ly", [(32, 128, 1.0, 3.0), (256, 64, 4.0, 4.0), (16, 16, 0.5, 2.0)])
def test_poisson_rectangular_closed_form(nx, ny, lx, ly):
    ms = W.poisson_source(nx, ny, seed=7, lx=lx, ly=ly, kmax=min(8, nx // 2 - 1, ny // 2 - 1))
    u = oracle.solve_poisson(ms.field, lx, ly)
    assert oracle.rel_l2(u, _poisson_closed_form(ms)) <= 1e-13


def test_poisson_ignores_source_mean():
    """g = s - mean(s): adding a constant to s does not change u (Eq. (Poisson2))."""
    ms = W.poisson_source(64, 32, seed=3)
    u1 = oracle.solve_poisson(ms.field, 1.0, 1.0)
    u2 = oracle.solve_poisson(ms.field + 5.0, 1.0, 1.0)
    assert oracle.rel_l2(u2, u1) <= 1e-13


def test_poisson_solution_satisfies_discrete_laplacian_spectrally():
    """Apply -|k|^2 to the solution's spectrum (numpy FFT): recovers the source."""
    ms = W.poisson_source(64, 128, seed=9, lx=2.0, ly=1.0)
    u = oracle.solve_poisson(ms.field, 2.0, 1.0)
    kx = oracle.signed_wavenumbers(64, 2.0)
    ky = oracle.signed_wavenumbers(128, 1.0)
    lap = np.fft.ifft2(-(ky[:, None] ** 2 + kx[None, :] ** 2) * np.fft.fft2(u))
    assert oracle.rel_l2(lap, ms.field - ms.field.mean()) <= 1e-12


def _image_gaussian(n, t, kappa=0.01, s0=0.05, L=2.0, origin=-1.0):
    x = W.grid(n, L, origin)
    X, Y = np.meshgrid(x, x)
    st2 = s0 ** 2 + 2 * kappa * t
    u = np.zeros_like(X)
    for m in (-1, 0, 1):
        for q in (-1, 0, 1):
            u += np.exp(-((X - L * m) ** 2 + (Y - L * q) ** 2) / (2 * st2))
    return (s0 ** 2 / st2) * u


@pytest.mark.parametrize("t", [1e-3, 0.1, 1.0])
def test_diffusion_periodic_image_gaussian(t):
    ic = W.diffusion_ic(256, seed=2, noise_std=0.0)
    u = oracle.solve_diffusion(ic.field, 2.0, 2.0, 0.01, t, threads=THREADS)
    assert oracle.rel_l2(u, _image_gaussian(256, t)) <= 1e-12


@pytest.mark.slow
def test_diffusion_config2_full_size_closed_form():
    ic = W.diffusion_ic(1024, seed=2, noise_std=0.0)
    u = oracle.solve_diffusion(ic.field, 2.0, 2.0, 0.01, 1.0, threads=THREADS)
    assert oracle.rel_l2(u, _image_gaussian(1024, 1.0)) <= 1e-12


def test_diffusion_mean_conservation_and_decay():
    """mean(u)/mean(f) = 1 (Sec. III.B) and the L2 norm decays."""
    ic = W.diffusion_ic(128, seed=2)
    f = ic.field
    prev = oracle.l2_from_spectrum(oracle.fft2d(f), 2.0, 2.0)
    for t in (0.5, 2.0, 10.0):
        u = oracle.solve_diffusion(f, 2.0, 2.0, 1.0, t)
        assert abs(np.mean(u) / np.mean(f) - 1) <= 1e-12
        e = oracle.l2_from_spectrum(oracle.fft2d(u), 2.0, 2.0)
        assert e <= prev * (1 + 1e-14)
        # the mean's share, area * |mean|^2, never decays
        assert e >= 4.0 * abs(np.mean(f)) ** 2 * (1 - 1e-12)
        prev = e
    # by t = 10 every non-zero mode has decayed and only the mean's share is left
    assert prev == pytest.approx(4.0 * abs(np.mean(f)) ** 2, rel=1e-12)


def test_diffusion_semigroup():
    ic = W.diffusion_ic(128, seed=5)
    a = oracle.solve_diffusion(oracle.solve_diffusion(ic.field, 2, 2, 0.01, 0.3), 2, 2, 0.01, 0.45)
    b = oracle.solve_diffusion(ic.field, 2, 2, 0.01, 0.75)
    assert oracle.rel_l2(a, b) <= 1e-14


def test_diffusion_t0_is_identity_and_rejects_negative_time():
    f = W.random_field((32, 64), seed=1)
    assert oracle.rel_l2(oracle.solve_diffusion(f, 1, 1, 0.5, 0.0), f) <= 1e-15
    with pytest.raises(ValueError):
        oracle.solve_diffusion(f, 1, 1, 0.5, -1.0)


@pytest.mark.parametrize("t", [0.0, 0.013, 0.5])
def test_wave_standing_mode(t, closed_forms):
    n = 256
    ic = W.wave_ic(n, seed=3, pulse=False)
    u, v = oracle.solve_wave(ic.field, None, 1.0, 1.0, 1.0, t, want_v=True)
    w = closed_forms["standing_omega"]
    assert w == pytest.approx(2 * math.pi * math.sqrt(34), rel=1e-15)
    assert oracle.rel_l2(u, ic.field * math.cos(w * t)) <= 1e-13 + 1e-12 * (t > 0)
    assert np.max(np.abs(v + w * math.sin(w * t) * ic.field)) <= 1e-11
    F = oracle.fft2d(ic.field)
    U, V = oracle.wave_spectra(F, None, 1.0, 1.0, 1.0, t)
    e = oracle.wave_energy_from_spectra(U, V, 1.0, 1.0, 1.0)
    assert e == pytest.approx(closed_forms["standing_energy"], rel=1e-12)


def test_wave_velocity_initial_data():
    """u0 = 0, v0 = sin(2 pi x): u(t) = sin(2 pi x) sin(w t)/w with w = 2 pi c;
    v0 = 1 (the w = 0 mode): u(t) = u0 + t (Eq. (OmegaZero) with s = 0)."""
    n, c, t = 64, 1.5, 0.37
    x = W.grid(n, 1.0)
    X, _ = np.meshgrid(x, x)
    v0 = np.sin(2 * math.pi * X).astype(np.complex128)
    u, v = oracle.solve_wave(np.zeros_like(v0), v0, 1.0, 1.0, c, t, want_v=True)
    w = 2 * math.pi * c
    assert np.max(np.abs(u - v0 * math.sin(w * t) / w)) <= 1e-14
    assert np.max(np.abs(v - v0 * math.cos(w * t))) <= 1e-14
    ones = np.ones((n, n), dtype=np.complex128)
    u1, v1 = oracle.solve_wave(np.zeros_like(ones), ones, 1.0, 1.0, c, t, want_v=True)
    assert np.max(np.abs(u1 - t)) <= 1e-14
    assert np.max(np.abs(v1 - 1.0)) <= 1e-14


def test_wave_mean_and_energy_conservation():
    ic = W.wave_ic(128, seed=11)
    F = oracle.fft2d(ic.field)
    G = oracle.fft2d(W.random_field((128, 128), seed=4))
    G[0, 0] = 0.0  # zero-mean velocity keeps the mean constant (Sec. III.C plot)
    U0, V0 = oracle.wave_spectra(F, G, 1.0, 1.0, 1.0, 0.0)
    e0 = oracle.wave_energy_from_spectra(U0, V0, 1.0, 1.0, 1.0)
    for t in (0.1, 1.0, 2.0):
        U, V = oracle.wave_spectra(F, G, 1.0, 1.0, 1.0, t)
        assert abs(oracle.mean_from_spectrum(U) / oracle.mean_from_spectrum(U0) - 1) <= 1e-12
        assert abs(oracle.wave_energy_from_spectra(U, V, 1.0, 1.0, 1.0) / e0 - 1) <= 1e-12


def test_wave_time_reversibility():
    u0 = W.random_field((64, 32), seed=21)
    v0 = W.random_field((64, 32), seed=22)
    u1, v1 = oracle.solve_wave(u0, v0, 2.0, 1.0, 0.7, 0.9, want_v=True)
    u2, v2 = oracle.solve_wave(u1, -v1, 2.0, 1.0, 0.7, 0.9, want_v=True)
    assert oracle.rel_l2(u2, u0) <= 1e-13
    assert oracle.rel_l2(-v2, v0) <= 1e-13


def test_wave_matches_second_order_ode_per_mode():
    """d^2 U/dt^2 = -w^2 U for every mode: centred second difference in time."""
    F = oracle.fft2d(W.random_field((16, 16), seed=8))
    G = oracle.fft2d(W.random_field((16, 16), seed=9))
    t, h = 0.4, 1e-4
    Um, _ = oracle.wave_spectra(F, G, 1, 1, 1, t - h)
    U0, _ = oracle.wave_spectra(F, G, 1, 1, 1, t)
    Up, _ = oracle.wave_spectra(F, G, 1, 1, 1, t + h)
    kx = oracle.signed_wavenumbers(16, 1.0)
    w2 = kx[:, None] ** 2 + kx[None, :] ** 2
    acc = (Up - 2 * U0 + Um) / h ** 2
    assert oracle.rel_l2(acc, -w2 * U0) <= 1e-5


def test_spectral_diagnostics_match_grid_sums_and_closed_forms():
    """mean_from_spectrum and l2_from_spectrum against sums over the grid
    (Parseval), and the L2 norm of a narrow Gaussian exp(-r^2/(2 s^2)) against
    its closed form: the integral of exp(-r^2/s^2) over the plane is pi s^2."""
    n, length, s = 256, 2.0, 0.05
    x = W.grid(n, length, -1.0)
    g = np.outer(np.exp(-x ** 2 / (2 * s * s)), np.exp(-x ** 2 / (2 * s * s))).astype(np.complex128)
    f = g + 0.3 + 0.1j
    F = oracle.fft2d(f)
    dx = length / n
    assert abs(oracle.mean_from_spectrum(F) - f.mean()) <= 1e-14
    direct = float(np.sum(np.abs(f) ** 2)) * dx * dx
    assert abs(oracle.l2_from_spectrum(F, length, length) / direct - 1) <= 1e-13
    # the Gaussian alone: its tails at the box edge are exp(-200), far below rounding
    assert abs(oracle.l2_from_spectrum(oracle.fft2d(g), length, length) / (math.pi * s * s) - 1) <= 1e-12
