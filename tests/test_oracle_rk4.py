"""Pins of the oracle's RK4 wave integrator with a time-dependent source
(Sec. III.C, the first-order system of the forced oscillators integrated by
the classical fourth-order Runge-Kutta method).

Fixed by mathematics rather than by the integrator itself: fourth-order
convergence (error ratio 16 when dt halves) to the exact source-free
solution and to the exact constant-source solution (both from the oracle's
closed forms, which have their own pins), and the self-convergence test of
Sec. III.C on the orbiting source, (u2 - u1)/(u3 - u2) close to 2^4 for the
domain mean at resolutions N, 2N, 4N with dt = h/4."""
import math

import numpy as np

import oracle
import workloads as W


def _smooth(n, seed):
    """A field of a few low Fourier modes (w dt stays small)."""
    rng = np.random.default_rng(seed)
    x = W.grid(n, 1.0)
    X, Y = np.meshgrid(x, x)
    u = np.zeros((n, n), dtype=np.complex128)
    for _ in range(4):
        m, k = rng.integers(-2, 3, size=2)
        u += rng.standard_normal() * np.cos(2 * math.pi * (m * X + k * Y) + rng.uniform(0, 2 * math.pi))
    return u


def test_rk4_converges_at_fourth_order_to_the_source_free_solution():
    n, c, T = 16, 1.0, 0.8
    f, g = _smooth(n, 1), _smooth(n, 2)
    exact, _ = oracle.solve_wave(f, g, 1.0, 1.0, c, T)
    zero = lambda t: np.zeros((n, n), dtype=np.complex128)  # noqa: E731
    errs = []
    # w dt <= 0.45 for the largest mode: the asymptotic regime of the method
    for steps in (32, 64, 128):
        u, _ = oracle.wave_rk4(f, g, 1.0, 1.0, c, 0.0, T / steps, steps, zero)
        errs.append(oracle.rel_l2(u, exact))
    assert 13.0 < errs[0] / errs[1] < 19.0 and 13.0 < errs[1] / errs[2] < 19.0


def test_rk4_converges_at_fourth_order_to_the_constant_source_solution():
    """gamma = Omega = 0: a static Gaussian source, exact by the forced oscillator."""
    n, c, T = 16, 0.7, 0.6
    f = _smooth(n, 3)
    src = dict(amplitude=2.0, sigma=0.3, radius=0.2, omega=0.0, gamma=0.0)
    s = oracle.orbiting_source(n, n, 0.0, 0.0, 1.0, 1.0, 0.0, **src)
    exact, _ = oracle.solve_wave_source(f, None, s, 1.0, 1.0, c, T)
    source = lambda t: oracle.orbiting_source(n, n, 0.0, 0.0, 1.0, 1.0, t, **src)  # noqa: E731
    errs = []
    # every mode of the grid is excited (rounding); w dt < 2.8 keeps RK4 stable
    for steps in (32, 64, 128):
        u, _ = oracle.wave_rk4(f, None, 1.0, 1.0, c, 0.0, T / steps, steps, source)
        errs.append(oracle.rel_l2(u, exact))
    assert 13.0 < errs[0] / errs[1] < 19.0 and 13.0 < errs[1] / errs[2] < 19.0


def test_orbiting_source_self_convergence_factor_is_about_16():
    """Sec. III.C: D = [-2, 2]^2, h = 4/N, dt = h/4, A = 1, sigma = 0.1, Omega = 5,
    gamma = 10, orbit radius 1, zero initial data; N = 64, 128, 256."""
    src = dict(amplitude=1.0, sigma=0.1, radius=1.0, omega=5.0, gamma=10.0)
    T = 0.5
    means = []
    for n in (64, 128, 256):
        h = 4.0 / n
        dt = 0.25 * h
        steps = int(round(T / dt))
        source = lambda t, n=n: oracle.orbiting_source(n, n, -2.0, -2.0, 4.0, 4.0, t, **src)  # noqa: E731
        z = np.zeros((n, n), dtype=np.complex128)
        u, _ = oracle.wave_rk4(z, None, 4.0, 4.0, 1.0, 0.0, dt, steps, source, threads=oracle.default_threads())
        means.append(u.real.mean())
    factor = (means[1] - means[0]) / (means[2] - means[1])
    assert 14.0 < factor < 18.0, factor


def test_orbiting_source_field_is_the_stated_gaussian():
    n = 32
    src = dict(amplitude=1.5, sigma=0.2, radius=0.5, omega=2.0, gamma=3.0)
    t = 0.3
    s = oracle.orbiting_source(n, n, -1.0, -1.0, 2.0, 2.0, t, **src)
    xs, ys = 0.5 * math.cos(2.0 * t), 0.5 * math.sin(2.0 * t)
    j, k = 20, 9
    x, y = -1.0 + j * 2.0 / n, -1.0 + k * 2.0 / n
    ref = 1.5 * math.exp(-((x - xs) ** 2 + (y - ys) ** 2) / 0.04) * math.cos(3.0 * t)
    assert abs(s[k, j] - ref) <= 1e-15
    assert np.all(s.imag == 0)
