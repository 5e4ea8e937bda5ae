"""Seeded synthetic inputs for the spectral PDE solvers.

This module only *draws* and *samples* input fields: grids, random mode
lists, Gaussian pulses, noise, request mixes.  It holds none of the
solvers' arithmetic (no transform, no spectral operator, no closed-form
solution), so both the CPU oracle and the GPU path can take their inputs
from here without sharing any of the method.

Grid convention (Sec. II.B and II.D of the paper): a periodic box of length
L sampled at N points, x_j = x0 + j*L/N for j = 0..N-1, endpoint excluded.
Fields are complex in general; the real fields used here carry a zero
imaginary part.  Arrays are [ny][nx] with x contiguous.

Every generator takes an explicit seed and uses numpy's PCG64
(`numpy.random.default_rng`), so a given seed always gives the same field.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


def grid(n: int, length: float, origin: float = 0.0) -> np.ndarray:
    """Sample points x_j = origin + j*length/n, j = 0..n-1 (periodic, endpoint excluded)."""
    return origin + np.arange(n, dtype=np.float64) * (length / n)


# ---------------------------------------------------------------------------
# Poisson sources: a manufactured sine term plus a seeded sum of Fourier modes
# ---------------------------------------------------------------------------

@dataclass
class ModeSum:
    """s(x, y) = sine_amp * sin(2 pi x/lx) sin(2 pi y/ly)
                 + sum_j a_j cos(theta_j) + b_j sin(theta_j),
    theta_j = 2 pi (m_j x / lx + n_j y / ly)."""
    nx: int
    ny: int
    lx: float
    ly: float
    m: np.ndarray          # int, x mode numbers
    n: np.ndarray          # int, y mode numbers
    a: np.ndarray          # cosine amplitudes
    b: np.ndarray          # sine amplitudes
    sine_amp: float        # amplitude of the sin*sin term (0 => absent)
    field: np.ndarray = dc_field(repr=False, default=None)  # complex128 [ny][nx]


def draw_modes(rng: np.random.Generator, count: int, kmax: int) -> Tuple[np.ndarray, ...]:
    """Draw `count` integer mode pairs uniformly from [-kmax, kmax]^2 minus (0, 0),
    with N(0,1) cosine and sine amplitudes."""
    ms, ns = [], []
    while len(ms) < count:
        m, n = (int(v) for v in rng.integers(-kmax, kmax + 1, size=2))
        if m == 0 and n == 0:
            continue
        ms.append(m)
        ns.append(n)
    a = rng.standard_normal(count)
    b = rng.standard_normal(count)
    return np.array(ms, dtype=np.int64), np.array(ns, dtype=np.int64), a, b


def _sample_mode_sum(nx, ny, lx, ly, m, n, a, b, sine_amp) -> np.ndarray:
    """Sample the mode sum on the grid with separable 1D tables.

    a cos(p+q) + b sin(p+q) = cos q (a cos p + b sin p) + sin q (b cos p - a sin p)
    with p = 2 pi m x/lx, q = 2 pi n y/ly: a trigonometric identity used only to
    sample the input faster; it is not part of any solver."""
    x = grid(nx, lx)
    y = grid(ny, ly)
    out = np.zeros((ny, nx), dtype=np.float64)
    for mj, nj, aj, bj in zip(m, n, a, b):
        px = TWO_PI * mj * x / lx
        qy = TWO_PI * nj * y / ly
        cp, sp = np.cos(px), np.sin(px)
        cq, sq = np.cos(qy), np.sin(qy)
        out += np.outer(cq, aj * cp + bj * sp)
        out += np.outer(sq, bj * cp - aj * sp)
    if sine_amp != 0.0:
        out += sine_amp * np.outer(np.sin(TWO_PI * y / ly), np.sin(TWO_PI * x / lx))
    return out


def poisson_source(nx: int = 64, ny: int = 64, seed: int = 1, *, lx: float = 1.0,
                   ly: float = 1.0, n_modes: int = 16, kmax: int = 8,
                   with_sine: bool = True) -> ModeSum:
    """Poisson source of the 64x64 FP64 case: -8 pi^2 sin(2 pi x) sin(2 pi y) plus 16
    seeded Fourier modes with |m|,|n| <= 8 and N(0,1) amplitudes; mean removed.

    Every mode has (m, n) != (0, 0), so the sampled sum is mean-zero up to
    rounding; the residual mean is subtracted anyway.  Modes must lie below
    the Nyquist index (|m| < nx/2, |n| < ny/2) for the closed-form comparison
    to be exact; callers on very small grids pass a smaller kmax."""
    rng = np.random.default_rng(seed)
    m, n, a, b = draw_modes(rng, n_modes, kmax)
    # sin(2 pi x/lx) sin(2 pi y/ly) scaled by -((2 pi/lx)^2 + (2 pi/ly)^2), which
    # is -8 pi^2 on the unit square, so its Poisson solution has unit amplitude.
    amp = -((TWO_PI / lx) ** 2 + (TWO_PI / ly) ** 2) if with_sine else 0.0
    f = _sample_mode_sum(nx, ny, lx, ly, m, n, a, b, amp)
    f -= f.mean()
    ms = ModeSum(nx, ny, lx, ly, m, n, a, b, amp)
    ms.field = f.astype(np.complex128)
    return ms


def batch_shapes(count: int = 1024, seed: int = 4,
                 sides: Sequence[int] = (32, 64, 128, 256, 512, 1024)) -> List[Tuple[int, int]]:
    """Shapes (nx, ny) of the uneven batch: each side drawn independently and
    uniformly from `sides`."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(sides), size=(count, 2))
    return [(int(sides[i]), int(sides[j])) for i, j in idx]


def batch_sources(shapes: Sequence[Tuple[int, int]], seed: int = 4,
                  n_modes: int = 16, kmax: int = 8) -> List[ModeSum]:
    """One 16-mode source per shape (no sine term), seeded by (seed, index)."""
    out = []
    for i, (nx, ny) in enumerate(shapes):
        k = min(kmax, nx // 2 - 1, ny // 2 - 1)
        out.append(poisson_source(nx, ny, seed=_child_seed(seed, i), n_modes=n_modes,
                                  kmax=k, with_sine=False))
    return out


def _child_seed(seed: int, index: int) -> int:
    """A deterministic per-item seed derived from (seed, index)."""
    ss = np.random.SeedSequence([seed, index])
    return int(ss.generate_state(1, dtype=np.uint32)[0])


# ---------------------------------------------------------------------------
# Diffusion: Gaussian initial profile plus seeded noise on [-1, 1]^2
# ---------------------------------------------------------------------------

@dataclass
class GaussianIC:
    n: int
    length: float
    origin: float
    sigma: float
    center: Tuple[float, float]
    noise_std: float
    standing: Optional[Tuple[int, int]]     # (p, q): adds sin(2 pi p x) sin(2 pi q y)
    field: np.ndarray = dc_field(repr=False, default=None)
    clean: np.ndarray = dc_field(repr=False, default=None)  # the field without noise


def _periodic_offset(x: np.ndarray, c: float, length: float) -> np.ndarray:
    """Minimum-image offset of x from c on a circle of circumference `length`."""
    d = x - c
    return d - length * np.round(d / length)


def gaussian_field(n: int, length: float, origin: float, sigma: float,
                   center: Tuple[float, float]) -> np.ndarray:
    """exp(-d^2 / (2 sigma^2)) with d the periodic minimum-image distance to `center`."""
    x = grid(n, length, origin)
    dx = _periodic_offset(x, center[0], length)
    dy = _periodic_offset(x, center[1], length)
    return np.outer(np.exp(-dy ** 2 / (2 * sigma ** 2)), np.exp(-dx ** 2 / (2 * sigma ** 2)))


def diffusion_ic(n: int = 1024, seed: int = 2, *, sigma: float = 0.05,
                 noise_std: float = 1e-3, length: float = 2.0,
                 origin: float = -1.0) -> GaussianIC:
    """u0 = exp(-r^2/(2 sigma^2)) + N(0, noise_std^2) on [-1,1)^2 (1024^2 case)."""
    rng = np.random.default_rng(seed)
    clean = gaussian_field(n, length, origin, sigma, (0.0, 0.0))
    noise = rng.normal(0.0, noise_std, size=(n, n)) if noise_std > 0 else 0.0
    ic = GaussianIC(n, length, origin, sigma, (0.0, 0.0), noise_std, None)
    ic.clean = clean.astype(np.complex128)
    ic.field = (clean + noise).astype(np.complex128)
    return ic


def wave_ic(n: int = 2048, seed: int = 3, *, sigma: float = 0.02,
            standing: Optional[Tuple[int, int]] = (3, 5), pulse: bool = True) -> GaussianIC:
    """u0 on [0,1)^2: a Gaussian pulse of width sigma at a seeded centre plus the
    standing mode sin(2 pi 3 x) sin(2 pi 5 y); v0 = 0 (2048^2 case)."""
    rng = np.random.default_rng(seed)
    center = tuple(float(v) for v in rng.uniform(0.0, 1.0, size=2))
    f = np.zeros((n, n))
    if pulse:
        f = f + gaussian_field(n, 1.0, 0.0, sigma, center)
    if standing is not None:
        x = grid(n, 1.0)
        p, q = standing
        f = f + np.outer(np.sin(TWO_PI * q * x), np.sin(TWO_PI * p * x))
    ic = GaussianIC(n, 1.0, 0.0, sigma, center, 0.0, standing)
    ic.field = f.astype(np.complex128)
    ic.clean = ic.field
    return ic


def serving_input(kind: int, nx: int, ny: int, seed: int = 5) -> Tuple[np.ndarray, float, float]:
    """(field, lx, ly) of a serving request: the recipe of the kind's single
    case at an nx-by-ny grid -- Poisson: a 16-mode mean-zero source on [0,1)^2
    (no sine term); diffusion: Gaussian (sigma 0.05) plus N(0, 1e-3^2) noise on
    [-1,1)^2; wave: a Gaussian pulse (sigma 0.02) at a seeded centre plus the
    standing mode sin(2 pi 3 x) sin(2 pi 5 y) on [0,1)^2."""
    rng = np.random.default_rng(_child_seed(seed, kind * 10007 + nx * 13 + ny))
    if kind == POISSON:
        k = max(1, min(8, nx // 2 - 1, ny // 2 - 1))
        ms = poisson_source(nx, ny, seed=int(rng.integers(1 << 31)), kmax=k, with_sine=False)
        return ms.field, 1.0, 1.0
    if kind == DIFFUSION:
        x, y = grid(nx, 2.0, -1.0), grid(ny, 2.0, -1.0)
        g = np.outer(np.exp(-y ** 2 / (2 * 0.05 ** 2)), np.exp(-x ** 2 / (2 * 0.05 ** 2)))
        return (g + rng.normal(0.0, 1e-3, size=(ny, nx))).astype(np.complex128), 2.0, 2.0
    cx_, cy_ = (float(v) for v in rng.uniform(0.0, 1.0, size=2))
    x, y = grid(nx, 1.0), grid(ny, 1.0)
    dx, dy = _periodic_offset(x, cx_, 1.0), _periodic_offset(y, cy_, 1.0)
    f = np.outer(np.exp(-dy ** 2 / (2 * 0.02 ** 2)), np.exp(-dx ** 2 / (2 * 0.02 ** 2)))
    f = f + np.outer(np.sin(TWO_PI * 5 * y), np.sin(TWO_PI * 3 * x))
    return f.astype(np.complex128), 1.0, 1.0


def random_field(shape: Tuple[int, ...], seed: int) -> np.ndarray:
    """Complex128 field with i.i.d. N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# Serving: open-loop Poisson arrivals of mixed requests
# ---------------------------------------------------------------------------

POISSON, DIFFUSION, WAVE = 0, 1, 2


@dataclass
class Request:
    arrival: float          # seconds from the start of the trace
    kind: int               # POISSON, DIFFUSION or WAVE
    nx: int
    ny: int
    steps: int              # 1 for Poisson; time steps for diffusion / wave
    dt: float
    coef: float             # kappa (diffusion) or c (wave); unused for Poisson


def serving_trace(seed: int = 5, rate: float = 2000.0, duration: float = 11.0,
                  mix: Tuple[float, float, float] = (0.5, 0.3, 0.2),
                  log2_sides: Tuple[int, int] = (6, 12)) -> List[Request]:
    """Poisson-process arrivals (exponential gaps, mean 1/rate) of a request mix:
    50% Poisson, 30% diffusion (10..200 steps, dt 1e-3, kappa 0.01), 20% wave
    (10..500 steps, dt 1e-4, c 1); each side drawn log-uniformly from
    {2^6, ..., 2^12} independently."""
    rng = np.random.default_rng(seed)
    out: List[Request] = []
    t = 0.0
    lo, hi = log2_sides
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        u = rng.uniform()
        nx = 1 << int(rng.integers(lo, hi + 1))
        ny = 1 << int(rng.integers(lo, hi + 1))
        if u < mix[0]:
            out.append(Request(t, POISSON, nx, ny, 1, 0.0, 0.0))
        elif u < mix[0] + mix[1]:
            out.append(Request(t, DIFFUSION, nx, ny, int(rng.integers(10, 201)), 1e-3, 0.01))
        else:
            out.append(Request(t, WAVE, nx, ny, int(rng.integers(10, 501)), 1e-4, 1.0))
    return out
