"""FP64 CPU oracle for the spectral PDE solvers (arXiv 2412.12308).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are its only callers.  The product library
never imports, links or runs anything here, and nothing here imports the
product package; the two share no code.  See `fft_oracle.c` for the
paper passages each routine follows.

The C part (`fft_oracle.c`) holds the transforms and the three solves;
this wrapper marshals numpy complex128 arrays and adds the diagnostics
(mean, energy) that the paper's conservation plots show, computed from
spectra in numpy FP64.

Parity pins (tests/test_oracle_*.py): brute-force O(N^2) DFT from the
matrix W of Sec. II.B on N <= 32 (1D and 2D, rectangular); inverse of
forward = identity; Parseval; the conjugation identity of the iDFT;
periodicity; single complex exponentials; butterfly identities; numpy.fft
on large sizes; manufactured Poisson modes; the periodic-image Gaussian
for diffusion; the standing wave and its energy 17 pi^2; mean
conservation; diffusion semigroup; wave time reversibility.  Sources
constant in time (tests/test_oracle_sources.py): single modes against the
forced oscillator and forced decay, constant fields against the k = 0 ODE,
the equations checked by finite differences in time, the source-free limit,
the long-time diffusion limit against the Poisson solve.  The RK4 wave
integrator with a time-dependent source (tests/test_oracle_rk4.py): fourth-
order convergence to the exact source-free and constant-source solutions,
and the self-convergence factor of Sec. III.C on the orbiting source.  3D
(tests/test_oracle_3d.py): brute-force 3D DFT, numpy.fft.fftn, inverse,
Parseval, manufactured Poisson modes, single-mode diffusion and standing
waves in closed form.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fft_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FORWARD, BACKWARD = -1, +1


def build(force: bool = False) -> str:
    """Compile fft_oracle.c with gcc -O2 -ffp-contract=off (no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.c_void_p
        i, d = ctypes.c_int, ctypes.c_double
        lib.oracle_fft1d.argtypes = [dp, dp, i, i]
        lib.oracle_fft2d.argtypes = [dp, dp, i, i, i, i]
        lib.oracle_ifft2d.argtypes = [dp, dp, i, i, i]
        lib.oracle_solve_poisson.argtypes = [dp, dp, i, i, d, d, i]
        lib.oracle_solve_diffusion.argtypes = [dp, dp, i, i, d, d, d, d, i]
        lib.oracle_wave_spectra.argtypes = [dp, dp, dp, dp, i, i, d, d, d, d]
        lib.oracle_solve_wave.argtypes = [dp, dp, dp, dp, i, i, d, d, d, d, i]
        lib.oracle_solve_diffusion_source.argtypes = [dp, dp, dp, i, i, d, d, d, d, i]
        lib.oracle_solve_wave_source.argtypes = [dp, dp, dp, dp, dp, i, i, d, d, d, d, i]
        lib.oracle_fft3d.argtypes = [dp, dp, i, i, i, i, i]
        lib.oracle_ifft3d.argtypes = [dp, dp, i, i, i, i]
        lib.oracle_solve3d.argtypes = [dp, dp, i, i, i, d, d, d, i, d, d, i]
        for f in (lib.oracle_fft3d, lib.oracle_ifft3d, lib.oracle_solve3d,
                  lib.oracle_fft1d, lib.oracle_fft2d, lib.oracle_ifft2d, lib.oracle_solve_poisson,
                  lib.oracle_solve_diffusion, lib.oracle_wave_spectra, lib.oracle_solve_wave,
                  lib.oracle_solve_diffusion_source, lib.oracle_solve_wave_source):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def default_threads() -> int:
    return max(1, os.cpu_count() or 1)


# ---------------------------------------------------------------------------
# transforms
# ---------------------------------------------------------------------------

def fft1d(x, sign: int = FORWARD) -> np.ndarray:
    """Unnormalised 1D transform sum_j x_j exp(sign 2 pi i j k / N)."""
    x = _c128(x)
    out = np.empty_like(x)
    _check(_load().oracle_fft1d(_ptr(x), _ptr(out), x.shape[0], sign), "fft1d")
    return out


def ifft1d(x) -> np.ndarray:
    """Inverse 1D transform: exp(+) sum times 1/N (Sec. II.B iDFT)."""
    return fft1d(x, BACKWARD) / x.shape[0]


def fft2d(x, sign: int = FORWARD, threads: int = 1) -> np.ndarray:
    """Unnormalised 2D transform of a [ny][nx] field, rows then columns."""
    x = _c128(x)
    ny, nx = x.shape
    out = np.empty_like(x)
    _check(_load().oracle_fft2d(_ptr(x), _ptr(out), nx, ny, sign, threads), "fft2d")
    return out


def ifft2d(x, threads: int = 1) -> np.ndarray:
    """Inverse 2D transform: exp(+) sum times 1/(nx*ny)."""
    x = _c128(x)
    ny, nx = x.shape
    out = np.empty_like(x)
    _check(_load().oracle_ifft2d(_ptr(x), _ptr(out), nx, ny, threads), "ifft2d")
    return out


def rfft2d(x, threads: int = 1) -> np.ndarray:
    """Half spectrum of a real [ny][nx] field: columns a = 0 .. nx/2 of its
    forward 2D transform (the others follow from X[-b][-a] = conj(X[b][a])
    for real data, Sec. II.B)."""
    x = np.asarray(x, dtype=np.float64)
    ny, nx = x.shape
    return fft2d(x.astype(np.complex128), threads=threads)[:, : nx // 2 + 1].copy()


def hermitian_extension(X, nx: int) -> np.ndarray:
    """The full [ny][nx] spectrum of which the half spectrum X ([ny][nx//2+1])
    is the Hermitian part: columns 0 < a < nx/2 as given, a > nx/2 from
    conj(X[-b][nx - a]), and the columns that the symmetry maps to
    themselves (a = 0, and a = nx/2 when nx is even) replaced by
    (X[b][a] + conj(X[-b][a])) / 2.  For odd nx the half spectrum holds
    columns 0 .. (nx-1)/2, all but a = 0 as given."""
    X = np.asarray(X, dtype=np.complex128)
    ny, h = X.shape
    assert h == nx // 2 + 1 and nx >= 1
    full = np.empty((ny, nx), dtype=np.complex128)
    for b in range(ny):
        bm = (-b) % ny
        for a in range(nx):
            if a == 0 or 2 * a == nx:
                full[b, a] = (X[b, a] + np.conj(X[bm, a])) / 2
            elif 2 * a < nx:
                full[b, a] = X[b, a]
            else:
                full[b, a] = np.conj(X[bm, nx - a])
    return full


def irfft2d(X, nx: int, threads: int = 1) -> np.ndarray:
    """The real field whose half spectrum is the Hermitian part of X: the
    inverse 2D transform (1/(nx*ny)) of hermitian_extension(X, nx)."""
    z = ifft2d(hermitian_extension(X, nx), threads=threads)
    return z.real.copy()


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

def solve_poisson(s, lx: float, ly: float, threads: int = 1) -> np.ndarray:
    """Zero-mean u with lap(u) = s - mean(s) on a periodic lx-by-ly box."""
    s = _c128(s)
    ny, nx = s.shape
    u = np.empty_like(s)
    _check(_load().oracle_solve_poisson(_ptr(s), _ptr(u), nx, ny, lx, ly, threads), "poisson")
    return u


def solve_diffusion(u0, lx: float, ly: float, kappa: float, t: float,
                    threads: int = 1) -> np.ndarray:
    """u(t) for u_t = kappa lap(u), u(0) = u0, periodic box."""
    u0 = _c128(u0)
    ny, nx = u0.shape
    u = np.empty_like(u0)
    _check(_load().oracle_solve_diffusion(_ptr(u0), _ptr(u), nx, ny, lx, ly, kappa, t, threads),
           "diffusion")
    return u


def solve_wave(u0, v0, lx: float, ly: float, c: float, t: float, want_v: bool = False,
               threads: int = 1) -> Tuple[np.ndarray, Optional[np.ndarray]]:
    """(u(t), u_t(t)) for u_tt = c^2 lap(u), u(0) = u0, u_t(0) = v0 (None => 0)."""
    u0 = _c128(u0)
    v0 = None if v0 is None else _c128(v0)
    ny, nx = u0.shape
    u = np.empty_like(u0)
    v = np.empty_like(u0) if want_v else None
    _check(_load().oracle_solve_wave(_ptr(u0), _ptr(v0), _ptr(u), _ptr(v), nx, ny, lx, ly, c, t,
                                     threads), "wave")
    return u, v


def solve_diffusion_source(f, s, lx: float, ly: float, kappa: float, t: float,
                           threads: int = 1) -> np.ndarray:
    """u(t) for u_t = kappa lap(u) + s, u(0) = f, with s constant in time."""
    f, s = _c128(f), _c128(s)
    ny, nx = f.shape
    u = np.empty_like(f)
    _check(_load().oracle_solve_diffusion_source(_ptr(f), _ptr(s), _ptr(u), nx, ny, lx, ly, kappa, t,
                                                 threads), "diffusion_source")
    return u


def solve_wave_source(f, g, s, lx: float, ly: float, c: float, t: float, want_v: bool = False,
                      threads: int = 1) -> Tuple[np.ndarray, Optional[np.ndarray]]:
    """(u(t), u_t(t)) for u_tt = c^2 lap(u) + s, u(0) = f, u_t(0) = g (None => 0),
    s constant in time."""
    f, s = _c128(f), _c128(s)
    g = None if g is None else _c128(g)
    ny, nx = f.shape
    u = np.empty_like(f)
    v = np.empty_like(f) if want_v else None
    _check(_load().oracle_solve_wave_source(_ptr(f), _ptr(g), _ptr(s), _ptr(u), _ptr(v), nx, ny, lx, ly,
                                            c, t, threads), "wave_source")
    return u, v


def fft3d(x, sign: int = FORWARD, threads: int = 1) -> np.ndarray:
    """Unnormalised 3D transform of an [nz][ny][nx] field: x lines, y lines, z lines."""
    x = _c128(x)
    nz, ny, nx = x.shape
    out = np.empty_like(x)
    _check(_load().oracle_fft3d(_ptr(x), _ptr(out), nx, ny, nz, sign, threads), "fft3d")
    return out


def ifft3d(x, threads: int = 1) -> np.ndarray:
    """Inverse 3D transform: exp(+) sum times 1/(nx*ny*nz)."""
    x = _c128(x)
    nz, ny, nx = x.shape
    out = np.empty_like(x)
    _check(_load().oracle_ifft3d(_ptr(x), _ptr(out), nx, ny, nz, threads), "ifft3d")
    return out


def solve3d(u0, lx: float, ly: float, lz: float, op: int, coef: float = 0.0, t: float = 0.0,
            threads: int = 1) -> np.ndarray:
    """The three solves on a periodic box in 3D: op 0 Poisson (zero-mean u with
    lap(u) = s - mean(s)), op 1 diffusion (kappa = coef), op 2 wave with zero
    initial velocity (c = coef)."""
    u0 = _c128(u0)
    nz, ny, nx = u0.shape
    out = np.empty_like(u0)
    _check(_load().oracle_solve3d(_ptr(u0), _ptr(out), nx, ny, nz, lx, ly, lz, op, coef, t, threads), "solve3d")
    return out


def orbiting_source(nx: int, ny: int, x0: float, y0: float, lx: float, ly: float, t: float, amplitude: float,
                    sigma: float, radius: float, omega: float, gamma: float, cx: float = 0.0,
                    cy: float = 0.0) -> np.ndarray:
    """s(t, x, y) = A exp(-d^2/sigma^2) cos(gamma t) on the grid x_j = x0 + j lx/nx,
    y_k = y0 + k ly/ny, with d the periodic (minimum-image) distance to the
    centre (cx + r cos(Omega t), cy + r sin(Omega t)) -- the orbiting source
    of Sec. III.C."""
    xs = cx + radius * math.cos(omega * t)
    ys = cy + radius * math.sin(omega * t)
    x = x0 + np.arange(nx) * (lx / nx)
    y = y0 + np.arange(ny) * (ly / ny)
    dx = x - xs
    dx -= lx * np.round(dx / lx)
    dy = y - ys
    dy -= ly * np.round(dy / ly)
    d2 = dy[:, None] ** 2 + dx[None, :] ** 2
    return (amplitude * np.exp(-d2 / (sigma * sigma)) * math.cos(gamma * t)).astype(np.complex128)


def wave_rk4(f, g, lx: float, ly: float, c: float, t0: float, dt: float, steps: int, source,
             threads: int = 1) -> Tuple[np.ndarray, np.ndarray]:
    """(u, u_t) at t0 + steps dt for u_tt = c^2 lap(u) + s(t), u(t0) = f,
    u_t(t0) = g (None => 0), by the classical fourth-order Runge-Kutta method
    on the first-order system of Sec. III.C, u^' = v^, v^' = -w^2 u^ + s^(t)
    (w = c|k|), for every Fourier coefficient.  source(t) returns the field
    s(t) on the grid; its spectrum is taken at t, t + dt/2 and t + dt of each
    step (the stage times of the method)."""
    f = _c128(f)
    ny, nx = f.shape
    U = fft2d(f, threads=threads)
    V = fft2d(_c128(g), threads=threads) if g is not None else np.zeros_like(U)
    kx = signed_wavenumbers(nx, lx)
    ky = signed_wavenumbers(ny, ly)
    w2 = c * c * (ky[:, None] ** 2 + kx[None, :] ** 2)

    def rhs(u, v, s):
        return v, -w2 * u + s

    for n in range(steps):
        t = t0 + n * dt
        s1 = fft2d(source(t), threads=threads)
        s2 = fft2d(source(t + 0.5 * dt), threads=threads)
        s3 = fft2d(source(t + dt), threads=threads)
        a1, b1 = rhs(U, V, s1)
        a2, b2 = rhs(U + 0.5 * dt * a1, V + 0.5 * dt * b1, s2)
        a3, b3 = rhs(U + 0.5 * dt * a2, V + 0.5 * dt * b2, s2)
        a4, b4 = rhs(U + dt * a3, V + dt * b3, s3)
        U = U + dt / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4)
        V = V + dt / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4)
    return ifft2d(U, threads=threads), ifft2d(V, threads=threads)


def wave_spectra(F, G, lx: float, ly: float, c: float, t: float):
    """Spectra (U, V) of the wave solution at time t from the spectra F, G of (u0, v0)."""
    F = _c128(F)
    G = None if G is None else _c128(G)
    ny, nx = F.shape
    U = np.empty_like(F)
    V = np.empty_like(F)
    _check(_load().oracle_wave_spectra(_ptr(F), _ptr(G), _ptr(U), _ptr(V), nx, ny, lx, ly, c, t),
           "wave_spectra")
    return U, V


# ---------------------------------------------------------------------------
# diagnostics (the conservation plots of Sec. III.B and III.C)
# ---------------------------------------------------------------------------

def signed_wavenumbers(n: int, length: float) -> np.ndarray:
    """Angular wavenumbers 2 pi a'/L, a' = a for a < n/2 else a - n."""
    a = np.arange(n)
    a = np.where(a < n // 2, a, a - n)
    return 2.0 * math.pi * a / length


def mean_from_spectrum(U) -> complex:
    """Domain mean of the field = k = 0 coefficient / (nx*ny)."""
    U = np.asarray(U)
    return complex(U[0, 0]) / U.size


def l2_from_spectrum(U, lx: float, ly: float) -> float:
    """integral |u|^2 dx dy = (dx dy / P) sum_k |U_k|^2 (Parseval)."""
    U = np.asarray(U)
    ny, nx = U.shape
    return float((lx / nx) * (ly / ny) / U.size * np.sum(np.abs(U) ** 2))


def wave_energy_from_spectra(U, V, lx: float, ly: float, c: float) -> float:
    """E = 1/2 integral (|u_t|^2 + c^2 |grad u|^2) = dx dy/(2P) sum_k (|V_k|^2 + c^2|k|^2 |U_k|^2)."""
    U = np.asarray(U)
    V = np.asarray(V)
    ny, nx = U.shape
    kx = signed_wavenumbers(nx, lx)
    ky = signed_wavenumbers(ny, ly)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    s = np.sum(np.abs(V) ** 2 + c * c * k2 * np.abs(U) ** 2)
    return float((lx / nx) * (ly / ny) / (2.0 * U.size) * s)


def rel_l2(y, ref) -> float:
    """||y - ref||_2 / ||ref||_2 over all real and imaginary components
    (absolute ||y||_2 when ||ref||_2 = 0)."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((y - ref).ravel())
    return float(num / den) if den > 0 else float(num)
