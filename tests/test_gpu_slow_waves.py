"""Waves whose speed is 0 or so small that w = c|k| underflows the FP32
scale factors: the propagators must take their w -> 0 limits (u0 + v0 t,
and s t^2/2 for a constant source) instead of dividing by w.  Against the
FP64 oracle, which forms every factor in FP64."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import as_oracle_input, rel_err_vs_input, say, to_dev, to_host, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("c", [0.0, 1e-30, 1e-12])
def test_wave_with_velocity_at_vanishing_speed(fp, dt, c):
    nx, ny, t = 64, 32, 0.7
    say(f"slow wave c={c} {dt}")
    u0, v0 = W.random_field((ny, nx), seed=1), W.random_field((ny, nx), seed=2)
    u, v = fp.solve_wave(to_dev(u0, dt), to_dev(v0, dt), c, t, 1.0, 1.0, want_v=True)
    ru, rv = oracle.solve_wave(as_oracle_input(u0, dt), as_oracle_input(v0, dt), 1.0, 1.0, c, t, want_v=True)
    norm = np.linalg.norm(u0) + np.linalg.norm(v0)
    hu, hv = to_host(u), to_host(v)
    assert np.all(np.isfinite(hu)) and np.all(np.isfinite(hv))
    assert rel_err_vs_input(hu, ru, norm) <= tol(dt, nx, ny, 2)
    assert rel_err_vs_input(hv, rv, norm) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("c", [0.0, 1e-30, 1e-12])
def test_source_wave_at_vanishing_speed(fp, dt, c):
    """Here the reference is the w -> 0 limit itself, in real space:
    u = f + g t + s t^2/2 and u_t = g + s t, exact to O((c k t)^2) <= 1e-19.
    (The oracle's printed form (f - s/w^2) cos(w t) + ... + s/w^2 cancels
    s/w^2 against itself and is meaningless at these w.)"""
    nx, ny, t = 32, 64, 0.4
    say(f"slow source wave c={c} {dt}")
    f, g, s = (W.random_field((ny, nx), seed=k) for k in (3, 4, 5))
    u, v = fp.solve_wave_source(to_dev(f, dt), to_dev(g, dt), to_dev(s, dt), c, t, 1.0, 1.0, want_v=True)
    fi, gi, si = (as_oracle_input(a, dt) for a in (f, g, s))
    ru, rv = fi + gi * t + si * t * t / 2, gi + si * t
    norm = np.linalg.norm(f) + np.linalg.norm(g) + np.linalg.norm(s)
    hu, hv = to_host(u), to_host(v)
    assert np.all(np.isfinite(hu)) and np.all(np.isfinite(hv))
    assert rel_err_vs_input(hu, ru, norm) <= tol(dt, nx, ny, 2)
    assert rel_err_vs_input(hv, rv, norm) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("nx,ny", [(64, 32), (60, 45), (16, 16)])
@pytest.mark.parametrize("c", [1e-30, 1e-12])
def test_wave_without_velocity_at_vanishing_speed(fp, dt, nx, ny, c):
    """u = u0 to within rounding: the power-of-two path, the mixed-radix path
    (60 x 45) and the single-workgroup path (16 x 16)."""
    say(f"slow wave no velocity {nx}x{ny} c={c} {dt}")
    u0 = W.random_field((ny, nx), seed=6)
    u, _ = fp.solve_wave(to_dev(u0, dt), None, c, 0.9, 1.0, 1.0)
    ref, _ = oracle.solve_wave(as_oracle_input(u0, dt), None, 1.0, 1.0, c, 0.9)
    hu = to_host(u)
    assert np.all(np.isfinite(hu))
    assert rel_err_vs_input(hu, ref, np.linalg.norm(u0)) <= tol(dt, nx, ny, 2)
