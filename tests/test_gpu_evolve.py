"""Time evolution with resident spectra against the FP64 oracle, at the named
cases' sizes and checked steps: diffusion 1024^2 (kappa 0.01, dt 1e-3, steps
1..1000) in FP64 and FP32, wave 2048^2 FP32 with FP64 phases (c 1, dt 1e-4,
steps 1..5000); the diagnostics (mean and energy from the spectra) against
the oracle's spectra and the paper's conservation statements."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import as_oracle_input, rel_err_vs_input, say, to_dev, to_host, tol

pytestmark = pytest.mark.gpu
THREADS = oracle.default_threads()


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_diffusion_1024_steps(fp, dt):
    ic = W.diffusion_ic(1024, seed=2)
    x = as_oracle_input(ic.field, dt)
    with fp.Evolution(fp.DIFFUSION, to_dev(ic.field, dt), coef=0.01, lx=2.0, ly=2.0) as ev:
        means = []
        for n in (1, 10, 100, 1000):
            say(f"evolve diffusion 1024 {dt} n={n}")
            u, _, d = ev.step(n, 1e-3, diag=True)
            t = n * 1e-3
            ref = oracle.solve_diffusion(x, 2.0, 2.0, 0.01, t, threads=THREADS)
            assert oracle.rel_l2(to_host(u), ref) <= tol(dt, 1024, 1024, 2)
            d = d.cpu().numpy()[0]
            U = oracle.fft2d(ref, threads=THREADS)
            # the energy is quadratic in the spectrum, which the FP32 path holds in FP32
            e_tol = 1e-10 if dt == "c128" else 2 * tol("c64", 1024, 1024, 1)
            assert d[2] == pytest.approx(oracle.l2_from_spectrum(U, 2.0, 2.0), rel=e_tol)
            means.append(d[0])
        # mean conservation (Sec. III.B): the k = 0 mode is never changed
        assert all(abs(m / means[0] - 1) <= 1e-12 for m in means)
        assert means[0] == pytest.approx(x.mean().real, rel=1e-10 if dt == "c128" else 1e-6)


def test_wave_2048_fp32_steps_and_energy(fp):
    ic = W.wave_ic(2048, seed=3)
    x = as_oracle_input(ic.field, "c64")
    with fp.Evolution(fp.WAVE, to_dev(ic.field, "c64"), coef=1.0) as ev:
        energies = []
        for n in (1, 100, 1000, 5000):
            say(f"evolve wave 2048 c64 n={n}")
            u, _, d = ev.step(n, 1e-4, diag=True)
            ref, _ = oracle.solve_wave(x, None, 1.0, 1.0, 1.0, n * 1e-4, threads=THREADS)
            assert oracle.rel_l2(to_host(u), ref) <= tol("c64", 2048, 2048, 2)
            energies.append(d.cpu().numpy()[0, 2])
        # energy from the resident spectra is conserved mode by mode
        assert all(abs(e / energies[0] - 1) <= 1e-12 for e in energies)
        F = oracle.fft2d(x, threads=THREADS)
        U, V = oracle.wave_spectra(F, None, 1.0, 1.0, 1.0, 0.5)
        assert energies[-1] == pytest.approx(oracle.wave_energy_from_spectra(U, V, 1.0, 1.0, 1.0),
                                             rel=2 * tol("c64", 2048, 2048, 1))


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_wave_standing_mode_energy_and_closed_form(fp, dt, closed_forms):
    ic = W.wave_ic(256, seed=3, pulse=False)
    w = 2 * math.pi * math.sqrt(34)
    with fp.Evolution(fp.WAVE, to_dev(ic.field, dt), coef=1.0) as ev:
        for n in (0, 7, 1234):
            say(f"evolve standing {dt} n={n}")
            u, v, d = ev.step(n, 1e-4, want_v=True, diag=True)
            t = n * 1e-4
            u0n = np.linalg.norm(ic.field)
            if dt == "c128":
                assert oracle.rel_l2(to_host(u), ic.field * math.cos(w * t)) <= 1e-12
            else:
                assert rel_err_vs_input(to_host(u), ic.field * math.cos(w * t), u0n) <= tol(dt, 256, 256, 2)
            vref = -w * math.sin(w * t) * ic.field
            if n:
                if dt == "c128":
                    assert oracle.rel_l2(to_host(v), vref) <= 1e-12
                else:
                    assert rel_err_vs_input(to_host(v), vref, w * u0n) <= tol(dt, 256, 256, 2)
            assert d.cpu().numpy()[0, 2] == pytest.approx(closed_forms["standing_energy"], rel=1e-10 if dt == "c128" else 1e-6)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_wave_with_velocity_batch(fp, dt):
    u0 = W.random_field((2, 64, 128), seed=31)
    v0 = W.random_field((2, 64, 128), seed=32)
    with fp.Evolution(fp.WAVE, to_dev(u0, dt), to_dev(v0, dt), coef=0.7, lx=2.0, ly=1.0) as ev:
        for n in (3, -5):
            say(f"evolve wave velocity {dt} n={n}")
            u, v, d = ev.step(n, 0.05, want_v=True, diag=True)
            u, v, d = to_host(u), to_host(v), d.cpu().numpy()
            for b in range(2):
                ru, rv = oracle.solve_wave(as_oracle_input(u0[b], dt), as_oracle_input(v0[b], dt), 2.0, 1.0, 0.7,
                                           n * 0.05, want_v=True)
                assert oracle.rel_l2(u[b], ru) <= tol(dt, 128, 64, 2)
                assert oracle.rel_l2(v[b], rv) <= tol(dt, 128, 64, 2)
                assert d[b, 0] + 1j * d[b, 1] == pytest.approx(ru.mean(), rel=1e-9 if dt == "c128" else 1e-4, abs=1e-12)


def test_diagnostics_only_step_writes_nothing(fp):
    f = W.random_field((32, 32), seed=3)
    with fp.Evolution(fp.DIFFUSION, to_dev(f, "c128"), coef=0.5) as ev:
        u, v, d = ev.step(4, 0.01, want_u=False, diag=True)
        assert u is None and v is None
        U = oracle.fft2d(oracle.solve_diffusion(f, 1.0, 1.0, 0.5, 0.04))
        assert d.cpu().numpy()[0, 2] == pytest.approx(oracle.l2_from_spectrum(U, 1.0, 1.0), rel=1e-12)
