"""GPU spectral solves against the FP64 oracle (and closed forms).

Workloads follow the paper's three examples at the sizes of the five named
cases: Poisson 64^2 FP64 (manufactured source), diffusion 1024^2 FP64 and
FP32 (Gaussian + noise, kappa = 0.01, steps of dt = 1e-3), wave 2048^2 FP32
with FP64 phases (Gaussian pulse + standing mode, c = 1, dt = 1e-4), plus
rectangular boxes and the wave with an initial velocity."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import TOL_FP64, as_oracle_input, say, to_dev, to_host, tol

pytestmark = pytest.mark.gpu
THREADS = oracle.default_threads()


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


def _poisson_closed_form(ms):
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


def test_poisson_64_fp64_vs_oracle_and_closed_form(fp):
    say("poisson 64x64 c128")
    ms = W.poisson_source(64, 64, seed=1)
    u = to_host(fp.solve_poisson(to_dev(ms.field, "c128"), 1.0, 1.0))
    ref = oracle.solve_poisson(ms.field, 1.0, 1.0)
    assert oracle.rel_l2(u, ref) <= TOL_FP64
    assert oracle.rel_l2(u, _poisson_closed_form(ms)) <= 1e-13
    assert abs(u.mean()) <= 1e-14


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("nx,ny,lx,ly", [(32, 256, 1.0, 3.0), (512, 64, 2.0, 0.5), (2, 2, 1.0, 1.0),
                                          (4096, 16, 4.0, 1.0), (16, 4096, 1.0, 1.0), (1024, 1024, 1.0, 1.0)])
def test_poisson_rectangular(fp, nx, ny, lx, ly, dt):
    say(f"poisson {nx}x{ny} {dt}")
    k = max(1, min(8, nx // 2 - 1, ny // 2 - 1))
    ms = W.poisson_source(nx, ny, seed=nx + ny, lx=lx, ly=ly, kmax=k)
    s = ms.field
    u = to_host(fp.solve_poisson(to_dev(s, dt), lx, ly))
    ref = oracle.solve_poisson(as_oracle_input(s, dt), lx, ly, threads=THREADS)
    assert oracle.rel_l2(u, ref) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_poisson_random_source_batch(fp, dt):
    say(f"poisson random batch {dt}")
    s = W.random_field((3, 128, 64), seed=17)
    u = to_host(fp.solve_poisson(to_dev(s, dt), 1.0, 2.0))
    for b in range(3):
        ref = oracle.solve_poisson(as_oracle_input(s[b], dt), 1.0, 2.0)
        assert oracle.rel_l2(u[b], ref) <= tol(dt, 64, 128, 2)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("step", [1, 10, 100, 1000])
def test_diffusion_1024(fp, dt, step):
    say(f"diffusion 1024 {dt} step={step}")
    ic = W.diffusion_ic(1024, seed=2)
    t = step * 1e-3
    u = to_host(fp.solve_diffusion(to_dev(ic.field, dt), 0.01, t, 2.0, 2.0))
    ref = oracle.solve_diffusion(as_oracle_input(ic.field, dt), 2.0, 2.0, 0.01, t, threads=THREADS)
    assert oracle.rel_l2(u, ref) <= tol(dt, 1024, 1024, 2)
    # mean conservation (the diffusion plot of Sec. III.B)
    assert abs(u.mean() / ic.field.mean() - 1) <= (1e-12 if dt == "c128" else 1e-5)


def test_diffusion_1024_closed_form_fp64(fp):
    say("diffusion 1024 closed form c128")
    ic = W.diffusion_ic(1024, seed=2, noise_std=0.0)
    u = to_host(fp.solve_diffusion(to_dev(ic.clean, "c128"), 0.01, 1.0, 2.0, 2.0))
    x = W.grid(1024, 2.0, -1.0)
    X, Y = np.meshgrid(x, x)
    st2 = 0.05 ** 2 + 2 * 0.01 * 1.0
    ref = sum(np.exp(-((X - 2 * m) ** 2 + (Y - 2 * q) ** 2) / (2 * st2)) for m in (-1, 0, 1) for q in (-1, 0, 1))
    ref = ref * 0.05 ** 2 / st2
    assert oracle.rel_l2(u, ref) <= 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("nx,ny", [(64, 256), (2, 8), (4096, 32)])
def test_diffusion_rectangular(fp, nx, ny, dt):
    say(f"diffusion {nx}x{ny} {dt}")
    f = W.random_field((ny, nx), seed=3)
    u = to_host(fp.solve_diffusion(to_dev(f, dt), 0.3, 0.02, 1.0, 3.0))
    ref = oracle.solve_diffusion(as_oracle_input(f, dt), 1.0, 3.0, 0.3, 0.02, threads=THREADS)
    assert oracle.rel_l2(u, ref) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("step", [1, 100, 1000, 5000])
def test_wave_2048_fp32(fp, step):
    say(f"wave 2048 c64 step={step}")
    ic = W.wave_ic(2048, seed=3)
    t = step * 1e-4
    u, _ = fp.solve_wave(to_dev(ic.field, "c64"), None, 1.0, t, 1.0, 1.0)
    u = to_host(u)
    ref, _ = oracle.solve_wave(as_oracle_input(ic.field, "c64"), None, 1.0, 1.0, 1.0, t, threads=THREADS)
    assert oracle.rel_l2(u, ref) <= tol("c64", 2048, 2048, 2)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_wave_standing_mode_closed_form(fp, dt):
    say(f"wave standing 256 {dt}")
    ic = W.wave_ic(256, seed=3, pulse=False)
    w = 2 * math.pi * math.sqrt(34)
    for t in (0.0, 0.0123, 0.5):
        u, _ = fp.solve_wave(to_dev(ic.field, dt), None, 1.0, t)
        err = oracle.rel_l2(to_host(u), ic.field * math.cos(w * t))
        assert err <= (1e-12 if dt == "c128" else tol("c64", 256, 256, 2))


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("nx,ny", [(128, 128), (64, 512), (2048, 64), (8, 4096)])
def test_wave_with_velocity(fp, nx, ny, dt):
    say(f"wave u0,v0 {nx}x{ny} {dt}")
    u0 = W.random_field((ny, nx), seed=1)
    v0 = W.random_field((ny, nx), seed=2)
    for t in (0.0, 0.3, -0.7):
        u, v = fp.solve_wave(to_dev(u0, dt), to_dev(v0, dt), 0.8, t, 2.0, 1.0, want_v=True)
        ru, rv = oracle.solve_wave(as_oracle_input(u0, dt), as_oracle_input(v0, dt), 2.0, 1.0, 0.8, t,
                                   want_v=True, threads=THREADS)
        assert oracle.rel_l2(to_host(u), ru) <= tol(dt, nx, ny, 2)
        assert oracle.rel_l2(to_host(v), rv) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_wave_velocity_only_variants(fp, dt):
    """v0 given but v not requested (workspace path), and v requested with v0 = 0."""
    say(f"wave variants {dt}")
    u0 = W.random_field((64, 128), seed=4)
    v0 = W.random_field((64, 128), seed=5)
    u, v = fp.solve_wave(to_dev(u0, dt), to_dev(v0, dt), 1.0, 0.25)
    assert v is None
    ru, _ = oracle.solve_wave(as_oracle_input(u0, dt), as_oracle_input(v0, dt), 1.0, 1.0, 1.0, 0.25)
    assert oracle.rel_l2(to_host(u), ru) <= tol(dt, 128, 64, 2)
    u, v = fp.solve_wave(to_dev(u0, dt), None, 1.0, 0.25, want_v=True)
    ru, rv = oracle.solve_wave(as_oracle_input(u0, dt), None, 1.0, 1.0, 1.0, 0.25, want_v=True)
    assert oracle.rel_l2(to_host(u), ru) <= tol(dt, 128, 64, 2)
    assert oracle.rel_l2(to_host(v), rv) <= tol(dt, 128, 64, 2)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_solves_in_place(fp, dt):
    say(f"solves in place {dt}")
    f = W.random_field((256, 128), seed=8)
    t = to_dev(f, dt)
    fp.solve_diffusion(t, 0.1, 0.05, 1.0, 1.0, out=t)
    ref = oracle.solve_diffusion(as_oracle_input(f, dt), 1.0, 1.0, 0.1, 0.05)
    assert oracle.rel_l2(to_host(t), ref) <= tol(dt, 128, 256, 2)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("op,nx,ny,batch", [("wave", 2048, 2048, 2), ("wave", 256, 512, 3),
                                            ("diffusion", 512, 128, 2), ("diffusion", 4, 4096, 2),
                                            ("wave", 4096, 16, 3)])
def test_multi_field_solves_vs_oracle(fp, dt, op, nx, ny, batch):
    """Diffusion and wave solves over several fields of 3-pass shapes (tiles
    within one column block, and narrow fields whose tiles span fields):
    every field against the oracle."""
    say(f"multi-field {op} {nx}x{ny}x{batch} {dt}")
    f = W.random_field((batch, ny, nx), seed=nx + ny + batch)
    x = to_dev(f, dt)
    if op == "wave":
        out = to_host(fp.solve_wave(x, None, 0.9, 0.37, 1.0, 2.0)[0])
    else:
        out = to_host(fp.solve_diffusion(x, 0.05, 0.21, 2.0, 1.0))
    for k in range(batch):
        g = as_oracle_input(f[k], dt)
        if op == "wave":
            ref, _ = oracle.solve_wave(g, None, 1.0, 2.0, 0.9, 0.37, threads=THREADS)
        else:
            ref = oracle.solve_diffusion(g, 2.0, 1.0, 0.05, 0.21, threads=THREADS)
        assert oracle.rel_l2(out[k], ref) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("nx,ny,batch", [(2048, 2048, 2), (1024, 512, 3), (4096, 64, 2), (64, 4096, 1),
                                         (8, 2048, 5), (4, 1024, 3)])
def test_tiled_intermediate_is_bit_identical(fp, dt, nx, ny, batch):
    """The solve's spectrum between passes in column blocks (default) or
    row-major: the same arithmetic, so the same bits, for every operator;
    and the tiled result against the oracle."""
    import torch
    say(f"tiled vs row-major {nx}x{ny}x{batch} {dt}")
    x = to_dev(W.random_field((batch, ny, nx), seed=nx + 3 * ny), dt)
    outs = {}
    try:
        for mode in (128, 8, 1024, 0):
            fp.plan_tiled(mode)
            outs[mode] = (fp.solve_poisson(x, 1.0, 2.0), fp.solve_diffusion(x, 0.01, 0.3, 1.0, 2.0),
                          fp.solve_wave(x, None, 1.0, 0.37, 1.0, 2.0)[0])
    finally:
        fp.plan_tiled(1024)
    for mode in (128, 8, 1024):
        for a, b in zip(outs[mode], outs[0]):
            assert torch.equal(a, b)
    ref = oracle.solve_poisson(as_oracle_input(W.random_field((batch, ny, nx), seed=nx + 3 * ny)[-1], dt), 1.0, 2.0,
                               threads=THREADS)
    assert oracle.rel_l2(to_host(outs[128][0])[-1], ref) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_chunked_batches_are_bit_identical(fp, dt):
    """A batch run in chunks (one field, three fields with a ragged last
    chunk, the default) gives the same bits as the whole batch at once, in
    both layouts."""
    import torch
    nx, ny, batch = 256, 512, 7
    field = nx * ny * (8 if dt == "c64" else 16)
    say(f"chunked {nx}x{ny}x{batch} {dt}")
    x = to_dev(W.random_field((batch, ny, nx), seed=17), dt)
    outs = []
    try:
        for tiled in (1024, 0):
            fp.plan_tiled(tiled)
            for chunk in (0, field, 3 * field, 256 << 20):
                fp.plan_chunk(chunk)
                outs.append(fp.solve_wave(x, None, 1.0, 0.41, 1.0, 2.0)[0])
    finally:
        fp.plan_tiled(1024)
        fp.plan_chunk(256 << 20)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_chunked_transforms_wave_velocity_and_evolution_are_bit_identical(fp, dt):
    """Every multi-pass path run in chunks (one field, three with a ragged
    last chunk) gives the bits of the whole batch at once: 2D transforms, the
    wave with an initial velocity and a velocity output, evolution steps."""
    import torch
    nx, ny, batch = 128, 256, 5
    field = nx * ny * (8 if dt == "c64" else 16)
    say(f"chunked paths {nx}x{ny}x{batch} {dt}")
    u0 = to_dev(W.random_field((batch, ny, nx), seed=21), dt)
    v0 = to_dev(W.random_field((batch, ny, nx), seed=22), dt)
    runs = []
    try:
        for chunk in (0, field, 3 * field):
            fp.plan_chunk(chunk)
            r = [fp.fft2d_forward(u0), fp.fft2d_inverse(u0)]
            r += list(fp.solve_wave(u0, v0, 0.8, 0.3, 1.0, 2.0, want_v=True))
            r.append(fp.solve_wave(u0, v0, 0.8, 0.3, 1.0, 2.0)[0])
            with fp.Evolution(fp.WAVE, u0, v0, 0.8, 1.0, 2.0) as ev:
                u, v, _ = ev.step(7, 0.05, want_v=True)
                r += [u, v]
            with fp.Evolution(fp.DIFFUSION, u0, None, 0.01, 1.0, 2.0) as ev:
                r.append(ev.step(3, 0.1)[0])
            runs.append(r)
    finally:
        fp.plan_chunk(256 << 20)
    for r in runs[1:]:
        for a, b in zip(r, runs[0]):
            assert torch.equal(a, b)
