"""Solves with a source constant in time against the FP64 oracle: diffusion
(forced decay) and the wave (forced oscillator, with the constant particular
solution), complex and real fields, FP32 and FP64."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import TOL_FP64, as_oracle_input, say, to_dev, to_host, tol, tol_fp32

pytestmark = pytest.mark.gpu
THREADS = oracle.default_threads()


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


def _rel(y, ref, scale):
    return float(np.linalg.norm(np.asarray(y) - ref) / scale)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("nx,ny,batch", [(256, 128, 2), (2048, 2048, 1), (8, 1024, 3), (4096, 4, 2)])
def test_diffusion_source_vs_oracle(fp, dt, nx, ny, batch):
    say(f"diffusion source {nx}x{ny}x{batch} {dt}")
    f = W.random_field((batch, ny, nx), seed=nx + 2 * ny)
    s = W.random_field((batch, ny, nx), seed=nx + 2 * ny + 1)
    kappa, t, lx, ly = 0.02, 0.7, 2.0, 1.0
    u = to_host(fp.solve_diffusion_source(to_dev(f, dt), to_dev(s, dt), kappa, t, lx, ly))
    for k in range(batch):
        ref = oracle.solve_diffusion_source(as_oracle_input(f[k], dt), as_oracle_input(s[k], dt), lx, ly, kappa, t,
                                            threads=THREADS)
        # the source term grows with t; bound relative to the larger of the result and the data
        scale = max(np.linalg.norm(ref), np.linalg.norm(f[k]), np.linalg.norm(s[k]) * t)
        assert _rel(u[k], ref, scale) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("nx,ny,batch", [(128, 256, 2), (2048, 2048, 1), (1024, 8, 3)])
def test_wave_source_vs_oracle(fp, dt, nx, ny, batch):
    say(f"wave source {nx}x{ny}x{batch} {dt}")
    f = W.random_field((batch, ny, nx), seed=3 * nx + ny)
    g = W.random_field((batch, ny, nx), seed=3 * nx + ny + 1)
    s = W.random_field((batch, ny, nx), seed=3 * nx + ny + 2)
    c, lx, ly = 0.8, 1.0, 2.0
    for t in (0.37, -1.3):
        u, v = fp.solve_wave_source(to_dev(f, dt), to_dev(g, dt), to_dev(s, dt), c, t, lx, ly, want_v=True)
        u, v = to_host(u), to_host(v)
        u2, none = fp.solve_wave_source(to_dev(f, dt), None, to_dev(s, dt), c, t, lx, ly)
        assert none is None
        u2 = to_host(u2)
        for k in range(batch):
            fk, gk, sk = (as_oracle_input(a[k], dt) for a in (f, g, s))
            ru, rv = oracle.solve_wave_source(fk, gk, sk, lx, ly, c, t, want_v=True, threads=THREADS)
            ru2, _ = oracle.solve_wave_source(fk, None, sk, lx, ly, c, t, threads=THREADS)
            # the k = 0 mode grows as s t^2/2; bound relative to the data and the result
            scale = max(np.linalg.norm(ru), np.linalg.norm(fk), np.linalg.norm(gk) * abs(t), np.linalg.norm(sk) * t * t)
            assert _rel(u[k], ru, scale) <= tol(dt, nx, ny, 2)
            assert _rel(u2[k], ru2, max(scale, np.linalg.norm(ru2))) <= tol(dt, nx, ny, 2)
            vscale = max(np.linalg.norm(rv), np.linalg.norm(gk), np.linalg.norm(sk) * abs(t))
            # the velocity carries w f^: its rounding scales with max w ||f||
            wmax = c * 2 * np.pi * np.hypot(nx / 2 / lx, ny / 2 / ly)
            vscale = max(vscale, wmax * np.linalg.norm(fk))
            assert _rel(v[k], rv, vscale) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["r32", "r64"])
def test_source_solves_on_real_fields(fp, dt):
    import torch
    nx, ny, batch = 256, 64, 3
    say(f"sources on real fields {nx}x{ny}x{batch} {dt}")
    tdt = torch.float32 if dt == "r32" else torch.float64
    f = W.random_field((batch, ny, nx), seed=51).real
    g = W.random_field((batch, ny, nx), seed=52).real
    s = W.random_field((batch, ny, nx), seed=53).real
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(tdt).cuda()  # noqa: E731
    seen = lambda a: a.astype(np.float32).astype(np.float64) if dt == "r32" else a  # noqa: E731
    ud = fp.solve_diffusion_source(dev(f), dev(s), 0.05, 0.4, 1.0, 1.0).cpu().numpy().astype(np.float64)
    uw, vw = fp.solve_wave_source(dev(f), dev(g), dev(s), 1.1, 0.6, 1.0, 1.0, want_v=True)
    uw, vw = (x.cpu().numpy().astype(np.float64) for x in (uw, vw))
    bound = TOL_FP64 if dt == "r64" else tol_fp32(nx, ny, 2)
    wmax = 1.1 * 2 * np.pi * np.hypot(nx / 2, ny / 2)
    for k in range(batch):
        p = k - (k % 2)
        pair = slice(p, p + 2)
        rd = oracle.solve_diffusion_source(seen(f[k]), seen(s[k]), 1.0, 1.0, 0.05, 0.4).real
        ru, rv = oracle.solve_wave_source(seen(f[k]), seen(g[k]), seen(s[k]), 1.0, 1.0, 1.1, 0.6, want_v=True)
        # per field, relative to the pair's data (the transforms' rounding scales with the pair's norm)
        data = np.sqrt(sum(np.linalg.norm(a[pair]) ** 2 for a in (f, g, s)))
        assert np.linalg.norm(ud[k] - rd) / max(data, np.linalg.norm(rd)) <= bound
        assert np.linalg.norm(uw[k] - ru.real) / max(data, np.linalg.norm(ru)) <= bound
        assert np.linalg.norm(vw[k] - rv.real) / max(wmax * data, np.linalg.norm(rv)) <= bound


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_zero_source_matches_the_source_free_solves(fp, dt):
    nx, ny = 128, 64
    say(f"zero source {dt}")
    f = W.random_field((2, ny, nx), seed=61)
    g = W.random_field((2, ny, nx), seed=62)
    z = np.zeros_like(f)
    u, v = fp.solve_wave_source(to_dev(f, dt), to_dev(g, dt), to_dev(z, dt), 1.0, 0.45, want_v=True)
    ru, rv = fp.solve_wave(to_dev(f, dt), to_dev(g, dt), 1.0, 0.45, want_v=True)
    assert oracle.rel_l2(to_host(u), to_host(ru)) <= tol(dt, nx, ny, 2)
    assert oracle.rel_l2(to_host(v), to_host(rv)) <= tol(dt, nx, ny, 2)
    d = fp.solve_diffusion_source(to_dev(f, dt), to_dev(z, dt), 0.1, 0.3)
    rd = fp.solve_diffusion(to_dev(f, dt), 0.1, 0.3)
    assert oracle.rel_l2(to_host(d), to_host(rd)) <= tol(dt, nx, ny, 2)
