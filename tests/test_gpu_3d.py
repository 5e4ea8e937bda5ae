"""3D transforms and solves against the FP64 oracle (x rows, y columns per
plane, z columns with the symbol fused), FP32 and FP64."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import TOL_FP64, as_oracle_input, say, to_dev, to_host


def tol3(dt, nx, ny, nz, transforms):
    """FP64: 1e-12.  FP32: 2e-6 log2(nx ny nz) per 3D transform (the 1D bound
    of each direction, summed over the three directions)."""
    return TOL_FP64 if dt == "c128" else transforms * 2e-6 * np.log2(nx * ny * nz)

pytestmark = pytest.mark.gpu
THREADS = oracle.default_threads()


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


SHAPES = [(8, 16, 32, 2), (64, 64, 64, 1), (128, 32, 8, 3), (2, 4, 2, 2), (256, 256, 16, 1)]


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("nx,ny,nz,batch", SHAPES)
def test_fft3d_vs_oracle(fp, dt, nx, ny, nz, batch):
    say(f"fft3d {nx}x{ny}x{nz}x{batch} {dt}")
    x = W.random_field((batch, nz, ny, nx), seed=nx + ny + nz)
    X = to_host(fp.fft3d_forward(to_dev(x, dt)))
    back = to_host(fp.fft3d_inverse(to_dev(X, dt)))
    for b in range(batch):
        ref = oracle.fft3d(as_oracle_input(x[b], dt), threads=THREADS)
        assert oracle.rel_l2(X[b], ref) <= tol3(dt, nx, ny, nz, 1)
    assert oracle.rel_l2(back, as_oracle_input(x, dt)) <= tol3(dt, nx, ny, nz, 2)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("op", [0, 1, 2])
@pytest.mark.parametrize("nx,ny,nz,batch", [(32, 16, 64, 2), (128, 128, 128, 1), (4, 256, 8, 2)])
def test_solves3d_vs_oracle(fp, dt, op, nx, ny, nz, batch):
    say(f"solve3d op={op} {nx}x{ny}x{nz}x{batch} {dt}")
    f = W.random_field((batch, nz, ny, nx), seed=op + nx + 2 * ny + 3 * nz)
    lx, ly, lz, coef, t = 1.0, 2.0, 0.5, 0.3, 0.21
    x = to_dev(f, dt)
    if op == 0:
        u = fp.solve_poisson_3d(x, lx, ly, lz)
    elif op == 1:
        u = fp.solve_diffusion_3d(x, coef, t, lx, ly, lz)
    else:
        u = fp.solve_wave_3d(x, coef, t, lx, ly, lz)
    u = to_host(u)
    for b in range(batch):
        g = as_oracle_input(f[b], dt)
        ref = oracle.solve3d(g, lx, ly, lz, op, coef, t, threads=THREADS)
        # |symbol| <= 1 for diffusion and wave: relative to the larger of result and input
        scale = max(np.linalg.norm(ref), np.linalg.norm(g) if op else 0.0)
        assert np.linalg.norm(u[b] - ref) / scale <= tol3(dt, nx, ny, nz, 2)


def test_3d_wave_standing_mode_closed_form(fp):
    nx, ny, nz = 32, 16, 64
    x, y, z = W.grid(nx, 1.0), W.grid(ny, 1.0), W.grid(nz, 1.0)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    mode = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * 2 * Y) * np.sin(2 * np.pi * 3 * Z)
    w = 2 * np.pi * np.sqrt(1 + 4 + 9)
    for t in (0.0, 0.05, 0.33):
        u = to_host(fp.solve_wave_3d(to_dev(mode[None], "c128"), 1.0, t))[0]
        assert np.abs(u - np.cos(w * t) * mode).max() <= 1e-12
