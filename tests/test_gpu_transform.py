"""GPU 2D FFT parity against the FP64 oracle (through the C ABI binding).

Shapes cover every power-of-two side 2..4096 along x and along y, square and
rectangular grids that span several tiles, batches whose last tile is ragged,
and the largest side.  FP64 must match to relative L2 <= 1e-12, FP32 to
2e-6 * log2(max side)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import as_oracle_input, say, to_dev, to_host, tol

pytestmark = pytest.mark.gpu

SIDES = [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]
SHAPES = sorted(set(
    [(n, 8) for n in SIDES] + [(8, n) for n in SIDES] +
    [(n, n) for n in SIDES if n <= 1024] +
    [(2, 2), (4, 2), (32, 1024), (1024, 32), (512, 2048), (2048, 256), (4096, 64), (64, 4096)]))
THREADS = oracle.default_threads()


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_forward_and_inverse(fp, nx, ny, dt):
    say(f"fft2d nx={nx} ny={ny} {dt}")
    x = W.random_field((ny, nx), seed=nx * 7919 + ny)
    xin = as_oracle_input(x, dt)
    ref = oracle.fft2d(xin, threads=THREADS)
    X = fp.fft2d_forward(to_dev(x, dt))
    got = to_host(X)
    assert oracle.rel_l2(got, ref) <= tol(dt, nx, ny, 1)
    # inverse of the exact spectrum
    back = to_host(fp.fft2d_inverse(to_dev(ref, dt)))
    assert oracle.rel_l2(back, oracle.ifft2d(as_oracle_input(ref, dt), threads=THREADS)) <= tol(dt, nx, ny, 1)
    # inverse of forward is the identity
    ident = to_host(fp.fft2d_inverse(X))
    assert oracle.rel_l2(ident, xin) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("nx,ny,batch", [(64, 32, 5), (16, 2048, 3), (2048, 16, 3), (4, 4, 9), (256, 512, 2)])
def test_batched_fields_match_solo(fp, nx, ny, batch, dt):
    say(f"fft2d batch nx={nx} ny={ny} b={batch} {dt}")
    x = W.random_field((batch, ny, nx), seed=batch * 31 + nx)
    X = to_host(fp.fft2d_forward(to_dev(x, dt)))
    for b in range(batch):
        solo = to_host(fp.fft2d_forward(to_dev(x[b], dt)))
        assert np.array_equal(X[b], solo), "batched result differs from the solo result"
        ref = oracle.fft2d(as_oracle_input(x[b], dt), threads=THREADS)
        assert oracle.rel_l2(X[b], ref) <= tol(dt, nx, ny, 1)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_in_place(fp, dt):
    say(f"fft2d in-place {dt}")
    x = W.random_field((128, 256), seed=5)
    t = to_dev(x, dt)
    fp.fft2d_forward(t, out=t)
    ref = oracle.fft2d(as_oracle_input(x, dt))
    assert oracle.rel_l2(to_host(t), ref) <= tol(dt, 256, 128, 1)
    fp.fft2d_inverse(t, out=t)
    assert oracle.rel_l2(to_host(t), as_oracle_input(x, dt)) <= tol(dt, 256, 128, 2)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_single_mode_is_a_delta(fp, dt):
    """exp(+2 pi i (m x + n y)) -> nx*ny at slot (m, n): pins sign and index order."""
    nx, ny, m, n = 64, 32, 5, 29
    j = np.arange(nx)[None, :]
    k = np.arange(ny)[:, None]
    x = np.exp(2j * np.pi * (m * j / nx + n * k / ny))
    X = to_host(fp.fft2d_forward(to_dev(x, dt)))
    ref = np.zeros((ny, nx), dtype=np.complex128)
    ref[n, m] = nx * ny
    assert np.max(np.abs(X - ref)) <= (1e-10 if dt == "c128" else 2e-3)
