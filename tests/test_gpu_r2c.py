"""GPU half-spectrum transforms of real fields (fft2d_r2c / fft2d_c2r)
against the FP64 oracle's rfft2d / irfft2d (columns 0..nx/2 of the 2D
transform, and the inverse of the Hermitian part), on powers of two and on
7-smooth sides (odd nx: no Nyquist column)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import TOL_FP64, say, tol

pytestmark = pytest.mark.gpu
THREADS = oracle.default_threads()

SHAPES = [(2, 4), (8, 2), (64, 32), (256, 1024), (4096, 16), (16, 4096), (2048, 2048)]
# half-row passes (nx, ny >= 16 and a column tile no wider than nx/2): every
# row length from 16 to 4096 and column lengths 16..4096
SHAPES += [(32, 1024), (512, 64), (1024, 16), (128, 4096), (4096, 256), (16, 2048)]
# 7-smooth sides (the mixed-radix passes), odd and even nx
SHAPES += [(3, 2), (5, 7), (12, 20), (45, 64), (64, 45), (96, 30), (105, 7), (1536, 10), (9, 2048), (4050, 3)]


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


def _real(shape, seed, dt):
    x = np.random.default_rng(seed).standard_normal(shape)
    return x.astype(np.float32).astype(np.float64) if dt == "f32" else x


def _dev(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.float32 if dt == "f32" else torch.float64).cuda()


def _tol(dt, nx, ny):
    return TOL_FP64 if dt == "f64" else tol("c64", nx, ny, 1)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("batch", [1, 3])
def test_r2c_vs_oracle(fp, nx, ny, dt, batch):
    if nx * ny * batch > 2048 * 2048:
        batch = 1
    say(f"r2c {nx}x{ny} b={batch} {dt}")
    x = _real((batch, ny, nx), nx + ny + batch, dt)
    X = fp.fft2d_r2c(_dev(x, dt)).cpu().numpy().astype(np.complex128)
    assert X.shape == (batch, ny, nx // 2 + 1)
    for k in range(batch):
        ref = oracle.rfft2d(x[k], threads=THREADS)
        assert oracle.rel_l2(X[k], ref) <= _tol(dt, nx, ny), k


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_c2r_vs_oracle_and_round_trip(fp, nx, ny, dt):
    import torch
    batch = 2 if nx * ny < 2048 * 2048 else 1
    say(f"c2r {nx}x{ny} b={batch} {dt}")
    x = _real((batch, ny, nx), 5 * nx + ny, dt)
    X = fp.fft2d_r2c(_dev(x, dt))
    y = fp.fft2d_c2r(X, nx).cpu().numpy()
    assert y.shape == (batch, ny, nx)
    for k in range(batch):
        assert np.linalg.norm(y[k] - x[k]) <= 2 * _tol(dt, nx, ny) * np.linalg.norm(x[k])
    # a half spectrum that is not Hermitian in its self-conjugate columns
    rng = np.random.default_rng(nx * ny)
    H = rng.standard_normal((batch, ny, nx // 2 + 1)) + 1j * rng.standard_normal((batch, ny, nx // 2 + 1))
    cdt = torch.complex64 if dt == "f32" else torch.complex128
    Hd = torch.from_numpy(H).to(cdt).cuda()
    Hin = Hd.cpu().numpy().astype(np.complex128)
    got = fp.fft2d_c2r(Hd, nx).cpu().numpy()
    for k in range(batch):
        ref = oracle.irfft2d(Hin[k], nx, threads=THREADS)
        assert np.linalg.norm(got[k] - ref) <= _tol(dt, nx, ny) * np.linalg.norm(ref), k


def test_odd_batch_last_field_alone(fp):
    """An odd batch pairs its last field with zero: the other results must not
    depend on it, and the last one must be right on its own."""
    nx, ny = 128, 64
    say("r2c odd batch")
    x = _real((5, ny, nx), 3, "f64")
    X = fp.fft2d_r2c(_dev(x, "f64")).cpu().numpy()
    X4 = fp.fft2d_r2c(_dev(x[4:], "f64")).cpu().numpy()
    assert np.abs(X[4] - X4[0]).max() <= 1e-12 * np.abs(X4).max()
    y = fp.fft2d_c2r(fp.fft2d_r2c(_dev(x, "f64")), nx).cpu().numpy()
    assert np.abs(y - x).max() <= 1e-13 * np.abs(x).max()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_smallest_fields(fp, dt):
    """2 x 2 fields: the half spectrum is the whole spectrum (columns 0 and 1)."""
    say(f"r2c 2x2 {dt}")
    x = _real((1, 2, 2), 9, dt)
    X = fp.fft2d_r2c(_dev(x, dt)).cpu().numpy().astype(np.complex128)
    ref = oracle.rfft2d(x[0])
    assert np.abs(X[0] - ref).max() <= (1e-15 if dt == "f64" else 1e-6) * np.abs(ref).max()
    y = fp.fft2d_c2r(fp.fft2d_r2c(_dev(x, dt)), 2).cpu().numpy()
    assert np.abs(y - x).max() <= (1e-15 if dt == "f64" else 1e-6) * np.abs(x).max()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_real_side_not_aligned_like_complex_points(fp, dt):
    """A real input (or output) that starts one element into its buffer is
    not aligned like the complex points the half-row passes read: the pair
    route takes it, with the same results."""
    import torch
    nx, ny = 256, 128
    say(f"r2c unaligned {dt}")
    x = _real((1, ny, nx), 17, dt)
    buf = torch.zeros(nx * ny + 1, dtype=torch.float32 if dt == "f32" else torch.float64, device="cuda:0")
    view = buf[1:].view(1, ny, nx)
    view.copy_(_dev(x, dt))
    X = fp.fft2d_r2c(view).cpu().numpy().astype(np.complex128)
    ref = oracle.rfft2d(x[0], threads=THREADS)
    assert oracle.rel_l2(X[0], ref) <= _tol(dt, nx, ny)
    Xa = fp.fft2d_r2c(_dev(x, dt)).cpu().numpy().astype(np.complex128)
    assert oracle.rel_l2(Xa[0], ref) <= _tol(dt, nx, ny)
    out = torch.zeros_like(buf)
    fp.fft2d_c2r(fp.fft2d_r2c(_dev(x, dt)), nx, out=out[1:].view(1, ny, nx))
    y = out[1:].view(1, ny, nx).cpu().numpy()
    assert np.linalg.norm(y[0] - x[0]) <= 2 * _tol(dt, nx, ny) * np.linalg.norm(x[0])
