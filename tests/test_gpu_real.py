"""Real-field solves (FFTPDE_R32 / FFTPDE_R64) against the FP64 oracle.

The solves' symbols are real and even in k, so each solve maps real fields to
real fields and is complex linear; the library solves fields 2p and 2p+1 as
the real and imaginary parts of one complex field.  Every real field is
checked against the oracle run on that field alone (imaginary part 0).  The
FP32 bound is the complex path's, taken relative to the pair's joint norm
(the rounding of a complex transform scales with the norm of its input)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import TOL_FP64, say, tol_fp32

pytestmark = pytest.mark.gpu
THREADS = oracle.default_threads()


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


def _dev(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to({"r32": torch.float32, "r64": torch.float64}[dt]).cuda()


def _host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _seen(a, dt):
    """The values the GPU sees (FP32 inputs rounded first), in FP64."""
    a = np.asarray(a, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if dt == "r32" else a


def _ref(op, g, lx, ly, coef, t, v0=None, want_v=False):
    g = g.astype(np.complex128)
    if op == "poisson":
        return oracle.solve_poisson(g, lx, ly, threads=THREADS), None
    if op == "diffusion":
        return oracle.solve_diffusion(g, lx, ly, coef, t, threads=THREADS), None
    return oracle.solve_wave(g, None if v0 is None else v0.astype(np.complex128), lx, ly, coef, t,
                             want_v=want_v, threads=THREADS)


def _check_pairs(got, refs, dt, nx, ny):
    """Per field: ||u_k - ref_k|| / ||(ref_2p, ref_2p+1)|| within the bound,
    and the reference itself real (the oracle's imaginary part is rounding)."""
    bound = TOL_FP64 if dt == "r64" else tol_fp32(nx, ny, 2)
    for k, ref in enumerate(refs):
        assert np.linalg.norm(ref.imag) <= 1e-12 * max(np.linalg.norm(ref.real), 1e-300)
        p = k - (k % 2)
        pair = [r.real for r in refs[p:p + 2]]
        denom = max(np.sqrt(sum(np.linalg.norm(r) ** 2 for r in pair)), 1e-300)
        err = np.linalg.norm(got[k] - ref.real) / denom
        assert err <= bound, (k, err, bound)


@pytest.mark.parametrize("dt", ["r32", "r64"])
@pytest.mark.parametrize("op,nx,ny,batch", [
    ("poisson", 64, 64, 1), ("wave", 2048, 2048, 3), ("diffusion", 256, 512, 5), ("wave", 4096, 16, 2),
    ("poisson", 8, 2048, 4), ("diffusion", 2, 4, 3), ("poisson", 1024, 2, 2)])
def test_real_solves_vs_oracle(fp, dt, op, nx, ny, batch):
    say(f"real {op} {nx}x{ny}x{batch} {dt}")
    f = W.random_field((batch, ny, nx), seed=7 * nx + ny + batch).real
    x = _dev(f, dt)
    lx, ly, coef, t = 1.0, 2.0, 0.3, 0.41
    if op == "poisson":
        u = fp.solve_poisson(x, lx, ly)
    elif op == "diffusion":
        u = fp.solve_diffusion(x, coef, t, lx, ly)
    else:
        u = fp.solve_wave(x, None, coef, t, lx, ly)[0]
    assert u.dtype == x.dtype and u.shape == x.shape
    got = _host(u)
    refs = [_ref(op, _seen(f[k], dt), lx, ly, coef, t)[0] for k in range(batch)]
    _check_pairs(got, refs, dt, nx, ny)


@pytest.mark.parametrize("dt", ["r32", "r64"])
@pytest.mark.parametrize("nx,ny,batch", [(128, 256, 3), (2048, 64, 2)])
def test_real_wave_with_velocity(fp, dt, nx, ny, batch):
    """u0 and v0 real, u and u_t requested; v0 given without u_t; u_t without v0."""
    say(f"real wave u0,v0 {nx}x{ny}x{batch} {dt}")
    u0 = W.random_field((batch, ny, nx), seed=31).real
    v0 = W.random_field((batch, ny, nx), seed=32).real
    c, t, lx, ly = 0.8, -0.37, 2.0, 1.0
    u, v = fp.solve_wave(_dev(u0, dt), _dev(v0, dt), c, t, lx, ly, want_v=True)
    refs = [_ref("wave", _seen(u0[k], dt), lx, ly, c, t, v0=_seen(v0[k], dt), want_v=True) for k in range(batch)]
    _check_pairs(_host(u), [r[0] for r in refs], dt, nx, ny)
    _check_pairs(_host(v), [r[1] for r in refs], dt, nx, ny)
    u2, none = fp.solve_wave(_dev(u0, dt), _dev(v0, dt), c, t, lx, ly)
    assert none is None
    _check_pairs(_host(u2), [r[0] for r in refs], dt, nx, ny)
    u3, v3 = fp.solve_wave(_dev(u0, dt), None, c, t, lx, ly, want_v=True)
    refs0 = [_ref("wave", _seen(u0[k], dt), lx, ly, c, t, v0=None, want_v=True) for k in range(batch)]
    _check_pairs(_host(u3), [r[0] for r in refs0], dt, nx, ny)
    _check_pairs(_host(v3), [r[1] for r in refs0], dt, nx, ny)


@pytest.mark.parametrize("dt", ["r32", "r64"])
def test_real_solve_in_place_chunked_and_against_complex_path(fp, dt):
    """In place (out = in), in chunks of one pair with a ragged last chunk, and
    against the same fields solved one by one as complex fields (imaginary 0)."""
    import torch
    nx, ny, batch = 256, 128, 5
    say(f"real in place / chunks {nx}x{ny}x{batch} {dt}")
    f = W.random_field((batch, ny, nx), seed=41).real
    x = _dev(f, dt)
    whole = fp.solve_diffusion(x, 0.05, 0.3, 1.0, 1.0)
    pair_bytes = nx * ny * (8 if dt == "r32" else 16)
    try:
        fp.plan_chunk(pair_bytes)
        chunked = fp.solve_diffusion(x, 0.05, 0.3, 1.0, 1.0)
    finally:
        fp.plan_chunk(256 << 20)
    assert torch.equal(whole, chunked)
    y = x.clone()
    fp.solve_diffusion(y, 0.05, 0.3, 1.0, 1.0, out=y)
    assert torch.equal(y, whole)
    cdt = torch.complex64 if dt == "r32" else torch.complex128
    zc = fp.solve_diffusion(x.to(cdt), 0.05, 0.3, 1.0, 1.0)
    bound = TOL_FP64 if dt == "r64" else tol_fp32(nx, ny, 2)
    err = np.linalg.norm(_host(whole) - zc.real.cpu().numpy()) / np.linalg.norm(zc.real.cpu().numpy())
    assert err <= bound


def test_real_fields_are_rejected_where_complex_is_required(fp):
    import torch
    x = torch.zeros((4, 4), dtype=torch.float32, device="cuda:0")
    with pytest.raises(TypeError):
        fp.fft2d_forward(x)
    with pytest.raises((TypeError, ValueError)):
        fp.solve_wave(torch.zeros((4, 4), dtype=torch.complex64, device="cuda:0"), x)
    with pytest.raises(TypeError):
        fp.Evolution(fp.WAVE, x)
