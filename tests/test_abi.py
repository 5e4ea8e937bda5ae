"""The C ABI without a GPU: the library loads, exports every function that
include/fftpde.h declares, and rejects bad arguments with FFTPDE_EINVAL before
touching the device."""
import ctypes
import math
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "fftpde.h")


def _lib():
    import paper_2412_12308_amd as fp
    if not os.path.exists(fp.LIB_PATH):
        pytest.skip("libfftpde.so not built (run __graft_entry__.build())")
    return fp, fp.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char \*|void)\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("fftpde_create", "fftpde_destroy", "fftpde_strerror", "fft2d_forward", "fft2d_inverse",
              "solve_poisson", "solve_diffusion", "solve_wave"):
        assert n in names


def test_library_exports_every_declared_symbol():
    fp, L = _lib()
    for name in declared_functions():
        assert hasattr(L, name), f"libfftpde.so does not export {name}"


def test_strerror_and_version():
    fp, L = _lib()
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, 99):
        assert isinstance(fp.strerror(code), str) and fp.strerror(code)
    assert "gfx950" in fp.version()


def test_binding_fails_loudly_without_a_device_tensor():
    fp, _ = _lib()
    import torch
    x = torch.zeros(4, 4, dtype=torch.complex64)
    with pytest.raises(ValueError, match="ROCm device"):
        fp.fft2d_forward(x)


# A non-null dummy context: every call below has at least one invalid argument,
# so the library must return EINVAL before it ever reads the context.
_DUMMY = ctypes.create_string_buffer(64)
DUMMY = ctypes.cast(_DUMMY, ctypes.c_void_p).value
BUF = ctypes.create_string_buffer(256)
P = (ctypes.cast(BUF, ctypes.c_void_p).value + 15) // 16 * 16  # 16-byte aligned "field"


# sides must be 7-smooth (powers of two, or the mixed-radix path) in [2, 4096]
@pytest.mark.parametrize("nx,ny,batch,dtype", [
    (11, 4, 1, 0), (4, 13, 1, 0), (22, 77, 1, 1), (4097, 4, 1, 0), (1, 4, 1, 0), (4, 1, 1, 1), (8192, 4, 1, 0),
    (4, 8192, 1, 1), (0, 4, 1, 0), (-4, 4, 1, 0), (4, 4, 0, 0), (4, 4, -1, 1), (4, 4, 1, 4), (4, 4, 1, -1),
    (4, 11, 1, 2), (13, 4, 1, 3),
])
def test_transforms_reject_bad_shape_or_dtype(nx, ny, batch, dtype):
    fp, L = _lib()
    assert L.fft2d_forward(DUMMY, P, P, nx, ny, batch, dtype, None) == fp.EINVAL
    assert L.fft2d_inverse(DUMMY, P, P, nx, ny, batch, dtype, None) == fp.EINVAL
    assert L.solve_poisson(DUMMY, P, P, nx, ny, batch, 1.0, 1.0, dtype, None) == fp.EINVAL


@pytest.mark.parametrize("dtype", [2, 3])
def test_transforms_take_complex_fields_only(dtype):
    """Real dtypes (FFTPDE_R32 / R64) are for the solves; the 2D transforms
    reject them before touching the context."""
    fp, L = _lib()
    assert (fp.R32, fp.R64) == (2, 3)
    assert L.fft2d_forward(DUMMY, P, P, 4, 4, 1, dtype, None) == fp.EINVAL
    assert L.fft2d_inverse(DUMMY, P, P, 4, 4, 1, dtype, None) == fp.EINVAL


def test_real_fields_need_their_own_alignment():
    fp, L = _lib()
    assert L.solve_poisson(DUMMY, P + 2, P, 4, 4, 1, 1.0, 1.0, 2, None) == fp.EINVAL  # FP32 needs 4 B
    assert L.solve_poisson(DUMMY, P + 4, P, 4, 4, 1, 1.0, 1.0, 3, None) == fp.EINVAL  # FP64 needs 8 B


def test_null_context_and_null_or_misaligned_pointers():
    fp, L = _lib()
    assert L.fft2d_forward(None, P, P, 4, 4, 1, 0, None) == fp.EINVAL
    assert L.fft2d_forward(DUMMY, None, P, 4, 4, 1, 0, None) == fp.EINVAL
    assert L.fft2d_forward(DUMMY, P, None, 4, 4, 1, 0, None) == fp.EINVAL
    assert L.fft2d_forward(DUMMY, P + 4, P, 4, 4, 1, 0, None) == fp.EINVAL   # FP32 needs 8 B
    assert L.fft2d_forward(DUMMY, P + 8, P, 4, 4, 1, 1, None) == fp.EINVAL   # FP64 needs 16 B
    assert L.solve_wave(DUMMY, None, None, P, None, 4, 4, 1, 1.0, 1.0, 1.0, 0.5, 0, None) == fp.EINVAL


@pytest.mark.parametrize("lx,ly", [(0.0, 1.0), (1.0, -1.0), (math.inf, 1.0), (1.0, math.nan)])
def test_solves_reject_bad_box(lx, ly):
    fp, L = _lib()
    assert L.solve_poisson(DUMMY, P, P, 4, 4, 1, lx, ly, 0, None) == fp.EINVAL
    assert L.solve_diffusion(DUMMY, P, P, 4, 4, 1, lx, ly, 0.1, 0.1, 0, None) == fp.EINVAL
    assert L.solve_wave(DUMMY, P, None, P, None, 4, 4, 1, lx, ly, 1.0, 0.1, 0, None) == fp.EINVAL


@pytest.mark.parametrize("kappa,t", [(-0.1, 1.0), (0.1, -1e-9), (math.nan, 1.0), (0.1, math.inf)])
def test_diffusion_rejects_bad_coefficients_and_backward_time(kappa, t):
    fp, L = _lib()
    assert L.solve_diffusion(DUMMY, P, P, 4, 4, 1, 1.0, 1.0, kappa, t, 1, None) == fp.EINVAL


def test_wave_rejects_bad_speed_time_and_aliasing():
    fp, L = _lib()
    assert L.solve_wave(DUMMY, P, None, P, None, 4, 4, 1, 1.0, 1.0, -1.0, 0.1, 0, None) == fp.EINVAL
    assert L.solve_wave(DUMMY, P, None, P, None, 4, 4, 1, 1.0, 1.0, 1.0, math.nan, 0, None) == fp.EINVAL
    # the velocity output may not alias the displacement
    Q = P + 64
    assert L.solve_wave(DUMMY, P, None, Q, Q, 4, 4, 1, 1.0, 1.0, 1.0, 0.1, 0, None) == fp.EINVAL
    assert L.solve_wave(DUMMY, P, Q, Q, None, 4, 4, 1, 1.0, 1.0, 1.0, 0.1, 0, None) == fp.EINVAL


def test_create_without_a_gpu_fails_cleanly():
    fp, L = _lib()
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p(123)
    rc = L.fftpde_create(ctypes.byref(h), 0)
    assert rc != fp.OK and h.value is None
    assert L.fftpde_destroy(None) == fp.OK


def test_evolve_rejects_bad_arguments():
    fp, L = _lib()
    h = ctypes.c_void_p(7)
    # diffusion with a velocity field, unknown kind, bad sizes, negative coefficient
    assert L.fftpde_evolve_create(DUMMY, fp.DIFFUSION, P, P, 4, 4, 1, 1.0, 1.0, 0.1, 0, None, ctypes.byref(h)) == fp.EINVAL
    assert h.value is None
    assert L.fftpde_evolve_create(DUMMY, 7, P, None, 4, 4, 1, 1.0, 1.0, 0.1, 0, None, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_evolve_create(DUMMY, fp.WAVE, P, None, 6, 4, 1, 1.0, 1.0, 0.1, 0, None, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_evolve_create(DUMMY, fp.WAVE, P, None, 4, 4, 1, 1.0, 1.0, -1.0, 0, None, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_evolve_create(None, fp.WAVE, P, None, 4, 4, 1, 1.0, 1.0, 1.0, 0, None, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_evolve_step(None, 1, 0.1, None, None, None, None) == fp.EINVAL
    assert L.fftpde_evolve_destroy(None) == fp.OK


def _jobs(*specs):
    """fftpde_job array from (op, nx, ny, lx, ly, coef, t, in, out) tuples."""
    import paper_2412_12308_amd as fp
    arr = (fp.FftpdeJob * len(specs))()
    for k, s in enumerate(specs):
        arr[k] = fp.FftpdeJob(*s)
    return arr


# Fake device addresses: batch planning checks every job (shape, box,
# coefficients, alignment, overlaps) before touching the context or device.
A = 1 << 32
FIELD = 64 * 64 * 8  # a 64x64 FP32 field


@pytest.mark.parametrize("job", [
    (3, 64, 64, 1.0, 1.0, 0.0, 0.0, A, A + FIELD),          # unknown operator
    (0, 8, 64, 1.0, 1.0, 0.0, 0.0, A, A + FIELD),           # side below 16
    (0, 64, 8192, 1.0, 1.0, 0.0, 0.0, A, A + (1 << 24)),    # side above 4096
    (0, 48, 64, 1.0, 1.0, 0.0, 0.0, A, A + FIELD),          # not a power of two
    (0, 64, 64, 0.0, 1.0, 0.0, 0.0, A, A + FIELD),          # empty box
    (1, 64, 64, 1.0, 1.0, -0.1, 0.1, A, A + FIELD),         # negative diffusivity
    (1, 64, 64, 1.0, 1.0, 0.1, -0.1, A, A + FIELD),         # backward heat equation
    (2, 64, 64, 1.0, 1.0, -1.0, 0.1, A, A + FIELD),         # negative wave speed
    (2, 64, 64, 1.0, 1.0, 1.0, math.inf, A, A + FIELD),     # non-finite time
    (0, 64, 64, 1.0, 1.0, 0.0, 0.0, None, A + FIELD),       # null input
    (0, 64, 64, 1.0, 1.0, 0.0, 0.0, A + 4, A + FIELD),      # misaligned input
    (0, 64, 64, 1.0, 1.0, 0.0, 0.0, A, A + FIELD // 2),     # in and out partly overlap
])
def test_batch_rejects_bad_jobs(job):
    fp, L = _lib()
    h = ctypes.c_void_p(9)
    good = (0, 64, 64, 1.0, 1.0, 0.0, 0.0, A + 8 * FIELD, A + 9 * FIELD)
    assert L.fftpde_batch_create(DUMMY, _jobs(good, job), 2, fp.C64, ctypes.byref(h)) == fp.EINVAL
    assert h.value is None


def test_batch_rejects_overlapping_outputs_and_bad_arguments():
    fp, L = _lib()
    h = ctypes.c_void_p()
    j1 = (0, 64, 64, 1.0, 1.0, 0.0, 0.0, A, A + 4 * FIELD)
    j2 = (1, 64, 64, 1.0, 1.0, 0.1, 0.1, A + FIELD, A + 4 * FIELD + FIELD // 2)   # outputs overlap
    j3 = (0, 64, 64, 1.0, 1.0, 0.0, 0.0, A + 4 * FIELD, A + 6 * FIELD)           # reads j1's output
    assert L.fftpde_batch_create(DUMMY, _jobs(j1, j2), 2, fp.C64, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_batch_create(DUMMY, _jobs(j1, j3), 2, fp.C64, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_batch_create(None, _jobs(j1), 1, fp.C64, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_batch_create(DUMMY, _jobs(j1), 0, fp.C64, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_batch_create(DUMMY, _jobs(j1), 1, 2, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_batch_create(DUMMY, _jobs(j1), 1, fp.C64, None) == fp.EINVAL
    # FP64 needs 16-byte alignment
    j4 = (0, 64, 64, 1.0, 1.0, 0.0, 0.0, A + 8, A + 8 * FIELD)
    assert L.fftpde_batch_create(DUMMY, _jobs(j4), 1, fp.C128, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_batch_run(None, 1, None) == fp.EINVAL
    assert L.fftpde_batch_status(None, None) == fp.EINVAL
    assert L.fftpde_batch_info(None, None, None, None) == fp.EINVAL
    assert L.fftpde_batch_destroy(None) == fp.OK


def test_job_struct_layout_matches_the_header():
    """ctypes' fftpde_job must have the C layout (int, int, int, 4 doubles,
    2 pointers, natural alignment)."""
    import paper_2412_12308_amd as fp
    J = fp.FftpdeJob
    assert J.lx.offset == 16 and J.t.offset == 40 and J.inp.offset == 48 and J.out.offset == 56
    assert ctypes.sizeof(J) == 64


def test_server_rejects_bad_arguments():
    fp, L = _lib()
    h = ctypes.c_void_p(5)
    assert L.fftpde_server_create(None, 1 << 20, 4, 2, ctypes.byref(h)) == fp.EINVAL and h.value is None
    assert L.fftpde_server_create(DUMMY, 1 << 20, 0, 2, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_server_create(DUMMY, 1 << 20, 4, 9, ctypes.byref(h)) == fp.EINVAL
    assert L.fftpde_server_create(DUMMY, 16, 4, 2, ctypes.byref(h)) == fp.EINVAL
    cb = fp.HOST_EXEC(lambda *a: 0)
    assert L.fftpde_server_create_host(1 << 40, 4, cb, None, ctypes.byref(h)) == fp.EINVAL  # host pool <= 1 GiB
    assert L.fftpde_server_create_host(1 << 20, 0, cb, None, ctypes.byref(h)) == fp.EINVAL
    r = fp.FftpdeResult()
    st = fp.FftpdeStats()
    rid = ctypes.c_ulonglong()
    req = fp.FftpdeRequest()
    assert L.fftpde_server_submit(None, ctypes.byref(req), ctypes.byref(rid)) == fp.EINVAL
    assert L.fftpde_server_poll(None, 1, ctypes.byref(r)) == fp.EINVAL
    assert L.fftpde_server_wait(None, 1, 0.0, ctypes.byref(r)) == fp.EINVAL
    assert L.fftpde_server_cancel(None, 1) == fp.EINVAL
    assert L.fftpde_server_release(None, 1) == fp.EINVAL
    assert L.fftpde_server_copy_out(None, 1, P, None) == fp.EINVAL
    assert L.fftpde_server_stats(None, 0, ctypes.byref(st)) == fp.EINVAL
    assert L.fftpde_server_destroy(None) == fp.OK


def test_request_structs_match_the_header():
    import paper_2412_12308_amd as fp
    R = fp.FftpdeRequest
    assert (R.lx.offset, R.steps.offset, R.inp.offset, R.deadline.offset, R.flags.offset) == (16, 48, 56, 88, 96)
    assert R.stream.offset == 104 and ctypes.sizeof(R) == 112 and ctypes.sizeof(fp.FftpdeResult) == 48
    assert ctypes.sizeof(fp.FftpdeStats) == 14 * 8 + 5 * 8


def test_plan_tiled_rejects_bad_block_sizes():
    fp, L = _lib()
    for bad in (-1, 3, 100, 1 << 17):
        assert L.fftpde_plan_tiled(DUMMY, bad) == fp.EINVAL
    assert L.fftpde_plan_tiled(None, 128) == fp.EINVAL


def test_plan_chunk_rejects_negative_sizes():
    fp, L = _lib()
    assert L.fftpde_plan_chunk(DUMMY, -1) == fp.EINVAL
    assert L.fftpde_plan_chunk(None, 1 << 20) == fp.EINVAL


def test_source_solves_reject_bad_arguments():
    fp, L = _lib()
    # bad shape, bad box, backward diffusion, negative speed, v == u
    assert L.solve_diffusion_source(DUMMY, P, P, P, 3, 4, 1, 1.0, 1.0, 0.1, 0.5, 0, None) == fp.EINVAL
    assert L.solve_diffusion_source(DUMMY, P, P, P, 4, 4, 1, 0.0, 1.0, 0.1, 0.5, 0, None) == fp.EINVAL
    assert L.solve_diffusion_source(DUMMY, P, P, P, 4, 4, 1, 1.0, 1.0, 0.1, -0.5, 0, None) == fp.EINVAL
    assert L.solve_diffusion_source(DUMMY, P, None, P, 4, 4, 1, 1.0, 1.0, 0.1, 0.5, 0, None) == fp.EINVAL
    assert L.solve_wave_source(DUMMY, P, None, P, P, None, 4, 4, 1, 1.0, 1.0, -1.0, 0.5, 0, None) == fp.EINVAL
    assert L.solve_wave_source(DUMMY, P, None, None, P, None, 4, 4, 1, 1.0, 1.0, 1.0, 0.5, 0, None) == fp.EINVAL
    assert L.solve_wave_source(DUMMY, P, None, P, P, P, 4, 4, 1, 1.0, 1.0, 1.0, 0.5, 0, None) == fp.EINVAL
    assert L.solve_wave_source(None, P, None, P, P, None, 4, 4, 1, 1.0, 1.0, 1.0, 0.5, 0, None) == fp.EINVAL
    assert L.solve_wave_source(DUMMY, P, None, P, P, None, 4, 4, 1, 1.0, 1.0, 1.0, 0.5, 5, None) == fp.EINVAL


def test_wave_rk4_rejects_bad_arguments():
    fp, L = _lib()
    ok = fp.FftpdeOrbitSource(1.0, 0.1, 1.0, 5.0, 10.0, 0.0, 0.0)
    bad_sigma = fp.FftpdeOrbitSource(1.0, 0.0, 1.0, 5.0, 10.0, 0.0, 0.0)
    bad_nan = fp.FftpdeOrbitSource(math.nan, 0.1, 1.0, 5.0, 10.0, 0.0, 0.0)
    args = lambda src, steps=4, dt=0.01, c=1.0, v=None, dtype=0: (  # noqa: E731
        DUMMY, src, P, None, P, v, 4, 4, 1, -2.0, -2.0, 4.0, 4.0, c, 0.0, dt, steps, dtype, None)
    assert ctypes.sizeof(fp.FftpdeOrbitSource) == 7 * 8
    assert L.fftpde_wave_rk4(*args(None)) == fp.EINVAL
    assert L.fftpde_wave_rk4(*args(ctypes.byref(bad_sigma))) == fp.EINVAL
    assert L.fftpde_wave_rk4(*args(ctypes.byref(bad_nan))) == fp.EINVAL
    assert L.fftpde_wave_rk4(*args(ctypes.byref(ok), steps=-1)) == fp.EINVAL
    assert L.fftpde_wave_rk4(*args(ctypes.byref(ok), dt=math.inf)) == fp.EINVAL
    assert L.fftpde_wave_rk4(*args(ctypes.byref(ok), c=-1.0)) == fp.EINVAL
    assert L.fftpde_wave_rk4(*args(ctypes.byref(ok), v=P)) == fp.EINVAL
    assert L.fftpde_wave_rk4(*args(ctypes.byref(ok), dtype=2)) == fp.EINVAL   # complex only


@pytest.mark.parametrize("nx,ny,nz", [(3, 4, 4), (4, 4, 1), (4, 4, 8192), (4096, 8192, 2), (4096, 4096, 0)])
def test_3d_entry_points_reject_bad_shapes(nx, ny, nz):
    fp, L = _lib()
    assert L.fft3d_forward(DUMMY, P, P, nx, ny, nz, 1, 0, None) == fp.EINVAL
    assert L.fft3d_inverse(DUMMY, P, P, nx, ny, nz, 1, 1, None) == fp.EINVAL
    assert L.solve_poisson_3d(DUMMY, P, P, nx, ny, nz, 1, 1.0, 1.0, 1.0, 0, None) == fp.EINVAL


def test_3d_solves_reject_bad_coefficients_and_real_dtypes():
    fp, L = _lib()
    assert L.solve_poisson_3d(DUMMY, P, P, 4, 4, 4, 1, 1.0, 1.0, 0.0, 0, None) == fp.EINVAL
    assert L.solve_diffusion_3d(DUMMY, P, P, 4, 4, 4, 1, 1.0, 1.0, 1.0, 0.1, -1.0, 0, None) == fp.EINVAL
    assert L.solve_wave_3d(DUMMY, P, P, 4, 4, 4, 1, 1.0, 1.0, 1.0, -1.0, 0.5, 0, None) == fp.EINVAL
    assert L.fft3d_forward(DUMMY, P, P, 4, 4, 4, 1, 2, None) == fp.EINVAL
    assert L.fft3d_forward(None, P, P, 4, 4, 4, 1, 0, None) == fp.EINVAL


@pytest.mark.parametrize("nx,ny,dtype", [(4, 6, 2), (12, 4, 3)])
def test_complex_transforms_reject_real_dtypes_on_7_smooth_sides(nx, ny, dtype):
    fp, L = _lib()
    assert L.fft2d_forward(DUMMY, P, P, nx, ny, 1, dtype, None) == fp.EINVAL
    assert L.fft2d_inverse(DUMMY, P, P, nx, ny, 1, dtype, None) == fp.EINVAL


def test_sides_that_are_not_powers_of_two_only_reach_the_mixed_radix_entry_points():
    """3D, sources, evolution and the uneven batch stay on powers of two."""
    fp, L = _lib()
    assert L.solve_diffusion_source(DUMMY, P, P, P, 12, 4, 1, 1.0, 1.0, 0.1, 0.5, 0, None) == fp.EINVAL
    assert L.solve_wave_source(DUMMY, P, None, P, P, None, 4, 6, 1, 1.0, 1.0, 1.0, 0.5, 0, None) == fp.EINVAL
    assert L.fft3d_forward(DUMMY, P, P, 6, 4, 4, 1, 0, None) == fp.EINVAL
    h = ctypes.c_void_p()
    assert L.fftpde_evolve_create(DUMMY, fp.WAVE, P, None, 12, 4, 1, 1.0, 1.0, 0.1, 0, None,
                                  ctypes.byref(h)) == fp.EINVAL


def test_half_spectrum_transforms_reject_bad_arguments():
    """fft2d_r2c / fft2d_c2r: real dtypes only, 7-smooth sides, aligned, and
    input and output must not overlap -- all before touching the context."""
    fp, L = _lib()
    big = ctypes.create_string_buffer(1 << 16)
    A = (ctypes.cast(big, ctypes.c_void_p).value + 255) // 256 * 256
    B = A + 8192
    for fn in (L.fft2d_r2c, L.fft2d_c2r):
        for dtype in (0, 1, 4, -1):                          # complex or unknown dtypes
            assert fn(DUMMY, A, B, 8, 8, 1, dtype, None) == fp.EINVAL
        assert fn(DUMMY, A, B, 11, 8, 1, 2, None) == fp.EINVAL  # prime factor 11
        assert fn(DUMMY, A, B, 8, 4097, 1, 3, None) == fp.EINVAL  # side above 4096
        assert fn(DUMMY, A, B, 8, 1, 1, 2, None) == fp.EINVAL   # side below 2
        assert fn(DUMMY, A, B, 8, 8, 0, 3, None) == fp.EINVAL   # empty batch
        assert fn(None, A, B, 8, 8, 1, 2, None) == fp.EINVAL
    # overlapping real field (8x8 floats = 256 B) and half spectrum (8x5 complex64)
    assert L.fft2d_r2c(DUMMY, A, A + 128, 8, 8, 1, 2, None) == fp.EINVAL
    assert L.fft2d_c2r(DUMMY, A + 64, A, 8, 8, 1, 2, None) == fp.EINVAL
    # half spectra are complex: FP64 needs 16-byte alignment
    assert L.fft2d_r2c(DUMMY, A, B + 8, 8, 8, 1, 3, None) == fp.EINVAL
