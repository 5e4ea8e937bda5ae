"""solve_wave_noalloc: the solve that allocates no device memory.  Its
results equal solve_wave's bit for bit (same kernels, same plan; the
spectrum between the passes sits in the library's fixed array instead of the
context workspace), on two calls in a row with the second smaller, with and
without a velocity; sizes whose spectrum exceeds the array are rejected
before any work; and a call on a fresh stream leaves the device's free
memory unchanged."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import as_oracle_input, rel_err_vs_input, say, to_dev, to_host

pytestmark = pytest.mark.gpu
EINVAL = -1


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


def _pair(fp, torch, shape, dtype, seed, c, t, velocity=False):
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    u0 = torch.randn(shape, dtype=dtype, device="cuda:0", generator=g)
    v0 = torch.randn(shape, dtype=dtype, device="cuda:0", generator=g) if velocity else None
    ref_u, ref_v = fp.solve_wave(u0, v0, c=c, t=t, lx=1.0, ly=2.0, want_v=velocity)
    out = torch.full_like(u0, float("nan"))
    v_out = torch.full_like(u0, float("nan")) if velocity else None
    got_u, got_v = fp.solve_wave_noalloc(u0, v0, c=c, t=t, lx=1.0, ly=2.0, out=out, v_out=v_out)
    torch.cuda.synchronize()
    return u0, v0, ref_u, ref_v, got_u, got_v


@pytest.mark.parametrize("dtype_name", ["c64", "c128"])
def test_two_calls_in_a_row_equal_solve_wave(fp, dtype_name):
    import torch
    dtype = {"c64": torch.complex64, "c128": torch.complex128}[dtype_name]
    for shape, seed in (((3, 2048, 2048), 11), ((2, 256, 512), 12)):
        say(f"noalloc {dtype_name} {shape}")
        _, _, ref_u, _, got_u, _ = _pair(fp, torch, shape, dtype, seed, 1.0, 0.37)
        assert torch.equal(got_u, ref_u), shape


def test_velocity_in_and_out_equal_solve_wave(fp):
    import torch
    for shape, seed in (((2, 2048, 2048), 21), ((1, 1024, 512), 22)):
        say(f"noalloc velocity {shape}")
        _, _, ref_u, ref_v, got_u, got_v = _pair(fp, torch, shape, torch.complex64, seed, 0.8, 0.21, velocity=True)
        assert torch.equal(got_u, ref_u) and torch.equal(got_v, ref_v), shape


def test_small_case_against_the_oracle(fp):
    import torch
    x = W.random_field((128, 256), seed=31)
    g = W.random_field((128, 256), seed=32)
    u0, v0 = to_dev(x, "c128"), to_dev(g, "c128")
    say("noalloc vs oracle 256x128 c128")
    u, v = fp.solve_wave_noalloc(u0, v0, c=1.3, t=0.6, lx=1.0, ly=2.0, want_v=True)
    ref_u, ref_v = oracle.solve_wave(as_oracle_input(x, "c128"), as_oracle_input(g, "c128"), 1.0, 2.0, 1.3, 0.6,
                                     want_v=True)
    assert oracle.rel_l2(to_host(u), ref_u) <= 1e-12
    assert oracle.rel_l2(to_host(v), ref_v) <= 1e-12


def test_oversized_and_unsupported_requests_are_rejected(fp):
    import torch
    big = torch.zeros((4096, 4096), dtype=torch.complex64, device="cuda:0")   # spectrum 128 MiB > 64 MiB
    out = torch.empty_like(big)
    with pytest.raises(fp.FftpdeError) as e:
        fp.solve_wave_noalloc(big, None, c=1.0, t=0.1, out=out)
    assert e.value.status == EINVAL
    odd = torch.zeros((96, 96), dtype=torch.complex64, device="cuda:0")     # not a power of two
    with pytest.raises(fp.FftpdeError):
        fp.solve_wave_noalloc(odd, None, c=1.0, t=0.1)
    # real fields, straight through the C ABI (the binding takes complex only)
    real = torch.zeros((64, 64), dtype=torch.float32, device="cuda:0")
    real_out = torch.empty_like(real)
    rc = fp.lib().solve_wave_noalloc(fp.context(0), real.data_ptr(), None, real_out.data_ptr(), None, 64, 64, 1,
                                     1.0, 1.0, 1.0, 0.1, fp.R32, torch.cuda.current_stream().cuda_stream)
    assert rc == EINVAL


def test_no_device_memory_is_allocated(fp):
    """On a stream the context has not used (and that has run one kernel, so
    the runtime's own set-up of its queue is done), solve_wave grows a new
    workspace (hipMalloc); solve_wave_noalloc leaves the device's free memory
    unchanged."""
    import torch
    x = torch.randn((4, 2048, 2048), dtype=torch.complex64, device="cuda:0")
    out = torch.empty_like(x)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out.zero_()   # the runtime's own first-use set-up of the stream's queue
        s.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        fp.solve_wave_noalloc(x, None, c=1.0, t=0.2, out=out)
        s.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        fp.solve_wave(x, None, c=1.0, t=0.2, out=out)
        s.synchronize()
        free2 = torch.cuda.mem_get_info()[0]
    say(f"free memory: {free0 >> 20} MiB, after noalloc {free1 >> 20} MiB, after solve_wave {free2 >> 20} MiB")
    assert free1 == free0
