"""fftpde -- FFT spectral solvers for periodic 2D PDEs on AMD Instinct MI355X.

A thin ctypes binding over libfftpde.so (C ABI in include/fftpde.h).  Every
step of every transform and solve runs in the library's HIP kernels; this
module only checks tensors, passes device pointers and the current HIP
stream, and turns status codes into exceptions.  PyTorch provides device
memory and streams.  There is no CPU fallback: if the library is missing or
no GPU is present, calls raise.

Tensors are complex64 (FP32 complex) or complex128 (FP64 complex) on a ROCm
device, contiguous, shaped [..., ny, nx] with x contiguous; leading
dimensions form the batch.  The solves also take real float32 / float64
fields (solved two per complex transform, see FFTPDE_R32 in fftpde.h).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
from typing import Optional, Tuple

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfftpde.so")

OK, PENDING = 0, 1
EINVAL, ENOMEM, EDEVICE, EBUDGET, ENOTFOUND, ECANCELED, ETIMEOUT = -1, -2, -3, -4, -5, -6, -7
C64, C128 = 0, 1
R32, R64 = 2, 3
POISSON, DIFFUSION, WAVE = 0, 1, 2


class FftpdeError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {strerror(status)} ({status})"
        if detail:
            msg += f" [{detail}]"
        super().__init__(msg)


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """Load libfftpde.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_2412_12308_amd.build`")
            # PyTorch-ROCm carries its own HIP runtime and makes its symbols
            # global.  Importing torch first makes libfftpde.so bind to that
            # same runtime, so tensors, streams and kernels share one HIP
            # instance (loading the library first would start a second runtime
            # from /opt/rocm that torch cannot share the GPU with).
            import torch  # noqa: F401
            L = ctypes.CDLL(LIB_PATH)
            _declare(L)
            _lib = L
    return _lib


class FftpdeOrbitSource(ctypes.Structure):
    """fftpde_orbit_source: the orbiting Gaussian source of fftpde_wave_rk4."""
    _fields_ = [("amplitude", ctypes.c_double), ("sigma", ctypes.c_double), ("radius", ctypes.c_double),
                ("omega", ctypes.c_double), ("gamma", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double)]


class FftpdeJob(ctypes.Structure):
    """struct fftpde_job of the C ABI."""
    _fields_ = [("op", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("coef", ctypes.c_double),
                ("t", ctypes.c_double), ("inp", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class FftpdeRequest(ctypes.Structure):
    """struct fftpde_request of the C ABI."""
    _fields_ = [("op", ctypes.c_int), ("dtype", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("coef", ctypes.c_double),
                ("dt", ctypes.c_double), ("steps", ctypes.c_longlong), ("inp", ctypes.c_void_p),
                ("v0", ctypes.c_void_p), ("out", ctypes.c_void_p), ("diag", ctypes.c_void_p),
                ("deadline", ctypes.c_double), ("flags", ctypes.c_int), ("stream", ctypes.c_void_p)]


class FftpdeResult(ctypes.Structure):
    """struct fftpde_result of the C ABI."""
    _fields_ = [("status", ctypes.c_int), ("state", ctypes.c_int), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("out", ctypes.c_void_p),
                ("footprint", ctypes.c_longlong)]


class FftpdeStats(ctypes.Structure):
    """struct fftpde_stats of the C ABI."""
    _fields_ = [(n, ctypes.c_longlong) for n in (
        "submitted", "rejected", "admitted", "completed", "failed", "canceled", "timed_out", "queued", "running",
        "hbm_budget", "hbm_in_use", "hbm_high_water", "iterations", "latency_count")] + \
        [(n, ctypes.c_double) for n in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "now")]


HOST_EXEC = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_ulonglong, ctypes.POINTER(FftpdeRequest),
                             ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_int)


def _declare(L):
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.fftpde_create.argtypes = [ctypes.POINTER(vp), i]
    L.fftpde_destroy.argtypes = [vp]
    L.fftpde_strerror.argtypes = [i]
    L.fftpde_strerror.restype = ctypes.c_char_p
    L.fftpde_version.restype = ctypes.c_char_p
    L.fftpde_last_error.restype = ctypes.c_char_p
    L.fft2d_forward.argtypes = [vp, vp, vp, i, i, i, i, vp]
    L.fft2d_r2c.argtypes = [vp, vp, vp, i, i, i, i, vp]
    L.fft2d_c2r.argtypes = [vp, vp, vp, i, i, i, i, vp]
    L.fft2d_inverse.argtypes = [vp, vp, vp, i, i, i, i, vp]
    L.solve_poisson.argtypes = [vp, vp, vp, i, i, i, d, d, i, vp]
    L.solve_diffusion.argtypes = [vp, vp, vp, i, i, i, d, d, d, d, i, vp]
    L.solve_wave.argtypes = [vp, vp, vp, vp, vp, i, i, i, d, d, d, d, i, vp]
    L.solve_wave_noalloc.argtypes = [vp, vp, vp, vp, vp, i, i, i, d, d, d, d, i, vp]
    L.solve_diffusion_source.argtypes = [vp, vp, vp, vp, i, i, i, d, d, d, d, i, vp]
    L.solve_wave_source.argtypes = [vp, vp, vp, vp, vp, vp, i, i, i, d, d, d, d, i, vp]
    L.fft3d_forward.argtypes = [vp, vp, vp, i, i, i, i, i, vp]
    L.fft3d_inverse.argtypes = [vp, vp, vp, i, i, i, i, i, vp]
    L.solve_poisson_3d.argtypes = [vp, vp, vp, i, i, i, i, d, d, d, i, vp]
    L.solve_diffusion_3d.argtypes = [vp, vp, vp, i, i, i, i, d, d, d, d, d, i, vp]
    L.solve_wave_3d.argtypes = [vp, vp, vp, i, i, i, i, d, d, d, d, d, i, vp]
    L.fftpde_wave_rk4.argtypes = [vp, ctypes.POINTER(FftpdeOrbitSource), vp, vp, vp, vp, i, i, i, d, d, d, d, d,
                                  d, d, i, i, vp]
    L.fftpde_profile.argtypes = [vp, i]
    L.fftpde_profile_read.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t,
                                      ctypes.POINTER(ctypes.c_size_t)]
    L.fftpde_plan_variants.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t,
                                       ctypes.POINTER(ctypes.c_size_t)]
    L.fftpde_plan_select.argtypes = [vp, ctypes.c_char_p]
    L.fftpde_plan_small.argtypes = [vp, i]
    L.fftpde_plan_tiled.argtypes = [vp, i]
    L.fftpde_plan_chunk.argtypes = [vp, ctypes.c_longlong]
    L.fftpde_autotune.argtypes = [vp, i, i, i, i, i, i, vp, ctypes.c_char_p, ctypes.c_size_t,
                                  ctypes.POINTER(ctypes.c_size_t)]
    L.fftpde_plan_save.argtypes = [vp, ctypes.c_char_p]
    L.fftpde_plan_load.argtypes = [vp, ctypes.c_char_p]
    L.fftpde_evolve_create.argtypes = [vp, i, vp, vp, i, i, i, d, d, d, i, vp, ctypes.POINTER(vp)]
    L.fftpde_evolve_step.argtypes = [vp, ctypes.c_longlong, d, vp, vp, vp, vp]
    L.fftpde_evolve_destroy.argtypes = [vp]
    L.fftpde_batch_create.argtypes = [vp, ctypes.POINTER(FftpdeJob), i, i, ctypes.POINTER(vp)]
    L.fftpde_batch_run.argtypes = [vp, i, vp]
    L.fftpde_batch_status.argtypes = [vp, vp]
    L.fftpde_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(i),
                                    ctypes.POINTER(d)]
    L.fftpde_batch_plan.argtypes = [vp, i, i, i]
    L.fftpde_batch_tune.argtypes = [vp, i, vp]
    L.fftpde_batch_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.fftpde_batch_destroy.argtypes = [vp]
    ull, ll = ctypes.c_ulonglong, ctypes.c_longlong
    L.fftpde_server_create.argtypes = [vp, ll, i, i, ctypes.POINTER(vp)]
    L.fftpde_server_create_host.argtypes = [ll, i, HOST_EXEC, vp, ctypes.POINTER(vp)]
    L.fftpde_server_submit.argtypes = [vp, ctypes.POINTER(FftpdeRequest), ctypes.POINTER(ull)]
    L.fftpde_server_poll.argtypes = [vp, ull, ctypes.POINTER(FftpdeResult)]
    L.fftpde_server_wait.argtypes = [vp, ull, d, ctypes.POINTER(FftpdeResult)]
    L.fftpde_server_cancel.argtypes = [vp, ull]
    L.fftpde_server_copy_out.argtypes = [vp, ull, vp, vp]
    L.fftpde_server_release.argtypes = [vp, ull]
    L.fftpde_server_stats.argtypes = [vp, i, ctypes.POINTER(FftpdeStats)]
    L.fftpde_server_destroy.argtypes = [vp]
    for f in ("fftpde_server_create", "fftpde_server_create_host", "fftpde_server_submit", "fftpde_server_poll",
              "fftpde_server_wait", "fftpde_server_cancel", "fftpde_server_copy_out", "fftpde_server_release",
              "fftpde_server_stats", "fftpde_server_destroy",
              "fftpde_batch_create", "fftpde_batch_run", "fftpde_batch_status", "fftpde_batch_info",
              "fftpde_batch_plan", "fftpde_batch_tune", "fftpde_batch_describe", "fftpde_batch_destroy", "fftpde_plan_small", "fftpde_plan_tiled", "fftpde_plan_chunk", "fftpde_evolve_create", "fftpde_evolve_step", "fftpde_evolve_destroy", "fftpde_autotune", "fftpde_plan_save", "fftpde_plan_load", "fftpde_plan_variants",
              "fftpde_plan_select", "fftpde_profile", "fftpde_profile_read", "fftpde_create", "fftpde_destroy", "fft2d_forward", "fft2d_inverse", "fft2d_r2c", "fft2d_c2r", "solve_poisson",
              "solve_diffusion", "solve_wave", "solve_wave_noalloc", "solve_diffusion_source", "solve_wave_source", "fftpde_wave_rk4",
              "fft3d_forward", "fft3d_inverse", "solve_poisson_3d", "solve_diffusion_3d", "solve_wave_3d"):
        getattr(L, f).restype = i


def strerror(status: int) -> str:
    try:
        return lib().fftpde_strerror(status).decode()
    except ImportError:
        return f"status {status}"


def version() -> str:
    return lib().fftpde_version().decode()


def _check(rc: int, where: str):
    if rc != OK:
        detail = ""
        if rc == EDEVICE:
            detail = lib().fftpde_last_error().decode(errors="replace")
        raise FftpdeError(rc, where, detail)


# ---------------------------------------------------------------------------
# contexts (one per device, created on first use)
# ---------------------------------------------------------------------------
_ctx = {}


def context(device: int) -> int:
    h = _ctx.get(device)
    if h is None:
        p = ctypes.c_void_p()
        _check(lib().fftpde_create(ctypes.byref(p), int(device)), "fftpde_create")
        h = _ctx[device] = p.value
    return h


@atexit.register
def _destroy_contexts():
    if _lib is None:
        return
    for dev, h in list(_ctx.items()):
        _lib.fftpde_destroy(h)
    _ctx.clear()


def profile(device: int, enable: bool):
    """Time every kernel launched on `device` from now on with HIP events."""
    _check(lib().fftpde_profile(context(device), 1 if enable else 0), "fftpde_profile")


def profile_read(device: int):
    """Per-kernel launches, total milliseconds and algorithmic bytes since profiling began."""
    import json
    need = ctypes.c_size_t(0)
    _check(lib().fftpde_profile_read(context(device), None, 0, ctypes.byref(need)), "fftpde_profile_read")
    buf = ctypes.create_string_buffer(max(2, need.value))
    _check(lib().fftpde_profile_read(context(device), buf, len(buf), None), "fftpde_profile_read")
    return json.loads(buf.value.decode())


def plan_variants(device: int = 0):
    """Every compiled kernel variant, with the one in use per slot marked active."""
    import json
    need = ctypes.c_size_t(0)
    _check(lib().fftpde_plan_variants(context(device), None, 0, ctypes.byref(need)), "fftpde_plan_variants")
    buf = ctypes.create_string_buffer(max(2, need.value))
    _check(lib().fftpde_plan_variants(context(device), buf, len(buf), None), "fftpde_plan_variants")
    return json.loads(buf.value.decode())


def plan_small(enable: bool, device: int = 0):
    """Use (default) or bypass the single-pass small-grid kernels."""
    _check(lib().fftpde_plan_small(context(device), 1 if enable else 0), "fftpde_plan_small")


def plan_chunk(nbytes: int = 256 << 20, device: int = 0):
    """Run batches of 3-pass solves in chunks of about `nbytes` of field data
    (fftpde_plan_chunk; 0 = whole batch).  Results are bit-identical."""
    _check(lib().fftpde_plan_chunk(context(device), int(nbytes)), "fftpde_plan_chunk")


def plan_tiled(block_bytes: int = 1024, device: int = 0):
    """Layout of the spectrum between the passes of 3-pass solves
    (fftpde_plan_tiled): column blocks of block_bytes per row (default 1024),
    0 row-major.  Results are bit-identical for every block size."""
    _check(lib().fftpde_plan_tiled(context(device), int(block_bytes)), "fftpde_plan_tiled")


def plan_select(name: Optional[str], device: int = 0):
    """Use the named kernel variant for its slot (None restores all defaults)."""
    _check(lib().fftpde_plan_select(context(device), None if name is None else name.encode()),
           "fftpde_plan_select")


def autotune(nx: int, ny: int, batch: int = 1, dtype: str = "c64", op: int = POISSON, reps: int = 5,
             device: int = 0):
    """Time every kernel variant for this solve shape and keep the fastest (see
    fftpde_autotune); returns the library's JSON report as a dict."""
    import json
    torch = _torch()
    code = {"c64": C64, "c128": C128}[dtype]
    stream = torch.cuda.current_stream(device).cuda_stream
    need = ctypes.c_size_t(0)
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().fftpde_autotune(context(device), nx, ny, batch, code, op, reps, stream, buf, len(buf),
                                 ctypes.byref(need)), "fftpde_autotune")
    return json.loads(buf.value.decode())


def plan_save(path: str, device: int = 0):
    _check(lib().fftpde_plan_save(context(device), os.fsencode(path)), "fftpde_plan_save")


def plan_load(path: str, device: int = 0):
    _check(lib().fftpde_plan_load(context(device), os.fsencode(path)), "fftpde_plan_load")


# ---------------------------------------------------------------------------
# tensor marshalling
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _dtype_code(t, real_ok: bool = False) -> int:
    torch = _torch()
    if t.dtype == torch.complex64:
        return C64
    if t.dtype == torch.complex128:
        return C128
    if real_ok and t.dtype == torch.float32:
        return R32
    if real_ok and t.dtype == torch.float64:
        return R64
    raise TypeError(f"expected complex64 or complex128{' (or float32 / float64)' if real_ok else ''}, "
                    f"got {t.dtype}")


def _field(t, name: str, real_ok: bool = False):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a ROCm device (got {t.device}); there is no CPU path")
    if t.dim() < 2:
        raise ValueError(f"{name} must have shape [..., ny, nx]")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    ny, nx = t.shape[-2], t.shape[-1]
    batch = t.numel() // (nx * ny) if nx * ny else 0
    return nx, ny, batch, _dtype_code(t, real_ok)


def _like(x, out, name="out"):
    torch = _torch()
    if out is None:
        return torch.empty_like(x)
    if out.shape != x.shape or out.dtype != x.dtype or out.device != x.device:
        raise ValueError(f"{name} must match the input's shape, dtype and device")
    if not out.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return out


def _stream(t) -> int:
    return _torch().cuda.current_stream(t.device).cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ---------------------------------------------------------------------------
# API (names as in the C ABI)
# ---------------------------------------------------------------------------
def fft2d_forward(x, out=None):
    """Unnormalised forward 2D FFT, exponent exp(-2 pi i (a j/nx + b k/ny))."""
    nx, ny, batch, dt = _field(x, "x")
    out = _like(x, out)
    _check(lib().fft2d_forward(context(x.device.index), _ptr(x), _ptr(out), nx, ny, batch, dt,
                               _stream(x)), "fft2d_forward")
    return out


def fft2d_inverse(x, out=None):
    """Inverse 2D FFT, exponent exp(+2 pi i ...) times 1/(nx ny)."""
    nx, ny, batch, dt = _field(x, "x")
    out = _like(x, out)
    _check(lib().fft2d_inverse(context(x.device.index), _ptr(x), _ptr(out), nx, ny, batch, dt,
                               _stream(x)), "fft2d_inverse")
    return out


def fft2d_r2c(x, out=None):
    """Half spectrum [..., ny, nx/2 + 1] (complex) of real fields x [..., ny, nx]
    (float32 -> complex64, float64 -> complex128): columns 0..nx/2 of the
    unnormalised forward 2D FFT."""
    torch = _torch()
    nx, ny, batch, dt = _field(x, "x", True)
    if dt not in (R32, R64):
        raise ValueError("fft2d_r2c takes real fields (float32 / float64)")
    shape = tuple(x.shape[:-1]) + (nx // 2 + 1,)
    cdt = torch.complex64 if dt == R32 else torch.complex128
    if out is None:
        out = torch.empty(shape, dtype=cdt, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != cdt or not out.is_contiguous() or out.device != x.device:
        raise ValueError(f"out must be a contiguous {cdt} tensor of shape {shape}")
    _check(lib().fft2d_r2c(context(x.device.index), _ptr(x), _ptr(out), nx, ny, batch, dt, _stream(x)),
           "fft2d_r2c")
    return out


def fft2d_c2r(X, nx: int, out=None):
    """Real fields [..., ny, nx] whose half spectrum is the Hermitian part of
    X [..., ny, nx/2 + 1] (complex64 -> float32, complex128 -> float64),
    inverse 2D FFT times 1/(nx ny)."""
    torch = _torch()
    h, ny, batch, cdt = _field(X, "X")
    if h != nx // 2 + 1:
        raise ValueError(f"X has {h} columns; a half spectrum of width nx = {nx} has {nx // 2 + 1}")
    dt = R32 if cdt == C64 else R64
    shape = tuple(X.shape[:-1]) + (nx,)
    rdt = torch.float32 if dt == R32 else torch.float64
    if out is None:
        out = torch.empty(shape, dtype=rdt, device=X.device)
    elif tuple(out.shape) != shape or out.dtype != rdt or not out.is_contiguous() or out.device != X.device:
        raise ValueError(f"out must be a contiguous {rdt} tensor of shape {shape}")
    _check(lib().fft2d_c2r(context(X.device.index), _ptr(X), _ptr(out), nx, ny, batch, dt, _stream(X)),
           "fft2d_c2r")
    return out


def solve_poisson(s, lx: float = 1.0, ly: float = 1.0, out=None):
    """Zero-mean u with lap(u) = s - mean(s) on a periodic lx-by-ly box."""
    nx, ny, batch, dt = _field(s, "s", True)
    out = _like(s, out)
    _check(lib().solve_poisson(context(s.device.index), _ptr(s), _ptr(out), nx, ny, batch,
                               float(lx), float(ly), dt, _stream(s)), "solve_poisson")
    return out


def solve_diffusion(u0, kappa: float, t: float, lx: float = 1.0, ly: float = 1.0, out=None):
    """u(t) for u_t = kappa lap(u), u(0) = u0, periodic box, t >= 0."""
    nx, ny, batch, dt = _field(u0, "u0", True)
    out = _like(u0, out)
    _check(lib().solve_diffusion(context(u0.device.index), _ptr(u0), _ptr(out), nx, ny, batch,
                                 float(lx), float(ly), float(kappa), float(t), dt, _stream(u0)),
           "solve_diffusion")
    return out


def solve_wave(u0, v0=None, c: float = 1.0, t: float = 0.0, lx: float = 1.0, ly: float = 1.0,
               out=None, v_out=None, want_v: bool = False) -> Tuple:
    """(u(t), u_t(t) or None) for u_tt = c^2 lap(u), u(0) = u0, u_t(0) = v0 (None => 0)."""
    nx, ny, batch, dt = _field(u0, "u0", True)
    if v0 is not None:
        if _field(v0, "v0", True) != (nx, ny, batch, dt) or v0.device != u0.device:
            raise ValueError("v0 must match u0")
    out = _like(u0, out)
    if want_v or v_out is not None:
        v_out = _like(u0, v_out, "v_out")
    _check(lib().solve_wave(context(u0.device.index), _ptr(u0), _ptr(v0), _ptr(out), _ptr(v_out),
                            nx, ny, batch, float(lx), float(ly), float(c), float(t), dt,
                            _stream(u0)), "solve_wave")
    return out, v_out


def solve_wave_noalloc(u0, v0=None, c: float = 1.0, t: float = 0.0, lx: float = 1.0, ly: float = 1.0,
                       out=None, v_out=None, want_v: bool = False) -> Tuple:
    """solve_wave through the entry point that allocates no device memory (its
    scratch is a fixed array of the library; complex fields, power-of-two
    sides).  Pass `out` (and `v_out`) to keep the call free of allocations on
    the Python side too."""
    nx, ny, batch, dt = _field(u0, "u0")
    if v0 is not None:
        if _field(v0, "v0") != (nx, ny, batch, dt) or v0.device != u0.device:
            raise ValueError("v0 must match u0")
    out = _like(u0, out)
    if want_v or v_out is not None:
        v_out = _like(u0, v_out, "v_out")
    _check(lib().solve_wave_noalloc(context(u0.device.index), _ptr(u0), _ptr(v0), _ptr(out), _ptr(v_out),
                                    nx, ny, batch, float(lx), float(ly), float(c), float(t), dt,
                                    _stream(u0)), "solve_wave_noalloc")
    return out, v_out


def solve_diffusion_source(f, s, kappa: float, t: float, lx: float = 1.0, ly: float = 1.0, out=None):
    """u(t) for u_t = kappa lap(u) + s, u(0) = f, with s constant in time."""
    nx, ny, batch, dt = _field(f, "f", True)
    if _field(s, "s", True) != (nx, ny, batch, dt) or s.device != f.device:
        raise ValueError("s must match f")
    out = _like(f, out)
    _check(lib().solve_diffusion_source(context(f.device.index), _ptr(f), _ptr(s), _ptr(out), nx, ny, batch,
                                        float(lx), float(ly), float(kappa), float(t), dt, _stream(f)),
           "solve_diffusion_source")
    return out


def solve_wave_source(f, g, s, c: float = 1.0, t: float = 0.0, lx: float = 1.0, ly: float = 1.0,
                      out=None, v_out=None, want_v: bool = False) -> Tuple:
    """(u(t), u_t(t) or None) for u_tt = c^2 lap(u) + s, u(0) = f, u_t(0) = g (None => 0),
    s constant in time."""
    nx, ny, batch, dt = _field(f, "f", True)
    for name, x in (("g", g), ("s", s)):
        if x is not None and (_field(x, name, True) != (nx, ny, batch, dt) or x.device != f.device):
            raise ValueError(f"{name} must match f")
    if s is None:
        raise ValueError("s is required (use solve_wave without a source)")
    out = _like(f, out)
    if want_v or v_out is not None:
        v_out = _like(f, v_out, "v_out")
    _check(lib().solve_wave_source(context(f.device.index), _ptr(f), _ptr(g), _ptr(s), _ptr(out), _ptr(v_out),
                                   nx, ny, batch, float(lx), float(ly), float(c), float(t), dt, _stream(f)),
           "solve_wave_source")
    return out, v_out


def wave_rk4(f, g=None, *, amplitude: float, sigma: float, radius: float, omega: float, gamma: float,
             cx: float = 0.0, cy: float = 0.0, x0: float = 0.0, y0: float = 0.0, lx: float = 1.0,
             ly: float = 1.0, c: float = 1.0, t0: float = 0.0, dt: float, steps: int, out=None, v_out=None,
             want_v: bool = False) -> Tuple:
    """(u, u_t) at t0 + steps*dt for u_tt = c^2 lap(u) + s(t) with the orbiting
    Gaussian source s = A exp(-d^2/sigma^2) cos(gamma t) (centre cx + r cos(Omega t),
    cy + r sin(Omega t)), RK4 in Fourier space (fftpde_wave_rk4)."""
    nx, ny, batch, dt_code = _field(f, "f")
    if g is not None and (_field(g, "g") != (nx, ny, batch, dt_code) or g.device != f.device):
        raise ValueError("g must match f")
    out = _like(f, out)
    if want_v or v_out is not None:
        v_out = _like(f, v_out, "v_out")
    src = FftpdeOrbitSource(float(amplitude), float(sigma), float(radius), float(omega), float(gamma),
                            float(cx), float(cy))
    _check(lib().fftpde_wave_rk4(context(f.device.index), ctypes.byref(src), _ptr(f), _ptr(g), _ptr(out),
                                 _ptr(v_out), nx, ny, batch, float(x0), float(y0), float(lx), float(ly), float(c),
                                 float(t0), float(dt), int(steps), dt_code, _stream(f)), "fftpde_wave_rk4")
    return out, v_out


def _field3d(t, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a torch.Tensor on a ROCm device (there is no CPU path)")
    if t.dim() < 3:
        raise ValueError(f"{name} must have shape [..., nz, ny, nx]")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    nz, ny, nx = t.shape[-3], t.shape[-2], t.shape[-1]
    pts = nx * ny * nz
    return nx, ny, nz, (t.numel() // pts if pts else 0), _dtype_code(t)


def fft3d_forward(x, out=None):
    """Unnormalised forward 3D FFT of [..., nz, ny, nx] fields."""
    nx, ny, nz, batch, dt = _field3d(x, "x")
    out = _like(x, out)
    _check(lib().fft3d_forward(context(x.device.index), _ptr(x), _ptr(out), nx, ny, nz, batch, dt, _stream(x)),
           "fft3d_forward")
    return out


def fft3d_inverse(x, out=None):
    """Inverse 3D FFT, exponent exp(+...) times 1/(nx ny nz)."""
    nx, ny, nz, batch, dt = _field3d(x, "x")
    out = _like(x, out)
    _check(lib().fft3d_inverse(context(x.device.index), _ptr(x), _ptr(out), nx, ny, nz, batch, dt, _stream(x)),
           "fft3d_inverse")
    return out


def solve_poisson_3d(s, lx: float = 1.0, ly: float = 1.0, lz: float = 1.0, out=None):
    """Zero-mean u with lap(u) = s - mean(s) on a periodic 3D box."""
    nx, ny, nz, batch, dt = _field3d(s, "s")
    out = _like(s, out)
    _check(lib().solve_poisson_3d(context(s.device.index), _ptr(s), _ptr(out), nx, ny, nz, batch, float(lx),
                                  float(ly), float(lz), dt, _stream(s)), "solve_poisson_3d")
    return out


def solve_diffusion_3d(u0, kappa: float, t: float, lx: float = 1.0, ly: float = 1.0, lz: float = 1.0, out=None):
    """u(t) for u_t = kappa lap(u) on a periodic 3D box."""
    nx, ny, nz, batch, dt = _field3d(u0, "u0")
    out = _like(u0, out)
    _check(lib().solve_diffusion_3d(context(u0.device.index), _ptr(u0), _ptr(out), nx, ny, nz, batch, float(lx),
                                    float(ly), float(lz), float(kappa), float(t), dt, _stream(u0)),
           "solve_diffusion_3d")
    return out


def solve_wave_3d(u0, c: float = 1.0, t: float = 0.0, lx: float = 1.0, ly: float = 1.0, lz: float = 1.0, out=None):
    """u(t) for u_tt = c^2 lap(u), u(0) = u0, u_t(0) = 0, on a periodic 3D box."""
    nx, ny, nz, batch, dt = _field3d(u0, "u0")
    out = _like(u0, out)
    _check(lib().solve_wave_3d(context(u0.device.index), _ptr(u0), _ptr(out), nx, ny, nz, batch, float(lx),
                               float(ly), float(lz), float(c), float(t), dt, _stream(u0)), "solve_wave_3d")
    return out


class Evolution:
    """Time evolution of the diffusion or wave equation with the forward spectra
    of the initial data resident on the device (fftpde_evolve_*).

    step(n, dt) evaluates the exact solution at t = n * dt."""

    def __init__(self, kind: int, u0, v0=None, coef: float = 1.0, lx: float = 1.0, ly: float = 1.0):
        nx, ny, batch, dt = _field(u0, "u0")
        if v0 is not None and (_field(v0, "v0") != (nx, ny, batch, dt) or v0.device != u0.device):
            raise ValueError("v0 must match u0")
        self.shape, self.dtype, self.device = tuple(u0.shape), u0.dtype, u0.device
        self.kind, self.coef, self.lx, self.ly = kind, coef, lx, ly
        self.batch = batch
        h = ctypes.c_void_p()
        _check(lib().fftpde_evolve_create(context(u0.device.index), int(kind), _ptr(u0), _ptr(v0), nx, ny, batch,
                                          float(lx), float(ly), float(coef), dt, _stream(u0), ctypes.byref(h)),
               "fftpde_evolve_create")
        self._h = h.value

    def step(self, n: int, dt: float, out=None, v_out=None, want_u: bool = True, want_v: bool = False,
             diag: bool = False):
        """(u(t), u_t(t) or None, diag or None) at t = n dt; diag is a float64
        device tensor [batch, 3] = (mean re, mean im, energy)."""
        torch = _torch()
        if self._h is None:
            raise RuntimeError("evolution destroyed")
        if want_u or out is not None:
            out = out if out is not None else torch.empty(self.shape, dtype=self.dtype, device=self.device)
        if want_v or v_out is not None:
            v_out = v_out if v_out is not None else torch.empty(self.shape, dtype=self.dtype, device=self.device)
        d = torch.empty((self.batch, 3), dtype=torch.float64, device=self.device) if diag else None
        _check(lib().fftpde_evolve_step(self._h, int(n), float(dt), _ptr(out), _ptr(v_out), _ptr(d),
                                        torch.cuda.current_stream(self.device).cuda_stream), "fftpde_evolve_step")
        return out, v_out, d

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.fftpde_evolve_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many independent solves of uneven power-of-two shapes run by one
    persistent kernel (fftpde_batch_*), replayed from a captured HIP graph.

    jobs: sequence of dicts with keys op (POISSON / DIFFUSION / WAVE), inp (a
    [ny, nx] complex device tensor), and optionally out (default: a new
    tensor; inp itself for in place), lx, ly (default 1.0), coef (kappa or c)
    and t.  The tensors are kept alive by the batch; run() recomputes every
    out from the current contents of every inp."""

    def __init__(self, jobs):
        torch = _torch()
        jobs = list(jobs)
        if not jobs:
            raise ValueError("a batch needs at least one job")
        first = jobs[0]["inp"]
        self.device, self.dtype = first.device, first.dtype
        self.inputs, self.outputs = [], []
        arr = (FftpdeJob * len(jobs))()
        dt = None
        for k, j in enumerate(jobs):
            inp = j["inp"]
            nx, ny, b, code = _field(inp, f"jobs[{k}].inp")
            if b != 1 or inp.dim() != 2:
                raise ValueError("each job is one [ny, nx] field")
            if inp.device != self.device or inp.dtype != self.dtype:
                raise ValueError("all jobs must share one device and dtype")
            out = j.get("out")
            if out is None:
                out = torch.empty_like(inp)
            elif tuple(out.shape) != tuple(inp.shape) or out.dtype != inp.dtype or not out.is_contiguous():
                raise ValueError(f"jobs[{k}].out must match jobs[{k}].inp")
            dt = code
            self.inputs.append(inp)
            self.outputs.append(out)
            arr[k] = FftpdeJob(int(j["op"]), nx, ny, float(j.get("lx", 1.0)), float(j.get("ly", 1.0)),
                               float(j.get("coef", 0.0)), float(j.get("t", 0.0)), inp.data_ptr(),
                               out.data_ptr())
        # the plan's copies are synchronous: order them after pending work
        torch.cuda.current_stream(self.device).synchronize()
        h = ctypes.c_void_p()
        _check(lib().fftpde_batch_create(context(self.device.index), arr, len(jobs), dt, ctypes.byref(h)),
               "fftpde_batch_create")
        self._h = h.value
        items, grid, nbytes = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_double()
        _check(lib().fftpde_batch_info(self._h, ctypes.byref(items), ctypes.byref(grid), ctypes.byref(nbytes)),
               "fftpde_batch_info")
        self.items, self.grid, self.bytes = items.value, grid.value, nbytes.value

    def run(self, use_graph: bool = True):
        """Enqueue one run on the current stream; returns the output tensors."""
        if self._h is None:
            raise RuntimeError("batch destroyed")
        s = _torch().cuda.current_stream(self.device).cuda_stream
        _check(lib().fftpde_batch_run(self._h, 1 if use_graph else 0, s), "fftpde_batch_run")
        return self.outputs

    def status(self):
        """Wait for the current stream; raise if a dependency wait timed out."""
        s = _torch().cuda.current_stream(self.device).cuda_stream
        _check(lib().fftpde_batch_status(self._h, s), "fftpde_batch_status")

    def set_plan(self, kind: int, logn: int, plan: int):
        """Radix plan of one class (kind 0 rows / 1 columns of log2 length
        logn): 0 = radix up to 8, 1 = up to 16 (FP32) / 4 (FP64)."""
        _torch().cuda.current_stream(self.device).synchronize()
        _check(lib().fftpde_batch_plan(self._h, kind, logn, plan), "fftpde_batch_plan")

    def tune(self, reps: int = 10):
        """Time each class's other plan on the current inputs and keep the
        faster within tolerance (fftpde_batch_tune); overwrites the outputs.
        Returns describe()."""
        s = _torch().cuda.current_stream(self.device).cuda_stream
        _check(lib().fftpde_batch_tune(self._h, reps, s), "fftpde_batch_tune")
        return self.describe()

    def describe(self):
        """Plans, single-pass items and the last tuning, as a dict."""
        import json
        need = ctypes.c_size_t(0)
        _check(lib().fftpde_batch_describe(self._h, None, 0, ctypes.byref(need)), "fftpde_batch_describe")
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().fftpde_batch_describe(self._h, buf, len(buf), ctypes.byref(need)), "fftpde_batch_describe")
        return json.loads(buf.value.decode())

    def close(self):
        if self._h is not None and _lib is not None:
            _torch().cuda.current_stream(self.device).synchronize()
            _lib.fftpde_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


AUTORELEASE = 1
STATE_QUEUED, STATE_RUNNING, STATE_ENDED = 0, 1, 2


class Server:
    """Request server (fftpde_server_*): continuous batching of Poisson solves
    and diffusion / wave evolutions on one GPU, admission by an HBM budget.

    Server(budget_bytes, max_slots, streams, device) runs on the GPU;
    Server.host(budget_bytes, max_slots, exec_fn) runs the same scheduler with
    a host backend that calls exec_fn(id, request, out_address, phase, n0, nt)
    for every piece of work (phase 0 start, 1 steps n0..n0+nt-1, 2 final
    field) -- for testing the scheduler without a GPU."""

    def __init__(self, budget: int, max_slots: int = 16, streams: int = 4, device: int = 0, _host=None):
        self._h = None
        self._keep = {}
        h = ctypes.c_void_p()
        if _host is None:
            self.device = device
            _check(lib().fftpde_server_create(context(device), int(budget), int(max_slots), int(streams),
                                              ctypes.byref(h)), "fftpde_server_create")
        else:
            self.device = None
            self._cb = _host
            _check(lib().fftpde_server_create_host(int(budget), int(max_slots), _host, None, ctypes.byref(h)),
                   "fftpde_server_create_host")
        self._h = h.value

    @classmethod
    def host(cls, budget: int, max_slots: int, exec_fn):
        def tramp(user, rid, req, out, phase, n0, nt):
            try:
                rc = exec_fn(int(rid), req.contents, out, int(phase), int(n0), int(nt))
                return int(rc or 0)
            except Exception:  # a failing callback fails its request
                import traceback
                traceback.print_exc()
                return -3
        return cls(budget, max_slots, _host=HOST_EXEC(tramp))

    def submit_raw(self, req: FftpdeRequest, keep=()) -> int:
        rid = ctypes.c_ulonglong()
        _check(lib().fftpde_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)), "fftpde_server_submit")
        if keep:
            self._keep[rid.value] = keep
        return rid.value

    def submit(self, op: int, inp, *, out=None, v0=None, diag=None, steps: int = 1, dt: float = 0.0,
               coef: float = 0.0, lx: float = 1.0, ly: float = 1.0, deadline: float = 0.0,
               autorelease: bool = False) -> int:
        """Submit a request on device tensors ([ny, nx] complex inp, optional
        out / v0 of the same shape, optional float64 diag of 3*steps)."""
        nx, ny, b, code = _field(inp, "inp")
        if b != 1 or inp.dim() != 2:
            raise ValueError("a request is one [ny, nx] field")
        for t, name in ((out, "out"), (v0, "v0")):
            if t is not None and (tuple(t.shape) != tuple(inp.shape) or t.dtype != inp.dtype or not t.is_contiguous()):
                raise ValueError(f"{name} must match inp")
        if diag is not None and (diag.dtype != _torch().float64 or diag.numel() < 3 * steps or not diag.is_contiguous()):
            raise ValueError("diag must be a contiguous float64 tensor of 3*steps values")
        req = FftpdeRequest(int(op), code, nx, ny, float(lx), float(ly), float(coef), float(dt), int(steps),
                            inp.data_ptr(), _ptr(v0), _ptr(out), _ptr(diag), float(deadline),
                            AUTORELEASE if autorelease else 0, _stream(inp))
        return self.submit_raw(req, keep=(inp, out, v0, diag))

    def _result(self, rc, res, rid):
        if rc == ENOTFOUND:
            raise FftpdeError(rc, "fftpde_server_poll", f"unknown request {rid}")
        return dict(status=res.status, state=res.state, t_submit=res.t_submit, t_admit=res.t_admit,
                    t_done=res.t_done, out=res.out, footprint=res.footprint)

    def poll(self, rid: int) -> dict:
        res = FftpdeResult()
        return self._result(lib().fftpde_server_poll(self._h, rid, ctypes.byref(res)), res, rid)

    def wait(self, rid: int, timeout: float = -1.0) -> dict:
        res = FftpdeResult()
        return self._result(lib().fftpde_server_wait(self._h, rid, float(timeout), ctypes.byref(res)), res, rid)

    def cancel(self, rid: int):
        _check(lib().fftpde_server_cancel(self._h, rid), "fftpde_server_cancel")

    def copy_out(self, rid: int, dst):
        """Copy an ended request's output into dst (a device tensor, or for the
        host backend a numpy array)."""
        if hasattr(dst, "data_ptr"):
            s = _torch().cuda.current_stream(dst.device).cuda_stream
            _check(lib().fftpde_server_copy_out(self._h, rid, dst.data_ptr(), s), "fftpde_server_copy_out")
        else:
            _check(lib().fftpde_server_copy_out(self._h, rid, dst.ctypes.data, None), "fftpde_server_copy_out")
        return dst

    def release(self, rid: int):
        _check(lib().fftpde_server_release(self._h, rid), "fftpde_server_release")
        self._keep.pop(rid, None)

    def stats(self, reset: bool = False) -> dict:
        st = FftpdeStats()
        _check(lib().fftpde_server_stats(self._h, 1 if reset else 0, ctypes.byref(st)), "fftpde_server_stats")
        return {n: getattr(st, n) for n, _ in FftpdeStats._fields_}

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.fftpde_server_destroy(self._h)
        self._h = None
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
