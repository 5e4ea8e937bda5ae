"""Shared helpers of the GPU parity tests: device transfer, tolerances."""
import math
import sys

import numpy as np

# FP64 GPU results must match the FP64 oracle to this relative L2 error.
TOL_FP64 = 1e-12


def tol_fp32(nx: int, ny: int, transforms: int) -> float:
    """FP32 bound: 2e-6 * log2(max side) per transform; a bare 2D FFT is one
    transform, a solve (forward + inverse) two."""
    return transforms * 2e-6 * math.log2(max(nx, ny))


def rel_err_vs_input(y, ref, input_norm: float) -> float:
    """||y - ref|| / max(||ref||, input_norm): the FP32 bound is per transform,
    and a transform's rounding error scales with the norm of its input.  For
    solves whose symbol has |M| <= 1 (diffusion, wave) a result much smaller
    than the initial data (e.g. cos(w t) near 0) keeps the forward transform's
    error floor, relative to ||u0||."""
    y = np.asarray(y, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    return float(np.linalg.norm(y - ref) / max(np.linalg.norm(ref), input_norm))


def tol(dtype_name: str, nx: int, ny: int, transforms: int) -> float:
    return TOL_FP64 if dtype_name == "c128" else tol_fp32(nx, ny, transforms)


def torch_dtype(name):
    import torch
    return {"c64": torch.complex64, "c128": torch.complex128}[name]


def to_dev(a: np.ndarray, name: str):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(torch_dtype(name))
    return t.to("cuda:0")


def as_oracle_input(a: np.ndarray, name: str) -> np.ndarray:
    """The values the GPU actually sees, in FP64: FP32 inputs are rounded first,
    so the comparison measures the path and not the input rounding."""
    a = np.asarray(a, dtype=np.complex128)
    return a.astype(np.complex64).astype(np.complex128) if name == "c64" else a


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.complex128)


def say(*a):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(*a, flush=True)
    sys.stdout.flush()
