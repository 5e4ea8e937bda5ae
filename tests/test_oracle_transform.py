"""Pins of the oracle's 1D and 2D transforms (CPU only).

Each check uses something other than the oracle itself: the DFT matrix W of
Sec. II.B written out (brute force), hand-derived golden values, closed-form
spectra of single exponentials, the identities stated in Sec. II.B (periodicity,
W^-1 = W^dagger / N, the conjugation form of the iDFT) and Sec. II.C (the
butterfly pair), Parseval, and numpy.fft as an independent library routine.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import golden_path

RNG = np.random.default_rng(12345)


def _rand(shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def _w_matrix(n, sign=-1):
    """The DFT matrix W_{kj} = w^{jk}, w = exp(sign 2 pi i / n) (Sec. II.B)."""
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


def _brute_dft(x, sign=-1):
    """O(N^2) sum written as explicit loops over j for each k."""
    n = len(x)
    out = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        acc = 0j
        for j in range(n):
            acc += x[j] * complex(math.cos(sign * 2 * math.pi * j * k / n),
                                  math.sin(sign * 2 * math.pi * j * k / n))
        out[k] = acc
    return out


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_matches_bruteforce(n, sign):
    x = _rand(n)
    ref = _brute_dft(x, sign)
    got = oracle.fft1d(x, sign)
    assert oracle.rel_l2(got, ref) <= 1e-13
    # and the matrix form P = W p
    assert oracle.rel_l2(got, _w_matrix(n, sign) @ x) <= 1e-13


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 4), (4, 2), (8, 8), (16, 4), (2, 32), (32, 16)])
def test_fft2d_matches_bruteforce(nx, ny):
    """2D DFT P_ab = sum_j sum_k p_jk exp(-2 pi i (aj/nx + bk/ny)), written as
    W_y p W_x^T with p stored [ny][nx]; rectangular shapes catch swapped axes."""
    p = _rand((ny, nx))
    ref = _w_matrix(ny) @ p @ _w_matrix(nx).T
    assert oracle.rel_l2(oracle.fft2d(p), ref) <= 1e-13
    # direct quadruple sum on one shape as a second, loop-level check
    if nx * ny <= 64:
        full = np.zeros((ny, nx), dtype=np.complex128)
        for b in range(ny):
            for a in range(nx):
                s = 0j
                for k in range(ny):
                    for j in range(nx):
                        s += p[k, j] * np.exp(-2j * np.pi * (a * j / nx + b * k / ny))
                full[b, a] = s
        assert oracle.rel_l2(oracle.fft2d(p), full) <= 1e-13


def test_golden_small_dfts():
    with open(golden_path("dft_small.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) >= 5
    for row in rows:
        name, n, xin, xout = [s.strip() for s in row.split("|")]
        parse = lambda s: np.array([complex(float(a), float(b)) for a, b in
                                    (t.split(",") for t in s.split())])
        x, ref = parse(xin), parse(xout)
        assert len(x) == int(n)
        got = oracle.fft1d(x)
        assert np.max(np.abs(got - ref)) <= 1e-13, name


@pytest.mark.parametrize("n", [2, 8, 64, 1024, 4096])
def test_inverse_of_forward_is_identity(n):
    x = _rand(n)
    y = oracle.ifft1d(oracle.fft1d(x))
    assert oracle.rel_l2(y, x) <= 1e-14 * max(1, math.log2(n))


@pytest.mark.parametrize("nx,ny", [(2, 2), (64, 16), (128, 256)])
def test_inverse_of_forward_is_identity_2d(nx, ny):
    x = _rand((ny, nx))
    y = oracle.ifft2d(oracle.fft2d(x))
    assert oracle.rel_l2(y, x) <= 1e-14 * math.log2(nx * ny)


@pytest.mark.parametrize("n", [4, 256, 2048])
def test_parseval(n):
    """sum |p|^2 = sum |P|^2 / N, a consequence of W^-1 = W^dagger / N."""
    x = _rand(n)
    P = oracle.fft1d(x)
    lhs = np.sum(np.abs(x) ** 2)
    rhs = np.sum(np.abs(P) ** 2) / n
    assert abs(lhs - rhs) / lhs <= 1e-13


def test_conjugation_identity():
    """iDFT(P) = DFT(P*)* / N (Sec. II.B)."""
    P = _rand(512)
    a = oracle.ifft1d(P)
    b = np.conj(oracle.fft1d(np.conj(P))) / 512
    assert oracle.rel_l2(a, b) <= 1e-15


@pytest.mark.parametrize("n,m", [(8, 3), (32, 0), (64, 31), (64, 32), (1024, 1000)])
def test_single_exponential_is_a_delta(n, m):
    """p_j = exp(+2 pi i m j / N) has forward spectrum N delta_{k,m}; mode m + N
    samples to the same values (aliasing / periodicity, Sec. II.A-B)."""
    j = np.arange(n)
    x = np.exp(2j * np.pi * m * j / n)
    x_alias = np.exp(2j * np.pi * (m + n) * j / n)
    ref = np.zeros(n, dtype=np.complex128)
    ref[m] = n
    got = oracle.fft1d(x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * n
    assert np.max(np.abs(oracle.fft1d(x_alias) - ref)) <= 1e-9 * n


def test_periodicity_of_the_dft():
    """P_{k+N} = P_k: evaluating the defining sum at k + N reproduces P_k."""
    n = 16
    x = _rand(n)
    P = oracle.fft1d(x)
    j = np.arange(n)
    for k in range(n):
        pk_shift = np.sum(x * np.exp(-2j * np.pi * j * (k + n) / n))
        assert abs(pk_shift - P[k]) <= 1e-12


@pytest.mark.parametrize("n", [16, 512])
def test_butterfly_pair(n):
    """P_k = E_k + w^k O_k and P_{k+N/2} = E_k - w^k O_k (Sec. II.C), with E, O the
    half-length transforms of the even and odd samples, taken by brute force."""
    x = _rand(n)
    P = oracle.fft1d(x)
    E = _w_matrix(n // 2) @ x[0::2]
    O = _w_matrix(n // 2) @ x[1::2]
    k = np.arange(n // 2)
    w = np.exp(-2j * np.pi * k / n)
    assert oracle.rel_l2(P[: n // 2], E + w * O) <= 1e-12
    assert oracle.rel_l2(P[n // 2:], E - w * O) <= 1e-12


def test_linearity():
    x, y = _rand((32, 64)), _rand((32, 64))
    a, b = 0.3 - 1.2j, 2.5
    lhs = oracle.fft2d(a * x + b * y)
    rhs = a * oracle.fft2d(x) + b * oracle.fft2d(y)
    assert oracle.rel_l2(lhs, rhs) <= 1e-14


@pytest.mark.parametrize("nx,ny", [(2048, 2048), (4096, 16), (2, 4096)])
def test_fft2d_matches_numpy(nx, ny):
    """numpy.fft (pocketfft) is an independent implementation of the same sum."""
    x = _rand((ny, nx))
    got = oracle.fft2d(x, threads=oracle.default_threads())
    assert oracle.rel_l2(got, np.fft.fft2(x)) <= 1e-14
    assert oracle.rel_l2(oracle.ifft2d(got, threads=oracle.default_threads()), x) <= 1e-14


def test_threads_do_not_change_results():
    x = _rand((256, 128))
    a = oracle.fft2d(x, threads=1)
    b = oracle.fft2d(x, threads=7)
    assert np.array_equal(a, b)


def test_rejects_empty_lengths_and_bad_signs():
    # any length >= 1 is accepted (lengths that are not powers of two have
    # their own pins); empty axes and exponent signs other than +-1 are not
    with pytest.raises(ValueError):
        oracle.fft1d(np.ones(0))
    with pytest.raises(ValueError):
        oracle.fft2d(np.ones((0, 8)))
    with pytest.raises(ValueError):
        oracle.fft1d(np.ones(8), sign=2)
