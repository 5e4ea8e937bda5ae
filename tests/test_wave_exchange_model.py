"""Host model of the in-wave exchanges of the 2048-point FP32 fused column
pass (ColMapWave in fft_engine.hpp), for one column of a tile: 128 threads
(8 wavefronts of 16 lanes of this column) with 16 registers each.

The model runs the Stockham stages of the forward plan 16 16 8 and the
reversed plan 8 16 16 with the map's butterfly layouts, an LDS exchange where
the kernel uses LDS, and the kernel's three lane-bit / register-bit swaps
(the semantics of DPP row_ror:8, v_permlane16_swap and v_permlane32_swap)
where it stays in the wavefront, and checks both against numpy's FFT.  It
also checks the mirror pairing the symbol evaluation relies on.  No GPU."""
import numpy as np

N, TH = 2048, 128


def residue(t):
    w, kb = t >> 4, t & 1          # t: thread of this column; lane bit 2 of the kernel = bit 0 here
    return (16 - w if w else 8) if kb else w


def butterfly(layout, t, q):
    h = (t >> 1) & 7               # lane bits 3-5 of the kernel
    if layout == 0:
        return t + TH * q          # ColMap: the HBM-facing stages
    k = residue(t)
    if layout == 1:
        return 16 * h + k
    if layout == 2:
        return 16 * (h + 8 * q) + k
    return 8 * k + h


def run_stage(x, R, ns, layout):
    for t in range(TH):
        for q in range(16 // R):
            j = butterfly(layout, t, q)
            v = x[t, q * R:(q + 1) * R] * np.exp(-2j * np.pi * np.arange(R) * (j % ns) / (ns * R))
            x[t, q * R:(q + 1) * R] = np.fft.fft(v)


def lds_exchange(x, R, ns, lay, R2, lay2):
    y = np.zeros(N, complex)
    for t in range(TH):
        for q in range(16 // R):
            j = butterfly(lay, t, q)
            k = j % ns
            for r in range(R):
                y[(j - k) * R + k + r * ns] = x[t, q * R + r]
    for t in range(TH):
        for q in range(16 // R2):
            j = butterfly(lay2, t, q)
            for r in range(R2):
                x[t, q * R2 + r] = y[j + r * (N // R2)]


def swap_bits(x, lane_bit, reg_bit):
    """A lane with the lane bit clear keeps register rb = 0 and receives its
    partner's rb = 0 register in place of rb = 1; a lane with the bit set
    receives its partner's rb = 1 register in place of rb = 0."""
    b = lane_bit - 2
    out = x.copy()
    for t in range(TH):
        p, hi = t ^ (1 << b), (t >> b) & 1
        for r in range(16):
            if (r >> reg_bit) & 1:
                continue
            lo_r, hi_r = r, r | (1 << reg_bit)
            if hi:
                out[t, lo_r] = x[p, hi_r]
            else:
                out[t, hi_r] = x[p, lo_r]
    return out


def in_wave_exchange(x):
    return swap_bits(swap_bits(swap_bits(x, 3, 0), 4, 1), 5, 2)


def test_layouts_are_bijections():
    for layout, R in ((1, 16), (2, 8), (3, 16)):
        js = sorted(butterfly(layout, t, q) for t in range(TH) for q in range(16 // R))
        assert js == list(range(N // R))


def test_swaps_stay_within_wavefronts():
    for b in (3, 4, 5):
        for t in range(TH):
            assert (t ^ (1 << (b - 2))) >> 4 == t >> 4


def test_forward_plan_matches_fft():
    u = np.random.default_rng(5).standard_normal(N) + 1j * np.random.default_rng(6).standard_normal(N)
    x = np.array([[u[t + r * 128] for r in range(16)] for t in range(TH)])
    run_stage(x, 16, 1, 0)
    lds_exchange(x, 16, 1, 0, 16, 1)
    run_stage(x, 16, 16, 1)
    x = in_wave_exchange(x)
    run_stage(x, 8, 256, 2)
    got = np.zeros(N, complex)
    for t in range(TH):
        for q in range(2):
            j = butterfly(2, t, q)
            got[j + 256 * np.arange(8)] = x[t, q * 8:(q + 1) * 8]
    ref = np.fft.fft(u)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_reversed_plan_matches_fft():
    u = np.random.default_rng(7).standard_normal(N) + 1j * np.random.default_rng(8).standard_normal(N)
    x = np.zeros((TH, 16), complex)
    for t in range(TH):
        for q in range(2):
            x[t, q * 8:(q + 1) * 8] = u[butterfly(2, t, q) + 256 * np.arange(8)]
    run_stage(x, 8, 1, 2)
    x = in_wave_exchange(x)
    run_stage(x, 16, 8, 3)
    lds_exchange(x, 16, 8, 3, 16, 0)
    run_stage(x, 16, 128, 0)
    got = np.zeros(N, complex)
    for t in range(TH):
        got[t + 128 * np.arange(16)] = x[t]
    ref = np.fft.fft(u)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_mirror_partner_lanes():
    """In wavefronts 1-7 the row of register 8 + t (slot 1) of lane l is the
    mirror (2048 - n) of the row of register 7 - t (slot 0) of lane l ^ 60,
    i.e. this column's thread t ^ 15; wavefront 0 pairs differently."""
    for t in range(16, TH):
        p = t ^ 15
        for r in range(8):
            n1 = butterfly(2, t, 1) + 256 * r
            n0 = butterfly(2, p, 0) + 256 * (7 - r)
            assert (n0 + n1) % N == 0
    assert any((butterfly(2, t, 1) + butterfly(2, t ^ 15, 0) + 256 * 7) % N for t in range(16))
