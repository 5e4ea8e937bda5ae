#!/usr/bin/env python3
"""Throughput of the fused FFT spectral solve on one MI355X.

Workload: the 2D wave equation u_tt = c^2 lap(u) on the periodic unit square
at 2048 x 2048 (c = 1, dt = 1e-4, u0 = Gaussian pulse of width 0.02 at a
seeded centre plus the standing mode sin(6 pi x) sin(10 pi y), v0 = 0).
One step solves a batch of B independent such problems (seeded centres)
at t_n = n dt: forward 2D FFT -> propagator cos(c|k| t_n) -> inverse 2D FFT,
FP32 butterflies with FP64 twiddle generation and FP64 phase.  The batch
keeps the working set (2 x 512 MiB at B = 16) well above the 256 MiB
Infinity Cache, so the passes run from HBM.  The same workload in FP64
(B = 8) is reported beside it.

The same problems stored as real fields (the initial data are real) are
timed beside them: two real fields per complex transform, half the bytes per
solve (`real_fields`; 2B FP32 / B FP64 fields).

Beside it: the batched uneven launch (1024 Poisson solves, sides drawn from
32..1024, one persistent kernel replayed from a HIP graph, FP32 with its
radix plans tuned by fftpde_batch_tune and FP64, and the FP64 solves one at
a time), and the request server under an open
loop of Poisson arrivals at 2000 requests/s (50 % Poisson, 30 % diffusion
with 10..200 steps, 20 % wave with 10..500 steps, sides log-uniform in
2^6..2^12, 64 GiB budget, per-step diagnostics from resident spectra):
p50 / p99 latency over 10 s after 1 s of warm-up.

Prints one JSON line.  Inputs are resident in HBM before timing starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "2D spectral solves/s + HBM GB/s at N=2048, FP32 vs FP64; serving p50/p99 ms"
HBM_PEAK_GBS = 8000.0
N_SIDE = 2048
DT = 1e-4
C_SPEED = 1.0
BURN_IN = 64  # untimed steps between the cold window and the timed one (run_leg)


# Counter traffic comes from the committed rocprofv3 summary, valid only for
# the kernel sources it was measured on.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "wave2d_2048_hbm_traffic.md")
KERNEL_SOURCES = ("fft_engine.hpp", "kernels.hpp", "rows_f32.hip", "rows_f64.hip", "cols_f32_nf1.hip",
                  "cols_f64_nf1.hip", "cols_f32_nf2.hip", "cols_f64_nf2.hip")


def kernel_sources_hash() -> str:
    """sha256 over the row / column kernel sources (name and contents)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(ROOT, "paper_2412_12308_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(kernel: str):
    """HBM bytes per launch of `kernel` (a plan variant name) from the counter
    summary; None if the summary is missing, lacks the kernel, or was taken on
    other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"kernel sources sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != kernel_sources_hash():
        return None
    for line in text.splitlines():
        if line.startswith(f"| `{kernel}` |"):
            try:
                return float(line.strip().strip("|").split("|")[-1])
            except ValueError:
                return None
    return None


def make_inputs(n: int, batch: int, seed: int = 3):
    import numpy as np

    import workloads as W
    out = np.empty((batch, n, n), dtype=np.complex128)
    for i in range(batch):
        s = seed if i == 0 else W._child_seed(seed, i)
        out[i] = W.wave_ic(n, seed=s).field
    return out


def run_leg(fp, torch, host_fields, dtype_name: str, steps: int, warmup: int):
    """Time `steps` batched solves; returns a dict of measurements."""
    dev = torch.device("cuda:0")
    tdt = {"c64": torch.complex64, "c128": torch.complex128, "r32": torch.float32, "r64": torch.float64}[dtype_name]
    real = dtype_name in ("r32", "r64")
    u0 = torch.from_numpy(host_fields.real.copy() if real else host_fields).to(tdt).to(dev)
    out = torch.empty_like(u0)
    batch, ny, nx = u0.shape
    bpp = {"c64": 8, "c128": 16, "r32": 4, "r64": 8}[dtype_name]
    stream = torch.cuda.current_stream(dev)

    def window():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for s in range(steps):
            fp.solve_wave(u0, None, C_SPEED, (s + 1) * DT, 1.0, 1.0, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), time.perf_counter() - t0

    for w in range(warmup):
        fp.solve_wave(u0, None, C_SPEED, (w + 1) * DT, 1.0, 1.0, out=out)
    # The first ~40 ms of back-to-back solves after the GPU idled run up to
    # 15 % slower than the steady state (clock and power management settling;
    # measured step by step).  The K steps right after the W warm-up steps are
    # reported as `cold`; then BURN_IN more untimed steps, and the K timed
    # steps behind `value` run in the steady state of a long job.
    cold_ms, _ = window()
    for b in range(BURN_IN):
        fp.solve_wave(u0, None, C_SPEED, (b + 1) * DT, 1.0, 1.0, out=out)
    ms, wall = window()
    # Per-kernel durations: the same steps again with an event pair around
    # every launch (on the launch stream).  The events add a few microseconds
    # per launch, so this pass is kept out of the throughput above.
    fp.profile(0, True)
    for s in range(steps):
        fp.solve_wave(u0, None, C_SPEED, (s + 1) * DT, 1.0, 1.0, out=out)
    torch.cuda.synchronize()
    kstats = fp.profile_read(0)
    fp.profile(0, False)
    solves = batch * steps
    alg_bytes = 6.0 * bpp * nx * ny * solves
    # dominant kernel: the one with the largest share of the timed region
    dom = max(kstats, key=lambda k: k["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return {
        "batch": batch, "steps": steps, "ms_total": ms, "wall_s": wall,
        "solves_per_s": solves / (ms * 1e-3),
        "ms_per_step": ms / steps,
        "cold_ms_per_step": cold_ms / steps,
        "eff_gbs": alg_bytes / (ms * 1e-3) / 1e9,
        "kernels": [{**k, "avg_us": 1e3 * k["total_ms"] / k["launches"],
                     "gbs": (k["bytes"] / k["launches"]) / (k["total_ms"] / k["launches"] * 1e-3) / 1e9}
                    for k in kstats],
        "dominant": {"kernel": dom["kernel"], "avg_us": 1e3 * avg_ms,
                     "bytes_per_launch": bytes_per_launch, "achieved_gbs": achieved},
        "last_out": out, "last_t": steps * DT,
    }


def source_leg(fp, torch, host_fields, steps: int, warmup: int, check: bool):
    """The wave problem with an initial velocity and a source constant in time
    (u_tt = c^2 lap(u) + s): f = the pulse fields, g and s seeded random
    fields, FP32 complex.  Algorithmic bytes per solve: three fields read and
    three spectra written by the row passes, three read and one written by the
    column pass, one read and one written by the inverse row pass: 12 b P."""
    import numpy as np

    import workloads as W
    dev = torch.device("cuda:0")
    batch, ny, nx = host_fields.shape
    f = torch.from_numpy(host_fields).to(torch.complex64).to(dev)
    g = torch.from_numpy(W.random_field((batch, ny, nx), seed=71)).to(torch.complex64).to(dev)
    s = torch.from_numpy(W.random_field((batch, ny, nx), seed=72)).to(torch.complex64).to(dev)
    out = torch.empty_like(f)
    for w in range(warmup):
        fp.solve_wave_source(f, g, s, C_SPEED, (w + 1) * DT, 1.0, 1.0, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        fp.solve_wave_source(f, g, s, C_SPEED, (k + 1) * DT, 1.0, 1.0, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    alg = 12.0 * 8 * nx * ny * batch * steps
    res = {"workload": "wave2d_2048 with u_t(0) and a source constant in time, FP32 complex",
           "batch": batch, "solves_per_s": round(batch * steps / (ms * 1e-3), 2),
           "ms_per_step": round(ms / steps, 4), "alg_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
           "alg_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if check:
        import oracle
        t = steps * DT
        x = lambda a: a.cpu().numpy()[0].astype(np.complex128)  # noqa: E731
        ref, _ = oracle.solve_wave_source(x(f), x(g), x(s), 1.0, 1.0, C_SPEED, t, threads=oracle.default_threads())
        res["err_vs_oracle"] = oracle.rel_l2(out.cpu().numpy()[0].astype(np.complex128), ref)
    return res


def leg_3d(fp, torch, steps: int, warmup: int, check: bool):
    """3D wave solves, 256^3 FP32 complex, batch 4 (512 MiB): five passes,
    algorithmic bytes 10 b P per solve."""
    import numpy as np

    import workloads as W
    n, batch = 256, 4
    host = W.random_field((batch, n, n, n), seed=81).astype(np.complex64)
    u0 = torch.from_numpy(host).to("cuda:0")
    del host
    out = torch.empty_like(u0)
    for w in range(warmup):
        fp.solve_wave_3d(u0, C_SPEED, (w + 1) * DT, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        fp.solve_wave_3d(u0, C_SPEED, (k + 1) * DT, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    alg = 10.0 * 8 * n ** 3 * batch * steps
    res = {"workload": "wave3d_256^3_periodic_unit_cube, FP32 complex, random initial data", "batch": batch,
           "solves_per_s": round(batch * steps / (ms * 1e-3), 2), "ms_per_step": round(ms / steps, 4),
           "alg_gbs": round(alg / (ms * 1e-3) / 1e9, 1), "alg_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if check:
        import oracle
        x = u0[0].cpu().numpy().astype(np.complex128)
        ref = oracle.solve3d(x, 1.0, 1.0, 1.0, 2, C_SPEED, steps * DT, threads=oracle.default_threads())
        res["err_vs_oracle"] = oracle.rel_l2(out[0].cpu().numpy().astype(np.complex128), ref)
    del u0, out
    return res


def mixed_leg(fp, torch, steps: int, warmup: int, check: bool, n: int = 1536, batch: int = 8):
    """The wave problem on a side that is not a power of two (1536 = 3 x 2^9:
    a radix-3 step around the 512-point register engine), FP32 complex,
    batch 8: three passes, algorithmic bytes 6 b P per solve; per-pass times
    from a second, profiled run."""
    import numpy as np

    dev = torch.device("cuda:0")
    host = make_inputs(n, batch, seed=5)
    u0 = torch.from_numpy(host).to(torch.complex64).to(dev)
    out = torch.empty_like(u0)
    for w in range(warmup):
        fp.solve_wave(u0, None, C_SPEED, (w + 1) * DT, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        fp.solve_wave(u0, None, C_SPEED, (k + 1) * DT, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    alg = 6.0 * 8 * n * n * batch * steps
    res = {"workload": f"wave2d_{n}x{n}_periodic_unit_square (3 x 512: radix-3 step + 512-point engine), FP32 complex",
           "batch": batch, "solves_per_s": round(batch * steps / (ms * 1e-3), 2),
           "ms_per_step": round(ms / steps, 4), "alg_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
           "alg_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    fp.profile(0, True)
    for k in range(min(steps, 5)):
        fp.solve_wave(u0, None, C_SPEED, (k + 1) * DT, out=out)
    torch.cuda.synchronize()
    prof = fp.profile_read(0)
    fp.profile(0, False)
    res["kernels"] = [{"kernel": k["kernel"], "launches": k["launches"],
                       "avg_us": round(k["total_ms"] / k["launches"] * 1e3, 2),
                       "gbs": round(k["bytes"] / (k["total_ms"] * 1e-3) / 1e9, 1)} for k in prof]
    if check:
        t = min(steps, 5) * DT
        res["err_vs_oracle"] = oracle_check(out[0], host[0], "c64", t)
        res["err_tol"] = 2 * 2e-6 * math.log2(n)
    del u0, out
    return res


def half_spectrum_leg(fp, torch, host_fields, steps: int, warmup: int, check: bool):
    """fft2d_r2c and fft2d_c2r of real FP32 fields (the real parts of the
    pulse fields).  Algorithmic bytes of one transform: the real fields
    (4 B per point) and the half spectra (8 B per point of [ny][nx/2+1])."""
    import numpy as np

    batch, ny, nx = host_fields.shape
    x = torch.from_numpy(np.ascontiguousarray(host_fields.real)).to(torch.float32).to("cuda:0")
    X = fp.fft2d_r2c(x)
    y = torch.empty_like(x)
    alg = (4.0 * nx * ny + 8.0 * (nx // 2 + 1) * ny) * batch
    res = {"workload": f"half spectra of {batch} real {nx}x{ny} FP32 fields", "batch": batch}
    for name, fn in (("r2c", lambda: fp.fft2d_r2c(x, out=X)), ("c2r", lambda: fp.fft2d_c2r(X, nx, out=y))):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"ms": round(ms, 4), "fields_per_s": round(batch / (ms * 1e-3), 1),
                     "alg_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
                     "alg_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        # per-kernel split (HIP events around each launch, outside the timed loop)
        fp.profile(0, True)
        for _ in range(min(steps, 5)):
            fn()
        torch.cuda.synchronize()
        prof = fp.profile_read(0)
        fp.profile(0, False)
        res[name]["kernels"] = [{"kernel": k["kernel"], "launches": k["launches"],
                                 "avg_us": round(k["total_ms"] / k["launches"] * 1e3, 2),
                                 "gbs": round(k["bytes"] / (k["total_ms"] * 1e-3) / 1e9, 1)} for k in prof]
    if check:
        import oracle
        x0 = x[0].cpu().numpy().astype(np.float64)
        ref = oracle.rfft2d(x0, threads=oracle.default_threads())
        res["r2c_err_vs_oracle"] = oracle.rel_l2(X[0].cpu().numpy().astype(np.complex128), ref)
        res["round_trip_err"] = float(np.linalg.norm(y[0].cpu().numpy() - x0) / np.linalg.norm(x0))
    del x, X, y
    return res


def oracle_check(out_dev, host_field, dtype_name, t):
    """Relative L2 error of one GPU result against the FP64 oracle."""
    import numpy as np

    import oracle
    x = host_field.real.astype(np.complex128) if dtype_name in ("r32", "r64") else host_field
    x = x.astype(np.complex64).astype(np.complex128) if dtype_name in ("c64", "r32") else x
    ref, _ = oracle.solve_wave(x, None, 1.0, 1.0, C_SPEED, t, threads=oracle.default_threads())
    got = out_dev.cpu().numpy().astype(np.complex128)
    return oracle.rel_l2(got, ref)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(host_field, seconds: float = 10.0):
    """The FP64 oracle (recursive radix-2) on the same workload: as many
    single-field solves as fit in about `seconds` on all host threads, then
    a shorter sample on one thread."""
    import oracle

    def timed(threads, budget):
        t0 = time.perf_counter()
        n = 0
        while True:
            oracle.solve_wave(host_field, None, 1.0, 1.0, C_SPEED, (n + 1) * DT, threads=threads)
            n += 1
            if time.perf_counter() - t0 >= budget:
                break
        return n, time.perf_counter() - t0

    threads = oracle.default_threads()
    n, el = timed(threads, 0.7 * seconds)
    n1, el1 = timed(1, 0.3 * seconds)
    return {"value": n / el, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} FP64 wave solves of one 2048x2048 field (fwd 2D FFT, propagator, "
                      f"inverse 2D FFT), {el:.1f} s on {threads} threads",
            "single_thread": {"value": n1 / el1, "unit": "solves/s", "cores": 1,
                              "sample": f"{n1} of the same solves, {el1:.1f} s on 1 thread"},
            "cpu_model": cpu_model()}


def batch_leg(fp, torch, reps: int, warmup: int, check: bool):
    """1024 uneven Poisson solves per launch (graph replay), FP32 and FP64;
    the FP64 solves also one at a time through the single-field path."""
    import numpy as np

    import oracle
    import workloads as W
    shapes = W.batch_shapes()
    srcs = W.batch_sources(shapes)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    out = {"workload": "poisson_uneven_batch_1024", "jobs": len(srcs),
           "sides": "nx, ny independently uniform in {32..1024}"}
    for name, tdt in (("fp32", torch.complex64), ("fp64", torch.complex128)):
        ins = [torch.from_numpy(ms.field).to(tdt).cuda() for ms in srcs]
        b = fp.Batch([dict(op=0, inp=x, lx=ms.lx, ly=ms.ly) for x, ms in zip(ins, srcs)])

        def timed():
            for _ in range(warmup):
                b.run()
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record()
            for _ in range(reps):
                b.run()
            e1.record()
            torch.cuda.synchronize()
            b.status()
            return e0.elapsed_time(e1) / reps

        ms_default = timed()
        ms = ms_default
        d = b.describe()
        if name == "fp32":  # FP64 batches have one radix plan
            d = b.tune(reps=10)
            ms = timed()
        leg = {"ms_per_launch": round(ms, 4), "solves_per_s": round(len(srcs) / (ms * 1e-3), 1),
               "alg_gbs": round(b.bytes / (ms * 1e-3) / 1e9, 1),
               "alg_frac": round(b.bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "default_plan_ms_per_launch": round(ms_default, 4),
               "plans": {f"{c['kind']}{1 << c['logn']}": c["max_radix"] for c in d["classes"]},
               "single_pass": d["single_pass"],
               "items": b.items, "workgroups": b.grid, "alg_bytes": b.bytes}
        if check:
            errs = []
            for i in (int(np.argmax([m.nx * m.ny for m in srcs])), 0, 511):
                x = srcs[i].field
                x = x.astype(np.complex64).astype(np.complex128) if name == "fp32" else x
                ref = oracle.solve_poisson(x, srcs[i].lx, srcs[i].ly, threads=oracle.default_threads())
                errs.append(oracle.rel_l2(b.outputs[i].cpu().numpy().astype(np.complex128), ref))
            leg["err_vs_oracle_max"] = max(errs)
        if name == "fp64":
            solo = [torch.empty_like(x) for x in ins]
            for _ in range(2):
                for x, o, m in zip(ins, solo, srcs):
                    fp.solve_poisson(x, m.lx, m.ly, out=o)
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record()
            for x, o, m in zip(ins, solo, srcs):
                fp.solve_poisson(x, m.lx, m.ly, out=o)
            e1.record()
            torch.cuda.synchronize()
            ms1 = e0.elapsed_time(e1)
            out["fp64_one_at_a_time"] = {"ms": round(ms1, 3), "solves_per_s": round(len(srcs) / (ms1 * 1e-3), 1)}
        out[name] = leg
        b.close()
        del ins
    return out


def serving_leg(fp, torch, duration: float = 11.0, warm: float = 1.0, budget_gib: int = 64,
                slots: int = 64, streams: int = 4, check: bool = True):
    """Open-loop serving: requests are submitted at their arrival times from
    a client thread; the main thread waits for each, records its latency and
    releases it.  Latency = completion (device timestamp) - submission."""
    import threading

    import numpy as np

    import workloads as W
    trace = W.serving_trace(seed=5, rate=2000.0, duration=duration)
    dev = torch.device("cuda:0")
    inputs = {}
    for t in trace:
        key = (t.kind, t.nx, t.ny)
        if key not in inputs:
            f, lx, ly = W.serving_input(t.kind, t.nx, t.ny)
            inputs[key] = (torch.from_numpy(f).to(torch.complex64).to(dev), lx, ly)
    max_steps = max(t.steps for t in trace)
    ring = 4096  # diagnostics slots: far more than requests in flight
    diag = torch.zeros((ring, 3 * max_steps), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    srv = fp.Server(budget_gib << 30, slots, streams)
    reqs = []
    for i, t in enumerate(trace):
        x, lx, ly = inputs[(t.kind, t.nx, t.ny)]
        d = diag[i % ring].data_ptr() if t.kind != 0 else None
        reqs.append(fp.FftpdeRequest(t.kind, 0, t.nx, t.ny, lx, ly, t.coef, t.dt, t.steps, x.data_ptr(), None,
                                     None, d, 0.0, 0, None))
    ids = [None] * len(trace)
    lag = [0.0] * len(trace)
    started = threading.Event()
    t0_box = []

    def client():
        t0 = time.perf_counter()
        t0_box.append(t0)
        started.set()
        for i, (t, r) in enumerate(zip(trace, reqs)):
            while True:
                now = time.perf_counter() - t0
                if now >= t.arrival:
                    break
                if t.arrival - now > 2e-4:
                    time.sleep(min(t.arrival - now - 1e-4, 1e-3))
            lag[i] = time.perf_counter() - t0 - t.arrival
            ids[i] = srv.submit_raw(r)

    th = threading.Thread(target=client, daemon=True)
    th.start()
    started.wait()
    # a sample of served results is kept for a check against the FP64 oracle
    # after the run: the largest request of each kind and every 2000th
    largest = {k: max((i for i, t in enumerate(trace) if t.kind == k), key=lambda i: trace[i].nx * trace[i].ny)
               for k in (0, 1, 2) if any(t.kind == k for t in trace)}
    keep_ids = set(largest.values()) | set(range(0, len(trace), 2000))
    kept = {}
    lat, kinds, arr = [], [], []
    failed = 0
    for i, t in enumerate(trace):
        while ids[i] is None:
            time.sleep(1e-4)
        res = srv.wait(ids[i], 120.0)
        if res["status"] != 0:
            failed += 1
        else:
            lat.append((res["t_done"] - res["t_submit"]) * 1e3 + lag[i] * 1e3)
            kinds.append(t.kind)
            arr.append(t.arrival)
            if check and i in keep_ids:
                kept[i] = srv.copy_out(ids[i], torch.empty((t.ny, t.nx), dtype=torch.complex64, device=dev))
        srv.release(ids[i])
    th.join()
    st = srv.stats()
    srv.close()
    lat, kinds, arr = np.array(lat), np.array(kinds), np.array(arr)
    m = arr >= warm
    window = duration - warm

    def q(v, p):
        return float(np.percentile(v, p, method="inverted_cdf")) if len(v) else None
    checked = []
    if kept:
        import oracle
        th_n = oracle.default_threads()
        for i in sorted(kept):
            t = trace[i]
            f, lx, ly = W.serving_input(t.kind, t.nx, t.ny)
            x = f.astype(np.complex64).astype(np.complex128)
            T = t.steps * t.dt
            if t.kind == 0:
                ref = oracle.solve_poisson(x, lx, ly, threads=th_n)
            elif t.kind == 1:
                ref = oracle.solve_diffusion(x, lx, ly, t.coef, T, threads=th_n)
            else:
                ref = oracle.solve_wave(x, None, lx, ly, t.coef, T, threads=th_n)[0]
            got = kept[i].cpu().numpy().astype(np.complex128)
            den = max(float(np.linalg.norm(ref)), float(np.linalg.norm(x)) if t.kind else 0.0)
            err = float(np.linalg.norm(got - ref) / den)
            checked.append({"kind": ("poisson", "diffusion", "wave")[t.kind], "nx": t.nx, "ny": t.ny,
                            "steps": t.steps, "err_vs_oracle": err,
                            "tol": 2 * 2e-6 * np.log2(max(t.nx, t.ny))})
    per_kind = {name: {"p50_ms": q(lat[m & (kinds == k)], 50), "p99_ms": q(lat[m & (kinds == k)], 99),
                       "count": int((m & (kinds == k)).sum())}
                for k, name in ((0, "poisson"), (1, "diffusion"), (2, "wave"))}
    return {"workload": "serving_mix_poisson_arrivals_2000rps", "requests": len(trace),
            "measured_requests": int(m.sum()), "failed": failed,
            "offered_rps": round(sum(1 for t in trace if t.arrival >= warm) / window, 1),
            "achieved_rps": round(int(m.sum()) / window, 1),
            "p50_ms": q(lat[m], 50), "p99_ms": q(lat[m], 99), "mean_ms": float(lat[m].mean()),
            "max_ms": float(lat[m].max()), "per_kind": per_kind,
            "submit_lag_p99_ms": round(float(np.percentile(np.array(lag), 99)) * 1e3, 3),
            "hbm_budget_gib": budget_gib, "hbm_high_water_gib": round(st["hbm_high_water"] / 2 ** 30, 3),
            "max_slots": slots, "streams": streams, "iterations": st["iterations"],
            "checked_vs_oracle": checked,
            "latency": "device completion - submission + client submit lag",
            "steps": "diagnostics (mean, energy) at every step from the resident spectra, "
                     "u materialised at the final step"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=16, help="FP32 batch (FP64 uses half)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-real", action="store_true", help="skip the real-field legs")
    ap.add_argument("--no-source", action="store_true", help="skip the constant-source leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-radix (1536^2) leg")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain elementwise copy of the FP32 batch (512 MiB at B = 16), "
                         "the known-size reference for hardware byte counters")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-seconds", type=float, default=11.0)
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(independent solves would shard by request across GPUs).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2412_12308_amd as fp
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    print(f"# generating inputs: {a.batch} x {N_SIDE}^2", file=sys.stderr, flush=True)
    fields = make_inputs(N_SIDE, a.batch)
    if a.copy_probe:
        src = torch.from_numpy(fields).to(torch.complex64).to("cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0, out=dst)
        torch.cuda.synchronize()
        print(f"# copy probe: 3 x {src.numel() * 8} bytes read + written", file=sys.stderr, flush=True)
        del src, dst
    print("# fp32 leg", file=sys.stderr, flush=True)
    r32 = run_leg(fp, torch, fields, "c64", a.steps, a.warmup)
    err32 = None if a.no_check else oracle_check(r32["last_out"][0], fields[0], "c64", r32["last_t"])
    r64 = None
    err64 = None
    if not a.no_fp64:
        print("# fp64 leg", file=sys.stderr, flush=True)
        f64 = fields[: max(1, a.batch // 2)]
        r64 = run_leg(fp, torch, f64, "c128", a.steps, a.warmup)
        err64 = None if a.no_check else oracle_check(r64["last_out"][0], f64[0], "c128", r64["last_t"])
    real = {}
    half = None
    if not a.no_real:
        # the same real-valued initial data as real fields, two per complex
        # transform: 2B FP32 / B FP64 fields, the complex legs' bytes in flight
        for name, nb in (("r32", 2 * a.batch), ("r64", a.batch)):
            print(f"# real {name} leg", file=sys.stderr, flush=True)
            rf = make_inputs(N_SIDE, nb) if nb > len(fields) else fields[:nb]
            rr = run_leg(fp, torch, rf, name, a.steps, a.warmup)
            err = None if a.no_check else oracle_check(rr["last_out"][0], rf[0], name, rr["last_t"])
            real[name] = {"value": round(rr["solves_per_s"], 2), "unit": "solves/s", "batch": rr["batch"],
                          "ms_per_step": round(rr["ms_per_step"], 4), "eff_hbm_gbs": round(rr["eff_gbs"], 1),
                          "eff_hbm_frac": round(rr["eff_gbs"] / HBM_PEAK_GBS, 4), "err_vs_oracle": err,
                          "err_tol": 1e-12 if name == "r64" else 2 * 2e-6 * math.log2(N_SIDE),
                          "kernels": [{"kernel": k["kernel"], "launches": k["launches"],
                                       "avg_us": round(k["avg_us"], 2), "gbs": round(k["gbs"], 1)}
                                      for k in rr["kernels"]]}
            del rr
        print("# half-spectrum leg", file=sys.stderr, flush=True)
        half = half_spectrum_leg(fp, torch, fields, a.steps, a.warmup, not a.no_check)
    three = None
    if not a.no_3d:
        print("# 3d leg", file=sys.stderr, flush=True)
        three = leg_3d(fp, torch, a.steps, a.warmup, not a.no_check)
    mixed = None
    if not a.no_mixed:
        print("# mixed-radix leg", file=sys.stderr, flush=True)
        mixed = mixed_leg(fp, torch, a.steps, a.warmup, not a.no_check)
    source = None
    if not a.no_source:
        print("# wave with a constant source leg", file=sys.stderr, flush=True)
        source = source_leg(fp, torch, fields[: max(1, a.batch // 2)], a.steps, a.warmup, not a.no_check)
    batch = None
    if not a.no_batch:
        print("# uneven batch leg", file=sys.stderr, flush=True)
        batch = batch_leg(fp, torch, 20, 3, not a.no_check)
    serve = None
    if not a.no_serve:
        print("# serving leg", file=sys.stderr, flush=True)
        serve = serving_leg(fp, torch, duration=a.serve_seconds, check=not a.no_check)
    cpu = None
    if not a.no_cpu:
        print("# cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(fields[0], a.cpu_seconds)

    dom = r32["dominant"]
    tol32 = 2 * 2e-6 * math.log2(N_SIDE)
    line = {
        "metric": METRIC,
        "value": round(r32["solves_per_s"], 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "timing": {"burn_in_steps": BURN_IN, "cold_ms_per_step": round(r32["cold_ms_per_step"], 4),
                   "cold_solves_per_s": round(r32["batch"] / (r32["cold_ms_per_step"] * 1e-3), 2),
                   "note": "value: K steps after the W warm-up steps, a cold window of K steps and "
                           "burn_in_steps more untimed steps (steady state); cold: the K steps right "
                           "after the W warm-up steps"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "wave2d_2048x2048_periodic_unit_square", "nx": N_SIDE, "ny": N_SIDE,
                   "batch": r32["batch"], "c": C_SPEED, "dt": DT,
                   "precision": "FP32 butterflies; FP64 twiddle generation and FP64 phase",
                   "solve": "fwd 2D FFT + cos(c|k|t_n) + inverse 2D FFT, 3 HBM passes"},
        "eff_hbm_gbs": round(r32["eff_gbs"], 1),
        "eff_hbm_frac": round(r32["eff_gbs"] / HBM_PEAK_GBS, 4),
        "err_vs_oracle": err32,
        "err_tol": tol32,
        "roofline": {"bound": "hbm", "achieved": round(dom["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom["achieved_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": traffic_for(dom["kernel"]), "kernel": dom["kernel"],
                     "avg_us": round(dom["avg_us"], 2), "bytes_per_launch": dom["bytes_per_launch"],
                     "solve_achieved": round(r32["eff_gbs"], 1),
                     "solve_frac": round(r32["eff_gbs"] / HBM_PEAK_GBS, 4),
                     "note": "achieved/frac: the dominant kernel (largest share of the step); "
                             "solve_*: the whole fused solve, 6 b P bytes per solve"},
        "kernels": [{"kernel": k["kernel"], "launches": k["launches"], "avg_us": round(k["avg_us"], 2),
                     "gbs": round(k["gbs"], 1)} for k in r32["kernels"]],
        "cpu_baseline": cpu,
    }
    if r64:
        line["fp64"] = {"value": round(r64["solves_per_s"], 2), "unit": "solves/s", "batch": r64["batch"],
                        "ms_per_step": round(r64["ms_per_step"], 4),
                        "cold_ms_per_step": round(r64["cold_ms_per_step"], 4),
                        "eff_hbm_gbs": round(r64["eff_gbs"], 1),
                        "eff_hbm_frac": round(r64["eff_gbs"] / HBM_PEAK_GBS, 4), "err_vs_oracle": err64,
                        "err_tol": 1e-12,
                        "kernels": [{"kernel": k["kernel"], "launches": k["launches"],
                                     "avg_us": round(k["avg_us"], 2), "gbs": round(k["gbs"], 1)}
                                    for k in r64["kernels"]]}
    if real:
        line["real_fields"] = {"workload": "the same wave problems with u0 stored as real fields, solved two "
                                           "per complex transform (S(u1 + i u2) = S(u1) + i S(u2): the symbol "
                                           "is real and even)", **real}
    if half:
        line["half_spectrum"] = half
    if three:
        line["wave3d"] = three
    if mixed:
        line["wave_mixed_radix"] = mixed
    if source:
        line["wave_source"] = source
    if batch:
        line["batch"] = batch
    if serve:
        line["serving"] = serve
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
