"""The request server on the GPU: every result against the FP64 oracle and
against the same request run alone (bit for bit: the same kernels run in the
same order on the request's own data), per-step diagnostics against the
evolution API, server-owned outputs, and admission under a small budget."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import as_oracle_input, rel_err_vs_input, say, to_dev, to_host, tol

pytestmark = pytest.mark.gpu
POISSON, DIFFUSION, WAVE = 0, 1, 2


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


def _expect(op, x, lx, ly, coef, t, threads=1):
    if op == POISSON:
        return oracle.solve_poisson(x, lx, ly, threads=threads)
    if op == DIFFUSION:
        return oracle.solve_diffusion(x, lx, ly, coef, t, threads=threads)
    return oracle.solve_wave(x, None, lx, ly, coef, t, threads=threads)[0]


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_each_operator_matches_the_oracle_and_the_evolution_api(fp, dt):
    import torch
    say(f"server operators {dt}")
    with fp.Server(1 << 30, 8, 4) as srv:
        cases = []
        for k, (op, nx, ny, steps, tstep, coef) in enumerate([
                (POISSON, 128, 64, 1, 0.0, 0.0), (DIFFUSION, 256, 256, 40, 1e-3, 0.01),
                (WAVE, 64, 512, 37, 1e-4, 1.0), (WAVE, 2048, 16, 3, 0.01, 0.5)]):
            x = W.random_field((ny, nx), seed=50 + k)
            inp = to_dev(x, dt)
            out = torch.empty_like(inp)
            diag = torch.zeros(3 * steps, dtype=torch.float64, device="cuda:0") if op != POISSON else None
            rid = srv.submit(op, inp, out=out, diag=diag, steps=steps, dt=tstep, coef=coef, lx=1.0, ly=2.0)
            cases.append((rid, op, x, inp, out, diag, steps, tstep, coef))
        for rid, op, x, inp, out, diag, steps, tstep, coef in cases:
            res = srv.wait(rid, 60)
            assert res["status"] == 0, res
            ny, nx = x.shape
            xo = as_oracle_input(x, dt)
            ref = _expect(op, xo, 1.0, 2.0, coef, steps * tstep)
            got = to_host(out)
            err = oracle.rel_l2(got, ref) if op == POISSON else rel_err_vs_input(got, ref, float(np.linalg.norm(xo)))
            assert err <= tol(dt, nx, ny, 2), (op, nx, ny, err)
            if diag is not None:
                # the evolution API evaluates one time per launch; the server 16
                with fp.Evolution(op, inp.view(1, ny, nx), None, coef, 1.0, 2.0) as ev:
                    for n in (1, steps // 2 + 1, steps):
                        _, _, d = ev.step(n, tstep, want_u=False, diag=True)
                        a = diag.view(steps, 3)[n - 1].cpu().numpy()
                        b = d[0].cpu().numpy()
                        assert np.allclose(a, b, rtol=1e-12, atol=1e-300), (n, a, b)
            srv.release(rid)
        st = srv.stats()
        assert st["completed"] == 4 and st["hbm_in_use"] == 0 and st["failed"] == 0


def test_results_alone_equal_results_in_the_mix(fp):
    """At least 200 logged requests of the serving mix (sides 2^6..2^9),
    submitted together, then each alone: identical fields and diagnostics."""
    import torch
    trace = W.serving_trace(seed=5, rate=2000.0, duration=0.11, log2_sides=(6, 9))
    assert len(trace) >= 200
    say(f"server alone vs mix: {len(trace)} requests")
    inputs = {}

    def inp_for(t):
        key = (t.kind, t.nx, t.ny)
        if key not in inputs:
            inputs[key] = to_dev(W.random_field((t.ny, t.nx), seed=t.nx * 7 + t.ny + t.kind), "c64")
        return inputs[key]

    def submit(srv, t):
        out = torch.empty((t.ny, t.nx), dtype=torch.complex64, device="cuda:0")
        diag = torch.zeros(3 * t.steps, dtype=torch.float64, device="cuda:0") if t.kind != POISSON else None
        rid = srv.submit(t.kind, inp_for(t), out=out, diag=diag, steps=t.steps, dt=t.dt, coef=t.coef)
        return rid, out, diag

    with fp.Server(8 << 30, 16, 4) as srv:
        mix = [submit(srv, t) for t in trace]
        for rid, _, _ in mix:
            assert srv.wait(rid, 120)["status"] == 0
        st = srv.stats()
        say(f"  mix: p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms, iterations {st['iterations']}")
        for t, (rid_m, out_m, diag_m) in zip(trace, mix):
            rid, out, diag = submit(srv, t)
            assert srv.wait(rid, 60)["status"] == 0
            assert torch.equal(out, out_m), (t.kind, t.nx, t.ny)
            if diag is not None:
                assert torch.equal(diag, diag_m)
            srv.release(rid)
            srv.release(rid_m)
        # a sample against the oracle
        for t, (_, out_m, _) in list(zip(trace, mix))[:12]:
            x = as_oracle_input(to_host(inp_for(t)), "c64")
            ref = _expect(t.kind, x, 1.0, 1.0, t.coef, t.steps * t.dt)
            got = to_host(out_m)
            err = oracle.rel_l2(got, ref) if t.kind == POISSON else rel_err_vs_input(got, ref, float(np.linalg.norm(x)))
            assert err <= tol("c64", t.nx, t.ny, 2)


def test_results_alone_equal_results_in_the_mix_at_every_side(fp):
    """The serving mix over its whole side range (2^6..2^12 on each axis),
    with the largest requests added: 4096^2 wave, diffusion and Poisson
    solves and 4096 x 64 / 64 x 4096 / 4096 x 128 rectangles (multi-tile,
    chunked and tiled-intermediate paths; a Poisson solve's spectrum lives in
    the server's pool).  Every request alone equals itself in the mix, bit
    for bit, and a sample that includes the largest sides of each kind
    matches the FP64 oracle."""
    import torch
    trace = list(W.serving_trace(seed=5, rate=2000.0, duration=0.1, log2_sides=(6, 12)))
    big = [W.Request(0.0, WAVE, 4096, 4096, 37, 1e-4, 1.0), W.Request(0.0, DIFFUSION, 4096, 4096, 25, 1e-3, 0.01),
           W.Request(0.0, POISSON, 4096, 4096, 1, 0.0, 0.0), W.Request(0.0, POISSON, 4096, 64, 1, 0.0, 0.0),
           W.Request(0.0, WAVE, 64, 4096, 50, 1e-4, 1.0), W.Request(0.0, DIFFUSION, 4096, 128, 12, 1e-3, 0.01)]
    for k, r in enumerate(big):   # spread through the mix
        trace.insert(min(len(trace), 5 + 30 * k), r)
    assert len(trace) >= 200 and max(t.nx for t in trace) == 4096 and min(t.nx for t in trace) == 64
    say(f"server alone vs mix, sides 2^6..2^12: {len(trace)} requests")
    inputs = {}

    def inp_for(t):
        key = (t.kind, t.nx, t.ny)
        if key not in inputs:
            g = torch.Generator(device="cuda:0").manual_seed(t.nx * 7919 + t.ny * 31 + t.kind)
            inputs[key] = torch.randn((t.ny, t.nx), dtype=torch.complex64, device="cuda:0", generator=g)
        return inputs[key]

    def submit(srv, t):
        out = torch.empty((t.ny, t.nx), dtype=torch.complex64, device="cuda:0")
        diag = torch.zeros(3 * t.steps, dtype=torch.float64, device="cuda:0") if t.kind != POISSON else None
        rid = srv.submit(t.kind, inp_for(t), out=out, diag=diag, steps=t.steps, dt=t.dt, coef=t.coef)
        return rid, out, diag

    with fp.Server(8 << 30, 16, 4) as srv:
        mix = [submit(srv, t) for t in trace]
        for rid, _, _ in mix:
            assert srv.wait(rid, 120)["status"] == 0
        st = srv.stats()
        assert st["hbm_high_water"] <= 8 << 30
        say(f"  mix: p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms, high water {st['hbm_high_water'] >> 20} MiB")
        for t, (rid_m, out_m, diag_m) in zip(trace, mix):
            rid, out, diag = submit(srv, t)
            assert srv.wait(rid, 60)["status"] == 0
            assert torch.equal(out, out_m), (t.kind, t.nx, t.ny)
            if diag is not None:
                assert torch.equal(diag, diag_m), (t.kind, t.nx, t.ny)
            srv.release(rid)
            srv.release(rid_m)
        # against the oracle: the largest request of each kind, the added
        # rectangles and a few of the trace
        by_size = sorted(range(len(trace)), key=lambda i: trace[i].nx * trace[i].ny)
        sample = {max((i for i in by_size if trace[i].kind == k), key=lambda i: trace[i].nx * trace[i].ny)
                  for k in (POISSON, DIFFUSION, WAVE)}
        sample |= {i for i, t in enumerate(trace) if t in big} | set(range(0, len(trace), 37))
        for i in sorted(sample):
            t, (_, out_m, _) = trace[i], mix[i]
            say(f"  oracle {t.kind} {t.nx}x{t.ny} steps {t.steps}")
            x = to_host(inp_for(t))
            ref = _expect(t.kind, x, 1.0, 1.0, t.coef, t.steps * t.dt, threads=oracle.default_threads())
            got = to_host(out_m)
            err = oracle.rel_l2(got, ref) if t.kind == POISSON else rel_err_vs_input(got, ref, float(np.linalg.norm(x)))
            assert err <= tol("c64", t.nx, t.ny, 2), (t.kind, t.nx, t.ny, err)


def test_server_owned_output_and_small_budget_admission(fp):
    """A budget of three 512^2 FP32 evolutions: requests wait for memory, the
    high-water mark stays within the budget, server-owned outputs are read
    back with copy_out and released."""
    import torch
    fb = 512 * 512 * 8
    budget = 3 * (4 * fb)   # in + F + scratch + server-owned out, with room to spare
    say("server small budget")
    with fp.Server(budget, 16, 4) as srv:
        x = W.random_field((512, 512), seed=9)
        inp = to_dev(x, "c64")
        ids = [srv.submit(DIFFUSION, inp, steps=20, dt=1e-3, coef=0.01 * (k + 1)) for k in range(10)]
        for k, rid in enumerate(ids):
            assert srv.wait(rid, 60)["status"] == 0
            got = to_host(srv.copy_out(rid, torch.empty_like(inp)))
            ref = oracle.solve_diffusion(as_oracle_input(x, "c64"), 1.0, 1.0, 0.01 * (k + 1), 20 * 1e-3)
            assert rel_err_vs_input(got, ref, float(np.linalg.norm(x))) <= tol("c64", 512, 512, 2)
            srv.release(rid)
        st = srv.stats()
        assert st["hbm_high_water"] <= budget and st["hbm_in_use"] == 0 and st["completed"] == 10
