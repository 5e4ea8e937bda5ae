"""The persistent batch kernel (fftpde_batch_*): many independent solves of
uneven shapes in one launch, replayed from a captured HIP graph.

Every job is checked against the FP64 oracle (on sampled jobs for the
1024-job uneven Poisson batch, whose other jobs are checked against the
single-field solve path on the GPU), against the closed form of its
mode-sum source, and the graph replay against a direct launch, bit for bit."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import TOL_FP64 as TOL64, as_oracle_input, rel_err_vs_input, say, to_dev, to_host, tol

pytestmark = pytest.mark.gpu
THREADS = oracle.default_threads()


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    return fp


def _oracle_solve(job, x):
    op = job["op"]
    if op == 0:
        return oracle.solve_poisson(x, job["lx"], job["ly"], threads=THREADS)
    if op == 1:
        return oracle.solve_diffusion(x, job["lx"], job["ly"], job["coef"], job["t"], threads=THREADS)
    return oracle.solve_wave(x, None, job["lx"], job["ly"], job["coef"], job["t"], threads=THREADS)[0]


def _mixed_jobs(dt, seed):
    """Every operator, sides 16..512 (square, wide, tall), boxes != 1, times of
    both signs for the wave, some jobs in place."""
    rng = np.random.default_rng(seed)
    shapes = [(16, 16), (16, 512), (512, 16), (32, 64), (64, 32), (128, 128), (256, 64), (64, 256),
              (512, 512), (32, 32), (256, 256), (128, 16)]
    jobs = []
    for k, (nx, ny) in enumerate(shapes):
        op = k % 3
        lx, ly = float(rng.uniform(0.5, 3.0)), float(rng.uniform(0.5, 3.0))
        coef = [0.0, float(rng.uniform(0.001, 0.05)), float(rng.uniform(0.5, 2.0))][op]
        t = [0.0, float(rng.uniform(0.0, 0.2)), float(rng.uniform(-0.5, 0.5))][op]
        x = W.random_field((ny, nx), seed=seed * 100 + k)
        jobs.append(dict(op=op, x=x, lx=lx, ly=ly, coef=coef, t=t, inplace=(k % 4 == 3)))
    return jobs


def _make_batch(fp, jobs, dt):
    specs = []
    for j in jobs:
        inp = to_dev(j["x"], dt)
        spec = dict(op=j["op"], inp=inp, lx=j["lx"], ly=j["ly"], coef=j["coef"], t=j["t"])
        if j.get("inplace"):
            spec["out"] = inp
        specs.append(spec)
    return fp.Batch(specs)


def _check_job(j, got, dt):
    x = as_oracle_input(j["x"], dt)
    ref = _oracle_solve(j, x)
    ny, nx = x.shape
    if j["op"] == 0:
        err = oracle.rel_l2(got, ref)
    else:
        # |symbol| <= 1: the FP32 error floor is relative to the input
        err = rel_err_vs_input(got, ref, float(np.linalg.norm(x)))
    assert err <= tol(dt, nx, ny, 2), (j["op"], nx, ny, err)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_mixed_batch_matches_oracle(fp, dt):
    jobs = _mixed_jobs(dt, seed=7)
    say(f"batch mixed {len(jobs)} jobs {dt}")
    with _make_batch(fp, jobs, dt) as b:
        outs = b.run()
        b.status()
        for j, o in zip(jobs, outs):
            _check_job(j, to_host(o), dt)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_graph_replays_match_direct_launch_and_follow_new_inputs(fp, dt):
    """Replays with eager work and synchronisations between them; each replay
    is checked against a direct (uncaptured) launch of the same kernels, and
    new data written into the inputs between replays is picked up."""
    import torch
    jobs = [j for j in _mixed_jobs(dt, seed=11) if not j["inplace"]]
    say(f"batch graph replays {len(jobs)} jobs {dt}")
    with _make_batch(fp, jobs, dt) as b:
        for rep in range(3):
            if rep:
                for k, (j, inp) in enumerate(zip(jobs, b.inputs)):
                    j["x"] = W.random_field(j["x"].shape, seed=1000 * rep + k)
                    inp.copy_(to_dev(j["x"], dt))
            scratch = torch.randn(1 << 20, device="cuda:0").sum()  # eager work between replays
            torch.cuda.synchronize()
            direct = [o.clone() for o in b.run(use_graph=False)]
            b.status()
            graph = b.run(use_graph=True)
            b.status()
            assert bool(torch.isfinite(scratch))
            for j, d, g in zip(jobs, direct, graph):
                assert torch.equal(d, g), "graph replay differs from the direct launch"
            for i in (0, len(jobs) // 2, len(jobs) - 1):
                _check_job(jobs[i], to_host(graph[i]), dt)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_extreme_sides_and_shared_input(fp, dt):
    """Sides 16 and 4096 (one row or one column per tile), and several jobs
    reading the same input buffer (inputs may be shared; outputs not)."""
    x1 = W.random_field((16, 4096), seed=3)
    x2 = W.random_field((4096, 16), seed=4)
    say(f"batch extreme sides {dt}")
    shared = to_dev(x1, dt)
    specs = [dict(op=0, inp=shared, lx=2.0, ly=1.0), dict(op=1, inp=shared, coef=0.01, t=0.5),
             dict(op=2, inp=to_dev(x2, dt), coef=1.0, t=0.3, lx=1.0, ly=4.0)]
    with fp.Batch(specs) as b:
        outs = [to_host(o) for o in b.run()]
        b.status()
    _check_job(dict(op=0, x=x1, lx=2.0, ly=1.0, coef=0.0, t=0.0), outs[0], dt)
    _check_job(dict(op=1, x=x1, lx=1.0, ly=1.0, coef=0.01, t=0.5), outs[1], dt)
    _check_job(dict(op=2, x=x2, lx=1.0, ly=4.0, coef=1.0, t=0.3), outs[2], dt)


def test_rejects_overlapping_outputs_and_bad_jobs(fp):
    import torch
    x = torch.zeros((64, 64), dtype=torch.complex64, device="cuda:0")
    y = torch.zeros((64, 64), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(fp.FftpdeError):
        fp.Batch([dict(op=0, inp=x, out=y), dict(op=0, inp=x, out=y)])   # shared output
    with pytest.raises(fp.FftpdeError):
        fp.Batch([dict(op=0, inp=x, out=y), dict(op=0, inp=y, out=x)])   # output is another job's input
    with pytest.raises(fp.FftpdeError):
        fp.Batch([dict(op=1, inp=x, coef=0.1, t=-1.0)])                   # backward heat equation
    with pytest.raises(fp.FftpdeError):
        fp.Batch([dict(op=0, inp=torch.zeros((8, 8), dtype=torch.complex64, device="cuda:0"))])  # side < 16
    big = torch.zeros(2 * 64 * 64, dtype=torch.complex64, device="cuda:0")
    with pytest.raises(fp.FftpdeError):  # in and out of one job partly overlap
        fp.Batch([dict(op=0, inp=big[:4096].view(64, 64), out=big[2048:6144].view(64, 64))])


def _poisson_closed_form(ms):
    assert ms.sine_amp == 0
    x = W.grid(ms.nx, ms.lx)
    y = W.grid(ms.ny, ms.ly)
    u = np.zeros((ms.ny, ms.nx))
    for m, n, a, b in zip(ms.m, ms.n, ms.a, ms.b):
        th = 2 * math.pi * (m * x[None, :] / ms.lx + n * y[:, None] / ms.ly)
        k2 = (2 * math.pi * m / ms.lx) ** 2 + (2 * math.pi * n / ms.ly) ** 2
        u -= (a * np.cos(th) + b * np.sin(th)) / k2
    return u


def test_uneven_poisson_1024_fp32(fp):
    """1024 Poisson solves, sides drawn from 32..1024 (the uneven-batch
    workload): every job against the single-field solve on the GPU; 24
    sampled jobs (the largest and smallest included) against the oracle and
    the closed form of the mode-sum source."""
    import torch
    shapes = W.batch_shapes()
    srcs = W.batch_sources(shapes)
    dt = "c64"
    say(f"batch uneven poisson {len(shapes)} jobs {dt}")
    specs = [dict(op=0, inp=to_dev(ms.field, dt), lx=ms.lx, ly=ms.ly) for ms in srcs]
    with fp.Batch(specs) as b:
        outs = b.run()
        b.status()
        worst = 0.0
        for ms, s, o in zip(srcs, specs, outs):
            solo = fp.solve_poisson(s["inp"], ms.lx, ms.ly)
            d = (torch.linalg.vector_norm(o - solo) / torch.linalg.vector_norm(solo)).item()
            worst = max(worst, d)
            assert d <= 2 * tol(dt, ms.nx, ms.ny, 2), (ms.nx, ms.ny, d)
        say(f"  worst batch-vs-solo rel err {worst:.2e}")
        sizes = [ms.nx * ms.ny for ms in srcs]
        pick = {int(np.argmax(sizes)), int(np.argmin(sizes))}
        pick |= set(np.random.default_rng(0).choice(len(srcs), 22, replace=False).tolist())
        for i in sorted(pick):
            ms = srcs[i]
            got = to_host(outs[i])
            x = as_oracle_input(ms.field, dt)
            ref = oracle.solve_poisson(x, ms.lx, ms.ly, threads=THREADS)
            assert oracle.rel_l2(got, ref) <= tol(dt, ms.nx, ms.ny, 2), (i, ms.nx, ms.ny)
            # the closed form differs from the oracle by the FP32 rounding of the input
            assert oracle.rel_l2(got, _poisson_closed_form(ms)) <= tol(dt, ms.nx, ms.ny, 2) + 1e-6


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_single_pass_items_full_and_partial(fp, dt):
    """Jobs that fit one tile run as single-pass items of up to tile / P jobs
    of one shape and operator: 37 jobs of 32 x 16 (three operators: items of
    16 / 8 jobs and partial last items), 5 of 16 x 16 in place, and one job
    of exactly a tile beside three-pass jobs; all against the oracle."""
    rng = np.random.default_rng(21)
    jobs = []
    for k in range(37):
        op = k % 3
        jobs.append(dict(op=op, x=W.random_field((16, 32), seed=2100 + k), lx=float(rng.uniform(0.5, 2.0)),
                         ly=float(rng.uniform(0.5, 2.0)), coef=[0.0, 0.02, 1.3][op],
                         t=[0.0, 0.1, float(rng.uniform(-0.4, 0.4))][op]))
    for k in range(5):
        jobs.append(dict(op=2, x=W.random_field((16, 16), seed=2200 + k), lx=1.0, ly=1.5, coef=0.7, t=0.25,
                         inplace=True))
    side = (64, 128) if dt == "c64" else (64, 64)  # exactly one tile
    jobs.append(dict(op=1, x=W.random_field(side, seed=2300), lx=1.0, ly=1.0, coef=0.01, t=0.3))
    jobs.append(dict(op=0, x=W.random_field((256, 128), seed=2301), lx=2.0, ly=1.0, coef=0.0, t=0.0))
    say(f"batch single-pass items {len(jobs)} jobs {dt}")
    with _make_batch(fp, jobs, dt) as b:
        d = b.describe()
        assert d["single_pass"]["jobs"] == len(jobs) - 1, d
        per = (8192 if dt == "c64" else 4096) // 512
        assert d["single_pass"]["items"] == sum(-(-n // per) for n in (13, 12, 12)) + 1 + 1, d
        outs = b.run()
        b.status()
        for j, o in zip(jobs, outs):
            _check_job(j, to_host(o), dt)


def test_fp64_batches_have_one_plan(fp):
    jobs = [j for j in _mixed_jobs("c128", seed=13) if not j["inplace"]]
    with _make_batch(fp, jobs, "c128") as b:
        c = b.describe()["classes"][0]
        assert c["plan"] == 0 and c["max_radix"] == 8
        b.set_plan(0 if c["kind"] == "row" else 1, c["logn"], 0)
        with pytest.raises(fp.FftpdeError):
            b.set_plan(0 if c["kind"] == "row" else 1, c["logn"], 1)


def test_alternate_radix_plans_match_oracle(fp):
    """Every FP32 class switched to the other compiled radix plan (radix up to
    16): still every job against the oracle, and the plan table reported
    back."""
    dt = "c64"
    jobs = [j for j in _mixed_jobs(dt, seed=13) if not j["inplace"]]
    jobs.append(dict(op=2, x=W.random_field((16, 4096), seed=5), lx=1.0, ly=1.0, coef=1.0, t=0.2))
    jobs.append(dict(op=0, x=W.random_field((4096, 16), seed=6), lx=1.0, ly=1.0, coef=0.0, t=0.0))
    say(f"batch alternate plans {len(jobs)} jobs {dt}")
    with _make_batch(fp, jobs, dt) as b:
        for c in b.describe()["classes"]:
            b.set_plan(0 if c["kind"] == "row" else 1, c["logn"], 1)
        d = b.describe()
        assert all(c["plan"] == 1 for c in d["classes"]), d
        assert all(c["max_radix"] == 16 for c in d["classes"]), d
        outs = b.run()
        b.status()
        for j, o in zip(jobs, outs):
            _check_job(j, to_host(o), dt)
    with pytest.raises(fp.FftpdeError):
        with _make_batch(fp, jobs[:1], dt) as b:
            b.set_plan(1, 3, 1)  # no class of log2 length 3


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_tuner_keeps_results_within_tolerance(fp, dt):
    """fftpde_batch_tune on 96 uneven Poisson jobs: every candidate it kept is
    within its tolerance, the tuned plan's outputs match the oracle on sampled
    jobs, and a batch with a job in place is refused."""
    shapes = W.batch_shapes(count=96, seed=9)
    srcs = W.batch_sources(shapes, seed=9)
    say(f"batch tune {len(shapes)} jobs {dt}")
    specs = [dict(op=0, inp=to_dev(ms.field, dt), lx=ms.lx, ly=ms.ly) for ms in srcs]
    with fp.Batch(specs) as b:
        d = b.tune(reps=3)
        log = d["tune"]
        assert log and log[0]["kind"] == "start", d
        ncls = len(d["classes"]) if dt == "c64" else 0  # FP64: one plan
        assert len(log) == 1 + ncls, d
        for cand in log[1:]:
            assert cand["kept"] in (0, 1) and (not cand["kept"] or cand["ok"]), cand
            assert cand["err"] <= (1e-12 if dt == "c128" else 4e-6 * 10), cand
        outs = b.run()
        b.status()
        for i in (0, len(srcs) // 2, len(srcs) - 1):
            ms = srcs[i]
            ref = oracle.solve_poisson(as_oracle_input(ms.field, dt), ms.lx, ms.ly, threads=THREADS)
            assert oracle.rel_l2(to_host(outs[i]), ref) <= tol(dt, ms.nx, ms.ny, 2), (i, ms.nx, ms.ny)
    x = to_dev(W.random_field((64, 64), seed=1), dt)
    with fp.Batch([dict(op=0, inp=x, out=x)]) as b:
        with pytest.raises(fp.FftpdeError):
            b.tune(reps=1)


def test_uneven_poisson_1024_fp64(fp):
    """The uneven-batch workload in FP64: every job against the single-field
    solve on the GPU; 24 sampled jobs (the largest and smallest included)
    against the oracle and the closed form of the mode-sum source."""
    import torch
    shapes = W.batch_shapes()
    srcs = W.batch_sources(shapes)
    dt = "c128"
    say(f"batch uneven poisson {len(shapes)} jobs {dt}")
    specs = [dict(op=0, inp=to_dev(ms.field, dt), lx=ms.lx, ly=ms.ly) for ms in srcs]
    with fp.Batch(specs) as b:
        d = b.describe()
        assert d["single_pass"]["jobs"] == sum(1 for ms in srcs if ms.nx * ms.ny <= 4096), d
        outs = b.run()
        b.status()
        worst = 0.0
        for ms, s, o in zip(srcs, specs, outs):
            solo = fp.solve_poisson(s["inp"], ms.lx, ms.ly)
            dd = (torch.linalg.vector_norm(o - solo) / torch.linalg.vector_norm(solo)).item()
            worst = max(worst, dd)
            assert dd <= 2 * TOL64, (ms.nx, ms.ny, dd)
        say(f"  worst batch-vs-solo rel err {worst:.2e}")
        sizes = [ms.nx * ms.ny for ms in srcs]
        pick = {int(np.argmax(sizes)), int(np.argmin(sizes))}
        pick |= set(np.random.default_rng(1).choice(len(srcs), 22, replace=False).tolist())
        for i in sorted(pick):
            ms = srcs[i]
            got = to_host(outs[i])
            ref = oracle.solve_poisson(as_oracle_input(ms.field, dt), ms.lx, ms.ly, threads=THREADS)
            assert oracle.rel_l2(got, ref) <= TOL64, (i, ms.nx, ms.ny)
            assert oracle.rel_l2(got, _poisson_closed_form(ms)) <= TOL64, (i, ms.nx, ms.ny)
