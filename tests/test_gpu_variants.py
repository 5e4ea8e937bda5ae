"""Every compiled kernel variant (every plan the autotuner may choose) against
the FP64 oracle: each row variant on a grid whose x side is its length, each
column variant on a grid whose y side is its length, with a batch whose last
tile is ragged where the tile holds several lines."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import as_oracle_input, say, to_dev, to_host, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fp():
    import paper_2412_12308_amd as fp
    yield fp
    fp.plan_select(None)


def _variants():
    import paper_2412_12308_amd as fp
    try:
        return fp.plan_variants()
    except Exception:  # no GPU / library: the test body will report it
        return []


def _cases():
    out = []
    for v in _variants():
        if v["pass"] in ("row", "col"):
            out.append(pytest.param(v, id=v["name"]))
    return out


def _small_cases():
    return [pytest.param(v, id=v["name"]) for v in _variants() if v["pass"] == "small"]


@pytest.mark.parametrize("v", _small_cases())
def test_small_grid_kernel(fp, v):
    """The single-pass kernel for each compiled shape: forward, inverse and
    the three solves against the oracle, and the solve against the 3-pass path."""
    dt = "c64" if v["dtype"] == 0 else "c128"
    nx, ny, batch = 1 << v["lognx"], 1 << v["logny"], 5
    say(f"small {v['name']} batch={batch}")
    x = W.random_field((batch, ny, nx), seed=nx * 3 + ny)
    xd = to_dev(x, dt)
    X = to_host(fp.fft2d_forward(xd))
    Y = to_host(fp.fft2d_inverse(xd))
    for b in (0, batch - 1):
        xb = as_oracle_input(x[b], dt)
        assert oracle.rel_l2(X[b], oracle.fft2d(xb)) <= tol(dt, nx, ny, 1)
        assert oracle.rel_l2(Y[b], oracle.ifft2d(xb)) <= tol(dt, nx, ny, 1)
    u_p = to_host(fp.solve_poisson(xd, 1.0, 2.0))
    u_d = to_host(fp.solve_diffusion(xd, 0.05, 0.02, 1.0, 2.0))
    u_w, _ = fp.solve_wave(xd, None, 1.0, 0.37, 1.0, 2.0)
    u_w = to_host(u_w)
    for b in (0, batch - 1):
        xb = as_oracle_input(x[b], dt)
        assert oracle.rel_l2(u_p[b], oracle.solve_poisson(xb, 1.0, 2.0)) <= tol(dt, nx, ny, 2)
        assert oracle.rel_l2(u_d[b], oracle.solve_diffusion(xb, 1.0, 2.0, 0.05, 0.02)) <= tol(dt, nx, ny, 2)
        assert oracle.rel_l2(u_w[b], oracle.solve_wave(xb, None, 1.0, 2.0, 1.0, 0.37)[0]) <= tol(dt, nx, ny, 2)
    fp.plan_small(False)
    try:
        u3 = to_host(fp.solve_poisson(xd, 1.0, 2.0))
    finally:
        fp.plan_small(True)
    assert oracle.rel_l2(u_p, u3) <= tol(dt, nx, ny, 2)


@pytest.mark.parametrize("v", _cases())
def test_variant_matches_oracle(fp, v):
    dt = "c64" if v["dtype"] == 0 else "c128"
    n = 1 << v["logn"]
    if v["pass"] == "row":
        nx, ny = n, 16 if n <= 1024 else 4
    else:
        nx, ny = 8 if n >= 1024 else 16, n
    batch = 3
    fp.plan_select(None)
    fp.plan_select(v["name"])
    say(f"variant {v['name']} nx={nx} ny={ny} batch={batch}")
    try:
        if v["fields"] == 1:
            s = W.random_field((batch, ny, nx), seed=v["logn"] * 97 + v["dtype"])
            u = to_host(fp.solve_poisson(to_dev(s, dt), 1.0, 2.0))
            for b in range(batch):
                ref = oracle.solve_poisson(as_oracle_input(s[b], dt), 1.0, 2.0)
                assert oracle.rel_l2(u[b], ref) <= tol(dt, nx, ny, 2)
            X = to_host(fp.fft2d_forward(to_dev(s, dt)))
            assert oracle.rel_l2(X[batch - 1], oracle.fft2d(as_oracle_input(s[batch - 1], dt))) <= tol(dt, nx, ny, 1)
        elif v["fields"] == 3:
            f = W.random_field((batch, ny, nx), seed=13)
            g = W.random_field((batch, ny, nx), seed=14)
            s = W.random_field((batch, ny, nx), seed=15)
            u, vv = fp.solve_wave_source(to_dev(f, dt), to_dev(g, dt), to_dev(s, dt), 0.9, 0.3, 1.0, 1.0,
                                         want_v=True)
            u, vv = to_host(u), to_host(vv)
            for b in range(batch):
                fb, gb, sb = (as_oracle_input(a[b], dt) for a in (f, g, s))
                ru, rv = oracle.solve_wave_source(fb, gb, sb, 1.0, 1.0, 0.9, 0.3, want_v=True)
                scale = max(np.linalg.norm(ru), np.linalg.norm(fb), np.linalg.norm(sb) * 0.09)
                assert np.linalg.norm(u[b] - ru) / scale <= tol(dt, nx, ny, 2)
                wmax = 0.9 * 2 * np.pi * np.hypot(nx / 2, ny / 2)
                vscale = max(np.linalg.norm(rv), wmax * np.linalg.norm(fb))
                assert np.linalg.norm(vv[b] - rv) / vscale <= tol(dt, nx, ny, 2)
        else:
            u0 = W.random_field((batch, ny, nx), seed=11)
            v0 = W.random_field((batch, ny, nx), seed=12)
            u, vv = fp.solve_wave(to_dev(u0, dt), to_dev(v0, dt), 0.9, 0.3, 1.0, 1.0, want_v=True)
            u, vv = to_host(u), to_host(vv)
            for b in range(batch):
                ru, rv = oracle.solve_wave(as_oracle_input(u0[b], dt), as_oracle_input(v0[b], dt), 1.0, 1.0,
                                           0.9, 0.3, want_v=True)
                assert oracle.rel_l2(u[b], ru) <= tol(dt, nx, ny, 2)
                assert oracle.rel_l2(vv[b], rv) <= tol(dt, nx, ny, 2)
    finally:
        fp.plan_select(None)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_autotune_picks_an_admitted_variant_and_round_trips(fp, dt, tmp_path):
    say(f"autotune 256x512 {dt}")
    fp.plan_select(None)
    rep = fp.autotune(256, 512, batch=2, dtype=dt, op=fp.DIFFUSION, reps=2)
    assert rep["nx"] == 256 and rep["ny"] == 512
    names = {c["name"] for c in rep["candidates"] if c["ok"]}
    assert rep["row"] in names and rep["col"] in names
    assert all(c["err"] <= (1e-12 if dt == "c128" else 2 * 2e-6 * 9) for c in rep["candidates"] if c["ok"])
    active = {v["name"] for v in fp.plan_variants() if v["active"]}
    assert rep["row"] in active and rep["col"] in active
    # the layout stage: every block size timed, the chosen one among the admitted
    layouts = {c["name"]: c for c in rep["candidates"] if c["pass"] == "layout"}
    assert set(layouts) == {"tiled_0", "tiled_256", "tiled_1024", "tiled_4096"}
    assert layouts[f"tiled_{rep['tiled_bytes']}"]["ok"]
    chunks = {c["name"]: c for c in rep["candidates"] if c["pass"] == "chunk"}
    assert len(chunks) == 5 and chunks[f"chunk_{rep['chunk_bytes']}"]["ok"]
    # results with the tuned plan still match the oracle
    f = W.random_field((512, 256), seed=5)
    u = to_host(fp.solve_diffusion(to_dev(f, dt), 0.2, 0.01, 1.0, 1.0))
    ref = oracle.solve_diffusion(as_oracle_input(f, dt), 1.0, 1.0, 0.2, 0.01)
    assert oracle.rel_l2(u, ref) <= tol(dt, 256, 512, 2)
    # save, reset, load: the same variants become active again
    path = str(tmp_path / "plan.txt")
    fp.plan_save(path)
    fp.plan_select(None)
    fp.plan_load(path)
    active2 = {v["name"] for v in fp.plan_variants() if v["active"]}
    assert rep["row"] in active2 and rep["col"] in active2
    code = 0 if dt == "c64" else 1
    assert f"tiled {code} 8 9 {rep['tiled_bytes']}" in open(path).read()
    assert f"chunk {code} 8 9 {rep['chunk_bytes']}" in open(path).read()
    fp.plan_select(None)


def _xw_cases():
    return [pytest.param(v, id=v["name"]) for v in _variants() if v["name"].endswith("_xw")]


@pytest.mark.parametrize("v", _xw_cases())
def test_in_wave_exchange_variant_all_symbols(fp, v):
    """The fused column pass whose exchanges around the radix-8 stage stay in
    each wavefront (2048-row columns, 4-column tiles): the Poisson, diffusion
    and wave solves against the oracle, on 6 tiles per field and a batch of 2.
    The wave solve's symbol is shared between mirrored rows across lanes, and
    wave 0 of each tile takes the residues 0 and 8, which pair differently:
    every tile has both kinds, so a wrong pairing shows at any column."""
    nx, ny, batch = 24, 2048, 2
    fp.plan_select(None)
    fp.plan_select(v["name"])
    say(f"variant {v['name']} nx={nx} ny={ny} batch={batch}")
    try:
        x = W.random_field((batch, ny, nx), seed=2048 + 24)
        xd = to_dev(x, "c64")
        u_p = to_host(fp.solve_poisson(xd, 1.0, 2.0))
        u_d = to_host(fp.solve_diffusion(xd, 0.05, 0.02, 1.0, 2.0))
        u_w, _ = fp.solve_wave(xd, None, 1.0, 0.37, 1.0, 2.0)
        u_w = to_host(u_w)
        for b in range(batch):
            xb = as_oracle_input(x[b], "c64")
            assert oracle.rel_l2(u_p[b], oracle.solve_poisson(xb, 1.0, 2.0)) <= tol("c64", nx, ny, 2)
            assert oracle.rel_l2(u_d[b], oracle.solve_diffusion(xb, 1.0, 2.0, 0.05, 0.02)) <= tol("c64", nx, ny, 2)
            assert oracle.rel_l2(u_w[b], oracle.solve_wave(xb, None, 1.0, 2.0, 1.0, 0.37)[0]) <= tol("c64", nx, ny, 2)
    finally:
        fp.plan_select(None)
