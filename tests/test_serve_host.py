"""The request server's scheduler on the CPU: the same server code with a
host backend (fftpde_server_create_host) whose "device" is a Python function
that computes each request with the FP64 oracle on host arrays.  Covers
admission by budget and slots, first-come first-served order, rejection of
requests larger than the budget, cancellation, deadlines, a failing job
(its slot and budget come back, others are unaffected), server-owned
outputs and the pool they come from, step chunking, and that every result
is the same alone and in a mix."""
import ctypes
import threading
import time

import numpy as np
import pytest

import oracle
import workloads as W

fp = pytest.importorskip("paper_2412_12308_amd")

C128 = 1
POISSON, DIFFUSION, WAVE = 0, 1, 2
PENDING, EINVAL, EBUDGET, ENOTFOUND, ECANCELED, ETIMEOUT = 1, -1, -4, -5, -6, -7


def _lib_or_skip():
    import os
    if not os.path.exists(fp.LIB_PATH):
        pytest.skip("libfftpde.so not built")
    fp.lib()


def field_bytes(nx, ny):
    return nx * ny * 16


def _view(addr, shape):
    n = int(np.prod(shape))
    buf = (ctypes.c_double * (2 * n)).from_address(addr)
    return np.frombuffer(buf, dtype=np.complex128).reshape(shape)


class FakeDevice:
    """Executes requests with the oracle.  Each call is logged; a request id
    can be made to block (until released) or to fail."""

    def __init__(self):
        self.log = []
        self.lock = threading.Lock()
        self.gates = {}       # id -> threading.Event to wait on before working
        self.default_gate = None  # gate for ids without one (set before a submission)
        self.fail = set()     # ids whose final phase fails
        self.inputs = {}      # address -> numpy input (kept alive by the test)
        self.active = 0
        self.max_active = 0

    def __call__(self, rid, req, out, phase, n0, nt):
        with self.lock:
            self.log.append((rid, phase, n0, nt))
            if phase == 0:
                self.active += 1
                self.max_active = max(self.max_active, self.active)
        gate = self.gates.get(rid, self.default_gate)
        if gate is not None and phase == 0:
            assert gate.wait(20), "test gate never opened"
        if phase == 1 and req.diag:
            d = np.ctypeslib.as_array((ctypes.c_double * (3 * req.steps)).from_address(req.diag))
            for n in range(n0, n0 + nt):
                d[3 * (n - 1)] += n   # each step once: the test checks d == 1..steps
        if phase == 2:
            with self.lock:
                self.active -= 1
            if rid in self.fail:
                return -3
            x = self.inputs[req.inp]
            if req.op == POISSON:
                u = oracle.solve_poisson(x, req.lx, req.ly)
            elif req.op == DIFFUSION:
                u = oracle.solve_diffusion(x, req.lx, req.ly, req.coef, req.steps * req.dt)
            else:
                u = oracle.solve_wave(x, None, req.lx, req.ly, req.coef, req.steps * req.dt)[0]
            _view(out, x.shape)[...] = u
        return 0


@pytest.fixture
def dev():
    _lib_or_skip()
    return FakeDevice()


def _req(dev, op, nx, ny, out=None, steps=1, dt=0.0, coef=0.0, diag=None, deadline=0.0, seed=0, flags=0):
    x = W.random_field((ny, nx), seed=seed).astype(np.complex128)
    dev.inputs[x.ctypes.data] = x
    r = fp.FftpdeRequest(op, C128, nx, ny, 1.0, 2.0, coef, dt, steps, x.ctypes.data, None,
                         None if out is None else out.ctypes.data, None if diag is None else diag.ctypes.data,
                         deadline, flags, None)
    return r, x


def _expect(x, r):
    if r.op == POISSON:
        return oracle.solve_poisson(x, r.lx, r.ly)
    if r.op == DIFFUSION:
        return oracle.solve_diffusion(x, r.lx, r.ly, r.coef, r.steps * r.dt)
    return oracle.solve_wave(x, None, r.lx, r.ly, r.coef, r.steps * r.dt)[0]


def test_every_operator_completes_with_the_oracle_result(dev):
    with fp.Server.host(1 << 24, 4, dev) as srv:
        cases = []
        for k, (op, steps) in enumerate([(POISSON, 1), (DIFFUSION, 37), (WAVE, 16), (WAVE, 1)]):
            out = np.zeros((32, 64), np.complex128)
            diag = np.zeros(3 * steps) if op != POISSON else None
            r, x = _req(dev, op, 64, 32, out=out, steps=steps, dt=1e-3, coef=0.5, diag=diag, seed=k)
            cases.append((srv.submit_raw(r), r, x, out, diag))
        for rid, r, x, out, diag in cases:
            res = srv.wait(rid, 20)
            assert res["status"] == 0 and res["state"] == fp.STATE_ENDED
            assert res["t_submit"] <= res["t_admit"] <= res["t_done"]
            assert np.array_equal(out, _expect(x, r))
            if diag is not None:   # every step exactly once, in chunks of at most 16
                assert np.array_equal(diag[0::3], np.arange(1, r.steps + 1))
                chunks = [(n0, nt) for (i, ph, n0, nt) in dev.log if i == rid and ph == 1]
                assert all(1 <= nt <= 16 for _, nt in chunks)
                assert [n0 for n0, _ in chunks] == sorted(n0 for n0, _ in chunks)
            phases = [ph for (i, ph, _, _) in dev.log if i == rid]
            assert phases[0] == 0 and phases[-1] == 2
            srv.release(rid)
        st = srv.stats()
        assert st["completed"] == 4 and st["failed"] == 0 and st["hbm_in_use"] == 0
        assert st["latency_count"] == 4 and 0 <= st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_budget_admission_waits_and_is_first_come_first_served(dev):
    """Budget for one 64x64 request at a time (in + out + the spectrum
    between the passes = 3 fields): B waits while A runs; C (small) may not
    overtake B, although it would fit."""
    big = 3 * field_bytes(64, 64)
    small = 3 * field_bytes(16, 16)
    with fp.Server.host(big + small, 8, dev) as srv:
        outs = [np.zeros((64, 64), np.complex128) for _ in range(2)] + [np.zeros((16, 16), np.complex128)]
        ra, xa = _req(dev, POISSON, 64, 64, out=outs[0], seed=1)
        rb, xb = _req(dev, POISSON, 64, 64, out=outs[1], seed=2)
        rc, xc = _req(dev, POISSON, 16, 16, out=outs[2], seed=3)
        dev.default_gate = threading.Event()
        a = srv.submit_raw(ra)
        dev.gates[a], dev.default_gate = dev.default_gate, None
        time.sleep(0.05)
        b, c = srv.submit_raw(rb), srv.submit_raw(rc)
        time.sleep(0.2)
        assert srv.poll(b)["state"] == fp.STATE_QUEUED
        assert srv.poll(c)["state"] == fp.STATE_QUEUED   # behind b, although it would fit
        st = srv.stats()
        assert st["queued"] == 2 and st["running"] == 1 and st["hbm_in_use"] == big
        dev.gates[a].set()
        for rid in (a, b, c):
            assert srv.wait(rid, 20)["status"] == 0
        ta, tb, tc = (srv.poll(r)["t_admit"] for r in (a, b, c))
        assert ta <= tb <= tc
        assert srv.stats()["hbm_high_water"] <= big + small


def test_slots_bound_concurrency(dev):
    with fp.Server.host(1 << 24, 2, dev) as srv:
        gate = threading.Event()
        ids = []
        dev.default_gate = gate   # every request below holds until the gate opens
        for k in range(5):
            out = np.zeros((16, 16), np.complex128)
            r, x = _req(dev, POISSON, 16, 16, out=out, seed=k)
            rid = srv.submit_raw(r, keep=(out,))
            ids.append(rid)
        time.sleep(0.2)
        st = srv.stats()
        assert st["running"] <= 2 and st["queued"] >= 3
        gate.set()
        for rid in ids:
            assert srv.wait(rid, 20)["status"] == 0
        assert dev.max_active <= 2


def test_rejection_cancellation_deadline_and_failure(dev):
    fb = field_bytes(32, 32)
    with fp.Server.host(4 * fb, 1, dev) as srv:
        # larger than the whole budget: rejected at submission
        o0 = np.zeros((128, 128), np.complex128)
        r, _ = _req(dev, POISSON, 128, 128, out=o0)
        with pytest.raises(fp.FftpdeError) as e:
            srv.submit_raw(r)
        assert e.value.status == EBUDGET
        # invalid requests
        bad, _ = _req(dev, POISSON, 32, 32, steps=2)
        with pytest.raises(fp.FftpdeError):
            srv.submit_raw(bad)
        bad, _ = _req(dev, DIFFUSION, 32, 32, dt=-1.0, coef=0.1)
        with pytest.raises(fp.FftpdeError):
            srv.submit_raw(bad)
        # a blocking request holds the only slot
        o1 = np.zeros((32, 32), np.complex128)
        r1, _ = _req(dev, POISSON, 32, 32, out=o1, seed=1)
        # the gate is in place before the submission, so the scheduler cannot
        # start the request before it holds
        dev.default_gate = threading.Event()
        a = srv.submit_raw(r1)
        dev.gates[a], dev.default_gate = dev.default_gate, None
        time.sleep(0.05)
        # queued requests: one cancelled, one past its deadline, one that fails
        o2, o3, o4, o5 = (np.zeros((32, 32), np.complex128) for _ in range(4))
        r2, _ = _req(dev, POISSON, 32, 32, out=o2, seed=2)
        r3, _ = _req(dev, POISSON, 32, 32, out=o3, seed=3, deadline=0.05)
        r4, _ = _req(dev, POISSON, 32, 32, out=o4, seed=4)
        r5, x5 = _req(dev, DIFFUSION, 32, 32, out=o5, seed=5, steps=5, dt=0.01, coef=0.1)
        b, c, d, f = (srv.submit_raw(r) for r in (r2, r3, r4, r5))
        dev.fail.add(d)
        srv.cancel(b)
        assert srv.poll(b)["status"] == ECANCELED
        time.sleep(0.2)
        assert srv.poll(c)["status"] == ETIMEOUT
        dev.gates[a].set()
        assert srv.wait(a, 20)["status"] == 0
        assert srv.wait(d, 20)["status"] < 0              # the failed job
        assert srv.wait(f, 20)["status"] == 0             # others unaffected
        assert np.array_equal(o5, _expect(x5, r5))
        st = srv.stats()
        assert st["canceled"] == 1 and st["timed_out"] == 1 and st["failed"] == 1 and st["rejected"] == 1
        assert st["hbm_in_use"] == 0 and st["running"] == 0 and st["queued"] == 0
        # cancelling a running request: no further work is issued
        o6, d6 = np.zeros((32, 32), np.complex128), np.zeros(300)   # alive until the request ends
        r6, _ = _req(dev, WAVE, 32, 32, out=o6, steps=100, dt=1e-3, coef=1.0, diag=d6, seed=6)
        dev.default_gate = threading.Event()
        g = srv.submit_raw(r6)
        dev.gates[g], dev.default_gate = dev.default_gate, None
        time.sleep(0.05)
        srv.cancel(g)
        dev.gates[g].set()
        assert srv.wait(g, 20)["status"] == ECANCELED
        assert not [1 for (i, ph, _, _) in dev.log if i == g and ph == 2]
        for rid in (a, b, c, d, f, g):
            srv.release(rid)
        with pytest.raises(fp.FftpdeError):
            srv.poll(a)


def test_server_owned_outputs_come_from_the_pool_and_coalesce(dev):
    """out = NULL: the output lives in the server's pool until release.  Four
    quarter-budget requests, released in an interleaved order, leave a pool
    that must coalesce for a request that needs all of it."""
    fb = field_bytes(32, 32)
    with fp.Server.host(4 * 3 * fb, 4, dev) as srv:   # each request: in + scratch + server-owned out
        ids, xs = [], []
        for k in range(4):
            r, x = _req(dev, POISSON, 32, 32, seed=10 + k)
            ids.append(srv.submit_raw(r))
            xs.append((x, r))
        for rid, (x, r) in zip(ids, xs):
            res = srv.wait(rid, 20)
            assert res["status"] == 0 and res["footprint"] == fb   # the output stays charged
            got = srv.copy_out(rid, np.zeros((32, 32), np.complex128))
            assert np.array_equal(got, _expect(x, r))
        assert srv.stats()["hbm_in_use"] == 4 * fb
        for k in (1, 3, 0, 2):
            srv.release(ids[k])
        assert srv.stats()["hbm_in_use"] == 0
        # one request with in + scratch + out = the whole budget needs the coalesced pool
        r, x = _req(dev, POISSON, 64, 64, seed=20)
        rid = srv.submit_raw(r)
        assert srv.wait(rid, 20)["status"] == 0
        assert np.array_equal(srv.copy_out(rid, np.zeros((64, 64), np.complex128)), _expect(x, r))


def test_autorelease_forgets_the_request(dev):
    with fp.Server.host(1 << 22, 2, dev) as srv:
        r, _ = _req(dev, POISSON, 16, 16, seed=1, flags=fp.AUTORELEASE)
        rid = srv.submit_raw(r)
        deadline = time.time() + 20
        while time.time() < deadline:
            try:
                srv.poll(rid)
            except fp.FftpdeError:
                break
            time.sleep(0.01)
        else:
            pytest.fail("autoreleased request still known")
        st = srv.stats()
        assert st["completed"] == 1 and st["hbm_in_use"] == 0


def test_results_alone_equal_results_in_a_mix(dev):
    """Logged requests of the serving mix (small sides), run together and then
    one at a time: identical outputs and diagnostics."""
    trace = W.serving_trace(seed=5, rate=2000.0, duration=0.03, log2_sides=(4, 6))
    assert len(trace) >= 30

    def build(t, k):
        out = np.zeros((t.ny, t.nx), np.complex128)
        diag = np.zeros(3 * t.steps) if t.kind != POISSON else None
        r, x = _req(dev, t.kind, t.nx, t.ny, out=out, steps=t.steps, dt=t.dt, coef=t.coef, diag=diag, seed=k)
        return r, x, out, diag

    with fp.Server.host(1 << 26, 8, dev) as srv:
        mix = [build(t, k) for k, t in enumerate(trace)]
        ids = [srv.submit_raw(m[0]) for m in mix]
        for rid in ids:
            assert srv.wait(rid, 60)["status"] == 0
        for k, (t, m) in enumerate(zip(trace, mix)):
            alone = build(t, k)
            rid = srv.submit_raw(alone[0])
            assert srv.wait(rid, 20)["status"] == 0
            assert np.array_equal(alone[2], m[2])
            if m[3] is not None:
                assert np.array_equal(alone[3], m[3])
