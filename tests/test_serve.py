"""Serving loop: admission and overlap on the CPU with a fake executor; on the GPU, a
request's result alone equals its result in a mix, and a request that outgrows its
reservation fails alone."""
import threading
import time

import numpy as np
import pytest

from tests.parity import compare_exports, oracle_layer_step

from paper_2606_20441_amd import serve, workloads as W


class _Req:
    def __init__(self, rid, arrival, wl):
        self.rid, self.arrival_s, self.workload = rid, arrival, wl


class _WL:
    """Just enough of a workload for the reservation rule."""

    def __init__(self, n_qubits=16, cap=1 << 10, precision="f64", mode="greedy", name="w"):
        class _C:
            pass
        self.circuit = _C()
        self.circuit.n_qubits = n_qubits
        self.max_terms, self.precision, self.mode, self.name = cap, precision, mode, name


def test_reservation_rule():
    wl = _WL(n_qubits=56, cap=1 << 22)
    assert serve.term_bytes(56, "f64", "greedy") == 24
    assert serve.term_bytes(128, "f32k", "greedy") == 36
    assert serve.term_bytes(56, "f64", "error_order") == 25
    assert serve.reservation_bytes(wl) == int(32.0 * (1 << 22) * 24)
    assert serve.reservation_bytes(_WL(cap=1)) == 1 << 30   # floor


def test_scheduler_fifo_slots_budget_reject():
    reserve = lambda wl: wl.max_terms
    s = serve.Scheduler(n_slots=2, budget_bytes=100, reserve=reserve)
    reqs = [_Req(i, 0.0, _WL(cap=c)) for i, c in enumerate([40, 50, 60, 20])]
    for r in reqs:
        assert s.offer(r) is None
    assert s.offer(_Req(9, 0.0, _WL(cap=101))) == "rejected"
    got = s.admit()
    assert [r.rid for _, r, _ in got] == [0, 1]          # two slots
    assert s.running == 2 and s.reserved == 90
    assert s.admit() == []                               # no slot
    s.release(got[0][0], 40)
    got2 = s.admit()
    assert got2 == []                                    # head (60) does not fit in 100 - 50
    s.release(got[1][0], 50)
    got3 = s.admit()
    assert [r.rid for _, r, _ in got3] == [2, 3]         # arrival order kept
    assert s.peak_reserved <= 100


def test_server_overlap_and_deferral_with_fake_executor():
    lock = threading.Lock()
    live = {"now": 0, "peak": 0}

    def fake(slot, req, need, res):
        with lock:
            live["now"] += 1
            live["peak"] = max(live["peak"], live["now"])
        time.sleep(0.05)
        with lock:
            live["now"] -= 1
        res.status = "ok"
        res.expectation = float(req.rid)
        res.term_updates = 10

    reserve = lambda wl: wl.max_terms
    reqs = [_Req(i, 0.002 * i, _WL(cap=30)) for i in range(12)]
    reqs.append(_Req(99, 0.0, _WL(cap=1000)))             # larger than the budget
    srv = serve.Server(n_slots=4, hbm_budget_bytes=90, executor=fake, reserve=reserve)
    out = srv.run(reqs)
    by = {r.rid: r for r in out}
    assert by[99].status == "rejected"
    ok = [r for r in out if r.status == "ok"]
    assert len(ok) == 12
    assert all(r.expectation == r.rid for r in ok)
    assert live["peak"] == 3                              # budget 90 admits three of 30 at once
    assert srv.sched.peak_reserved <= 90
    for r in ok:
        assert r.admitted >= r.arrival - 1e-9 and r.finished >= r.admitted + 0.045
    s = serve.summarize(out, offered_rate=500.0)
    assert s["ok"] == 12 and s["rejected"] == 1
    assert s["p99_latency_ms"] >= s["p50_latency_ms"] >= 45.0
    assert s["term_updates_per_s"] > 0


def test_server_continuous_admission():
    """A request arriving while others run starts when a slot frees, not after a batch."""
    def fake(slot, req, need, res):
        time.sleep(0.2 if req.rid == 0 else 0.02)
        res.status = "ok"

    reqs = [_Req(0, 0.0, _WL()), _Req(1, 0.0, _WL()), _Req(2, 0.05, _WL())]
    srv = serve.Server(n_slots=2, hbm_budget_bytes=10**12, executor=fake)
    out = {r.rid: r for r in srv.run(reqs)}
    # request 2 arrives after 1 finished and takes its slot while 0 is still running
    assert out[2].admitted < out[0].finished
    assert out[2].finished < out[0].finished


def _small_stream(n, seed=7):
    return W.serving_stream(n, rate_hz=1000.0, seed_arrivals=seed, seed_requests=seed + 1,
                            rows=(3, 4), cols=(3, 5), steps=(2, 3), max_terms=1 << 16)


@pytest.mark.gpu
def test_serving_alone_equals_mix_and_oracle():
    from oracle import oracle
    reqs = _small_stream(8)
    alone = serve.Server(n_slots=1, hbm_budget_bytes=200 * 10**9)
    try:
        ra = {r.rid: r for r in alone.run(reqs, time_scale=0.0)}
    finally:
        alone.close()
    mix = serve.Server(n_slots=4, hbm_budget_bytes=200 * 10**9)
    try:
        rm = {r.rid: r for r in mix.run(reqs, time_scale=0.0)}
    finally:
        mix.close()
    assert mix.sched.peak_running > 1
    from paper_2606_20441_amd import pp
    ctx = pp.Context(0)
    try:
        for r in reqs:
            a, m = ra[r.rid], rm[r.rid]
            assert a.status == "ok" and m.status == "ok", (a.message, m.message)
            assert a.n_terms == m.n_terms
            assert a.expectation == m.expectation        # deterministic kernels: bit-identical
            wl = r.workload
            if wl.precision != "f64":
                continue
            # The same request through the library directly, with the reference fed the
            # device's terms before every layer call (the two round the noise products in a
            # different order, so an unfed walk may put a term within an ulp of the threshold
            # or of a cut on different sides): every call term by term, and the end result
            # equal to the served one bit for bit.
            state = [None]
            n = wl.circuit.n_qubits
            g0 = pp.Observable.from_sum(ctx, wl.observable, eps=wl.eps, max_terms=wl.max_terms)
            state[0] = g0.export()
            g0.destroy()

            def on_layer(step, kind, mm, obs, wl=wl, n=n, state=state, rid=r.rid):
                ref = oracle_layer_step(oracle, n, state[0], wl, kind, mm)
                got = obs.export()
                rr = ref.export()
                cut = float(np.abs(rr[2]).min()) if len(rr[2]) else 0.0
                compare_exports(got, rr, thresholds=[wl.eps, cut], context=f"request {rid} call {step}")
                assert abs(obs.expectation() - ref.expectation()) < 1e-10
                state[0] = got

            d = pp.run_workload(ctx, wl, on_layer=on_layer)
            assert d.expectation() == a.expectation, (r.rid, d.expectation(), a.expectation)
            d.destroy()
    finally:
        ctx.close()


@pytest.mark.gpu
def test_serving_oom_fails_alone():
    reqs = _small_stream(4, seed=11)
    victim = reqs[1].workload.name
    reserve = lambda wl: 4096 if wl.name == victim else serve.reservation_bytes(wl)
    srv = serve.Server(n_slots=2, hbm_budget_bytes=200 * 10**9, reserve=reserve)
    try:
        out = {r.rid: r for r in srv.run(reqs, time_scale=0.0)}
    finally:
        srv.close()
    assert out[reqs[1].rid].status == "oom"
    assert all(out[r.rid].status == "ok" for r in reqs if r.rid != reqs[1].rid)
    assert srv.sched.reserved == 0


@pytest.mark.gpu
def test_serving_budget_defers_on_device():
    """The HBM budget binds on the device: with room for two reservations, four slots and
    six requests arriving at once, at most two run together; each later request is admitted
    only when an earlier one has finished and returned its memory; every result equals the
    same request served alone."""
    reqs = _small_stream(6, seed=21)
    need = 1 << 30                                      # the reservation floor of these requests
    assert all(serve.reservation_bytes(r.workload) == need for r in reqs)
    srv = serve.Server(n_slots=4, hbm_budget_bytes=int(2.5 * need))
    try:
        out = srv.run(reqs, time_scale=0.0)
    finally:
        srv.close()
    assert all(r.status == "ok" for r in out), [r.message for r in out]
    assert srv.sched.peak_running == 2 and srv.sched.peak_reserved == 2 * need
    by_admit = sorted(out, key=lambda r: r.admitted)
    for k, r in enumerate(by_admit[2:], start=2):
        # two reservations at most: someone admitted earlier had finished by then
        assert any(o.finished <= r.admitted + 1e-6 for o in by_admit[:k]), r.rid
    alone = serve.Server(n_slots=1, hbm_budget_bytes=200 * 10**9)
    try:
        ra = {r.rid: r for r in alone.run(reqs, time_scale=0.0)}
    finally:
        alone.close()
    for r in out:
        assert r.expectation == ra[r.rid].expectation and r.n_terms == ra[r.rid].n_terms
