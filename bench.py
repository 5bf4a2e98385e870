#!/usr/bin/env python3
"""Benchmark: noise-canceling Pauli propagation of the 56-qubit TFIM configuration on one GPU.

One step = one full propagation O -> O~ = D O (backward through 19 gate layers, the first
inverse-noise layer, then 19 forward gate layers each followed by its inverse Pauli-Lindblad
layer) of the 7x8 transverse-field Ising Trotter circuit (10 steps, Clifford ZZ layers at
theta_J = -pi/2, theta_h = 0.5, rates U[1e-4, 2e-3]), observable = mean of Z over the 56
sites, threshold 1e-5, cap 2^24 terms.  Inputs are synthetic and seeded.

Metric: term-updates/s (one live term passed through one layer call), for FP64 coefficients
(`value`) and for FP32 coefficients with compensated merges (`fp32k`), with the dominant
kernel's achieved bandwidth from HIP events against the 8 TB/s HBM peak, and the CPU FP64
reference timed on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME] [--layers]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of the dominant kernels, taken from FETCH_SIZE / WRITE_SIZE counter runs and
# scaled by the same counters read on a plain device copy of known size.  The figure is
# reported only while the kernel sources still hash to the value recorded with it.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gate_tile_tfim7x8_pna.md")
KERNEL_SOURCES = ["paper_2606_20441_amd/csrc/pp_layer.hpp", "paper_2606_20441_amd/csrc/pp_common.hpp",
                  "paper_2606_20441_amd/csrc/pp_gate.hpp", "paper_2606_20441_amd/csrc/pp_misc.hpp",
                  "paper_2606_20441_amd/csrc/pp_sort.hpp",
                  "paper_2606_20441_amd/csrc/pp_api.hip"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(ctx, wl, precision, steps, warmup, layers_verbose=False, progress=False):
    import torch
    from paper_2606_20441_amd import pp

    def one(verbose=False):
        upd = [0]
        io = [0]
        t_layer = [time.perf_counter()]

        def on_layer(step, phase, m, obs):
            st = obs.last_layer_stats()
            upd[0] += st["n_in"]
            io[0] += st["n_in"] + st["n_out"]
            if verbose:
                now = time.perf_counter()
                log(f"  {step:3d} {phase:8s} m={m:2d} in={st['n_in']:>10d} out={st['n_out']:>10d} "
                    f"peak={st['n_peak']:>10d} fallback={st['n_fallback']:>8d} capped={st['n_capped']:>9d} "
                    f"{1e3 * (now - t_layer[0]):8.2f} ms")
                t_layer[0] = now

        obs = pp.run_workload(ctx, wl, precision=precision, on_layer=on_layer)
        e = obs.expectation()
        n = len(obs)
        obs.destroy()
        return upd[0], e, n, io[0]

    for i in range(warmup):
        tw = time.perf_counter()
        one(verbose=layers_verbose and i == 0)
        log(f"   warmup propagation {i + 1}/{warmup}: {1e3 * (time.perf_counter() - tw):.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_upd = 0
    total_io = 0
    res = None
    for i in range(steps):
        u, e, n, q = one(verbose=progress)
        total_upd += u
        total_io += q
        res = (e, n)
        log(f"   timed propagation {i + 1}/{steps} done at {1e3 * (time.perf_counter() - t0):.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel HIP-event timing on the library's stream, in one extra step of its own (the
    # event records and byte counters are kept out of the timed steps above)
    ctx.timing_read(reset=True)
    ctx.timing(True)
    ts = time.perf_counter()
    one(verbose=progress)
    torch.cuda.synchronize()
    log(f"   statistics propagation (HIP events on every launch): {1e3 * (time.perf_counter() - ts):.1f} ms")
    ctx.timing(False)
    kstats = ctx.timing_read(reset=True)
    return dict(seconds=t1 - t0, updates=total_upd, layer_terms_io=total_io, expectation=res[0], terms=res[1],
                kernels=kstats)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str, kernel: str, precision: str):
    """HBM bytes per launch recorded for `kernel` at `precision` on `workload`, or None when
    absent or stale (kernel sources changed since the counters were taken)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    src = kernel_source_hash()
    for line in text.splitlines():
        # machine-readable lines:
        #   "traffic: <workload> <kernel> <precision> <bytes per launch> <source hash>"
        if line.startswith("traffic:"):
            parts = line.split()
            if (len(parts) == 6 and parts[1] == workload and parts[2] == kernel and parts[3] == precision
                    and parts[5] == src):
                return float(parts[4])
    return None


def copy_probe(nbytes: int, reps: int = 5):
    """A plain device-to-device copy of known size: the calibration run for the HBM counters."""
    import torch
    n = nbytes // 4
    a = torch.arange(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    assert bool((b[-1] == n - 1).item())
    log(f"copy probe: {reps} copies of {n * 4} bytes")


def copy_ceiling(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Measured device copy bandwidth (bytes read + written per second, GB/s): the practical
    HBM ceiling of this machine, reported beside the vendor peak."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def roofline(kstats, workload, precision="f64", copy_gbs=None):
    """The dominant kernel (largest device time) against the HBM roofline.

    `achieved` counts the algorithmic bytes of the work unit: a layer call reads its input
    terms once and writes its output terms once, (N_in + N_out) B.  A kernel that applies one
    gate per pass over the whole array is charged 1/G of its layer's bytes per pass (G gates
    in that layer call); per-gate re-reads are overhead.  The per-pass rate (every pass
    counted as one read and one write of what it handled) is reported beside it as
    `pass_gbs`, and the counted DRAM traffic (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy's counters) as `traffic` per launch."""
    timed = [k for k in kstats if k["total_ms"] > 0]
    total = sum(k["total_ms"] for k in timed)
    dom = max(timed, key=lambda k: k["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    layer_bytes = dom["layer_bytes"] / dom["launches"]
    pass_bytes = dom["algo_bytes"] / dom["launches"]
    achieved = layer_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    pass_gbs = pass_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = recorded_traffic(workload, dom["name"], precision)
    out = {"bound": "hbm", "kernel": dom["name"], "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
           "traffic": None if traffic is None else round(traffic),
           "algo_bytes_per_launch": round(layer_bytes),
           "avg_launch_ms": round(avg_ms, 4), "launches": dom["launches"],
           "share_of_device_time": round(dom["total_ms"] / total, 3),
           "pass_bytes_per_launch": round(pass_bytes), "pass_gbs": round(pass_gbs, 1),
           "pass_frac": round(pass_gbs / HBM_PEAK_GBS, 4)}
    if traffic is not None and avg_ms > 0:
        tg = traffic / (avg_ms * 1e-3) / 1e9   # counted DRAM bytes per second
        out["traffic_gbs"] = round(tg, 1)
        out["traffic_frac"] = round(tg / HBM_PEAK_GBS, 4)
        out["traffic_over_pass_bytes"] = round(traffic / pass_bytes, 3) if pass_bytes else None
    if copy_gbs:
        out["copy_ceiling_gbs"] = round(copy_gbs, 1)
        out["pass_frac_of_copy"] = round(pass_gbs / copy_gbs, 4)
    return out


def noisy_check(ctx, wl, precision):
    """Propagate O~ back through the noisy circuit (the check that the mitigated observable
    recovers the ideal value): Tr[O~ rho_noisy], its time and term-updates/s, once."""
    import torch
    from paper_2606_20441_amd import pp
    obs = pp.run_workload(ctx, wl, precision=precision)
    torch.cuda.synchronize()
    upd = [0]

    def on_layer(m, o):
        upd[0] += o.last_layer_stats()["n_in"]

    t0 = time.perf_counter()
    v = pp.noisy_evaluation(wl.circuit, obs, on_layer=on_layer)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = len(obs)
    obs.destroy()
    log(f"   noisy evaluation: Tr[O~ rho_noisy] = {v!r} in {1e3 * dt:.1f} ms ({upd[0] / dt:.4g} term-updates/s)")
    return {"value": v, "ms": round(1e3 * dt, 3), "term_updates_per_s": round(upd[0] / dt, 1), "terms_out": n}


def pna_walk(ctx, steps: int, eps: float, cap: int, eps_fwd: float, cap_fwd: int, kmax: int,
             forward: str = "batched", weights: bool = False):
    """One propagated-noise-absorption walk (Section I.A) on the headline lattice, angles
    and noise at `steps` Trotter steps: every generator's error carried forward through the
    later gates (a layer's errors together, forward="batched"; threshold eps_fwd, each E'
    cut to its cap_fwd largest terms before it is absorbed), then absorbed into O one update
    per generator, E' O E' limited to its kmax most significant products when kmax > 0
    (Appendix B), O thresholded at eps and capped at `cap` after every update.  Timed whole,
    uninstrumented, with one progress line per layer.  weights=True also reads every E' back
    and reports how much of its unit weight (sum of c^2; conjugation by the later gates keeps
    it at 1) the forward threshold and cap removed; that read-back is inside the timing."""
    import numpy as np
    import torch
    from paper_2606_20441_amd import pp, workloads as W
    wl = W.named_workload("tfim7x8_pna", steps=steps)
    circ = wl.circuit
    n_maps = sum(l.n_gen for l in circ.layers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seen = {"t": -1}

    lost = {"sum": 0.0, "max": 0.0, "n": 0}

    def on_map(t, k, obs):
        if t != seen["t"] and k == circ.layers[t].n_gen - 1:
            seen["t"] = t
            extra = ""
            if weights:
                extra = (f", E' weight lost: mean {lost['sum'] / max(1, lost['n']):.2e}, "
                         f"max {lost['max']:.2e}")
            log(f"   PNA walk: layer {t + 1}/{len(circ.layers)} absorbed at {time.perf_counter() - t0:.1f} s, "
                f"|O| = {len(obs)}, <O~> = {obs.expectation():.6g}{extra}")

    def on_error(t, k, e):
        c = e.export()[2]
        d = 1.0 - float(np.dot(c, c))
        lost["sum"] += d
        lost["max"] = max(lost["max"], d)
        lost["n"] += 1

    g = pp.pna(ctx, circ, wl.observable, eps=eps, max_terms=cap, eps_fwd=eps_fwd, max_terms_fwd=cap_fwd,
               max_products=kmax, forward=forward, on_map=on_map, on_error=on_error if weights else None)
    v = g.expectation()
    n_out = len(g)
    g.destroy()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {"workload": f"tfim7x8_pna at {steps} Trotter steps: 56q, {len(circ.layers)} layers, {n_maps} maps; "
                       f"K_O {cap or 'none'}, eps {eps:g}; K_E {cap_fwd or 'none'}, forward eps {eps_fwd:g}, "
                       f"{forward} forward propagation; products per map {kmax or 'all'}",
           "maps": n_maps, "ms": round(1e3 * dt, 1), "maps_per_s": round(n_maps / dt, 1), "expectation": v,
           "terms_out": n_out}
    if weights:
        res["eprime_weight_lost"] = {"mean": lost["sum"] / max(1, lost["n"]), "max": lost["max"]}
    log(f"   PNA walk: {n_maps} maps in {dt:.1f} s ({n_maps / dt:.0f} maps/s), <O~> = {v!r}, {n_out} terms")
    return res


def pna_check(ctx, cpu: bool, prefix_maps: int = 300, topk=(), batches=()):
    """Propagated noise absorption (Section I.A) on the same 7x8 lattice, angles and noise
    as the headline workload at 2 Trotter steps (4 layers, 4164 generators): every
    generator's error propagated forward through the later gates on the device (threshold
    1e-4), then absorbed into O (threshold 1e-5), one update per generator.  Timed whole,
    uninstrumented, once, and again with per-launch HIP events for the kernel breakdown; the
    oracle and the device are also timed on the same prefix of the walk.  Each
    value in `topk` reruns the walk with E' O E' limited to that many most significant
    products (Appendix B), and each (C, order) in `batches` reruns it with the maps of a
    layer absorbed C at a time to that order in the number of errors (Appendix C); both
    report their time and the shift of <O~> from the exact walk."""
    import torch
    from paper_2606_20441_amd import pp, workloads as W
    wl = W.named_workload("tfim7x8_pna", steps=2)
    eps, eps_fwd = wl.eps, 1e-4
    circ = wl.circuit
    n_maps = sum(l.n_gen for l in circ.layers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = pp.pna(ctx, circ, wl.observable, eps=eps, eps_fwd=eps_fwd)
    v = g.expectation()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_out = len(g)
    g.destroy()
    # kernel breakdown from a second walk with HIP events around every launch (slower)
    ctx.timing(True)
    ctx.timing_read(reset=True)
    pp.pna(ctx, circ, wl.observable, eps=eps, eps_fwd=eps_fwd).destroy()
    torch.cuda.synchronize()
    ks = ctx.timing_read(reset=True)
    ctx.timing(False)
    top = sorted(ks, key=lambda k: -k["total_ms"])[:6]
    out = {"workload": "tfim7x8_pna at 2 Trotter steps: 56q, 4 layers, eps 1e-5, forward eps 1e-4, no cap",
           "maps": n_maps, "ms": round(1e3 * dt, 1), "maps_per_s": round(n_maps / dt, 1), "expectation": v,
           "terms_out": n_out,
           "kernels": [{"name": k["name"], "launches": k["launches"], "total_ms": round(k["total_ms"], 2)} for k in top]}
    log(f"   PNA: {n_maps} maps in {1e3 * dt:.0f} ms ({n_maps / dt:.0f} maps/s), <O~> = {v!r}, {n_out} terms")
    for k in top:
        log(f"      {k['name']:24s} {k['launches']:6d} launches {k['total_ms']:9.2f} ms")
    out["topk"] = []
    for mp in topk:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gk = pp.pna(ctx, circ, wl.observable, eps=eps, eps_fwd=eps_fwd, max_products=int(mp))
        vk = gk.expectation()
        torch.cuda.synchronize()
        dk = time.perf_counter() - t0
        out["topk"].append({"max_products": int(mp), "ms": round(1e3 * dk, 1), "expectation": vk,
                            "abs_shift_vs_exact": abs(vk - v), "terms_out": len(gk)})
        gk.destroy()
        log(f"   PNA, at most {int(mp)} products per map: {1e3 * dk:.0f} ms, <O~> = {vk!r} (shift {abs(vk - v):.3e})")
    out["batches"] = []
    for C_, order in batches:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gb = pp.pna(ctx, circ, wl.observable, eps=eps, eps_fwd=eps_fwd, batch=int(C_), batch_order=int(order))
        vb = gb.expectation()
        torch.cuda.synchronize()
        db = time.perf_counter() - t0
        out["batches"].append({"batch": int(C_), "order": int(order), "ms": round(1e3 * db, 1), "expectation": vb,
                               "abs_shift_vs_exact": abs(vb - v), "terms_out": len(gb)})
        gb.destroy()
        log(f"   PNA, batches of {int(C_)} to order {int(order)}: {1e3 * db:.0f} ms, <O~> = {vb!r} (shift {abs(vb - v):.3e})")
    if cpu:
        from oracle import oracle
        maps = [(t, k) for t, l in enumerate(circ.layers) for k in range(l.n_gen)][:prefix_maps]
        t0 = time.perf_counter()
        o = oracle.OracleSum.from_sum(wl.observable)
        for t, k in maps:
            o.antinoise(oracle.propagated_error(circ, t, k, eps_fwd), oracle.antinoise_q(circ.layers[t].lam[k]))
            o.truncate(eps, 0)
        t_cpu = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gg = pp.Observable.from_sum(ctx, wl.observable, eps=eps)
        for t, k in maps:
            e = pp.propagated_error(ctx, circ, t, k, eps_fwd)
            gg.apply_antinoise(e, circ.layers[t].lam[k])
            e.destroy()
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
        same = abs(gg.expectation() - o.expectation())
        gg.destroy()
        out["cpu_baseline"] = {"kind": "oracle", "cores": 1, "maps": len(maps),
                               "sample": f"the first {len(maps)} maps of the walk (errors of the first layer, carried through 3 layers)",
                               "oracle_s": round(t_cpu, 3), "gpu_s": round(t_gpu, 3),
                               "maps_per_s": round(len(maps) / t_cpu, 2), "abs_diff_expectation": same}
        log(f"   PNA prefix of {len(maps)} maps: oracle {t_cpu:.2f} s, device {t_gpu:.3f} s, |d<O~>| = {same:.2e}")
    return out


def sine_order_check(ctx, wl, orders):
    """The headline propagation in the sine-order mode (Euclid appendix, CPT order), circuit
    in the Clifford interaction picture, for each tag limit K: time, term count and <O~>."""
    import torch
    from paper_2606_20441_amd import pp
    ip = wl.circuit   # the library writes it in the interaction picture
    out = []
    for K in orders:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = pp.noise_canceling(ctx, ip, wl.observable, eps=wl.eps, max_terms=wl.max_terms, mode="sine_order",
                               max_order=int(K))
        v = g.expectation()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.append({"max_sine_order": int(K), "ms": round(1e3 * dt, 1), "terms_out": len(g), "expectation": v})
        log(f"   sine order <= {int(K)}: {1e3 * dt:.0f} ms, {len(g)} terms, <O~> = {v!r}")
        g.destroy()
    return out


def _cpu_sample(wl, budget_s):
    """The FP64 CPU reference (one thread) on a bounded prefix of the propagation: layer calls
    in the same order until the time budget is spent.  Returns (term-updates, seconds, calls)."""
    from oracle import oracle
    c = wl.circuit
    M = len(c.layers)
    mode = 1 if wl.mode == "error_order" else 0
    s = oracle.OracleSum.from_sum(wl.observable)
    calls = [(m, +1, True, False) for m in range(M - 1, 0, -1)] + [(0, -1, False, True)] + \
            [(m, -1, True, True) for m in range(1, M)]
    t0 = time.perf_counter()
    upd = 0
    done = 0
    last = prev = 0.0
    for m, d, g, nz in calls:
        n_in = len(s)
        spent = time.perf_counter() - t0
        # stop before a call whose predicted time (the last call's, grown by the last ratio)
        # would take the sample past twice the budget
        predicted = last * max(1.0, last / prev) if prev > 0 else last
        if done and (spent > budget_s or spent + predicted > 2.0 * budget_s):
            break
        t_call = time.perf_counter()
        s.apply_layer(c.layers[m], d, with_gates=g, with_noise=nz, eps=wl.eps, max_terms=wl.max_terms,
                      mode=mode, max_order=wl.max_order)
        prev, last = last, time.perf_counter() - t_call
        upd += n_in
        done += 1
    return upd, time.perf_counter() - t0, done, len(calls)


def _host_cpu():
    """Host CPU facts for the report: logical CPUs, CPUs this process may run on, model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "allowed_cpus": allowed, "model": model}


def cpu_baseline(wl, workload, max_terms, budget_s=15.0, workers=16):
    """The oracle as it stands (single-threaded C++) on the host's cores: `workers` processes
    (the machine's CPU share, at most the CPUs this process may use), each running the same
    bounded prefix of the propagation at once; the value is their summed term-updates over
    the wall time of the set.  One worker's own rate is reported beside it."""
    import subprocess
    host = _host_cpu()
    p = max(1, min(workers, host["allowed_cpus"]))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", "--workload", workload,
           "--cpu-budget", str(budget_s), "--trotter-steps", str(len(wl.circuit.layers) // 2)]
    if max_terms is not None:
        cmd += ["--max-terms", str(max_terms)]
    t0 = time.perf_counter()
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True) for _ in range(p)]
    outs = [json.loads(pr.communicate()[0].strip().splitlines()[-1]) for pr in procs]
    wall = time.perf_counter() - t0
    if any(pr.returncode for pr in procs):
        raise RuntimeError("a CPU reference worker failed")
    upd = sum(o["updates"] for o in outs)
    one = outs[0]
    return {"value": round(upd / wall, 1), "unit": "term-updates/s", "cores": p, "kind": "oracle",
            "sample": f"{p} concurrent single-threaded oracle processes, each the first {one['calls']} of "
                      f"{one['of']} layer calls of the same propagation ({one['updates']} term-updates, "
                      f"{one['seconds']:.1f} s); {upd} term-updates in {wall:.1f} s wall",
            "single_thread_value": round(one["updates"] / one["seconds"], 1),
            "host": host}


def run_serving(n_requests: int, rate_hz: float, n_slots: int, warmup: int):
    """The serving form: a seeded Poisson stream of mixed propagation requests replayed
    against the wall clock; latency is arrival to result."""
    from paper_2606_20441_amd import serve, workloads as W
    reqs = W.serving_stream(n_requests + warmup, rate_hz=rate_hz)
    srv = serve.Server(n_slots=n_slots, hbm_budget_bytes=200 * 10**9)
    done = [0]

    def on_done(res):
        done[0] += 1
        if done[0] % 10 == 0 or done[0] == len(reqs):
            log(f"   served {done[0]}/{len(reqs)} (last: request {res.rid}, {res.status}, "
                f"latency {1e3 * res.latency:.0f} ms)")

    try:
        out = srv.run(reqs, on_done=on_done)
    finally:
        srv.close()
    measured = [r for r in out if r.rid >= warmup]
    s = serve.summarize(measured, rate_hz)
    s.update({"slots": n_slots, "warmup_requests": warmup, "hbm_budget_bytes": 200 * 10**9,
              "peak_reserved_bytes": srv.sched.peak_reserved, "peak_running": srv.sched.peak_running})
    return s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tfim7x8_pna")
    ap.add_argument("--precision", default="both", choices=["both", "f64", "f32k"])
    ap.add_argument("--layers", action="store_true", help="print per-layer counts of the first warmup step")
    ap.add_argument("--progress", action="store_true", help="print per-layer counts of the timed steps too")
    ap.add_argument("--max-terms", type=int, default=None, help="override the workload's cap")
    ap.add_argument("--trotter-steps", type=int, default=None, help="override the workload's Trotter steps")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-noisy-check", action="store_true",
                    help="skip propagating O~ back through the noisy circuit")
    ap.add_argument("--no-pna", action="store_true", help="skip the propagated-noise-absorption leg")
    ap.add_argument("--pna-only", action="store_true", help="run only the propagated-noise-absorption leg")
    ap.add_argument("--pna-topk", default="", help="comma-separated product limits for extra PNA walks")
    ap.add_argument("--pna-batch", default="", help="comma-separated C:order pairs for batched PNA walks")
    ap.add_argument("--pna-walk", action="store_true",
                    help="run only one PNA walk with the --pna-* settings below and print its JSON")
    ap.add_argument("--pna-steps", type=int, default=10)
    ap.add_argument("--pna-eps", type=float, default=1e-5)
    ap.add_argument("--pna-cap", type=int, default=1 << 16, help="K_O: terms kept in O after every update")
    ap.add_argument("--pna-eps-fwd", type=float, default=1e-4)
    ap.add_argument("--pna-fwd-cap", type=int, default=256, help="K_E: terms kept in each evolved error")
    ap.add_argument("--pna-kmax", type=int, default=1 << 18, help="most significant products per update (0: all)")
    ap.add_argument("--pna-forward", default="each", choices=["batched", "each"],
                    help="each: every error alone, K_E after every non-Clifford gate; batched: 256 "
                         "errors of a layer together, K_E once at the end")
    ap.add_argument("--pna-weights", action="store_true",
                    help="read every evolved error back and report the weight its truncation removed")
    ap.add_argument("--sine-orders", default="", help="comma-separated CPT-order limits: run only the "
                    "workload in the sine-order mode for each")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="concurrent CPU reference processes (the box's CPU share)")
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--serve-requests", type=int, default=30,
                    help="measured requests of the serving stream per arrival rate (0: skip it)")
    ap.add_argument("--serve-rates", default="200,0.5",
                    help="arrival rates (req/s): the configured one and one the device sustains")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving stream (--serve-requests measured after --serve-warmup, "
                         "at each of --serve-rates) and print its JSON")
    ap.add_argument("--serve-warmup", type=int, default=10)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args()
    if args.cpu_worker:
        # one CPU reference process of the baseline (no GPU use): prints its sample as JSON
        from paper_2606_20441_amd import workloads as W
        over = {} if args.max_terms is None else {"max_terms": args.max_terms}
        if args.trotter_steps is not None:
            over["steps"] = args.trotter_steps
        wl = W.named_workload(args.workload, **over)
        u, dt, done, of = _cpu_sample(wl, args.cpu_budget)
        print(json.dumps({"updates": u, "seconds": dt, "calls": done, "of": of}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_20441_amd import pp, workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    pp.lib()
    over = {} if args.max_terms is None else {"max_terms": args.max_terms}
    if args.trotter_steps is not None:
        over["steps"] = args.trotter_steps
    wl = W.named_workload(args.workload, **over)
    ctx = pp.Context(0)
    if args.sine_orders:
        so = sine_order_check(ctx, wl, [int(v) for v in args.sine_orders.split(",") if v])
        print(json.dumps({"sine_order": so, "workload": args.workload}), flush=True)
        ctx.close()
        return
    if args.serve_only:
        out = []
        for rate in [float(r) for r in args.serve_rates.split(",") if r]:
            log(f"== serving: {args.serve_requests} requests after {args.serve_warmup} at {rate:g}/s, "
                f"{args.serve_slots} slots")
            t0 = time.perf_counter()
            res = run_serving(args.serve_requests, rate, args.serve_slots, args.serve_warmup)
            res["wall_s"] = round(time.perf_counter() - t0, 1)
            out.append(res)
            log(f"   {res}")
        print(json.dumps({"serving": out}), flush=True)
        return
    if args.pna_walk:
        res = pna_walk(ctx, args.pna_steps, args.pna_eps, args.pna_cap, args.pna_eps_fwd, args.pna_fwd_cap,
                       args.pna_kmax, args.pna_forward, args.pna_weights)
        print(json.dumps({"pna_walk": res}), flush=True)
        ctx.close()
        return
    if args.pna_only:
        tk = [int(v) for v in args.pna_topk.split(",") if v]
        bt = [tuple(int(x) for x in v.split(":")) for v in args.pna_batch.split(",") if v]
        print(json.dumps({"pna": pna_check(ctx, not args.no_cpu, topk=tk, batches=bt)}), flush=True)
        ctx.close()
        return
    Wd = wl.circuit.W
    results = {}
    copy_gbs = copy_ceiling()
    log(f"device copy ceiling: {copy_gbs:.0f} GB/s (read + write)")
    precs = ["f64", "f32k"] if args.precision == "both" else [args.precision]
    for prec in precs:
        log(f"== {args.workload} {prec}: warmup {args.warmup}, steps {args.steps}")
        r = run_gpu(ctx, wl, prec, args.steps, args.warmup, layers_verbose=args.layers, progress=args.progress)
        tb = 16 * Wd + (8 if prec == "f64" else 4) + (1 if wl.mode == "error_order" else 0)
        r["term_bytes"] = tb
        r["roofline"] = roofline(r["kernels"], args.workload, prec, copy_gbs)
        r["step_algo_gbs"] = tb * r["layer_terms_io"] / r["seconds"] / 1e9
        results[prec] = r
        log(f"   {r['updates'] / r['seconds']:.4g} term-updates/s, {1e3 * r['seconds'] / args.steps:.1f} ms/step, "
            f"<O> = {r['expectation']!r}, {r['terms']} terms")
        for k in sorted(r["kernels"], key=lambda k: -k["total_ms"])[:20]:
            avg = k["total_ms"] / k["launches"]
            bw = k["algo_bytes"] / k["launches"] / (avg * 1e-3) / 1e9 if avg > 0 and k["algo_bytes"] else 0
            log(f"   {k['name']:24s} {k['launches']:6d} launches {k['total_ms']:9.2f} ms  avg {avg:8.4f} ms  "
                f"algo {bw:8.1f} GB/s")
    main_prec = precs[0]
    noisy = noisy_check(ctx, wl, main_prec) if not args.no_noisy_check else None
    pna = pna_check(ctx, not args.no_cpu) if not args.no_pna else None
    r = results[main_prec]
    value = r["updates"] / r["seconds"]
    line = {
        "metric": "Pauli-term updates/s + HBM GB/s (56q TFIM, FP64 vs FP32); p50/p99 latency",
        "value": round(value, 1),
        "unit": "term-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["seconds"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.circuit.n_qubits}q "
                               f"{'x'.join(wl.circuit.name.split('_')[1:2])} TFIM, {len(wl.circuit.layers) // 2} Trotter steps, "
                               f"eps {wl.eps:g}, cap {wl.max_terms}, {wl.mode}",
                   "terms_out": r["terms"], "expectation": r["expectation"],
                   "term_updates_per_step": r["updates"] // args.steps, "parallelism": "1 GPU"},
        "roofline": r["roofline"],
        "step_algo": {"gbs": round(r["step_algo_gbs"], 2), "frac": round(r["step_algo_gbs"] / HBM_PEAK_GBS, 5),
                      "bytes_per_step": int(r["term_bytes"] * r["layer_terms_io"] / args.steps),
                      "note": "sum over the layer calls of (N_in + N_out) x term bytes, over ms_per_step"},
    }
    if noisy is not None:
        line["noisy_evaluation"] = noisy
    if pna is not None:
        line["pna"] = pna
    if "f32k" in results and main_prec != "f32k":
        f = results["f32k"]
        line["fp32k"] = {"value": round(f["updates"] / f["seconds"], 1),
                         "ms_per_step": round(1e3 * f["seconds"] / args.steps, 3),
                         "speedup_vs_f64": round(r["seconds"] / f["seconds"], 3),
                         "expectation": f["expectation"],
                         "abs_err_vs_f64_gpu": abs(f["expectation"] - r["expectation"]),
                         "step_algo_gbs": round(f["step_algo_gbs"], 2),
                         "roofline": f["roofline"]}
    if args.serve_requests > 0:
        line["serving"] = []
        for rate in [float(r) for r in args.serve_rates.split(",") if r]:
            log(f"== serving: {args.serve_requests} requests at {rate:g}/s, {args.serve_slots} slots")
            res = run_serving(args.serve_requests, rate, args.serve_slots, args.serve_warmup)
            line["serving"].append(res)
            log(f"   {res}")
    if not args.no_cpu:
        log("== CPU reference sample")
        line["cpu_baseline"] = cpu_baseline(wl, args.workload, args.max_terms, args.cpu_budget, args.cpu_workers)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
