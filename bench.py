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
        t_layer = [time.perf_counter()]

        def on_layer(step, phase, m, obs):
            st = obs.last_layer_stats()
            upd[0] += st["n_in"]
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
        return upd[0], e, n

    for i in range(warmup):
        one(verbose=layers_verbose and i == 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_upd = 0
    res = None
    for _ in range(steps):
        u, e, n = one(verbose=progress)
        total_upd += u
        res = (e, n)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel HIP-event timing on the library's stream, in one extra step of its own (the
    # event records and byte counters are kept out of the timed steps above)
    ctx.timing_read(reset=True)
    ctx.timing(True)
    one()
    torch.cuda.synchronize()
    ctx.timing(False)
    kstats = ctx.timing_read(reset=True)
    return dict(seconds=t1 - t0, updates=total_upd, expectation=res[0], terms=res[1], kernels=kstats)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, precision: str):
    """HBM bytes per launch recorded for `kernel` at `precision`, or None when absent or stale."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    src = kernel_source_hash()
    for line in text.splitlines():
        # machine-readable lines: "traffic: <kernel> <precision> <bytes per launch> <source hash>"
        if line.startswith("traffic:"):
            parts = line.split()
            if len(parts) == 5 and parts[1] == kernel and parts[2] == precision and parts[4] == src:
                return float(parts[3])
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


def roofline(kstats, term_bytes, precision="f64", copy_gbs=None):
    timed = [k for k in kstats if k["total_ms"] > 0]
    total = sum(k["total_ms"] for k in timed)
    dom = max(timed, key=lambda k: k["total_ms"])
    fused = next((k for k in timed if k["name"] == "layer_fused_wave"), None)
    pick = dom
    avg_ms = pick["total_ms"] / pick["launches"]
    per_launch_bytes = pick["algo_bytes"] / pick["launches"]
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = recorded_traffic(pick["name"], precision)
    out = {"bound": "hbm", "kernel": pick["name"], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": None if traffic is None else round(traffic),
           "algo_bytes_per_launch": round(per_launch_bytes),
           "share_of_device_time": round(pick["total_ms"] / total, 3),
           "avg_launch_ms": round(avg_ms, 4), "launches": pick["launches"]}
    if traffic is not None and avg_ms > 0:
        tg = traffic / (avg_ms * 1e-3) / 1e9   # counted DRAM bytes per second
        out["traffic_gbs"] = round(tg, 1)
        out["traffic_frac"] = round(tg / HBM_PEAK_GBS, 4)
    if copy_gbs:
        out["copy_ceiling_gbs"] = round(copy_gbs, 1)
        out["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if fused is not None and fused is not pick:
        f_ms = fused["total_ms"] / fused["launches"]
        f_ach = fused["algo_bytes"] / fused["launches"] / (f_ms * 1e-3) / 1e9
        out["layer_fused_wave"] = {"achieved": round(f_ach, 1), "frac": round(f_ach / HBM_PEAK_GBS, 4),
                              "avg_launch_ms": round(f_ms, 4), "share_of_device_time": round(fused["total_ms"] / total, 3)}
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


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 CPU reference (single thread) on a bounded prefix of the same propagation:
    layer calls in the same order until the time budget is spent."""
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
    dt = time.perf_counter() - t0
    return {"value": round(upd / dt, 1), "unit": "term-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {len(calls)} layer calls of the same propagation ({upd} term-updates, {dt:.1f} s)"}


def run_serving(n_requests: int, rate_hz: float, n_slots: int, warmup: int):
    """The serving form: a seeded Poisson stream of mixed propagation requests replayed
    against the wall clock; latency is arrival to result."""
    from paper_2606_20441_amd import serve, workloads as W
    reqs = W.serving_stream(n_requests + warmup, rate_hz=rate_hz)
    srv = serve.Server(n_slots=n_slots, hbm_budget_bytes=200 * 10**9)
    try:
        out = srv.run(reqs)
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
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-noisy-check", action="store_true",
                    help="skip propagating O~ back through the noisy circuit")
    ap.add_argument("--no-pna", action="store_true", help="skip the propagated-noise-absorption leg")
    ap.add_argument("--pna-only", action="store_true", help="run only the propagated-noise-absorption leg")
    ap.add_argument("--pna-topk", default="", help="comma-separated product limits for extra PNA walks")
    ap.add_argument("--pna-batch", default="", help="comma-separated C:order pairs for batched PNA walks")
    ap.add_argument("--sine-orders", default="", help="comma-separated CPT-order limits: run only the "
                    "workload in the sine-order mode for each")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--serve-requests", type=int, default=30,
                    help="measured requests of the serving stream per arrival rate (0: skip it)")
    ap.add_argument("--serve-rates", default="200,0.5",
                    help="arrival rates (req/s): the configured one and one the device sustains")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-warmup", type=int, default=10)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args()
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
    wl = W.named_workload(args.workload, **({} if args.max_terms is None else {"max_terms": args.max_terms}))
    ctx = pp.Context(0)
    if args.sine_orders:
        so = sine_order_check(ctx, wl, [int(v) for v in args.sine_orders.split(",") if v])
        print(json.dumps({"sine_order": so, "workload": args.workload}), flush=True)
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
        r["roofline"] = roofline(r["kernels"], tb, prec, copy_gbs)
        results[prec] = r
        log(f"   {r['updates'] / r['seconds']:.4g} term-updates/s, {1e3 * r['seconds'] / args.steps:.1f} ms/step, "
            f"<O> = {r['expectation']!r}, {r['terms']} terms")
        for k in sorted(r["kernels"], key=lambda k: -k["total_ms"])[:12]:
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
        "metric": "Pauli-term updates/s (56q TFIM noise-canceling propagation)",
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
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
