"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU reference.

Strings and orders are compared exactly, coefficients to 1e-12 relative (FP64), terms within
1e-12 of a truncation threshold are exempt, and <O> must agree within 1e-10 absolute.  Whole
propagations where a cap binds are compared layer call by layer call, the reference fed the
device's input (tests/test_gpu_fullsteps.py); the end-to-end cases here are uncapped.
"""
import math
import sys

import numpy as np
import pytest

from paper_2606_20441_amd import workloads as W
from tests.parity import cap_cut, compare_sums

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_20441_amd import pp as _pp
    _pp.lib()
    return _pp


@pytest.fixture(scope="module")
def ctx(pp):
    c = pp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    from oracle import build
    build.build(force=False)
    from oracle import oracle
    return oracle


def random_gate_layer(n, n_gates, seed, kind="any", clifford_frac=0.3):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(n_gates):
        w = int(rng.integers(1, 4))
        qs = rng.choice(n, w, replace=False)
        letters = {"any": "XYZ", "x": "X", "z": "Z"}[kind]
        ops = {int(q): letters[int(rng.integers(0, len(letters)))] for q in qs}
        if rng.random() < clifford_frac:
            th = float(rng.integers(-4, 5)) * math.pi / 2
        else:
            th = float(rng.uniform(-3, 3))
        gates.append((ops, th))
    return W.make_layer(n, gates, [])


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [9, 56, 100, 140, 256])
def test_create_and_export(pp, ctx, orc, n):
    log(f"create n={n}")
    ps = W.random_pauli_sum(n, 500, seed=n)
    # duplicates and an exact cancellation
    x = np.concatenate([ps.x, ps.x[:50], ps.x[:3]])
    z = np.concatenate([ps.z, ps.z[:50], ps.z[:3]])
    c = np.concatenate([ps.c, ps.c[:50] * 0.5, -1.5 * ps.c[:3]])
    g = pp.Observable(ctx, n, x, z, c)
    o = orc.OracleSum(n, x, z, c)
    compare_sums(g.as_dict(), o.as_dict(), rtol=1e-15, atol=0.0, context="create")
    assert len(g) == len(o)


@pytest.mark.parametrize("n", [5, 56, 128, 200, 256])
@pytest.mark.parametrize("direction", [1, -1])
def test_general_gates_one_by_one(pp, ctx, orc, n, direction):
    log(f"general gates n={n} dir={direction}")
    ps = W.random_pauli_sum(n, 300, seed=7 * n + direction)
    layer = random_gate_layer(n, 6, seed=n + 3)
    g = pp.Observable.from_sum(ctx, ps, eps=1e-3)
    o = orc.OracleSum.from_sum(ps)
    g.apply_layer(layer, direction, with_noise=False)
    o.apply_layer(layer, direction, with_noise=False, eps=1e-3)
    compare_sums(g.as_dict(), o.as_dict(), thresholds=[1e-3], rtol=1e-12, atol=1e-15, context="general gates")


@pytest.mark.parametrize("name,steps", [("tfim7x8_pna", 1), ("tfim8x16", 1), ("tfim3x3", 1)])
@pytest.mark.parametrize("direction", [1, -1])
def test_tfim_layers_exact(pp, ctx, orc, name, steps, direction):
    """X-type and Z-type layers (fused LDS kernel) and Clifford layers, FP64."""
    wl = W.named_workload(name, steps=steps)
    n = wl.circuit.n_qubits
    ps = W.random_pauli_sum(n, 2000, seed=11, weight=3)
    eps = 1e-4
    for li, layer in enumerate(wl.circuit.layers):
        log(f"tfim layer {name} #{li} dir={direction}")
        g = pp.Observable.from_sum(ctx, ps, eps=eps)
        o = orc.OracleSum.from_sum(ps)
        g.apply_layer(layer, direction, with_noise=False)
        o.apply_layer(layer, direction, with_noise=False, eps=eps)
        compare_sums(g.as_dict(), o.as_dict(), thresholds=[eps], rtol=1e-12, atol=1e-15, context=f"layer {li}")


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("name", ["tfim7x8_pna", "tfim8x16"])
def test_noise_greedy(pp, ctx, orc, name, sign):
    log(f"noise greedy {name} sign={sign}")
    wl = W.named_workload(name, steps=1)
    layer = wl.circuit.layers[0]
    n = wl.circuit.n_qubits
    ps = W.random_pauli_arrays(n, 5000, seed=3, density=0.2)
    g = pp.Observable.from_sum(ctx, ps)
    o = orc.OracleSum.from_sum(ps)
    g.apply_layer(layer, with_gates=False, noise_sign=sign)
    o.noise(layer.ex, layer.ez, layer.lam, sign=sign)
    compare_sums(g.as_dict(), o.as_dict(), rtol=1e-13, context="noise")


def test_noise_general_generators(pp, ctx, orc):
    """Generators of weight > 2 (tested one by one) and mixed supports."""
    n = 70
    rng = np.random.default_rng(5)
    gens = []
    for _ in range(40):
        w = int(rng.integers(1, 5))
        ops = {int(q): "XYZ"[int(rng.integers(0, 3))] for q in rng.choice(n, w, replace=False)}
        gens.append((ops, float(rng.uniform(1e-4, 5e-2))))
    layer = W.make_layer(n, [], gens)
    ps = W.random_pauli_arrays(n, 3000, seed=8, density=0.3)
    g = pp.Observable.from_sum(ctx, ps)
    o = orc.OracleSum.from_sum(ps)
    g.apply_layer(layer, with_gates=False)
    o.noise(layer.ex, layer.ez, layer.lam)
    compare_sums(g.as_dict(), o.as_dict(), rtol=1e-13, context="noise general")


@pytest.mark.parametrize("variant", ["interleaved", "with_weight3"])
def test_noise_runs(pp, ctx, orc, variant):
    """The device multiplies the factors of each run of consecutive generators on the same
    qubits together (one table value per run a string touches); the reference applies the
    local channels one generator at a time.  Supports that come back later in the list (a
    new run) and lists with a weight-3 generator (every generator tested on its own) agree
    to rounding."""
    log(f"noise runs {variant}")
    n = 12
    rng = np.random.default_rng(21)
    gens = []
    for _ in range(60):
        if variant == "with_weight3" and rng.random() < 0.1:
            qs = rng.choice(n, 3, replace=False)
        elif rng.random() < 0.5:
            qs = [int(rng.integers(0, n))]
        else:
            q = int(rng.integers(0, n - 1))
            qs = [q, q + 1]
        ops = {int(q): "XYZ"[int(rng.integers(0, 3))] for q in qs}
        # runs of 1-3 generators on the same qubits
        for _ in range(int(rng.integers(1, 4))):
            ops2 = {q: "XYZ"[int(rng.integers(0, 3))] for q in ops}
            gens.append((ops2, float(rng.uniform(1e-3, 5e-2))))
    layer = W.make_layer(n, [], gens)
    ps = W.random_pauli_arrays(n, 3000, seed=9, density=0.5)
    for sign in (1, -1):
        g = pp.Observable.from_sum(ctx, ps)
        o = orc.OracleSum.from_sum(ps)
        g.apply_layer(layer, with_gates=False, noise_sign=sign)
        o.noise(layer.ex, layer.ez, layer.lam, sign=sign)
        compare_sums(g.as_dict(), o.as_dict(), rtol=1e-13, atol=0.0, context=f"noise runs {variant} {sign}")


@pytest.mark.parametrize("max_order", [0, 1, 2, 3])
def test_noise_error_order(pp, ctx, orc, max_order):
    log(f"error-order noise M={max_order}")
    wl = W.named_workload("tfim7x8_cd", steps=1, rate_lo=1e-3, rate_hi=2e-2)
    n = wl.circuit.n_qubits
    ps = W.random_pauli_arrays(n, 3000, seed=9, density=0.15)
    g = pp.Observable.from_sum(ctx, ps, mode="error_order", max_order=max_order, eps=1e-9)
    o = orc.OracleSum.from_sum(ps)
    for layer in wl.circuit.layers:
        g.apply_layer(layer, with_gates=False)
        o.apply_layer(layer, 1, with_gates=False, eps=1e-9, mode=1, max_order=max_order)
    compare_sums(g.as_dict(), o.as_dict(), thresholds=[1e-9], rtol=1e-12, atol=1e-16, context="error order")


def test_truncate_threshold_and_cap_with_ties(pp, ctx, orc):
    rng = np.random.default_rng(21)
    ps = W.random_pauli_sum(90, 6000, seed=21, allow_duplicates=False)
    ps.c = rng.choice([0.5, -0.5, 0.25, -0.25, 0.125, 1e-3, -2e-3, 3e-4], len(ps.c))
    for eps, cap in [(1e-3, 0), (0.2, 0), (0.0, 700), (1e-3, 2500), (0.3, 50), (0.0, 5999)]:
        log(f"truncate eps={eps} cap={cap}")
        g = pp.Observable.from_sum(ctx, ps)
        o = orc.OracleSum.from_sum(ps)
        g.truncate(eps, cap)
        o.truncate(eps, cap)
        assert g.as_dict() == o.as_dict()


@pytest.mark.parametrize("n", [6, 56, 130])
def test_expectation(pp, ctx, orc, n):
    ps = W.random_pauli_sum(n, 4000, seed=n, weight=None)
    # make a good share diagonal
    ps.x[: len(ps.c) // 2] = 0
    g = pp.Observable.from_sum(ctx, ps)
    o = orc.OracleSum.from_sum(ps)
    rng = np.random.default_rng(1)
    for _ in range(4):
        b = np.zeros(W.n_words(n), np.uint64)
        for q in rng.choice(n, n // 3, replace=False):
            b[q // 64] |= np.uint64(1) << np.uint64(q % 64)
        assert abs(g.expectation(b) - o.expectation(b)) < 1e-10
    assert abs(g.expectation() - o.expectation()) < 1e-10


def test_empty_and_vanishing(pp, ctx, orc):
    layer = W.named_workload("tfim7x8_pna", steps=1).circuit.layers[1]
    g = pp.Observable(ctx, 56, np.zeros((0, 1), np.uint64), np.zeros((0, 1), np.uint64), np.zeros(0))
    g.apply_layer(layer, -1)
    assert len(g) == 0 and g.expectation() == 0.0
    x, z, c, o = g.export()
    assert len(c) == 0
    ps = W.random_pauli_sum(56, 100, seed=2)
    ps.c[:] = 1e-6
    g = pp.Observable.from_sum(ctx, ps, eps=1e-3)
    g.apply_layer(layer, -1, with_noise=False)     # every anticommuting child falls below eps
    o = orc.OracleSum.from_sum(ps)
    o.apply_layer(layer, -1, with_noise=False, eps=1e-3)
    assert g.as_dict() == o.as_dict()


def test_group_overflow_falls_back(pp, ctx, orc):
    """A single z-group that outgrows LDS (2^14 children) goes through the per-gate path."""
    n = 56
    ops = {q: "Z" for q in range(0, 56, 4)}         # z-weight 14
    ps = W.pauli_sum(n, [(ops, 1.0), ({1: "Z", 2: "X"}, 0.5)])
    layer = W.make_layer(n, [({q: "X"}, 0.7) for q in range(n)], [])
    g = pp.Observable.from_sum(ctx, ps, eps=1e-12)
    o = orc.OracleSum.from_sum(ps)
    g.apply_layer(layer, 1, with_noise=False)
    st = g.last_layer_stats()
    o.apply_layer(layer, 1, with_noise=False, eps=1e-12)
    assert st["n_fallback"] > 0
    compare_sums(g.as_dict(), o.as_dict(), thresholds=[1e-12], rtol=1e-12, atol=1e-15, context="overflow")


@pytest.mark.parametrize("cap", [40000, 15000])
@pytest.mark.parametrize("W_qubits", [20, 100])
def test_capped_gates_with_oversize_classes(pp, ctx, orc, cap, W_qubits):
    """Gate by gate under a binding cap, with z-classes far larger than an LDS tile: 2^14
    strings share one z (all x patterns on its 14 qubits), plus smaller classes; every X
    rotation on those qubits pairs the whole class."""
    n = W_qubits
    rng = np.random.default_rng(5 + n)
    zq = list(range(14))
    terms = []
    for xm in range(1 << 14):
        ops = {q: ("Y" if (xm >> i) & 1 else "Z") for i, q in enumerate(zq)}
        terms.append((ops, float(rng.uniform(-1, 1))))
    for k in range(3000):   # smaller classes elsewhere
        qs = rng.choice(np.arange(14, n), 4, replace=False)
        terms.append(({int(q): "XYZ"[int(rng.integers(0, 3))] for q in qs}, float(rng.uniform(-1, 1))))
    ps = W.pauli_sum(n, terms)
    layer = W.make_layer(n, [({q: "X"}, 0.4 + 0.01 * q) for q in range(n)], [])
    log(f"oversize classes: n={n} cap={cap} terms={len(ps.c)}")
    for direction in (1, -1):
        g = pp.Observable.from_sum(ctx, ps, eps=1e-4, max_terms=cap)
        o = orc.OracleSum.from_sum(ps)
        g.apply_layer(layer, direction, with_noise=False)
        st = g.last_layer_stats()
        o.apply_layer(layer, direction, with_noise=False, eps=1e-4, max_terms=cap)
        assert st["n_fallback"] > 0
        gd, od = g.as_dict(), o.as_dict()
        compare_sums(gd, od, thresholds=[1e-4, cap_cut(od)], rtol=1e-12, atol=1e-15, context="capped classes")
        assert len(gd) <= cap


def test_invalid_arguments_leave_state(pp, ctx):
    ps = W.random_pauli_sum(56, 50, seed=1)
    g = pp.Observable.from_sum(ctx, ps)
    before = g.as_dict()
    bad = W.make_layer(56, [({3: "X"}, 0.3)], [({3: "Z"}, 0.01)])
    bad.lam[:] = -1.0
    with pytest.raises(pp.PPError) as e:
        g.apply_layer(bad)
    assert e.value.status == pp.PP_ERR_INVALID
    bad2 = W.make_layer(56, [({3: "X"}, 0.3)], [])
    bad2.gx[0, 0] |= np.uint64(1) << np.uint64(60)    # bit above n_qubits
    with pytest.raises(pp.PPError):
        g.apply_layer(bad2)
    with pytest.raises(pp.PPError):
        g.apply_layer(bad2, direction=0)
    with pytest.raises(pp.PPError):
        pp.Observable(ctx, 56, [[1 << 60]], [[0]], [1.0])
    with pytest.raises(pp.PPError):
        pp.Observable(ctx, 56, [[1]], [[0]], [1.0], mode="error_order", max_order=9)
    assert g.as_dict() == before


# ------------------------------------------------------------------------------------------
# Whole method on the named workloads (small sizes the reference finishes in seconds).
# ------------------------------------------------------------------------------------------
def run_both(pp, ctx, orc, wl, precision="f64"):
    g = pp.run_workload(ctx, wl, precision=precision)
    o = orc.run_workload(wl)
    return g, o


@pytest.mark.parametrize("wname,kw", [
    ("tfim3x3", {}),
    ("tfim3x3", dict(eps=1e-6)),
    ("tfim3x3", dict(noise="entangling", steps=5)),
    ("tfim7x8_pna", dict(steps=2)),
    ("tfim7x8_pna", dict(steps=3, eps=1e-4)),
    ("tfim7x8_cd", dict(steps=2)),
    ("tfim7x8_cd", dict(steps=3, eps=1e-5)),
    ("tfim8x16", dict(steps=1, eps=1e-4)),
    ("tfim8x16", dict(steps=2, eps=2e-3)),
])
def test_workload_parity(pp, ctx, orc, wname, kw):
    wl = W.named_workload(wname, **kw)
    log(f"workload {wname} {kw}")
    g, o = run_both(pp, ctx, orc, wl)
    od = o.as_dict()
    thr = [wl.eps] + ([cap_cut(od)] if wl.max_terms else [])
    rep = compare_sums(g.as_dict(), od, thresholds=thr, rtol=1e-12, atol=1e-15, context=f"{wname} {kw}")
    eg, eo = g.expectation(), o.expectation()
    log(f"  terms {rep['n_gpu']} vs {rep['n_ref']}, <O> {eg!r} vs {eo!r}")
    assert abs(eg - eo) < 1e-10


@pytest.mark.parametrize("wname,kw", [
    ("tfim3x3", dict(eps=0.0)),
    ("tfim3x3", {}),
    ("tfim7x8_pna", dict(steps=2)),
    ("tfim7x8_pna", dict(steps=3, eps=1e-4)),
])
def test_noisy_evaluation(pp, ctx, orc, wname, kw):
    """O~ propagated back through the noisy circuit on the GPU: Tr[O~ rho_noisy] against the
    reference's same walk, and against the ideal value (statevector) at zero threshold."""
    wl = W.named_workload(wname, **kw)
    log(f"noisy evaluation {wname} {kw}")
    g, o = run_both(pp, ctx, orc, wl)
    vg = pp.noisy_evaluation(wl.circuit, g)
    vo = orc.noisy_evaluation(wl.circuit, o, eps=wl.eps, max_terms=wl.max_terms)
    log(f"  Tr[O~ rho_noisy]: {vg!r} vs {vo!r}")
    assert abs(vg - vo) < 1e-10
    if wl.eps == 0.0 and wl.circuit.n_qubits <= 10:
        from oracle import brute as B
        psi = B.statevector(wl.circuit)
        om = B.pauli_sum_matrix(wl.circuit.n_qubits, wl.observable.x, wl.observable.z, wl.observable.c)
        assert abs(vg - np.vdot(psi, om @ psi).real) < 1e-10


@pytest.mark.parametrize("wname,kw", [
    ("tfim3x3", {}),
    ("tfim7x8_pna", dict(steps=2)),
    ("tfim8x16", dict(steps=1, eps=1e-4)),
])
def test_workload_fp32_error(pp, ctx, orc, wname, kw):
    """FP32 coefficients (compensated merges, FP64 noise factors and reduction): report and
    bound the error of <O> against the FP64 reference."""
    wl = W.named_workload(wname, **kw)
    g = pp.run_workload(ctx, wl, precision="f32k")
    o = orc.run_workload(wl)
    eg, eo = g.expectation(), o.expectation()
    norm1 = float(np.abs(wl.observable.c).sum())
    log(f"fp32 {wname} {kw}: <O> {eg!r} vs {eo!r}, |d| = {abs(eg - eo):.3e}, terms {len(g)} vs {len(o)}")
    assert abs(eg - eo) <= 1e-6 * max(1.0, norm1)
