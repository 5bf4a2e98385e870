"""GPU parity of the sine-order mode (Euclid appendix: the CPT order kappa = k + 2p of a term,
counted as the sine factors along its path, in the Clifford interaction picture).

Each case runs D O in the sine-order mode on the device (which writes each layer in the
interaction picture itself) and in the FP64 reference (given the circuit rewritten by its own,
independent rewrite), with the first layer's gate pair kept on both sides, and compares
every (string, tag) term (terms within 1e-12 of a threshold exempt, coefficients to
1e-11 relative, <O~> to 1e-10).  At a tag limit above the number of rotations, the tags
summed equal the greedy propagation.
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


def _wide_angles(circ, seed):
    rng = np.random.default_rng(seed)
    for layer in circ.layers:
        if layer.n_gates:
            th = np.array(layer.theta, np.float64)
            th = th + rng.choice([0.0, math.pi / 2, -math.pi / 2, math.pi], th.shape[0]) + rng.uniform(-0.5, 0.5, th.shape[0])
            layer.theta = th
    return circ


@pytest.mark.parametrize("name,kw,K,eps,cap,wide", [
    ("tfim3x3", dict(steps=2), 0, 0.0, 0, False),
    ("tfim3x3", dict(steps=2), 1, 0.0, 0, False),
    ("tfim3x3", dict(steps=2), 3, 0.0, 0, True),
    ("tfim3x3", dict(steps=3), 4, 1e-6, 0, True),
    ("tfim3x3", dict(steps=3), 3, 0.0, 25, True),
    ("tfim7x8_pna", dict(steps=2), 2, 1e-5, 0, False),
    ("tfim8x16", dict(steps=1), 2, 1e-4, 0, True),
    ("tfim7x8_pna", dict(steps=2), 2, 1e-6, 400, False),
    ("tfim8x16", dict(steps=1), 2, 1e-5, 1000, True),
])
def test_sine_order_parity(pp, ctx, orc, name, kw, K, eps, cap, wide):
    wl = W.named_workload(name, **kw)
    circ = _wide_angles(wl.circuit, 5) if wide else wl.circuit
    log(f"sine order {name} {kw} K={K} eps={eps} cap={cap} wide={wide}")
    ipo = orc.interaction_picture(circ)      # the library writes the device's layers in it itself
    g = pp.noise_canceling(ctx, circ, wl.observable, eps=eps, max_terms=cap, mode="sine_order", max_order=K)
    r = orc.noise_canceling(ipo, wl.observable, eps=eps, max_terms=cap, mode="sine_order", max_order=K)
    ref = r.as_dict()
    got = g.as_dict()
    th = [eps] + ([cap_cut(ref)] if cap else [])
    rep = compare_sums(got, ref, thresholds=th, context=f"sine {name}")
    assert max((k[2] for k in got), default=0) <= K
    eg, eo = g.expectation(), r.expectation()
    log(f"  {rep}; <O~> {eg!r} vs {eo!r}")
    assert abs(eg - eo) < 1e-10
    g.destroy()


@pytest.mark.parametrize("K", [1, 3])
@pytest.mark.parametrize("cap", [40000, 12000])
def test_sine_order_capped_oversize_classes(pp, ctx, orc, K, cap):
    """Sine order under a binding cap, through the tiled gate passes: 2^14 strings share one
    z (all x patterns on 14 qubits, a class far larger than an LDS tile) plus small classes
    elsewhere; every X rotation pairs a whole class and the sin parts step the tags up to K.
    The angles stay within pi/4, so the interaction picture adds no Clifford gate."""
    n = 40
    rng = np.random.default_rng(17)
    terms = []
    for xm in range(1 << 14):
        terms.append(({q: ("Y" if (xm >> q) & 1 else "Z") for q in range(14)}, float(rng.uniform(-1, 1))))
    for k in range(3000):
        qs = rng.choice(np.arange(14, n), 4, replace=False)
        terms.append(({int(q): "XYZ"[int(rng.integers(0, 3))] for q in qs}, float(rng.uniform(-1, 1))))
    ps = W.pauli_sum(n, terms)
    layer = W.make_layer(n, [({q: "X"}, 0.2 + 0.01 * q) for q in range(n)], [])
    log(f"sine order, oversize classes: K={K} cap={cap} terms={len(ps.c)}")
    for direction in (1, -1):
        g = pp.Observable.from_sum(ctx, ps, eps=1e-5, max_terms=cap, mode="sine_order", max_order=K)
        o = orc.OracleSum.from_sum(ps)
        g.apply_layer(layer, direction, with_noise=False)
        st = g.last_layer_stats()
        o.apply_layer(layer, direction, with_noise=False, eps=1e-5, max_terms=cap, mode=2, max_order=K)
        gd, od = g.as_dict(), o.as_dict()
        assert st["n_fallback"] > 0
        rep = compare_sums(gd, od, thresholds=[1e-5, cap_cut(od)], rtol=1e-12, atol=1e-15,
                           context=f"sine order, oversize classes, direction {direction}")
        log(f"  direction {direction}: {rep}")
        assert len(gd) <= cap
        assert max(k[2] for k in gd) <= K
        g.destroy()


def test_sine_order_all_tags_equal_greedy(pp, ctx):
    wl = W.named_workload("tfim3x3", steps=2)
    ip = _wide_angles(wl.circuit, 9)
    a = pp.noise_canceling(ctx, ip, wl.observable, mode="sine_order", max_order=250)
    b = pp.noise_canceling(ctx, ip, wl.observable)
    tot = {}
    for (x, z, o), v in a.as_dict().items():
        tot[(x, z, 0)] = tot.get((x, z, 0), 0.0) + v
    compare_sums(tot, b.as_dict(), context="sine order, all tags vs greedy")
    assert abs(a.expectation() - b.expectation()) < 1e-10
    a.destroy()
    b.destroy()


def test_sine_order_argument_errors(pp, ctx):
    wl = W.named_workload("tfim3x3", steps=1)
    with pytest.raises(pp.PPError):
        pp.Observable.from_sum(ctx, wl.observable, mode="sine_order", max_order=251)
    with pytest.raises(pp.PPError):
        pp.Observable.from_sum(ctx, wl.observable, mode="sine_order", max_order=-1)
