"""GPU parity at the full step counts of the two capped workloads, with the cap binding.

The 56-qubit propagated-noise-absorption workload (7x8 lattice, 10 Trotter steps: 39 layer
calls of D) with a cap of 2^16 terms, and the 128-qubit workload (8x16 lattice, 8 steps, two
words per string: 31 layer calls) with a cap of 2^14, run through the device's normal path,
one layer call after the other.  Before each call the device's terms are exported and handed
to the FP64 reference, which applies the same call with the same threshold and cap; the two
results are compared term by term (strings exact, coefficients to 1e-12 relative, terms
within 1e-12 of the threshold or of the cut exempt) and <O~> to 1e-10.

Why the reference is fed the device's input before each call: the cap binds after nearly
every non-Clifford gate, and the device multiplies the inverse-noise factors of a local
channel's generators together before applying them, the reference applies one generator
after the other, so the two round the noise differently (by about one unit in the last
place).  A cut falling between two terms that close would keep a different term on each side
of an unfed walk, and the difference would propagate.  Within one call the gates' arithmetic
is the same on both sides (the same cos and sin, and sums of two products), so each call's
cuts are identical.  The unfed end-to-end difference and the FP32-Kahan error against the
FP64 reference are measured and reported.
"""
import sys
import time

import numpy as np
import pytest

from paper_2606_20441_amd import workloads as W
from tests.parity import compare_exports, oracle_layer_step

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


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,kw", [
    ("tfim7x8_pna", dict(steps=10, max_terms=1 << 16)),
    ("tfim8x16", dict(steps=8, max_terms=1 << 14)),
])
def test_capped_full_schedule_layer_fed(pp, ctx, orc, name, kw):
    wl = W.named_workload(name, **kw)
    n = wl.circuit.n_qubits
    log(f"full schedule {name} {kw}: eps {wl.eps}, {len(wl.circuit.layers)} layers")
    state = [None]
    g0 = pp.Observable.from_sum(ctx, wl.observable, eps=wl.eps, max_terms=wl.max_terms)
    state[0] = g0.export()
    g0.destroy()
    n_capped = [0]
    worst = [0.0]
    t0 = time.time()

    def on_layer(step, kind, m, obs):
        r = oracle_layer_step(orc, n, state[0], wl, kind, m)
        got = obs.export()
        ref = r.export()
        st = obs.last_layer_stats()
        n_capped[0] += int(st["n_capped"] > 0)
        cut = float(np.abs(ref[2]).min()) if len(ref[2]) else 0.0
        rep = compare_exports(got, ref, thresholds=[wl.eps, cut], context=f"{name} call {step} ({kind} {m})")
        eg, eo = obs.expectation(), r.expectation()
        assert abs(eg - eo) < 1e-10, (step, eg, eo)
        worst[0] = max(worst[0], rep["worst_rel"])
        log(f"  call {step:2d} {kind:8s} layer {m:2d}: {rep['n_gpu']} terms (ref {rep['n_ref']}), capped "
            f"{st['n_capped']}, worst rel {rep['worst_rel']:.1e}, <O~> {eg:.12f}  [{time.time() - t0:.0f} s]")
        state[0] = got

    g = pp.noise_canceling(ctx, wl.circuit, wl.observable, wl.eps, wl.max_terms, on_layer=on_layer)
    assert n_capped[0] >= 10, "the cap should bind in many layer calls"
    eg = g.expectation()
    g.destroy()
    # Unfed, end to end: the reference's own walk, and FP32-Kahan on the device.
    r = orc.run_workload(wl)
    eo = r.expectation()
    f = pp.run_workload(ctx, wl, precision="f32k")
    ef = f.expectation()
    f.destroy()
    norm1 = float(np.abs(wl.observable.c).sum())
    log(f"  {name}: {n_capped[0]} capped calls, worst coefficient rel. error {worst[0]:.1e}; unfed <O~>: "
        f"device {eg!r}, reference {eo!r}, |d| = {abs(eg - eo):.2e}; FP32-Kahan {ef!r}, "
        f"|d| vs reference {abs(ef - eo):.2e} (relative to ||O||_1 = {norm1:g}: {abs(ef - eo) / norm1:.2e})")
