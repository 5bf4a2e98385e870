"""Host logic of the binding that needs no GPU: the Clifford interaction-picture rewrite
(Euclid appendix) against the reference's own, independently written rewrite."""
import math

import numpy as np
import pytest

from paper_2606_20441_amd import workloads as W


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_interaction_picture_matches_reference(seed):
    from oracle import oracle
    from paper_2606_20441_amd import pp
    rng = np.random.default_rng(seed)
    wl = W.named_workload("tfim3x3", steps=2)
    circ = wl.circuit
    for layer in circ.layers:
        th = np.asarray(layer.theta, np.float64).copy()
        # mix of small, wide, exact Clifford and whole-turn angles
        th = th + rng.choice([0.0, math.pi / 2, -math.pi / 2, math.pi, 2 * math.pi], th.shape[0])
        th[0] = math.pi / 2
        th[-1] = 2 * math.pi + 0.2
        layer.theta = th
    a = pp.interaction_picture(circ)
    b = oracle.interaction_picture(circ)
    for la, lb in zip(a.layers, b.layers):
        assert np.array_equal(np.asarray(la.gx, np.uint64), np.asarray(lb.gx, np.uint64))
        assert np.array_equal(np.asarray(la.gz, np.uint64), np.asarray(lb.gz, np.uint64))
        assert np.array_equal(np.asarray(la.theta), np.asarray(lb.theta))
        for t in la.theta:
            k = t / (math.pi / 2)
            assert abs(t) <= math.pi / 4 + 1e-12 or abs(k - round(k)) < 1e-12


def test_interaction_picture_keeps_the_circuit():
    from paper_2606_20441_amd import pp
    wl = W.named_workload("tfim3x3", steps=1)
    a = pp.interaction_picture(wl.circuit)
    for la, lo in zip(a.layers, wl.circuit.layers):
        assert la.n_gates == lo.n_gates          # angles 0.3 and 0.7 are already residuals
        assert np.array_equal(np.asarray(la.theta), np.asarray(lo.theta))
        assert np.array_equal(np.asarray(la.ex), np.asarray(lo.ex))
