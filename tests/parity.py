"""Comparison helpers for the GPU-vs-oracle parity tests (term sets and coefficients)."""
from __future__ import annotations

import math
from typing import Dict, Tuple

Key = Tuple[tuple, tuple, int]


def compare_sums(gpu: Dict[Key, float], ref: Dict[Key, float], thresholds=(), boundary: float = 1e-12,
                 rtol: float = 1e-11, atol: float = 1e-14, context: str = "") -> dict:
    """Strings and orders must agree exactly, except terms whose |c| lies within `boundary`
    (relative) of one of the truncation `thresholds` (eps, or the cap's cut value) or that are
    below 1e-12 in magnitude (rounding residue of cancellations).  Shared coefficients must agree
    to rtol/atol.  Returns a small report."""
    only_g = set(gpu) - set(ref)
    only_r = set(ref) - set(gpu)

    def exempt(v: float) -> bool:
        a = abs(v)
        if a <= 1e-12:
            return True
        return any(abs(a - t) <= boundary * max(t, 1e-300) + boundary for t in thresholds if t > 0)

    bad_g = [k for k in only_g if not exempt(gpu[k])]
    bad_r = [k for k in only_r if not exempt(ref[k])]
    assert not bad_g, f"{context}: {len(bad_g)} strings only on the GPU, e.g. {bad_g[:3]} -> {[gpu[k] for k in bad_g[:3]]}"
    assert not bad_r, f"{context}: {len(bad_r)} strings missing on the GPU, e.g. {bad_r[:3]} -> {[ref[k] for k in bad_r[:3]]}"
    worst = 0.0
    for k in set(gpu) & set(ref):
        a, b = gpu[k], ref[k]
        err = abs(a - b)
        tol = atol + rtol * abs(b)
        assert err <= tol, f"{context}: coefficient mismatch at {k}: gpu {a!r} oracle {b!r}"
        if b != 0:
            worst = max(worst, err / abs(b))
    return dict(n_gpu=len(gpu), n_ref=len(ref), only_gpu=len(only_g), only_ref=len(only_r), worst_rel=worst)


def cap_cut(ref: Dict[Key, float]) -> float:
    """Smallest kept |c| (the cap's cut value) of a capped result."""
    return min((abs(v) for v in ref.values()), default=0.0)
