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


def _keys(x, z, o):
    """Rows of (x words, z words, order) as one structured array, sortable and comparable."""
    import numpy as np
    n, w = x.shape
    dt = [(f"x{i}", "<u8") for i in range(w)] + [(f"z{i}", "<u8") for i in range(w)] + [("o", "u1")]
    k = np.zeros(n, dtype=dt)
    for i in range(w):
        k[f"x{i}"] = x[:, i]
        k[f"z{i}"] = z[:, i]
    k["o"] = o
    return k


def compare_exports(g, r, thresholds=(), boundary: float = 1e-12, rtol: float = 1e-12, atol: float = 1e-15,
                    context: str = "") -> dict:
    """compare_sums for two exports (x, z, c, ord), vectorised for large sums: strings and
    orders exact except terms within `boundary` (relative) of a truncation threshold or below
    1e-12, shared coefficients to rtol/atol."""
    import numpy as np
    gk, rk = _keys(g[0], g[1], g[3]), _keys(r[0], r[1], r[3])
    gc, rc = np.asarray(g[2], np.float64), np.asarray(r[2], np.float64)
    common, gi, ri = np.intersect1d(gk, rk, assume_unique=True, return_indices=True)
    only_g = np.setdiff1d(np.arange(len(gk)), gi)
    only_r = np.setdiff1d(np.arange(len(rk)), ri)

    def exempt(v):
        a = np.abs(v)
        ok = a <= 1e-12
        for t in thresholds:
            if t > 0:
                ok |= np.abs(a - t) <= boundary * t + boundary
        return ok

    bad_g = only_g[~exempt(gc[only_g])]
    bad_r = only_r[~exempt(rc[only_r])]
    assert len(bad_g) == 0, f"{context}: {len(bad_g)} strings only on the GPU, e.g. |c| {np.abs(gc[bad_g[:3]])}"
    assert len(bad_r) == 0, f"{context}: {len(bad_r)} strings missing on the GPU, e.g. |c| {np.abs(rc[bad_r[:3]])}"
    a, b = gc[gi], rc[ri]
    err = np.abs(a - b)
    tol = atol + rtol * np.abs(b)
    bad = np.nonzero(err > tol)[0]
    assert len(bad) == 0, f"{context}: {len(bad)} coefficient mismatches, e.g. gpu {a[bad[:3]]} oracle {b[bad[:3]]}"
    nz = b != 0
    worst = float((err[nz] / np.abs(b[nz])).max()) if nz.any() else 0.0
    return dict(n_gpu=len(gk), n_ref=len(rk), only_gpu=len(only_g), only_ref=len(only_r), worst_rel=worst)


def oracle_layer_step(orc, n: int, state, wl, kind: str, m: int):
    """The reference's version of one layer call of D on the state (x, z, c, ord) exported by the
    device just before that call.  `kind` is the schedule step the library reported: backward
    through G_m without noise, the inverse noise N_m^-1 alone, or forward through G_m followed
    by N_m^-1; the workload's threshold, cap and mode apply as on the device."""
    x, z, c, o = state
    r = orc.OracleSum(n, x, z, c, o)
    layer = wl.circuit.layers[m]
    kw = dict(eps=wl.eps, max_terms=wl.max_terms, mode=orc.MODES[wl.mode], max_order=wl.max_order)
    if kind == "backward":
        r.apply_layer(layer, +1, with_noise=False, **kw)
    elif kind == "noise":
        r.apply_layer(layer, -1, with_gates=False, noise_sign=1, **kw)
    else:
        r.apply_layer(layer, -1, noise_sign=1, noise_after_gates=True, **kw)
    return r

