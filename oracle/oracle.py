"""ctypes front end of the CPU FP64 reference (``libpp_oracle.so``).

Test infrastructure only (test suite, smoke check, benchmark CPU-baseline leg).  It
imports nothing from the HIP package; circuits and observables are passed as plain
numpy arrays or duck-typed objects with the same fields as the seeded input generators
produce (``n_qubits``, ``layers[m].gx/gz/theta/ex/ez/lam``, ``x/z/c``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

from . import build as _build

_LIB = None

_u64p = C.POINTER(C.c_uint64)
_f64p = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_i32p = C.POINTER(C.c_int)


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=True)
        lib = C.CDLL(path)
        lib.or_create.restype = C.c_void_p
        lib.or_create.argtypes = [C.c_int, C.c_int64, _u64p, _u64p, _f64p, _u8p]
        lib.or_clone.restype = C.c_void_p
        lib.or_clone.argtypes = [C.c_void_p]
        lib.or_free.argtypes = [C.c_void_p]
        lib.or_size.restype = C.c_int64
        lib.or_size.argtypes = [C.c_void_p]
        lib.or_export.argtypes = [C.c_void_p, _u64p, _u64p, _f64p, _u8p]
        lib.or_rotate.restype = C.c_int
        lib.or_rotate.argtypes = [C.c_void_p, _u64p, _u64p, C.c_double, C.c_int]
        lib.or_noise.argtypes = [C.c_void_p, C.c_int, _u64p, _u64p, _f64p, C.c_int, C.c_int, C.c_int]
        lib.or_truncate.argtypes = [C.c_void_p, C.c_double, C.c_int64]
        lib.or_apply_layer.argtypes = [C.c_void_p, C.c_int, _u64p, _u64p, _f64p, C.c_int, C.c_int,
                                       _u64p, _u64p, _f64p, C.c_int, C.c_int, C.c_double, C.c_int64,
                                       C.c_int, C.c_int]
        lib.or_noise_canceling.restype = C.c_void_p
        lib.or_noise_canceling.argtypes = [C.c_void_p, C.c_int, _i32p, _u64p, _u64p, _f64p, _i32p,
                                           _u64p, _u64p, _f64p, C.c_double, C.c_int64, C.c_int, C.c_int]
        lib.or_antinoise.argtypes = [C.c_void_p, C.c_void_p, C.c_double]
        lib.or_antinoise_topk.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_int64]
        lib.or_antinoise_batch.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_void_p), _f64p, C.c_int, C.c_double]
        lib.or_expectation.restype = C.c_double
        lib.or_expectation.argtypes = [C.c_void_p, _u64p]
        lib.or_norm2.restype = C.c_double
        lib.or_norm2.argtypes = [C.c_void_p]
        _LIB = lib
    return _LIB


def _p(a: Optional[np.ndarray], t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _u64(a, w: int) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(-1, w))


class OracleSum:
    """A Pauli sum held by the CPU reference."""

    def __init__(self, n_qubits: int, x, z, c, ord_=None, _handle=None):
        self.n = int(n_qubits)
        self.W = (self.n + 63) // 64
        lib = _lib()
        if _handle is not None:
            self._h = _handle
            return
        x = _u64(x, self.W)
        z = _u64(z, self.W)
        c = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(-1))
        o = None if ord_ is None else np.ascontiguousarray(np.asarray(ord_, dtype=np.uint8))
        self._h = lib.or_create(self.n, c.shape[0], _p(x, _u64p), _p(z, _u64p), _p(c, _f64p), _p(o, _u8p))

    @classmethod
    def from_sum(cls, ps) -> "OracleSum":
        return cls(ps.n_qubits, ps.x, ps.z, ps.c)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib().or_free(h)
            self._h = None

    def clone(self) -> "OracleSum":
        return OracleSum(self.n, None, None, None, _handle=_lib().or_clone(self._h))

    def __len__(self) -> int:
        return int(_lib().or_size(self._h))

    def export(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        n = len(self)
        x = np.zeros((n, self.W), np.uint64)
        z = np.zeros((n, self.W), np.uint64)
        c = np.zeros(n, np.float64)
        o = np.zeros(n, np.uint8)
        _lib().or_export(self._h, _p(x, _u64p), _p(z, _u64p), _p(c, _f64p), _p(o, _u8p))
        return x, z, c, o

    def rotate(self, rx, rz, theta: float, direction: int) -> bool:
        rx = _u64(rx, self.W)
        rz = _u64(rz, self.W)
        return bool(_lib().or_rotate(self._h, _p(rx, _u64p), _p(rz, _u64p), float(theta), int(direction)))

    def noise(self, ex, ez, lam, sign: int = 1, mode: int = 0, max_order: int = 2) -> None:
        ex = _u64(ex, self.W)
        ez = _u64(ez, self.W)
        lam = np.ascontiguousarray(np.asarray(lam, np.float64))
        _lib().or_noise(self._h, lam.shape[0], _p(ex, _u64p), _p(ez, _u64p), _p(lam, _f64p),
                        int(sign), int(mode), int(max_order))

    def truncate(self, eps: float, max_terms: int = 0) -> None:
        _lib().or_truncate(self._h, float(eps), int(max_terms))

    def antinoise(self, eprime: "OracleSum", q: float) -> None:
        """O -> (1 - q) O + q E' O E' (Section I.A, Eq. applyantinoise); no truncation."""
        _lib().or_antinoise(self._h, eprime._h, float(q))

    def antinoise_batch(self, eprimes, qs, order: int = 1, eps1: float = 0.0) -> None:
        """A batch of commuting antinoise maps to first or second order in the number of
        errors (Appendix C); exact for one map.  The second-order pass takes the
        first-order part without its terms below eps1."""
        hs = (C.c_void_p * len(eprimes))(*[e._h for e in eprimes])
        qa = np.ascontiguousarray(np.asarray(qs, np.float64))
        _lib().or_antinoise_batch(self._h, len(eprimes), hs, _p(qa, _f64p), int(order), float(eps1))

    def antinoise_topk(self, eprime: "OracleSum", q: float, k: int) -> None:
        """As ``antinoise`` with E' O E' limited to the k most significant products
        (Appendix B; ties with the k-th kept)."""
        _lib().or_antinoise_topk(self._h, eprime._h, float(q), int(k))

    def apply_layer(self, layer, direction: int, with_gates: bool = True, with_noise: bool = True,
                    noise_sign: int = 1, noise_after_gates: bool = True, eps: float = 0.0,
                    max_terms: int = 0, mode: int = 0, max_order: int = 2) -> None:
        W = self.W
        ng = layer.n_gates if with_gates else 0
        nk = layer.n_gen if with_noise else 0
        gx = _u64(layer.gx, W) if ng else np.zeros((1, W), np.uint64)
        gz = _u64(layer.gz, W) if ng else np.zeros((1, W), np.uint64)
        th = np.ascontiguousarray(layer.theta, np.float64) if ng else np.zeros(1)
        ex = _u64(layer.ex, W) if nk else np.zeros((1, W), np.uint64)
        ez = _u64(layer.ez, W) if nk else np.zeros((1, W), np.uint64)
        lam = np.ascontiguousarray(layer.lam, np.float64) if nk else np.zeros(1)
        _lib().or_apply_layer(self._h, ng, _p(gx, _u64p), _p(gz, _u64p), _p(th, _f64p), int(direction),
                              nk, _p(ex, _u64p), _p(ez, _u64p), _p(lam, _f64p), int(noise_sign),
                              int(bool(noise_after_gates)), float(eps), int(max_terms), int(mode),
                              int(max_order))

    def expectation(self, basis=None) -> float:
        b = None if basis is None else _u64(basis, self.W).reshape(-1)
        return float(_lib().or_expectation(self._h, _p(b, _u64p)))

    def norm2(self) -> float:
        return float(_lib().or_norm2(self._h))

    def as_dict(self):
        x, z, c, o = self.export()
        return {(tuple(int(v) for v in x[i]), tuple(int(v) for v in z[i]), int(o[i])): float(c[i])
                for i in range(len(c))}


def _circuit_arrays(circuit):
    W = (circuit.n_qubits + 63) // 64
    ng = np.array([l.n_gates for l in circuit.layers], dtype=np.int32)
    nk = np.array([l.n_gen for l in circuit.layers], dtype=np.int32)

    def cat(name, w):
        parts = [np.asarray(getattr(l, name)).reshape(-1, w) if w else np.asarray(getattr(l, name)).reshape(-1)
                 for l in circuit.layers]
        arr = np.concatenate(parts) if parts else np.zeros((0, w) if w else 0)
        if arr.size == 0:
            arr = np.zeros((1, w) if w else 1, dtype=arr.dtype)
        return np.ascontiguousarray(arr)

    gx = cat("gx", W).astype(np.uint64)
    gz = cat("gz", W).astype(np.uint64)
    th = cat("theta", 0).astype(np.float64)
    ex = cat("ex", W).astype(np.uint64)
    ez = cat("ez", W).astype(np.uint64)
    lam = cat("lam", 0).astype(np.float64)
    return ng, nk, gx, gz, th, ex, ez, lam


MODES = {"greedy": 0, "error_order": 1, "sine_order": 2}


def interaction_picture(circuit):
    """The Clifford interaction picture of the Euclid appendix: every rotation angle theta
    is split into its nearest multiple m pi/2 (an exact Clifford rotation about the same
    Pauli, applied first; the two commute) and a residual with |theta'| <= pi/4, so every
    sine the expansion counts is at most 1/sqrt 2.  A whole turn (m = 0 mod 4) is only a
    phase under conjugation and is left out; Clifford angles are kept as they are."""
    import copy
    import math
    out = copy.deepcopy(circuit)
    half = math.pi / 2
    for layer in out.layers:
        if layer.n_gates == 0:
            continue
        gx = np.asarray(layer.gx, np.uint64).reshape(layer.n_gates, -1)
        gz = np.asarray(layer.gz, np.uint64).reshape(layer.n_gates, -1)
        xs, zs, th = [], [], []
        for g in range(layer.n_gates):
            t = float(layer.theta[g])
            m = round(t / half)
            r = t - m * half
            if abs(r) <= 1e-12 * half:
                parts = [t]
            elif m % 4 == 0:
                parts = [r]
            else:
                parts = [m * half, r]
            for a in parts:
                xs.append(gx[g])
                zs.append(gz[g])
                th.append(a)
        layer.gx = np.array(xs, np.uint64).reshape(len(th), -1)
        layer.gz = np.array(zs, np.uint64).reshape(len(th), -1)
        layer.theta = np.array(th, np.float64)
    return out


def noise_canceling(circuit, observable, eps: float = 0.0, max_terms: int = 0,
                    mode: str = "greedy", max_order: int = 2) -> OracleSum:
    """O~ = D O for a layered circuit (see ``or_noise_canceling`` in pp_oracle.h)."""
    obs = observable if isinstance(observable, OracleSum) else OracleSum.from_sum(observable)
    ng, nk, gx, gz, th, ex, ez, lam = _circuit_arrays(circuit)
    h = _lib().or_noise_canceling(obs._h, len(circuit.layers), _p(ng, _i32p), _p(gx, _u64p), _p(gz, _u64p),
                                  _p(th, _f64p), _p(nk, _i32p), _p(ex, _u64p), _p(ez, _u64p), _p(lam, _f64p),
                                  float(eps), int(max_terms), MODES[mode], int(max_order))
    return OracleSum(circuit.n_qubits, None, None, None, _handle=h)


def noisy_evaluation(circuit, obs: OracleSum, eps: float = 0.0, max_terms: int = 0) -> float:
    """Tr[O~ rho_noisy] by noisy Pauli propagation (Section III's check that the mitigated
    observable recovers the ideal value): C_noisy = N_M G_M .. N_1 G_1 (noise after every
    layer's gates), so its adjoint applies, from m = M down to 1, the channel N_m itself
    (a Pauli channel is self-adjoint) and then G_m^dag.  Changes `obs` in place."""
    for layer in reversed(circuit.layers):
        obs.apply_layer(layer, +1, with_gates=True, with_noise=True, noise_sign=-1, noise_after_gates=False,
                        eps=eps, max_terms=max_terms)
    return obs.expectation()


def antinoise_q(lam: float) -> float:
    """Quasi-probability of one generator's inverse map (Section I: the channel applies
    E with probability p = (1 - e^{-2 lambda})/2; the inverse negates lambda)."""
    return (1.0 - np.exp(2.0 * lam)) / 2.0


def propagated_error(circuit, t: int, k: int, eps_fwd: float = 0.0, max_terms_fwd: int = 0) -> OracleSum:
    """E'_{t,k} = U E U^dag: generator k of layer t's noise carried through the gates of
    layers t+1..M, forward in time (Section I.A, Eq. channel_prop; truncation per non-Clifford gate)."""
    layer = circuit.layers[t]
    W = (circuit.n_qubits + 63) // 64
    ex = np.asarray(layer.ex, np.uint64).reshape(-1, W)[k:k + 1]
    ez = np.asarray(layer.ez, np.uint64).reshape(-1, W)[k:k + 1]
    e = OracleSum(circuit.n_qubits, ex, ez, np.ones(1))
    for later in circuit.layers[t + 1:]:
        e.apply_layer(later, -1, with_gates=True, with_noise=False, eps=eps_fwd, max_terms=max_terms_fwd)
    return e


def pna(circuit, observable, eps: float = 0.0, max_terms: int = 0, eps_fwd: float = 0.0,
        max_terms_fwd: int = 0, max_products: int = 0, batch: int = 1, batch_order: int = 1,
        fwd_cap: str = "gate") -> OracleSum:
    """Propagated noise absorption (Section I.A).  The hardware circuit is
    C_noisy = N_M G_M .. N_1 G_1.  Writing each ideal layer as N_t^{-1} N_t G_t and carrying
    the inverse maps to the end one at a time, from t = 1 up, through the later gates only,
    gives C_ideal = N'_1^{-1} .. N'_M^{-1} C_noisy, where N'_t^{-1} applies, for every
    generator E of N_t, the evolved error E' = U E U^dag with quasi-probability q.  The
    adjoint of that product acts on O with N'_1^{-1} first, so
    O~ = N'_M^{-1}( .. N'_1^{-1}(O)), each generator's map being
    O -> (1 - q) O + q E' O E' (Eq. applyantinoise; a generator's maps within one layer
    commute).  After every update |c| < eps is dropped and the cap applied.  With
    max_products > 0, E' O E' keeps only that many most significant products (Appendix B).
    With batch > 1, a layer's maps are taken batch at a time, each batch expanded to
    batch_order in the number of errors (Appendix C), then truncated once.
    fwd_cap="gate": each E' keeps its max_terms_fwd largest terms after every non-Clifford
    gate of its propagation; "final": only the eps_fwd threshold during the propagation, and
    the max_terms_fwd largest terms of the evolved E' kept once, before it is absorbed."""
    if fwd_cap not in ("gate", "final"):
        raise ValueError("fwd_cap must be 'gate' or 'final'")

    def evolved(t, k):
        if fwd_cap == "gate":
            return propagated_error(circuit, t, k, eps_fwd, max_terms_fwd)
        e = propagated_error(circuit, t, k, eps_fwd, 0)
        e.truncate(0.0, max_terms_fwd)
        return e

    o = observable.clone() if isinstance(observable, OracleSum) else OracleSum.from_sum(observable)
    if batch > 1:
        for t, layer in enumerate(circuit.layers):
            lam = np.asarray(layer.lam, np.float64)
            for k0 in range(0, layer.n_gen, batch):
                ks = range(k0, min(k0 + batch, layer.n_gen))
                es = [evolved(t, k) for k in ks]
                o.antinoise_batch(es, [antinoise_q(float(lam[k])) for k in ks], batch_order, eps)
                o.truncate(eps, max_terms)
        return o
    for t, layer in enumerate(circuit.layers):
        for k in range(layer.n_gen):
            e = evolved(t, k)
            qk = antinoise_q(float(np.asarray(layer.lam)[k]))
            if max_products > 0:
                o.antinoise_topk(e, qk, max_products)
            else:
                o.antinoise(e, qk)
            o.truncate(eps, max_terms)
    return o


def run_workload(wl) -> OracleSum:
    return noise_canceling(wl.circuit, wl.observable, wl.eps, wl.max_terms, wl.mode, wl.max_order)
