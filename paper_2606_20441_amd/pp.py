"""ctypes binding of ``libpp.so`` (C ABI in ``include/pp.h``).

Argument marshalling only: every step of the propagation runs in the library's HIP
kernels.  PyTorch supplies the HIP stream and, optionally, device memory through its
caching allocator.  Loading fails loudly if the library was not built.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpp.so")

PP_OK, PP_ERR_INVALID, PP_ERR_OOM, PP_ERR_DEVICE, PP_ERR_UNSUPPORTED = 0, 1, 2, 3, 4
PP_F64, PP_F32_KAHAN = 0, 1
PP_MODE_GREEDY, PP_MODE_ERROR_ORDER, PP_MODE_SINE_ORDER = 0, 1, 2
PP_HEISENBERG, PP_FORWARD = 1, -1

PRECISIONS = {"f64": PP_F64, "f32k": PP_F32_KAHAN}
MODES = {"greedy": PP_MODE_GREEDY, "error_order": PP_MODE_ERROR_ORDER, "sine_order": PP_MODE_SINE_ORDER}


class PPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pp status {status}: {msg}")
        self.status = status


class pp_trunc(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_terms", C.c_int64), ("max_order", C.c_int)]


_u64p = C.POINTER(C.c_uint64)
_f64p = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)


class pp_layer(C.Structure):
    _fields_ = [("n_gates", C.c_int), ("gx", _u64p), ("gz", _u64p), ("theta", _f64p), ("dir", C.c_int),
                ("n_gen", C.c_int), ("ex", _u64p), ("ez", _u64p), ("lambda_", _f64p),
                ("noise_sign", C.c_int), ("noise_after_gates", C.c_int)]


class pp_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("algo_bytes", C.c_double), ("items", C.c_double), ("layer_bytes", C.c_double)]


class pp_layer_stats(C.Structure):
    _fields_ = [("n_in", C.c_int64), ("n_out", C.c_int64), ("n_peak", C.c_int64), ("n_fallback", C.c_int64),
                ("n_capped", C.c_int64), ("dropped_l1", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None
_lib_lock = threading.Lock()

# Live handles, released before interpreter shutdown tears PyTorch down (the library may
# call back into PyTorch's allocator while releasing device memory).
import atexit
import weakref

_live_obs = weakref.WeakSet()
_live_ctx = weakref.WeakSet()


@atexit.register
def _release_all():
    for o in list(_live_obs):
        try:
            o.destroy()
        except Exception:
            pass
    for c in list(_live_ctx):
        try:
            c.close()
        except Exception:
            pass

EXPORTED = ["pp_ctx_create", "pp_ctx_destroy", "pp_create_observable", "pp_apply_layer", "pp_truncate",
            "pp_expectation", "pp_expectation_noalloc", "pp_size", "pp_export", "pp_destroy", "pp_last_error", "pp_timing_enable",
            "pp_timing_read", "pp_last_layer_stats"]


def lib():
    """Load ``libpp.so`` (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_20441_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.pp_last_error.restype = C.c_char_p
        L.pp_ctx_create.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]
        L.pp_ctx_create.restype = C.c_int
        L.pp_ctx_destroy.argtypes = [C.c_void_p]
        L.pp_create_observable.argtypes = [C.c_void_p, C.c_int, C.c_int64, _u64p, _u64p, _f64p, C.c_int, C.c_int,
                                           pp_trunc, C.POINTER(C.c_void_p)]
        L.pp_create_observable.restype = C.c_int
        L.pp_set_terms.argtypes = [C.c_void_p, C.c_int64, _u64p, _u64p, _f64p]
        L.pp_set_terms.restype = C.c_int
        L.pp_apply_layer.argtypes = [C.c_void_p, C.POINTER(pp_layer)]
        L.pp_apply_layer.restype = C.c_int
        L.pp_truncate.argtypes = [C.c_void_p, C.c_double, C.c_int64]
        L.pp_apply_antinoise.argtypes = [C.c_void_p, C.c_void_p, C.c_double]
        L.pp_apply_antinoise.restype = C.c_int
        L.pp_apply_antinoise_topk.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_int64]
        L.pp_apply_antinoise_topk.restype = C.c_int
        L.pp_apply_antinoise_batch.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), _f64p, C.c_int, C.c_int]
        L.pp_apply_antinoise_batch.restype = C.c_int
        L.pp_truncate.restype = C.c_int
        L.pp_expectation.argtypes = [C.c_void_p, _u64p, _f64p]
        L.pp_expectation.restype = C.c_int
        L.pp_expectation_noalloc.argtypes = [C.c_void_p, _u64p, _f64p]
        L.pp_expectation_noalloc.restype = C.c_int
        L.pp_size.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.pp_size.restype = C.c_int
        L.pp_export.argtypes = [C.c_void_p, _u64p, _u64p, _f64p, _u8p]
        L.pp_export.restype = C.c_int
        L.pp_destroy.argtypes = [C.c_void_p]
        L.pp_timing_enable.argtypes = [C.c_void_p, C.c_int]
        L.pp_timing_enable.restype = C.c_int
        L.pp_timing_read.argtypes = [C.c_void_p, C.POINTER(pp_kernel_stat), C.c_int, C.c_int]
        L.pp_timing_read.restype = C.c_int
        L.pp_last_layer_stats.argtypes = [C.c_void_p, C.POINTER(pp_layer_stats)]
        L.pp_last_layer_stats.restype = C.c_int
        _lib = L
        return L


def _check(status: int):
    if status != PP_OK:
        raise PPError(status, lib().pp_last_error().decode())


def _ptr(a: Optional[np.ndarray], t):
    return None if a is None else a.ctypes.data_as(t)


def _words(a, w: int) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(-1, w))


class Context:
    """A device, a HIP stream and (optionally) PyTorch's caching allocator."""

    def __init__(self, device: int = 0, stream=None, torch_allocator: bool = True,
                 limit_bytes: Optional[int] = None):
        """`limit_bytes` (torch allocator only) caps the device bytes this context may hold at
        once; an allocation beyond it fails, and the library reports PP_ERR_OOM."""
        import torch
        self.device = device
        self._torch_stream = stream if stream is not None else torch.cuda.current_stream(device)
        handle = C.c_void_p(self._torch_stream.cuda_stream)
        self._alloc_cb = None
        self._release_cb = None
        self.limit_bytes = limit_bytes
        self.live_bytes = 0
        self.peak_bytes = 0
        self.n_allocs = 0
        self._sizes = {}
        if torch_allocator:
            dev = torch.device("cuda", device)
            st = self._torch_stream

            def _alloc(nbytes, _user):
                nbytes = int(nbytes)
                if self.limit_bytes is not None and self.live_bytes + nbytes > self.limit_bytes:
                    return None
                try:
                    p = int(torch.cuda.caching_allocator_alloc(nbytes, dev, st))
                except Exception:
                    return None
                self._sizes[p] = nbytes
                self.n_allocs += 1
                self.live_bytes += nbytes
                self.peak_bytes = max(self.peak_bytes, self.live_bytes)
                return p

            def _release(p, _user):
                self.live_bytes -= self._sizes.pop(int(p), 0)
                torch.cuda.caching_allocator_delete(int(p))

            self._alloc_cb = ALLOC_FN(_alloc)
            self._release_cb = RELEASE_FN(_release)
        out = C.c_void_p()
        a = C.cast(self._alloc_cb, C.c_void_p) if self._alloc_cb else None
        r = C.cast(self._release_cb, C.c_void_p) if self._release_cb else None
        _check(lib().pp_ctx_create(device, handle, a, r, None, C.byref(out)))
        self._h = out
        self._obs = weakref.WeakSet()
        _live_ctx.add(self)

    def close(self):
        if getattr(self, "_h", None):
            for o in list(getattr(self, "_obs", ())):
                o.destroy()
            lib().pp_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timing(self, enable: bool = True):
        _check(lib().pp_timing_enable(self._h, int(enable)))

    def timing_read(self, reset: bool = True) -> List[dict]:
        n = lib().pp_timing_read(self._h, None, 0, 0)
        if n < 0:
            raise PPError(PP_ERR_DEVICE, lib().pp_last_error().decode())
        arr = (pp_kernel_stat * max(n, 1))()
        lib().pp_timing_read(self._h, arr, n, int(reset))
        return [dict(name=arr[i].name.decode(), launches=int(arr[i].launches), total_ms=float(arr[i].total_ms),
                     algo_bytes=float(arr[i].algo_bytes), items=float(arr[i].items),
                     layer_bytes=float(arr[i].layer_bytes)) for i in range(n)]


class Observable:
    """A Pauli sum resident on the device (``pp_obs``)."""

    def __init__(self, ctx: Context, n_qubits: int, x, z, c, precision: str = "f64", mode: str = "greedy",
                 eps: float = 0.0, max_terms: int = 0, max_order: int = 2):
        self.ctx = ctx
        self.n = int(n_qubits)
        self.W = (self.n + 63) // 64
        self.mode = mode
        xw = _words(x, self.W)
        zw = _words(z, self.W)
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(-1))
        out = C.c_void_p()
        tr = pp_trunc(float(eps), int(max_terms), int(max_order))
        _check(lib().pp_create_observable(ctx._h, self.n, cc.shape[0], _ptr(xw, _u64p), _ptr(zw, _u64p),
                                          _ptr(cc, _f64p), PRECISIONS[precision], MODES[mode], tr, C.byref(out)))
        self._h = out
        ctx._obs.add(self)
        _live_obs.add(self)

    @classmethod
    def from_sum(cls, ctx: Context, ps, **kw) -> "Observable":
        return cls(ctx, ps.n_qubits, ps.x, ps.z, ps.c, **kw)

    def destroy(self):
        if getattr(self, "_h", None):
            lib().pp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def apply_layer(self, layer, direction: int = PP_HEISENBERG, with_gates: bool = True, with_noise: bool = True,
                    noise_sign: int = 1, noise_after_gates: bool = True):
        W = self.W
        ng = layer.n_gates if with_gates else 0
        nk = layer.n_gen if with_noise else 0
        keep = []
        L = pp_layer()
        L.n_gates = ng
        L.dir = int(direction)
        if ng:
            gx, gz = _words(layer.gx, W), _words(layer.gz, W)
            th = np.ascontiguousarray(layer.theta, np.float64)
            keep += [gx, gz, th]
            L.gx, L.gz, L.theta = _ptr(gx, _u64p), _ptr(gz, _u64p), _ptr(th, _f64p)
        L.n_gen = nk
        if nk:
            ex, ez = _words(layer.ex, W), _words(layer.ez, W)
            lam = np.ascontiguousarray(layer.lam, np.float64)
            keep += [ex, ez, lam]
            L.ex, L.ez, L.lambda_ = _ptr(ex, _u64p), _ptr(ez, _u64p), _ptr(lam, _f64p)
        L.noise_sign = int(noise_sign)
        L.noise_after_gates = int(bool(noise_after_gates))
        _check(lib().pp_apply_layer(self._h, C.byref(L)))
        del keep

    def apply_antinoise(self, eprime: "Observable", lam: float):
        """O -> (1 - q) O + q E' O E' for a generator of strength lam, q taken by the
        library (``pp_apply_antinoise``)."""
        _check(lib().pp_apply_antinoise(self._h, eprime._h, float(lam)))

    def apply_antinoise_batch(self, eprimes, lams, order: int = 1):
        """A batch of commuting antinoise maps to first or second order in the number of
        errors (``pp_apply_antinoise_batch``); lams are the generators' strengths."""
        hs = (C.c_void_p * len(eprimes))(*[e._h.value if isinstance(e._h, C.c_void_p) else e._h for e in eprimes])
        la = np.ascontiguousarray(np.asarray(lams, np.float64))
        _check(lib().pp_apply_antinoise_batch(self._h, hs, _ptr(la, _f64p), len(eprimes), int(order)))

    def apply_antinoise_topk(self, eprime: "Observable", lam: float, max_products: int):
        """As ``apply_antinoise`` with E' O E' limited to its most significant products
        (``pp_apply_antinoise_topk``)."""
        _check(lib().pp_apply_antinoise_topk(self._h, eprime._h, float(lam), int(max_products)))

    def set_terms(self, x, z, c):
        """Replace the terms, keeping the device buffers (``pp_set_terms``)."""
        xw = _words(x, self.W)
        zw = _words(z, self.W)
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(-1))
        _check(lib().pp_set_terms(self._h, cc.shape[0], _ptr(xw, _u64p), _ptr(zw, _u64p), _ptr(cc, _f64p)))

    def truncate(self, eps: float, max_terms: int = 0):
        _check(lib().pp_truncate(self._h, float(eps), int(max_terms)))

    def expectation(self, basis=None) -> float:
        out = C.c_double()
        b = None if basis is None else _words(basis, self.W).reshape(-1)
        _check(lib().pp_expectation(self._h, _ptr(b, _u64p), C.byref(out)))
        return float(out.value)

    def expectation_noalloc(self, basis=None) -> float:
        """<b|O|b> without any device allocation (``pp_expectation_noalloc``)."""
        out = C.c_double()
        b = None if basis is None else _words(basis, self.W).reshape(-1)
        _check(lib().pp_expectation_noalloc(self._h, _ptr(b, _u64p), C.byref(out)))
        return float(out.value)

    def __len__(self) -> int:
        out = C.c_int64()
        _check(lib().pp_size(self._h, C.byref(out)))
        return int(out.value)

    def export(self):
        n = len(self)
        x = np.zeros((n, self.W), np.uint64)
        z = np.zeros((n, self.W), np.uint64)
        c = np.zeros(n, np.float64)
        o = np.zeros(n, np.uint8)
        if n:
            _check(lib().pp_export(self._h, _ptr(x, _u64p), _ptr(z, _u64p), _ptr(c, _f64p), _ptr(o, _u8p)))
        return x, z, c, o

    def as_dict(self):
        x, z, c, o = self.export()
        return {(tuple(int(v) for v in x[i]), tuple(int(v) for v in z[i]), int(o[i])): float(c[i])
                for i in range(len(c))}

    def last_layer_stats(self) -> dict:
        s = pp_layer_stats()
        _check(lib().pp_last_layer_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in pp_layer_stats._fields_}


def noise_canceling(ctx: Context, circuit, observable, eps: float = 0.0, max_terms: int = 0,
                    mode: str = "greedy", max_order: int = 2, precision: str = "f64",
                    on_layer=None) -> Observable:
    """O~ = D O with D = (C_ideal C_noisy^{-1})^dag (Section I.B of the paper).

    For a circuit of layers m = 1..M (gates G_m, then Pauli-Lindblad channel N_m),
    C_ideal C_noisy^{-1} = G_M..G_2 N_1^{-1} G_2^{-1} N_2^{-1} .. G_M^{-1} N_M^{-1} (the first
    layer's gates cancel).  Its adjoint applied to O therefore walks backward through
    G_M .. G_2 without noise (U^dag P U), applies N_1^{-1}, then for m = 2..M goes forward
    through G_m (U P U^dag) followed by N_m^{-1}.  In the sine-order mode the G_1 pair is
    kept (backward through G_1, then forward through G_1 before N_1^{-1}): the Euclid
    appendix expands D over every gate of C_ideal, and with a cut on the number of sines
    the two halves of the pair no longer cancel.  The library writes that mode's layers in
    the Clifford interaction picture itself.
    """
    obs = Observable.from_sum(ctx, observable, precision=precision, mode=mode, eps=eps, max_terms=max_terms,
                              max_order=max_order)
    layers = circuit.layers
    M = len(layers)
    first = 0 if mode == "sine_order" else 1
    step = 0
    for m in range(M - 1, first - 1, -1):
        obs.apply_layer(layers[m], PP_HEISENBERG, with_noise=False)
        if on_layer:
            on_layer(step, "backward", m, obs)
        step += 1
    obs.apply_layer(layers[0], PP_FORWARD, with_gates=first == 0, noise_sign=1)
    if on_layer:
        on_layer(step, "noise", 0, obs)
    step += 1
    for m in range(1, M):
        obs.apply_layer(layers[m], PP_FORWARD, noise_sign=1, noise_after_gates=True)
        if on_layer:
            on_layer(step, "forward", m, obs)
        step += 1
    return obs


def noisy_evaluation(circuit, obs_tilde: "Observable", on_layer=None) -> float:
    """Tr[O~ rho_noisy] by noisy Pauli propagation, with rho_noisy = C_noisy(|0><0|).

    This is the paper's check that propagating the mitigated observable back through the
    noisy circuit recovers the ideal value (Section III).  C_noisy = N_M G_M .. N_1 G_1, so
    its adjoint on O~ walks back from m = M to 1 applying the channel N_m itself (noise
    sign -1; a Pauli channel is its own adjoint) and then G_m^dag (U^dag P U).  The
    observable keeps its own threshold and cap, and is changed in place.
    """
    layers = circuit.layers
    for m in range(len(layers) - 1, -1, -1):
        obs_tilde.apply_layer(layers[m], PP_HEISENBERG, noise_sign=-1, noise_after_gates=False)
        if on_layer:
            on_layer(m, obs_tilde)
    return obs_tilde.expectation()


def propagated_error(ctx: Context, circuit, t: int, k: int, eps_fwd: float = 0.0, max_terms_fwd: int = 0,
                     precision: str = "f64", into: Optional[Observable] = None) -> Observable:
    """E' = U E U^dag for generator k of layer t's noise: E carried forward in time
    through the gates of layers t+1..M (Section I.A, Eq. channel_prop), on the device.  With `into` (an
    observable of the same qubit count, precision, eps_fwd and cap) its buffers are reused."""
    W = (circuit.n_qubits + 63) // 64
    layer = circuit.layers[t]
    ex = _words(layer.ex, W)[k:k + 1]
    ez = _words(layer.ez, W)[k:k + 1]
    if into is not None:
        e = into
        e.set_terms(ex, ez, np.ones(1))
    else:
        e = Observable(ctx, circuit.n_qubits, ex, ez, np.ones(1), precision=precision, eps=eps_fwd,
                       max_terms=max_terms_fwd)
    for later in circuit.layers[t + 1:]:
        e.apply_layer(later, PP_FORWARD, with_noise=False)
    return e


TAG_QUBITS = 8   # extra qubits that carry a generator's index in a batched forward propagation


class _GateLayer:
    """A layer's gates only, as pp_apply_layer reads them (no noise)."""

    def __init__(self, gx, gz, theta):
        self.gx, self.gz, self.theta = gx, gz, theta
        self.ex = self.ez = np.zeros((0, gx.shape[1]), np.uint64)
        self.lam = np.zeros(0)

    @property
    def n_gates(self) -> int:
        return int(self.theta.shape[0])

    @property
    def n_gen(self) -> int:
        return 0


def _widened_gates(circuit, n_total: int):
    """The circuit's gate layers written on n_total >= n qubits (the extra qubits untouched)."""
    W, Wt = (circuit.n_qubits + 63) // 64, (n_total + 63) // 64
    out = []
    for layer in circuit.layers:
        G = layer.n_gates
        gx = np.zeros((G, Wt), np.uint64)
        gz = np.zeros((G, Wt), np.uint64)
        if G:
            gx[:, :W] = _words(layer.gx, W)
            gz[:, :W] = _words(layer.gz, W)
        out.append(_GateLayer(gx, gz, np.ascontiguousarray(layer.theta, np.float64)))
    return out


def evolved_errors(ctx: Context, circuit, t: int, ks, eps_fwd: float = 0.0, precision: str = "f64",
                   widened=None):
    """E'_k = U E_k U^dag for the generators ks (at most 2^TAG_QUBITS of them) of layer t's
    noise, carried forward together through the gates of layers t+1..M (Section I.A,
    Eq. channel_prop) in one propagation on the device: generator ks[j] enters as
    E_{ks[j]} (x) Z^j on TAG_QUBITS extra qubits that no gate touches, so the strings of
    different generators never merge and each term keeps its generator's index; the
    threshold eps_fwd follows every non-Clifford gate, as for one generator alone.  Returns
    {k: (x, z, c)} with the extra qubits removed."""
    n = circuit.n_qubits
    nt = n + TAG_QUBITS
    W, Wt = (n + 63) // 64, (nt + 63) // 64
    ks = list(ks)
    assert len(ks) <= (1 << TAG_QUBITS)
    layer = circuit.layers[t]
    ex = _words(layer.ex, W)
    ez = _words(layer.ez, W)
    x0 = np.zeros((len(ks), Wt), np.uint64)
    z0 = np.zeros((len(ks), Wt), np.uint64)
    x0[:, :W] = ex[ks]
    z0[:, :W] = ez[ks]
    for j in range(len(ks)):
        for b in range(TAG_QUBITS):
            if (j >> b) & 1:
                q = n + b
                z0[j, q // 64] |= np.uint64(1) << np.uint64(q % 64)
    if widened is None:
        widened = _widened_gates(circuit, nt)
    e = Observable(ctx, nt, x0, z0, np.ones(len(ks)), precision=precision, eps=eps_fwd)
    try:
        for later in widened[t + 1:]:
            e.apply_layer(later, PP_FORWARD, with_noise=False)
        x, z, c, _ = e.export()
    finally:
        e.destroy()
    tag = np.zeros(len(c), np.int64)
    for b in range(TAG_QUBITS):
        q = n + b
        bit = (z[:, q // 64] >> np.uint64(q % 64)) & np.uint64(1)
        tag |= bit.astype(np.int64) << b
        z[:, q // 64] &= ~(np.uint64(1) << np.uint64(q % 64))
    x, z = np.ascontiguousarray(x[:, :W]), np.ascontiguousarray(z[:, :W])
    order = np.argsort(tag, kind="stable")
    bounds = np.searchsorted(tag[order], np.arange(len(ks) + 1))
    return {k: (x[order[bounds[j]:bounds[j + 1]]], z[order[bounds[j]:bounds[j + 1]]], c[order[bounds[j]:bounds[j + 1]]])
            for j, k in enumerate(ks)}


def pna(ctx: Context, circuit, observable, eps: float = 0.0, max_terms: int = 0, eps_fwd: float = 0.0,
        max_terms_fwd: int = 0, precision: str = "f64", on_map=None, max_products: int = 0, batch: int = 1,
        batch_order: int = 1, forward: str = "batched", on_error=None) -> Observable:
    """Propagated noise absorption (Section I.A).

    With C_noisy = N_M G_M .. N_1 G_1, inserting N_t^{-1} N_t after every G_t and carrying
    each inverse map to the end of the circuit, from t = 1 up and through the later gates
    only, gives C_ideal = N'_1^{-1} .. N'_M^{-1} C_noisy.  The adjoint of that product acts
    on O with N'_1^{-1} first: for t = 1..M and every generator E of N_t (whose maps
    commute), O -> (1 - q) O + q E' O E' with E' = U E U^dag (Eq. applyantinoise), then the
    observable's eps threshold and cap.  With max_products > 0 each E' O E' keeps only that
    many most significant products (Appendix B's heuristic conjugation).  With batch > 1 a
    layer's maps are absorbed `batch` at a time, each batch expanded to `batch_order` in the
    number of errors and merged once (Appendix C).

    forward="batched" carries up to 2^TAG_QUBITS generators of a layer forward in one
    propagation (evolved_errors), with the threshold eps_fwd after every non-Clifford gate;
    each E' is then cut to its max_terms_fwd largest terms once, on the device, before it is
    absorbed.  forward="each" propagates every generator on its own with eps_fwd and the
    max_terms_fwd cap after every non-Clifford gate.  on_error(t, k, e) sees every evolved
    error E' (an Observable) just before it is absorbed.
    """
    if forward not in ("batched", "each"):
        raise ValueError("forward must be 'batched' or 'each'")
    obs = Observable.from_sum(ctx, observable, precision=precision, eps=eps, max_terms=max_terms)
    n, W = circuit.n_qubits, (circuit.n_qubits + 63) // 64
    empty = np.zeros((0, W), np.uint64)
    # the evolved errors live in a pool of observables whose buffers are reused
    pool = [Observable(ctx, n, empty, empty, np.zeros(0), precision=precision, eps=eps_fwd, max_terms=max_terms_fwd)
            for _ in range(max(1, batch))]
    widened = _widened_gates(circuit, n + TAG_QUBITS) if forward == "batched" else None
    try:
        for t, layer in enumerate(circuit.layers):
            lam = np.asarray(layer.lam, np.float64)
            step = max(1, batch)
            evolved = {}
            for k0 in range(0, layer.n_gen, step):
                ks = range(k0, min(k0 + step, layer.n_gen))
                if forward == "batched":
                    es = []
                    for i, k in enumerate(ks):
                        if k not in evolved:
                            evolved = evolved_errors(ctx, circuit, t, range(k, min(k + (1 << TAG_QUBITS), layer.n_gen)),
                                                     eps_fwd, precision, widened)
                        x, z, c = evolved.pop(k)
                        pool[i].set_terms(x, z, c)
                        if max_terms_fwd > 0:
                            pool[i].truncate(0.0, max_terms_fwd)
                        es.append(pool[i])
                else:
                    es = [propagated_error(ctx, circuit, t, k, eps_fwd, max_terms_fwd, precision, into=pool[i])
                          for i, k in enumerate(ks)]
                if on_error:
                    for k, e in zip(ks, es):
                        on_error(t, k, e)
                if batch > 1:
                    obs.apply_antinoise_batch(es, [lam[k] for k in ks], batch_order)
                elif max_products > 0:
                    obs.apply_antinoise_topk(es[0], lam[k0], max_products)
                else:
                    obs.apply_antinoise(es[0], lam[k0])
                if on_map:
                    on_map(t, ks[-1], obs)
    finally:
        for e in pool:
            e.destroy()
    return obs


def run_workload(ctx: Context, wl, precision: Optional[str] = None, on_layer=None) -> Observable:
    return noise_canceling(ctx, wl.circuit, wl.observable, wl.eps, wl.max_terms, wl.mode, wl.max_order,
                           precision or wl.precision, on_layer=on_layer)
