"""Seeded synthetic inputs for the noise-canceling Pauli-propagation path.

This module builds the *inputs* only: square lattices, transverse-field Ising
Trotter circuits written as lists of Pauli-rotation generators with their angles,
Pauli-Lindblad generator lists with seeded rates, observables, random Pauli sums
and the seeded request stream of the serving loop.  It holds none of the method's
arithmetic (no anticommutation test, branching, rescaling, merging, truncation or
expectation), so the CPU reference and the HIP path can both consume it without
sharing any of the computation they are compared on.

Conventions
-----------
* A Pauli string on ``n`` qubits is two bit vectors ``x`` and ``z`` packed into
  ``W = ceil(n / 64)`` little-endian ``uint64`` words each: qubit ``q`` lives in
  word ``q // 64``, bit ``q % 64``.  ``(x_q, z_q) = (1, 0)`` is X, ``(0, 1)`` is Z
  and ``(1, 1)`` is Y (the Hermitian string ``i^{|x&z|} X^x Z^z``).
* A circuit is a time-ordered list of layers.  Each layer is a list of Pauli
  rotations ``exp(-i theta R / 2)`` (the gate form of the paper's Section I,
  Eq. evolve_gate) applied in list order, followed by one Pauli-Lindblad channel:
  a composition of local channels, one per generator ``E_k`` with strength
  ``lambda_k`` (Section I, the channel form above Eq. evolve_gate).
* The lattice of an ``R x C`` configuration has ``R`` rows and ``C`` columns,
  site ``(r, c)`` is qubit ``r * C + c``; edges are listed horizontal first
  (row-major), then vertical (row-major).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

PAULI_BITS = {"I": (0, 0), "X": (1, 0), "Y": (1, 1), "Z": (0, 1)}


def n_words(n_qubits: int) -> int:
    """Number of 64-bit words per bit vector for ``n_qubits`` qubits."""
    if n_qubits <= 0:
        raise ValueError("n_qubits must be positive")
    return (n_qubits + 63) // 64


def _set_bit(words: np.ndarray, q: int) -> None:
    words[q // 64] |= np.uint64(1) << np.uint64(q % 64)


def pauli_masks(n_qubits: int, ops: Dict[int, str]) -> Tuple[np.ndarray, np.ndarray]:
    """Pack ``{qubit: 'X'|'Y'|'Z'|'I'}`` into ``(x[W], z[W])`` uint64 words."""
    w = n_words(n_qubits)
    x = np.zeros(w, dtype=np.uint64)
    z = np.zeros(w, dtype=np.uint64)
    for q, p in ops.items():
        if not 0 <= q < n_qubits:
            raise ValueError(f"qubit {q} outside 0..{n_qubits - 1}")
        bx, bz = PAULI_BITS[p]
        if bx:
            _set_bit(x, q)
        if bz:
            _set_bit(z, q)
    return x, z


def pauli_label(x: np.ndarray, z: np.ndarray, n_qubits: int) -> str:
    """Dense label, qubit 0 first (debugging aid)."""
    out = []
    for q in range(n_qubits):
        bx = (int(x[q // 64]) >> (q % 64)) & 1
        bz = (int(z[q // 64]) >> (q % 64)) & 1
        out.append("IZXY"[bx * 2 + bz])
    return "".join(out)


# ----------------------------------------------------------------------------------------
# Lattice
# ----------------------------------------------------------------------------------------
@dataclass(frozen=True)
class Lattice:
    rows: int
    cols: int

    @property
    def n(self) -> int:
        return self.rows * self.cols

    def site(self, r: int, c: int) -> int:
        return r * self.cols + c

    @property
    def horizontal_edges(self) -> List[Tuple[int, int]]:
        return [(self.site(r, c), self.site(r, c + 1))
                for r in range(self.rows) for c in range(self.cols - 1)]

    @property
    def vertical_edges(self) -> List[Tuple[int, int]]:
        return [(self.site(r, c), self.site(r + 1, c))
                for r in range(self.rows - 1) for c in range(self.cols)]

    @property
    def edges(self) -> List[Tuple[int, int]]:
        return self.horizontal_edges + self.vertical_edges

    @property
    def plaquettes(self) -> List[Tuple[int, int, int, int]]:
        return [(self.site(r, c), self.site(r, c + 1), self.site(r + 1, c), self.site(r + 1, c + 1))
                for r in range(self.rows - 1) for c in range(self.cols - 1)]


# ----------------------------------------------------------------------------------------
# Circuits
# ----------------------------------------------------------------------------------------
@dataclass
class Layer:
    """One circuit layer: rotations (applied in list order), then one PL channel."""
    gx: np.ndarray          # uint64 [G, W]   rotation generators R_g, x part
    gz: np.ndarray          # uint64 [G, W]   z part
    theta: np.ndarray       # float64 [G]     U_g = exp(-i theta_g R_g / 2)
    ex: np.ndarray          # uint64 [K, W]   Pauli-Lindblad generators E_k, x part
    ez: np.ndarray          # uint64 [K, W]
    lam: np.ndarray         # float64 [K]     strengths lambda_k >= 0

    @property
    def n_gates(self) -> int:
        return int(self.theta.shape[0])

    @property
    def n_gen(self) -> int:
        return int(self.lam.shape[0])


@dataclass
class Circuit:
    n_qubits: int
    layers: List[Layer] = field(default_factory=list)
    name: str = ""

    @property
    def W(self) -> int:
        return n_words(self.n_qubits)


def _stack(masks: Sequence[Tuple[np.ndarray, np.ndarray]], w: int) -> Tuple[np.ndarray, np.ndarray]:
    if not masks:
        return np.zeros((0, w), np.uint64), np.zeros((0, w), np.uint64)
    return (np.stack([m[0] for m in masks]).astype(np.uint64),
            np.stack([m[1] for m in masks]).astype(np.uint64))


def make_layer(n_qubits: int, gates: Sequence[Tuple[Dict[int, str], float]],
               gens: Sequence[Tuple[Dict[int, str], float]]) -> Layer:
    """Build a layer from label dictionaries: ``gates`` = [(ops, theta)], ``gens`` = [(ops, lambda)]."""
    w = n_words(n_qubits)
    gx, gz = _stack([pauli_masks(n_qubits, ops) for ops, _ in gates], w)
    ex, ez = _stack([pauli_masks(n_qubits, ops) for ops, _ in gens], w)
    return Layer(gx, gz, np.array([t for _, t in gates], dtype=np.float64),
                 ex, ez, np.array([l for _, l in gens], dtype=np.float64))


def pl_generator_labels(lat: Lattice) -> List[Dict[int, str]]:
    """Generator list of one noise layer: every weight-1 Pauli per site (sites row-major,
    X, Y, Z), then the nine weight-2 Paulis of every edge (horizontal edges first, each
    edge's ``(P_a, P_b)`` in lexicographic X < Y < Z order)."""
    labels: List[Dict[int, str]] = []
    for q in range(lat.n):
        for p in "XYZ":
            labels.append({q: p})
    for a, b in lat.edges:
        for pa in "XYZ":
            for pb in "XYZ":
                labels.append({a: pa, b: pb})
    return labels


def tfim_circuit(rows: int, cols: int, steps: int, theta_j: float, theta_h: float,
                 rate_lo: float, rate_hi: float, seed: int = 0,
                 noise: str = "every_layer") -> Circuit:
    """First-order TFIM Trotter circuit on an open ``rows x cols`` lattice.

    Each step is a layer of ``R_ZZ(theta_j)`` on every edge followed by a layer of
    ``R_X(theta_h)`` on every site.  ``noise='every_layer'`` puts a Pauli-Lindblad
    channel after both layers; ``'entangling'`` only after the ``R_ZZ`` layers (the
    placement of the paper's numerics, Fig. 3 caption); ``'none'`` draws no channel.
    Rates are drawn with ``numpy.random.default_rng(seed)``: one ``uniform(lo, hi, K)``
    vector per noisy layer, in time order.
    """
    lat = Lattice(rows, cols)
    n = lat.n
    rng = np.random.default_rng(seed)
    gen_labels = pl_generator_labels(lat)
    k = len(gen_labels)
    w = n_words(n)
    ex, ez = _stack([pauli_masks(n, g) for g in gen_labels], w)
    zz = [({a: "Z", b: "Z"}, theta_j) for a, b in lat.edges]
    xx = [({q: "X"}, theta_h) for q in range(n)]
    layers: List[Layer] = []
    for _ in range(steps):
        for kind, gates in (("zz", zz), ("x", xx)):
            noisy = noise == "every_layer" or (noise == "entangling" and kind == "zz")
            gx, gz = _stack([pauli_masks(n, ops) for ops, _ in gates], w)
            theta = np.array([t for _, t in gates], dtype=np.float64)
            if noisy:
                lam = rng.uniform(rate_lo, rate_hi, k)
                layers.append(Layer(gx, gz, theta, ex.copy(), ez.copy(), lam))
            else:
                layers.append(Layer(gx, gz, theta, np.zeros((0, w), np.uint64),
                                    np.zeros((0, w), np.uint64), np.zeros(0)))
    return Circuit(n, layers, name=f"tfim_{rows}x{cols}_s{steps}")


# ----------------------------------------------------------------------------------------
# Observables (Pauli sums)
# ----------------------------------------------------------------------------------------
@dataclass
class PauliSum:
    n_qubits: int
    x: np.ndarray      # uint64 [N, W]
    z: np.ndarray      # uint64 [N, W]
    c: np.ndarray      # float64 [N]

    @property
    def W(self) -> int:
        return n_words(self.n_qubits)

    def __len__(self) -> int:
        return int(self.c.shape[0])


def pauli_sum(n: int, terms: Sequence[Tuple[Dict[int, str], float]]) -> PauliSum:
    w = n_words(n)
    x, z = _stack([pauli_masks(n, ops) for ops, _ in terms], w)
    return PauliSum(n, x, z, np.array([c for _, c in terms], dtype=np.float64))


def obs_single_z(n: int, q: int) -> PauliSum:
    return pauli_sum(n, [({q: "Z"}, 1.0)])


def obs_mean_z(n: int) -> PauliSum:
    return pauli_sum(n, [({q: "Z"}, 1.0 / n) for q in range(n)])


def obs_edge_zz(n: int, a: int, b: int) -> PauliSum:
    return pauli_sum(n, [({a: "Z", b: "Z"}, 1.0)])


def obs_sum_horizontal_zz(lat: Lattice) -> PauliSum:
    return pauli_sum(lat.n, [({a: "Z", b: "Z"}, 1.0) for a, b in lat.horizontal_edges])


def obs_plaquette(lat: Lattice, r: int, c: int) -> PauliSum:
    a, b, d, e = lat.plaquettes[r * (lat.cols - 1) + c]
    return pauli_sum(lat.n, [({a: "Z", b: "Z", d: "Z", e: "Z"}, 1.0)])


def random_pauli_sum(n: int, n_terms: int, seed: int, weight: Optional[int] = None,
                     scale: float = 1.0, allow_duplicates: bool = True) -> PauliSum:
    """Random Pauli sum: each term's letters i.i.d. uniform over {I,X,Y,Z} (or exactly
    ``weight`` non-identity letters), coefficients ``scale * N(0,1)``.  Duplicated strings
    are kept unless ``allow_duplicates`` is False."""
    rng = np.random.default_rng(seed)
    w = n_words(n)
    xs = np.zeros((n_terms, w), np.uint64)
    zs = np.zeros((n_terms, w), np.uint64)
    for i in range(n_terms):
        if weight is None:
            letters = rng.integers(0, 4, n)
        else:
            letters = np.zeros(n, dtype=np.int64)
            sup = rng.choice(n, size=weight, replace=False)
            letters[sup] = rng.integers(1, 4, weight)
        for q in range(n):
            l = int(letters[q])
            if l & 1:
                xs[i, q // 64] |= np.uint64(1) << np.uint64(q % 64)
            if l & 2:
                zs[i, q // 64] |= np.uint64(1) << np.uint64(q % 64)
    c = scale * rng.standard_normal(n_terms)
    if not allow_duplicates:
        _, idx = np.unique(np.concatenate([xs, zs], axis=1), axis=0, return_index=True)
        idx = np.sort(idx)
        xs, zs, c = xs[idx], zs[idx], c[idx]
    return PauliSum(n, xs, zs, c)


def random_pauli_arrays(n: int, n_terms: int, seed: int, density: float = 0.5) -> PauliSum:
    """Vectorised random strings for large sizes: each x/z bit is 1 with probability
    ``density``; coefficients uniform in ``(-1, 1)`` excluding a small band around 0."""
    rng = np.random.default_rng(seed)
    w = n_words(n)
    bits = rng.random((n_terms, 2, n)) < density
    words = np.zeros((n_terms, 2, w), np.uint64)
    for q in range(n):
        words[:, :, q // 64] |= bits[:, :, q].astype(np.uint64) << np.uint64(q % 64)
    c = rng.uniform(0.05, 1.0, n_terms) * rng.choice([-1.0, 1.0], n_terms)
    return PauliSum(n, np.ascontiguousarray(words[:, 0]), np.ascontiguousarray(words[:, 1]), c)


# ----------------------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    circuit: Circuit
    observable: PauliSum
    eps: float
    max_terms: int          # 0 = no cap
    mode: str               # "greedy" (propagated noise absorption) | "error_order" (Clifford-Dyson)
    max_order: int          # error-order mode only
    precision: str          # "f64" | "f32k"


def tfim_workload(name: str, rows: int, cols: int, steps: int, theta_j: float, theta_h: float,
                  rate_lo: float, rate_hi: float, obs: str, eps: float, max_terms: int = 0,
                  mode: str = "greedy", max_order: int = 2, precision: str = "f64",
                  seed: int = 0, noise: str = "every_layer", obs_site: Optional[Tuple[int, int]] = None) -> Workload:
    lat = Lattice(rows, cols)
    circ = tfim_circuit(rows, cols, steps, theta_j, theta_h, rate_lo, rate_hi, seed=seed, noise=noise)
    if obs == "center_z":
        o = obs_single_z(lat.n, lat.site(rows // 2, cols // 2))
    elif obs == "site_z":
        assert obs_site is not None
        o = obs_single_z(lat.n, lat.site(*obs_site))
    elif obs == "mean_z":
        o = obs_mean_z(lat.n)
    elif obs == "horizontal_zz":
        o = obs_sum_horizontal_zz(lat)
    else:
        raise ValueError(obs)
    return Workload(name, circ, o, eps, max_terms, mode, max_order, precision)


HALF_PI = math.pi / 2


def named_workload(name: str, **overrides) -> Workload:
    """The named configurations (sizes as stated; ``overrides`` shrink them for tests):

    * ``tfim3x3``     -- 3x3, 4 steps, theta_J 0.3, theta_h 0.7, rates U[1e-4,1e-3],
                         Z on the centre qubit, eps 1e-4, no cap, FP64.
    * ``tfim7x8_pna`` -- 7x8 (56 q), 10 steps, theta_J -pi/2 (Clifford), theta_h 0.5,
                         rates U[1e-4,2e-3], mean of Z, eps 1e-5, cap 2^24.
    * ``tfim7x8_cd``  -- 7x8, 12 steps, theta_J -pi/2, theta_h 0.3, rates U[1e-4,2e-3],
                         Z at site (3,4), eps 1e-6, error orders <= 2.
    * ``tfim8x16``    -- 8x16 (128 q), 8 steps, theta_J 0.25, theta_h 0.6,
                         rates U[1e-4,1e-3], sum of horizontal ZZ, eps 1e-6, cap 2^28.
    """
    base = {
        "tfim3x3": dict(rows=3, cols=3, steps=4, theta_j=0.3, theta_h=0.7, rate_lo=1e-4,
                        rate_hi=1e-3, obs="center_z", eps=1e-4, max_terms=0),
        "tfim7x8_pna": dict(rows=7, cols=8, steps=10, theta_j=-HALF_PI, theta_h=0.5, rate_lo=1e-4,
                            rate_hi=2e-3, obs="mean_z", eps=1e-5, max_terms=1 << 24),
        "tfim7x8_cd": dict(rows=7, cols=8, steps=12, theta_j=-HALF_PI, theta_h=0.3, rate_lo=1e-4,
                           rate_hi=2e-3, obs="site_z", obs_site=(3, 4), eps=1e-6, max_terms=0,
                           mode="error_order", max_order=2),
        "tfim8x16": dict(rows=8, cols=16, steps=8, theta_j=0.25, theta_h=0.6, rate_lo=1e-4,
                         rate_hi=1e-3, obs="horizontal_zz", eps=1e-6, max_terms=1 << 28),
    }[name]
    base.update(overrides)
    return tfim_workload(name, **base)


# ----------------------------------------------------------------------------------------
# Serving request stream
# ----------------------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival_s: float
    workload: Workload


def serving_stream(n_requests: int, rate_hz: float = 200.0, seed_arrivals: int = 0,
                   seed_requests: int = 1, rows=(4, 8), cols=(4, 16), steps=(5, 20),
                   rate_lo: float = 1e-4, rate_hi: float = 1e-3,
                   max_terms: int = 1 << 22) -> List[Request]:
    """Poisson arrivals (exponential gaps, ``seed_arrivals``) of TFIM propagation requests.

    Per request (``seed_requests`` stream): rows ~ U{rows}, cols ~ U{cols}, steps ~ U{steps},
    theta_J, theta_h ~ U[-pi/2, pi/2], observable uniform over {single Z at a random site,
    ZZ on a random edge, ZZZZ on a random plaquette}, eps uniform over {1e-4,1e-5,1e-6},
    precision uniform over {f32k, f64}, rates U[rate_lo, rate_hi] drawn with the request's
    own seed, per-request cap ``max_terms``.
    """
    ra = np.random.default_rng(seed_arrivals)
    rq = np.random.default_rng(seed_requests)
    t = 0.0
    out: List[Request] = []
    for rid in range(n_requests):
        t += float(ra.exponential(1.0 / rate_hz))
        r = int(rq.integers(rows[0], rows[1] + 1))
        c = int(rq.integers(cols[0], cols[1] + 1))
        s = int(rq.integers(steps[0], steps[1] + 1))
        tj = float(rq.uniform(-HALF_PI, HALF_PI))
        th = float(rq.uniform(-HALF_PI, HALF_PI))
        kind = int(rq.integers(0, 3))
        eps = [1e-4, 1e-5, 1e-6][int(rq.integers(0, 3))]
        prec = ["f32k", "f64"][int(rq.integers(0, 2))]
        seed = int(rq.integers(0, 2**31 - 1))
        lat = Lattice(r, c)
        circ = tfim_circuit(r, c, s, tj, th, rate_lo, rate_hi, seed=seed)
        if kind == 0:
            o = obs_single_z(lat.n, int(rq.integers(0, lat.n)))
        elif kind == 1:
            a, b = lat.edges[int(rq.integers(0, len(lat.edges)))]
            o = obs_edge_zz(lat.n, a, b)
        else:
            p = int(rq.integers(0, len(lat.plaquettes)))
            o = obs_plaquette(lat, p // (c - 1), p % (c - 1))
        wl = Workload(f"req{rid}", circ, o, eps, max_terms, "greedy", 2, prec)
        out.append(Request(rid, t, wl))
    return out
