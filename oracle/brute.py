"""Dense brute force for small qubit counts (n <= ~10): statevector, density matrix,
Heisenberg superoperators on explicit 2^n x 2^n matrices, and Pauli decomposition.

Test infrastructure only.  It never uses the symplectic bookkeeping of the Pauli
propagators: Paulis are explicit (permutation, phase) matrices, gates are
U = exp(-i theta R / 2) = cos(theta/2) I - i sin(theta/2) R, and channels act on
matrices as (1 - p) M + p E M E (Section I's channel definition).  That makes it an
independent pin for the FP64 reference and the HIP path.

Basis index j = sum_q b_q 2^q (qubit 0 is the least significant bit).  The Hermitian
Pauli of bit masks (x, z) is i^{|x&z|} X^x Z^z, so P|j> = i^{|x&z|} (-1)^{|z&j|} |j ^ x>.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np


def _mask(words) -> int:
    words = np.asarray(words, dtype=np.uint64).reshape(-1)
    v = 0
    for i, w in enumerate(words):
        v |= int(w) << (64 * i)
    return v


def _popc_vec(a: np.ndarray) -> np.ndarray:
    a = a.astype(np.int64)
    c = np.zeros_like(a)
    while np.any(a):
        c += a & 1
        a >>= 1
    return c


class PauliOp:
    """Explicit Pauli operator on n qubits as a permutation and a phase vector."""

    def __init__(self, n: int, x, z):
        self.n = n
        self.xm = _mask(x) if not isinstance(x, int) else x
        self.zm = _mask(z) if not isinstance(z, int) else z
        dim = 1 << n
        j = np.arange(dim, dtype=np.int64)
        self.perm = j ^ self.xm
        sign = 1 - 2 * (_popc_vec(j & self.zm) & 1)
        self.phase = (1j ** (bin(self.xm & self.zm).count("1") % 4)) * sign.astype(np.complex128)

    def matrix(self) -> np.ndarray:
        dim = 1 << self.n
        m = np.zeros((dim, dim), np.complex128)
        m[self.perm, np.arange(dim)] = self.phase
        return m

    def left(self, m: np.ndarray) -> np.ndarray:      # P @ M
        out = np.empty_like(m)
        out[self.perm, :] = self.phase[:, None] * m
        return out

    def right(self, m: np.ndarray) -> np.ndarray:     # M @ P
        return m[:, self.perm] * self.phase[None, :]

    def apply(self, psi: np.ndarray) -> np.ndarray:   # P |psi>
        out = np.empty_like(psi)
        out[self.perm] = self.phase * psi
        return out

    def conj(self, m: np.ndarray) -> np.ndarray:      # P M P
        return self.right(self.left(m))


def conj_forward(m: np.ndarray, r: PauliOp, theta: float) -> np.ndarray:
    """U M U^dag with U = cos(t/2) I - i sin(t/2) R."""
    a, b = np.cos(theta / 2), np.sin(theta / 2)
    rm, mr = r.left(m), r.right(m)
    return a * a * m + 1j * a * b * (mr - rm) + b * b * r.right(rm)


def conj_backward(m: np.ndarray, r: PauliOp, theta: float) -> np.ndarray:
    """U^dag M U with U = cos(t/2) I - i sin(t/2) R."""
    a, b = np.cos(theta / 2), np.sin(theta / 2)
    rm, mr = r.left(m), r.right(m)
    return a * a * m + 1j * a * b * (rm - mr) + b * b * r.right(rm)


def channel(m: np.ndarray, gens: Sequence[PauliOp], lam: np.ndarray, sign: int) -> np.ndarray:
    """Composition of local Pauli-Lindblad maps (1-p) M + p E M E with
    p = (1 - exp(-2 sign lambda))/2; sign = -1 gives the inverse map's quasi-probability."""
    for e, l in zip(gens, lam):
        p = (1.0 - np.exp(-2.0 * sign * l)) / 2.0
        m = (1.0 - p) * m + p * e.conj(m)
    return m


def pauli_sum_matrix(n: int, x: np.ndarray, z: np.ndarray, c: np.ndarray) -> np.ndarray:
    dim = 1 << n
    m = np.zeros((dim, dim), np.complex128)
    for i in range(len(c)):
        p = PauliOp(n, x[i], z[i])
        m[p.perm, np.arange(dim)] += c[i] * p.phase
    return m


def _wht(v: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform along the last axis (length 2^n)."""
    v = v.copy()
    n = v.shape[-1]
    h = 1
    while h < n:
        v = v.reshape(v.shape[:-1] + (n // (2 * h), 2, h))
        a = v[..., 0, :].copy()
        b = v[..., 1, :].copy()
        v[..., 0, :] = a + b
        v[..., 1, :] = a - b
        v = v.reshape(v.shape[:-3] + (n,))
        h *= 2
    return v


def pauli_decompose(m: np.ndarray, n: int, tol: float = 0.0) -> Dict[Tuple[int, int], complex]:
    """Coefficients c(x, z) = Tr(P(x,z) M) / 2^n for every Pauli with |c| > tol."""
    dim = 1 << n
    k = np.arange(dim, dtype=np.int64)
    v = m[k[None, :], k[None, :] ^ k[:, None]]     # v[x, k] = M[k, k ^ x]
    t = _wht(v)                                    # t[x, z] = sum_k (-1)^{|z&k|} M[k, k^x]
    xs = k[:, None]
    zs = k[None, :]
    ph = 1j ** (_popc_vec(xs & zs) % 4)
    coef = ph * t / dim
    out = {}
    nz = np.argwhere(np.abs(coef) > tol)
    for xi, zi in nz:
        out[(int(xi), int(zi))] = complex(coef[xi, zi])
    return out


def _layer_ops(n: int, layer) -> Tuple[List[Tuple[PauliOp, float]], List[PauliOp], np.ndarray]:
    gates = [(PauliOp(n, layer.gx[g], layer.gz[g]), float(layer.theta[g])) for g in range(layer.n_gates)]
    gens = [PauliOp(n, layer.ex[k], layer.ez[k]) for k in range(layer.n_gen)]
    return gates, gens, np.asarray(layer.lam, np.float64)


def statevector(circuit) -> np.ndarray:
    """Ideal circuit C_ideal |0>: every gate U = exp(-i theta R/2) in time order, no noise."""
    n = circuit.n_qubits
    psi = np.zeros(1 << n, np.complex128)
    psi[0] = 1.0
    for layer in circuit.layers:
        gates, _, _ = _layer_ops(n, layer)
        for r, th in gates:
            psi = np.cos(th / 2) * psi - 1j * np.sin(th / 2) * r.apply(psi)
    return psi


def density_matrix(circuit, noisy: bool = True) -> np.ndarray:
    """rho = C_noisy(|0><0|): each layer's gates in time order, then its channel."""
    n = circuit.n_qubits
    dim = 1 << n
    rho = np.zeros((dim, dim), np.complex128)
    rho[0, 0] = 1.0
    for layer in circuit.layers:
        gates, gens, lam = _layer_ops(n, layer)
        for r, th in gates:
            rho = conj_forward(rho, r, th)
        if noisy and gens:
            rho = channel(rho, gens, lam, +1)
    return rho


def _deconvolution_sequence(circuit):
    """Schroedinger-picture maps of C_ideal o C_noisy^{-1}, earliest first.

    C_noisy = N_M G_M ... N_1 G_1, so C_noisy^{-1} applies N_M^{-1}, then G_M^{-1}, ...,
    N_1^{-1}, G_1^{-1}; C_ideal then applies G_1 .. G_M.  G^{-1} undoes the layer's gates
    (last gate first, each U^dag . U)."""
    n = circuit.n_qubits
    seq = []
    layers = [_layer_ops(n, l) for l in circuit.layers]
    for gates, gens, lam in reversed(layers):
        if gens:
            seq.append(("noise_inv", gens, lam))
        for r, th in reversed(gates):
            seq.append(("u_inv", r, th))
    for gates, gens, lam in layers:
        for r, th in gates:
            seq.append(("u", r, th))
    return seq


def deconvolved_observable(circuit, obs_matrix: np.ndarray) -> np.ndarray:
    """D O = (C_ideal C_noisy^{-1})^dag O (Section I.B): the adjoint of a composition is the
    composition of adjoints in reverse order; (U . U^dag)^dag = U^dag . U, the adjoint of
    U^dag . U is U . U^dag, and Pauli maps are self-adjoint."""
    m = obs_matrix.copy()
    for op in reversed(_deconvolution_sequence(circuit)):
        if op[0] == "u":
            m = conj_backward(m, op[1], op[2])
        elif op[0] == "u_inv":
            m = conj_forward(m, op[1], op[2])
        else:
            m = channel(m, op[1], op[2], -1)
    return m


def deconvolved_orders(circuit, obs_matrix: np.ndarray, max_order: int) -> List[np.ndarray]:
    """D O as a power series in a formal parameter t that marks each inverse-noise
    generator: the inverse local map is written M + t x_k A_k(M) with
    A_k(M) = (M - E_k M E_k)/2 (the part of M anticommuting with E_k) and
    x_k = exp(2 lambda_k) - 1; returns the coefficient matrices of t^0 .. t^max_order."""
    series = [obs_matrix.copy()] + [np.zeros_like(obs_matrix) for _ in range(max_order)]
    for op in reversed(_deconvolution_sequence(circuit)):
        if op[0] == "u":
            series = [conj_backward(m, op[1], op[2]) for m in series]
        elif op[0] == "u_inv":
            series = [conj_forward(m, op[1], op[2]) for m in series]
        else:
            for e, l in zip(op[1], op[2]):
                xk = np.expm1(2.0 * l)
                for j in range(max_order, 0, -1):
                    prev = series[j - 1]
                    series[j] = series[j] + xk * (prev - e.conj(prev)) / 2.0
    return series


def expectation(m: np.ndarray, rho: np.ndarray) -> complex:
    return complex(np.trace(m @ rho))
