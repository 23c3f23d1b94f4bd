"""Brute-force numpy checker for up to six qubits -- TEST INFRASTRUCTURE.

An independent second route to the same definitions, used only to pin the
C oracle:

* rotation gates are matrix exponentials of their generators computed by
  ``scipy.linalg.expm`` (RX/RY/RZ(t) = exp(-i t P/2), RZZ(t) =
  exp(-i t Z(x)Z/2), the controlled rotations exp(-i t |1><1| (x) P / 2),
  U3 as a phase times RZ RY RZ), controlled gates are built from projectors
  (|0><0| (x) I + |1><1| (x) V), the swap as (I + XX + YY + ZZ)/2 and the
  Hadamard as (X + Z)/sqrt(2);
* a gate on wires (w_1..w_k) of an n-qubit register is embedded as a full
  2^n x 2^n matrix by Kronecker products, ``kron(I_left, U, I_right)``, after
  permuting the wires into a contiguous ascending block (wire 0 = leftmost
  factor = most significant bit);
* observables are Kronecker products of 2x2 Pauli matrices.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.linalg import expm

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
P0 = np.array([[1, 0], [0, 0]], dtype=complex)
P1 = np.array([[0, 0], [0, 1]], dtype=complex)
PAULI = {"I": I2, "X": PX, "Y": PY, "Z": PZ}


def named(op: str, theta: float = 0.0) -> np.ndarray:
    if op == "h":
        return (PX + PZ) / np.sqrt(2.0)
    if op in ("x", "y", "z"):
        return PAULI[op.upper()].copy()
    if op in ("rx", "ry", "rz"):
        return expm(-0.5j * theta * PAULI[op[1].upper()])
    if op == "cnot":
        return np.kron(P0, I2) + np.kron(P1, PX)
    if op == "cz":
        return np.kron(P0, I2) + np.kron(P1, PZ)
    if op == "cp":
        return np.kron(P0, I2) + np.kron(P1, np.diag([1.0, np.exp(1j * theta)]))
    if op == "swap":
        return (np.eye(4) + np.kron(PX, PX) + np.kron(PY, PY) + np.kron(PZ, PZ)) / 2.0
    if op == "rzz":
        return expm(-0.5j * theta * np.kron(PZ, PZ))
    if op in ("rxx", "ryy"):
        P = PAULI[op[1].upper()]
        return expm(-0.5j * theta * np.kron(P, P))
    if op in ("crx", "cry", "crz"):
        return expm(-0.5j * theta * np.kron(P1, PAULI[op[2].upper()]))
    raise ValueError(op)


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    """e^{i (phi + lambda)/2} RZ(phi) RY(theta) RZ(lambda), each rotation a
    matrix exponential of its generator."""
    rz = lambda a: expm(-0.5j * a * PZ)
    return np.exp(0.5j * (phi + lam)) * rz(phi) @ expm(-0.5j * theta * PY) @ rz(lam)


def _perm_matrix(n: int, order) -> np.ndarray:
    """Permutation matrix Q with (Q psi) having wire order[i] at position i."""
    N = 1 << n
    Q = np.zeros((N, N))
    for j in range(N):
        bits = [(j >> (n - 1 - w)) & 1 for w in range(n)]
        newbits = [bits[order[i]] for i in range(n)]
        jj = int("".join(map(str, newbits)), 2) if n else 0
        Q[jj, j] = 1.0
    return Q


def embed(U: np.ndarray, wires, n: int) -> np.ndarray:
    k = len(wires)
    rest = [w for w in range(n) if w not in wires]
    order = list(wires) + rest           # target wires first, in the given order
    Q = _perm_matrix(n, order)
    full = np.kron(U, np.eye(1 << (n - k)))
    return Q.T @ full @ Q


def embed_adjacent(U: np.ndarray, first: int, n: int) -> np.ndarray:
    """kron(I_{2^first}, U, I_rest) for ascending adjacent wires."""
    k = int(np.log2(U.shape[0]))
    return np.kron(np.kron(np.eye(1 << first), U), np.eye(1 << (n - first - k)))


def gate_angle(g, params, data, b=0, k=0) -> float:
    if g.src == "param":
        p = np.asarray(params, float)
        return g.scale * (p[b, g.idx + k] if p.ndim == 2 else p[g.idx + k])
    if g.src == "data":
        return g.scale * float(np.asarray(data, float)[b, g.idx + k])
    return g.scale


def gate_full(g, n, params=None, data=None, b=0) -> np.ndarray:
    if g.op == "unitary":
        U = np.asarray(g.matrix, complex)
    elif g.op == "u3":
        U = u3(*(gate_angle(g, params, data, b, k) for k in range(3)))
    else:
        U = named(g.op, gate_angle(g, params, data, b))
    return embed(U, list(g.wires), n)


def circuit_unitary(circuit, params=None, data=None, b=0) -> np.ndarray:
    assert circuit.n <= 6, "brute force only for tiny registers"
    U = np.eye(1 << circuit.n, dtype=complex)
    for g in circuit.gates:
        U = gate_full(g, circuit.n, params, data, b) @ U
    return U


def state(circuit, params=None, data=None, b=0) -> np.ndarray:
    return circuit_unitary(circuit, params, data, b)[:, 0].copy()


def pauli_full(letters: str) -> np.ndarray:
    M = np.ones((1, 1), dtype=complex)
    for l in letters:
        M = np.kron(M, PAULI[l])
    return M


def expval(psi, observable) -> float:
    return float(sum(c * np.vdot(psi, pauli_full(l) @ psi).real for c, l in observable))


def all_wire_tuples(n: int, k: int):
    return list(itertools.permutations(range(n), k))
