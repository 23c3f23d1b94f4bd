"""Seeded synthetic inputs shared by the HIP path, the oracle and the bench.

This module holds circuit *structure* and random draws only: gate lists
(which gate on which wires, which angle source), parameter and data arrays,
and Pauli-sum observables.  It contains none of the simulator's arithmetic
(no gate matrices, no state updates, no expectation values), so both sides
of every parity test can consume the same bytes without sharing code.

Conventions (paper section 4.2, API overview; listing "code:qubitcircuit"):

* a circuit is an ordered gate list on ``n`` wires, applied to |0...0>;
* a gate's angle is ``scale * v`` where ``v`` is ``params[idx]`` (src
  ``'param'``), ``data[idx]`` (src ``'data'``, the ``encode=True`` gates of the
  paper) or 1 (src ``'none'``: a fixed angle stored in ``scale``);
* ``wires`` of a controlled gate are ``(control, target)``; for ``unitary`` the
  first listed wire is the most significant bit of the matrix index;
* an observable is a list of ``(coef, letters)`` terms, ``letters`` a string
  over ``IXYZ`` with ``letters[w]`` acting on wire ``w``.

Seeds: config ``c`` draws from ``numpy.random.default_rng(1000 + c)`` in the
order params, data, structure, observables.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

ONE_QUBIT_FIXED = ("h", "x", "y", "z")
ONE_QUBIT_ROT = ("rx", "ry", "rz")
TWO_QUBIT_FIXED = ("cnot", "cz", "swap")
TWO_QUBIT_ROT = ("cp", "rzz")
# the other two-qubit rotations (exp(-i t X(x)X / 2), exp(-i t Y(x)Y / 2)); not in
# ALL_OPS, so that the seeded random circuits of the other tests stay as they are
TWO_QUBIT_ROT_XY = ("rxx", "ryy")
# the general one-qubit gate U3(theta, phi, lambda) (three consecutive angle
# entries idx, idx+1, idx+2) and the controlled rotations (control, target);
# likewise outside ALL_OPS
ONE_QUBIT_U3 = ("u3",)
CONTROLLED_ROT = ("crx", "cry", "crz")
ALL_OPS = ONE_QUBIT_FIXED + ONE_QUBIT_ROT + TWO_QUBIT_FIXED + TWO_QUBIT_ROT + ("unitary",)
KNOWN_OPS = ALL_OPS + TWO_QUBIT_ROT_XY + ONE_QUBIT_U3 + CONTROLLED_ROT
ROTATIONS = ONE_QUBIT_ROT + TWO_QUBIT_ROT + TWO_QUBIT_ROT_XY + ONE_QUBIT_U3 + CONTROLLED_ROT
ARITY = {**{o: 1 for o in ONE_QUBIT_FIXED + ONE_QUBIT_ROT + ONE_QUBIT_U3},
         **{o: 2 for o in TWO_QUBIT_FIXED + TWO_QUBIT_ROT + TWO_QUBIT_ROT_XY + CONTROLLED_ROT}}


def n_angles(op: str) -> int:
    """Angle entries a gate reads: U3 takes theta, phi, lambda."""
    return 3 if op == "u3" else 1


@dataclass(frozen=True)
class Gate:
    op: str
    wires: Tuple[int, ...]
    src: str = "none"          # 'none' | 'param' | 'data'
    idx: int = -1
    scale: float = 1.0
    matrix: Optional[np.ndarray] = field(default=None, compare=False, hash=False)

    @property
    def nq(self) -> int:
        return len(self.wires)


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    n_params: int = 0
    n_data: int = 0

    def __post_init__(self):
        for g in self.gates:
            assert g.op in KNOWN_OPS, g.op
            if g.op != "unitary":
                assert g.nq == ARITY[g.op], g
            assert len(set(g.wires)) == g.nq and all(0 <= w < self.n for w in g.wires), g
            if g.src == "param":
                assert 0 <= g.idx and g.idx + n_angles(g.op) <= self.n_params, g
            elif g.src == "data":
                assert 0 <= g.idx and g.idx + n_angles(g.op) <= self.n_data, g


Term = Tuple[float, str]
Observable = List[Term]


@dataclass
class Workload:
    """One batch of one circuit (configs 1, 2, 3, 5 and the test cases)."""
    name: str
    circuit: Circuit
    dtype: str                    # 'c64' | 'c128'
    batch: int
    params: np.ndarray            # [P] shared, or [B, P] per sample
    data: Optional[np.ndarray]    # [B, D] or None
    observables: List[Observable]
    grad: bool                    # forward + adjoint gradient wanted
    seed: int = 0

    @property
    def per_sample_params(self) -> bool:
        return self.params.ndim == 2


@dataclass
class MultiWorkload:
    """Config 4: many circuits of uneven size, one launch."""
    name: str
    items: List[Workload]
    seed: int = 0


# ---------------------------------------------------------------- builders
def hea_layers(n: int, layers: int, rot: Sequence[str], entangler: str,
               first_param: int = 0, pairs=None) -> Tuple[List[Gate], int]:
    """Hardware-efficient ansatz: per layer, each rotation kind in ``rot`` on
    every wire (kind-major, wire-minor), then the entangler.  Parameter
    index = layer*len(rot)*n + kind*n + wire (+ first_param)."""
    gates: List[Gate] = []
    p = first_param
    for layer in range(layers):
        for r in rot:
            for q in range(n):
                gates.append(Gate(r, (q,), "param", p))
                p += 1
        if entangler == "ring":
            gates += cnot_ring(n)
        elif entangler == "czladder":
            gates += [Gate("cz", (i, i + 1)) for i in range(n - 1)]
        elif entangler == "pairs":
            gates += [Gate("cnot", (c, t)) for (c, t) in pairs[layer]]
        elif entangler == "none":
            pass
        else:
            raise ValueError(entangler)
    return gates, p


def cnot_ring(n: int) -> List[Gate]:
    """CNOT(i, (i+1) mod n) for ascending i (the order that reproduces the
    printed numbers of the paper's first listing)."""
    if n < 2:
        return []
    return [Gate("cnot", (i, (i + 1) % n)) for i in range(n)]


def z_string(n: int, wires: Sequence[int], letters: str) -> str:
    s = ["I"] * n
    for w, l in zip(wires, letters):
        s[w] = l
    return "".join(s)


def sum_z(n: int) -> Observable:
    return [(1.0, z_string(n, [i], "Z")) for i in range(n)]


def sum_zz_open(n: int) -> Observable:
    return [(1.0, z_string(n, [i, i + 1], "ZZ")) for i in range(n - 1)]


def tfim_open(n: int, hx: float = 0.5) -> Observable:
    return sum_zz_open(n) + [(hx, z_string(n, [i], "X")) for i in range(n)]


def random_pauli_sum(rng, n: int, nterms: int) -> Observable:
    terms: Observable = []
    while len(terms) < nterms:
        letters = "".join("IXYZ"[k] for k in rng.integers(0, 4, size=n))
        if set(letters) == {"I"}:
            continue
        terms.append((float(rng.standard_normal()), letters))
    return terms


def random_unitary(rng, k: int) -> np.ndarray:
    d = 1 << k
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def random_pairs(rng, n: int) -> List[Tuple[int, int]]:
    perm = rng.permutation(n)
    return [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(n // 2)]


# ---------------------------------------------------------------- configs
def config(cid: int, **over) -> object:
    """The five benchmark configurations (seed 1000 + cid).  Keyword
    overrides (``n``, ``layers``, ``batch``) shrink a config within its own
    family for parity tests."""
    rng = np.random.default_rng(1000 + cid)
    two_pi = 2.0 * np.pi
    if cid == 1:
        n, L = over.get("n", 10), over.get("layers", 4)
        gates, P = hea_layers(n, L, ("ry", "rz"), "ring")
        params = rng.uniform(0.0, two_pi, size=P)
        return Workload("cfg1-hea-n%d-L%d-b1-c128" % (n, L), Circuit(n, gates, P), "c128", 1,
                        params, None, [[(1.0, z_string(n, [0], "Z"))]], True, 1001)
    if cid == 2:
        n, L, B = over.get("n", 16), over.get("layers", 8), over.get("batch", 256)
        enc = [Gate("rx", (q,), "data", q) for q in range(n)]
        gates, P = hea_layers(n, L, ("ry", "rz"), "ring")
        params = rng.uniform(0.0, two_pi, size=P)
        data = rng.uniform(0.0, np.pi, size=(B, n))
        return Workload("cfg2-enc-hea-n%d-L%d-b%d-c64" % (n, L, B), Circuit(n, enc + gates, P, n),
                        "c64", B, params, data, [sum_z(n)], over.get("grad", False), 1002)
    if cid == 3:
        n, L, B = over.get("n", 20), over.get("layers", 12), over.get("batch", 16)
        gates, P = hea_layers(n, L, ("rx", "ry", "rz"), "czladder")
        params = rng.uniform(0.0, two_pi, size=(B, P))
        return Workload("cfg3-hea3-cz-n%d-L%d-b%d-c64" % (n, L, B), Circuit(n, gates, P), "c64", B,
                        params, None, [tfim_open(n, 0.5)], True, 1003)
    if cid == 4:
        count = over.get("count", 64)
        nlo, nhi = over.get("nmin", 12), over.get("nmax", 22)
        llo, lhi = over.get("lmin", 4), over.get("lmax", 16)
        ns = rng.integers(nlo, nhi + 1, size=count)
        Ls = rng.integers(llo, lhi + 1, size=count)
        params = [rng.uniform(0.0, two_pi, size=2 * int(n) * int(L)) for n, L in zip(ns, Ls)]
        items = []
        for c in range(count):
            n, L = int(ns[c]), int(Ls[c])
            pairs = [random_pairs(rng, n) for _ in range(L)]
            gates, P = hea_layers(n, L, ("ry", "rz"), "pairs", pairs=pairs)
            items.append(Workload("cfg4-item%d-n%d-L%d" % (c, n, L), Circuit(n, gates, P), "c64", 1,
                                  params[c], None, [], True, 1004))
        for it in items:
            it.observables = [random_pauli_sum(rng, it.circuit.n, 8)]
        return MultiWorkload("cfg4-uneven-%d" % count, items, 1004)
    if cid == 5:
        n, L = over.get("n", 32), over.get("layers", 20)
        gates, P = hea_layers(n, L, ("ry", "rz"), "ring")
        params = rng.uniform(0.0, two_pi, size=P)
        return Workload("cfg5-hea-n%d-L%d-b1-c64" % (n, L), Circuit(n, gates, P), "c64", 1,
                        params, None, [sum_zz_open(n)], True, 1005)
    raise ValueError(cid)


# ---------------------------------------------------------------- test circuits
def random_circuit(rng, n: int, ngates: int, ops: Sequence[str] = ALL_OPS,
                   with_data: bool = False, max_unitary_k: int = 3) -> Circuit:
    """Random gate list over ``ops`` at random wires; rotations take a fresh
    parameter (or, when ``with_data``, sometimes a data column)."""
    gates: List[Gate] = []
    P = D = 0
    for _ in range(ngates):
        op = ops[int(rng.integers(0, len(ops)))]
        if op == "unitary":
            k = int(rng.integers(1, min(max_unitary_k, n) + 1))
            wires = tuple(int(w) for w in rng.choice(n, size=k, replace=False))
            gates.append(Gate("unitary", wires, matrix=random_unitary(rng, k)))
            continue
        a = ARITY[op]
        if a > n:
            continue
        wires = tuple(int(w) for w in rng.choice(n, size=a, replace=False))
        if op in ROTATIONS:
            k = n_angles(op)
            if with_data and rng.random() < 0.3:
                gates.append(Gate(op, wires, "data", D, float(rng.choice([1.0, -0.5, 2.0]))))
                D += k
            else:
                gates.append(Gate(op, wires, "param", P))
                P += k
        else:
            gates.append(Gate(op, wires))
    return Circuit(n, gates, P, D)


def random_params(rng, circuit: Circuit, batch: int = 1, per_sample: bool = False):
    if per_sample:
        params = rng.uniform(0.0, 2 * np.pi, size=(batch, circuit.n_params))
    else:
        params = rng.uniform(0.0, 2 * np.pi, size=circuit.n_params)
    data = rng.uniform(0.0, np.pi, size=(batch, circuit.n_data)) if circuit.n_data else None
    return params, data


# ---------------------------------------------------------------- paper circuits
def listing1(theta: Sequence[float], data: Sequence[float] = (1.0, 2.0, 3.0)):
    """The three-qubit example of the paper's API overview (listing
    "code:qubitcircuit"): H(0); CNOT(0,1); X on wire 2 controlled by wire 0;
    RY(data[q]) on wire q; CNOT ring; RY(theta[q]) on wire q; observable
    X0 Z1 X2."""
    g = [Gate("h", (0,)), Gate("cnot", (0, 1)), Gate("cnot", (0, 2))]
    g += [Gate("ry", (q,), "data", q) for q in range(3)]
    g += cnot_ring(3)
    g += [Gate("ry", (q,), "param", q) for q in range(3)]
    c = Circuit(3, g, 3, 3)
    return c, np.asarray(theta, float), np.asarray([data], float), [[(1.0, "XZX")]]


def dist_listing():
    """The four-qubit example of the distributed-simulation section (listing
    "code:dist"): RY(data[q]) on wire q, CNOT ring, observables Z0 and X1,
    data = arange(4); gradient taken with respect to the data."""
    g = [Gate("ry", (q,), "data", q) for q in range(4)] + cnot_ring(4)
    c = Circuit(4, g, 0, 4)
    return c, np.zeros(0), np.arange(4, dtype=float)[None, :], [[(1.0, "ZIII")], [(1.0, "IXII")]]


def qresnet(residual: bool = True):
    """The curve-fitting model of the QResNet listing ("code:qresnet",
    section 4.3).  Residual form on two wires: RY(theta) on wire 0, U3 on
    wire 1, the data encoded as an RY on wire 1 controlled by wire 0, RY on
    wire 0, U3 on wire 1; observables Z1 and Z0 Z1.  Plain form on one wire:
    U3, RY(data), U3; observable Z0.  Parameters in gate order (U3 takes
    three); one data column.  Returns (circuit, observables)."""
    if residual:
        g = [Gate("ry", (0,), "param", 0), Gate("u3", (1,), "param", 1), Gate("cry", (0, 1), "data", 0),
             Gate("ry", (0,), "param", 4), Gate("u3", (1,), "param", 5)]
        return Circuit(2, g, 8, 1), [[(1.0, "IZ")], [(1.0, "ZZ")]]
    g = [Gate("u3", (0,), "param", 0), Gate("ry", (0,), "data", 0), Gate("u3", (0,), "param", 3)]
    return Circuit(1, g, 6, 1), [[(1.0, "Z")]]


def qcnn(n: int = 12):
    """The QCNN of its listing ("code:qcnn_demo", section 4.3) on n = 12
    wires: data encoded by RY on all 12 wires, a convolution (RXX then RYY
    on pairs (i, i+1), i even), pooling (CRY with control 2i+1 and target
    2i); RY encoding on wires 0..5, convolution and pooling on 6 wires; RY
    encoding on wires 0..2, RXX and RYY on (0,1) and (1,2), then CRY(1, 0)
    and CRY(2, 0).  21 data columns (12 + 6 + 3), parameters in gate order;
    observable Z on wire 0.  Returns (circuit, observables)."""
    assert n == 12, "the listing's layer sizes are those of 12 wires"
    g: List[Gate] = []
    P = D = 0

    def enc(wires):
        nonlocal D
        for q in wires:
            g.append(Gate("ry", (q,), "data", D))
            D += 1

    def rot(op, wires):
        nonlocal P
        g.append(Gate(op, wires, "param", P))
        P += 1

    def conv(m):
        for i in range(0, m - 1, 2):
            rot("rxx", (i, i + 1))
            rot("ryy", (i, i + 1))

    def pool(m):
        for i in range(m // 2):
            rot("cry", (2 * i + 1, 2 * i))

    enc(range(12))
    conv(12)
    pool(12)
    enc(range(6))
    conv(6)
    pool(6)
    enc(range(3))
    for i in range(2):
        rot("rxx", (i, i + 1))
        rot("ryy", (i, i + 1))
    rot("cry", (1, 0))
    rot("cry", (2, 0))
    return Circuit(n, g, P, D), [[(1.0, z_string(n, [0], "Z"))]]


def qft(n: int, reverse: bool = False) -> Circuit:
    """QFT of the distributed-QFT listing ("code:dist_qft"): per wire i a
    Hadamard then controlled phases pi/2^(k-1) from wires i+1.., then the
    wire-reversing swaps."""
    g: List[Gate] = []
    for i in range(n):
        g.append(Gate("h", (i,)))
        k = 2
        for j in range(i, n - 1):
            g.append(Gate("cp", (j + 1, i), "none", -1, float(np.pi / 2 ** (k - 1))))
            k += 1
    if not reverse:
        for i in range(n // 2):
            g.append(Gate("swap", (i, n - 1 - i)))
    return Circuit(n, g)


def trotter_step(n: int, J: float, h: float, dt: float, periodic: bool = True) -> Circuit:
    """One second-order Trotter step of the TFIM listing ("code:mps_tfim"):
    rx(-h dt) on every wire, rzz(-2 J dt) on even then odd bonds (then the
    periodic bond), rx(-h dt) again."""
    g: List[Gate] = [Gate("rx", (i,), "none", -1, -h * dt) for i in range(n)]
    g += [Gate("rzz", (i, i + 1), "none", -1, -2 * J * dt) for i in range(0, n - 1, 2)]
    g += [Gate("rzz", (i, i + 1), "none", -1, -2 * J * dt) for i in range(1, n - 1, 2)]
    if periodic:
        g.append(Gate("rzz", (n - 1, 0), "none", -1, -2 * J * dt))
    g += [Gate("rx", (i,), "none", -1, -h * dt) for i in range(n)]
    return Circuit(n, g)
