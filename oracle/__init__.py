"""The oracle -- TEST INFRASTRUCTURE, not part of the product.

A plain, slow, complex128 CPU simulator of what the HIP path computes,
written from the paper's definitions and pinned by the ``-m "not gpu"``
tests against values the paper prints, closed forms, library routines
(``numpy.fft``, ``scipy.linalg.expm``) and brute force.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the product package never does.

* ``dq_oracle.c``: gate matrices, the textbook gather/multiply/scatter loop,
  Pauli-string expectations (letters applied as ordinary gates), marginal
  probabilities.  Pure-state evolution is the equation of paper section 4.1;
  expectations and measurement follow the API overview of section 4.2.
* this module: per-gate angles (``scale * source``; U3 reads three
  consecutive entries as theta, phi, lambda), batching over samples, and the
  two reference gradients -- the parameter-shift rule and central finite
  differences.  The two-term shift rule is exact for gates exp(-i t G/2)
  whose generator G has eigenvalues +-1, for the controlled phase (generator
  eigenvalues 0 and 1) and for each angle of U3 (each enters as such a
  rotation, up to a global phase); the controlled rotations, whose
  generator |1><1| (x) P has eigenvalues 0 and +-1, take the four-term rule
  dE/dt = d+ [E(t + pi/2) - E(t - pi/2)] - d- [E(t + 3 pi/2) - E(t - 3 pi/2)],
  d+- = (sqrt 2 +- 1) / (4 sqrt 2), exact for the two frequencies 1/2 and 1
  that such a gate gives E.  The adjoint method that the paper names for its
  distributed simulator (section 7.2) is *not* re-implemented here: the
  oracle's gradients come from the definition of the derivative.
* ``kron.py``: an independent numpy brute-force checker (tensor
  contraction / Kronecker products) for up to six qubits.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dq_oracle.c")
_SO = os.path.join(_HERE, "_dq_oracle.so")

OPCODE = {"h": 0, "x": 1, "y": 2, "z": 3, "rx": 4, "ry": 5, "rz": 6, "cnot": 7, "cz": 8,
          "swap": 9, "cp": 10, "rzz": 11, "unitary": 12, "rxx": 13, "ryy": 14,
          "u3": 15, "crx": 16, "cry": 17, "crz": 18}
# gates whose derivative the two-term shift rule gives exactly
SHIFT_RULE_GATES = ("rx", "ry", "rz", "rzz", "cp", "rxx", "ryy", "u3")
# gates that need the four-term rule (generator eigenvalues 0, +-1)
FOUR_TERM_GATES = ("crx", "cry", "crz")
_D_PLUS = (np.sqrt(2.0) + 1.0) / (4.0 * np.sqrt(2.0))
_D_MINUS = (np.sqrt(2.0) - 1.0) / (4.0 * np.sqrt(2.0))


def n_angles(op: str) -> int:
    return 3 if op == "u3" else 1


_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)          # when missing or older than its source
            L = ctypes.CDLL(_SO)
            dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
            L.orc_gate_matrix.argtypes = [ctypes.c_int, ctypes.c_double, dp]
            L.orc_gate_matrix.restype = ctypes.c_int
            L.orc_u3_matrix.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
            L.orc_u3_matrix.restype = None
            L.orc_apply.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, dp]
            L.orc_apply.restype = None
            L.orc_run.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, dp, dp]
            L.orc_run.restype = ctypes.c_int
            L.orc_pauli_expval.argtypes = [ctypes.c_int, dp, ctypes.c_char_p, dp]
            L.orc_pauli_expval.restype = ctypes.c_double
            L.orc_prob_zero.argtypes = [ctypes.c_int, dp, ctypes.c_int]
            L.orc_prob_zero.restype = ctypes.c_double
            _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# ------------------------------------------------------------ circuit encoding
class _Encoded:
    """The gate list as flat int/double arrays for the C loop."""

    def __init__(self, circuit):
        G = len(circuit.gates)
        self.n = circuit.n
        self.ops = np.array([OPCODE[g.op] for g in circuit.gates], dtype=np.intc)
        self.nq = np.array([g.nq for g in circuit.gates], dtype=np.intc)
        self.wires = np.zeros(5 * max(G, 1), dtype=np.intc)
        for i, g in enumerate(circuit.gates):
            self.wires[5 * i:5 * i + g.nq] = g.wires
        dense = [np.ascontiguousarray(g.matrix, dtype=np.complex128).ravel()
                 for g in circuit.gates if g.op == "unitary"]
        self.dense = (np.concatenate(dense) if dense else np.zeros(1, np.complex128)).view(np.float64)
        self.gates = circuit.gates

    def angles(self, params, data, b: int) -> np.ndarray:
        """[G, 3]: theta_g,k = scale * (params[idx + k] | data[idx + k] | 1)
        for the gate's k-th angle (k < 3 for U3, k = 0 otherwise)."""
        th = np.zeros((max(len(self.gates), 1), 3))
        for i, g in enumerate(self.gates):
            for k in range(n_angles(g.op)):
                if g.src == "param":
                    p = np.asarray(params, float)
                    th[i, k] = g.scale * (p[b, g.idx + k] if p.ndim == 2 else p[g.idx + k])
                elif g.src == "data":
                    th[i, k] = g.scale * float(np.asarray(data, float)[b, g.idx + k])
                else:
                    th[i, k] = g.scale
        return th


def _run_angles(enc: _Encoded, theta: np.ndarray, psi0: Optional[np.ndarray] = None) -> np.ndarray:
    psi = np.zeros(1 << enc.n, dtype=np.complex128)
    if psi0 is None:
        psi[0] = 1.0
    else:
        psi[:] = psi0
    pv = psi.view(np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    rc = lib().orc_run(enc.n, _dp(pv), len(enc.gates), _ip(enc.ops), _ip(enc.nq), _ip(enc.wires),
                       _dp(theta), _dp(enc.dense))
    if rc != 0:
        raise ValueError("oracle: unknown gate")
    return psi


# ------------------------------------------------------------ public API
def u3_matrix(theta: float, phi: float, lam: float) -> np.ndarray:
    buf = np.zeros(8)
    lib().orc_u3_matrix(float(theta), float(phi), float(lam), _dp(buf))
    return buf.view(np.complex128).reshape(2, 2).copy()


def gate_matrix(op: str, theta: float = 0.0) -> np.ndarray:
    buf = np.zeros(32)
    k = lib().orc_gate_matrix(OPCODE[op], float(theta), _dp(buf))
    if k < 0:
        raise ValueError(op)
    d = 1 << k
    return buf[:2 * d * d].view(np.complex128).reshape(d, d).copy()


def apply_matrix(n: int, psi: np.ndarray, wires: Sequence[int], U: np.ndarray) -> np.ndarray:
    """Apply a dense matrix to ``wires`` of a copy of ``psi``."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    Ui = np.ascontiguousarray(U, dtype=np.complex128)
    w = np.array(wires, dtype=np.intc)
    lib().orc_apply(n, _dp(out.view(np.float64)), len(wires), _ip(w), _dp(Ui.view(np.float64)))
    return out


def state(circuit, params=None, data=None, b: int = 0, psi0=None) -> np.ndarray:
    """Final state of sample ``b`` (complex128, length 2^n)."""
    enc = _Encoded(circuit)
    return _run_angles(enc, enc.angles(params, data, b), psi0)


def pauli_expval(n: int, psi: np.ndarray, letters: str, check_imag: float = 1e-10) -> float:
    im = ctypes.c_double(0.0)
    pv = np.ascontiguousarray(psi, dtype=np.complex128).view(np.float64)
    re = lib().orc_pauli_expval(n, _dp(pv), letters.encode("ascii"), ctypes.byref(im))
    if not np.isfinite(re) or abs(im.value) > check_imag * max(1.0, np.vdot(psi, psi).real):
        raise ValueError("oracle: <P> not real (%r, %r)" % (re, im.value))
    return re


def expvals(n: int, psi: np.ndarray, observables) -> np.ndarray:
    """E[o] = sum_k c_k <psi|P_k|psi> for each observable o."""
    out = np.zeros(len(observables))
    for o, obs in enumerate(observables):
        out[o] = sum(c * pauli_expval(n, psi, letters) for c, letters in obs)
    return out


def prob_zero(n: int, psi: np.ndarray, wire: int) -> float:
    pv = np.ascontiguousarray(psi, dtype=np.complex128).view(np.float64)
    return lib().orc_prob_zero(n, _dp(pv), wire)


def probs(n: int, psi: np.ndarray, wires: Sequence[int]) -> np.ndarray:
    """Marginal probabilities of a computational-basis measurement of
    ``wires`` (measurement of section 4.2; the Born rule behind the state
    evolution of section 4.1): P[m] = sum of |psi_j|^2 over the basis states
    j whose measured wires read m, wires[0] being the most significant bit
    of m and wire w being bit n-1-w of j."""
    j = np.arange(1 << n, dtype=np.int64)
    m = np.zeros(1 << n, dtype=np.int64)
    for w in wires:
        m = (m << 1) | ((j >> (n - 1 - w)) & 1)
    out = np.zeros(1 << len(wires))
    np.add.at(out, m, np.abs(np.asarray(psi, dtype=np.complex128)) ** 2)
    return out


def sample(p: Sequence[float], u: Sequence[float]) -> np.ndarray:
    """Shots by inverse transform (sampling of section 4.2's measurement):
    for each uniform x the smallest outcome m with x < p[0] + ... + p[m]
    (summed in this order), else the last outcome of nonzero probability
    (x not below the total), else 0 (no probability at all)."""
    out = []
    for x in u:
        c, last, res = 0.0, -1, -1
        for m, pm in enumerate(p):
            if pm > 0:
                last = m
            c += pm
            if x < c:
                res = m
                break
        out.append(res if res >= 0 else (last if last >= 0 else 0))
    return np.array(out, dtype=np.int64)


def _pool(threads: Optional[int]):
    return ThreadPoolExecutor(max_workers=threads or 1)


def forward(circuit, params, data, observables, batch: int, threads: Optional[int] = None,
            samples: Optional[Sequence[int]] = None) -> np.ndarray:
    """Expectations E[b, o] for the listed samples (default: all)."""
    enc = _Encoded(circuit)
    samples = list(range(batch)) if samples is None else list(samples)

    def one(b):
        return expvals(circuit.n, _run_angles(enc, enc.angles(params, data, b)), observables)

    with _pool(threads) as ex:
        rows = list(ex.map(one, samples))
    return np.array(rows).reshape(len(samples), len(observables))


def _source_gates(circuit):
    return [i for i, g in enumerate(circuit.gates) if g.src in ("param", "data")]


def grad_param_shift(circuit, params, data, observables, weights, batch: int,
                     threads: Optional[int] = None, samples: Optional[Sequence[int]] = None,
                     gate_subset: Optional[Sequence[int]] = None):
    """Vector-Jacobian product of L = sum_{b,o} w[b,o] E[b,o] by the
    parameter-shift rule, applied to every angle of every gate occurrence
    that reads a parameter or a data entry:
        dE/dtheta = (E(theta + pi/2) - E(theta - pi/2)) / 2           (two-term)
        dE/dtheta = d+ [E(theta + pi/2) - E(theta - pi/2)]
                  - d- [E(theta + 3 pi/2) - E(theta - 3 pi/2)]         (controlled rotations)
    chained through theta = scale * source.
    Returns (grad_params shaped like params, grad_data shaped like data)."""
    enc = _Encoded(circuit)
    w = np.asarray(weights, float).reshape(batch, len(observables))
    p = np.asarray(params, float) if params is not None else np.zeros(0)
    gp = np.zeros_like(p)
    gd = None if data is None else np.zeros_like(np.asarray(data, float))
    samples = list(range(batch)) if samples is None else list(samples)
    gates = _source_gates(circuit) if gate_subset is None else list(gate_subset)
    for i in gates:
        if circuit.gates[i].op not in SHIFT_RULE_GATES + FOUR_TERM_GATES:
            raise ValueError("no shift rule for %s" % circuit.gates[i].op)

    jobs = [(b, i, k) for b in samples for i in gates for k in range(n_angles(circuit.gates[i].op))]

    def L_at(b, th):
        return float(np.dot(w[b], expvals(circuit.n, _run_angles(enc, th), observables)))

    def shifted(b, th, i, k, s):
        t2 = th.copy()
        t2[i, k] += s
        return L_at(b, t2)

    def one(job):
        b, i, k = job
        th = enc.angles(params, data, b)
        if circuit.gates[i].op in FOUR_TERM_GATES:
            a = shifted(b, th, i, k, np.pi / 2) - shifted(b, th, i, k, -np.pi / 2)
            c = shifted(b, th, i, k, 3 * np.pi / 2) - shifted(b, th, i, k, -3 * np.pi / 2)
            return _D_PLUS * a - _D_MINUS * c
        return (shifted(b, th, i, k, np.pi / 2) - shifted(b, th, i, k, -np.pi / 2)) / 2.0

    with _pool(threads) as ex:
        vals = list(ex.map(one, jobs))
    for (b, i, k), v in zip(jobs, vals):
        g = circuit.gates[i]
        if g.src == "param":
            if gp.ndim == 2:
                gp[b, g.idx + k] += g.scale * v
            else:
                gp[g.idx + k] += g.scale * v
        else:
            gd[b, g.idx + k] += g.scale * v
    return gp, gd


def _shift_rule(op: str):
    """(coefficients, shifts) of a gate angle's derivative rule,
    dE/dt = sum_i c_i E(t + s_i): two-term for generators with two
    eigenvalues a distance 1 apart, four-term for the controlled rotations."""
    if op in FOUR_TERM_GATES:
        return ((_D_PLUS, -_D_PLUS, -_D_MINUS, _D_MINUS),
                (np.pi / 2, -np.pi / 2, 3 * np.pi / 2, -3 * np.pi / 2))
    if op in SHIFT_RULE_GATES:
        return ((0.5, -0.5), (np.pi / 2, -np.pi / 2))
    raise ValueError("no shift rule for %s" % op)


def hessian_param_shift(circuit, params, data, observables, weights, threads: Optional[int] = None):
    """Hessian d^2 L / dtheta_p dtheta_q of L = sum_o w[o] E_o for one
    sample with shared parameters params[P] (data: one row or None) -- the
    second-order benchmark of paper section 3.1.  Each gate-angle occurrence
    a (gate i, angle k, reading params[idx + k] with chain factor scale) has
    the derivative rule D_a of its gate; D_a D_b L is that rule applied
    along angle a to the function that the rule along b gives,
        D_a D_b L = sum_i sum_j c_i c_j L(angles + s_i e_a + s_j e_b),
    (for a = b both shifts land on the same angle).  This is exact: E, and
    its derivative along b, are trigonometric polynomials in angle a with
    the frequencies of a's generator, for which D_a is exact.  Chained
    through theta = scale * source:
        H[p, q] = sum_{a reads p} sum_{b reads q} scale_a scale_b D_a D_b L.
    Returns H [P, P] (float64)."""
    enc = _Encoded(circuit)
    w = np.asarray(weights, float).reshape(len(observables))
    p = np.asarray(params, float).reshape(-1)
    dat = None if data is None else np.asarray(data, float).reshape(1, -1)
    occ = [(i, k) for i, g in enumerate(circuit.gates) if g.src == "param" for k in range(n_angles(g.op))]
    th0 = enc.angles(p, dat, 0)

    def L_at(th):
        return float(np.dot(w, expvals(circuit.n, _run_angles(enc, th), observables)))

    def one(pair):
        a, b = pair
        (ia, ka), (ib, kb) = occ[a], occ[b]
        ca, sa = _shift_rule(circuit.gates[ia].op)
        cb, sb = _shift_rule(circuit.gates[ib].op)
        v = 0.0
        for ci, si in zip(ca, sa):
            for cj, sj in zip(cb, sb):
                th = th0.copy()
                th[ia, ka] += si
                th[ib, kb] += sj
                v += ci * cj * L_at(th)
        return v

    pairs = [(a, b) for a in range(len(occ)) for b in range(a, len(occ))]
    with _pool(threads) as ex:
        vals = list(ex.map(one, pairs))
    H = np.zeros((len(p), len(p)))
    for (a, b), v in zip(pairs, vals):
        ga, gb = circuit.gates[occ[a][0]], circuit.gates[occ[b][0]]
        pa, pb = ga.idx + occ[a][1], gb.idx + occ[b][1]
        f = ga.scale * gb.scale * v
        H[pa, pb] += f
        if a != b:               # D_a D_b = D_b D_a: the mirrored pair
            H[pb, pa] += f
    return H


def grad_fd(circuit, params, data, observables, weights, batch: int, h: float = 1e-6,
            threads: Optional[int] = None, samples: Optional[Sequence[int]] = None,
            param_subset: Optional[Sequence[int]] = None, with_data: bool = True):
    """Central finite differences (L(x+h) - L(x-h)) / 2h of the same VJP, on
    each parameter (and each data entry)."""
    w = np.asarray(weights, float).reshape(batch, len(observables))
    p = np.asarray(params, float) if params is not None else np.zeros(0)
    samples = list(range(batch)) if samples is None else list(samples)
    gp = np.zeros_like(p)
    dat = None if data is None else np.asarray(data, float)
    gd = None if dat is None else np.zeros_like(dat)
    P = circuit.n_params
    pidx = list(range(P)) if param_subset is None else list(param_subset)

    def L(pp, dd, bs):
        E = forward(circuit, pp, dd, observables, batch, threads=threads, samples=bs)
        return float(sum(np.dot(w[b], E[k]) for k, b in enumerate(bs)))

    if p.ndim == 2:
        for b in samples:
            for j in pidx:
                pp, pm = p.copy(), p.copy()
                pp[b, j] += h
                pm[b, j] -= h
                gp[b, j] = (L(pp, dat, [b]) - L(pm, dat, [b])) / (2 * h)
    else:
        for j in pidx:
            pp, pm = p.copy(), p.copy()
            pp[j] += h
            pm[j] -= h
            gp[j] = (L(pp, dat, samples) - L(pm, dat, samples)) / (2 * h)
    if dat is not None and with_data:
        for b in samples:
            for j in range(dat.shape[1]):
                dp_, dm_ = dat.copy(), dat.copy()
                dp_[b, j] += h
                dm_[b, j] -= h
                gd[b, j] = (L(p, dp_, [b]) - L(p, dm_, [b])) / (2 * h)
    return gp, gd
