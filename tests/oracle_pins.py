"""Pins of the oracle to things other than itself.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with
a value the paper prints, a closed form, a library routine or brute force.
``test_oracle_pins.py`` runs them against the oracle; ``test_oracle_mutants``
re-runs them against copies of the oracle with planted mistakes and checks
that every mistake is caught by at least one pin.
"""
import json
import os

import numpy as np
from scipy.linalg import expm

import oracle
import workloads as W
from oracle import kron

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _close(a, b, tol, what):
    a, b = np.asarray(a), np.asarray(b)
    err = float(np.max(np.abs(a - b))) if a.size else 0.0
    assert err <= tol, "%s: max|diff| = %.3e > %.1e" % (what, err, tol)


def _rand_state(rng, n):
    x = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return x / np.linalg.norm(x)


def pin_listing1_printed_values():
    """Paper 4.2, listing code:qubitcircuit: <X0Z1X2>, three gradients and
    P(wire 0 = 0) as printed (4 decimals)."""
    g = json.load(open(os.path.join(GOLDEN, "listing1.json")))
    c, th, data, obs = W.listing1(g["theta"], g["data"])
    psi = oracle.state(c, th, data)
    _close(oracle.expvals(3, psi, obs)[0], g["expval"], g["tol"], "listing1 <X0Z1X2>")
    gp, _ = oracle.grad_param_shift(c, th, data, obs, np.ones((1, 1)), 1)
    _close(gp, g["grad"], g["tol"], "listing1 gradients")
    _close(oracle.prob_zero(3, psi, 0), g["p0_wire0"], g["tol"], "listing1 P(q0=0)")


def pin_bloch_state():
    """Paper 4.1: cos(t/2)|0> + e^{i phi} sin(t/2)|1> is reached by RZ(phi) RY(t)
    from |0>, up to a global phase; RY(t)|0> has no phase at all."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        t, ph = rng.uniform(0, 2 * np.pi, 2)
        c = W.Circuit(1, [W.Gate("ry", (0,), "param", 0), W.Gate("rz", (0,), "param", 1)], 2)
        psi = oracle.state(c, [t, ph])
        want = np.array([np.cos(t / 2), np.exp(1j * ph) * np.sin(t / 2)])
        _close(abs(np.vdot(want, psi)), 1.0, 1e-12, "Bloch state fidelity")
        _close(psi * np.exp(1j * ph / 2), want, 1e-12, "Bloch state with RZ phase")
        c1 = W.Circuit(1, [W.Gate("ry", (0,), "param", 0)], 1)
        _close(oracle.state(c1, [t]), [np.cos(t / 2), np.sin(t / 2)], 1e-14, "RY|0>")


def pin_ghz():
    """GHZ / Bell states (paper 5.x EPR/GHZ definitions): H(0) then a CNOT
    chain gives (|0..0> + |1..1>)/sqrt 2, and Listing 1's prefix H(0) CNOT(0,1)
    gives a Bell pair on wires 0,1."""
    for n in range(2, 8):
        g = [W.Gate("h", (0,))] + [W.Gate("cnot", (i, i + 1)) for i in range(n - 1)]
        psi = oracle.state(W.Circuit(n, g))
        want = np.zeros(1 << n, complex)
        want[0] = want[-1] = 1 / np.sqrt(2)
        _close(psi, want, 1e-15, "GHZ n=%d" % n)
    # a CNOT whose control is a *lower* wire than the target flips the later bit
    psi = oracle.state(W.Circuit(2, [W.Gate("x", (0,)), W.Gate("cnot", (0, 1))]))
    _close(psi, [0, 0, 0, 1], 0, "X0 then CNOT(0,1) = |11>")
    psi = oracle.state(W.Circuit(2, [W.Gate("x", (1,)), W.Gate("cnot", (0, 1))]))
    _close(psi, [0, 1, 0, 0], 0, "X1 then CNOT(0,1) = |01> (control 0 not set)")


def pin_cnot_from_cz():
    """Paper eq. in 5.x (dual-rail CNOT): CNOT = (I (x) H) CZ (I (x) H)."""
    rng = np.random.default_rng(2)
    n = 4
    for c, t in [(0, 1), (1, 0), (0, 3), (3, 1), (2, 0)]:
        x = _rand_state(rng, n)
        a = oracle.state(W.Circuit(n, [W.Gate("cnot", (c, t))]), psi0=x)
        b = oracle.state(W.Circuit(n, [W.Gate("h", (t,)), W.Gate("cz", (c, t)), W.Gate("h", (t,))]), psi0=x)
        _close(a, b, 1e-14, "CNOT vs H CZ H on (%d,%d)" % (c, t))


def pin_rotation_generators():
    """RX/RY/RZ(t) = expm(-i t P/2), RZZ(t) = expm(-i t ZZ/2) (scipy), CP from
    projectors, H = (X+Z)/sqrt 2, SWAP = (I+XX+YY+ZZ)/2."""
    for t in (0.0, 0.37, -1.9, 3.1, 5.5):
        for op in ("rx", "ry", "rz", "rzz", "cp"):
            _close(oracle.gate_matrix(op, t), kron.named(op, t), 1e-14, "%s(%g)" % (op, t))
    for op in ("h", "x", "y", "z", "cnot", "cz", "swap"):
        _close(oracle.gate_matrix(op), kron.named(op), 1e-15, op)


def pin_kron_bruteforce():
    """Random circuits over every gate kind on every wire position at n<=6
    equal the product of full Kronecker-embedded matrices."""
    rng = np.random.default_rng(3)
    for n in range(1, 7):
        for trial in range(4):
            ops = W.ALL_OPS if n >= 2 else ("h", "x", "y", "z", "rx", "ry", "rz", "unitary")
            c = W.random_circuit(rng, n, 25, ops=ops, with_data=True, max_unitary_k=min(3, n))
            params, data = W.random_params(rng, c, 1)
            _close(oracle.state(c, params, data), kron.state(c, params, data), 1e-12,
                   "kron n=%d trial %d" % (n, trial))
    # every ordered wire pair / triple of a dense unitary at n=4
    n = 4
    for k in (1, 2, 3):
        for wires in kron.all_wire_tuples(n, k):
            U = W.random_unitary(rng, k)
            x = _rand_state(rng, n)
            _close(oracle.apply_matrix(n, x, wires, U), kron.embed(U, list(wires), n) @ x, 1e-13,
                   "dense %s" % (wires,))
    # adjacent ascending wires through literal np.kron
    U = W.random_unitary(rng, 2)
    x = _rand_state(rng, 5)
    _close(oracle.apply_matrix(5, x, (1, 2), U), kron.embed_adjacent(U, 1, 5) @ x, 1e-13, "kron adjacent")


def pin_qft_is_dft():
    """Paper 7.3, listing code:dist_qft: the QFT circuit equals the unitary DFT
    (numpy.fft.ifft, orthonormal) -- true only with wire 0 as the most
    significant bit."""
    rng = np.random.default_rng(4)
    for n in range(1, 8):
        x = _rand_state(rng, n)
        _close(oracle.state(W.qft(n), psi0=x), np.fft.ifft(x, norm="ortho"), 1e-13, "QFT n=%d" % n)


def pin_norm_preserved():
    """Unitarity (paper 4.1): the norm stays 1 through every gate."""
    rng = np.random.default_rng(5)
    for n in (3, 7, 11):
        c = W.random_circuit(rng, n, 60, with_data=True, max_unitary_k=3)
        params, data = W.random_params(rng, c, 1)
        _close(np.linalg.norm(oracle.state(c, params, data)), 1.0, 1e-13, "norm n=%d" % n)


def pin_shift_equals_fd():
    """Parameter shift (exact) equals central finite differences (h=1e-6)."""
    rng = np.random.default_rng(6)
    for n in (2, 4, 5):
        c = W.random_circuit(rng, n, 30, ops=("h", "rx", "ry", "rz", "cnot", "cz", "rzz", "cp", "swap"),
                             with_data=True)
        params, data = W.random_params(rng, c, 2)
        obs = [W.random_pauli_sum(rng, n, 3), W.random_pauli_sum(rng, n, 2)]
        w = rng.standard_normal((2, 2))
        a = oracle.grad_param_shift(c, params, data, obs, w, 2)
        b = oracle.grad_fd(c, params, data, obs, w, 2)
        _close(a[0], b[0], 2e-8, "shift vs FD params n=%d" % n)
        _close(a[1], b[1], 2e-8, "shift vs FD data n=%d" % n)


def pin_special_cases():
    """Closed forms: zero angles make the ansatz the identity on |0..0>;
    RY(a)RZ(b) gives <Z>=cos a, <X>=sin a cos b; RX(x)|0> gives <Z>=cos x,
    <Y>=-sin x and d<Z>/dx = -sin x."""
    n = 6
    gates, P = W.hea_layers(n, 3, ("ry", "rz"), "ring")
    c = W.Circuit(n, gates, P)
    psi = oracle.state(c, np.zeros(P))
    _close(oracle.expvals(n, psi, [[(1.0, W.z_string(n, [i], "Z"))] for i in range(n)]), np.ones(n), 1e-14, "Z_i")
    _close(oracle.expvals(n, psi, [W.sum_zz_open(n)])[0], n - 1, 1e-14, "sum ZZ")
    _close(oracle.expvals(n, psi, [W.tfim_open(n, 0.5)])[0], n - 1, 1e-14, "TFIM at 0")
    g, _ = oracle.grad_param_shift(c, np.zeros(P), None, [W.tfim_open(n, 0.5)], np.ones((1, 1)), 1)
    ry = [i for i, gg in enumerate(gates) if gg.op == "ry"]
    _close(g[[gates[i].idx for i in ry]], 0.0, 1e-14, "RY gradients at 0")
    for a, b in [(0.3, 1.1), (2.5, -0.7), (4.0, 3.0)]:
        c2 = W.Circuit(1, [W.Gate("ry", (0,), "param", 0), W.Gate("rz", (0,), "param", 1)], 2)
        psi = oracle.state(c2, [a, b])
        _close(oracle.pauli_expval(1, psi, "Z"), np.cos(a), 1e-14, "<Z> = cos a")
        _close(oracle.pauli_expval(1, psi, "X"), np.sin(a) * np.cos(b), 1e-14, "<X> = sin a cos b")
        _close(oracle.pauli_expval(1, psi, "Y"), np.sin(a) * np.sin(b), 1e-14, "<Y> = sin a sin b")
        c3 = W.Circuit(1, [W.Gate("rx", (0,), "data", 0)], 0, 1)
        psi = oracle.state(c3, None, np.array([[a]]))
        _close(oracle.pauli_expval(1, psi, "Z"), np.cos(a), 1e-14, "RX: <Z>")
        _close(oracle.pauli_expval(1, psi, "Y"), -np.sin(a), 1e-14, "RX: <Y>")
        _, gd = oracle.grad_param_shift(c3, np.zeros(0), np.array([[a]]), [[(1.0, "Z")]], np.ones((1, 1)), 1)
        _close(gd[0, 0], -np.sin(a), 1e-13, "RX: d<Z>/dx")


def pin_trotter_vs_expm():
    """Paper 7.3 TFIM: one second-order Trotter step (listing code:mps_tfim)
    approximates expm(-i H dt) with error O(dt^3), H = -J sum ZZ - h sum X
    (periodic)."""
    n, J, h = 6, -1.0, -1.2
    H = np.zeros((1 << n, 1 << n), complex)
    for i in range(n):
        j = (i + 1) % n
        H += -J * kron.pauli_full(W.z_string(n, sorted([i, j]), "ZZ"))
        H += -h * kron.pauli_full(W.z_string(n, [i], "X"))
    rng = np.random.default_rng(7)
    x = _rand_state(rng, n)
    errs = []
    for dt in (0.1, 0.05, 0.025):
        a = oracle.state(W.trotter_step(n, J, h, dt), psi0=x)
        b = expm(-1j * H * dt) @ x
        errs.append(np.linalg.norm(a - b))
    assert errs[0] < 5e-3, errs
    for e1, e2 in zip(errs, errs[1:]):
        assert 6.0 < e1 / e2 < 10.0, "Trotter error not O(dt^3): %s" % errs


def pin_pauli_expectations():
    """<P> against the Kronecker product of Pauli matrices; |<P>| <= 1;
    linearity in the coefficients; a Pauli sum is bounded by sum |c|."""
    rng = np.random.default_rng(8)
    for n in (1, 3, 5, 6):
        x = _rand_state(rng, n)
        for _ in range(6):
            letters = "".join("IXYZ"[k] for k in rng.integers(0, 4, n))
            v = oracle.pauli_expval(n, x, letters)
            _close(v, np.vdot(x, kron.pauli_full(letters) @ x).real, 1e-13, "<%s>" % letters)
            assert abs(v) <= 1 + 1e-12
        obs = W.random_pauli_sum(rng, n, 5)
        e = oracle.expvals(n, x, [obs])[0]
        _close(e, sum(c * oracle.pauli_expval(n, x, l) for c, l in obs), 1e-13, "linearity")
        assert abs(e) <= sum(abs(c) for c, _ in obs) + 1e-12


def pin_marginal_probability():
    """P(wire w = 0) = sum of |amp|^2 over the half with that bit clear:
    on a product state of RY(t_w) it is cos^2(t_w/2)."""
    rng = np.random.default_rng(9)
    n = 5
    t = rng.uniform(0, 2 * np.pi, n)
    c = W.Circuit(n, [W.Gate("ry", (q,), "param", q) for q in range(n)], n)
    psi = oracle.state(c, t)
    for w in range(n):
        _close(oracle.prob_zero(n, psi, w), np.cos(t[w] / 2) ** 2, 1e-14, "P(w=%d)" % w)


def pin_marginal_distribution():
    """Marginals of several wires (first listed wire = most significant bit
    of the outcome): on a product of RY(t_w)|0> states the Kronecker product
    of the per-wire [cos^2(t/2), sin^2(t/2)] in the listed order; on
    (|0..0> + |1..1>)/sqrt(2) half on all-zero and half on all-one; over all
    wires in order |psi|^2 itself and in reverse order its bit reversal; a
    single wire agrees with the C routine's P(w = 0)."""
    rng = np.random.default_rng(11)
    n = 5
    t = rng.uniform(0, 2 * np.pi, n)
    c = W.Circuit(n, [W.Gate("ry", (q,), "param", q) for q in range(n)], n)
    psi = oracle.state(c, t)
    for wires in ([3, 0, 4], [0], [4, 1], [2, 3, 1, 0]):
        want = np.ones(1)
        for w in wires:
            want = np.kron(want, [np.cos(t[w] / 2) ** 2, np.sin(t[w] / 2) ** 2])
        _close(oracle.probs(n, psi, wires), want, 1e-14, "product-state marginal %s" % wires)
    ghz = np.zeros(1 << n, complex)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    _close(oracle.probs(n, ghz, [2, 0]), [0.5, 0, 0, 0.5], 1e-15, "GHZ two-wire marginal")
    x = _rand_state(rng, n)
    _close(oracle.probs(n, x, list(range(n))), np.abs(x) ** 2, 1e-15, "all wires")
    rev = np.array([int(format(j, "0%db" % n)[::-1], 2) for j in range(1 << n)])
    _close(oracle.probs(n, x, list(range(n))[::-1]), (np.abs(x) ** 2)[rev], 1e-15, "all wires reversed")
    for w in range(n):
        p0 = oracle.prob_zero(n, x, w)
        _close(oracle.probs(n, x, [w]), [p0, 1 - p0], 1e-14, "single wire %d vs the C routine" % w)


def pin_sampling():
    """Inverse transform on a hand-made distribution at and around its
    cumulative sums (a uniform equal to a cumulative sum belongs to the next
    outcome; zero-probability outcomes are never drawn; a uniform not below
    the total gives the last outcome of nonzero probability), and the
    frequencies of 200000 seeded uniforms within 5 standard deviations."""
    p = [0.2, 0.0, 0.5, 0.3, 0.0]
    u = [0.0, 0.1999999, 0.2, 0.6999999, 0.7, 0.9999999, 1.0, 1.5]
    assert list(oracle.sample(p, u)) == [0, 0, 2, 2, 3, 3, 3, 3], list(oracle.sample(p, u))
    assert list(oracle.sample([0.0, 0.0], [0.3])) == [0]
    rng = np.random.default_rng(12)
    q = rng.dirichlet(np.ones(6))
    N = 200000
    counts = np.bincount(oracle.sample(q, rng.uniform(0, 1, N)), minlength=6)
    sd = np.sqrt(N * q * (1 - q))
    assert np.all(np.abs(counts - N * q) <= 5 * sd + 1), (counts, N * q)


def pin_two_qubit_xy_rotations():
    """RXX(t) and RYY(t) are the matrix exponentials exp(-i t P(x)P / 2)
    (scipy's expm of the Kronecker product; first listed wire = most
    significant bit), and their parameter-shift gradient equals central
    differences in a small circuit."""
    X = np.array([[0, 1], [1, 0]], complex)
    Y = np.array([[0, -1j], [1j, 0]])
    rng = np.random.default_rng(13)
    for name, P in (("rxx", X), ("ryy", Y)):
        for t in rng.uniform(-2 * np.pi, 2 * np.pi, 3):
            _close(oracle.gate_matrix(name, t), expm(-0.5j * t * np.kron(P, P)), 1e-14, "%s(%.3f)" % (name, t))
    n = 4
    c = W.Circuit(n, [W.Gate("h", (q,)) for q in range(n)] + [W.Gate("ry", (1,), "param", 0),
                  W.Gate("rxx", (0, 2), "param", 1), W.Gate("ryy", (3, 1), "param", 2), W.Gate("cnot", (2, 3)),
                  W.Gate("ryy", (2, 0), "param", 3), W.Gate("rxx", (1, 3), "param", 4)], 5)
    th = rng.uniform(0, 2 * np.pi, 5)
    obs = [[(0.7, "ZXIY"), (-0.4, "YZZI")]]
    gp, _ = oracle.grad_param_shift(c, th, None, obs, np.ones((1, 1)), 1)
    gf, _ = oracle.grad_fd(c, th, None, obs, np.ones((1, 1)), 1)
    _close(gp, gf, 1e-8, "shift vs central differences (rxx, ryy)")


def pin_u3_gate():
    """U3(theta, phi, lambda) = e^{i(phi+lambda)/2} RZ(phi) RY(theta) RZ(lambda)
    (each rotation scipy's expm of its generator); special cases U3(t,0,0) =
    RY(t), U3(0,0,l) = diag(1, e^{i l}), U3(pi/2, 0, pi) = H; unitary."""
    rng = np.random.default_rng(14)
    for _ in range(6):
        a = rng.uniform(-2 * np.pi, 2 * np.pi, 3)
        U = oracle.u3_matrix(*a)
        _close(U, kron.u3(*a), 1e-14, "U3%s" % (tuple(np.round(a, 3)),))
        _close(U.conj().T @ U, np.eye(2), 1e-14, "U3 unitary")
        _close(oracle.u3_matrix(a[0], 0, 0), kron.named("ry", a[0]), 1e-15, "U3(t,0,0) = RY(t)")
        _close(oracle.u3_matrix(0, 0, a[2]), np.diag([1, np.exp(1j * a[2])]), 1e-15, "U3(0,0,l)")
    _close(oracle.u3_matrix(np.pi / 2, 0, np.pi), kron.named("h"), 1e-15, "U3(pi/2,0,pi) = H")


def pin_controlled_rotations():
    """CRX/CRY/CRZ(t) on (control, target) = exp(-i t |1><1| (x) P / 2)
    (scipy's expm; control = most significant bit of the 4x4): the identity
    where the control reads 0, the rotation where it reads 1; in a register
    the control is the first listed wire."""
    rng = np.random.default_rng(15)
    for op in ("crx", "cry", "crz"):
        for t in rng.uniform(-2 * np.pi, 2 * np.pi, 3):
            U = oracle.gate_matrix(op, t)
            _close(U, kron.named(op, t), 1e-14, "%s(%.3f)" % (op, t))
            _close(U[:2, :2], np.eye(2), 0, "%s control-0 block" % op)
            _close(U[2:, 2:], kron.named("r" + op[2], t), 1e-14, "%s control-1 block" % op)
    # CRY with control wire 2 and target wire 0 of three, from |1 0 1> vs |0 0 1>
    t = 1.1
    c = W.Circuit(3, [W.Gate("x", (2,)), W.Gate("cry", (2, 0), "param", 0)], 1)
    want = np.zeros(8, complex)
    want[0b001], want[0b101] = np.cos(t / 2), np.sin(t / 2)
    _close(oracle.state(c, [t]), want, 1e-15, "CRY(2 -> 0) with the control set")
    c = W.Circuit(3, [W.Gate("cry", (2, 0), "param", 0)], 1)
    _close(oracle.state(c, [t]), np.eye(8)[0], 0, "CRY(2 -> 0) with the control clear")


def pin_u3_and_controlled_rotations_bruteforce():
    """Random circuits with U3 and controlled rotations among the other
    gates (parameters and data) at n <= 5 equal the Kronecker-embedded
    product, with U3's three angles read from consecutive entries."""
    rng = np.random.default_rng(16)
    ops = ("h", "rx", "ry", "rz", "cnot", "cz", "u3", "crx", "cry", "crz", "rxx")
    for n in (2, 3, 5):
        for trial in range(3):
            c = W.random_circuit(rng, n, 20, ops=ops, with_data=True)
            P = c.n_params        # at least one U3 and one controlled rotation, whatever was drawn
            extra = [W.Gate("u3", (n - 1,), "param", P), W.Gate(("crx", "cry", "crz")[trial], (n - 1, 0), "param", P + 3)]
            c = W.Circuit(n, extra[:1] + c.gates + extra[1:], P + 4, c.n_data)
            params, data = W.random_params(rng, c, 1)
            _close(oracle.state(c, params, data), kron.state(c, params, data), 1e-12,
                   "kron with u3 / cr n=%d trial %d" % (n, trial))


def pin_four_term_shift_equals_fd():
    """The four-term rule of the controlled rotations and the two-term rule
    on each U3 angle equal central finite differences (parameters and
    data), and a plain two-term rule would miss a controlled rotation's
    derivative."""
    rng = np.random.default_rng(17)
    ops = ("h", "ry", "cnot", "u3", "crx", "cry", "crz")
    for n in (2, 4):
        c = W.random_circuit(rng, n, 16, ops=ops, with_data=True)
        params, data = W.random_params(rng, c, 2)
        obs = [W.random_pauli_sum(rng, n, 3)]
        w = rng.standard_normal((2, 1))
        a = oracle.grad_param_shift(c, params, data, obs, w, 2)
        b = oracle.grad_fd(c, params, data, obs, w, 2)
        _close(a[0], b[0], 2e-8, "shift vs FD params n=%d" % n)
        _close(a[1], b[1], 2e-8, "shift vs FD data n=%d" % n)
    # one controlled rotation: the two-term rule alone is not its derivative
    c = W.Circuit(2, [W.Gate("h", (0,)), W.Gate("ry", (1,), "param", 1), W.Gate("crx", (0, 1), "param", 0)], 2)
    th = np.array([0.9, 0.4])
    obs = [[(1.0, "XI"), (0.5, "IZ")]]        # X on the control sees both branches
    fd = oracle.grad_fd(c, th, None, obs, np.ones((1, 1)), 1)[0][0]
    e = lambda t: oracle.forward(c, np.array([t, 0.4]), None, obs, 1)[0, 0]
    two = (e(0.9 + np.pi / 2) - e(0.9 - np.pi / 2)) / 2
    assert abs(two - fd) > 1e-3, "two-term rule matched a controlled rotation"
    _close(oracle.grad_param_shift(c, th, None, obs, np.ones((1, 1)), 1)[0][0], fd, 2e-8, "four-term CRX")


def pin_hessian_closed_forms():
    """Second derivatives in closed form.  (a) RY(a) on wire 0, RY(2b) on
    wire 1, observable Z0 Z1: E = cos a cos 2b, so H = [[-cos a cos 2b,
    2 sin a sin 2b], [2 sin a sin 2b, -4 cos a cos 2b]] (the factor 2 of the
    second gate's scale is chained in).  (b) H on wire 0, CRY(t) from wire 0
    to wire 1, observable Z1: E = (1 + cos t) / 2, E'' = -cos(t) / 2 (the
    four-term rule applied twice).  (c) U3(theta, phi, lambda)|0> has
    <X> = sin(theta) cos(phi), independent of lambda."""
    a, b = 0.7, -1.1
    c = W.Circuit(2, [W.Gate("ry", (0,), "param", 0), W.Gate("ry", (1,), "param", 1, 2.0)], 2)
    H = oracle.hessian_param_shift(c, np.array([a, b]), None, [[(1.0, "ZZ")]], [1.0])
    want = np.array([[-np.cos(a) * np.cos(2 * b), 2 * np.sin(a) * np.sin(2 * b)],
                     [2 * np.sin(a) * np.sin(2 * b), -4 * np.cos(a) * np.cos(2 * b)]])
    _close(H, want, 1e-12, "Hessian of cos a cos 2b")
    for t in (0.3, 2.0, -2.6):
        c = W.Circuit(2, [W.Gate("h", (0,)), W.Gate("cry", (0, 1), "param", 0)], 1)
        H = oracle.hessian_param_shift(c, np.array([t]), None, [[(1.0, "IZ")]], [1.0])
        _close(H, [[-np.cos(t) / 2]], 1e-12, "CRY second derivative t=%g" % t)
    th, ph, la = 1.2, -0.4, 2.2
    c = W.Circuit(1, [W.Gate("u3", (0,), "param", 0)], 3)
    H = oracle.hessian_param_shift(c, np.array([th, ph, la]), None, [[(1.0, "X")]], [1.0])
    want = np.array([[-np.sin(th) * np.cos(ph), -np.cos(th) * np.sin(ph), 0],
                     [-np.cos(th) * np.sin(ph), -np.sin(th) * np.cos(ph), 0], [0, 0, 0]])
    _close(H, want, 1e-12, "U3 Hessian of sin(theta) cos(phi)")


def pin_hessian_equals_fd_of_gradient():
    """The Hessian against central differences of the shift-rule gradient
    (h = 1e-5: truncation ~h^2, rounding ~1e-16/h), on random circuits with
    every differentiable gate kind, a parameter read by two gates with
    different scales, and data-encoded gates (held fixed); and it is
    symmetric."""
    rng = np.random.default_rng(23)
    ops = ("h", "rx", "ry", "rz", "cnot", "cz", "cp", "rzz", "rxx", "ryy", "u3", "crx", "cry", "crz")
    for n in (2, 3):
        c = W.random_circuit(rng, n, 10, ops=ops, with_data=True)
        P = c.n_params
        c = W.Circuit(n, c.gates + [W.Gate("rx", (0,), "param", 0, -1.5)], P, c.n_data)
        params, data = W.random_params(rng, c, 1)
        obs = [W.random_pauli_sum(rng, n, 3), W.random_pauli_sum(rng, n, 2)]
        w = rng.standard_normal(2)
        H = oracle.hessian_param_shift(c, params, data, obs, w)
        h = 1e-5
        F = np.zeros((P, P))
        for q in range(P):
            pp, pm = params.copy(), params.copy()
            pp[q] += h
            pm[q] -= h
            gp = oracle.grad_param_shift(c, pp, data, obs, w[None, :], 1)[0]
            gm = oracle.grad_param_shift(c, pm, data, obs, w[None, :], 1)[0]
            F[:, q] = (gp - gm) / (2 * h)
        _close(H, F, 1e-8, "Hessian vs FD of the gradient n=%d" % n)
        _close(H, H.T, 1e-12, "Hessian symmetry n=%d" % n)


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
