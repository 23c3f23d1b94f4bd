"""HIP path vs the oracle, element by element, through the C ABI.

Sizes are small enough for the oracle to finish in seconds and still span
several register tiles (n >= 7 splits the register into 64-lane x 2^R
tiles) with every wire position as lane bit and as register bit."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_helpers import DEV, RTOL, assert_state, gpu_forward, normwise, rand_state, t64

import paper_2512_18995_amd as dq

pytestmark = pytest.mark.gpu
DTYPES = ["c64", "c128"]
FUSION = [True, False]


def _id(x):
    return str(x)


# ------------------------------------------------------------------ single gates
ONE_Q = ["h", "x", "y", "z", "rx", "ry", "rz"]
TWO_Q = ["cnot", "cz", "swap", "cp", "rzz"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fusion", FUSION, ids=["tile", "plain"])
@pytest.mark.parametrize("n", [5, 9])
def test_every_gate_every_wire(dtype, fusion, n):
    """Each gate kind on every wire (one-qubit) / ordered wire pair
    (two-qubit), applied to a random state."""
    rng = np.random.default_rng(100 + n)
    x = rand_state(rng, n)
    for op in ONE_Q + TWO_Q:
        if op in ONE_Q:
            wire_sets = [(w,) for w in range(n)]
        else:
            wire_sets = [(a, b) for a in range(n) for b in range(n) if a != b]
        for wires in wire_sets:
            theta = float(rng.uniform(0, 2 * np.pi))
            src = "param" if op in W.ROTATIONS else "none"
            c = W.Circuit(n, [W.Gate(op, wires, src, 0 if src == "param" else -1)], 1 if src == "param" else 0)
            params = np.array([theta]) if src == "param" else None
            _, st = gpu_forward(c, params, None, 1, dtype, fusion, init=x)
            want = oracle.state(c, params, None, psi0=x)
            assert_state(st.cpu().numpy()[0], want, dtype, 1, "%s%s n=%d" % (op, wires, n))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fusion", FUSION, ids=["tile", "plain"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_dense_unitary(dtype, fusion, k):
    rng = np.random.default_rng(200 + k)
    n = 9
    x = rand_state(rng, n)
    for trial in range(6):
        wires = tuple(int(w) for w in rng.choice(n, size=k, replace=False))
        c = W.Circuit(n, [W.Gate("unitary", wires, matrix=W.random_unitary(rng, k))])
        _, st = gpu_forward(c, None, None, 1, dtype, fusion, init=x)
        assert_state(st.cpu().numpy()[0], oracle.state(c, psi0=x), dtype, 1, "unitary%s" % (wires,))


# ------------------------------------------------------------------ random circuits
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fusion", FUSION, ids=["tile", "plain"])
@pytest.mark.parametrize("n,batch,per_sample", [(3, 2, False), (7, 3, True), (10, 2, False), (12, 3, True)])
def test_random_circuit_states_and_expvals(dtype, fusion, n, batch, per_sample):
    rng = np.random.default_rng(300 + n)
    c = W.random_circuit(rng, n, 12 * n, with_data=True, max_unitary_k=min(3, n))
    params, data = W.random_params(rng, c, batch, per_sample)
    obs = [W.random_pauli_sum(rng, n, 4), W.random_pauli_sum(rng, n, 3), [(1.0, "Z" + "I" * (n - 1))]]
    plan, st = gpu_forward(c, params, data, batch, dtype, fusion)
    got = st.cpu().numpy()
    O = dq.Observable(n, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    for b in range(batch):
        want = oracle.state(c, params, data, b)
        assert_state(got[b], want, dtype, len(c.gates), "sample %d" % b)
        normwise(E[b], oracle.expvals(n, want, obs), RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12,
                 "expval sample %d" % b)


def _diag_sums(rng, n, nobs, nterms):
    """Sums whose X-free terms take the diagonal-observable kernel: Z on
    random wires, on wires that are bits 6..10 of an amplitude index only
    (the register part of its 2048-amplitude tile), on the other wires only,
    an identity term, and in every other observable an X-carrying term that
    takes the general path beside them; observables are interleaved term by
    term in the list handed over."""
    def zs(wires):
        s = ["I"] * n
        for w in wires:
            s[int(w)] = "Z"
        return "".join(s)
    mid = [n - 1 - b for b in range(6, 11)]
    rest = [w for w in range(n) if w not in mid]
    obs = [[] for _ in range(nobs)]
    for k in range(nterms):
        for o in range(nobs):
            pick = (k + o) % 3
            pool = range(n) if pick == 0 else (mid if pick == 1 else rest)
            wires = rng.choice(list(pool), size=int(rng.integers(1, 4)), replace=False)
            obs[o].append((float(rng.standard_normal()), zs(wires)))
    obs[0].append((0.25, "I" * n))
    for o in range(1, nobs, 2):
        obs[o].append((0.7, "X" + "I" * (n - 2) + "Z"))
    return obs


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,batch,nobs", [(11, 2, 3), (13, 1, 10), (17, 2, 2)])
def test_diagonal_observables(dtype, n, batch, nobs):
    """Expectations and adjoint gradients of Z-string sums (the diagonal
    kernel: one tile at n = 11, one block at 13, many at 17; more than
    eight observables leave the expectation on the general kernel and keep
    the gradient seed on the diagonal one) against the oracle."""
    rng = np.random.default_rng(500 + n)
    ops = ("h", "rx", "ry", "rz", "cnot", "cz", "rzz")
    c = W.random_circuit(rng, n, 3 * n, ops=ops)
    params, data = W.random_params(rng, c, batch, per_sample=True)
    obs = _diag_sums(rng, n, nobs, 5)
    plan, st = gpu_forward(c, params, data, batch, dtype)
    O = dq.Observable(n, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    tol = 1e-6 if dtype == "c64" else 1e-12
    for b in range(batch):
        want = oracle.state(c, params, data, b)
        normwise(E[b], oracle.expvals(n, want, obs), RTOL[dtype], tol, "expval sample %d" % b)
    w = rng.standard_normal((batch, nobs))
    gp, _ = dq.adjoint_grad(plan, O, st, t64(params), t64(data), t64(w))
    gp = gp.cpu().numpy()
    src = [i for i, g in enumerate(c.gates) if g.src == "param"]
    subset = src if n <= 13 else [src[k] for k in np.random.default_rng(5).choice(len(src), 6, replace=False)]
    rp, _ = oracle.grad_param_shift(c, params, data, obs, w, batch, threads=8, gate_subset=subset)
    idx = sorted(c.gates[i].idx for i in subset)
    normwise(gp[:, idx], rp[:, idx], RTOL[dtype], tol, "d/dparams")


def _one_x_sums(rng, n, nobs):
    """Sums of terms with one X or Y (times Z on random other wires) on every
    wire, one wire with more such terms than one tile launch takes, beside a
    Z-only and a two-X term; physical bits 0..5 are lane bits of the tiles,
    6..10 registers of the first set, higher ones later sets."""
    def term(h, letter, zw):
        s = ["I"] * n
        s[h] = letter
        for w in zw:
            if int(w) != h:
                s[int(w)] = "Z"
        return "".join(s)
    obs = [[] for _ in range(nobs)]
    for o in range(nobs):
        for h in range(n):
            zw = rng.choice(n, size=int(rng.integers(0, 4)), replace=False)
            obs[o].append((float(rng.standard_normal()), term(h, "XY"[int(rng.integers(2))], zw)))
        crowd = int(rng.integers(n))
        for k in range(14):
            zw = rng.choice(n, size=int(rng.integers(1, 5)), replace=False)
            obs[o].append((float(rng.standard_normal()), term(crowd, "XY"[k % 2], zw)))
        obs[o].append((float(rng.standard_normal()), "ZZ" + "I" * (n - 2)))
        obs[o].append((float(rng.standard_normal()), "XX" + "I" * (n - 2)))
    return obs


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [11, 13, 17])
def test_one_x_terms_expval_and_adjoint(dtype, n):
    """Observables of one-X (or one-Y) terms times Z strings, as the
    transverse field of an Ising Hamiltonian: complex64 plans take them in
    register tiles (one state read per set of bits), complex128 plans by
    pairs; expectations and adjoint gradients against the oracle."""
    rng = np.random.default_rng(950 + n)
    batch = 2
    c = W.random_circuit(rng, n, 3 * n, ops=("h", "rx", "ry", "rz", "cnot", "cz"), with_data=False)
    params, _ = W.random_params(rng, c, batch, True)
    obs = _one_x_sums(rng, n, 2)
    plan, st = gpu_forward(c, params, None, batch, dtype, True)
    O = dq.Observable(n, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    for b in range(batch):
        want = oracle.state(c, params, None, b)
        normwise(E[b], oracle.expvals(n, want, obs), RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12,
                 "expval sample %d" % b)
    w = rng.standard_normal((batch, len(obs)))
    gp, _ = dq.adjoint_grad(plan, O, st, t64(params), None, t64(w))
    rp, _ = oracle.grad_param_shift(c, params, None, obs, w, batch, threads=8)
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "d/dparams")


@pytest.mark.parametrize("dtype", DTYPES)
def test_fold_init_matches_unfolded(dtype):
    rng = np.random.default_rng(7)
    n = 11
    gates = [W.Gate("rx", (q,), "data", q) for q in range(n)] + [W.Gate("h", (0,)), W.Gate("ry", (3,), "param", 0)]
    gates += W.hea_layers(n, 2, ("ry", "rz"), "ring", first_param=1)[0]
    c = W.Circuit(n, gates, 1 + 4 * n, n)
    params, data = W.random_params(rng, c, 3)
    a = gpu_forward(c, params, data, 3, dtype, True, fold=True)[1].cpu().numpy()
    b = gpu_forward(c, params, data, 3, dtype, True, fold=False)[1].cpu().numpy()
    for s in range(3):
        want = oracle.state(c, params, data, s)
        assert_state(a[s], want, dtype, len(gates), "folded")
        assert_state(b[s], want, dtype, len(gates), "unfolded")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fusion", FUSION, ids=["tile", "plain"])
@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
@pytest.mark.parametrize("n", [1, 2])
def test_one_and_two_qubit_registers(dtype, fusion, jit, n):
    """The smallest registers the ABI accepts (no register tile fits: every
    gate takes a whole-state sweep): random circuits of every gate kind
    that fits, states, expectations and adjoint gradients (parameters and
    data) against the oracle, and the product-state fold."""
    rng = np.random.default_rng(40 + n)
    ops = ONE_Q + (TWO_Q + ["unitary"] if n == 2 else ["unitary"])
    c = W.random_circuit(rng, n, 24, ops=ops, with_data=True, max_unitary_k=n)
    params, data = W.random_params(rng, c, 3, True)
    obs = [W.random_pauli_sum(rng, n, 3), [(1.0, "Z" * n)]]
    w = rng.standard_normal((3, len(obs)))
    plan = dq.Plan(c, dtype, fusion=fusion, jit=jit)
    st = plan.state(3, DEV)
    dq.apply_circuit(plan, st, t64(params), t64(data), from_zero=True)
    got = st.cpu().numpy()
    O = dq.Observable(n, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    tol = 1e-6 if dtype == "c64" else 1e-12
    for b in range(3):
        want = oracle.state(c, params, data, b)
        assert_state(got[b], want, dtype, len(c.gates), "n=%d sample %d" % (n, b))
        normwise(E[b], oracle.expvals(n, want, obs), RTOL[dtype], tol, "expval sample %d" % b)
    gp, gd = dq.adjoint_grad(plan, O, st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, 3, threads=4)
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], tol, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL[dtype], tol, "d/ddata")


# ------------------------------------------------------------------ adjoint gradients
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fusion", FUSION, ids=["tile", "plain"])
@pytest.mark.parametrize("n,batch,per_sample", [(4, 2, False), (8, 2, True), (11, 3, False)])
def test_adjoint_vs_parameter_shift(dtype, fusion, n, batch, per_sample):
    rng = np.random.default_rng(400 + n)
    ops = ("h", "x", "rx", "ry", "rz", "cnot", "cz", "swap", "cp", "rzz", "unitary")
    c = W.random_circuit(rng, n, 8 * n, ops=ops, with_data=True, max_unitary_k=2)
    params, data = W.random_params(rng, c, batch, per_sample)
    obs = [W.random_pauli_sum(rng, n, 5), W.random_pauli_sum(rng, n, 2)]
    w = rng.standard_normal((batch, len(obs)))
    plan, st = gpu_forward(c, params, data, batch, dtype, fusion)
    O = dq.Observable(n, obs)
    gp, gd = dq.adjoint_grad(plan, O, st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, batch, threads=8)
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "d/ddata")


@pytest.mark.parametrize("dtype", DTYPES)
def test_autograd_function(dtype):
    rng = np.random.default_rng(11)
    n, B = 9, 4
    c = W.random_circuit(rng, n, 60, ops=("h", "rx", "ry", "rz", "cnot", "cz"), with_data=True)
    params, data = W.random_params(rng, c, B)
    obs = [W.tfim_open(n, 0.5)]
    plan, O = dq.Plan(c, dtype), dq.Observable(n, obs)
    p = torch.tensor(params, device=DEV, requires_grad=True)
    d = torch.tensor(data, device=DEV, requires_grad=True)
    E = dq.expectation(plan, O, p, d)
    w = torch.tensor(rng.standard_normal((B, 1)), device=DEV)
    (E * w).sum().backward()
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w.cpu().numpy(), B, threads=8)
    normwise(p.grad.cpu().numpy(), rp, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "autograd params")
    normwise(d.grad.cpu().numpy(), rd, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "autograd data")


# ------------------------------------------------------------------ paper examples
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fusion", FUSION, ids=["tile", "plain"])
def test_listing1_printed_values(dtype, fusion):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "listing1.json")))
    c, th, data, obs = W.listing1(g["theta"], g["data"])
    plan, st = gpu_forward(c, th, data, 1, dtype, fusion)
    O = dq.Observable(3, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    assert abs(E[0, 0] - g["expval"]) <= g["tol"]
    gp, _ = dq.adjoint_grad(plan, O, st, t64(th), t64(data), t64(np.ones((1, 1))))
    assert np.max(np.abs(gp.cpu().numpy() - g["grad"])) <= g["tol"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [4, 10, 13])
def test_qft_is_dft(dtype, n):
    rng = np.random.default_rng(500 + n)
    x = rand_state(rng, n)
    c = W.qft(n)
    _, st = gpu_forward(c, None, None, 1, dtype, True, init=x)
    assert_state(st.cpu().numpy()[0], np.fft.ifft(x, norm="ortho"), dtype, len(c.gates), "QFT")


def test_dist_listing_data_gradient():
    c, params, data, obs = W.dist_listing()
    plan, st = gpu_forward(c, params, data, 1, "c128", True)
    O = dq.Observable(4, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    normwise(E[0], oracle.forward(c, params, data, obs, 1)[0], 1e-12, 1e-14, "expvals")
    _, gd = dq.adjoint_grad(plan, O, st, None, t64(data), t64(np.ones((1, 2))))
    _, rd = oracle.grad_param_shift(c, params, data, obs, np.ones((1, 2)), 1)
    normwise(gd.cpu().numpy(), rd, 1e-11, 1e-13, "data gradient")


# ------------------------------------------------------------------ properties
def test_deterministic_bitwise():
    rng = np.random.default_rng(13)
    n, B = 14, 4
    c = W.random_circuit(rng, n, 80, ops=("h", "rx", "ry", "rz", "cnot", "cz", "rzz"))
    params, _ = W.random_params(rng, c, B, True)
    obs = [W.random_pauli_sum(rng, n, 6)]
    O = dq.Observable(n, obs)
    outs = []
    for _ in range(2):
        plan, st = gpu_forward(c, params, None, B, "c64", True)
        E = dq.expval(plan, O, st)
        gp, _ = dq.adjoint_grad(plan, O, st, t64(params), None, t64(np.ones((B, 1))))
        outs.append((E.cpu().numpy(), gp.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_norm_preserved_deep_c64():
    rng = np.random.default_rng(17)
    n, B = 16, 2
    c = W.random_circuit(rng, n, 600, ops=("h", "rx", "ry", "rz", "cnot", "cz", "rzz", "cp", "swap"))
    params, _ = W.random_params(rng, c, B)
    _, st = gpu_forward(c, params, None, B, "c64", True)
    norms = torch.linalg.vector_norm(st.to(torch.complex128), dim=1).cpu().numpy()
    assert np.all(np.abs(norms - 1) < 1e-5), norms


# ------------------------------------------------------------------ matrix-core dense blocks
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [4, 5])
def test_dense_unitary_on_matrix_cores(dtype, k):
    """A dense 4- or 5-qubit unitary in a fused plan runs as one MFMA sweep;
    target bits low, high, mixed and unordered."""
    rng = np.random.default_rng(600 + k)
    n = 13
    x = rand_state(rng, n)
    placements = [tuple(range(n - k, n)), tuple(range(k)), tuple(range(k))[::-1],
                  tuple(int(w) for w in rng.choice(n, size=k, replace=False)),
                  tuple(int(w) for w in rng.choice(n, size=k, replace=False))]
    for wires in placements:
        c = W.Circuit(n, [W.Gate("unitary", wires, matrix=W.random_unitary(rng, k))])
        plan, st = gpu_forward(c, None, None, 1, dtype, True, init=x)
        assert plan.stats()["fwd_dense_blocks"] == 1
        assert_state(st.cpu().numpy()[0], oracle.state(c, psi0=x), dtype, 2, "dense unitary %s" % (wires,))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [4, 5])
@pytest.mark.parametrize("n,batch,per_sample", [(11, 2, False), (14, 3, True)])
def test_dense_fuse_forward_and_adjoint(dtype, k, n, batch, per_sample):
    """Forward sweep fused into dense k-qubit blocks (matrix cores), adjoint
    through register tiles: states, expectations and gradients vs the oracle."""
    rng = np.random.default_rng(700 + n + k)
    ops = ("h", "x", "y", "rx", "ry", "rz", "cnot", "cz", "swap", "cp", "rzz")
    c = W.random_circuit(rng, n, 10 * n, ops=ops, with_data=True)
    params, data = W.random_params(rng, c, batch, per_sample)
    obs = [W.random_pauli_sum(rng, n, 4)]
    from gpu_helpers import DEV as _dev
    plan = dq.Plan(c, dtype, dense_fuse=k)
    assert plan.stats()["fwd_dense_blocks"] > 0
    st = plan.state(batch, _dev)
    dq.apply_circuit(plan, st, t64(params), t64(data), from_zero=True)
    got = st.cpu().numpy()
    for b in range(batch):
        assert_state(got[b], oracle.state(c, params, data, b), dtype, len(c.gates), "dense-fused sample %d" % b)
    O = dq.Observable(n, obs)
    w = rng.standard_normal((batch, 1))
    gp, gd = dq.adjoint_grad(plan, O, st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, batch, threads=8)
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "d/ddata")


@pytest.mark.parametrize("k", [4, 5])
def test_dense_fuse_hea_family(k):
    """The 32-qubit workload's circuit family at 16 qubits: dense-fused forward
    equals the tiled forward and the oracle."""
    wl = W.config(5, n=16, layers=4)
    c = wl.circuit
    a = gpu_forward(c, wl.params, None, 1, "c64", True)[1].cpu().numpy()[0]
    plan = dq.Plan(c, "c64", dense_fuse=k)
    st = plan.state(1, DEV)
    dq.apply_circuit(plan, st, t64(wl.params), None, from_zero=True)
    b = st.cpu().numpy()[0]
    want = oracle.state(c, wl.params)
    assert_state(a, want, "c64", len(c.gates), "tiles")
    assert_state(b, want, "c64", len(c.gates), "dense blocks")


# ------------------------------------------------------------------ uneven batches
def _uneven(count=7, nmin=10, nmax=14, lmin=2, lmax=4):
    # sizes chosen so that both the shared tile launches (several circuits)
    # and the single-plan path inside the multi-plan calls are exercised
    return W.config(4, count=count, nmin=nmin, nmax=nmax, lmin=lmin, lmax=lmax)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("variant", ["mixed", "grouped_observables", "first_circuit_8_qubits", "compiled_plans"])
def test_multi_plan_matches_oracle(dtype, variant):
    """Circuits of uneven size in one multi-plan: every circuit's state,
    expectation and gradient equal the oracle's (and the single-plan path).
    Random Pauli sums hold one term per X mask (the expectation sweep's
    4-term build); grouped_observables adds the transverse-field Ising sum,
    whose n - 1 ZZ terms share the X mask 0 (the 32-term build).  Variants
    whose tile shape has no multi-circuit kernel (a first circuit of 8
    qubits sets 2 register bits; compiled plans) run every circuit on the
    single-plan path inside the same calls."""
    mw = _uneven()
    if variant == "first_circuit_8_qubits":
        mw.items.insert(0, W.config(4, count=1, nmin=8, nmax=8, lmin=2, lmax=2).items[0])
    if variant == "grouped_observables":
        for it in mw.items:
            it.observables = [W.tfim_open(it.circuit.n, 0.5)] + it.observables
    plans = [dq.Plan(it.circuit, dtype, jit=variant == "compiled_plans") for it in mw.items]
    obs = [dq.Observable(it.circuit.n, it.observables) for it in mw.items]
    M = dq.Multi(plans, obs)
    if variant in ("mixed", "grouped_observables"):
        assert sum(M.batched) >= 2
    else:
        assert not any(M.batched)
    st = M.states(DEV)
    ws = M.workspace(DEV)
    params = M.pack_params([it.params for it in mw.items], DEV)
    M.apply(st, params, ws)
    E = M.expval(st, ws).cpu().numpy()
    got = st.cpu().numpy()
    for c, it in enumerate(mw.items):
        want = oracle.state(it.circuit, it.params)
        assert_state(M.state_of(torch.as_tensor(got), c).numpy(), want, dtype, len(it.circuit.gates), "circuit %d" % c)
        no = len(it.observables)
        normwise(E[M.out_off[c]:M.out_off[c] + no], oracle.expvals(it.circuit.n, want, it.observables), RTOL[dtype],
                 1e-6 if dtype == "c64" else 1e-12, "expval %d" % c)
    w = torch.as_tensor(np.random.default_rng(3).standard_normal(M.nout), device=DEV)
    g = M.adjoint_grad(st, params, w, ws).cpu().numpy()
    wn = w.cpu().numpy()
    for c, it in enumerate(mw.items):
        no = len(it.observables)
        rp, _ = oracle.grad_param_shift(it.circuit, it.params, None, it.observables,
                                        wn[M.out_off[c]:M.out_off[c] + no][None, :], 1, threads=8)
        normwise(g[M.param_off[c]:M.param_off[c] + it.circuit.n_params], rp, RTOL[dtype],
                 1e-6 if dtype == "c64" else 1e-12, "gradient %d" % c)


def test_multi_plan_graph_replay():
    """The multi-plan step captured in a HIP graph: several replays with eager
    work in between each equal the eager result."""
    mw = _uneven()
    plans = [dq.Plan(it.circuit, "c64") for it in mw.items]
    obs = [dq.Observable(it.circuit.n, it.observables) for it in mw.items]
    M = dq.Multi(plans, obs)
    assert sum(M.batched) >= 2
    st, ws = M.states(DEV), M.workspace(DEV)
    params = M.pack_params([it.params for it in mw.items], DEV)
    w = torch.ones(M.nout, dtype=torch.float64, device=DEV)
    E, G = torch.empty(M.nout, dtype=torch.float64, device=DEV), torch.empty_like(params)

    def step():
        M.apply(st, params, ws)
        M.expval(st, ws, E)
        M.adjoint_grad(st, params, w, ws, G)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                       # warm-up: plan tables uploaded outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref_E, ref_G = E.clone(), G.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for r in range(3):
        E.zero_()
        G.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(E, ref_E) and torch.equal(G, ref_G), "replay %d differs" % r
        step()                       # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(E, ref_E)


def test_uneven_full_config_multi_equals_single_plans():
    """The full 64-circuit uneven batch (12..22 qubits): the multi-plan's
    expectations and gradients equal those of each circuit run alone through
    the single-plan path; circuits of up to 14 qubits also against the oracle."""
    mw = W.config(4)
    plans = [dq.Plan(it.circuit, "c64") for it in mw.items]
    obs = [dq.Observable(it.circuit.n, it.observables) for it in mw.items]
    M = dq.Multi(plans, obs)
    assert all(M.batched)
    st, ws = M.states(DEV), M.workspace(DEV)
    params = M.pack_params([it.params for it in mw.items], DEV)
    w = torch.ones(M.nout, dtype=torch.float64, device=DEV)
    M.apply(st, params, ws)
    E = M.expval(st, ws).cpu().numpy()
    G = M.adjoint_grad(st, params, w, ws).cpu().numpy()
    bad = []
    for c, it in enumerate(mw.items):
        n = it.circuit.n
        s1 = plans[c].state(1, DEV)
        p1 = t64(it.params)
        dq.apply_circuit(plans[c], s1, p1, None, from_zero=True)
        e1 = dq.expval(plans[c], obs[c], s1).cpu().numpy()[0, 0]
        g1, _ = dq.adjoint_grad(plans[c], obs[c], s1, p1, None, t64(np.ones((1, 1))))
        g1 = g1.cpu().numpy()
        gm = G[M.param_off[c]:M.param_off[c] + it.circuit.n_params]
        ok_e = abs(E[M.out_off[c]] - e1) <= 1e-9 * max(1.0, abs(e1))
        ok_g = np.all(np.isfinite(gm)) and np.linalg.norm(gm - g1) <= 1e-9 * max(1e-12, np.linalg.norm(g1))
        if not (ok_e and ok_g):
            bad.append((c, n, len(it.circuit.gates), float(E[M.out_off[c]]), float(e1),
                        float(np.linalg.norm(gm - g1)), bool(np.all(np.isfinite(gm)))))
        if n <= 14:
            want = oracle.expvals(n, oracle.state(it.circuit, it.params), it.observables)[0]
            normwise([e1], [want], 1e-5, 1e-6, "circuit %d expval vs oracle" % c)
    assert not bad, "multi vs single plan differ (c, n, gates, E_multi, E_single, |dg|, finite): %s" % bad[:8]


@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
def test_layout_search_keeps_canonical_order(jit):
    """For a large state the planner may relabel physical bits and append
    the undoing swaps: the state handed back stays in the canonical order,
    and expectations and gradients equal those of the canonical plan."""
    n = 24
    w = W.config(5, n=n, layers=4)
    obs = dq.Observable(n, w.observables)
    out = {}
    for lay in ("auto", "canonical"):
        plan = dq.Plan(w.circuit, "c64", jit=jit, layout=lay)
        assert (plan.stats()["layout_swaps"] > 0) == (lay == "auto")
        st = plan.state(1, DEV)
        p = t64(w.params)
        dq.apply_circuit(plan, st, p, None, from_zero=True)
        S = st.cpu().numpy()[0]
        E = dq.expval(plan, obs, st).cpu().numpy()
        g, _ = dq.adjoint_grad(plan, obs, st, p, None, t64(np.ones((1, 1))))
        out[lay] = (S, E, g.cpu().numpy())
    assert_state(out["auto"][0], out["canonical"][0].astype(np.complex128), "c64", 2 * len(w.circuit.gates), "state")
    normwise(out["auto"][1], out["canonical"][1], RTOL["c64"], 1e-7, "expval")
    normwise(out["auto"][2], out["canonical"][2], RTOL["c64"], 1e-7, "gradient")


# ------------------------------------------------------------------ measurement
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,batch", [(5, 2), (9, 3), (13, 2)])
def test_marginal_probabilities_and_sampling(dtype, n, batch):
    """Marginals of several wire lists (the top wire, the bottom wire, mixed
    order, a random set, every wire when n <= 12) against the oracle on
    random circuit states; shots drawn from the device marginals for seeded
    uniforms, some equal to a cumulative sum (the boundary case) or above
    the total, against the oracle's inverse transform of the same float64
    marginals (an integer decision on identical inputs: bit-exact)."""
    rng = np.random.default_rng(700 + n)
    c = W.random_circuit(rng, n, 6 * n, with_data=True, max_unitary_k=min(3, n))
    params, data = W.random_params(rng, c, batch, per_sample=True)
    plan, st = gpu_forward(c, params, data, batch, dtype)
    lists = [[0], [n - 1], [n - 1, 0, n // 2], [int(w) for w in rng.choice(n, min(4, n), replace=False)]]
    if n <= 12:
        lists.append(list(range(n)))
    states = [oracle.state(c, params, data, b) for b in range(batch)]
    for wires in lists:
        P = dq.probs(plan, st, wires)
        Pn = P.cpu().numpy()
        for b in range(batch):
            want = oracle.probs(n, states[b], wires)
            normwise(Pn[b], want, RTOL[dtype], 1e-7 if dtype == "c64" else 1e-14, "marginal %s, sample %d" % (wires, b))
        shots = 300
        u = rng.uniform(0, 1, (batch, shots))
        cs = np.cumsum(Pn, axis=1)
        k = min(shots - 1, Pn.shape[1])
        u[:, :k] = cs[:, :k]                     # exactly on the cumulative sums
        u[:, -1] = 1.0                           # not below the total
        got = dq.sample(P, torch.as_tensor(u, device=DEV)).cpu().numpy()
        for b in range(batch):
            want = oracle.sample(Pn[b], u[b])
            assert np.array_equal(got[b], want), ("shots", wires, b, np.flatnonzero(got[b] != want)[:5])


def test_marginals_of_a_large_product_state():
    """26 qubits (a 512 MiB complex64 state, beyond the last-level cache):
    after RY(t_w) on every wire the marginal of wires [25, 0, 13] is the
    Kronecker product of [cos^2(t/2), sin^2(t/2)] in that order, and the
    marginal of one wire sums to 1."""
    n = 26
    rng = np.random.default_rng(26)
    t = rng.uniform(0, 2 * np.pi, n)
    c = W.Circuit(n, [W.Gate("ry", (q,), "param", q) for q in range(n)], n)
    plan, st = gpu_forward(c, t, None, 1, "c64")
    wires = [25, 0, 13]
    want = np.ones(1)
    for w in wires:
        want = np.kron(want, [np.cos(t[w] / 2) ** 2, np.sin(t[w] / 2) ** 2])
    P = dq.probs(plan, st, wires).cpu().numpy()[0]
    normwise(P, want, 1e-5, 1e-7, "product-state marginal at 26 qubits")
    assert abs(dq.probs(plan, st, [7]).cpu().numpy()[0].sum() - 1.0) < 1e-5
    del st
    torch.cuda.empty_cache()


@pytest.mark.parametrize("jit", [True, False], ids=["compiled", "interpreted"])
def test_large_states_against_references(jit):
    """24 qubits (a 128 MiB complex64 state: low physical bits pinned into
    every tile, qubit layout searched): the QFT of a random state (applied
    to a given state, so the relabelled layout must be entered first) equals
    numpy's inverse DFT, and two HEA layers from |0..0> equal the oracle's
    state, give its ZZ-chain expectation (the diagonal-observable kernel) and
    the adjoint gradient of two of its parameters (parameter shift on
    the oracle); in both cases with the searched layout and the canonical
    one."""
    n = 24
    rng = np.random.default_rng(24)
    x = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    x /= np.linalg.norm(x)
    want = np.fft.ifft(x, norm="ortho")
    c = W.qft(n)
    w = W.config(5, n=n, layers=2)
    ref = oracle.state(w.circuit, w.params)
    e_ref = oracle.expvals(n, ref, w.observables)
    # parameter shift on the oracle for two parameters
    pick = [0, 2 * n + n // 2]                # an RY of the first and of the second layer
    gates = [i for i, gt in enumerate(w.circuit.gates) if gt.src == "param" and gt.idx in pick]
    rp, _ = oracle.grad_param_shift(w.circuit, w.params, None, w.observables, np.ones((1, 1)), 1, threads=8,
                                    gate_subset=gates)
    g_ref = [float(np.asarray(rp).reshape(-1)[k]) for k in pick]
    for layout in ("auto", "canonical"):
        plan = dq.Plan(c, "c64", jit=jit, layout=layout)
        assert (plan.stats()["layout_swaps"] > 0) == (layout == "auto")
        st = plan.state(1, DEV)
        dq.state_init(plan, st, torch.as_tensor(x.astype(np.complex64), device=DEV))
        dq.apply_circuit(plan, st, None, None, from_zero=False)
        assert_state(st.cpu().numpy()[0], want, "c64", len(c.gates), "QFT, layout %s" % layout)
        del st
        plan = dq.Plan(w.circuit, "c64", jit=jit, layout=layout)
        st = plan.state(1, DEV)
        dq.apply_circuit(plan, st, t64(w.params), None, from_zero=True)
        assert_state(st.cpu().numpy()[0], ref, "c64", len(w.circuit.gates), "HEA, layout %s" % layout)
        O = dq.Observable(n, w.observables)
        E = dq.expval(plan, O, st).cpu().numpy()[0]
        normwise(E, e_ref, RTOL["c64"], 1e-7, "ZZ-chain expectation, layout %s" % layout)
        g, _ = dq.adjoint_grad(plan, O, st, t64(w.params), None, t64(np.ones((1, 1))))
        g = g.cpu().numpy()
        # each entry relative to itself (1e-5), with a floor of 1e-5 of the
        # gradient vector's norm for entries that nearly cancel
        gn = float(np.linalg.norm(g))
        for k, r in zip(pick, g_ref):
            assert abs(g[k] - r) <= 1e-5 * max(abs(r), gn), ("d/dtheta_%d, layout %s" % (k, layout), g[k], r, gn)
        del st
        torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
@pytest.mark.parametrize("n,batch,per_sample", [(6, 2, True), (11, 2, False)])
def test_xx_yy_rotations_forward_and_adjoint(dtype, jit, n, batch, per_sample):
    """RXX and RYY (planned as basis changes around an RZZ that carries the
    angle) among one- and two-qubit gates: states against the oracle, which
    applies their 4x4 matrices directly, and adjoint gradients (parameters
    and data) against its parameter shift."""
    rng = np.random.default_rng(800 + n)
    ops = ("h", "rx", "ry", "rz", "cnot", "rxx", "ryy", "rzz")
    c = W.random_circuit(rng, n, 8 * n, ops=ops, with_data=True)
    assert any(g.op == "rxx" for g in c.gates) and any(g.op == "ryy" for g in c.gates)
    params, data = W.random_params(rng, c, batch, per_sample)
    obs = [W.random_pauli_sum(rng, n, 4), W.random_pauli_sum(rng, n, 2)]
    w = rng.standard_normal((batch, len(obs)))
    plan, st = gpu_forward(c, params, data, batch, dtype, True, jit=jit)
    got = st.cpu().numpy()
    for b in range(batch):
        assert_state(got[b], oracle.state(c, params, data, b), dtype, 5 * len(c.gates), "sample %d" % b)
    gp, gd = dq.adjoint_grad(plan, dq.Observable(n, obs), st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, batch, threads=8)
    tol = 1e-6 if dtype == "c64" else 1e-12
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], tol, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL[dtype], tol, "d/ddata")


MODES = {"plain": dict(fusion=False), "interpreted": dict(fusion=True, jit=False), "compiled": dict(fusion=True, jit=True)}


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("n,batch,per_sample", [(3, 2, True), (7, 2, False), (12, 2, True)])
def test_u3_and_controlled_rotations(dtype, mode, n, batch, per_sample):
    """U3 and the controlled rotations CRX, CRY, CRZ (the planner expands U3
    into phase, RY, phase and each controlled rotation into two half-angle
    rotations around two CNOT or CZ gates) among the other gates: states
    against the oracle, which applies their matrices directly, and adjoint
    gradients for parameters and data against its shift rules (two-term for
    U3's angles, four-term for the controlled rotations)."""
    rng = np.random.default_rng(900 + n)
    ops = ("h", "rx", "ry", "rz", "cnot", "cz", "u3", "crx", "cry", "crz", "rxx")
    c = W.random_circuit(rng, n, 6 * n, ops=ops, with_data=True)
    # one more of each new kind in the middle of the list, reading fresh
    # parameters and a fresh data column
    P, D, mid = c.n_params, c.n_data, len(c.gates) // 2
    extra = [W.Gate("u3", (n - 1,), "param", P), W.Gate("crx", (1, 0), "param", P + 3),
             W.Gate("cry", (n - 1, 1), "data", D, -0.5), W.Gate("crz", (0, n - 1), "param", P + 4)]
    c = W.Circuit(n, c.gates[:mid] + extra + c.gates[mid:], P + 5, D + 1)
    params, data = W.random_params(rng, c, batch, per_sample)
    obs = [W.random_pauli_sum(rng, n, 4), W.random_pauli_sum(rng, n, 2)]
    w = rng.standard_normal((batch, len(obs)))
    m = MODES[mode]
    plan, st = gpu_forward(c, params, data, batch, dtype, m["fusion"], jit=m.get("jit", False))
    got = st.cpu().numpy()
    for b in range(batch):
        assert_state(got[b], oracle.state(c, params, data, b), dtype, 4 * len(c.gates), "sample %d" % b)
    gp, gd = dq.adjoint_grad(plan, dq.Observable(n, obs), st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, batch, threads=8)
    tol = 1e-6 if dtype == "c64" else 1e-12
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], tol, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL[dtype], tol, "d/ddata")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
def test_qcnn_listing_circuit(dtype, jit):
    """The 12-qubit QCNN of the paper's listing (RY data encoding in three
    stages, RXX / RYY convolutions, CRY pooling; observable Z0) on a batch
    of 4 encoded samples: expectations, parameter gradients (summed over
    the batch) and data gradients (per sample) against the oracle."""
    rng = np.random.default_rng(1212)
    c, obs = W.qcnn(12)
    B = 4
    params = rng.uniform(0, 2 * np.pi, c.n_params)
    data = rng.uniform(0, np.pi, (B, c.n_data))
    w = rng.standard_normal((B, 1))
    plan, st = gpu_forward(c, params, data, B, dtype, True, jit=jit)
    O = dq.Observable(c.n, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    normwise(E, oracle.forward(c, params, data, obs, B, threads=8), RTOL[dtype], 1e-7, "expval")
    gp, gd = dq.adjoint_grad(plan, O, st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, B, threads=8)
    tol = 1e-6 if dtype == "c64" else 1e-12
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], tol, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL[dtype], tol, "d/ddata")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("residual", [True, False], ids=["residual", "plain"])
def test_qresnet_listing_circuit(dtype, residual):
    """The QResNet curve-fitting circuit of the paper's listing (U3 layers,
    an RY-encoded input, controlled by wire 0 in the residual form) over a
    batch of 16 inputs: expectations and gradients for the eight (six)
    parameters and the inputs against the oracle."""
    rng = np.random.default_rng(77)
    c, obs = W.qresnet(residual)
    B = 16
    params = rng.uniform(0, 2 * np.pi, c.n_params)
    data = np.linspace(-np.pi, np.pi, B)[:, None]
    w = rng.standard_normal((B, len(obs)))
    plan, st = gpu_forward(c, params, data, B, dtype, True)
    O = dq.Observable(c.n, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    normwise(E, oracle.forward(c, params, data, obs, B, threads=8), RTOL[dtype], 1e-7, "expval")
    gp, gd = dq.adjoint_grad(plan, O, st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, B, threads=8)
    tol = 1e-6 if dtype == "c64" else 1e-12
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], tol, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL[dtype], tol, "d/ddata")


@pytest.mark.parametrize("n,batch,per_sample", [(7, 2, True), (12, 3, False)])
def test_arith64_forward_and_adjoint(n, batch, per_sample):
    """Complex64 states swept with float64 arithmetic (compiled passes):
    states, expectations and gradients for parameters and data against the
    oracle, every gate kind; the state error stays within the complex64
    bound for one rounding per pass."""
    rng = np.random.default_rng(640 + n)
    ops = ("h", "x", "rx", "ry", "rz", "cnot", "cz", "swap", "cp", "rzz", "rxx", "u3", "cry", "crz", "unitary")
    c = W.random_circuit(rng, n, 8 * n, ops=ops, with_data=True, max_unitary_k=1)
    params, data = W.random_params(rng, c, batch, per_sample)
    obs = [W.random_pauli_sum(rng, n, 4), W.tfim_open(n, 0.5)]
    w = rng.standard_normal((batch, len(obs)))
    plan = dq.Plan(c, "c64", jit=True, arith64=True)
    st = plan.state(batch, DEV)
    dq.apply_circuit(plan, st, t64(params), t64(data), from_zero=True)
    got = st.cpu().numpy()
    for b in range(batch):
        assert_state(got[b], oracle.state(c, params, data, b), "c64", plan.stats()["fwd_tile_passes"] + 1,
                     "sample %d" % b)
    O = dq.Observable(n, obs)
    E = dq.expval(plan, O, st).cpu().numpy()
    normwise(E, oracle.forward(c, params, data, obs, batch, threads=8), RTOL["c64"], 1e-7, "expval")
    gp, gd = dq.adjoint_grad(plan, O, st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, batch, threads=8)
    normwise(gp.cpu().numpy(), rp, RTOL["c64"], 1e-6, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL["c64"], 1e-6, "d/ddata")
