"""Compiled register-tile passes (plan option jit): the straight-line kernels
compiled with hipRTC give the oracle's states, expectations and gradients,
and agree with the interpreted passes."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_helpers import DEV, RTOL, assert_state, gpu_forward, normwise, t64

import paper_2512_18995_amd as dq

pytestmark = pytest.mark.gpu
DTYPES = ["c64", "c128"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,batch,per_sample", [(8, 2, True), (12, 3, False)])
def test_jit_random_circuit_states_and_expvals(dtype, n, batch, per_sample):
    rng = np.random.default_rng(500 + n)
    c = W.random_circuit(rng, n, 10 * n, with_data=True, max_unitary_k=min(3, n))
    params, data = W.random_params(rng, c, batch, per_sample)
    obs = [W.random_pauli_sum(rng, n, 4), [(1.0, "Z" + "I" * (n - 1))]]
    plan, st = gpu_forward(c, params, data, batch, dtype, True, jit=True)
    assert len(plan.jit_sources()) > 0
    got = st.cpu().numpy()
    E = dq.expval(plan, dq.Observable(n, obs), st).cpu().numpy()
    for b in range(batch):
        want = oracle.state(c, params, data, b)
        assert_state(got[b], want, dtype, len(c.gates), "sample %d" % b)
        normwise(E[b], oracle.expvals(n, want, obs), RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12,
                 "expval sample %d" % b)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,batch,per_sample", [(8, 2, True), (11, 2, False)])
def test_jit_adjoint_vs_parameter_shift(dtype, n, batch, per_sample):
    rng = np.random.default_rng(600 + n)
    ops = ("h", "x", "rx", "ry", "rz", "cnot", "cz", "swap", "cp", "rzz", "unitary")
    c = W.random_circuit(rng, n, 8 * n, ops=ops, with_data=True, max_unitary_k=2)
    params, data = W.random_params(rng, c, batch, per_sample)
    obs = [W.random_pauli_sum(rng, n, 5), W.random_pauli_sum(rng, n, 2)]
    w = rng.standard_normal((batch, len(obs)))
    plan, st = gpu_forward(c, params, data, batch, dtype, True, jit=True)
    gp, gd = dq.adjoint_grad(plan, dq.Observable(n, obs), st, t64(params), t64(data), t64(w))
    rp, rd = oracle.grad_param_shift(c, params, data, obs, w, batch, threads=8)
    normwise(gp.cpu().numpy(), rp, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "d/dparams")
    normwise(gd.cpu().numpy(), rd, RTOL[dtype], 1e-6 if dtype == "c64" else 1e-12, "d/ddata")


def _step(plan, obs, params, n):
    st = plan.state(1, DEV)
    p = t64(params)
    dq.apply_circuit(plan, st, p, None, from_zero=True)
    E = dq.expval(plan, obs, st).cpu().numpy()
    g, _ = dq.adjoint_grad(plan, obs, st, p, None, t64(np.ones((1, 1))))
    return E, g.cpu().numpy()


@pytest.mark.parametrize("n", [16, 22, 25])
def test_jit_hea_ring_family_equals_interpreted(n):
    """The flagship circuit family (RY, RZ layers and a CNOT ring; open ZZ
    chain): compiled and interpreted passes run the same operations in the
    same order, so expectations and gradients agree to float64 summation
    order; at n = 16 both also match the oracle.  At n = 25 the state (256
    MiB) is large enough that every tile holds physical bits 3 (a lane bit) and
    4 (a register bit), and the
    compiled plan uses the larger tiles (6 forward, 5 adjoint register bits)."""
    w = W.config(5, n=n, layers=6 if n < 25 else 3)
    obs = dq.Observable(n, w.observables)
    big = {"tile_bits": 6, "adj_tile_bits": 5} if n >= 25 else {}
    pj = dq.Plan(w.circuit, "c64", jit=True, **big)
    if n >= 25:
        assert all(" lbits=3," in l and " rbits=4," in l for l in pj.describe().splitlines() if " tile " in l)
    Ej, gj = _step(pj, obs, w.params, n)
    Ei, gi = _step(dq.Plan(w.circuit, "c64", jit=False), obs, w.params, n)
    normwise(Ej, Ei, 1e-6, 1e-9, "expval jit vs interpreted")
    normwise(gj, gi, 1e-6, 1e-9, "gradient jit vs interpreted")
    if n <= 16:
        want = oracle.expvals(n, oracle.state(w.circuit, w.params), w.observables)
        normwise(Ej[0], want, RTOL["c64"], 1e-6, "expval vs oracle")
        rp, _ = oracle.grad_param_shift(w.circuit, w.params, None, w.observables, np.ones((1, 1)), 1, threads=8)
        normwise(gj, rp, RTOL["c64"], 1e-6, "gradient vs oracle")


def test_jit_graph_replay():
    """A compiled plan's forward + adjoint captured in a HIP graph: replays
    with eager work in between equal the eager result."""
    n = 14
    w = W.config(5, n=n, layers=3)
    plan = dq.Plan(w.circuit, "c64", jit=True)
    obs = dq.Observable(n, w.observables)
    st = plan.state(1, DEV)
    p = t64(w.params)
    ws = plan.workspace(1, False, 1, obs, DEV)
    go = t64(np.ones((1, 1)))
    E = torch.empty((1, 1), dtype=torch.float64, device=DEV)
    G = torch.empty_like(p)

    def step():
        dq.apply_circuit(plan, st, p, None, from_zero=True, ws=ws)
        dq.expval(plan, obs, st, ws=ws, out=E)
        g, _ = dq.adjoint_grad(plan, obs, st, p, None, go, ws=ws)
        G.copy_(g)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    E0, G0 = E.clone(), G.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for _ in range(3):
        st.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(E, E0) and torch.equal(G, G0)


def test_jit_qft_is_dft():
    """The compiled passes of the QFT (Hadamards, controlled phases, the
    wire-reversing swaps) applied to a random 17-qubit state equal the
    unitary inverse DFT of that state."""
    from gpu_helpers import rand_state
    n = 17
    rng = np.random.default_rng(517)
    x = rand_state(rng, n)
    c = W.qft(n)
    plan, st = gpu_forward(c, None, None, 1, "c64", True, init=x, jit=True)
    assert len(plan.jit_sources()) > 0
    assert_state(st.cpu().numpy()[0], np.fft.ifft(x, norm="ortho"), "c64", len(c.gates), "QFT")
