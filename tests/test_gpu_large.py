"""Registers beyond 2^32 amplitudes on one GPU: 33 qubits (68.7 GB
complex64 state; forward, expectation and the adjoint gradient, whose two
states fill 137 GB) and 34 qubits (137 GB; forward and expectation).  One
layer of the benchmark circuit (RY, RZ on every wire, then the CNOT ring)
has closed forms for everything the path computes, so every physical bit up
to 33 is checked without a reference simulator:

* amplitudes: the RZ(phi) RY(theta) product state read at the ring's
  preimage of the index;
* Z-string expectations, Heisenberg picture: the ring maps Z strings to Z
  strings (conjugation by CNOT(c, t) adds Z_c where Z_t is present), and on
  the product state <prod_{q in M} Z_q> = prod_{q in M} cos(theta_q), with
  no dependence on phi;
* gradients: d/dtheta_q of that product is -sin(theta_q) times the other
  cosines; d/dphi_q = 0.

The 34-qubit register also runs the QFT of a basis state (closed-form
amplitudes exp(2 pi i j k / 2^n) / 2^(n/2))."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import DEV, t64

import paper_2512_18995_amd as dq

pytestmark = pytest.mark.gpu


def _ring_preimage(j, n):
    bit = lambda x, w: (x >> (n - 1 - w)) & 1
    for c in list(range(n))[::-1]:
        t = (c + 1) % n
        if bit(j, c):
            j ^= 1 << (n - 1 - t)
    return j


def _ring_heisenberg(mask, n):
    """The wire set of U^dagger Z_mask U for U = CNOT(0,1) ... CNOT(n-1,0):
    conjugate by the ring's gates from the last to the first."""
    m = set(mask)
    for c in list(range(n))[::-1]:
        t = (c + 1) % n
        if t in m:
            m ^= {c}
    return m


def _closed_forms(n, th):
    """E = sum_i <Z_i Z_{i+1}> (open chain) and dE/dtheta after one layer."""
    E = 0.0
    g = np.zeros(n)
    cs, sn = np.cos(th), np.sin(th)
    for i in range(n - 1):
        M = sorted(_ring_heisenberg([i, i + 1], n))
        E += np.prod(cs[M])
        for q in M:
            g[q] += -sn[q] * np.prod([cs[r] for r in M if r != q])
    return E, g


def _sample_indices(n, rng):
    N = 1 << n
    return np.concatenate([rng.integers(0, N, 4090, dtype=np.int64),
                           [0, 1, N - 1, N - 2, N >> 1, (N >> 1) - 1]]).astype(np.int64)


def _check_amplitudes(st, js, th, ph, n):
    got = st[0, torch.as_tensor(js, device=DEV)].cpu().numpy().astype(np.complex128)
    u = np.stack([np.exp(-0.5j * ph) * np.cos(th / 2), np.exp(0.5j * ph) * np.sin(th / 2)], axis=1)
    want = np.empty(len(js), dtype=np.complex128)
    for i, j in enumerate(js.tolist()):
        pre = _ring_preimage(j, n)
        want[i] = np.prod([u[q, (pre >> (n - 1 - q)) & 1] for q in range(n)])
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print("n=%d one layer: max |err| / max |amp| = %.2e" % (n, err), flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("n", [33, 34])
def test_one_layer_beyond_2_32_amplitudes(n):
    rng = np.random.default_rng(n)
    w = W.config(5, n=n, layers=1)
    th, ph = w.params[:n], w.params[n:2 * n]
    plan = dq.Plan(w.circuit, "c64", jit=True)
    obs = dq.Observable(n, w.observables + [[(1.0, "I" * n)]])   # sum Z_i Z_{i+1}, and the norm
    st = plan.state(1, DEV)
    p = t64(w.params)
    dq.apply_circuit(plan, st, p, None, from_zero=True)
    print("n=%d forward done" % n, flush=True)
    _check_amplitudes(st, _sample_indices(n, rng), th, ph, n)
    E = dq.expval(plan, obs, st).cpu().numpy()[0]
    E_ref, g_ref = _closed_forms(n, th)
    print("n=%d: E = %.9f (closed form %.9f), norm^2 = %.9f" % (n, E[0], E_ref, E[1]), flush=True)
    assert abs(E[1] - 1.0) < 1e-5
    assert abs(E[0] - E_ref) <= 1e-5 * max(1.0, abs(E_ref))
    if n == 33:
        o1 = dq.Observable(n, w.observables)
        g, _ = dq.adjoint_grad(plan, o1, st, p, None, t64(np.ones((1, 1))))
        g = g.cpu().numpy()
        print("n=33 adjoint done: |g_theta| = %.6f" % np.linalg.norm(g[:n]), flush=True)
        err = np.linalg.norm(g[:n] - g_ref) / np.linalg.norm(g_ref)
        assert err <= 1e-5, err
        assert np.max(np.abs(g[n:])) <= 1e-6 * np.linalg.norm(g_ref)
    del st, plan
    torch.cuda.empty_cache()


def test_qft_of_a_basis_state_at_34_qubits():
    n = 34
    N = 1 << n
    rng = np.random.default_rng(3434)
    js = _sample_indices(n, rng)
    plan = dq.Plan(W.qft(n), "c64", jit=True)
    st = plan.state(1, DEV)
    k = 0x2545F4914 % N
    st.zero_()
    st[0, k] = 1.0
    dq.apply_circuit(plan, st, None, None, from_zero=False)
    got = st[0, torch.as_tensor(js, device=DEV)].cpu().numpy().astype(np.complex128)
    scale = np.sqrt(N)
    want = np.exp(2j * np.pi * ((js.astype(object) * k) % N).astype(np.float64) / N) / scale
    err = float(np.max(np.abs(got - want)) * scale)
    print("QFT|k> at 34 qubits: max |err| x 2^(n/2) = %.2e" % err, flush=True)
    assert err <= 2e-5
    nrm = dq.expval(plan, dq.Observable(n, [[(1.0, "I" * n)]]), st).cpu().numpy()[0, 0]
    assert abs(nrm - 1.0) < 1e-5
    del st, plan
    torch.cuda.empty_cache()
