"""Hessians (paper section 3.1, the second-order gradient benchmark) on the
GPU against the oracle's double application of the shift rules: closed
forms, random circuits with every differentiable gate kind and data
encodings, the 10-qubit workload in full, and batching of the shifted
circuits (max_shifts)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_helpers import DEV, normwise, t64

import paper_2512_18995_amd as dq

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-11}
ATOL = {"c64": 1e-6, "c128": 1e-12}


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_hessian_closed_form(dtype):
    """RY(a) on wire 0, RY(2b) on wire 1, observable Z0 Z1: E = cos a cos 2b."""
    a, b = 0.7, -1.1
    c = W.Circuit(2, [W.Gate("ry", (0,), "param", 0), W.Gate("ry", (1,), "param", 1, 2.0)], 2)
    plan, obs = dq.Plan(c, dtype), dq.Observable(2, [[(1.0, "ZZ")]])
    H = dq.hessian(plan, obs, t64([a, b])).cpu().numpy()
    want = np.array([[-np.cos(a) * np.cos(2 * b), 2 * np.sin(a) * np.sin(2 * b)],
                     [2 * np.sin(a) * np.sin(2 * b), -4 * np.cos(a) * np.cos(2 * b)]])
    assert np.max(np.abs(H - want)) <= (1e-6 if dtype == "c64" else 1e-13), (H, want)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
@pytest.mark.parametrize("n", [3, 8])
def test_hessian_random_circuits(dtype, jit, n):
    """Every differentiable gate kind (U3's three angles, the controlled
    rotations' two half-angle occurrences, RXX / RYY / RZZ / CP), a
    parameter read by two gates with different scales, data-encoded
    gates held fixed, two weighted observables; symmetric up to rounding;
    the same Hessian with the shifted circuits in batches of 3."""
    rng = np.random.default_rng(300 + n)
    ops = ("h", "rx", "ry", "rz", "cnot", "cz", "cp", "rzz", "rxx", "ryy", "u3", "crx", "cry", "crz")
    c = W.random_circuit(rng, n, 4 * n, ops=ops, with_data=True)
    P = c.n_params
    c = W.Circuit(n, c.gates + [W.Gate("rx", (0,), "param", 0, -1.5)], P, c.n_data)
    params, data = W.random_params(rng, c, 1)
    obs = [W.random_pauli_sum(rng, n, 3), W.random_pauli_sum(rng, n, 2)]
    w = rng.standard_normal(2)
    plan, O = dq.Plan(c, dtype, jit=jit), dq.Observable(n, obs)
    d = None if data is None else t64(data[0])
    H = dq.hessian(plan, O, t64(params), d, t64(w)).cpu().numpy()
    ref = oracle.hessian_param_shift(c, params, data, obs, w, threads=8)
    normwise(H, ref, TOL[dtype], ATOL[dtype], "Hessian n=%d" % n)
    normwise(H, H.T, TOL[dtype], ATOL[dtype], "symmetry")
    H3 = dq.hessian(plan, O, t64(params), d, t64(w), max_shifts=3).cpu().numpy()
    normwise(H3, H, TOL[dtype], ATOL[dtype], "max_shifts=3")


def test_hessian_config1_full():
    """The 10-qubit, 4-layer workload (80 parameters, complex128): all 6400
    entries against the oracle."""
    wl = W.config(1)
    c = wl.circuit
    plan, O = dq.Plan(c, "c128", jit=True), dq.Observable(c.n, wl.observables)
    H = dq.hessian(plan, O, t64(wl.params)).cpu().numpy()
    ref = oracle.hessian_param_shift(c, wl.params, None, wl.observables, [1.0], threads=16)
    rel = normwise(H, ref, 1e-11, 1e-13, "config 1 Hessian")
    print("config 1 Hessian: relative error %.2e, ||H|| = %.3e" % (rel, np.linalg.norm(ref)), flush=True)


def test_hessian_deterministic():
    """Two calls give bitwise equal Hessians (fixed-order reductions)."""
    wl = W.config(1, n=8, layers=2)
    c = wl.circuit
    plan, O = dq.Plan(c, "c64"), dq.Observable(c.n, wl.observables)
    a = dq.hessian(plan, O, t64(wl.params)).cpu().numpy()
    b = dq.hessian(plan, O, t64(wl.params)).cpu().numpy()
    assert np.array_equal(a, b)
