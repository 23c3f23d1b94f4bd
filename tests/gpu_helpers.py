"""Shared helpers of the GPU parity tests: run a workload through the HIP
library (C ABI via the binding) and compare with the oracle."""
import numpy as np
import torch

import paper_2512_18995_amd as dq

DEV = "cuda:0"
CT = {"c64": torch.complex64, "c128": torch.complex128}


def t64(x):
    return None if x is None else torch.as_tensor(np.asarray(x, dtype=np.float64), device=DEV)


def rand_state(rng, n):
    x = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return x / np.linalg.norm(x)


def gpu_forward(circuit, params, data, batch, dtype, fusion=True, init=None, tile_bits=0, fold=True, jit=False):
    """Final states [B, 2^n] (numpy complex128) of the HIP path."""
    plan = dq.Plan(circuit, dtype, fusion=fusion, tile_bits=tile_bits, fold_init=fold, jit=jit)
    st = plan.state(batch, DEV)
    if init is not None:
        dq.state_init(plan, st, torch.as_tensor(np.asarray(init), dtype=CT[dtype], device=DEV))
        dq.apply_circuit(plan, st, t64(params), t64(data), from_zero=False)
    else:
        dq.apply_circuit(plan, st, t64(params), t64(data), from_zero=True)
    torch.cuda.synchronize()
    return plan, st


def state_tol(dtype, ngates):
    """Bound on ||psi - psi_ref||_2 for a unit state after `ngates` gates:
    each gate rounds every amplitude once and its matrix once (unit roundoff
    u = 2^-24 complex64, 2^-53 complex128), so the error grows at most
    linearly, typically like sqrt(ngates); 8 u sqrt(ngates) + 8 u with a
    factor 2 margin per complex multiply-add."""
    u = 2.0 ** -24 if dtype == "c64" else 2.0 ** -53
    return 16 * u * (np.sqrt(max(ngates, 1)) + 1) * 4


def assert_state(got, want, dtype, ngates, what=""):
    got = np.asarray(got, dtype=np.complex128).reshape(want.shape)
    err = np.linalg.norm(got - want)
    tol = state_tol(dtype, ngates)
    assert err <= tol, "%s: ||psi - psi_ref|| = %.3e > %.3e" % (what, err, tol)
    return err


def normwise(got, want, rtol, atol=0.0, what=""):
    """||v - v_ref||_2 <= rtol ||v_ref||_2 + atol (the per-output-tensor
    criterion), reporting the worst element too."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    err = np.linalg.norm(got - want)
    ref = np.linalg.norm(want)
    worst = float(np.max(np.abs(got - want))) if want.size else 0.0
    assert err <= rtol * ref + atol, "%s: ||v-v_ref||=%.3e > %.1e*||v_ref||(=%.3e) + %.1e; worst element %.3e" % (
        what, err, rtol, ref, atol, worst)
    return err / max(ref, 1e-300)


# tolerance of expectations / gradients, relative normwise (C64: the 1e-5
# target; C128: rounding of ~1e3 gates)
RTOL = {"c64": 1e-5, "c128": 1e-11}
