"""The allocation-free forward entry point (dq_apply_circuit_noalloc),
called through the C ABI: identical states to dq_apply_circuit on two calls
in a row (the second with a smaller batch and different angles, so that
stale scratch contents would show), for interpreted and compiled plans and
per-sample data; host-side rejection of a plan not yet resident on the
device and of matrix blocks beyond the scratch, with the state untouched."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import DEV, t64

import paper_2512_18995_amd as dq
from paper_2512_18995_amd import _lib

pytestmark = pytest.mark.gpu


def _noalloc(plan, st, p, d, from_zero=True):
    s = torch.cuda.current_stream().cuda_stream
    return _lib.lib().dq_apply_circuit_noalloc(plan.handle, st.data_ptr(), st.shape[0],
                                               None if p is None else p.data_ptr(), 0 if p is None or p.dim() < 2 else p.shape[1],
                                               None if d is None else d.data_ptr(), 0 if d is None or d.dim() < 2 else d.shape[1],
                                               1 if from_zero else 0, s)


@pytest.mark.parametrize("jit", [False, True], ids=["interpreted", "compiled"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_equals_apply_circuit(jit, dtype):
    rng = np.random.default_rng(4242)
    n = 12
    ops = ("h", "rx", "ry", "rz", "cnot", "cz", "u3", "cry", "rzz")
    c = W.random_circuit(rng, n, 10 * n, ops=ops, with_data=True)
    plan = dq.Plan(c, dtype, jit=jit)
    for B in (6, 3):                      # the second call is smaller
        params, data = W.random_params(rng, c, B, per_sample=True)
        p, d = t64(params), t64(data)
        ref = plan.state(B, DEV)
        dq.apply_circuit(plan, ref, p, d, from_zero=True)
        got = plan.state(B, DEV)
        got.fill_(float("nan"))
        assert _noalloc(plan, got, p, d) == 0, _lib.lib().dq_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), float((got - ref).abs().max())
    # from a given state (not |0..0>): the same input state for both paths
    params, data = W.random_params(rng, c, 2, per_sample=True)
    p, d = t64(params), t64(data)
    x = torch.randn(2, 1 << n, dtype=plan.state(1, DEV).dtype, device=DEV)
    ref, got = x.clone(), x.clone()
    dq.apply_circuit(plan, ref, p, d, from_zero=False)
    assert _noalloc(plan, got, p, d, from_zero=False) == 0, _lib.lib().dq_last_error()
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_rejections_leave_the_state_alone():
    rng = np.random.default_rng(7)
    c = W.random_circuit(rng, 8, 40, ops=("h", "ry", "rz", "cnot"))
    params, _ = W.random_params(rng, c, 1)
    plan = dq.Plan(c, "c64")
    st = plan.state(2, DEV)
    st.fill_(3.0)
    # never used on this device: nothing uploaded, nothing enqueued
    assert _noalloc(plan, st, t64(params), None) == 1
    assert "not yet resident" in _lib.lib().dq_last_error().decode()
    torch.cuda.synchronize()
    assert bool((st == 3.0).all())
    dq.apply_circuit(plan, plan.state(1, DEV), t64(params), None)
    # per-sample matrix blocks beyond the 16 MiB scratch
    big = W.random_circuit(rng, 8, 600, ops=("u3",))
    pb = dq.Plan(big, "c128")
    x = pb.state(256, DEV)
    P = t64(rng.uniform(0, 6, (256, big.n_params)))
    dq.apply_circuit(pb, x, P, None)
    need = pb.workspace_size(256, per_sample=True)
    assert need > 16 << 20, need
    x.fill_(3.0)
    assert _noalloc(pb, x, P, None) == 4
    assert "scratch" in _lib.lib().dq_last_error().decode()
    torch.cuda.synchronize()
    assert bool((x == 3.0).all())
    assert _noalloc(plan, st, t64(params), None) == 0
    torch.cuda.synchronize()
