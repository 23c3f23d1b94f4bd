"""The autotuners on the GPU: the tile shape picked for an uneven batch
(and the options picked for a single plan, compiled passes included) is one
of the candidates, a second call is served from the cache, and the plans
built with the pick match the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_helpers import DEV, RTOL, normwise, t64

import paper_2512_18995_amd as dq

pytestmark = pytest.mark.gpu


def test_autotune_multi_pick_matches_oracle(tmp_path):
    mw = W.config(4, count=6, nmin=12, nmax=14, lmin=2, lmax=4)
    circuits = [it.circuit for it in mw.items]
    obsl = [it.observables for it in mw.items]
    params = [it.params for it in mw.items]
    cache = str(tmp_path / "tune.json")
    r = dq.autotune_multi(circuits, obsl, params, "c64", cache_path=cache, device=DEV)
    assert not r["cached"]
    assert {"tile_bits": r["tile_bits"], "adj_tile_bits": r["adj_tile_bits"]} in dq.multi_candidates("c64")
    assert len(r["tried"]) == len(dq.multi_candidates("c64"))
    r2 = dq.autotune_multi(circuits, obsl, params, "c64", cache_path=cache, device=DEV)
    assert r2["cached"] and (r2["tile_bits"], r2["adj_tile_bits"]) == (r["tile_bits"], r["adj_tile_bits"])
    plans = [dq.Plan(c, "c64", tile_bits=r["tile_bits"], adj_tile_bits=r["adj_tile_bits"]) for c in circuits]
    M = dq.Multi(plans, [dq.Observable(c.n, o) for c, o in zip(circuits, obsl)])
    assert all(M.batched)
    st, ws = M.states(DEV), M.workspace(DEV)
    p = M.pack_params(params, DEV)
    M.apply(st, p, ws)
    E = M.expval(st, ws).cpu().numpy()
    for c, it in enumerate(mw.items):
        ref = oracle.forward(it.circuit, it.params, None, it.observables, 1)[0]
        normwise(E[M.out_off[c]:M.out_off[c] + len(ref)], ref, RTOL["c64"], 1e-7, "circuit %d" % c)
    w = torch.ones(M.nout, dtype=torch.float64, device=DEV)
    G = M.adjoint_grad(st, p, w, ws).cpu().numpy()
    it = mw.items[0]
    gref, _ = oracle.grad_param_shift(it.circuit, it.params, None, it.observables, np.ones((1, 1)), 1, threads=8)
    normwise(G[M.param_off[0]:M.param_off[0] + it.circuit.n_params], gref, RTOL["c64"], 1e-6, "gradient")


def test_autotune_single_plan_compiled(tmp_path):
    wl = W.config(3, n=10, layers=2, batch=2)
    c = wl.circuit
    obs = dq.Observable(c.n, wl.observables)
    cache = str(tmp_path / "tune.json")
    r = dq.autotune(c, "c64", obs, t64(wl.params), batch=2, cache_path=cache, device=DEV, jit=True)
    assert not r["cached"] and r["jit"]
    assert {k: r[k] for k in ("tile_bits", "dense_fuse", "jit")} in dq.candidate_options("c64", c.n, True)
    assert dq.autotune(c, "c64", obs, t64(wl.params), batch=2, cache_path=cache, device=DEV, jit=True)["cached"]
    plan = dq.Plan(c, "c64", tile_bits=r["tile_bits"], dense_fuse=r["dense_fuse"], jit=True)
    st = plan.state(2, DEV)
    dq.apply_circuit(plan, st, t64(wl.params), None)
    E = dq.expval(plan, obs, st).cpu().numpy()
    normwise(E, oracle.forward(c, wl.params, None, wl.observables, 2), RTOL["c64"], 1e-7, "expval")
