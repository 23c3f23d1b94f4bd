"""The autotuners' candidate sets and cache keys (host only): the
single-plan candidates include the compiled passes' wider tiles when jit is
on, the uneven-batch candidates are exactly the tile shapes the
multi-circuit kernels exist for (every circuit of the 64-circuit workload
joins the shared launches at each of them), and the cache key separates
jit from interpreted tuning."""
import numpy as np

import workloads as W
from paper_2512_18995_amd import engine


def test_single_plan_candidates():
    c64 = engine.candidate_options("c64", 20, jit=False)
    c64j = engine.candidate_options("c64", 20, jit=True)
    c128j = engine.candidate_options("c128", 20, jit=True)
    assert max(o["tile_bits"] for o in c64) == 5 and max(o["tile_bits"] for o in c64j) == 6
    assert max(o["tile_bits"] for o in c128j) == 5
    assert all(o["jit"] for o in c64j) and not any(o["jit"] for o in c64)
    assert {o["dense_fuse"] for o in c64} == {0, 4, 5}
    # small registers: no tile wider than the register allows
    assert max(o["tile_bits"] for o in engine.candidate_options("c64", 9, jit=True)) == 3


def test_cache_key_separates_jit_and_structure():
    c = W.config(1, n=8, layers=2).circuit
    k0 = engine._structure_key(c, "c64", 1, False, True, "gfx950", jit=False)
    k1 = engine._structure_key(c, "c64", 1, False, True, "gfx950", jit=True)
    k2 = engine._structure_key(W.config(1, n=8, layers=3).circuit, "c64", 1, False, True, "gfx950", jit=False)
    assert len({k0, k1, k2}) == 3
    assert k0 == engine._structure_key(c, "c64", 1, False, True, "gfx950", jit=False)


def test_multi_candidates_batch_every_circuit():
    mw = W.config(4)
    for dtype in ("c64", "c128"):
        cands = engine.multi_candidates(dtype)
        assert cands
        for opt in cands:
            plans = [engine.Plan(it.circuit, dtype, tile_bits=opt["tile_bits"], adj_tile_bits=opt["adj_tile_bits"])
                     for it in mw.items]
            obs = [engine.Observable(it.circuit.n, it.observables) for it in mw.items]
            M = engine.Multi(plans, obs)
            assert all(M.batched), (dtype, opt, M.batched)
