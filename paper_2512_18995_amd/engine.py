"""Python face of libdq: plans, observables and the four hot-path calls.

Thin wrappers: validation of tensor shapes / dtypes / devices, then one call
into the C ABI with raw device pointers and torch's current HIP stream.
PyTorch provides device memory and streams only.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import check, lib

CDTYPE = {"c64": torch.complex64, "c128": torch.complex128}


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Plan:
    """A circuit planned for one qubit count and precision (host only until
    its first use on a device)."""

    def __init__(self, circuit, dtype: str = "c64", fusion: bool = True, tile_bits: int = 0,
                 fold_init: bool = True, dense_fuse: int = 0, jit: bool = False, adj_tile_bits: int = 0,
                 low_bits: int = 0, layout: str = "auto", arith64: bool = False):
        self.n = int(circuit.n)
        self.dtype = dtype
        self.nparams = int(circuit.n_params)
        self.ndata = int(circuit.n_data)
        self.gates = list(circuit.gates)
        arr, keep = _lib.gate_array(self.gates)
        opt = _lib.DqOptions(1 if fusion else 0, int(tile_bits), 1 if fold_init else 0, int(dense_fuse),
                             1 if jit else 0, int(adj_tile_bits), int(low_bits),
                             {"auto": 0, "canonical": 1}[layout], 1 if arith64 else 0)
        self.jit = bool(jit)
        h = ctypes.c_void_p()
        check(lib().dq_plan_create(ctypes.byref(h), self.n, arr, len(self.gates), self.nparams, self.ndata,
                                   _lib.C64 if dtype == "c64" else _lib.C128, ctypes.byref(opt)), "dq_plan_create")
        self._h = h
        del keep

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().dq_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    def stats(self) -> dict:
        s = _lib.DqPlanStats()
        check(lib().dq_plan_get_stats(self._h, ctypes.byref(s)), "dq_plan_get_stats")
        out = {k: getattr(s, k) for k, _ in _lib.DqPlanStats._fields_ if k not in ("tile_ops", "pad")}
        kinds = ["1q", "1q_diag", "cnot", "cz", "2q_diag", "swap", "1q_real", "1q_rx"]
        for w, prog in enumerate(("fwd", "adj")):
            for where, name in enumerate(("lane", "reg")):
                out["%s_ops_%s" % (prog, name)] = {kinds[k]: int(s.tile_ops[w][where][k]) for k in range(8)
                                                   if s.tile_ops[w][where][k]}
        return out

    def describe(self) -> str:
        """One line per kernel step of the forward and adjoint programs."""
        need = ctypes.c_size_t()
        check(lib().dq_plan_describe(self._h, None, 0, ctypes.byref(need)), "dq_plan_describe")
        buf = ctypes.create_string_buffer(need.value)
        check(lib().dq_plan_describe(self._h, buf, need.value, None), "dq_plan_describe")
        return buf.value.decode()

    def jit_sources(self) -> list:
        """Sources of the plan's compiled pass kernels (jit plans; else empty)."""
        cnt = ctypes.c_int32()
        check(lib().dq_plan_jit_source(self._h, -1, None, 0, None, ctypes.byref(cnt)), "dq_plan_jit_source")
        out = []
        for i in range(cnt.value):
            need = ctypes.c_size_t()
            check(lib().dq_plan_jit_source(self._h, i, None, 0, ctypes.byref(need), None), "dq_plan_jit_source")
            buf = ctypes.create_string_buffer(need.value)
            check(lib().dq_plan_jit_source(self._h, i, buf, need.value, None, None), "dq_plan_jit_source")
            out.append(buf.value.decode())
        return out

    def profile_enable(self, on: bool = True):
        """Bracket every kernel launch of this plan with hipEvents."""
        check(lib().dq_profile_enable(self._h, 1 if on else 0), "dq_profile_enable")

    def profile_read(self, reset: bool = True) -> dict:
        """{family: {"launches", "ms", "bytes"}} summed since the last reset."""
        p = _lib.DqProfile()
        check(lib().dq_profile_read(self._h, ctypes.byref(p), 1 if reset else 0), "dq_profile_read")
        return {k: {"launches": p.launches[i], "ms": p.ms[i], "bytes": p.bytes[i], "flops": p.flops[i]}
                for i, k in enumerate(_lib.PROF_KINDS)}

    def workspace_size(self, batch: int, per_sample: bool = False, grad: int = 0, obs: "Observable" = None) -> int:
        n = ctypes.c_size_t(0)
        check(lib().dq_workspace_size(self._h, obs.handle if obs else None, batch, 1 if per_sample else 0, grad,
                                      ctypes.byref(n)), "dq_workspace_size")
        return n.value

    def state(self, batch: int, device="cuda") -> torch.Tensor:
        return torch.empty((batch, 1 << self.n), dtype=CDTYPE[self.dtype], device=device)

    def workspace(self, batch: int, per_sample=False, grad=0, obs=None, device="cuda") -> torch.Tensor:
        return torch.empty(max(self.workspace_size(batch, per_sample, grad, obs), 1), dtype=torch.uint8,
                           device=device)


class Observable:
    """nobs Pauli sums; each a list of (coef, letters) with letters[w] on wire w."""

    def __init__(self, n: int, observables: Sequence):
        self.n = int(n)
        self.nobs = len(observables)
        terms, off = _lib.pauli_arrays(self.n, observables)
        h = ctypes.c_void_p()
        check(lib().dq_obs_create(ctypes.byref(h), self.n, terms, off, self.nobs), "dq_obs_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().dq_obs_destroy(h)
            except Exception:
                pass
            self._h = None


def _check_state(plan: Plan, state: torch.Tensor):
    if state.dtype != CDTYPE[plan.dtype] or not state.is_cuda or not state.is_contiguous():
        raise ValueError("state must be a contiguous %s CUDA tensor" % CDTYPE[plan.dtype])
    if state.dim() != 2 or state.shape[1] != (1 << plan.n):
        raise ValueError("state must have shape [batch, 2^%d]" % plan.n)


def _f64(t: Optional[torch.Tensor], device) -> Optional[torch.Tensor]:
    if t is None:
        return None
    t = t.detach()
    if t.dtype != torch.float64 or t.device != torch.device(device) or not t.is_contiguous():
        t = t.to(device=device, dtype=torch.float64).contiguous()
    return t


def _stride(t: Optional[torch.Tensor]) -> int:
    return 0 if t is None or t.dim() < 2 else int(t.shape[1])


def state_init(plan: Plan, state: torch.Tensor, init: Optional[torch.Tensor] = None):
    _check_state(plan, state)
    check(lib().dq_state_init(plan.handle, state.data_ptr(), state.shape[0], _ptr(init), _stream(state.device)),
          "dq_state_init")


def apply_circuit(plan: Plan, state: torch.Tensor, params=None, data=None, from_zero: bool = True,
                  ws: Optional[torch.Tensor] = None):
    """Apply the circuit to every sample of ``state`` in place.  ``params``:
    [P] (shared) or [B, P]; ``data``: [B, D] or [D] (shared)."""
    _check_state(plan, state)
    dev = state.device
    B = state.shape[0]
    p, d = _f64(params, dev), _f64(data, dev)
    per_sample = _stride(p) != 0 or _stride(d) != 0
    if ws is None:
        ws = plan.workspace(B, per_sample, 0, None, dev)
    check(lib().dq_apply_circuit(plan.handle, state.data_ptr(), B, _ptr(p), _stride(p), _ptr(d), _stride(d),
                                 1 if from_zero else 0, ws.data_ptr(), ws.numel(), _stream(dev)), "dq_apply_circuit")
    return state


def apply_circuit_noalloc(plan: Plan, state: torch.Tensor, params=None, data=None, from_zero: bool = True):
    """apply_circuit with the gate matrices in the library's device scratch:
    no workspace and no allocation (params / data must already be float64
    contiguous tensors on the state's device; the plan must have run
    apply_circuit on this device once)."""
    _check_state(plan, state)
    dev = state.device
    for t in (params, data):
        if t is not None and (t.dtype != torch.float64 or t.device != dev or not t.is_contiguous()):
            raise ValueError("params / data must be contiguous float64 tensors on %s" % dev)
    check(lib().dq_apply_circuit_noalloc(plan.handle, state.data_ptr(), state.shape[0], _ptr(params),
                                         _stride(params), _ptr(data), _stride(data), 1 if from_zero else 0,
                                         _stream(dev)), "dq_apply_circuit_noalloc")
    return state


def expval(plan: Plan, obs: Observable, state: torch.Tensor, ws: Optional[torch.Tensor] = None,
           out: Optional[torch.Tensor] = None) -> torch.Tensor:
    _check_state(plan, state)
    dev = state.device
    B = state.shape[0]
    if out is None:
        out = torch.empty((B, obs.nobs), dtype=torch.float64, device=dev)
    if ws is None:
        ws = plan.workspace(B, False, 0, obs, dev)
    check(lib().dq_expval(plan.handle, obs.handle, state.data_ptr(), B, out.data_ptr(), ws.data_ptr(), ws.numel(),
                          _stream(dev)), "dq_expval")
    return out


def probs(plan: Plan, state: torch.Tensor, wires, ws: Optional[torch.Tensor] = None,
          out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Marginal probabilities [B, 2^k] of measuring ``wires`` (k <= 12; the
    first listed wire is the most significant bit of the outcome index)."""
    _check_state(plan, state)
    dev = state.device
    B = state.shape[0]
    w = (ctypes.c_int32 * len(wires))(*[int(x) for x in wires])
    if out is None:
        out = torch.empty((B, 1 << len(wires)), dtype=torch.float64, device=dev)
    if ws is None:
        n = ctypes.c_size_t(0)
        check(lib().dq_probs_workspace_size(plan.handle, B, len(wires), ctypes.byref(n)), "dq_probs_workspace_size")
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=dev)
    check(lib().dq_probs(plan.handle, state.data_ptr(), B, w, len(wires), out.data_ptr(), ws.data_ptr(), ws.numel(),
                         _stream(dev)), "dq_probs")
    return out


def sample(p: torch.Tensor, u: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Outcomes [B, shots] (int64) of the distributions p [B, nout] (float64)
    for the caller's uniforms u [B, shots] in [0, 1): inverse transform."""
    if p.dtype != torch.float64 or u.dtype != torch.float64 or p.dim() != 2 or u.dim() != 2 or \
            p.shape[0] != u.shape[0] or not p.is_contiguous() or not u.is_contiguous() or p.device != u.device:
        raise ValueError("p [B, nout] and u [B, shots]: contiguous float64 on one device")
    if out is None:
        out = torch.empty(u.shape, dtype=torch.int64, device=u.device)
    check(lib().dq_sample(p.data_ptr(), p.shape[0], p.shape[1], u.data_ptr(), u.shape[1], out.data_ptr(),
                          _stream(u.device)), "dq_sample")
    return out


def adjoint_grad(plan: Plan, obs: Observable, state: torch.Tensor, params, data, grad_out: torch.Tensor,
                 preserve_state: bool = False, ws: Optional[torch.Tensor] = None, want_data: bool = True):
    """VJP of sum_{b,o} grad_out[b,o] E[b,o] w.r.t. params and data (adjoint
    sweep).  ``state`` must hold the final states; it is consumed unless
    ``preserve_state``."""
    _check_state(plan, state)
    dev = state.device
    B = state.shape[0]
    p, d = _f64(params, dev), _f64(data, dev)
    go = _f64(grad_out, dev)
    if go.shape != (B, obs.nobs):
        raise ValueError("grad_out must be [batch, nobs]")
    per_sample = _stride(p) != 0 or _stride(d) != 0
    if ws is None:
        ws = plan.workspace(B, per_sample, 2 if preserve_state else 1, obs, dev)
    gp = torch.empty_like(p) if p is not None else None
    gd = torch.empty_like(d) if (d is not None and want_data) else None
    check(lib().dq_adjoint_grad(plan.handle, obs.handle, state.data_ptr(), B, _ptr(p), _stride(p), _ptr(d),
                                _stride(d), go.data_ptr(), _ptr(gp), _ptr(gd), 1 if preserve_state else 0,
                                ws.data_ptr(), ws.numel(), _stream(dev)), "dq_adjoint_grad")
    return gp, gd


def hessian(plan: Plan, obs: Observable, params, data=None, weights=None, max_shifts: int = 0,
            ws: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Hessian [P, P] of sum_o weights[o] E_o (one sample, shared ``params``
    [P]; ``data`` one row [D] or None; ``weights`` [nobs], default ones) by
    parameter-shifted adjoint sweeps; ``max_shifts`` bounds the shifted
    circuits per batch (0 = all)."""
    p = _f64(params, "cuda" if not torch.is_tensor(params) else params.device)
    dev = p.device
    d = _f64(data, dev)
    if d is not None:
        d = d.reshape(-1)
    w = torch.ones(obs.nobs, dtype=torch.float64, device=dev) if weights is None else _f64(weights, dev).reshape(-1)
    if p.dim() != 1 or p.numel() != plan.nparams or w.numel() != obs.nobs:
        raise ValueError("params must be [P] and weights [nobs]")
    if out is None:
        out = torch.empty((plan.nparams, plan.nparams), dtype=torch.float64, device=dev)
    if ws is None:
        n = ctypes.c_size_t(0)
        check(lib().dq_hessian_workspace_size(plan.handle, obs.handle, int(max_shifts), ctypes.byref(n)),
              "dq_hessian_workspace_size")
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=dev)
    check(lib().dq_hessian(plan.handle, obs.handle, p.data_ptr(), _ptr(d), w.data_ptr(), out.data_ptr(),
                           int(max_shifts), ws.data_ptr(), ws.numel(), _stream(dev)), "dq_hessian")
    return out


class ExpvalFunction(torch.autograd.Function):
    """E[b, o] = <psi_b(params, data)| H_o |psi_b(...)> with the adjoint
    method as its backward (the custom autograd Function of the paper's
    distributed simulator, section 7.2, here on one GPU)."""

    @staticmethod
    def forward(ctx, params, data, plan: Plan, obs: Observable, batch: int):
        dev = params.device if params is not None else data.device
        state = plan.state(batch, dev)
        apply_circuit(plan, state, params, data, from_zero=True)
        E = expval(plan, obs, state)
        ctx.plan, ctx.obs = plan, obs
        ctx.save_for_backward(params, data, state)
        return E

    @staticmethod
    def backward(ctx, grad_out):
        params, data, state = ctx.saved_tensors
        want_data = data is not None and ctx.needs_input_grad[1]
        gp, gd = adjoint_grad(ctx.plan, ctx.obs, state, params, data, grad_out, preserve_state=True,
                              want_data=want_data)
        if gp is not None and params is not None:
            gp = gp.to(params.dtype)
        if gd is not None:
            gd = gd.to(data.dtype)
        return gp, gd, None, None, None


def expectation(plan: Plan, obs: Observable, params, data=None, batch: Optional[int] = None) -> torch.Tensor:
    """Differentiable [batch, nobs] expectations."""
    if batch is None:
        batch = data.shape[0] if data is not None and data.dim() == 2 else (
            params.shape[0] if params is not None and params.dim() == 2 else 1)
    return ExpvalFunction.apply(params, data, plan, obs, batch)


# ---------------------------------------------------------------- uneven batches
class Multi:
    """Several circuits of different sizes run together (one tile launch per
    pass depth across all circuits).  States and parameters are packed: use
    ``states()``, ``pack_params()`` and the offsets."""

    def __init__(self, plans: Sequence[Plan], observables: Sequence[Observable]):
        self.plans, self.obs = list(plans), list(observables)
        n = len(self.plans)
        ph = (ctypes.c_void_p * n)(*[p.handle.value for p in self.plans])
        oh = (ctypes.c_void_p * n)(*[o.handle.value for o in self.obs])
        h = ctypes.c_void_p()
        check(lib().dq_multi_create(ctypes.byref(h), ph, oh, n), "dq_multi_create")
        self._h = h
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        so, po, oo = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
        check(lib().dq_multi_layout(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), so, po, oo), "dq_multi_layout")
        self.state_amps, self.param_count, self.nout = a.value, b.value, c.value
        self.state_off, self.param_off, self.out_off = list(so), list(po), list(oo)
        sz = ctypes.c_size_t()
        check(lib().dq_multi_workspace_size(h, ctypes.byref(sz)), "dq_multi_workspace_size")
        self.ws_bytes = sz.value
        self.dtype = self.plans[0].dtype
        flags = (ctypes.c_int32 * n)()
        check(lib().dq_multi_batched(h, flags, None), "dq_multi_batched")
        self.batched = [bool(f) for f in flags]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().dq_multi_destroy(h)
            except Exception:
                pass
            self._h = None

    def states(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.state_amps, dtype=CDTYPE[self.dtype], device=device)

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)

    def pack_params(self, per_circuit, device="cuda") -> torch.Tensor:
        out = torch.zeros(max(self.param_count, 1), dtype=torch.float64, device=device)
        for off, p in zip(self.param_off, per_circuit):
            p = torch.as_tensor(p, dtype=torch.float64, device=device).reshape(-1)
            out[off:off + p.numel()] = p
        return out

    def state_of(self, states: torch.Tensor, c: int) -> torch.Tensor:
        return states[self.state_off[c]:self.state_off[c] + (1 << self.plans[c].n)]

    def apply(self, states, params, ws):
        check(lib().dq_multi_apply(self._h, states.data_ptr(), params.data_ptr(), ws.data_ptr(), ws.numel(),
                                   _stream(states.device)), "dq_multi_apply")

    def expval(self, states, ws, out=None):
        if out is None:
            out = torch.empty(self.nout, dtype=torch.float64, device=states.device)
        check(lib().dq_multi_expval(self._h, states.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                    _stream(states.device)), "dq_multi_expval")
        return out

    def adjoint_grad(self, states, params, grad_out, ws, grad=None):
        if grad is None:
            grad = torch.empty_like(params)
        check(lib().dq_multi_adjoint_grad(self._h, states.data_ptr(), params.data_ptr(), grad_out.data_ptr(),
                                          grad.data_ptr(), ws.data_ptr(), ws.numel(), _stream(states.device)),
              "dq_multi_adjoint_grad")
        return grad


# ---------------------------------------------------------------- autotuner
def _arch(device) -> str:
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name)


def _structure_key(circuits, dtype: str, batch: int, per_sample: bool, grad: bool, arch: str, jit=None) -> str:
    """Cache key of a tuning result: circuit structure (gates, wires, angle
    sources; not the angles), dtype, batch, per-sample flag, gradient flag,
    the jit flag and the GPU architecture."""
    import hashlib
    h = hashlib.sha256()
    h.update(("%s|%d|%d|%d|%s|" % (dtype, batch, per_sample, grad, jit)).encode())
    for circuit in (circuits if isinstance(circuits, (list, tuple)) else [circuits]):
        h.update(("n%d|" % circuit.n).encode())
        for g in circuit.gates:
            h.update(("%s:%s:%s;" % (g.op, ",".join(map(str, g.wires)), g.src)).encode())
    h.update(arch.encode())
    return h.hexdigest()[:24]


def candidate_options(dtype: str, n: int, jit: bool = False):
    """Fusion width / tile shape candidates: register bits per tile (the
    gates of one HBM sweep act on up to 6 + tile_bits wires) and the
    dense-block width of the forward sweep; with jit, the compiled passes'
    wider tiles (6 register bits for complex64, 5 for complex128) too."""
    top = (6 if dtype == "c64" else 5) if jit else (5 if dtype == "c64" else 4)
    tiles = [r for r in range(3, top + 1) if r <= n - 6] or [0]
    out = [{"tile_bits": r, "dense_fuse": 0, "jit": bool(jit)} for r in tiles]
    if dtype == "c64":
        out += [{"tile_bits": min(tiles[-1], 5), "dense_fuse": k, "jit": bool(jit)} for k in (4, 5) if n >= k + 5]
    return out


def _load_cache(path):
    import json
    import os
    if os.path.exists(path):
        try:
            return json.load(open(path))
        except (OSError, ValueError):
            return {}
    return {}


def _store_cache(path, cache):
    import json
    import os
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass


def _time_ms(step, reps, device):
    step()
    torch.cuda.synchronize(device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    torch.cuda.synchronize(device)
    return e0.elapsed_time(e1) / reps


def multi_candidates(dtype: str):
    """Tile shapes of the uneven-batch kernels (forward, adjoint register
    bits): those the multi-circuit kernels are built for."""
    fwd = (3, 4, 5) if dtype == "c64" else (3, 4)
    adj = (3, 4) if dtype == "c64" else (3,)
    return [{"tile_bits": f, "adj_tile_bits": a} for f in fwd for a in adj if a <= f]


def autotune_multi(circuits, observables, params, dtype: str = "c64", reps: int = 2,
                   cache_path: Optional[str] = None, device="cuda:0", verbose: bool = False) -> dict:
    """Pick the tile shape (forward and adjoint register bits, i.e. the
    fusion width of a sweep) of an uneven batch with the lowest measured
    time of one forward + expectation + adjoint step of the multi-plan on
    this device; cached like autotune().  Circuits whose plan cannot join
    the shared launches at a candidate shape still run (single-plan path)."""
    import os
    path = cache_path or os.environ.get("DQ_AUTOTUNE_CACHE", os.path.expanduser("~/.cache/dq_autotune.json"))
    key = "multi|" + _structure_key(list(circuits), dtype, 1, False, True, _arch(device))
    cache = _load_cache(path)
    if key in cache:
        return dict(cache[key], cached=True)
    best, timings = None, []
    for opt in multi_candidates(dtype):
        plans = [Plan(c, dtype, tile_bits=opt["tile_bits"], adj_tile_bits=opt["adj_tile_bits"]) for c in circuits]
        obs = [Observable(c.n, o) for c, o in zip(circuits, observables)]
        M = Multi(plans, obs)
        st, ws = M.states(device), M.workspace(device)
        p = M.pack_params(params, device)
        w = torch.ones(M.nout, dtype=torch.float64, device=device)

        def step():
            M.apply(st, p, ws)
            M.expval(st, ws)
            M.adjoint_grad(st, p, w, ws)

        ms = _time_ms(step, reps, device)
        timings.append(dict(opt, ms=ms, batched=sum(M.batched)))
        if verbose:
            print("autotune_multi", opt, "%.3f ms" % ms, flush=True)
        if best is None or ms < best["ms"]:
            best = dict(opt, ms=ms)
        del M, plans, obs, st, ws
    result = {"tile_bits": best["tile_bits"], "adj_tile_bits": best["adj_tile_bits"], "ms": best["ms"],
              "tried": timings}
    cache[key] = result
    _store_cache(path, cache)
    return dict(result, cached=False)


def autotune(circuit, dtype, obs: Observable, params, data=None, batch: int = 1, grad: bool = True,
             reps: int = 2, cache_path: Optional[str] = None, device="cuda:0", verbose: bool = False,
             jit: bool = False) -> dict:
    """Pick the plan options (tile bits, dense-fusion width) with the lowest
    measured time of one forward (+ adjoint) step on this device; results are
    cached in a JSON file keyed by circuit structure, dtype, batch, the jit
    flag and GPU architecture (DQ_AUTOTUNE_CACHE, default
    ~/.cache/dq_autotune.json).  With jit the candidates are compiled passes
    (their compiles fall in the first, untimed call of each candidate)."""
    import os
    path = cache_path or os.environ.get("DQ_AUTOTUNE_CACHE", os.path.expanduser("~/.cache/dq_autotune.json"))
    p = _f64(params, device) if params is not None else None
    d = _f64(data, device) if data is not None else None
    per_sample = _stride(p) != 0 or _stride(d) != 0
    key = _structure_key(circuit, dtype, batch, per_sample, grad, _arch(device), jit=bool(jit))
    cache = _load_cache(path)
    if key in cache:
        return dict(cache[key], cached=True)
    gout = torch.ones((batch, obs.nobs), dtype=torch.float64, device=device)
    best, timings = None, []
    for opt in candidate_options(dtype, circuit.n, jit):
        plan = Plan(circuit, dtype, tile_bits=opt["tile_bits"], dense_fuse=opt["dense_fuse"], jit=opt["jit"])
        st = plan.state(batch, device)
        ws = plan.workspace(batch, per_sample, 1 if grad else 0, obs, device)

        def step():
            apply_circuit(plan, st, p, d, from_zero=True, ws=ws)
            expval(plan, obs, st, ws=ws)
            if grad:
                adjoint_grad(plan, obs, st, p, d, gout, ws=ws, want_data=False)

        ms = _time_ms(step, reps, device)
        timings.append(dict(opt, ms=ms))
        if verbose:
            print("autotune", opt, "%.3f ms" % ms, flush=True)
        if best is None or ms < best["ms"]:
            best = dict(opt, ms=ms)
        del plan, st, ws
    result = {"tile_bits": best["tile_bits"], "dense_fuse": best["dense_fuse"], "jit": best["jit"], "ms": best["ms"],
              "tried": timings}
    cache[key] = result
    _store_cache(path, cache)
    return dict(result, cached=False)
