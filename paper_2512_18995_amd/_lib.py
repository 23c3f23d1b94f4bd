"""ctypes binding of libdq.so (include/dq.h): argument marshalling only.

Every computation runs in the HIP library; this module converts gate lists
and Pauli sums into the C structs and passes device pointers and the
current HIP stream.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdq.so")

OPS = {"h": 0, "x": 1, "y": 2, "z": 3, "rx": 4, "ry": 5, "rz": 6, "cnot": 7, "cz": 8, "swap": 9,
       "cp": 10, "rzz": 11, "unitary": 12, "rxx": 13, "ryy": 14, "u3": 15, "crx": 16, "cry": 17,
       "crz": 18}
SRC = {"none": 0, "param": 1, "data": 2}
STATUS = {0: "DQ_OK", 1: "DQ_ERR_INVALID_ARG", 2: "DQ_ERR_UNSUPPORTED", 3: "DQ_ERR_WORKSPACE",
          4: "DQ_ERR_OUT_OF_RANGE", 5: "DQ_ERR_HIP", 6: "DQ_ERR_INTERNAL"}
C64, C128 = 0, 1

EXPORTS = ["dq_plan_create", "dq_plan_destroy", "dq_plan_get_stats", "dq_obs_create", "dq_obs_destroy",
           "dq_workspace_size", "dq_state_init", "dq_apply_circuit", "dq_expval", "dq_adjoint_grad",
           "dq_last_error", "dq_version", "dq_profile_enable", "dq_profile_read",
           "dq_multi_create", "dq_multi_destroy", "dq_multi_layout", "dq_multi_workspace_size", "dq_multi_apply",
           "dq_multi_expval", "dq_multi_adjoint_grad", "dq_multi_batched", "dq_plan_describe",
           "dq_plan_jit_source", "dq_probs_workspace_size", "dq_probs", "dq_sample",
           "dq_hessian_workspace_size", "dq_hessian", "dq_apply_circuit_noalloc"]
PROF_KINDS = ["fwd_tile", "adj_tile", "gate", "grad_gate", "expval", "lambda", "init", "other", "dense"]


class DqGate(ctypes.Structure):
    _fields_ = [("op", c_int32), ("nq", c_int32), ("wires", c_int32 * 5), ("src", c_int32),
                ("idx", c_int64), ("scale", c_double), ("matrix", POINTER(c_double))]


class DqPauliTerm(ctypes.Structure):
    _fields_ = [("coef", c_double), ("xmask", c_uint64), ("zmask", c_uint64)]


class DqOptions(ctypes.Structure):
    _fields_ = [("fusion", c_int32), ("tile_bits", c_int32), ("fold_init", c_int32), ("dense_fuse", c_int32),
                ("jit", c_int32), ("adj_tile_bits", c_int32), ("low_bits", c_int32), ("layout", c_int32),
                ("arith64", c_int32)]


class DqPlanStats(ctypes.Structure):  # noqa: E302
    _fields_ = [("nqubits", c_int32), ("dtype", c_int32), ("ngates", c_int64), ("fwd_steps", c_int64),
                ("fwd_tile_passes", c_int64), ("fwd_dense_blocks", c_int64), ("adj_steps", c_int64),
                ("folded_gates", c_int64), ("grad_gates", c_int64), ("tile_bits", c_int32), ("adj_tile_bits", c_int32), ("layout_swaps", c_int32), ("pad", c_int32),
                ("tile_ops", ((c_int64 * 8) * 2) * 2)]


class DqProfile(ctypes.Structure):
    _fields_ = [("launches", c_int64 * 9), ("ms", c_double * 9), ("bytes", c_double * 9), ("flops", c_double * 9)]


class DqError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s: %s (%s)" % (where, msg, STATUS.get(status, status)))
        self.status = status


_lib = None


def lib():
    """Load libdq.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdq.so not built: run python -m paper_2512_18995_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp = c_void_p
        L.dq_plan_create.argtypes = [POINTER(vp), c_int32, POINTER(DqGate), c_int64, c_int64, c_int64, c_int32,
                                     POINTER(DqOptions)]
        L.dq_plan_destroy.argtypes = [vp]
        L.dq_plan_destroy.restype = None
        L.dq_plan_get_stats.argtypes = [vp, POINTER(DqPlanStats)]
        L.dq_obs_create.argtypes = [POINTER(vp), c_int32, POINTER(DqPauliTerm), POINTER(c_int64), c_int32]
        L.dq_obs_destroy.argtypes = [vp]
        L.dq_obs_destroy.restype = None
        L.dq_workspace_size.argtypes = [vp, vp, c_int64, c_int32, c_int32, POINTER(c_size_t)]
        L.dq_state_init.argtypes = [vp, vp, c_int64, vp, vp]
        L.dq_apply_circuit.argtypes = [vp, vp, c_int64, vp, c_int64, vp, c_int64, c_int32, vp, c_size_t, vp]
        L.dq_expval.argtypes = [vp, vp, vp, c_int64, vp, vp, c_size_t, vp]
        L.dq_adjoint_grad.argtypes = [vp, vp, vp, c_int64, vp, c_int64, vp, c_int64, vp, vp, vp, c_int32, vp,
                                      c_size_t, vp]
        L.dq_profile_enable.argtypes = [vp, c_int32]
        L.dq_profile_read.argtypes = [vp, POINTER(DqProfile), c_int32]
        L.dq_multi_create.argtypes = [POINTER(vp), POINTER(vp), POINTER(vp), c_int32]
        L.dq_multi_destroy.argtypes = [vp]
        L.dq_multi_destroy.restype = None
        i64p = POINTER(c_int64)
        L.dq_multi_layout.argtypes = [vp, i64p, i64p, i64p, i64p, i64p, i64p]
        L.dq_multi_workspace_size.argtypes = [vp, POINTER(c_size_t)]
        L.dq_multi_batched.argtypes = [vp, POINTER(c_int32), POINTER(c_int32)]
        L.dq_plan_describe.argtypes = [vp, c_char_p, c_size_t, POINTER(c_size_t)]
        L.dq_plan_jit_source.argtypes = [vp, c_int32, c_char_p, c_size_t, POINTER(c_size_t), POINTER(c_int32)]
        L.dq_multi_apply.argtypes = [vp, vp, vp, vp, c_size_t, vp]
        L.dq_multi_expval.argtypes = [vp, vp, vp, vp, c_size_t, vp]
        L.dq_multi_adjoint_grad.argtypes = [vp, vp, vp, vp, vp, vp, c_size_t, vp]
        L.dq_probs_workspace_size.argtypes = [vp, c_int64, c_int32, POINTER(c_size_t)]
        L.dq_probs.argtypes = [vp, vp, c_int64, POINTER(c_int32), c_int32, vp, vp, c_size_t, vp]
        L.dq_sample.argtypes = [vp, c_int64, c_int32, vp, c_int32, vp, vp]
        L.dq_hessian_workspace_size.argtypes = [vp, vp, c_int32, POINTER(c_size_t)]
        L.dq_hessian.argtypes = [vp, vp, vp, vp, vp, vp, c_int32, vp, c_size_t, vp]
        L.dq_apply_circuit_noalloc.argtypes = [vp, vp, c_int64, vp, c_int64, vp, c_int64, c_int32, vp]
        L.dq_last_error.restype = c_char_p
        L.dq_version.restype = c_int32
        for f in ("dq_plan_create", "dq_plan_get_stats", "dq_obs_create", "dq_workspace_size", "dq_state_init",
                  "dq_apply_circuit", "dq_expval", "dq_adjoint_grad", "dq_profile_enable", "dq_profile_read",
                  "dq_multi_create", "dq_multi_layout", "dq_multi_workspace_size", "dq_multi_apply",
                  "dq_multi_expval", "dq_multi_adjoint_grad", "dq_multi_batched", "dq_plan_describe", "dq_plan_jit_source",
                  "dq_probs_workspace_size", "dq_probs", "dq_sample", "dq_hessian_workspace_size", "dq_hessian",
                  "dq_apply_circuit_noalloc"):
            getattr(L, f).restype = c_int32
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != 0:
        raise DqError(status, where, lib().dq_last_error().decode())


def gate_array(gates):
    """Gate-like objects (op, wires, src, idx, scale, matrix) -> (DqGate[], keepalive)."""
    arr = (DqGate * max(len(gates), 1))()
    keep = []
    for i, g in enumerate(gates):
        G = arr[i]
        G.op = OPS[g.op]
        G.nq = len(g.wires)
        for k, w in enumerate(g.wires):
            G.wires[k] = int(w)
        G.src = SRC[g.src]
        G.idx = int(g.idx)
        G.scale = float(g.scale)
        if g.op == "unitary" and g.matrix is not None:
            import numpy as np
            m = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128)).view(np.float64).ravel()
            keep.append(m)
            G.matrix = m.ctypes.data_as(POINTER(c_double))
    return arr, keep


def pauli_arrays(n: int, observables):
    """[[(coef, letters), ...], ...] -> (DqPauliTerm[], int64 offsets[nobs+1])."""
    terms = []
    offs = [0]
    for obs in observables:
        for coef, letters in obs:
            if len(letters) != n:
                raise ValueError("Pauli string %r is not of length %d" % (letters, n))
            x = z = 0
            for w, l in enumerate(letters):
                if l in "XY":
                    x |= 1 << w
                if l in "ZY":
                    z |= 1 << w
                if l not in "IXYZ":
                    raise ValueError("bad Pauli letter %r" % l)
            terms.append((float(coef), x, z))
        offs.append(len(terms))
    arr = (DqPauliTerm * max(len(terms), 1))()
    for i, (c, x, z) in enumerate(terms):
        arr[i].coef, arr[i].xmask, arr[i].zmask = c, x, z
    off = (c_int64 * len(offs))(*offs)
    return arr, off
