"""dq: an MI355X (gfx950) state-vector engine for batched parameterised
qubit circuits -- gate application, Pauli-sum expectations and adjoint
gradients -- after the qubit simulator of DeepQuantum (arXiv 2512.18995,
sections 4 and 7).

The compute path is the HIP library ``libdq.so`` (C ABI in include/dq.h);
this package only marshals arguments.  There is no CPU fallback: importing
the engine without a built library raises.
"""
from ._lib import DqError, LIB_PATH, lib  # noqa: F401

__all__ = ["DqError", "LIB_PATH", "lib", "Plan", "Observable", "state_init", "apply_circuit", "expval", "autotune",
           "adjoint_grad", "expectation", "ExpvalFunction", "Multi", "probs", "sample", "hessian",
           "apply_circuit_noalloc", "autotune_multi", "candidate_options",
           "multi_candidates"]


def __getattr__(name):
    # torch-facing API loaded on first use (keeps `import paper_2512_18995_amd` cheap)
    if name in __all__:
        from . import engine
        return getattr(engine, name)
    raise AttributeError(name)
