"""The C ABI without a GPU: the library loads, exports every function that
include/dq.h declares, and rejects bad arguments on the host with the
documented status codes (no device work is reached by these calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dq.h")


def _built():
    from paper_2512_18995_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2512_18995_amd import build
        build.build()
    return _lib


@pytest.fixture(scope="module")
def L():
    return _built()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dq_[a-z_]+)\s*\(", text)))


def test_exports_every_header_function(L):
    names = header_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), "libdq.so does not export %s" % n
    assert sorted(L.EXPORTS) == names


def test_version(L):
    assert L.lib().dq_version() == 1


class G:
    def __init__(self, op, wires, src="none", idx=-1, scale=1.0, matrix=None):
        self.op, self.wires, self.src, self.idx, self.scale, self.matrix = op, tuple(wires), src, idx, scale, matrix


def _create(L, n, gates, nparams=0, ndata=0, dtype=0, opt=None):
    arr, keep = L.gate_array(gates)
    h = ctypes.c_void_p()
    st = L.lib().dq_plan_create(ctypes.byref(h), n, arr, len(gates), nparams, ndata, dtype,
                                ctypes.byref(opt) if opt is not None else None)
    return st, h


def test_unknown_op_and_expanded_gates(L):
    """Op codes beyond the last one are rejected; RXX and RYY are planned as
    basis changes around an RZZ (four more internal gates each), U3 as
    phase, RY, phase (three gates, one gradient slot per angle), and the
    controlled rotations as two half-angle rotations around two CNOT / CZ
    (four gates, two gradient slots)."""
    arr, keep = L.gate_array([G("h", (0,))])
    for bad in (19, -1, 32):
        arr[0].op = bad
        h = ctypes.c_void_p()
        assert L.lib().dq_plan_create(ctypes.byref(h), 3, arr, 1, 0, 0, 0, None) == 1
        assert "unknown op" in L.lib().dq_last_error().decode()
    st, h = _create(L, 3, [G("rxx", (0, 2), "param", 0), G("ryy", (1, 0), "param", 1)], 2, 0)
    assert st == 0
    s = L.DqPlanStats()
    assert L.lib().dq_plan_get_stats(h, ctypes.byref(s)) == 0
    assert s.ngates == 10
    L.lib().dq_plan_destroy(h)
    gates = [G("u3", (1,), "param", 0), G("crx", (0, 2), "param", 3), G("cry", (2, 1), "data", 0),
             G("crz", (1, 0), "param", 4), G("u3", (0,), "none", -1, 0.3)]
    st, h = _create(L, 3, gates, 5, 1)
    assert st == 0, L.lib().dq_last_error()
    assert L.lib().dq_plan_get_stats(h, ctypes.byref(s)) == 0
    assert s.ngates == 3 + 3 * 4 + 3
    assert s.grad_gates == 3 + 3 * 2          # the fixed U3 carries no gradient
    L.lib().dq_plan_destroy(h)



@pytest.mark.parametrize("n,gates,np_,nd,code", [
    (0, [], 0, 0, 4),                                         # nqubits out of range
    (35, [], 0, 0, 4),
    (3, [G("h", (3,))], 0, 0, 1),                             # wire out of range
    (3, [G("cnot", (1, 1))], 0, 0, 1),                        # repeated wire
    (3, [G("cnot", (1,))], 0, 0, 1),                          # wrong arity
    (3, [G("ry", (0,), "param", 5)], 2, 0, 1),                # param index out of range
    (3, [G("ry", (0,), "data", 0)], 2, 0, 1),                 # data index without data
    (3, [G("h", (0,), "param", 0)], 2, 0, 1),                 # angle on a fixed gate
    (3, [G("unitary", (0, 1))], 0, 0, 1),                     # unitary without matrix
    (3, [G("rxx", (0,), "param", 0)], 1, 0, 1),               # two-qubit rotation on one wire
    (3, [G("ryy", (2, 2), "param", 0)], 1, 0, 1),             # repeated wire
    (3, [G("u3", (0,), "param", 1)], 3, 0, 1),                # U3 reads idx..idx+2: 3 > 2
    (3, [G("u3", (0,), "data", 0)], 0, 2, 1),
    (3, [G("u3", (0, 1), "param", 0)], 3, 0, 1),              # U3 on two wires
    (3, [G("cry", (1,), "param", 0)], 1, 0, 1),               # controlled rotation on one wire
    (3, [G("crz", (0, 0), "param", 0)], 1, 0, 1),
    (3, [G("crx", (0, 1), "param", 1)], 1, 0, 1),
])
def test_plan_create_rejects(L, n, gates, np_, nd, code):
    st, h = _create(L, n, gates, np_, nd)
    assert st == code, (st, L.lib().dq_last_error())
    assert h.value is None
    assert L.lib().dq_last_error().decode() != ""


def test_plan_create_and_stats(L):
    gates = [G("ry", (q,), "param", q) for q in range(10)] + [G("cnot", (q, (q + 1) % 10)) for q in range(10)]
    st, h = _create(L, 10, gates, 10, 0)
    assert st == 0, L.lib().dq_last_error()
    assert L.lib().dq_last_error().decode() == ""
    s = L.DqPlanStats()
    assert L.lib().dq_plan_get_stats(h, ctypes.byref(s)) == 0
    assert s.nqubits == 10 and s.ngates == 20 and s.grad_gates == 10
    assert s.folded_gates == 10          # every leading RY folds into the first write
    assert s.tile_bits == 4              # n - 6 register bits at n = 10
    assert s.fwd_tile_passes == 1        # the whole register fits one wave tile
    sz = ctypes.c_size_t(0)
    assert L.lib().dq_workspace_size(h, None, 4, 1, 0, ctypes.byref(sz)) == 0 and sz.value > 0
    assert L.lib().dq_workspace_size(h, None, 4, 1, 1, ctypes.byref(sz)) == 1   # adjoint needs an observable
    assert L.lib().dq_workspace_size(h, None, 0, 0, 0, ctypes.byref(sz)) == 1   # batch >= 1
    L.lib().dq_plan_destroy(h)


def test_plain_path_has_one_step_per_gate(L):
    gates = [G("h", (q,)) for q in range(8)] + [G("cz", (0, 1)), G("rzz", (2, 5), "none", -1, 0.3)]
    st, h = _create(L, 8, gates, 0, 0, 0, L.DqOptions(0, 0, 1, 0))
    assert st == 0
    s = L.DqPlanStats()
    L.lib().dq_plan_get_stats(h, ctypes.byref(s))
    assert s.fwd_steps == 10 and s.fwd_tile_passes == 0 and s.folded_gates == 0
    L.lib().dq_plan_destroy(h)


def test_obs_create_validation(L):
    terms, off = L.pauli_arrays(3, [[(1.0, "XZX")], [(0.5, "ZZI"), (2.0, "IIY")]])
    h = ctypes.c_void_p()
    assert L.lib().dq_obs_create(ctypes.byref(h), 3, terms, off, 2) == 0
    L.lib().dq_obs_destroy(h)
    bad = (L.DqPauliTerm * 1)()
    bad[0].coef, bad[0].xmask, bad[0].zmask = 1.0, 1 << 3, 0          # wire 3 of a 3-qubit register
    off1 = (ctypes.c_int64 * 2)(0, 1)
    assert L.lib().dq_obs_create(ctypes.byref(h), 3, bad, off1, 1) == 1
    off_bad = (ctypes.c_int64 * 2)(1, 0)
    assert L.lib().dq_obs_create(ctypes.byref(h), 3, bad, off_bad, 1) == 1
    with pytest.raises(ValueError):
        L.pauli_arrays(3, [[(1.0, "XZ")]])


def test_calls_validate_before_device_work(L):
    gates = [G("ry", (q,), "param", q) for q in range(8)]
    st, h = _create(L, 8, gates, 8, 0)
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    # NULL state
    assert lib.dq_apply_circuit(h, None, 1, fake, 0, None, 0, 1, fake, 1 << 20, None) == 1
    # params missing
    assert lib.dq_apply_circuit(h, fake, 1, None, 0, None, 0, 1, fake, 1 << 20, None) == 1
    # params stride shorter than a row
    assert lib.dq_apply_circuit(h, fake, 2, fake, 3, None, 0, 1, fake, 1 << 20, None) == 1
    # workspace too small
    assert lib.dq_apply_circuit(h, fake, 1, fake, 0, None, 0, 1, fake, 16, None) == 3
    assert "workspace" in lib.dq_last_error().decode()
    # batch out of range
    assert lib.dq_apply_circuit(h, fake, 0, fake, 0, None, 0, 1, fake, 1 << 20, None) == 1
    assert lib.dq_apply_circuit(h, fake, 70000, fake, 0, None, 0, 1, fake, 1 << 40, None) == 4
    # observable for another register size
    terms, off = L.pauli_arrays(4, [[(1.0, "ZIII")]])
    o = ctypes.c_void_p()
    assert lib.dq_obs_create(ctypes.byref(o), 4, terms, off, 1) == 0
    assert lib.dq_expval(h, o, fake, 1, fake, fake, 1 << 20, None) == 1
    assert lib.dq_adjoint_grad(h, o, fake, 1, fake, 0, None, 0, fake, fake, None, 0, fake, 1 << 20, None) == 1
    lib.dq_obs_destroy(o)
    lib.dq_plan_destroy(h)


def test_probs_and_sample_validate_before_device_work(L):
    """Marginal probabilities and sampling reject bad arguments on the host
    with the documented codes, and report the workspace the reduction needs
    (one float64 partial per block of 4096 amplitudes per outcome)."""
    n = 14
    st, h = _create(L, n, [G("h", (q,)) for q in range(n)])
    assert st == 0
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced
    size = ctypes.c_size_t()
    for B, k in ((1, 1), (3, 4), (2, 12)):
        assert lib.dq_probs_workspace_size(h, B, k, ctypes.byref(size)) == 0
        blocks = -(-(1 << (n - k)) // 4096)
        assert size.value == -(-(B * (1 << k) * blocks * 8) // 256) * 256, (B, k, size.value)
    assert lib.dq_probs_workspace_size(h, 1, 0, ctypes.byref(size)) == 1
    assert lib.dq_probs_workspace_size(h, 1, 13, ctypes.byref(size)) == 1
    assert lib.dq_probs_workspace_size(h, 0, 2, ctypes.byref(size)) == 1
    assert lib.dq_probs_workspace_size(h, 70000, 2, ctypes.byref(size)) == 4

    def probs(wires, B=1, ws=1 << 30, state=fake, out=fake):
        w = (ctypes.c_int32 * max(len(wires), 1))(*wires)
        return lib.dq_probs(h, state, B, w, len(wires), out, fake, ws, None)
    assert probs([0, n]) == 1                    # wire beyond the register
    assert probs([-1]) == 1
    assert probs([3, 5, 3]) == 1                 # repeated wire
    assert "twice" in lib.dq_last_error().decode()
    assert probs([]) == 1
    assert probs(list(range(13))) == 1           # more than 12 wires
    assert probs([1, 2], state=None) == 1
    assert probs([1, 2], out=None) == 1
    assert probs([1, 2], ws=64) == 3             # workspace too small
    assert "workspace" in lib.dq_last_error().decode()
    # sampling
    assert lib.dq_sample(None, 1, 4, fake, 8, fake, None) == 1
    assert lib.dq_sample(fake, 1, 4, None, 8, fake, None) == 1
    assert lib.dq_sample(fake, 1, 4, fake, 8, None, None) == 1
    assert lib.dq_sample(fake, 1, 0, fake, 8, fake, None) == 1
    assert lib.dq_sample(fake, 1, (1 << 20) + 1, fake, 8, fake, None) == 1
    assert lib.dq_sample(fake, 1, 4, fake, -1, fake, None) == 1
    assert lib.dq_sample(fake, 0, 4, fake, 8, fake, None) == 4
    assert lib.dq_sample(fake, 1, 4, fake, 0, fake, None) == 0    # no shots: nothing to do
    lib.dq_plan_destroy(h)


def test_jit_option_validation_and_sources(L):
    """jit must be 0 or 1; a jit plan lists one kernel per distinct tile pass,
    and passes that repeat (equal operation lists) share a kernel."""
    from workloads import config
    st, h = _create(L, 8, [G("ry", (q,), "param", q) for q in range(8)], 8, 0, opt=L.DqOptions(1, 0, 1, 0, 2))
    assert st == 1 and "jit" in L.lib().dq_last_error().decode()
    import paper_2512_18995_amd as dq
    w = config(5, n=16, layers=8)
    plain = dq.Plan(w.circuit, "c64")
    assert plain.jit_sources() == []
    p = dq.Plan(w.circuit, "c64", jit=True)
    srcs = p.jit_sources()
    steps = [l for l in p.describe().splitlines() if " tile " in l]
    assert 0 < len(srcs) < len(steps)
    assert all('#include "tile_dev.h"' in s and "dq::op_s<" in s for s in srcs)
    assert any("dq::gen_s<" in s for s in srcs)   # adjoint passes accumulate gradient terms


def test_jit_helper_compiles_passes(L, tmp_path):
    """The helper program beside the library (one hipRTC compile per process,
    so that a plan's passes compile in parallel) turns a pass source into a
    gfx950 code object holding that kernel, and reports a broken source with
    a non-zero status and the compiler's message."""
    import subprocess
    import paper_2512_18995_amd as dq
    from workloads import config
    helper = os.path.join(os.path.dirname(L.LIB_PATH), "dq_jitc")
    assert os.access(helper, os.X_OK)
    w = config(5, n=12, layers=2)
    src = dq.Plan(w.circuit, "c64", jit=True).jit_sources()[-1]
    (tmp_path / "p.hip").write_text(src)
    r = subprocess.run([helper, "gfx950", str(tmp_path / "p.hip"), str(tmp_path / "p.co")], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    code = (tmp_path / "p.co").read_bytes()
    assert code[:4] == b"\x7fELF"
    name = re.search(r"void (dqj_[0-9a-f]{16})\(", src).group(1)
    assert name.encode() in code
    (tmp_path / "bad.hip").write_text(src.replace("dq::jit_", "dq::no_such_"))
    r = subprocess.run([helper, "gfx950", str(tmp_path / "bad.hip"), str(tmp_path / "bad.co")], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 1 and "no_such_" in r.stderr
    assert not (tmp_path / "bad.co").exists()


@pytest.mark.skipif(not os.path.exists("/opt/rocm/lib/libhiprtc.so"), reason="hipRTC not installed")
def test_jit_source_compiles_for_gfx950(L):
    """The generated pass kernels compile with hipRTC against tile_dev.h for
    gfx950 (host-side check; no device needed), and the packed FP32
    instructions stay disabled."""
    import subprocess
    import tempfile
    import paper_2512_18995_amd as dq
    from workloads import config
    rtc = ctypes.CDLL("/opt/rocm/lib/libhiprtc.so")
    hdr = open(os.path.join(os.path.dirname(L.LIB_PATH), "csrc", "tile_dev.h")).read().encode()
    w = config(5, n=12, layers=2)
    srcs = dq.Plan(w.circuit, "c64", jit=True).jit_sources()
    opts = [b"-O3", b"-std=c++17", b"-Xclang", b"-target-feature", b"-Xclang", b"-packed-fp32-ops",
            b"--offload-arch=gfx950"]
    for src in (srcs[0], srcs[-1]):   # a forward and an adjoint pass
        prog = ctypes.c_void_p()
        hs, hn = (ctypes.c_char_p * 1)(hdr), (ctypes.c_char_p * 1)(b"tile_dev.h")
        assert rtc.hiprtcCreateProgram(ctypes.byref(prog), src.encode(), b"pass.hip", 1, hs, hn) == 0
        r = rtc.hiprtcCompileProgram(prog, len(opts), (ctypes.c_char_p * len(opts))(*opts))
        n = ctypes.c_size_t()
        rtc.hiprtcGetProgramLogSize(prog, ctypes.byref(n))
        log = ctypes.create_string_buffer(n.value + 1)
        rtc.hiprtcGetProgramLog(prog, log)
        assert r == 0, log.value.decode()[:2000]
        rtc.hiprtcGetCodeSize(prog, ctypes.byref(n))
        code = ctypes.create_string_buffer(n.value)
        rtc.hiprtcGetCode(prog, code)
        rtc.hiprtcDestroyProgram(ctypes.byref(prog))
        name = re.search(r"void (dqj_[0-9a-f]{16})\(", src).group(1)
        with tempfile.NamedTemporaryFile(suffix=".co") as f:
            f.write(code.raw)
            f.flush()
            dis = subprocess.run(["/opt/rocm/llvm/bin/llvm-objdump", "-d", f.name], capture_output=True, text=True).stdout
        assert name in dis
        assert not re.search(r"v_pk_(add|mul|fma)_f32", dis)


_ALLOC_FAIL_SCRIPT = r"""
import ctypes, resource, sys
sys.path.insert(0, %r)
import numpy as np
from paper_2512_18995_amd import _lib
L = _lib.lib()
n = 4 << 20
arr = (_lib.DqGate * n)()
a = np.frombuffer(arr, dtype=np.int32).reshape(n, ctypes.sizeof(_lib.DqGate) // 4)
a[:, 1] = 1                                  # H on wire 0, no angle source
vm = [int(l.split()[1]) for l in open("/proc/self/status") if l.startswith("VmSize:")][0] * 1024
soft, hard = resource.getrlimit(resource.RLIMIT_AS)
resource.setrlimit(resource.RLIMIT_AS, (vm + (96 << 20), hard))
h = ctypes.c_void_p()
st = L.dq_plan_create(ctypes.byref(h), 4, arr, n, 0, 0, 0, None)
msg = L.dq_last_error().decode()
resource.setrlimit(resource.RLIMIT_AS, (soft, hard))
ok = ctypes.c_void_p()
st2 = L.dq_plan_create(ctypes.byref(ok), 4, arr, 8, 0, 0, 0, None)
print("|".join(map(str, (st, h.value is None, msg, st2))))
"""


def test_host_allocation_failure_returns_a_status(L, tmp_path):
    """A host allocation that fails inside an entry point (here the gate
    table of a 4M-gate plan under an address-space limit) comes back as
    DQ_ERR_INTERNAL with a message: no C++ exception crosses the C ABI,
    and the library stays usable afterwards."""
    import subprocess
    import sys
    script = tmp_path / "alloc_fail.py"
    script.write_text(_ALLOC_FAIL_SCRIPT % ROOT)
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    st, null_handle, msg, st2 = r.stdout.strip().splitlines()[-1].split("|")
    assert int(st) == 6 and null_handle == "True", r.stdout
    assert "allocation" in msg
    assert int(st2) == 0


def _tile_steps(plan):
    """(direction, R, compiled, operation count) of every register-tile step."""
    out = []
    for line in plan.describe().splitlines():
        if " tile " not in line:
            continue
        R = int(re.search(r" R=(\d+)", line).group(1))
        ops = line.split(" ops=")[1]
        out.append((line.split()[0], R, " kernel=" in line, len(ops.split(";")) if ops else 0))
    return out


def test_benchmark_plans_have_no_interpreted_wide_tiles():
    """Every plan the benchmark times (compiled passes): no register-tile
    step with 64 amplitudes per lane runs interpreted (that kernel does not
    exist: it kept its tile in scratch memory, and passes that fell back to
    it ran for minutes), and every compiled pass stays within the compile
    limit of 2048 operations x amplitudes per lane."""
    import paper_2512_18995_amd as dq
    import workloads as W
    plans = [(W.config(c).circuit, W.config(c).dtype) for c in (1, 2, 3, 5)]
    plans += [(W.qft(30), "c64"), (W.qft(32), "c64")]
    for circuit, dtype in plans:
        steps = _tile_steps(dq.Plan(circuit, dtype, jit=True))
        assert steps
        for d, R, compiled, nops in steps:
            assert compiled or R <= 5, (circuit.n, d, R)
            if compiled:
                assert nops << R <= 2048, (circuit.n, d, R, nops)


def test_streaming_kernels_keep_no_registers_in_scratch(L):
    """The build records the compiler's resource report of every kernel and
    fails if a kernel that streams the state (tiles, dense blocks, per-gate
    sweeps, init, expectations) keeps registers in scratch memory; the
    record holds every interpreted tile kernel the launchers can reach."""
    import json
    from paper_2512_18995_amd import build as B
    path = os.path.join(os.path.dirname(L.LIB_PATH), "_build", "kernel_resources.json")
    res = json.load(open(path))
    bases = {}
    for k, v in res.items():
        bases.setdefault(B.demangled_base(k), []).append(v)
        if B.demangled_base(k).startswith(B.NO_SCRATCH):
            assert v["scratch"] == 0, (k, v)
    # complex64 forward tiles 1..5, complex128 1..4; adjoint 1..4 and 1..3
    assert len(bases["k_tile_fwd"]) == 9 and len(bases["k_tile_adj"]) == 7, \
        (len(bases["k_tile_fwd"]), len(bases["k_tile_adj"]))
    assert len(bases["k_dense_f32"]) == 2 and len(bases["k_dense_f64"]) == 2


def test_interpreted_tiles_are_clamped_to_the_built_kernels():
    """Requested tile widths beyond the interpreted kernels that exist are
    clamped on the host: complex128 forward 4 register bits, adjoint 3;
    complex64 forward 5, adjoint 4."""
    import paper_2512_18995_amd as dq
    import workloads as W
    c = W.config(5, n=14, layers=2).circuit
    s = dq.Plan(c, "c128", tile_bits=5, adj_tile_bits=4).stats()
    assert (s["tile_bits"], s["adj_tile_bits"]) == (4, 3), s
    s = dq.Plan(c, "c64", tile_bits=5, adj_tile_bits=4).stats()
    assert (s["tile_bits"], s["adj_tile_bits"]) == (5, 4), s
    s = dq.Plan(c, "c64", tile_bits=6, jit=True).stats()      # compiled: the wide tiles stay
    assert (s["tile_bits"], s["adj_tile_bits"]) == (6, 5), s


def test_adjoint_passes_balanced_for_float64_arithmetic():
    """Compiled float64-arithmetic plans cap the operations per adjoint pass
    at the smallest value that adds no pass: the 32-qubit ring workload keeps
    121 adjoint passes with at most 18 operations each (greedy packing gave
    one pass per layer 21); float32 arithmetic keeps the greedy packing."""
    import paper_2512_18995_amd as dq
    import workloads as W
    c = W.config(5).circuit

    def adj_ops(plan):
        return [len(l.split(" ops=")[1].split(";")) for l in plan.describe().splitlines()
                if l.startswith("adj") and " tile " in l]
    a64 = dq.Plan(c, "c64", jit=True, arith64=True)
    ops = adj_ops(a64)
    assert len(ops) == 121 and max(ops) == 18, (len(ops), max(ops))
    ops = adj_ops(dq.Plan(c, "c64", jit=True))
    assert len(ops) == 100 and max(ops) == 26, (len(ops), max(ops))


def test_float64_arithmetic_forward_keeps_rz_out_of_ry_and_every_pass_compiled():
    """With float64 arithmetic the forward keeps diagonal one-qubit gates in
    slots of their own (RZ runs apart from RY), and the pass selection counts
    them as separate operations: random circuits of every gate kind still
    compile every pass (arith64 plans refuse interpreted ones), and the
    32-qubit ring workload keeps 101 forward passes with its 608 RY as real
    matrices and its 608 RZ as diagonals."""
    import paper_2512_18995_amd as dq
    import workloads as W
    ops = ("h", "x", "rx", "ry", "rz", "cnot", "cz", "swap", "cp", "rzz", "rxx", "u3", "cry", "crz", "unitary")
    for n in (7, 12, 16):
        for seed in range(4):
            rng = np.random.default_rng(640 + n + 1000 * seed)
            c = W.random_circuit(rng, n, 8 * n, ops=ops, with_data=True, max_unitary_k=1)
            dq.Plan(c, "c64", jit=True, arith64=True)
    s = dq.Plan(W.config(5).circuit, "c64", jit=True, arith64=True).stats()
    assert s["fwd_tile_passes"] == 101, s
    assert s["fwd_ops_reg"].get("1q_diag") == 608 and "1q" not in s["fwd_ops_reg"], s["fwd_ops_reg"]
    assert s["fwd_ops_lane"].get("1q_real", 0) + s["fwd_ops_reg"].get("1q_real", 0) == 608, s
    s32 = dq.Plan(W.config(5).circuit, "c64", jit=True).stats()
    assert "1q_diag" not in s32["fwd_ops_reg"] and s32["fwd_ops_reg"].get("1q", 0) > 0, s32["fwd_ops_reg"]


def test_multi_plan_runs_unbatched_shapes_on_the_single_plan_path():
    """Circuits whose common tile shape has no multi-circuit kernel (an
    8-qubit first circuit gives 2 register bits; compiled plans use 6) are
    not batched: they take the single-plan path instead of failing at launch."""
    import paper_2512_18995_amd as dq
    import workloads as W
    a, b = W.config(5, n=8, layers=2), W.config(5, n=12, layers=2)
    obs = [dq.Observable(w.circuit.n, w.observables) for w in (a, b)]
    m = dq.Multi([dq.Plan(a.circuit, "c64"), dq.Plan(b.circuit, "c64")], obs)
    assert m.batched == [False, False]
    m = dq.Multi([dq.Plan(b.circuit, "c64", jit=True), dq.Plan(b.circuit, "c64", jit=True)], [obs[1], obs[1]])
    assert m.batched == [False, False]
    m = dq.Multi([dq.Plan(b.circuit, "c64"), dq.Plan(b.circuit, "c64")], [obs[1], obs[1]])
    assert m.batched == [True, True]


def test_hessian_validates_before_device_work(L):
    """dq_hessian rejects bad arguments on the host: NULL pointers, a plan
    without parameters, a negative or too large max_shifts, a short
    workspace; the workspace query builds the derived plan on the host."""
    lib = L.lib()
    vp = ctypes.c_void_p
    terms, off = L.pauli_arrays(3, [[(1.0, "ZZI")]])
    obs = vp()
    assert lib.dq_obs_create(ctypes.byref(obs), 3, terms, off, 1) == 0
    gates = [G("u3", (0,), "param", 0), G("cry", (0, 1), "param", 3), G("ry", (2,), "data", 0)]
    st, h = _create(L, 3, gates, 4, 1)
    assert st == 0, lib.dq_last_error()
    sz = ctypes.c_size_t(0)
    assert lib.dq_hessian_workspace_size(h, obs, 0, ctypes.byref(sz)) == 0 and sz.value > 0
    full = sz.value
    assert lib.dq_hessian_workspace_size(h, obs, 2, ctypes.byref(sz)) == 0 and 0 < sz.value < full
    assert lib.dq_hessian_workspace_size(h, obs, -1, ctypes.byref(sz)) == 1
    fake = vp(256)   # never dereferenced: every call below fails validation first
    assert lib.dq_hessian(h, obs, fake, fake, None, fake, 0, fake, full, None) == 1        # weights NULL
    assert lib.dq_hessian(h, obs, None, fake, fake, fake, 0, fake, full, None) == 1        # params NULL
    assert lib.dq_hessian(h, obs, fake, None, fake, fake, 0, fake, full, None) == 1        # data NULL
    assert lib.dq_hessian(h, obs, fake, fake, fake, fake, -2, fake, full, None) == 1       # max_shifts < 0
    assert lib.dq_hessian(h, obs, fake, fake, fake, fake, 0, fake, full - 1, None) == 3    # workspace short
    assert lib.dq_hessian(h, obs, fake, fake, fake, fake, 0, None, full, None) == 3
    L.lib().dq_plan_destroy(h)
    st, h = _create(L, 3, [G("h", (0,))], 0, 0)
    assert lib.dq_hessian(h, obs, fake, None, fake, fake, 0, fake, full, None) == 1        # no parameters
    assert "no parameters" in lib.dq_last_error().decode()
    L.lib().dq_plan_destroy(h)
    lib.dq_obs_destroy(obs)


def test_noalloc_apply_validates_on_the_host(L):
    """dq_apply_circuit_noalloc: bad arguments and matrix blocks beyond the
    16 MiB scratch are rejected before any device call."""
    lib = L.lib()
    gates = [G("u3", (q % 8,), "param", 3 * q) for q in range(600)]
    st, h = _create(L, 8, gates, 1800, 0, dtype=1)
    assert st == 0, lib.dq_last_error()
    fake = ctypes.c_void_p(256)   # never dereferenced
    assert lib.dq_apply_circuit_noalloc(h, None, 1, fake, 0, None, 0, 1, None) == 1
    assert lib.dq_apply_circuit_noalloc(h, fake, 0, fake, 0, None, 0, 1, None) == 1
    assert lib.dq_apply_circuit_noalloc(h, fake, 256, fake, 1800, None, 0, 1, None) == 4
    assert "scratch" in lib.dq_last_error().decode()
    lib.dq_plan_destroy(h)


def test_arith64_option_validation(L):
    """Float64 arithmetic on complex64 states: only for compiled, fused
    complex64 plans without dense blocks; its tiles hold one register bit
    less than complex64 arithmetic (as complex128 tiles do)."""
    gates = [G("ry", (q,), "param", q) for q in range(20)] + [G("cnot", (q, (q + 1) % 20)) for q in range(20)]

    def opt(**kw):
        o = L.DqOptions(1, 0, 1, 0, 1, 0, 0, 0, 1)
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    for bad, code in ((dict(jit=0), 2), (dict(fusion=0), 2), (dict(dense_fuse=4), 2), (dict(arith64=2), 1)):
        st, h = _create(L, 20, gates, 20, 0, opt=opt(**bad))
        assert st == code, (bad, st, L.lib().dq_last_error())
    st, h = _create(L, 20, gates, 20, 0, dtype=1, opt=opt())
    assert st == 2
    # dense unitaries of two or more wires run as per-gate sweeps: not in arith64 plans
    U = np.eye(4, dtype=np.complex128)
    st, h = _create(L, 20, gates + [G("unitary", (3, 11), matrix=U)], 20, 0, opt=opt())
    assert st == 2 and "compiled tile pass" in L.lib().dq_last_error().decode()
    st, h = _create(L, 20, gates, 20, 0, opt=opt())
    assert st == 0, L.lib().dq_last_error()
    s = L.DqPlanStats()
    assert L.lib().dq_plan_get_stats(h, ctypes.byref(s)) == 0
    assert (s.tile_bits, s.adj_tile_bits) == (5, 4)
    L.lib().dq_plan_destroy(h)
    st, h = _create(L, 20, gates, 20, 0, opt=opt(arith64=0))
    assert L.lib().dq_plan_get_stats(h, ctypes.byref(s)) == 0
    assert (s.tile_bits, s.adj_tile_bits) == (6, 5)
    L.lib().dq_plan_destroy(h)
