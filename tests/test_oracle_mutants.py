"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch every one of them: a dropped term, a wrong sign, a
wrong index or bit order, a transposed operand."""
import os
import shutil
import subprocess
import sys

import pytest

import oracle
import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "dq_oracle.c")

# the controlled rotations' matrix: identity block, then the rotation block
CR_BLOCK = """        U[0 * 4 + 0] = 1.0;
        U[1 * 4 + 1] = 1.0;
        U[2 * 4 + 2] = R[0] + I * R[1];
        U[2 * 4 + 3] = R[2] + I * R[3];
        U[3 * 4 + 2] = R[4] + I * R[5];
        U[3 * 4 + 3] = R[6] + I * R[7];"""

# (name, exact text in dq_oracle.c, replacement)
MUTANTS = [
    ("ry-sign", "U[0] = c; U[1] = -s; U[2] = s; U[3] = c;", "U[0] = c; U[1] = s; U[2] = -s; U[3] = c;"),
    ("rx-sign", "U[0] = c; U[1] = -I * s; U[2] = -I * s;", "U[0] = c; U[1] = I * s; U[2] = I * s;"),
    ("rz-sign", "U[0] = cexp(-I * theta / 2.0); U[3] = cexp(I * theta / 2.0);",
     "U[0] = cexp(I * theta / 2.0); U[3] = cexp(-I * theta / 2.0);"),
    ("full-angle", "double c = cos(theta / 2.0), s = sin(theta / 2.0);", "double c = cos(theta), s = sin(theta);"),
    ("y-sign", "k = 1; U[1] = -I; U[2] = I;", "k = 1; U[1] = I; U[2] = -I;"),
    ("h-sign", "U[2] = 1.0 / sqrt(2.0); U[3] = -1.0 / sqrt(2.0);", "U[2] = -1.0 / sqrt(2.0); U[3] = 1.0 / sqrt(2.0);"),
    ("cnot-swapped-roles", "U[0 * 4 + 0] = 1.0; U[1 * 4 + 1] = 1.0; U[2 * 4 + 3] = 1.0; U[3 * 4 + 2] = 1.0;",
     "U[0 * 4 + 0] = 1.0; U[1 * 4 + 3] = 1.0; U[2 * 4 + 2] = 1.0; U[3 * 4 + 1] = 1.0;"),
    ("cz-wrong-corner", "U[0] = 1.0; U[5] = 1.0; U[10] = 1.0; U[15] = -1.0;",
     "U[0] = -1.0; U[5] = 1.0; U[10] = 1.0; U[15] = 1.0;"),
    ("cp-conj", "U[15] = cexp(I * theta);", "U[15] = cexp(-I * theta);"),
    ("rzz-sign", "U[10] = cexp(I * theta / 2.0); U[15] = cexp(-I * theta / 2.0);",
     "U[10] = cexp(-I * theta / 2.0); U[15] = cexp(I * theta / 2.0);"),
    ("lsb-wire0", ["target_mask |= 1LL << (n - 1 - wires[t]);", "off[a] += 1LL << (n - 1 - wires[t]);"],
     ["target_mask |= 1LL << wires[t];", "off[a] += 1LL << wires[t];"]),
    ("matrix-transposed", "acc += U[r * dim + c] * in[c];", "acc += U[c * dim + r] * in[c];"),
    ("subindex-order", "if ((a >> (k - 1 - t)) & 1)", "if ((a >> t) & 1)"),
    ("dropped-conj", "acc += conj(psi[j]) * phi[j];", "acc += psi[j] * phi[j];"),
    ("prob-wrong-half", "if (!(j & bit))", "if (j & bit)"),
    ("rxx-sign", "U[0 * 4 + 3] = -I * s; U[1 * 4 + 2] = -I * s; U[2 * 4 + 1] = -I * s; U[3 * 4 + 0] = -I * s;",
     "U[0 * 4 + 3] = I * s; U[1 * 4 + 2] = I * s; U[2 * 4 + 1] = I * s; U[3 * 4 + 0] = I * s;"),
    ("ryy-as-rxx", "U[0 * 4 + 3] = I * s; U[1 * 4 + 2] = -I * s; U[2 * 4 + 1] = -I * s; U[3 * 4 + 0] = I * s;",
     "U[0 * 4 + 3] = -I * s; U[1 * 4 + 2] = -I * s; U[2 * 4 + 1] = -I * s; U[3 * 4 + 0] = -I * s;"),
    ("u3-phi-lambda-swapped", ["U[1] = -cexp(I * lambda) * sh;", "U[2] = cexp(I * phi) * sh;"],
     ["U[1] = -cexp(I * phi) * sh;", "U[2] = cexp(I * lambda) * sh;"]),
    ("u3-dropped-phase", "U[3] = cexp(I * (phi + lambda)) * ch;", "U[3] = ch;"),
    ("u3-half-angle-dropped", "double ch = cos(theta / 2.0);", "double ch = cos(theta);"),
    ("cr-block-transposed", ["U[2 * 4 + 3] = R[2] + I * R[3];", "U[3 * 4 + 2] = R[4] + I * R[5];"],
     ["U[2 * 4 + 3] = R[4] + I * R[5];", "U[3 * 4 + 2] = R[2] + I * R[3];"]),
    ("crx-as-cry", "op == ORC_CRX ? ORC_RX", "op == ORC_CRX ? ORC_RY"),
    ("cr-control-on-zero", CR_BLOCK, CR_BLOCK.replace("U[0 * 4 + 0] = 1.0;", "U[3 * 4 + 3] = 1.0;")
     .replace("U[1 * 4 + 1] = 1.0;", "U[2 * 4 + 2] = 1.0;").replace("U[2 * 4 + 2] = R", "U[0 * 4 + 0] = R")
     .replace("U[2 * 4 + 3] = R", "U[0 * 4 + 1] = R").replace("U[3 * 4 + 2] = R", "U[1 * 4 + 0] = R")
     .replace("U[3 * 4 + 3] = R", "U[1 * 4 + 1] = R")),
]


def _build(tmp_path, name, old, new):
    text = open(SRC).read()
    olds, news = (old, new) if isinstance(old, list) else ([old], [new])
    for o, nw in zip(olds, news):
        assert text.count(o) == 1, "mutant %s: anchor text not found once" % name
        text = text.replace(o, nw)
    src = tmp_path / ("m_%s.c" % name)
    src.write_text(text)
    so = tmp_path / ("m_%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", str(so), str(src), "-lm"])
    return str(so)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    so = _build(tmp_path, name, old, new)
    tests_dir = os.path.dirname(os.path.abspath(__file__))
    r = subprocess.run([sys.executable, "-c", _RUNNER, so], cwd=tests_dir, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    caught = [l for l in r.stdout.splitlines() if l.startswith("CAUGHT")]
    assert caught, "planted mistake %r passed every pin" % name


_RUNNER = """
import ctypes, os, sys
sys.path.insert(0, os.path.dirname(os.getcwd()))
sys.path.insert(0, os.getcwd())
import oracle, oracle_pins
real = oracle.lib()
L = ctypes.CDLL(sys.argv[1])
for fn in ("orc_gate_matrix", "orc_u3_matrix", "orc_apply", "orc_run", "orc_pauli_expval", "orc_prob_zero"):
    getattr(L, fn).argtypes = getattr(real, fn).argtypes
    getattr(L, fn).restype = getattr(real, fn).restype
oracle._lib = L
for pin in oracle_pins.ALL_PINS:
    try:
        pin()
    except Exception as e:
        print("CAUGHT", pin.__name__, str(e)[:100].replace(chr(10), " "))
"""


# Planted mistakes in the numpy part of the oracle (marginals and sampling):
# (name, function, exact text in its source, replacement, pins that must fail)
PY_MUTANTS = [
    ("probs-lsb-wire0", "probs", "((j >> (n - 1 - w)) & 1)", "((j >> w) & 1)", ["pin_marginal_distribution"]),
    ("probs-order-reversed", "probs", "for w in wires:", "for w in list(wires)[::-1]:",
     ["pin_marginal_distribution"]),
    ("probs-amplitude-not-squared", "probs", "np.abs(np.asarray(psi, dtype=np.complex128)) ** 2",
     "np.abs(np.asarray(psi, dtype=np.complex128))", ["pin_marginal_distribution"]),
    ("sample-le", "sample", "if x < c:", "if x <= c:", ["pin_sampling"]),
    ("sample-no-fallback", "sample", "out.append(res if res >= 0 else (last if last >= 0 else 0))",
     "out.append(res if res >= 0 else 0)", ["pin_sampling"]),
    ("four-term-sign", "grad_param_shift", "return _D_PLUS * a - _D_MINUS * c", "return _D_PLUS * a + _D_MINUS * c",
     ["pin_four_term_shift_equals_fd"]),
    ("four-term-as-two-term", "grad_param_shift", "if circuit.gates[i].op in FOUR_TERM_GATES:",
     "if False:", ["pin_four_term_shift_equals_fd"]),
    ("u3-angle-not-chained", "grad_param_shift", "gp[g.idx + k] += g.scale * v", "gp[g.idx] += g.scale * v",
     ["pin_four_term_shift_equals_fd"]),
    ("hessian-no-mirror", "hessian_param_shift", "        if a != b:", "        if False:",
     ["pin_hessian_closed_forms", "pin_hessian_equals_fd_of_gradient"]),
    ("hessian-diagonal-mirrored", "hessian_param_shift", "        if a != b:", "        if True:",
     ["pin_hessian_closed_forms", "pin_hessian_equals_fd_of_gradient"]),
    ("hessian-one-scale", "hessian_param_shift", "f = ga.scale * gb.scale * v", "f = ga.scale * v",
     ["pin_hessian_closed_forms", "pin_hessian_equals_fd_of_gradient"]),
    ("hessian-second-shift-dropped", "hessian_param_shift", "th[ib, kb] += sj", "pass",
     ["pin_hessian_closed_forms", "pin_hessian_equals_fd_of_gradient"]),
    ("hessian-u3-angle-index", "hessian_param_shift", "pa, pb = ga.idx + occ[a][1], gb.idx + occ[b][1]",
     "pa, pb = ga.idx, gb.idx", ["pin_hessian_closed_forms", "pin_hessian_equals_fd_of_gradient"]),
]


@pytest.mark.parametrize("name,func,old,new,pins", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_python_mutant_is_caught(monkeypatch, name, func, old, new, pins):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(getattr(oracle, func)))
    assert src.count(old) == 1, "mutant %s: anchor text not found once" % name
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), "<mutant %s>" % name, "exec"), ns)
    monkeypatch.setattr(oracle, func, ns[func])
    for pin in pins:
        with pytest.raises(AssertionError):
            getattr(oracle_pins, pin)()
