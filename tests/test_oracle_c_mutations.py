"""Planted mistakes in the C oracle (on the CPU): a mutated copy of
oracle/lbm_oracle.c is compiled into a temporary library, loaded in place of
the real one for the duration of the test, and each plausible slip must make
at least one pin fail. The real oracle is untouched."""
import ctypes
import os
import shutil
import subprocess

import pytest

from oracle import oracle as O

import test_oracle_pins as P
from conftest import load_golden

SRC = os.path.join(os.path.dirname(O.__file__), "lbm_oracle.c")

MUTATIONS = {
    # opposite directions of two diagonals exchanged (bounce-back and the table)
    "opposites": ("static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};",
                  "static const int OPP[Q] = {0, 3, 4, 1, 2, 8, 7, 6, 5};"),
    # the drag halved twice over in the Brinkman velocity
    "drag": ("double denom = rho * (1.0 + p->eps * p->nu / (2.0 * kappa));",
             "double denom = rho * (1.0 + p->eps * p->nu / kappa);"),
    # a sign slip in the Shan-Chen shifted velocity
    "shift_sign": ("double uex = 2.0 * p->tau * ux + (1.0 - 2.0 * p->tau) * jx / rho;",
                   "double uex = 2.0 * p->tau * ux - (1.0 - 2.0 * p->tau) * jx / rho;"),
    # streaming in the wrong direction along x
    "stream_x": ("int xd = wrap(x + EX[a], nx);", "int xd = wrap(x - EX[a], nx);"),
    # bounce-back that forgets to reverse the population
    "bounce": ("fnew[c * Q + OPP[a]] = fs[a];", "fnew[c * Q + a] = fs[a];"),
    # the Guo forcing term with 1 - 1/tau instead of 1 - 1/(2 tau)
    "guo_factor": ("(1.0 - 1.0 / (2.0 * p->tau))", "(1.0 - 1.0 / p->tau)"),
    # kxy and kyx exchanged in the tensor velocity solve (K^T instead of K);
    # the third entry picks the occurrence when the text appears more than once
    "tensor_transpose": ("double kxx = perm[0], kxy = perm[1], kyx = perm[2], kyy = perm[3];",
                         "double kxx = perm[0], kxy = perm[2], kyx = perm[1], kyy = perm[3];", 0),
    # the same exchange in the Guo form's tensor drag force only
    "tensor_transpose_guo": ("double kxx = perm[0], kxy = perm[1], kyx = perm[2], kyy = perm[3];",
                             "double kxx = perm[0], kxy = perm[2], kyx = perm[1], kyy = perm[3];", 1),
    # the inverse tensor's off-diagonal signs dropped
    "tensor_inverse_sign": ("ixy = -kxy / det, iyx = -kyx / det, iyy = kxx / det; /* K^{-1} */",
                            "ixy = kxy / det, iyx = kyx / det, iyy = kxx / det; /* K^{-1} */"),
}


def _pins():
    """(name, callable) of the pins a mutation may break."""
    return [
        ("lattice", P.test_lattice_matches_d2q9_definition),
        ("transient", lambda: P.test_uniform_transient_closed_form(0.8, 0)),
        ("transient_guo", lambda: P.test_uniform_transient_closed_form(0.8, 1)),
        ("steady", lambda: P.test_uniform_steady_state_eq_f_steady(0.8)),
        ("guo_eq_sc", lambda: P.test_guo_form_equals_shan_chen_form(0.8, 1)),
        ("poiseuille", lambda: P.test_poiseuille_discrete_closed_form(0.8)),
        ("table1", lambda: P.test_table1_layered_perpendicular(load_golden)),
        ("table2", lambda: P.test_table2_layered_parallel(load_golden)),
        ("tensor_steady", lambda: P.test_uniform_nonsymmetric_tensor_steady_state(0.8, 0)),
        ("tensor_steady_guo", lambda: P.test_uniform_nonsymmetric_tensor_steady_state(0.8, 1)),
        ("tensor_guo_eq_sc", lambda: P.test_guo_form_equals_shan_chen_form_tensor(0.8)),
    ]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(tmp_path, monkeypatch, name):
    old, new, *which = MUTATIONS[name]
    src = open(SRC).read()
    if which:
        # replace the given occurrence of a text that appears more than once
        parts = src.split(old)
        assert len(parts) > which[0] + 1, name
        src = old.join(parts[:which[0] + 1]) + new + old.join(parts[which[0] + 1:])
    else:
        assert src.count(old) == 1, name
        src = src.replace(old, new)
    mutated = tmp_path / "lbm_oracle_mutated.c"
    mutated.write_text(src)
    lib = tmp_path / "liblbm_oracle_mutated.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", str(mutated), "-o",
                    str(lib), "-lm"], check=True)
    monkeypatch.setattr(O, "_LIB", str(lib))
    monkeypatch.setattr(O, "build", lambda force=False: str(lib))
    monkeypatch.setattr(O, "_lib", None)
    failed = []
    for pin, fn in _pins():
        try:
            fn()
        except AssertionError:
            failed.append(pin)
    assert failed, f"no pin caught the planted mistake {name!r}"
    print(name, "caught by", failed)
