"""Mutation check of the oracle's pins: plant plausible mistakes in a copy of
the oracle's C source (on the CPU, in a temporary directory), rebuild it, and
check that the LAPACK pin rejects every mutant while accepting the original.
This shows that the pins can see a dropped term, a wrong sign, a wrong index
or a transposed operand."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import random_dd

SRC = os.path.join(os.path.dirname(oracle.__file__), "pent_oracle.c")

MUTANTS = {
    "forward_sign_eps": ("(row[j] - eps * g2 - bet * g1)", "(row[j] + eps * g2 - bet * g1)"),
    "forward_drop_beta": ("(row[j] - eps * g2 - bet * g1)", "(row[j] - eps * g2)"),
    "backward_index": ("row[j] - gam * x1 - del * x2", "row[j] - gam * x2 - del * x1"),
    "factor_beta_index": ("beta[i] = bi - ai * gam2;", "beta[i] = bi - ai * gam1;"),
    "factor_gamma_index": ("(di - beta[i] * del1)", "(di - beta[i] * del2)"),
    "factor_transposed": ("double bi = (i >= 1) ? b[i] : 0.0;", "double bi = (i >= 1) ? d[i - 1] : 0.0;"),
    "factor_delta_nodiv": ("delta[i] = ei / alpha[i];", "delta[i] = ei;"),
    "forward_mul_alpha": ("- bet * g1) / alpha[i];", "- bet * g1) * alpha[i];"),
    "alpha_drop_term": ("alpha[i] = c[i] - ai * del2 - beta[i] * gam1;",
                        "alpha[i] = c[i] - beta[i] * gam1;"),
}


def _build(tmp_path, name, src):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c), "-lm"])
    lib = ctypes.CDLL(str(so))
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.orc_factor.argtypes = [I64, P, P, P, P, P, P, P, P, P, ctypes.POINTER(I64)]
    lib.orc_solve.argtypes = [I64, P, P, P, P, P, P, I64, I64]
    return lib


def _pin_passes(lib):
    """The dense-LAPACK pin of test_oracle_pins, run against ``lib``."""
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    for n in (5, 17, 32):
        dg = random_dd(n, seed=100 + n)
        fac = [np.zeros(n) for _ in range(4)]
        bad = ctypes.c_int64(-1)
        if lib.orc_factor(n, *[p(np.ascontiguousarray(v)) for v in dg], *[p(v) for v in fac],
                          ctypes.byref(bad)) != 0:
            return False
        F = np.random.Generator(np.random.PCG64(7 + n)).uniform(-1, 1, (n, 5))
        X = F.copy()
        lib.orc_solve(n, p(np.ascontiguousarray(dg.a)), *[p(v) for v in fac], p(X), 5, 5)
        ref = np.linalg.solve(oracle.dense(dg), F)
        kappa = np.linalg.cond(oracle.dense(dg), 1)
        if not np.max(np.abs(X - ref)) <= 64 * 1.1e-16 * kappa * np.max(np.abs(ref)):
            return False
    return True


def test_original_passes(tmp_path):
    assert _pin_passes(_build(tmp_path, "orig", open(SRC).read()))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    assert not _pin_passes(_build(tmp_path, name, src.replace(old, new)))
