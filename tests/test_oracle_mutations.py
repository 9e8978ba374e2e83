"""Mistakes planted in a copy of the oracle (on the CPU) must trip the pins.

Each mutation is a plausible slip (dropped term, wrong sign, wrong operand,
transposed role of C and Ct).  The mutated copy is built from the oracle's
own source text in a private namespace; the real module is untouched.
"""
import inspect
import json
import os
import random
import types
from fractions import Fraction as F

import pytest

from oracle import rg_ref
from oracle import ref_c
from tests import test_oracle_rank_test as R
from tests.test_oracle_exact import _planted

MUTATIONS = {
    "ct_update_sign": ("st.Ct[k][j] - gamma[k] * K[j]", "st.Ct[k][j] + gamma[k] * K[j]"),
    "ct_update_dropped": ("st.Ct[k][j] - gamma[k] * K[j]", "st.Ct[k][j]"),
    "pinv_downdate_sign": ("st.Pinv[i][k] - zeta[i] * zeta[k] / den", "st.Pinv[i][k] + zeta[i] * zeta[k] / den"),
    "den_missing_one": ("den = (z + 1) + sum", "den = z + sum"),
    "residual_sign": ("dy = y - sum", "dy = y + sum"),
    "rejection_uses_dual": ("st.C[k][j] * gamma[k] for k", "st.Ct[k][j] * gamma[k] for k"),
    "projection_uses_basis": ("st.Ct[k][j] * Gamma[j] for j", "st.C[k][j] * Gamma[j] for j"),
    "gain_uses_raw_row": ("K = [v / nrm2 for v in Gamma_r]", "K = [v / nrm2 for v in Gamma]"),
    "pinv_border_two": ("[[z] * r + [z + 1]]", "[[z] * r + [z + 2]]"),
    "basis_stores_rejection": ("st.C.append(list(Gamma))", "st.C.append(list(Gamma_r))"),
    "gain_dependent_no_den": ("for k in range(r)), z) / den for j", "for k in range(r)), z) for j"),
    # the relative clause of the rank test (Section 3), float and rational branches
    "rank_rel_dropped": ("return nr < eps or nr < eps * ng", "return nr < eps"),
    "rank_rel_squared": ("return nr < eps or nr < eps * ng", "return nr < eps or nr < eps * ng * ng"),
    "rank_rel_not_strict": ("return nr < eps or nr < eps * ng", "return nr < eps or nr <= eps * ng"),
    "rank_rel_dropped_exact": ("return s < e2 or s < e2 * g", "return s < e2"),
    "rank_rel_squared_exact": ("return s < e2 or s < e2 * g", "return s < e2 or s < e2 * g * g"),
    "rank_rel_not_strict_exact": ("return s < e2 or s < e2 * g", "return s < e2 or s <= e2 * g"),
}

# The same three slips planted in the C oracle's rank test.
C_MUTATIONS = {
    "c_rank_rel_dropped": ("(nr < eps) || (nr < eps * ng)", "(nr < eps)"),
    "c_rank_rel_squared": ("(nr < eps) || (nr < eps * ng)", "(nr < eps) || (nr < eps * ng * ng)"),
    "c_rank_rel_not_strict": ("(nr < eps) || (nr < eps * ng)", "(nr < eps) || (nr <= eps * ng)"),
}


def _mutant(old, new):
    src = inspect.getsource(rg_ref)
    assert src.count(old) >= 1, old
    mod = types.ModuleType("rg_ref_mutant")
    exec(compile(src.replace(old, new), "rg_ref_mutant", "exec"), mod.__dict__)
    return mod


def _pins_pass(mod):
    """A subset of the oracle pins, run against module ``mod``."""
    for rows, eps, want in R.CASES.values():
        if R.python_float_decisions(mod, rows, eps) != want or R.python_exact_decisions(mod, rows, eps) != want:
            return False
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example_m2.json")))
    st = mod.RGState(2, F(0))
    for row, y in zip(gold["rows"], gold["y"]):
        mod.update_least_squares(st, [F(v) for v in row], F(y), 0)
    if st.X != [F(*p) for p in gold["x_after_each_row"][-1]]:
        return False
    for seed in range(12):
        rng = random.Random(seed)
        m, n, r = rng.randint(1, 7), rng.randint(1, 18), 0
        r = rng.randint(1, min(m, 5))
        A, Y = _planted(rng, n, m, r)
        try:
            s = mod.solve_stream(A, Y, exact=True)
        except ZeroDivisionError:
            return False
        x, rank = rg_ref.lstsq_exact(A, Y)
        if s.r != rank or s.X != x:
            return False
    return True


def test_unmutated_passes():
    assert _pins_pass(rg_ref)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    old, new = MUTATIONS[name]
    assert not _pins_pass(_mutant(old, new))


def _c_pins_pass(lib_path):
    return all(R.c_decisions(rows, eps, lib_path) == want for rows, eps, want in R.CASES.values())


def test_c_unmutated_passes(tmp_path):
    assert _c_pins_pass(ref_c.build_from_source(ref_c.source(), str(tmp_path / "librg_ref_copy.so")))


@pytest.mark.parametrize("name", sorted(C_MUTATIONS))
def test_c_mutation_is_caught(name, tmp_path):
    old, new = C_MUTATIONS[name]
    src = ref_c.source()
    assert src.count(old) == 1, old
    lib = ref_c.build_from_source(src.replace(old, new), str(tmp_path / ("librg_ref_%s.so" % name)))
    assert not _c_pins_pass(lib)
