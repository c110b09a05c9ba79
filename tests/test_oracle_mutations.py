"""The oracle's pins must catch plausible mistakes.  Each case plants one mistake in a
copy of the oracle's source (on the CPU, in a temporary directory), builds it, and runs
the pins that should catch it; they must fail."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ccmc_oracle.c")

MUTATIONS = [
    ("creator sign dropped", "    (*n)++;\n    return (k & 1) ? -1 : 1;", "    (*n)++;\n    return 1;",
     "excitor_sign_bruteforce or collapse_bruteforce"),
    ("exchange integral dropped", "return orc_u2(S, p, q, r, s) - orc_u2(S, p, q, s, r);",
     "return orc_u2(S, p, q, r, s);", "slater_condon_molecular"),
    ("s! missing from p(c)", "fact *= (double)a;", "fact *= 1.0;", "exact_expectation_molecular"),
    ("same-spin path factor missing in UEG p_gen",
     "pgen = (((i & 1) == (j & 1)) ? 2.0 : 1.0) / ((double)np * (double)half);",
     "pgen = 1.0 / ((double)np * (double)half);", "exact_expectation_ueg"),
    ("shift sign flipped in death", "return -tau * (K - shift) * A;", "return -tau * (K + shift) * A;",
     "exact_expectation_molecular"),
    ("composite sizes start at 1", "int lo = composite ? 2 : 0, hi = R->l + 2;",
     "int lo = composite ? 1 : 0, hi = R->l + 2;", "exact_expectation_molecular"),
    ("reference amplitude power", "for (int a = 1; a < s; ++a) Ac *= R->amps[idx[a]] / R->n0;",
     "for (int a = 1; a < s; ++a) Ac *= R->amps[idx[a]];", "exact_expectation_molecular"),
    ("Philox key schedule", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;", "philox"),
    ("biased spawn rounding", "x = copysign(R->opt.spawn_cutoff, x);",
     "x = copysign(0.5 * R->opt.spawn_cutoff, x);", "full_step_mean"),
    ("excitor draws cover half the weight", "uint64_t r = below(draw(R, PURPOSE_SELECT, k, 0, 1 + a), R->qtot);",
     "uint64_t r = below(draw(R, PURPOSE_SELECT, k, 0, 1 + a), R->qtot / 2);", "full_step_mean"),
]


@pytest.mark.parametrize("name,old,new,selector", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, selector):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    with tempfile.TemporaryDirectory() as tmp:
        csrc = os.path.join(tmp, "ccmc_oracle.c")
        with open(csrc, "w") as f:
            f.write(src.replace(old, new))
        with open(os.path.join(tmp, "ccmc_oracle.h"), "w") as f:
            f.write(open(os.path.join(ROOT, "oracle", "ccmc_oracle.h")).read())
        so = os.path.join(tmp, "libmut.so")
        subprocess.check_call(["gcc", "-std=c11", "-D_GNU_SOURCE", "-O2", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", so, csrc, "-lm"])
        env = dict(os.environ, CCMC_ORACLE_LIB=so)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", selector],
                           env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
        assert r.returncode == 1, f"{name}: pins did not fail\n{r.stdout[-2000:]}"
