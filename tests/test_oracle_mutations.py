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
PINS, PLACE = "test_oracle_pins.py", "test_oracle_placement.py"

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
    ("excitor draws cover half the weight", "uint64_t r = below(draw(R, PURPOSE_SELECT, k, 0, 1 + a), qnorm);",
     "uint64_t r = below(draw(R, PURPOSE_SELECT, k, 0, 1 + a), qnorm / 2);", "full_step_mean"),
    # virtual processors (Sec. III)
    ("MurmurHash2 tail byte shifted", "if (len == 3) h ^= (uint32_t)b[2] << 16;",
     "if (len == 3) h ^= (uint32_t)b[2] << 8;", "murmur2", PLACE),
    ("offset never applied", "    d[0] ^= o;\n", "    d[0] ^= 0;\n", "moves_only", PLACE),
    ("processor factor N_p^-s", "for (int a = 1; a < s; ++a) d *= (double)n_ranks;",
     "for (int a = 0; a < s; ++a) d *= (double)n_ranks;", "unbiased_over_placements", PLACE),
    ("reference cluster not scaled", "            p *= (double)n_ranks;\n", "            p *= 1.0;\n",
     "unbiased_over_placements", PLACE),
    ("selections per processor rounded down", "n_sel / np + (rank < n_sel % np ? 1 : 0)", "n_sel / np",
     "one_placement", PLACE),
]


@pytest.mark.parametrize("name,old,new,selector,tests", [m if len(m) == 5 else (*m, PINS) for m in MUTATIONS],
                         ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, selector, tests):
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
                            os.path.join(ROOT, "tests", tests), "-k", selector],
                           env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
        assert r.returncode == 1, f"{name}: pins did not fail\n{r.stdout[-2000:]}"
