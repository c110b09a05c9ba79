"""The oracle and its host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): a small C driver built with the oracle's source and -fsanitize=address,undefined runs
UEG and molecule-like steps through the oracle's C API -- original and full non-composite
selection, multi-spawn, virtual processors, import / export and the record list -- and must
end cleanly (any sanitizer report aborts it)."""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "ccmc_oracle.h"

static int run(orc_system *S, int l, int fnc, int kmin, double thr, uint32_t ranks, double init, double tau, int steps)
{
    orc_options o;
    memset(&o, 0, sizeof o);
    o.full_noncomposite = fnc; o.min_spawn_attempts = kmin; o.multispawn_threshold = thr;
    o.noncomposite_threshold = 1.0; o.spawn_cutoff = 0.01; o.occupation_threshold = 1.0; o.init_pop = init;
    o.p_single = 0.2; o.seed = 4321; o.n_ranks = ranks; o.move_shift = 2; o.hash_seed = 0;
    orc_run *R = NULL;
    if (orc_run_create(S, l, &o, &R)) return 1;
    orc_stats st;
    uint64_t nsel = (uint64_t)init;
    for (int t = 0; t < steps; ++t) {
        if (orc_step(R, tau, -0.01 * t, nsel, &st)) return 2;
        nsel = (uint64_t)(st.n_total + 0.5);
    }
    uint64_t n = 0, nr = 0, step = 0;
    double n0 = 0;
    int ne = 0, M = 0, W = 0;
    orc_system_dims(S, &ne, &M, &W);
    orc_export_size(R, &n);
    uint64_t *keys = calloc((n ? n : 1) * W, sizeof(uint64_t));
    double *amps = calloc(n ? n : 1, sizeof(double));
    if (orc_export(R, keys, amps, &n0, &step)) return 3;
    if (orc_import(R, keys, amps, n, n0, step)) return 4;
    orc_records_size(R, &nr);
    uint64_t *rk = calloc((nr ? nr : 1) * W, sizeof(uint64_t)), *ids = calloc(nr ? nr : 1, sizeof(uint64_t));
    double *ra = calloc(nr ? nr : 1, sizeof(double));
    if (orc_records(R, rk, ra, ids)) return 5;
    if (orc_step(R, tau, 0.0, nsel, &st)) return 6;
    printf("ok %llu excitors %llu records\n", (unsigned long long)n, (unsigned long long)nr);
    free(keys); free(amps); free(rk); free(ids); free(ra);
    orc_run_free(R);
    return 0;
}

int main(void)
{
    orc_system *U = NULL, *V = NULL, *Mo = NULL;
    if (orc_system_ueg(14, 2, 1.0, &U) || orc_system_ueg(14, 4, 0.5, &V)) return 10;
    int n = 5, nc = 6;
    double h[25], *B = calloc((size_t)nc * n * n, sizeof(double));
    srand(7);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q <= p; ++q) {
            double x = (p == q) ? -1.0 + 0.4 * p : 0.02 * ((rand() % 200) / 100.0 - 1.0);
            h[p * n + q] = h[q * n + p] = x;
        }
    for (int L = 0; L < nc; ++L)
        for (int p = 0; p < n; ++p)
            for (int q = 0; q <= p; ++q) {
                double x = 0.1 * ((rand() % 200) / 100.0 - 1.0);
                B[(L * n + p) * n + q] = B[(L * n + q) * n + p] = x;
            }
    if (orc_system_mol(4, n, h, B, nc, &Mo)) return 11;
    int rc = 0;
    rc |= run(U, 2, 0, 1, 0.0, 1, 300.0, 0.005, 12);
    rc |= run(V, 3, 1, 4, 1.0, 1, 300.0, 0.004, 8);
    rc |= run(V, 3, 1, 2, 1.0, 24, 300.0, 0.004, 6);
    rc |= run(Mo, 4, 0, 1, 0.0, 1, 200.0, 0.01, 12);
    rc |= run(Mo, 2, 1, 3, 0.7, 3, 200.0, 0.01, 12);
    orc_system_free(U); orc_system_free(V); orc_system_free(Mo);
    free(B);
    return rc;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"),
           str(src), os.path.join(ROOT, "oracle", "ccmc_oracle.c"), "-lm", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "cannot find" in (r.stderr or "") and "asan" in (r.stderr or ""):
        pytest.skip("no sanitizer runtime: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert out.stdout.count("ok ") == 5, out.stdout
