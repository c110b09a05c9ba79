"""Annihilation at a size where the radix histogram takes its 1024-thread blocks (at least 256
tiles of 2048 records): one FP64 step of the molecule-like 16e/92so CCSDTQ system at
N_tot ~ 2.5e6 (several million records), checked against sums formed on the host from the
step's own records and the store before it.  These are properties that hold at any size
(Sec. II): the spawned and death amounts of a determinant add to its amplitude, the reference's
to N_0; occupation rounding only touches |N| below the threshold, where it gives 0 or
+-threshold with the sign of N; no determinant appears that neither the store nor a record
holds; the store stays strictly ascending."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1807_03749_amd import ccmc, driver, inputs

pytestmark = pytest.mark.gpu


def _say(msg: str):
    print(msg, flush=True)


def _group(keys: np.ndarray, vals: np.ndarray):
    """Unique two-word keys (ascending, word 1 most significant) and the sums of their values."""
    order = np.lexsort((keys[:, 0], keys[:, 1]))
    k = keys[order]
    v = vals[order]
    new = np.ones(len(k), bool)
    new[1:] = (k[1:, 0] != k[:-1, 0]) | (k[1:, 1] != k[:-1, 1])
    starts = np.flatnonzero(new)
    return k[starts], np.add.reduceat(v, starts), np.add.reduceat(np.abs(v), starts)


def _index(keys: np.ndarray, query: np.ndarray):
    """Position of each query key in the ascending `keys`, or -1."""
    # lexicographic search on (word 1, word 0) with a structured view
    kv = np.ascontiguousarray(keys[:, ::-1]).view([("hi", "<u8"), ("lo", "<u8")]).ravel()
    qv = np.ascontiguousarray(query[:, ::-1]).view([("hi", "<u8"), ("lo", "<u8")]).ravel()
    pos = np.searchsorted(kv, qv)
    pos_c = np.minimum(pos, len(kv) - 1)
    hit = (pos < len(kv)) & (kv[pos_c] == qv)
    return np.where(hit, pos_c, -1)


def test_large_step_annihilation_sums():
    w = inputs.WORKLOADS["mol16_92_ccsdtq_fp32"]
    h, B = inputs.molecule_like(n_spatial=w.n_spatial, n_electrons=w.n_electrons, n_chol=w.n_chol)
    st = ccmc.State("mol", w.n_electrons, w.truncation, h=h, chol=B, precision="fp64", full_noncomposite=1,
                    min_spawn_attempts=w.min_spawn_attempts, multispawn_threshold=w.multispawn_threshold,
                    noncomposite_threshold=w.noncomposite_threshold, init_pop=1e5, seed=w.seed, keep_spawn_ids=1)
    try:
        nsel = driver.selections(1e5)
        s = None
        for it in range(200):  # growth at the shift 0
            s = st.ccmc_step(w.tau, 0.0, nsel)
            nsel = driver.selections(s["n_total"])
            if s["n_total"] >= 2.5e6:
                break
        _say(f"[large] grown in {it + 1} steps: N_tot {s['n_total']:.3e}, {s['n_excitors']} excitors")
        k0, a0, n0_0, _ = st.ccmc_export()
        s = st.ccmc_step(w.tau, 0.0, nsel)
        rk, ra, rid = st.ccmc_export_spawns()
        k1, a1, n0_1, _ = st.ccmc_export()
        _say(f"[large] step: {len(rk)} records, {s['n_excitors']} excitors after")
        assert len(rk) >= 256 * 2048, "the step must cover at least 256 radix tiles"
        theta = st.options.occupation_threshold
    finally:
        st.close()

    # the store stays strictly ascending (word 1 most significant)
    hi, lo = k1[:, 1], k1[:, 0]
    assert np.all((hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1])))
    assert s["n_excitors"] == len(k1)

    # the reference's records add to N_0 (it is not rounded)
    hf = np.array([(1 << w.n_electrons) - 1, 0], np.uint64)
    is_hf = (rk[:, 0] == hf[0]) & (rk[:, 1] == hf[1])
    ref_sum = ra[is_hf].sum()
    ref_mag = np.abs(ra[is_hf]).sum() + abs(n0_0)
    assert abs(n0_1 - (n0_0 + ref_sum)) <= 1e-12 * ref_mag + 1e-12

    # every determinant: old amplitude plus its records
    keys = np.concatenate([k0, rk[~is_hf]])
    vals = np.concatenate([a0, ra[~is_hf]])
    uk, usum, umag = _group(keys, vals)
    pos = _index(k1, uk)
    new = np.where(pos >= 0, a1[np.maximum(pos, 0)], 0.0)
    assert (pos >= 0).sum() == len(k1), "a determinant of the new store that no record or old entry holds"
    tol = 1e-12 * umag + 1e-300
    above = np.abs(usum) >= theta * (1 + 1e-9)
    below = np.abs(usum) < theta * (1 - 1e-9)
    assert np.all(np.abs(new[above] - usum[above]) <= tol[above]), "summed amplitudes differ"
    nb = new[below]
    assert np.all((nb == 0) | (np.abs(np.abs(nb) - theta) <= 1e-12 * theta)), "a rounded amplitude is not 0 or theta"
    assert np.all((nb == 0) | (np.sign(nb) == np.sign(usum[below]))), "a rounded amplitude changed sign"
    _say(f"[large] {len(uk)} determinants checked ({above.sum()} summed, {below.sum()} rounded)")
