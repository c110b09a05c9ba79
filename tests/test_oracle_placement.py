"""Pins of the oracle's virtual processors (Sec. III, eq. 9) against things other
than itself (no GPU).

* MurmurHash2: SMHasher's published verification value (tests/golden/murmur2_verification.txt).
* Placement: nu_move >= 64 is the static eq. 8, hash(D) mod N_p; with nu_move the
  processor can change only where (hash(D) + i_tau) crosses a multiple of 2^nu_move; the
  processors are evenly used.
* Co-location sums: brute force over pairs and iterations.
* Ranked selection: averaged over every placement of the excitors, the expected amplitude
  that one step's selections put on each cluster is the one-processor value (the N_p^(1-s)
  factor); and the mean of many oracle steps at one placement matches the exact
  enumeration of that placement's selections.
"""
from __future__ import annotations

import itertools
import math
import os
from collections import defaultdict

import numpy as np
import pytest

from oracle import binding as ob
from paper_1807_03749_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return {ln.split()[0]: ln.split()[1] for ln in f if ln.strip() and not ln.startswith("#")}


# ----------------------------------------------------------------------- MurmurHash2

def test_murmur2_smhasher_verification():
    g = _golden("murmur2_verification.txt")
    key = bytearray(256)
    out = bytearray()
    for i in range(256):
        key[i] = i
        out += ob.murmur2(bytes(key[:i]), 256 - i).to_bytes(4, "little")
    assert ob.murmur2(bytes(out), 0) == int(g["verification"], 16)
    assert ob.murmur2(b"", 0) == int(g["empty_seed0"], 16)


def _det_bytes(d):
    return b"".join(int(w).to_bytes(8, "little") for w in d)


def _random_dets(rng, n, W, M):
    dets = set()
    while len(dets) < n:
        occ = rng.choice(M, 14, replace=False)
        d = [0] * W
        for p in occ:
            d[p >> 6] |= 1 << int(p & 63)
        dets.add(tuple(d))
    return np.array(sorted(dets), np.uint64)


# ------------------------------------------------------------------------- placement

def test_static_placement_is_hash_mod_np():
    rng = np.random.default_rng(3)
    for d in _random_dets(rng, 50, 2, 114):
        want = ob.murmur2(_det_bytes(d), 17) % 7
        for t in (0, 1, 1000, 2 ** 40):
            assert ob.placement(d, t, 7, 64, 17) == want
    assert ob.placement(np.array([5, 0], np.uint64), 3, 1, 2, 0) == 0


def test_moves_only_at_offset_boundaries():
    rng = np.random.default_rng(4)
    nu, np_ = 3, 5
    changes = 0
    for d in _random_dets(rng, 40, 3, 186):
        h = ob.murmur2(_det_bytes(d), 9)
        prev = ob.placement(d, 0, np_, nu, 9)
        for t in range(1, 70):
            cur = ob.placement(d, t, np_, nu, 9)
            if (h + t) % (1 << nu) != 0:
                assert cur == prev, (t, h)
            else:
                changes += cur != prev
            prev = cur
    assert changes > 0  # it does move


def test_placement_evenly_spread():
    rng = np.random.default_rng(5)
    dets = _random_dets(rng, 4000, 2, 114)
    np_ = 16
    for t in (0, 77):
        counts = np.bincount([ob.placement(d, t, np_, 5, 0) for d in dets], minlength=np_)
        chi2 = float(((counts - len(dets) / np_) ** 2 / (len(dets) / np_)).sum())
        assert chi2 < 50.0  # 15 degrees of freedom: P(chi2 > 50) < 1e-5


def test_codistribution_sums_brute_force():
    rng = np.random.default_rng(6)
    dets = _random_dets(rng, 23, 2, 66)
    cps = [0, 1, 5, 16, 40]
    for np_, nu in ((3, 2), (8, 4), (4, 64)):
        s1, s2 = ob.codistribution(dets, np_, nu, 11, cps)
        pl = np.array([[ob.placement(d, t, np_, nu, 11) for d in dets] for t in range(cps[-1])])
        for c, T in enumerate(cps):
            same = (pl[:T, :, None] == pl[:T, None, :]).sum(0)
            iu = np.triu_indices(len(dets), 1)
            cnt = same[iu].astype(np.uint64)
            assert int(s1[c]) == int(cnt.sum()) and int(s2[c]) == int((cnt * cnt).sum())


def test_codistribution_mean_is_one_over_np():
    """The long-time co-location frequency of two excitors is 1/N_p (Sec. III.B)."""
    rng = np.random.default_rng(7)
    dets = _random_dets(rng, 120, 2, 114)
    npairs = len(dets) * (len(dets) - 1) // 2
    for np_ in (2, 4, 8):
        T = 256
        s1, s2 = ob.codistribution(dets, np_, 2, 0, [T])
        mean = float(s1[0]) / (npairs * T)
        assert abs(mean * np_ - 1.0) < 0.05


# -------------------------------------------------------------- ranked selection

def _mol_state(n=4, seed=2):
    h, B = inputs.molecule_like(n_spatial=5, n_electrons=4, n_chol=6, seed=4)
    S = ob.System.molecular(4, h, B)
    import sq
    hf = sq.to_int(S.hf)
    rng = np.random.default_rng(seed)
    pool = [d for d in sq.sz_determinants(S.M, S.n_el) if d != hf and 1 <= S.level(sq.to_words(d, S.W)) <= 2]
    pick = sorted(pool[i] for i in rng.choice(len(pool), n, replace=False))
    keys = np.array([sq.to_words(d, S.W) for d in pick], np.uint64)
    amps = np.array([1.25, -2.0, 0.75, 3.5, -1.5, 2.25][:n])
    return S, keys, amps


def _sizes(l, fnc):
    lo, hi = (2, l + 2) if fnc else (0, l + 2)
    return {s: (2.0 ** -(s - lo + 1) if s < hi else 2.0 ** -(hi - lo)) for s in range(lo, hi + 1)}


@pytest.mark.parametrize("fnc,np_", [(False, 2), (True, 2), (False, 3), (True, 3)])
def test_ranked_selection_unbiased_over_placements(fnc, np_):
    """Sum over placements (each excitor on each processor with probability 1/N_p), over the
    processors (one selection each) and over every draw: the expected cluster amplitude on
    each determinant equals the one-processor value."""
    S, keys, amps = _mol_state()
    l, n0 = 2, 3.0
    run = ob.Run(S, l, ob.RunOptions(full_noncomposite=fnc, init_pop=n0))
    run.import_state(keys, amps, n0)
    q = np.array([ob.weight(a) for a in amps], dtype=np.int64)
    n = len(amps)
    one = defaultdict(float)
    for s, ps in _sizes(l, fnc).items():
        for tup in itertools.product(range(n), repeat=s):
            c = run.cluster(list(tup), 1, fnc)
            if c is not None:
                one[tuple(c[0])] += ps * np.prod([q[i] / q.sum() for i in tup]) * c[1]
    many = defaultdict(float)
    for where in itertools.product(range(np_), repeat=n):
        pw = np_ ** -n
        for r in range(np_):
            mine = [i for i in range(n) if where[i] == r]
            Qr = int(q[mine].sum()) if mine else 0
            for s, ps in _sizes(l, fnc).items():
                if s > 0 and not mine:
                    continue
                for tup in itertools.product(mine, repeat=s):
                    c = run.cluster_ranked(list(tup), 1, Qr, np_, fnc)
                    if c is not None:
                        many[tuple(c[0])] += pw * ps * np.prod([q[i] / Qr for i in tup]) * c[1]
    scale = max(abs(v) for v in one.values())
    for d in set(one) | set(many):
        assert many.get(d, 0.0) == pytest.approx(one.get(d, 0.0), abs=1e-12 * scale), d


@pytest.mark.parametrize("fnc", [False, True])
def test_ranked_step_matches_enumeration_at_one_placement(fnc):
    """Many oracle steps (different Philox keys) at one step index, hence one placement: the
    mean death amount recorded for the sampled clusters on each determinant matches the exact
    enumeration of that placement's selections, within 5 standard errors."""
    S, keys, amps = _mol_state(n=5, seed=3)
    l, n0, tau, shift, nsel, np_, t0 = 2, 3.0, 0.02, -0.1, 7, 3, 11
    where = [ob.placement(k, t0, np_, 1, 5) for k in keys]
    q = np.array([ob.weight(a) for a in amps], dtype=np.int64)
    base = ob.Run(S, l, ob.RunOptions(full_noncomposite=fnc, init_pop=n0, n_ranks=np_, move_shift=1, hash_seed=5))
    base.import_state(keys, amps, n0, t0)
    exact = defaultdict(float)
    for r in range(np_):
        count = nsel // np_ + (1 if r < nsel % np_ else 0)
        mine = [i for i in range(len(amps)) if where[i] == r]
        Qr = int(q[mine].sum()) if mine else 0
        for s, ps in _sizes(l, fnc).items():
            if s > 0 and not mine:
                continue
            for tup in itertools.product(mine, repeat=s):
                c = base.cluster_ranked(list(tup), count, Qr, np_, fnc)
                if c is None or c[2] > l:
                    continue
                prob = count * ps * np.prod([q[i] / Qr for i in tup])
                exact[tuple(c[0])] += prob * base.death(c[0], c[1], tau, shift)
    dets = sorted(exact)
    idx = {d: i for i, d in enumerate(dets)}
    nrep = 4000
    samples = np.zeros((nrep, len(dets)))
    for rep in range(nrep):
        run = ob.Run(S, l, ob.RunOptions(full_noncomposite=fnc, init_pop=n0, seed=500 + rep, n_ranks=np_,
                                         move_shift=1, hash_seed=5))
        run.import_state(keys, amps, n0, t0)
        run.step(tau, shift, nsel)
        rk, ra, ri = run.records()
        sampled_death = ((ri >> np.uint64(62)) == 1) & ((ri & np.uint64((1 << 30) - 1)) == 0)
        for k, a in zip(rk[sampled_death], ra[sampled_death]):
            samples[rep, idx[tuple(int(x) for x in k)]] += a
    mean = samples.mean(0)
    err = samples.std(0, ddof=1) / math.sqrt(nrep)
    for d in dets:
        i = idx[d]
        assert abs(mean[i] - exact[d]) <= 5 * err[i] + 1e-12 * abs(exact[d]), (d, mean[i], exact[d], err[i])


def test_ccsd_determinant_set_of_the_codistribution_study():
    """The input set of the co-distribution study: 3813 distinct determinants for 14e/186so
    (the count printed in Sec. III.B), all within CCSD and momentum-conserving (each double
    couples to the reference)."""
    rows = {(int(r[0]), int(r[1]), int(r[2])): int(r[3]) for r in
            (ln.split() for ln in open(os.path.join(GOLDEN, "ueg_space_sizes.txt")) if ln.strip() and ln[0] != "#")}
    dets = inputs.ueg_ccsd_determinants(14, 8)
    assert len(dets) == rows[(14, 186, 2)] and len({tuple(d) for d in dets}) == len(dets)
    S = ob.System.ueg(14, 8, 1.0)
    assert S.W == dets.shape[1]
    levels = [S.level(d) for d in dets]
    assert levels.count(0) == 1 and set(levels) == {0, 2}
    rng = np.random.default_rng(1)
    for d in dets[rng.choice(len(dets), 40, replace=False)]:
        if S.level(d) == 2:
            assert S.hamiltonian(S.hf, d) != 0.0
