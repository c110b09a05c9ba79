"""ctypes binding of the CPU oracle (``oracle/libccmc_oracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU
baseline of the benchmark.  The product package never imports it.

The oracle follows Spencer et al., arXiv:1807.03749, Sec. II (cluster sampling, spawning,
death, annihilation, projected energy) and Sec. IV (full non-composite sampling,
multi-spawn); see ``ccmc_oracle.h`` for the readings it takes where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# CCMC_ORACLE_LIB points the tests at a deliberately broken copy (mutation tests only).
LIB_PATH = os.environ.get("CCMC_ORACLE_LIB") or os.path.join(HERE, "libccmc_oracle.so")
SRC_PATH = os.path.join(HERE, "ccmc_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (serial C, FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-std=c11", "-D_GNU_SOURCE", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
            "-Wall", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Options(C.Structure):
    _fields_ = [
        ("full_noncomposite", C.c_int),
        ("min_spawn_attempts", C.c_int),
        ("multispawn_threshold", C.c_double),
        ("noncomposite_threshold", C.c_double),
        ("spawn_cutoff", C.c_double),
        ("occupation_threshold", C.c_double),
        ("init_pop", C.c_double),
        ("p_single", C.c_double),
        ("seed", C.c_uint64),
        ("n_ranks", C.c_uint32),
        ("move_shift", C.c_uint32),
        ("hash_seed", C.c_uint32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("step", C.c_uint64),
        ("n_selections", C.c_uint64),
        ("n_discarded", C.c_uint64),
        ("n_spawn_attempts", C.c_uint64),
        ("n_spawns", C.c_uint64),
        ("n_deaths", C.c_uint64),
        ("n_excitors", C.c_uint64),
        ("max_attempts_per_cluster", C.c_uint64),
        ("n_total", C.c_double),
        ("n_ref", C.c_double),
        ("eproj_num", C.c_double),
        ("eproj_den", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        sig = {
            "orc_system_ueg": (C.c_int, [C.c_int, C.c_int, C.c_double, C.POINTER(vp)]),
            "orc_system_mol": (C.c_int, [C.c_int, C.c_int, _f64p, _f64p, C.c_int, C.POINTER(vp)]),
            "orc_system_free": (None, [vp]),
            "orc_system_dims": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "orc_ueg_nvec": (C.c_int, [vp, _i32p]),
            "orc_ueg_box_length": (C.c_double, [vp]),
            "orc_h1": (C.c_double, [vp, C.c_int, C.c_int]),
            "orc_u2": (C.c_double, [vp, C.c_int, C.c_int, C.c_int, C.c_int]),
            "orc_hamiltonian": (C.c_double, [vp, _u64p, _u64p]),
            "orc_ehf": (C.c_double, [vp]),
            "orc_excitor_sign": (C.c_int, [vp, _u64p]),
            "orc_excitation_level": (C.c_int, [vp, _u64p]),
            "orc_collapse": (C.c_int, [vp, C.c_int, _u64p, _u64p, C.POINTER(C.c_int)]),
            "orc_run_create": (C.c_int, [vp, C.c_int, C.POINTER(Options), C.POINTER(vp)]),
            "orc_run_free": (None, [vp]),
            "orc_import": (C.c_int, [vp, _u64p, _f64p, C.c_uint64, C.c_double, C.c_uint64]),
            "orc_export_size": (C.c_int, [vp, C.POINTER(C.c_uint64)]),
            "orc_export": (C.c_int, [vp, _u64p, _f64p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
            "orc_step": (C.c_int, [vp, C.c_double, C.c_double, C.c_uint64, C.POINTER(Stats)]),
            "orc_records_size": (C.c_int, [vp, C.POINTER(C.c_uint64)]),
            "orc_records": (C.c_int, [vp, _u64p, _f64p, _u64p]),
            "orc_weight": (C.c_uint64, [C.c_double]),
            "orc_cluster": (C.c_int, [vp, C.c_int, _u64p, C.c_uint64, C.c_int, _u64p,
                                      C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_uint64)]),
            "orc_attempts": (C.c_int, [vp, C.c_double, C.c_int, C.POINTER(C.c_uint64)]),
            "orc_attempt": (C.c_int, [vp, _u64p, C.c_double, C.c_uint64, _u64p, C.c_double, _u64p,
                                      C.POINTER(C.c_double)]),
            "orc_death": (C.c_double, [vp, _u64p, C.c_double, C.c_double, C.c_double]),
            "orc_philox": (None, [_u32p, _u32p, _u32p]),
            "orc_cluster_ranked": (C.c_int, [vp, C.c_int, _u64p, C.c_uint64, C.c_uint64, C.c_uint32, C.c_int, _u64p,
                                             C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_uint64)]),
            "orc_murmur2": (C.c_uint32, [C.c_char_p, C.c_int, C.c_uint32]),
            "orc_placement": (C.c_uint32, [C.c_int, _u64p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]),
            "orc_codistribution": (C.c_int, [C.c_int, _u64p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p,
                                             C.c_int, _u64p, _u64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def murmur2(data: bytes, seed: int) -> int:
    return int(lib().orc_murmur2(bytes(data), len(data), int(seed)))


def placement(det, i_tau: int, n_ranks: int, move_shift: int, seed: int) -> int:
    d = np.ascontiguousarray(det, np.uint64)
    return int(lib().orc_placement(len(d), d, int(i_tau), int(n_ranks), int(move_shift), int(seed)))


def codistribution(keys, n_ranks: int, move_shift: int, seed: int, checkpoints):
    """Sums over pairs i < j of c_ij and c_ij^2 at each checkpoint (c_ij: iterations on the
    same processor)."""
    keys = np.ascontiguousarray(np.asarray(keys, np.uint64))
    n, W = keys.shape
    cp = np.ascontiguousarray(checkpoints, np.uint64)
    s1 = np.zeros(len(cp), np.uint64)
    s2 = np.zeros(len(cp), np.uint64)
    _check(lib().orc_codistribution(W, keys.ravel(), n, int(n_ranks), int(move_shift), int(seed), cp, len(cp), s1, s2),
           "codistribution")
    return s1, s2


def weight(amp: float) -> int:
    return int(lib().orc_weight(float(amp)))


class System:
    """A UEG or molecule-like system held by the oracle."""

    def __init__(self, handle, kind: str):
        self._h = handle
        self.kind = kind
        ne, M, W = C.c_int(), C.c_int(), C.c_int()
        lib().orc_system_dims(self._h, C.byref(ne), C.byref(M), C.byref(W))
        self.n_el, self.M, self.W = ne.value, M.value, W.value

    @classmethod
    def ueg(cls, n_el: int, n2max: int, rs: float) -> "System":
        h = C.c_void_p()
        _check(lib().orc_system_ueg(n_el, n2max, rs, C.byref(h)), "system_ueg")
        return cls(h, "ueg")

    @classmethod
    def molecular(cls, n_el: int, h1: np.ndarray, chol: np.ndarray) -> "System":
        h = C.c_void_p()
        h1 = np.ascontiguousarray(h1, np.float64)
        chol = np.ascontiguousarray(chol, np.float64)
        n = h1.shape[0]
        if chol.size == 0:
            chol = np.zeros(1, np.float64)
            nchol = 0
        else:
            nchol = chol.shape[0]
        _check(lib().orc_system_mol(n_el, n, h1.ravel(), chol.ravel(), nchol, C.byref(h)), "system_mol")
        return cls(h, "mol")

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.orc_system_free(self._h)
            self._h = None

    # --- helpers
    def det(self, orbitals) -> np.ndarray:
        d = np.zeros(self.W, np.uint64)
        for p in orbitals:
            d[p >> 6] |= np.uint64(1) << np.uint64(p & 63)
        return d

    @property
    def hf(self) -> np.ndarray:
        return self.det(range(self.n_el))

    def nvec(self) -> np.ndarray:
        out = np.zeros((self.M // 2, 3), np.int32)
        _check(lib().orc_ueg_nvec(self._h, out.ravel()), "ueg_nvec")
        return out

    def box_length(self) -> float:
        return lib().orc_ueg_box_length(self._h)

    def h1(self, p, q) -> float:
        return lib().orc_h1(self._h, p, q)

    def u2(self, p, q, r, s) -> float:
        return lib().orc_u2(self._h, p, q, r, s)

    def hamiltonian(self, bra, ket) -> float:
        return lib().orc_hamiltonian(self._h, np.ascontiguousarray(bra, np.uint64),
                                     np.ascontiguousarray(ket, np.uint64))

    def ehf(self) -> float:
        return lib().orc_ehf(self._h)

    def excitor_sign(self, det) -> int:
        return lib().orc_excitor_sign(self._h, np.ascontiguousarray(det, np.uint64))

    def level(self, det) -> int:
        return lib().orc_excitation_level(self._h, np.ascontiguousarray(det, np.uint64))

    def collapse(self, dets):
        keys = np.ascontiguousarray(np.asarray(dets, np.uint64).reshape(-1))
        out = np.zeros(self.W, np.uint64)
        sign = C.c_int()
        ok = lib().orc_collapse(self._h, len(dets), keys, out, C.byref(sign))
        return (out, sign.value) if ok else (None, 0)


@dataclass
class RunOptions:
    full_noncomposite: bool = False
    min_spawn_attempts: int = 1
    multispawn_threshold: float = 0.0
    noncomposite_threshold: float = 1.0
    spawn_cutoff: float = 0.01
    occupation_threshold: float = 1.0
    init_pop: float = 10.0
    p_single: float = 0.1
    seed: int = 1234
    n_ranks: int = 1
    move_shift: int = 5
    hash_seed: int = 0

    def to_c(self) -> Options:
        return Options(int(self.full_noncomposite), int(self.min_spawn_attempts),
                       float(self.multispawn_threshold), float(self.noncomposite_threshold),
                       float(self.spawn_cutoff), float(self.occupation_threshold), float(self.init_pop),
                       float(self.p_single), int(self.seed), int(self.n_ranks), int(self.move_shift),
                       int(self.hash_seed))


class Run:
    """One CCMC calculation held by the oracle."""

    def __init__(self, system: System, truncation: int, options: RunOptions | None = None):
        self.system = system
        self.truncation = truncation
        self.options = options or RunOptions()
        self._opt = self.options.to_c()
        h = C.c_void_p()
        _check(lib().orc_run_create(system._h, truncation, C.byref(self._opt), C.byref(h)), "run_create")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.orc_run_free(self._h)
            self._h = None

    def import_state(self, keys, amps, n_ref: float, step: int = 0):
        keys = np.ascontiguousarray(np.asarray(keys, np.uint64).reshape(-1, self.system.W))
        amps = np.ascontiguousarray(amps, np.float64)
        _check(lib().orc_import(self._h, keys.ravel() if keys.size else np.zeros(1, np.uint64),
                                amps if amps.size else np.zeros(1), len(amps), float(n_ref), int(step)),
               "import")

    def export_state(self):
        n = C.c_uint64()
        lib().orc_export_size(self._h, C.byref(n))
        keys = np.zeros((max(n.value, 1), self.system.W), np.uint64)
        amps = np.zeros(max(n.value, 1), np.float64)
        n_ref, step = C.c_double(), C.c_uint64()
        lib().orc_export(self._h, keys.ravel(), amps, C.byref(n_ref), C.byref(step))
        return keys[: n.value], amps[: n.value], n_ref.value, step.value

    def step(self, tau: float, shift: float, n_sel: int) -> dict:
        st = Stats()
        _check(lib().orc_step(self._h, tau, shift, int(n_sel), C.byref(st)), "step")
        return st.as_dict()

    def records(self):
        n = C.c_uint64()
        lib().orc_records_size(self._h, C.byref(n))
        m = max(n.value, 1)
        keys = np.zeros((m, self.system.W), np.uint64)
        amps = np.zeros(m, np.float64)
        ids = np.zeros(m, np.uint64)
        lib().orc_records(self._h, keys.ravel(), amps, ids)
        return keys[: n.value], amps[: n.value], ids[: n.value]

    # --- components
    def cluster(self, idx, n_sel: int, composite: bool):
        s = len(idx)
        arr = np.ascontiguousarray(idx, np.uint64) if s else np.zeros(1, np.uint64)
        det = np.zeros(self.system.W, np.uint64)
        A, L, n = C.c_double(), C.c_int(), C.c_uint64()
        ok = lib().orc_cluster(self._h, s, arr, int(n_sel), int(composite), det,
                               C.byref(A), C.byref(L), C.byref(n))
        _check(ok, "cluster")
        return (det, A.value, L.value, n.value) if ok else None

    def cluster_ranked(self, idx, count: int, qnorm: int, n_ranks: int, composite: bool):
        s = len(idx)
        arr = np.ascontiguousarray(idx, np.uint64) if s else np.zeros(1, np.uint64)
        det = np.zeros(self.system.W, np.uint64)
        A, L, n = C.c_double(), C.c_int(), C.c_uint64()
        ok = lib().orc_cluster_ranked(self._h, s, arr, int(count), int(qnorm), int(n_ranks), int(composite), det,
                                      C.byref(A), C.byref(L), C.byref(n))
        _check(ok, "cluster_ranked")
        return (det, A.value, L.value, n.value) if ok else None

    def attempts(self, A: float, noncomposite: bool) -> int:
        n = C.c_uint64()
        _check(lib().orc_attempts(self._h, float(A), int(noncomposite), C.byref(n)), "attempts")
        return n.value

    def attempt(self, det, A: float, n: int, choice, tau: float):
        tgt = np.zeros(self.system.W, np.uint64)
        x = C.c_double()
        ch = np.zeros(4, np.uint64)
        ch[: len(choice)] = choice
        ok = lib().orc_attempt(self._h, np.ascontiguousarray(det, np.uint64), float(A), int(n), ch, float(tau),
                               tgt, C.byref(x))
        return (tgt, x.value) if ok else None

    def death(self, det, A: float, tau: float, shift: float) -> float:
        return lib().orc_death(self._h, np.ascontiguousarray(det, np.uint64), float(A), float(tau), float(shift))
