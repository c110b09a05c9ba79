"""Thin ctypes binding of the HIP CCMC library (``libccmc.so``, C ABI in ``include/ccmc.h``).

Argument marshalling only: every step of the CCMC time step runs in the library's HIP
kernels.  There is no CPU fallback -- if the library is missing or no GPU is visible, the
calls fail loudly.

Names follow the C ABI: ``ccmc_init`` / ``ccmc_step`` / ``ccmc_energy`` / ``ccmc_free`` and the
import / export extensions, wrapped by the :class:`State` class.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccmc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ccmc.h")

CCMC_UEG, CCMC_MOLECULAR = 1, 2
CCMC_FP64, CCMC_FP32 = 0, 1
STATUS = {0: "CCMC_OK", -1: "CCMC_EINVAL", -2: "CCMC_ENOMEM", -3: "CCMC_EOVERFLOW", -4: "CCMC_EDEVICE",
          -5: "CCMC_EBLOWUP"}


class CCMCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class ccmc_system(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_electrons", C.c_int), ("n_spin_orbitals", C.c_int), ("rs", C.c_double),
                ("n2_max", C.c_int)]


class ccmc_integrals(C.Structure):
    _fields_ = [("n_spatial", C.c_int), ("h", C.POINTER(C.c_double)), ("chol", C.POINTER(C.c_double)),
                ("n_chol", C.c_int), ("eri", C.POINTER(C.c_double)), ("e_core", C.c_double)]


class ccmc_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("full_noncomposite", C.c_int), ("min_spawn_attempts", C.c_int),
                ("multispawn_threshold", C.c_double), ("noncomposite_threshold", C.c_double),
                ("spawn_cutoff", C.c_double), ("occupation_threshold", C.c_double), ("init_pop", C.c_double),
                ("p_single", C.c_double), ("seed", C.c_uint64), ("hbm_budget_bytes", C.c_uint64),
                ("hip_stream", C.c_void_p), ("keep_spawn_ids", C.c_int), ("n_ranks", C.c_uint32),
                ("move_shift", C.c_uint32), ("hash_seed", C.c_uint32), ("blowup_factor", C.c_double)]


class ccmc_stats(C.Structure):
    _fields_ = [("step", C.c_uint64), ("n_selections", C.c_uint64), ("n_discarded", C.c_uint64),
                ("n_spawn_attempts", C.c_uint64), ("n_spawns", C.c_uint64), ("n_deaths", C.c_uint64),
                ("n_excitors", C.c_uint64), ("max_attempts_per_cluster", C.c_uint64), ("n_total", C.c_double),
                ("n_ref", C.c_double), ("eproj_num", C.c_double), ("eproj_den", C.c_double), ("ms", C.c_double),
                ("status", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ccmc_shift_control(C.Structure):
    """The library's population control (``ccmc_shift_update``): the same rule as
    ``driver.ShiftControl``, with its state held in the struct."""
    _fields_ = [("target", C.c_double), ("damping", C.c_double), ("period", C.c_int), ("varying", C.c_int),
                ("shift", C.c_double), ("since", C.c_int), ("n_hist", C.c_double * 64)]

    @classmethod
    def new(cls, target: float, shift: float = 0.0, damping: float = 0.05, period: int = 10,
            started_at: float | None = None) -> "ccmc_shift_control":
        """A fresh control; with `started_at` (an N_tot) it is already varying from that step."""
        c = cls(target=target, damping=damping, period=period, varying=0, shift=shift, since=0)
        if started_at is not None:
            c.varying = 1
            c.n_hist[0] = started_at
        return c


class ccmc_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_uint64), ("ms", C.c_double), ("bytes", C.c_double),
                ("items", C.c_double)]


EXPORTED = ["ccmc_options_default", "ccmc_init", "ccmc_step", "ccmc_step_noalloc", "ccmc_step_batch", "ccmc_energy", "ccmc_free",
            "ccmc_last_error",
            "ccmc_export_size", "ccmc_export", "ccmc_import", "ccmc_spawns_size", "ccmc_export_spawns",
            "ccmc_profile", "ccmc_profile_read", "ccmc_dims", "ccmc_memory", "ccmc_set_budget",
            "ccmc_codistribution", "ccmc_shift_update", "ccmc_run"]

_lib = None
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def lib():
    """Load libccmc.so (built in-tree by ``__graft_entry__.build()``); raise if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, st = C.c_void_p, C.c_int
        sig = {
            "ccmc_options_default": (st, [C.POINTER(ccmc_options)]),
            "ccmc_init": (st, [C.POINTER(ccmc_system), C.POINTER(ccmc_integrals), C.c_int, C.POINTER(ccmc_options),
                               C.POINTER(vp)]),
            "ccmc_step": (st, [vp, C.c_double, C.c_double, C.c_uint64, C.POINTER(ccmc_stats)]),
            "ccmc_step_noalloc": (st, [vp, C.c_double, C.c_double, C.c_uint64, C.POINTER(ccmc_stats)]),
            "ccmc_step_batch": (st, [C.POINTER(vp), C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_uint64), C.POINTER(ccmc_stats)]),
            "ccmc_energy": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
            "ccmc_free": (None, [vp]),
            "ccmc_last_error": (C.c_char_p, [vp]),
            "ccmc_export_size": (st, [vp, C.POINTER(C.c_uint64)]),
            "ccmc_export": (st, [vp, _u64p, _f64p, C.c_uint64, C.POINTER(C.c_uint64), C.POINTER(C.c_double),
                                 C.POINTER(C.c_uint64)]),
            "ccmc_import": (st, [vp, _u64p, _f64p, C.c_uint64, C.c_double, C.c_uint64]),
            "ccmc_spawns_size": (st, [vp, C.POINTER(C.c_uint64)]),
            "ccmc_export_spawns": (st, [vp, _u64p, _f64p, _u64p, C.c_uint64, C.POINTER(C.c_uint64)]),
            "ccmc_profile": (st, [vp, C.c_char_p]),
            "ccmc_profile_read": (st, [vp, C.POINTER(ccmc_kernel_time), C.c_int, C.POINTER(C.c_int)]),
            "ccmc_memory": (st, [vp, C.POINTER(C.c_uint64)]),
            "ccmc_set_budget": (st, [vp, C.c_uint64]),
            "ccmc_dims": (st, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "ccmc_codistribution": (st, [C.c_int, _u64p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p,
                                         C.c_int, _u64p, _u64p]),
            "ccmc_shift_update": (st, [C.POINTER(ccmc_shift_control), C.c_double, C.c_double]),
            "ccmc_run": (st, [vp, C.c_int, C.c_double, C.POINTER(ccmc_shift_control), C.POINTER(C.c_uint64),
                              C.POINTER(ccmc_stats), C.POINTER(C.c_int)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def options(**kw) -> ccmc_options:
    o = ccmc_options()
    lib().ccmc_options_default(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = CCMC_FP32 if v.lower() == "fp32" else CCMC_FP64
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


CCMC_EINVAL_STATUS = -1
CCMC_ENOMEM_STATUS = -2


class State:
    """One CCMC calculation resident on the GPU (wraps ``ccmc_state*``)."""

    def __init__(self, system: str, n_electrons: int, truncation: int, *, n2_max: int = 0, rs: float = 1.0,
                 h: np.ndarray | None = None, chol: np.ndarray | None = None, eri: np.ndarray | None = None,
                 e_core: float = 0.0, **opts):
        self._h = None
        sysc = ccmc_system()
        sysc.kind = CCMC_UEG if system == "ueg" else CCMC_MOLECULAR
        sysc.n_electrons = n_electrons
        sysc.rs = rs
        sysc.n2_max = n2_max
        ints = None
        self._keep = []
        if system != "ueg":
            h = np.ascontiguousarray(h, np.float64)
            dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None
            chol = np.ascontiguousarray(chol, np.float64) if chol is not None else None
            eri = np.ascontiguousarray(eri, np.float64) if eri is not None else None
            self._keep += [h, chol, eri]
            ints = ccmc_integrals(h.shape[0], dp(h), dp(chol), chol.shape[0] if chol is not None else 0, dp(eri),
                                  float(e_core))
            sysc.n_spin_orbitals = 2 * h.shape[0]
        self.options = options(**opts)
        handle = C.c_void_p()
        rc = lib().ccmc_init(C.byref(sysc), C.byref(ints) if ints is not None else None, truncation,
                             C.byref(self.options), C.byref(handle))
        if rc != 0:
            raise CCMCError(rc, lib().ccmc_last_error(None).decode())
        self._h = handle
        self.system = sysc
        self.truncation = truncation
        self.n_electrons, self.n_spin_orbitals, self.n_words = self.ccmc_dims()

    def _check(self, rc: int):
        if rc != 0:
            raise CCMCError(rc, lib().ccmc_last_error(self._h).decode())

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.ccmc_free(self._h)
        self._h = None

    def __del__(self):
        self.close()

    # ------------------------------------------------------------------- C ABI calls
    def ccmc_step(self, tau: float, shift: float, n_attempts: int) -> dict:
        out = ccmc_stats()
        self._check(lib().ccmc_step(self._h, float(tau), float(shift), int(n_attempts), C.byref(out)))
        return out.as_dict()

    step = ccmc_step

    def ccmc_step_noalloc(self, tau: float, shift: float, n_attempts: int) -> dict:
        """ccmc_step without any allocation: the step area is the GPU's fixed array and the
        state's buffers must already be large enough (CCMC_ENOMEM otherwise)."""
        out = ccmc_stats()
        self._check(lib().ccmc_step_noalloc(self._h, float(tau), float(shift), int(n_attempts), C.byref(out)))
        return out.as_dict()

    def ccmc_run(self, n_steps: int, tau: float, ctl: ccmc_shift_control, n_attempts: int):
        """`n_steps` steps in the library's own loop under the population control `ctl`
        (updated in place).  Returns the per-step statistics (a ctypes array of ccmc_stats)
        and the next step's selection count."""
        out = (ccmc_stats * max(n_steps, 1))()
        n = C.c_uint64(int(n_attempts))
        done = C.c_int(0)
        rc = lib().ccmc_run(self._h, int(n_steps), float(tau), C.byref(ctl), C.byref(n), out, C.byref(done))
        self._check(rc)
        return out, n.value

    run = ccmc_run

    def ccmc_energy(self):
        e, n, d = C.c_double(), C.c_double(), C.c_double()
        self._check(lib().ccmc_energy(self._h, C.byref(e), C.byref(n), C.byref(d)))
        return e.value, n.value, d.value

    energy = ccmc_energy

    def ccmc_dims(self):
        ne, M, W = C.c_int(), C.c_int(), C.c_int()
        self._check(lib().ccmc_dims(self._h, C.byref(ne), C.byref(M), C.byref(W)))
        return ne.value, M.value, W.value

    def ccmc_import(self, keys: np.ndarray, amps: np.ndarray, n_ref: float, step: int = 0):
        keys = np.ascontiguousarray(np.asarray(keys, np.uint64).reshape(-1, self.n_words))
        amps = np.ascontiguousarray(amps, np.float64)
        k = keys.ravel() if keys.size else np.zeros(1, np.uint64)
        a = amps if amps.size else np.zeros(1, np.float64)
        self._check(lib().ccmc_import(self._h, k, a, len(amps), float(n_ref), int(step)))

    import_state = ccmc_import

    def ccmc_export(self):
        n = C.c_uint64()
        self._check(lib().ccmc_export_size(self._h, C.byref(n)))
        m = max(n.value, 1)
        keys = np.zeros((m, self.n_words), np.uint64)
        amps = np.zeros(m, np.float64)
        n_ref, step, got = C.c_double(), C.c_uint64(), C.c_uint64()
        self._check(lib().ccmc_export(self._h, keys.ravel(), amps, m, C.byref(got), C.byref(n_ref), C.byref(step)))
        return keys[: got.value], amps[: got.value], n_ref.value, step.value

    export_state = ccmc_export

    def ccmc_export_spawns(self):
        n = C.c_uint64()
        self._check(lib().ccmc_spawns_size(self._h, C.byref(n)))
        m = max(n.value, 1)
        keys = np.zeros((m, self.n_words), np.uint64)
        amps = np.zeros(m, np.float64)
        ids = np.zeros(m, np.uint64)
        got = C.c_uint64()
        self._check(lib().ccmc_export_spawns(self._h, keys.ravel(), amps, ids, m, C.byref(got)))
        return keys[: got.value], amps[: got.value], ids[: got.value]

    records = ccmc_export_spawns

    def ccmc_profile(self, kernels="*"):
        """Time launches with HIP events: "*" every launch, a comma-separated list of kernel
        names, or None / False to stop."""
        if kernels is True:
            kernels = "*"
        arg = kernels.encode() if kernels else None
        self._check(lib().ccmc_profile(self._h, arg))

    def ccmc_profile_read(self) -> dict:
        buf = (ccmc_kernel_time * 64)()
        n = C.c_int()
        self._check(lib().ccmc_profile_read(self._h, buf, 64, C.byref(n)))
        return {buf[i].name.decode(): dict(launches=buf[i].launches, ms=buf[i].ms, bytes=buf[i].bytes,
                                           items=buf[i].items) for i in range(n.value)}

    def ccmc_set_budget(self, hbm_budget_bytes: int):
        self._check(lib().ccmc_set_budget(self._h, int(hbm_budget_bytes)))
        self.options.hbm_budget_bytes = int(hbm_budget_bytes)

    def ccmc_memory(self) -> int:
        b = C.c_uint64()
        self._check(lib().ccmc_memory(self._h, C.byref(b)))
        return b.value


def ccmc_step_batch(states, tau, shift, n_attempts):
    """One step of every state in shared launches (``ccmc_step_batch``).  Returns a list with
    each state's statistics dict, or the CCMCError of that state when its step failed (the
    state is then unchanged); raises on invalid arguments."""
    n = len(states)
    if n == 0:
        return []
    hs = (C.c_void_p * n)(*[s_._h for s_ in states])
    ta = (C.c_double * n)(*[float(x) for x in tau])
    sa = (C.c_double * n)(*[float(x) for x in shift])
    na = (C.c_uint64 * n)(*[int(x) for x in n_attempts])
    outs = (ccmc_stats * n)()
    rc = lib().ccmc_step_batch(hs, n, ta, sa, na, outs)
    if rc == CCMC_EINVAL_STATUS:
        raise CCMCError(rc, "; ".join(filter(None, (lib().ccmc_last_error(h).decode() for h in hs))) or
                        "ccmc_step_batch: invalid arguments")
    res = []
    for i, st in enumerate(states):
        own = outs[i].status  # each state's own outcome
        res.append(CCMCError(own, lib().ccmc_last_error(hs[i]).decode()) if own != 0 else outs[i].as_dict())
    return res


def ccmc_shift_update(ctl: ccmc_shift_control, n_total: float, tau: float) -> float:
    """The library's control update after a step ending at N_tot = n_total (host only)."""
    rc = lib().ccmc_shift_update(C.byref(ctl), float(n_total), float(tau))
    if rc != 0:
        raise CCMCError(rc, "ccmc_shift_update: bad control or population")
    return ctl.shift


def ccmc_codistribution(keys, n_ranks: int, move_shift: int, hash_seed: int, checkpoints):
    """Co-location sums of the placement over iterations 0 .. T-1 (``ccmc_codistribution``):
    for each checkpoint, the sums over pairs i < j of c_ij and c_ij^2."""
    keys = np.ascontiguousarray(np.asarray(keys, np.uint64))
    if keys.ndim != 2:
        raise ValueError("keys must be [n][n_words]")
    cp = np.ascontiguousarray(checkpoints, np.uint64)
    s1 = np.zeros(len(cp), np.uint64)
    s2 = np.zeros(len(cp), np.uint64)
    kk = keys.ravel() if keys.size else np.zeros(1, np.uint64)
    rc = lib().ccmc_codistribution(keys.shape[1], kk, keys.shape[0], int(n_ranks), int(move_shift), int(hash_seed), cp,
                                   len(cp), s1, s2)
    if rc != 0:
        raise CCMCError(rc, lib().ccmc_last_error(None).decode())
    return s1, s2
