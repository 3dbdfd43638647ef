"""Python handle on the CPU oracle (oracle/ea_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the library.  The oracle stores
one spin per byte and shares no code with the HIP path; see ea_oracle.c for
the definition it implements and the paper sections each step follows.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libea_oracle.so")

MAX_TEMPS = 64

_i8p = ctypes.POINTER(ctypes.c_int8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)


class _OrcSim(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int), ("n_T", ctypes.c_int), ("R", ctypes.c_int), ("rng", ctypes.c_int),
        ("seed", ctypes.c_uint64), ("t", ctypes.c_int64),
        ("rid", _i32p), ("J", _i8p), ("betas", _f64p),
        ("spins", _i8p), ("temp_of_slot", _i32p), ("Urun", _i64p),
        ("flip_tries", _i64p), ("flip_acc", _i64p),
        ("swap_tries", _i64p), ("swap_acc", _i64p),
        ("h", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _build
            _build.build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_flip_threshold.argtypes = [ctypes.c_double, ctypes.c_int]
        L.orc_flip_threshold.restype = ctypes.c_uint32
        L.orc_flip_draw.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_int, ctypes.c_int]
        L.orc_flip_draw.restype = ctypes.c_uint32
        L.orc_swap_threshold.argtypes = [ctypes.c_double, ctypes.c_int64]
        L.orc_swap_threshold.restype = ctypes.c_uint32
        L.orc_n_phases.argtypes = [ctypes.c_int]
        L.orc_n_phases.restype = ctypes.c_int
        L.orc_colour.argtypes = [ctypes.c_int] * 4
        L.orc_colour.restype = ctypes.c_int
        L.orc_local_unsat.argtypes = [ctypes.c_int, _i8p, _i8p, ctypes.c_int]
        L.orc_local_unsat.restype = ctypes.c_int
        L.orc_unsat_bonds.argtypes = [ctypes.c_int, _i8p, _i8p]
        L.orc_unsat_bonds.restype = ctypes.c_int64
        for name in ("orc_init", "orc_reset_running_energy"):
            getattr(L, name).argtypes = [ctypes.POINTER(_OrcSim)]
            getattr(L, name).restype = None
        L.orc_sweep.argtypes = [ctypes.POINTER(_OrcSim), ctypes.c_int64, ctypes.c_int]
        L.orc_sweep.restype = ctypes.c_int
        L.orc_observables.argtypes = [ctypes.POINTER(_OrcSim), _i32p, _i32p]
        L.orc_observables.restype = None
        L.orc_measure.argtypes = [ctypes.POINTER(_OrcSim), _i64p, _i64p, ctypes.POINTER(ctypes.c_uint64), _i64p]
        L.orc_measure.restype = None
        L.orc_magnetization.argtypes = [ctypes.POINTER(_OrcSim), _i32p]
        L.orc_magnetization.restype = None
        L.orc_flip_threshold_h.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_flip_threshold_h.restype = ctypes.c_uint32
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


RNG_WORDS, RNG_PLANES = 0, 1
RNGS = {"words": RNG_WORDS, "planes": RNG_PLANES}


def flip_draw(seed, rng, i, t, r, c, slot):
    """The flip draw of (realization id r, copy c, slot, sweep t, site i)."""
    return int(lib().orc_flip_draw(int(seed) & (2 ** 64 - 1), RNGS.get(rng, rng), int(i), int(t), int(r), int(c),
                                   int(slot)))


def flip_threshold_h(beta, u, S, h):
    """Threshold of a flip with cost 12 - 4u + 2h(2S - 1) (2^32 - 1 when the cost is <= 0)."""
    return int(lib().orc_flip_threshold_h(float(beta), int(u), int(S), float(h)))


def flip_threshold(beta, u):
    return int(lib().orc_flip_threshold(float(beta), int(u)))


def swap_threshold(dbeta_abs, n):
    return int(lib().orc_swap_threshold(float(dbeta_abs), int(n)))


def n_phases(L):
    return int(lib().orc_n_phases(int(L)))


def colour(L, x, y, z):
    return int(lib().orc_colour(int(L), int(x), int(y), int(z)))


def unsat_bonds(L, J, s):
    J = np.ascontiguousarray(J, dtype=np.int8)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return int(lib().orc_unsat_bonds(int(L), _ptr(J, ctypes.c_int8), _ptr(s, ctypes.c_int8)))


def local_unsat(L, J, s, i):
    J = np.ascontiguousarray(J, dtype=np.int8)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return int(lib().orc_local_unsat(int(L), _ptr(J, ctypes.c_int8), _ptr(s, ctypes.c_int8), int(i)))


class OracleSim:
    """State of R realizations x 2 copies x n_T slots, one spin per byte.

    couplings: int8 [R][N][3] in {+1,-1}; betas: float64 [n_T];
    rid: realization ids (Philox counter word 2), default 0..R-1.
    """

    def __init__(self, L, couplings, betas, seed, rid=None, track_energy=False, stats=False, rng="words", h=0.0):
        self.L = int(L)
        self.N = self.L ** 3
        self.J = np.ascontiguousarray(couplings, dtype=np.int8)
        assert self.J.ndim == 3 and self.J.shape[1:] == (self.N, 3)
        self.R = self.J.shape[0]
        self.betas = np.ascontiguousarray(betas, dtype=np.float64)
        self.n_T = len(self.betas)
        assert 1 <= self.n_T <= MAX_TEMPS
        self.rid = np.ascontiguousarray(np.arange(self.R) if rid is None else rid, dtype=np.int32)
        assert self.rid.shape == (self.R,)
        self.seed = int(seed) & (2 ** 64 - 1)
        self.spins = np.zeros((self.R, 2, self.n_T, self.N), dtype=np.int8)
        self.temp_of_slot = np.zeros((self.R, 2, self.n_T), dtype=np.int32)
        self.Urun = np.zeros((self.R, 2, self.n_T), dtype=np.int64) if track_energy else None
        if stats:
            self.flip_tries = np.zeros((self.n_T, 7), dtype=np.int64)
            self.flip_acc = np.zeros((self.n_T, 7), dtype=np.int64)
            self.swap_tries = np.zeros(max(self.n_T - 1, 1), dtype=np.int64)
            self.swap_acc = np.zeros(max(self.n_T - 1, 1), dtype=np.int64)
        else:
            self.flip_tries = self.flip_acc = self.swap_tries = self.swap_acc = None
        self._s = _OrcSim()
        s = self._s
        self.rng = RNGS.get(rng, rng)
        assert self.rng in (RNG_WORDS, RNG_PLANES)
        s.L, s.n_T, s.R, s.seed, s.t, s.rng = self.L, self.n_T, self.R, self.seed, 0, self.rng
        self.h = float(h)
        assert abs(self.h) <= 8.0 and self.h * 4.0 == round(self.h * 4.0), "h must be a multiple of 1/4 in [-8, 8]"
        s.h = self.h
        s.rid = _ptr(self.rid, ctypes.c_int32)
        s.J = _ptr(self.J, ctypes.c_int8)
        s.betas = _ptr(self.betas, ctypes.c_double)
        s.spins = _ptr(self.spins, ctypes.c_int8)
        s.temp_of_slot = _ptr(self.temp_of_slot, ctypes.c_int32)
        s.Urun = _ptr(self.Urun, ctypes.c_int64) if self.Urun is not None else None
        for name in ("flip_tries", "flip_acc", "swap_tries", "swap_acc"):
            a = getattr(self, name)
            setattr(s, name, _ptr(a, ctypes.c_int64) if a is not None else None)
        lib().orc_init(ctypes.byref(s))

    @property
    def t(self):
        return int(self._s.t)

    def set_state(self, spins, temp_of_slot, t):
        self.spins[...] = np.asarray(spins, dtype=np.int8)
        self.temp_of_slot[...] = np.asarray(temp_of_slot, dtype=np.int32)
        self._s.t = int(t)
        lib().orc_reset_running_energy(ctypes.byref(self._s))

    def sweep(self, n_sweeps, swap_every):
        rc = lib().orc_sweep(ctypes.byref(self._s), int(n_sweeps), int(swap_every))
        if rc != 0:
            raise RuntimeError(f"oracle sweep failed with status {rc}")

    def observables(self):
        energy = np.zeros((self.R, 2, self.n_T), dtype=np.int32)
        overlap = np.zeros((self.R, self.n_T), dtype=np.int32)
        lib().orc_observables(ctypes.byref(self._s), _ptr(energy, ctypes.c_int32), _ptr(overlap, ctypes.c_int32))
        return energy, overlap

    def magnetization(self):
        """sum_i s_i [R][2][n_T] by temperature index."""
        m = np.zeros((self.R, 2, self.n_T), dtype=np.int32)
        lib().orc_magnetization(ctypes.byref(self._s), _ptr(m, ctypes.c_int32))
        return m

    def new_measurements(self):
        """Zeroed accumulators: count, sum_q2 [R][n_T], sum_q4 [R][n_T][2] (lo, hi), sum_c [R][n_T][L]."""
        return (np.zeros((self.R, self.n_T), np.int64), np.zeros((self.R, self.n_T), np.int64),
                np.zeros((self.R, self.n_T, 2), np.uint64), np.zeros((self.R, self.n_T, self.L), np.int64))

    def measure(self, acc):
        """Add one measurement of the current state into `acc` (from new_measurements)."""
        count, q2, q4, c = acc
        lib().orc_measure(ctypes.byref(self._s), _ptr(count, ctypes.c_int64), _ptr(q2, ctypes.c_int64),
                          _ptr(q4, ctypes.c_uint64), _ptr(c, ctypes.c_int64))
        return acc


def binder_and_xi(acc, L):
    """Spin-glass Binder ratio g = (3 - [<q^4>] / [<q^2>]^2) / 2 and correlation
    length over L per temperature index from measurement accumulators; [.] is
    the average over realizations.  xi = sqrt(chi(0) / chi(k) - 1) / (2 sin(k / 2))
    with k = 2 pi / L along each axis, chi(0) = [<q^2>] / N and chi(k) the
    axis-averaged [<|sum_i q_i e^{i k x}|^2>] / N = [<sum_d C[d] cos(k d)>] / (3 N);
    nan where chi(0) / chi(k) < 1."""
    count, q2, q4, c = acc
    N = L ** 3
    n = count.astype(np.float64)
    m2 = (q2 / n).mean(axis=0)
    q4v = q4[..., 0].astype(np.float64) + q4[..., 1].astype(np.float64) * 2.0 ** 64
    m4 = (q4v / n).mean(axis=0)
    g = 0.5 * (3.0 - m4 / (m2 * m2))
    k = 2.0 * math.pi / L
    w = np.cos(k * np.arange(L))
    chik = ((c @ w) / n / (3.0 * N)).mean(axis=0)
    chi0 = m2 / N
    ratio = chi0 / chik
    xi = np.where(ratio >= 1.0, np.sqrt(np.maximum(ratio - 1.0, 0.0)) / (2.0 * math.sin(k / 2.0)), np.nan)
    return g, xi / L
