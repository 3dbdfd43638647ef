"""ctypes binding over the C ABI in include/ea.h (argument marshalling only).

Every step of the simulation runs in the HIP kernels of libea_mi355x.so; this
module converts numpy arrays to pointers and back.  When torch with a GPU is
available, device memory comes from torch's caching allocator and the work
runs on a torch stream; otherwise the library's own hipMalloc and the default
stream are used.  A missing library is an error, never a fallback.
"""
import atexit
import ctypes
import os
import re
import weakref

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libea_mi355x.so")
HEADER = os.path.join(ROOT, "include", "ea.h")

EA_OK, EA_EINVAL, EA_ENOMEM, EA_EDEVICE, EA_ESTATE, EA_EBUSY = 0, -1, -2, -3, -4, -5
LAYOUT_CAMSC, LAYOUT_AMSC4 = 0, 1
LAYOUT_AMSC3, LAYOUT_AMSC1 = 2, 3
LAYOUTS = {"camsc": LAYOUT_CAMSC, "amsc4": LAYOUT_AMSC4, "amsc3": LAYOUT_AMSC3, "amsc1": LAYOUT_AMSC1}
RNG_WORDS, RNG_PLANES = 0, 1
RNGS = {"words": RNG_WORDS, "planes": RNG_PLANES}
MAX_TEMPS = 64

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [
        ("layout", ctypes.c_int), ("block_threads", ctypes.c_int),
        ("words_resident", ctypes.c_int), ("split", ctypes.c_int), ("rng", ctypes.c_int),
        ("field", ctypes.c_double), ("stream", ctypes.c_void_p),
        ("dev_alloc", _ALLOC_FN), ("dev_free", _FREE_FN), ("alloc_ctx", ctypes.c_void_p),
        ("site_order", ctypes.c_int),
    ]


class PlanOptions(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int), ("autotune", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("reserved_", ctypes.c_int), ("stream", ctypes.c_void_p)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("quantum_sweeps", ctypes.c_int), ("layout", ctypes.c_int),
                ("max_active", ctypes.c_int), ("autotune", ctypes.c_int), ("keep_state", ctypes.c_int),
                ("rng", ctypes.c_int), ("policy", ctypes.c_int), ("fill_ladders", ctypes.c_int),
                ("pack_rounds", ctypes.c_int), ("stream", ctypes.c_void_p)]


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_CANCELLED, JOB_FAILED = 0, 1, 2, 3, 4


class EAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def lib():
    """Open libea_mi355x.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i8p, i32p, i64p = (ctypes.POINTER(t) for t in (ctypes.c_int8, ctypes.c_int32, ctypes.c_int64))
        u32p, u64p, f64p = (ctypes.POINTER(t) for t in (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double))
        sig = {
            "ea_default_options": (None, [ctypes.POINTER(Options)]),
            "ea_create": (ctypes.c_int, [ctypes.c_int, i8p, f64p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.POINTER(Options), ctypes.POINTER(P)]),
            "ea_sweep": (ctypes.c_int, [P, ctypes.c_int64, ctypes.c_int]),
            "ea_sweep_batch": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, i64p, i32p]),
            "ea_sweep_batch_noalloc": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, i64p, i32p]),
            "ea_observables": (ctypes.c_int, [P, i32p, i32p]),
            "ea_state": (ctypes.c_int, [P, i8p, i32p, i64p]),
            "ea_set_state": (ctypes.c_int, [P, i8p, i32p, ctypes.c_int64]),
            "ea_swap_acceptance": (ctypes.c_int, [P, u64p]),
            "ea_get_dims": (ctypes.c_int, [P, i32p, i32p, i32p, i32p]),
            "ea_destroy": (None, [P]),
            "ea_last_error": (ctypes.c_char_p, []),
            "ea_flip_thresholds": (ctypes.c_int, [f64p, ctypes.c_int, u32p]),
            "ea_swap_threshold": (ctypes.c_uint32, [ctypes.c_double, ctypes.c_int64]),
            "ea_version": (ctypes.c_char_p, []),
            "ea_default_plan_options": (None, [ctypes.POINTER(PlanOptions)]),
            "ea_plan_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, ctypes.c_int, i32p,
                                              ctypes.POINTER(PlanOptions), ctypes.POINTER(P)]),
            "ea_plan_run": (ctypes.c_int, [P, ctypes.c_int64]),
            "ea_plan_info": (ctypes.c_int, [P, i32p, i32p, i32p, ctypes.POINTER(ctypes.c_size_t), i32p, i32p]),
            "ea_plan_destroy": (None, [P]),
            "ea_default_server_options": (None, [ctypes.POINTER(ServerOptions)]),
            "ea_server_create": (ctypes.c_int, [ctypes.POINTER(ServerOptions), ctypes.POINTER(P)]),
            "ea_server_submit": (ctypes.c_int, [P, ctypes.c_int, i8p, f64p, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, i64p]),
            "ea_server_step": (ctypes.c_int, [P, i32p, i32p, i32p]),
            "ea_server_status": (ctypes.c_int, [P, ctypes.c_int64, i32p, i64p]),
            "ea_server_result": (ctypes.c_int, [P, ctypes.c_int64, i32p, i32p]),
            "ea_server_final_state": (ctypes.c_int, [P, ctypes.c_int64, i8p, i32p]),
            "ea_server_cancel": (ctypes.c_int, [P, ctypes.c_int64]),
            "ea_server_release": (ctypes.c_int, [P, ctypes.c_int64]),
            "ea_server_stats": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                               i64p, i64p, i64p]),
            "ea_server_destroy": (None, [P]),
            "ea_job_footprint": (ctypes.c_int, [ctypes.c_int, f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_size_t)]),
            "ea_sim_footprint": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
            "ea_sim_info": (ctypes.c_int, [P, i32p, i32p, i32p, ctypes.POINTER(ctypes.c_size_t)]),
            "ea_sim_split": (ctypes.c_int, [P, i32p, i32p]),
            "ea_measure": (ctypes.c_int, [P]),
            "ea_magnetization": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int32)]),
            "ea_measure_read": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int64)]),
            "ea_measure_reset": (ctypes.c_int, [P]),
            "ea_binder_xi": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions():
    """Names of the functions include/ea.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ea_[a-z_0-9]+)\s*\(", text, re.M)))


def last_error():
    return lib().ea_last_error().decode()


def check(rc):
    if rc != EA_OK:
        raise EAError(rc, last_error())


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def flip_thresholds(betas):
    b = np.ascontiguousarray(betas, dtype=np.float64)
    out = np.zeros((len(b), 3), dtype=np.uint32)
    check(lib().ea_flip_thresholds(_p(b, ctypes.c_double), len(b), _p(out, ctypes.c_uint32)))
    return out


def swap_threshold(dbeta_abs, n):
    return int(lib().ea_swap_threshold(float(dbeta_abs), int(n)))


# Live handles, closed in dependency order (servers, plans, then jobs) when
# the interpreter exits, while torch and this module are still intact: a
# handle's device memory may come from torch's caching allocator, whose
# callbacks must not run during interpreter teardown.
_LIVE = {"server": weakref.WeakSet(), "plan": weakref.WeakSet(), "sim": weakref.WeakSet()}


@atexit.register
def _close_live_handles():
    for kind in ("server", "plan", "sim"):
        for h in list(_LIVE[kind]):
            h.close()


class TorchAllocator:
    """Device memory for the library from torch's caching allocator."""

    def __init__(self, device=0):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self.alloc_cb = _ALLOC_FN(self._alloc)
        self.free_cb = _FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=f"cuda:{self.device}")
        except Exception:   # out of memory: the library reports EA_ENOMEM
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, ctx):
        self.live.pop(ptr, None)


def _torch_gpu():
    try:
        import torch
        return torch if torch.cuda.is_available() else None
    except Exception:
        return None


class Sim:
    """One job: R realizations x 2 copies x n_T temperature slots on the GPU.

    layout: "camsc" (default), "amsc4", "amsc3", "amsc1"; rng: "words" or
    "planes"; split: True/"auto" (the library's choice), False/"never",
    "always" (whenever the job allows: by lattice halves for two parts, else
    by slot groups), "slots" (whenever possible, by slot groups only);
    site_order: "natural" or "by_class"; h: the external field (a multiple
    of 1/4); allocator: an object with ctypes callbacks alloc_cb / free_cb
    (default torch's caching allocator when torch sees a GPU).  info()
    reports the launch: block_threads, words_resident, split_parts,
    lds_bytes, split_by_halves."""

    def __init__(self, L, couplings, betas, seed, layout="camsc", block_threads=0, words_resident=0,
                 stream=None, torch_memory=True, split=True, rng="words", h=0.0, site_order="natural",
                 allocator=None):
        L = int(L)
        J = np.ascontiguousarray(couplings, dtype=np.int8)
        if J.ndim != 3 or J.shape[1:] != (L ** 3, 3):
            raise ValueError(f"couplings must have shape [R][{L ** 3}][3]")
        b = np.ascontiguousarray(betas, dtype=np.float64)
        opt = Options()
        lib().ea_default_options(ctypes.byref(opt))
        opt.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
        opt.block_threads = int(block_threads)
        opt.words_resident = int(words_resident)
        # True/"auto": library choice; False: one workgroup per ladder; "always": split when possible
        # "slots": whenever possible, by slot groups only (not by lattice halves)
        opt.split = {True: 0, "auto": 0, False: 1, "never": 1, "always": 2, "slots": 3}[split]
        opt.rng = RNGS[rng] if isinstance(rng, str) else int(rng)
        opt.field = float(h)
        opt.site_order = {"natural": 0, "by_class": 1}[site_order] if isinstance(site_order, str) else int(site_order)
        # allocator: an object with ctypes callbacks alloc_cb / free_cb (TorchAllocator's
        # interface); default torch's caching allocator when torch sees a GPU, else hipMalloc
        self._alloc = allocator
        torch = _torch_gpu() if (torch_memory or stream is not None) else None
        if stream is not None:
            opt.stream = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        if self._alloc is None and torch is not None and torch_memory:
            self._alloc = TorchAllocator(torch.cuda.current_device())
        if self._alloc is not None:
            opt.dev_alloc = self._alloc.alloc_cb
            opt.dev_free = self._alloc.free_cb
        self.stream = stream
        self.L, self.N, self.R, self.n_T = L, L ** 3, J.shape[0], len(b)
        self.layout = opt.layout
        self._h = ctypes.c_void_p()
        check(lib().ea_create(L, _p(J, ctypes.c_int8), _p(b, ctypes.c_double), len(b), J.shape[0],
                              ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), ctypes.byref(opt), ctypes.byref(self._h)))
        _LIVE["sim"].add(self)

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.ea_destroy(self._h)
            self._h = ctypes.c_void_p()

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def sweep(self, n_sweeps, swap_every=1):
        check(lib().ea_sweep(self._h, int(n_sweeps), int(swap_every)))

    def observables(self):
        E = np.zeros((self.R, 2, self.n_T), dtype=np.int32)
        q = np.zeros((self.R, self.n_T), dtype=np.int32)
        check(lib().ea_observables(self._h, _p(E, ctypes.c_int32), _p(q, ctypes.c_int32)))
        return E, q

    def state(self):
        s = np.zeros((self.R, 2, self.n_T, self.N), dtype=np.int8)
        perm = np.zeros((self.R, 2, self.n_T), dtype=np.int32)
        t = ctypes.c_int64()
        check(lib().ea_state(self._h, _p(s, ctypes.c_int8), _p(perm, ctypes.c_int32), ctypes.byref(t)))
        return s, perm, int(t.value)

    def set_state(self, spins, temp_of_slot, sweeps_done):
        s = np.ascontiguousarray(spins, dtype=np.int8)
        p = np.ascontiguousarray(temp_of_slot, dtype=np.int32)
        check(lib().ea_set_state(self._h, _p(s, ctypes.c_int8), _p(p, ctypes.c_int32), int(sweeps_done)))

    def magnetization(self):
        """sum_i s_i [R][2][n_T] by temperature index."""
        m = np.zeros((self.R, 2, self.n_T), np.int32)
        check(lib().ea_magnetization(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return m

    def measure(self):
        """Add one measurement of the current state to the device accumulators."""
        check(lib().ea_measure(self._h))

    def measurements(self):
        """(count, sum_q2 [R][n_T], sum_q4 [R][n_T][2] uint64 lo/hi, sum_c [R][n_T][L])."""
        R, n_T, L = self.R, self.n_T, self.L
        count = np.zeros((R, n_T), np.int64)
        q2 = np.zeros((R, n_T), np.int64)
        q4 = np.zeros((R, n_T, 2), np.uint64)
        c = np.zeros((R, n_T, L), np.int64)
        check(lib().ea_measure_read(self._h, count.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    q2.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    q4.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return count, q2, q4, c

    def reset_measurements(self):
        check(lib().ea_measure_reset(self._h))

    def binder_xi(self):
        """Binder ratio and xi / L per temperature index."""
        g = np.zeros(self.n_T, np.float64)
        x = np.zeros(self.n_T, np.float64)
        check(lib().ea_binder_xi(self._h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return g, x

    def info(self):
        bt, wr, parts = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lds = ctypes.c_size_t()
        check(lib().ea_sim_info(self._h, ctypes.byref(bt), ctypes.byref(wr), ctypes.byref(parts), ctypes.byref(lds)))
        halves = ctypes.c_int()
        check(lib().ea_sim_split(self._h, None, ctypes.byref(halves)))
        return dict(block_threads=bt.value, words_resident=wr.value, split_parts=parts.value, lds_bytes=int(lds.value),
                    split_by_halves=bool(halves.value))

    def footprint(self):
        b = ctypes.c_size_t()
        check(lib().ea_sim_footprint(self._h, ctypes.byref(b)))
        return int(b.value)

    def swap_acceptance(self):
        a = np.zeros((self.R, 2, max(self.n_T - 1, 0)), dtype=np.uint64)
        check(lib().ea_swap_acceptance(self._h, _p(a, ctypes.c_uint64)))
        return a


def sweep_batch(sims, n_sweeps, swap_every):
    """One launch over several jobs; n_sweeps / swap_every are per-job lists."""
    n = len(sims)
    hs = (ctypes.c_void_p * n)(*[s.handle.value for s in sims])
    ns = np.ascontiguousarray(n_sweeps, dtype=np.int64)
    se = np.ascontiguousarray(swap_every, dtype=np.int32)
    check(lib().ea_sweep_batch(hs, n, _p(ns, ctypes.c_int64), _p(se, ctypes.c_int32)))


def sweep_batch_noalloc(sims, n_sweeps, swap_every):
    """sweep_batch through the entry point that allocates no device memory
    (its launch arrays live in the library's static per-device workspace)."""
    n = len(sims)
    hs = (ctypes.c_void_p * n)(*[s.handle.value for s in sims])
    ns = np.ascontiguousarray(n_sweeps, dtype=np.int64)
    se = np.ascontiguousarray(swap_every, dtype=np.int32)
    check(lib().ea_sweep_batch_noalloc(hs, n, _p(ns, ctypes.c_int64), _p(se, ctypes.c_int32)))


def job_footprint(L, betas, n_realizations, layout="camsc"):
    """Device bytes a job of this shape needs (host-only)."""
    b = np.ascontiguousarray(betas, dtype=np.float64)
    out = ctypes.c_size_t()
    lay = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
    check(lib().ea_job_footprint(int(L), _p(b, ctypes.c_double), len(b), int(n_realizations), lay, ctypes.byref(out)))
    return int(out.value)


class Plan:
    """One step (sweeps_per_step sweeps of every job) captured in a hipGraph and replayed."""

    def __init__(self, sims, sweeps_per_step, swap_every, block_threads=0, autotune=True, use_graph=True,
                 stream=None):
        self.sims = list(sims)
        n = len(self.sims)
        hs = (ctypes.c_void_p * n)(*[x.handle.value for x in self.sims])
        se = np.ascontiguousarray(swap_every if np.ndim(swap_every) else [swap_every] * n, dtype=np.int32)
        opt = PlanOptions()
        lib().ea_default_plan_options(ctypes.byref(opt))
        opt.block_threads, opt.autotune, opt.use_graph = int(block_threads), int(bool(autotune)), int(bool(use_graph))
        if stream is not None:
            opt.stream = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        self._h = ctypes.c_void_p()
        check(lib().ea_plan_create(hs, n, int(sweeps_per_step), _p(se, ctypes.c_int32), ctypes.byref(opt),
                                   ctypes.byref(self._h)))
        _LIVE["plan"].add(self)

    def run(self, n_steps=1):
        check(lib().ea_plan_run(self._h, int(n_steps)))

    def info(self):
        bt, grid, units, g, parts = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lds = ctypes.c_size_t()
        check(lib().ea_plan_info(self._h, ctypes.byref(bt), ctypes.byref(grid), ctypes.byref(units),
                                 ctypes.byref(lds), ctypes.byref(g), ctypes.byref(parts)))
        return dict(block_threads=bt.value, grid=grid.value, units=units.value, lds_bytes=int(lds.value),
                    uses_graph=bool(g.value), split_parts=parts.value)

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.ea_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    __del__ = close


class Server:
    """Continuous-batching job server (see ea_server_* in include/ea.h)."""

    def __init__(self, hbm_budget_bytes=0, quantum_sweeps=400, layout="camsc", max_active=0, autotune=False,
                 keep_state=False, rng="words", policy="ratio", fill_ladders=0, pack_rounds=True):
        opt = ServerOptions()
        lib().ea_default_server_options(ctypes.byref(opt))
        opt.hbm_budget_bytes = int(hbm_budget_bytes)
        opt.quantum_sweeps = int(quantum_sweeps)
        opt.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
        opt.max_active = int(max_active)
        opt.autotune = int(bool(autotune))
        opt.keep_state = int(bool(keep_state))
        opt.rng = RNGS[rng] if isinstance(rng, str) else int(rng)
        opt.policy = {"fifo": 0, "shortest": 1, "ratio": 2}[policy] if isinstance(policy, str) else int(policy)
        opt.fill_ladders = int(fill_ladders)
        opt.pack_rounds = int(bool(pack_rounds))
        self._h = ctypes.c_void_p()
        self.shapes = {}
        check(lib().ea_server_create(ctypes.byref(opt), ctypes.byref(self._h)))
        _LIVE["server"].add(self)

    def submit(self, L, couplings, betas, seed, n_sweeps, swap_every=1):
        J = np.ascontiguousarray(couplings, dtype=np.int8)
        b = np.ascontiguousarray(betas, dtype=np.float64)
        jid = ctypes.c_int64()
        check(lib().ea_server_submit(self._h, int(L), _p(J, ctypes.c_int8), _p(b, ctypes.c_double), len(b),
                                     J.shape[0], ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), int(n_sweeps),
                                     int(swap_every), ctypes.byref(jid)))
        self.shapes[jid.value] = (int(L), J.shape[0], len(b))
        return jid.value

    def step(self):
        r, q, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().ea_server_step(self._h, ctypes.byref(r), ctypes.byref(q), ctypes.byref(f)))
        return r.value, q.value, f.value

    def status(self, jid):
        st, done = ctypes.c_int(), ctypes.c_int64()
        check(lib().ea_server_status(self._h, int(jid), ctypes.byref(st), ctypes.byref(done)))
        return st.value, done.value

    def result(self, jid):
        L, R, n_T = self.shapes[jid]
        E = np.zeros((R, 2, n_T), dtype=np.int32)
        q = np.zeros((R, n_T), dtype=np.int32)
        check(lib().ea_server_result(self._h, int(jid), _p(E, ctypes.c_int32), _p(q, ctypes.c_int32)))
        return E, q

    def final_state(self, jid):
        L, R, n_T = self.shapes[jid]
        s = np.zeros((R, 2, n_T, L ** 3), dtype=np.int8)
        p = np.zeros((R, 2, n_T), dtype=np.int32)
        check(lib().ea_server_final_state(self._h, int(jid), _p(s, ctypes.c_int8), _p(p, ctypes.c_int32)))
        return s, p

    def cancel(self, jid):
        check(lib().ea_server_cancel(self._h, int(jid)))

    def release(self, jid):
        check(lib().ea_server_release(self._h, int(jid)))
        self.shapes.pop(jid, None)

    def stats(self):
        used, budget = ctypes.c_size_t(), ctypes.c_size_t()
        steps, plans, replays = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().ea_server_stats(self._h, ctypes.byref(used), ctypes.byref(budget), ctypes.byref(steps),
                                    ctypes.byref(plans), ctypes.byref(replays)))
        return dict(hbm_used=int(used.value), hbm_budget=int(budget.value), steps=steps.value,
                    plans_built=plans.value, launches_replayed=replays.value)

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.ea_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    __del__ = close
