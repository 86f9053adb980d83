"""ctypes binding of libpamc.so (the C ABI declared in include/pamc.h).

Argument marshalling only: every step of the method runs in the library's
gfx950 kernels.  The module-level functions carry the C names; ``Instance``
is a thin owner object around a ``pamc_instance*``.  Importing this module
without the built library raises immediately -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpamc.so")

PAMC_OK, PAMC_ERR_INVALID_ARG, PAMC_ERR_OUT_OF_MEMORY, PAMC_ERR_DEVICE, PAMC_ERR_STATE, \
    PAMC_ERR_UNSUPPORTED = range(6)
HEATBATH, METROPOLIS = 0, 1
MAXCUT, ISING = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
FLAG_FIXED_CLASS_ORDER = 1
FLAG_FIELDS_PUSH = 2
FLAG_FIELDS_PULL = 4
POTTS_SOFTMAX, POTTS_CASCADE = 0, 1

EXPORTED = [
    "pamc_create_instance_csr", "pamc_create_instance_dense_i8", "pamc_create_instance_dense_random",
    "pamc_create_instance_max3cut", "pamc_create_instance_potts", "pamc_destroy_instance", "pamc_reset_population", "pamc_get_info", "pamc_anneal",
    "pamc_sweep", "pamc_resample", "pamc_cluster_move", "pamc_update_best", "pamc_best",
    "pamc_get_state", "pamc_get_trace", "pamc_max3cut_decode", "pamc_pair_distance",
    "pamc_profile_enable", "pamc_profile_read", "pamc_synchronize", "pamc_last_error",
    "pamc_set_state", "pamc_checkpoint_size", "pamc_get_checkpoint", "pamc_set_checkpoint", "pamc_autotune",
    "pamc_pair_distance_hist", "pamc_get_dh_trace",
    "pamc_anneal_batch", "pamc_anneal_batch_noalloc", "pamc_server_create", "pamc_server_submit",
    "pamc_server_tick",
    "pamc_server_drain", "pamc_server_poll", "pamc_server_latency", "pamc_server_forget",
    "pamc_server_destroy", "pamc_server_get_stats",
]


class PamcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pamc status {status}: {msg}")
        self.status = status


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class pamc_allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class pamc_config(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("replicas", C.c_int32), ("rule", C.c_int32),
                ("device", C.c_int32), ("stream", C.c_void_p), ("flags", C.c_uint32),
                ("alloc", C.c_void_p)]


class Allocator:
    """A pamc_allocator made of two Python callables: alloc(nbytes, stream)
    returning a device pointer as an int (0 or an exception: failure) and
    free(ptr, stream).  It must outlive every instance or server made with
    it (the Instance and Server wrappers keep a reference)."""

    def __init__(self, alloc, free):
        def _alloc(ctx, nbytes, stream):
            try:
                return alloc(int(nbytes), int(stream or 0)) or None
            except Exception:
                return None

        def _free(ctx, ptr, stream):
            free(int(ptr), int(stream or 0))

        self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
        self.struct = pamc_allocator(None, self._cb[0], self._cb[1])

    @property
    def ptr(self):
        return C.cast(C.pointer(self.struct), C.c_void_p)


def torch_allocator(device=0):
    """Device memory from torch's caching allocator, on the stream the
    library names for each block."""
    import torch
    return Allocator(lambda n, s: torch.cuda.caching_allocator_alloc(n, device, s),
                     lambda p, s: torch.cuda.caching_allocator_delete(p))


def _alloc_ptr(allocator):
    return allocator.ptr if allocator is not None else None


class pamc_info(C.Structure):
    _fields_ = [("n", C.c_int32), ("replicas", C.c_int32), ("num_classes", C.c_int32),
                ("dense", C.c_int32), ("pull", C.c_int32), ("nnz", C.c_int64), ("W", C.c_int64), ("X", C.c_int64),
                ("device_bytes", C.c_int64), ("tiles_per_wave", C.c_int32), ("quads_per_wave", C.c_int32),
                ("coupling_mode", C.c_int32), ("potts_K", C.c_int32), ("tile_sweeps", C.c_int32),
                ("hubs", C.c_int32)]


class pamc_schedule(C.Structure):
    _fields_ = [("beta0", C.c_double), ("dbeta", C.c_double), ("steps", C.c_int32),
                ("sweeps", C.c_int32), ("z_rst", C.c_int32), ("augmented", C.c_int32),
                ("resample", C.c_int32), ("win_short", C.c_int32), ("win_long", C.c_int32),
                ("max_distinct_short", C.c_int32), ("max_distinct_long", C.c_int32),
                ("reheat", C.c_double), ("tau", C.c_int32), ("n_top", C.c_int32),
                ("mis_trials", C.c_int32), ("target", C.c_int64), ("stop_at_target", C.c_int32),
                ("literal_break", C.c_int32), ("resume", C.c_int32), ("dh_every", C.c_int32)]


class pamc_result(C.Structure):
    _fields_ = [("best_cut", C.c_int64), ("best_energy", C.c_int64), ("steps_run", C.c_int32),
                ("step_reached", C.c_int32), ("sum_lnq", C.c_double),
                ("n_cluster_moves", C.c_int32), ("n_reheats", C.c_int32),
                ("n_reversals", C.c_int32), ("n_restarts", C.c_int32),
                ("seconds_total", C.c_double), ("seconds_to_target", C.c_double)]


class pamc_tune_result(C.Structure):
    _fields_ = [("tile_sweeps", C.c_int32), ("tiles_per_wave", C.c_int32), ("quads_per_wave", C.c_int32),
                ("candidates", C.c_int32), ("cached", C.c_int32), ("best_ms_per_sweep", C.c_double),
                ("default_ms_per_sweep", C.c_double)]


class pamc_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("finished", C.c_int64), ("failed", C.c_int64), ("ticks", C.c_int64),
                ("steps", C.c_int64), ("request_steps", C.c_int64), ("prep_seconds", C.c_double),
                ("admit_seconds", C.c_double), ("step_seconds", C.c_double), ("peak_active", C.c_int64),
                ("peak_bytes", C.c_int64), ("in_use_bytes", C.c_int64), ("active", C.c_int64),
                ("queued", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def schedule(**kw) -> pamc_schedule:
    """Algorithm 1 inputs with the paper's controller constants as defaults
    (windows 25/40, at most 3 / 5 distinct values, reheat factor 0.8)."""
    s = pamc_schedule(beta0=0.1, dbeta=0.02, steps=10, sweeps=1, z_rst=0, augmented=0, resample=1,
                      win_short=25, win_long=40, max_distinct_short=3, max_distinct_long=5,
                      reheat=0.8, tau=25, n_top=1, mis_trials=4, target=2**62, stop_at_target=0,
                      literal_break=0, resume=0, dh_every=0)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _load():
    # torch first, when it is installed: it ships its own HIP runtime, and
    # loaded first that runtime also serves this library, so the process has
    # one runtime and torch's memory and streams are usable by the library
    # (PAMC_NO_TORCH=1 skips this: the library then uses the HIP runtime it
    # was built against, for tools that must not load a second one)
    if os.environ.get("PAMC_NO_TORCH", "0") != "1":
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    PP = C.POINTER(C.c_void_p)
    st = C.c_int
    L.pamc_last_error.restype = C.c_char_p
    sig = {
        "pamc_create_instance_csr": [C.c_int32, P, P, P, C.c_int, C.c_int32, C.POINTER(pamc_config), PP],
        "pamc_create_instance_dense_i8": [C.c_int32, P, C.c_int64, C.c_int, C.c_int32, C.POINTER(pamc_config), PP],
        "pamc_create_instance_dense_random": [C.c_int32, C.c_uint64, C.POINTER(pamc_config), PP],
        "pamc_create_instance_max3cut": [C.c_int32, P, P, P, C.POINTER(pamc_config), PP],
        "pamc_create_instance_potts": [C.c_int32, P, P, P, C.c_int32, C.c_int32, C.c_double,
                                       C.POINTER(pamc_config), PP],
        "pamc_get_info": [P, C.POINTER(pamc_info)],
        "pamc_reset_population": [P, C.c_uint64],
        "pamc_anneal": [P, C.POINTER(pamc_schedule), C.POINTER(pamc_result)],
        "pamc_sweep": [P, C.c_double, C.c_int32],
        "pamc_resample": [P, C.c_double, P],
        "pamc_cluster_move": [P, C.c_int32, C.c_int32, P],
        "pamc_update_best": [P],
        "pamc_best": [P, P, P, P],
        "pamc_get_state": [P, P, P, P, P],
        "pamc_get_trace": [P, C.c_int32, P, P, P, P, P, P],
        "pamc_max3cut_decode": [P, P, P, P],
        "pamc_pair_distance": [P, P],
        "pamc_profile_enable": [P, C.c_int32],
        "pamc_profile_read": [P, P, P, P, P],
        "pamc_synchronize": [P],
        "pamc_set_state": [P, P, P, P],
        "pamc_autotune": [P, C.c_double, C.c_int32, C.c_int32, C.POINTER(pamc_tune_result)],
        "pamc_pair_distance_hist": [P, C.c_int32, P, P],
        "pamc_get_dh_trace": [P, C.c_int32, P, P],
        "pamc_checkpoint_size": [P, C.POINTER(C.c_int64)],
        "pamc_get_checkpoint": [P, P, C.c_int64],
        "pamc_set_checkpoint": [P, P, C.c_int64],
        "pamc_anneal_batch": [P, P, C.c_int32, P],
        "pamc_anneal_batch_noalloc": [P, P, C.c_int32, P],
        "pamc_server_create": [C.c_int64, C.c_int32, C.POINTER(pamc_config), PP],
        "pamc_server_submit": [P, C.c_int32, P, P, P, C.c_int32, C.c_uint64, C.POINTER(pamc_schedule),
                               C.POINTER(C.c_uint64)],
        "pamc_server_tick": [P, C.c_int32, P, P],
        "pamc_server_drain": [P],
        "pamc_server_poll": [P, C.c_uint64, P, P, P],
        "pamc_server_latency": [P, C.c_uint64, P, P],
        "pamc_server_forget": [P, C.c_uint64],
        "pamc_server_get_stats": [P, C.POINTER(pamc_server_stats)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.pamc_destroy_instance.argtypes = [P]
    L.pamc_destroy_instance.restype = None
    L.pamc_server_destroy.argtypes = [P]
    L.pamc_server_destroy.restype = None
    return L


lib = _load()


def _check(status):
    if status != PAMC_OK:
        raise PamcError(status, lib.pamc_last_error().decode(errors="replace"))


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


# ---------------------------------------------------------------- C names
def pamc_create_instance_csr(n, row_ptr, col, w, objective=MAXCUT, *, seed=0, replicas=64,
                             rule=HEATBATH, device=0, stream=None, flags=0, allocator=None):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    cl = np.ascontiguousarray(col, np.int32)
    ww = np.ascontiguousarray(w, np.int32)
    cfg = pamc_config(seed, replicas, rule, device, stream, flags, _alloc_ptr(allocator))
    h = C.c_void_p()
    _check(lib.pamc_create_instance_csr(int(n), _ptr(rp), _ptr(cl), _ptr(ww), MEM_HOST, objective,
                                        C.byref(cfg), C.byref(h)))
    return h


def pamc_create_instance_dense_i8(J, objective=ISING, *, seed=0, replicas=64, rule=HEATBATH,
                                  device=0, stream=None, flags=0, allocator=None):
    J = np.ascontiguousarray(J, np.int8)
    cfg = pamc_config(seed, replicas, rule, device, stream, flags, _alloc_ptr(allocator))
    h = C.c_void_p()
    _check(lib.pamc_create_instance_dense_i8(int(J.shape[0]), _ptr(J), int(J.shape[1]), MEM_HOST,
                                             objective, C.byref(cfg), C.byref(h)))
    return h


def pamc_create_instance_dense_random(n, graph_seed, *, seed=0, replicas=64, rule=HEATBATH,
                                      device=0, stream=None, flags=0, allocator=None):
    cfg = pamc_config(seed, replicas, rule, device, stream, flags, _alloc_ptr(allocator))
    h = C.c_void_p()
    _check(lib.pamc_create_instance_dense_random(int(n), int(graph_seed), C.byref(cfg), C.byref(h)))
    return h


def pamc_create_instance_potts(n, row_ptr, col, w, K, potts_rule=POTTS_SOFTMAX, gamma=1.0, *, seed=0,
                               replicas=64, device=0, stream=None, flags=0, allocator=None):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    cl = np.ascontiguousarray(col, np.int32)
    ww = np.ascontiguousarray(w, np.int32)
    cfg = pamc_config(seed, replicas, HEATBATH, device, stream, flags, _alloc_ptr(allocator))
    h = C.c_void_p()
    _check(lib.pamc_create_instance_potts(int(n), _ptr(rp), _ptr(cl), _ptr(ww), int(K), int(potts_rule),
                                          float(gamma), C.byref(cfg), C.byref(h)))
    return h


def pamc_create_instance_max3cut(n, row_ptr, col, w, *, seed=0, replicas=64, rule=HEATBATH,
                                 device=0, stream=None, flags=0, allocator=None):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    cl = np.ascontiguousarray(col, np.int32)
    ww = np.ascontiguousarray(w, np.int32)
    cfg = pamc_config(seed, replicas, rule, device, stream, flags, _alloc_ptr(allocator))
    h = C.c_void_p()
    _check(lib.pamc_create_instance_max3cut(int(n), _ptr(rp), _ptr(cl), _ptr(ww), C.byref(cfg), C.byref(h)))
    return h


def pamc_destroy_instance(h):
    lib.pamc_destroy_instance(h)


def pamc_reset_population(h, seed):
    _check(lib.pamc_reset_population(h, int(seed)))


def pamc_get_info(h) -> pamc_info:
    info = pamc_info()
    _check(lib.pamc_get_info(h, C.byref(info)))
    return info


def pamc_anneal(h, sched: pamc_schedule) -> pamc_result:
    res = pamc_result()
    _check(lib.pamc_anneal(h, C.byref(sched), C.byref(res)))
    return res


def pamc_sweep(h, beta, nsweeps=1):
    _check(lib.pamc_sweep(h, float(beta), int(nsweeps)))


def pamc_resample(h, delta, want_log_q=True):
    q = C.c_double()
    _check(lib.pamc_resample(h, float(delta), C.byref(q) if want_log_q else None))
    return q.value if want_log_q else None


def pamc_cluster_move(h, n_top, mis_trials, want_flipped=True):
    f = C.c_int32()
    _check(lib.pamc_cluster_move(h, int(n_top), int(mis_trials), C.byref(f) if want_flipped else None))
    return f.value if want_flipped else None


def pamc_update_best(h):
    _check(lib.pamc_update_best(h))


def pamc_best(h, n):
    cut, en = C.c_int64(), C.c_int64()
    spins = np.zeros(n, np.int8)
    _check(lib.pamc_best(h, C.byref(cut), C.byref(en), _ptr(spins)))
    return cut.value, en.value, spins


def pamc_get_state(h, n, R):
    s = np.zeros((R, n), np.int8)
    f = np.zeros((R, n), np.int32)
    E = np.zeros(R, np.int64)
    fam = np.zeros(R, np.int32)
    _check(lib.pamc_get_state(h, _ptr(s), _ptr(f), _ptr(E), _ptr(fam)))
    return s, f, E, fam


def pamc_get_trace(h, capacity):
    m = np.zeros(capacity, np.int64)
    b = np.zeros(capacity, np.float64)
    q = np.zeros(capacity, np.float64)
    ev = np.zeros(capacity, np.int32)
    t = np.zeros(capacity, np.float64)
    k = C.c_int32()
    _check(lib.pamc_get_trace(h, int(capacity), _ptr(m), _ptr(b), _ptr(q), _ptr(ev), _ptr(t), C.byref(k)))
    k = k.value
    return {"mstar": m[:k], "beta": b[:k], "lnq": q[:k], "events": ev[:k], "seconds": t[:k]}


def pamc_max3cut_decode(h, m3_n, spins=None):
    labels = np.zeros(m3_n, np.int32)
    cut = C.c_int64()
    sp = np.ascontiguousarray(spins, np.int8) if spins is not None else None
    _check(lib.pamc_max3cut_decode(h, _ptr(sp), _ptr(labels), C.byref(cut)))
    return cut.value, labels


def pamc_pair_distance(h):
    d = C.c_double()
    _check(lib.pamc_pair_distance(h, C.byref(d)))
    return d.value


def pamc_profile_enable(h, on=True):
    _check(lib.pamc_profile_enable(h, int(bool(on))))


def pamc_profile_read(h):
    ms, la, at, fl = C.c_double(), C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib.pamc_profile_read(h, C.byref(ms), C.byref(la), C.byref(at), C.byref(fl)))
    return {"ms": ms.value, "launches": la.value, "attempts": at.value, "flips": fl.value}


def pamc_synchronize(h):
    _check(lib.pamc_synchronize(h))


def pamc_pair_distance_hist(h, nbins):
    counts = np.zeros(int(nbins), np.int64)
    mean = C.c_double()
    _check(lib.pamc_pair_distance_hist(h, int(nbins), _ptr(counts), C.byref(mean)))
    return counts, mean.value


def pamc_get_dh_trace(h, capacity):
    dh = np.zeros(int(capacity), np.float64)
    k = C.c_int32()
    _check(lib.pamc_get_dh_trace(h, int(capacity), _ptr(dh), C.byref(k)))
    return dh[:k.value]


def pamc_autotune(h, beta, sweeps=4, force=False) -> pamc_tune_result:
    r = pamc_tune_result()
    _check(lib.pamc_autotune(h, float(beta), int(sweeps), int(bool(force)), C.byref(r)))
    return r


def pamc_set_state(h, spins, family=None, counters=None):
    sp = np.ascontiguousarray(spins, np.int8)
    fa = None if family is None else np.ascontiguousarray(family, np.int32)
    co = None if counters is None else np.ascontiguousarray(counters, np.uint32)
    _check(lib.pamc_set_state(h, _ptr(sp), _ptr(fa), _ptr(co)))


def pamc_get_checkpoint(h) -> bytes:
    size = C.c_int64()
    _check(lib.pamc_checkpoint_size(h, C.byref(size)))
    buf = np.zeros(size.value, np.uint8)
    _check(lib.pamc_get_checkpoint(h, _ptr(buf), size.value))
    return buf.tobytes()


def pamc_set_checkpoint(h, blob: bytes):
    buf = np.frombuffer(blob, np.uint8).copy()
    _check(lib.pamc_set_checkpoint(h, _ptr(buf), buf.size))


def pamc_anneal_batch(handles, scheds):
    """One batched run over several instances (one schedule each)."""
    k = len(handles)
    if len(scheds) != k:
        raise ValueError("one schedule per instance")
    hs = (C.c_void_p * k)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    ss = (pamc_schedule * k)(*scheds)
    rs = (pamc_result * k)()
    _check(lib.pamc_anneal_batch(C.cast(hs, C.c_void_p), C.cast(ss, C.c_void_p), k, C.cast(rs, C.c_void_p)))
    return list(rs)


def pamc_anneal_batch_noalloc(handles, scheds):
    """pamc_anneal_batch without device allocation (fixed device scratch)."""
    k = len(handles)
    if len(scheds) != k:
        raise ValueError("one schedule per instance")
    hs = (C.c_void_p * k)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    ss = (pamc_schedule * k)(*scheds)
    rs = (pamc_result * k)()
    _check(lib.pamc_anneal_batch_noalloc(C.cast(hs, C.c_void_p), C.cast(ss, C.c_void_p), k,
                                         C.cast(rs, C.c_void_p)))
    return list(rs)


def pamc_server_create(hbm_budget_bytes, max_slots, *, replicas=64, rule=HEATBATH, device=0, stream=None,
                       flags=0, allocator=None):
    cfg = pamc_config(0, replicas, rule, device, stream, flags, _alloc_ptr(allocator))
    h = C.c_void_p()
    _check(lib.pamc_server_create(int(hbm_budget_bytes), int(max_slots), C.byref(cfg), C.byref(h)))
    return h


def pamc_server_submit(srv, n, row_ptr, col, w, objective, seed, sched):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    cl = np.ascontiguousarray(col, np.int32)
    ww = np.ascontiguousarray(w, np.int32)
    t = C.c_uint64()
    _check(lib.pamc_server_submit(srv, int(n), _ptr(rp), _ptr(cl), _ptr(ww), int(objective), int(seed),
                                  C.byref(sched), C.byref(t)))
    return t.value


def pamc_server_tick(srv, max_steps=0):
    a, q = C.c_int32(), C.c_int32()
    _check(lib.pamc_server_tick(srv, int(max_steps), C.byref(a), C.byref(q)))
    return a.value, q.value


def pamc_server_drain(srv):
    _check(lib.pamc_server_drain(srv))


def pamc_server_poll(srv, ticket, n=None):
    d = C.c_int32()
    res = pamc_result()
    spins = np.zeros(n, np.int8) if n is not None else None
    _check(lib.pamc_server_poll(srv, int(ticket), C.byref(d), C.byref(res), _ptr(spins)))
    if not d.value:
        return None
    return (res, spins) if n is not None else res


def pamc_server_latency(srv, ticket):
    q, t = C.c_double(), C.c_double()
    _check(lib.pamc_server_latency(srv, int(ticket), C.byref(q), C.byref(t)))
    return q.value, t.value


def pamc_server_forget(srv, ticket):
    _check(lib.pamc_server_forget(srv, int(ticket)))


def pamc_server_get_stats(srv):
    st = pamc_server_stats()
    _check(lib.pamc_server_get_stats(srv, C.byref(st)))
    return st.as_dict()


def pamc_server_destroy(srv):
    lib.pamc_server_destroy(srv)


# ---------------------------------------------------------------- owner object
class Instance:
    """Owns one ``pamc_instance*``; methods forward to the C functions."""

    def __init__(self, handle, n, replicas, m3_n=0, allocator=None):
        self.h = handle
        self.n = int(n)
        self.R = int(replicas)
        self.m3_n = m3_n
        self.allocator = allocator  # kept alive while the instance exists

    @classmethod
    def csr(cls, g, *, replicas, seed, rule=HEATBATH, objective=MAXCUT, shuffle=True, stream=None, fields=None,
            allocator=None):
        flags = 0 if shuffle else FLAG_FIXED_CLASS_ORDER
        flags |= {None: 0, "push": FLAG_FIELDS_PUSH, "pull": FLAG_FIELDS_PULL}[fields]
        h = pamc_create_instance_csr(g.n, g.row_ptr, g.col, g.w, objective, seed=seed, replicas=replicas,
                                     rule=rule, stream=stream, flags=flags, allocator=allocator)
        return cls(h, g.n, replicas, allocator=allocator)

    @classmethod
    def max3cut(cls, g, *, replicas, seed, rule=HEATBATH, shuffle=True, stream=None, fields=None):
        flags = 0 if shuffle else FLAG_FIXED_CLASS_ORDER
        flags |= {None: 0, "push": FLAG_FIELDS_PUSH, "pull": FLAG_FIELDS_PULL}[fields]
        h = pamc_create_instance_max3cut(g.n, g.row_ptr, g.col, g.w, seed=seed, replicas=replicas, rule=rule,
                                         stream=stream, flags=flags)
        return cls(h, 3 * g.n + 1, replicas, m3_n=g.n)

    @classmethod
    def potts(cls, g, K, *, replicas, seed, potts_rule=POTTS_SOFTMAX, gamma=1.0, shuffle=True, stream=None):
        flags = 0 if shuffle else FLAG_FIXED_CLASS_ORDER
        h = pamc_create_instance_potts(g.n, g.row_ptr, g.col, g.w, K, potts_rule, gamma, seed=seed,
                                       replicas=replicas, stream=stream, flags=flags)
        return cls(h, g.n, replicas)

    @classmethod
    def dense(cls, J, *, replicas, seed, rule=HEATBATH, objective=ISING, stream=None):
        h = pamc_create_instance_dense_i8(J, objective, seed=seed, replicas=replicas, rule=rule, stream=stream)
        return cls(h, J.shape[0], replicas)

    @classmethod
    def dense_random(cls, n, graph_seed, *, replicas, seed, rule=HEATBATH, stream=None, allocator=None):
        h = pamc_create_instance_dense_random(n, graph_seed, seed=seed, replicas=replicas, rule=rule,
                                              stream=stream, allocator=allocator)
        return cls(h, n, replicas, allocator=allocator)

    def close(self):
        if self.h:
            pamc_destroy_instance(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return pamc_get_info(self.h)

    def reset(self, seed):
        pamc_reset_population(self.h, seed)

    def anneal(self, sched):
        return pamc_anneal(self.h, sched)

    def sweep(self, beta, nsweeps=1):
        pamc_sweep(self.h, beta, nsweeps)

    def resample(self, delta):
        return pamc_resample(self.h, delta)

    def cluster_move(self, n_top, mis_trials):
        return pamc_cluster_move(self.h, n_top, mis_trials)

    def update_best(self):
        pamc_update_best(self.h)

    def best(self):
        return pamc_best(self.h, self.n)

    def state(self):
        return pamc_get_state(self.h, self.n, self.R)

    def trace(self, capacity):
        return pamc_get_trace(self.h, capacity)

    def max3cut_decode(self, spins=None):
        return pamc_max3cut_decode(self.h, self.m3_n, spins)

    def pair_distance(self):
        return pamc_pair_distance(self.h)

    def pair_distance_hist(self, nbins):
        return pamc_pair_distance_hist(self.h, nbins)

    def dh_trace(self, capacity):
        return pamc_get_dh_trace(self.h, capacity)

    def autotune(self, beta, sweeps=4, force=False):
        return pamc_autotune(self.h, beta, sweeps, force)

    def set_state(self, spins, family=None, counters=None):
        pamc_set_state(self.h, spins, family, counters)

    def checkpoint(self) -> bytes:
        return pamc_get_checkpoint(self.h)

    def restore(self, blob: bytes):
        pamc_set_checkpoint(self.h, blob)

    def synchronize(self):
        pamc_synchronize(self.h)


def anneal_batch(instances, scheds):
    """Batched run of several ``Instance`` objects; returns their results."""
    return pamc_anneal_batch([i.h for i in instances], scheds)


def anneal_batch_noalloc(instances, scheds):
    """``anneal_batch`` through the entry point that allocates no device memory."""
    return pamc_anneal_batch_noalloc([i.h for i in instances], scheds)


class Server:
    """Owns one ``pamc_server*`` (continuous batching of annealing requests)."""

    def __init__(self, hbm_budget_bytes, max_slots, *, replicas, rule=HEATBATH, device=0, stream=None,
                 fields=None, allocator=None):
        flags = {None: 0, "push": FLAG_FIELDS_PUSH, "pull": FLAG_FIELDS_PULL}[fields]
        self.allocator = allocator
        self.h = pamc_server_create(hbm_budget_bytes, max_slots, replicas=replicas, rule=rule, device=device,
                                    stream=stream, flags=flags, allocator=allocator)
        self.sizes = {}

    def submit(self, g, seed, sched, objective=MAXCUT):
        t = pamc_server_submit(self.h, g.n, g.row_ptr, g.col, g.w, objective, seed, sched)
        self.sizes[t] = g.n
        return t

    def tick(self, max_steps=0):
        return pamc_server_tick(self.h, max_steps)

    def drain(self):
        pamc_server_drain(self.h)

    def poll(self, ticket, spins=False):
        return pamc_server_poll(self.h, ticket, self.sizes[ticket] if spins else None)

    def latency(self, ticket):
        return pamc_server_latency(self.h, ticket)

    def forget(self, ticket):
        pamc_server_forget(self.h, ticket)

    def stats(self):
        return pamc_server_get_stats(self.h)

    def close(self):
        if self.h:
            pamc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
