"""CPU oracle for augmented PAMC -- TEST INFRASTRUCTURE ONLY.

A plain, slow, single-threaded C implementation of the method (pamc_oracle.c)
wrapped with ctypes.  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library and never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "pamc_oracle.c")

TAG_INIT, TAG_SWEEP, TAG_RS, TAG_CL, TAG_ORDER, TAG_DENSE, TAG_POTTS = range(7)
HEATBATH, METROPOLIS = 0, 1
POTTS_SOFTMAX, POTTS_CASCADE = 0, 1
MAXCUT, ISING = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction of a*b+c into fma)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
               "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Schedule(C.Structure):
    _fields_ = [("beta0", C.c_double), ("dbeta", C.c_double),
                ("steps", C.c_int32), ("sweeps", C.c_int32), ("z_rst", C.c_int32),
                ("augmented", C.c_int32), ("resample", C.c_int32),
                ("win_short", C.c_int32), ("win_long", C.c_int32),
                ("max_distinct_short", C.c_int32), ("max_distinct_long", C.c_int32),
                ("reheat", C.c_double), ("tau", C.c_int32), ("n_top", C.c_int32),
                ("mis_trials", C.c_int32), ("target", C.c_int64),
                ("stop_at_target", C.c_int32), ("literal_break", C.c_int32), ("resume", C.c_int32),
                ("dh_every", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("best_cut", C.c_int64), ("best_energy", C.c_int64),
                ("steps_run", C.c_int32), ("step_reached", C.c_int32),
                ("sum_lnq", C.c_double), ("n_cluster_moves", C.c_int32),
                ("n_reheats", C.c_int32), ("n_reversals", C.c_int32),
                ("n_restarts", C.c_int32)]


class Trace(C.Structure):
    _fields_ = [("mstar", C.POINTER(C.c_int64)), ("beta", C.POINTER(C.c_double)),
                ("lnq", C.POINTER(C.c_double)), ("events", C.POINTER(C.c_int32)),
                ("dh", C.POINTER(C.c_double))]


class Ctrl(C.Structure):
    _fields_ = [("beta", C.c_double), ("delta", C.c_double), ("z", C.c_int32),
                ("cycle", C.c_int32), ("cooldown", C.c_int32), ("enable", C.c_int32),
                ("hist_len", C.c_int32), ("stop", C.c_int32), ("hist", C.c_int64 * 64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C")
        L.orc_philox4x32_10.argtypes = [np.ctypeslib.ndpointer(np.uint32), np.ctypeslib.ndpointer(np.uint32),
                                        np.ctypeslib.ndpointer(np.uint32)]
        L.orc_pexp.argtypes = [C.c_double]
        L.orc_pexp.restype = C.c_double
        L.orc_threshold.argtypes = [C.c_double, C.c_int32, C.c_int64]
        L.orc_threshold.restype = C.c_uint32
        L.orc_colour.argtypes = [C.c_int32, i32p, i32p, i32p]
        L.orc_colour.restype = C.c_int32
        L.orc_max3cut_colour.argtypes = [C.c_int32, i32p, i32p, i32p]
        L.orc_max3cut_colour.restype = C.c_int32
        L.orc_dense_random.argtypes = [C.c_int32, C.c_uint64, i8p]
        L.orc_create_sparse.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, C.c_int32,
                                        C.c_uint64, C.c_int32, C.c_int32, C.c_char_p, C.c_int32]
        L.orc_create_sparse.restype = P
        L.orc_create_dense.argtypes = [C.c_int32, i8p, C.c_int32, C.c_int32, C.c_uint64,
                                       C.c_int32, C.c_char_p, C.c_int32]
        L.orc_create_dense.restype = P
        L.orc_create_max3cut.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, C.c_uint64,
                                         C.c_int32, C.c_int32, C.c_char_p, C.c_int32]
        L.orc_create_max3cut.restype = P
        L.orc_create_potts.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, C.c_int32, C.c_uint64,
                                       C.c_int32, C.c_double, C.c_int32, C.c_char_p, C.c_int32]
        L.orc_create_potts.restype = P
        L.orc_potts_energy.argtypes = [P, C.c_int32]
        L.orc_potts_energy.restype = C.c_int64
        L.orc_potts_choose.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double,
                                       np.ctypeslib.ndpointer(np.int64), np.ctypeslib.ndpointer(np.uint32)]
        L.orc_potts_choose.restype = C.c_int32
        L.orc_destroy.argtypes = [P]
        for f, rt in (("orc_n", C.c_int32), ("orc_replicas", C.c_int32),
                      ("orc_num_classes", C.c_int32), ("orc_W", C.c_int64), ("orc_X", C.c_int64)):
            getattr(L, f).argtypes = [P]
            getattr(L, f).restype = rt
        L.orc_internal_ids.argtypes = [P, i32p]
        L.orc_class_ptr.argtypes = [P, i32p]
        L.orc_counters.argtypes = [P, np.ctypeslib.ndpointer(np.uint32)]
        L.orc_sweep.argtypes = [P, C.c_double, C.c_int32]
        L.orc_resample.argtypes = [P, C.c_double, P]
        L.orc_resample.restype = C.c_double
        L.orc_cluster.argtypes = [P, C.c_int32, C.c_int32, P]
        L.orc_cluster.restype = C.c_int32
        L.orc_update_best.argtypes = [P]
        L.orc_update_best.restype = C.c_int64
        L.orc_best.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), P]
        L.orc_get_state.argtypes = [P, P, P, P, P]
        L.orc_anneal.argtypes = [P, C.POINTER(Schedule), C.POINTER(Result), C.POINTER(Trace)]
        L.orc_max3cut_decode.argtypes = [P, i8p, i32p]
        L.orc_max3cut_decode.restype = C.c_int64
        L.orc_max3cut_value.argtypes = [P, i32p]
        L.orc_max3cut_value.restype = C.c_int64
        L.orc_controller_step.argtypes = [C.POINTER(Ctrl), C.POINTER(Schedule), C.c_int64]
        L.orc_controller_step.restype = C.c_int32
        L.orc_mean_pair_distance.argtypes = [P]
        L.orc_mean_pair_distance.restype = C.c_double
        L.orc_set_population.argtypes = [P, i8p, P]
        L.orc_set_population.restype = C.c_int32
        L.orc_set_counters.argtypes = [P, np.ctypeslib.ndpointer(np.uint32)]
        L.orc_pair_distances.argtypes = [P, np.ctypeslib.ndpointer(np.float64)]
        L.orc_checkpoint_size.argtypes = [P]
        L.orc_checkpoint_size.restype = C.c_int64
        L.orc_get_checkpoint.argtypes = [P, np.ctypeslib.ndpointer(np.uint8)]
        L.orc_set_checkpoint.argtypes = [P, np.ctypeslib.ndpointer(np.uint8), C.c_int64]
        L.orc_set_checkpoint.restype = C.c_int32
        _lib = L
    return _lib


# ---------------------------------------------------------------- primitives
def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c, k, out)
    return out


def pexp(x: float) -> float:
    return lib().orc_pexp(float(x))


def threshold(beta: float, rule: int, x: int) -> int:
    return int(lib().orc_threshold(float(beta), int(rule), int(x)))


def colour(n, row_ptr, col):
    out = np.zeros(n, dtype=np.int32)
    k = lib().orc_colour(n, np.ascontiguousarray(row_ptr, np.int32), np.ascontiguousarray(col, np.int32), out)
    return k, out


def max3cut_colour(n, row_ptr, col):
    """The Max-3-Cut embedding's colouring (3n + 1 spins) from the base
    graph (n vertices): (class count, colour per spin)."""
    out = np.zeros(3 * n + 1, dtype=np.int32)
    k = lib().orc_max3cut_colour(n, np.ascontiguousarray(row_ptr, np.int32), np.ascontiguousarray(col, np.int32),
                                 out)
    return k, out


def dense_random(n: int, seed: int) -> np.ndarray:
    J = np.zeros((n, n), dtype=np.int8)
    lib().orc_dense_random(n, seed, J)
    return J


def potts_choose(K: int, rule: int, gamma: float, beta: float, syn, u) -> int:
    """The label one Potts update picks (Eqs. 8-9 or the cascaded sampler)."""
    sv = np.zeros(4, np.int64)
    sv[:K] = np.asarray(syn, np.int64)
    uv = np.zeros(4, np.uint32)
    uv[:len(u)] = np.asarray(u, np.uint32)
    return int(lib().orc_potts_choose(int(K), int(rule), float(gamma), float(beta), sv, uv))


def default_schedule(**kw) -> Schedule:
    s = Schedule(beta0=0.1, dbeta=0.02, steps=10, sweeps=1, z_rst=0, augmented=0, resample=1,
                 win_short=25, win_long=40, max_distinct_short=3, max_distinct_long=5,
                 reheat=0.8, tau=25, n_top=1, mis_trials=4, target=2**62,
                 stop_at_target=0, literal_break=0, resume=0, dh_every=0)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


# ---------------------------------------------------------------- instances
class Oracle:
    """One oracle instance: graph + population of R replicas."""

    def __init__(self, handle, kind):
        if not handle:
            raise ValueError("oracle rejected the instance")
        self._h = handle
        self.kind = kind
        L = lib()
        self.n = L.orc_n(handle)
        self.R = L.orc_replicas(handle)

    @classmethod
    def sparse(cls, n, row_ptr, col, w, replicas, seed, rule=HEATBATH, objective=MAXCUT, shuffle=True):
        err = C.create_string_buffer(256)
        h = lib().orc_create_sparse(int(n), np.ascontiguousarray(row_ptr, np.int32),
                                    np.ascontiguousarray(col, np.int32), np.ascontiguousarray(w, np.int32),
                                    objective, replicas, seed, rule, int(bool(shuffle)), err, 256)
        if not h:
            raise ValueError(err.value.decode())
        return cls(h, "sparse")

    @classmethod
    def dense(cls, J, replicas, seed, rule=HEATBATH, objective=ISING):
        J = np.ascontiguousarray(J, dtype=np.int8)
        err = C.create_string_buffer(256)
        h = lib().orc_create_dense(int(J.shape[0]), J, objective, replicas, seed, rule, err, 256)
        if not h:
            raise ValueError(err.value.decode())
        return cls(h, "dense")

    @classmethod
    def max3cut(cls, n, row_ptr, col, w, replicas, seed, rule=HEATBATH, shuffle=True):
        err = C.create_string_buffer(256)
        h = lib().orc_create_max3cut(int(n), np.ascontiguousarray(row_ptr, np.int32),
                                     np.ascontiguousarray(col, np.int32), np.ascontiguousarray(w, np.int32),
                                     replicas, seed, rule, int(bool(shuffle)), err, 256)
        if not h:
            raise ValueError(err.value.decode())
        o = cls(h, "max3cut")
        o.m3_n = int(n)
        return o

    @classmethod
    def potts(cls, n, row_ptr, col, w, K, replicas, seed, rule=POTTS_SOFTMAX, gamma=1.0, shuffle=True):
        err = C.create_string_buffer(256)
        h = lib().orc_create_potts(int(n), np.ascontiguousarray(row_ptr, np.int32),
                                   np.ascontiguousarray(col, np.int32), np.ascontiguousarray(w, np.int32),
                                   int(K), replicas, seed, int(rule), float(gamma), int(bool(shuffle)), err, 256)
        if not h:
            raise ValueError(err.value.decode())
        o = cls(h, "potts")
        o.K = int(K)
        return o

    def potts_energy(self, r):
        return lib().orc_potts_energy(self._h, int(r))

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    # facts
    @property
    def W(self):
        return lib().orc_W(self._h)

    @property
    def X(self):
        return lib().orc_X(self._h)

    @property
    def num_classes(self):
        return lib().orc_num_classes(self._h)

    def internal_ids(self):
        out = np.zeros(self.n, np.int32)
        lib().orc_internal_ids(self._h, out)
        return out

    def class_ptr(self):
        out = np.zeros(self.num_classes + 1, np.int32)
        lib().orc_class_ptr(self._h, out)
        return out

    def counters(self):
        out = np.zeros(3, np.uint32)
        lib().orc_counters(self._h, out)
        return out

    # steps
    def sweep(self, beta, nsweeps=1):
        lib().orc_sweep(self._h, float(beta), int(nsweeps))

    def resample(self, delta, return_parents=False):
        parents = np.zeros(self.R, np.int32)
        lnq = lib().orc_resample(self._h, float(delta), parents.ctypes.data)
        return (lnq, parents) if return_parents else lnq

    def cluster(self, n_top, mis_trials):
        sizes = np.zeros(max(1, n_top), np.int32)
        tot = lib().orc_cluster(self._h, int(n_top), int(mis_trials), sizes.ctypes.data)
        return tot, sizes[:min(n_top, self.R)]

    def update_best(self):
        return lib().orc_update_best(self._h)

    def best(self):
        cut, en = C.c_int64(), C.c_int64()
        spins = np.zeros(self.n, np.int8)
        lib().orc_best(self._h, C.byref(cut), C.byref(en), spins.ctypes.data)
        return cut.value, en.value, spins

    def state(self):
        s = np.zeros((self.R, self.n), np.int8)
        h = np.zeros((self.R, self.n), np.int32)
        E = np.zeros(self.R, np.int64)
        f = np.zeros(self.R, np.int32)
        lib().orc_get_state(self._h, s.ctypes.data, h.ctypes.data, E.ctypes.data, f.ctypes.data)
        return s, h, E, f

    def anneal(self, sched: Schedule, trace: bool = False):
        res = Result()
        tr = None
        arrays = None
        if trace:
            n = sched.steps
            arrays = (np.zeros(n, np.int64), np.zeros(n, np.float64), np.zeros(n, np.float64),
                      np.zeros(n, np.int32), np.full(n, -1.0))
            tr = Trace(arrays[0].ctypes.data_as(C.POINTER(C.c_int64)),
                       arrays[1].ctypes.data_as(C.POINTER(C.c_double)),
                       arrays[2].ctypes.data_as(C.POINTER(C.c_double)),
                       arrays[3].ctypes.data_as(C.POINTER(C.c_int32)),
                       arrays[4].ctypes.data_as(C.POINTER(C.c_double)))
        lib().orc_anneal(self._h, C.byref(sched), C.byref(res), C.byref(tr) if tr is not None else None)
        if trace:
            return res, {"mstar": arrays[0], "beta": arrays[1], "lnq": arrays[2], "events": arrays[3],
                         "dh": arrays[4]}
        return res

    def max3cut_decode(self, spins):
        labels = np.zeros(self.m3_n, np.int32)
        cut = lib().orc_max3cut_decode(self._h, np.ascontiguousarray(spins, np.int8), labels)
        return cut, labels

    def max3cut_value(self, labels):
        return lib().orc_max3cut_value(self._h, np.ascontiguousarray(labels, np.int32))

    def mean_pair_distance(self):
        return lib().orc_mean_pair_distance(self._h)

    def pair_distances(self):
        out = np.zeros(self.R * (self.R - 1) // 2, np.float64)
        lib().orc_pair_distances(self._h, out)
        return out

    def set_population(self, spins, family=None):
        s = np.ascontiguousarray(spins, np.int8).reshape(self.R, self.n)
        f = None if family is None else np.ascontiguousarray(family, np.int32)
        if lib().orc_set_population(self._h, s, None if f is None else f.ctypes.data) != 0:
            raise ValueError("spin or label out of range")

    def checkpoint(self) -> bytes:
        buf = np.zeros(lib().orc_checkpoint_size(self._h), np.uint8)
        lib().orc_get_checkpoint(self._h, buf)
        return buf.tobytes()

    def restore(self, blob: bytes):
        buf = np.frombuffer(blob, np.uint8).copy()
        if lib().orc_set_checkpoint(self._h, buf, buf.size) != 0:
            raise ValueError("not a checkpoint of this instance")

    def set_counters(self, gs, g_rs, g_cl):
        lib().orc_set_counters(self._h, np.array([gs, g_rs, g_cl], np.uint32))


def controller_step(ctrl: Ctrl, sched: Schedule, mstar: int) -> int:
    return lib().orc_controller_step(C.byref(ctrl), C.byref(sched), int(mstar))
