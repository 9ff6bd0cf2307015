"""ctypes wrapper of the plain C oracle (pcpd_oracle.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use this module. The product path never imports it.

Every function here is marshalling only; the arithmetic lives in
pcpd_oracle.c, which documents the paper passage each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcpd_oracle.c")
_LIB = os.path.join(_HERE, "libpcpd_oracle.so")

MODEL_N = {"dp": 1, "pcpd": 2, "tcpd": 3, "qcpd": 4}
INIT_KIND = {"full": 0, "empty": 1, "host": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over independent units)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-Wall",
             "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("B", ctypes.c_uint32),
        ("L", ctypes.c_uint64),
        ("seed", ctypes.c_uint32),
        ("stream", ctypes.c_uint32),
        ("plane", ctypes.c_uint32),
        ("p", ctypes.c_double),
        ("d", ctypes.c_double),
        ("samples", ctypes.c_uint64),
        ("init", ctypes.c_int32),
        ("init_words", ctypes.POINTER(ctypes.c_uint64)),
        ("t0", ctypes.c_uint64),
        ("n_times", ctypes.c_uint32),
        ("times", ctypes.POINTER(ctypes.c_uint64)),
        ("words_out", ctypes.POINTER(ctypes.c_uint64)),
        ("n_out", ctypes.POINTER(ctypes.c_uint64)),
        ("pair_out", ctypes.POINTER(ctypes.c_uint64)),
        ("connected", ctypes.c_int32),
        ("mask_bits", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u32, u64 = ctypes.c_uint32, ctypes.c_uint64
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(u32), ctypes.POINTER(u32),
                                        ctypes.POINTER(u32)]
        L.orc_philox4x32_10.restype = None
        L.orc_threshold.argtypes = [ctypes.c_double]
        L.orc_threshold.restype = u64
        L.orc_decide.argtypes = [u64, u64, u32, u64, ctypes.c_int]
        L.orc_decide.restype = ctypes.c_int
        L.orc_threshold_m.argtypes = [ctypes.c_double, ctypes.c_int]
        L.orc_threshold_m.restype = u64
        L.orc_decide_m.argtypes = [ctypes.POINTER(u64), ctypes.c_int, u32, u64, ctypes.c_int]
        L.orc_decide_m.restype = ctypes.c_int
        L.orc_offset.argtypes = [u32, u32, u32, u64, u32]
        L.orc_offset.restype = u32
        L.orc_rule_window.argtypes = [ctypes.c_int, u32, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int]
        L.orc_rule_window.restype = u32
        L.orc_simulate.argtypes = [ctypes.POINTER(_Params)]
        L.orc_simulate.restype = ctypes.c_int
        L.orc_simulate_many.argtypes = [ctypes.POINTER(_Params), ctypes.c_int32,
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.orc_simulate_many.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int32
        L.orc_connected_substep.argtypes = [ctypes.c_int, u32, u64, u32, u32, u32, u64, u64, u64,
                                            ctypes.POINTER(ctypes.c_uint8)]
        L.orc_connected_substep.restype = None
        _lib = L
    return _lib


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def threshold(q: float) -> int:
    return int(lib().orc_threshold(float(q)))


def decide(x1: int, x2: int, g: int, K: int, b: int) -> int:
    return int(lib().orc_decide(x1, x2, g, K, b))


def threshold_m(q: float, m: int) -> int:
    """K = rint(q * 2^(32+m)) for m decorrelation bits (2 or 4)."""
    return int(lib().orc_threshold_m(float(q), int(m)))


def decide_m(xs, g: int, K: int, b: int) -> int:
    """U_b < K with U_b = (bits b of xs[0..m-1], most significant first) * 2^32 + g."""
    arr = (ctypes.c_uint64 * len(xs))(*[int(x) for x in xs])
    return int(lib().orc_decide_m(arr, len(xs), int(g), int(K), int(b)))


def offset(seed: int, stream: int, plane: int, s: int, B: int) -> int:
    return int(lib().orc_offset(seed, stream, plane, s, B))


def rule_window(n: int, window: int, D: int, A: int, R: int) -> int:
    return int(lib().orc_rule_window(n, window, D, A, R))


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


class Run:
    """One (instance, plane) unit: inputs plus the output arrays it fills."""

    def __init__(self, *, model="pcpd", B=64, L, seed=1, stream=0, plane=0, p, d,
                 samples=(1 << 64) - 1, init="full", init_words=None, t0=0, times,
                 connected=False, mask_bits=2):
        self.times = np.ascontiguousarray(np.asarray(times, dtype=np.uint64))
        self.words = np.zeros(int(L), dtype=np.uint64)
        self.n = np.zeros((len(self.times), 64), dtype=np.uint64)
        self.pair = np.zeros((len(self.times), 64), dtype=np.uint64)
        self.init_words = None
        if init == "host":
            self.init_words = np.ascontiguousarray(np.asarray(init_words, dtype=np.uint64))
            assert self.init_words.shape == (int(L),)
        self.samples = int(samples)
        P = _Params()
        P.n = MODEL_N[model] if isinstance(model, str) else int(model)
        P.B = int(B)
        P.L = int(L)
        P.seed = int(seed)
        P.stream = int(stream)
        P.plane = int(plane)
        P.p = float(p)
        P.d = float(d)
        P.samples = self.samples
        P.init = INIT_KIND[init]
        P.init_words = _ptr(self.init_words) if self.init_words is not None else None
        P.t0 = int(t0)
        P.n_times = len(self.times)
        P.times = _ptr(self.times)
        P.words_out = _ptr(self.words)
        P.n_out = _ptr(self.n)
        P.pair_out = _ptr(self.pair)
        P.connected = 1 if connected else 0
        P.mask_bits = int(mask_bits)
        self.params = P

    # aggregated observables over the simulated samples, per record
    def counts(self):
        """(N, N_pair, alive) per record, summed over the simulated samples."""
        N = self.n.sum(axis=1, dtype=np.uint64)
        NP = self.pair.sum(axis=1, dtype=np.uint64)
        alive = np.zeros(len(self.times), dtype=np.uint64)
        for b in range(64):
            alive |= (self.n[:, b] > 0).astype(np.uint64) << np.uint64(b)
        return N, NP, alive


def connected_substep(model, B, L, seed, stream, plane, p, d, s, sites):
    """One substep s on a joined ring of 64 L sites given as a uint8 array
    (global site order); returns the new array."""
    q = np.ascontiguousarray(np.asarray(sites, dtype=np.uint8)).copy()
    assert q.shape == (64 * int(L),)
    n = MODEL_N[model] if isinstance(model, str) else int(model)
    lib().orc_connected_substep(n, int(B), int(L), int(seed), int(stream), int(plane),
                                threshold(d), threshold(p), int(s),
                                q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return q


def simulate(run: Run) -> Run:
    rc = lib().orc_simulate(ctypes.byref(run.params))
    if rc != 0:
        raise ValueError(f"oracle rejected the run (status {rc})")
    return run


def simulate_many(runs, n_threads: int = 0):
    arr = (_Params * len(runs))(*[r.params for r in runs])
    status = (ctypes.c_int32 * len(runs))()
    rc = lib().orc_simulate_many(arr, len(runs), int(n_threads), status)
    if rc != 0:
        raise ValueError(f"oracle rejected a run (status {rc})")
    return runs


def max_threads() -> int:
    return int(lib().orc_max_threads())
