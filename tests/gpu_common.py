"""Helpers shared by the GPU tests: per-sample observables of packed words
and oracle runs for a GPU context's instances. Test infrastructure only."""
from __future__ import annotations

import numpy as np

from oracle import oracle

MODEL_NAME = {1: "dp", 2: "pcpd", 3: "tcpd", 4: "qcpd"}


def sample_bits(words: np.ndarray) -> np.ndarray:
    """[L, 64] uint8 matrix: bit b of word j."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    return np.unpackbits(w.view(np.uint8).reshape(-1, 8), axis=1, bitorder="little")


def per_sample_counts(words: np.ndarray):
    """(N_b, N_pair_b) for the 64 samples of one plane (ring of len(words))."""
    bits = sample_bits(words).astype(np.int64)
    n = bits.sum(axis=0)
    pair = (bits & np.roll(bits, -1, axis=0)).sum(axis=0)
    return n, pair


def aggregate_counts(words: np.ndarray):
    """(N, N_pair, alive) of one plane, as the GPU reports them."""
    n, pair = per_sample_counts(words)
    alive = 0
    for b in range(64):
        if n[b] > 0:
            alive |= 1 << b
    return int(n.sum()), int(pair.sum()), alive


def oracle_runs(model, B, planes, seed, instances, times, t0=0, samples=(1 << 64) - 1,
                which=None, init_words=None, connected=False, mask_bits=2):
    """One oracle.Run per (instance, plane) in `which` (default: all)."""
    runs = []
    keys = which if which is not None else [(i, q) for i in range(len(instances))
                                            for q in range(planes)]
    for (i, q) in keys:
        inst = instances[i]
        init = {0: "full", 1: "empty", 2: "host"}[int(inst.init)]
        iw = None
        if init == "host":
            L = int(inst.L)
            src = inst.host_words if init_words is None else init_words[i]
            iw = np.asarray(src, dtype=np.uint64)[q * L:(q + 1) * L]
        runs.append(oracle.Run(model=MODEL_NAME[model], B=B, L=int(inst.L), seed=seed,
                               stream=int(inst.stream_id), plane=q, p=inst.p, d=inst.d,
                               samples=samples, init=init, init_words=iw, t0=t0, times=times,
                               connected=connected, mask_bits=mask_bits))
    oracle.simulate_many(runs)
    return keys, runs
