"""Seeded synthetic workloads: the inputs that the GPU path and the oracle share.

This module holds no arithmetic of the method. It only states the workloads
(lattice sizes, rates, seeds, record schedules, random starting lattices) so
that both sides are fed identical inputs. It imports neither side.

The paper's production workload (Sec. 5.3) is a ring of L = 2^18 sites started
fully occupied, with rates near the critical point; the configurations below
follow that shape at the sizes the benchmark and the tests use.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

DP, PCPD, TCPD, QCPD = 1, 2, 3, 4
INIT_FULL, INIT_EMPTY, INIT_HOST = 0, 1, 2


@dataclass
class Instance:
    p: float
    d: float
    L: int
    stream_id: int
    init: int = INIT_FULL
    host_words: np.ndarray | None = None  # planes*L uint64 words if init == INIT_HOST


@dataclass
class Workload:
    name: str
    model: int
    B: int
    planes: int
    seed: int
    instances: List[Instance]
    steps: int                      # Monte Carlo steps of the whole run
    times: List[int] = field(default_factory=list)  # record times (MC steps)

    def site_updates(self, steps: int | None = None) -> int:
        """64 samples x planes x L sites per instance, per Monte Carlo step."""
        st = self.steps if steps is None else steps
        return sum(64 * self.planes * inst.L for inst in self.instances) * st


def log_times(T: int, count: int = 64) -> List[int]:
    """`count` distinct, strictly increasing record times ending exactly at T:
    t_k = max(t_{k-1} + 1, floor(T^(k/count) + 1/2)), t_0 = 0."""
    out, prev = [], 0
    for k in range(1, count + 1):
        t = max(prev + 1, int(math.floor(T ** (k / count) + 0.5)))
        out.append(t)
        prev = t
    assert out[-1] == T, (T, out[-1])
    return out


def cfg1() -> Workload:
    """PCPD ring L=1024, one plane, d=0.5, p=0.1, fully occupied, 1000 MC steps,
    Philox seed 1, records every 10th step."""
    return Workload("pcpd_L1024_1plane_d0.5_p0.1", PCPD, 64, 1, 1,
                    [Instance(0.1, 0.5, 1024, 0)], 1000, list(range(10, 1001, 10)))


def cfg2(steps: int = 100_000) -> Workload:
    """PCPD ring L=2^20, 4 planes (256 samples), d=0.1, 16 p values
    linspace(0.05, 0.20, 16), fully occupied, 64 log-spaced records."""
    ps = np.linspace(0.05, 0.20, 16)
    inst = [Instance(float(p), 0.1, 1 << 20, i) for i, p in enumerate(ps)]
    return Workload("pcpd_L2^20_4planes_16p_d0.1", PCPD, 64, 4, 1, inst, steps,
                    log_times(steps))


def cfg3(steps: int = 10_000, count: int = 512) -> Workload:
    """Batched PCPD: `count` instances, L log-uniform in [2^12, 2^18] rounded
    down to a multiple of 64, d uniform in {0.1, 0.5, 0.9}, p uniform in
    [0.05, 0.25], one plane each, drawn from numpy default_rng(2013)."""
    rng = np.random.default_rng(2013)
    u = rng.uniform(12.0, 18.0, size=count)
    ds = rng.choice(np.array([0.1, 0.5, 0.9]), size=count)
    ps = rng.uniform(0.05, 0.25, size=count)
    inst = []
    for i in range(count):
        L = 64 * int(math.floor(2.0 ** u[i] / 64.0))
        inst.append(Instance(float(ps[i]), float(ds[i]), L, i))
    return Workload("batched_pcpd_512x_L2^12..2^18", PCPD, 64, 1, 1, inst, steps,
                    log_times(steps))


def cfg4(steps: int = 100_000) -> Workload:
    """TCPD ring L=2^18, one plane, d=0.5, p = linspace(0.02, 0.15, 8)."""
    ps = np.linspace(0.02, 0.15, 8)
    inst = [Instance(float(p), 0.5, 1 << 18, i) for i, p in enumerate(ps)]
    return Workload("tcpd_L2^18_8p_d0.5", TCPD, 64, 1, 1, inst, steps, log_times(steps))


def dp_absorbing(steps: int = 100_000) -> Workload:
    """DP (n = 1) rings of 2^18 sites, one plane, d = 0.5, 16 values of
    p = linspace(0.05, 0.6, 16), fully occupied start: the rings deep in the
    absorbing phase die out in every sample (the empty lattice is DP's only
    absorbing state), the others stay active. For rates with empty tiles
    skipped, which depend on the state."""
    ps = np.linspace(0.05, 0.6, 16)
    inst = [Instance(float(p), 0.5, 1 << 18, i) for i, p in enumerate(ps)]
    return Workload("dp_L2^18_16p_d0.5", DP, 64, 1, 1, inst, steps, log_times(steps))


def random_lattice(L: int, planes: int, density: float, seed: int) -> np.ndarray:
    """planes*L uint64 words with each bit set independently with `density`."""
    rng = np.random.default_rng(seed)
    bits = rng.random((planes * L, 64)) < density
    w = np.zeros(planes * L, dtype=np.uint64)
    for b in range(64):
        w |= bits[:, b].astype(np.uint64) << np.uint64(b)
    return w
