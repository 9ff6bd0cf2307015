"""Write the expected results of the long-horizon GPU parity cases.

Every expected value in the horizon_*.json files comes from this script, and
this script calls only the CPU oracle (oracle/) on the seeded workloads of
paper_1301_6082_amd.workloads (input recipes, no arithmetic of the method).
Nothing here reads a GPU result.

    python tests/golden/make_horizon_golden.py [--case NAME ...] [--threads N]

For each case and each simulated (instance, plane) unit the file holds:
  - the sha256 of the unit's final lattice (L little-endian uint64 words; bits
    of samples the case does not simulate are zero),
  - per record time, the particle count N, the pair count N_pair and the
    alive mask over the simulated samples (all 64 unless `samples` says
    otherwise), and for sampled units the per-sample N and N_pair.
The GPU test (tests/test_gpu_horizons.py) rebuilds the same workload from
the recipe named in the file and compares bit for bit.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_1301_6082_amd import workloads as wl  # noqa: E402

ALL = (1 << 64) - 1
MODEL_NAME = {1: "dp", 2: "pcpd", 3: "tcpd", 4: "qcpd"}


def ring1024(model: int) -> wl.Workload:
    """One ring of 1024 sites, one plane, B = 64, seed 1, stream 0, run to
    10^5 Monte Carlo steps with the 64 log-spaced records."""
    p = {1: 0.1, 2: 0.1, 3: 0.02}[model]
    return wl.Workload(f"ring1024_n{model}", model, 64, 1, 1,
                       [wl.Instance(p, 0.5, 1024, 0)], 100_000, wl.log_times(100_000))


def cfg3_pick32():
    """32 of the 512 batched instances, drawn without replacement."""
    return sorted(int(i) for i in np.random.default_rng(7).choice(512, 32, replace=False))


# name -> (workload builder, record times, units [(inst, plane, samples)] or None = all)
def cases():
    c2 = wl.cfg2
    out = {
        "cfg2_all_t8": (c2, [1, 2, 4, 8], None),
        "cfg2_pends_t64": (c2, [1, 2, 4, 8, 16, 32, 64],
                           [(i, q, ALL) for i in (0, 15) for q in range(4)]),
        "cfg2_sampled_t600": (c2, [512, 600], [(3, 1, 1 << 17), (12, 3, 1 << 40)]),
        "cfg3_all_t16": (wl.cfg3, [1, 2, 4, 8, 16], None),
        "cfg3_pick32_t256": (wl.cfg3, [16, 64, 256], [(i, 0, ALL) for i in cfg3_pick32()]),
        "cfg4_all_t256": (wl.cfg4, [16, 64, 256], None),
    }
    for n in (1, 2, 3):
        out[f"ring1024_n{n}_t1e5"] = (lambda n=n: ring1024(n), wl.log_times(100_000), None)
    return out


def run_case(name, threads):
    build, times, units = cases()[name]
    w = build()
    if units is None:
        units = [(i, q, ALL) for i in range(len(w.instances)) for q in range(w.planes)]
    runs = []
    for i, q, samples in units:
        inst = w.instances[i]
        runs.append(oracle.Run(model=MODEL_NAME[w.model], B=w.B, L=int(inst.L), seed=w.seed,
                               stream=int(inst.stream_id), plane=q, p=inst.p, d=inst.d,
                               samples=samples, times=times))
    t0 = time.perf_counter()
    oracle.simulate_many(runs, n_threads=threads)
    dt = time.perf_counter() - t0
    recs = []
    for (i, q, samples), r in zip(units, runs):
        N, NP, alive = r.counts()
        rec = {"inst": i, "plane": q, "samples": hex(samples),
               "words_sha256": hashlib.sha256(r.words.astype("<u8").tobytes()).hexdigest(),
               "n": [int(v) for v in N], "n_pair": [int(v) for v in NP],
               "alive": [hex(int(v)) for v in alive]}
        if samples != ALL:
            bits = [b for b in range(64) if (samples >> b) & 1]
            rec["per_sample"] = {str(b): {"n": [int(v) for v in r.n[:, b]],
                                          "n_pair": [int(v) for v in r.pair[:, b]]}
                                 for b in bits}
        recs.append(rec)
    su = sum(64 * int(r.params.L) * (int(times[-1])) for r in runs)
    doc = {
        "what": "expected results of a long-horizon parity case, written by the CPU oracle",
        "script": "tests/golden/make_horizon_golden.py",
        "case": name,
        "workload": w.name,
        "model": w.model, "B": w.B, "planes": w.planes, "seed": w.seed,
        "instances": [[inst.p, inst.d, int(inst.L), int(inst.stream_id)] for inst in w.instances],
        "times": [int(t) for t in times],
        "units": recs,
        "oracle_seconds": round(dt, 1),
        "oracle_threads": threads if threads > 0 else oracle.max_threads(),
        "oracle_site_updates_upper_bound": su,
    }
    path = os.path.join(HERE, f"horizon_{name}.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(f"{name}: {len(units)} units, {dt:.1f} s -> {os.path.relpath(path, ROOT)}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", action="append", default=None)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    oracle.build(force=False)
    for name in (a.case or list(cases())):
        run_case(name, a.threads)


if __name__ == "__main__":
    main()
