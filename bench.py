"""Benchmark: site-updates/s of the multispin PCPD sweep on one MI355X.

Workload: PCPD, periodic ring L = 2^20, 4 planes of 64 samples (256 samples),
d = 0.1, 16 values of p = linspace(0.05, 0.20, 16), fully occupied start,
Philox seed 1, density recorded at the 64 log-spaced times of a 10^5-step run.
One benchmark step = 1000 Monte Carlo steps of all 16 x 4 planes (4.3e12
site updates), with the density records that fall inside it plus one at its
end; consecutive steps continue the same trajectory, so warmup + timed steps
cover a prefix of the 10^5-step run.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mc-per-step M]
                    [--workload cfg2|cfg3|cfg4|dp_absorbing] [--autotune]
                    [--tile-cols C] [--phase-max S] [--teams T] [--persistent]
                    [--skip-empty] [--graph]

Prints one JSON line. Also reports the dominant kernel (the phase kernel of
the sweep) against the integer-VALU roofline, and the CPU oracle on a bounded
sample of the same workload. The default workload is the one above; cfg3 (512
batched PCPD rings of uneven length, one plane), cfg4 (TCPD, 8 rings of 2^18
sites, one plane) and dp_absorbing (DP, 16 rings of 2^18 sites across the
absorbing transition) report the same metric on those workloads, without the
CPU leg. --autotune times the library's tile shapes on the workload before the
timed region; --skip-empty skips tiles with no particle (exact; the rate then
depends on the state, so it is reported apart).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Integer-VALU op model of one word-update (64 site updates): the VALU
# instructions of the method's per-site arithmetic as issued on gfx950, each
# one issue slot per lane (32x32->64 products run at full rate on gfx950):
# three Philox-4x32-10 draws = 47 products + 54 XORs, two probability
# decisions = 8, and the bit-sliced attempt = 20 (DP), 22 (PCPD), 26 (TCPD) or
# 30 (QCPD).
# Work that is uniform across a wavefront (the counter words and keys of the
# first two rounds) runs on the scalar unit and is not counted; neither are
# addressing, register moves, halo windows and tile copies.
OPS_PER_WORD_UPDATE = {1: 129, 2: 131, 3: 135, 4: 139}
PEAK_SLOTS = 256 * 64 * 2.4e9          # CUs x 64 lanes x 2.4 GHz = 3.93e13 ops/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "brs_phase_pcpd_L2p20_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1301_6082_amd", "csrc", "brs_phase.h")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mc-per-step", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-units", type=int, default=0,
                    help="(instance, plane) units for the oracle timing; 0 = one per host thread")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device-to-device three times first (counter calibration)")
    ap.add_argument("--workload", choices=("cfg2", "cfg3", "cfg4", "dp_absorbing"), default="cfg2")
    ap.add_argument("--autotune", action="store_true",
                    help="time the library's tile shapes on the workload first (untimed)")
    ap.add_argument("--teams", type=int, default=0, choices=(0, 2, 4),
                    help="lanes per block of the phase kernel (0 = the library's default)")
    ap.add_argument("--tile-cols", type=int, default=0,
                    help="tile width in blocks, halo included (0 = the library's default)")
    ap.add_argument("--phase-max", type=int, default=0,
                    help="most substeps per phase launch (0 = the library's default)")
    ap.add_argument("--skip-empty", action="store_true",
                    help="tiles with no particle in their loaded range skip their substeps "
                         "(state-dependent rate; exact)")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured HIP graphs in the timed region (profiling off there); "
                         "the kernel time comes from one more, profiled step after it")
    ap.add_argument("--persistent", action="store_true",
                    help="all phases between records in one ticket-dispatched launch")
    return ap.parse_args()


def kernel_traffic(tile):
    """HBM bytes per phase launch from the committed counter profile, if it
    was taken on the current kernel source and tile shape (columns x substeps
    x teams); else None."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch:", "kernel_sha256:", "tile:")))
    digest = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if fields.get("kernel_sha256", "").strip() != digest:
        return None
    if fields.get("tile", "").strip() != f"{tile[0]}x{tile[1]}x{tile[2]}":
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(wl, n_units: int):
    """The oracle as it stands, on (instance, plane) units of the same
    workload, 2 MC steps each, all host cores (OpenMP over units)."""
    from oracle import oracle

    oracle.build(force=False)
    if n_units <= 0:
        n_units = max(1, oracle.max_threads())
    units = []
    steps = 2
    for u in range(n_units):
        i, q = u % len(wl.instances), (u // len(wl.instances)) % wl.planes
        inst = wl.instances[i]
        units.append(oracle.Run(model="pcpd", B=wl.B, L=inst.L, seed=wl.seed,
                                stream=inst.stream_id, plane=q, p=inst.p, d=inst.d,
                                times=[steps]))
    threads = min(oracle.max_threads(), n_units)
    t0 = time.perf_counter()
    oracle.simulate_many(units, n_threads=threads)
    dt = time.perf_counter() - t0
    su = sum(64 * r.params.L * steps for r in units)
    return {"value": su / dt, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_units} (instance, plane) units of the workload, L=2^20, 64 samples "
                      f"each, {steps} MC steps from the full start ({su:.3e} site updates, "
                      f"{dt:.1f} s wall)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the instances shard across GPUs with no exchange, but this build runs on one).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1301_6082_amd import pcpd
    from paper_1301_6082_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    M = args.mc_per_step
    total_steps = (args.warmup + args.steps) * M
    wl = {"cfg2": workloads.cfg2, "cfg3": workloads.cfg3, "cfg4": workloads.cfg4,
          "dp_absorbing": workloads.dp_absorbing}[args.workload]()
    rec_times = [t for t in wl.times]
    su_per_mc = sum(64 * wl.planes * inst.L for inst in wl.instances)

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    sim = pcpd.Sim(wl.model, wl.B, wl.planes, wl.seed, wl.instances)
    if args.teams or args.tile_cols or args.phase_max:
        sim.set_tuning(args.tile_cols, args.phase_max, args.teams)
    if args.persistent or args.skip_empty or args.graph:
        sim.set_options(graph=args.graph, persistent=args.persistent, skip_empty=args.skip_empty)
    if args.autotune:
        sim.autotune()

    def step_times(k):
        lo, hi = k * M, (k + 1) * M
        ts = [t for t in rec_times if lo < t < hi]
        return ts + [hi]

    for k in range(args.warmup):
        sim.run(step_times(k))
    torch.cuda.synchronize()

    # the dominant kernel (the sweep's phase kernel) is timed by HIP events
    # that the library records around each launch on its own stream; with
    # --graph the timed region replays graphs unprofiled (profiling launches
    # directly), and one more step after it is profiled instead
    if not args.graph:
        sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    counts = None
    for k in range(args.warmup, args.warmup + args.steps):
        counts = sim.run(step_times(k))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert sim.time == total_steps
    if args.graph:
        sim.profile(True)
        sim.run(step_times(args.warmup + args.steps))
        torch.cuda.synchronize()
    kernel_ms, launches = sim.profile_read()
    sim.profile(False)
    site_updates = su_per_mc * M * args.steps
    value = site_updates / elapsed

    tuning = sim.get_tuning()
    launch_ms = kernel_ms / launches
    if args.graph:   # the timed steps' launches at the profiled step's rate
        launches = launches * args.steps
        kernel_ms = launch_ms * launches
    word_updates = site_updates / 64          # interior windows, all launches
    ops_word = OPS_PER_WORD_UPDATE[wl.model]
    ops_per_launch = ops_word * word_updates / launches
    achieved = ops_per_launch / (launch_ms * 1e-3)
    # the committed counter profile covers the default workload only
    traffic = kernel_traffic(tuning) if args.workload == "cfg2" else None
    Ls = np.array([inst.L for inst in wl.instances], dtype=np.float64)
    rho = counts[-1, :, :, 0].astype(np.float64).sum(axis=1) / (64 * wl.planes * Ls)

    cpu = None
    if not args.no_cpu_baseline and args.workload == "cfg2":
        cpu = cpu_baseline(wl, args.cpu_sample_units)

    if args.workload == "cfg2":
        config = {"workload": wl.name, "L": 1 << 20, "planes": wl.planes,
                  "samples_per_instance": 64 * wl.planes, "instances": len(wl.instances),
                  "d": 0.1, "p": "linspace(0.05,0.20,16)", "B": wl.B}
    else:
        ds = sorted({inst.d for inst in wl.instances})
        config = {"workload": wl.name, "model": {1: "DP", 2: "PCPD", 3: "TCPD", 4: "QCPD"}[wl.model],
                  "L": [int(Ls.min()), int(Ls.max())], "total_sites": int(Ls.sum()),
                  "planes": wl.planes, "samples_per_instance": 64 * wl.planes,
                  "instances": len(wl.instances), "d": ds if len(ds) > 1 else ds[0],
                  "p": [round(min(i.p for i in wl.instances), 4),
                        round(max(i.p for i in wl.instances), 4)], "B": wl.B}
    config.update({"mc_steps_per_bench_step": M, "mc_steps_total": total_steps,
                   "records": "the workload's log-spaced record times, plus each step end",
                   "tile_cols": tuning[0], "phase_max": tuning[1], "teams": tuning[2],
                   "persistent": args.persistent, "skip_empty": args.skip_empty,
                   "graph": args.graph,
                   "autotuned": args.autotune})

    out = {
        "metric": "site-updates/sec (samples x sites x MC steps) at 1 GPU",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": config,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tops/s (int32 VALU lane-ops)",
                     "frac": achieved / PEAK_SLOTS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "kernel": f"brs_phase<{wl.model}>", "launch_ms": launch_ms,
                     "launches": launches, "ops_per_word_update": ops_word,
                     "site_updates_per_s_at_peak": PEAK_SLOTS / ops_word * 64,
                     "kernel_share_of_wall": kernel_ms * 1e-3 / elapsed},
        "cpu_baseline": cpu,
        "rho_at_end": [round(float(x), 5) for x in rho],
    }
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
