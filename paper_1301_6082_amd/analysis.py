"""Effective exponents of the particle and pair densities near p_c (paper
Sec. 5.3, Figs. 5-6).

At the critical point the density is expected to decay as a power law with
strong corrections to scaling, rho(t) = c1 t^-delta + c2 t^-2delta + ...; then
the effective exponent delta_eff = -d ln rho / d ln t, plotted against rho,
approaches a straight line whose value at rho = 0 is delta, and the particle
density and the pair density (nearest-neighbour pairs per site) extrapolate
to the same delta. This module computes delta_eff(rho) for both densities from
the counts the sweep records (N and N_pair at log-spaced times, summed over
independent runs) and the straight-line extrapolation to rho = 0.

Simulations run on the GPU through the C ABI (`run_near_pc`); the analysis
itself is a few array operations on the recorded counts.

    python -m paper_1301_6082_amd.analysis --d 0.25 --p 0.125141 --L 262144 \\
        --runs 64 --steps 100000
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import workloads


def delta_eff(times, rho, span: int = 1):
    """delta_eff between records k and k + span: -(ln rho_{k+span} - ln rho_k) /
    (ln t_{k+span} - ln t_k), at the geometric midpoint of the two times and
    of the two densities. Records with rho = 0 are dropped. Returns (t_mid,
    rho_mid, delta_eff)."""
    t = np.asarray(times, float)
    r = np.asarray(rho, float)
    keep = (t > 0) & (r > 0)
    t, r = t[keep], r[keep]
    if len(t) <= span:
        return np.empty(0), np.empty(0), np.empty(0)
    lt, lr = np.log(t), np.log(r)
    d = -(lr[span:] - lr[:-span]) / (lt[span:] - lt[:-span])
    return np.exp(0.5 * (lt[span:] + lt[:-span])), np.exp(0.5 * (lr[span:] + lr[:-span])), d


def extrapolate(rho_mid, d_eff, rho_max: float, rho_min: float = 0.0):
    """Straight-line fit delta_eff = delta + a * rho over the points with
    rho_min < rho <= rho_max; returns (delta, a), the value at rho = 0 and the
    slope (nan, nan if fewer than two points)."""
    rho_mid = np.asarray(rho_mid, float)
    d_eff = np.asarray(d_eff, float)
    sel = (rho_mid > rho_min) & (rho_mid <= rho_max) & np.isfinite(d_eff)
    if sel.sum() < 2:
        return float("nan"), float("nan")
    a, delta = np.polyfit(rho_mid[sel], d_eff[sel], 1)
    return float(delta), float(a)


@dataclass
class Curves:
    """Densities at the record times, summed over runs, and their effective
    exponents."""
    times: np.ndarray
    rho: np.ndarray        # particles per site
    rho_pair: np.ndarray   # nearest-neighbour pairs per site
    runs: int

    def particle(self, span: int = 1):
        return delta_eff(self.times, self.rho, span)

    def pair(self, span: int = 1):
        return delta_eff(self.times, self.rho_pair, span)


def curves_from_counts(times, counts, L: int, planes: int) -> Curves:
    """counts uint64 [n_times, n_runs, planes, 3] (N, N_pair, alive) as
    pcpd.Sim.run returns them, every run of ring length L."""
    c = np.asarray(counts)
    sites = 64.0 * planes * L * c.shape[1]
    N = c[:, :, :, 0].astype(np.float64).sum(axis=(1, 2))
    NP = c[:, :, :, 1].astype(np.float64).sum(axis=(1, 2))
    return Curves(np.asarray(times, float), N / sites, NP / sites, int(c.shape[1]))


def run_near_pc(p: float, d: float, L: int = 1 << 18, runs: int = 16, planes: int = 1,
                steps: int = 100_000, records: int = 64, model: int = workloads.PCPD,
                B: int = 64, seed: int = 7, first_stream: int = 0, layout: int = 0) -> Curves:
    """`runs` independent runs (Philox streams first_stream ..) of one (p, d)
    from the full lattice, batched in one GPU context; densities at
    log-spaced times."""
    from . import pcpd

    times = workloads.log_times(steps, records)
    insts = [workloads.Instance(float(p), float(d), int(L), first_stream + k) for k in range(runs)]
    with pcpd.Sim(model, B, planes, seed, insts, layout=layout) as sim:
        sim.set_options(graph=True)
        counts = sim.run(times)
    return curves_from_counts(times, counts, L, planes)


def _deviations(per_run, ref, runs):
    """Largest |mean difference| / its standard error over the records, per key."""
    dev = {}
    for k, r in per_run.items():
        sigma = np.sqrt(r.var(axis=1, ddof=1) / runs + per_run[ref].var(axis=1, ddof=1) / runs)
        diff = np.abs(r.mean(axis=1) - per_run[ref].mean(axis=1))
        z = np.where(sigma > 0, diff / np.maximum(sigma, 1e-300), 0.0)
        dev[k] = float(z.max())
    return dev


def _scheme_runs(p, d, L, runs, planes, steps, B, layout, mask_bits):
    from . import pcpd

    times = workloads.log_times(steps, 64)
    insts = [workloads.Instance(float(p), float(d), int(L), k) for k in range(runs)]
    with pcpd.Sim(workloads.PCPD, int(B), planes, 7, insts, layout=layout,
                  mask_bits=mask_bits) as sim:
        sim.set_options(graph=True)
        c = sim.run(times)
    return times, c


def compare_block_widths(p: float, d: float, widths=(16, 64, 256), L: int = 1 << 18,
                         runs: int = 16, planes: int = 1, steps: int = 100_000, span: int = 4,
                         layout: int = 0, mask_bits: int = 2):
    """The paper's numerical-accuracy check (Sec. 5.2): rho(t) near p_c for
    several block widths B (the number of sites that share one randomly chosen
    local site per substep; the paper's workgroup sizes 512 .. 32 at its
    L = 2^18 correspond to B = 16 .. 256). The same runs (Philox streams) at
    every B; returns {B: Curves} and, per B, the largest deviation of rho(t)
    from the curve at the largest B, in units of the statistical error of the
    difference of the two means over runs at that record."""
    out, per_run = {}, {}
    for B in widths:
        times, c = _scheme_runs(p, d, L, runs, planes, steps, B, layout, mask_bits)
        out[B] = curves_from_counts(times, c, L, planes)
        per_run[B] = c[:, :, :, 0].astype(np.float64).sum(axis=2) / (64.0 * planes * L)
    return out, _deviations(per_run, max(widths), runs)


def compare_mask_bits(p: float, d: float, bits=(2, 4), L: int = 1 << 18, runs: int = 16,
                      planes: int = 1, steps: int = 100_000, B: int = 64, layout: int = 0):
    """The other half of the Sec. 5.2 check: rho(t) near p_c with m = 2 and
    m = 4 decorrelation bits per decision (independent random bits per sample
    under the word-wide comparison), the same streams; deviations from the
    largest m as in compare_block_widths."""
    out, per_run = {}, {}
    for m in bits:
        times, c = _scheme_runs(p, d, L, runs, planes, steps, B, layout, m)
        out[m] = curves_from_counts(times, c, L, planes)
        per_run[m] = c[:, :, :, 0].astype(np.float64).sum(axis=2) / (64.0 * planes * L)
    return out, _deviations(per_run, max(bits), runs)


def main(argv: Optional[Sequence[str]] = None):
    import argparse
    import json

    ap = argparse.ArgumentParser(description="delta_eff(rho) of particles and pairs near p_c")
    ap.add_argument("--p", type=float, required=True)
    ap.add_argument("--d", type=float, required=True)
    ap.add_argument("--L", type=int, default=1 << 18)
    ap.add_argument("--runs", type=int, default=16)
    ap.add_argument("--planes", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--span", type=int, default=4, help="records between the two ends of a slope")
    ap.add_argument("--rho-max", type=float, default=0.05,
                    help="densities up to this enter the straight-line extrapolation")
    ap.add_argument("--layout", type=int, default=0, help="0 classical, 1 connected (Sec. 4)")
    ap.add_argument("--compare-B", type=str, default=None,
                    help="comma-separated block widths: the Sec. 5.2 accuracy check instead")
    ap.add_argument("--compare-m", type=str, default=None,
                    help="comma-separated decorrelation bits (2,4): the same check over m")
    a = ap.parse_args(argv)
    if a.compare_m:
        bits = tuple(int(v) for v in a.compare_m.split(","))
        curves, dev = compare_mask_bits(a.p, a.d, bits, a.L, a.runs, a.planes, a.steps,
                                        layout=a.layout)
        for m in bits:
            t, r, de = curves[m].particle(a.span)
            print(f"m={m}: rho(T)={curves[m].rho[-1]:.6g}, late delta_eff={de[-1]:.3f}, "
                  f"largest |rho - rho(m={max(bits)})| / sigma = {dev[m]:.2f}", flush=True)
        print(json.dumps({"p": a.p, "d": a.d, "L": a.L, "runs": a.runs, "steps": a.steps,
                          "deviation_sigma": {str(k): v for k, v in dev.items()},
                          "rho": {str(m): curves[m].rho.tolist() for m in bits},
                          "times": curves[bits[0]].times.tolist()}), flush=True)
        return
    if a.compare_B:
        widths = tuple(int(v) for v in a.compare_B.split(","))
        curves, dev = compare_block_widths(a.p, a.d, widths, a.L, a.runs, a.planes, a.steps,
                                           a.span, a.layout)
        for B in widths:
            t, r, de = curves[B].particle(a.span)
            print(f"B={B}: rho(T)={curves[B].rho[-1]:.5g}, late delta_eff={de[-1]:.3f}, "
                  f"largest |rho - rho(B={max(widths)})| / sigma = {dev[B]:.2f}", flush=True)
        print(json.dumps({"p": a.p, "d": a.d, "L": a.L, "runs": a.runs, "steps": a.steps,
                          "deviation_sigma": {str(k): v for k, v in dev.items()},
                          "rho": {str(B): curves[B].rho.tolist() for B in widths},
                          "times": curves[widths[0]].times.tolist()}), flush=True)
        return
    c = run_near_pc(a.p, a.d, a.L, a.runs, a.planes, a.steps, layout=a.layout)
    out = {"p": a.p, "d": a.d, "L": a.L, "runs": a.runs, "planes": a.planes, "steps": a.steps}
    for name, (t, r, de) in (("particles", c.particle(a.span)), ("pairs", c.pair(a.span))):
        delta, slope = extrapolate(r, de, a.rho_max)
        out[name] = {"t": t.tolist(), "rho": r.tolist(), "delta_eff": de.tolist(),
                     "delta_at_rho0": delta, "slope": slope}
        print(f"{name}: delta_eff from {de[0]:.3f} (rho {r[0]:.3g}) to {de[-1]:.3f} "
              f"(rho {r[-1]:.3g}); straight line to rho = 0: delta = {delta:.4f}", flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
