"""Search for the critical annihilation rate p_c (paper Sec. 2: active phase
for p < p_c, inactive for p > p_c, p_c depends on d), by plain bisection on a
p-grid and by bisection guided by the density surrogate.

Every run is a GPU simulation through the C ABI; the surrogate only proposes
where to run. Site updates are counted for every run (the ledger), so the two
searches can be compared on the work they need to reach their bracket.

Classification of a density curve rho(t_k) (the order parameter, Sec. 1),
motivated by the power law at p_c and its corrections to scaling (Sec. 5.3):
the effective exponent delta_eff = -d log rho / d log t is roughly constant
at p_c (about 0.2 for PCPD), falls towards 0 in the active phase (rho
saturates) and rises in the inactive phase towards the 1/2 of diffusing,
pair-annihilating particles (pairs vanish quickly; lone particles only meet
by diffusion). A curve is inactive if all its samples died, or if delta_eff
over the last half-decade of t is above DELTA_HIGH, or if it exceeds both its
value over the half-decade before and DELTA_FLOOR; otherwise active.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import workloads

DELTA_FLOOR = 0.05
DELTA_HIGH = 0.35


# p enters the surrogate centred and scaled: one cell of the 2^10-point search
# grid then moves the input by 0.004, which is the resolution of the bfloat16
# activations of the network's hidden products. Scaled as p / 0.25, a cell moved
# it by 0.001 and neighbouring cells got identical predictions.
P_MID, P_SCALE = 0.16, 0.07


def features(p, d, t):
    """Surrogate inputs ((p - P_MID) / P_SCALE, d, log10(t) / 6), float32 [..., 3]."""
    p, d, t = np.broadcast_arrays(np.asarray(p, float), np.asarray(d, float), np.asarray(t, float))
    return np.stack([(p - P_MID) / P_SCALE, d, np.log10(t) / 6.0], axis=-1).astype(np.float32)


def _slope(logt, logr):
    A = np.stack([logt, np.ones_like(logt)], axis=1)
    return float(np.linalg.lstsq(A, logr, rcond=None)[0][0])


def delta_eff_windows(times, rho) -> Tuple[float, float]:
    """delta_eff fitted over [T/10, T/sqrt(10)] and [T/sqrt(10), T]."""
    t = np.asarray(times, float)
    r = np.asarray(rho, float)
    T = t[-1]
    lt, lr = np.log10(t), np.log10(np.maximum(r, 1e-300))
    a = (t >= T / 10.0 * 0.999) & (t <= T / math.sqrt(10.0) * 1.001)
    b = t >= T / math.sqrt(10.0) * 0.999
    return -_slope(lt[a], lr[a]), -_slope(lt[b], lr[b])


def classify(times, rho) -> bool:
    """True if the curve is inactive (p above the finite-time p_c)."""
    r = np.asarray(rho, float)
    if r[-1] <= 0.0:
        return True
    prev, last = delta_eff_windows(times, r)
    return bool(last > DELTA_HIGH or (last > prev and last > DELTA_FLOOR))


@dataclass
class Ledger:
    runs: int = 0
    site_updates: int = 0
    # (grid index, p, inactive, delta_eff previous half-decade, last half-decade, rho(T))
    path: List[Tuple] = field(default_factory=list)


@dataclass
class RunSpec:
    L: int = 1 << 18
    planes: int = 4
    steps: int = 1_000_000
    records: int = 64
    B: int = 64
    model: int = workloads.PCPD
    tune: bool = True   # autotune the kernel shape of each batched verification run

    def times(self):
        return workloads.log_times(self.steps, self.records)

    def site_updates(self):
        return 64 * self.planes * self.L * self.steps


SEED = 1000  # Philox key word 0 of every verification run; the stream id is d's index


def simulate_curves(spec: RunSpec, probes: Sequence[Tuple[float, float, int]]):
    """Verification runs of several (p, d, stream) probes as one batched GPU
    run (each instance is simulated exactly as it would be alone); returns
    (times, [rho per probe])."""
    from . import pcpd

    insts = [workloads.Instance(float(p), float(d), spec.L, int(st)) for p, d, st in probes]
    times = spec.times()
    with pcpd.Sim(spec.model, spec.B, spec.planes, SEED, insts) as sim:
        if spec.tune:
            sim.autotune(2)   # cached per lattice shape; never changes results
        sim.set_options(graph=True)
        c = sim.run(times)
    N = c[:, :, :, 0].astype(np.float64).sum(axis=2)           # [times, instance]
    rho = N / (64.0 * spec.planes * spec.L)
    return np.asarray(times, float), [rho[:, k] for k in range(len(insts))]


def simulate_curve(spec: RunSpec, p: float, d: float, stream: int):
    """One verification run on the GPU; returns (times, rho)."""
    times, rhos = simulate_curves(spec, [(p, d, stream)])
    return times, rhos[0]


class Grid:
    """2^bits points uniform on [lo, hi]. Every run at diffusion index d_idx
    uses key (SEED, d_idx): common random numbers across the grid, so the
    class of a grid point is a fixed function of the point and neighbouring
    points see the same draws (classes change smoothly with p)."""

    def __init__(self, lo=0.02, hi=0.30, bits=10):
        self.p = np.linspace(lo, hi, 1 << bits)

    def __len__(self):
        return len(self.p)


# Searches are generators: they yield the grid index to simulate next and
# receive (times, rho, inactive); they return the final bracket. Each keeps
# its own ledger and cache, so two searches never share a run.


def _record(ledger, grid, i, times, rho, ina, spec):
    ledger.runs += 1
    ledger.site_updates += spec.site_updates()
    dp, dl = delta_eff_windows(times, rho) if rho[-1] > 0 else (float("nan"), float("nan"))
    ledger.path.append((i, float(grid.p[i]), ina, round(dp, 4), round(dl, 4), float(rho[-1])))


def plain_steps(grid: Grid, lo: int, hi: int):
    """Midpoint bisection; the ends are taken as active (lo) and inactive (hi)."""
    while hi - lo > 1:
        mid = (lo + hi) // 2
        _, _, ina = yield mid
        if ina:
            hi = mid
        else:
            lo = mid
    return lo, hi


CALIBRATED_PROBES = 4     # probes placed by the calibrated surrogate before midpoints
LEVEL_STEP = 0.0025       # delta_eff change per grid cell above which the level calibrates


def match_index(ys, sim_log10, late) -> int:
    """Grid index whose predicted curve is closest (mean |log10 rho| gap over
    the late times) to a simulated curve."""
    err = np.mean(np.abs(ys[:, late] - sim_log10[late]), axis=1)
    return int(np.argmin(err))


def level_index(levels, level_sim: float, probe: int, lo: int = 0, hi: Optional[int] = None) -> int:
    """Grid index in [lo, hi] whose predicted delta_eff level (last
    half-decade) is closest to the simulated one; near-ties (within 1e-3) go
    to the index nearest the probe. Near p_c the level rises steeply with p
    (about 0.2 at p_c towards 1/2 in the inactive phase), so it places a
    simulated run on the network's p axis to about a cell even where the
    curves themselves are nearly alike."""
    levels = np.asarray(levels, float)
    hi = len(levels) - 1 if hi is None else hi
    lo, hi = max(0, lo), min(len(levels) - 1, hi)
    idx = np.arange(lo, hi + 1)
    gap = np.abs(levels[lo:hi + 1] - level_sim)
    gap = np.where(np.isfinite(gap), gap, np.inf)
    best = gap.min()
    if not np.isfinite(best):
        return probe
    near = idx[gap <= best + 1e-3]
    return int(near[np.argmin(np.abs(near - probe))])


def rising_segment(levels, f0: int, tol: float = 0.01) -> Tuple[int, int]:
    """The stretch [a, b] around the surrogate's flip f0 over which its
    predicted delta_eff level rises with p: extended down while the level
    does not go up by more than `tol` per cell, and up while it does not go
    down by more than `tol` (small wiggles of the network pass)."""
    levels = np.asarray(levels, float)
    n = len(levels)
    f0 = min(max(int(f0), 0), n - 1)
    a = b = f0
    while a > 0 and np.isfinite(levels[a - 1]) and levels[a - 1] <= levels[a] + tol:
        a -= 1
    while b + 1 < n and np.isfinite(levels[b + 1]) and levels[b + 1] >= levels[b] - tol:
        b += 1
    return a, b


def crossing_index(levels, level_sim: float, f0: int, tol: float = 0.01) -> float:
    """Where the predicted level equals a simulated run's level, on the
    rising stretch around f0 and nearest f0: from f0 down to the first cell
    at or below the simulated level when that lies below the level at f0,
    else up to the first cell at or above it (linear between cells). A level
    below the whole lower stretch goes to the foot of the rise, the last cell
    below f0 within `tol` of the stretch's floor; one above the upper stretch
    goes to its top. Near p_c the level of a run rises by a tenth or more per
    cell, so a run placed this way tells how far the surrogate's flip is off;
    the same level far from the flip, where the predicted curves are flat or
    saturated, does not."""
    levels = np.asarray(levels, float)
    a, b = rising_segment(levels, f0, tol)
    f = min(max(int(f0), a), b)
    if not np.isfinite(levels[f]):
        return float(f)
    if level_sim <= levels[f]:
        i = f
        while i > a and levels[i] > level_sim:
            i -= 1
        if levels[i] > level_sim:
            floor = float(np.min(levels[a:f + 1]))
            return float(a + int(np.nonzero(levels[a:f + 1] <= floor + tol)[0][-1]))
        if i == f:
            return float(f)
        lo, hi = levels[i], levels[i + 1]
        return i + (float((level_sim - lo) / (hi - lo)) if hi > lo else 0.0)
    i = f
    while i < b and levels[i] < level_sim:
        i += 1
    if levels[i] < level_sim:
        return float(b)
    lo, hi = levels[i - 1], levels[i]
    return i - 1 + (float((level_sim - lo) / (hi - lo)) if hi > lo else 1.0)


def predicted_levels(ys, times):
    """delta_eff over the last half-decade of each predicted log10 rho curve."""
    ys = np.asarray(ys, float)
    out = np.full(len(ys), np.nan)
    for j in range(len(ys)):
        if np.all(np.isfinite(ys[j])):
            out[j] = delta_eff_windows(times, 10.0 ** ys[j])[1]
    return out


def restrict_to_domain(ys, cls, grid: Grid, domain=None):
    """Outside the p range the network was trained on, its predictions are
    extrapolations. There its classes are taken as active below the range and
    inactive above it, and its curves are kept out of calibration matches."""
    if domain is None:
        return ys, cls
    below, above = grid.p < domain[0], grid.p > domain[1]
    ys = np.array(ys, float)
    cls = np.array(cls, bool)
    cls[below], cls[above] = False, True
    ys[below | above] = np.inf
    return ys, cls


def surrogate_steps(ys, cls, grid: Grid, times, lo: int, hi: int,
                    calibrated: int = CALIBRATED_PROBES, calibration: str = "crossing"):
    """Bracket search whose probes the surrogate places. `ys` [grid, times]
    are its log10 rho curves for the whole grid and `cls` their classes; its
    flip f0 is where its last run of inactive predictions inside the bracket
    starts.
    Each simulated probe calibrates it: the grid index j where the surrogate
    puts the simulated curve, so that its flip moves by (probe - j). With
    calibration="crossing" (the default) j is where the predicted delta_eff
    level of the last half-decade, on its rising stretch around the flip,
    equals the simulated run's (crossing_index). Otherwise j is the
    index whose predicted curve is closest over the last decade of t
    (match_index, calibration="shape"); with calibration="level", where the
    predicted delta_eff level of the last half-decade changes by LEVEL_STEP
    or more per cell, j is instead the index with the closest level
    (level_index): near and above the flip the level rises steeply with p
    while the curves just below it are nearly alike. The next
    probe is the calibrated flip, or the point below it when the flip is
    already the upper end of the bracket; when the estimate keeps pressing
    against an end of the bracket the step from that end doubles. Once both
    ends of the bracket come from simulations, an interior proposal outside
    the middle half of the bracket, or a repeated press against an end, is
    replaced by the midpoint. After `calibrated` such
    probes, or after an extinct run (which calibrates nothing), probes are
    midpoints. The simulation decides every class."""
    ys = np.asarray(ys, float)
    cls = np.asarray(cls, bool)
    late = np.asarray(times, float) >= float(times[-1]) / 10.0
    levels = predicted_levels(ys, times) if calibration in ("level", "crossing") else None
    # the surrogate's flip: the start of its last run of inactive predictions
    # inside the bracket (spurious inactive predictions far below it, e.g.
    # where the network extrapolates, do not count)
    active_pred = np.nonzero(~cls[lo + 1:hi + 1])[0]
    f0 = lo + 2 + int(active_pred[-1]) if active_pred.size else lo + 1
    f0 = min(f0, hi)
    shift, placed, streak, last_end = 0.0, 0, 0, None
    lo_seen = hi_seen = False  # ends of the bracket established by simulation
    while hi - lo > 1:
        by_surrogate = placed < calibrated
        if by_surrogate:
            f = int(round(f0 + shift))
            end = "hi" if f >= hi else ("lo" if f <= lo + 1 else None)
            streak = streak + 1 if (end is not None and end == last_end) else 0
            last_end = end
            step = 1 << streak
            if end == "hi":
                probe = max(hi - step, lo + 1)
            elif end == "lo":
                probe = min(lo + step, hi - 1)
            else:
                probe = f
            if lo_seen and hi_seen:
                # both ends simulated: an interior proposal outside the middle
                # half of the bracket, or a repeated press against one end, is
                # replaced by the midpoint; a first press (the point next to an
                # end, which closes the bracket if the surrogate is right) stays
                q = (hi - lo) // 4
                if (end is None and not (lo + q <= probe <= hi - q)) or streak > 0:
                    probe = (lo + hi) // 2
            placed += 1
        else:
            probe = (lo + hi) // 2
        _, rho, ina = yield probe
        lo0, hi0 = lo, hi  # the bracket the probe was placed in
        if ina:
            hi, hi_seen = probe, True
        else:
            lo, lo_seen = probe, True
        if by_surrogate:
            if rho[-1] > 0 and calibration == "crossing":
                shift = probe - crossing_index(levels, delta_eff_windows(times, rho)[1], f0)
            elif rho[-1] > 0:
                j = match_index(ys, np.log10(np.maximum(rho, 1e-300)), late)
                if levels is not None:
                    # the level places the run where it discriminates (it
                    # changes by LEVEL_STEP or more per cell there); where it
                    # is flat (deep in the active phase) the curve shape does
                    jl = level_index(levels, delta_eff_windows(times, rho)[1], probe, lo0, hi0)
                    a, b = max(jl - 1, 0), min(jl + 1, len(levels) - 1)
                    if np.isfinite(levels[a]) and np.isfinite(levels[b]) and \
                            abs(levels[b] - levels[a]) >= 2 * LEVEL_STEP:
                        j = jl
                shift = probe - j
            else:
                placed = calibrated  # extinct: no calibration, midpoints from here on
    return lo, hi


def drive(searches, spec: RunSpec, grid: Grid, runner=None, log=None):
    """Run searches in lockstep. `searches` maps a name to (generator, d,
    stream); every round simulates the pending probe of each unfinished
    search in one batched run (`runner(spec, [(p, d, stream)])` ->
    (times, [rho])). Returns {name: ((lo, hi), ledger)}."""
    runner = runner or simulate_curves
    state = {}
    rounds = 0
    for name, (gen, d, st) in searches.items():
        try:
            state[name] = [gen, d, st, next(gen), Ledger(), {}, None]
        except StopIteration as e:
            state[name] = [None, d, st, None, Ledger(), {}, e.value]
    while True:
        live = [n for n, v in state.items() if v[0] is not None]
        if not live:
            break
        todo = [n for n in live if state[n][3] not in state[n][5]]
        if todo:
            times, rhos = runner(spec, [(grid.p[state[n][3]], state[n][1], state[n][2]) for n in todo])
            rounds += 1
            if log:
                log(f"round {rounds}: simulated {len(todo)} probes "
                    f"{[(str(n), int(state[n][3])) for n in todo]}")
            for n, rho in zip(todo, rhos):
                i = state[n][3]
                ina = classify(times, rho)
                state[n][5][i] = (times, rho, ina)
                _record(state[n][4], grid, i, times, rho, ina, spec)
        for n in live:
            v = state[n]
            try:
                v[3] = v[0].send(v[5][v[3]])
            except StopIteration as e:
                v[0], v[6] = None, e.value
    return {n: (tuple(v[6]), v[4]) for n, v in state.items()}


def _sequential(runner):
    """Adapt a one-curve runner(spec, p, d, stream) to drive()."""
    def run(spec, probes):
        out = [runner(spec, p, d, st) for p, d, st in probes]
        return out[0][0], [r for _, r in out]
    return run


def plain_bisect(d, d_idx, grid: Grid, spec: RunSpec, runner=simulate_curve,
                 lo: int = 0, hi: Optional[int] = None):
    """Plain bisection alone; returns ((lo, hi), ledger)."""
    hi = len(grid) - 1 if hi is None else hi
    res = drive({"plain": (plain_steps(grid, lo, hi), d, d_idx)}, spec, grid,
                _sequential(runner))
    return res["plain"]


def predicted_class(times, log10_rho, flip_level: float = DELTA_HIGH) -> bool:
    """Class of a surrogate curve for placing probes: inactive when its
    delta_eff over the last half-decade exceeds `flip_level`. The network
    reproduces the level of delta_eff near p_c (about 0.2 at p_c, 1/2 for
    decaying runs) better than the change of delta_eff between half-decades,
    on which classify() also relies; simulated runs are classified by
    classify(). `flip_level` is the level at which classify() turns to
    inactive on the training curves of this d (flip_levels), DELTA_HIGH
    without one."""
    r = 10.0 ** np.asarray(log10_rho, float)
    return bool(delta_eff_windows(times, r)[1] > flip_level)


def flip_levels(p, d, t, y, m, times):
    """For each d of a training set, the delta_eff level (last half-decade)
    that best separates its curves into the classes classify() gives them:
    the threshold with the fewest curves on the wrong side. Rows are
    (p, d, t, log10 rho, mask); a curve is the rows of one (p, d). Returns
    {d: level}."""
    p, d, t, y, m = (np.asarray(a, float) for a in (p, d, t, y, m))
    out = {}
    for dv in np.unique(d):
        sel = d == dv
        pc, inv = np.unique(p[sel], return_inverse=True)
        levels, classes = [], []
        for c in range(len(pc)):
            rows = np.nonzero(inv == c)[0]
            order = np.argsort(t[sel][rows])
            tt = t[sel][rows][order]
            rho = np.where(m[sel][rows][order] > 0, 10.0 ** y[sel][rows][order], 0.0)
            if len(tt) != len(times):
                continue
            ina = classify(tt, rho)
            lvl = delta_eff_windows(tt, rho)[1] if rho[-1] > 0 else np.inf
            levels.append(lvl)
            classes.append(ina)
        levels, classes = np.asarray(levels), np.asarray(classes, bool)
        finite = np.sort(np.unique(levels[np.isfinite(levels)]))
        if finite.size < 2:
            out[float(dv)] = DELTA_HIGH
            continue
        cands = 0.5 * (finite[1:] + finite[:-1])
        errors = np.array([int(np.sum((levels > c) != classes)) for c in cands])
        # the middle of the run of candidates with the fewest errors
        best = np.nonzero(errors == errors.min())[0]
        out[float(dv)] = float(0.5 * (cands[best[0]] + cands[best[-1]]))
    return out


def level_for(flip: Optional[dict], d: float) -> float:
    """flip_levels value for d (linear in d between the training d values)."""
    if not flip:
        return DELTA_HIGH
    ds = np.array(sorted(flip), float)
    return float(np.interp(d, ds, [flip[k] for k in sorted(flip)]))


def predicted_classes(net, d, idx: Sequence[int], grid: Grid, spec: RunSpec,
                      flip: Optional[dict] = None):
    """Surrogate curves log10 rho(p_j, d, t_k) and their classes
    (predicted_class at the flip level for d) for grid indices idx."""
    import torch

    times = np.asarray(spec.times(), float)
    P = np.repeat(grid.p[np.asarray(idx)], len(times))
    T = np.tile(times, len(idx))
    x = torch.from_numpy(features(P, d, T)).cuda()
    y = net.predict(x).cpu().numpy().astype(np.float64).reshape(len(idx), len(times))
    lvl = level_for(flip, d)
    cls = [predicted_class(times, y[k], lvl) for k in range(len(idx))]
    return y, np.array(cls, dtype=bool)


def surrogate_bisect(net, d, d_idx, grid: Grid, spec: RunSpec, runner=simulate_curve,
                     lo: int = 0, hi: Optional[int] = None, predictor=None,
                     calibrated: int = CALIBRATED_PROBES, domain=None,
                     calibration: str = "crossing"):
    """The surrogate-guided search alone; `predictor(d, idx)` -> (log10 rho
    [len(idx), times], classes) replaces the network (tests). `domain` is the
    network's training p range (see restrict_to_domain)."""
    hi = len(grid) - 1 if hi is None else hi
    predictor = predictor or (lambda dd, idx: predicted_classes(net, dd, idx, grid, spec))
    ys, cls = restrict_to_domain(*predictor(d, list(range(len(grid)))), grid, domain)
    gen = surrogate_steps(ys, cls, grid, spec.times(), lo, hi, calibrated, calibration)
    res = drive({"surrogate": (gen, d, d_idx)}, spec, grid, _sequential(runner))
    return res["surrogate"]


# --------------------------------------------------------------------------
# training data from the simulator and training on the GPU


def training_batch(count: int, spec: RunSpec, seed: int, d_values=(0.1, 0.5, 0.9),
                   p_range=(0.05, 0.25), L_range=(1 << 14, 1 << 16)):
    """Instances of one batched run (config-3 style: uneven L, d from a set,
    p uniform), drawn from numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log2(L_range[0]), math.log2(L_range[1]), size=count)
    ds = rng.choice(np.asarray(d_values, float), size=count)
    ps = rng.uniform(p_range[0], p_range[1], size=count)
    insts = [workloads.Instance(float(ps[i]), float(ds[i]), 64 * int(2.0 ** u[i] // 64), i)
             for i in range(count)]
    return insts


def training_rows(insts, times):
    """(p, d, t) of every row of simulate_training_set, in its order."""
    P = np.array([i.p for i in insts], float)[None, :].repeat(len(times), 0)
    D = np.array([i.d for i in insts], float)[None, :].repeat(len(times), 0)
    T = np.asarray(times, float)[:, None].repeat(len(insts), 1)
    return P.ravel(), D.ravel(), T.ravel()


def simulate_training_set(insts, spec: RunSpec, seed: int, graph: bool = True):
    """One batched GPU run of all instances (one plane each) with records at
    spec.times(); returns (features [n,3], log10 rho [n], mask [n], site updates)."""
    from . import pcpd

    times = spec.times()
    with pcpd.Sim(spec.model, spec.B, 1, seed, insts) as sim:
        sim.set_options(graph=graph)
        c = sim.run(times)
    N = c[:, :, 0, 0].astype(np.float64)                       # [times, inst]
    L = np.array([i.L for i in insts], float)
    rho = N / (64.0 * L[None, :])
    x = features(*training_rows(insts, times))
    mask = (rho.ravel() > 0).astype(np.float32)
    y = np.log10(np.where(rho.ravel() > 0, rho.ravel(), 1.0)).astype(np.float32)
    su = int(sum(64 * i.L for i in insts) * spec.steps)
    return x, y, mask, su


def train(net, x, y, mask, epochs: int = 200, batch: int = 8192, lr: float = 2e-3,
          seed: int = 0, log: Optional[Callable[[str], None]] = None):
    """Minibatch Adam on the GPU; returns the final full-set loss."""
    import torch

    rng = np.random.default_rng(seed)
    X = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    Y = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    M = torch.from_numpy(np.ascontiguousarray(mask, np.float32)).cuda()
    n = X.shape[0]
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        step_lr = lr * (0.5 * (1 + math.cos(math.pi * ep / epochs)) * 0.9 + 0.1)
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            net.train_step(X[idx].contiguous(), Y[idx].contiguous(), M[idx].contiguous(), lr=step_lr)
        if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {net.loss(X, Y, M):.5f}")
    return net.loss(X, Y, M)


# --------------------------------------------------------------------------
# end-to-end comparison


def build_surrogate(d_values=(0.1, 0.5, 0.9), spec: Optional[RunSpec] = None,
                    train_count: int = 512, train_batches: int = 2, train_L=(1 << 14, 1 << 16),
                    epochs: int = 150, seed: int = 2013, log=print, p_range=(0.04, 0.30),
                    data_path: Optional[str] = None, max_data_s: float = float("inf")):
    """Simulate the training curves (batched runs at the search's horizon) and
    train a surrogate on them. Returns (net, training summary). With
    `data_path`, the simulated set (features, targets, mask, site updates) is
    read from that .npz file if it exists, else written there, each batch
    also to a file of its own; batches not yet cached are simulated only
    while less than `max_data_s` seconds have passed (TimeoutError after)."""
    import os
    import time

    from . import pcpd

    spec = spec or RunSpec()
    t0 = time.perf_counter()
    if data_path and os.path.exists(data_path):
        with np.load(data_path) as z:
            P, D, T = z["p"], z["d"], z["t"]
            y, m, train_su = z["y"], z["m"], int(z["site_updates"])
        log(f"training set read from {data_path}: {len(y)} rows")
    else:
        raws, ys, ms, train_su = [], [], [], 0
        for b in range(train_batches):
            # each batch is cached on its own, so a long set can be simulated
            # over several processes
            bpath = f"{os.path.splitext(data_path)[0]}.b{b}.npz" if data_path else None
            if bpath and os.path.exists(bpath):
                with np.load(bpath) as z:
                    raw, y, m, su = (z["p"], z["d"], z["t"]), z["y"], z["m"], int(z["site_updates"])
            else:
                if time.perf_counter() - t0 > max_data_s:
                    raise TimeoutError(f"training batch {b}: time budget spent; cached batches "
                                       f"are kept, run again to continue")
                insts = training_batch(train_count, spec, seed + b, d_values=d_values,
                                       L_range=train_L, p_range=p_range)
                _, y, m, su = simulate_training_set(insts, spec, seed + b)
                raw = training_rows(insts, spec.times())
                if bpath:
                    np.savez(bpath, p=raw[0], d=raw[1], t=raw[2], y=y, m=m,
                             site_updates=np.int64(su))
            raws.append(raw), ys.append(y), ms.append(m)
            train_su += su
            log(f"training batch {b + 1}/{train_batches}: {len(y) // len(spec.times())} curves, "
                f"{time.perf_counter() - t0:.1f} s")
        P, D, T = (np.concatenate([r[k] for r in raws]) for k in range(3))
        y, m = np.concatenate(ys), np.concatenate(ms)
        if data_path:
            np.savez(data_path, p=P, d=D, t=T, y=y, m=m, site_updates=np.int64(train_su))
    x = features(P, D, T)
    t_data = time.perf_counter() - t0
    flip = flip_levels(P, D, T, y, m, spec.times())
    log(f"flip levels from the training curves: {flip}")
    net = pcpd.Surrogate(seed=seed)
    t1 = time.perf_counter()
    loss = train(net, x, y, m, epochs=epochs, seed=seed, log=log)
    t_train = time.perf_counter() - t1
    return net, {"curves": int(len(y) // len(spec.times())), "rows": int(len(y)),
                 "site_updates": train_su, "data_s": t_data, "train_s": t_train,
                 "final_loss": loss, "flip_levels": flip}


def run_searches(net, d_values, d_indices, spec: RunSpec, grid: Grid, log=print, runner=None,
                 predictor=None, domain=None, calibration: str = "crossing",
                 flip: Optional[dict] = None):
    """Plain and surrogate-guided searches for every d, all driven in
    lockstep (one batched GPU run per round), each with its own ledger and
    cache: no run is shared between searches. `domain` is the network's
    training p range. Returns one record per d."""
    import time

    predictor = predictor or (lambda dd, idx: predicted_classes(net, dd, idx, grid, spec, flip))
    hi = len(grid) - 1
    searches = {}
    for d, k in zip(d_values, d_indices):
        ys, cls = restrict_to_domain(*predictor(d, list(range(len(grid)))), grid, domain)
        searches[("plain", k)] = (plain_steps(grid, 0, hi), d, k)
        searches[("surrogate", k)] = (surrogate_steps(ys, cls, grid, spec.times(), 0, hi,
                                                      calibration=calibration), d, k)
    t0 = time.perf_counter()
    res = drive(searches, spec, grid, runner, log)
    wall = time.perf_counter() - t0
    out = []
    for d, k in zip(d_values, d_indices):
        pb, pl = res[("plain", k)]
        sb, sl = res[("surrogate", k)]
        log(f"d={d}: plain {pb} in {pl.runs} runs, surrogate {sb} in {sl.runs} runs")
        out.append({"d": d,
                    "plain": {"bracket": [float(grid.p[pb[0]]), float(grid.p[pb[1]])],
                              "idx": list(pb), "runs": pl.runs, "site_updates": pl.site_updates,
                              "path": pl.path},
                    "surrogate": {"bracket": [float(grid.p[sb[0]]), float(grid.p[sb[1]])],
                                  "idx": list(sb), "runs": sl.runs,
                                  "site_updates": sl.site_updates, "path": sl.path},
                    "same_bracket": pb == sb,
                    "gain": pl.site_updates / max(sl.site_updates, 1),
                    "wall_s_all_searches": wall})
    return out


def compare(d_values=(0.1, 0.5, 0.9), spec: Optional[RunSpec] = None, bits: int = 10,
            train_count: int = 512, train_batches: int = 2, train_L=(1 << 14, 1 << 16),
            epochs: int = 150, seed: int = 2013, log=print, p_range=(0.04, 0.30)):
    """Train the surrogate on simulator curves, then search p_c for each d both
    ways. Returns a summary dict; training site updates are reported
    separately from the searches'."""
    spec = spec or RunSpec()
    grid = Grid(bits=bits)
    net, training = build_surrogate(d_values, spec, train_count, train_batches, train_L,
                                    epochs, seed, log, p_range=p_range)
    out = {"spec": {"L": spec.L, "planes": spec.planes, "steps": spec.steps, "grid": len(grid),
                    "p_range": [float(grid.p[0]), float(grid.p[-1])]},
           "training": training, "searches": []}
    try:
        out["searches"] = run_searches(net, d_values, range(len(d_values)), spec, grid, log,
                                       domain=p_range)
    finally:
        net.close()
    return out


def main(argv=None):
    import argparse
    import json
    import os

    ap = argparse.ArgumentParser(description="p_c search, plain vs surrogate-guided")
    ap.add_argument("--L", type=int, default=1 << 18)
    ap.add_argument("--planes", type=int, default=4)
    ap.add_argument("--steps", type=int, default=1_000_000)
    ap.add_argument("--bits", type=int, default=10)
    ap.add_argument("--train-count", type=int, default=512)
    ap.add_argument("--train-batches", type=int, default=2)
    ap.add_argument("--train-L", type=str, default="16384,65536")
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--d", type=str, default="0.1,0.5,0.9")
    ap.add_argument("--d-index", type=str, default=None,
                    help="comma-separated indices into --d to search (default: all)")
    ap.add_argument("--save-net", type=str, default=None, help="write trained parameters (.npy)")
    ap.add_argument("--load-net", type=str, default=None, help="read parameters, skip training")
    ap.add_argument("--train-only", action="store_true")
    ap.add_argument("--train-p", type=str, default="0.04,0.30",
                    help="p range of the training curves, also the range where the network's "
                         "predictions are trusted (give the loaded network's with --load-net)")
    ap.add_argument("--train-data", type=str, default=None,
                    help="training set cache (.npz): read if present, else simulated and written")
    ap.add_argument("--train-d", type=str, default=None,
                    help="d values of the training curves (default: the searched --d)")
    ap.add_argument("--calibration", choices=("crossing", "level", "shape"), default="crossing",
                    help="how a simulated probe is placed on the network's p axis")
    ap.add_argument("--seed", type=int, default=2013, help="training set and network seed")
    ap.add_argument("--max-data-s", type=float, default=float("inf"),
                    help="stop simulating training batches after this many seconds "
                         "(cached batches are kept; run again to continue)")
    ap.add_argument("--no-flip-levels", action="store_true",
                    help="place probes with the fixed level DELTA_HIGH, not the learned ones")
    a = ap.parse_args(argv)
    from . import pcpd

    log = lambda s: print(s, flush=True)  # noqa: E731
    spec = RunSpec(L=a.L, planes=a.planes, steps=a.steps)
    grid = Grid(bits=a.bits)
    d_values = tuple(float(v) for v in a.d.split(","))
    res = {"spec": {"L": spec.L, "planes": spec.planes, "steps": spec.steps, "grid": len(grid),
                    "p_range": [float(grid.p[0]), float(grid.p[-1])]},
           "training": None, "searches": []}
    flip = None
    if a.load_net:
        net = pcpd.Surrogate(seed=0)
        net.set_params(np.load(a.load_net))
        meta = os.path.splitext(a.load_net)[0] + ".json"
        if os.path.exists(meta):
            with open(meta) as f:
                flip = {float(k): float(v) for k, v in json.load(f)["flip_levels"].items()}
    else:
        train_d = d_values if a.train_d is None else tuple(float(v) for v in a.train_d.split(","))
        net, res["training"] = build_surrogate(
            train_d, spec, a.train_count, a.train_batches,
            tuple(int(v) for v in a.train_L.split(",")), a.epochs, seed=a.seed, log=log,
            p_range=tuple(float(v) for v in a.train_p.split(",")), data_path=a.train_data,
            max_data_s=a.max_data_s)
        print(json.dumps({"training": res["training"]}), flush=True)
        flip = res["training"]["flip_levels"]
    if a.save_net:
        np.save(a.save_net, net.params())
        with open(os.path.splitext(a.save_net)[0] + ".json", "w") as f:
            json.dump({"flip_levels": {str(k): v for k, v in (flip or {}).items()},
                       "train_p": [float(v) for v in a.train_p.split(",")],
                       "train_d": a.train_d or a.d, "train_L": a.train_L,
                       "spec": {"L": spec.L, "planes": spec.planes, "steps": spec.steps,
                                "bits": a.bits}}, f, indent=1)
    if not a.train_only:
        keep = range(len(d_values)) if a.d_index is None else [int(v) for v in a.d_index.split(",")]
        res["searches"] = run_searches(net, [d_values[k] for k in keep], list(keep), spec, grid,
                                       log, domain=tuple(float(v) for v in a.train_p.split(",")),
                                       calibration=a.calibration,
                                       flip=None if a.no_flip_levels else flip)
    net.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
