"""GPU parity: the HIP sweep (through the C ABI) against the CPU oracle,
bit-exact on lattice words and on every recorded count."""
import numpy as np
import pytest

from paper_1301_6082_amd import workloads as wl
from paper_1301_6082_amd.workloads import Instance

from gpu_common import aggregate_counts, oracle_runs, per_sample_counts

pytestmark = pytest.mark.gpu

FULL = (1 << 64) - 1


@pytest.fixture(scope="module")
def pcpd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_6082_amd import pcpd as mod
    return mod


def _compare_full(pcpd, model, B, planes, seed, instances, times, tuning=None, t0=0,
                  options=None, layout=0, mask_bits=2):
    """GPU run with records at `times` vs the oracle on every plane, all samples."""
    print(f"[parity] model={model} B={B} planes={planes} n_inst={len(instances)} "
          f"L={[i.L for i in instances]} times={times[:4]}..{times[-1]} tuning={tuning} "
          f"options={options} layout={layout} mask_bits={mask_bits}", flush=True)
    with pcpd.Sim(model, B, planes, seed, instances, t0=t0, layout=layout,
                  mask_bits=mask_bits) as sim:
        if tuning:
            sim.set_tuning(*tuning)
        if options:
            sim.set_options(**options)
        counts = sim.run(times)
        lat = [sim.get_lattice(i) for i in range(len(instances))]
    keys, runs = oracle_runs(model, B, planes, seed, instances, times, t0=t0,
                             connected=layout == 1, mask_bits=mask_bits)
    for (i, q), r in zip(keys, runs):
        L = instances[i].L
        np.testing.assert_array_equal(lat[i][q * L:(q + 1) * L], r.words,
                                      err_msg=f"lattice inst {i} plane {q}")
        N, NP, alive = r.counts()
        np.testing.assert_array_equal(counts[:, i, q, 0], N, err_msg=f"N inst {i} plane {q}")
        np.testing.assert_array_equal(counts[:, i, q, 1], NP, err_msg=f"Npair inst {i} plane {q}")
        np.testing.assert_array_equal(counts[:, i, q, 2], alive, err_msg=f"alive {i} {q}")
    return counts, lat


def test_cfg1_full_parity(pcpd):
    """PCPD ring L=1024, d=0.5, p=0.1, 1000 MC steps, all 100 records."""
    c = wl.cfg1()
    counts, _ = _compare_full(pcpd, c.model, c.B, c.planes, c.seed, c.instances,
                              [0] + c.times)
    assert counts[0, 0, 0, 0] == 64 * 1024


def test_several_tiles_and_ragged_tail(pcpd):
    # 537 blocks: four full 116-block tiles and a ragged 73-block tile per plane
    insts = [Instance(0.13, 0.3, 64 * 537, 0), Instance(0.2, 0.7, 64 * 300, 5)]
    _compare_full(pcpd, 2, 64, 2, 7, insts, [0, 1, 3, 12])


@pytest.mark.parametrize("teams", [2, 4])
@pytest.mark.parametrize("model", [1, 3, 4])
def test_dp_tcpd_qcpd_parity(pcpd, model, teams):
    insts = [Instance(0.08, 0.5, 64 * 260, 1), Instance(0.3, 0.1, 64 * 17, 2)]
    _compare_full(pcpd, model, 64, 1, 3, insts, [2, 9], tuning=(0, 0, teams))


@pytest.mark.parametrize("teams", [2, 4])
@pytest.mark.parametrize("shape", [(256, 64), (128, 64), (64, 16), (9, 1), (40, 7), (200, 33),
                                   (128, 128), (96, 61)])
def test_tile_shape_does_not_change_results(pcpd, shape, teams):
    """Tile width, phase length (including phases that end inside a group of
    substeps) and team count never change the results."""
    insts = [Instance(0.12, 0.4, 64 * 301, 3)]
    _compare_full(pcpd, 2, 64, 1, 11, insts, [4], tuning=(*shape, teams))


@pytest.mark.parametrize("teams", [2, 4])
@pytest.mark.parametrize("L,B,model", [(4, 4, 2), (5, 5, 2), (8, 4, 2), (6, 6, 3), (3, 3, 1),
                                       (192, 192, 2), (96, 32, 2), (1000, 8, 2), (6, 6, 4),
                                       (7, 7, 4), (12, 6, 4), (1200, 12, 4)])
def test_small_rings_and_block_widths(pcpd, L, B, model, teams):
    insts = [Instance(0.2, 0.3, L, 0), Instance(0.05, 0.9, L, 1)]
    _compare_full(pcpd, model, B, 2, 1, insts, [1, 2, 17], tuning=(0, 0, teams))


@pytest.mark.parametrize("teams", [2, 4])
@pytest.mark.parametrize("L,B,model", [(32 * 700, 32, 2), (96 * 150, 96, 2), (16 * 1500, 16, 3),
                                       (64 * 700, 64, 1), (15 * 1400, 15, 2), (9 * 2000, 9, 3),
                                       (64 * 700, 64, 4), (11 * 1800, 11, 4)])
def test_block_widths_over_many_tiles(pcpd, L, B, model, teams):
    """Block widths other than 64 over many tiles per ring: even widths move
    tiles as 16-byte site pairs, odd widths one word at a time."""
    insts = [Instance(0.15, 0.4, L, 5), Instance(0.1, 0.7, L + 2 * B, 6)]
    _compare_full(pcpd, model, B, 2, 4, insts, [3, 10], tuning=(0, 0, teams))


def test_host_init_resume_and_chunking(pcpd):
    L = 64 * 40
    start = wl.random_lattice(L, 2, 0.4, 21)
    insts = [Instance(0.1, 0.25, L, 4, wl.INIT_HOST, start)]
    # one run to 30 vs 7 + 23 via a stored lattice and t0 = 7
    with pcpd.Sim(2, 64, 2, 5, insts) as sim:
        sim.sweep(7)
        mid = sim.get_lattice(0)
        assert sim.time == 7
        sim.sweep(10)
        sim.sweep(13)
        end = sim.get_lattice(0)
    resumed = [Instance(0.1, 0.25, L, 4, wl.INIT_HOST, mid)]
    with pcpd.Sim(2, 64, 2, 5, resumed, t0=7) as sim:
        sim.sweep(23)
        end2 = sim.get_lattice(0)
        dens = sim.density()
    np.testing.assert_array_equal(end, end2)
    keys, runs = oracle_runs(2, 64, 2, 5, insts, [30])
    for (i, q), r in zip(keys, runs):
        np.testing.assert_array_equal(end[q * L:(q + 1) * L], r.words)
        N, NP, alive = r.counts()
        assert (dens[0, q] == [N[0], NP[0], alive[0]]).all()


def test_set_lattice_then_sweep(pcpd):
    L = 64 * 20
    a = wl.random_lattice(L, 1, 0.5, 3)
    insts = [Instance(0.15, 0.5, L, 0)]
    with pcpd.Sim(2, 64, 1, 9, insts) as sim:
        sim.set_lattice(0, a)
        np.testing.assert_array_equal(sim.get_lattice(0), a)
        sim.sweep(5)
        got = sim.get_lattice(0)
    host = [Instance(0.15, 0.5, L, 0, wl.INIT_HOST, a)]
    _, runs = oracle_runs(2, 64, 1, 9, host, [5])
    np.testing.assert_array_equal(got, runs[0].words)


def test_empty_and_absorbing(pcpd):
    insts = [Instance(0.1, 0.5, 64 * 10, 0, wl.INIT_EMPTY)]
    with pcpd.Sim(2, 64, 1, 1, insts) as sim:
        c = sim.run([0, 5, 50])
        assert (c == 0).all()
        assert (sim.get_lattice(0) == 0).all()


def test_density_kernel_matches_lattice(pcpd):
    L = 64 * 700
    insts = [Instance(0.11, 0.2, L, 0, wl.INIT_HOST, wl.random_lattice(L, 3, 0.3, 8))]
    with pcpd.Sim(2, 64, 3, 1, insts) as sim:
        sim.sweep(3)
        dens = sim.density()
        words = sim.get_lattice(0)
    for q in range(3):
        assert tuple(int(x) for x in dens[0, q]) == aggregate_counts(words[q * L:(q + 1) * L])


def test_cfg2_full_size_sampled(pcpd):
    """The full PCPD L=2^20, 4-plane, 16-p workload in the benchmark's launch
    shape, 8 MC steps with records at t = 1..8; sampled (instance, plane,
    sample) trajectories against the oracle, every site, every record, plus
    count properties on all planes."""
    c = wl.cfg2()
    times = [1, 2, 3, 4, 5, 6, 7, 8]
    picks = [(0, 0, 0), (5, 3, 17), (9, 1, 63), (15, 2, 40), (15, 0, 5), (11, 3, 31)]
    snaps = {}
    with pcpd.Sim(c.model, c.B, c.planes, c.seed, c.instances) as sim:
        counts = sim.run([0])
        assert (counts[0, :, :, 0] == 64 * (1 << 20)).all()
        for t in times:
            counts = sim.run([t])
            for (i, q, b) in picks:
                w = sim.get_lattice(i)[q << 20:(q + 1) << 20]
                snaps[(i, q, b, t)] = (w >> np.uint64(b)) & np.uint64(1)
            # properties of every plane
            n, npair = counts[0, :, :, 0], counts[0, :, :, 1]
            assert (npair <= n).all() and (n <= 64 * (1 << 20)).all()
    which = [(i, q) for (i, q, _) in picks]
    for k, (i, q, b) in enumerate(picks):
        _, runs = oracle_runs(c.model, c.B, c.planes, c.seed, c.instances, times,
                              samples=1 << b, which=[(i, q)])
        r = runs[0]
        final = (r.words >> np.uint64(b)) & np.uint64(1)
        np.testing.assert_array_equal(snaps[(i, q, b, times[-1])], final,
                                      err_msg=f"inst {i} plane {q} sample {b}")
        for ti, t in enumerate(times):
            bits = snaps[(i, q, b, t)].astype(np.int64)
            assert bits.sum() == int(r.n[ti, b]), (i, q, b, t)
            assert (bits & np.roll(bits, -1)).sum() == int(r.pair[ti, b]), (i, q, b, t)
    assert len(which) == len(picks)


def test_cfg4_tcpd_full_size_sampled(pcpd):
    """TCPD ring L=2^18, 8 p values, 32 MC steps; one sample of every instance."""
    c = wl.cfg4()
    with pcpd.Sim(c.model, c.B, c.planes, c.seed, c.instances) as sim:
        counts = sim.run([32])
        lat = [sim.get_lattice(i) for i in range(len(c.instances))]
    for i in range(len(c.instances)):
        b = (7 * i + 3) % 64
        _, runs = oracle_runs(c.model, c.B, 1, c.seed, c.instances, [32], samples=1 << b,
                              which=[(i, 0)])
        np.testing.assert_array_equal(lat[i] & np.uint64(1 << b), runs[0].words)
        assert tuple(int(x) for x in counts[0, i, 0]) == aggregate_counts(lat[i])


def test_cfg3_batch_sampled(pcpd):
    """The 512-instance batch of uneven L in one context: sampled instances,
    all 64 samples, against the oracle run alone."""
    c = wl.cfg3()
    times = [4, 16]
    with pcpd.Sim(c.model, c.B, c.planes, c.seed, c.instances) as sim:
        counts = sim.run(times)
        Ls = np.array([i.L for i in c.instances])
        picks = [int(np.argmin(Ls)), 7, 100, 255, 511]
        lat = {i: sim.get_lattice(i) for i in picks}
    for i in picks:
        samples = FULL if Ls[i] <= 20000 else (1 << 3) | (1 << 60)
        _, runs = oracle_runs(c.model, c.B, 1, c.seed, c.instances, times, samples=samples,
                              which=[(i, 0)])
        r = runs[0]
        np.testing.assert_array_equal(lat[i] & np.uint64(samples), r.words, err_msg=f"inst {i}")
        if samples == FULL:
            N, NP, alive = r.counts()
            np.testing.assert_array_equal(counts[:, i, 0, 0], N)
            np.testing.assert_array_equal(counts[:, i, 0, 1], NP)
            np.testing.assert_array_equal(counts[:, i, 0, 2], alive)
        else:
            n, pair = per_sample_counts(lat[i])
            for b in (3, 60):
                assert n[b] == r.n[-1, b] and pair[b] == r.pair[-1, b]


def test_profiling_does_not_change_results(pcpd):
    insts = [Instance(0.12, 0.4, 64 * 301, 3)]
    out = []
    for prof in (False, True):
        with pcpd.Sim(2, 64, 1, 11, insts) as sim:
            sim.profile(prof)
            sim.sweep(6)
            ms, n = sim.profile_read()
            out.append(sim.get_lattice(0))
            if prof:
                assert n == -(-6 * 64 // sim.get_tuning()[1]) and ms > 0
            else:
                assert n == 0
    np.testing.assert_array_equal(out[0], out[1])


def test_graph_replays_match_direct_launches(pcpd):
    """PCPD_OPT_GRAPH: segments of a fixed number of steps are captured once
    and replayed (phases of 4 substeps: 16 steps per segment, so every run
    below replays segments and launches remainders and records directly);
    every replay, with eager work between replays, must equal direct
    launches."""
    insts = [Instance(0.1, 0.3, 64 * 200, 0), Instance(0.22, 0.6, 64 * 37, 1)]
    with pcpd.Sim(2, 64, 2, 4, insts) as g, pcpd.Sim(2, 64, 2, 4, insts) as d:
        g.set_tuning(128, 4)
        g.set_options(graph=True)
        for rep in range(4):
            t = g.time
            sched = [t + 20, t + 40, t + 75]
            cg, cd = g.run(sched), d.run(sched)
            np.testing.assert_array_equal(cg, cd, err_msg=f"replay {rep}")
            for i in range(2):
                np.testing.assert_array_equal(g.get_lattice(i), d.get_lattice(i))
            if rep == 1:
                g.sweep(1)   # eager work between replays (flips the copy parity)
                d.sweep(1)
        assert g.time == d.time
        final = [g.get_lattice(i) for i in range(2)]
        T = g.time
    keys, runs = oracle_runs(2, 64, 2, 4, insts, [T])
    for (i, q), r in zip(keys, runs):
        L = insts[i].L
        np.testing.assert_array_equal(final[i][q * L:(q + 1) * L], r.words)


def test_autotune_keeps_results(pcpd):
    insts = [Instance(0.12, 0.4, 64 * 1500, 3), Instance(0.2, 0.1, 64 * 300, 4)]
    with pcpd.Sim(2, 64, 1, 11, insts) as sim:
        before = sim.get_lattice(0)
        chosen = sim.autotune(reps=2)
        assert sim.get_tuning() == chosen
        np.testing.assert_array_equal(sim.get_lattice(0), before)   # trials leave the state
        counts = sim.run([3, 6])
        lat = [sim.get_lattice(i) for i in range(2)]
    print(f"[autotune] chose {chosen}", flush=True)
    keys, runs = oracle_runs(2, 64, 1, 11, insts, [3, 6])
    for (i, q), r in zip(keys, runs):
        np.testing.assert_array_equal(lat[i], r.words)
        N, NP, alive = r.counts()
        np.testing.assert_array_equal(counts[:, i, 0, 0], N)


def test_batch_in_one_graph_launch_matches_instances_alone(pcpd):
    """Instances of uneven L batched in one context and one graph launch per
    run give the same lattices as each instance in a context of its own."""
    c = wl.cfg3(count=24)
    with pcpd.Sim(c.model, c.B, 1, c.seed, c.instances) as sim:
        sim.set_tuning(128, 4)   # 16-step graph segments
        sim.set_options(graph=True)
        batch = sim.run([5, 40])
        lat = [sim.get_lattice(i) for i in range(len(c.instances))]
    for i in (0, 5, 17, 23):
        with pcpd.Sim(c.model, c.B, 1, c.seed, [c.instances[i]]) as alone:
            a = alone.run([5, 40])
            np.testing.assert_array_equal(alone.get_lattice(0), lat[i], err_msg=f"inst {i}")
            np.testing.assert_array_equal(a[:, 0], batch[:, i])


# ---- persistent launches ----------------------------------------------------

@pytest.mark.parametrize("teams", [2, 4])
@pytest.mark.parametrize("shape", [(128, 128), (64, 16), (40, 7), (200, 33), (9, 1)])
def test_persistent_launch_matches_oracle(pcpd, shape, teams):
    """All phases between records in one ticket-dispatched launch: rings of
    many tiles, one tile, and fewer blocks than the halo (every tile depends
    on every other), with phases that end inside a group of substeps."""
    insts = [Instance(0.12, 0.4, 64 * 301, 3), Instance(0.2, 0.1, 64 * 7, 4),
             Instance(0.05, 0.8, 64 * 1200, 5)]
    _compare_full(pcpd, 2, 64, 2, 11, insts, [0, 1, 4, 13], tuning=(*shape, teams),
                  options={"persistent": True})


@pytest.mark.parametrize("L,B,model", [(64 * 260, 64, 1), (64 * 260, 64, 3), (64 * 260, 64, 4),
                                       (15 * 1400, 15, 2), (1000, 8, 2), (6, 6, 4)])
def test_persistent_launch_models_and_block_widths(pcpd, L, B, model):
    insts = [Instance(0.15, 0.4, L, 5), Instance(0.1, 0.7, L + 2 * B, 6)]
    _compare_full(pcpd, model, B, 2, 4, insts, [3, 10], options={"persistent": True})


def test_persistent_launch_in_graphs_matches_direct(pcpd):
    """Persistent launches captured in graph segments and replayed, with
    eager work between replays, against direct per-phase launches."""
    insts = [Instance(0.1, 0.3, 64 * 200, 0), Instance(0.22, 0.6, 64 * 37, 1)]
    with pcpd.Sim(2, 64, 2, 4, insts) as g, pcpd.Sim(2, 64, 2, 4, insts) as d:
        g.set_tuning(128, 4)
        g.set_options(graph=True, persistent=True)
        for rep in range(3):
            t = g.time
            sched = [t + 20, t + 40, t + 75]
            cg, cd = g.run(sched), d.run(sched)
            np.testing.assert_array_equal(cg, cd, err_msg=f"replay {rep}")
            for i in range(2):
                np.testing.assert_array_equal(g.get_lattice(i), d.get_lattice(i))
            if rep == 0:
                g.sweep(1)
                d.sweep(1)


def test_persistent_cfg3_batch_matches_direct(pcpd):
    """The 512 uneven rings of the batched workload: persistent launches
    against per-phase launches, lattices and counts at every record."""
    c = wl.cfg3()
    times = [3, 8]
    with pcpd.Sim(c.model, c.B, c.planes, c.seed, c.instances) as p, \
            pcpd.Sim(c.model, c.B, c.planes, c.seed, c.instances) as d:
        p.set_options(persistent=True)
        cp, cd = p.run(times), d.run(times)
        np.testing.assert_array_equal(cp, cd)
        for i in (0, 77, 300, 511):
            np.testing.assert_array_equal(p.get_lattice(i), d.get_lattice(i), err_msg=f"inst {i}")


# ---- connected multispin layout ----------------------------------------------

@pytest.mark.parametrize("teams", [2, 4])
@pytest.mark.parametrize("shape", [(128, 128), (64, 16), (40, 7), (9, 1)])
def test_connected_layout_matches_oracle(pcpd, shape, teams):
    """The 64 bits of each plane joined into one ring (paper Sec. 4): rings of
    many tiles, of one tile, and of fewer blocks than the halo (columns many
    laps around the word ring, each rotated by its lap count)."""
    insts = [Instance(0.12, 0.4, 64 * 301, 3), Instance(0.2, 0.1, 64 * 7, 4),
             Instance(0.05, 0.8, 64 * 1200, 5), Instance(0.3, 0.5, 64, 6)]
    _compare_full(pcpd, 2, 64, 2, 11, insts, [0, 1, 4, 9], tuning=(*shape, teams), layout=1)


@pytest.mark.parametrize("L,B,model", [(64 * 260, 64, 1), (64 * 260, 64, 3), (64 * 40, 64, 4),
                                       (15 * 1400, 15, 2), (1000, 8, 2), (6, 6, 4), (12, 4, 2)])
def test_connected_layout_models_and_block_widths(pcpd, L, B, model):
    start = wl.random_lattice(L, 2, 0.5, 77)
    insts = [Instance(0.15, 0.4, L, 5, wl.INIT_HOST, start), Instance(0.1, 0.7, L, 6)]
    _compare_full(pcpd, model, B, 2, 4, insts, [3, 10], layout=1)


def test_connected_layout_persistent_and_graph(pcpd):
    insts = [Instance(0.1, 0.3, 64 * 200, 0), Instance(0.22, 0.6, 64 * 37, 1)]
    _compare_full(pcpd, 2, 64, 2, 4, insts, [2, 5, 11], tuning=(64, 16, 2),
                  options={"persistent": True}, layout=1)
    _compare_full(pcpd, 2, 64, 2, 4, insts, [2, 40], tuning=(128, 4, 2),
                  options={"graph": True}, layout=1)


# ---- empty-tile skip ------------------------------------------------------------

def _clustered(L, planes, centres, width, seed):
    """Host start: all words empty except random words in a few clusters (so
    that some tiles of a phase hold particles and the rest do not)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(planes * L, dtype=np.uint64)
    for q in range(planes):
        for c in centres:
            lo = q * L + (c % L)
            for j in range(width):
                w[q * L + (c + j) % L] = rng.integers(0, 1 << 63, dtype=np.uint64) | np.uint64(1)
    return w


@pytest.mark.parametrize("model", [1, 2, 3])
@pytest.mark.parametrize("shape", [(128, 128, 2), (64, 16, 4), (40, 7, 2)])
def test_skip_empty_tiles_matches_oracle(pcpd, model, shape):
    """Sparse states: particles in a few clusters of a long ring, empty tiles
    in between that the clusters grow into; every record and the final lattice
    bit-exact against the oracle with empty tiles skipped."""
    L = 64 * 900
    start = _clustered(L, 2, [100, 20000, 40000 + 33, L - 10], 12, 5)
    insts = [Instance(0.1, 0.5, L, 2, wl.INIT_HOST, start),
             Instance(0.25, 0.2, L, 3, wl.INIT_HOST, start),
             Instance(0.1, 0.5, 64 * 5, 4, wl.INIT_EMPTY)]
    _compare_full(pcpd, model, 64, 2, 9, insts, [1, 2, 5, 12], tuning=shape,
                  options={"skip_empty": True})


def test_skip_empty_tiles_through_extinction(pcpd):
    """Small rings deep in the absorbing phase die out; from then on every
    tile is skipped, before that only some. Direct, persistent and graph
    launches, and the connected layout."""
    insts = [Instance(0.6, 0.1, 64 * 12, k) for k in range(6)] + \
            [Instance(0.3, 0.5, 64 * 300, 7), Instance(0.9, 0.05, 64 * 40, 8)]
    times = [1, 4, 16, 64, 200]
    _compare_full(pcpd, 2, 64, 1, 3, insts, times, options={"skip_empty": True})
    _compare_full(pcpd, 2, 64, 1, 3, insts, times, tuning=(64, 32, 2),
                  options={"skip_empty": True, "persistent": True})
    _compare_full(pcpd, 2, 64, 1, 3, insts, times, options={"skip_empty": True, "graph": True})
    _compare_full(pcpd, 2, 64, 1, 3, insts, times, options={"skip_empty": True}, layout=1)


def test_skip_option_change_drops_graphs(pcpd):
    """Options switched between runs of one context (graphs captured before
    the change are not replayed after it): the trajectory is the oracle's."""
    L = 64 * 300
    start = _clustered(L, 1, [50, 9000], 20, 8)
    insts = [Instance(0.2, 0.4, L, 1, wl.INIT_HOST, start)]
    with pcpd.Sim(2, 64, 1, 6, insts) as sim:
        sim.set_tuning(64, 8, 2)
        sim.set_options(graph=True)
        sim.sweep(40)
        sim.set_options(graph=True, skip_empty=True)
        sim.sweep(40)
        sim.set_options(skip_empty=True)
        sim.sweep(7)
        got = sim.get_lattice(0)
    _, runs = oracle_runs(2, 64, 1, 6, insts, [87])
    np.testing.assert_array_equal(got, runs[0].words)


def test_autotune_disk_cache_and_forced_shape(pcpd, tmp_path, monkeypatch):
    """PCPD_TUNE_CACHE: a hand-written entry for this lattice forces its shape
    (no timing), the run matches the oracle; a lattice without an entry is
    timed and appended to the file."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    insts = [Instance(0.12, 0.4, 64 * 1300, 3), Instance(0.2, 0.1, 64 * 700, 4)]
    nb = [i.L // 64 for i in insts]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{arch} 2 64 2 {sum(nb)} {max(nb)} {min(nb)} 96 48 4\n")
    monkeypatch.setenv("PCPD_TUNE_CACHE", str(cache))
    with pcpd.Sim(2, 64, 1, 11, insts) as sim:
        assert sim.autotune(reps=1) == (96, 48, 4)
        assert sim.get_tuning() == (96, 48, 4)
        sim.run([5])
        lat = [sim.get_lattice(i) for i in range(2)]
    keys, runs = oracle_runs(2, 64, 1, 11, insts, [5])
    for (i, q), r in zip(keys, runs):
        np.testing.assert_array_equal(lat[i], r.words)
    other = [Instance(0.1, 0.5, 64 * 333, 0)]
    with pcpd.Sim(2, 64, 1, 1, other) as sim:
        chosen = sim.autotune(reps=1)
    lines = cache.read_text().splitlines()
    assert len(lines) == 2
    assert lines[1].split() == [arch, "2", "64", "1", "333", "333", "333", *map(str, chosen)]


# ---- four decorrelation bits ------------------------------------------------------

@pytest.mark.parametrize("teams", [2, 4])
@pytest.mark.parametrize("model", [1, 2, 3, 4])
def test_four_decorrelation_bits_match_oracle(pcpd, model, teams):
    """mask_bits = 4 (two more Philox draws per window, thresholds rint(q 2^36)):
    rates in sixteenths and off them, the edges q = 0 and 1, many tiles and a
    ragged tail."""
    insts = [Instance(0.13, 0.37, 64 * 260, 1), Instance(0.0, 1.0, 64 * 40, 2),
             Instance(1.0, 0.0, 64 * 30, 3), Instance(0.5625, 0.0625, 64 * 77, 4),
             Instance(0.9, 0.6, 64 * 50, 5)]
    _compare_full(pcpd, model, 64, 2, 8, insts, [1, 3, 7], tuning=(128, 64, teams), mask_bits=4)


def test_four_decorrelation_bits_other_layouts_and_launches(pcpd):
    insts = [Instance(0.2, 0.3, 64 * 150, 0), Instance(0.11, 0.5, 64 * 9, 1)]
    _compare_full(pcpd, 2, 64, 1, 5, insts, [2, 6], mask_bits=4, layout=1)
    _compare_full(pcpd, 2, 64, 1, 5, insts, [2, 6], tuning=(64, 16, 2), mask_bits=4,
                  options={"persistent": True, "skip_empty": True})
    _compare_full(pcpd, 3, 15, 2, 5, [Instance(0.17, 0.45, 15 * 333, 3)], [4], mask_bits=4)
