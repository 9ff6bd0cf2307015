"""GPU parity at the long horizons of the configured workloads.

The HIP sweep runs each workload whole, in the benchmark's default launch
shape, through the C ABI, and must reproduce bit for bit the expected results
that the CPU oracle wrote into tests/golden/horizon_*.json (written by
tests/golden/make_horizon_golden.py, which calls only the oracle): the
sha256 of every simulated (instance, plane) lattice at the last record, and
N, N_pair and the alive mask at every record. Units that the oracle simulated
for a subset of the 64 samples are compared on those samples only, with
per-sample counts taken from lattices read back at each record.

The rings of 1024 sites run the 64 log-spaced records of a 10^5-step run for
n = 1, 2, 3, once with direct launches and once replaying captured graph
segments.

Also here: the rate edges of eq. (1) (p or d at 0 or 1, and p >= 1/2), where
every integer part of the decision thresholds selects its own kernel copy,
checked bit-exactly against the oracle and against the invariants the model
fixes at those rates.
"""
import hashlib
import importlib.util
import json
import os

import numpy as np
import pytest

from paper_1301_6082_amd import workloads as wl
from paper_1301_6082_amd.workloads import Instance

from gpu_common import oracle_runs, per_sample_counts

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
ALL = (1 << 64) - 1


def _golden_module():
    spec = importlib.util.spec_from_file_location(
        "make_horizon_golden", os.path.join(GOLDEN, "make_horizon_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


_GM = _golden_module()
CASES = sorted(_GM.cases())


@pytest.fixture(scope="module")
def pcpd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_6082_amd import pcpd as mod
    return mod


def _load(name):
    with open(os.path.join(GOLDEN, f"horizon_{name}.json")) as f:
        return json.load(f)


def _sha(words):
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest()


def _workload(doc, name):
    """The seeded recipe named by the case, checked against the stored inputs."""
    build, times, _ = _GM.cases()[name]
    w = build()
    assert [int(t) for t in times] == doc["times"]
    assert (w.model, w.B, w.planes, w.seed) == (doc["model"], doc["B"], doc["planes"], doc["seed"])
    got = [[inst.p, inst.d, int(inst.L), int(inst.stream_id)] for inst in w.instances]
    assert got == doc["instances"], "workload recipe changed since the oracle wrote the case"
    return w


def _check_case(pcpd, name, graph=False):
    doc = _load(name)
    w = _workload(doc, name)
    times = doc["times"]
    units = doc["units"]
    sampled = [u for u in units if int(u["samples"], 16) != ALL]
    print(f"[horizon] case={name} model={w.model} n_inst={len(w.instances)} planes={w.planes} "
          f"units={len(units)} times={times[0]}..{times[-1]} graph={graph}", flush=True)
    need = sorted({u["inst"] for u in sampled})
    snaps = {}
    with pcpd.Sim(w.model, w.B, w.planes, w.seed, w.instances) as sim:
        if graph:
            sim.set_options(graph=True)
        if sampled:
            # one record at a time, reading back the sampled instances each time
            recs = []
            for t in times:
                recs.append(sim.run([t])[0])
                for i in need:
                    snaps[(i, t)] = sim.get_lattice(i)
            counts = np.stack(recs)
        else:
            counts = sim.run(times)
        tuning = sim.get_tuning()
        lat = {i: sim.get_lattice(i) for i in sorted({u["inst"] for u in units})}
    print(f"[horizon] case={name} tile={tuning}", flush=True)
    for u in units:
        i, q, samples = u["inst"], u["plane"], int(u["samples"], 16)
        L = int(w.instances[i].L)
        words = lat[i][q * L:(q + 1) * L] & np.uint64(samples)
        assert _sha(words) == u["words_sha256"], f"{name}: lattice inst {i} plane {q}"
        if samples == ALL:
            np.testing.assert_array_equal(counts[:, i, q, 0], u["n"], err_msg=f"{name} N {i} {q}")
            np.testing.assert_array_equal(counts[:, i, q, 1], u["n_pair"],
                                          err_msg=f"{name} N_pair {i} {q}")
            np.testing.assert_array_equal(counts[:, i, q, 2], [int(a, 16) for a in u["alive"]],
                                          err_msg=f"{name} alive {i} {q}")
        else:
            for k, t in enumerate(times):
                n, pair = per_sample_counts(snaps[(i, t)][q * L:(q + 1) * L])
                for b, ref in u["per_sample"].items():
                    assert int(n[int(b)]) == ref["n"][k], (name, i, q, b, t)
                    assert int(pair[int(b)]) == ref["n_pair"][k], (name, i, q, b, t)
            # every plane's aggregate counts stay consistent
            assert (counts[:, :, :, 1] <= counts[:, :, :, 0]).all()
    return tuning


@pytest.mark.parametrize("name", [c for c in CASES if not c.startswith("ring1024")])
def test_configured_workload_at_its_horizon(pcpd, name):
    tuning = _check_case(pcpd, name)
    if name.startswith("cfg2"):
        # the benchmark's launch: 128-column tiles, phases of 128 substeps
        assert tuning[:2] == (128, 128)


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("name", [c for c in CASES if c.startswith("ring1024")])
def test_ring1024_to_1e5_steps(pcpd, name, graph):
    _check_case(pcpd, name, graph=graph)


# ---- rate edges -----------------------------------------------------------

# (p, d) pairs whose thresholds K = rint(q 2^34) have every integer part
# floor(K / 2^32) in 0..4 for both rates, including the exact values 0, 1/4,
# 1/2, 3/4 and 1 (K a multiple of 2^32) and p >= 1/2.
EDGE_RATES = [(0.0, 0.0), (0.0, 1.0), (1.0, 0.0), (1.0, 1.0), (0.6, 0.3), (0.8, 0.6),
              (0.55, 0.8), (0.25, 0.75), (0.5, 0.5), (0.75, 0.25), (0.3, 0.95), (0.97, 0.03)]


@pytest.mark.parametrize("teams", [2, 4])
@pytest.mark.parametrize("model", [1, 2, 3, 4])
def test_rate_edges_match_oracle(pcpd, model, teams):
    L = 64 * 150
    start = wl.random_lattice(L, 1, 0.6, 40 + model)
    insts = [Instance(p, d, L, k, wl.INIT_HOST, start) for k, (p, d) in enumerate(EDGE_RATES)]
    times = [0, 1, 2, 5, 9]
    print(f"[edges] model={model} teams={teams} L={L} rates={EDGE_RATES}", flush=True)
    with pcpd.Sim(model, 64, 1, 3, insts) as sim:
        sim.set_tuning(0, 0, teams)
        counts = sim.run(times)
        lat = [sim.get_lattice(i) for i in range(len(insts))]
    keys, runs = oracle_runs(model, 64, 1, 3, insts, times)
    for (i, q), r in zip(keys, runs):
        np.testing.assert_array_equal(lat[i], r.words, err_msg=f"rates {EDGE_RATES[i]}")
        N, NP, alive = r.counts()
        np.testing.assert_array_equal(counts[:, i, 0, 0], N, err_msg=f"N {EDGE_RATES[i]}")
        np.testing.assert_array_equal(counts[:, i, 0, 1], NP, err_msg=f"N_pair {EDGE_RATES[i]}")
        np.testing.assert_array_equal(counts[:, i, 0, 2], alive, err_msg=f"alive {EDGE_RATES[i]}")
    # invariants of eq. (1), read off the GPU's own output, per sample
    n0, _ = per_sample_counts(start)
    for i, (p, d) in enumerate(EDGE_RATES):
        n_end, _ = per_sample_counts(lat[i])
        N = counts[:, i, 0, 0].astype(np.int64)
        if d == 1.0:                      # pure diffusion conserves every sample's count
            assert (N == N[0]).all() and (n_end == n0).all(), (p, d)
        elif d == 0.0 and p == 1.0:       # pure annihilation: counts never grow
            assert (np.diff(N) <= 0).all() and (n_end <= n0).all(), (p, d)
        elif d == 0.0 and p == 0.0:       # fission only: counts never shrink
            assert (np.diff(N) >= 0).all() and (n_end >= n0).all(), (p, d)


@pytest.mark.parametrize("model", [2, 3])
def test_absorbing_states_on_the_gpu(pcpd, model):
    """An empty ring stays empty; a lone PCPD particle (or a TCPD pair) can only
    diffuse, at any rates."""
    L = 64 * 12
    lone = np.zeros(L, dtype=np.uint64)
    lone[100] = np.uint64(ALL)               # one particle in every sample
    if model == 3:
        lone[400] = np.uint64(ALL)           # a second one: TCPD needs three
    empty = np.zeros(L, dtype=np.uint64)
    insts = [Instance(p, d, L, k, wl.INIT_HOST, s)
             for k, (p, d, s) in enumerate([(0.0, 0.0, lone), (0.5, 0.2, lone), (0.1, 0.9, lone),
                                            (0.0, 0.0, empty), (1.0, 1.0, empty)])]
    with pcpd.Sim(model, 64, 1, 8, insts) as sim:
        counts = sim.run([1, 10, 40])
    want = model - 1
    for i in range(3):
        assert (counts[:, i, 0, 0] == 64 * want).all()
    for i in (3, 4):
        assert (counts[:, i, 0] == 0).all()
