"""pcpd_run_noalloc, the allocation-free run, against pcpd_init + pcpd_run.

Both go through the C ABI on the same seeded start; the lattice after the last
record and every count record must agree bit for bit. Two calls in a row, the
second on a smaller problem, so that what the first left in the shared
workspace (spare lattice copy, tables, records) cannot leak into the second.
"""
import numpy as np
import pytest

from paper_1301_6082_amd import workloads as wl
from paper_1301_6082_amd.workloads import Instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcpd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_6082_amd import pcpd as mod
    return mod


def _compare(pcpd, model, B, planes, seed, insts, t0, times, label):
    import torch
    start = np.concatenate([np.asarray(i.host_words, dtype=np.uint64) for i in insts])
    print(f"[noalloc] {label}: model={model} B={B} planes={planes} n_inst={len(insts)} "
          f"words={start.size} t0={t0} times={times[0]}..{times[-1]}", flush=True)
    with pcpd.Sim(model, B, planes, seed, insts, t0=t0) as sim:
        want = sim.run(times)
        want_lat = np.concatenate([sim.get_lattice(i) for i in range(len(insts))])
    lat = torch.from_numpy(start.view(np.int64).copy()).cuda()
    got = pcpd.run_noalloc(model, B, planes, seed, insts, t0, lat, times)
    torch.cuda.synchronize()
    got_lat = lat.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, want, err_msg=f"{label}: count records")
    np.testing.assert_array_equal(got_lat, want_lat, err_msg=f"{label}: final lattice")
    return got


def test_noalloc_matches_the_context_run_twice_second_smaller(pcpd):
    B = 64
    # first call: three uneven rings, two planes, PCPD, odd number of phases
    Ls = [64 * 300, 64 * 45, 64 * 1200]
    rates = [(0.12, 0.3), (0.6, 0.9), (0.05, 0.0)]
    insts = [Instance(p, d, L, 10 + k, wl.INIT_HOST, wl.random_lattice(L, 2, 0.7, 100 + k))
             for k, ((p, d), L) in enumerate(zip(rates, Ls))]
    first = _compare(pcpd, 2, B, 2, 5, insts, 3, [3, 4, 7, 12, 21], "first")
    # second call: one smaller ring of another model, one plane, even phase count
    L = 64 * 20
    small = [Instance(0.2, 0.5, L, 4, wl.INIT_HOST, wl.random_lattice(L, 1, 0.5, 7))]
    second = _compare(pcpd, 3, B, 1, 9, small, 0, [1, 2, 6], "second")
    assert first.shape != second.shape


def test_noalloc_rejects_beyond_its_workspace(pcpd):
    import torch
    L = pcpd.NOALLOC_MAX_WORDS  # one plane of this ring fits exactly; two planes do not
    inst = [Instance(0.1, 0.5, L, 0, wl.INIT_FULL, None)]
    lat = torch.zeros(2 * L, dtype=torch.int64, device="cuda")
    with pytest.raises(pcpd.PcpdError) as err:
        pcpd.run_noalloc(2, 64, 2, 1, inst, 0, lat, [1])
    assert err.value.status == pcpd.PCPD_ELIMIT
