"""Pins the oracle's Philox-4x32-10 to two independent implementations that
ship in this image: PyTorch's at::Philox4_32 and rocRAND's
philox4x32_10_engine, each compiled for the host from its own header and
driven through its public (seed, subsequence, offset) interface."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
PROBES = os.path.join(HERE, "probes")


def _cases():
    rng = np.random.default_rng(12345)
    cases = [
        (0, 0, 0, 0, 0, 0),
        (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF),
        (1, 2, 3, 4, 5, 6),
        (0, 7, 0, 0, 1, 0),            # substep-offset draw, plane 0, s = 0
        (16383, (3 << 3) | 2, 640000, 0, 1, 15),  # window draw, plane 3
        (5, 1, 0xFFFFFFFF, 1, 1, 511),  # substep index crossing 2^32
    ]
    for _ in range(200):
        c = [int(x) for x in rng.integers(0, 2**32, size=6, dtype=np.uint64)]
        c[1] &= (1 << 29) - 1  # the rocRAND offset interface takes 4*(c0|c1<<32) < 2^64
        cases.append(tuple(c))
    return cases


def _run_probe(exe, cases):
    inp = "".join(" ".join(str(v) for v in c) + "\n" for c in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]


@pytest.fixture(scope="module")
def torch_probe(tmp_path_factory):
    import torch  # noqa: F401  (only to locate the headers)
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path_factory.mktemp("kat") / "philox_torch")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", inc, "-o", exe,
                           os.path.join(PROBES, "philox_torch.cpp")])
    return exe


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("kat") / "philox_rocrand")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-host-only", "-o", exe,
                           os.path.join(PROBES, "philox_rocrand.cpp")])
    return exe


def test_philox_matches_pytorch(torch_probe):
    cases = _cases()
    ref = _run_probe(torch_probe, cases)
    got = [oracle.philox(c[:4], c[4:]) for c in cases]
    assert got == ref


def test_philox_matches_rocrand(rocrand_probe):
    # its offset argument counts 32-bit outputs, so c1 must stay below 2^30
    cases = [c for c in _cases() if c[1] < (1 << 30)]
    assert len(cases) > 200
    ref = _run_probe(rocrand_probe, cases)
    got = [oracle.philox(c[:4], c[4:]) for c in cases]
    assert got == ref


def test_offset_is_uniform_over_block():
    """o = floor(x0 * B / 2^32) is uniform on [0, B): chi-square over 64 cells."""
    B = 64
    counts = np.zeros(B)
    n = 64 * 400
    for s in range(n):
        counts[oracle.offset(1, 3, 2, s, B)] += 1
    exp = n / B
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 63 degrees of freedom: P(chi2 > 120) < 1e-5
    assert chi2 < 120, chi2
    assert counts.min() > 0


def test_offset_depends_on_plane_stream_and_substep():
    base = [oracle.offset(1, 0, 0, s, 1 << 20) for s in range(32)]
    assert base != [oracle.offset(1, 1, 0, s, 1 << 20) for s in range(32)]
    assert base != [oracle.offset(1, 0, 1, s, 1 << 20) for s in range(32)]
    assert base != [oracle.offset(2, 0, 0, s, 1 << 20) for s in range(32)]
    assert len(set(base)) > 25
