"""The C ABI library loads, exports every symbol include/pcpd.h declares, and
validates its arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("pcpd.h", "pcpd_mlp.h")]


def declared():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"PCPD_API\s+[\w\s\*]*?\b(pcpd_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def mod():
    from paper_1301_6082_amd import pcpd
    return pcpd


def test_header_declares_the_boundary():
    names = declared()
    for must in ("pcpd_init", "pcpd_sweep", "pcpd_density", "pcpd_run", "pcpd_free"):
        assert must in names


def test_library_exports_every_declared_symbol(mod):
    out = subprocess.run(["nm", "-D", "--defined-only", mod.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    assert sorted(mod.EXPORTS + mod.MLP_EXPORTS) == declared()
    # nothing else with the pcpd_ prefix leaks out
    assert sorted(n for n in exported if n.startswith("pcpd_")) == declared()


def test_strerror(mod):
    lib = mod._lib
    assert lib.pcpd_strerror(0) == b"success"
    assert lib.pcpd_strerror(-1) == b"invalid argument"
    assert lib.pcpd_strerror(-5) == b"substep counter overflow"
    assert lib.pcpd_strerror(42) == b"unknown status"


def _cfg(mod, model=2, B=64, planes=1, seed=1, layout=0):
    return mod.Config(model, B, planes, seed, layout)


def _inst(mod, p=0.1, d=0.5, L=1024, init=0, words=None):
    arr = (mod.InstanceC * 1)()
    arr[0].p, arr[0].d, arr[0].L, arr[0].stream_id, arr[0].init = p, d, L, 0, init
    arr[0].host_words = words
    return arr


BAD = [
    dict(cfg=dict(model=0)), dict(cfg=dict(model=5)), dict(cfg=dict(B=3)),
    dict(cfg=dict(model=3, B=4)), dict(cfg=dict(model=4, B=5)), dict(cfg=dict(planes=0)), dict(cfg=dict(planes=1 << 29)),
    dict(inst=dict(p=-0.1)), dict(inst=dict(p=1.5)), dict(inst=dict(d=float("nan"))),
    dict(inst=dict(d=float("inf"))), dict(inst=dict(L=100)), dict(inst=dict(L=32)),
    dict(inst=dict(L=0)), dict(inst=dict(init=3)), dict(inst=dict(init=2, words=None)),
    dict(inst=dict(L=64 << 32)), dict(cfg=dict(layout=2)),
]


@pytest.mark.parametrize("case", BAD)
def test_invalid_arguments_are_rejected_on_the_host(mod, case):
    cfg = _cfg(mod, **case.get("cfg", {}))
    inst = _inst(mod, **case.get("inst", {}))
    size = ctypes.c_size_t(12345)
    assert mod._lib.pcpd_lattice_bytes(ctypes.byref(cfg), inst, 1, ctypes.byref(size)) == -1
    assert size.value == 12345
    ctx = ctypes.c_void_p(0xABC)
    rc = mod._lib.pcpd_init(ctypes.byref(ctx), ctypes.byref(cfg), inst, 1, 0, None)
    assert rc == -1
    assert ctx.value == 0xABC  # untouched


def test_lattice_bytes(mod):
    cfg = _cfg(mod, planes=4)
    arr = (mod.InstanceC * 2)()
    for i, L in enumerate((1024, 4096)):
        arr[i].p, arr[i].d, arr[i].L, arr[i].init = 0.1, 0.1, L, 0
    size = ctypes.c_size_t()
    assert mod._lib.pcpd_lattice_bytes(ctypes.byref(cfg), arr, 2, ctypes.byref(size)) == 0
    assert size.value == 2 * 8 * 4 * (1024 + 4096)
    assert mod._lib.pcpd_lattice_bytes(ctypes.byref(cfg), arr, 0, ctypes.byref(size)) == -1


def test_null_context_calls(mod):
    lib = mod._lib
    assert lib.pcpd_sweep(None, 1) == -1
    assert lib.pcpd_sync(None) == -1
    assert lib.pcpd_free(None) == -1
    assert lib.pcpd_init(None, None, None, 0, 0, None) == -1


def test_overflowing_start_time_is_rejected(mod):
    cfg = _cfg(mod)
    inst = _inst(mod)
    ctx = ctypes.c_void_p()
    rc = mod._lib.pcpd_init(ctypes.byref(ctx), ctypes.byref(cfg), inst, 1, 2**64 // 64 + 1, None)
    assert rc == -5


def test_noalloc_run_checks_its_limits_before_any_device_work(mod):
    """pcpd_run_noalloc validates like pcpd_init + pcpd_run and refuses what
    exceeds its fixed workspace with PCPD_ELIMIT, all before touching a
    device (here there is none)."""
    lib = mod._lib
    assert lib.pcpd_strerror(-6).startswith(b"exceeds the fixed workspace")
    fake = ctypes.c_void_p(0x1000)          # never dereferenced on these paths
    times = (mod.u64 * 2)(5, 9)
    out = (mod.CountsC * 8)()
    cfg = _cfg(mod, planes=2)
    big = _inst(mod, L=mod.NOALLOC_MAX_WORDS)          # 2 planes: twice the limit
    assert lib.pcpd_run_noalloc(ctypes.byref(cfg), big, 1, 0, fake, times, 2, out, None) == -6
    one = _cfg(mod, planes=1)
    ok = _inst(mod, L=1024)
    assert lib.pcpd_run_noalloc(ctypes.byref(one), ok, 1, 0, None, times, 2, out, None) == -1
    assert lib.pcpd_run_noalloc(ctypes.byref(one), ok, 1, 6, fake, times, 2, out, None) == -1
    desc = (mod.u64 * 2)(9, 5)
    assert lib.pcpd_run_noalloc(ctypes.byref(one), ok, 1, 0, fake, desc, 2, out, None) == -1
    bad = _inst(mod, p=2.0)
    assert lib.pcpd_run_noalloc(ctypes.byref(one), bad, 1, 0, fake, times, 2, out, None) == -1
    late = (mod.u64 * 1)(2**64 // 64 + 1)
    assert lib.pcpd_run_noalloc(ctypes.byref(one), ok, 1, 0, fake, late, 1, out, None) == -5
    # no records: nothing to do, the lattice is left as it is
    assert lib.pcpd_run_noalloc(ctypes.byref(one), ok, 1, 0, fake, None, 0, None, None) == 0


def test_mlp_limits_match_the_header(mod):
    import os
    import re
    text = open(os.path.join(os.path.dirname(__file__), "..", "include", "pcpd_mlp.h")).read()
    macros = {k: eval(v.replace("u", "")) for k, v in
              re.findall(r"#define (PCPD_MLP_\w+) \(?([0-9u <]+)\)?", text)}
    assert macros["PCPD_MLP_PARAMS"] == mod.MLP_PARAMS
    assert macros["PCPD_MLP_MAX_ROWS"] == mod.MLP_MAX_ROWS
    assert macros["PCPD_MLP_MAX_TRAIN_ROWS"] == mod.MLP_MAX_TRAIN_ROWS


def test_mlp_calls_refuse_bad_arguments_without_a_device(mod):
    lib = mod._lib
    f = ctypes.c_float()
    assert lib.pcpd_mlp_loss(None, None, None, None, 1, None, ctypes.byref(f)) == mod.PCPD_EINVAL


def test_mask_bits_other_than_2_or_4_are_refused(mod):
    out = ctypes.c_size_t()
    for m, ok in ((0, True), (2, True), (4, True), (3, False), (1, False), (8, False)):
        cfg = mod.Config(2, 64, 1, 1, 0, m)
        st = mod._lib.pcpd_lattice_bytes(ctypes.byref(cfg), _inst(mod), 1, ctypes.byref(out))
        assert (st == mod.PCPD_OK) == ok, m
