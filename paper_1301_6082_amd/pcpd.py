"""ctypes binding of libpcpd (include/pcpd.h). Argument marshalling only:
every step of the sweep runs in the library's HIP kernels.

PyTorch supplies device memory (the two lattice copies are one torch tensor)
and the stream (torch's current stream); it is imported before the library so
that both share one HIP runtime. There is no fallback: if libpcpd.so is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpcpd.so")

OPT_GRAPH, OPT_PERSISTENT, OPT_SKIP_EMPTY = 1, 2, 4
PCPD_OK, PCPD_EINVAL, PCPD_ENOMEM, PCPD_EDEVICE, PCPD_ESTATE, PCPD_EOVERFLOW = 0, -1, -2, -3, -4, -5
PCPD_ELIMIT = -6
NOALLOC_MAX_WORDS = 1 << 22
DP, PCPD, TCPD, QCPD = 1, 2, 3, 4
INIT_FULL, INIT_EMPTY, INIT_HOST = 0, 1, 2

u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32


LAYOUT_CLASSICAL, LAYOUT_CONNECTED = 0, 1


class Config(ctypes.Structure):
    _fields_ = [("model", i32), ("B", u32), ("planes", u32), ("seed", u32), ("layout", u32),
                ("mask_bits", u32)]


class InstanceC(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("d", ctypes.c_double), ("L", u64),
                ("stream_id", u32), ("init", i32), ("host_words", ctypes.POINTER(u64))]


class Device(ctypes.Structure):
    _fields_ = [("hip_stream", ctypes.c_void_p), ("dev_buf", ctypes.c_void_p),
                ("dev_buf_bytes", ctypes.c_size_t)]


class CountsC(ctypes.Structure):
    _fields_ = [("n", u64), ("n_pair", u64), ("alive", u64)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_cols", u32), ("phase_max", u32), ("teams", u32)]


EXPORTS = ["pcpd_lattice_bytes", "pcpd_init", "pcpd_sweep", "pcpd_density", "pcpd_run",
           "pcpd_get_lattice", "pcpd_set_lattice", "pcpd_time", "pcpd_sync",
           "pcpd_set_tuning", "pcpd_get_tuning", "pcpd_set_options", "pcpd_autotune",
           "pcpd_profile", "pcpd_profile_read", "pcpd_run_noalloc",
           "pcpd_device_error", "pcpd_free", "pcpd_strerror"]
MLP_EXPORTS = ["pcpd_mlp_init", "pcpd_mlp_get_params", "pcpd_mlp_set_params", "pcpd_mlp_predict",
               "pcpd_mlp_loss", "pcpd_mlp_grads", "pcpd_mlp_train_step", "pcpd_mlp_free"]
MLP_PARAMS = 33665
MLP_MAX_ROWS = 1 << 24
MLP_MAX_TRAIN_ROWS = 1 << 20


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"libpcpd.so not built ({path}); run python -m paper_1301_6082_amd.build")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    sig = {
        "pcpd_lattice_bytes": ([P(Config), P(InstanceC), u32, P(ctypes.c_size_t)], ctypes.c_int),
        "pcpd_init": ([P(vp), P(Config), P(InstanceC), u32, u64, P(Device)], ctypes.c_int),
        "pcpd_sweep": ([vp, u64], ctypes.c_int),
        "pcpd_density": ([vp, P(CountsC)], ctypes.c_int),
        "pcpd_run": ([vp, P(u64), u32, P(CountsC)], ctypes.c_int),
        "pcpd_get_lattice": ([vp, u32, P(u64)], ctypes.c_int),
        "pcpd_set_lattice": ([vp, u32, P(u64)], ctypes.c_int),
        "pcpd_time": ([vp, P(u64)], ctypes.c_int),
        "pcpd_sync": ([vp], ctypes.c_int),
        "pcpd_set_tuning": ([vp, P(Tuning)], ctypes.c_int),
        "pcpd_get_tuning": ([vp, P(Tuning)], ctypes.c_int),
        "pcpd_set_options": ([vp, u32], ctypes.c_int),
        "pcpd_autotune": ([vp, u32, P(Tuning)], ctypes.c_int),
        "pcpd_profile": ([vp, ctypes.c_int], ctypes.c_int),
        "pcpd_profile_read": ([vp, P(ctypes.c_double), P(u64)], ctypes.c_int),
        "pcpd_run_noalloc": ([P(Config), P(InstanceC), u32, u64, vp, P(u64), u32, P(CountsC), vp],
                             ctypes.c_int),
        "pcpd_free": ([vp], ctypes.c_int),
        "pcpd_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "pcpd_device_error": ([vp], ctypes.c_char_p),
        "pcpd_mlp_init": ([P(vp), u32, P(Device)], ctypes.c_int),
        "pcpd_mlp_get_params": ([vp, P(ctypes.c_float)], ctypes.c_int),
        "pcpd_mlp_set_params": ([vp, P(ctypes.c_float)], ctypes.c_int),
        "pcpd_mlp_predict": ([vp, vp, u32, vp], ctypes.c_int),
        "pcpd_mlp_loss": ([vp, vp, vp, vp, u32, vp, P(ctypes.c_float)], ctypes.c_int),
        "pcpd_mlp_grads": ([vp, vp, vp, vp, u32, P(ctypes.c_float), P(ctypes.c_float)], ctypes.c_int),
        "pcpd_mlp_train_step": ([vp, vp, vp, vp, u32, ctypes.c_float, P(ctypes.c_float)], ctypes.c_int),
        "pcpd_mlp_free": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = load_library()


class PcpdError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        extra = f" [{detail}]" if detail else ""
        super().__init__(f"{where}: {_lib.pcpd_strerror(status).decode()} ({status}){extra}")


def _check(status: int, where: str, ctx=None):
    if status != PCPD_OK:
        detail = ""
        if ctx is not None and status in (PCPD_EDEVICE, PCPD_ENOMEM):
            detail = _lib.pcpd_device_error(ctx).decode()
        raise PcpdError(status, where, detail)


def _u64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(u64))


def _instances(insts, planes):
    arr = (InstanceC * len(insts))()
    keep = []
    for i, it in enumerate(insts):
        arr[i].p = float(it.p)
        arr[i].d = float(it.d)
        arr[i].L = int(it.L)
        arr[i].stream_id = int(it.stream_id)
        arr[i].init = int(it.init)
        if int(it.init) == INIT_HOST:
            w = np.ascontiguousarray(np.asarray(it.host_words, dtype=np.uint64))
            if w.shape != (planes * int(it.L),):
                raise ValueError("host_words must hold planes*L words")
            keep.append(w)
            arr[i].host_words = _u64p(w)
        else:
            arr[i].host_words = None
    return arr, keep


def lattice_bytes(model: int, B: int, planes: int, seed: int, instances, layout: int = 0,
                  mask_bits: int = 2) -> int:
    cfg = Config(int(model), int(B), int(planes), int(seed), int(layout), int(mask_bits))
    arr, _ = _instances(instances, planes)
    out = ctypes.c_size_t()
    _check(_lib.pcpd_lattice_bytes(ctypes.byref(cfg), arr, len(instances), ctypes.byref(out)),
           "pcpd_lattice_bytes")
    return int(out.value)


class Sim:
    """A context of one or more instances (workloads.Instance-like objects with
    p, d, L, stream_id, init, host_words) sharing model, B, planes and seed."""

    def __init__(self, model: int, B: int, planes: int, seed: int, instances, t0: int = 0,
                 device: int | None = None, torch_buffer: bool = True, layout: int = 0,
                 mask_bits: int = 2):
        if not torch.cuda.is_available():
            raise RuntimeError("libpcpd needs a ROCm GPU; none is visible")
        self.model, self.B, self.planes, self.seed = int(model), int(B), int(planes), int(seed)
        self.layout = int(layout)
        self.mask_bits = int(mask_bits)
        self.instances = list(instances)
        self.n_inst = len(self.instances)
        self.Ls = [int(i.L) for i in self.instances]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        cfg = Config(self.model, self.B, self.planes, self.seed, self.layout, self.mask_bits)
        arr, keep = _instances(self.instances, self.planes)
        dev = Device()
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            dev.hip_stream = ctypes.c_void_p(self.stream.cuda_stream)
            self._buf = None
            if torch_buffer:
                nbytes = lattice_bytes(self.model, self.B, self.planes, self.seed, self.instances,
                                       self.layout, self.mask_bits)
                self._buf = torch.empty(nbytes // 8, dtype=torch.int64, device=self.device)
                dev.dev_buf = ctypes.c_void_p(self._buf.data_ptr())
                dev.dev_buf_bytes = nbytes
            self._ctx = ctypes.c_void_p()
            _check(_lib.pcpd_init(ctypes.byref(self._ctx), ctypes.byref(cfg), arr, self.n_inst,
                                  int(t0), ctypes.byref(dev)), "pcpd_init")
        del keep

    # -- stepping and observables
    def sweep(self, n_steps: int):
        _check(_lib.pcpd_sweep(self._ctx, int(n_steps)), "pcpd_sweep", self._ctx)

    def sync(self):
        _check(_lib.pcpd_sync(self._ctx), "pcpd_sync", self._ctx)

    def density(self) -> np.ndarray:
        """uint64 [n_inst, planes, 3] = (N, N_pair, alive)."""
        out = (CountsC * (self.n_inst * self.planes))()
        _check(_lib.pcpd_density(self._ctx, out), "pcpd_density", self._ctx)
        return np.frombuffer(out, dtype=np.uint64).reshape(self.n_inst, self.planes, 3).copy()

    def run(self, times: Sequence[int]) -> np.ndarray:
        """uint64 [n_times, n_inst, planes, 3] at each record time."""
        t = np.ascontiguousarray(np.asarray(times, dtype=np.uint64))
        out = (CountsC * (len(t) * self.n_inst * self.planes))()
        _check(_lib.pcpd_run(self._ctx, _u64p(t), len(t), out), "pcpd_run", self._ctx)
        return np.frombuffer(out, dtype=np.uint64).reshape(len(t), self.n_inst, self.planes, 3).copy()

    # -- state
    def get_lattice(self, inst: int) -> np.ndarray:
        w = np.empty(self.planes * self.Ls[inst], dtype=np.uint64)
        _check(_lib.pcpd_get_lattice(self._ctx, int(inst), _u64p(w)), "pcpd_get_lattice", self._ctx)
        return w

    def set_lattice(self, inst: int, words) -> None:
        w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
        if w.shape != (self.planes * self.Ls[inst],):
            raise ValueError("set_lattice needs planes*L words")
        _check(_lib.pcpd_set_lattice(self._ctx, int(inst), _u64p(w)), "pcpd_set_lattice", self._ctx)

    @property
    def time(self) -> int:
        t = u64()
        _check(_lib.pcpd_time(self._ctx, ctypes.byref(t)), "pcpd_time")
        return int(t.value)

    def set_tuning(self, tile_cols: int = 0, phase_max: int = 0, teams: int = 0):
        """All 0: the default shape; otherwise a 0 keeps the current value."""
        tu = Tuning(int(tile_cols), int(phase_max), int(teams))
        _check(_lib.pcpd_set_tuning(self._ctx, ctypes.byref(tu)), "pcpd_set_tuning", self._ctx)

    def get_tuning(self):
        tu = Tuning()
        _check(_lib.pcpd_get_tuning(self._ctx, ctypes.byref(tu)), "pcpd_get_tuning")
        return int(tu.tile_cols), int(tu.phase_max), int(tu.teams)

    def set_options(self, graph: bool = False, persistent: bool = False, skip_empty: bool = False):
        """graph=True: capture sweep segments into HIP graphs and replay them;
        persistent=True: all phases between two records in one ticket-dispatched launch;
        skip_empty=True: tiles with no particle in their loaded range skip their substeps."""
        flags = ((OPT_GRAPH if graph else 0) | (OPT_PERSISTENT if persistent else 0) |
                 (OPT_SKIP_EMPTY if skip_empty else 0))
        _check(_lib.pcpd_set_options(self._ctx, flags), "pcpd_set_options", self._ctx)

    def autotune(self, reps: int = 3):
        """Time candidate tile shapes on this lattice (state unchanged); returns the choice."""
        tu = Tuning()
        _check(_lib.pcpd_autotune(self._ctx, int(reps), ctypes.byref(tu)), "pcpd_autotune", self._ctx)
        return int(tu.tile_cols), int(tu.phase_max), int(tu.teams)

    def profile(self, enable: bool = True):
        """Bracket every phase-kernel launch with HIP events on the stream."""
        _check(_lib.pcpd_profile(self._ctx, 1 if enable else 0), "pcpd_profile", self._ctx)

    def profile_read(self):
        """(summed phase-kernel milliseconds, launches) since the last read."""
        ms, n = ctypes.c_double(), u64()
        _check(_lib.pcpd_profile_read(self._ctx, ctypes.byref(ms), ctypes.byref(n)),
               "pcpd_profile_read", self._ctx)
        return float(ms.value), int(n.value)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            _lib.pcpd_free(self._ctx)
            self._ctx = ctypes.c_void_p()
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def run_noalloc(model: int, B: int, planes: int, seed: int, instances, t0: int,
                lattice: torch.Tensor, times: Sequence[int], layout: int = 0,
                mask_bits: int = 2) -> np.ndarray:
    """pcpd_run_noalloc: advance the lattice held in `lattice` (a contiguous
    int64 CUDA tensor of planes * sum L words, instance-major then
    plane-major) from step t0 through `times`, in place, without any device
    allocation; returns uint64 [n_times, n_inst, planes, 3] like Sim.run."""
    instances = list(instances)
    words = planes * sum(int(i.L) for i in instances)
    if not (isinstance(lattice, torch.Tensor) and lattice.is_cuda and lattice.dtype == torch.int64
            and lattice.is_contiguous() and lattice.numel() == words):
        raise ValueError(f"lattice must be a contiguous int64 CUDA tensor of {words} words")
    cfg = Config(int(model), int(B), int(planes), int(seed), int(layout), int(mask_bits))
    arr, keep = _instances(instances, planes)
    t = np.ascontiguousarray(np.asarray(times, dtype=np.uint64))
    out = (CountsC * (len(t) * len(instances) * planes))()
    with torch.cuda.device(lattice.device):
        stream = torch.cuda.current_stream(lattice.device).cuda_stream
        _check(_lib.pcpd_run_noalloc(ctypes.byref(cfg), arr, len(instances), int(t0),
                                     ctypes.c_void_p(lattice.data_ptr()), _u64p(t), len(t), out,
                                     ctypes.c_void_p(stream)), "pcpd_run_noalloc")
    del keep
    return np.frombuffer(out, dtype=np.uint64).reshape(len(t), len(instances), planes, 3).copy()


def _dev_f32(t, shape, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape {shape}")
    return ctypes.c_void_p(t.data_ptr())


class Surrogate:
    """The density surrogate (include/pcpd_mlp.h): 3-128-128-128-1 GELU
    network on log10 rho; inputs and targets are float32 CUDA tensors."""

    def __init__(self, seed: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate needs a ROCm GPU; none is visible")
        dev = Device()
        dev.hip_stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        self._net = ctypes.c_void_p()
        _check(_lib.pcpd_mlp_init(ctypes.byref(self._net), int(seed), ctypes.byref(dev)),
               "pcpd_mlp_init")

    def params(self) -> np.ndarray:
        out = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(_lib.pcpd_mlp_get_params(self._net, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "pcpd_mlp_get_params")
        return out

    def set_params(self, theta) -> None:
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        if th.shape != (MLP_PARAMS,):
            raise ValueError("parameter vector must hold 33665 values")
        _check(_lib.pcpd_mlp_set_params(self._net, th.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "pcpd_mlp_set_params")

    def predict(self, x: torch.Tensor) -> torch.Tensor:
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(_lib.pcpd_mlp_predict(self._net, _dev_f32(x, (n, 3), "x"), n,
                                     ctypes.c_void_p(y.data_ptr())), "pcpd_mlp_predict")
        return y

    def loss(self, x, target, mask=None) -> float:
        """Masked mean squared error, forward pass only (no gradient scratch)."""
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        m = _dev_f32(mask, (n,), "mask") if mask is not None else None
        _check(_lib.pcpd_mlp_loss(self._net, _dev_f32(x, (n, 3), "x"),
                                  _dev_f32(target, (n,), "target"), m, n,
                                  ctypes.c_void_p(y.data_ptr()), ctypes.byref(loss)),
               "pcpd_mlp_loss")
        return float(loss.value)

    def grads(self, x, target, mask=None):
        n = x.shape[0]
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        m = _dev_f32(mask, (n,), "mask") if mask is not None else None
        _check(_lib.pcpd_mlp_grads(self._net, _dev_f32(x, (n, 3), "x"), _dev_f32(target, (n,), "target"),
                                   m, n, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   ctypes.byref(loss)), "pcpd_mlp_grads")
        return float(loss.value), g

    def train_step(self, x, target, mask=None, lr: float = 1e-3, want_loss: bool = False):
        n = x.shape[0]
        loss = ctypes.c_float()
        m = _dev_f32(mask, (n,), "mask") if mask is not None else None
        _check(_lib.pcpd_mlp_train_step(self._net, _dev_f32(x, (n, 3), "x"),
                                        _dev_f32(target, (n,), "target"), m, n, float(lr),
                                        ctypes.byref(loss) if want_loss else None),
               "pcpd_mlp_train_step")
        return float(loss.value) if want_loss else None

    def close(self):
        if getattr(self, "_net", None) and self._net.value:
            _lib.pcpd_mlp_free(self._net)
            self._net = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
