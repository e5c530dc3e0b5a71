"""Python binding of libsft, the MI355X sparse Fourier transform library.

Argument marshalling only: every step of the transform runs in the HIP
kernels of ``libsft.so`` behind the C ABI declared in ``include/sft.h``.
PyTorch supplies device memory (tensors) and streams.  There is no CPU
fallback: if the library is not built or no HIP device is present the calls
raise.

    import torch, paper_1706_02740_amd as sft
    plan = sft.Plan(N, s)                       # dmsft6 preset
    freqs, coefs, count = plan.execute(f)       # f: complex64 tensor [N] on cuda
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsft.so")

SFT_OK = 0
SFT_EINVAL = -1
SFT_ENOMEM = -2
SFT_EHIP = -3
SFT_EBUDGET = -4
SFT_EUNSUPPORTED = -5
SFT_EOVERFLOW = -6

PRESET_DMSFT6 = 0
PRESET_DMSFT4 = 1
PRESET_THEORY = 2
PRESETS = {"dmsft6": PRESET_DMSFT6, "dmsft4": PRESET_DMSFT4, "theory": PRESET_THEORY}

IDENT_RESIDUE = 0
IDENT_PHASE = 1
IDENTS = {"residue": IDENT_RESIDUE, "phase": IDENT_PHASE}

FETCH_SAMPLES = 0
FETCH_BINS = 1
FETCH_HEAVY = 2
FETCH_BANDS = 3
FETCH_SAMPLES_SHIFTED = 4
FETCH_BINS_SHIFTED = 5
FETCH_CLASSES = 6

KERNEL_GATHER = 0
KERNEL_DFT = 1
KERNEL_IDENTIFY = 2
KERNEL_MERGE = 3
KERNEL_DFT_ROWS = 4
KERNEL_DFT_COLS = 5
KERNEL_SELECT = 6
KERNEL_DFT_MX = 7
KERNEL_DFT_COLS_MX = 8
KERNEL_GATHER_MX = 9
KERNEL_NAMES = {KERNEL_GATHER: "k_gather", KERNEL_DFT: "k_dft", KERNEL_IDENTIFY: "k_identify",
                KERNEL_MERGE: "k_merge", KERNEL_DFT_ROWS: "k_dft_rows", KERNEL_DFT_COLS: "k_dft_cols",
                KERNEL_SELECT: "k_select", KERNEL_DFT_MX: "k_dft_mx", KERNEL_DFT_COLS_MX: "k_dft_cols_mx",
                KERNEL_GATHER_MX: "k_gather_mx"}

MAX_MODULI = 15

EXPORTED = [
    "sft_params_default", "sft_plan_describe", "sft_plan_create", "sft_plan_get_info",
    "sft_plan_footprint", "sft_execute", "sft_execute_many", "sft_plan_status",
    "sft_plan_fetch", "sft_plan_destroy", "sft_last_error", "sft_profile_enable",
    "sft_profile_reset", "sft_profile_read", "sft_batch_create", "sft_batch_launch",
    "sft_batch_graph_launch", "sft_batch_destroy", "sft_plan_workspace_bytes",
    "sft_execute_many_status", "sft_execute_many_reserve", "sft_execute_many_release",
    "sft_batch_status", "sft_execute_noalloc",
]


class SftError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsft error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("preset", ctypes.c_int32), ("kappa", ctypes.c_int32), ("sigma_t", ctypes.c_double),
                ("tau", ctypes.c_double), ("r", ctypes.c_double), ("s1_mult", ctypes.c_int32),
                ("group", ctypes.c_int32), ("heavy_T", ctypes.c_int32), ("dft_path", ctypes.c_int32),
                ("ident", ctypes.c_int32), ("gather_path", ctypes.c_int32), ("dft_split", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("s", ctypes.c_int32), ("preset", ctypes.c_int32),
                ("kappa", ctypes.c_int32), ("Q", ctypes.c_int32), ("L", ctypes.c_int64),
                ("q_first", ctypes.c_int64), ("s1", ctypes.c_int32), ("G", ctypes.c_int32),
                ("K", ctypes.c_int32), ("T", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("ident", ctypes.c_int32), ("sigma_t", ctypes.c_double), ("beta", ctypes.c_double),
                ("c1", ctypes.c_double), ("tau", ctypes.c_double), ("alpha", ctypes.c_double),
                ("c2", ctypes.c_double), ("r", ctypes.c_double),
                ("primes", ctypes.c_int32 * MAX_MODULI), ("dft_path", ctypes.c_int32),
                ("P", ctypes.c_int64 * MAX_MODULI), ("M", ctypes.c_int64), ("dft_split", ctypes.c_int32),
                ("gather_path", ctypes.c_int32)]


_lib = None


def load_library():
    """Load libsft.so (built in-tree).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1706_02740_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp = c.c_void_p
    lib.sft_params_default.argtypes = [c.POINTER(Params), c.c_int32]
    lib.sft_plan_describe.argtypes = [c.c_int64, c.c_int32, c.POINTER(Params), c.POINTER(PlanInfo)]
    lib.sft_plan_create.argtypes = [c.POINTER(vp), c.c_int64, c.c_int32, c.POINTER(Params)]
    lib.sft_plan_get_info.argtypes = [vp, c.POINTER(PlanInfo)]
    lib.sft_plan_footprint.argtypes = [vp, c.POINTER(c.c_size_t)]
    lib.sft_execute.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.sft_execute_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.sft_execute_many.argtypes = [c.POINTER(vp), c.c_int32, c.POINTER(vp), c.POINTER(vp),
                                     c.POINTER(vp), vp, vp]
    lib.sft_plan_status.argtypes = [vp, c.POINTER(c.c_int32)]
    lib.sft_plan_fetch.argtypes = [vp, c.c_int32, vp, c.c_size_t, c.POINTER(c.c_size_t)]
    lib.sft_plan_destroy.argtypes = [vp]
    lib.sft_plan_destroy.restype = None
    lib.sft_last_error.argtypes = []
    lib.sft_last_error.restype = c.c_char_p
    lib.sft_profile_enable.argtypes = [c.c_int32]
    lib.sft_profile_reset.argtypes = []
    lib.sft_profile_read.argtypes = [c.c_int32, c.POINTER(c.c_int64), c.POINTER(c.c_double)]
    lib.sft_batch_create.argtypes = [c.POINTER(vp), c.POINTER(vp), c.c_int32, c.POINTER(vp), c.POINTER(vp),
                                     c.POINTER(vp), vp]
    lib.sft_batch_launch.argtypes = [vp, vp]
    lib.sft_batch_graph_launch.argtypes = [vp, vp]
    lib.sft_batch_destroy.argtypes = [vp]
    lib.sft_batch_destroy.restype = None
    lib.sft_plan_workspace_bytes.argtypes = [vp, c.POINTER(c.c_size_t)]
    lib.sft_execute_many_status.argtypes = [vp, c.c_int32, c.POINTER(c.c_int32)]
    lib.sft_execute_many_reserve.argtypes = [vp, c.c_size_t, c.c_int32]
    lib.sft_execute_many_release.argtypes = [vp]
    lib.sft_batch_status.argtypes = [vp, c.POINTER(c.c_int32)]
    for name in EXPORTED:
        if name not in ("sft_plan_destroy", "sft_last_error", "sft_batch_destroy"):
            getattr(lib, name).restype = c.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != SFT_OK:
        raise SftError(rc, load_library().sft_last_error().decode())


def require_device():
    """Fail loudly unless the HIP library is built and a device is visible."""
    import torch
    load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible to torch")


def make_params(preset=PRESET_DMSFT6, kappa=0, sigma_t=0.0, tau=0.0, r=0.0, s1_mult=0,
                group=0, heavy_T=0, dft_path=0, ident=IDENT_RESIDUE, gather_path=0, dft_split=0) -> Params:
    if isinstance(preset, str):
        preset = PRESETS[preset]
    if isinstance(ident, str):
        ident = IDENTS[ident]
    p = Params()
    _check(load_library().sft_params_default(ctypes.byref(p), int(preset)))
    p.kappa, p.sigma_t, p.tau, p.r = int(kappa), float(sigma_t), float(tau), float(r)
    p.s1_mult, p.group, p.heavy_T, p.dft_path = int(s1_mult), int(group), int(heavy_T), int(dft_path)
    p.ident = int(ident)
    p.gather_path = int(gather_path)
    p.dft_split = int(dft_split)
    return p


def _info_dict(info: PlanInfo) -> dict:
    K = info.K
    d = {name: getattr(info, name) for name, _ in PlanInfo._fields_
         if name not in ("primes", "P")}
    d["primes"] = tuple(int(info.primes[j]) for j in range(K))
    d["P"] = tuple(int(info.P[j]) for j in range(K))
    d["q"] = tuple(info.q_first + 2 * b * info.L for b in range(info.Q))
    return d


def describe(N: int, s: int, **params) -> dict:
    """The plan the library derives for (N, s, params); host only, no device."""
    info = PlanInfo()
    p = make_params(**params)
    _check(load_library().sft_plan_describe(int(N), int(s), ctypes.byref(p), ctypes.byref(info)))
    return _info_dict(info)


def _check_input(f, N: int):
    import torch
    if not isinstance(f, torch.Tensor) or f.dtype != torch.complex64 or f.dim() != 1 or f.shape[0] != N \
            or not f.is_cuda:
        raise ValueError("f must be a complex64 cuda tensor of its plan's length")
    if not f.is_contiguous():
        raise ValueError("f must be contiguous")


def _check_outputs(w, c, s: int, device, n=None):
    """Caller-supplied outputs: int64[s] frequencies and complex64[s]
    coefficients (and an int32 count tensor), contiguous, on f's device."""
    import torch
    for t, dt, name in ((w, torch.int64, "freqs"), (c, torch.complex64, "coefs")):
        if not isinstance(t, torch.Tensor) or t.dtype != dt or t.dim() != 1 or t.shape[0] < s \
                or t.device != device or not t.is_contiguous():
            raise ValueError(f"output {name} must be a contiguous {dt} tensor of at least {s} entries on {device}")
    if n is not None and (not isinstance(n, torch.Tensor) or n.dtype != torch.int32 or n.numel() < 1
                          or n.device != device or not n.is_contiguous()):
        raise ValueError(f"output count must be a contiguous int32 tensor on {device}")


def _check_counts(counts, n: int, device):
    import torch
    if not isinstance(counts, torch.Tensor) or counts.dtype != torch.int32 or counts.numel() < n \
            or counts.device != device or not counts.is_contiguous():
        raise ValueError(f"counts must be a contiguous int32 tensor of at least {n} entries on {device}")


def _stream_handle(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A plan for transforms of length N with sparsity s (device tables + workspace)."""

    def __init__(self, N: int, s: int, **params):
        lib = load_library()
        self._h = ctypes.c_void_p()
        p = make_params(**params)
        _check(lib.sft_plan_create(ctypes.byref(self._h), int(N), int(s), ctypes.byref(p)))
        info = PlanInfo()
        _check(lib.sft_plan_get_info(self._h, ctypes.byref(info)))
        self.info = _info_dict(info)
        self.N = int(N)
        self.s = int(s)

    @property
    def handle(self):
        return self._h

    def footprint(self) -> int:
        """Device bytes the plan holds now (tables; its sft_execute workspace once allocated)."""
        v = ctypes.c_size_t()
        _check(load_library().sft_plan_footprint(self._h, ctypes.byref(v)))
        return int(v.value)

    def workspace_bytes(self) -> int:
        """Device workspace one transform of this plan needs (alone or in a batch)."""
        v = ctypes.c_size_t()
        _check(load_library().sft_plan_workspace_bytes(self._h, ctypes.byref(v)))
        return int(v.value)

    def outputs(self, device=None):
        import torch
        dev = device or torch.device("cuda")
        return (torch.empty(self.s, dtype=torch.int64, device=dev),
                torch.empty(self.s, dtype=torch.complex64, device=dev),
                torch.empty(1, dtype=torch.int32, device=dev))

    def execute(self, f, out=None, stream=None):
        """Enqueue one transform of the complex64 device tensor f (shape [N]).
        Returns (freqs int64[s], coefs complex64[s], count int32[1]) device tensors."""
        _check_input(f, self.N)
        w, c, n = out if out is not None else self.outputs(f.device)
        _check_outputs(w, c, self.s, f.device, n)
        _check(load_library().sft_execute(self._h, ctypes.c_void_p(f.data_ptr()),
                                          ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                          ctypes.c_void_p(n.data_ptr()), _stream_handle(stream)))
        return w, c, n

    def execute_noalloc(self, f, out, stream=None):
        """As execute(), through sft_execute_noalloc: the library allocates
        nothing (its per-device scratch is the workspace); the caller supplies
        the outputs (freqs int64[s], coefs complex64[s], count int32[1])."""
        _check_input(f, self.N)
        w, c, n = out
        _check_outputs(w, c, self.s, f.device, n)
        _check(load_library().sft_execute_noalloc(self._h, ctypes.c_void_p(f.data_ptr()),
                                                  ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                                  ctypes.c_void_p(n.data_ptr()), _stream_handle(stream)))
        return w, c, n

    def status(self) -> int:
        flags = ctypes.c_int32(0)
        rc = load_library().sft_plan_status(self._h, ctypes.byref(flags))
        if rc not in (SFT_OK, SFT_EOVERFLOW):
            _check(rc)
        return int(flags.value)

    def fetch(self, what: int) -> np.ndarray:
        """Copy an intermediate of the last execute() to host (synchronises)."""
        lib = load_library()
        need = ctypes.c_size_t()
        _check(lib.sft_plan_fetch(self._h, int(what), None, 0, ctypes.byref(need)))
        buf = np.empty(need.value, dtype=np.uint8)
        _check(lib.sft_plan_fetch(self._h, int(what), ctypes.c_void_p(buf.ctypes.data), need.value, None))
        if what in (FETCH_SAMPLES, FETCH_BINS, FETCH_SAMPLES_SHIFTED, FETCH_BINS_SHIFTED):
            return buf.view(np.complex64)
        if what in (FETCH_HEAVY, FETCH_CLASSES):
            return buf.view(np.int32)
        Q, s = self.info["Q"], self.s
        counts = buf[: 4 * Q].view(np.int32).copy()
        rec = buf[4 * Q:].view(np.dtype([("w", "<i8"), ("re", "<f8"), ("im", "<f8")])).reshape(Q, s)
        return counts, rec

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().sft_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def execute_many(plans: Sequence[Plan], fs, outs=None, counts=None, stream=None):
    """Enqueue len(plans) transforms in one batched launch sequence.
    Returns (list of (freqs, coefs) device tensors, counts int32[count])."""
    import torch
    n = len(plans)
    if len(fs) != n:
        raise ValueError("plans and fs differ in length")
    if outs is None:
        outs = [(torch.empty(p.s, dtype=torch.int64, device=f.device),
                 torch.empty(p.s, dtype=torch.complex64, device=f.device)) for p, f in zip(plans, fs)]
    if counts is None:
        counts = torch.empty(n, dtype=torch.int32, device=fs[0].device if n else "cuda")
    if len(outs) != n:
        raise ValueError("plans and outs differ in length")
    for p, f, o in zip(plans, fs, outs):
        _check_input(f, p.N)
        _check_outputs(o[0], o[1], p.s, f.device)
    if n:
        _check_counts(counts, n, fs[0].device)
    VP = ctypes.c_void_p * n
    hp = VP(*[p.handle.value for p in plans])
    hf = VP(*[f.data_ptr() for f in fs])
    hw = VP(*[o[0].data_ptr() for o in outs])
    hc = VP(*[o[1].data_ptr() for o in outs])
    _check(load_library().sft_execute_many(hp, n, hf, hw, hc, ctypes.c_void_p(counts.data_ptr()),
                                           _stream_handle(stream)))
    return outs, counts


def execute_many_status(stream, count: int) -> list:
    """Per-transform status flags of the last execute_many on `stream`
    (synchronises it); a nonzero entry is a device-side capacity overflow."""
    flags = (ctypes.c_int32 * max(1, count))()
    rc = load_library().sft_execute_many_status(_stream_handle(stream), int(count), flags)
    if rc not in (SFT_OK, SFT_EOVERFLOW):
        _check(rc)
    return [int(flags[i]) for i in range(count)]


def execute_many_reserve(stream, workspace_bytes: int, count: int):
    """Size the library's workspace of `stream` for batches of up to `count`
    transforms needing at most `workspace_bytes` (sum of workspace_bytes())."""
    _check(load_library().sft_execute_many_reserve(_stream_handle(stream), int(workspace_bytes), int(count)))


def execute_many_release(stream):
    """Free the library's workspace of `stream` (after its work completes)."""
    _check(load_library().sft_execute_many_release(_stream_handle(stream)))


class Batch:
    """A prepared batch (sft_batch_*): the plans, inputs and outputs of an
    execute_many fixed once; launch() enqueues the kernels only, graph_launch()
    replays them as a captured hipGraph.  Rewrite the input tensors in place
    between launches; launches of one batch must not overlap."""

    def __init__(self, plans: Sequence[Plan], fs, outs=None, counts=None):
        import torch
        n = len(plans)
        if n < 1 or len(fs) != n:
            raise ValueError("plans and fs must be non-empty and of equal length")
        for p, f in zip(plans, fs):
            _check_input(f, p.N)
        if outs is None:
            outs = [(torch.empty(p.s, dtype=torch.int64, device=f.device),
                     torch.empty(p.s, dtype=torch.complex64, device=f.device)) for p, f in zip(plans, fs)]
        if counts is None:
            counts = torch.empty(n, dtype=torch.int32, device=fs[0].device)
        if len(outs) != n:
            raise ValueError("plans and outs differ in length")
        for p, f, o in zip(plans, fs, outs):
            _check_outputs(o[0], o[1], p.s, f.device)
        _check_counts(counts, n, fs[0].device)
        # the batch holds device pointers: keep the tensors and plans alive with it
        self.plans, self.fs, self.outs, self.counts = list(plans), list(fs), outs, counts
        VP = ctypes.c_void_p * n
        self._h = ctypes.c_void_p()
        _check(load_library().sft_batch_create(
            ctypes.byref(self._h), VP(*[p.handle.value for p in plans]), n, VP(*[f.data_ptr() for f in fs]),
            VP(*[o[0].data_ptr() for o in outs]), VP(*[o[1].data_ptr() for o in outs]),
            ctypes.c_void_p(counts.data_ptr())))

    def launch(self, stream=None):
        _check(load_library().sft_batch_launch(self._h, _stream_handle(stream)))
        return self.outs, self.counts

    def graph_launch(self, stream=None):
        _check(load_library().sft_batch_graph_launch(self._h, _stream_handle(stream)))
        return self.outs, self.counts

    def status(self) -> list:
        """Per-transform status flags of the last launch (synchronises)."""
        n = len(self.plans)
        flags = (ctypes.c_int32 * n)()
        rc = load_library().sft_batch_status(self._h, flags)
        if rc not in (SFT_OK, SFT_EOVERFLOW):
            _check(rc)
        return [int(flags[i]) for i in range(n)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().sft_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True):
    _check(load_library().sft_profile_enable(1 if on else 0))


def profile_reset():
    _check(load_library().sft_profile_reset())


def profile_read(kernel: int):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load_library().sft_profile_read(int(kernel), ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def samples_natural(plan: Plan, flat: np.ndarray, b: int, j: int) -> np.ndarray:
    """Reorder the fetched samples of (band b, modulus j) into node order k."""
    info = plan.info
    Q, s1 = info["Q"], info["s1"]
    p, P = info["primes"][j], info["P"][j]
    off = Q * sum(info["P"][:j]) + b * P
    blk = flat[off: off + P]
    idx = np.arange(P)
    n1, n2 = idx % s1, idx // s1
    k = (n1 * p + n2 * s1) % P
    out = np.empty(P, dtype=flat.dtype)
    out[k] = blk
    return out


def bins_natural(plan: Plan, flat: np.ndarray, b: int, j: int) -> np.ndarray:
    """Reorder the fetched DFT bins of (band b, modulus j) into bin order h."""
    info = plan.info
    Q, s1 = info["Q"], info["s1"]
    p, P = info["primes"][j], info["P"][j]
    off = Q * sum(info["P"][:j]) + b * P
    blk = flat[off: off + P]
    h = np.arange(P)
    return blk[(h % p) * s1 + (h % s1)]


def heavy_block(plan: Plan, flat: np.ndarray, b: int, j: int) -> np.ndarray:
    info = plan.info
    Q, T = info["Q"], info["T"]
    return flat[(j * Q + b) * T: (j * Q + b + 1) * T]
