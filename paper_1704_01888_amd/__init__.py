"""Population annealing of the 2D q-state Potts model on MI355X (gfx950).

Python binding of the C ABI in ``include/pa.h`` (libpa.so).  Argument
marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch provides device memory (the workspace) and the stream.

Method: Barash, Weigel, Shchur, Janke, arXiv:1704.01888, Sec. 2-3.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpa.so")

PA_OK, PA_ERR_INVALID, PA_ERR_NOMEM, PA_ERR_DEVICE, PA_ERR_CAPACITY, PA_ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5
RESAMPLE_POISSON, RESAMPLE_MULTINOMIAL, RESAMPLE_NONE = 0, 1, 2
INIT_RANDOM, INIT_GROUND = 0, 1
OUT_HIST, OUT_MAG, OUT_FINAL, OUT_WIDTHS, OUT_DIGEST = 1, 2, 4, 8, 16
KERNEL_NAMES = ("init", "sweep", "post", "resample")

EXPORTS = [
    "pa_plan", "pa_plan_tables", "pa_weight_table", "pa_ctx_create", "pa_ctx_destroy",
    "pa_ctx_set_profiling", "pa_ctx_set_lanes", "pa_ctx_get_lanes", "pa_autotune",
    "pa_ctx_set_graphs", "pa_ctx_set_batch_mode", "pa_ctx_abort_batch",
    "pa_ctx_batch_info", "pa_tune", "pa_tune_set", "pa_tune_get", "pa_tune_save", "pa_tune_load",
    "pa_run", "pa_run_begin", "pa_run_advance", "pa_run_sync", "pa_run_read", "pa_run_load",
    "pa_run_read_free_energy",
    "pa_run_read_slots", "pa_run_finish", "pa_status_str", "pa_last_error",
    "pa_plan_batch", "pa_run_batch",
    "pa_serve_start", "pa_serve_submit", "pa_serve_wait", "pa_serve_cancel", "pa_serve_stop",
    "pa_width_maxima", "pa_free_energy_crossing", "pa_issue_probe",
    "pa_checkpoint", "pa_checkpoint_info", "pa_resume", "pa_serve_checkpoint", "pa_serve_resume",
    "pa_run_static",
]
STATIC_SCRATCH_BYTES = 64 << 20
PROBE_KINDS = ("xor", "bitop3", "mad64", "perm", "sad", "xad", "mulhi", "cmpsel", "mix")
PA_ERR_BUSY, PA_ERR_CANCELLED, PA_ERR_TIMEOUT = -6, -7, -8
BATCH_TEAM, BATCH_SEGMENTED = 0, 1


class PAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class RunDesc(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_uint32), ("q", ctypes.c_uint32), ("R", ctypes.c_uint64),
        ("K", ctypes.c_uint32), ("beta", ctypes.POINTER(ctypes.c_double)),
        ("theta", ctypes.c_uint32), ("seed", ctypes.c_uint64),
        ("resample", ctypes.c_int32), ("init", ctypes.c_int32), ("outputs", ctypes.c_uint32),
        ("bin_e", ctypes.c_uint32), ("bin_m", ctypes.c_uint32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("R_i", ctypes.c_void_p), ("E_sum", ctypes.c_void_p), ("E_mean", ctypes.c_void_p),
        ("lnQ", ctypes.c_void_p), ("minus_beta_F", ctypes.c_void_p), ("hist", ctypes.c_void_p),
        ("Mt_sum", ctypes.c_void_p), ("M_mean", ctypes.c_void_p), ("mhist", ctypes.c_void_p),
        ("width_e", ctypes.c_void_p), ("width_m", ctypes.c_void_p), ("digest", ctypes.c_void_p),
        ("final_spins", ctypes.c_void_p), ("final_E", ctypes.c_void_p),
        ("last_anc", ctypes.c_void_p), ("kernel_ms", ctypes.c_void_p),
        ("kernel_launches", ctypes.c_void_p),
    ]


class Timing(ctypes.Structure):
    _fields_ = [("arrival_us", ctypes.c_double), ("admit_us", ctypes.c_double),
                ("done_us", ctypes.c_double), ("attempts", ctypes.c_uint64)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("q_large", ctypes.c_uint32), ("r_class", ctypes.c_uint32),
                ("lanes", ctypes.c_uint32), ("waves_per_block", ctypes.c_uint32),
                ("attempts_per_ns", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("R_cap", ctypes.c_uint64), ("R_final", ctypes.c_uint64),
        ("workspace_bytes", ctypes.c_uint64), ("Kb", ctypes.c_uint32),
        ("n_tables", ctypes.c_uint32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libpa.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1704_01888_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32, dbl = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                              ctypes.c_double)
    P = ctypes.POINTER
    L.pa_plan.argtypes = [P(RunDesc), P(PlanInfo)]
    L.pa_plan_tables.argtypes = [P(RunDesc), vp, vp]
    L.pa_weight_table.argtypes = [dbl, u32, u32, vp, vp]
    L.pa_ctx_create.argtypes = [ctypes.c_int, P(vp)]
    L.pa_ctx_destroy.argtypes = [vp]
    L.pa_ctx_destroy.restype = None
    L.pa_ctx_set_profiling.argtypes = [vp, ctypes.c_int]
    L.pa_ctx_set_profiling.restype = i32
    L.pa_ctx_set_lanes.argtypes = [vp, u32, u32]
    L.pa_ctx_set_lanes.restype = i32
    L.pa_ctx_get_lanes.argtypes = [vp, u32, vp, vp, vp]
    L.pa_ctx_get_lanes.restype = i32
    L.pa_autotune.argtypes = [vp, u32, u32, vp, u64, vp, vp, vp]
    L.pa_autotune.restype = i32
    L.pa_tune.argtypes = [vp, u32, u32, u64, vp, u64, vp, P(TuneEntry), vp, u32, vp]
    L.pa_tune.restype = i32
    L.pa_tune_set.argtypes = [vp, P(TuneEntry)]
    L.pa_tune_set.restype = i32
    L.pa_tune_get.argtypes = [vp, u32, u32, u64, P(TuneEntry)]
    L.pa_tune_get.restype = i32
    L.pa_tune_save.argtypes = [vp, ctypes.c_char_p]
    L.pa_tune_save.restype = i32
    L.pa_tune_load.argtypes = [vp, ctypes.c_char_p, vp]
    L.pa_tune_load.restype = i32
    L.pa_ctx_set_graphs.argtypes = [vp, ctypes.c_int]
    L.pa_ctx_set_graphs.restype = i32
    L.pa_ctx_set_batch_mode.argtypes = [vp, ctypes.c_int]
    L.pa_ctx_set_batch_mode.restype = i32
    L.pa_ctx_abort_batch.argtypes = [vp]
    L.pa_ctx_batch_info.argtypes = [vp, vp, vp]
    L.pa_ctx_batch_info.restype = i32
    L.pa_ctx_abort_batch.restype = i32
    L.pa_run.argtypes = [vp, P(RunDesc), vp, u64, vp, P(Result)]
    L.pa_run_begin.argtypes = [vp, P(RunDesc), vp, u64, vp, P(vp)]
    L.pa_run_advance.argtypes = [vp, u32]
    L.pa_run_sync.argtypes = [vp]
    L.pa_run_read.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.pa_run_load.argtypes = [vp, u32, u64, vp, dbl]
    L.pa_run_read_free_energy.argtypes = [vp, vp, vp]
    L.pa_run_finish.argtypes = [vp, P(Result)]
    L.pa_run_read_slots.argtypes = [vp, ctypes.c_int, vp, u32, vp]
    L.pa_plan_batch.argtypes = [P(RunDesc), u32, P(u64)]
    L.pa_run_batch.argtypes = [vp, P(RunDesc), u32, vp, u64, vp, P(Result)]
    L.pa_serve_start.argtypes = [vp, vp, u64, u32, vp]
    L.pa_serve_submit.argtypes = [vp, P(RunDesc), P(Result), P(u64)]
    L.pa_serve_wait.argtypes = [vp, u64, ctypes.c_int64, P(Timing)]
    L.pa_serve_cancel.argtypes = [vp, u64]
    L.pa_serve_stop.argtypes = [vp]
    L.pa_width_maxima.argtypes = [vp, vp, u32, vp, vp, vp]
    L.pa_free_energy_crossing.argtypes = [vp, vp, vp, u32, vp]
    L.pa_run_static.argtypes = [vp, P(RunDesc), vp, P(Result)]
    L.pa_run_static.restype = i32
    L.pa_checkpoint.argtypes = [vp, ctypes.c_char_p]
    L.pa_checkpoint_info.argtypes = [ctypes.c_char_p, P(RunDesc), vp, u32, P(u32), P(u64)]
    L.pa_resume.argtypes = [vp, ctypes.c_char_p, vp, u64, vp, P(vp)]
    L.pa_serve_checkpoint.argtypes = [vp, u64, ctypes.c_char_p]
    L.pa_serve_resume.argtypes = [vp, ctypes.c_char_p, P(Result), P(u64)]
    for name in ("pa_checkpoint", "pa_checkpoint_info", "pa_resume", "pa_serve_checkpoint",
                 "pa_serve_resume"):
        getattr(L, name).restype = i32
    L.pa_issue_probe.argtypes = [vp, u32, vp, u64, vp, P(dbl)]
    L.pa_issue_probe.restype = i32
    L.pa_status_str.argtypes = [i32]
    L.pa_status_str.restype = ctypes.c_char_p
    L.pa_last_error.argtypes = []
    L.pa_last_error.restype = ctypes.c_char_p
    for name in ("pa_plan", "pa_plan_tables", "pa_weight_table", "pa_ctx_create", "pa_run",
                 "pa_run_begin", "pa_run_advance", "pa_run_sync", "pa_run_read", "pa_run_load",
                 "pa_run_read_slots", "pa_run_finish", "pa_plan_batch", "pa_run_batch",
                 "pa_serve_start", "pa_serve_submit", "pa_serve_wait", "pa_serve_cancel",
                 "pa_serve_stop"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(status: int):
    if status != PA_OK:
        raise PAError(status, lib().pa_last_error().decode())


def _ptr(a) -> int:
    return a.ctypes.data if a is not None else None


class Desc:
    """A run description (fields of ``pa_run_desc``)."""

    def __init__(self, L, q, R, beta, theta, seed, resample=RESAMPLE_POISSON, init=INIT_RANDOM,
                 outputs=0, bin_e=1, bin_m=1):
        self.L, self.q, self.R = int(L), int(q), int(R)
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        self.K = len(self.beta)
        self.theta, self.seed = int(theta), int(seed)
        self.resample, self.init, self.outputs = int(resample), int(init), int(outputs)
        self.bin_e, self.bin_m = int(bin_e), int(bin_m)

    @property
    def N(self):
        return self.L * self.L

    def c(self) -> RunDesc:
        d = RunDesc()
        d.L, d.q, d.R, d.K = self.L, self.q, self.R, self.K
        d.beta = self.beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.theta, d.seed = self.theta, self.seed
        d.resample, d.init, d.outputs = self.resample, self.init, self.outputs
        d.bin_e, d.bin_m = self.bin_e, self.bin_m
        return d


def pa_plan(desc: Desc) -> PlanInfo:
    info = PlanInfo()
    _check(lib().pa_plan(ctypes.byref(desc.c()), ctypes.byref(info)))
    return info


def pa_plan_tables(desc: Desc):
    T = np.zeros((desc.K, 4), dtype=np.uint64)
    R_sched = np.zeros(desc.K, dtype=np.uint64)
    _check(lib().pa_plan_tables(ctypes.byref(desc.c()), _ptr(T), _ptr(R_sched)))
    return T, R_sched


def pa_weight_table(abs_dbeta: float, Kb: int, N: int):
    W = np.zeros(2 * N + 1, dtype=np.uint64)
    D = ctypes.c_uint32(0)
    _check(lib().pa_weight_table(float(abs_dbeta), int(Kb), int(N), _ptr(W), ctypes.byref(D)))
    return W, int(D.value)


def width_maxima(beta, width):
    """(i_max, w_max, T_max) of a width curve (pa_width_maxima)."""
    b = np.ascontiguousarray(beta, dtype=np.float64)
    w = np.ascontiguousarray(width, dtype=np.float64)
    if len(b) != len(w):
        raise ValueError("beta and width differ in length")
    i = np.zeros(1, np.uint32)
    wm = np.zeros(1)
    tm = np.zeros(1)
    _check(lib().pa_width_maxima(_ptr(b), _ptr(w), len(b), _ptr(i), _ptr(wm), _ptr(tm)))
    return int(i[0]), float(wm[0]), float(tm[0])


def free_energy_crossing(beta, mbf_cool, mbf_heat) -> float:
    """Crossing of cooling and heating -beta F on an increasing beta grid
    (pa_free_energy_crossing)."""
    b = np.ascontiguousarray(beta, dtype=np.float64)
    c = np.ascontiguousarray(mbf_cool, dtype=np.float64)
    h = np.ascontiguousarray(mbf_heat, dtype=np.float64)
    if not (len(b) == len(c) == len(h)):
        raise ValueError("arrays differ in length")
    x = np.zeros(1)
    _check(lib().pa_free_energy_crossing(_ptr(b), _ptr(c), _ptr(h), len(b), _ptr(x)))
    return float(x[0])


def tune_cache_path(device: int = 0) -> str:
    """The cache of tuned sweep shapes shipped with the package (one file for
    every architecture; pa_tune_load keeps the lines of the device's)."""
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.jsonl")


class Context:
    """A device handle (``pa_ctx``) on torch's current HIP device.  With
    tune_cache (the default) the tuned sweep shapes of tune_cache_path() are
    loaded, so that every run on the context uses them."""

    def __init__(self, device: int | None = None, tune_cache: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        _check(lib().pa_ctx_create(self.device, ctypes.byref(h)))
        self.handle = h
        if tune_cache and os.path.exists(tune_cache_path(self.device)):
            try:
                self.tune_load(tune_cache_path(self.device))
            except PAError as e:          # a damaged cache leaves the default shapes
                import warnings
                warnings.warn(f"tuned shapes not loaded: {e}")

    def set_lanes(self, L: int, lanes: int):
        _check(lib().pa_ctx_set_lanes(self.handle, int(L), int(lanes)))

    def get_lanes(self, L: int):
        """(lanes in use, candidate list) for lattice side L."""
        cur = np.zeros(1, np.uint32)
        cand = np.zeros(2, np.uint32)
        n = np.zeros(1, np.uint32)
        _check(lib().pa_ctx_get_lanes(self.handle, int(L), _ptr(cur), _ptr(cand), _ptr(n)))
        return int(cur[0]), [int(x) for x in cand[: int(n[0])]]

    def autotune(self, L: int, q: int, workspace=None):
        """Time the lane candidates for (L, q); keep and return the fastest."""
        ws = workspace if workspace is not None else _workspace(256 << 20, self.device)
        best = np.zeros(1, np.uint32)
        rate = np.zeros(1, np.float64)
        _check(lib().pa_autotune(self.handle, int(L), int(q), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream_ptr(), _ptr(best), _ptr(rate)))
        return int(best[0]), float(rate[0])

    def tune(self, L: int, q: int, R: int, workspace=None) -> dict:
        """Time every sweep shape of L on R replicas (pa_tune); the fastest
        becomes the entry of the (L, q, R) class and is returned, with every
        shape's rate under "timed"."""
        d = Desc(L=int(L), q=int(q), R=int(R), beta=np.array([0.0, 0.5, 1.0]), theta=10, seed=12345,
                 resample=RESAMPLE_MULTINOMIAL)
        ws = workspace if workspace is not None else _workspace(pa_plan(d).workspace_bytes, self.device)
        e = TuneEntry()
        timed = (TuneEntry * 64)()
        n = ctypes.c_uint32(0)
        _check(lib().pa_tune(self.handle, int(L), int(q), int(R), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                             _stream_ptr(), ctypes.byref(e), timed, 64, ctypes.byref(n)))
        out = e.as_dict()
        out["timed"] = [timed[i].as_dict() for i in range(min(n.value, 64))]
        return out

    def tune_set(self, L: int, q_large: int, r_class: int, lanes: int, waves_per_block: int):
        """Install a tuned shape for a class (pa_tune_set)."""
        e = TuneEntry(int(L), int(q_large), int(r_class), int(lanes), int(waves_per_block), 0.0)
        _check(lib().pa_tune_set(self.handle, ctypes.byref(e)))

    def tune_get(self, L: int, q: int, R: int) -> dict:
        """The sweep shape later runs of (L, q, R) use (pa_tune_get)."""
        e = TuneEntry()
        _check(lib().pa_tune_get(self.handle, int(L), int(q), int(R), ctypes.byref(e)))
        return e.as_dict()

    def tune_save(self, path):
        _check(lib().pa_tune_save(self.handle, os.fsencode(str(path))))

    def tune_load(self, path) -> int:
        n = ctypes.c_uint32(0)
        _check(lib().pa_tune_load(self.handle, os.fsencode(str(path)), ctypes.byref(n)))
        return int(n.value)

    def issue_probe(self, kind: str) -> float:
        """Lane-instructions per second of a stream of one instruction kind
        (PROBE_KINDS; pa_issue_probe) on this device."""
        import torch
        props = torch.cuda.get_device_properties(self.device)
        out = _workspace(4 * 256 * 8 * props.multi_processor_count, self.device)
        rate = ctypes.c_double(0.0)
        _check(lib().pa_issue_probe(self.handle, PROBE_KINDS.index(kind),
                                    ctypes.c_void_p(out.data_ptr()), out.numel(), _stream_ptr(),
                                    ctypes.byref(rate)))
        return float(rate.value)

    def set_graphs(self, on: bool):
        _check(lib().pa_ctx_set_graphs(self.handle, 1 if on else 0))

    def set_batch_mode(self, mode: int):
        """BATCH_SEGMENTED (default) or BATCH_TEAM for later pa_run_batch calls."""
        _check(lib().pa_ctx_set_batch_mode(self.handle, int(mode)))

    def batch_info(self):
        """(runs finished in team launches, team launches) of the last batch."""
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().pa_ctx_batch_info(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def abort_batch(self):
        """Stop the pa_run_batch running on this context (from another thread)."""
        _check(lib().pa_ctx_abort_batch(self.handle))

    def set_profiling(self, on: bool):
        _check(lib().pa_ctx_set_profiling(self.handle, 1 if on else 0))

    def close(self):
        if self.handle:
            lib().pa_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _workspace(nbytes: int, device: int):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=f"cuda:{device}")


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _final_plan(desc: Desc):
    """The plan when the result needs its final population size, else None
    (planning builds the run's tables: tens of microseconds per run)."""
    return pa_plan(desc) if desc.outputs & OUT_FINAL else None


_ITEMSIZE = {np.uint8: 1, np.int32: 4, np.uint32: 4, np.int64: 8, np.uint64: 8, np.float64: 8}


def _alloc_result(desc: Desc, info):
    """Result arrays and the pa_result pointing at them; `info` (a plan) is
    needed for the final population's buffers only (OUT_FINAL).  The arrays
    are views of one zeroed buffer (one address lookup per result)."""
    K, N, o = desc.K, desc.N, desc.outputs
    fields = [("R_i", (K,), np.uint64), ("E_sum", (K,), np.int64), ("E_mean", (K,), np.float64),
              ("lnQ", (K,), np.float64), ("minus_beta_F", (K,), np.float64)]
    if o & OUT_HIST:
        fields.append(("hist", (K, 2 * N + 1), np.uint32))
    if o & OUT_MAG:
        fields += [("Mt_sum", (K,), np.int64), ("M_mean", (K,), np.float64)]
        if o & OUT_HIST:
            fields.append(("mhist", (K, N + 1), np.uint32))
    if o & OUT_WIDTHS:
        fields.append(("width_e", (K,), np.float64))
        if o & OUT_MAG:
            fields.append(("width_m", (K,), np.float64))
    if o & OUT_DIGEST:
        fields.append(("digest", (K,), np.uint64))
    if o & OUT_FINAL:
        RF = int(info.R_final)
        fields += [("final_spins", (RF, N), np.uint8), ("final_E", (RF,), np.int32),
                   ("last_anc", (RF,), np.uint32)]
    fields += [("kernel_ms", (len(KERNEL_NAMES),), np.float64),
               ("kernel_launches", (len(KERNEL_NAMES),), np.uint64)]
    spans, total = [], 0
    for name, shape, dt in fields:
        count = shape[0] * shape[1] if len(shape) == 2 else shape[0]
        nbytes = count * _ITEMSIZE[dt]
        spans.append((name, shape, dt, total, nbytes))
        total += (nbytes + 7) & ~7
    buf = np.zeros(max(total, 8), np.uint8)
    base = buf.ctypes.data
    out, res = {}, Result()
    for name, shape, dt, off, nbytes in spans:
        v = buf[off:off + nbytes].view(dt)
        out[name] = v if len(shape) == 1 else v.reshape(shape)
        setattr(res, name, base + off)
    return out, res


def pa_run(ctx: Context, desc: Desc, workspace=None):
    """Whole run on the current torch stream; returns a dict of numpy arrays."""
    info = pa_plan(desc) if workspace is None else _final_plan(desc)
    ws = workspace if workspace is not None else _workspace(info.workspace_bytes, ctx.device)
    out, res = _alloc_result(desc, info)
    _check(lib().pa_run(ctx.handle, ctypes.byref(desc.c()), ctypes.c_void_p(ws.data_ptr()),
                        ws.numel(), _stream_ptr(), ctypes.byref(res)))
    return out


def pa_run_static(ctx: Context, desc: Desc):
    """Whole run in the library's fixed device workspace (pa_run_static: no
    device allocation by the call); returns a dict of numpy arrays."""
    out, res = _alloc_result(desc, _final_plan(desc))
    _check(lib().pa_run_static(ctx.handle, ctypes.byref(desc.c()), _stream_ptr(), ctypes.byref(res)))
    return out


class Run:
    """Stepwise run (pa_run_begin / advance / read / load / finish)."""

    def __init__(self, ctx: Context, desc: Desc, workspace=None):
        self.desc = desc
        self.info = pa_plan(desc)
        self.ws = workspace if workspace is not None else _workspace(self.info.workspace_bytes,
                                                                     ctx.device)
        h = ctypes.c_void_p()
        _check(lib().pa_run_begin(ctx.handle, ctypes.byref(desc.c()),
                                  ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                  _stream_ptr(), ctypes.byref(h)))
        self.handle = h

    def advance(self, n: int = 1):
        _check(lib().pa_run_advance(self.handle, int(n)))

    def sync(self):
        _check(lib().pa_run_sync(self.handle))

    def read(self, spins=True, E=True, anc=True, counts=True):
        step = ctypes.c_uint32()
        R_cur, R_prev = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().pa_run_read(self.handle, ctypes.byref(step), ctypes.byref(R_cur),
                                 ctypes.byref(R_prev), None, None, None, None))
        rc, rp, N = int(R_cur.value), int(R_prev.value), self.desc.N
        out = {"step": int(step.value), "R_cur": rc, "R_prev": rp}
        bufs = {}
        if spins:
            bufs["spins"] = np.zeros((rc, N), np.uint8)
        if E:
            bufs["E"] = np.zeros(rc, np.int32)
        if anc:
            bufs["anc"] = np.zeros(rc, np.uint32)
        if counts:
            bufs["counts"] = np.zeros(rp, np.uint32)
        _check(lib().pa_run_read(self.handle, None, None, None, _ptr(bufs.get("spins")),
                                 _ptr(bufs.get("E")), _ptr(bufs.get("anc")),
                                 _ptr(bufs.get("counts"))))
        out.update(bufs)
        return out

    def load(self, step: int, spins: np.ndarray, minus_beta_F: float):
        s = np.ascontiguousarray(spins, dtype=np.uint8)
        _check(lib().pa_run_load(self.handle, int(step), int(s.shape[0]), _ptr(s),
                                 float(minus_beta_F)))

    def free_energy(self):
        """(step, -beta F of the current step)."""
        step, v = ctypes.c_uint32(), ctypes.c_double()
        _check(lib().pa_run_read_free_energy(self.handle, ctypes.byref(step), ctypes.byref(v)))
        return int(step.value), float(v.value)

    def checkpoint(self, path):
        """Write the current step, population and -beta F with the run
        description to `path` (pa_checkpoint; the binary format of pa.h)."""
        _check(lib().pa_checkpoint(self.handle, os.fsencode(str(path))))

    @classmethod
    def resume(cls, ctx: "Context", path, workspace=None) -> "Run":
        """A run continued from a checkpoint file (pa_resume); it finishes
        bit-identically to the run the checkpoint was taken from (results from
        the checkpoint step on)."""
        desc, _, _ = checkpoint_info(path)
        run = cls.__new__(cls)
        run.desc = desc
        run.info = pa_plan(desc)
        run.ws = workspace if workspace is not None else _workspace(run.info.workspace_bytes,
                                                                    ctx.device)
        h = ctypes.c_void_p()
        _check(lib().pa_resume(ctx.handle, os.fsencode(str(path)), ctypes.c_void_p(run.ws.data_ptr()),
                               run.ws.numel(), _stream_ptr(), ctypes.byref(h)))
        run.handle = h
        return run

    def read_slots(self, slots, previous=False):
        sl = np.ascontiguousarray(slots, dtype=np.uint32)
        out = np.zeros((len(sl), self.desc.N), np.uint8)
        _check(lib().pa_run_read_slots(self.handle, 1 if previous else 0, _ptr(sl), len(sl),
                                       _ptr(out)))
        return out

    def finish(self):
        out, res = _alloc_result(self.desc, self.info)
        h, self.handle = self.handle, None
        _check(lib().pa_run_finish(h, ctypes.byref(res)))
        return out

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                lib().pa_run_finish(self.handle, None)
            except Exception:
                pass


def checkpoint_info(path):
    """(Desc, step, R_cur) of a checkpoint file (pa_checkpoint_info)."""
    d = RunDesc()
    step, R_cur = ctypes.c_uint32(), ctypes.c_uint64()
    _check(lib().pa_checkpoint_info(os.fsencode(str(path)), ctypes.byref(d), None, 0,
                                    ctypes.byref(step), ctypes.byref(R_cur)))
    beta = np.zeros(d.K)
    _check(lib().pa_checkpoint_info(os.fsencode(str(path)), ctypes.byref(d), _ptr(beta), d.K, None,
                                    None))
    desc = Desc(d.L, d.q, d.R, beta, d.theta, d.seed, resample=d.resample, init=d.init,
                outputs=d.outputs, bin_e=d.bin_e, bin_m=d.bin_m)
    return desc, int(step.value), int(R_cur.value)


def _desc_array(descs):
    arr = (RunDesc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d.c()
    return arr


def pa_plan_batch(descs) -> int:
    n = ctypes.c_uint64(0)
    arr = _desc_array(descs)
    _check(lib().pa_plan_batch(arr, len(descs), ctypes.byref(n)))
    return int(n.value)


def pa_run_batch(ctx: Context, descs, workspace=None):
    """Several independent runs advanced together; returns one result dict per run."""
    ws = workspace if workspace is not None else _workspace(pa_plan_batch(descs), ctx.device)
    outs, ress = [], (Result * len(descs))()
    for i, d in enumerate(descs):
        o, r = _alloc_result(d, _final_plan(d))
        outs.append(o)
        ress[i] = r
    arr = _desc_array(descs)
    _check(lib().pa_run_batch(ctx.handle, arr, len(descs), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), _stream_ptr(), ress))
    return outs


class Server:
    """Continuous-batching server (pa_serve_*) on a context and a device arena."""

    def __init__(self, ctx: Context, arena_bytes: int, max_slots: int, arena=None):
        self.ctx = ctx
        self.arena = arena if arena is not None else _workspace(arena_bytes, ctx.device)
        self._live = {}
        _check(lib().pa_serve_start(ctx.handle, ctypes.c_void_p(self.arena.data_ptr()),
                                    self.arena.numel(), int(max_slots), _stream_ptr()))
        self.running = True

    def submit(self, desc: Desc) -> int:
        out, res = _alloc_result(desc, _final_plan(desc))
        t = ctypes.c_uint64(0)
        _check(lib().pa_serve_submit(self.ctx.handle, ctypes.byref(desc.c()), ctypes.byref(res),
                                     ctypes.byref(t)))
        self._live[int(t.value)] = (out, res, desc)
        return int(t.value)

    def wait(self, ticket: int, timeout_us: int = -1):
        """Returns (result dict, timing dict); raises PAError on failure."""
        tm = Timing()
        st = lib().pa_serve_wait(self.ctx.handle, int(ticket), int(timeout_us), ctypes.byref(tm))
        if st == PA_ERR_TIMEOUT:
            raise PAError(st, lib().pa_last_error().decode())
        out, res, desc = self._live.pop(int(ticket))
        _check(st)
        return out, {"arrival_us": tm.arrival_us, "admit_us": tm.admit_us, "done_us": tm.done_us,
                     "attempts": int(tm.attempts)}

    def cancel(self, ticket: int):
        _check(lib().pa_serve_cancel(self.ctx.handle, int(ticket)))

    def checkpoint(self, ticket: int, path):
        """Write a running ticket's state to `path` (pa_serve_checkpoint)."""
        _check(lib().pa_serve_checkpoint(self.ctx.handle, int(ticket), os.fsencode(str(path))))

    def resume(self, path) -> int:
        """Submit a request continuing a checkpoint file (pa_serve_resume)."""
        desc, _, _ = checkpoint_info(path)
        out, res = _alloc_result(desc, _final_plan(desc))
        t = ctypes.c_uint64(0)
        _check(lib().pa_serve_resume(self.ctx.handle, os.fsencode(str(path)), ctypes.byref(res),
                                     ctypes.byref(t)))
        self._live[int(t.value)] = (out, res, desc)
        return int(t.value)

    def stop(self):
        if self.running:
            _check(lib().pa_serve_stop(self.ctx.handle))
            self.running = False

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
