"""CPU oracle for population annealing of the 2D q-state Potts model.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does.  The
oracle shares no source with the GPU library.

The numerical work lives in ``pa_oracle.c`` (plain C, IEEE double), built into
``liboracle.so`` by :func:`build`; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RESAMPLE_POISSON, RESAMPLE_MULTINOMIAL, RESAMPLE_NONE = 0, 1, 2
INIT_RANDOM, INIT_GROUND = 0, 1
DOM_INIT, DOM_SWEEP, DOM_RESAMPLE, DOM_PLAN, DOM_GROUND = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP over replicas, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Desc(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_uint32), ("q", ctypes.c_uint32),
        ("R", ctypes.c_uint64), ("K", ctypes.c_uint32),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("theta", ctypes.c_uint32), ("seed", ctypes.c_uint64),
        ("resample", ctypes.c_int32), ("init", ctypes.c_int32),
        ("bin_e", ctypes.c_uint32), ("bin_m", ctypes.c_uint32),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("R_i", ctypes.c_void_p), ("E_sum", ctypes.c_void_p), ("E_mean", ctypes.c_void_p),
        ("lnQ", ctypes.c_void_p), ("minus_beta_F", ctypes.c_void_p),
        ("M_mean", ctypes.c_void_p), ("Mt_sum", ctypes.c_void_p), ("mhist", ctypes.c_void_p),
        ("width_e", ctypes.c_void_p), ("width_m", ctypes.c_void_p), ("digest", ctypes.c_void_p),
        ("hist", ctypes.c_void_p),
        ("final_spins", ctypes.c_void_p), ("final_E", ctypes.c_void_p),
        ("last_anc", ctypes.c_void_p), ("n_threads", ctypes.c_int),
    ]


class _Checkpoint(ctypes.Structure):
    _fields_ = [
        ("desc", _Desc), ("beta", ctypes.POINTER(ctypes.c_double)), ("step", ctypes.c_uint32),
        ("R_cur", ctypes.c_uint64), ("minus_beta_F", ctypes.c_double), ("E_sum", ctypes.c_int64),
        ("spins", ctypes.POINTER(ctypes.c_uint8)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, u32, u64, i32, dbl = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_int32, ctypes.c_double)
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_validate.argtypes = [ctypes.POINTER(_Desc)]
        L.orc_thresholds.argtypes = [dbl, vp]
        L.orc_weights.argtypes = [dbl, u32, u32, vp]
        L.orc_weights.restype = u32
        L.orc_poisson.argtypes = [dbl, dbl]
        L.orc_poisson.restype = u64
        L.orc_plan.argtypes = [ctypes.POINTER(_Desc), vp, vp, vp]
        L.orc_energy.argtypes = [u32, vp]
        L.orc_energy.restype = i32
        L.orc_mtilde.argtypes = [u32, u32, vp]
        L.orc_mtilde.restype = u32
        L.orc_init_replica.argtypes = [ctypes.POINTER(_Desc), u64, vp]
        L.orc_sweep_replica.argtypes = [ctypes.POINTER(_Desc), u32, u64, vp]
        L.orc_one_sweep.argtypes = [ctypes.POINTER(_Desc), u32, u32, u64, vp, vp]
        L.orc_resample.argtypes = [ctypes.POINTER(_Desc), u32, u32, vp, u64, u64, vp, vp, vp]
        L.orc_lnQ.argtypes = [u32, dbl, vp, u64, vp]
        L.orc_lnQ.restype = dbl
        L.orc_fwhm.argtypes = [vp, u32, u32]
        L.orc_fwhm.restype = dbl
        L.orc_width_maxima.argtypes = [vp, vp, u32, vp, vp, vp]
        L.orc_digest.argtypes = [ctypes.POINTER(_Desc), u32, vp, u64]
        L.orc_digest.restype = u64
        L.orc_crossing.argtypes = [vp, vp, vp, u32, vp]
        L.orc_run.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(_Result)]
        L.orc_step.argtypes = [ctypes.POINTER(_Desc), u32, u32, vp, vp, u64, u64, vp, vp, vp]
        L.orc_run_from.argtypes = [ctypes.POINTER(_Desc), u32, u64, vp, dbl, ctypes.POINTER(_Result)]
        L.orc_read_checkpoint.argtypes = [ctypes.c_char_p, ctypes.POINTER(_Checkpoint)]
        L.orc_free_checkpoint.argtypes = [ctypes.POINTER(_Checkpoint)]
        L.orc_free_checkpoint.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class Desc:
    """Run description (the same fields as the GPU library's run descriptor)."""

    def __init__(self, L, q, R, beta, theta, seed, resample=RESAMPLE_POISSON, init=INIT_RANDOM,
                 bin_e=1, bin_m=1):
        self.L, self.q, self.R = int(L), int(q), int(R)
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        self.K = len(self.beta)
        self.theta, self.seed = int(theta), int(seed)
        self.resample, self.init = int(resample), int(init)
        self.bin_e, self.bin_m = int(bin_e), int(bin_m)

    @property
    def N(self):
        return self.L * self.L

    def c(self) -> _Desc:
        d = _Desc()
        d.L, d.q, d.R, d.K = self.L, self.q, self.R, self.K
        d.beta = self.beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.theta, d.seed, d.resample, d.init = self.theta, self.seed, self.resample, self.init
        d.bin_e, d.bin_m = self.bin_e, self.bin_m
        self._keep = self.beta
        return d


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def validate(d: Desc) -> int:
    return lib().orc_validate(ctypes.byref(d.c()))


def thresholds(beta: float) -> np.ndarray:
    T = np.zeros(5, dtype=np.uint64)
    lib().orc_thresholds(float(beta), _ptr(T))
    return T


def weights(abs_dbeta: float, Kb: int, N: int):
    W = np.zeros(2 * N + 1, dtype=np.uint64)
    D = lib().orc_weights(float(abs_dbeta), int(Kb), int(N), _ptr(W))
    return W, int(D)


def poisson(lam: float, u: float) -> int:
    return int(lib().orc_poisson(float(lam), float(u)))


def plan(d: Desc):
    R_sched = np.zeros(d.K, dtype=np.uint64)
    cap = np.zeros(1, dtype=np.uint64)
    kb = np.zeros(1, dtype=np.uint32)
    rc = lib().orc_plan(ctypes.byref(d.c()), _ptr(R_sched), _ptr(cap), _ptr(kb))
    if rc:
        raise ValueError(f"orc_plan failed: {rc}")
    return R_sched, int(cap[0]), int(kb[0])


def energy(L: int, spins: np.ndarray) -> int:
    s = np.ascontiguousarray(spins, dtype=np.uint8)
    return int(lib().orc_energy(int(L), _ptr(s)))


def mtilde(L: int, q: int, spins: np.ndarray) -> int:
    s = np.ascontiguousarray(spins, dtype=np.uint8)
    return int(lib().orc_mtilde(int(L), int(q), _ptr(s)))


def init_replica(d: Desc, k: int) -> np.ndarray:
    s = np.zeros(d.N, dtype=np.uint8)
    lib().orc_init_replica(ctypes.byref(d.c()), int(k), _ptr(s))
    return s


def sweep_replica(d: Desc, i: int, k: int, spins: np.ndarray) -> np.ndarray:
    s = np.array(spins, dtype=np.uint8, copy=True)
    lib().orc_sweep_replica(ctypes.byref(d.c()), int(i), int(k), _ptr(s))
    return s


def one_sweep(d: Desc, i: int, t: int, k: int, T: np.ndarray, spins: np.ndarray) -> np.ndarray:
    s = np.array(spins, dtype=np.uint8, copy=True)
    TT = np.ascontiguousarray(T, dtype=np.uint64)
    lib().orc_one_sweep(ctypes.byref(d.c()), int(i), int(t), int(k), _ptr(TT), _ptr(s))
    return s


def resample(d: Desc, i: int, Kb: int, E: np.ndarray, n_new: int):
    E = np.ascontiguousarray(E, dtype=np.int32)
    r = np.zeros(len(E), dtype=np.uint32)
    anc = np.zeros(max(int(n_new), 1), dtype=np.uint32)
    eref = np.zeros(1, dtype=np.int32)
    rc = lib().orc_resample(ctypes.byref(d.c()), int(i), int(Kb), _ptr(E), len(E), int(n_new),
                            _ptr(r), _ptr(anc), _ptr(eref))
    if rc:
        raise ValueError(f"orc_resample failed: {rc}")
    return r, anc[: int(n_new)], int(eref[0])


def lnQ(N: int, dbeta: float, hist: np.ndarray, R_prev: int):
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    eref = np.zeros(1, dtype=np.int32)
    v = lib().orc_lnQ(int(N), float(dbeta), _ptr(h), int(R_prev), _ptr(eref))
    return float(v), int(eref[0])


def step(d: Desc, i: int, Kb: int, spins_old: np.ndarray, E_old: np.ndarray, R_new: int):
    spins_old = np.ascontiguousarray(spins_old, dtype=np.uint8)
    E_old = np.ascontiguousarray(E_old, dtype=np.int32)
    R_prev = len(E_old)
    spins_new = np.zeros((int(R_new), d.N), dtype=np.uint8)
    E_new = np.zeros(int(R_new), dtype=np.int32)
    anc = np.zeros(int(R_new), dtype=np.uint32)
    rc = lib().orc_step(ctypes.byref(d.c()), int(i), int(Kb), _ptr(spins_old), _ptr(E_old),
                        R_prev, int(R_new), _ptr(spins_new), _ptr(E_new), _ptr(anc))
    if rc:
        raise ValueError(f"orc_step failed: {rc}")
    return spins_new, E_new, anc


def fwhm(h: np.ndarray, B: int = 1) -> float:
    """Full width at half maximum of histogram h in bins of B levels (in levels)."""
    hh = np.ascontiguousarray(h, dtype=np.uint32)
    return float(lib().orc_fwhm(_ptr(hh), len(hh), int(B)))


def digest(d: Desc, i: int, spins: np.ndarray) -> int:
    """Digest of the population `spins` [R][N] at step i (orc_digest)."""
    s = np.ascontiguousarray(spins, dtype=np.uint8)
    return int(lib().orc_digest(ctypes.byref(d.c()), int(i), _ptr(s), s.shape[0]))


def width_maxima(beta, width):
    b = np.ascontiguousarray(beta, dtype=np.float64)
    w = np.ascontiguousarray(width, dtype=np.float64)
    i, wm, tm = np.zeros(1, np.uint32), np.zeros(1), np.zeros(1)
    if lib().orc_width_maxima(_ptr(b), _ptr(w), len(b), _ptr(i), _ptr(wm), _ptr(tm)):
        raise ValueError("empty width curve")
    return int(i[0]), float(wm[0]), float(tm[0])


def crossing(beta, f_cool, f_heat):
    b = np.ascontiguousarray(beta, dtype=np.float64)
    c = np.ascontiguousarray(f_cool, dtype=np.float64)
    h = np.ascontiguousarray(f_heat, dtype=np.float64)
    x = np.zeros(1)
    if lib().orc_crossing(_ptr(b), _ptr(c), _ptr(h), len(b), _ptr(x)):
        raise ValueError("no crossing")
    return float(x[0])


def _result(d: Desc, R_final: int, hist, final, magnetisation, widths, digest):
    K, N = d.K, d.N
    out = {
        "R_i": np.zeros(K, dtype=np.uint64), "E_sum": np.zeros(K, dtype=np.int64),
        "E_mean": np.zeros(K), "lnQ": np.zeros(K), "minus_beta_F": np.zeros(K),
    }
    res = _Result()
    for name in ("R_i", "E_sum", "E_mean", "lnQ", "minus_beta_F"):
        setattr(res, name, _ptr(out[name]))
    if magnetisation:
        out["M_mean"] = np.zeros(K)
        out["Mt_sum"] = np.zeros(K, dtype=np.int64)
        out["mhist"] = np.zeros((K, N + 1), dtype=np.uint32)
        res.M_mean = _ptr(out["M_mean"])
        res.Mt_sum = _ptr(out["Mt_sum"])
        res.mhist = _ptr(out["mhist"])
    if digest:
        out["digest"] = np.zeros(K, dtype=np.uint64)
        res.digest = _ptr(out["digest"])
    if widths:
        out["width_e"] = np.zeros(K)
        res.width_e = _ptr(out["width_e"])
        if magnetisation:
            out["width_m"] = np.zeros(K)
            res.width_m = _ptr(out["width_m"])
    if hist:
        out["hist"] = np.zeros((K, 2 * N + 1), dtype=np.uint32)
        res.hist = _ptr(out["hist"])
    if final:
        out["final_spins"] = np.zeros((R_final, N), dtype=np.uint8)
        out["final_E"] = np.zeros(R_final, dtype=np.int32)
        out["last_anc"] = np.zeros(R_final, dtype=np.uint32)
        res.final_spins = _ptr(out["final_spins"])
        res.final_E = _ptr(out["final_E"])
        res.last_anc = _ptr(out["last_anc"])
    return out, res


def run(d: Desc, hist=False, final=False, magnetisation=False, widths=False, digest=False):
    """Whole PA run; returns a dict of numpy arrays."""
    R_sched, R_cap, Kb = plan(d)
    out, res = _result(d, int(R_sched[-1]), hist, final, magnetisation, widths, digest)
    rc = lib().orc_run(ctypes.byref(d.c()), ctypes.byref(res))
    if rc:
        raise ValueError(f"orc_run failed: {rc}")
    out["n_threads"] = res.n_threads
    out["R_sched"], out["R_cap"], out["Kb"] = R_sched, R_cap, Kb
    return out


def run_from(d: Desc, step: int, spins: np.ndarray, minus_beta_F: float, hist=False, final=False,
             magnetisation=False, widths=False, digest=False):
    """The run continued from population `spins` [R][N] at `step` with -beta F
    there (orc_run_from); arrays filled from index `step` on."""
    R_sched, R_cap, Kb = plan(d)
    s = np.ascontiguousarray(spins, dtype=np.uint8)
    out, res = _result(d, int(R_sched[-1]) if step + 1 < d.K else s.shape[0], hist, final,
                       magnetisation, widths, digest)
    rc = lib().orc_run_from(ctypes.byref(d.c()), int(step), s.shape[0], _ptr(s), float(minus_beta_F),
                            ctypes.byref(res))
    if rc:
        raise ValueError(f"orc_run_from failed: {rc}")
    out["n_threads"] = res.n_threads
    return out


def read_checkpoint(path):
    """A checkpoint file of the GPU library (orc_read_checkpoint): its run
    description (Desc), step, population size, -beta F, energy sum and spins."""
    ck = _Checkpoint()
    rc = lib().orc_read_checkpoint(os.fsencode(str(path)), ctypes.byref(ck))
    if rc:
        raise ValueError(f"orc_read_checkpoint failed: {rc}")
    try:
        dd = ck.desc
        K, N = dd.K, dd.L * dd.L
        beta = np.ctypeslib.as_array(ck.beta, shape=(K,)).copy()
        spins = np.ctypeslib.as_array(ck.spins, shape=(ck.R_cur * N,)).copy().reshape(ck.R_cur, N)
        desc = Desc(dd.L, dd.q, dd.R, beta, dd.theta, dd.seed, resample=dd.resample, init=dd.init,
                    bin_e=dd.bin_e, bin_m=dd.bin_m)
        return {"desc": desc, "step": int(ck.step), "R_cur": int(ck.R_cur),
                "minus_beta_F": float(ck.minus_beta_F), "E_sum": int(ck.E_sum), "spins": spins}
    finally:
        lib().orc_free_checkpoint(ctypes.byref(ck))
