"""ctypes front end of the FP64 CPU oracle (``bp4_oracle.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline leg import this module.  It shares no code with the GPU library.

Paper: "Improved Belief Propagation Decoding Algorithms for Surface Codes"
(arXiv 2407.11523).  Functions cite the section / equation they follow.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bp4_oracle.c")
# BP4_ORACLE_SANITIZE=1: the AddressSanitizer + UndefinedBehaviorSanitizer build (the
# process must preload gcc's libasan and libubsan)
_SANITIZE = os.environ.get("BP4_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g"]

BP, MOMENTUM, ADAGRAD, EWAINIT, AEWA = 0, 1, 2, 3, 4
VARIANTS = {"bp": BP, "momentum": MOMENTUM, "adagrad": ADAGRAD, "ewainit": EWAINIT, "aewa": AEWA}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE semantics, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra"] + (SANITIZE_FLAGS if _SANITIZE else []) +
                              ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("stop_on_syndrome", ctypes.c_int32), ("adagrad_g_from_t1", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("gamma", ctypes.c_double),
                ("eps", ctypes.c_double), ("clamp", ctypes.c_double), ("alpha_t", ctypes.c_void_p),
                ("alpha_last", ctypes.c_double), ("alpha_steps", ctypes.c_int32), ("serial", ctypes.c_int32),
                ("gamma_t", ctypes.c_void_p)]


class _Outputs(ctypes.Structure):
    _fields_ = [("q_out", ctypes.c_void_p), ("mvc_out", ctypes.c_void_p),
                ("mcv_out", ctypes.c_void_p), ("q_trace", ctypes.c_void_p),
                ("m_trace", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.or_decode.restype = ctypes.c_int
        L.or_decode.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p, ctypes.POINTER(_Params),
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_double), u8p, u8p, u8p,
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_Outputs),
                                ctypes.c_int]
        L.or_sample.restype = ctypes.c_int
        L.or_sample.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p, ctypes.c_int64,
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint64,
                                ctypes.c_uint64, u8p, u8p, ctypes.c_int]
        L.or_bookkeep.restype = ctypes.c_int
        L.or_bookkeep.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p, ctypes.c_int, u8p, u8p,
                                  ctypes.c_int64, u8p, u8p, u8p, ctypes.POINTER(ctypes.c_int64)]
        L.or_philox4x64_10.restype = None
        L.or_philox4x64_10.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 3
        L.or_lambda.restype = ctypes.c_double
        L.or_lambda.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.or_phi.restype = ctypes.c_double
        L.or_phi.argtypes = [ctypes.c_double]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


@dataclass
class Params:
    """Decoder hyperparameters (section III; defaults are the readings in the design notes)."""
    variant: str = "bp"
    max_iter: int = 100
    stop_on_syndrome: bool = True
    adagrad_g_from_t1: bool = False
    alpha: float = 1.0
    gamma: float = 0.0
    eps: float = 1e-8
    clamp: float = 30.0
    alpha_t: Optional[np.ndarray] = None   # per-iteration EWAInit discount or Momentum step, entry t-1 at t
    gamma_t: Optional[np.ndarray] = None   # per-iteration Momentum decay, entry t-1 at iteration t
    alpha_last: float = 0.0                # AEWA: discount of the last attempt (alpha is the first)
    alpha_steps: int = 11                  # AEWA: number of attempts
    serial: bool = False                   # serial schedule (Alg. 1) instead of flooding (Alg. 2)

    def c(self) -> _Params:
        cp = _Params(VARIANTS[self.variant], int(self.max_iter), int(bool(self.stop_on_syndrome)),
                     int(bool(self.adagrad_g_from_t1)), float(self.alpha), float(self.gamma),
                     float(self.eps), float(self.clamp), None, float(self.alpha_last), int(self.alpha_steps),
                     int(bool(self.serial)))
        keep = []
        for name in ("alpha_t", "gamma_t"):
            v = getattr(self, name)
            if v is not None:
                a = np.ascontiguousarray(v, dtype=np.float64)
                if a.shape != (self.max_iter,):
                    raise ValueError(f"{name} needs one entry per iteration")
                keep.append(a)
                setattr(cp, name, a.ctypes.data)
        cp._keep = keep                       # keeps the buffers alive as long as the struct
        return cp


# ---------------------------------------------------------------------------
# Priors (section II-B1) and statistics (section IV)
# ---------------------------------------------------------------------------

def prior_llr(probs: np.ndarray) -> np.ndarray:
    """Pi_{v,W} = ln(p_v^I / p_v^W) for W in (X, Y, Z), p^I = 1 - p^X - p^Y - p^Z.

    Section II-B1 prints ln((1-p)/p) for the vector p_v; lambda is only a
    commutation LLR when e^{-Pi_W} = p_W / p_I, which fixes this reading.
    """
    probs = np.asarray(probs, dtype=np.float64)
    pi = 1.0 - probs.sum(axis=1, keepdims=True)
    return np.log(pi) - np.log(probs)


def wilson_ci(k: int, n: int, z: float = 1.959963984540054):
    """Wilson score interval for a binomial proportion k / n."""
    if n == 0:
        return (0.0, 1.0)
    ph = k / n
    den = 1 + z * z / n
    ctr = (ph + z * z / (2 * n)) / den
    half = z * math.sqrt(ph * (1 - ph) / n + z * z / (4 * n * n)) / den
    return (max(0.0, ctr - half), min(1.0, ctr + half))


# ---------------------------------------------------------------------------
# Wrappers
# ---------------------------------------------------------------------------

def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_p(c, ctypes.c_uint64), _p(k, ctypes.c_uint64), _p(out, ctypes.c_uint64))
    return out


def lam(pauli: int, l3) -> float:
    return lib().or_lambda(int(pauli), float(l3[0]), float(l3[1]), float(l3[2]))


def phi(x: float) -> float:
    return lib().or_phi(float(x))


def sample(hx, hz, shots: int, thr, seed: int, stream: int = 0, shot0: int = 0, nthreads: int = 0):
    """Errors [shots][n] (Pauli codes) and syndromes [shots][m] from the oracle's sampler."""
    hx, hz = _u8(hx), _u8(hz)
    m, n = hx.shape
    t = np.ascontiguousarray(thr, dtype=np.uint32)
    err = np.zeros((shots, n), np.uint8)
    syn = np.zeros((shots, m), np.uint8)
    rc = lib().or_sample(m, n, _p(hx, ctypes.c_uint8), _p(hz, ctypes.c_uint8), shots, shot0,
                         _p(t, ctypes.c_uint32), seed & (2 ** 64 - 1), stream & (2 ** 64 - 1),
                         _p(err, ctypes.c_uint8), _p(syn, ctypes.c_uint8), nthreads)
    if rc:
        raise ValueError("or_sample rejected its arguments")
    return err, syn


def decode(hx, hz, params: Params, pi0, synd, *, want_q=False, want_msgs=False,
           want_trace=False, nthreads: int = 0):
    """Decode syndromes [shots][m] with prior LLRs pi0 [n][3]; returns a dict."""
    hx, hz = _u8(hx), _u8(hz)
    m, n = hx.shape
    synd = _u8(synd).reshape(-1, m)
    shots = synd.shape[0]
    pi0 = np.ascontiguousarray(pi0, dtype=np.float64).reshape(n, 3)
    nnz = int(np.count_nonzero(hx | hz))
    est = np.zeros((shots, n), np.uint8)
    conv = np.zeros(shots, np.uint8)
    iters = np.zeros(shots, np.int32)
    o = _Outputs()
    res = {}
    if want_q:
        res["q"] = np.zeros((shots, n, 3))
        o.q_out = res["q"].ctypes.data
    if want_msgs:
        res["mvc"] = np.zeros((shots, nnz))
        res["mcv"] = np.zeros((shots, nnz))
        o.mvc_out = res["mvc"].ctypes.data
        o.mcv_out = res["mcv"].ctypes.data
    if want_trace:
        res["q_trace"] = np.zeros((shots, params.max_iter, n, 3))
        res["m_trace"] = np.zeros((shots, params.max_iter, n, 3))
        o.q_trace = res["q_trace"].ctypes.data
        o.m_trace = res["m_trace"].ctypes.data
    cp = params.c()
    rc = lib().or_decode(m, n, _p(hx, ctypes.c_uint8), _p(hz, ctypes.c_uint8), ctypes.byref(cp),
                         shots, _p(pi0, ctypes.c_double), _p(synd, ctypes.c_uint8),
                         _p(est, ctypes.c_uint8), _p(conv, ctypes.c_uint8),
                         _p(iters, ctypes.c_int32), ctypes.byref(o), nthreads)
    if rc:
        raise ValueError("or_decode rejected its arguments")
    res.update(est=est, conv=conv, iters=iters)
    return res


def bookkeep(hx, hz, lx, lz, err, est):
    """Per-shot failure kind (0 ok, 1 detected, 2 undetected) and the three counts."""
    hx, hz, lx, lz = _u8(hx), _u8(hz), _u8(lx), _u8(lz)
    m, n = hx.shape
    err = _u8(err).reshape(-1, n)
    est = _u8(est).reshape(-1, n)
    shots = err.shape[0]
    fail = np.zeros(shots, np.uint8)
    counts = np.zeros(3, np.int64)
    nlog = lx.shape[0]
    rc = lib().or_bookkeep(m, n, _p(hx, ctypes.c_uint8), _p(hz, ctypes.c_uint8), nlog,
                           _p(lx, ctypes.c_uint8), _p(lz, ctypes.c_uint8), shots,
                           _p(err, ctypes.c_uint8), _p(est, ctypes.c_uint8),
                           _p(fail, ctypes.c_uint8), _p(counts, ctypes.c_int64))
    if rc:
        raise ValueError("or_bookkeep rejected its arguments")
    return fail, counts
