"""ctypes front end of the C oracle (``oracle.c``).  Test infrastructure only."""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FP32, FP16, INT8, FP64 = 0, 1, 2, 3
FLIP_MSG, FLIP_LLR = 0, 1
OSD_NONE, OSD_0, OSD_CS = 0, 1, 2
FLAG_CONVERGED, FLAG_OSD, FLAG_OSD_INCONSISTENT = 1, 2, 4


class _Params(ctypes.Structure):
    _fields_ = [
        ("max_iter", ctypes.c_int32),
        ("scale_mode", ctypes.c_int32),
        ("scale", ctypes.c_double),
        ("msg", ctypes.c_int32),
        ("lottery", ctypes.c_int32),
        ("lottery_skip", ctypes.c_int32),
        ("flip", ctypes.c_int32),
        ("osd", ctypes.c_int32),
        ("osd_order", ctypes.c_int32),
        ("early_stop", ctypes.c_int32),
        ("policy", ctypes.c_int32),
        ("fx_int", ctypes.c_int32),
        ("fx_frac", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


@dataclass
class OracleParams:
    max_iter: int = 100
    scale_mode: int = 0          # 0: sigma_i = 1 - 2^-(i+1); 1: constant `scale`
    scale: float = 0.625
    msg: int = FP64
    lottery: bool = True
    lottery_skip: int = 6
    flip: int = FLIP_MSG
    osd: int = OSD_NONE
    osd_order: int = 10
    early_stop: bool = True
    policy: int = 0              # lottery variant: CN rule | VN rule << 4 (see lottery_pick)
    fx_int: int = 3              # INT8 messages are fixed point Int x.y: x integer bits,
    fx_frac: int = 4             # y fraction bits and a sign bit (Int3.4 by default)
    seed: int = 0

    def c(self) -> _Params:
        return _Params(self.max_iter, self.scale_mode, self.scale, self.msg, int(self.lottery),
                       self.lottery_skip, self.flip, self.osd, self.osd_order, int(self.early_stop),
                       self.policy, self.fx_int, self.fx_frac, self.seed & 0xFFFFFFFFFFFFFFFF)


# ORACLE_SANITIZE=1 builds and loads an AddressSanitizer + UndefinedBehaviorSanitizer
# build instead (host code only; the process must preload libasan, see sanitize_check.sh).
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_SAN_LIB = os.path.join(os.path.dirname(_LIB), "liboracle_san.so")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, -O2), or the sanitizer build."""
    lib = _SAN_LIB if _SANITIZE else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp"
        flags = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"] if _SANITIZE else ["-O2"])
        subprocess.check_call(["gcc"] + flags + ["-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-Wall",
                                                 "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, lib)
    return lib


_lib = None


def _get():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        lib.orc_philox4x64_10.argtypes = [P(ctypes.c_uint64), P(ctypes.c_uint64), P(ctypes.c_uint64)]
        lib.orc_store.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.orc_store.restype = ctypes.c_double
        lib.orc_prior_int8.argtypes = [ctypes.c_double]
        lib.orc_prior_int8.restype = ctypes.c_int
        lib.orc_prior_fixed.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int]
        lib.orc_prior_fixed.restype = ctypes.c_int
        lib.orc_decode.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, P(_Params), ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int32]
        lib.orc_decode.restype = ctypes.c_int
        lib.orc_osd.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_osd.restype = ctypes.c_int
        lib.orc_lottery_pick.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p]
        lib.orc_lottery_pick.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _csr(h):
    h = sp.csr_matrix(h)
    h.sort_indices()
    return (h.shape[0], h.shape[1], np.ascontiguousarray(h.indptr, dtype=np.int32),
            np.ascontiguousarray(h.indices, dtype=np.int32))


def philox4x64_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    P = ctypes.POINTER(ctypes.c_uint64)
    _get().orc_philox4x64_10(c.ctypes.data_as(P), k.ctypes.data_as(P), out.ctypes.data_as(P))
    return out


def store(fmt: int, x: float) -> float:
    return _get().orc_store(fmt, float(x))


def prior_int8(p: float) -> int:
    return _get().orc_prior_int8(float(p))


def prior_fixed(p: float, x: int, y: int) -> int:
    """Int x.y prior: 2^y ln((1-p)/p) rounded to nearest even, saturated to +-(2^(x+y) - 1)."""
    return _get().orc_prior_fixed(float(p), int(x), int(y))


def decode(h, prior, params: OracleParams, syndromes: np.ndarray, first_shot_id: int = 0,
           want_llr: bool = False, n_threads: int = 1):
    """Decode packed syndromes [shots, ceil(m/32)] uint32.

    Returns dict(corr [shots, ceil(n/32)] uint32, flags u8, iters i32, llr f64 or None).
    """
    m, n, rp, ci = _csr(h)
    prior = np.broadcast_to(np.asarray(prior, dtype=np.float64), (n,)).copy()
    syn = np.ascontiguousarray(syndromes, dtype=np.uint32)
    shots = syn.shape[0]
    corr = np.zeros((shots, (n + 31) // 32), dtype=np.uint32)
    flags = np.zeros(shots, dtype=np.uint8)
    iters = np.zeros(shots, dtype=np.int32)
    llr = np.zeros((shots, n), dtype=np.float64) if want_llr else None
    prm = params.c()
    rc = _get().orc_decode(m, n, _ptr(rp), _ptr(ci), _ptr(prior), ctypes.byref(prm), shots,
                           first_shot_id & 0xFFFFFFFFFFFFFFFF, _ptr(syn), _ptr(corr), _ptr(flags),
                           _ptr(iters), _ptr(llr), n_threads)
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return dict(corr=corr, flags=flags, iters=iters, llr=llr)


def osd(h, llr: np.ndarray, syndrome: np.ndarray, mode: int = OSD_0, order: int = 10):
    """OSD of one shot from a given lambda vector.  Returns (corr words, flag)."""
    m, n, rp, ci = _csr(h)
    lam = np.ascontiguousarray(llr, dtype=np.float64)
    syn = np.ascontiguousarray(syndrome, dtype=np.uint32)
    corr = np.zeros((n + 31) // 32, dtype=np.uint32)
    flag = np.zeros(1, dtype=np.uint8)
    rc = _get().orc_osd(m, n, _ptr(rp), _ptr(ci), mode, order, _ptr(lam), _ptr(syn), _ptr(corr), _ptr(flag))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return corr, int(flag[0])


# Lottery design-space rules (Sec. III-B, Table I); policy = CN rule | VN rule << 4.
CN_RANDOM, CN_WORST = 0, 1
VN_PROPOSED, VN_Q_FIRST, VN_UNRELIABLE, VN_RANDOM = 0, 1, 2, 3


def policy_code(cn: int = CN_RANDOM, vn: int = VN_PROPOSED) -> int:
    return cn | (vn << 4)


def lottery_pick(h, seed: int, shot_id: int, i: int, s, sprev, lam, is_int8: bool = False,
                 policy: int = 0, ehat=None) -> int:
    """Algorithm 3's selection on explicit state; returns v* (or -1 if no check is unsatisfied).

    ehat (n bytes, the current hard decision) is read only by the worst-check rule."""
    m, n, rp, ci = _csr(h)
    s8 = np.ascontiguousarray(s, dtype=np.uint8)
    p8 = np.ascontiguousarray(sprev, dtype=np.uint8)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    e8 = np.ascontiguousarray(ehat if ehat is not None else np.zeros(n), dtype=np.uint8)
    return _get().orc_lottery_pick(m, n, _ptr(rp), _ptr(ci), seed, shot_id, i, _ptr(s8), _ptr(p8), _ptr(lam),
                                   int(is_int8), int(policy), _ptr(e8))
