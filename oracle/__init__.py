"""CPU oracle for quantized layered BP decoding of LDPC syndromes (arXiv:1903.10107).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package. The product library never calls it;
the two share no code. The arithmetic lives in ``ldpc_oracle.c`` (plain C);
this module only marshals numpy arrays into it.

Every function here follows the paper: Alg. 1 (tau), Eqs. 4 and 7 (box-plus
folds), Eqs. 8 and 9 with Alg. 2 (variable node), Sec. 2 (layered schedule and
stopping rule). The C file's header states the integer conventions it fixes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

RULE_RCBP_FB = 0
RULE_RCBP_EQ7 = 1
RULE_MINSUM = 2

_lib = None


class _Params(C.Structure):
    _fields_ = [("msg_max", C.c_int32), ("e_max", C.c_int32), ("acc_bits", C.c_int32),
                ("cn_rule", C.c_int32), ("offset", C.c_void_p), ("offset_iters", C.c_int32),
                ("freeze", C.c_int32)]


def lib():
    """The oracle library, compiled with gcc on first use if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.oracle_tau.restype = C.c_int
        L.oracle_tau.argtypes = [C.c_int, C.c_int, C.c_int]
        for name in ("oracle_cn_rcbp_fb", "oracle_cn_rcbp_eq7", "oracle_cn_minsum"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.oracle_vn_update.restype = C.c_int
        L.oracle_vn_update.argtypes = [C.c_int] * 5
        L.oracle_decode.restype = C.c_int
        L.oracle_decode.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(_Params),
                                    C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.oracle_bp_fp64_decode.restype = C.c_int
        L.oracle_bp_fp64_decode.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                            C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.oracle_max_threads.restype = C.c_int
        for name in ("oracle_beta",):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double, C.c_double]
        for name in ("oracle_mag_tanh", "oracle_mag_phi", "oracle_mag_fold"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_void_p, C.c_int, C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None else None


# --- single-operation entry points (Alg. 1, Eq. 4/7, Alg. 2) ---------------

def tau(p: int, q: int, msg_max: int = 63) -> int:
    """Alg. 1: the integer table tau(p, q)."""
    return lib().oracle_tau(int(p), int(q), int(msg_max))


def tau_table(size: int = 64, msg_max: int = 63) -> np.ndarray:
    t = np.empty((size, size), dtype=np.int32)
    for p in range(size):
        for q in range(size):
            t[p, q] = tau(p, q, msg_max)
    return t


def cn_magnitudes(p, rule: int = RULE_RCBP_FB, msg_max: int = 63) -> np.ndarray:
    """Magnitudes of the CN->VN messages of one check row, given the clipped
    input magnitudes p (one per edge, in edge order)."""
    a = np.ascontiguousarray(p, dtype=np.int32)
    out = np.zeros_like(a)
    fn = {RULE_RCBP_FB: lib().oracle_cn_rcbp_fb, RULE_RCBP_EQ7: lib().oracle_cn_rcbp_eq7,
          RULE_MINSUM: lib().oracle_cn_minsum}[rule]
    fn(_ptr(a), len(a), int(msg_max), _ptr(out))
    return out


def vn_update(e: int, v: int, lnew: int, e_max: int = 127, freeze: bool = True) -> int:
    """Eq. 9 with the saturation rule of Alg. 2."""
    return lib().oracle_vn_update(int(e), int(v), int(lnew), int(e_max), int(bool(freeze)))


# --- whole decoder ----------------------------------------------------------

def decode(base, z: int, syn, llr, max_iter: int, *, msg_max: int = 63, e_max: int | None = None,
           acc_bits: int = 8, cn_rule: int = RULE_RCBP_FB, offsets=None, freeze: bool = True,
           want_state: bool = False, n_threads: int = 0):
    """Integer layered decoder over a batch. Returns a dict with bits (packed),
    conv, iters and, with want_state, L [F, n_blocks, Z] int8 and E [F, n] int16."""
    base = np.ascontiguousarray(base, dtype=np.int32)
    mb, nb = base.shape
    n, m = nb * z, mb * z
    nblk = int((base >= 0).sum())
    syn = np.ascontiguousarray(syn, dtype=np.uint8).reshape(-1, (m + 7) // 8)
    llr = np.ascontiguousarray(llr, dtype=np.int8).reshape(-1, n)
    F = llr.shape[0]
    if syn.shape[0] != F:
        raise ValueError("syndrome and llr batch sizes differ")
    if e_max is None:
        e_max = 32767 if acc_bits == 16 else 127
    off = None
    off_iters = 0
    if offsets is not None:
        off = np.ascontiguousarray(offsets, dtype=np.int8).reshape(-1, nblk)
        off_iters = off.shape[0]
    prm = _Params(msg_max, e_max, acc_bits, cn_rule, _ptr(off), off_iters, int(bool(freeze)))
    bits = np.zeros((F, (n + 7) // 8), dtype=np.uint8)
    conv = np.zeros(F, dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    Lo = np.zeros((F, nblk, z), dtype=np.int8) if want_state else None
    Eo = np.zeros((F, n), dtype=np.int16) if want_state else None
    rc = lib().oracle_decode(_ptr(base), mb, nb, z, C.byref(prm), _ptr(syn), _ptr(llr), F, int(max_iter),
                             _ptr(bits), _ptr(conv), _ptr(iters), _ptr(Lo), _ptr(Eo), int(n_threads))
    if rc != 0:
        raise ValueError("oracle_decode rejected its arguments")
    out = {"bits": bits, "conv": conv, "iters": iters}
    if want_state:
        out["L"], out["E"] = Lo, Eo
    return out


def bp_fp64_decode(base, z: int, syn, llr_f, max_iter: int, n_threads: int = 0):
    """FP64 layered BP with the exact box-plus (statistics only)."""
    base = np.ascontiguousarray(base, dtype=np.int32)
    mb, nb = base.shape
    n, m = nb * z, mb * z
    syn = np.ascontiguousarray(syn, dtype=np.uint8).reshape(-1, (m + 7) // 8)
    llr_f = np.ascontiguousarray(llr_f, dtype=np.float64).reshape(-1, n)
    F = llr_f.shape[0]
    bits = np.zeros((F, (n + 7) // 8), dtype=np.uint8)
    conv = np.zeros(F, dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    rc = lib().oracle_bp_fp64_decode(_ptr(base), mb, nb, z, _ptr(syn), _ptr(llr_f), F, int(max_iter),
                                     _ptr(bits), _ptr(conv), _ptr(iters), int(n_threads))
    if rc != 0:
        raise ValueError("oracle_bp_fp64_decode rejected its arguments")
    return {"bits": bits, "conv": conv, "iters": iters}


def beta(a: float, b: float) -> float:
    """Eq. 6 on magnitudes."""
    return lib().oracle_beta(float(a), float(b))


def _mag(fn, a, k):
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return fn(_ptr(arr), len(arr), int(k))


def mag_tanh(a, k):
    """Eq. 2 for the output to edge k."""
    return _mag(lib().oracle_mag_tanh, a, k)


def mag_phi(a, k):
    """Eq. 3 for the output to edge k."""
    return _mag(lib().oracle_mag_phi, a, k)


def mag_fold(a, k):
    """Eq. 7 for the output to edge k."""
    return _mag(lib().oracle_mag_fold, a, k)


def max_threads() -> int:
    return lib().oracle_max_threads()
