"""Seeded synthetic SMILES generator (input data only; no codec arithmetic).

The workloads stand in for the paper's SMILES datasets (GDB-17, MEDIATE,
EXSCALATE, MIXED; Sec. V-A), which are not available.  Every preset is a
grammar-driven generator with a per-line SplitMix64 counter stream, so line k
of a seed is the same bytes whatever range it is generated in.

Presets (lengths exclude the newline):
  small   uniform length 20..80                          (10k-line parity case)
  bulk    log-normal, median 45, sigma 0.5, clip 10..120  (10M-line bulk case)
  uneven  bulk mixed with 10% long lines, uniform 200..1000, deep branches
          and many simultaneously open rings so %nn labels occur
  test    uniform 1..80, with [NH3+] (digits inside brackets)
  long    long mode only, uniform 200..1000
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsmilesgen.so")


class Params(ctypes.Structure):
    _fields_ = [
        ("dist", ctypes.c_int32),
        ("lo", ctypes.c_int32),
        ("hi", ctypes.c_int32),
        ("median", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("long_frac", ctypes.c_double),
        ("long_lo", ctypes.c_int32),
        ("long_hi", ctypes.c_int32),
        ("bracket_digits", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


PRESETS = {
    "small": dict(dist=0, lo=20, hi=80),
    "bulk": dict(dist=1, lo=10, hi=120, median=45.0, sigma=0.5),
    "uneven": dict(dist=1, lo=10, hi=120, median=45.0, sigma=0.5,
                   long_frac=0.10, long_lo=200, long_hi=1000),
    "test": dict(dist=0, lo=1, hi=80, bracket_digits=1),
    "long": dict(dist=0, lo=200, hi=1000, long_frac=1.0, long_lo=200, long_hi=1000),
}


def build(force=False):
    """Compile libsmilesgen.so in place (plain C, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(src):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", src, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.smg_generate.restype = ctypes.c_int64
        lib.smg_generate.argtypes = [ctypes.POINTER(Params), ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


def params(preset):
    p = Params()
    for k, v in PRESETS[preset].items():
        setattr(p, k, v)
    return p


def generate(preset, seed, n, first=0, threads=0):
    """Return (buf uint8[N], off uint64[n+1]) for lines [first, first+n)."""
    lib = _load()
    p = params(preset)
    off = np.zeros(n + 1, dtype=np.uint64)
    total = lib.smg_generate(ctypes.byref(p), seed, first, n, None, 0,
                             off.ctypes.data_as(ctypes.c_void_p), threads)
    buf = np.empty(max(total, 1), dtype=np.uint8)
    got = lib.smg_generate(ctypes.byref(p), seed, first, n, buf.ctypes.data_as(ctypes.c_void_p),
                           buf.size, off.ctypes.data_as(ctypes.c_void_p), threads)
    if got != total:
        raise RuntimeError("smilesgen: generation failed")
    return buf[:total], off


def lines(preset, seed, n, first=0):
    """Convenience: list of bytes objects (no newline)."""
    buf, off = generate(preset, seed, n, first)
    b = buf.tobytes()
    return [b[int(off[k]):int(off[k + 1]) - 1] for k in range(n)]
