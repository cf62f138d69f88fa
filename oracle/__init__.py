"""oracle - TEST INFRASTRUCTURE ONLY.

Plain single-threaded CPU reference of the ZSMILES codec (zs_oracle.c), used
by the test suite, the smoke check and the benchmark's CPU-baseline leg.  The
product package never imports it.  It shares no code with the GPU path: it
has its own dictionary-file reader, its own build, its own C source.

brute.py next to it holds the independent checks that pin this oracle
(exhaustive parses, an explicit Dijkstra, a second ring-ID formulation).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libzsoracle.so")

OK, EINVAL, ENOSPC, ECORRUPT = 0, -1, -2, -3
F_PREPROCESS = 1
LMAX_CAP = 16


def build(force=False):
    """Compile the oracle with gcc -O2, no intrinsics, no threads."""
    srcs = [os.path.join(_HERE, f) for f in ("zs_oracle.c", "train_dict.c")]
    if not force and os.path.exists(_SO) and all(os.path.getmtime(_SO) >= os.path.getmtime(s) for s in srcs):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC"] + srcs + ["-o", tmp])
    os.replace(tmp, _SO)
    return _SO


_lib = None
_u8p = ctypes.POINTER(ctypes.c_uint8)
_vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.zo_sizeof_dict.restype = ctypes.c_uint64
        L.zo_dict_init.argtypes = [_vp, _vp, _vp]
        L.zo_dict_init.restype = ctypes.c_int
        L.zo_preprocess.argtypes = [_vp, ctypes.c_int64, _vp]
        L.zo_preprocess.restype = ctypes.c_int64
        L.zo_compress_line.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_uint32, _vp]
        L.zo_compress_line.restype = ctypes.c_int64
        L.zo_decompress_line.argtypes = [_vp, _vp, ctypes.c_int64, _vp]
        L.zo_decompress_line.restype = ctypes.c_int64
        L.zo_compress.argtypes = [_vp, _vp, ctypes.c_uint64, _vp, ctypes.c_uint64, ctypes.c_uint32,
                                  _vp, ctypes.c_uint64, _vp, _vp]
        L.zo_compress.restype = ctypes.c_int
        L.zo_decompress.argtypes = [_vp, _vp, ctypes.c_uint64, _vp, ctypes.c_uint64,
                                    _vp, ctypes.c_uint64, _vp, _vp]
        L.zo_decompress.restype = ctypes.c_int
        L.zo_decompress_lines.argtypes = [_vp, _vp, ctypes.c_uint64, _vp, ctypes.c_uint64, _vp,
                                          ctypes.c_uint64, _vp, ctypes.c_uint64, _vp, _vp]
        L.zo_decompress_lines.restype = ctypes.c_int
        L.zo_index_lines.argtypes = [_vp, ctypes.c_uint64, _vp, ctypes.c_uint64]
        L.zo_index_lines.restype = ctypes.c_int64
        L.zo_preprocess_buffer.argtypes = [_vp, _vp, ctypes.c_uint64, _vp, _vp]
        L.zo_preprocess_buffer.restype = None
        L.zo_postprocess.argtypes = [_vp, ctypes.c_int64, _vp]
        L.zo_postprocess.restype = ctypes.c_int64
        L.zo_postprocess_buffer.argtypes = [_vp, _vp, ctypes.c_uint64, _vp, _vp]
        L.zo_postprocess_buffer.restype = None
        L.zo_train_dict.argtypes = [_vp, _vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, _vp, _vp]
        L.zo_train_dict.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_vp) if a is not None and a.size else None


def _bytes_arr(b):
    a = np.frombuffer(bytes(b), dtype=np.uint8).copy()
    if a.size == 0:
        a = np.zeros(1, dtype=np.uint8)[:0]
    return a


class Dict:
    """A code table: code byte -> expansion (Sec. IV-B/IV-C)."""

    def __init__(self, entries):
        self.entries = {int(k): bytes(v) for k, v in entries.items()}
        self.len = np.zeros(256, dtype=np.uint8)
        self.exp = np.zeros((256, LMAX_CAP), dtype=np.uint8)
        for c, e in self.entries.items():
            if 0 <= c < 256 and 1 <= len(e) <= LMAX_CAP:
                self.len[c] = len(e)
                self.exp[c, :len(e)] = np.frombuffer(e, dtype=np.uint8)
            else:
                self.len[c % 256] = 255  # forces EINVAL below
        lib = _load()
        self._buf = ctypes.create_string_buffer(int(lib.zo_sizeof_dict()))
        self.status = lib.zo_dict_init(self._buf, _ptr(self.len), _ptr(self.exp))
        self.lmax = max((len(e) for e in self.entries.values()), default=0)

    @property
    def valid(self):
        return self.status == OK

    def _h(self):
        if not self.valid:
            raise ValueError("invalid dictionary")
        return self._buf

    @classmethod
    def load(cls, path):
        """Read a .zsd file: a 'ZSD1' header line, then '<hex code> <expansion>' lines."""
        with open(path, "rb") as f:
            data = f.read()
        rows = data.split(b"\n")
        if not rows or not rows[0].startswith(b"ZSD1"):
            raise ValueError("not a ZSD1 dictionary: %s" % path)
        entries = {}
        for row in rows[1:]:
            if not row:
                continue
            code, exp = row.split(b" ", 1)
            entries[int(code, 16)] = exp
        return cls(entries)


def preprocess(line):
    """Ring-ID pre-processing of one line (Sec. IV-A)."""
    lib = _load()
    x = _bytes_arr(line)
    y = np.zeros(3 * x.size + 1, dtype=np.uint8)
    m = lib.zo_preprocess(_ptr(x), x.size, _ptr(y))
    return y[:m].tobytes()


def preprocess_buffer(buf, off):
    """Pre-process every line of a buffer; returns (bytes, offsets)."""
    lib = _load()
    buf, off = _as_u8(buf), _as_u64(off)
    n = off.size - 1
    out = np.zeros(3 * buf.size + n + 1, dtype=np.uint8)
    out_off = np.zeros(n + 1, dtype=np.uint64)
    lib.zo_preprocess_buffer(_ptr(buf), _ptr(off), n, out.ctypes.data_as(_vp), _ptr(out_off))
    return out[:int(out_off[n])], out_off


def postprocess(line):
    """Post-processing of one decompressed line: ring labels renumbered in the writers'
    convention (our definition; the paper names the step, Sec. IV-D, without defining it)."""
    lib = _load()
    x = _bytes_arr(line)
    y = np.zeros(3 * x.size + 1, dtype=np.uint8)
    m = lib.zo_postprocess(_ptr(x), x.size, _ptr(y))
    return y[:m].tobytes()


def postprocess_buffer(buf, off):
    """Post-process every line of a buffer; returns (bytes, offsets)."""
    lib = _load()
    buf, off = _as_u8(buf), _as_u64(off)
    n = off.size - 1
    out = np.zeros(3 * buf.size + n + 1, dtype=np.uint8)
    out_off = np.zeros(n + 1, dtype=np.uint64)
    lib.zo_postprocess_buffer(_ptr(buf), _ptr(off), n, out.ctypes.data_as(_vp), _ptr(out_off))
    return out[:int(out_off[n])], out_off


def compress_line(d, line, preprocess=True):
    lib = _load()
    x = _bytes_arr(line)
    y = np.zeros(6 * x.size + 1, dtype=np.uint8)
    n = lib.zo_compress_line(d._h(), _ptr(x), x.size, F_PREPROCESS if preprocess else 0, _ptr(y))
    return y[:n].tobytes()


def decompress_line(d, c):
    """Returns the expansion, or None for corrupt input."""
    lib = _load()
    x = _bytes_arr(c)
    y = np.zeros(max(d.lmax, 1) * x.size + 1, dtype=np.uint8)
    n = lib.zo_decompress_line(d._h(), _ptr(x), x.size, _ptr(y))
    return None if n < 0 else y[:n].tobytes()


def _as_u8(buf):
    return np.ascontiguousarray(np.asarray(buf, dtype=np.uint8))


def _as_u64(off):
    return np.ascontiguousarray(np.asarray(off, dtype=np.uint64))


def compress(d, buf, off, preprocess=True, out_cap=None, size_only=False):
    """Compress a buffer of lines.  Returns (code, first_bad, out, out_off)."""
    lib = _load()
    buf, off = _as_u8(buf), _as_u64(off)
    n = off.size - 1
    out_off = np.zeros(n + 1, dtype=np.uint64)
    fb = ctypes.c_int64(-1)
    flags = F_PREPROCESS if preprocess else 0
    if out_cap is None:
        lib.zo_compress(d._h(), _ptr(buf), buf.size, _ptr(off), n, flags, None, 0,
                        _ptr(out_off), ctypes.byref(fb))
        out_cap = int(out_off[n])
    if size_only:
        code = lib.zo_compress(d._h(), _ptr(buf), buf.size, _ptr(off), n, flags, None, 0,
                               _ptr(out_off), ctypes.byref(fb))
        return code, fb.value, None, out_off
    out = np.zeros(max(out_cap, 1), dtype=np.uint8)
    code = lib.zo_compress(d._h(), _ptr(buf), buf.size, _ptr(off), n, flags, out.ctypes.data_as(_vp),
                           out_cap, _ptr(out_off), ctypes.byref(fb))
    return code, fb.value, out[:min(out_cap, int(out_off[n]))], out_off


def decompress(d, buf, off, out_cap=None, size_only=False):
    lib = _load()
    buf, off = _as_u8(buf), _as_u64(off)
    n = off.size - 1
    out_off = np.zeros(n + 1, dtype=np.uint64)
    fb = ctypes.c_int64(-1)
    if out_cap is None:
        lib.zo_decompress(d._h(), _ptr(buf), buf.size, _ptr(off), n, None, 0, _ptr(out_off), ctypes.byref(fb))
        out_cap = int(out_off[n])
    if size_only:
        code = lib.zo_decompress(d._h(), _ptr(buf), buf.size, _ptr(off), n, None, 0, _ptr(out_off),
                                 ctypes.byref(fb))
        return code, fb.value, None, out_off
    out = np.zeros(max(out_cap, 1), dtype=np.uint8)
    code = lib.zo_decompress(d._h(), _ptr(buf), buf.size, _ptr(off), n, out.ctypes.data_as(_vp), out_cap,
                             _ptr(out_off), ctypes.byref(fb))
    return code, fb.value, out[:min(out_cap, int(out_off[n]))], out_off


def decompress_lines(d, buf, off, ids, out_cap=None):
    lib = _load()
    buf, off, ids = _as_u8(buf), _as_u64(off), _as_u64(ids)
    n = off.size - 1
    k = ids.size
    out_off = np.zeros(k + 1, dtype=np.uint64)
    fb = ctypes.c_int64(-1)
    if out_cap is None:
        lib.zo_decompress_lines(d._h(), _ptr(buf), buf.size, _ptr(off), n, _ptr(ids), k, None, 0,
                                _ptr(out_off), ctypes.byref(fb))
        out_cap = int(out_off[k])
    out = np.zeros(max(out_cap, 1), dtype=np.uint8)
    code = lib.zo_decompress_lines(d._h(), _ptr(buf), buf.size, _ptr(off), n, _ptr(ids), k,
                                   out.ctypes.data_as(_vp), out_cap, _ptr(out_off), ctypes.byref(fb))
    return code, fb.value, out[:min(out_cap, int(out_off[k]))], out_off


def index_lines(buf):
    lib = _load()
    buf = _as_u8(buf)
    n = lib.zo_index_lines(_ptr(buf), buf.size, None, 0)
    off = np.zeros(n + 1, dtype=np.uint64)
    lib.zo_index_lines(_ptr(buf), buf.size, _ptr(off), n + 1)
    return off


def join_lines(lines):
    """bytes lines -> (buf, off) with a newline after every line."""
    data = b"".join(l + b"\n" for l in lines)
    off = np.zeros(len(lines) + 1, dtype=np.uint64)
    acc = 0
    for i, l in enumerate(lines):
        acc += len(l) + 1
        off[i + 1] = acc
    return np.frombuffer(data, dtype=np.uint8).copy() if data else np.zeros(0, np.uint8), off


def split_lines(buf, off):
    b = np.asarray(buf, dtype=np.uint8).tobytes()
    return [b[int(off[k]):int(off[k + 1]) - 1] for k in range(len(off) - 1)]


def train_patterns(buf, off, T, lmin=2, lmax=8, preprocess=True):
    """Algorithm 1 (Sec. IV-C): the T patterns of highest Eq. (1) rank, in selection order."""
    lib = _load()
    buf, off = _as_u8(buf), _as_u64(off)
    pat = np.zeros((max(T, 1), 16), dtype=np.uint8)
    plen = np.zeros(max(T, 1), dtype=np.uint8)
    got = lib.zo_train_dict(_ptr(buf), _ptr(off), off.size - 1, 1 if preprocess else 0, lmin, lmax, T,
                            _ptr(pat), _ptr(plen))
    if got < 0:
        raise RuntimeError("training failed (%d)" % got)
    return [pat[i, :plen[i]].tobytes() for i in range(got)]
