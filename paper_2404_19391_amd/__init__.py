"""ZSMILES codec on MI355X: Python binding of libzsmiles.so (include/zsmiles.h).

Argument marshalling only: every step of compression and decompression runs in
the HIP kernels of the library.  PyTorch provides device memory and the
stream (torch.cuda.current_stream()); tensors are uint8 for bytes and int64
for offsets, read as uint64 by the library.

    d = Dict.load(default_dict_path())
    c, c_off = compress(d, raw_u8, raw_off)          # Sec. IV-A + IV-D-1
    r, r_off = decompress(d, c, c_off)               # Sec. IV-D-2
    s, s_off = decompress_lines(d, c, c_off, ids)    # random access (Sec. I)

The library must be built (python -m paper_2404_19391_amd._build); without it
every call raises - there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libzsmiles.so")

OK, EINVAL, ENOSPC, ECORRUPT, EDEVICE, ENOMEM = 0, -1, -2, -3, -4, -5
F_PREPROCESS = 1
LMAX_CAP = 16
MAX_LINE = 4096
OP_COMPRESS, OP_DECOMPRESS, OP_DECOMPRESS_LINES, OP_INDEX = 1, 2, 3, 4

_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_lib = None


class ZsError(RuntimeError):
    def __init__(self, code, first_bad=-1, what=""):
        self.code = code
        self.first_bad = first_bad
        super().__init__("%s: %s (code %d, first bad %d)" % (what, status_str(code), code, first_bad))


def default_dict_path():
    return os.path.join(_PKG, "data", "default.zsd")


MAX_BINS = 8


class BinConfig(ctypes.Structure):
    """zs_bin_config: bins by raw line length (ascending edges), lines per tile and line-buffer layout
    per bin (large_lds: 0 LDS, 1 larger LDS batch, 2 line buffers in global memory)."""
    _fields_ = [("nbins", ctypes.c_uint32), ("edges", ctypes.c_uint32 * (MAX_BINS - 1)),
                ("lines_per_tile", ctypes.c_uint32 * MAX_BINS), ("large_lds", ctypes.c_uint32 * MAX_BINS)]

    @classmethod
    def make(cls, edges=(), lines_per_tile=None, large_lds=None):
        c = cls()
        c.nbins = len(edges) + 1
        for i, e in enumerate(edges):
            c.edges[i] = int(e)
        lpt = list(lines_per_tile) if lines_per_tile is not None else [256] * c.nbins
        lg = list(large_lds) if large_lds is not None else [0] * c.nbins
        for i in range(c.nbins):
            c.lines_per_tile[i] = int(lpt[i])
            c.large_lds[i] = int(lg[i])
        return c

    def as_dict(self):
        n = int(self.nbins)
        return {"nbins": n, "edges": [int(self.edges[i]) for i in range(n - 1)],
                "lines_per_tile": [int(self.lines_per_tile[i]) for i in range(n)],
                "large_lds": [int(self.large_lds[i]) for i in range(n)]}


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64), ("host_bytes", ctypes.c_uint64)]


class Reply(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("first_bad", ctypes.c_int64), ("n", ctypes.c_uint64),
                ("off", ctypes.POINTER(ctypes.c_uint64)), ("data", ctypes.POINTER(ctypes.c_uint8)),
                ("bytes", ctypes.c_uint64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("footprint", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("deferred", ctypes.c_uint64), ("peak_device_bytes", ctypes.c_uint64),
                ("device_bytes_in_use", ctypes.c_uint64), ("busy_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    """The loaded libzsmiles.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libzsmiles.so is not built: run python -m paper_2404_19391_amd._build")
        L = ctypes.CDLL(LIB_PATH)
        L.zs_status_str.restype = ctypes.c_char_p
        L.zs_status_str.argtypes = [ctypes.c_int]
        L.zs_dict_create.restype = ctypes.c_int
        L.zs_dict_create.argtypes = [_vp, _vp, ctypes.POINTER(_vp)]
        L.zs_dict_destroy.restype = None
        L.zs_dict_destroy.argtypes = [_vp]
        L.zs_dict_lmax.restype = ctypes.c_int
        L.zs_dict_lmax.argtypes = [_vp]
        L.zs_compress_bound.restype = _u64
        L.zs_compress_bound.argtypes = [_u64, _u64]
        L.zs_decompress_bound.restype = _u64
        L.zs_decompress_bound.argtypes = [_vp, _u64, _u64]
        L.zs_workspace_bytes.restype = ctypes.c_size_t
        L.zs_workspace_bytes.argtypes = [ctypes.c_int, _u64]
        L.zs_compress.restype = ctypes.c_int
        L.zs_compress.argtypes = [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, ctypes.c_uint32, _vp,
                                  ctypes.c_size_t, _vp, _vp]
        L.zs_decompress.restype = ctypes.c_int
        L.zs_decompress.argtypes = [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _vp, ctypes.c_size_t, _vp, _vp]
        L.zs_decompress_lines.restype = ctypes.c_int
        L.zs_decompress_lines.argtypes = [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _vp,
                                          ctypes.c_size_t, _vp, _vp]
        L.zs_decompress_lines_noalloc.restype = ctypes.c_int
        L.zs_decompress_lines_noalloc.argtypes = [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _vp, _vp]
        L.zs_index_lines.restype = ctypes.c_int
        L.zs_index_lines.argtypes = [_vp, _u64, _vp, _u64, _vp, _vp, ctypes.c_size_t, _vp, _vp]
        L.zs_binned_workspace_bytes.restype = ctypes.c_size_t
        L.zs_binned_workspace_bytes.argtypes = [_u64, _u64]
        L.zs_compress_binned.restype = ctypes.c_int
        L.zs_compress_binned.argtypes = [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, ctypes.c_uint32,
                                         ctypes.POINTER(BinConfig), _vp, ctypes.c_size_t, _vp, _vp]
        L.zs_autotune_binned.restype = ctypes.c_int
        L.zs_autotune_binned.argtypes = [_vp, _vp, _u64, _vp, _u64, ctypes.c_uint32, ctypes.POINTER(BinConfig),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_uint32), _vp]
        L.zs_graph_begin.restype = ctypes.c_int
        L.zs_graph_begin.argtypes = [_vp]
        L.zs_graph_end.restype = ctypes.c_int
        L.zs_graph_end.argtypes = [_vp, ctypes.POINTER(_vp)]
        L.zs_graph_launch.restype = ctypes.c_int
        L.zs_graph_launch.argtypes = [_vp, _vp]
        L.zs_graph_destroy.restype = None
        L.zs_graph_destroy.argtypes = [_vp]
        L.zs_server_create.restype = ctypes.c_int
        L.zs_server_create.argtypes = [_vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]
        L.zs_server_add_shard.restype = ctypes.c_int
        L.zs_server_add_shard.argtypes = [_vp, _vp, _u64, _vp, _u64, ctypes.POINTER(ctypes.c_uint32)]
        L.zs_server_submit_decompress.restype = ctypes.c_int
        L.zs_server_submit_decompress.argtypes = [_vp, ctypes.c_uint32, _vp, _u64, ctypes.POINTER(_u64)]
        L.zs_server_submit_compress.restype = ctypes.c_int
        L.zs_server_submit_compress.argtypes = [_vp, _vp, _u64, _vp, _u64, ctypes.c_uint32, ctypes.POINTER(_u64)]
        L.zs_server_wait.restype = ctypes.c_int
        L.zs_server_wait.argtypes = [_vp, _u64, ctypes.POINTER(Reply)]
        L.zs_server_release.restype = None
        L.zs_server_release.argtypes = [_vp, _u64]
        L.zs_server_get_stats.restype = ctypes.c_int
        L.zs_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
        L.zs_server_destroy.restype = None
        L.zs_server_destroy.argtypes = [_vp]
        L.zs_preprocess.restype = ctypes.c_int
        L.zs_preprocess.argtypes = [_vp, _u64, _vp, _u64, _vp, _u64, _vp, _vp, ctypes.c_size_t, _vp, _vp]
        L.zs_postprocess.restype = ctypes.c_int
        L.zs_postprocess.argtypes = [_vp, _u64, _vp, _u64, _vp, _u64, _vp, _vp, ctypes.c_size_t, _vp, _vp]
        L.zs_train_workspace_bytes.restype = ctypes.c_size_t
        L.zs_train_workspace_bytes.argtypes = [_u64, _u64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.zs_train_patterns.restype = ctypes.c_int
        L.zs_train_patterns.argtypes = [_vp, _u64, _vp, _u64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
        L.zsi_compile_dict_c.restype = ctypes.c_int
        L.zsi_compile_dict_c.argtypes = [_vp, _vp, _vp, _u64, ctypes.POINTER(_u64)]
        _lib = L
    return _lib


def status_str(code):
    try:
        return lib().zs_status_str(int(code)).decode()
    except RuntimeError:
        return "status %d" % code


def _torch():
    import torch
    return torch


# Pointer arguments are passed as plain ints (None for NULL): every entry point has
# c_void_p argtypes, so ctypes converts them without a wrapper object per argument.
def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _p(t):
    return t.data_ptr() if t is not None and t.numel() else None


def read_zsd(path):
    """Parse a .zsd dictionary file: a 'ZSD1' header line, then '<hex code> <expansion>' lines."""
    with open(path, "rb") as f:
        rows = f.read().split(b"\n")
    if not rows or not rows[0].startswith(b"ZSD1"):
        raise ValueError("not a ZSD1 dictionary: %s" % path)
    entries = {}
    for row in rows[1:]:
        if row:
            code, exp = row.split(b" ", 1)
            entries[int(code, 16)] = exp
    return entries


def table_arrays(entries):
    """code -> expansion dict as the (len[256], exp[256*16]) host arrays of zs_dict_create."""
    ln = np.zeros(256, dtype=np.uint8)
    ex = np.zeros((256, LMAX_CAP), dtype=np.uint8)
    for c, e in entries.items():
        e = bytes(e)
        if not (0 <= c < 256) or not (1 <= len(e) <= LMAX_CAP):
            raise ZsError(EINVAL, -1, "dictionary entry %r" % (c,))
        ln[c] = len(e)
        ex[c, :len(e)] = np.frombuffer(e, dtype=np.uint8)
    return ln, ex


class Dict:
    """A compiled dictionary resident on the current device (zs_dict)."""

    def __init__(self, entries):
        self.entries = {int(k): bytes(v) for k, v in entries.items()}
        ln, ex = table_arrays(self.entries)
        h = _vp()
        rc = lib().zs_dict_create(ln.ctypes.data_as(_vp), ex.ctypes.data_as(_vp), ctypes.byref(h))
        if rc != OK:
            raise ZsError(rc, -1, "zs_dict_create")
        self._h = h
        self.lmax = lib().zs_dict_lmax(h)

    @classmethod
    def load(cls, path=None):
        return cls(read_zsd(path or default_dict_path()))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().zs_dict_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compile_tables(entries):
    """Compile a dictionary into its kernel image on the host (no GPU needed); returns bytes."""
    ln, ex = table_arrays(entries)
    cap = 1 << 20
    buf = np.zeros(cap, dtype=np.uint8)
    size = _u64(0)
    rc = lib().zsi_compile_dict_c(ln.ctypes.data_as(_vp), ex.ctypes.data_as(_vp), buf.ctypes.data_as(_vp), cap,
                                  ctypes.byref(size))
    if rc != OK:
        raise ZsError(rc, -1, "compile dictionary")
    return buf[:size.value].tobytes()


def workspace_bytes(op, n):
    return int(lib().zs_workspace_bytes(op, n))


class Workspaces:
    """Device scratch reused across calls, one per operation (calls on one stream)."""

    def __init__(self, device="cuda"):
        self.device = device
        self._ws = {}

    def get(self, op, n):
        torch = _torch()
        need = max(workspace_bytes(op, n), 64)
        cur = self._ws.get(op)
        if cur is None or cur.numel() < need:
            cur = torch.empty(need + (need >> 3), dtype=torch.uint8, device=self.device)
            self._ws[op] = cur
        return cur


_default_ws = {}


def _ws_for(device):
    key = str(device)
    if key not in _default_ws:
        _default_ws[key] = Workspaces(device)
    return _default_ws[key]


def new_result(device="cuda"):
    return _torch().zeros(2, dtype=_torch().int64, device=device)


def read_result(res):
    v = res.cpu().numpy()
    code = int(np.int32(v[0] & 0xFFFFFFFF))
    return code, int(v[1])


def _check_rc(rc, what):
    if rc != OK:
        raise ZsError(rc, -1, what)


def _check_res(res, what, check):
    code, fb = read_result(res)
    if check and code != OK:
        raise ZsError(code, fb, what)
    return code, fb


# ---- raw entry points (preallocated device buffers; enqueue only) --------------------------------

def compress_into(d, buf, off, out, out_off, ws, res, preprocess=True, in_bytes=None):
    """zs_compress on preallocated tensors; out may be None (size-only)."""
    n = off.numel() - 1
    nb = buf.numel() if in_bytes is None else in_bytes
    rc = lib().zs_compress(d.handle, _p(buf), nb, _p(off), n, _p(out), out.numel() if out is not None else 0,
                           _p(out_off), F_PREPROCESS if preprocess else 0, _p(ws), ws.numel(), _p(res), _stream())
    _check_rc(rc, "zs_compress")


def preprocess_into(buf, off, out, out_off, ws, res, in_bytes=None):
    """zs_preprocess on preallocated tensors (ws: the OP_COMPRESS workspace); out may be None."""
    n = off.numel() - 1
    nb = buf.numel() if in_bytes is None else in_bytes
    rc = lib().zs_preprocess(_p(buf), nb, _p(off), n, _p(out), out.numel() if out is not None else 0,
                             _p(out_off), _p(ws), ws.numel(), _p(res), _stream())
    _check_rc(rc, "zs_preprocess")


def postprocess_into(buf, off, out, out_off, ws, res, in_bytes=None):
    """zs_postprocess on preallocated tensors (ws: the OP_COMPRESS workspace); out may be None."""
    n = off.numel() - 1
    nb = buf.numel() if in_bytes is None else in_bytes
    rc = lib().zs_postprocess(_p(buf), nb, _p(off), n, _p(out), out.numel() if out is not None else 0,
                              _p(out_off), _p(ws), ws.numel(), _p(res), _stream())
    _check_rc(rc, "zs_postprocess")


def train_workspace_bytes(in_bytes, n, lmin, lmax, preprocess=True):
    return int(lib().zs_train_workspace_bytes(in_bytes, n, lmin, lmax, F_PREPROCESS if preprocess else 0))


def train_patterns_into(buf, off, T, lmin, lmax, preprocess, pat, pat_len, n_chosen, ws, res, in_bytes=None):
    """zs_train_patterns on preallocated tensors: pat uint8 [T, 16], pat_len uint8 [T], n_chosen int32 [1]."""
    n = off.numel() - 1
    nb = buf.numel() if in_bytes is None else in_bytes
    rc = lib().zs_train_patterns(_p(buf), nb, _p(off), n, F_PREPROCESS if preprocess else 0, lmin, lmax, T,
                                 _p(pat), _p(pat_len), _p(n_chosen), _p(ws), ws.numel(), _p(res), _stream())
    _check_rc(rc, "zs_train_patterns")


def binned_workspace_bytes(n, out_cap):
    return int(lib().zs_binned_workspace_bytes(n, out_cap))


def compress_binned_into(d, buf, off, out, out_off, cfg, ws, res, preprocess=True, in_bytes=None):
    """zs_compress_binned on preallocated tensors; out may be None (size-only)."""
    n = off.numel() - 1
    nb = buf.numel() if in_bytes is None else in_bytes
    rc = lib().zs_compress_binned(d.handle, _p(buf), nb, _p(off), n, _p(out),
                                  out.numel() if out is not None else 0, _p(out_off),
                                  F_PREPROCESS if preprocess else 0, ctypes.byref(cfg), _p(ws), ws.numel(), _p(res),
                                  _stream())
    _check_rc(rc, "zs_compress_binned")


def autotune_binned(d, buf, off, preprocess=True):
    """zs_autotune_binned on device lines (a sample of the workload): (BinConfig, best_ms, plain_ms, tried)."""
    n = off.numel() - 1
    cfg = BinConfig()
    best, plain = ctypes.c_double(0), ctypes.c_double(0)
    tried = ctypes.c_uint32(0)
    rc = lib().zs_autotune_binned(d.handle, _p(buf), buf.numel(), _p(off), n, F_PREPROCESS if preprocess else 0,
                                  ctypes.byref(cfg), ctypes.byref(best), ctypes.byref(plain), ctypes.byref(tried),
                                  _stream())
    _check_rc(rc, "zs_autotune_binned")
    return cfg, best.value, plain.value, int(tried.value)


class Graph:
    """A HIP graph of codec calls: capture the calls made inside `with g.capture(stream):`, then replay()."""

    def __init__(self):
        self.handle = None
        self.stream = None

    def capture(self, stream):
        g = self

        class _Ctx:
            def __enter__(self_):
                g.stream = stream
                _check_rc(lib().zs_graph_begin(_vp(stream.cuda_stream)), "zs_graph_begin")
                return g

            def __exit__(self_, et, ev, tb):
                h = _vp()
                rc = lib().zs_graph_end(_vp(stream.cuda_stream), ctypes.byref(h))
                if et is None:
                    _check_rc(rc, "zs_graph_end")
                    g.handle = h
                return False

        return _Ctx()

    def replay(self, stream=None):
        s = stream if stream is not None else self.stream
        _check_rc(lib().zs_graph_launch(self.handle, _vp(s.cuda_stream)), "zs_graph_launch")

    def __del__(self):
        try:
            if self.handle:
                lib().zs_graph_destroy(self.handle)
        except Exception:
            pass


def decompress_into(d, buf, off, out, out_off, ws, res, in_bytes=None):
    n = off.numel() - 1
    nb = buf.numel() if in_bytes is None else in_bytes
    rc = lib().zs_decompress(d.handle, _p(buf), nb, _p(off), n, _p(out), out.numel() if out is not None else 0,
                             _p(out_off), _p(ws), ws.numel(), _p(res), _stream())
    _check_rc(rc, "zs_decompress")


def decompress_lines_into(d, buf, off, ids, out, out_off, ws, res, in_bytes=None):
    n = off.numel() - 1
    nb = buf.numel() if in_bytes is None else in_bytes
    rc = lib().zs_decompress_lines(d.handle, _p(buf), nb, _p(off), n, _p(ids), ids.numel(), _p(out),
                                   out.numel() if out is not None else 0, _p(out_off), _p(ws), ws.numel(),
                                   _p(res), _stream())
    _check_rc(rc, "zs_decompress_lines")


NOALLOC_MAX_IDS = 1 << 24


def decompress_lines_noalloc_into(d, buf, off, ids, out, out_off, res, in_bytes=None, n_ids=None):
    """zs_decompress_lines_noalloc: the library's static scratch instead of a workspace."""
    n = off.numel() - 1
    nb = buf.numel() if in_bytes is None else in_bytes
    k = ids.numel() if n_ids is None else n_ids
    rc = lib().zs_decompress_lines_noalloc(d.handle, _p(buf), nb, _p(off), n, _p(ids), k, _p(out),
                                           out.numel() if out is not None else 0, _p(out_off), _p(res), _stream())
    _check_rc(rc, "zs_decompress_lines_noalloc")


def index_into(buf, off, n_out, ws, res):
    rc = lib().zs_index_lines(_p(buf), buf.numel(), _p(off), off.numel(), _p(n_out), _p(ws), ws.numel(), _p(res),
                              _stream())
    _check_rc(rc, "zs_index_lines")


# ---- convenience: exact-size outputs (a size-only pass, one host read, then the call) -------------

def _sized(run, out_off, device, check, what):
    torch = _torch()
    res = new_result(device)
    run(None, res)
    total = int(out_off[-1].item())
    out = torch.empty(max(total, 1), dtype=torch.uint8, device=device)
    res = new_result(device)
    run(out, res)
    _check_res(res, what, check)
    return out[:total], out_off


def compress(d, buf, off, preprocess=True, check=True):
    """Compress a buffer of lines; returns (bytes uint8, offsets int64) on the same device."""
    torch = _torch()
    n = off.numel() - 1
    dev = buf.device if buf.numel() else off.device
    out_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ws = _ws_for(dev).get(OP_COMPRESS, n)
    return _sized(lambda out, res: compress_into(d, buf, off, out, out_off, ws, res, preprocess), out_off, dev,
                  check, "compress")


def compress_binned(d, buf, off, cfg, preprocess=True, check=True):
    """Length-binned compression; the same bytes and offsets as compress()."""
    torch = _torch()
    n = off.numel() - 1
    dev = buf.device if buf.numel() else off.device
    out_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    state = {}

    def run(out, res):
        cap = out.numel() if out is not None else 0
        need = max(binned_workspace_bytes(n, cap), 64)
        ws = state.get("ws")
        if ws is None or ws.numel() < need:
            ws = state["ws"] = torch.empty(need, dtype=torch.uint8, device=dev)
        compress_binned_into(d, buf, off, out, out_off, cfg, ws, res, preprocess)

    return _sized(run, out_off, dev, check, "compress_binned")


def preprocess(buf, off, check=True):
    """Ring-ID pre-processing of every line (Sec. IV-A); returns (bytes, offsets)."""
    torch = _torch()
    n = off.numel() - 1
    dev = buf.device if buf.numel() else off.device
    out_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ws = _ws_for(dev).get(OP_COMPRESS, n)
    return _sized(lambda out, res: preprocess_into(buf, off, out, out_off, ws, res), out_off, dev, check,
                  "preprocess")


def postprocess(buf, off, check=True):
    """Post-processing of decompressed lines: ring labels renumbered in the writers'
    convention (the library's definition of the step Sec. IV-D names); (bytes, offsets)."""
    torch = _torch()
    n = off.numel() - 1
    dev = buf.device if buf.numel() else off.device
    out_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ws = _ws_for(dev).get(OP_COMPRESS, n)
    return _sized(lambda out, res: postprocess_into(buf, off, out, out_off, ws, res), out_off, dev, check,
                  "postprocess")


def train_patterns(buf, off, T, lmin=2, lmax=8, preprocess=True, check=True):
    """Algorithm 1 (Sec. IV-C) on the device: the T substrings of highest Eq. (1) rank, in
    selection order, as a list of bytes (fewer when no candidate has a positive rank)."""
    torch = _torch()
    n = off.numel() - 1
    dev = buf.device if buf.numel() else off.device
    ws = torch.empty(max(train_workspace_bytes(buf.numel(), n, lmin, lmax, preprocess), 64), dtype=torch.uint8,
                     device=dev)
    pat = torch.zeros((max(T, 1), 16), dtype=torch.uint8, device=dev)
    plen = torch.zeros(max(T, 1), dtype=torch.uint8, device=dev)
    nch = torch.zeros(1, dtype=torch.int32, device=dev)
    res = new_result(dev)
    train_patterns_into(buf, off, T, lmin, lmax, preprocess, pat, plen, nch, ws, res)
    _check_res(res, "train_patterns", check)
    k = int(nch.item())
    ph, lh = pat.cpu().numpy(), plen.cpu().numpy()
    return [ph[i, :lh[i]].tobytes() for i in range(k)]


def decompress(d, buf, off, check=True):
    torch = _torch()
    n = off.numel() - 1
    dev = buf.device if buf.numel() else off.device
    out_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ws = _ws_for(dev).get(OP_DECOMPRESS, n)
    return _sized(lambda out, res: decompress_into(d, buf, off, out, out_off, ws, res), out_off, dev, check,
                  "decompress")


def decompress_lines(d, buf, off, ids, check=True):
    torch = _torch()
    k = ids.numel()
    dev = off.device
    out_off = torch.empty(k + 1, dtype=torch.int64, device=dev)
    ws = _ws_for(dev).get(OP_DECOMPRESS_LINES, k)
    return _sized(lambda out, res: decompress_lines_into(d, buf, off, ids, out, out_off, ws, res), out_off, dev,
                  check, "decompress_lines")


def index_lines(buf, check=True):
    """Line index of a newline-separated device buffer: int64 offsets (n+1)."""
    torch = _torch()
    dev = buf.device
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = _ws_for(dev).get(OP_INDEX, buf.numel())
    res = new_result(dev)
    probe = torch.empty(1, dtype=torch.int64, device=dev)
    index_into(buf, probe[:0], n_out, ws, res)  # count only
    n = int(n_out.item())
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    res = new_result(dev)
    index_into(buf, off, n_out, ws, res)
    _check_res(res, "index_lines", check)
    return off


# ---- request loop ----------------------------------------------------------------------------------

class Server:
    """zs_server: resident shards, requests from any thread, admission by exact device footprint.

    submit_* return a ticket; wait(ticket) returns (code, first_bad, data uint8 array, offsets uint64
    array, timings dict) and releases the request's host buffers."""

    def __init__(self, d, slots=8, device_bytes=4 << 30, host_bytes=2 << 30):
        self.d = d
        cfg = ServerConfig(slots, device_bytes, host_bytes)
        h = _vp()
        _check_rc(lib().zs_server_create(d.handle, ctypes.byref(cfg), ctypes.byref(h)), "zs_server_create")
        self.handle = h
        self._keep = []

    def add_shard(self, buf, off):
        """Register a device-resident compressed shard (uint8 bytes, int64 offsets); returns its id."""
        sid = ctypes.c_uint32(0)
        _check_rc(lib().zs_server_add_shard(self.handle, _p(buf), buf.numel(), _p(off), off.numel() - 1,
                                            ctypes.byref(sid)), "zs_server_add_shard")
        self._keep.append((buf, off))
        return int(sid.value)

    def submit_decompress(self, shard, ids):
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        t = _u64(0)
        _check_rc(lib().zs_server_submit_decompress(self.handle, shard, ids.ctypes.data_as(_vp), ids.size,
                                                    ctypes.byref(t)), "zs_server_submit_decompress")
        return int(t.value)

    def submit_compress(self, lines, off, preprocess=True):
        lines = np.ascontiguousarray(lines, dtype=np.uint8)
        off = np.ascontiguousarray(off, dtype=np.uint64)
        t = _u64(0)
        _check_rc(lib().zs_server_submit_compress(self.handle, lines.ctypes.data_as(_vp), lines.size,
                                                  off.ctypes.data_as(_vp), off.size - 1,
                                                  F_PREPROCESS if preprocess else 0, ctypes.byref(t)),
                  "zs_server_submit_compress")
        return int(t.value)

    def wait(self, ticket, copy=True):
        """Block until the request is done; (code, first_bad, data, offsets, times).  With
        copy=False the reply's bytes and offsets are not copied out (empty arrays; the byte
        count is in times["bytes"])."""
        r = Reply()
        _check_rc(lib().zs_server_wait(self.handle, ticket, ctypes.byref(r)), "zs_server_wait")
        n = int(r.n)
        # a request that failed before its output was written has no offsets
        off = np.ctypeslib.as_array(r.off, shape=(n + 1,)).copy() if (r.off and copy) else \
            np.zeros(0, dtype=np.uint64)
        data = np.ctypeslib.as_array(r.data, shape=(int(r.bytes),)).copy() if (r.bytes and copy) else \
            np.zeros(0, dtype=np.uint8)
        t = {"submit": r.t_submit, "admit": r.t_admit, "done": r.t_done, "footprint": int(r.footprint),
             "bytes": int(r.bytes)}
        code, fb = int(r.code), int(r.first_bad)
        lib().zs_server_release(self.handle, ticket)
        return code, fb, data, off, t

    def stats(self):
        st = ServerStats()
        _check_rc(lib().zs_server_get_stats(self.handle, ctypes.byref(st)), "zs_server_get_stats")
        return st.as_dict()

    def close(self):
        if self.handle:
            lib().zs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
