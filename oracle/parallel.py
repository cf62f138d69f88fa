"""TEST INFRASTRUCTURE: the oracle run as several host processes on disjoint line ranges.

Each worker is a fresh interpreter (multiprocessing "spawn": nothing of the parent,
whose process may have initialised a GPU, is inherited) that loads the oracle
library and the dictionary file itself, maps its input from a temporary file and
runs the plain single-threaded oracle (zs_oracle.c) on ranges of lines; the results
are concatenated in line order.  Used to compare full-size GPU outputs with the
oracle line for line, and for the all-cores CPU baseline.  Lines are independent
(one SMILES per line, Sec. I), so splitting the buffer by lines leaves every
line's result unchanged.
"""
import multiprocessing as mp
import os
import shutil
import tempfile
import time

import numpy as np

_W = {}


def _init(dict_path):
    import oracle
    _W["d"] = oracle.Dict.load(dict_path)
    _W["maps"] = {}


def _mapped(path, dtype, count):
    key = (path, count)
    m = _W["maps"].get(key)
    if m is None:
        m = np.memmap(path, dtype=dtype, mode="r", shape=(count,)) if count else np.zeros(0, dtype)
        _W["maps"] = {key: m}  # the input of the current call only
    return m


def _job(args):
    import oracle
    op, bp, nbuf, opath, noff, a, b, preprocess = args
    buf = _mapped(bp, np.uint8, nbuf)
    off = np.memmap(opath, dtype=np.uint64, mode="r", shape=(noff,))
    lo, hi = int(off[a]), int(off[b])
    sub = np.array(buf[lo:min(hi, buf.size)])
    soff = np.array(off[a:b + 1]) - off[a]
    t0 = time.perf_counter()
    if op == "c":
        code, fb, out, out_off = oracle.compress(_W["d"], sub, soff, preprocess=preprocess)
    else:
        code, fb, out, out_off = oracle.decompress(_W["d"], sub, soff)
    dt = time.perf_counter() - t0
    return a, code, (fb + a if fb >= 0 else -1), out.tobytes(), out_off, dt


def default_procs():
    """Host cores this process may use (its CPU affinity), at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _ranges(n, pieces):
    pieces = max(1, min(pieces, n))
    cuts = np.linspace(0, n, pieces + 1).astype(np.int64)
    return [(int(cuts[i]), int(cuts[i + 1])) for i in range(pieces) if cuts[i + 1] > cuts[i]]


class Pool:
    """Worker processes holding one dictionary; compress/decompress return
    (code, first_bad, out, out_off, wall_seconds, summed_worker_seconds), the wall
    time from handing out the work to having every result back (workers already
    started)."""

    def __init__(self, dict_path, procs=None):
        self.procs = procs or default_procs()
        self.tmp = tempfile.mkdtemp(prefix="zs_oracle_")
        self.seq = 0
        self.pool = mp.get_context("spawn").Pool(self.procs, initializer=_init, initargs=(dict_path,))

    def close(self):
        if self.pool is not None:
            self.pool.close()
            self.pool.join()
            self.pool = None
        shutil.rmtree(self.tmp, ignore_errors=True)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _run(self, op, buf, off, preprocess, pieces):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        off = np.ascontiguousarray(off, dtype=np.uint64)
        n = off.size - 1
        if n == 0:
            return 0, -1, np.zeros(0, np.uint8), np.zeros(1, np.uint64), 0.0, 0.0
        self.seq += 1
        bp = os.path.join(self.tmp, "buf%d" % self.seq)
        opath = os.path.join(self.tmp, "off%d" % self.seq)
        buf.tofile(bp)
        off.tofile(opath)
        jobs = [(op, bp, buf.size, opath, off.size, a, b, preprocess)
                for a, b in _ranges(n, pieces or 4 * self.procs)]
        t0 = time.perf_counter()
        parts = sorted(self.pool.map(_job, jobs, chunksize=1))
        wall = time.perf_counter() - t0
        os.remove(bp)
        os.remove(opath)
        code, fb = 0, -1
        outs, offs = [], [np.zeros(1, dtype=np.uint64)]
        base = 0
        for a, c, f, ob, oo, _ in parts:
            if c != 0 and code == 0:
                code, fb = c, f
            outs.append(ob)
            offs.append(oo[1:] + np.uint64(base))
            base += int(oo[-1])
        out = np.frombuffer(b"".join(outs), dtype=np.uint8)
        return code, fb, out, np.concatenate(offs), wall, sum(p[5] for p in parts)

    def compress(self, buf, off, preprocess=True, pieces=None):
        return self._run("c", buf, off, preprocess, pieces)

    def decompress(self, buf, off, pieces=None):
        return self._run("d", buf, off, True, pieces)


def compress(dict_path, buf, off, preprocess=True, procs=None, pieces=None):
    """Oracle compression of every line with `procs` worker processes."""
    with Pool(dict_path, procs) as p:
        return p.compress(buf, off, preprocess, pieces)


def decompress(dict_path, buf, off, procs=None, pieces=None):
    """Oracle decompression of every line with `procs` worker processes."""
    with Pool(dict_path, procs) as p:
        return p.decompress(buf, off, pieces)
