"""The oracle split over host processes gives the single-process oracle's bytes."""
import numpy as np

import oracle
from oracle import parallel

from conftest import DEFAULT_DICT


def test_parallel_compress_and_decompress_equal_serial(odict):
    import smilesgen
    buf, off = smilesgen.generate("uneven", 5, 3001)
    buf = buf[:-1].copy()          # last line ends at the virtual newline
    off = off.copy()
    assert int(off[-1]) == buf.size + 1
    want = oracle.compress(odict, buf, off)
    got = parallel.compress(DEFAULT_DICT, buf, off, procs=3, pieces=7)
    assert got[:2] == want[:2]
    assert got[2].tobytes() == want[2].tobytes() and np.array_equal(got[3], want[3])
    dw = oracle.decompress(odict, want[2], want[3])
    dg = parallel.decompress(DEFAULT_DICT, want[2], want[3], procs=2, pieces=5)
    assert dg[:2] == dw[:2] and dg[2].tobytes() == dw[2].tobytes() and np.array_equal(dg[3], dw[3])


def test_parallel_reports_first_bad_line(odict):
    lines = [b"CC"] * 50 + [b"C\x01"] + [b"CC"] * 20 + [b"\x7f"]
    buf, off = oracle.join_lines(lines)
    want = oracle.compress(odict, buf, off)
    got = parallel.compress(DEFAULT_DICT, buf, off, procs=2, pieces=6)
    assert got[:2] == want[:2] == (oracle.ECORRUPT, 50)
    assert got[2].tobytes() == want[2].tobytes()
