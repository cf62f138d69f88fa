"""GPU parity with every frozen dictionary, not only the default one: the L_max sweep
(Sec. V-C: L_max 5, 8, 15), the six Table I variants (Sec. V-B: pre-processing on/off x
pre-population Printable / SMILES alphabet / None), a dictionary with patterns of 9..16
bytes (the 16-wide parse window and the decoder's long expansions), and a sparse
hand-made dictionary whose bytes mostly fall outside every pattern. Byte-exact against
the oracle: compression (plain and binned), bulk decompression and random access."""
import os

import numpy as np
import pytest

import oracle
import smilesgen
from test_gpu_codec import _edge_lines

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2404_19391_amd", "data")

# (dictionary file, pre-processing flag the dictionary was trained for)
DICTS = [("lmax5", True), ("default", True), ("lmax15", True), ("long16", True),
         ("t1_prep_printable", True), ("t1_raw_printable", False), ("t1_prep_smiles", True),
         ("t1_raw_smiles", False), ("t1_prep_none", True), ("t1_raw_none", False)]

SPARSE = {ord("C"): b"C", ord("c"): b"c", ord("A"): b"CC", ord("D"): b"cc", ord("E"): b"C(", 0xA1: b"(C)",
          0xA2: b"CCCCCCCCCC", 0xA3: b"c1", ord("G"): b"=", 0xA4: b"C" * 16, 0xA5: b"C(C)C(C)C(C)C(C)",
          0xFF: b"c0ccccc0"}


@pytest.fixture(scope="module")
def zs():
    import paper_2404_19391_amd as zs
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return zs


def dev(buf, off):
    return (torch.from_numpy(np.ascontiguousarray(buf, dtype=np.uint8)).cuda(),
            torch.from_numpy(np.ascontiguousarray(off).astype(np.int64)).cuda())


def host(t):
    return t.cpu().numpy()


def _pair(zs, name):
    if name == "sparse":
        return zs.Dict(SPARSE), oracle.Dict(SPARSE)
    path = os.path.join(DATA, name + ".zsd")
    od = oracle.Dict.load(path)
    assert od.valid
    return zs.Dict.load(path), od


def _inputs(od, preprocess):
    """Edge lines and generated lines, without the few whose compressed form under
    this dictionary would exceed ZS_MAX_CLINE (the library rejects those, the
    oracle has no such limit; that case is tested in test_gpu_codec)."""
    lines = _edge_lines()
    lines += smilesgen.lines("test", 301, 3000)
    lines += smilesgen.lines("uneven", 302, 1500)
    lines = [l for l in lines if len(oracle.compress_line(od, l, preprocess)) <= 8192]
    return oracle.join_lines(lines)


def _check_all(zs, gd, od, buf, off, preprocess):
    code, fb, want, woff = oracle.compress(od, buf, off, preprocess=preprocess)
    b, o = dev(buf, off)
    got, goff = zs.compress(gd, b, o, preprocess=preprocess, check=False)
    torch.cuda.synchronize()
    assert np.array_equal(host(goff).astype(np.uint64), woff)
    assert host(got).tobytes() == want.tobytes()
    cfg = zs.BinConfig.make(edges=(64, 256), lines_per_tile=(256, 128, 32), large_lds=(0, 0, 1))
    bg, bgo = zs.compress_binned(gd, b, o, cfg, preprocess=preprocess, check=False)
    assert torch.equal(bg, got) and torch.equal(bgo, goff)
    # decode: the oracle's compressed bytes, in bulk and by line id
    dcode, dfb, back, boff = oracle.decompress(od, want, woff)
    assert dcode == 0
    cb, co = dev(want, woff)
    gb, gbo = zs.decompress(gd, cb, co, check=False)
    assert np.array_equal(host(gbo).astype(np.uint64), boff)
    assert host(gb).tobytes() == back.tobytes()
    n = woff.size - 1
    ids = np.random.default_rng(n).integers(0, n, 5000).astype(np.uint64)
    rcode, rfb, rw, rwo = oracle.decompress_lines(od, want, woff, ids)
    rg, rgo = zs.decompress_lines(gd, cb, co, torch.from_numpy(ids.astype(np.int64)).cuda(), check=False)
    assert np.array_equal(host(rgo).astype(np.uint64), rwo)
    assert host(rg).tobytes() == rw.tobytes()
    return code, want, woff


@pytest.mark.parametrize("name,prep", DICTS)
def test_dictionary_parity(zs, name, prep):
    gd, od = _pair(zs, name)
    buf, off = _inputs(od, prep)
    _check_all(zs, gd, od, buf, off, prep)


@pytest.mark.parametrize("name", ["t1_prep_none", "long16"])
def test_dictionary_parity_other_flag(zs, name):
    gd, od = _pair(zs, name)
    buf, off = _inputs(od, False)
    _check_all(zs, gd, od, buf, off, False)


def test_long_patterns_run_the_wide_window(zs):
    gd, od = _pair(zs, "long16")
    assert od.lmax > 8 and gd.lmax == od.lmax
    # lines made of the long patterns themselves: the long codes are chosen and the
    # decoder expands them
    longs = [e for e in od.entries.values() if len(e) > 8]
    rnd = np.random.default_rng(3)
    lines = [b"".join(longs[int(k)] for k in rnd.integers(0, len(longs), int(rnd.integers(1, 30))))
             for _ in range(4000)]
    buf, off = oracle.join_lines(lines)
    code, want, woff = _check_all(zs, gd, od, buf, off, False)
    assert code == 0 and want.size < 0.3 * buf.size


def test_sparse_dictionary(zs):
    gd, od = _pair(zs, "sparse")
    for prep in (True, False):
        buf, off = _inputs(od, prep)
        _check_all(zs, gd, od, buf, off, prep)
