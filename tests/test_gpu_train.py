"""GPU parity of the pre-processing call (zs_preprocess, Sec. IV-A) and of dictionary
generation on the device (zs_train_patterns: Algorithm 1 with the rank of Eq. (1),
Sec. IV-C) against the oracle: the same bytes and offsets, and the same patterns in the
same selection order (integer ranks and fixed tie-breaks, so the tolerance is zero)."""
import numpy as np
import pytest

import oracle
import smilesgen
from test_gpu_codec import _edge_lines
from test_oracle_train import HAND_CASES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def test_preprocess_matches_oracle(zs):
    lines = [l for l in _edge_lines() if len(l) <= 4096]
    lines += smilesgen.lines("uneven", 401, 3000) + smilesgen.lines("test", 402, 3000)
    buf, off = oracle.join_lines(lines)
    want, woff = oracle.preprocess_buffer(buf, off)
    b, o = dev(buf, off)
    got, goff = zs.preprocess(b, o)
    assert np.array_equal(host(goff).astype(np.uint64), woff)
    assert host(got).tobytes() == want.tobytes()
    # many tiles, and a last line ending at the virtual newline
    buf, off = smilesgen.generate("bulk", 403, 300000)
    buf = buf[:-1].copy()
    want, woff = oracle.preprocess_buffer(buf, off)
    b, o = dev(buf, off)
    got, goff = zs.preprocess(b, o)
    assert np.array_equal(host(goff).astype(np.uint64), woff)
    assert host(got).tobytes() == want.tobytes()


def test_preprocess_bad_lines(zs):
    lines = [b"C1CC1", b"C\x01C", b"C" * 4097, b"C1CC%10C1%10"]
    buf, off = oracle.join_lines(lines)
    b, o = dev(buf, off)
    got, goff = zs.preprocess(b, o, check=False)
    g = oracle.split_lines(host(got), host(goff))
    assert g == [oracle.preprocess(lines[0]), b"", b"", oracle.preprocess(lines[3])]
    ws = zs.Workspaces().get(zs.OP_COMPRESS, len(lines))
    res = zs.new_result()
    out = torch.empty(int(host(goff)[-1]), dtype=torch.uint8, device="cuda")
    zs.preprocess_into(b, o, out, goff, ws, res)
    assert zs.read_result(res) == (zs.ECORRUPT, 1)


def _gpu_train(zs, buf, off, T, lmin, lmax, preprocess, check=True):
    b, o = dev(buf, off)
    return zs.train_patterns(b, o, T, lmin=lmin, lmax=lmax, preprocess=preprocess, check=check)


@pytest.mark.parametrize("name", sorted(HAND_CASES))
def test_train_hand_worked(zs, name):
    lines, lmin, lmax, T, want = HAND_CASES[name]
    buf, off = oracle.join_lines(lines)
    assert _gpu_train(zs, buf, off, T, lmin, lmax, False) == want


@pytest.mark.parametrize("lmin,lmax,prep,n", [(2, 5, True, 10000), (2, 8, True, 10000), (2, 8, False, 10000),
                                              (2, 15, True, 3000), (9, 16, True, 3000), (1, 3, False, 2000)])
def test_train_matches_oracle(zs, lmin, lmax, prep, n):
    buf, off = smilesgen.generate("small", 1000, n)
    T = 146
    want = oracle.train_patterns(buf, off, T, lmin=lmin, lmax=lmax, preprocess=prep)
    got = _gpu_train(zs, buf, off, T, lmin, lmax, prep)
    assert got == want


def test_train_reproduces_frozen_dictionaries(zs):
    """The frozen default and L_max 5 dictionaries hold, after the SMILES alphabet, the
    patterns the device trainer selects on their corpus (in selection order)."""
    import os
    from oracle.make_default_dict import SMILES_ALPHABET
    from oracle.make_dicts import DATA, pattern_codes
    buf, off = smilesgen.generate("small", 1000, 10000)
    codes = pattern_codes(SMILES_ALPHABET)
    for name, lmax in (("default", 8), ("lmax5", 5)):
        od = oracle.Dict.load(os.path.join(DATA, name + ".zsd"))
        got = _gpu_train(zs, buf, off, len(codes), 2, lmax, True)
        assert [od.entries[c] for c in codes[:len(got)]] == got


def test_train_edge_cases(zs):
    # T = 0, more patterns asked than there are, a corpus of empty lines, no lines at all
    buf, off = oracle.join_lines([b"CCO", b"CCN"])
    assert _gpu_train(zs, buf, off, 0, 2, 3, False) == []
    assert _gpu_train(zs, buf, off, 50, 2, 3, False) == oracle.train_patterns(buf, off, 50, lmin=2, lmax=3,
                                                                                preprocess=False)
    buf, off = oracle.join_lines([b"", b"", b"C"])
    assert _gpu_train(zs, buf, off, 5, 2, 3, True) == []
    buf, off = np.zeros(0, np.uint8), np.zeros(1, np.uint64)
    assert _gpu_train(zs, buf, off, 5, 2, 3, True) == []
    # the virtual last newline and a sub-range of a larger buffer
    raw = np.frombuffer(b"XXXX\nCCOCC\nCCN", dtype=np.uint8).copy()
    off = np.array([5, 11, 15], dtype=np.uint64)
    want = oracle.train_patterns(raw, off, 10, lmin=2, lmax=4, preprocess=False)
    assert _gpu_train(zs, raw, off, 10, 2, 4, False) == want and want


def test_train_bad_corpus(zs):
    lines = [b"CCO", b"C\x02C", b"CC"]
    buf, off = oracle.join_lines(lines)
    for prep in (False, True):
        b, o = dev(buf, off)
        ws = torch.empty(zs.train_workspace_bytes(buf.size, 3, 2, 3, prep), dtype=torch.uint8, device="cuda")
        pat = torch.zeros((4, 16), dtype=torch.uint8, device="cuda")
        plen = torch.zeros(4, dtype=torch.uint8, device="cuda")
        nch = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        res = zs.new_result()
        zs.train_patterns_into(b, o, 4, 2, 3, prep, pat, plen, nch, ws, res)
        assert zs.read_result(res) == (zs.ECORRUPT, 1)
        assert int(nch.item()) == 0
    with pytest.raises(zs.ZsError):
        _gpu_train(zs, buf, off, 4, 3, 2, False)


def _ring_lines():
    from test_oracle_postprocess import _random_ring_line
    rng = np.random.default_rng(601)
    return [_random_ring_line(rng, int(rng.integers(1, 60))) for _ in range(3000)]


def test_postprocess_matches_oracle(zs):
    """Post-processing (the library's definition of the step Sec. IV-D names) of
    decompressed lines, raw lines and random ring structures (up to 60 rings, crossing,
    nested, %nn): byte-exact against the oracle, through all three ring paths."""
    lines = [l for l in _edge_lines() if len(l) <= 4096]
    lines += smilesgen.lines("uneven", 602, 3000) + _ring_lines()
    lines += [oracle.preprocess(l) for l in smilesgen.lines("uneven", 603, 3000)]
    lines = [l for l in lines if len(l) <= 4096]
    buf, off = oracle.join_lines(lines)
    want, woff = oracle.postprocess_buffer(buf, off)
    b, o = dev(buf, off)
    got, goff = zs.postprocess(b, o)
    assert np.array_equal(host(goff).astype(np.uint64), woff)
    assert host(got).tobytes() == want.tobytes()
    # decompress -> post-process gives the oracle's post-processed lines of the input
    d = zs.Dict.load()
    raw, roff = smilesgen.generate("bulk", 604, 200000)
    rb, ro = dev(raw, roff)
    c, co = zs.compress(d, rb, ro)
    back, boff = zs.decompress(d, c, co)
    p, po = zs.postprocess(back, boff)
    want, woff = oracle.postprocess_buffer(raw, roff)
    assert np.array_equal(host(po).astype(np.uint64), woff)
    assert host(p).tobytes() == want.tobytes()


def test_preprocess_ring_structures(zs):
    """Pre-processing of random ring structures (up to 60 rings) through the register and
    global-memory ring paths."""
    lines = _ring_lines()
    buf, off = oracle.join_lines(lines)
    want, woff = oracle.preprocess_buffer(buf, off)
    b, o = dev(buf, off)
    got, goff = zs.preprocess(b, o)
    assert np.array_equal(host(goff).astype(np.uint64), woff)
    assert host(got).tobytes() == want.tobytes()
