"""GPU parity of the length-binned compressor (zs_compress_binned) and of its
HIP-graph replay against the CPU oracle, byte for byte: every configuration must
give exactly the bytes, offsets and result word of the plain compressor, which
are the oracle's."""
import numpy as np
import pytest

import oracle
import smilesgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CONFIGS = [
    dict(edges=()),
    dict(edges=(128,), lines_per_tile=(256, 64), large_lds=(0, 1)),
    dict(edges=(64, 256), lines_per_tile=(256, 128, 32), large_lds=(0, 0, 1)),
    dict(edges=(16, 32, 48, 64, 96, 128, 400), lines_per_tile=(256, 200, 160, 128, 96, 64, 33, 32),
         large_lds=(1, 0, 1, 0, 1, 0, 1, 0)),
    # line buffers in global memory: for the long bin, and for every bin
    dict(edges=(128,), lines_per_tile=(256, 256), large_lds=(0, 2)),
    dict(edges=(64, 256), lines_per_tile=(256, 128, 64), large_lds=(2, 2, 2)),
]


@pytest.fixture(scope="module")
def zs():
    import paper_2404_19391_amd as zs
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return zs


@pytest.fixture(scope="module")
def gd(zs):
    return zs.Dict.load()


def dev(buf, off):
    return (torch.from_numpy(np.ascontiguousarray(buf, dtype=np.uint8)).cuda(),
            torch.from_numpy(np.ascontiguousarray(off).astype(np.int64)).cuda())


def host(t):
    return t.cpu().numpy()


def _check(zs, gd, odict, buf, off, cfgs=CONFIGS, preprocess=True):
    code, fb, want, woff = oracle.compress(odict, buf, off, preprocess=preprocess)
    b, o = dev(buf, off)
    for c in cfgs:
        cfg = zs.BinConfig.make(**c)
        got, goff = zs.compress_binned(gd, b, o, cfg, preprocess=preprocess, check=False)
        torch.cuda.synchronize()
        assert np.array_equal(host(goff).astype(np.uint64), woff), c
        assert host(got).tobytes() == want.tobytes(), c
    return code, fb


@pytest.mark.parametrize("preset,seed,n", [("uneven", 91, 4000), ("test", 92, 3000), ("long", 93, 500),
                                           ("small", 94, 3000)])
def test_binned_presets(zs, gd, odict, preset, seed, n):
    code, _ = _check(zs, gd, odict, *smilesgen.generate(preset, seed, n))
    assert code == oracle.OK


def test_binned_preprocess_off(zs, gd, odict):
    _check(zs, gd, odict, *smilesgen.generate("uneven", 95, 2000), preprocess=False)


def test_binned_edge_lines(zs, gd, odict):
    from test_gpu_codec import _edge_lines
    buf, off = oracle.join_lines(_edge_lines())
    _check(zs, gd, odict, buf, off)


def _ring_lines(seed, n):
    """Lines of ring labels only: up to 40 rings open at once (IDs past 31), labels
    opened and closed in either form ('5' / '%05'), repeated back to back, and
    some lines left with rings open (malformed) between well-formed ones."""
    rng = np.random.default_rng(seed)
    lines = []
    for _ in range(n):
        parts, open_ = [], []
        cap = int(rng.integers(1, 41))
        for _ in range(int(rng.integers(1, 160))):
            if rng.random() < 0.8:
                parts.append(b"C")
            if open_ and (len(open_) >= cap or rng.random() < 0.45):
                v = open_.pop(int(rng.integers(0, len(open_))))
            else:
                free = [x for x in range(100) if x not in open_]
                v = int(free[int(rng.integers(0, min(len(free), int(rng.integers(1, 101)))))])
                open_.append(v)
            parts.append(b"%d" % v if v < 10 and rng.random() < 0.8 else b"%%%02d" % v)
        if rng.random() < 0.85:
            while open_:
                parts.append(b"C")
                v = open_.pop()
                parts.append(b"%d" % v if v < 10 and rng.random() < 0.5 else b"%%%02d" % v)
        lines.append(b"".join(parts))
    return lines


def test_binned_ring_tables(zs, gd, odict):
    """Ring IDs of the global-memory layout (label tables, latest close per ID)
    against the oracle, over several tiles per workgroup."""
    lines = _ring_lines(97, 3000)
    assert max(len(x) for x in lines) <= 4096
    buf, off = oracle.join_lines(lines)
    _check(zs, gd, odict, buf, off, cfgs=[dict(edges=(), large_lds=(2,)), CONFIGS[4], dict(edges=())])


def test_binned_many_tiles(zs, gd, odict):
    """The uneven mix at 60,000 lines: hundreds of tiles in each bin."""
    _check(zs, gd, odict, *smilesgen.generate("uneven", 96, 60000), cfgs=CONFIGS[1:3])


def test_binned_repeated_calls_agree(zs, gd, odict):
    """300,000 uneven lines (thousands of tiles, long-line bins that take several
    batches) compressed ten times in a row with one workspace: every call gives the
    plain compressor's bytes and offsets (a regression test for tiles placed with
    stale bytes under load)."""
    buf, off = smilesgen.generate("uneven", 97, 300000)
    b, o = dev(buf, off)
    want, woff = zs.compress(gd, b, o)
    cfg = zs.BinConfig.make(edges=(128,), lines_per_tile=(256, 256), large_lds=(0, 0))
    total = int(host(woff)[-1])
    ws = torch.empty(zs.binned_workspace_bytes(300000, total), dtype=torch.uint8, device="cuda")
    out = torch.empty(total + 16, dtype=torch.uint8, device="cuda")
    ooff = torch.empty(300001, dtype=torch.int64, device="cuda")
    res = zs.new_result()
    for _ in range(10):
        out.fill_(0)
        zs.compress_binned_into(gd, b, o, out, ooff, cfg, ws, res)
        torch.cuda.synchronize()
        assert zs.read_result(res)[0] == 0
        assert torch.equal(ooff, woff)
        assert torch.equal(out[:total], want)


def test_binned_errors_and_sizes(zs, gd, odict):
    lines = [b"CCO", b"C\tC", b"c1ccccc1", b"N\x7f", b"C" * 4097, b"CC"] * 50 + [b"C" * 900, b"\xff"]
    buf, off = oracle.join_lines(lines)
    b, o = dev(buf, off)
    n = len(lines)
    ws_p = zs.Workspaces().get(zs.OP_COMPRESS, n)
    sizes = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    res = zs.new_result()
    zs.compress_into(gd, b, o, None, sizes, ws_p, res)
    plain_res = zs.read_result(res)
    total = int(sizes[-1].item())
    for c in CONFIGS:
        cfg = zs.BinConfig.make(**c)
        ws = torch.empty(zs.binned_workspace_bytes(n, total), dtype=torch.uint8, device="cuda")
        oo = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        res = zs.new_result()
        zs.compress_binned_into(gd, b, o, None, oo, cfg, ws, res)
        assert zs.read_result(res) == plain_res
        assert torch.equal(oo, sizes)
        out = torch.empty(total, dtype=torch.uint8, device="cuda")
        res = zs.new_result()
        zs.compress_binned_into(gd, b, o, out, oo, cfg, ws, res)
        assert zs.read_result(res) == plain_res == (oracle.ECORRUPT, 1)
        code, fb, want, woff = oracle.compress(odict, buf, off)
        g = oracle.split_lines(host(out), host(oo))
        w = oracle.split_lines(want, woff)
        assert all(g[i] == w[i] for i in range(n) if len(lines[i]) <= 4096)
    # ENOSPC, no bad line
    good, goff = oracle.join_lines([b"CCO", b"c1ccccc1" * 40] * 300)
    b2, o2 = dev(good, goff)
    n2 = goff.size - 1
    cfg = zs.BinConfig.make(**CONFIGS[1])
    ws = torch.empty(zs.binned_workspace_bytes(n2, 100), dtype=torch.uint8, device="cuda")
    oo = torch.empty(n2 + 1, dtype=torch.int64, device="cuda")
    res = zs.new_result()
    zs.compress_binned_into(gd, b2, o2, torch.empty(100, dtype=torch.uint8, device="cuda"), oo, cfg, ws, res)
    assert zs.read_result(res)[0] == zs.ENOSPC
    code, fb, want, woff = oracle.compress(odict, good, goff)
    assert np.array_equal(host(oo).astype(np.uint64), woff)


def test_binned_graph_replays(zs, gd, odict):
    """The binned call captured in a HIP graph: every replay, with eager work and
    synchronisations between replays, gives the oracle's bytes."""
    buf, off = smilesgen.generate("uneven", 97, 20000)
    code, fb, want, woff = oracle.compress(odict, buf, off)
    b, o = dev(buf, off)
    n = off.size - 1
    total = int(woff[-1])
    cfg = zs.BinConfig.make(**CONFIGS[2])
    ws = torch.empty(zs.binned_workspace_bytes(n, total), dtype=torch.uint8, device="cuda")
    out = torch.empty(total, dtype=torch.uint8, device="cuda")
    oo = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    res = zs.new_result()
    s = torch.cuda.Stream()
    g = zs.Graph()
    with torch.cuda.stream(s):
        with g.capture(s):
            zs.compress_binned_into(gd, b, o, out, oo, cfg, ws, res)
    for rep in range(3):
        out.fill_(0)
        oo.fill_(-1)
        res.fill_(7)
        torch.cuda.synchronize()
        g.replay(s)
        s.synchronize()
        assert zs.read_result(res) == (0, -1), rep
        assert np.array_equal(host(oo).astype(np.uint64), woff), rep
        assert host(out).tobytes() == want.tobytes(), rep
        # eager work between replays
        e, eo = zs.compress(gd, b, o)
        assert torch.equal(e, out)
    del g


def test_plain_graph_replays(zs, gd, odict):
    buf, off = smilesgen.generate("bulk", 98, 20000)
    code, fb, want, woff = oracle.compress(odict, buf, off)
    b, o = dev(buf, off)
    n = off.size - 1
    ws = zs.Workspaces().get(zs.OP_COMPRESS, n)
    out = torch.empty(int(woff[-1]), dtype=torch.uint8, device="cuda")
    oo = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    res = zs.new_result()
    s = torch.cuda.Stream()
    g = zs.Graph()
    with torch.cuda.stream(s):
        with g.capture(s):
            zs.compress_into(gd, b, o, out, oo, ws, res)
    for rep in range(3):
        out.fill_(0)
        torch.cuda.synchronize()
        g.replay(s)
        s.synchronize()
        assert zs.read_result(res) == (0, -1)
        assert host(out).tobytes() == want.tobytes(), rep
        assert np.array_equal(host(oo).astype(np.uint64), woff)


def test_autotune(zs, gd, odict):
    buf, off = smilesgen.generate("uneven", 99, 30000)
    b, o = dev(buf, off)
    cfg, best_ms, plain_ms, tried = zs.autotune_binned(gd, b, o)
    assert tried >= 10 and best_ms > 0 and plain_ms > 0
    d = cfg.as_dict()
    assert 1 <= d["nbins"] <= zs.MAX_BINS
    code, fb, want, woff = oracle.compress(odict, buf, off)
    got, goff = zs.compress_binned(gd, b, o, cfg)
    assert host(got).tobytes() == want.tobytes()
    assert np.array_equal(host(goff).astype(np.uint64), woff)
