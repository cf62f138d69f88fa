"""GPU tests of the request loop (zs_server): every reply equals the oracle's
bytes for the same request, whether the request runs alone or among many
concurrent ones, and whether memory is plentiful or tight (admission by exact
device footprint defers requests but never changes a result)."""
import threading

import numpy as np
import pytest

import oracle
import smilesgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def zs():
    import paper_2404_19391_amd as zs
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return zs


@pytest.fixture(scope="module")
def gd(zs):
    return zs.Dict.load()


@pytest.fixture(scope="module")
def shard(odict):
    """A compressed shard made by the oracle (30,000 lines) and its host copy."""
    buf, off = smilesgen.generate("bulk", 101, 30000)
    code, fb, c, co = oracle.compress(odict, buf, off)
    assert code == oracle.OK
    return c, co


@pytest.fixture(scope="module")
def requests(odict, shard):
    """A seeded mix: decompression requests of 1..5,000 ids (some repeated, one out of
    range), compression requests of 1..3,000 new lines (some bad lines), with the
    oracle's answers."""
    rnd = np.random.default_rng(102)
    c, co = shard
    n = co.size - 1
    pool_buf, pool_off = smilesgen.generate("uneven", 103, 20000)
    reqs = []
    for k in range(40):
        if k % 10 == 3:
            lines = smilesgen.lines("test", 104 + k, int(rnd.integers(1, 300)))
            if k == 13:
                lines[len(lines) // 2] = b"C\x01C"
            buf, off = oracle.join_lines(lines)
            want = oracle.compress(odict, buf, off)
            reqs.append(("c", buf, off, want))
        elif k % 3 == 0:
            m = int(np.exp(rnd.uniform(0, np.log(3000))))
            s0 = int(rnd.integers(0, pool_off.size - 1 - m))
            buf = pool_buf[int(pool_off[s0]):int(pool_off[s0 + m])].copy()
            off = (pool_off[s0:s0 + m + 1] - pool_off[s0]).astype(np.uint64)
            want = oracle.compress(odict, buf, off)
            reqs.append(("c", buf, off, want))
        else:
            m = int(np.exp(rnd.uniform(0, np.log(5000))))
            ids = rnd.integers(0, n, m).astype(np.uint64)
            if k == 7:
                ids[m // 2] = n + 5
            want = oracle.decompress_lines(odict, c, co, ids)
            reqs.append(("d", ids, None, want))
    return reqs


def _submit(srv, sid, r):
    if r[0] == "d":
        return srv.submit_decompress(sid, r[1])
    return srv.submit_compress(r[1], r[2])


def _same(got, want):
    code, fb, data, off, _ = got
    wcode, wfb, wdata, woff = want
    return code == wcode and fb == wfb and np.array_equal(off, woff) and data.tobytes() == wdata.tobytes()


def _server(zs, gd, shard, **kw):
    c, co = shard
    srv = zs.Server(gd, **kw)
    sid = srv.add_shard(torch.from_numpy(c).cuda(), torch.from_numpy(co.astype(np.int64)).cuda())
    return srv, sid


def test_alone_and_in_the_mix(zs, gd, shard, requests):
    srv, sid = _server(zs, gd, shard, slots=8, device_bytes=256 << 20, host_bytes=256 << 20)
    alone = []
    for r in requests:
        got = srv.wait(_submit(srv, sid, r))
        assert _same(got, r[3]), r[0]
        alone.append(got)
    # all at once, from four submitting threads
    tickets = [None] * len(requests)

    def sub(part):
        for i in part:
            tickets[i] = _submit(srv, sid, requests[i])

    th = [threading.Thread(target=sub, args=(range(j, len(requests), 4),)) for j in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, r in enumerate(requests):
        got = srv.wait(tickets[i])
        assert _same(got, r[3]), (i, r[0])
        assert got[2].tobytes() == alone[i][2].tobytes()
    st = srv.stats()
    assert st["completed"] == 2 * len(requests) and st["device_bytes_in_use"] == 0
    srv.close()


def test_tight_memory_agrees(zs, gd, shard, requests):
    """A device arena a few times the biggest request: requests wait for memory
    in arrival order when it is full (how often depends on timing), the arena is
    never exceeded, and every answer is still the oracle's."""
    srv, sid = _server(zs, gd, shard, slots=6, device_bytes=6 << 20, host_bytes=64 << 20)
    tickets = [_submit(srv, sid, r) for r in requests]
    for t, r in zip(tickets, requests):
        assert _same(srv.wait(t), r[3])
    st = srv.stats()
    assert st["peak_device_bytes"] <= 6 << 20
    assert st["completed"] == len(requests) and st["device_bytes_in_use"] == 0
    srv.close()


def test_request_too_large(zs, gd, shard):
    srv, sid = _server(zs, gd, shard, slots=2, device_bytes=2 << 20, host_bytes=64 << 20)
    with pytest.raises(zs.ZsError):
        srv.submit_decompress(sid, np.zeros(400000, dtype=np.uint64))
    srv.close()


def test_output_that_can_never_fit_ends_with_enospc(zs, gd, odict):
    """Inputs that fit the device arena but an output that cannot, even alone: the
    request ends with ZS_ENOSPC (it used to be sized again forever), and the loop
    goes on serving the requests behind it."""
    buf, off = smilesgen.generate("long", 105, 3000)
    code, fb, c, co = oracle.compress(odict, buf, off)
    assert code == oracle.OK
    srv, sid = _server(zs, gd, (c, co), slots=2, device_bytes=1 << 20, host_bytes=64 << 20)
    ids = np.arange(3000, dtype=np.uint64)  # about 1.5 MB of output, 48 KB of stage-1 buffers
    t_big = srv.submit_decompress(sid, ids)
    t_small = srv.submit_decompress(sid, ids[:5])
    got = srv.wait(t_big)
    assert got[0] == zs.ENOSPC and got[2].size == 0 and got[3].size == 0
    want = oracle.decompress_lines(odict, c, co, ids[:5])
    assert _same(srv.wait(t_small), want)
    st = srv.stats()
    assert st["device_bytes_in_use"] == 0
    srv.close()


def test_compress_output_larger_than_input(zs, gd, shard, odict):
    """A compression request whose output is larger than its input (bytes with no code
    are escaped, two bytes each): the first call, into an output the size of the input,
    ends with ZS_ENOSPC and the request runs again at the exact size; the reply is the
    oracle's.  Beside it, a request whose output fits the first call."""
    srv, sid = _server(zs, gd, shard, slots=2, device_bytes=64 << 20, host_bytes=64 << 20)
    big = [b"a" * 50, b"CC(=O)aa", b"", b"x" * 4000] * 50
    small = smilesgen.lines("bulk", 106, 500)
    for lines in (big, small):
        buf, off = oracle.join_lines(lines)
        want = oracle.compress(odict, buf, off)
        got = srv.wait(srv.submit_compress(buf, off))
        assert _same(got, want)
    srv.close()
