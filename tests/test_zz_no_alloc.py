"""The allocation-free random-access entry point (zs_decompress_lines_noalloc, for
callers that cannot allocate) against zs_decompress_lines, byte for byte, through the
C ABI: two calls in a row on the library's static scratch, the second smaller (its
tiles and result word must not keep anything of the first), plus a bad request and
the host-side rejection of a request set above the scratch's limit."""
import numpy as np
import pytest

import smilesgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def zs():
    import paper_2404_19391_amd as zs
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return zs


def _with_workspace(zs, d, c, co, ids):
    out_off = torch.empty(ids.numel() + 1, dtype=torch.int64, device="cuda")
    ws = torch.empty(max(zs.workspace_bytes(zs.OP_DECOMPRESS_LINES, ids.numel()), 64), dtype=torch.uint8,
                     device="cuda")
    res = zs.new_result()
    zs.decompress_lines_into(d, c, co, ids, None, out_off, ws, res)
    total = int(out_off[-1].item())
    out = torch.empty(max(total, 1), dtype=torch.uint8, device="cuda")
    res = zs.new_result()
    zs.decompress_lines_into(d, c, co, ids, out, out_off, ws, res)
    torch.cuda.synchronize()
    return out[:total].cpu().numpy().tobytes(), out_off.cpu().numpy(), zs.read_result(res)


def _without_workspace(zs, d, c, co, ids):
    out_off = torch.full((ids.numel() + 1,), -7, dtype=torch.int64, device="cuda")
    res = zs.new_result()
    zs.decompress_lines_noalloc_into(d, c, co, ids, None, out_off, res)
    total = int(out_off[-1].item())
    out = torch.empty(max(total, 1), dtype=torch.uint8, device="cuda")
    res = zs.new_result()
    zs.decompress_lines_noalloc_into(d, c, co, ids, out, out_off, res)
    torch.cuda.synchronize()
    return out[:total].cpu().numpy().tobytes(), out_off.cpu().numpy(), zs.read_result(res)


def test_noalloc_matches_workspace_call(zs):
    d = zs.Dict.load()
    buf, off = smilesgen.generate("bulk", 71, 300000)
    b = torch.from_numpy(buf).cuda()
    o = torch.from_numpy(off.astype(np.int64)).cuda()
    c, co = zs.compress(d, b, o)
    n = off.size - 1
    rng = np.random.default_rng(72)
    # first call: 200,000 ids (tiles of 256), one of them out of range
    ids1 = rng.integers(0, n, 200000).astype(np.int64)
    ids1[123457] = n + 5
    # second call, smaller: 700 ids (tiles of 32), all valid
    ids2 = rng.integers(0, n, 700).astype(np.int64)
    for ids_np, want_code, want_bad in ((ids1, zs.EINVAL, 123457), (ids2, zs.OK, -1)):
        print("noalloc call: %d ids" % ids_np.size, flush=True)
        ids = torch.from_numpy(ids_np).cuda()
        w_bytes, w_off, w_res = _with_workspace(zs, d, c, co, ids)
        g_bytes, g_off, g_res = _without_workspace(zs, d, c, co, ids)
        assert w_res == (want_code, want_bad)
        assert g_res == w_res
        assert np.array_equal(g_off, w_off)
        assert g_bytes == w_bytes


def test_noalloc_rejects_more_ids_than_its_scratch(zs):
    d = zs.Dict.load()
    buf, off = smilesgen.generate("small", 73, 100)
    b = torch.from_numpy(buf).cuda()
    o = torch.from_numpy(off.astype(np.int64)).cuda()
    c, co = zs.compress(d, b, o)
    ids = torch.zeros(4, dtype=torch.int64, device="cuda")
    out_off = torch.empty(5, dtype=torch.int64, device="cuda")
    res = zs.new_result()
    # rejected on the host before anything is enqueued: no kernel reads past the 4 ids
    with pytest.raises(zs.ZsError) as e:
        zs.decompress_lines_noalloc_into(d, c, co, ids, None, out_off, res, n_ids=zs.NOALLOC_MAX_IDS + 1)
    assert e.value.code == zs.EINVAL
