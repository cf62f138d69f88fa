"""Host-side checks of libzsmiles.so that need no GPU: the exported C ABI, dictionary
validation, and the compiled match automaton (the tables the kernels stage in LDS).

The automaton test walks each line backwards through the compiled transition table
and compares the pattern set it reports at every position with a direct check of
every dictionary entry (Sec. IV-D-1: the edges that leave node i).  The parse test
replays the kernel's (min,+) key recurrence over those tables and compares the result
with the oracle."""
import ctypes
import os
import random
import re
import struct

import numpy as np
import pytest

import paper_2404_19391_amd as zs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zsmiles.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(zs_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = zs.lib()
    names = _declared_functions()
    assert {"zs_compress", "zs_decompress", "zs_decompress_lines", "zs_index_lines",
            "zs_dict_create"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    assert zs.status_str(0) == "ok"
    assert "fit" in zs.status_str(zs.ENOSPC)


def test_workspace_sizes_grow_with_n():
    a = zs.workspace_bytes(zs.OP_COMPRESS, 1000)
    b = zs.workspace_bytes(zs.OP_COMPRESS, 10_000_000)
    assert 0 < a < b
    assert zs.workspace_bytes(zs.OP_DECOMPRESS, 10) > 0
    assert zs.workspace_bytes(zs.OP_INDEX, 1 << 20) > 0


@pytest.mark.parametrize("entries", [
    {0x20: b"C"}, {0x0A: b"C"}, {0x90: b"C"}, {ord("A"): b"C C"}, {ord("A"): b"C", ord("B"): b"C"},
    {ord("A"): b"C" * 17}, {0xFF: b"\x80C"},
])
def test_dict_create_rejects_invalid(entries):
    ln = np.zeros(256, dtype=np.uint8)
    ex = np.zeros((256, 16), dtype=np.uint8)
    for c, e in entries.items():
        ln[c] = min(len(e), 255)
        ex[c, :min(len(e), 16)] = np.frombuffer(e[:16], dtype=np.uint8)
    h = ctypes.c_void_p()
    rc = zs.lib().zs_dict_create(ln.ctypes.data_as(ctypes.c_void_p), ex.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(h))
    assert rc == zs.EINVAL


class Tables:
    """Reader of the compiled image (layout of csrc/zs_tables.hpp)."""

    def __init__(self, blob):
        h = struct.unpack_from("<16I", blob, 0)
        (self.lmax, self.lk, self.S, self.C, o_len, o_col, o_code1, o_trans, o_outk, o_code, o_exp,
         self.size, self.ncodes) = h[:13]
        assert self.size == len(blob)
        b = np.frombuffer(blob, dtype=np.uint8)
        self.len = b[o_len:o_len + 256]
        self.col = b[o_col:o_col + 256]
        self.code1 = b[o_code1:o_code1 + 256]
        self.trans = np.frombuffer(blob, dtype=np.uint16, count=self.S * self.C, offset=o_trans).reshape(self.S, self.C)
        # signed bytes: 31 - L, or -1 (as a 32-bit key mask: 0xFFFFFFFF) where no pattern of length L starts
        self.outk = (np.frombuffer(blob, dtype=np.int8, count=self.S * self.lk, offset=o_outk).astype(np.int64)
                     & 0xFFFFFFFF).astype(np.uint32).reshape(self.S, self.lk)
        self.code = b[o_code:o_code + self.S * self.lk].reshape(self.S, self.lk)
        self.exp = b[o_exp:o_exp + 256 * 16].reshape(256, 16)

    def walk(self, s):
        """States after consuming s[i] when reading s from its end: list indexed by i."""
        st = 0
        states = [0] * len(s)
        for i in range(len(s) - 1, -1, -1):
            st = int(self.trans[st, self.col[s[i]]])
            states[i] = st
        return states

    def parse(self, s):
        """The kernel's backward recurrence on keys (cost << 5 | 31 - L)."""
        INF = 0xFFFFFFFF
        lk = self.lk
        V = [32] + [INF] * (lk - 1)
        toks = [None] * len(s)
        st = 0
        for i in range(len(s) - 1, -1, -1):
            c = s[i]
            st = int(self.trans[st, self.col[c]])
            K = V[0] + 63
            for k in range(lk):
                K = min(K, (V[k] | int(self.outk[st, k])) & INF)
            ch = 31 - (K & 31)
            if ch == 0:
                toks[i] = (True, c)
            elif ch == 1:
                toks[i] = (False, int(self.code1[c]))
            else:
                toks[i] = (False, int(self.code[st, ch - 1]))
            V = [(K | 31) + 1] + V[:-1]
        out = bytearray()
        i = 0
        while i < len(s):
            esc, t = toks[i]
            if esc:
                out += bytes([32, t])
                i += 1
            else:
                out.append(t)
                i += int(self.len[t])
        return bytes(out), (V[0] >> 5) - 1


def _match_sets_direct(entries, s):
    inv = {bytes(e): c for c, e in entries.items()}
    return [{L: inv[s[i:i + L]] for L in range(1, 17) if i + L <= len(s) and s[i:i + L] in inv}
            for i in range(len(s))]


def _check_automaton(entries, strings):
    t = Tables(zs.compile_tables(entries))
    for s in strings:
        states = t.walk(s)
        direct = _match_sets_direct(entries, s)
        for i, st in enumerate(states):
            got = {L + 1 for L in range(t.lk) if t.outk[st, L] != 0xFFFFFFFF}
            assert got == set(direct[i]), (s, i)
            for L, code in direct[i].items():
                if L == 1:
                    assert t.code1[s[i]] == code
                else:
                    assert t.code[st, L - 1] == code
    return t


def test_automaton_on_default_dictionary():
    import smilesgen
    entries = zs.read_zsd(zs.default_dict_path())
    lines = smilesgen.lines("test", 51, 300) + [b"", b" ", b"C C", b"~~~", b"%%%%"]
    t = _check_automaton(entries, lines)
    assert t.lk == 8 and t.S <= 4096


def test_automaton_random_dictionaries():
    rnd = random.Random(7)
    codes = list(range(0x21, 0x7F)) + list(range(0xA1, 0x100))
    for trial in range(60):
        alphabet = b"abcd()=1"[:rnd.randint(2, 8)]
        ents = {}
        seen = set()
        rnd.shuffle(codes)
        for c in codes[:rnd.randint(1, 30)]:
            L = rnd.randint(1, 12 if trial % 3 == 0 else 5)
            e = bytes(rnd.choice(alphabet) for _ in range(L))
            if e not in seen:
                seen.add(e)
                ents[c] = e
        strings = [bytes(rnd.choice(alphabet + b"xy") for _ in range(rnd.randint(0, 30))) for _ in range(20)]
        _check_automaton(ents, strings)


def test_kernel_recurrence_matches_oracle():
    import oracle
    import smilesgen
    entries = zs.read_zsd(zs.default_dict_path())
    t = Tables(zs.compile_tables(entries))
    od = oracle.Dict(entries)
    for x in smilesgen.lines("test", 52, 400) + [b"C C", b"   ", b"aei", b"[NH+]x"]:
        p = oracle.preprocess(x)
        got, cost = t.parse(p)
        want = oracle.compress_line(od, x)
        assert got == want, x
        assert cost == len(want)
    rnd = random.Random(8)
    for trial in range(40):
        alphabet = b"abc"
        ents = {}
        seen = set()
        for c in rnd.sample(range(0x41, 0x5B), rnd.randint(1, 9)):
            e = bytes(rnd.choice(alphabet) for _ in range(rnd.randint(1, 11)))
            if e not in seen:
                seen.add(e)
                ents[c] = e
        t2 = Tables(zs.compile_tables(ents))
        od2 = oracle.Dict(ents)
        for _ in range(20):
            s = bytes(rnd.choice(alphabet) for _ in range(rnd.randint(0, 25)))
            got, _ = t2.parse(s)
            assert got == oracle.compress_line(od2, s, preprocess=False), (ents, s)


def test_binned_config_validation():
    """zs_compress_binned rejects bad bin configurations on the host, before any device work."""
    import ctypes
    import paper_2404_19391_amd as zs
    L = zs.lib()
    fake = ctypes.c_void_p(16)

    def call(cfg, flags=1, n=10):
        return L.zs_compress_binned(fake, fake, 100, fake, n, fake, 100, fake, flags, ctypes.byref(cfg), fake,
                                    1 << 40, fake, None)

    bad = [zs.BinConfig.make(edges=(128, 128)), zs.BinConfig.make(edges=(256, 128)),
           zs.BinConfig.make(edges=(0,)), zs.BinConfig.make(lines_per_tile=(0,)),
           zs.BinConfig.make(lines_per_tile=(31,)), zs.BinConfig.make(edges=(64,), lines_per_tile=(256, 7)),
           zs.BinConfig.make(lines_per_tile=(257,)), zs.BinConfig.make(large_lds=(3,))]
    for c in bad:
        assert call(c) == zs.EINVAL
    c = zs.BinConfig.make()
    c.nbins = 0
    assert call(c) == zs.EINVAL
    c.nbins = zs.MAX_BINS + 1
    assert call(c) == zs.EINVAL
    assert call(zs.BinConfig.make(), flags=4) == zs.EINVAL
    assert call(zs.BinConfig.make(), n=1 << 32) == zs.EINVAL
    assert L.zs_graph_begin(None) == zs.EINVAL
