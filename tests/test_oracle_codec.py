"""Pins of the oracle's compression and decompression (Sec. IV-D) to things other than
itself: exhaustive enumeration of parses and an explicit Dijkstra on the graph G
(oracle/brute.py), closed forms, the decoder definition, round trips, and the invariants
the paper states (one SMILES per line, readable output, no expansion with a pre-populated
dictionary; Sec. I, Sec. IV-B)."""
import itertools
import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import brute

SMILES_ALPHABET = b"BCNOPSFIHlrbcnops0123456789[]+-%=#$:/\\().@*"


def _rand_dict(rnd, alphabet, n_entries, max_len, codes=b"ABDEGJKLMQRTUVWXYZ"):
    entries = {}
    seen = set()
    for c in codes[:n_entries]:
        while True:
            L = rnd.randint(1, max_len)
            e = bytes(rnd.choice(alphabet) for _ in range(L))
            if e not in seen:
                seen.add(e)
                entries[c] = e
                break
    return entries


def test_exhaustive_small_alphabet_matches_brute_force():
    rnd = random.Random(1)
    alphabet = b"abc"
    for trial in range(12):
        entries = _rand_dict(rnd, alphabet, rnd.randint(1, 7), 4)
        d = oracle.Dict(entries)
        assert d.valid
        for n in range(0, 7):
            for t in itertools.product(alphabet, repeat=n):
                s = bytes(t)
                got = oracle.compress_line(d, s, preprocess=False)
                assert got == brute.brute_compress(entries, s), (entries, s)


def test_random_strings_match_brute_force_and_dijkstra():
    rnd = random.Random(2)
    for trial in range(150):
        alphabet = b"abcd"[:rnd.randint(2, 4)]
        entries = _rand_dict(rnd, alphabet, rnd.randint(0, 8), 4)
        d = oracle.Dict(entries)
        s = bytes(rnd.choice(alphabet) for _ in range(rnd.randint(0, 11)))
        got = oracle.compress_line(d, s, preprocess=False)
        assert len(got) == brute.dijkstra_cost(entries, s)
        if len(s) <= 9:
            assert got == brute.brute_compress(entries, s), (entries, s)
        assert brute.decompress_ref(entries, got) == s


def test_closed_form_identity_only_dictionary():
    d = oracle.Dict({c: bytes([c]) for c in SMILES_ALPHABET})
    import smilesgen
    for x in smilesgen.lines("test", 21, 300):
        assert oracle.compress_line(d, x) == oracle.preprocess(x)


def test_closed_form_empty_dictionary_escapes_everything():
    d = oracle.Dict({})
    assert d.valid
    s = b"CC(=O)N"
    assert oracle.compress_line(d, s, preprocess=False) == b"".join(b" " + bytes([c]) for c in s)


@pytest.mark.parametrize("n", range(0, 14))
def test_closed_form_runs_of_one_letter(n):
    # only {C, CC, CCC}: C^n takes ceil(n/3) codes, longest first (3, 3, ..., remainder)
    d = oracle.Dict({ord("x"): b"C", ord("y"): b"CC", ord("z"): b"CCC"})
    want = b"z" * (n // 3) + {0: b"", 1: b"x", 2: b"y"}[n % 3]
    assert oracle.compress_line(d, b"C" * n, preprocess=False) == want


def test_tie_break_prefers_longest_first_edge():
    # "abcd": {ab, cd, a, bcd} -> both (ab, cd) and (a, bcd) cost 2; T1 takes ab first.
    d = oracle.Dict({ord("P"): b"ab", ord("Q"): b"cd", ord("R"): b"a", ord("S"): b"bcd"})
    assert oracle.compress_line(d, b"abcd", preprocess=False) == b"PQ"
    # escape (cost 2) ties with a longer edge: the longer edge is taken
    d = oracle.Dict({ord("P"): b"ab", ord("Q"): b"b"})
    assert oracle.compress_line(d, b"ab", preprocess=False) == b"P"


def test_decoder_definition():
    d = oracle.Dict({ord("C"): b"C", ord("X"): b"c1ccc", ord(" ") + 0x81: b"(=O)"})
    assert oracle.decompress_line(d, b"CXC") == b"Cc1cccC"
    assert oracle.decompress_line(d, b"\xa1C") == b"(=O)C"
    # escape parity: "  C" = escaped space then code C; "   C" = escaped space, escaped C
    assert oracle.decompress_line(d, b"  C") == b" C"
    assert oracle.decompress_line(d, b"   C") == b" C"
    assert oracle.decompress_line(d, b"    C") == b"  C"
    assert oracle.decompress_line(d, b" a") == b"a"
    assert oracle.decompress_line(d, b"C ") is None          # dangling escape
    assert oracle.decompress_line(d, b"Z") is None           # not a code
    assert oracle.decompress_line(d, b" \n") is None         # literal outside 0x20..0x7E
    assert oracle.decompress_line(d, b"") == b""


def _allowed_out(b):
    return b == 0x0A or 0x20 <= b <= 0x7E or 0xA1 <= b <= 0xFF


@pytest.mark.parametrize("preset,seed,n", [("small", 1, 2000), ("test", 31, 2000), ("uneven", 32, 300)])
def test_round_trip_and_invariants(odict, preset, seed, n):
    import smilesgen
    buf, off = smilesgen.generate(preset, seed, n)
    code, fb, out, oo = oracle.compress(odict, buf, off)
    assert code == oracle.OK and fb == -1
    # one output line per input line, in order, no newline inside a line (Sec. I)
    assert int((out == 0x0A).sum()) == n
    assert np.all(out[oo[1:].astype(np.int64) - 1] == 0x0A)
    assert all(_allowed_out(int(b)) for b in np.unique(out))
    raw = oracle.split_lines(buf, off)
    comp = oracle.split_lines(out, oo)
    for x, c in zip(raw, comp):
        p = oracle.preprocess(x)
        # with every character pre-populated, never longer than the input (Sec. IV-B)
        assert len(c) <= len(p)
        assert oracle.decompress_line(odict, c) == p
    code, fb, back, bo = oracle.decompress(odict, out, oo)
    assert code == oracle.OK
    assert back.tobytes() == b"".join(oracle.preprocess(x) + b"\n" for x in raw)
    # without pre-processing the round trip is the identity
    code, fb, out2, oo2 = oracle.compress(odict, buf, off, preprocess=False)
    code, fb, back2, _ = oracle.decompress(odict, out2, oo2)
    assert back2.tobytes() == buf.tobytes()


@settings(max_examples=300, deadline=None)
@given(st.lists(st.binary(min_size=0, max_size=40).map(lambda b: bytes(32 + (c % 95) for c in b)),
                min_size=0, max_size=8))
def test_round_trip_any_printable(lines):
    d = oracle.Dict.load(__import__("conftest").DEFAULT_DICT)
    buf, off = oracle.join_lines(lines)
    for pre in (True, False):
        code, fb, out, oo = oracle.compress(d, buf, off, preprocess=pre)
        assert code == oracle.OK
        code, fb, back, _ = oracle.decompress(d, out, oo)
        assert code == oracle.OK
        want = [oracle.preprocess(x) if pre else x for x in lines]
        assert oracle.split_lines(back, _) == want
        assert all(_allowed_out(int(b)) for b in out)


def test_spaces_in_input_are_escaped(odict):
    c = oracle.compress_line(odict, b"C C", preprocess=False)
    assert c == b"C  C"
    assert oracle.decompress_line(odict, c) == b"C C"
    assert oracle.compress_line(odict, b"   ", preprocess=False) == b"      "


def test_errors_and_framing(odict):
    lines = [b"CCO", b"C\tC", b"c1ccccc1", b"N\x7f"]
    buf, off = oracle.join_lines(lines)
    code, fb, out, oo = oracle.compress(odict, buf, off)
    assert code == oracle.ECORRUPT and fb == 1
    comp = oracle.split_lines(out, oo)
    assert comp[1] == b"" and comp[3] == b""
    assert oracle.decompress_line(odict, comp[0]) == b"CCO"
    # a line whose terminator is missing -> EINVAL at that line
    buf2 = buf.copy()
    buf2[int(off[1]) - 1] = ord("C")
    code, fb, _, _ = oracle.compress(odict, buf2, off)
    assert code == oracle.EINVAL and fb == 0
    # virtual newline for an unterminated last line
    raw = np.frombuffer(b"CCO\nc1ccccc1", dtype=np.uint8).copy()
    off3 = oracle.index_lines(raw)
    assert list(off3) == [0, 4, 13]
    code, fb, out3, oo3 = oracle.compress(odict, raw, off3)
    assert code == oracle.OK and oracle.split_lines(out3, oo3)[1] == oracle.compress_line(odict, b"c1ccccc1")
    # ENOSPC, and size-only mode
    code, fb, out4, oo4 = oracle.compress(odict, buf, off, out_cap=3)
    assert code == oracle.ECORRUPT  # data errors win over ENOSPC
    good, goff = oracle.join_lines([b"CCO", b"c1ccccc1"])
    code, fb, _, oo5 = oracle.compress(odict, good, goff, out_cap=3)
    assert code == oracle.ENOSPC
    code, fb, _, oo6 = oracle.compress(odict, good, goff, size_only=True)
    assert code == oracle.OK and list(oo6) == list(oo5)


def test_decompress_errors(odict):
    lines = [b"CC", b"C ", b"\x80", b"C"]
    buf, off = oracle.join_lines(lines)
    code, fb, out, oo = oracle.decompress(odict, buf, off)
    assert code == oracle.ECORRUPT and fb == 1
    assert oracle.split_lines(out, oo) == [b"CC", b"", b"", b"C"]


def test_random_access_equals_rows_of_full_decompression(odict):
    import smilesgen
    buf, off = smilesgen.generate("bulk", 41, 3000)
    _, _, c, co = oracle.compress(odict, buf, off)
    _, _, full, fo = oracle.decompress(odict, c, co)
    rows = oracle.split_lines(full, fo)
    rnd = np.random.default_rng(3)
    ids = np.concatenate([rnd.integers(0, 3000, 500), np.arange(100, 140), [0, 2999, 7, 7]]).astype(np.uint64)
    code, fb, out, oo = oracle.decompress_lines(odict, c, co, ids)
    assert code == oracle.OK
    assert oracle.split_lines(out, oo) == [rows[int(i)] for i in ids]
    code, fb, out, oo = oracle.decompress_lines(odict, c, co, np.array([5, 3000, 9, 4000], dtype=np.uint64))
    assert code == oracle.EINVAL and fb == 1
    code, fb, out, oo = oracle.decompress_lines(odict, c, co, np.zeros(0, dtype=np.uint64))
    assert code == oracle.OK and list(oo) == [0]


def test_index_lines_matches_split():
    rnd = random.Random(4)
    for _ in range(200):
        parts = [bytes(rnd.choice(b"C\n") for _ in range(rnd.randint(0, 6))) for _ in range(rnd.randint(0, 5))]
        data = b"".join(parts)
        off = oracle.index_lines(np.frombuffer(data, dtype=np.uint8))
        pieces = data.split(b"\n")
        if data.endswith(b"\n") or data == b"":
            pieces = pieces[:-1]
        assert len(off) == len(pieces) + 1
        for k, p in enumerate(pieces):
            assert data[int(off[k]):int(off[k]) + len(p)] == p
        if data and not data.endswith(b"\n"):
            assert int(off[-1]) == len(data) + 1


def test_dictionary_validation():
    ok = {ord("C"): b"C", 0xA1: b"CC"}
    assert oracle.Dict(ok).valid
    assert not oracle.Dict({0x20: b"C"}).valid                 # space is the escape
    assert not oracle.Dict({0x0A: b"C"}).valid                 # newline is the separator
    assert not oracle.Dict({0x85: b"C"}).valid                 # C1 control range
    assert not oracle.Dict({ord("A"): b"C C"}).valid           # expansion byte outside 0x21..0x7E
    assert not oracle.Dict({ord("A"): b"C", ord("B"): b"C"}).valid  # duplicate expansion
    assert not oracle.Dict({ord("A"): b"C" * 17}).valid        # longer than 16
    assert not oracle.Dict({ord("A"): b""}).valid              # empty
    assert oracle.Dict({ord("A"): b"C" * 16}).valid
