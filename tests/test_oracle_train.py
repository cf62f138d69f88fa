"""Pins of the oracle's dictionary trainer (Algorithm 1 with the rank of Eq. (1), Sec. IV-C)
and of the buffer-level pre-processing framing.

The expected pattern lists below are worked out by hand in the comments: substring
counts (overlapping occurrences), the Eq. (1) rank occ * (len - overlap) at every step,
the overlap update (longest common substring with any pattern selected so far) and the
tie-breaks (higher rank, then longer, then bytewise smaller).  The last test plants
plausible mistakes in a temporary copy of the trainer's C source and checks that these
cases catch every one of them.
"""
import os
import shutil
import subprocess
import tempfile
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _train(lines, lmin, lmax, T, preprocess=False, lib=None):
    buf, off = oracle.join_lines(lines)
    if lib is None:
        return oracle.train_patterns(buf, off, T, lmin=lmin, lmax=lmax, preprocess=preprocess)
    # room for a few more patterns than asked: a planted mistake may select too many
    pat = np.zeros((T + 8, 16), dtype=np.uint8)
    plen = np.zeros(T + 8, dtype=np.uint8)
    got = lib.zo_train_dict(buf.ctypes.data_as(ctypes.c_void_p), off.ctypes.data_as(ctypes.c_void_p),
                            ctypes.c_uint64(off.size - 1), 1 if preprocess else 0, lmin, lmax, T,
                            pat.ctypes.data_as(ctypes.c_void_p), plen.ctypes.data_as(ctypes.c_void_p))
    return [pat[i, :plen[i]].tobytes() for i in range(got)]


# Case A: lines "CACCC" and "BA", Lmin 2, Lmax 3, T 4.
#   counts: CA 1, AC 1, CC 2 (positions 2 and 3 of CACCC overlap), CAC 1, ACC 1, CCC 1, BA 1
#   t=0  ranks: CC 2*2=4, CAC/ACC/CCC 3, CA/AC/BA 2                       -> CC
#        overlaps with CC: CA 1, AC 1, BA 0, CAC 1, ACC 2, CCC 2
#   t=1  ranks: CA 1, AC 1, BA 2, CAC 1*(3-1)=2, ACC 1, CCC 1
#        BA and CAC tie at 2 -> the longer one                          -> CAC
#        overlaps with CAC: CA 2, AC 2, BA 1 ("A"), ACC 2 ("AC"), CCC stays 2
#   t=2  ranks: CA 0, AC 0, BA 1, ACC 1, CCC 1
#        BA, ACC, CCC tie at 1 -> longer (ACC, CCC) -> bytewise smaller   -> ACC
#        overlaps with ACC: BA stays 1, CCC stays 2
#   t=3  ranks: BA 1, CCC 1 -> longer                                     -> CCC
CASE_A = ([b"CACCC", b"BA"], 2, 3, 4, [b"CC", b"CAC", b"ACC", b"CCC"])

# Case B: lines "AA" and "CCBBB", Lmin 2, Lmax 3, T 4.
#   counts: AA 1, CC 1, CB 1, BB 2, CCB 1, CBB 1, BBB 1
#   t=0  ranks: BB 4, CCB/CBB/BBB 3, AA/CC/CB 2                            -> BB
#        overlaps with BB: CB 1, CCB 1, CBB 2, BBB 2, AA 0, CC 0
#   t=1  ranks: AA 2, CC 2, CB 1, CCB 2, CBB 1, BBB 1 -> tie at 2, longer  -> CCB
#        overlaps with CCB: CC 2, CB 2, CBB 2 ("CB"), BBB stays 2, AA 0
#   t=2  ranks: AA 2, CC 0, CB 0, CBB 1, BBB 1                            -> AA
#   t=3  ranks: CBB 1, BBB 1 -> same length -> bytewise smaller            -> BBB
CASE_B = ([b"AA", b"CCBBB"], 2, 3, 4, [b"BB", b"CCB", b"AA", b"BBB"])

# Case C: one line "CCCCC", Lmin 2, Lmax 3, T 2.
#   counts: CC 4, CCC 3 (overlapping occurrences)
#   t=0  ranks: CC 8, CCC 9                                                -> CCC
#        overlap of CC with CCC: 2 -> rank 4 * (2 - 2) = 0
#   t=1  no candidate with a positive rank: the loop stops with one pattern
CASE_C = ([b"CCCCC"], 2, 3, 2, [b"CCC"])

# Case D: lines "AB" x3 and "XYZ", Lmin 2, Lmax 3, T 1.
#   counts: AB 3, XY 1, YZ 1, XYZ 1; ranks AB 6, XYZ 3, XY 2, YZ 2         -> AB
CASE_D = ([b"AB", b"AB", b"AB", b"XYZ"], 2, 3, 1, [b"AB"])

# Case E: lines "XYZ", "XYZ", "XY", Lmin 2, Lmax 3, T 2.
#   counts: XY 3, YZ 2, XYZ 2; ranks XY 6, XYZ 6, YZ 4 -> tie, longer     -> XYZ
#   overlaps with XYZ: XY 2, YZ 2 -> ranks 0: the loop stops
CASE_E = ([b"XYZ", b"XYZ", b"XY"], 2, 3, 2, [b"XYZ"])

HAND_CASES = {"A": CASE_A, "B": CASE_B, "C": CASE_C, "D": CASE_D, "E": CASE_E}


@pytest.mark.parametrize("name", sorted(HAND_CASES))
def test_trainer_hand_worked(name):
    lines, lmin, lmax, T, want = HAND_CASES[name]
    assert _train(lines, lmin, lmax, T) == want


def test_trainer_counts_overlapping_occurrences():
    # "CCCCC": CC occurs 4 times overlapping (2 without overlap), CCC 3 times (1):
    # only overlapping counts make CCC (3*3=9) beat CC (4*2=8)
    assert _train([b"CCCCC"], 2, 3, 1) == [b"CCC"]


def test_trainer_rank_uses_length_and_occurrences():
    # Case D: by occurrences alone AB wins as well, by length alone XYZ would;
    # Case C: by occurrences alone CC (4) would beat CCC (3)
    assert _train(*CASE_D[:4]) == [b"AB"]
    assert _train(*CASE_C[:4]) == [b"CCC"]


def test_trainer_overlap_is_longest_common_substring_with_all_selected():
    # Case A, t=1: CAC is reduced by its common substring "C" with CC (a common
    # prefix or suffix would also give 1 here), and at t=2 ACC keeps the overlap 2
    # it got from CC even though its overlap with the newest pattern CAC is 2 too;
    # at t=3 CCC must keep overlap 2 from CC although its overlap with ACC is 2 and
    # with CAC only 1 - with the overlap of the last pattern alone it would
    # still be ahead of BA at t=2.
    assert _train(*CASE_A[:4]) == CASE_A[4]
    # "XAB" shares the substring "AB" with the selected "AB" (no common prefix):
    # counts AB 5, XA 2, XAB 2, QR 1, RS 1, QRS 1 -> t0 AB (10); then XAB 2*(3-2)=2,
    # XA 2*(2-1)=2, QRS 3 -> t1 QRS (with a prefix overlap, XAB would keep 6)
    got = _train([b"AB", b"AB", b"AB", b"XAB", b"XAB", b"QRS"], 2, 3, 2)
    assert got == [b"AB", b"QRS"]


def test_trainer_tie_breaks():
    # equal rank and length: the bytewise smaller first
    assert _train([b"AB", b"BA"], 2, 2, 1) == [b"AB"]
    # equal rank: the longer first (Case E)
    assert _train(*CASE_E[:4]) == [b"XYZ"]


def test_trainer_stops_at_T_and_when_nothing_ranks():
    assert _train([b"CACCC", b"BA"], 2, 3, 2) == [b"CC", b"CAC"]
    assert _train([b"AB"], 2, 2, 5) == [b"AB"]
    assert _train([b"A", b""], 2, 3, 3) == []
    assert _train([b"ABAB"], 2, 2, 0) == []


def test_trainer_pre_processes_when_asked():
    # "C1CCC1" pre-processes to "C0CCC0" (one ring, ID 0, Sec. IV-A):
    # C0 2, 0C 1, CC 2 -> C0 and CC tie at 4 -> "C0" < "CC"
    assert _train([b"C1CCC1"], 2, 2, 1, preprocess=True) == [b"C0"]
    # without pre-processing: C1 2, 1C 1, CC 2 -> "C1" < "CC"
    assert _train([b"C1CCC1"], 2, 2, 1, preprocess=False) == [b"C1"]


def test_trainer_single_characters_and_long_patterns():
    # Lmin 1 (no pre-population): "CCO": C 2, O 1, CC 1, CO 1 -> C, CC and CO tie at 2,
    # CC and CO are longer, "CC" < "CO"
    assert _train([b"CCO"], 1, 2, 1) == [b"CC"]
    # patterns of 16 bytes: every substring of the line occurs twice, so the rank is
    # 2 * length and the whole 16-byte line wins
    line = b"ABCDEFGHIJKLMNOP"
    assert _train([line, line], 2, 16, 1) == [line]
    assert _train([line + b"Q", line + b"Q"], 2, 15, 1) == [line[:15]]


def test_trainer_rejects_bad_parameters():
    buf, off = oracle.join_lines([b"ABC"])
    with pytest.raises(RuntimeError):
        oracle.train_patterns(buf, off, 1, lmin=2, lmax=17)
    with pytest.raises(RuntimeError):
        oracle.train_patterns(buf, off, 1, lmin=3, lmax=2)
    with pytest.raises(RuntimeError):
        oracle.train_patterns(buf, off, 1, lmin=0, lmax=2)


# Planted mistakes: (name, text in train_dict.c, replacement).  Each one must make at
# least one hand-worked case fail.
MUTANTS = [
    ("rank by occurrences only", "(int64_t)((int)c[i].len - overlap[i])", "(int64_t)1"),
    ("rank by length only", "(int64_t)c[i].occ * (int64_t)((int)c[i].len - overlap[i])",
     "(int64_t)((int)c[i].len - overlap[i])"),
    ("no overlap update", "if (l > overlap[i]) overlap[i] = l;", "(void)l;"),
    ("overlap of the last pattern only", "if (l > overlap[i]) overlap[i] = l;", "overlap[i] = l;"),
    ("overlap from aligned positions only", "c[i][j] = (a[i - 1] == b[j - 1]) ? c[i - 1][j - 1] + 1 : 0;",
     "c[i][j] = (a[i - 1] == b[j - 1] && i == j) ? c[i - 1][j - 1] + 1 : 0;"),
    ("shorter first on equal rank", "return p1->len > p2->len;", "return p1->len < p2->len;"),
    ("bytewise larger first", "return memcmp(p1->b, p2->b, p1->len) < 0;",
     "return memcmp(p1->b, p2->b, p1->len) > 0;"),
    ("T + 1 selections", "for (int t = 0; t < T; t++) {", "for (int t = 0; t <= T; t++) {"),
    ("Lmax excluded", "L <= lmax && i + L <= m", "L < lmax && i + L <= m"),
    ("occurrences overlapping the previous one not counted", "tab[h].occ++;",
     "if (!(i >= 1 && memcmp(tmp + i - 1, s, (size_t)L) == 0)) tab[h].occ++;"),
]


def _build_variant(src_dir, text, repl, out_so):
    src = open(os.path.join(src_dir, "train_dict.c")).read()
    assert text in src, "mutation anchor not found: %r" % text
    d = os.path.dirname(out_so)
    with open(os.path.join(d, "train_dict.c"), "w") as f:
        f.write(src.replace(text, repl, 1))
    shutil.copy(os.path.join(src_dir, "zs_oracle.c"), os.path.join(d, "zs_oracle.c"))
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", os.path.join(d, "train_dict.c"),
                           os.path.join(d, "zs_oracle.c"), "-o", out_so])
    lib = ctypes.CDLL(out_so)
    lib.zo_train_dict.restype = ctypes.c_int
    return lib


@pytest.mark.parametrize("name,text,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_trainer_mistake_is_caught(name, text, repl):
    src_dir = os.path.dirname(os.path.abspath(oracle.__file__))
    with tempfile.TemporaryDirectory() as d:
        lib = _build_variant(src_dir, text, repl, os.path.join(d, "mut.so"))
        caught = [k for k, (lines, lmin, lmax, T, want) in HAND_CASES.items()
                  if _train(lines, lmin, lmax, T, lib=lib) != want]
        caught += ["XAB"] if _train([b"AB", b"AB", b"AB", b"XAB", b"XAB", b"QRS"], 2, 3, 2,
                                    lib=lib) != [b"AB", b"QRS"] else []
        assert caught, "the hand-worked cases do not catch: " + name


def test_preprocess_buffer_framing():
    """zo_preprocess_buffer: one pre-processed line per input line, each followed by a
    newline, offsets the running sum of (length + 1); empty lines stay empty; a last
    line ending at a virtual newline is framed like the others."""
    lines = [b"C1CC1", b"", b"c1ccc2ccccc2c1", b"", b"", b"N[NH3+]C%12CC%12", b"C1CC"]
    buf, off = oracle.join_lines(lines)
    out, out_off = oracle.preprocess_buffer(buf, off)
    want = [oracle.preprocess(l) for l in lines]
    # the per-line results themselves: ring IDs from 0, the inner ring (closed first)
    # taking the lower ID (Sec. IV-A); an unclosed ring leaves its line unchanged
    assert want == [b"C0CC0", b"", b"c1ccc0ccccc0c1", b"", b"", b"N[NH3+]C0CC0", b"C1CC"]
    assert out.tobytes() == b"".join(w + b"\n" for w in want)
    assert [int(x) for x in out_off] == list(np.cumsum([0] + [len(w) + 1 for w in want]))
    # the same lines with the last one unterminated (off[n] = len + 1)
    vbuf = buf[:-1].copy()
    voff = off.copy()
    voff[-1] = vbuf.size + 1
    vout, voff_out = oracle.preprocess_buffer(vbuf, voff)
    assert vout.tobytes() == out.tobytes()
    assert np.array_equal(voff_out, out_off)
    # no lines at all
    e, eo = oracle.preprocess_buffer(np.zeros(0, np.uint8), np.zeros(1, np.uint64))
    assert e.size == 0 and list(eo) == [0]
