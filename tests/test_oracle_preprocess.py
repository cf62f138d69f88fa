"""Pins of the oracle's ring-ID pre-processing (Sec. IV-A) to things other than itself:
the paper's worked example, hand-derived cases, a second algorithm (brute.preprocess_alt)
and the structural properties the paper states (nested rings never share an ID, Sec. II;
the inner ring gets the lower ID, Sec. IV-A; the result is still a valid ring numbering)."""
import os
import random

import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cases(name):
    rows = [r for r in open(os.path.join(GOLDEN, name), "rb").read().split(b"\n")
            if r and not r.startswith(b"#")]
    assert len(rows) % 2 == 0
    return [(rows[i], rows[i + 1]) for i in range(0, len(rows), 2)]


@pytest.mark.parametrize("raw,expected", _cases("preprocess_paper.txt"))
def test_paper_example(raw, expected):
    assert oracle.preprocess(raw) == expected


@pytest.mark.parametrize("raw,expected", _cases("preprocess_derived.txt"))
def test_derived_cases(raw, expected):
    assert oracle.preprocess(raw) == expected


def _nested(k):
    # k rings, each one inside the previous: C1C2C3 ... C3C2C1 (labels 1..k, %nn beyond 9)
    lab = [(b"%d" % v) if v < 10 else (b"%%%02d" % v) for v in range(1, k + 1)]
    return b"C" + b"C".join(lab) + b"CC" + b"C".join(reversed(lab)) + b"C"


def test_ten_and_more_nested_rings_use_percent_labels():
    x = _nested(12)
    y = oracle.preprocess(x)
    # innermost ring closes first -> 0; the outermost of 12 gets 11
    assert y == brute.preprocess_alt(x)
    assert b"%11" in y and b"%10" in y and b"%12" not in y
    assert y.count(b"0") >= 2


def _ids_by_ring(y):
    toks = brute._label_tokens(y)
    rings = brute.ring_intervals(y)
    return toks, rings


def _check_structure(x, y):
    """Properties of a valid renumbering of the rings of x."""
    rx = brute.ring_intervals(x)
    if rx is None:
        assert y == x
        return
    ry = brute.ring_intervals(y)
    # the same rings, i.e. the same pairing of label tokens
    assert ry == rx
    toks = brute._label_tokens(y)
    ids = {o: toks[o][2] for o, _ in ry}
    for o, c in ry:
        assert toks[c][2] == ids[o]
    # overlapping rings never share an ID; nested ones: inner lower
    for (o1, c1) in ry:
        for (o2, c2) in ry:
            if (o1, c1) == (o2, c2):
                continue
            if o1 < o2 < c1 or o2 < o1 < c2:
                assert ids[o1] != ids[o2]
            if o1 < o2 and c2 < c1:
                assert ids[o2] < ids[o1]
    # the IDs used are 0..k-1, and a proper colouring needs at least w = omega of them
    w = brute.omega(x)
    k = len(set(ids.values()))
    assert set(ids.values()) == set(range(k))
    assert k >= w
    # when no two rings cross (every pair nested or disjoint, the usual case), exactly w
    crossing = any(o1 < o2 < c1 < c2 for (o1, c1) in ry for (o2, c2) in ry)
    if not crossing:
        assert k == w


def _gen(preset, seed, n):
    import smilesgen
    return smilesgen.lines(preset, seed, n)


@pytest.mark.parametrize("preset,seed,n", [("test", 11, 3000), ("uneven", 12, 400), ("long", 13, 60)])
def test_matches_second_formulation_and_properties(preset, seed, n):
    for x in _gen(preset, seed, n):
        y = oracle.preprocess(x)
        assert y == brute.preprocess_alt(x), x
        _check_structure(x, y)


def test_crossing_rings_may_need_more_than_omega_ids():
    # Closing-order assignment is not an optimal colouring when rings cross:
    # here at most 3 rings are open at once, yet 4 IDs are used.
    x = b"CCOc[NH+]Cc=sO(O)c(ccO1)c(cOC1C(sc(c)ClO)C)S=CCFc2(n(n3o)C4)C=C25(c3)c6(C47(Cl657))"
    y = oracle.preprocess(x)
    assert y == b"CCOc[NH+]Cc=sO(O)c(ccO0)c(cOC0C(sc(c)ClO)C)S=CCFc0(n(n1o)C2)C=C03(c1)c0(C21(Cl031))"
    assert brute.omega(x) == 3
    _check_structure(x, y)


def test_idempotent():
    for x in _gen("uneven", 14, 300):
        y = oracle.preprocess(x)
        assert oracle.preprocess(y) == y


def test_random_ring_structures():
    rnd = random.Random(5)
    for _ in range(2000):
        # random label sequence over few values, atoms between, random brackets
        parts = []
        for _ in range(rnd.randint(0, 14)):
            r = rnd.random()
            if r < 0.45:
                v = rnd.randint(0, 12)
                parts.append((b"%d" % v) if v < 10 and rnd.random() < 0.7 else (b"%%%02d" % v))
            elif r < 0.55:
                parts.append(b"[NH3+]")
            elif r < 0.6:
                parts.append(rnd.choice([b"[", b"]", b"%", b"%1"]))
            else:
                parts.append(rnd.choice([b"C", b"c", b"N", b"(", b")", b"="]))
        x = b"C" + b"".join(parts)
        y = oracle.preprocess(x)
        assert y == brute.preprocess_alt(x), x
        _check_structure(x, y)


def test_empty_and_trivial():
    assert oracle.preprocess(b"") == b""
    assert oracle.preprocess(b"CCO") == b"CCO"
    assert oracle.preprocess(b" ") == b" "
