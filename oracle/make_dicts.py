"""Write the frozen variant dictionaries (run once; calls only oracle/ and the input generator).

Every dictionary is trained by Algorithm 1 (Sec. IV-C, rank of Eq. (1)) on
synthetic SMILES and written as a .zsd file next to the default one:

* L_max sweep (Sec. V-C sweeps L_max over 5, 8 and 15): the default recipe
  (10,000 lines of the small workload, seed 1000, pre-processed, SMILES
  alphabet pre-populated, 146 learned patterns, L_min 2) with L_max 5 and 15;
  the default dictionary itself is the L_max 8 point.
* Table I variants (Sec. V-B, Table I): pre-processing Yes/No x pre-population
  {Printable, SMILES alphabet, None}.  Each is trained on 50,000 lines of the
  small workload (seed 1001; the paper trains and tests on the same 50,000
  lines), L_min 2, L_max 8.  "Yes" trains on the pre-processed corpus and is
  meant to be used with pre-processing on; "No" trains on the raw corpus.
  Printable pre-populates the 94 printable ASCII characters other than the
  space (the escape byte), leaving the 95 codes 0xA1..0xFF for patterns; the
  SMILES alphabet leaves 146 codes; None leaves all 189.
* A long-pattern dictionary for tests and the kernel-window comparison: the
  default dictionary with its last 24 learned codes replaced by the patterns
  Algorithm 1 selects with L_min 9 and L_max 16 on the same corpus as the
  default one (they come out 9 to 11 bytes long).

    python -m oracle.make_dicts [name ...]
"""
import os
import sys

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import oracle  # noqa: E402
import smilesgen  # noqa: E402
from oracle.make_default_dict import SMILES_ALPHABET, write_zsd  # noqa: E402

DATA = os.path.join(_ROOT, "paper_2404_19391_amd", "data")
PRINTABLE = bytes(b for b in range(0x21, 0x7F))
EXTENDED = list(range(0xA1, 0x100))


def pattern_codes(prepop):
    """Code bytes left for learned patterns: 0xA1..0xFF first, then unused printable ASCII."""
    return EXTENDED + [b for b in range(0x21, 0x7F) if b not in prepop]


def train(prepop, preprocess, lmin=2, lmax=8, seed=1000, n=10000):
    codes = pattern_codes(prepop)
    buf, off = smilesgen.generate("small", seed, n)
    pats = oracle.train_patterns(buf, off, len(codes), lmin=lmin, lmax=lmax, preprocess=preprocess)
    entries = {c: bytes([c]) for c in prepop}
    for c, p in zip(codes, pats):
        entries[c] = p
    return entries


def long_pattern_entries(n_long=24):
    base = train(SMILES_ALPHABET, True)
    codes = pattern_codes(SMILES_ALPHABET)
    buf, off = smilesgen.generate("small", 1000, 10000)
    longs = oracle.train_patterns(buf, off, n_long, lmin=9, lmax=16, preprocess=True)
    assert len(longs) == n_long
    taken = set(base.values())
    for c, p in zip(codes[-n_long:], longs):
        assert p not in taken
        base[c] = p
    return base


RECIPES = {
    "lmax5": (lambda: train(SMILES_ALPHABET, True, lmax=5), "L_max 5, SMILES alphabet, pre-processed"),
    "lmax15": (lambda: train(SMILES_ALPHABET, True, lmax=15), "L_max 15, SMILES alphabet, pre-processed"),
    "t1_prep_printable": (lambda: train(PRINTABLE, True, seed=1001, n=50000), "Table I: pre-processing, Printable"),
    "t1_raw_printable": (lambda: train(PRINTABLE, False, seed=1001, n=50000), "Table I: no pre-processing, Printable"),
    "t1_prep_smiles": (lambda: train(SMILES_ALPHABET, True, seed=1001, n=50000),
                       "Table I: pre-processing, SMILES alphabet"),
    "t1_raw_smiles": (lambda: train(SMILES_ALPHABET, False, seed=1001, n=50000),
                      "Table I: no pre-processing, SMILES alphabet"),
    "t1_prep_none": (lambda: train(b"", True, seed=1001, n=50000), "Table I: pre-processing, no pre-population"),
    "t1_raw_none": (lambda: train(b"", False, seed=1001, n=50000), "Table I: no pre-processing, no pre-population"),
    "long16": (long_pattern_entries, "default with 24 patterns trained with L_min 9, L_max 16"),
}


def main():
    names = sys.argv[1:] or list(RECIPES)
    for name in names:
        make, what = RECIPES[name]
        entries = make()
        d = oracle.Dict(entries)
        assert d.valid, "trained dictionary %s failed validation" % name
        path = os.path.join(DATA, name + ".zsd")
        write_zsd(path, entries, header=b"ZSD1 " + what.encode())
        print("wrote %s: %d codes, longest pattern %d" % (path, len(entries), d.lmax), flush=True)


if __name__ == "__main__":
    main()
