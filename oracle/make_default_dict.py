"""Write the frozen default dictionary (run once; calls only oracle/ and the input generator).

Training corpus: 10,000 synthetic lines of the small workload (uniform length
20..80), seed 1000 - disjoint from every seed the tests and benchmarks use.
Pre-population with the SMILES alphabet (Sec. IV-B): 43 characters map to
themselves, so a well-formed line never needs an escape.  The remaining 146
printable code bytes (0xA1..0xFF first, the "extended ASCII" of Sec. IV-B,
then the unused printable ASCII bytes) receive the patterns of Algorithm 1,
lengths 2..8, trained on the pre-processed corpus (Sec. V-B), in selection
order.

    python -m oracle.make_default_dict [out_path]
"""
import os
import sys

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import oracle  # noqa: E402
import smilesgen  # noqa: E402

SMILES_ALPHABET = b"BCNOPSFIHlrbcnops0123456789[]+-%=#$:/\\().@*"
DEFAULT_OUT = os.path.join(_ROOT, "paper_2404_19391_amd", "data", "default.zsd")


def free_codes():
    ext = list(range(0xA1, 0x100))
    asc = [b for b in range(0x21, 0x7F) if b not in SMILES_ALPHABET]
    return ext + asc


def build_entries(seed=1000, n=10000, lmin=2, lmax=8):
    assert len(SMILES_ALPHABET) == 43 and len(set(SMILES_ALPHABET)) == 43
    codes = free_codes()
    buf, off = smilesgen.generate("small", seed, n)
    pats = oracle.train_patterns(buf, off, len(codes), lmin=lmin, lmax=lmax, preprocess=True)
    entries = {c: bytes([c]) for c in SMILES_ALPHABET}
    for c, p in zip(codes, pats):
        entries[c] = p
    return entries


def write_zsd(path, entries, header=b"ZSD1 default: SMILES alphabet + Algorithm 1 patterns, Lmax 8"):
    with open(path, "wb") as f:
        f.write(header + b"\n")
        for c in sorted(entries):
            f.write(b"%02x " % c + entries[c] + b"\n")


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else DEFAULT_OUT
    entries = build_entries()
    d = oracle.Dict(entries)
    assert d.valid, "trained dictionary failed validation"
    write_zsd(out, entries)
    print("wrote %s: %d codes, lmax %d" % (out, len(entries), d.lmax))


if __name__ == "__main__":
    main()
