"""Writes the stored expected values under tests/golden/ that do not come
from the paper: known-answer vectors of the oracle's dither generator and
codec.  Calls only the oracle.  Run: python tests/golden/make_golden.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    cases = []
    for idx, t, seed, mode in [(0, 0, 0, 1), (1, 0, 0, 1), (12345, 7, 42, 1), (2**31 + 5, 999, 3, 1),
                               (160_000_000 - 1, 500, 0, 1), (77, 3, 9, 2), (77, 4, 9, 2), (5, 5, 5, 0)]:
        xi, h = oracle.dither(idx, t, seed, mode)
        cases.append({"idx": idx, "t": t, "seed": seed, "mode": mode, "h1": h[0], "h2": h[1],
                      "xi": [float(v) for v in xi]})
    hashes = {str(v): oracle.pcg_hash(v) for v in [0, 1, 2, 3, 1000, 2**32 - 1, 0x9E3779B9]}
    codes = []
    for m, k, xi in [(1.0, 0, 0.0), (0.8, 0, 0.0), (1.5, 0, 0.0), (0.0, 1, 0.0), (0.05, 2, 0.25),
                     (-0.4, 3, 0.0), (0.4, 3, 0.0), (0.0, 4, 0.0), (0.1, 9, 0.0), (-0.1, 7, 0.49),
                     (2.0, 0, 0.0), (-1.0, 5, 0.0)]:
        codes.append({"m": m, "k": k, "xi": xi, "q": oracle.encode_one(m, k, xi)})
    out = {"_note": "written by tests/golden/make_golden.py from the oracle; definitions, not paper values",
           "dither": cases, "pcg_hash": hashes, "encode": codes}
    with open(os.path.join(HERE, "oracle_kat.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
