"""Write the oracle's full-size reference for the 1M-node / 20M-edge power-law workload.

Calls only the oracle (Algorithm 1 replay, processors split over host threads) and the input
generators; no value comes from the device library.  Output: config2_oracle.txt beside this
script, holding the 40 global counts, the sum of the local counts per group, and a SHA-256 of
the exact int64 arrays (global then local, little-endian), which the full-size GPU test
compares against.

    python tests/golden/make_reference_digests.py [--workers 8]
"""
import argparse
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

N, M, C, SEED = 1_000_000, 10, 40, 20181122


def digest(glob: np.ndarray, loc: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(glob, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(loc, dtype="<i8").tobytes())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    edges = synth.config2_stream()
    t0 = time.time()
    glob, loc = oracle.rept_threads(edges, N, M, C, SEED, workers=args.workers)
    dt = time.time() - t0
    path = os.path.join(HERE, "config2_oracle.txt")
    with open(path, "w") as f:
        f.write("# Oracle (Algorithm 1 replay) on the Chung-Lu stream: 1,000,000 nodes, 20,000,000 edges,\n")
        f.write("# exponent 2.1, max expected degree 5e4, generator seed 2, order seed 1002 (synth.config2_stream);\n")
        f.write(f"# m = {M}, c = {C} (four hash groups), hash seed {SEED}; local counts per group.\n")
        f.write("# Written by tests/golden/make_reference_digests.py (oracle only).\n")
        f.write(f"# replay time {dt:.0f} s on {args.workers} host threads\n")
        f.write(f"sha256: {digest(glob, loc)}\n")
        f.write("global: " + " ".join(str(int(x)) for x in glob) + "\n")
        f.write("local_row_sums: " + " ".join(str(int(x)) for x in loc.sum(axis=1)) + "\n")
    print(open(path).read())


if __name__ == "__main__":
    main()
