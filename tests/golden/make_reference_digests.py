"""Write the oracle's full-size references for the two large single-stream workloads.

Calls only the oracle (Algorithm 1 replay, processors spread over host threads) and the input
generators; no value comes from the device library.  Each output file beside this script holds
the global counts, the sum of the local counts per row, and a SHA-256 of the exact int64 arrays
(global then local, little-endian), which the full-size GPU tests compare against:

  config2_oracle.txt  Chung-Lu, 1,000,000 nodes, 20,000,000 edges; m = 10, c = 40 (four groups)
  config3_oracle.txt  R-MAT scale 24, edge factor 16, deduplicated, generation order
                      (260,384,039 edges); m = 100, c = 100

    python tests/golden/make_reference_digests.py [--config 2|3|all] [--workers 8]
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

SEED = 20181122
CONFIGS = {
    "2": dict(file="config2_oracle.txt", n=1_000_000, m=10, c=40, stream=synth.config2_stream,
              about=["Oracle (Algorithm 1 replay) on the Chung-Lu stream: 1,000,000 nodes, 20,000,000 edges,",
                     "exponent 2.1, max expected degree 5e4, generator seed 2, order seed 1002 (synth.config2_stream);",
                     f"m = 10, c = 40 (four hash groups), hash seed {SEED}; local counts per group."]),
    "3": dict(file="config3_oracle.txt", n=1 << 24, m=100, c=100, stream=synth.config3_stream,
              about=["Oracle (Algorithm 1 replay) on the R-MAT stream: scale 24 (16,777,216 nodes), edge factor 16,",
                     "(a, b, c) = (0.57, 0.19, 0.19), generator seed 3, self-loops and repeated pairs dropped, generation",
                     f"order (synth.config3_stream); m = 100, c = 100 (one hash group), hash seed {SEED}; local counts per group."]),
}


def digest(glob: np.ndarray, loc: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(glob, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(loc, dtype="<i8").tobytes())
    return h.hexdigest()


def write(key: str, workers: int) -> None:
    cfg = CONFIGS[key]
    edges = cfg["stream"]()
    t0 = time.time()
    glob, loc = oracle.rept_threads(edges, cfg["n"], cfg["m"], cfg["c"], SEED, workers=workers)
    dt = time.time() - t0
    path = os.path.join(HERE, cfg["file"])
    with open(path, "w") as f:
        for line in cfg["about"]:
            f.write(f"# {line}\n")
        f.write("# Written by tests/golden/make_reference_digests.py (oracle only).\n")
        f.write(f"# {len(edges)} stream edges; replay time {dt:.0f} s on {workers} host threads\n")
        f.write(f"sha256: {digest(glob, loc)}\n")
        f.write("global: " + " ".join(str(int(x)) for x in glob) + "\n")
        f.write("local_row_sums: " + " ".join(str(int(x)) for x in loc.sum(axis=1)) + "\n")
    print(open(path).read(), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="all", choices=["2", "3", "all"])
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    for key in (["2", "3"] if args.config == "all" else [args.config]):
        write(key, args.workers)


if __name__ == "__main__":
    main()
