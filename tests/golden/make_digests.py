"""Write fixpoint digests of the full-size workloads, computed by the oracle.

Run from the repository root:  python tests/golden/make_digests.py [names...]
It calls only oracle/ (and the input generators) and writes
tests/golden/fixpoint_digests.json: per workload and relation the tuple count
and the SHA-256 of the row-sorted uint32 tuples (little-endian, row-major),
plus the per-round delta sizes.  GPU tests compare the engine's export with
these digests where running the oracle inside the test would take minutes.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2501_13051_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fixpoint_digests.json")

WORKLOADS = {
    "tc_er_n2000_m3000": W.config_tc,
    "sg_forest_t64_n1024": W.config_sg,
    "pointsto_n200000": W.config_pointsto,
    "rdfs_20000000": W.config_rdfs,
}


def digest(rows: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(rows, dtype="<u4").tobytes()).hexdigest()


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        w = WORKLOADS[name]()
        t = time.time()
        r = oracle.evaluate(w.program, w.edb, relations=list(w.idb))
        data[name] = {"relations": {n: {"count": int(len(r[n])), "sha256": digest(r[n])} for n in w.idb},
                      "deltas": r.delta_sizes, "oracle_seconds": round(r.seconds, 2)}
        print(name, {n: len(r[n]) for n in w.idb}, f"{time.time() - t:.1f}s", flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
