"""Full-size workloads against fixpoint digests written by the oracle
(tests/golden/make_digests.py): tuple counts, SHA-256 of the row-sorted
relations and the per-round delta sizes."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2501_13051_amd import fv
from paper_2501_13051_amd import workloads as W

pytestmark = pytest.mark.gpu
DIGESTS = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "fixpoint_digests.json")))
MAKERS = {"tc_er_n2000_m3000": W.config_tc, "sg_forest_t64_n1024": W.config_sg,
          "pointsto_n200000": W.config_pointsto, "rdfs_20000000": W.config_rdfs}


def _digest(rows):
    return hashlib.sha256(np.ascontiguousarray(rows, dtype="<u4").tobytes()).hexdigest()


MODES = {"plain": None, "tuned": {"radix_bits": 11, "fuse_dedup": 1}, "ranges": {"dedup_ranges": 1}}


@pytest.mark.parametrize("name", sorted(MAKERS))
@pytest.mark.parametrize("mode", sorted(MODES))
def test_full_size_matches_oracle_digest(name, mode):
    w = MAKERS[name]()
    ref = DIGESTS[name]
    tuning = MODES[mode]
    got, stats, deltas, _ = fv.evaluate(w.program, w.edb, relations=list(w.idb), tuning=tuning)
    for rel, d in ref["relations"].items():
        assert len(got[rel]) == d["count"], rel
        assert _digest(got[rel]) == d["sha256"], rel
    assert deltas == ref["deltas"]
    # the per-round deltas count derived tuples only (input facts are seeds)
    assert stats["derived_tuples"] == sum(ref["deltas"])
