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


MODES = {"plain": None, "tuned": {"radix_bits": 11, "fuse_dedup": 1}, "ranges": {"dedup_ranges": 1},
         "blocks": {"block_log2": [[7, 7, 9, 9], [7, 7, 9, 9]]}, "merge": {"dedup_ranges": 2}}


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


def _plain_traces():
    """Join traces the plain engine logs on the transitive-closure,
    same-generation, points-to and batched transitive-closure workloads --
    the predictor's training data, as the benchmark collects it."""
    rows = []
    for w in (W.config_tc(), W.config_sg(), W.config_pointsto()):
        *_, trace = fv.evaluate(w.program, w.edb, flags=fv.FV_LOG_JOINS, relations=list(w.idb), with_trace=True)
        rows.append(trace)
    engines = []
    for x in W.batched_tc_instances():
        e = fv.Engine(flags=fv.FV_LOG_JOINS)
        e.relation("edge", 2)
        e.relation("path", 2)
        e.load("edge", x.edb["edge"])
        e.program(x.program)
        engines.append(e)
    fv.run_batch(engines)
    rows.append(engines[0].join_trace())
    for e in engines:
        e.close()
    return np.concatenate(rows)


def test_rdfs_full_size_learned_mode_matches_oracle_digest():
    """The 20M-triple RDFS workload in its learned mode: the predictor on,
    trained (on the GPU) from the plain engine's traces of the transitive-
    closure, same-generation, points-to and batched transitive-closure
    workloads."""
    T = _plain_traces()
    params, loss = fv.mlp_train(T[:, :8], T[:, 8], steps=2000, lr=3e-3, seed=1)
    assert np.isfinite(loss)
    w = W.config_rdfs()
    ref = DIGESTS["rdfs_20000000"]
    got, stats, deltas, _ = fv.evaluate(w.program, w.edb, relations=["t"], flags=fv.FV_LEARNED, predictor=params)
    assert len(got["t"]) == ref["relations"]["t"]["count"]
    assert _digest(got["t"]) == ref["relations"]["t"]["sha256"]
    assert deltas == ref["deltas"]
    assert stats["derived_tuples"] == sum(ref["deltas"]) and stats["predicted_joins"] > 0
