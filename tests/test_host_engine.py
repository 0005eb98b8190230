"""The host evaluator (FV_HOST): the same plans and operators on host threads,
checked tuple for tuple and round for round against the oracle.  It needs no
GPU: these tests run in the CPU suite."""
import random

import numpy as np
import pytest

import oracle
from progs import random_edb, random_program
from paper_2501_13051_amd import fv
from paper_2501_13051_amd import workloads as W


def _check(program, edb, relations=None):
    ref = oracle.evaluate(program, edb)
    names = relations or list(ref.relations)
    got, stats, deltas, _ = fv.evaluate(program, edb, flags=fv.FV_HOST, relations=names)
    for n in names:
        assert np.array_equal(got[n], ref[n]), n
    assert deltas == ref.delta_sizes, (deltas, ref.delta_sizes)
    return got, stats, ref


@pytest.mark.parametrize("n", [2, 3, 64, 65])
def test_chain_and_cycle(n):
    _check(W.TC_PROGRAM, {"edge": W.chain(n)})
    _check(W.TC_PROGRAM, {"edge": W.cycle(n)})


def test_tc_forms_and_sg_forms():
    _check(W.TC_PROGRAM, {"edge": W.er_graph(400, 800, seed=11)})
    _check(W.TC_PROGRAM_PAPER_FORM, {"edge": W.er_graph(400, 800, seed=11)})
    edge = W.forest(4, 200, 0.05, seed=1002)
    _check(W.SG_PROGRAM, {"edge": edge})
    _check(W.SG_PROGRAM_PAPER_FORM, {"edge": edge})


@pytest.mark.parametrize("seed", range(20))
def test_random_programs(seed):
    rnd = random.Random(seed)
    _check(random_program(rnd), random_edb(rnd))


def test_pointsto_and_rdfs_small():
    w = W.config_pointsto(scale=0.02)
    _check(w.program, w.edb, relations=list(w.idb))
    d = W.rdfs_triples(n_triples=30_000, class_depth=4, n_entities=4_000, trans_tree=16, seed=9)
    _check(W.RDFS_PROGRAM, {"t": d["t"]}, relations=["t"])


def test_ack_reachability():
    w = W.ack_reach(4)
    for name, (a, b) in w.edb.items():
        assert np.all(a // 256 == b // 256), name          # edges stay inside a group
        assert len(np.unique((a.astype(np.uint64) << np.uint64(32)) | b)) == len(a), name
    _check(w.program, w.edb, relations=["r"])


def test_wide_ids_renumbered():
    from test_gpu_parity import wide_rdfs_case
    prog, edb = wide_rdfs_case()
    got, _, _ = _check(prog, edb, relations=["t"])
    assert int(got["t"][:, 1].max()) == 4294967294


def test_too_many_distinct_values_for_a_packed_triple():
    n = 700_000
    i = np.arange(n, dtype=np.uint32)
    e = fv.Engine(flags=fv.FV_HOST)
    e.relation("a", 3)
    e.relation("b", 3)
    e.load("a", [3 * i, 3 * i + 1, 3 * i + 2])
    e.program("b(x, y, z) :- a(x, y, z).")
    with pytest.raises(fv.FvError) as ei:
        e.run()
    assert ei.value.status == "FV_ENOTSUP" and "renumbered" in str(ei.value)
    e.close()


def test_empty_duplicates_and_reserved():
    _check(W.TC_PROGRAM, {"edge": [np.zeros(0, np.uint32), np.zeros(0, np.uint32)]}, relations=["path", "edge"])
    got, _, _ = _check(W.TC_PROGRAM, {"edge": [np.array([1, 1, 2], np.uint32), np.array([2, 2, 3], np.uint32)]})
    assert got["path"].tolist() == [[1, 2], [1, 3], [2, 3]]
    e = fv.Engine(flags=fv.FV_HOST)
    e.relation("edge", 2)
    with pytest.raises(fv.FvError) as ei:
        e.load("edge", [np.array([1, 2], np.uint32), np.array([0xFFFFFFFF, 3], np.uint32)])
    assert ei.value.status == "FV_ERESERVED"
    e.close()


def test_host_rejects_gpu_only_modes():
    for flags in (fv.FV_LEARNED, fv.FV_GRAPH, fv.FV_LOG_JOINS):
        with pytest.raises(fv.FvError) as ei:
            fv.Engine(flags=fv.FV_HOST | flags,
                      predictor=np.zeros(fv.MLP_PARAMS, np.float32))
        assert ei.value.status == "FV_EINVAL"


def test_bounds_under_constant_conditions():
    from progs import CONDITIONED_PROGRAM, conditioned_edb
    got, _, _ = _check(CONDITIONED_PROGRAM, conditioned_edb())
    assert int(got["p"][:, 1].max()) == 1_000_099
    assert [5, 40] in got["s"].tolist() and [5, 41] in got["s"].tolist()
