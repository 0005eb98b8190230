"""Parity of the HIP engine (through the C ABI) with the oracle.

Every comparison is exact: the exported relations (row-sorted uint32) must
be byte-identical to the oracle's fixpoint, and the per-round delta sizes
must match the oracle's round structure.
"""
import glob
import json
import os
import random

import numpy as np
import pytest

import oracle
from progs import random_edb, random_program
from paper_2501_13051_amd import fv
from paper_2501_13051_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


TUNINGS = {
    "default": None,
    "radix11": {"radix_bits": 11},
    "fused": {"fuse_dedup": 1},
    "radix11_fused_tight": {"radix_bits": 11, "fuse_dedup": 1, "set_load": 0.75, "index_load": 0.75,
                            "max_blocks": 256},
    "index_rebuild": {"index_rebuild": 1},
    "index_sort": {"index_sort": 2},     # every join index built by sorting
    "index_count": {"index_sort": 1},    # every join index built by counting
    "no_lookahead": {"lookahead": 1},    # every round waits for the one before
    "ranges": {"dedup_ranges": 1},       # Algorithm 2's difference over per-column indices of full
    "ranges_count": {"dedup_ranges": 1, "index_sort": 1},
    "merge": {"dedup_ranges": 2},        # difference against full's sorted keys, merged in every round
    "merge_tight": {"dedup_ranges": 2, "radix_bits": 11, "max_blocks": 256},
    # join and difference kernels in 128- or 512-thread blocks, or mixed by launch size
    "blocks128": {"block_log2": [[7, 7, 7, 7], [7, 7, 7, 7]]},
    "blocks512": {"block_log2": [[9, 9, 9, 9], [9, 9, 9, 9]]},
    "blocks_mixed": {"block_log2": [[7, 9, 8, 9], [9, 7, 9, 7]], "fuse_dedup": 1},
}


def _check(program, edb, relations=None, flags=fv.FV_PLAIN, tuning=None, predictor=None):
    ref = oracle.evaluate(program, edb)
    names = relations or list(ref.relations)
    got, stats, deltas, _ = fv.evaluate(program, edb, flags=flags, relations=names, tuning=tuning,
                                        predictor=predictor)
    for n in names:
        assert got[n].shape == ref[n].shape, (n, got[n].shape, ref[n].shape)
        assert np.array_equal(got[n], ref[n]), n
    assert deltas == ref.delta_sizes, (deltas, ref.delta_sizes)
    return got, stats, ref


def _edb_from_rows(d):
    return {k: [np.asarray(v, np.uint32)[:, c].copy() for c in range(len(v[0]))] for k, v in d.items()}


@pytest.mark.parametrize("path", sorted(f for f in glob.glob(os.path.join(GOLDEN, "*.json")) if "digest" not in f), ids=os.path.basename)
def test_golden(path):
    g = json.load(open(path))
    edb = _edb_from_rows(g["edb"])
    for pk, ek in [("program", "expect"), ("program_paper_form", "expect_paper_form")]:
        if pk in g:
            got, _, _ = _check(g[pk], edb)
            for name, rows in g[ek].items():
                assert np.array_equal(got[name], np.asarray(rows, np.uint32))


@pytest.mark.parametrize("n", [2, 3, 64, 65, 300])
def test_tc_chain_and_cycle(n):
    _check(W.TC_PROGRAM, {"edge": W.chain(n)})
    _check(W.TC_PROGRAM, {"edge": W.cycle(n)})


def test_tc_paper_form_and_dag():
    _check(W.TC_PROGRAM_PAPER_FORM, {"edge": W.er_graph(500, 900, seed=11)})
    _check(W.TC_PROGRAM, {"edge": W.complete_dag(40)})


@pytest.mark.parametrize("seed", range(30))
def test_random_programs(seed):
    rnd = random.Random(seed)
    prog = random_program(rnd)
    _check(prog, random_edb(rnd))


@pytest.mark.parametrize("tuning", list(TUNINGS), ids=list(TUNINGS))
@pytest.mark.parametrize("seed", range(30, 38))
def test_random_programs_tuned(seed, tuning):
    rnd = random.Random(seed)
    prog = random_program(rnd)
    _check(prog, random_edb(rnd), tuning=TUNINGS[tuning])


@pytest.mark.parametrize("tuning", list(TUNINGS), ids=list(TUNINGS))
def test_tuned_workloads(tuning):
    t = TUNINGS[tuning]
    _check(W.TC_PROGRAM, {"edge": W.er_graph(700, 1400, seed=5)}, tuning=t)
    _check(W.SG_PROGRAM, {"edge": W.forest(8, 256, 0.05, seed=1002)}, tuning=t)
    w = W.config_pointsto(scale=0.05)
    _check(w.program, w.edb, relations=list(w.idb), tuning=t)
    d = W.rdfs_triples(n_triples=60_000, class_depth=5, n_entities=8_000, trans_tree=32, seed=9)
    _check(W.RDFS_PROGRAM, {"t": d["t"]}, relations=["t"], tuning=t)


def test_autotune_picks_a_stored_tuning_with_the_same_fixpoint(tmp_path):
    edb = {"edge": W.forest(8, 256, 0.05, seed=1002)}
    rules = fv.parse_program(W.SG_PROGRAM)

    def make(t):
        e = fv.Engine(tuning=t)
        e.relation("edge", 2)
        e.relation("sg", 2)
        e.load("edge", edb["edge"])
        for head, body, neq in rules:
            e.add_rule(head, body, neq)
        return e

    cache = str(tmp_path / "tuning.json")
    best = fv.autotune(make, key="sg_small", cache_path=cache, reps=1)
    assert best["radix_bits"] in (8, 11) and best["fuse_dedup"] in (0, 1)
    assert best["max_blocks"] in (1024, 2048, 4096)
    assert all(b in (7, 8, 9) for row in best["block_log2"] for b in row)
    assert fv.tuning_load(cache, "sg_small") == best
    _check(W.SG_PROGRAM, edb, relations=["sg"], tuning=best)


@pytest.mark.parametrize("tuning", ["default", "index_sort"])
@pytest.mark.parametrize("zipf_s", [0.0, 1.0])
def test_join_case_small(zipf_s, tuning):
    w = W.join_case(1 << 14, 1 << 10, zipf_s)
    _check(w.program, w.edb, relations=["out"], tuning=TUNINGS[tuning])


@pytest.mark.parametrize("tuning", ["default", "index_count"])
@pytest.mark.parametrize("zipf_s", [0.0, 1.5])
def test_join_case_past_the_sorted_build_size(zipf_s, tuning):
    # 2^21 probe rows: the default knobs build a's index by sorting (a build
    # of at least 2^20 rows), index_count by hashing; same join either way
    w = W.join_case(1 << 21, 1 << 16, zipf_s, seed=1010)
    got, stats, ref = _check(w.program, w.edb, relations=["out"], tuning=TUNINGS[tuning])
    assert stats["derived_tuples"] == 1 << 21


def test_empty_and_duplicate_inputs():
    e0 = [np.zeros(0, np.uint32), np.zeros(0, np.uint32)]
    _check(W.TC_PROGRAM, {"edge": e0}, relations=["path", "edge"])
    # repeated facts in the load are one fact
    dup = [np.array([1, 1, 1, 2, 2], np.uint32), np.array([2, 2, 2, 3, 3], np.uint32)]
    got, _, _ = _check(W.TC_PROGRAM, {"edge": dup})
    assert got["path"].tolist() == [[1, 2], [1, 3], [2, 3]]


def test_large_ids_and_wide_keys():
    # ids near the top of the uint32 range: 32-bit columns, 64-bit packed keys
    rng = W.SplitMix64(5)
    src = (0xFFFFFFFE - rng.below(3000, 4000)).astype(np.uint32)
    dst = (0xFFFFFFFE - rng.below(3000, 4000)).astype(np.uint32)
    keep = src != dst
    _check(W.TC_PROGRAM, {"edge": [src[keep], dst[keep]]})


def spread_ids(col, keep_below=6):
    """Ids >= keep_below mapped one-to-one over [keep_below, 2^32 - 3]
    (v -> keep_below + v * 2654435761 mod (2^32 - 8), a unit modulo 2^32 - 8):
    the same relations with ids of full 32-bit magnitude."""
    v = np.asarray(col, np.uint64)
    m = np.uint64(2**32 - 8)
    with np.errstate(over="ignore"):
        f = np.uint64(keep_below) + (v * np.uint64(2654435761)) % m
    return np.where(v < keep_below, v, f).astype(np.uint32)


WIDE_EXTRA_RULES = """
t(o, 4294967294, s) :- t(s, {p}, o).
t(s, 4000000000, o) :- t(s, 3999999999, o).
"""


def wide_rdfs_case():
    d = W.rdfs_triples(n_triples=60_000, class_depth=5, n_entities=8_000, trans_tree=32, seed=9)
    t = [spread_ids(c) for c in d["t"]]
    prog = W.RDFS_PROGRAM + WIDE_EXTRA_RULES.format(p=int(t[1][t[1] >= 6][0]))
    return prog, {"t": t}


@pytest.mark.parametrize("flags", [fv.FV_PLAIN, fv.FV_LEARNED], ids=["plain", "learned"])
def test_packed_tuples_wider_than_64_bits(flags):
    """Triples whose three columns hold ids of full 32-bit magnitude (96 bits
    packed), rules with large constants (one absent from the facts): values
    are renumbered densely before the fixpoint and mapped back on export; the
    oracle works on the raw values."""
    prog, edb = wide_rdfs_case()
    kw = {"flags": flags}
    if flags & fv.FV_LEARNED:
        kw["predictor"] = np.zeros(fv.MLP_PARAMS, np.float32)
    ref = oracle.evaluate(prog, edb)
    got, stats, deltas, _ = fv.evaluate(prog, edb, relations=["t"], **kw)
    assert np.array_equal(got["t"], ref["t"])
    assert deltas == ref.delta_sizes
    assert int(got["t"][:, 1].max()) == 4294967294


def test_two_wide_columns_at_the_top_of_the_range():
    # both columns reach 0xFFFFFFFE: 33 + 33 bits with the empty-slot margin
    rng = W.SplitMix64(6)
    src = (0xFFFFFFFE - rng.below(3000, 4000)).astype(np.uint32)
    dst = (0xFFFFFFFE - rng.below(3000, 4000)).astype(np.uint32)
    src[0], dst[0] = 0xFFFFFFFE, 0xFFFFFFFD
    src[1], dst[1] = 0xFFFFFFFD, 0xFFFFFFFE
    keep = src != dst
    _check(W.TC_PROGRAM, {"edge": [src[keep], dst[keep]]})


def test_too_many_distinct_values_for_a_packed_triple():
    """2.1M distinct values over three columns still need 3 x 22 bits after
    renumbering: FV_ENOTSUP, and the context can be destroyed."""
    n = 700_000
    i = np.arange(n, dtype=np.uint32)
    e = fv.Engine()
    e.relation("a", 3)
    e.relation("b", 3)
    e.load("a", [3 * i, 3 * i + 1, 3 * i + 2])
    e.program("b(x, y, z) :- a(x, y, z).")
    with pytest.raises(fv.FvError) as ei:
        e.run()
    assert ei.value.status == "FV_ENOTSUP" and "renumbered" in str(ei.value)
    e.close()


def test_bounds_under_constant_conditions():
    from progs import CONDITIONED_PROGRAM, conditioned_edb
    got, _, _ = _check(CONDITIONED_PROGRAM, conditioned_edb())
    assert int(got["p"][:, 1].max()) == 1_000_099
    got, _, _ = _check(CONDITIONED_PROGRAM, conditioned_edb(), flags=fv.FV_LEARNED,
                       predictor=np.zeros(fv.MLP_PARAMS, np.float32))
    assert int(got["p"][:, 1].max()) == 1_000_099


def test_sg_forest_small_both_forms():
    edge = W.forest(8, 256, 0.05, seed=1002)
    _check(W.SG_PROGRAM, {"edge": edge})
    _check(W.SG_PROGRAM_PAPER_FORM, {"edge": edge})


def test_device_resident_load_and_export():
    import torch
    edge = W.er_graph(400, 800, seed=3)
    eng = fv.Engine()
    eng.relation("edge", 2)
    eng.relation("path", 2)
    eng.load("edge", [torch.from_numpy(c.astype(np.int32)).cuda() for c in edge])
    eng.program(W.TC_PROGRAM)
    eng.run()
    cols = eng.export("path", device=True)
    got = np.stack([c.cpu().numpy().view(np.uint32) for c in cols], axis=1)
    ref = oracle.evaluate(W.TC_PROGRAM, {"edge": edge})
    assert np.array_equal(got, ref["path"])
    eng.close()


def test_reserved_value_rejected():
    eng = fv.Engine()
    eng.relation("edge", 2)
    with pytest.raises(fv.FvError) as ei:
        eng.load("edge", [np.array([1, 0xFFFFFFFF], np.uint32), np.array([2, 3], np.uint32)])
    assert ei.value.status == "FV_ERESERVED"
    eng.close()


def test_config_tc_full_size():
    w = W.config_tc()
    got, stats, ref = _check(w.program, w.edb, relations=["path"])
    assert stats["derived_tuples"] == len(ref["path"])


@pytest.mark.parametrize("tuning", ["default", "radix11_fused_tight"])
def test_config_sg_full_size(tuning):
    w = W.config_sg()
    got, stats, ref = _check(w.program, w.edb, relations=["sg"], tuning=TUNINGS[tuning])
    assert stats["derived_tuples"] == len(ref["sg"])


def test_pointsto_small():
    w = W.config_pointsto(scale=0.05)
    _check(w.program, w.edb, relations=list(w.idb))


@pytest.mark.parametrize("tuning", ["index_rebuild", "default", "index_sort"])
def test_pointsto_full_size(tuning):
    w = W.config_pointsto()
    got, stats, ref = _check(w.program, w.edb, relations=list(w.idb), tuning=TUNINGS[tuning])
    assert stats["derived_tuples"] == sum(len(ref[n]) for n in w.idb)


def test_rdfs_small():
    d = W.rdfs_triples(n_triples=60_000, class_depth=5, n_entities=8_000, trans_tree=32, seed=9)
    _check(W.RDFS_PROGRAM, {"t": d["t"]}, relations=["t"])


def _batch_engines(instances, tuning=None, flags=fv.FV_PLAIN):
    engines = []
    for w in instances:
        e = fv.Engine(tuning=tuning, flags=flags)
        for name, cols in w.edb.items():
            e.relation(name, len(cols))
        e.relation("path", 2)
        for name, cols in w.edb.items():
            e.load(name, cols)
        e.program(w.program)
        engines.append(e)
    return engines


@pytest.mark.parametrize("n_inst,tuning", [(1, "default"), (7, "default"), (64, "default"), (7, "index_sort"),
                                           (7, "merge"), (64, "blocks_mixed")])
def test_batched_tc_matches_per_instance_oracle(n_inst, tuning):
    insts = W.batched_tc_instances(n_instances=n_inst, seed=77 + n_inst)
    engines = _batch_engines(insts, TUNINGS[tuning])
    stats = fv.run_batch(engines)
    total = 0
    per_round = []
    for w, e in zip(insts, engines):
        ref = oracle.evaluate(w.program, w.edb)
        got = e.export("path")
        assert np.array_equal(got, ref["path"])
        assert e.size("path") == len(ref["path"])
        assert np.array_equal(e.export("edge"), np.unique(np.stack(w.edb["edge"], 1), axis=0))
        total += len(ref["path"])
        per_round.append(ref.delta_sizes)
    merged = engines[0].delta_sizes()
    for e in engines:
        e.close()
    assert stats["derived_tuples"] == total
    # the merged rounds are the instances' rounds added up
    width = max(len(d) for d in per_round)
    summed = [sum(d[r] if r < len(d) else 0 for d in per_round) for r in range(width)]
    assert stats["iterations"] == width
    assert merged == summed


def test_batched_rejects_constants_and_disconnected_bodies():
    def mk(prog):
        e = fv.Engine()
        e.relation("edge", 2)
        e.relation("path", 2)
        e.load("edge", W.chain(4))
        e.program(prog)
        return e
    for prog in ["path(x, y) :- edge(x, y), edge(3, y).", "path(x, y) :- edge(x, z), edge(w, y)."]:
        es = [mk(prog), mk(prog)]
        with pytest.raises(fv.FvError) as ei:
            fv.run_batch(es)
        assert ei.value.status == "FV_ENOTSUP"
        for e in es:
            e.close()


@pytest.mark.parametrize("flags", [fv.FV_PLAIN, fv.FV_GRAPH], ids=["eager", "graph"])
def test_batched_config_full_size(flags):
    """All 512 instances of the batched workload, each against its own oracle
    fixpoint (eager rounds, and the recursive round captured as a graph)."""
    insts = W.batched_tc_instances()
    engines = _batch_engines(insts, flags=flags)
    stats = fv.run_batch(engines)
    total = 0
    for k, (w, e) in enumerate(zip(insts, engines)):
        ref = oracle.evaluate(w.program, w.edb)
        assert np.array_equal(e.export("path"), ref["path"]), k
        total += len(ref["path"])
    assert stats["derived_tuples"] == total
    if flags == fv.FV_GRAPH:
        assert stats["graph_captures"] >= 1 and stats["graph_replays"] >= 1, stats
    for e in engines:
        e.close()


# ------------------------------------------------------------------ captured rounds
@pytest.mark.parametrize("case", ["tc_chain", "tc_er", "sg", "pointsto", "rdfs"])
def test_graph_rounds_match_oracle(case):
    """FV_GRAPH: the recursive round captured once as a HIP graph and replayed
    (re-captured when a buffer grows)."""
    if case == "tc_chain":
        prog, edb, rels = W.TC_PROGRAM, {"edge": W.chain(300)}, ["path"]
    elif case == "tc_er":
        prog, edb, rels = W.TC_PROGRAM, {"edge": W.er_graph(700, 1400, seed=5)}, ["path"]
    elif case == "sg":
        prog, edb, rels = W.SG_PROGRAM, {"edge": W.forest(8, 256, 0.05, seed=1002)}, ["sg"]
    elif case == "pointsto":
        w = W.config_pointsto(scale=0.05)
        prog, edb, rels = w.program, w.edb, list(w.idb)
    else:
        d = W.rdfs_triples(n_triples=60_000, class_depth=5, n_entities=8_000, trans_tree=32, seed=9)
        prog, edb, rels = W.RDFS_PROGRAM, {"t": d["t"]}, ["t"]
    _, stats, _ = _check(prog, edb, relations=rels, flags=fv.FV_GRAPH)
    assert stats["graph_replays"] >= 1, stats


@pytest.mark.parametrize("seed", range(30, 38))
def test_graph_random_programs(seed):
    rnd = random.Random(seed)
    prog = random_program(rnd)
    _check(prog, random_edb(rnd), flags=fv.FV_GRAPH)


@pytest.mark.parametrize("n_inst", [7, 64])
def test_batched_graph_matches_per_instance_oracle(n_inst):
    insts = W.batched_tc_instances(n_instances=n_inst, seed=77 + n_inst)
    engines = _batch_engines(insts, flags=fv.FV_GRAPH)
    stats = fv.run_batch(engines)
    for w, e in zip(insts, engines):
        assert np.array_equal(e.export("path"), oracle.evaluate(w.program, w.edb)["path"])
        e.close()
    assert stats["graph_replays"] >= 1


# ------------------------------------------------------------------ fault injection
def _workload(case):
    if case == "tc":
        return W.TC_PROGRAM, {"edge": W.er_graph(700, 1400, seed=5)}, ["path"]
    if case == "sg":
        return W.SG_PROGRAM, {"edge": W.forest(8, 256, 0.05, seed=1002)}, ["sg"]
    if case == "pointsto":
        w = W.config_pointsto(scale=0.05)
        return w.program, w.edb, list(w.idb)
    d = W.rdfs_triples(n_triples=60_000, class_depth=5, n_entities=8_000, trans_tree=32, seed=9)
    return W.RDFS_PROGRAM, {"t": d["t"]}, ["t"]


@pytest.mark.parametrize("case", ["tc", "sg", "pointsto", "rdfs"])
def test_rounds_that_fail_run_again(case, monkeypatch):
    """Rounds made to fail (test hook: as if a join had overflowed) commit
    nothing and run again.  TC and SG run with look-ahead, so a round fails
    while the next one is already queued: that one must do nothing at all."""
    prog, edb, rels = _workload(case)
    monkeypatch.setenv("FV_TEST_FAIL_ROUNDS", "1,2,4,5,6,9,10,13,17")
    _, stats, _ = _check(prog, edb, relations=rels)
    assert stats["redo_rounds"] >= 3, stats


@pytest.mark.parametrize("case", ["tc", "sg", "pointsto", "rdfs"])
def test_learned_rounds_that_fail_fall_back(case, monkeypatch):
    prog, edb, rels = _workload(case)
    monkeypatch.setenv("FV_TEST_FAIL_ROUNDS", "1,3,4,7")
    params = np.zeros(fv.MLP_PARAMS, np.float32)
    _, stats, _ = _check(prog, edb, relations=rels, flags=fv.FV_LEARNED, predictor=params)
    assert stats["redo_rounds"] >= 2, stats


@pytest.mark.parametrize("case", ["tc", "sg", "pointsto", "rdfs"])
@pytest.mark.parametrize("flags", [fv.FV_PLAIN, fv.FV_GRAPH], ids=["eager", "graph"])
def test_tiny_initial_capacities_grow(case, flags, monkeypatch):
    """Every new-tuple and intermediate buffer starts at 256 rows (test hook):
    rounds overflow, buffers grow, rounds run again."""
    prog, edb, rels = _workload(case)
    monkeypatch.setenv("FV_TEST_SMALL_CAPS", "1")
    _, stats, _ = _check(prog, edb, relations=rels, flags=flags)
    assert stats["redo_rounds"] >= 1, stats


@pytest.mark.parametrize("case", ["tc", "sg", "pointsto", "rdfs"])
@pytest.mark.parametrize("flags", [fv.FV_PLAIN, fv.FV_GRAPH], ids=["eager", "graph"])
def test_merge_difference_with_failed_rounds_and_growth(case, flags, monkeypatch):
    """The difference by merge keeps a sorted copy of full that a round
    replaces only when it succeeds: rounds made to fail and buffers that start
    at 256 rows (the sorted copies grow with them) leave the fixpoint as the
    oracle's, eager and with the recursive round captured."""
    prog, edb, rels = _workload(case)
    monkeypatch.setenv("FV_TEST_SMALL_CAPS", "1")
    monkeypatch.setenv("FV_TEST_FAIL_ROUNDS", "2,3,6")
    _, stats, _ = _check(prog, edb, relations=rels, flags=flags, tuning={"dedup_ranges": 2})
    assert stats["redo_rounds"] >= 3, stats


@pytest.mark.parametrize("seed", range(38, 46))
def test_random_programs_with_failures_and_tiny_capacities(seed, monkeypatch):
    rnd = random.Random(seed)
    prog = random_program(rnd)
    monkeypatch.setenv("FV_TEST_SMALL_CAPS", "1")
    monkeypatch.setenv("FV_TEST_FAIL_ROUNDS", "2,3,5")
    _check(prog, random_edb(rnd))


def test_device_memory_is_handed_back():
    """Contexts, including a batch's merged result, return every allocation
    to the caller's allocator when they are destroyed."""
    import gc
    import torch
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    _check(W.SG_PROGRAM, {"edge": W.forest(4, 128, 0.05, seed=3)}, relations=["sg"])
    insts = W.batched_tc_instances(n_instances=9, seed=5)
    engines = _batch_engines(insts)
    fv.run_batch(engines)
    for w, e in zip(insts, engines):
        assert np.array_equal(e.export("path"), oracle.evaluate(w.program, w.edb)["path"])
    for e in engines:
        e.close()
    del engines
    gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_batched_with_failures(monkeypatch):
    insts = W.batched_tc_instances(n_instances=16, seed=91)
    monkeypatch.setenv("FV_TEST_FAIL_ROUNDS", "2,3,6")
    monkeypatch.setenv("FV_TEST_SMALL_CAPS", "1")
    engines = _batch_engines(insts)
    stats = fv.run_batch(engines)
    for w, e in zip(insts, engines):
        assert np.array_equal(e.export("path"), oracle.evaluate(w.program, w.edb)["path"])
        e.close()
    assert stats["redo_rounds"] >= 3


def _raw_tc_context(L, opt):
    """A TC program set up through the C ABI directly; returns the handle,
    the path relation, the edges, the status of the load (0 if it worked)
    and the error text the load left."""
    import ctypes
    h = ctypes.c_void_p()
    rc = L.fv_ctx_create(ctypes.byref(h), ctypes.byref(opt) if opt is not None else None)
    assert rc == 0
    e, p = ctypes.c_uint32(), ctypes.c_uint32()
    assert L.fv_relation_create(h, b"edge", 2, ctypes.byref(e)) == 0
    assert L.fv_relation_create(h, b"path", 2, ctypes.byref(p)) == 0
    edge = W.er_graph(500, 1000, seed=3)
    cols = [np.ascontiguousarray(c, np.uint32) for c in edge]
    ptrs = (ctypes.c_void_p * 2)(cols[0].ctypes.data, cols[1].ctypes.data)
    rc = L.fv_load_columns(h, e.value, ptrs, len(cols[0]), 0)
    err = L.fv_last_error(h)          # valid until the next call on the context
    keep = []
    for head, body, neq in fv.parse_program(W.TC_PROGRAM):
        def atom(a):
            name, ts = a
            arr = (fv.Term * len(ts))(*[fv.Term(v, 1 if k == "c" else 0) for k, v in ts])
            keep.append(arr)
            return fv.Atom(e.value if name == "edge" else p.value, len(ts), arr)
        r = fv.Rule()
        r.head = atom(head)
        r.body = (fv.Atom * len(body))(*[atom(b) for b in body])
        keep.append(r.body)
        r.n_body = len(body)
        r.n_neq = 0
        assert L.fv_add_rule(h, ctypes.byref(r)) == 0
    return h, p.value, edge, rc, err


def test_allocator_failure_is_enomem_and_the_context_stays_destroyable():
    """The allocator hook returns NULL from its k-th call on: the call that
    needed the memory returns FV_ENOMEM, later calls refuse, and the context
    can still be destroyed (everything it did allocate is handed back)."""
    import ctypes
    import torch
    L = fv.lib()
    dev = torch.cuda.current_device()
    stream = torch.cuda.Stream()

    def run(fail_after):
        count, live = [0], set()

        def _alloc(nbytes, s, user):
            count[0] += 1
            if count[0] > fail_after:
                return None
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream.cuda_stream)
            live.add(ptr)
            return ptr

        def _free(ptr, s, user):
            live.discard(ptr)
            torch.cuda.caching_allocator_delete(ptr)

        a, f = fv.ALLOC_FN(_alloc), fv.FREE_FN(_free)
        opt = fv.Options()
        opt.stream = ctypes.c_void_p(stream.cuda_stream)
        opt.dev_alloc, opt.dev_free = a, f
        h, path, _, rc, err = _raw_tc_context(L, opt)
        if rc == 0:
            st = fv.Stats()
            rc = L.fv_run_fixpoint(h, ctypes.byref(st))
            err = L.fv_last_error(h)
        if rc != 0:
            n = ctypes.c_uint64()
            assert L.fv_export(h, path, None, 0, ctypes.byref(n), 0) != 0   # a failed context refuses
        L.fv_ctx_destroy(h)
        assert not live, f"{len(live)} allocations not handed back"
        return rc, count[0], err

    rc, total, _ = run(10 ** 9)
    assert rc == 0 and total > 10
    for k in (0, 2, total // 3, total // 2, total - 1):
        rc, _, err = run(k)
        assert rc == -2, (k, rc, err)          # FV_ENOMEM
        assert b"allocation" in err, err
    # the device is still fine afterwards
    _check(W.TC_PROGRAM, {"edge": W.chain(50)})


def test_export_into_a_short_buffer_is_etrunc():
    import ctypes
    L = fv.lib()
    h, path, edge, rc, _ = _raw_tc_context(L, None)
    assert rc == 0
    try:
        st = fv.Stats()
        assert L.fv_run_fixpoint(h, ctypes.byref(st)) == 0
        n = ctypes.c_uint64()
        assert L.fv_export(h, path, None, 0, ctypes.byref(n), 0) == 0
        ref = oracle.evaluate(W.TC_PROGRAM, {"edge": edge})["path"]
        assert n.value == len(ref)
        bufs = [np.full(n.value, 7, np.uint32) for _ in range(2)]
        ptrs = (ctypes.c_void_p * 2)(bufs[0].ctypes.data, bufs[1].ctypes.data)
        m = ctypes.c_uint64()
        assert L.fv_export(h, path, ptrs, n.value - 1, ctypes.byref(m), 0) == -8   # FV_ETRUNC
        assert m.value == n.value and np.all(bufs[0] == 7)                          # nothing written
        assert L.fv_export(h, path, ptrs, n.value, ctypes.byref(m), 0) == 0
        assert np.array_equal(np.stack(bufs, 1), ref)
        assert L.fv_run_fixpoint(h, ctypes.byref(st)) == -5                         # FV_ESTATE: ran already
    finally:
        L.fv_ctx_destroy(h)
