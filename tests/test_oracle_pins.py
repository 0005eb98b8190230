"""Pins for the oracle: hand-derived fixtures, closed forms, brute force.

The oracle (oracle/) is checked here against things other than itself:
values derived by hand from the rule definitions (tests/golden), closed
forms of the closure on shapes whose answer is known (chain, cycle,
complete DAG, trees, stars), reachability by BFS, the matrix formulation of
same generation, and T_P applied literally over every variable assignment
on random tiny programs.  Each of the plausible mistakes -- a dropped rule
variant, a wrong join column, a missed duplicate, a wrong delta bookkeeping
-- changes at least one of these.
"""
import glob
import json
import math
import os
import random

import numpy as np
import pytest

import brute
from progs import random_program, random_edb
import oracle
from paper_2501_13051_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _edb_from_rows(d):
    out = {}
    for name, rows in d.items():
        a = np.asarray(rows, dtype=np.uint32)
        out[name] = [a[:, k].copy() for k in range(a.shape[1])]
    return out


@pytest.mark.parametrize("path", sorted(f for f in glob.glob(os.path.join(GOLDEN, "*.json")) if "digest" not in f), ids=os.path.basename)
@pytest.mark.parametrize("naive", [False, True])
def test_golden_by_hand(path, naive):
    g = json.load(open(path))
    edb = _edb_from_rows(g["edb"])
    for prog_key, exp_key, d_key in [("program", "expect", "deltas"),
                                     ("program_paper_form", "expect_paper_form", "deltas_paper_form")]:
        if prog_key not in g:
            continue
        r = oracle.evaluate(g[prog_key], edb, naive=naive)
        for name, rows in g[exp_key].items():
            exp = np.asarray(rows, dtype=np.uint32)
            assert np.array_equal(r[name], exp), (name, r[name].tolist())
        assert r.delta_sizes == g[d_key]


@pytest.mark.parametrize("n", [1, 2, 3, 10, 57])
def test_tc_chain_closed_form(n):
    r = oracle.evaluate(W.TC_PROGRAM, {"edge": W.chain(n)} if n > 1 else
                        {"edge": [np.zeros(0, np.uint32), np.zeros(0, np.uint32)]})
    assert len(r["path"]) == n * (n - 1) // 2
    # one round per path length, then the empty round
    assert r.delta_sizes == [n - 1 - k for k in range(n - 1)] + [0]


@pytest.mark.parametrize("n", [1, 2, 5, 31])
def test_tc_cycle_closed_form(n):
    edge = W.cycle(n) if n > 1 else [np.array([0], np.uint32), np.array([0], np.uint32)]
    r = oracle.evaluate(W.TC_PROGRAM, {"edge": edge})
    assert len(r["path"]) == n * n


@pytest.mark.parametrize("n", [2, 6, 20])
def test_tc_complete_dag_closed_form(n):
    r = oracle.evaluate(W.TC_PROGRAM, {"edge": W.complete_dag(n)})
    assert len(r["path"]) == math.comb(n, 2)
    # every pair is already an edge: round 0 copies them, round 1 adds nothing
    assert r.delta_sizes == [math.comb(n, 2), 0]


def _depths(src, dst, n):
    parent = {int(v): int(u) for u, v in zip(src, dst)}
    d = np.zeros(n, dtype=np.int64)
    for v in range(n):
        k, x = 0, v
        while x in parent:
            x = parent[x]
            k += 1
        d[v] = k
    return d


@pytest.mark.parametrize("seed", [3, 4])
def test_tc_tree_closed_form(seed):
    rng = W.SplitMix64(seed)
    e = W.recursive_tree_edges(300, 0, rng)
    src, dst = e[:, 0].astype(np.uint32), e[:, 1].astype(np.uint32)
    r = oracle.evaluate(W.TC_PROGRAM, {"edge": [src, dst]})
    assert len(r["path"]) == int(_depths(src, dst, 300).sum())


def test_tc_config_graph_equals_bfs():
    w = W.config_tc()
    r = oracle.evaluate(w.program, w.edb)
    assert np.array_equal(r["path"], brute.tc_bfs(*w.edb["edge"]))
    # the paper's left-recursive form reaches the same fixpoint (same set)
    r2 = oracle.evaluate(W.TC_PROGRAM_PAPER_FORM, w.edb)
    assert np.array_equal(r2["reach"], r["path"])


def test_sg_pure_forest_closed_form():
    # 6 trees of 200 nodes, no extra edges: sg = distinct pairs at equal depth
    edge = W.forest(6, 200, 0.0, seed=77)
    r = oracle.evaluate(W.SG_PROGRAM, {"edge": edge})
    exp = 0
    for t in range(6):
        m = (edge[0] >= t * 200) & (edge[0] < (t + 1) * 200)
        d = _depths(edge[0][m] - t * 200, edge[1][m] - t * 200, 200)
        _, cnt = np.unique(d[d >= 1], return_counts=True)
        exp += int((cnt * (cnt - 1)).sum())
    assert len(r["sg"]) == exp


@pytest.mark.parametrize("k", [1, 2, 7])
def test_sg_star_and_chain(k):
    assert len(oracle.evaluate(W.SG_PROGRAM, {"edge": W.star(k)})["sg"]) == k * (k - 1)
    assert len(oracle.evaluate(W.SG_PROGRAM, {"edge": W.chain(k + 1)})["sg"]) == 0


@pytest.mark.parametrize("paper_form", [False, True])
def test_sg_forest_equals_matrix_form(paper_form):
    nodes, trees = 256, 3
    edge = W.forest(trees, nodes, 0.05, seed=1002)
    prog = W.SG_PROGRAM_PAPER_FORM if paper_form else W.SG_PROGRAM
    r = oracle.evaluate(prog, {"edge": edge})
    exp = brute.sg_matrix(edge[0].astype(np.int64), edge[1].astype(np.int64), trees * nodes,
                          neq_recursive=paper_form)
    assert np.array_equal(r["sg"], exp)


# ------------------------------------------------------- random tiny programs
@pytest.mark.parametrize("seed", range(40))
def test_random_programs_agree_with_assignment_brute_force(seed):
    rnd = random.Random(seed)
    prog = random_program(rnd)
    edb = random_edb(rnd)
    facts, deltas = brute.naive_by_assignment(prog, edb)
    semi = oracle.evaluate(prog, edb)
    naive = oracle.evaluate(prog, edb, naive=True, relations=list(semi.relations))
    for name in semi.relations:
        ar = {"e": 2, "c": 1, "p": 2, "q": 2, "r": 3, "u": 1}[name]
        exp = brute.as_rows(facts.get(name, set()), ar)
        if name in ("e", "c"):
            exp = brute.rows(edb[name]) if len(edb[name][0]) else exp
        assert np.array_equal(semi[name], exp), (prog, name)
        assert np.array_equal(naive[name], exp), (prog, name)
    assert semi.delta_sizes == deltas, prog
    assert naive.delta_sizes == deltas, prog


def test_oracle_rejects_bad_programs():
    with pytest.raises(oracle.OracleError):
        oracle.evaluate("p(x, y) :- e(x, x).", {"e": [np.zeros(0, np.uint32)] * 2})   # unsafe head var
    with pytest.raises(oracle.OracleError):
        oracle.evaluate("p(x) :- e(x, y), x != z.", {"e": [np.zeros(0, np.uint32)] * 2})  # unsafe !=
    with pytest.raises(oracle.OracleError):
        oracle.evaluate("p(x) :- e(x).", {"e": [np.zeros(0, np.uint32)] * 2})        # arity clash
