"""The learned join-cardinality path: identical fixpoints whatever the
predictor says, join traces, and a predictor trained on the plain engine's
traces."""
import numpy as np
import pytest

import oracle
from paper_2501_13051_amd import fv
from paper_2501_13051_amd import workloads as W

pytestmark = pytest.mark.gpu

ZERO = np.zeros(fv.MLP_PARAMS, np.float32)
HUGE = np.zeros(fv.MLP_PARAMS, np.float32)
HUGE[-1] = 2.0          # b3: predicts log2(1+m) = 32 for every join


def _cases():
    d = W.rdfs_triples(n_triples=60_000, class_depth=5, n_entities=8_000, trans_tree=32, seed=9)
    pt = W.config_pointsto(scale=0.05)
    return [
        (W.TC_PROGRAM, {"edge": W.er_graph(700, 1400, seed=5)}, ["path"]),
        (W.SG_PROGRAM, {"edge": W.forest(8, 256, 0.05, seed=1002)}, ["sg"]),
        (pt.program, pt.edb, list(pt.idb)),
        (W.RDFS_PROGRAM, {"t": d["t"]}, ["t"]),
    ]


def _skewed_join():
    """Every probe row hits the one build key that owns 100,000 rows, among
    1,000 single-row keys: the uniform-key estimate (probe rows x mean run,
    about 100) is 1,000x short, so presized buffers overflow."""
    a_x = np.arange(50, dtype=np.uint32)
    a_y = np.zeros(50, dtype=np.uint32)
    b_y = np.concatenate([np.zeros(100_000, np.uint32), np.arange(1, 1001, dtype=np.uint32)])
    b_z = np.arange(len(b_y), dtype=np.uint32)
    return W.JOIN_PROGRAM, {"a": [a_x, a_y], "b": [b_y, b_z]}, ["out"]


@pytest.mark.parametrize("stub", ["zero", "huge"])
def test_stub_predictors_leave_the_fixpoint_unchanged(stub):
    params = ZERO if stub == "zero" else HUGE
    overflows = 0
    for program, edb, rels in _cases() + [_skewed_join()]:
        print(f"learned, {stub} predictor: {rels}", flush=True)
        ref = oracle.evaluate(program, edb)
        got, stats, deltas, _ = fv.evaluate(program, edb, flags=fv.FV_LEARNED, relations=rels, predictor=params)
        for r in rels:
            assert np.array_equal(got[r], ref[r]), r
        assert deltas == ref.delta_sizes
        assert stats["predicted_joins"] > 0
        overflows += stats["overflows"] + (stats["redo_rounds"] if stub == "zero" else 0)
    if stub == "zero":
        # presized buffers are at least the uniform-key estimate and never
        # below max(2^16, 2 x facts) rows; the skewed join exceeds both, so its
        # round runs again with exact sizes
        assert overflows > 0
    else:
        assert overflows == 0


def _true_sizes(trace):
    """Join output sizes recorded in a trace (column 8 holds log2(1 + m) / 16)."""
    return np.exp2(trace[:, 8].astype(np.float64) * 16) - 1


def test_join_trace_records_true_sizes():
    program, edb, rels = _cases()[1]
    got, stats, deltas, _, trace = fv.evaluate(program, edb, flags=fv.FV_LOG_JOINS, relations=rels,
                                               with_trace=True)
    assert trace.shape[1] == fv.TRACE_COLS and len(trace) >= 2 * (len(deltas) - 1)
    assert np.all(trace[:, 9] == -1)
    assert np.all(trace[:, 8] >= 0)
    assert stats["join_output_tuples"] > 0


def test_join_trace_sizes_equal_nested_loop_counts():
    """A chain of three atoms: the trace's two joins must report |a join b|
    and |(a join b) join c| before any filter, as bags, counted here by
    nested loops over the distinct rows (the relations are sets)."""
    rng = np.random.default_rng(21)

    def rel(n, hi0, hi1):
        r = np.unique(np.stack([rng.integers(0, hi0, n), rng.integers(0, hi1, n)], 1).astype(np.uint32), axis=0)
        return r

    a, b, c = rel(300, 200, 40), rel(900, 40, 60), rel(2500, 60, 500)   # |a| < |b| < |c|: a is probed first
    prog = "out(x, w) :- a(x, y), b(y, z), c(z, w)."
    edb = {k: [v[:, 0].copy(), v[:, 1].copy()] for k, v in (("a", a), ("b", b), ("c", c))}
    m1 = sum(1 for (_, y) in a for (y2, _) in b if y == y2)
    m2 = sum(1 for (_, y) in a for (y2, z) in b if y == y2 for (z2, _) in c if z == z2)
    *_, trace = fv.evaluate(prog, edb, flags=fv.FV_LOG_JOINS, relations=["out"], with_trace=True)
    steps = trace[:, 7]
    got1 = _true_sizes(trace[steps == 0])
    got2 = _true_sizes(trace[steps == 1])
    assert len(got1) == 1 and len(got2) == 1, trace
    assert abs(got1[0] - m1) <= 1e-4 * m1 + 0.5, (got1, m1)
    assert abs(got2[0] - m2) <= 1e-4 * m2 + 0.5, (got2, m2)


def test_recursive_join_trace_sizes_follow_shortest_path_layers():
    """Transitive closure path(x, z) :- path(x, y), edge(y, z): round j joins
    the pairs first derived in round j - 1 -- the pairs at shortest walk
    length exactly j -- with edge, so it outputs the sum of out-degree(y)
    over those pairs (computed here from boolean matrix powers)."""
    n = 300
    edge = W.er_graph(n, 600, seed=12)
    A = np.zeros((n, n), np.int64)
    A[edge[0], edge[1]] = 1
    outdeg = A.sum(1)
    seen = A.astype(bool)
    layer = A.astype(bool)           # pairs at shortest length exactly 1
    expect = [0]                     # round 0 joins the still empty path relation
    while layer.any():
        expect.append(int((layer * outdeg[None, :]).sum()))
        nxt = (layer.astype(np.int64) @ A) > 0
        layer = nxt & ~seen
        seen |= nxt
    *_, trace = fv.evaluate(W.TC_PROGRAM, {"edge": edge}, flags=fv.FV_LOG_JOINS, relations=["path"],
                            with_trace=True)
    got = np.rint(_true_sizes(trace)).astype(np.int64).tolist()
    assert got == expect, (got, expect)


def _predictor_rows(program, edb, rels, params):
    *_, trace = fv.evaluate(program, edb, flags=fv.FV_LEARNED, relations=rels, predictor=params, with_trace=True)
    return trace


def _bf16_sizes(X, params):
    """Sizes the reference network predicts (a negative size reads as 0)."""
    from oracle import mlp
    y = mlp.forward_bf16(X, params).astype(np.float64)
    return np.maximum(np.exp2(16 * y) - 1, 0)


def test_on_device_predictions_equal_the_bf16_reference():
    """k_predict (the inference the engine runs every round) against the
    FP64-structured BF16 reference on the same features.  First-step joins
    only: a later step's probe size is the previous prediction on the device
    but the true intermediate size in the trace.  A hand-built network
    predicts (1 + probe)^0.898 - 1, below every join's worst case (probe rows
    x longest build run), so no prediction is clamped and each must equal the
    reference's, truncated to an integer."""
    hand = np.zeros(fv.MLP_PARAMS, np.float32)
    hand[0] = 1.0                       # W1[0][0]: hidden unit 0 = probe feature
    hand[64 * 8 + 64 + 0] = 1.0         # W2[0][0]
    hand[64 * 8 + 64 + 64 * 64 + 64 + 0] = 0.9   # W3[0]
    checked = 0
    for program, edb, rels in _cases():
        T = _predictor_rows(program, edb, rels, hand)
        sel = (T[:, 7] == 0) & (T[:, 1] > 0)
        ref = _bf16_sizes(T[sel, :8], hand)
        got = T[sel, 9].astype(np.float64)
        assert np.all(np.abs(got - np.floor(ref)) <= 1 + 1e-5 * ref), np.c_[got, ref][:10]
        checked += int(sel.sum())
    assert checked > 20


def test_trained_predictions_within_the_bf16_reference():
    rows = []
    for program, edb, rels in _cases()[:3]:
        *_, trace = fv.evaluate(program, edb, flags=fv.FV_LOG_JOINS, relations=rels, with_trace=True)
        rows.append(trace)
    T0 = np.concatenate(rows)
    params, _ = fv.mlp_train(T0[:, :8], T0[:, 8], steps=800, lr=3e-3, seed=5)
    exact_rows = 0
    for program, edb, rels in _cases():
        T = _predictor_rows(program, edb, rels, params)
        sel = T[:, 7] == 0
        ref = _bf16_sizes(T[sel, :8], params)
        got = T[sel, 9].astype(np.float64)
        probe = np.exp2(T[sel, 0].astype(np.float64)) - 1
        # clamping to the worst case only lowers a prediction
        assert np.all(got <= ref * (1 + 1e-4) + 1), np.c_[got, ref][:10]
        # a prediction at most the probe rows is never clamped (longest run >= 1)
        unclamped = (ref <= probe) & (T[sel, 1] > 0)
        assert np.all(np.abs(got[unclamped] - np.floor(ref[unclamped])) <= 1 + 1e-4 * ref[unclamped])
        exact_rows += int(unclamped.sum())
    assert exact_rows > 0


def test_trained_predictor_on_plain_traces():
    rows = []
    for program, edb, rels in _cases()[:3]:
        *_, trace = fv.evaluate(program, edb, flags=fv.FV_LOG_JOINS, relations=rels, with_trace=True)
        rows.append(trace)
    T = np.concatenate(rows)
    params, loss = fv.mlp_train(T[:, :8], T[:, 8], steps=1500, lr=3e-3, seed=3)
    assert np.isfinite(loss)
    program, edb, rels = _cases()[3]     # held out: RDFS
    ref = oracle.evaluate(program, edb)
    got, stats, deltas, _ = fv.evaluate(program, edb, flags=fv.FV_LEARNED, relations=rels, predictor=params)
    assert np.array_equal(got["t"], ref["t"]) and deltas == ref.delta_sizes
    assert stats["predicted_joins"] > 0 and stats["qerror_median"] >= 1.0


def test_trained_predictor_gains_over_plain_engine():
    """What the network buys on an RDFS workload it never saw: the same
    fixpoint with fewer join count passes (light joins run presized in one
    pass) and no more re-run rounds than the plain engine's capacity guess."""
    rows = []
    for program, edb, rels in _cases()[:3]:
        *_, trace = fv.evaluate(program, edb, flags=fv.FV_LOG_JOINS, relations=rels, with_trace=True)
        rows.append(trace)
    T = np.concatenate(rows)
    params, _ = fv.mlp_train(T[:, :8], T[:, 8], steps=1500, lr=3e-3, seed=3)
    w = W.config_rdfs(scale=0.02)
    ref = oracle.evaluate(w.program, w.edb, relations=["t"])
    runs = {}
    for name, flags in (("plain", fv.FV_TRACE), ("learned", fv.FV_TRACE | fv.FV_LEARNED)):
        got, stats, deltas, prof = fv.evaluate(w.program, w.edb, flags=flags, relations=["t"], predictor=params)
        assert np.array_equal(got["t"], ref["t"]) and deltas == ref.delta_sizes, name
        runs[name] = (stats, {k["name"]: k for k in prof})
        print(name, stats["ms_total"], "ms, redo", stats["redo_rounds"], flush=True)
    count_passes = {n: r[1].get("join_probe", {"launches": 0})["launches"] for n, r in runs.items()}
    assert count_passes["learned"] < count_passes["plain"], count_passes
    assert runs["learned"][1]["join_onepass"]["launches"] > 0
    assert runs["learned"][0]["redo_rounds"] <= runs["plain"][0]["redo_rounds"]


def test_trained_predictor_picks_the_join_order_with_fewer_rows():
    """r(x, z) :- r(x, y), fan(y, z), ack(z, x) can join fan (about 128 rows
    per key) or ack (about 16) right after the delta atom.  The default order
    takes fan (a tie on bound variables, broken by body order); the zero stub
    predicts nothing for either order and keeps it.  A network trained on the
    plain engine's traces expects fewer rows from ack first and runs that
    order: the same fixpoint with fewer join output rows (intermediates
    included)."""
    rows = []
    w = W.ack_reach(32)
    for program, edb, rels in _cases()[:3] + [(w.program, w.edb, ["r"])]:
        *_, trace = fv.evaluate(program, edb, flags=fv.FV_LOG_JOINS, relations=rels, with_trace=True)
        rows.append(trace)
    T = np.concatenate(rows)
    params, _ = fv.mlp_train(T[:, :8], T[:, 8], steps=1500, lr=3e-3, seed=3)
    ref = oracle.evaluate(w.program, w.edb)
    runs = {}
    for name, kw in (("plain", {}), ("zero", dict(flags=fv.FV_LEARNED, predictor=ZERO)),
                     ("trained", dict(flags=fv.FV_LEARNED, predictor=params))):
        got, stats, deltas, _ = fv.evaluate(w.program, w.edb, relations=["r"], **kw)
        assert np.array_equal(got["r"], ref["r"]) and deltas == ref.delta_sizes, name
        runs[name] = stats
        print(name, stats["join_output_tuples"], "join rows, reordered", stats["reordered_rounds"], flush=True)
    assert runs["zero"]["reordered_rounds"] == 0
    assert runs["zero"]["join_output_tuples"] == runs["plain"]["join_output_tuples"]
    assert runs["trained"]["reordered_rounds"] > 0
    assert runs["trained"]["join_output_tuples"] < runs["zero"]["join_output_tuples"] // 2


def _hand_net(feature):
    """A network whose output is feature `feature` itself: it predicts
    m = 2^(16 x feature / 16) - 1 (build rows for feature 1, distinct probe
    keys for feature 3), clamped to the join's worst case."""
    net = np.zeros(fv.MLP_PARAMS, np.float32)
    net[feature] = 1.0                        # W1[0][feature]
    net[64 * 8 + 64 + 0] = 1.0                # W2[0][0]
    net[64 * 8 + 64 + 64 * 64 + 64 + 0] = 1.0   # W3[0]
    return net


def test_join_orders_are_parity_green_whichever_is_chosen():
    """Every join order the learned engine may pick gives the oracle's
    fixpoint, on the three-atom rules of the acknowledged-reachability and
    points-to programs: a predictor that expects huge outputs (each clamped to
    its join's worst case, probe rows x longest build run, so the order with
    the smaller worst case wins), one that predicts the build side's rows, and
    one that predicts the probe key's distinct values."""
    w = W.ack_reach(8)
    pt = W.config_pointsto(scale=0.05)
    reordered = {}
    for name, program, edb, rels in (("ack", w.program, w.edb, ["r"]), ("pointsto", pt.program, pt.edb, list(pt.idb))):
        ref = oracle.evaluate(program, edb)
        for pname, params in (("huge", HUGE), ("build_rows", _hand_net(1)), ("probe_ndv", _hand_net(3))):
            print(f"join orders: {name} with the {pname} predictor", flush=True)
            got, stats, deltas, _ = fv.evaluate(program, edb, flags=fv.FV_LEARNED, relations=rels, predictor=params)
            for r in rels:
                assert np.array_equal(got[r], ref[r]), (name, pname, r)
            assert deltas == ref.delta_sizes, (name, pname)
            reordered[name, pname] = stats["reordered_rounds"]
    # ack (16 rows per key) is both the smaller build and the smaller worst case
    assert reordered["ack", "huge"] > 0 and reordered["ack", "build_rows"] > 0, reordered


def test_a_failed_round_in_a_predicted_order_returns_to_the_default(monkeypatch):
    """A round run in a join order the predictions picked that fails (forced
    here through the test hook on the first recursive round) runs again in
    the default order, and its group keeps the default order for the rest of
    the fixpoint: the same result, fewer reordered rounds."""
    w = W.ack_reach(8)
    ref = oracle.evaluate(w.program, w.edb)
    net = _hand_net(1)
    _, free, _, _ = fv.evaluate(w.program, w.edb, flags=fv.FV_LEARNED, relations=["r"], predictor=net)
    monkeypatch.setenv("FV_TEST_FAIL_ROUNDS", "2")
    got, stats, deltas, _ = fv.evaluate(w.program, w.edb, flags=fv.FV_LEARNED, relations=["r"], predictor=net)
    assert np.array_equal(got["r"], ref["r"]) and deltas == ref.delta_sizes
    assert stats["redo_rounds"] >= 1
    assert free["reordered_rounds"] >= 2 and stats["reordered_rounds"] == 1, (free, stats)
