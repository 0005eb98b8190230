"""Benchmark: derived tuples/s to fixpoint on one MI355X.

Headline (`value`): whole fixpoints of RDFS reasoning over the 20M-triple
synthetic triple table (class hierarchy of 8 levels with fan-out 6, 200
properties in a 4-level sub-property tree, domain and range axioms on half of
them, 10 transitive properties, Zipf-distributed entities and types; 102.5M
derived triples) with the learned join-cardinality predictor on: an MLP
trained at the start of the run, on this GPU, by the library's own kernels
from join traces the plain engine logs on the transitive-closure,
same-generation, points-to and batched transitive-closure workloads.  One
step = one fv_run_fixpoint: ingest of the EDB, index builds and every round of
join / radix sort / difference / merge to the fixpoint, from the call until the
stream is synchronized.  Inputs are generated and copied to the device, and
each step's context is created and loaded from those resident columns, before
its timed region (the metric excludes the load); the K timed regions are
summed.  The engine's knobs come from its own autotuner (stored choice).

The JSON line also carries: the roofline of the dominant kernel class
(algorithmic bytes over its kernels' device-clock time inside the timed
region, against 8 TB/s), the same workload run by the plain engine and with a
zero predictor (what the trained network adds), the oracle timed on one host
core on a bounded sample of the same workload, and the engine's other forms --
same generation, 512 batched transitive-closure instances vs the same
instances run one after another, a large single join, and autotuned points-to.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="headline only (no batched/learned/autotune forms)")
    ap.add_argument("--no-autotune", action="store_true", help="default knobs for the headline")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even if the cache holds a choice")
    ap.add_argument("--tuning-cache", default=os.path.join(ROOT, "paper_2501_13051_amd", "tuning_cache.json"))
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="copy this many MiB device-to-device once before timing (a known-size kernel for "
                         "calibrating HBM byte counters)")
    ap.add_argument("--save-predictor", default=None, help="write the trained predictor's parameters here (.npy)")
    ap.add_argument("--load-predictor", default=None,
                    help="use these parameters (.npy written by --save-predictor) instead of training, so that a "
                         "profiled run holds only the headline workload's kernels")
    ap.add_argument("--sweep-only", action="store_true",
                    help="run only the large-join sweep (for profiling it) and print its result")
    ap.add_argument("--sweep-case", type=int, default=-1,
                    help="with --sweep-only: run only this case of the sweep (0, 1 or 2)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain and zero-predictor runs beside the headline")
    return ap.parse_args()


# Kernel classes -> the source file that holds their kernel (for the traffic
# record's staleness check).
KERNEL_SOURCES = {"sort_pass": "kern_sort.hip", "sort_pass_dedup": "kern_sort.hip", "sort_hist": "kern_sort.hip",
                  "join_probe": "kern_join.hip", "join_write": "kern_join.hip", "dedup_append": "kern_join.hip",
                  "join_onepass": "kern_join.hip", "select": "kern_join.hip", "index_build": "kern_index.hip",
                  "index_upd_count": "kern_index.hip", "index_upd_reserve": "kern_index.hip",
                  "index_upd_move": "kern_index.hip", "index_upd_fill": "kern_index.hip",
                  "index_upd_keys": "kern_index.hip",
                  "index_upds_reserve": "kern_index.hip", "index_upds_fill": "kern_index.hip"}


def source_digest(kernel_class):
    import hashlib
    name = KERNEL_SOURCES.get(kernel_class)
    if not name:
        return None
    csrc = os.path.join(ROOT, "paper_2501_13051_amd", "csrc")
    h = hashlib.sha256()
    for f in (name, "fv_device.h", "fv_types.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_class):
    """HBM bytes per launch of a kernel class from the committed counter
    summary, if it was taken on the kernel's current source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel_class)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source") != source_digest(kernel_class):
        return None
    return rec.get("bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Runner:
    """Builds loaded contexts for one workload (EDB resident on the device)."""

    def __init__(self, fv, torch, np, program, edb, relations):
        self.fv, self.torch = fv, torch
        self.rules = fv.parse_program(program)
        self.arity = {}
        for head, body, _ in self.rules:
            for name, ts in [head] + body:
                self.arity.setdefault(name, len(ts))
        self.edb = {k: [torch.from_numpy(np.asarray(c).astype(np.int32)).cuda() for c in v] for k, v in edb.items()}
        for k, v in edb.items():
            self.arity.setdefault(k, len(v))
        self.relations = relations
        torch.cuda.synchronize()

    @staticmethod
    def arity_of(fv, program, edb):
        ar = {}
        for head, body, _ in fv.parse_program(program):
            for name, ts in [head] + body:
                ar.setdefault(name, len(ts))
        for k, v in edb.items():
            ar.setdefault(k, len(v))
        return ar

    def make(self, **kw):
        e = self.fv.Engine(**kw)
        for name, a in self.arity.items():
            e.relation(name, a)
        for name, cols in self.edb.items():
            e.load(name, cols)
        for head, body, neq in self.rules:
            e.add_rule(head, body, neq)
        return e

    def run_once(self, **kw):
        e = self.make(**kw)
        try:
            st = e.run()
            prof = e.profile()
            trace = e.join_trace() if kw.get("flags", 0) & (self.fv.FV_LOG_JOINS | self.fv.FV_LEARNED) else None
            return st, prof, trace
        finally:
            e.close()

    def time_runs(self, reps, **kw):
        """Median fv_run_fixpoint time (ms) over fresh contexts; last stats."""
        ms, st = [], None
        for _ in range(reps):
            st, _, _ = self.run_once(**kw)
            ms.append(st["ms_total"])
        return sorted(ms)[len(ms) // 2], st


def training_suite(W):
    """Plain-engine runs whose join traces train the predictor: transitive
    closure, same generation, points-to and acknowledged reachability (its
    recursive rule in both body orders, so that both join orders appear) at
    several sizes and seeds, and single joins of uniform and Zipf keys.  The
    RDFS headline workload is held out."""
    ack_swapped = W.ACK_PROGRAM.replace("fan(y, z), ack(z, x)", "ack(z, x), fan(y, z)")
    suite = [(W.TC_PROGRAM, {"edge": W.config_tc().edb["edge"]}, ["path"])]
    for n, m, seed in ((1000, 3000, 21), (4000, 6000, 22), (500, 2500, 23)):
        suite.append((W.TC_PROGRAM, {"edge": W.er_graph(n, m, seed=seed)}, ["path"]))
    suite.append((W.SG_PROGRAM, W.config_sg().edb, ["sg"]))
    for trees, nodes, extra, seed in ((16, 512, 0.10, 31), (32, 256, 0.02, 32)):
        suite.append((W.SG_PROGRAM, {"edge": W.forest(trees, nodes, extra, seed=seed)}, ["sg"]))
    for scale, seed in ((1.0, 1003), (0.2, 1013), (0.05, 1023)):
        pt = W.config_pointsto(seed=seed, scale=scale)
        suite.append((pt.program, pt.edb, list(pt.idb)))
    for args in ((32, 256, 128, 16, 1007), (128, 128, 32, 32, 41), (64, 512, 64, 8, 42)):
        a = W.ack_reach(*args)
        suite.append((a.program, a.edb, ["r"]))
        suite.append((ack_swapped, a.edb, ["r"]))
    for n_probe, n_keys, zipf_s in ((1 << 16, 1 << 12, 0.0), (1 << 18, 1 << 10, 1.0), (1 << 17, 1 << 16, 0.5)):
        j = W.join_case(n_probe, n_keys, zipf_s)
        suite.append((j.program, j.edb, ["out"]))
    return suite


def collect_traces(fv, W, torch, np):
    """Join traces (features, true sizes) the plain engine logs on the
    training suite and on the batched transitive-closure instances: the
    predictor's training data."""
    rows = []
    for program, edb, rels in training_suite(W):
        r = Runner(fv, torch, np, program, edb, rels)
        _, _, trace = r.run_once(flags=fv.FV_LOG_JOINS)
        rows.append(trace)
        del r
    insts = W.batched_tc_instances()
    es = []
    for x in insts:
        e = fv.Engine(flags=fv.FV_LOG_JOINS)
        e.relation("edge", 2)
        e.relation("path", 2)
        e.load("edge", x.edb["edge"])
        e.program(x.program)
        es.append(e)
    fv.run_batch(es)
    rows.append(es[0].join_trace())   # the merged run's trace is reported on the first instance
    for e in es:
        e.close()
    return np.concatenate(rows)


def qerror_by_step(trace, np):
    """Median and max q-error (max(m/p, p/m) on sizes + 1) per position in
    the join chain, from a learned run's trace."""
    out = {}
    m = np.exp2(trace[:, 8].astype(np.float64) * 16) - 1
    p = trace[:, 9].astype(np.float64)
    for step in sorted(set(trace[:, 7].astype(int).tolist())):
        sel = trace[:, 7] == step
        q = np.maximum((m[sel] + 1) / (p[sel] + 1), (p[sel] + 1) / (m[sel] + 1))
        out[f"step{step}"] = {"joins": int(sel.sum()), "median": round(float(np.median(q)), 3),
                              "max": round(float(q.max()), 3)}
    return out


def compare_learned(fv, np, rd, args, tuning, learned, T, train_loss, trace, reps):
    """The headline workload and knobs without the network: the plain engine,
    and the learned path with a zero predictor (presizing from the
    uniform-key estimate alone), untraced, median of `reps` fixpoints each."""
    plain_ms, plain_st = rd.time_runs(reps, tuning=tuning)
    zero_ms, zero_st = rd.time_runs(reps, tuning=tuning, flags=fv.FV_LEARNED,
                                    predictor=np.zeros(fv.MLP_PARAMS, np.float32))
    trained_ms, trained_st = rd.time_runs(reps, tuning=tuning, **learned)
    return {
        "train_records": int(len(T)), "train_loss": round(train_loss, 6),
        "plain_ms": round(plain_ms, 2), "zero_predictor_ms": round(zero_ms, 2), "trained_ms": round(trained_ms, 2),
        "speedup_vs_plain": round(plain_ms / trained_ms, 3), "speedup_vs_zero_predictor": round(zero_ms / trained_ms, 3),
        "plain_redo_rounds": plain_st["redo_rounds"], "zero_predictor_redo_rounds": zero_st["redo_rounds"],
        "zero_predictor_overflow_fallbacks": zero_st["overflows"],
        "trained_redo_rounds": trained_st["redo_rounds"], "trained_overflow_fallbacks": trained_st["overflows"],
        "predicted_joins": trained_st["predicted_joins"], "qerror_median": round(trained_st["qerror_median"], 3),
        "qerror_max": round(trained_st["qerror_max"], 3), "qerror_by_chain_step": qerror_by_step(trace, np)}


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this engine runs on a single "
              "device and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2501_13051_amd import fv
    from paper_2501_13051_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.sweep_only:
        copy_probe(torch, args)
        print(json.dumps({"large_join_sweep": join_sweep(fv, W, torch, np, args.sweep_case)}), flush=True)
        return

    # the predictor: trained here, on this GPU, from the plain engine's traces
    if args.load_predictor:
        params = np.load(args.load_predictor).astype(np.float32)
        T, train_loss = np.zeros((0, 10), np.float32), float("nan")
        log(f"predictor parameters from {args.load_predictor}")
    else:
        log("collecting join traces of the plain engine (training suite, batched TC)")
        T = collect_traces(fv, W, torch, np)
        params, train_loss = fv.mlp_train(T[:, :8], T[:, 8], steps=4000, lr=3e-3, seed=1)
        log(f"trained the predictor on {len(T)} join records, loss {train_loss:.5f}")
    if args.save_predictor:
        np.save(args.save_predictor, params)

    w = W.config_rdfs()
    rd = Runner(fv, torch, np, w.program, w.edb, ["t"])
    learned = dict(flags=fv.FV_LEARNED, predictor=params)

    tuning, tuning_source = None, "defaults"
    if not args.no_autotune:
        key = "rdfs_t20000000_learned"
        tuning = None if args.retune or not os.path.exists(args.tuning_cache) else fv.tuning_load(args.tuning_cache, key)
        tuning_source = "autotuner cache"
        if tuning is None:
            log("autotuning the engine on the learned RDFS workload")
            tuning = fv.autotune(lambda t: rd.make(tuning=t, **learned), key=key, cache_path=args.tuning_cache,
                                 reps=3)
            tuning_source = "autotuner (this run)"
        log(f"tuning {tuning} ({tuning_source})")
    copy_probe(torch, args)

    # dominant kernel class: most time over three traced passes (outside the timed region)
    per_class = {}
    for _ in range(3):
        _, prof, _ = rd.run_once(flags=fv.FV_TRACE | fv.FV_LEARNED, predictor=params, tuning=tuning)
        for k in prof:
            if not k["name"].startswith("host_"):   # host phases of a round are not kernels
                per_class[k["name"]] = per_class.get(k["name"], 0.0) + k["ms"]
    dom_name = max(per_class, key=per_class.get)
    log(f"dominant kernel class: {dom_name}")

    traced = dict(flags=fv.FV_TRACE | fv.FV_LEARNED, predictor=params, tuning=tuning, trace_only=dom_name)
    for _ in range(args.warmup):
        rd.run_once(**traced)
    # A step is one fixpoint (fv_run_fixpoint: EDB ingest, index builds and
    # every round to the fixpoint).  Each step's context is created and loaded
    # from the resident EDB before its timed region, as the metric excludes
    # the load, and read and closed after it; the timed regions are summed.
    log(f"timing {args.steps} steps")
    dom = {"launches": 0, "ms": 0.0, "algo_bytes": 0.0, "items": 0}
    derived = iters = st = trace = None
    elapsed = 0.0
    for _ in range(args.steps):
        e = rd.make(**traced)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = e.run()
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        derived, iters = st["derived_tuples"], st["iterations"]
        for k in e.profile():
            if k["name"] == dom_name:
                for f in dom:
                    dom[f] += k[f]
        trace = e.join_trace()
        e.close()
    ms_per_step = elapsed * 1000.0 / max(args.steps, 1)
    value = derived * args.steps / elapsed if elapsed > 0 else 0.0
    achieved = dom["algo_bytes"] / (dom["ms"] * 1e-3) / 1e9 if dom["ms"] > 0 else 0.0
    traffic = measured_traffic(dom_name)
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": round(traffic, 1) if traffic is not None else None,
                "avg_launch_ms": round(dom["ms"] / max(dom["launches"], 1), 5),
                "launches_per_step": dom["launches"] / max(args.steps, 1),
                "algo_bytes_per_launch": round(dom["algo_bytes"] / max(dom["launches"], 1), 1)}

    # the same workload and knobs without the network: the plain engine, and
    # the learned path with a zero predictor (presizing from the uniform-key
    # estimate alone), untraced, median of three fixpoints each
    reps = max(3, args.steps // 3)
    learned_form = None
    if not args.no_compare:
        learned_form = compare_learned(fv, np, rd, args, tuning, learned, T, train_loss, trace, reps)

    out = {
        "metric": "derived tuples/s to fixpoint",
        "value": round(value, 1),
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "RDFS reasoning to fixpoint over 20M synthetic triples (class tree of 8 levels x "
                               "fan-out 6, 200 properties in 4 levels, domain/range on every second property, 10 "
                               "transitive properties, Zipf(1) entities, types and properties), seed 1005, learned "
                               "join-cardinality MLP on",
                   "triples": w.meta["triples"], "derived_tuples": derived, "rounds": iters,
                   "engine": "semi-naive, learned presizing with exact count-then-write fallback, autotuned knobs",
                   "tuning": tuning, "tuning_source": tuning_source,
                   "redo_rounds": st["redo_rounds"], "overflow_fallbacks": st["overflows"]},
        "roofline": roofline,
        "cpu_baseline": None,
        "learned_vs_plain": learned_form,
    }

    if not args.no_extras:
        out["forms"] = extras(fv, W, torch, np, args)
        out["forms"]["learned_join_order"] = join_order_form(fv, W, torch, np, params, reps)
        out["forms"]["difference_ab"] = difference_form(fv, W, torch, np, rd, tuning, learned, args)
        out["forms"]["host_engine"] = host_form(fv, W, torch, np)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W):
    """The oracle (single-threaded sorted-vector semi-naive) on the same
    workload at 1/10 scale, pinned to one host core, once."""
    import oracle
    log("timing the oracle on a 1/10-scale sample of the RDFS workload")
    sample = W.config_rdfs(scale=0.1)
    old = os.sched_getaffinity(0)
    core = min(old)
    try:
        os.sched_setaffinity(0, {core})
        r = oracle.evaluate(sample.program, sample.edb, relations=["t"])
    finally:
        os.sched_setaffinity(0, old)
    derived = sum(r.delta_sizes)
    return {"value": round(derived / r.seconds, 1), "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": f"the RDFS generator at 1/10 scale ({sample.meta['triples']} triples, same rules and "
                      f"hierarchies): {derived} derived tuples in {r.seconds:.2f} s, one run pinned to host core "
                      f"{core} ({cpu_model()}; {len(old)} cores available to the process)"}


def extras(fv, W, torch, np, args):
    forms = {}
    # --- same generation (the round-1 headline), autotuned knobs
    log("same-generation form")
    wsg = W.config_sg()
    sg = Runner(fv, torch, np, wsg.program, wsg.edb, ["sg"])
    key = "sg_forest_t64_n1024"
    sg_tune = fv.tuning_load(args.tuning_cache, key) if os.path.exists(args.tuning_cache) else None
    sg.run_once(tuning=sg_tune)
    sg_ms, sg_st = sg.time_runs(max(5, args.steps), tuning=sg_tune)
    forms["sg_forest_64x1024"] = {"ms_per_fixpoint": round(sg_ms, 3), "derived_tuples": int(sg_st["derived_tuples"]),
                                  "tuples_per_s": round(sg_st["derived_tuples"] / (sg_ms * 1e-3), 1),
                                  "rounds": sg_st["iterations"], "tuning": sg_tune}
    del sg

    # --- batched: 512 independent TC instances, one fixpoint vs 512 fixpoints
    log("batched form: 512 transitive-closure instances")
    insts = W.batched_tc_instances()
    runners = [Runner(fv, torch, np, x.program, x.edb, ["path"]) for x in insts]

    def serial():
        es = [r.make() for r in runners]
        torch.cuda.synchronize()
        t = time.perf_counter()
        tot = 0
        for e in es:
            tot += e.run()["derived_tuples"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        for e in es:
            e.close()
        return dt, tot

    def batched(flags):
        es = [r.make(flags=flags) for r in runners]
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = fv.run_batch(es)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        for e in es:
            e.close()
        return dt, st

    serial()
    ts, tot = serial()
    batched(0)
    tb, stb = batched(0)
    batched(fv.FV_GRAPH)
    tg, stg = batched(fv.FV_GRAPH)
    forms["batched_tc_512"] = {
        "derived_tuples": int(tot), "serial_plain_ms": round(ts * 1e3, 2), "batched_ms": round(tb * 1e3, 2),
        "batched_graph_ms": round(tg * 1e3, 2), "speedup": round(ts / min(tb, tg), 2),
        "rounds": stb["iterations"], "graph_replays": stg["graph_replays"],
        "tuples_per_s_batched": round(tot / min(tb, tg), 1)}
    del runners

    # --- one join at large sizes: per-kernel bandwidth where sizes are not
    # latency-bound (probe 2^24..2^26 rows against 2^20..2^22 keys)
    log("large-join sweep")
    forms["large_join_sweep"] = join_sweep(fv, W, torch, np)

    # --- autotuned single-instance points-to
    log("autotuned form: points-to")
    pt = W.config_pointsto()
    pr = Runner(fv, torch, np, pt.program, pt.edb, list(pt.idb))
    pr.run_once()
    p_ms, p_st = pr.time_runs(3)
    key = "pointsto_n200000"
    tune = fv.tuning_load(args.tuning_cache, key) if os.path.exists(args.tuning_cache) and not args.retune else None
    if tune is None:
        tune = fv.autotune(lambda t: pr.make(tuning=t), key=key, cache_path=args.tuning_cache, reps=3)
    t_ms, t_st = pr.time_runs(3, tuning=tune)
    forms["autotuned_pointsto"] = {"plain_ms": round(p_ms, 2), "tuned_ms": round(t_ms, 2),
                                   "speedup": round(p_ms / t_ms, 3), "tuning": tune,
                                   "derived_tuples": int(t_st["derived_tuples"]),
                                   "tuples_per_s_tuned": round(t_st["derived_tuples"] / (t_ms * 1e-3), 1)}
    return forms


def join_order_form(fv, W, torch, np, params, reps):
    """The acknowledged-reachability program (1024 groups of 256 nodes): its
    recursive rule can join fan (about 128 rows per key) or ack (about 16)
    first.  The plain engine and the zero predictor keep the default order;
    the trained network picks the order from its predicted intermediate
    sizes.  Untraced, median of `reps` fixpoints each."""
    log("learned join order: acknowledged reachability")
    w = W.ack_reach(1024)
    r = Runner(fv, torch, np, w.program, w.edb, ["r"])
    out = {"workload": w.name, "edb_rows": {k: int(len(v[0])) for k, v in w.edb.items()}}
    for name, kw in (("plain", {}),
                     ("zero_predictor", dict(flags=fv.FV_LEARNED, predictor=np.zeros(fv.MLP_PARAMS, np.float32))),
                     ("trained", dict(flags=fv.FV_LEARNED, predictor=params))):
        r.run_once(**kw)
        ms, st = r.time_runs(reps, **kw)
        out[name] = {"ms": round(ms, 2), "join_output_tuples": int(st["join_output_tuples"]),
                     "reordered_rounds": int(st["reordered_rounds"]), "derived_tuples": int(st["derived_tuples"])}
    out["speedup_trained_vs_zero_predictor"] = round(out["zero_predictor"]["ms"] / out["trained"]["ms"], 3)
    out["speedup_trained_vs_plain"] = round(out["plain"]["ms"] / out["trained"]["ms"], 3)
    del r
    return out


def difference_form(fv, W, torch, np, rd, tuning, learned, args):
    """The three differences against full side by side: the tuple set of
    full's packed tuples (the default), Algorithm 2's range test over
    per-column indices of full, and the search of each sorted tile's window
    of full's sorted keys with a merge after every round (dedup_ranges 0, 1,
    2), on the headline (same knobs otherwise) and on the same-generation
    forest.  Median of three fixpoints (five on the forest), one for
    Algorithm 2 on RDFS."""
    log("difference A/B: tuple set, Algorithm 2, sorted merge")
    names = {0: "tuple_set", 1: "ranges", 2: "sorted_merge"}
    out = {}
    base = dict(tuning) if tuning else {}
    # (Algorithm 2 takes about 20 s per RDFS fixpoint: one run, no warm-up)
    for mode, reps in ((0, 3), (2, 3), (1, 1)):
        t = dict(base, dedup_ranges=mode)
        if mode != 1:
            rd.run_once(tuning=t, **learned)
        ms, st = rd.time_runs(reps, tuning=t, **learned)
        out[f"rdfs_20M_learned_{names[mode]}_ms"] = round(ms, 2)
    wsg = W.config_sg()
    sg = Runner(fv, torch, np, wsg.program, wsg.edb, ["sg"])
    for mode in (0, 2, 1):
        t = {"dedup_ranges": mode}
        sg.run_once(tuning=t)
        ms, _ = sg.time_runs(5, tuning=t)
        out[f"sg_forest_64x1024_{names[mode]}_ms"] = round(ms, 3)
    del sg
    return out


def host_form(fv, W, torch, np):
    """The same engine on host threads (FV_HOST) against the GPU engine, on
    the same-generation forest and on the RDFS generator at 1/20 scale; the
    process is held to 16 host cores (its share of the machine) while the
    host engine runs, and the GPU runs are the plain engine with default
    knobs.  Median of three fixpoints each."""
    out = {}
    old = os.sched_getaffinity(0)
    cores = sorted(old)[:16]
    for label, w, rels in (("sg_forest_64x1024", W.config_sg(), ["sg"]),
                           ("rdfs_1M_triples", W.config_rdfs(scale=0.05), ["t"])):
        log(f"host engine form: {label}")
        g = Runner(fv, torch, np, w.program, w.edb, rels)
        g.run_once()
        g_ms, g_st = g.time_runs(3)
        del g
        h_ms = []
        try:
            os.sched_setaffinity(0, set(cores))
            for _ in range(3):
                e = fv.Engine(flags=fv.FV_HOST)
                for name, a in Runner.arity_of(fv, w.program, w.edb).items():
                    e.relation(name, a)
                for name, cols in w.edb.items():
                    e.load(name, [np.ascontiguousarray(np.asarray(c, np.uint32)) for c in cols])
                e.program(w.program)
                st = e.run()
                h_ms.append(st["ms_total"])
                assert st["derived_tuples"] == g_st["derived_tuples"], (label, st["derived_tuples"])
                e.close()
        finally:
            os.sched_setaffinity(0, old)
        h = sorted(h_ms)[1]
        out[label] = {"gpu_ms": round(g_ms, 2), "host_ms": round(h, 2), "host_threads": len(cores),
                      "gpu_over_host": round(h / g_ms, 2), "derived_tuples": int(g_st["derived_tuples"]),
                      "host_cpu": cpu_model()}
    return out


def copy_probe(torch, args):
    """A device copy of known size, for calibrating the HBM traffic counters."""
    if args.copy_probe_mb <= 0:
        return
    n = args.copy_probe_mb << 18
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    log(f"copy probe: {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written")
    del x, y


def join_sweep(fv, W, torch, np, only=-1):
    cases = []
    sizes = ((1 << 24, 1 << 20, 0.0), (1 << 26, 1 << 22, 0.0), (1 << 25, 1 << 21, 1.0))
    for i, (n_probe, n_keys, zipf_s) in enumerate(sizes):
        if only >= 0 and i != only:
            continue
        w = W.join_case(n_probe, n_keys, zipf_s)
        r = Runner(fv, torch, np, w.program, w.edb, ["out"])
        r.run_once(flags=fv.FV_TRACE)
        st, prof, _ = r.run_once(flags=fv.FV_TRACE)
        kernels = {}
        for k in prof:
            if not k["launches"] or k["ms"] <= 0 or k["name"].startswith("host_"):
                continue
            gbs = k["algo_bytes"] / (k["ms"] * 1e-3) / 1e9
            kernels[k["name"]] = {"ms": round(k["ms"], 3), "launches": k["launches"], "GB_s": round(gbs, 1),
                                  "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
        cases.append({"case": w.name, "derived_tuples": int(st["derived_tuples"]),
                      "ms_fixpoint": round(st["ms_total"], 3),
                      "tuples_per_s": round(st["derived_tuples"] / (st["ms_total"] * 1e-3), 1), "kernels": kernels})
        del r
        torch.cuda.empty_cache()
    return cases


if __name__ == "__main__":
    main()
