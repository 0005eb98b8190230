"""Seeded synthetic inputs and the Datalog programs that run on them.

This module is the one place both sides of a parity check take their inputs
from: it draws edge lists and triple tables from a counter-based SplitMix64
stream and holds the rule texts.  It contains none of the evaluation
arithmetic (no joins, no deduplication, no fixpoint): it only produces EDB
relations as uint32 column arrays and program texts.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): output k of a stream with seed s is
mix64(s + (k + 1) * 0x9E3779B97F4A7C15) with the finalizer below.  Because
every output is a pure function of (seed, k), a stream can be consumed in
vectorised blocks.

The paper evaluates on SuiteSparse/SNAP graphs and on LUBM (Section 5);
none of those datasets is available, so the generators below stand in for
them with graphs and triple tables of the same kind (directed graphs with
recursive closure, forests with same-generation structure, power-law
assignment graphs, an RDFS-style triple store).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Counter-based SplitMix64 stream; `take(k)` returns the next k outputs."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.counter = 0

    def take(self, k: int) -> np.ndarray:
        idx = np.arange(self.counter + 1, self.counter + 1 + k, dtype=np.uint64)
        self.counter += k
        with np.errstate(over="ignore"):
            return _mix64(self.seed + idx * GOLDEN)

    def below(self, n, k: int) -> np.ndarray:
        """k integers uniform in [0, n) (n scalar or array, n < 2^32):
        the high 32 bits of an output times n, shifted down 32."""
        x = self.take(k) >> np.uint64(32)
        return ((x * np.asarray(n, dtype=np.uint64)) >> np.uint64(32)).astype(np.int64)

    def unit(self, k: int) -> np.ndarray:
        """k floats uniform in [0, 1): top 53 bits times 2^-53."""
        return (self.take(k) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _cols(pairs) -> list[np.ndarray]:
    a = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
    return [np.ascontiguousarray(a[:, 0]), np.ascontiguousarray(a[:, 1])]


# ---------------------------------------------------------------- programs
# Rule texts in a small Datalog syntax: `head(t,..) :- atom(t,..), ..., x != y.`
# Terms are variables (identifiers) or unsigned decimal constants; `_` is a
# fresh variable at every occurrence; `%` starts a comment.

TC_PROGRAM = """
path(x, y) :- edge(x, y).
path(x, z) :- path(x, y), edge(y, z).
"""

# Transitive closure in the left-recursive form the paper states it in
# (Section 2): the recursive atom is the second body atom.
TC_PROGRAM_PAPER_FORM = """
reach(x, y) :- edge(x, y).
reach(x, z) :- edge(x, y), reach(y, z).
"""

# Same generation as the benchmark configuration states it: the x != y
# filter sits only on the base rule.
SG_PROGRAM = """
sg(x, y) :- edge(p, x), edge(p, y), x != y.
sg(x, y) :- edge(a, x), sg(a, b), edge(b, y).
"""

# Same generation exactly as Section 5.2 prints it: x != y on both rules.
SG_PROGRAM_PAPER_FORM = """
sg(x, y) :- edge(p, x), edge(p, y), x != y.
sg(x, y) :- edge(a, x), sg(a, b), edge(b, y), x != y.
"""


# ---------------------------------------------------------------- workloads
@dataclass
class Workload:
    name: str
    program: str
    edb: dict = field(default_factory=dict)      # name -> list of uint32 column arrays
    idb: tuple = ()                              # relations whose fixpoint is compared
    meta: dict = field(default_factory=dict)

    def n_edb_rows(self) -> int:
        return sum(len(c[0]) for c in self.edb.values())


def er_graph(n_nodes: int, n_edges: int, seed: int) -> list[np.ndarray]:
    """Directed Erdos-Renyi-style graph: candidate (u, v) pairs drawn
    uniformly from [0, n)^2 in stream order; self-loops and repeats are
    rejected until exactly n_edges distinct edges remain."""
    if n_edges > n_nodes * (n_nodes - 1):
        raise ValueError("more edges than ordered node pairs")
    rng = SplitMix64(seed)
    seen, out = set(), []
    while len(out) < n_edges:
        need = n_edges - len(out)
        cand = rng.below(n_nodes, 2 * max(64, 2 * need)).reshape(-1, 2)
        for u, v in cand.tolist():
            if u == v or (u, v) in seen:
                continue
            seen.add((u, v))
            out.append((u, v))
            if len(out) == n_edges:
                break
    return _cols(out)


def recursive_tree_edges(n_nodes: int, n_extra: int, rng: SplitMix64, base: int = 0):
    """A random recursive tree on nodes 0..n-1 (node i >= 1 attaches to a
    parent drawn uniformly from [0, i)), parent->child edges, plus n_extra
    distinct forward edges (a, b) with a < b in insertion order.  Ids are
    offset by `base`."""
    i = np.arange(1, n_nodes, dtype=np.int64)
    parent = rng.below(i, n_nodes - 1) if n_nodes > 1 else np.zeros(0, np.int64)
    edges = set(zip(parent.tolist(), i.tolist()))
    extra = []
    if n_extra > n_nodes * (n_nodes - 1) // 2 - (n_nodes - 1):
        raise ValueError("too many extra forward edges")
    while len(extra) < n_extra:
        cand = rng.below(n_nodes, 2 * max(16, 2 * (n_extra - len(extra)))).reshape(-1, 2)
        for a, b in cand.tolist():
            if a == b:
                continue
            if a > b:
                a, b = b, a
            if (a, b) in edges:
                continue
            edges.add((a, b))
            extra.append((a, b))
            if len(extra) == n_extra:
                break
    pairs = list(zip(parent.tolist(), i.tolist())) + extra
    arr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2) + base
    return arr


def forest(n_trees: int, nodes_per_tree: int, extra_frac: float, seed: int,
           id_stride: int | None = None) -> list[np.ndarray]:
    """Random forest: n_trees random recursive trees, each with
    round(extra_frac * (nodes-1)) extra in-tree forward edges; tree t's
    node i gets global id t * id_stride + i."""
    rng = SplitMix64(seed)
    stride = nodes_per_tree if id_stride is None else id_stride
    n_extra = int(round(extra_frac * (nodes_per_tree - 1)))
    parts = [recursive_tree_edges(nodes_per_tree, n_extra, rng, base=t * stride)
             for t in range(n_trees)]
    arr = np.concatenate(parts, axis=0) if parts else np.zeros((0, 2), np.int64)
    return _cols(arr)


def config_tc(seed: int = 1001, n_nodes: int = 2000, n_edges: int = 3000) -> Workload:
    """Transitive closure over a directed G(n=2000, m=3000) graph."""
    return Workload(
        name=f"tc_er_n{n_nodes}_m{n_edges}", program=TC_PROGRAM,
        edb={"edge": er_graph(n_nodes, n_edges, seed)}, idb=("path",),
        meta={"nodes": n_nodes, "edges": n_edges, "seed": seed})


def config_sg(seed: int = 1002, n_trees: int = 64, nodes: int = 1024,
              extra_frac: float = 0.05) -> Workload:
    """Same generation over a forest of 64 random recursive trees of 1,024
    nodes with 5% extra forward edges per tree."""
    edge = forest(n_trees, nodes, extra_frac, seed)
    return Workload(
        name=f"sg_forest_t{n_trees}_n{nodes}", program=SG_PROGRAM,
        edb={"edge": edge}, idb=("sg",),
        meta={"trees": n_trees, "nodes_per_tree": nodes, "extra_frac": extra_frac,
              "seed": seed, "edges": int(len(edge[0]))})


def batched_tc_instances(seed: int = 1004, n_instances: int = 512, nodes: int = 256,
                         min_trees: int = 2, max_trees: int = 64,
                         extra_frac: float = 0.10) -> list[Workload]:
    """Independent transitive-closure instances for the batched form: each
    is a forest of round(exp(U(ln 2, ln 64))) trees of 256 nodes with 10%
    extra in-tree forward edges; local ids are tree * 256 + i."""
    rng = SplitMix64(seed)
    u = rng.unit(n_instances)
    trees = np.rint(np.exp(math.log(min_trees) + u * (math.log(max_trees) - math.log(min_trees))))
    out = []
    for k in range(n_instances):
        edge = forest(int(trees[k]), nodes, extra_frac, seed * 1_000_003 + k)
        out.append(Workload(name=f"tc_forest_inst{k}", program=TC_PROGRAM,
                            edb={"edge": edge}, idb=("path",),
                            meta={"trees": int(trees[k]), "nodes_per_tree": nodes}))
    return out


# ---------------------------------------------------------------- tiny shapes
def chain(n: int) -> list[np.ndarray]:
    return _cols([(i, i + 1) for i in range(n - 1)])


def cycle(n: int) -> list[np.ndarray]:
    return _cols([(i, (i + 1) % n) for i in range(n)])


def complete_dag(n: int) -> list[np.ndarray]:
    return _cols([(i, j) for i in range(n) for j in range(i + 1, n)])


def star(k: int) -> list[np.ndarray]:
    return _cols([(0, j) for j in range(1, k + 1)])


# ---------------------------------------------------------------- points-to
# Inclusion-based (Andersen-style) alias analysis, written from the
# context-free-language formulation of Zheng and Rugina ("Demand-driven alias
# analysis for C", POPL 2008):  value flow F ::= (assign M?)*,  memory alias
# M ::= deref^-1 V deref,  value alias V ::= F^-1 M? F.
# assign(a, b) is the statement a = b (the value of b flows into a);
# dereference(p, l) says l is the memory expression *p.
POINTSTO_PROGRAM = """
valueFlow(x, x) :- assign(x, _).
valueFlow(x, x) :- assign(_, x).
valueFlow(b, a) :- assign(a, b).
valueFlow(u, w) :- assign(v, u), memoryAlias(v, w).
valueFlow(x, z) :- valueFlow(x, y), valueFlow(y, z).
memoryAlias(l, m) :- dereference(p, l), valueAlias(p, q), dereference(q, m).
valueAlias(p, q) :- valueFlow(v, p), valueFlow(v, q).
valueAlias(p, q) :- valueFlow(u, p), memoryAlias(u, w), valueFlow(w, q).
"""


def zipf_sources(n_nodes: int, n_edges: int, s: float, rng: SplitMix64) -> np.ndarray:
    """Edge sources whose out-degrees follow Zipf's law with exponent s over
    a random ranking of the nodes: the node of rank k is drawn with
    probability proportional to k^-s (many nodes get no edge at all)."""
    rank_of = np.argsort(rng.take(n_nodes), kind="stable")      # random permutation
    w = 1.0 / np.arange(1, n_nodes + 1, dtype=np.float64) ** s
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.unit(n_edges)
    r = np.minimum(np.searchsorted(cdf, u, side="right"), n_nodes - 1)
    return rank_of[r]


def pointsto_graph(n_nodes: int = 200_000, n_assign: int = 400_000, n_deref: int = 100_000,
                   s: float = 1.5, seed: int = 1003) -> dict:
    """assign: n_assign distinct non-loop edges (a, b), sources a with Zipf
    out-degrees, targets b uniform over the nodes.  dereference: n_deref
    edges from uniformly drawn pointer nodes to fresh location nodes (ids
    n_nodes ..), one location per edge."""
    rng = SplitMix64(seed)
    seen, out = set(), []
    while len(out) < n_assign:
        need = n_assign - len(out)
        a = zipf_sources(n_nodes, 2 * need + 64, s, rng)
        b = rng.below(n_nodes, 2 * need + 64)
        for x, y in zip(a.tolist(), b.tolist()):
            if x == y or (x, y) in seen:
                continue
            seen.add((x, y))
            out.append((x, y))
            if len(out) == n_assign:
                break
    ptr = rng.below(n_nodes, n_deref)
    loc = np.arange(n_nodes, n_nodes + n_deref, dtype=np.int64)
    return {"assign": _cols(out), "dereference": _cols(np.stack([ptr, loc], axis=1))}


def config_pointsto(seed: int = 1003, scale: float = 1.0) -> Workload:
    """Andersen-style points-to over a power-law assignment graph of 200,000
    nodes / 400,000 edges and 100,000 dereference edges (scale shrinks all
    three counts together)."""
    n = max(8, int(200_000 * scale))
    edb = pointsto_graph(n, int(400_000 * scale), int(100_000 * scale), 1.5, seed)
    return Workload(name=f"pointsto_n{n}", program=POINTSTO_PROGRAM, edb=edb,
                    idb=("valueFlow", "valueAlias", "memoryAlias"),
                    meta={"nodes": n, "assign": int(400_000 * scale), "deref": int(100_000 * scale),
                          "zipf_s": 1.5, "seed": seed})


# ---------------------------------------------------------------- RDFS
# RDFS entailment over one triple relation t(s, p, o), after the W3C RDF 1.1
# Semantics entailment patterns (rdfs2, rdfs3, rdfs5, rdfs7, rdfs9, rdfs11)
# plus the transitive-property rule of OWL 2 RL (prp-trp).  Reserved ids:
# 0 type, 1 subClassOf, 2 subPropertyOf, 3 domain, 4 range, 5 the class of
# transitive properties.
RDF_TYPE, RDFS_SC, RDFS_SP, RDFS_DOM, RDFS_RNG, OWL_TRANS = 0, 1, 2, 3, 4, 5
RDFS_PROGRAM = """
t(c, 1, e) :- t(c, 1, d), t(d, 1, e).
t(p, 2, r) :- t(p, 2, q), t(q, 2, r).
t(s, q, o) :- t(s, p, o), t(p, 2, q).
t(s, 0, c) :- t(s, p, o), t(p, 3, c).
t(o, 0, c) :- t(s, p, o), t(p, 4, c).
t(s, 0, d) :- t(s, 0, c), t(c, 1, d).
t(x, p, z) :- t(p, 0, 5), t(x, p, y), t(y, p, z).
"""


def _zipf_pick(n: int, k: int, s: float, rng: SplitMix64, ranked: np.ndarray | None = None) -> np.ndarray:
    """k draws from n items with P(rank r) proportional to r^-s; `ranked`
    maps rank -> item (default: a random permutation)."""
    if ranked is None:
        ranked = np.argsort(rng.take(n), kind="stable")
    w = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** s
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    r = np.minimum(np.searchsorted(cdf, rng.unit(k), side="right"), n - 1)
    return ranked[r]


def rdfs_triples(n_triples: int = 20_000_000, class_depth: int = 8, fanout: int = 6,
                 n_props: int = 200, n_entities: int = 1_700_000, n_trans: int = 10,
                 trans_share: float = 0.1, trans_tree: int = 256, seed: int = 1005) -> dict:
    """Synthetic RDFS triple table.

    * classes: a complete `fanout`-ary tree with `class_depth` levels
      (root = level 0), one subClassOf triple per non-root class;
    * properties: 8 root properties and three more levels (24, 72, 96
      properties, 200 in all) under subPropertyOf;
    * every second property gets a domain and a range class;
    * n_trans properties are typed as transitive; their triples form random
      recursive trees of `trans_tree` entities (acyclic, so the closure stays
      bounded: sum of depths);
    * each entity gets one type, the class drawn Zipf(1.0) over a random
      class ranking; the remaining triples draw subject and object Zipf(1.0)
      over a random entity ranking and the property Zipf(1.0) over the
      properties in hierarchy order (roots most frequent).
    Ids: reserved 0..5, properties from 6, then classes, then entities."""
    rng = SplitMix64(seed)
    P0 = 6
    n_classes = (fanout ** class_depth - 1) // (fanout - 1)
    C0 = P0 + n_props
    E0 = C0 + n_classes
    s_, p_, o_ = [], [], []

    def add(s, p, o):
        s_.append(np.asarray(s, np.int64))
        p_.append(np.broadcast_to(np.asarray(p, np.int64), np.shape(s)).copy())
        o_.append(np.asarray(o, np.int64))

    k = np.arange(1, n_classes, dtype=np.int64)
    add(C0 + k, RDFS_SC, C0 + (k - 1) // fanout)
    # property hierarchy: levels of 8, 24, 72, 96
    levels = [8, 24, 72, n_props - 104]
    parent = np.full(n_props, -1, np.int64)
    start = 0
    for lv in range(1, 4):
        prev_start, prev_n = start, levels[lv - 1]
        start += prev_n
        idx = np.arange(start, start + levels[lv])
        parent[idx] = prev_start + (idx - start) % prev_n
    child = np.nonzero(parent >= 0)[0]
    add(P0 + child, RDFS_SP, P0 + parent[child])
    dprops = np.arange(0, n_props, 2)
    add(P0 + dprops, RDFS_DOM, C0 + rng.below(n_classes, len(dprops)))
    add(P0 + dprops, RDFS_RNG, C0 + rng.below(n_classes, len(dprops)))
    trans = np.arange(n_props - n_trans, n_props)          # deepest properties
    add(P0 + trans, RDF_TYPE, np.full(n_trans, OWL_TRANS))
    ent = E0 + np.arange(n_entities, dtype=np.int64)
    add(ent, RDF_TYPE, C0 + _zipf_pick(n_classes, n_entities, 1.0, rng))
    used = sum(len(x) for x in s_)
    rest = n_triples - used
    n_tr = int(rest * trans_share)
    per = n_tr // n_trans
    for j in trans:
        nodes = rng.below(n_entities, per + 1)              # tree vertices (may repeat: merged nodes)
        i = np.arange(1, per + 1, dtype=np.int64)
        i = i[np.arange(len(i)) % trans_tree != 0]          # every trans_tree-th vertex starts a new tree
        par = i - 1 - rng.below(np.minimum(i % trans_tree, i), len(i))
        keep = nodes[par] < nodes[i]                        # orient by entity order: acyclic
        add(E0 + nodes[par][keep], P0 + j, E0 + nodes[i][keep])
    used = sum(len(x) for x in s_)
    rest = n_triples - used
    ents = np.argsort(rng.take(n_entities), kind="stable")
    props = np.arange(n_props - n_trans)                    # hierarchy order: roots first
    add(E0 + _zipf_pick(n_entities, rest, 1.0, rng, ents),
        P0 + _zipf_pick(len(props), rest, 1.0, rng, props),
        E0 + _zipf_pick(n_entities, rest, 1.0, rng, ents))
    s = np.concatenate(s_).astype(np.uint32)
    p = np.concatenate(p_).astype(np.uint32)
    o = np.concatenate(o_).astype(np.uint32)
    return {"t": [s, p, o], "ids": {"properties": P0, "classes": C0, "entities": E0,
                                     "n_classes": n_classes, "max_id": int(E0 + n_entities - 1)}}


def config_rdfs(seed: int = 1005, scale: float = 1.0) -> Workload:
    """RDFS-style reasoning over a 20M-triple synthetic table (scale shrinks
    the triple and entity counts together; the class and property
    hierarchies keep their shape)."""
    d = rdfs_triples(n_triples=int(20_000_000 * scale), n_entities=max(1000, int(1_700_000 * scale)),
                     seed=seed)
    return Workload(name=f"rdfs_{int(20_000_000 * scale)}", program=RDFS_PROGRAM, edb={"t": d["t"]},
                    idb=("t",), meta={"triples": int(20_000_000 * scale), **d["ids"], "seed": seed})


# ---------------------------------------------------------------- join sweep
# Reachability confirmed by the target: x reaches z over an edge y -> z of
# `fan` only if z acknowledges x.  The recursive rule closes a triangle
# (r, fan, ack share x, y, z), so after the delta atom r(x, y) either fan
# (keyed on y) or ack (keyed on x) can be joined first: the same result,
# intermediates of different sizes.
ACK_PROGRAM = """
r(x, y) :- e(x, y).
r(x, z) :- r(x, y), fan(y, z), ack(z, x).
"""


def ack_reach(n_groups: int, group: int = 256, fan: int = 128, acks: int = 16, seed: int = 1007) -> Workload:
    """Nodes in n_groups groups of `group` consecutive ids.  Every node has
    one e edge, `fan` fan edges and `acks` ack edges, each to a uniform node of
    its own group (duplicate pairs dropped).  A delta row r(x, y) meets about
    `fan` fan rows on y but about `acks` ack rows on x, so joining ack first
    keeps the intermediate result fan/acks times smaller."""
    rng = SplitMix64(seed)
    n = n_groups * group

    def edges(per_node):
        src = np.repeat(np.arange(n, dtype=np.int64), per_node)
        dst = (src // group) * group + rng.below(group, len(src))
        key = np.unique((src << 32) | dst)
        return [(key >> 32).astype(np.uint32), (key & 0xFFFFFFFF).astype(np.uint32)]

    e, f, a = edges(1), edges(fan), edges(acks)
    return Workload(name=f"ack_reach_g{n_groups}x{group}_f{fan}_a{acks}", program=ACK_PROGRAM,
                    edb={"e": e, "fan": f, "ack": a}, idb=("r",),
                    meta={"groups": n_groups, "group": group, "fan": fan, "acks": acks, "seed": seed})


JOIN_PROGRAM = """
out(x, z) :- a(x, y), b(y, z).
"""


def join_case(n_probe: int, n_keys: int, zipf_s: float = 0.0, seed: int = 1006) -> Workload:
    """One non-recursive join at large sizes: a(x, y) has n_probe rows with
    distinct x and y drawn from n_keys keys (uniform, or Zipf(s) over a random
    key ranking); b(y, z) has one row per key.  out has exactly n_probe
    distinct tuples; the build side of the join is a's index on y, whose runs
    follow the key distribution."""
    rng = SplitMix64(seed)
    x = np.arange(n_probe, dtype=np.uint32)
    if zipf_s > 0:
        y = _zipf_pick(n_keys, n_probe, zipf_s, rng).astype(np.uint32)
    else:
        y = rng.below(n_keys, n_probe).astype(np.uint32)
    by = np.arange(n_keys, dtype=np.uint32)
    bz = rng.below(1 << 30, n_keys).astype(np.uint32)
    name = f"join_p{n_probe}_k{n_keys}_" + (f"zipf{zipf_s:g}" if zipf_s > 0 else "uniform")
    return Workload(name=name, program=JOIN_PROGRAM, edb={"a": [x, y], "b": [by, bz]}, idb=("out",),
                    meta={"probe_rows": n_probe, "keys": n_keys, "zipf_s": zipf_s, "seed": seed})
