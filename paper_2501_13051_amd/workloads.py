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
