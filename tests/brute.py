"""Independent brute-force evaluators used to pin the oracle.

None of this shares code with oracle/ or with the engine.  Each function
computes a fixpoint by a different route from the oracle's sorted-vector
semi-naive joins:

* `naive_by_assignment`: T_P applied literally -- every assignment of every
  rule variable over the active domain is tried against the current facts
  (only for tiny domains).
* `tc_bfs`: transitive closure as reachability, one BFS per source node.
* `sg_matrix`: same generation as the least solution of S = B U A^T S A
  with B = A^T A minus its diagonal, in boolean matrix products.
"""
from __future__ import annotations

import itertools
import re
from collections import defaultdict, deque

import numpy as np


def parse(program: str):
    """Tiny parser for `h(t,..) :- a(t,..), ..., x != y.` rules.
    Returns [(head, [atoms], [neq pairs], [vars])], atom = (rel, terms),
    term = ('c', int) | ('v', name)."""
    text = "\n".join(line.split("%")[0] for line in program.splitlines())
    rules = []
    fresh = itertools.count()
    for stmt in text.split("."):
        stmt = stmt.strip()
        if not stmt:
            continue
        head_s, body_s = stmt.split(":-")

        def term(tok):
            tok = tok.strip()
            if tok.isdigit():
                return ("c", int(tok))
            if tok == "_":
                return ("v", f"_{next(fresh)}")
            return ("v", tok)

        def atom(s):
            m = re.fullmatch(r"\s*([A-Za-z_]\w*)\s*\((.*)\)\s*", s)
            return (m.group(1), [term(t) for t in m.group(2).split(",")])

        head = atom(head_s)
        atoms, neqs = [], []
        for part in re.findall(r"[A-Za-z_]\w*\s*\([^()]*\)|[^,]+!=[^,]+", body_s):
            if "!=" in part:
                a, b = part.split("!=")
                neqs.append((a.strip(), b.strip()))
            else:
                atoms.append(atom(part))
        vs = sorted({t[1] for _, ts in atoms for t in ts if t[0] == "v"})
        rules.append((head, atoms, neqs, vs))
    return rules


def naive_by_assignment(program: str, edb: dict):
    """Least fixpoint by the definition: repeat F <- F U T_P(F), where
    T_P(F) tries every assignment of the rule's variables over the active
    domain (all values in the EDB and the rules).  Returns (facts, deltas)
    where facts maps relation -> set of tuples and deltas lists how many
    facts each round added."""
    rules = parse(program)
    facts = defaultdict(set)
    dom = set()
    for name, cols in edb.items():
        rows = list(zip(*[list(map(int, c)) for c in cols])) if len(cols[0]) else []
        facts[name] |= set(rows)
        for r in rows:
            dom |= set(r)
    for head, atoms, _, _ in rules:
        for _, ts in [head] + atoms:
            dom |= {t[1] for t in ts if t[0] == "c"}
    dom = sorted(dom)
    deltas = []
    while True:
        derived = defaultdict(set)
        for (hrel, hts), atoms, neqs, vs in rules:
            for vals in itertools.product(dom, repeat=len(vs)):
                env = dict(zip(vs, vals))
                if any(env[a] == env[b] for a, b in neqs):
                    continue
                ok = True
                for rel, ts in atoms:
                    tup = tuple(t[1] if t[0] == "c" else env[t[1]] for t in ts)
                    if tup not in facts[rel]:
                        ok = False
                        break
                if ok:
                    derived[hrel].add(tuple(t[1] if t[0] == "c" else env[t[1]] for t in hts))
        added = 0
        for rel, s in derived.items():
            new = s - facts[rel]
            added += len(new)
            facts[rel] |= new
        deltas.append(added)
        if added == 0:
            return facts, deltas


def tc_bfs(src: np.ndarray, dst: np.ndarray):
    """All (u, v) with a non-empty path u -> v, by one BFS per node."""
    adj = defaultdict(list)
    for u, v in zip(src.tolist(), dst.tolist()):
        adj[u].append(v)
    out = []
    for s in list(adj.keys()):
        seen = set()
        dq = deque(adj[s])
        while dq:
            v = dq.popleft()
            if v in seen:
                continue
            seen.add(v)
            dq.extend(adj.get(v, ()))
        out.extend((s, v) for v in seen)
    return np.array(sorted(out), dtype=np.uint32).reshape(-1, 2)


def sg_matrix(src: np.ndarray, dst: np.ndarray, n: int, neq_recursive: bool = False):
    """Same generation on a graph of n nodes as boolean matrices:
    S <- B U A^T S A (minus the diagonal on the recursive part when that
    rule carries x != y), with B = A^T A minus the diagonal, iterated from
    S = B until S stops growing (Kleene iteration of a monotone operator)."""
    A = np.zeros((n, n), dtype=np.float32)
    A[src, dst] = 1.0
    eye = np.eye(n, dtype=bool)
    B = ((A.T @ A) > 0) & ~eye
    S = B.copy()
    while True:
        step = (A.T @ S.astype(np.float32) @ A) > 0
        if neq_recursive:
            step &= ~eye
        nxt = S | B | step
        if (nxt == S).all():
            break
        S = nxt
    xs, ys = np.nonzero(S)
    return np.stack([xs, ys], axis=1).astype(np.uint32)


def rows(cols) -> np.ndarray:
    """Column list -> row-sorted unique (n, k) uint32 array."""
    a = np.stack([np.asarray(c, dtype=np.uint32) for c in cols], axis=1)
    if len(a) == 0:
        return a.reshape(0, len(cols))
    return np.unique(a, axis=0)


def as_rows(s, arity: int) -> np.ndarray:
    if not s:
        return np.zeros((0, arity), dtype=np.uint32)
    return np.array(sorted(s), dtype=np.uint32).reshape(-1, arity)
