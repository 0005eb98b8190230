"""Random tiny Datalog programs and inputs for cross-checks (seeded)."""
import random

import numpy as np

ARITY = {"e": 2, "c": 1, "p": 2, "q": 2, "r": 3, "u": 1}


def random_program(rnd: random.Random):
    """Random safe rules over EDB e/2, c/1 and IDB p/2, q/2, r/3, u/1 with
    constants, repeated variables, != and mutual recursion."""
    arity = ARITY
    idb = ["p", "q", "r", "u"]
    rules = []
    for _ in range(rnd.randint(2, 5)):
        head = rnd.choice(idb)
        nb = rnd.randint(1, 3)
        vars_ = ["x", "y", "z", "w"]
        body = []
        for _ in range(nb):
            rel = rnd.choice(["e", "e", "c"] + idb)
            terms = []
            for _ in range(arity[rel]):
                if rnd.random() < 0.12:
                    terms.append(str(rnd.randint(0, 4)))
                else:
                    terms.append(rnd.choice(vars_))
            body.append(f"{rel}({', '.join(terms)})")
        bound = sorted({t for a in body for t in a[a.index('(') + 1:-1].split(', ') if not t.isdigit()})
        if not bound:
            continue
        hterms = [rnd.choice(bound) if rnd.random() > 0.1 else str(rnd.randint(0, 4))
                  for _ in range(arity[head])]
        neq = ""
        if len(bound) >= 2 and rnd.random() < 0.3:
            a, b = rnd.sample(bound, 2)
            neq = f", {a} != {b}"
        rules.append(f"{head}({', '.join(hterms)}) :- {', '.join(body)}{neq}.")
    # make sure each IDB relation exists with the right arity
    rules.append("u(x) :- c(x).")
    rules.append("p(x, y) :- e(x, y).")
    return "\n".join(rules) + "\n"



def random_edb(rnd: random.Random, dom: int = 5):
    ne = rnd.randint(0, 9)
    e = [(rnd.randrange(dom), rnd.randrange(dom)) for _ in range(ne)]
    c = [rnd.randrange(dom) for _ in range(rnd.randint(0, 3))]
    return {"e": [np.array([a for a, _ in e], np.uint32), np.array([b for _, b in e], np.uint32)],
            "c": [np.array(c, np.uint32)]}


# Column bounds under constant conditions: p's middle column holds only small
# constants in the facts, but the second rule fills it with values of rows
# whose middle column is 2, and the first rule makes such rows from q, whose
# values are large; q(5, 3) also lets the second rule make rows whose middle
# column is 3, which that rule reads again.  A bound for p's middle column
# that missed either path would cut values off.
CONDITIONED_PROGRAM = """
p(x, 2, y) :- q(x, y).
p(x, y, z) :- p(x, 2, y), p(y, 3, z).
s(x, y) :- p(x, 3, y).
"""


def conditioned_edb():
    import numpy as np
    i = np.arange(100, dtype=np.uint32)
    q = [np.concatenate([i, [5]]).astype(np.uint32), np.concatenate([1_000_000 + i, [3]]).astype(np.uint32)]
    ps = np.concatenate([1_000_000 + i, [3, 3, 7]]).astype(np.uint32)
    pm = np.full(len(ps), 3, np.uint32)
    po = np.concatenate([i % 7 + 10, [40, 41, 42]]).astype(np.uint32)
    return {"q": q, "p": [ps, pm, po]}
