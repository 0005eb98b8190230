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
