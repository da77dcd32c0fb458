"""Parser for the small text fixtures under tests/golden/."""
import os

import synth

INF_I32 = 2**31 - 1
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    """Returns (problem, input_names, facts) where facts maps a keyword to the
    list of its token lists."""
    n = None
    inputs = None
    G = None
    pairs = {}
    facts = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            key = tok[0]
            if key == "states":
                n = int(tok[1])
            elif key == "inputs":
                inputs = tok[1:]
            elif key == "terminal":
                G = [INF_I32 if t == "INF" else int(t) for t in tok[1:]]
            elif key == "pair":
                x = int(tok[1]) - 1
                u = inputs.index(tok[2])
                c = INF_I32 if tok[3] == "INF" else int(tok[3])
                pairs[(x, u)] = (c, [int(t) - 1 for t in tok[4:]])
            else:
                facts.setdefault(key, []).append(tok[1:])
    K = len(inputs)
    rows, g = [], []
    for x in range(n):
        for u in range(K):
            c, succ = pairs[(x, u)]
            rows.append(succ)
            g.append(c)
    prob = synth.explicit_problem(n, K, rows, g, G, name=name)
    return prob, inputs, facts
