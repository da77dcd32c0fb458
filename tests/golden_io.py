"""Parser for the small text fixtures under tests/golden/."""
import os

import numpy as np

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
    edges = {}
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
            elif key == "edge":
                # per-edge costs h of a pair, one per successor in the listed order
                x = int(tok[1]) - 1
                u = inputs.index(tok[2])
                edges[(x, u)] = [int(t) for t in tok[3:]]
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
    if edges:
        h = []
        for x in range(n):
            for u in range(K):
                succ = pairs[(x, u)][1]
                assert succ == sorted(succ), f"{name}: successors of pair {x + 1} {inputs[u]} must be ascending"
                hv = edges[(x, u)]
                assert len(hv) == len(succ), f"{name}: one edge cost per successor of pair {x + 1} {inputs[u]}"
                h.extend(hv)
        prob.g_edge = np.array(h, dtype=np.int32)
    return prob, inputs, facts


def expected(facts, inputs, n):
    """The hand-computed value function and canonical policy stated in a
    fixture (`value <state> <v|INF>`, `policy <state> <input|HANDOVER|NONE>`)."""
    V = np.full(n, INF_I32, dtype=np.int64)
    pol = np.full(n, -3, dtype=np.int32)
    for st, v in facts["value"]:
        V[int(st) - 1] = INF_I32 if v == "INF" else int(v)
    for st, u in facts["policy"]:
        pol[int(st) - 1] = {"HANDOVER": -1, "NONE": -2}.get(u, inputs.index(u) if u in inputs else -3)
    assert len(facts["value"]) == n and len(facts["policy"]) == n and (pol != -3).all()
    return V.astype(np.int32), pol
