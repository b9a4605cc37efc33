"""Shared test helpers: golden-fixture parsing and result comparison."""
from __future__ import annotations

import os
from collections import defaultdict

import numpy as np

import hypergen as hg

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_toy(path: str = os.path.join(GOLDEN, "toy_paper_example.txt")):
    """Parse the worked-example fixture -> (Incidence, keep, L, dual)."""
    n = None
    edges = {}
    keep = {}
    lines = defaultdict(list)
    dual = defaultdict(list)
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "n":
                n = int(tok[1])
            elif tok[0] == "edge":
                edges[int(tok[1])] = [int(x) for x in tok[2:]]
            elif tok[0] == "keep":
                keep[int(tok[1])] = [int(x) for x in tok[2:]]
            elif tok[0] == "L":
                s, i, j, w = map(int, tok[1:])
                lines[s].append((i, j, w))
            elif tok[0] == "dual":
                s, i, j, w = map(int, tok[1:])
                dual[s].append((i, j, w))
    inc = hg.from_rows([edges[k] for k in sorted(edges)], n=n)
    return inc, keep, lines, dual


def edges_of(lg) -> list:
    """(i, j, w) tuples of an oracle LineGraph, in stored order."""
    return [(int(a), int(b), int(c)) for a, b, c in zip(lg.i, lg.j, lg.w)]


def brute_force_sets(rows, s):
    """Python-set evaluation of the definition, for tiny inputs only."""
    sets = [set(r) for r in rows]
    out = []
    for i in range(len(sets)):
        if len(sets[i]) < s:
            continue
        for j in range(i + 1, len(sets)):
            if len(sets[j]) < s:
                continue
            w = len(sets[i] & sets[j])
            if w >= s:
                out.append((i, j, w))
    return out


def rows_of(inc):
    return [list(map(int, inc.row(i))) for i in range(inc.m)]


def assert_same_graph(a_rowptr, a_i, a_j, a_w, b_rowptr, b_i, b_j, b_w, what=""):
    np.testing.assert_array_equal(np.asarray(a_rowptr, np.int64), np.asarray(b_rowptr, np.int64),
                                  err_msg=f"{what}: row_ptr")
    np.testing.assert_array_equal(np.asarray(a_i), np.asarray(b_i), err_msg=f"{what}: i")
    np.testing.assert_array_equal(np.asarray(a_j), np.asarray(b_j), err_msg=f"{what}: j")
    np.testing.assert_array_equal(np.asarray(a_w), np.asarray(b_w), err_msg=f"{what}: w")


def load_toy_components(path: str = os.path.join(GOLDEN, "toy_components.txt")):
    """Parse the components/squeeze fixture -> ({s: labels}, {s: new ids})."""
    cc, sq = {}, {}
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            vals = [int(x) for x in tok[2:]]
            (cc if tok[0] == "cc" else sq)[int(tok[1])] = vals
    return cc, sq


def load_toy_symmetric(path: str = os.path.join(GOLDEN, "toy_symmetric.txt")):
    """Parse the symmetric-adjacency fixture -> {s: [[(partner, overlap), ...] per row]}."""
    out = {}
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            s, r = int(tok[1]), int(tok[2])
            rows = out.setdefault(s, [])
            while len(rows) <= r:
                rows.append([])
            rows[r] = [tuple(int(x) for x in t.split(":")) for t in tok[3:]]
    return out


def load_toy_preprocess(path: str = os.path.join(GOLDEN, "toy_preprocess.txt")):
    """Parse the preprocessing fixture -> {"asc": [...], "desc": [...], "top": [...]}."""
    out = {}
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if line:
                tok = line.split()
                out[tok[0]] = [int(x) for x in tok[1:]]
    return out


def with_subsets(seed: int, m: int, n: int, kmax: int, extra: int):
    """Input construction for toplex tests: random hyperedges, then `extra`
    more that are random subsets (some empty, some whole copies) of earlier
    ones, all shuffled together."""
    import hypergen as hg
    rng = np.random.default_rng(seed)
    base = hg.random_small(seed, m, n, kmax, 0.9)
    rows = [base.row(i).tolist() for i in range(base.m)]
    for _ in range(extra):
        src = rows[int(rng.integers(0, len(rows)))]
        pick = rng.random(len(src)) < rng.choice([0.0, 0.5, 0.9, 1.0])
        rows.append([v for v, p in zip(src, pick) if p])
    perm = rng.permutation(len(rows))
    return hg.from_rows([rows[i] for i in perm], n=n)
