"""Shared helpers for the oracle pin tests."""
import itertools

import oracle as O


def spanning_trees(edges, k):
    """All spanning trees of the motif's underlying undirected multigraph, as
    sorted tuples of motif edge indices."""
    for sub in itertools.combinations(range(len(edges)), k - 1):
        comp = list(range(k))
        ok = True
        for p in sub:
            a, b = comp[edges[p][0]], comp[edges[p][1]]
            if a == b:
                ok = False
                break
            comp = [a if c == b else c for c in comp]
        if ok:
            yield sub


def all_tree_choices(edges):
    k = 1 + max(max(e) for e in edges)
    for sub in spanning_trees(edges, k):
        for c in sub:
            yield O.make_tree(sub, c)
