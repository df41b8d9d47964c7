"""Error paths of the oracle: every invalid input is reported, never guessed."""
import numpy as np
import pytest

import oracle as O
from paper_2507_20441_amd import workloads as W


def _g(edges, n=4):
    e = np.array(edges, dtype=np.int64)
    return O.Graph(e[:, 0], e[:, 1], e[:, 2], n)


def test_graph_errors():
    with pytest.raises(O.OracleError) as ex:
        _g([(0, 0, 1)])
    assert ex.value.code == O.OR_ESELFLOOP
    with pytest.raises(O.OracleError) as ex:
        _g([(0, 1, 1), (0, 1, 1)])
    assert ex.value.code == O.OR_EDUP
    with pytest.raises(O.OracleError) as ex:
        _g([(0, 5, 1)])
    assert ex.value.code == O.OR_EINVAL
    with pytest.raises(O.OracleError) as ex:
        _g([(0, 1, -(2**62)), (1, 2, 2**62)])
    assert ex.value.code == O.OR_ERANGE
    # same pair, different time, and same time, different pair, are fine
    _g([(0, 1, 1), (0, 1, 2), (1, 0, 1), (2, 3, 1)])


def test_motif_and_tree_errors():
    G = _g([(0, 1, 1), (1, 2, 2), (2, 0, 3)])
    bad_motifs = [
        O.make_motif([(0, 1), (2, 3)], 5),          # disconnected
        O.make_motif([(0, 1), (1, 2)], 0),          # delta <= 0
        O.make_motif([(0, 0), (0, 1)], 5),          # self loop
        O.make_motif([(0, 1)] * 3 + [(1, 8)], 5),   # more than 8 vertices
    ]
    for mo in bad_motifs:
        with pytest.raises(O.OracleError):
            O.Prep(G, mo)
    mo = O.make_motif(W.MOTIFS["3cycle"], 5)
    for tr in (O.make_tree([0, 1], 2), O.make_tree([0], 0), O.make_tree([0, 0], 0),
               O.make_tree([0, 1, 2], 0)):
        with pytest.raises(O.OracleError):
            O.Prep(G, mo, tr)
    two_cycle = O.make_motif([(0, 1), (1, 0)], 5)
    with pytest.raises(O.OracleError):
        O.Prep(G, two_cycle, O.make_tree([0, 1], 0))   # not a tree on 2 vertices
