"""CPU checks of the ordering arguments the GPU path relies on (no GPU):

* a sub-round's decisions do not depend on the order in which its vertices
  are taken (every decision reads the same snapshot), so the order of a
  bucket list and the assignment of vertices to blocks change nothing;
* the small-level schedule with two state copies (sub-round s reads copy
  s mod 2, applies its own moves to the other copy and replays sub-round
  s - 1's moves into it; the iteration end replays the last sub-round into
  the lagging copy) gives, after every sub-round, the clustering of the
  plain schedule that applies each sub-round's moves to one state;
* an iteration queued after an iteration without moves changes nothing:
  under the rule "all vertices" every vertex decides to stay against the
  state it leaves; under the frontier list rules its frontier is empty.

Decisions come from the oracle; the schedules around them are modelled here
in a few lines each."""
import numpy as np
import pytest

import oracle as O
from paper_2108_01731_amd import graphgen as G
from tests import helpers as H


def graphs():
    return [
        ("sbm", H.to_oracle(G.c1_sbm(3)), 1, 100),
        ("signed", H.to_oracle(G.random_signed(800, 4000, 5, wmin=-3, wmax=6, kmax=3)), 1, 9),
        ("chung_lu", H.to_oracle(G.chung_lu_planted(3000, 30000, 2.1, 0.3, seed=4)), 1, 60000),
    ]


@pytest.mark.parametrize("idx", range(3))
def test_decisions_do_not_depend_on_vertex_order(idx):
    name, g, p, q = graphs()[idx]
    rng = np.random.default_rng(idx)
    C = rng.integers(0, max(1, g.n // 10), size=g.n).astype(np.int32)
    U = rng.permutation(g.n).astype(np.int32)[: g.n // 2]
    D = O.decide_many(g, p, q, C, U)
    perm = rng.permutation(len(U))
    D2 = O.decide_many(g, p, q, C, U[perm])
    assert np.array_equal(D[perm], D2)
    # one vertex at a time, in reverse: the same decisions
    D3 = np.array([O.decide_many(g, p, q, C, U[i:i + 1])[0] for i in range(len(U) - 1, len(U) - 40, -1)])
    assert np.array_equal(D3, D[len(U) - 1:len(U) - 40:-1])


def color_lists(n, S, seed, level, it):
    h = O.round_hash(seed, level, 0, it)
    col = np.array([O.color(h, v, S) for v in range(n)])
    return [np.nonzero(col == s)[0].astype(np.int32) for s in range(S)]


@pytest.mark.parametrize("idx", range(3))
@pytest.mark.parametrize("S", [1, 2, 3, 4])
def test_two_copy_schedule_equals_plain_schedule(idx, S):
    """allow_isolate = 0 keeps every id in [0, n) (no fresh ids), so the
    plain schedule is a chain of oracle sub-rounds."""
    name, g, p, q = graphs()[idx]
    n = g.n
    C0 = np.arange(n, dtype=np.int32)
    copies = [C0.copy(), C0.copy()]
    plain = C0.copy()
    for it in range(2):
        Us = color_lists(n, S, seed=11, level=0, it=it)
        Ds = []
        for s in range(S):
            read, write = copies[s % 2], copies[(s + 1) % 2]
            D = O.decide_many(g, p, q, read, Us[s], allow_isolate=0)
            Ds.append(D)
            # the launch: replay of sub-round s - 1 into the write copy, then
            # its own moves (disjoint vertices; the order between them is free)
            if s > 0:
                U1, D1 = Us[s - 1], Ds[s - 1]
                diff = D1 != write[U1]
                write[U1[diff]] = D1[diff]
            diff = D != read[Us[s]]
            write[Us[s][diff]] = D[diff]
            plain, Dp, _ = O.subround(g, p, q, plain, Us[s], allow_isolate=0)
            assert np.array_equal(D, Dp)
            assert np.array_equal(write, plain), (name, S, it, s)
        # iteration end: the copy the last sub-round read lags by its moves
        lag = copies[(S - 1) % 2]
        diff = Ds[S - 1] != lag[Us[S - 1]]
        lag[Us[S - 1][diff]] = Ds[S - 1][diff]
        assert np.array_equal(copies[0], plain) and np.array_equal(copies[1], plain)


@pytest.mark.parametrize("idx", range(3))
def test_iteration_after_a_still_one_changes_nothing_all_vertices(idx):
    """Rule "all vertices": an iteration without moves took every vertex
    against one unchanged state, so against that state every vertex stays,
    under any later sub-round assignment."""
    name, g, p, q = graphs()[idx]
    C, st = O.best_move(g, p, q, O.Params(S=3, num_iter=200, frontier=O.FRONTIER_ALL))
    assert st["term"] == O.TERM_NO_MOVES
    D = O.decide_many(g, p, q, C, np.arange(g.n, dtype=np.int32))
    assert np.array_equal(D, C)
    C2, st2 = O.best_move(g, p, q, O.Params(S=3, num_iter=5, frontier=O.FRONTIER_ALL), C, level=0, phase=1)
    assert np.array_equal(C2, C) and st2["moves"] == 0


@pytest.mark.parametrize("frontier", [O.FRONTIER_NBR, O.FRONTIER_CLUSTERS])
def test_frontier_after_an_iteration_without_moves_is_empty(frontier):
    """The frontier list rules: the iteration after one without movers has no
    vertex to take (no mover marks neighbors, no cluster was left), so an
    iteration queued past the end has no work.  (A vertex outside the
    frontier may still prefer another cluster: the rule never looks at it.)
    From a clustering where every vertex stays (the end of an all-vertices
    run), a call under the rule ends after its first iteration, which moved
    nothing, and the frontier of no movers is empty."""
    name, g, p, q = graphs()[0]
    rng = np.random.default_rng(2)
    C = rng.integers(0, 50, size=g.n).astype(np.int32)
    Cs, _ = O.best_move(g, p, q, O.Params(S=2, num_iter=200, frontier=O.FRONTIER_ALL), C)
    _, st = O.best_move(g, p, q, O.Params(S=2, num_iter=3, frontier=frontier), Cs, level=0, phase=1)
    assert st["iterations"] == 1 and st["moves"] == 0 and st["term"] == O.TERM_NO_MOVES
    assert np.array_equal(O.frontier_nbr(g, np.zeros(0, np.int32)), np.zeros(g.n, np.uint8))
