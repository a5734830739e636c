"""Pins of the oracle's VerticesSplitting / VerticesGrouping (Section 5.2).

* A second, literal transliteration over Python sets (linear scans instead of
  heaps) must agree exactly with the oracle on random small graphs.
* The paper's design goals (a)-(c): the classes cover V, are disjoint and are
  internally unconnected in S (read as S or S^T); each class is a maximal
  independent set of what was left; the colour count is at most
  max degree + 1 (Proposition "Upper bound estimation"); the algorithm
  terminates with c <= |V| (Proposition "Finite termination").
* With theta = 0 on a 7-point grid (bipartite adjacency), the frontier
  sweeps one parity class per connected component, so exactly 2 colours,
  masked or not, and every colour block of A is diagonal (Proposition
  "Matrix diagonalization").
"""
import numpy as np

from oracle import coloring, strength
from oracle.sparse import csr_from_dense, pattern_lists
from workloads import blackoil as bo
from oracle.cpr import Bsr, pressure_matrix


def literal_grouping(n, S):
    """Algorithms VerticesSplitting/VerticesGrouping over Python sets."""
    infl = [len(s) for s in S]
    V = set(range(n))
    colours = []
    while V:
        W, Wbar, What = set(), set(), set()
        Vcur = set(V)
        while Vcur:
            cand = (What & Vcur) or Vcur
            best = min(cand, key=lambda v: (-infl[v], v))
            if not (set(S[best]) & W):
                W.add(best)
                Vcur.discard(best)
                What.discard(best)
                Si = set(S[best]) & Vcur
                Wbar |= Si
                Vcur -= Si
                ring = set()
                for k in S[best]:
                    ring |= set(S[k])
                ring -= set(S[best]) | {best}
                What |= ring & Vcur
            else:
                Wbar.add(best)
                Vcur.discard(best)
                What.discard(best)
        colours.append(sorted(W))
        V = Wbar
    return colours


def _random_strength(rng, n, density):
    d = (rng.uniform(size=(n, n)) < density).astype(float)
    np.fill_diagonal(d, 0)
    if rng.uniform() < 0.5:
        d = np.maximum(d, d.T)
    return [list(np.nonzero(d[i])[0]) for i in range(n)]


def _check_goals(n, S, colours):
    allv = sorted(v for c in colours for v in c)
    assert allv == list(range(n))  # (a) cover and (b) disjoint
    col = coloring.colour_array(n, colours)
    sym = [set(S[i]) for i in range(n)]
    for i in range(n):
        for j in S[i]:
            sym[j].add(i)
    for i in range(n):
        for j in sym[i]:
            assert col[i] != col[j]  # (c) independent
    remaining = set(range(n))
    for c in colours:  # maximal independent in what was left
        cs = set(c)
        for v in remaining - cs:
            assert sym[v] & cs
        remaining -= cs
    maxdeg = max((len(s) for s in sym), default=0)
    assert len(colours) <= maxdeg + 1
    assert len(colours) <= n


def test_literal_and_heap_agree_on_random_graphs():
    rng = np.random.default_rng(11)
    for trial in range(1500):
        n = int(rng.integers(1, 28))
        S = _random_strength(rng, n, rng.uniform(0.02, 0.5))
        got = coloring.vertices_grouping(n, S)
        want = literal_grouping(n, S)
        assert got == want, (trial, S)
        _check_goals(n, S, got)


def test_goals_on_generated_pressure_levels():
    case = bo.case_small(shape=(8, 7, 4))
    App = pressure_matrix(Bsr.from_case(case))
    for theta in (0.0, 0.05, 0.1, 0.3):
        _, (ip, ix) = strength.color_strength(App, theta)
        S = pattern_lists(ip, ix)
        colours = coloring.vertices_grouping(App.n_rows, S)
        _check_goals(App.n_rows, S, colours)
        assert colours == literal_grouping(App.n_rows, S)


def test_theta0_seven_point_grid_two_colours_and_diagonal_blocks():
    for shape, frac, seed in (((9, 8, 5), 0.0, 3), ((10, 7, 6), 0.1, 4), ((13, 11, 3), 0.25, 5)):
        rng = np.random.default_rng(seed)
        perm = bo.perm_iid_lognormal(shape, rng)
        active = bo.random_mask(shape, rng, frac)
        case = bo.assemble(shape, active, bo.make_faces(shape, perm, active, 1.0, rng))
        App = pressure_matrix(Bsr.from_case(case))
        _, (ip, ix) = strength.color_strength(App, 0.0)
        S = pattern_lists(ip, ix)
        colours = coloring.vertices_grouping(App.n_rows, S)
        assert len(colours) == 2
        d = App.to_dense()
        for c in colours:
            blk = d[np.ix_(c, c)]
            assert np.count_nonzero(blk - np.diag(np.diag(blk))) == 0


def test_theta_one_single_colour():
    case = bo.case_small(shape=(5, 4, 3))
    App = pressure_matrix(Bsr.from_case(case))
    _, (ip, ix) = strength.color_strength(App, 1.0)
    colours = coloring.vertices_grouping(App.n_rows, pattern_lists(ip, ix))
    assert colours == [list(range(App.n_rows))]


def test_dense_graph_needs_n_colours():
    n = 9
    S = [[j for j in range(n) if j != i] for i in range(n)]
    colours = coloring.vertices_grouping(n, S)
    assert len(colours) == n
