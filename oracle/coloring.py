"""Vertex grouping on the matrix of strong connections (oracle; test infrastructure only).

Follows Section 5.2 of the paper: Algorithm "VerticesSplitting" splits the
still-uncoloured vertex set V into one colour class W and a deferred set W-bar;
Algorithm "VerticesGrouping" repeats the split on W-bar until nothing is left.

Notation (Section 5.2): S_i is the set of j with S_ij = 1 (row i of the strong
matrix); |S_i| is the influence of vertex i; the "second circle" of i is the
union of S_k over k in S_i, minus S_i and i itself.

Readings where the printed algorithm is ambiguous:

* selection: the vertex of largest influence |S_i|, ties broken by the
  smallest vertex index; the influence is the static row count of S;
* the frontier (the paper's W-hat) is searched first whenever it still holds
  an undecided vertex; vertices that have left V are skipped lazily;
* the second-circle definition uses "there exists k in S_i" (the printed
  "for all" cannot be meant: the worked example of the notation figure lists
  vertices adjacent to a single neighbour of i);
* "v is not strongly connected to any vertex of W" tests row v of S; vertices
  joining W-bar are taken from V only (already coloured vertices stay put);
* colours are numbered in the order they are created and the members of each
  colour are listed in ascending index order.
"""
from __future__ import annotations

import heapq

import numpy as np

UNDECIDED, IN_W, IN_WBAR, OUTSIDE = 0, 1, 2, 3


def vertices_splitting(V, S, influence):
    """Algorithm VerticesSplitting on the vertex list V; returns (W, Wbar) sorted."""
    n = len(S)
    state = np.full(n, OUTSIDE, dtype=np.int8)
    state[V] = UNDECIDED
    remaining = len(V)
    heap_v = [(-influence[v], v) for v in V]
    heapq.heapify(heap_v)
    heap_f = []  # the frontier W-hat
    W, Wbar = [], []

    def pop(heap):
        while heap:
            _, v = heapq.heappop(heap)
            if state[v] == UNDECIDED:
                return v
        return -1

    while remaining > 0:
        v = pop(heap_f)
        if v < 0:
            v = pop(heap_v)
        if not any(state[j] == IN_W for j in S[v]):
            state[v] = IN_W
            W.append(v)
            remaining -= 1
            for j in S[v]:
                if state[j] == UNDECIDED:
                    state[j] = IN_WBAR
                    Wbar.append(j)
                    remaining -= 1
            for k in S[v]:
                for j in S[k]:
                    if state[j] == UNDECIDED:
                        heapq.heappush(heap_f, (-influence[j], j))
        else:
            state[v] = IN_WBAR
            Wbar.append(v)
            remaining -= 1
    return sorted(W), sorted(Wbar)


def vertices_grouping(n, S):
    """Algorithm VerticesGrouping: list of colour classes (each an ascending list).

    S is a list of Python lists, S[i] = strong neighbours of i (row i of S).
    """
    influence = [len(s) for s in S]
    V = list(range(n))
    colours = []
    while V:
        W, Wbar = vertices_splitting(V, S, influence)
        colours.append(W)
        V = Wbar
    return colours


def colour_array(n, colours):
    c = np.full(n, -1, dtype=np.int64)
    for ell, members in enumerate(colours):
        c[members] = ell
    return c
