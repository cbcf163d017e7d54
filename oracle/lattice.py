"""Forward pass over an input lattice instead of a string (CPU oracle).

TEST INFRASTRUCTURE ONLY: used by the test suite; the product path never
imports it.  It shares no code with the GPU library.

The paper (section 3) reads one input string and has no epsilon arcs, and
names lattices as a generalisation its prefix-sum idea does not cover
(section 6.1).  Here the input is an acyclic weighted lattice: nodes
0..n-1 in topological order (every arc goes from a lower to a higher node),
node 0 the start and node n-1 the end; an arc (u, v, a, w) reads input
symbol a with log weight w, or reads nothing when a = -1 (epsilon).  The
total weight is Eq. 1 summed over the lattice's paths, i.e. the
composition of the lattice (as an acceptor) with the FST:

    A_0 = the start vector (0 at the start state, -inf elsewhere),
    A_v[q'] = LSE over arcs e = (u, v, a, w):
                a = -1:  A_u[q'] + w
                else:    LSE over FST arcs k with ilabel a, dst q' of (A_u[src_k] + theta_k) + w,
    log Z = LSE_q (A_{n-1}[q] + final[q]),

all in FP64.
"""
from __future__ import annotations

import numpy as np


def _lse2(a, b):
    m = np.maximum(a, b)
    out = np.full_like(m, -np.inf)
    fin = m > -np.inf
    out[fin] = m[fin] + np.log(np.exp(a[fin] - m[fin]) + np.exp(b[fin] - m[fin]))
    return out


def label_index(fst):
    """(order, bounds): the FST's arc ids stably sorted by input label, and
    where each label's run starts (label a: order[bounds[a]:bounds[a+1]])."""
    order = np.argsort(np.asarray(fst.ilabel), kind="stable")
    bounds = np.searchsorted(np.asarray(fst.ilabel)[order], np.arange(fst.num_ilabels + 1))
    return order, bounds


def lattice_forward(fst, n_nodes, arcs, index=None):
    """(log Z, node vectors f64[n_nodes, Q]) of one lattice; arcs = list of
    (u, v, label, log weight) with u < v < n_nodes, label in [-1, M).
    index: label_index(fst), when the caller reuses it over many lattices."""
    Q = fst.num_states
    order, bounds = index if index is not None else label_index(fst)
    by_label = {a: order[bounds[a]:bounds[a + 1]] for a in {int(e[2]) for e in arcs if e[2] >= 0}}
    A = np.full((n_nodes, Q), -np.inf)
    A[0, fst.start] = 0.0
    for v in range(1, n_nodes):
        for (u, t, a, w) in arcs:
            if t != v:
                continue
            if a < 0:
                A[v] = _lse2(A[v], A[u] + w)
                continue
            contrib = np.full(Q, -np.inf)
            for k in by_label.get(int(a), []):
                x = A[u, fst.src[k]] + float(fst.arc_score[k]) + w
                d = fst.dst[k]
                contrib[d] = np.logaddexp(contrib[d], x) if contrib[d] > -np.inf else x
            A[v] = _lse2(A[v], contrib)
    last = A[n_nodes - 1] + fst.final_score.astype(np.float64)
    m = np.max(last)
    log_z = -np.inf if m == -np.inf else float(m + np.log(np.sum(np.exp(last[last > -np.inf] - m))))
    return log_z, A
