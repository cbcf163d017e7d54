"""EM re-estimation of arc scores from expected counts (CPU oracle).

TEST INFRASTRUCTURE ONLY: used by the test suite; the product path never
imports it.  It shares no code with the GPU library.

The paper (section 4) computes expected arc counts with Algorithm 2 in order
to run expectation-maximisation on the transducer's weights.  The reading
taken here: the WFST is a locally normalised model, p(arc | source state),
with the final weights held fixed.  The E-step is the oracle's
forward-backward (expected count of every arc over the batch); the M-step
sets every arc's probability to its expected count divided by the total
expected count of the arcs leaving the same source state,

    theta'_k = log(c_k + lam) - log(sum_{j: src_j = src_k} (c_j + lam)),

with add-lam smoothing (lam = 0: plain EM).  A state whose arcs received no
count keeps its scores.  For lam = 0 each iteration cannot decrease the
batch log-likelihood sum_b log Z_b (the standard EM guarantee).
"""
from __future__ import annotations

import numpy as np

from . import forward_backward


def m_step(fst, counts, smoothing=0.0):
    """New log-domain arc scores (FP64, arc-id order) from expected counts."""
    c = np.asarray(counts, np.float64) + float(smoothing)
    tot = np.zeros(fst.num_states, np.float64)
    np.add.at(tot, fst.src, c)
    new = fst.arc_score.astype(np.float64).copy()
    live = tot[fst.src] > 0
    with np.errstate(divide="ignore"):
        new[live] = np.log(c[live]) - np.log(tot[fst.src[live]])
    return new


def em_step(fst, batch, smoothing=0.0):
    """One EM iteration: (new scores f64[A], log-likelihood of the batch under
    the current scores, expected counts f64[A])."""
    log_z, counts, _, status = forward_backward(fst, batch)
    ll = float(np.sum(log_z[status == 0]))
    return m_step(fst, counts, smoothing), ll, counts
