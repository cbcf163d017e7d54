"""Brute-force path enumeration and a dense-matrix form of Eq. (1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  These are the plain
definitions the C oracle must reproduce:

* Viterbi score = max over accepting paths of the path score, each path score
  accumulated left to right in FP32 (0 + s_1 + s_2 + ... + s_n + final), one
  binary32 rounding per addition.
* log Z = log of the sum over accepting paths of exp(path score) (FP64).
* arc posterior of arc k = sum over paths of P(path) * (uses of k in path).

``dense_log_z`` evaluates Eq. (1), s^T (prod_t delta[w_t]) f, with dense
log-semiring matrix-vector products (torch.logsumexp in FP64).
"""
from __future__ import annotations

import math

import numpy as np


def enumerate_paths(fst, tokens):
    """All label-consistent accepting paths: list of (arc tuple, final state)."""
    tokens = [int(x) for x in tokens]
    out_arcs = {}
    for k in range(fst.num_arcs):
        out_arcs.setdefault((int(fst.src[k]), int(fst.ilabel[k])), []).append(k)
    paths = []

    def rec(q, t, acc):
        if t == len(tokens):
            if fst.final_score[q] != -np.inf:
                paths.append((tuple(acc), q))
            return
        for k in out_arcs.get((q, tokens[t]), ()):
            acc.append(k)
            rec(int(fst.dst[k]), t + 1, acc)
            acc.pop()

    rec(int(fst.start), 0, [])
    return paths


def path_score_f32(fst, arcs, q_final):
    s = np.float32(0.0)
    for k in arcs:
        s = np.float32(s + fst.arc_score[k])
    return np.float32(s + fst.final_score[q_final])


def path_score_f64(fst, arcs, q_final):
    return float(sum(float(fst.arc_score[k]) for k in arcs)) + float(fst.final_score[q_final])


def brute_viterbi(fst, tokens):
    """(best FP32 score or -inf, set of arc tuples attaining it)."""
    paths = enumerate_paths(fst, tokens)
    if not paths:
        return np.float32(-np.inf), set()
    scores = [path_score_f32(fst, a, q) for a, q in paths]
    best = max(scores)
    return best, {paths[i][0] for i, s in enumerate(scores) if s == best}


def brute_forward_backward(fst, tokens):
    """(log Z, arc posteriors f64[A], final-state posteriors f64[Q])."""
    paths = enumerate_paths(fst, tokens)
    post = np.zeros(fst.num_arcs, np.float64)
    fpost = np.zeros(fst.num_states, np.float64)
    if not paths:
        return -math.inf, post, fpost
    sc = np.array([path_score_f64(fst, a, q) for a, q in paths])
    m = sc.max()
    log_z = m + math.log(np.exp(sc - m).sum())
    for (arcs, q), s in zip(paths, sc):
        p = math.exp(s - log_z)
        for k in arcs:
            post[k] += p
        fpost[q] += p
    return log_z, post, fpost


def dense_log_z(fst, tokens):
    """Eq. (1) with dense |Q|x|Q| log-semiring matrices (small |Q| only)."""
    import torch

    Q = fst.num_states
    ninf = -math.inf
    mats = {}
    for a in set(int(x) for x in tokens):
        m = torch.full((Q, Q), ninf, dtype=torch.float64)
        sel = np.nonzero(fst.ilabel == a)[0]
        for k in sel:
            i, j = int(fst.src[k]), int(fst.dst[k])
            m[i, j] = torch.logaddexp(m[i, j], torch.tensor(float(fst.arc_score[k]), dtype=torch.float64))
        mats[a] = m
    alpha = torch.full((Q,), ninf, dtype=torch.float64)
    alpha[int(fst.start)] = 0.0
    for a in tokens:
        alpha = torch.logsumexp(alpha[:, None] + mats[int(a)], dim=0)
    f = torch.as_tensor(fst.final_score.astype(np.float64))
    return float(torch.logsumexp(alpha + f, dim=0))
