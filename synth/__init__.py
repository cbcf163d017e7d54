"""Seeded synthetic workloads: weighted finite-state transducers and input batches.

This module only draws random structures and numbers.  It computes nothing of
the decoding method (no path scores, no semiring arithmetic); both the oracle
and the GPU path consume what it returns.

Every workload is a weighted FST in the tuple form of section 3 of the paper
(states, input alphabet, one start state, final weights, per-symbol transition
matrices; no epsilon arcs), stored as a flat arc list.  Scores are log-domain:
``arc_score = log p`` (higher is better), ``final_score = -inf`` marks a
non-final state.

Random streams: ``np.random.SeedSequence(seed).spawn(3)`` gives one stream
each for structure, weights and sentences, so a workload is a pure function of
its seed and parameters.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Fst", "Batch", "zipf_probs", "zipf_tokens", "lognormal_lengths",
    "tiny_random_fst", "random_batch", "hmm_bigram", "hmm_trigram",
    "powerlaw_fst", "random_walk_batch", "config", "random_lattice", "confusion_network",
]


@dataclass
class Fst:
    num_states: int
    num_ilabels: int
    start: int
    src: np.ndarray          # int32 [A]
    dst: np.ndarray          # int32 [A]
    ilabel: np.ndarray       # int32 [A]
    olabel: np.ndarray       # int32 [A]
    arc_score: np.ndarray    # float32 [A]  (log-domain, higher is better)
    final_score: np.ndarray  # float32 [Q]  (-inf = non-final)
    meta: dict = field(default_factory=dict)

    @property
    def num_arcs(self) -> int:
        return int(self.src.shape[0])


@dataclass
class Batch:
    offsets: np.ndarray  # int64 [B+1], offsets[0] = 0
    tokens: np.ndarray   # int32 [offsets[-1]]
    meta: dict = field(default_factory=dict)

    @property
    def size(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def sentence(self, b: int) -> np.ndarray:
        return self.tokens[self.offsets[b]:self.offsets[b + 1]]

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)


def _streams(seed: int):
    ss = np.random.SeedSequence(seed).spawn(3)
    return tuple(np.random.default_rng(s) for s in ss)


def zipf_probs(n: int, s: float) -> np.ndarray:
    """Finite Zipf law over ids 0..n-1: P(id = r-1) proportional to r^-s."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def zipf_tokens(rng, n: int, s: float, size: int) -> np.ndarray:
    p = zipf_probs(n, s)
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    return np.searchsorted(cdf, rng.random(size), side="right").astype(np.int32)


def lognormal_lengths(rng, size: int, mean: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    mu = np.log(mean) - 0.5 * sigma * sigma
    return np.clip(np.rint(rng.lognormal(mu, sigma, size)), lo, hi).astype(np.int64)


def _batch_from_lengths(lengths: np.ndarray, tokens: np.ndarray, meta=None) -> Batch:
    offsets = np.zeros(lengths.shape[0] + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    assert offsets[-1] == tokens.shape[0]
    return Batch(offsets=offsets, tokens=tokens.astype(np.int32), meta=dict(meta or {}))


def random_batch(seed: int, num_ilabels: int, lengths, zipf_s: float | None = None) -> Batch:
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    lengths = np.asarray(lengths, dtype=np.int64)
    n = int(lengths.sum())
    if zipf_s is None:
        toks = rng.integers(0, num_ilabels, n).astype(np.int32)
    else:
        toks = zipf_tokens(rng, num_ilabels, zipf_s, n)
    return _batch_from_lengths(lengths, toks)


# --------------------------------------------------------------------------
# Tiny random transducers (brute-force territory)
# --------------------------------------------------------------------------

def tiny_random_fst(seed: int, num_states: int = 4, num_ilabels: int = 2, num_arcs: int = 10,
                    integer_scores: bool = False, final_prob: float = 0.6) -> Fst:
    """A small random nondeterministic WFST; duplicate arcs and self-loops allowed.

    With ``integer_scores`` every score is drawn from {0, -1, -2}, which makes
    ties between paths the rule rather than the exception.
    """
    rs, rw, _ = _streams(seed)
    src = rs.integers(0, num_states, num_arcs).astype(np.int32)
    dst = rs.integers(0, num_states, num_arcs).astype(np.int32)
    ilab = rs.integers(0, num_ilabels, num_arcs).astype(np.int32)
    olab = rs.integers(0, 3, num_arcs).astype(np.int32)
    if integer_scores:
        sc = -rw.integers(0, 3, num_arcs).astype(np.float32)
        fin = np.where(rs.random(num_states) < final_prob,
                       -rw.integers(0, 2, num_states).astype(np.float32), -np.inf)
    else:
        sc = np.log(rw.uniform(0.05, 1.0, num_arcs)).astype(np.float32)
        fin = np.where(rs.random(num_states) < final_prob,
                       np.log(rw.uniform(0.1, 1.0, num_states)), -np.inf)
    return Fst(num_states, num_ilabels, 0, src, dst, ilab, olab,
               sc.astype(np.float32), fin.astype(np.float32), meta={"kind": "tiny", "seed": seed})


# --------------------------------------------------------------------------
# HMM taggers written as WFSTs
# --------------------------------------------------------------------------

def _tags_per_word(rng, vocab: int, n_tags: int, rule: str) -> list[np.ndarray]:
    if rule == "uniform123":
        c = rng.integers(1, 4, vocab)
    elif rule == "geometric0.6cap8":
        # 1 + G with G ~ Geometric(0.6) counted as failures, i.e. trials capped at 8
        c = np.minimum(rng.geometric(0.6, vocab), 8)
    else:
        raise ValueError(rule)
    order = np.argsort(rng.random((vocab, n_tags)), axis=1)
    return c.astype(np.int64), order


def _emission_logprobs(rng, c: np.ndarray, order: np.ndarray, n_tags: int, alpha: float):
    """log p(w | t) with p(. | t) ~ Dirichlet(alpha) over the words allowed tag t."""
    vocab = c.shape[0]
    words = np.repeat(np.arange(vocab), c)
    col = np.arange(words.shape[0]) - np.repeat(np.cumsum(c) - c, c)
    tags = order[words, col]
    g = rng.gamma(alpha, 1.0, words.shape[0])
    g = np.maximum(g, np.finfo(np.float64).tiny)
    tot = np.bincount(tags, weights=g, minlength=n_tags)
    return words, tags, np.log(g) - np.log(tot[tags])


def _dirichlet_rows(rng, n_rows: int, n: int, alpha: float) -> np.ndarray:
    g = rng.gamma(alpha, 1.0, (n_rows, n))
    g = np.maximum(g, np.finfo(np.float64).tiny)
    return np.log(g) - np.log(g.sum(axis=1, keepdims=True))


def _assemble(vocab, c, words, tags, emis, n_ctx, next_state, trans_logp):
    """Arcs in id order (word, context state, tag): ctx --w:tag--> next_state[ctx, tag]."""
    word_start = np.zeros(vocab + 1, dtype=np.int64)
    np.cumsum(c * n_ctx, out=word_start[1:])
    A = int(word_start[-1])
    src = np.empty(A, np.int32)
    dst = np.empty(A, np.int32)
    ilab = np.empty(A, np.int32)
    olab = np.empty(A, np.int32)
    sc = np.empty(A, np.float32)
    pair_start = np.cumsum(c) - c
    ctx = np.arange(n_ctx, dtype=np.int64)
    for cc in np.unique(c):
        ws = np.nonzero(c == cc)[0]
        cols = np.arange(cc)
        pidx = pair_start[ws][:, None] + cols[None, :]              # (n, cc)
        tg = tags[pidx]                                             # (n, cc)
        em = emis[pidx]                                             # (n, cc)
        pos = (word_start[ws][:, None, None] + ctx[None, :, None] * cc + cols[None, None, :])
        pos = pos.reshape(-1)
        src[pos] = np.broadcast_to(ctx[None, :, None], (ws.size, n_ctx, cc)).reshape(-1)
        dst[pos] = next_state[ctx[None, :, None], tg[:, None, :]].reshape(-1)
        ilab[pos] = np.broadcast_to(ws[:, None, None], (ws.size, n_ctx, cc)).reshape(-1)
        olab[pos] = np.broadcast_to(tg[:, None, :], (ws.size, n_ctx, cc)).reshape(-1)
        th = trans_logp[ctx[None, :, None], tg[:, None, :]] + em[:, None, :]
        sc[pos] = th.reshape(-1).astype(np.float32)
        del pos, th
    return src, dst, ilab, olab, sc


def hmm_bigram(seed: int, n_tags: int, vocab: int, tags_rule: str = "uniform123",
               alpha: float = 1.0) -> Fst:
    """Bigram HMM tagger as a WFST.

    States: 0 = start, 1 + t = "previous tag was t".  Arc (q, w) -> 1 + t for
    every state q and every tag t allowed for word w, with score
    log p(t | q) + log p(w | t).  Every state is final with score 0.
    """
    rs, rw, _ = _streams(seed)
    c, order = _tags_per_word(rs, vocab, n_tags, tags_rule)
    words, tags, emis = _emission_logprobs(rw, c, order, n_tags, alpha)
    n_ctx = n_tags + 1
    trans = _dirichlet_rows(rw, n_ctx, n_tags, alpha)
    next_state = np.broadcast_to(1 + np.arange(n_tags)[None, :], (n_ctx, n_tags))
    src, dst, ilab, olab, sc = _assemble(vocab, c, words, tags, emis, n_ctx, next_state, trans)
    fin = np.zeros(n_ctx, np.float32)
    return Fst(n_ctx, vocab, 0, src, dst, ilab, olab, sc, fin,
               meta={"kind": "hmm_bigram", "seed": seed, "n_tags": n_tags, "vocab": vocab,
                     "tags_rule": tags_rule, "alpha": alpha, "tags_per_word": c})


def hmm_trigram(seed: int, n_tags: int = 45, vocab: int = 50000,
                tags_rule: str = "geometric0.6cap8", alpha: float = 0.5) -> Fst:
    """Trigram HMM tagger as a WFST over tag-pair states.

    States: 0 = (<s>,<s>), 1 + t = (<s>, t), 1 + n + n*t1 + t2 = (t1, t2).
    Arc (x, y) --w:t3--> (y, t3) for every state and every tag t3 allowed for
    w, with score log p(t3 | x, y) + log p(w | t3).  All states final, score 0.
    """
    rs, rw, _ = _streams(seed)
    n = n_tags
    c, order = _tags_per_word(rs, vocab, n, tags_rule)
    words, tags, emis = _emission_logprobs(rw, c, order, n, alpha)
    Q = 1 + n + n * n
    trans = _dirichlet_rows(rw, Q, n, alpha)
    t3 = np.arange(n)
    next_state = np.empty((Q, n), np.int64)
    next_state[0] = 1 + t3
    next_state[1:1 + n] = 1 + n + n * np.arange(n)[:, None] + t3[None, :]
    t2 = (np.arange(n * n) % n)
    next_state[1 + n:] = 1 + n + n * t2[:, None] + t3[None, :]
    src, dst, ilab, olab, sc = _assemble(vocab, c, words, tags, emis, Q, next_state, trans)
    fin = np.zeros(Q, np.float32)
    return Fst(Q, vocab, 0, src, dst, ilab, olab, sc, fin,
               meta={"kind": "hmm_trigram", "seed": seed, "n_tags": n, "vocab": vocab,
                     "tags_rule": tags_rule, "alpha": alpha, "tags_per_word": c})


# --------------------------------------------------------------------------
# Random sparse power-law transducer
# --------------------------------------------------------------------------

def powerlaw_fst(seed: int, num_states: int = 1_000_000, num_ilabels: int = 10_000,
                 num_arcs: int = 50_000_000, exponent: float = 2.1, d_min: int = 10,
                 d_max: int = 5000, label_zipf: float = 1.0) -> Fst:
    """Random nondeterministic WFST with power-law out-degrees.

    Out-degree d ~ P(d) proportional to d^-exponent on [d_min, d_max], then
    topped up one arc at a time at uniformly random states below the cap until
    there are exactly ``num_arcs`` arcs (or trimmed if the draw overshoots).
    Destinations uniform, input labels Zipf(label_zipf), output = input label,
    score = -Exp(1).  Start 0, every state final with score 0.  Arcs are listed
    grouped by source state.
    """
    rs, rw, _ = _streams(seed)
    d = np.arange(d_min, d_max + 1, dtype=np.float64)
    p = d ** (-exponent)
    p /= p.sum()
    deg = rs.choice(np.arange(d_min, d_max + 1), size=num_states, p=p).astype(np.int64)
    total = int(deg.sum())
    while total < num_arcs:
        need = num_arcs - total
        cand = rs.integers(0, num_states, need)
        cand = cand[deg[cand] < d_max]
        np.add.at(deg, cand, 1)
        deg = np.minimum(deg, d_max)
        total = int(deg.sum())
    while total > num_arcs:
        over = total - num_arcs
        cand = rs.integers(0, num_states, over)
        cand = cand[deg[cand] > d_min]
        np.add.at(deg, cand, -1)
        deg = np.maximum(deg, d_min)
        total = int(deg.sum())
    src = np.repeat(np.arange(num_states, dtype=np.int32), deg)
    dst = rs.integers(0, num_states, num_arcs).astype(np.int32)
    ilab = zipf_tokens(rs, num_ilabels, label_zipf, num_arcs)
    sc = (-rw.exponential(1.0, num_arcs)).astype(np.float32)
    fin = np.zeros(num_states, np.float32)
    return Fst(num_states, num_ilabels, 0, src, dst, ilab, ilab.copy(), sc, fin,
               meta={"kind": "powerlaw", "seed": seed, "exponent": exponent,
                     "d_min": d_min, "d_max": d_max, "out_degree": deg})


def random_walk_batch(seed: int, fst: Fst, batch: int, length: int) -> Batch:
    """Input strings read off random walks from the start state.

    At each state one out-arc is picked uniformly; its input label is the next
    token.  Needs arcs grouped by source state (as ``powerlaw_fst`` lists them).
    """
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    Q = fst.num_states
    if np.any(np.diff(fst.src) < 0):
        raise ValueError("random_walk_batch needs arcs grouped by source state")
    out_start = np.zeros(Q + 1, np.int64)
    np.cumsum(np.bincount(fst.src, minlength=Q), out=out_start[1:])
    deg = np.diff(out_start)
    toks = np.empty((batch, length), np.int32)
    state = np.full(batch, fst.start, np.int64)
    for t in range(length):
        if np.any(deg[state] == 0):
            raise ValueError("random walk reached a state with no out-arcs")
        k = out_start[state] + (rng.random(batch) * deg[state]).astype(np.int64)
        toks[:, t] = fst.ilabel[k]
        state = fst.dst[k]
    lengths = np.full(batch, length, np.int64)
    return _batch_from_lengths(lengths, toks.reshape(-1), meta={"kind": "random_walk"})


# --------------------------------------------------------------------------
# The five workload configurations
# --------------------------------------------------------------------------

def config(i: int, seed: int = 0, **kw):
    """Return (Fst, Batch) for workload configuration ``i`` (1..5).

    Keyword overrides shrink a configuration for quick tests (vocab, batch,
    num_states, ...); the defaults are the full sizes.
    1: bigram tagger, 12 tags, vocab 1000, one sentence of 30 tokens.
    2: trigram tagger, 45 tags, vocab 50k, 4096 sentences, lognormal lengths.
    3: the FST of 2 with 1024 sentences (training batch).
    4: bigram tagger, 45 tags, vocab 200k, 16384 sentences of length U{1..200}.
    5: power-law WFST, 1M states, 50M arcs, 1024 random-walk strings of 100.
    """
    if i == 1:
        fst = hmm_bigram(seed, kw.get("n_tags", 12), kw.get("vocab", 1000), "uniform123", 1.0)
        _, _, rb = _streams(seed)
        B = kw.get("batch", 1)
        L = kw.get("length", 30)
        toks = zipf_tokens(rb, fst.num_ilabels, 1.1, B * L)
        return fst, _batch_from_lengths(np.full(B, L, np.int64), toks, {"config": 1})
    if i in (2, 3):
        fst = hmm_trigram(seed, kw.get("n_tags", 45), kw.get("vocab", 50000))
        _, _, rb = _streams(seed)
        if i == 3:
            rb = np.random.default_rng(np.random.SeedSequence(seed).spawn(4)[3])
        B = kw.get("batch", 4096 if i == 2 else 1024)
        lens = lognormal_lengths(rb, B, 25.0, 0.5, kw.get("min_len", 5), kw.get("max_len", 60))
        toks = zipf_tokens(rb, fst.num_ilabels, 1.1, int(lens.sum()))
        return fst, _batch_from_lengths(lens, toks, {"config": i})
    if i == 4:
        fst = hmm_bigram(seed, kw.get("n_tags", 45), kw.get("vocab", 200000), "uniform123", 1.0)
        _, _, rb = _streams(seed)
        B = kw.get("batch", 16384)
        lens = rb.integers(1, kw.get("max_len", 200) + 1, B).astype(np.int64)
        toks = zipf_tokens(rb, fst.num_ilabels, 1.1, int(lens.sum()))
        return fst, _batch_from_lengths(lens, toks, {"config": 4})
    if i == 5:
        fst = powerlaw_fst(seed, kw.get("num_states", 1_000_000), kw.get("num_ilabels", 10_000),
                           kw.get("num_arcs", 50_000_000), d_min=kw.get("d_min", 10),
                           d_max=kw.get("d_max", 5000))
        b = random_walk_batch(seed, fst, kw.get("batch", 1024), kw.get("length", 100))
        b.meta["config"] = 5
        return fst, b
    raise ValueError(f"unknown configuration {i}")


def random_lattice(seed: int, num_ilabels: int, n_nodes: int, n_arcs: int, eps: float = 0.2) -> list:
    """An acyclic input lattice as arcs (from, to, label, log weight): nodes in
    topological order, one arc into every node from an earlier one (so every
    node is reachable from node 0), then n_arcs random forward arcs; label -1
    (epsilon) with probability eps; weights log U(0.2, 1)."""
    rng = np.random.default_rng(seed)
    arcs = []
    for v in range(1, n_nodes):
        arcs.append((int(rng.integers(0, v)), v, int(rng.integers(0, num_ilabels)),
                     float(np.log(rng.uniform(0.2, 1.0)))))
    for _ in range(n_arcs):
        u = int(rng.integers(0, n_nodes - 1))
        v = int(rng.integers(u + 1, n_nodes))
        a = -1 if rng.random() < eps else int(rng.integers(0, num_ilabels))
        arcs.append((u, v, a, float(np.log(rng.uniform(0.2, 1.0)))))
    return arcs


def confusion_network(seed: int, tokens, num_ilabels: int, alternatives: int = 3, zipf_s: float = 1.1,
                      deletion: float = 0.1) -> tuple[int, list]:
    """A confusion network ("sausage") around a token sequence, the usual
    shape of a recogniser's output lattice: node t -> t+1 carries the token
    and `alternatives` Zipf-drawn competitors, and with probability `deletion`
    an epsilon arc; the slot's weights are the logs of a Dirichlet(1) draw.
    Returns (num_nodes, arcs)."""
    rng = np.random.default_rng(seed)
    tokens = np.asarray(tokens)
    alt = zipf_tokens(rng, num_ilabels, zipf_s, alternatives * tokens.size).reshape(tokens.size, alternatives)
    dele = rng.random(tokens.size) < deletion
    arcs = []
    for t, w in enumerate(tokens):
        labels = [int(w)] + [int(x) for x in alt[t]] + ([-1] if dele[t] else [])
        p = rng.dirichlet(np.ones(len(labels)))
        arcs += [(t, t + 1, a, float(np.log(max(pi, 1e-30)))) for a, pi in zip(labels, p)]
    return tokens.size + 1, arcs
