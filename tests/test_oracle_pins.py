"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each check is independent of the oracle's own code: the paper's worked
example (Figures 1-3), brute-force enumeration of paths on tiny FSTs, a dense
matrix formulation of Eq. (1), closed forms (single-state and deterministic
FSTs), invariants of forward-backward, and central finite differences.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
import synth
from oracle import brute
from conftest import fig1_fst

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------- worked example

def test_fig3_composition_arithmetic():
    """Figure 1's arc weights are LM x translation-table products (Figure 3)."""
    g, _, _ = fig1_fst()
    comp = g["composition"]
    for k, (lm, tm) in comp["arcs"].items():
        assert math.isclose(comp["lm"][lm] * comp["tm"][tm], g["P"][int(k)], rel_tol=1e-12)


def test_fig1_viterbi():
    g, fst, batch = fig1_fst()
    score, arcs, status = oracle.viterbi(fst, batch)
    assert status[0] == oracle.ST_OK
    assert arcs.tolist() == g["expected"]["viterbi_arcs"]
    outs = [g["output_symbols"][fst.olabel[k]] for k in arcs]
    assert outs == g["expected"]["viterbi_output"]
    # 0 + f32(log .48) + 0 + 0 + 0 is exact in FP32
    assert score[0] == np.float32(np.log(np.float64(g["expected"]["viterbi_prob"])))


def test_fig1_forward_backward():
    g, fst, batch = fig1_fst()
    lz, post, fpost, status = oracle.forward_backward(fst, batch, final_posteriors=True)
    assert status[0] == oracle.ST_OK
    # Z = 0.48 + 0.08 up to the FP32 rounding of the two log scores
    assert abs(lz[0] - math.log(g["expected"]["Z"])) < 1e-7
    np.testing.assert_allclose(post, g["expected"]["posteriors"], atol=1e-7)
    assert abs(post.sum() - 3.0) < 1e-12
    assert abs(fpost[5] - 1.0) < 1e-12 and np.all(fpost[:5] == 0)


# ---------------------------------------------------------------- brute force

def _check_against_brute(fst, tokens):
    batch = synth.Batch(np.array([0, len(tokens)], np.int64), np.asarray(tokens, np.int32))
    score, arcs, status = oracle.viterbi(fst, batch)
    best, argmaxes = brute.brute_viterbi(fst, tokens)
    if best == -np.inf:
        assert status[0] == oracle.ST_NO_PATH and score[0] == -np.inf
        assert np.all(arcs == -1)
    else:
        assert status[0] == oracle.ST_OK
        assert score[0].view(np.uint32) == np.float32(best).view(np.uint32)
        assert tuple(int(k) for k in arcs) in argmaxes
    lz, post, fpost, st2 = oracle.forward_backward(fst, batch, final_posteriors=True)
    blz, bpost, bfpost = brute.brute_forward_backward(fst, tokens)
    if blz == -math.inf:
        assert lz[0] == -np.inf and st2[0] == oracle.ST_NO_PATH
        assert np.all(post == 0) and not np.any(np.isnan(post))
    else:
        assert abs(lz[0] - blz) <= 1e-12 * max(1.0, abs(blz))
        np.testing.assert_allclose(post, bpost, atol=1e-10)
        np.testing.assert_allclose(fpost, bfpost, atol=1e-10)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), Q=st.integers(1, 5), M=st.integers(1, 3),
       A=st.integers(0, 12), n=st.integers(0, 6), integer=st.booleans())
def test_oracle_vs_brute_force(seed, Q, M, A, n, integer):
    fst = synth.tiny_random_fst(seed, Q, M, A, integer_scores=integer)
    rng = np.random.default_rng(seed + 1)
    tokens = rng.integers(0, M, n).astype(np.int32)
    _check_against_brute(fst, tokens)


def test_oracle_vs_brute_force_dense_ties():
    """Integer scores in {0,-1,-2}: many equal-score paths; the oracle's path must
    still attain the exact maximum."""
    hits = 0
    for seed in range(200):
        fst = synth.tiny_random_fst(seed, 4, 2, 12, integer_scores=True, final_prob=1.0)
        tokens = np.random.default_rng(seed).integers(0, 2, 5).astype(np.int32)
        best, argmaxes = brute.brute_viterbi(fst, tokens)
        hits += len(argmaxes) > 1
        _check_against_brute(fst, tokens)
    assert hits > 20  # the fixture really exercises ties


# ---------------------------------------------------------------- tie rule

def test_tie_lowest_arc_id_and_lowest_final_state():
    """Two parallel arcs with equal score: the lower id wins; two final states
    with equal total: the lower state wins."""
    fst = synth.Fst(3, 1, 0,
                    np.array([0, 0, 0, 0], np.int32), np.array([2, 2, 1, 1], np.int32),
                    np.array([0, 0, 0, 0], np.int32), np.zeros(4, np.int32),
                    np.array([-1, -1, -1, -1], np.float32), np.array([-np.inf, 0, 0], np.float32))
    batch = synth.Batch(np.array([0, 1], np.int64), np.array([0], np.int32))
    score, arcs, status = oracle.viterbi(fst, batch)
    # states 1 and 2 both reach -1; state 1 is lower; arcs into 1 are ids 2, 3 -> 2
    assert score[0] == np.float32(-1) and arcs.tolist() == [2]


# ---------------------------------------------------------------- dense Eq. (1)

def test_dense_matrix_form_config1():
    fst, batch = synth.config(1)
    lz, _, _, _ = oracle.forward_backward(fst, batch, arc_posteriors=False)
    assert abs(lz[0] - brute.dense_log_z(fst, batch.tokens)) < 1e-9


def test_dense_matrix_form_small_trigram():
    fst, batch = synth.config(2, n_tags=4, vocab=30, batch=3, min_len=3, max_len=8)
    lz, _, _, _ = oracle.forward_backward(fst, batch, arc_posteriors=False)
    for b in range(batch.size):
        assert abs(lz[b] - brute.dense_log_z(fst, batch.sentence(b))) < 1e-9


# ---------------------------------------------------------------- closed forms

def _single_state_fst(seed, M=4, per_label=3):
    rng = np.random.default_rng(seed)
    A = M * per_label
    ilab = np.repeat(np.arange(M), per_label).astype(np.int32)
    sc = np.log(rng.uniform(0.05, 1.0, A)).astype(np.float32)
    return synth.Fst(1, M, 0, np.zeros(A, np.int32), np.zeros(A, np.int32), ilab,
                     np.zeros(A, np.int32), sc, np.array([np.float32(-0.25)], np.float32))


def test_single_state_closed_form():
    """A one-state FST (like Figure 3b): Viterbi = sum_t max_k s_k (FP32, left to
    right) + final; log Z = sum_t LSE_k s_k + final."""
    fst = _single_state_fst(3)
    toks = np.array([0, 2, 1, 3, 3, 0, 2], np.int32)
    batch = synth.Batch(np.array([0, toks.size], np.int64), toks)
    score, arcs, _ = oracle.viterbi(fst, batch)
    s = np.float32(0)
    for a in toks:
        s = np.float32(s + fst.arc_score[fst.ilabel == a].max())
    s = np.float32(s + fst.final_score[0])
    assert score[0].view(np.uint32) == s.view(np.uint32)
    lz, post, _, _ = oracle.forward_backward(fst, batch)
    ref = sum(np.logaddexp.reduce(fst.arc_score[fst.ilabel == a].astype(np.float64)) for a in toks)
    assert abs(lz[0] - (ref + np.float64(fst.final_score[0]))) < 1e-12
    # each position's posterior over its label's arcs is a softmax of the scores
    for a in range(fst.num_ilabels):
        sel = fst.ilabel == a
        cnt = int((toks == a).sum())
        p = np.exp(fst.arc_score[sel].astype(np.float64))
        np.testing.assert_allclose(post[sel], cnt * p / p.sum(), atol=1e-12)


def test_deterministic_fst_log_z_equals_path_score():
    """With exactly one accepting path, log Z is that path's FP64 score."""
    fst, batch = synth.config(1)
    # keep the first arc of every (state, label): a deterministic FST
    keep = np.zeros(fst.num_arcs, bool)
    seen = set()
    for k in range(fst.num_arcs):
        key = (int(fst.src[k]), int(fst.ilabel[k]))
        if key not in seen:
            seen.add(key)
            keep[k] = True
    d = synth.Fst(fst.num_states, fst.num_ilabels, 0, fst.src[keep], fst.dst[keep], fst.ilabel[keep],
                  fst.olabel[keep], fst.arc_score[keep], fst.final_score)
    score, arcs, st_ = oracle.viterbi(d, batch)
    lz, _, _, _ = oracle.forward_backward(d, batch, arc_posteriors=False)
    assert st_[0] == oracle.ST_OK
    path64 = sum(float(d.arc_score[k]) for k in arcs) + float(d.final_score[d.dst[arcs[-1]]])
    assert abs(lz[0] - path64) < 1e-12


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("cfg", ["config1", "trigram_small"])
def test_forward_backward_invariants(cfg):
    if cfg == "config1":
        fst, batch = synth.config(1)
    else:
        fst, batch = synth.config(2, vocab=300, batch=4)
    for b in range(batch.size):
        toks = batch.sentence(b)
        sub = synth.Batch(np.array([0, toks.size], np.int64), toks)
        lz, post, fpost, _ = oracle.forward_backward(fst, sub, final_posteriors=True)
        la, lb = oracle.fb_tables(fst, toks)
        # alpha . beta = Z at every time step
        for t in range(toks.size + 1):
            assert abs(np.logaddexp.reduce(la[t] + lb[t]) - lz[0]) < 1e-9 * max(1, abs(lz[0]))
        assert abs(lb[0][fst.start] - lz[0]) < 1e-9 * max(1, abs(lz[0]))
        # no epsilon arcs: every accepting path uses exactly n arcs
        assert abs(post.sum() - toks.size) < 1e-8
        assert abs(fpost.sum() - 1.0) < 1e-10
        assert post.min() >= 0 and post.max() <= toks.size + 1e-9
        vs, _, _ = oracle.viterbi(fst, sub)
        assert float(vs[0]) <= lz[0] + 1e-4


def test_finite_differences():
    """d log Z / d score_k = E[count_k], by central differences in the FP64 oracle."""
    fst, batch = synth.config(1)
    lz, post, _, _ = oracle.forward_backward(fst, batch)
    used = np.nonzero(np.isin(fst.ilabel, batch.tokens))[0]
    rng = np.random.default_rng(0)
    ks = rng.choice(used, 24, replace=False)
    ks = np.concatenate([ks, np.argsort(-post)[:8]])
    for k in ks:
        plus = synth.Fst(**{**fst.__dict__})
        plus.arc_score = fst.arc_score.copy()
        minus = synth.Fst(**{**fst.__dict__})
        minus.arc_score = fst.arc_score.copy()
        plus.arc_score[k] = np.float32(fst.arc_score[k] + 1e-3)
        minus.arc_score[k] = np.float32(fst.arc_score[k] - 1e-3)
        h = float(plus.arc_score[k]) - float(minus.arc_score[k])
        lp, _, _, _ = oracle.forward_backward(plus, batch, arc_posteriors=False)
        lm, _, _, _ = oracle.forward_backward(minus, batch, arc_posteriors=False)
        assert abs((lp[0] - lm[0]) / h - post[k]) < 1e-6


def test_gradient_weights_scale_per_sentence():
    fst, batch = synth.config(2, vocab=200, batch=5)
    g = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    _, total, _, _ = oracle.forward_backward(fst, batch, grad_log_z=g)
    acc = np.zeros(fst.num_arcs)
    for b in range(batch.size):
        toks = batch.sentence(b)
        _, p, _, _ = oracle.forward_backward(fst, synth.Batch(np.array([0, toks.size]), toks))
        acc += g[b] * p
    np.testing.assert_allclose(total, acc, atol=1e-10)


# ---------------------------------------------------------------- special cases

def test_empty_sentence():
    fst, _ = synth.config(1)
    fst.final_score = fst.final_score.copy()
    fst.final_score[0] = np.float32(-0.75)
    batch = synth.Batch(np.array([0, 0], np.int64), np.zeros(0, np.int32))
    score, arcs, status = oracle.viterbi(fst, batch)
    assert status[0] == oracle.ST_OK and score[0] == np.float32(-0.75) and arcs.size == 0
    lz, post, _, _ = oracle.forward_backward(fst, batch)
    assert lz[0] == -0.75 and np.all(post == 0)


def test_no_path_and_bad_token():
    g, fst, _ = fig1_fst()
    batch = synth.Batch(np.array([0, 2, 4, 5], np.int64), np.array([1, 0, 0, 7, 2], np.int32))
    score, arcs, status = oracle.viterbi(fst, batch)
    assert status.tolist() == [oracle.ST_NO_PATH, oracle.ST_BAD_TOKEN, oracle.ST_NO_PATH]
    assert np.all(score == -np.inf) and np.all(arcs == -1)
    lz, post, _, st2 = oracle.forward_backward(fst, batch)
    assert st2.tolist() == status.tolist()
    assert np.all(lz == -np.inf) and np.all(post == 0) and not np.any(np.isnan(post))
