"""Pins of the oracle's EM step (oracle/em.py) against what the mathematics
fixes: the unigram maximum-likelihood estimate (closed form), brute-force
path enumeration, local normalisation, and the monotone likelihood of EM;
and plausible mistakes planted in a copy of the M-step must fail a pin."""
import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from oracle import em


def _one_state(seed, M, N):
    """One state, one self-loop per label, random scores: a unigram model."""
    rng = np.random.default_rng(seed)
    sc = np.log(rng.dirichlet(np.ones(M))).astype(np.float32)
    fst = synth.Fst(1, M, 0, np.zeros(M, np.int32), np.zeros(M, np.int32), np.arange(M, dtype=np.int32),
                    np.arange(M, dtype=np.int32), sc, np.zeros(1, np.float32))
    lens = rng.integers(0, 9, N)
    batch = synth.random_batch(seed, M, lens, zipf_s=1.2)
    return fst, batch


@pytest.mark.parametrize("seed", range(4))
def test_unigram_closed_form(seed):
    """One state with one arc per label: one EM step from any scores gives
    the relative frequencies of the labels in the batch."""
    fst, batch = _one_state(seed, 7, 30)
    new, _, _ = em.em_step(fst, batch)
    freq = np.bincount(batch.tokens, minlength=7) / batch.tokens.size
    seen = freq > 0
    np.testing.assert_allclose(np.exp(new[seen]), freq[seen], rtol=1e-12)
    np.testing.assert_array_equal(new[~seen], -np.inf)


def _brute_counts(fst, batch):
    tot = np.zeros(fst.num_arcs)
    for b in range(batch.size):
        _, post, _ = brute.brute_forward_backward(fst, batch.sentence(b))
        tot += post
    return tot


@pytest.mark.parametrize("seed", range(6))
def test_m_step_against_brute_force_counts(seed):
    fst = synth.tiny_random_fst(seed, 3, 2, 9, final_prob=0.8)
    batch = synth.random_batch(seed, 2, np.random.default_rng(seed).integers(0, 5, 6))
    new, _, counts = em.em_step(fst, batch)
    bc = _brute_counts(fst, batch)
    np.testing.assert_allclose(counts, bc, atol=1e-12)
    tot = np.bincount(fst.src, weights=bc, minlength=fst.num_states)
    for k in range(fst.num_arcs):
        if tot[fst.src[k]] > 0:
            assert abs(np.exp(new[k]) - bc[k] / tot[fst.src[k]]) <= 1e-12
        else:
            assert new[k] == fst.arc_score[k]


@pytest.mark.parametrize("seed", range(4))
def test_local_normalisation_and_smoothing(seed):
    fst, batch = synth.config(1, batch=4, length=12, seed=seed)
    for lam in (0.0, 0.5):
        new, _, counts = em.em_step(fst, batch, smoothing=lam)
        tot = np.bincount(fst.src, weights=counts, minlength=fst.num_states)
        mass = np.bincount(fst.src, weights=np.exp(new), minlength=fst.num_states)
        visited = tot > 0
        np.testing.assert_allclose(mass[visited], 1.0, atol=1e-12)
        if lam > 0:
            assert np.all(np.isfinite(new))


def _normalised(fst):
    """Scores replaced by a log-softmax over each source state's arcs."""
    f = synth.Fst(**{**fst.__dict__})
    s = fst.arc_score.astype(np.float64)
    m = np.full(fst.num_states, -np.inf)
    np.maximum.at(m, fst.src, s)
    z = np.zeros(fst.num_states)
    np.add.at(z, fst.src, np.exp(s - m[fst.src]))
    f.arc_score = (s - m[fst.src] - np.log(z[fst.src])).astype(np.float32)
    return f


@pytest.mark.parametrize("seed", range(5))
def test_em_likelihood_is_monotone(seed):
    fst = _normalised(synth.tiny_random_fst(seed, 4, 3, 24, final_prob=1.0))
    fst.final_score = np.zeros(fst.num_states, np.float32)
    batch = synth.random_batch(seed, 3, np.random.default_rng(seed).integers(1, 8, 20))
    lls = []
    for _ in range(6):
        new, ll, _ = em.em_step(fst, batch)
        lls.append(ll)
        fst.arc_score = new.astype(np.float32)
    assert all(b >= a - 1e-5 * max(1, abs(a)) for a, b in zip(lls, lls[1:])), lls
    assert lls[-1] > lls[0]


MUTANTS = {
    "per destination": lambda fst, c, lam: _mutant_norm(fst, c, lam, fst.dst),
    "per label": lambda fst, c, lam: _mutant_norm(fst, c, lam, fst.ilabel),
    "smoothing not in the total": lambda fst, c, lam: np.log(c + lam) - np.log(
        np.bincount(fst.src, weights=c, minlength=fst.num_states)[fst.src]),
    "unvisited set to zero": lambda fst, c, lam: np.where(
        np.bincount(fst.src, weights=c, minlength=fst.num_states)[fst.src] > 0,
        em.m_step(fst, c, lam), 0.0),
}


def _mutant_norm(fst, c, lam, group):
    c = c + lam
    tot = np.bincount(group, weights=c)
    with np.errstate(divide="ignore"):
        return np.log(c) - np.log(tot[group])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_are_caught(name):
    """Each planted mistake fails the brute-force or normalisation pin."""
    caught = False
    for seed in range(6):
        fst = synth.tiny_random_fst(seed, 3, 2, 9, final_prob=0.8)
        batch = synth.random_batch(seed, 2, np.random.default_rng(seed).integers(0, 5, 6))
        bc = _brute_counts(fst, batch)
        tot = np.bincount(fst.src, weights=bc + 0.5, minlength=fst.num_states)
        want = np.where(tot[fst.src] > 0, np.log(bc + 0.5) - np.log(np.maximum(tot[fst.src], 1e-300)),
                        fst.arc_score)
        got = MUTANTS[name](fst, bc, 0.5)
        if not np.allclose(got, want, atol=1e-9):
            caught = True
            break
    assert caught, name
