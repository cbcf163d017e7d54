"""Pins of the lattice oracle (oracle/lattice.py): a chain lattice is the
string it spells (the string oracle's log Z); on small lattices log Z equals
the log-sum over every lattice path of (path weight + log Z of the string it
reads), epsilon arcs reading nothing -- composition distributes over paths;
and planted mistakes fail a pin."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import lattice as lat


def random_lattice(seed, M, n_nodes, n_arcs, eps=0.2):
    return synth.random_lattice(seed, M, n_nodes, n_arcs, eps)


def _paths(n_nodes, arcs):
    out = {}
    for e, (u, v, a, w) in enumerate(arcs):
        out.setdefault(u, []).append((v, a, w))

    def walk(u):
        if u == n_nodes - 1:
            yield [], 0.0
            return
        for v, a, w in out.get(u, []):
            for labels, ww in walk(v):
                yield ([a] if a >= 0 else []) + labels, w + ww
    return list(walk(0))


def _string_log_z(fst, labels):
    b = synth.Batch(np.array([0, len(labels)], np.int64), np.array(labels, np.int32))
    lz, _, _, _ = oracle.forward_backward(fst, b, arc_posteriors=False)
    return float(lz[0])


@pytest.mark.parametrize("seed", range(8))
def test_chain_is_the_string(seed):
    fst = synth.tiny_random_fst(seed, 4, 3, 20, final_prob=0.7)
    toks = np.random.default_rng(seed).integers(0, 3, 6)
    arcs = [(t, t + 1, int(a), 0.0) for t, a in enumerate(toks)]
    lz, A = lat.lattice_forward(fst, len(toks) + 1, arcs)
    want = _string_log_z(fst, list(toks))
    assert (lz == want == -np.inf) or abs(lz - want) <= 1e-12 * max(1, abs(want))
    la, _ = oracle.fb_tables(fst, toks.astype(np.int32))
    np.testing.assert_allclose(A, la, atol=1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_sum_over_paths(seed):
    fst = synth.tiny_random_fst(seed, 3, 2, 14, final_prob=0.8)
    n = 4 + seed % 3
    arcs = random_lattice(seed, 2, n, 4 + seed % 4)
    lz, _ = lat.lattice_forward(fst, n, arcs)
    terms = [w + _string_log_z(fst, labels) for labels, w in _paths(n, arcs)]
    terms = [x for x in terms if x > -np.inf]
    want = -np.inf if not terms else float(np.logaddexp.reduce(terms))
    assert (lz == want == -np.inf) or abs(lz - want) <= 1e-10 * max(1, abs(want))


MUTANTS = {
    "lattice weights dropped": lambda fst, n, arcs: lat.lattice_forward(fst, n, [(u, v, a, 0.0) for u, v, a, w in arcs]),
    "epsilon read as label 0": lambda fst, n, arcs: lat.lattice_forward(fst, n, [(u, v, max(a, 0), w) for u, v, a, w in arcs]),
    "only the first incoming arc": lambda fst, n, arcs: lat.lattice_forward(
        fst, n, [e for i, e in enumerate(arcs) if all(f[1] != e[1] for f in arcs[:i])]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_are_caught(name):
    caught = False
    for seed in range(10):
        fst = synth.tiny_random_fst(seed, 3, 2, 14, final_prob=0.8)
        n = 4 + seed % 3
        arcs = random_lattice(seed, 2, n, 4 + seed % 4, eps=0.4)
        terms = [w + _string_log_z(fst, labels) for labels, w in _paths(n, arcs)]
        terms = [x for x in terms if x > -np.inf]
        want = -np.inf if not terms else float(np.logaddexp.reduce(terms))
        got, _ = MUTANTS[name](fst, n, arcs)
        if not ((got == want == -np.inf) or abs(got - want) <= 1e-9 * max(1, abs(want))):
            caught = True
            break
    assert caught, name
