"""Forward pass over input lattices (wfst_lattice_forward) against the FP64
lattice oracle: log Z within 1e-4 * max(1, |log Z|) and every node vector
within 1e-4 * max(1, |A_v[q]|) with the same support; statuses equal.  The
tolerance is the string forward pass's: node vectors are FP32 after
normalisation, each node one FP32 log-sum-exp per incoming arc, merged in
FP64.  Cases: tiny random FSTs x random lattices with epsilon and parallel
arcs, chain lattices against wfst_forward, confusion networks on the 12- and
45-tag bigram taggers and on a trigram tagger (2071 states: several
workgroup-wide slices per label), and the malformed and degenerate inputs."""
import numpy as np
import pytest

import synth
from gpu_common import say
from oracle import lattice as lat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wf():
    import torch
    import paper_1701_03038_amd as wf
    assert torch.cuda.is_available()
    wf.load_library()
    return wf


def _run(wf, d, lattices):
    import torch
    flat = wf.lattices_from_lists(lattices)
    lz, st, al = wf.lattice_forward(d, *flat, node_alpha=True)
    torch.cuda.synchronize()
    assert d.health() == 0, f"kernel health flags {d.health():#x}"
    return lz.cpu().numpy(), st.cpu().numpy(), al.cpu().numpy(), flat[0]


def _check(wf, fst, d, lattices, ctx):
    lz, st, al, noff = _run(wf, d, lattices)
    for b, (n, arcs) in enumerate(lattices):
        olz, A = lat.lattice_forward(fst, n, arcs)
        if olz == -np.inf:
            assert st[b] == wf.STATUS_NO_PATH and lz[b] == -np.inf, f"{ctx} b={b}: status {st[b]}"
        else:
            assert st[b] == wf.STATUS_OK, f"{ctx} b={b}: status {st[b]}"
            err = abs(float(lz[b]) - olz)
            assert err <= 1e-4 * max(1.0, abs(olz)), f"{ctx} b={b}: log Z {lz[b]} vs {olz} (err {err:.3g})"
        got = al[noff[b]:noff[b + 1]].astype(np.float64)
        fin = np.isfinite(A)
        np.testing.assert_array_equal(np.isfinite(got), fin, err_msg=f"{ctx} b={b} support")
        e = np.abs(got[fin] - A[fin])
        assert np.all(e <= 1e-4 * np.maximum(1.0, np.abs(A[fin]))), f"{ctx} b={b}: node err {e.max():.3g}"
    return lz, st


@pytest.mark.parametrize("seed", range(10))
def test_tiny_random(wf, seed):
    say(f"case: lattice tiny seed={seed}")
    fst = synth.tiny_random_fst(seed, 1 + seed % 6, 1 + seed % 4, 5 + 3 * seed, final_prob=0.7)
    rng = np.random.default_rng(100 + seed)
    lattices = []
    for i in range(12):
        n = int(rng.integers(1, 12))
        arcs = synth.random_lattice(1000 * seed + i, fst.num_ilabels, n, int(rng.integers(0, 3 * n + 1)),
                                    eps=0.25) if n > 1 else []
        lattices.append((n, arcs))
    _check(wf, fst, wf.Fst.from_synth(fst), lattices, f"seed={seed}")


def test_chain_equals_string_forward(wf):
    say("case: lattice chains vs wfst_forward, config 1")
    fst, batch = synth.config(1, batch=24, length=30)
    d = wf.Fst.from_synth(fst)
    lattices = []
    for b in range(batch.size):
        toks = batch.sentence(b)
        lattices.append((len(toks) + 1, [(t, t + 1, int(a), 0.0) for t, a in enumerate(toks)]))
    lz, st = _check(wf, fst, d, lattices, "chains")
    lz2, st2, tape = wf.forward(d, batch.offsets, batch.tokens)
    lz2, st2 = lz2.cpu().numpy(), st2.cpu().numpy()
    tape.free()
    np.testing.assert_array_equal(st, st2)
    fin = np.isfinite(lz2)
    assert np.all(np.abs(lz[fin] - lz2[fin]) <= 2e-4 * np.maximum(1, np.abs(lz2[fin])))


@pytest.mark.parametrize("cfg,kw", [(1, {"batch": 20}), (4, {"vocab": 3000, "batch": 20, "max_len": 40})])
def test_confusion_networks_bigram(wf, cfg, kw):
    say(f"case: lattice confusion networks, config {cfg}")
    fst, batch = synth.config(cfg, **kw)
    lattices = [synth.confusion_network(50 + b, batch.sentence(b), fst.num_ilabels, alternatives=3)
                for b in range(batch.size)]
    _check(wf, fst, wf.Fst.from_synth(fst), lattices, f"config {cfg}")


def test_confusion_networks_trigram(wf):
    say("case: lattice confusion networks, trigram tagger 2071 states")
    fst, batch = synth.config(2, vocab=400, batch=6, min_len=5, max_len=14)
    lattices = [synth.confusion_network(70 + b, batch.sentence(b), fst.num_ilabels, alternatives=2)
                for b in range(batch.size)]
    lattices.append((9, synth.random_lattice(77, fst.num_ilabels, 9, 16, eps=0.2)))
    _check(wf, fst, wf.Fst.from_synth(fst), lattices, "trigram")


def test_degenerate_and_malformed(wf):
    import torch
    say("case: lattice degenerate and malformed inputs")
    fst = synth.tiny_random_fst(3, 4, 3, 20, final_prob=1.0)
    d = wf.Fst.from_synth(fst)
    M = fst.num_ilabels
    good = (4, [(0, 1, 0, -0.1), (0, 1, -1, -0.5), (1, 2, 1, 0.0), (0, 2, 2, -1.0), (2, 3, -1, 0.0),
                (1, 3, 0, -0.2)])
    cases = [
        ("single node", (1, [])),                       # log Z = final[start]
        ("unreachable end", (3, [(0, 1, 0, 0.0)])),      # NO_PATH
        ("disabled arc", (2, [(0, 1, 0, -np.inf)])),     # NO_PATH
        ("epsilon only", (3, [(0, 1, -1, -0.3), (1, 2, -1, -0.4), (0, 2, -1, 0.1)])),
        ("parallel arcs", (2, [(0, 1, 1, -0.1), (0, 1, 1, -0.1), (0, 1, 1, -2.0)])),
        ("good", good),
    ]
    _check(wf, fst, d, [c[1] for c in cases], "degenerate")
    # malformed lattices: statuses, and the well-formed neighbour still right
    flat = list(wf.lattices_from_lists([good, good, good, good, good]))
    noff, aoff, fr, to, lab, w = flat
    a0 = aoff[1]
    lab[a0 + 2] = M                      # lattice 1: label out of range
    a0 = aoff[2]
    to[a0], to[a0 + 1] = to[a0 + 1] + 1, to[a0]   # lattice 2: arcs not sorted by target
    a0 = aoff[3]
    fr[a0] = to[a0]                      # lattice 3: arc from == to
    lz, st = wf.lattice_forward(d, noff, aoff, fr, to, lab, w)
    torch.cuda.synchronize()
    lz, st = lz.cpu().numpy(), st.cpu().numpy()
    olz, _ = lat.lattice_forward(fst, *good)
    assert list(st) == [wf.STATUS_OK, wf.STATUS_BAD_TOKEN, wf.STATUS_BAD_INPUT, wf.STATUS_BAD_INPUT, wf.STATUS_OK]
    assert np.all(lz[1:4] == -np.inf)
    for b in (0, 4):
        assert abs(float(lz[b]) - olz) <= 1e-4 * max(1.0, abs(olz))
    # non-monotone node offsets anywhere: the whole batch is BAD_INPUT
    noff2 = noff.copy()
    noff2[2] = noff2[1] - 1
    lz, st = wf.lattice_forward(d, noff2, aoff, fr, to, lab, w)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == wf.STATUS_BAD_INPUT)
    assert np.all(lz.cpu().numpy() == -np.inf)
    # empty batch
    lz, st = wf.lattice_forward(d, np.zeros(1, np.int32), np.zeros(1, np.int32), [], [], [], [])
    assert lz.numel() == 0 and st.numel() == 0
    assert d.health() == 0
