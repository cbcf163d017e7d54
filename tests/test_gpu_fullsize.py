"""The newer paths at the benchmark's full sizes, in the launch configuration
bench.py times, checked on sampled outputs the oracle computes one by one and
on properties that hold for every output:

- input lattices: the 4096 confusion networks around the trigram workload's
  sentences on the full trigram FST (172M arcs), one launch; three lattices
  against the FP64 lattice oracle (log Z within 1e-4 * max(1, |log Z|)), and
  for every lattice log Z >= log Z of its sentence + the weights of the
  sentence's own arcs (a lattice sums over more paths than that one);
- EM M-step: wfst_em_update on the full trigram FST with seeded counts (zeros
  included) against the oracle's M-step on the same counts, every arc, within
  a few FP32 rounding steps of the log probability;
- time-parallel scan: the full bigram tagger (46 states, vocabulary 200k) on
  sampled sentences including 200-token ones, log Z and log alpha against the
  oracle's forward pass.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import say
from oracle import em
from oracle import lattice as lat

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def wf():
    import torch
    import paper_1701_03038_amd as wf
    assert torch.cuda.is_available()
    wf.load_library()
    return wf


@pytest.fixture(scope="module")
def trigram(wf):
    say("case: full trigram FST: generating")
    fst, batch = synth.config(2)
    say("case: full trigram FST: building device layouts")
    d = wf.Fst.from_synth(fst)
    yield fst, batch, d
    d.close()


def test_lattices_full_trigram(wf, trigram):
    import torch
    fst, batch, d = trigram
    say("case: 4096 confusion networks: building")
    nets = [synth.confusion_network(1000 + b, batch.sentence(b), fst.num_ilabels, alternatives=3)
            for b in range(batch.size)]
    own = np.zeros(batch.size)  # weight of the sentence's own path: each slot's first arc reads its token
    for b, (n, arcs) in enumerate(nets):
        last = -1
        for (u, v, a, w) in arcs:
            if u != last:
                own[b] += w
                last = u
    say("case: 4096 confusion networks: one launch")
    flat = wf.lattices_from_lists(nets)
    lz, st = wf.lattice_forward(d, *flat)
    lz_s, st_s, tape = wf.forward(d, batch.offsets, batch.tokens)
    torch.cuda.synchronize()
    tape.free()
    assert d.health() == 0
    lz, st, lz_s = lz.cpu().numpy().astype(np.float64), st.cpu().numpy(), lz_s.cpu().numpy().astype(np.float64)
    assert np.all(st == wf.STATUS_OK) and np.all(st_s.cpu().numpy() == wf.STATUS_OK)
    slack = 1e-4 * np.maximum(1.0, np.abs(lz))
    low = lz_s + own
    assert np.all(lz >= low - slack), f"{np.sum(lz < low - slack)} lattices below their sentence path"
    lens = batch.lengths()
    index = lat.label_index(fst)
    for b in (0, int(np.argmax(lens)), batch.size - 1):
        say(f"case: lattice {b} against the oracle ({lens[b]} slots)")
        olz, _ = lat.lattice_forward(fst, *nets[b], index=index)
        assert abs(lz[b] - olz) <= 1e-4 * max(1.0, abs(olz)), f"lattice {b}: {lz[b]} vs {olz}"


def test_em_update_full_trigram(wf, trigram):
    import torch
    fst, _, d = trigram
    say("case: EM M-step on the full trigram FST")
    rng = np.random.default_rng(2024)
    counts = rng.exponential(1.0, fst.num_arcs).astype(np.float32)
    counts[rng.random(fst.num_arcs) < 0.3] = 0.0  # arcs no visit used
    dead = fst.src == 7  # a source state whose arcs all received nothing: scores stay
    counts[dead] = 0.0
    for smoothing in (0.0, 0.5):
        new = wf.em_update(d, torch.as_tensor(counts, device="cuda"), torch.as_tensor(fst.arc_score, device="cuda"),
                           smoothing=smoothing)
        torch.cuda.synchronize()
        new = new.cpu().numpy().astype(np.float64)
        want = em.m_step(fst, counts.astype(np.float64), smoothing)
        fin = np.isfinite(want)
        np.testing.assert_array_equal(np.isfinite(new), fin)
        err = np.abs(new[fin] - want[fin])
        tol = 4 * 2.0 ** -23 * np.maximum(1.0, np.abs(want[fin]))
        assert np.all(err <= tol), f"smoothing {smoothing}: max err {err.max():.3g}"
        if smoothing == 0.0:
            np.testing.assert_array_equal(new[dead], fst.arc_score[dead].astype(np.float64))


def test_scan_full_bigram(wf):
    import torch
    say("case: full bigram tagger (vocabulary 200k): generating")
    fst, batch = synth.config(4)
    d = wf.Fst.from_synth(fst)
    lens = batch.lengths()
    pick = np.concatenate([np.nonzero(lens == 200)[0][:4], np.arange(0, batch.size, batch.size // 60)])
    off, tok = wf.batch_from_sentences([batch.sentence(int(b)) for b in pick])
    sample = synth.Batch(off.astype(np.int64), tok)
    say(f"case: scan on {sample.size} sampled sentences")
    lz, st, al = wf.forward_scan(d, sample.offsets, sample.tokens, alpha=True)
    torch.cuda.synchronize()
    lz, st, al = lz.cpu().numpy(), st.cpu().numpy(), al.cpu().numpy()
    olz, _, _, ost = oracle.forward_backward(fst, sample, arc_posteriors=False)
    np.testing.assert_array_equal(st, ost)
    ok = ost == oracle.ST_OK
    err = np.abs(lz[ok].astype(np.float64) - olz[ok])
    assert np.all(err <= 1e-4 * np.maximum(1, np.abs(olz[ok]))), f"log Z max err {err.max():.3g}"
    for k in range(4):
        la, _ = oracle.fb_tables(fst, sample.sentence(k))
        got = al[sample.offsets[k]:sample.offsets[k + 1]].astype(np.float64)
        want = la[1:]
        fin = np.isfinite(want)
        np.testing.assert_array_equal(np.isfinite(got), fin)
        e = np.abs(got[fin] - want[fin])
        assert np.all(e <= 1e-4 * np.maximum(1, np.abs(want[fin]))), f"sentence {k}: alpha err {e.max():.3g}"
    d.close()
