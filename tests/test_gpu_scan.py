"""The forward pass as a time-parallel scan (wfst_forward_scan) against the
FP64 oracle: log Z within 1e-4 * max(1, |log Z|), every log alpha_t within
1e-4 * max(1, |log alpha_t|) of the oracle's forward table, statuses equal;
tiny FSTs with duplicate arcs and self-loops, empty / bad-token / no-path
sentences, the 12- and 45-tag bigram taggers, sentences of 200 tokens."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wf():
    import torch
    import paper_1701_03038_amd as wf
    assert torch.cuda.is_available()
    wf.load_library()
    return wf


def _check(wf, fst, batch, d, ctx, alpha_sentences=8):
    import torch
    lz, st, al = wf.forward_scan(d, batch.offsets, batch.tokens, alpha=True)
    torch.cuda.synchronize()
    lz, st, al = lz.cpu().numpy(), st.cpu().numpy(), al.cpu().numpy()
    olz, _, _, ost = oracle.forward_backward(fst, batch, arc_posteriors=False)
    np.testing.assert_array_equal(st, ost, err_msg=ctx)
    ok = ost == oracle.ST_OK
    assert np.all(lz[~ok] == -np.inf)
    err = np.abs(lz[ok].astype(np.float64) - olz[ok])
    assert np.all(err <= 1e-4 * np.maximum(1, np.abs(olz[ok]))), f"{ctx}: log Z err {err.max():.3g}"
    for b in range(min(batch.size, alpha_sentences)):
        if ost[b] == oracle.ST_BAD_TOKEN or batch.lengths()[b] == 0:
            continue
        la, _ = oracle.fb_tables(fst, batch.sentence(b))
        got = al[batch.offsets[b]:batch.offsets[b + 1]].astype(np.float64)
        want = la[1:]
        fin = np.isfinite(want)
        np.testing.assert_array_equal(np.isfinite(got), fin, err_msg=f"{ctx} b={b} support")
        d_ = np.abs(got[fin] - want[fin])
        assert np.all(d_ <= 1e-4 * np.maximum(1, np.abs(want[fin]))), f"{ctx} b={b}: alpha err {d_.max():.3g}"
    return lz


@pytest.mark.parametrize("seed", range(12))
def test_tiny(wf, seed):
    say(f"case: scan tiny seed={seed}")
    fst = synth.tiny_random_fst(seed, 1 + seed % 6, 1 + seed % 3, 5 + 3 * seed, final_prob=0.7)
    lens = np.random.default_rng(seed).integers(0, 12, 30)
    batch = synth.random_batch(seed, fst.num_ilabels, lens)
    toks = batch.tokens.copy()
    if toks.size > 5:
        toks[5] = fst.num_ilabels  # a bad token
    batch = synth.Batch(batch.offsets, toks)
    _check(wf, fst, batch, wf.Fst.from_synth(fst), f"seed={seed}")


def test_bigram_taggers(wf):
    for cfg, kw in ((1, {"batch": 16}), (4, {"vocab": 3000, "batch": 40, "max_len": 200})):
        say(f"case: scan config {cfg}")
        fst, batch = synth.config(cfg, **kw)
        d = wf.Fst.from_synth(fst)
        lz = _check(wf, fst, batch, d, f"config {cfg}")
        lz2, _, tape = wf.forward(d, batch.offsets, batch.tokens)
        lz2 = lz2.cpu().numpy()
        tape.free()
        fin = np.isfinite(lz)
        assert np.all(np.abs(lz[fin] - lz2[fin]) <= 2e-4 * np.maximum(1, np.abs(lz2[fin])))


def test_long_sentences(wf):
    fst, batch = synth.config(4, vocab=5000, batch=6, max_len=200)
    toks = synth.random_batch(9, fst.num_ilabels, [200, 200, 137, 1, 0, 64], zipf_s=1.1)
    say("case: scan T=200")
    _check(wf, fst, toks, wf.Fst.from_synth(fst), "T=200")


def test_too_many_states(wf):
    fst = synth.tiny_random_fst(1, 65, 2, 100)
    d = wf.Fst.from_synth(fst)
    with pytest.raises(wf.WfstError) as e:
        wf.forward_scan(d, np.array([0, 2]), np.array([0, 1]))
    assert e.value.code == wf.WFST_EUNSUPPORTED
