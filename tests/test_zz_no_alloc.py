"""The no-allocation Viterbi entry point against wfst_viterbi: bit-equal
scores, paths and statuses on two calls in a row (the second smaller), and
its size limit."""
import numpy as np
import pytest

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


def _both(wf, d, batch):
    import torch
    a = [x.cpu().numpy() for x in wf.viterbi(d, batch.offsets, batch.tokens, olabels=True)]
    b = [x.cpu().numpy() for x in wf.viterbi_noalloc(d, batch.offsets, batch.tokens, olabels=True)]
    torch.cuda.synchronize()
    assert d.health() == 0
    return a, b


def _check_equal(a, b, ctx):
    for x, y, name in zip(a, b, ("score", "arcs", "status", "olabels")):
        assert x.dtype == y.dtype and x.shape == y.shape, (ctx, name)
        assert x.tobytes() == y.tobytes(), f"{ctx}: {name} differs"


def test_noalloc_matches_viterbi_two_calls(wf):
    fst, batch = synth.config(3, vocab=2000, batch=120)
    d = wf.Fst.from_synth(fst)
    say("case: no-alloc trigram 120 sentences")
    a, b = _both(wf, d, batch)
    _check_equal(a, b, "first call")
    small = synth.Batch(batch.offsets[:31].copy(), batch.tokens[:int(batch.offsets[30])].copy())
    say("case: no-alloc trigram 30 sentences (second, smaller call)")
    a, b = _both(wf, d, small)
    _check_equal(a, b, "second call")


def test_noalloc_edge_cases_and_ties(wf):
    """Empty, bad-token and no-path sentences; integer scores with dense ties."""
    for seed in range(400, 406):
        fst = synth.tiny_random_fst(seed, 3 + seed % 4, 2, 18, integer_scores=True, final_prob=0.7)
        lens = np.random.default_rng(seed).integers(0, 9, 40 - seed % 7)
        batch = synth.random_batch(seed, fst.num_ilabels, lens)
        toks = batch.tokens.copy()
        if toks.size > 3:
            toks[3] = fst.num_ilabels + 2  # one bad token
        batch = synth.Batch(batch.offsets, toks)
        d = wf.Fst.from_synth(fst)
        say(f"case: no-alloc tiny seed={seed}")
        a, b = _both(wf, d, batch)
        _check_equal(a, b, f"seed={seed}")


def test_noalloc_rejects_oversize_and_global_form(wf):
    fst, _ = synth.config(3, vocab=2000, batch=1)
    d = wf.Fst.from_synth(fst)
    segs = d.info()["max_fwd_segments_per_label"]
    n = int(1.1 * (256 << 20) / (8 * segs)) + 1  # tokens whose back-pointer bound exceeds 256 MiB
    lens = np.full((n + 59) // 60, 60)
    batch = synth.random_batch(9, fst.num_ilabels, lens)
    with pytest.raises(wf.WfstError) as e:
        wf.viterbi_noalloc(d, batch.offsets, batch.tokens)
    assert e.value.code == wf.WFST_EUNSUPPORTED
    ok = synth.random_batch(9, fst.num_ilabels, lens[:len(lens) // 2])  # half of it fits
    a, b = _both(wf, d, ok)
    _check_equal(a, b, "half")
    tiny = synth.tiny_random_fst(5, 4, 2, 12)
    g = wf.Fst.from_synth(tiny, state_memory=2)
    b = synth.random_batch(5, tiny.num_ilabels, [3, 4])
    with pytest.raises(wf.WfstError) as e:
        wf.viterbi_noalloc(g, b.offsets, b.tokens)
    assert e.value.code == wf.WFST_EUNSUPPORTED
