"""Autotuner of the batched passes (wfst_fst_autotune through the C ABI).

It changes only launch configuration (workgroup size per sentence, count
path, and with chunk tuning the arcs per lane chunk, which rebuilds both
layouts from the device layout), so after tuning the results must still
match the oracle to the usual bar: Viterbi bit-exact, log Z within 1e-4
relative, posteriors within 1e-5 per visit.  The cache file replays a choice
without timing.
"""
import json
import os

import numpy as np
import pytest

import synth
from gpu_common import assert_fb_parity, assert_viterbi_parity, say

pytestmark = pytest.mark.gpu

SIZES = (64, 128, 256, 512, 1024)


@pytest.fixture(scope="module")
def wf():
    import torch
    import paper_1701_03038_amd as wf
    assert torch.cuda.is_available()
    wf.load_library()
    return wf


def _tune(d, batch, **kw):
    import torch
    out = d.autotune(batch.offsets, batch.tokens, **kw)
    torch.cuda.synchronize()
    assert d.health() == 0, f"kernel health flags {d.health():#x}"
    return out


@pytest.mark.parametrize("case", ["tiny", "trigram"])
def test_autotune_keeps_parity(wf, case):
    say(f"case: autotune {case}")
    if case == "tiny":
        fst, batch = synth.config(1, batch=48)
    else:
        fst, batch = synth.config(2, vocab=200, batch=24)
    d = wf.Fst.from_synth(fst)
    r = _tune(d, batch)
    assert r["threads_per_sentence"] in SIZES and r["count_path"] in ("records", "grouped", "fixed_point")
    assert r["tried"] == len(r["times"]) and r["tried"] >= 10
    assert r["best_ms"] == min(r["times"].values())
    assert r["times"][(r["chunk_arcs"], r["threads_per_sentence"], r["count_path"])] == r["best_ms"]
    say(f"  chosen {r['threads_per_sentence']} / {r['count_path']}: best {r['best_ms']} ms")
    assert_viterbi_parity(fst, batch, d, ctx=f"autotuned {case}")
    assert_fb_parity(fst, batch, d, ctx=f"autotuned {case}")


def test_autotune_chunks_and_cache(wf, tmp_path):
    """Chunk tuning rebuilds the layouts (with the current scores, which the
    oracle FST carries after set_scores); the cache file replays the choice on
    a fresh FST without timing; a tape made before a rebuild is refused."""
    import torch
    fst, batch = synth.config(4, vocab=3000, batch=64, max_len=40)
    new = (fst.arc_score + np.random.default_rng(2).normal(0, 0.2, fst.num_arcs)).astype(np.float32)
    f2 = synth.Fst(**{**fst.__dict__})
    f2.arc_score = new
    d = wf.Fst.from_synth(fst, chunk_arcs=16)
    d.set_scores(torch.tensor(new, device="cuda"))
    _, _, old_tape = wf.forward(d, batch.offsets, batch.tokens)
    cache = str(tmp_path / "tune.json")
    say("case: autotune with chunk lengths")
    r = _tune(d, batch, cache_path=cache, tune_chunk=True)
    assert not r["from_cache"]
    assert {c for (c, _, _) in r["times"]} == {4, 8, 16, 32}
    assert d.info()["chunk_arcs"] == r["chunk_arcs"]
    assert_viterbi_parity(f2, batch, d, ctx="chunk-tuned")
    assert_fb_parity(f2, batch, d, ctx="chunk-tuned")
    if r["chunk_arcs"] != 16:
        with pytest.raises(wf.WfstError):
            wf.backward(d, old_tape)
    old_tape.free()
    entries = json.load(open(cache))
    assert len(entries) == 1
    (e,) = entries.values()
    assert e["chunk_arcs"] == r["chunk_arcs"] and e["threads_per_sentence"] == r["threads_per_sentence"]
    say("case: autotune from the cache")
    d2 = wf.Fst.from_synth(f2, chunk_arcs=16)
    r2 = _tune(d2, batch, cache_path=cache, tune_chunk=True)
    assert r2["from_cache"] and r2["tried"] == 0
    assert (r2["chunk_arcs"], r2["threads_per_sentence"], r2["count_path"]) == \
        (r["chunk_arcs"], r["threads_per_sentence"], r["count_path"])
    assert d2.info()["chunk_arcs"] == r["chunk_arcs"]
    assert_viterbi_parity(f2, batch, d2, ctx="from cache")
    assert_fb_parity(f2, batch, d2, ctx="from cache")
    assert os.path.exists(cache) and not os.path.exists(cache + ".tmp")


def test_autotune_empty_batch(wf):
    say("case: autotune empty batch")
    fst, _ = synth.config(1, batch=1)
    d = wf.Fst.from_synth(fst, threads_per_sentence=128)
    r = d.autotune(np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert r["threads_per_sentence"] == 128 and r["tried"] == 0 and r["times"] == {}
