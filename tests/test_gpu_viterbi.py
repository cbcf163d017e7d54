"""Viterbi on the GPU vs the serial oracle: bit-exact scores, identical paths.

Every case goes through the C ABI (wfst_fst_create / wfst_viterbi) via the
ctypes binding.  Scores are compared as uint32 bit patterns.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import fig1_fst
from gpu_common import assert_viterbi_parity, run_viterbi, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wf():
    import torch
    import paper_1701_03038_amd as wf
    assert torch.cuda.is_available()
    wf.load_library()
    return wf


def _random_sentences(seed, M, n, max_len):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, n)
    return synth.random_batch(seed, M, lens)


def test_fig1(wf):
    say("case: fig1 viterbi")
    g, fst, batch = fig1_fst()
    d = wf.Fst.from_synth(fst)
    score, arcs, status, ol = (x.cpu().numpy() for x in wf.viterbi(d, batch.offsets, batch.tokens, olabels=True))
    assert status[0] == 0
    assert arcs.tolist() == g["expected"]["viterbi_arcs"]
    assert [g["output_symbols"][o] for o in ol] == g["expected"]["viterbi_output"]
    assert score[0] == np.float32(np.log(0.48))


@pytest.mark.parametrize("chunk,nt", [(16, 256), (1, 64), (2, 128), (3, 1024)])
@pytest.mark.parametrize("integer", [False, True])
def test_tiny_random(wf, chunk, nt, integer):
    for seed in range(12):
        say(f"case: tiny viterbi seed={seed} chunk={chunk} nt={nt} int={integer}")
        fst = synth.tiny_random_fst(seed, 1 + seed % 6, 1 + seed % 3, 4 + 3 * seed, integer_scores=integer)
        batch = _random_sentences(seed, fst.num_ilabels, 50, 7)
        d = wf.Fst.from_synth(fst, chunk_arcs=chunk, threads_per_sentence=nt)
        assert_viterbi_parity(fst, batch, d, f"seed={seed}")


def test_dense_ties_multichunk(wf):
    """Integer scores and long parallel-arc segments split over several chunks."""
    rng = np.random.default_rng(5)
    Q, M, A = 6, 2, 400
    fst = synth.Fst(Q, M, 0, rng.integers(0, Q, A).astype(np.int32), rng.integers(0, Q, A).astype(np.int32),
                    rng.integers(0, M, A).astype(np.int32), np.zeros(A, np.int32),
                    -rng.integers(0, 2, A).astype(np.float32), np.zeros(Q, np.float32))
    batch = _random_sentences(7, M, 64, 12)
    for chunk in (1, 4, 16, 64):
        say(f"case: dense ties chunk={chunk}")
        d = wf.Fst.from_synth(fst, chunk_arcs=chunk)
        assert_viterbi_parity(fst, batch, d, f"chunk={chunk}")


def test_config1(wf):
    say("case: config1")
    fst, batch = synth.config(1)
    d = wf.Fst.from_synth(fst)
    assert_viterbi_parity(fst, batch, d, "config1")
    fst, batch = synth.config(1, batch=64)
    assert_viterbi_parity(fst, batch, d, "config1 x64")


@pytest.mark.parametrize("nt", [64, 256, 1024])
def test_trigram_small(wf, nt):
    say(f"case: trigram small nt={nt}")
    fst, batch = synth.config(2, vocab=2000, batch=300)
    d = wf.Fst.from_synth(fst, threads_per_sentence=nt)
    assert_viterbi_parity(fst, batch, d, f"trigram small nt={nt}")


def test_edge_cases(wf):
    say("case: edge cases")
    g, fst, _ = fig1_fst()
    d = wf.Fst.from_synth(fst)
    # no path, bad token, empty sentence (start not final -> no path), valid
    batch = synth.Batch(np.array([0, 2, 4, 4, 7], np.int64), np.array([1, 0, 0, 7, 0, 1, 2], np.int32))
    score, arcs, status = run_viterbi(d, batch)
    assert status.tolist() == [oracle.ST_NO_PATH, oracle.ST_BAD_TOKEN, oracle.ST_NO_PATH, oracle.ST_OK]
    assert np.all(score[:3] == -np.inf) and np.all(arcs[:4] == -1)
    assert arcs[4:].tolist() == [0, 2, 4]
    # empty batch
    out = wf.viterbi(d, np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert out[0].numel() == 0
    # empty sentence with a final start state scores f[start]
    f2 = synth.Fst(**{**fst.__dict__})
    f2.final_score = fst.final_score.copy()
    f2.final_score[0] = np.float32(-1.25)
    d2 = wf.Fst.from_synth(f2)
    batch = synth.Batch(np.array([0, 0, 3, 3], np.int64), np.array([0, 1, 2], np.int32))
    assert_viterbi_parity(f2, batch, d2, "empty sentences")


def test_bad_offsets_flagged(wf):
    say("case: bad offsets")
    _, fst, _ = fig1_fst()
    d = wf.Fst.from_synth(fst)
    score, arcs, status = run_viterbi(d, synth.Batch(np.array([0, 3, 2], np.int64), np.array([0, 1, 2], np.int32)))
    assert status.tolist() == [0, 3]


def test_many_states_lds_only_rejected_else_global(wf):
    """70000 states: the state vectors do not fit LDS (and Viterbi's segment
    indices exceed 16 bits).  With state_memory=1 (LDS only) the passes are
    refused with WFST_EUNSUPPORTED before any sweep runs; by default they run
    in the global-memory form and match the oracle."""
    from gpu_common import assert_fb_parity
    say("case: 70000 states")
    Q = 70000
    src = np.array([0, 1, 2, 0], np.int32)
    dst = np.array([1, 2, Q - 1, 2], np.int32)
    lab = np.array([0, 0, 1, 0], np.int32)
    fin = np.full(Q, -np.inf, np.float32)
    fin[Q - 1] = 0.0
    sc = np.array([-0.5, -1.0, -0.25, -2.0], np.float32)
    d = wf.Fst(Q, 2, 0, src, dst, lab, sc, fin, state_memory=1)
    with pytest.raises(wf.WfstError) as e:
        wf.viterbi(d, np.array([0, 2], np.int32), np.array([0, 1], np.int32))
    assert e.value.code == wf.WFST_EUNSUPPORTED
    with pytest.raises(wf.WfstError) as e:
        wf.forward(d, np.array([0, 2], np.int32), np.array([0, 1], np.int32))
    assert e.value.code == wf.WFST_EUNSUPPORTED
    fst = synth.Fst(Q, 2, 0, src, dst, lab, np.zeros(4, np.int32), sc, fin)
    batch = synth.Batch(np.array([0, 2, 5, 5, 6], np.int64), np.array([0, 1, 0, 0, 1, 0], np.int32))
    d = wf.Fst.from_synth(fst)
    assert_viterbi_parity(fst, batch, d, "70000 states")
    assert_fb_parity(fst, batch, d, "70000 states")


def test_rejects_bad_scores(wf):
    _, fst, _ = fig1_fst()
    sc = fst.arc_score.copy()
    sc[2] = np.nan
    with pytest.raises(wf.WfstError):
        wf.Fst(fst.num_states, fst.num_ilabels, 0, fst.src, fst.dst, fst.ilabel, sc, fst.final_score)


def test_deterministic_repeat(wf):
    fst, batch = synth.config(2, vocab=1000, batch=128)
    d = wf.Fst.from_synth(fst)
    a = run_viterbi(d, batch)
    b = run_viterbi(d, batch)
    for x, y in zip(a, b):
        assert x.tobytes() == y.tobytes()


@pytest.mark.slow
def test_config2_full(wf):
    """The full trigram workload: 172M arcs, 4096 sentences, bit-exact on all."""
    say("case: config2 full: generating")
    fst, batch = synth.config(2)
    say("case: config2 full: building device FST")
    d = wf.Fst.from_synth(fst)
    say("case: config2 full: decoding + oracle")
    assert_viterbi_parity(fst, batch, d, "config2 full")


def test_att_fig1_output_string(wf):
    """Figure 1 read from AT&T text, decoded on the GPU: the best path's
    output symbols (looked up from best_olabels) are the figure's."""
    from test_att_reader import fig1_att
    text, isyms, osyms = fig1_att()
    f = wf.read_att(text, isyms, osyms)
    d = wf.Fst.from_synth(f)
    toks = f.encode(["le", "chat", "</s>"])
    score, arcs, status, ol = (x.cpu().numpy() for x in wf.viterbi(d, np.array([0, 3]), toks, olabels=True))
    assert status[0] == 0 and list(arcs) == [0, 2, 4]
    assert f.output_strings(ol, np.array([0, 3])) == [["the", "cat", "</s>"]]
    assert score[0] == np.float32(np.log(np.float64(0.48)))  # the cost, rounded once to FP32
