"""FSTs whose per-sentence state vectors do not fit on chip: the sweeps keep
them in a slot of global memory per workgroup (the forward sweep, in auto
mode, as a team of workgroups per sentence), and the expected counts are
accumulated in fixed point during the backward sweep.

Forced onto small FSTs (state_memory=2) so that the oracle's brute-force-
pinned territory and the edge cases run through the same kernels; then a
~40k-state FST (the size class of the paper's larger transducers) and 16
strings of the 1M-state power-law workload, where the global form is chosen
automatically.  Viterbi bit-exact; log Z within 1e-4 * max(1, |log Z|);
batch-summed posteriors within 1e-5 * max(1, n_k).
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import fig1_fst
from gpu_common import (assert_fb_parity, assert_final_parity, assert_viterbi_parity, oracle_fb_parallel, say,
                        visits_per_arc)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wf():
    import torch
    import paper_1701_03038_amd as wf
    assert torch.cuda.is_available()
    wf.load_library()
    return wf


def test_fig1_global_state(wf):
    say("case: fig1 global state")
    g, fst, batch = fig1_fst()
    d = wf.Fst.from_synth(fst, state_memory=2)
    assert_viterbi_parity(fst, batch, d, "fig1 gmem")
    lz, post, st = assert_fb_parity(fst, batch, d, "fig1 gmem")
    np.testing.assert_allclose(post, g["expected"]["posteriors"], atol=1e-6)
    edge = synth.Batch(np.array([0, 2, 4, 4, 7], np.int64), np.array([1, 0, 0, 7, 0, 1, 2], np.int32))
    assert_viterbi_parity(fst, edge, d, "fig1 gmem edge")
    assert_fb_parity(fst, edge, d, "fig1 gmem edge")
    assert_final_parity(fst, edge, d, "fig1 gmem edge")


@pytest.mark.parametrize("chunk,nt", [(16, 256), (2, 64), (5, 128)])
def test_tiny_global_state(wf, chunk, nt):
    for seed in range(300, 310):
        say(f"case: tiny gmem seed={seed} chunk={chunk} nt={nt}")
        fst = synth.tiny_random_fst(seed, 2 + seed % 6, 1 + seed % 3, 6 + 2 * (seed % 13), final_prob=0.8)
        lens = np.random.default_rng(seed).integers(0, 9, 50)
        batch = synth.random_batch(seed, fst.num_ilabels, lens)
        d = wf.Fst.from_synth(fst, chunk_arcs=chunk, threads_per_sentence=nt, state_memory=2)
        assert_viterbi_parity(fst, batch, d, f"gmem seed={seed}")
        assert_fb_parity(fst, batch, d, f"gmem seed={seed}")


@pytest.mark.parametrize("chunk,nt,ck", [(16, 256, 0), (2, 64, 1), (5, 128, 1), (16, 1024, 0)])
def test_tiny_team_forward(wf, chunk, nt, ck):
    """The team form of the forward sweep (state_memory=3: the workgroups on
    one XCD share each step and meet at a barrier), plain and checkpointed
    (its block recompute runs as a team too); the other sweeps in global
    memory per workgroup.  Includes empty, one-token and bad-token sentences."""
    for seed in range(340, 348):
        say(f"case: tiny team forward seed={seed} chunk={chunk} nt={nt} ck={ck}")
        fst = synth.tiny_random_fst(seed, 2 + seed % 6, 1 + seed % 3, 6 + 2 * (seed % 13), final_prob=0.8)
        lens = np.random.default_rng(seed).integers(0, 12, 40)
        batch = synth.random_batch(seed, fst.num_ilabels, lens)
        toks = batch.tokens.copy()
        if toks.size > 3:
            toks[3] = fst.num_ilabels  # a bad token
        batch = synth.Batch(batch.offsets, toks)
        d = wf.Fst.from_synth(fst, chunk_arcs=chunk, threads_per_sentence=nt, state_memory=3, checkpoint=ck)
        assert_fb_parity(fst, batch, d, f"team seed={seed}")
        assert d.health() == 0


def test_team_barrier_timeout_is_reported(wf):
    """Failure handling of the team sweep, forced from the host: with a poll
    limit of 1 a team stops at the first barrier its members do not pass at
    once; the call returns, health bit 64 reports it.  With the default limit
    again the same FST computes the right results."""
    import torch
    say("case: team barrier timeout (poll limit 1)")
    fst = synth.tiny_random_fst(351, 5, 2, 18, final_prob=0.8)
    batch = synth.random_batch(351, fst.num_ilabels, np.random.default_rng(351).integers(1, 10, 64))
    d = wf.Fst.from_synth(fst, state_memory=3)
    d.debug_team_spin(1)
    lz, st, tape = wf.forward(d, batch.offsets, batch.tokens)
    torch.cuda.synchronize()
    tape.free()
    assert d.health(clear=True) & 64, "a team with a poll limit of 1 should have stopped"
    d.debug_team_spin(0)
    assert_fb_parity(fst, batch, d, "team after a stopped run")
    assert d.health() == 0


def test_tiny_integer_ties_global_state(wf):
    """Integer scores (dense ties): the lowest-arc-id path, bit for bit."""
    for seed in range(320, 330):
        say(f"case: tiny integer gmem seed={seed}")
        fst = synth.tiny_random_fst(seed, 3 + seed % 4, 2, 20, integer_scores=True, final_prob=0.7)
        batch = synth.random_batch(seed, fst.num_ilabels, np.random.default_rng(seed).integers(0, 10, 40))
        d = wf.Fst.from_synth(fst, state_memory=2)
        assert_viterbi_parity(fst, batch, d, f"int gmem seed={seed}")


@pytest.mark.parametrize("state_memory", [1, 2])
def test_fixed_point_counts(wf, state_memory):
    """count_records=-2 (fixed-point accumulation) on chip and in global
    memory, with and without checkpointing, against the oracle; repeat is
    bitwise equal."""
    import torch
    fst, batch = synth.config(3, vocab=2000, batch=200)
    olz, opost, ofin, ost = oracle.forward_backward(fst, batch, final_posteriors=True)
    n_k = visits_per_arc(fst, batch)
    got = []
    for ck in (2, 1):
        say(f"case: fixed-point counts state_memory={state_memory} checkpoint={ck}")
        d = wf.Fst.from_synth(fst, count_records=-2, checkpoint=ck, state_memory=state_memory)
        r = []
        for _ in range(2):
            lz, post, st = wf.forward_backward(d, batch.offsets, batch.tokens)
            torch.cuda.synchronize()
            assert d.health() == 0
            r.append(post.cpu().numpy())
        assert r[0].tobytes() == r[1].tobytes()
        np.testing.assert_array_equal(st.cpu().numpy(), ost)
        assert np.all(np.abs(r[0] - opost) <= 1e-5 * np.maximum(1, n_k)), f"ck={ck}"
        got.append(r[0])
    assert got[0].tobytes() == got[1].tobytes(), "fixed-point counts differ with checkpointing"


def test_autograd_global_state(wf):
    """log_partition through the global-memory form: gradient = expected
    counts under weights g_b (FP64 oracle)."""
    import torch
    fst = synth.tiny_random_fst(17, 7, 3, 40, final_prob=0.7)
    batch = synth.random_batch(17, fst.num_ilabels, np.random.default_rng(17).integers(0, 12, 64))
    d = wf.Fst.from_synth(fst, state_memory=2)
    theta = torch.tensor(fst.arc_score, device="cuda", requires_grad=True)
    g = torch.linspace(-1.0, 2.0, batch.size, device="cuda")
    lz, st = wf.log_partition(theta, d, batch.offsets, batch.tokens)
    ok = st == 0
    (torch.where(ok, lz, torch.zeros_like(lz)) * g).sum().backward()
    gn = (g * ok).cpu().numpy().astype(np.float64)
    _, ograd, _, _ = oracle.forward_backward(fst, batch, grad_log_z=gn)
    n_k = visits_per_arc(fst, batch)
    assert np.all(np.abs(theta.grad.cpu().numpy() - ograd) <= 2e-5 * np.maximum(1, n_k))


def _powerlaw(num_states, num_arcs, labels, strings, length, seed=0):
    fst = synth.powerlaw_fst(seed, num_states, labels, num_arcs, d_min=10, d_max=min(5000, num_states))
    batch = synth.random_walk_batch(seed, fst, strings, length)
    return fst, batch


def test_40k_states(wf):
    """A 40k-state power-law WFST (2M arcs, 1000 labels): state vectors of
    40k states exceed LDS, so all three sweeps run in the global form."""
    say("case: 40k states: generating")
    fst, batch = _powerlaw(40_000, 2_000_000, 1000, 24, 30)
    d = wf.Fst.from_synth(fst)
    say("case: 40k states: Viterbi")
    assert_viterbi_parity(fst, batch, d, "40k")
    say("case: 40k states: forward-backward")
    assert_fb_parity(fst, batch, d, "40k")
    assert_final_parity(fst, batch, d, "40k")
    say("case: 40k states: checkpointed")
    d2 = wf.Fst.from_synth(fst, checkpoint=1)
    assert_fb_parity(fst, batch, d2, "40k ckpt")


@pytest.mark.slow
def test_powerlaw_1m_subset(wf):
    """16 random-walk strings of 100 symbols on the 1M-state, 50M-arc
    power-law WFST: Viterbi bit-exact, forward-backward and the gradient
    (through LogPartition) within tolerance of the FP64 oracle."""
    import torch
    say("case: 1M states: generating")
    fst, batch = synth.config(5, batch=16)
    say("case: 1M states: building device FST")
    d = wf.Fst.from_synth(fst)
    say("case: 1M states: Viterbi")
    assert_viterbi_parity(fst, batch, d, "1M")
    say("case: 1M states: LogPartition")
    theta = torch.tensor(fst.arc_score, device="cuda", requires_grad=True)
    lz, st = wf.log_partition(theta, d, batch.offsets, batch.tokens)
    lz.sum().backward()
    torch.cuda.synchronize()
    assert d.health() == 0
    say("case: 1M states: oracle (one part per host thread)")
    olz, opost, _, ost = oracle_fb_parallel(fst, batch)
    np.testing.assert_array_equal(st.cpu().numpy(), ost)
    err = np.abs(lz.detach().cpu().numpy().astype(np.float64) - olz)
    assert np.all(err <= 1e-4 * np.maximum(1, np.abs(olz))), f"log Z max err {err.max():.3g}"
    n_k = visits_per_arc(fst, batch)
    perr = np.abs(theta.grad.cpu().numpy().astype(np.float64) - opost)
    assert np.all(perr <= 1e-5 * np.maximum(1, n_k)), f"posterior max err {perr.max():.3g}"
