"""HIP graphs of whole batched pass sequences (wfst_graph_* through the C ABI).

Every replay is checked against eager calls on an FST with the same options,
bit for bit (the graph takes fixed-point counts where the eager default
would take records, so the eager reference uses count_records=-2), with the
program's own eager work and synchronisations between replays; and against
the oracle to the usual bar.
"""
import numpy as np
import pytest

import synth
from gpu_common import say, visits_per_arc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wf():
    import torch
    import paper_1701_03038_amd as wf
    assert torch.cuda.is_available()
    wf.load_library()
    return wf


def _eager(wf, d, off, tok):
    import torch
    s, a, st = wf.viterbi(d, off, tok)
    lz, post, fpost, st2 = wf.forward_backward(d, off, tok, final_posteriors=True)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (s, a, st, lz, post, fpost, st2)]


def _graph_out(g):
    import torch
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (g.best_score, g.best_arcs, g.status, g.log_z, g.status, g.grad,
                                      g.grad_final, g.status)]


def _same(a, b, ctx):
    for i, (x, y) in enumerate(zip(a, b)):
        assert x.tobytes() == y.tobytes(), f"{ctx}: output {i} differs"


@pytest.mark.parametrize("count_records", [0, -1, -2])
def test_graph_replays_match_eager(wf, count_records):
    import torch
    import oracle
    fst, batch = synth.config(4, vocab=3000, batch=96, max_len=60)
    other = synth.random_batch(7, fst.num_ilabels, np.random.default_rng(7).integers(0, 50, 40))
    dev = torch.device("cuda", 0)
    off = torch.as_tensor(batch.offsets.astype(np.int32), device=dev)
    tok = torch.as_tensor(batch.tokens, device=dev)
    d = wf.Fst.from_synth(fst, count_records=count_records)
    ref = wf.Fst.from_synth(fst, count_records=-2 if count_records == 0 else count_records)
    want = _eager(wf, ref, off, tok)
    want = want[:3] + [want[3], want[6], want[4], want[5], want[6]]
    say(f"case: graph count_records={count_records}")
    g = wf.Graph(d, off, tok, final=True)
    _same(_graph_out(g), want, "eager pass of creation")
    for rep in range(3):
        wf.forward_backward(d, other.offsets, other.tokens)  # eager work on the same FST in between
        torch.cuda.synchronize()
        g.replay()
        _same(_graph_out(g), want, f"replay {rep}")
    assert d.health() == 0
    olz, opost, _, ost = oracle.forward_backward(fst, batch)
    np.testing.assert_array_equal(g.status.cpu().numpy(), ost)
    n_k = visits_per_arc(fst, batch)
    assert np.all(np.abs(g.grad.cpu().numpy() - opost) <= 1e-5 * np.maximum(1, n_k))
    g.close()


def test_graph_new_tokens_in_place(wf):
    """Tokens rewritten in the bound buffer between replays: each replay
    decodes what the buffer holds."""
    import torch
    fst, batch = synth.config(1, batch=32)
    dev = torch.device("cuda", 0)
    off = torch.as_tensor(batch.offsets.astype(np.int32), device=dev)
    tok = torch.as_tensor(batch.tokens, device=dev)
    d = wf.Fst.from_synth(fst, count_records=-2)
    g = wf.Graph(d, off, tok, final=True)
    for seed in range(3):
        new = synth.random_batch(50 + seed, fst.num_ilabels, batch.lengths())
        tok.copy_(torch.as_tensor(new.tokens, device=dev))
        torch.cuda.synchronize()
        want = _eager(wf, d, off, tok)
        want = want[:3] + [want[3], want[6], want[4], want[5], want[6]]
        g.replay()
        _same(_graph_out(g), want, f"tokens {seed}")
    g.close()


def test_training_graph_with_scores(wf):
    """set_scores + forward + backward in one graph: new scores written into
    the bound score buffer are used by the next replay; the eager tape of an
    earlier forward is refused after a replay that replaced the scores."""
    import torch
    fst, batch = synth.config(3, vocab=1500, batch=64)
    dev = torch.device("cuda", 0)
    off = torch.as_tensor(batch.offsets.astype(np.int32), device=dev)
    tok = torch.as_tensor(batch.tokens, device=dev)
    theta = torch.tensor(fst.arc_score, device=dev)
    d = wf.Fst.from_synth(fst, count_records=-2)
    g = wf.Graph(d, off, tok, viterbi=False, arc_score=theta)
    _, _, tape = wf.forward(d, off, tok)
    rng = np.random.default_rng(1)
    for rep in range(3):
        new = (fst.arc_score + rng.normal(0, 0.2, fst.num_arcs)).astype(np.float32)
        theta.copy_(torch.as_tensor(new, device=dev))
        g.replay()
        torch.cuda.synchronize()
        got = (g.log_z.cpu().numpy(), g.grad.cpu().numpy())
        d.set_scores(torch.as_tensor(new, device=dev))
        lz, post, _ = wf.forward_backward(d, off, tok)
        torch.cuda.synchronize()
        assert got[0].tobytes() == lz.cpu().numpy().tobytes(), f"log Z replay {rep}"
        assert got[1].tobytes() == post.cpu().numpy().tobytes(), f"counts replay {rep}"
    with pytest.raises(wf.WfstError):
        wf.backward(d, tape)
    tape.free()
    g.close()


def test_graph_refusals(wf):
    """Forced checkpointing (plans from device totals) and the null stream
    are refused; autotune chunk rebuilds are refused while a graph exists."""
    import torch
    fst, batch = synth.config(1, batch=8)
    d = wf.Fst.from_synth(fst, checkpoint=1)
    with pytest.raises(wf.WfstError) as e:
        wf.Graph(d, batch.offsets, batch.tokens)
    assert e.value.code == wf.WFST_EUNSUPPORTED
    d2 = wf.Fst.from_synth(fst)
    g = wf.Graph(d2, batch.offsets, batch.tokens)
    with pytest.raises(wf.WfstError):
        d2.autotune(batch.offsets, batch.tokens, tune_chunk=True)
    g.close()
    torch.cuda.synchronize()
    assert d2.health() == 0
