"""EM re-estimation on the GPU (wfst_em_update after the batched
forward-backward) against the oracle's EM step: from the same scores, the
re-estimated arc probabilities agree within the bound the count tolerance
implies; iterating, the batch log-likelihood never decreases; repeats are
bitwise equal."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import say, visits_per_arc
from oracle import em

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wf():
    import torch
    import paper_1701_03038_amd as wf
    assert torch.cuda.is_available()
    wf.load_library()
    return wf


def _check_step(fst, batch, theta, new_gpu, smoothing):
    """p = exp(new) on the GPU vs the oracle's M-step from the same scores:
    |dp| <= 1e-5 * (n_k + p * N_q) / T_q + 1e-6, where T_q is the oracle's
    total count of the source state and N_q the sum of n_j over its arcs."""
    f = synth.Fst(**{**fst.__dict__})
    f.arc_score = theta
    want, _, counts = em.em_step(f, batch, smoothing)
    n_k = visits_per_arc(fst, batch)
    tot = np.bincount(fst.src, weights=counts + smoothing, minlength=fst.num_states)[fst.src]
    nq = np.bincount(fst.src, weights=n_k, minlength=fst.num_states)[fst.src]
    p_w, p_g = np.exp(want), np.exp(new_gpu.astype(np.float64))
    live = tot > 0
    bound = 1e-5 * (n_k + p_w * nq) / np.where(live, tot, 1.0) + 1e-6
    bad = np.nonzero(live & (np.abs(p_g - p_w) > bound))[0]
    assert bad.size == 0, f"{bad.size} arcs off, first {bad[:3]}: gpu {p_g[bad[:3]]} oracle {p_w[bad[:3]]}"
    np.testing.assert_array_equal(new_gpu[~live], theta[~live])


@pytest.mark.parametrize("case", ["bigram12", "bigram45", "tiny"])
def test_em_iterations(wf, case):
    import torch
    if case == "bigram12":
        fst, batch = synth.config(1, batch=64)
        smoothing = 0.0
    elif case == "bigram45":
        fst, batch = synth.config(4, vocab=3000, batch=200, max_len=60)
        smoothing = 0.0
    else:
        fst = synth.tiny_random_fst(3, 5, 3, 30, final_prob=1.0)
        fst.final_score = np.zeros(fst.num_states, np.float32)
        batch = synth.random_batch(3, 3, np.random.default_rng(3).integers(1, 9, 40))
        smoothing = 0.1
    d = wf.Fst.from_synth(fst)
    theta = torch.tensor(fst.arc_score, device="cuda")
    lls = []
    for it in range(5):
        say(f"case: EM {case} iteration {it}")
        new, ll = wf.em_step(d, theta, batch.offsets, batch.tokens, smoothing)
        torch.cuda.synchronize()
        assert d.health() == 0
        _check_step(fst, batch, theta.cpu().numpy(), new.cpu().numpy(), smoothing)
        lls.append(float(ll))
        theta = new
    if smoothing == 0.0:
        assert all(b >= a - 1e-4 * max(1.0, abs(a)) for a, b in zip(lls, lls[1:])), lls
        assert lls[-1] > lls[0]


def test_em_update_repeat_and_alias(wf):
    import torch
    fst, batch = synth.config(1, batch=16)
    d = wf.Fst.from_synth(fst)
    lz, counts, st = wf.forward_backward(d, batch.offsets, batch.tokens)
    theta = torch.tensor(fst.arc_score, device="cuda")
    a = wf.em_update(d, counts, theta)
    b = wf.em_update(d, counts, theta)
    c = theta.clone()
    wf.em_update(d, counts, c, out=c)
    torch.cuda.synchronize()
    assert a.cpu().numpy().tobytes() == b.cpu().numpy().tobytes() == c.cpu().numpy().tobytes()
    with pytest.raises(wf.WfstError):
        wf.em_update(d, counts, theta, smoothing=-1.0)
