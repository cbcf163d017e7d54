"""Autotuner of the batched passes (wfst_fst_autotune through the C ABI).

It only changes the workgroup size per sentence, so after tuning the results
must still match the oracle to the usual bar: Viterbi bit-exact, log Z within
1e-4 relative, posteriors within 1e-5 per visit.
"""
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


@pytest.mark.parametrize("case", ["tiny", "trigram"])
def test_autotune_keeps_parity(wf, case):
    say(f"case: autotune {case}")
    if case == "tiny":
        fst, batch = synth.config(1, batch=48)
    else:
        fst, batch = synth.config(2, vocab=200, batch=24)
    d = wf.Fst.from_synth(fst)
    chosen, times = wf_tune(d, batch)
    assert chosen in SIZES
    assert times[chosen] is not None and times[chosen] > 0
    measured = [t for t in times.values() if t is not None]
    assert times[chosen] == min(measured)
    say(f"  chosen {chosen}: {times}")
    assert_viterbi_parity(fst, batch, d, ctx=f"autotuned {case}")
    assert_fb_parity(fst, batch, d, ctx=f"autotuned {case}")


def wf_tune(d, batch):
    import torch
    out = d.autotune(batch.offsets, batch.tokens)
    torch.cuda.synchronize()
    assert d.health() == 0, f"kernel health flags {d.health():#x}"
    return out


def test_autotune_empty_batch(wf):
    say("case: autotune empty batch")
    fst, _ = synth.config(1, batch=1)
    d = wf.Fst.from_synth(fst, threads_per_sentence=128)
    chosen, times = d.autotune(np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert chosen == 128 and all(t is None for t in times.values())
