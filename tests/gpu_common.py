"""Helpers shared by the GPU parity tests (they call the HIP path through the C ABI)."""
import sys

import numpy as np

import oracle
import synth


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_viterbi(fst_dev, batch, olabels=False):
    import torch
    import paper_1701_03038_amd as wf
    out = wf.viterbi(fst_dev, batch.offsets, batch.tokens, olabels=olabels)
    torch.cuda.synchronize()
    assert fst_dev.health() == 0, f"kernel health flags {fst_dev.health():#x}"
    return tuple(x.cpu().numpy() for x in out)


def assert_viterbi_parity(fst, batch, fst_dev, ctx=""):
    """Bit-exact best scores, identical paths and statuses."""
    score, arcs, status = run_viterbi(fst_dev, batch)
    osc, oarcs, ost = oracle.viterbi(fst, batch)
    np.testing.assert_array_equal(status, ost, err_msg=f"status {ctx}")
    bad = np.nonzero(score.view(np.uint32) != osc.view(np.uint32))[0]
    assert bad.size == 0, f"{ctx}: {bad.size} scores differ, first b={bad[:5]} gpu={score[bad[:5]]} oracle={osc[bad[:5]]}"
    diff = np.nonzero(arcs != oarcs)[0]
    assert diff.size == 0, f"{ctx}: {diff.size} path arcs differ, first token {diff[:5]}"
    return score, arcs, status


def visits_per_arc(fst, batch):
    """n_k: number of (sentence, step) visits whose input symbol is arc k's label."""
    cnt = np.bincount(batch.tokens, minlength=fst.num_ilabels)
    return cnt[fst.ilabel].astype(np.float64)


def assert_fb_parity(fst, batch, fst_dev, ctx="", per_sentence_tol=False):
    """log Z within 1e-4 relative; batch-summed posteriors within 1e-5 per visit."""
    import torch
    import paper_1701_03038_amd as wf
    lz, post, st = wf.forward_backward(fst_dev, batch.offsets, batch.tokens)
    torch.cuda.synchronize()
    assert fst_dev.health() == 0, f"kernel health flags {fst_dev.health():#x}"
    lz, post, st = lz.cpu().numpy(), post.cpu().numpy(), st.cpu().numpy()
    olz, opost, _, ost = oracle.forward_backward(fst, batch)
    np.testing.assert_array_equal(st, ost, err_msg=f"status {ctx}")
    ok = ost == oracle.ST_OK
    assert np.all(lz[~ok] == -np.inf)
    err = np.abs(lz[ok].astype(np.float64) - olz[ok])
    tol = 1e-4 * np.maximum(1.0, np.abs(olz[ok]))
    assert np.all(err <= tol), f"{ctx}: log Z max rel err {np.max(err / np.maximum(1, np.abs(olz[ok]))):.3g}"
    n_k = visits_per_arc(fst, batch)
    perr = np.abs(post.astype(np.float64) - opost)
    bound = 1e-5 * np.maximum(1.0, n_k)
    worst = np.argmax(perr / bound) if perr.size else 0
    assert np.all(perr <= bound), (f"{ctx}: posterior err {perr[worst]:.3g} at arc {worst} "
                                   f"(n_k={n_k[worst]}, gpu={post[worst]}, oracle={opost[worst]})")
    assert not np.any(np.isnan(post))
    return lz, post, st


def final_visits(fst, batch):
    """n_q: number of sentences whose last step can end in state q (the
    destinations of the last token's label; the start state for an empty one)."""
    n = np.zeros(fst.num_states, np.float64)
    last = {}
    for b in range(batch.size):
        o0, o1 = int(batch.offsets[b]), int(batch.offsets[b + 1])
        if o1 == o0:
            n[fst.start] += 1
            continue
        a = int(batch.tokens[o1 - 1])
        if not 0 <= a < fst.num_ilabels:
            continue
        if a not in last:
            last[a] = np.unique(fst.dst[fst.ilabel == a])
        n[last[a]] += 1
    return n


def assert_final_parity(fst, batch, fst_dev, ctx=""):
    """Batch-summed final-state posteriors within 1e-5 per sentence that can end there."""
    import torch
    import paper_1701_03038_amd as wf
    lz, post, fpost, st = wf.forward_backward(fst_dev, batch.offsets, batch.tokens, final_posteriors=True)
    torch.cuda.synchronize()
    assert fst_dev.health() == 0, f"kernel health flags {fst_dev.health():#x}"
    fpost = fpost.cpu().numpy().astype(np.float64)
    _, _, ofpost, ost = oracle.forward_backward(fst, batch, arc_posteriors=False, final_posteriors=True)
    np.testing.assert_array_equal(st.cpu().numpy(), ost, err_msg=f"status {ctx}")
    bound = 1e-5 * np.maximum(1.0, final_visits(fst, batch))
    err = np.abs(fpost - ofpost)
    worst = int(np.argmax(err / bound))
    assert np.all(err <= bound), f"{ctx}: final posterior err {err[worst]:.3g} at state {worst}"
    n_ok = int(np.sum(ost == oracle.ST_OK))
    assert abs(fpost.sum() - n_ok) <= 1e-5 * max(1, n_ok)
    return fpost


def oracle_fb_parallel(fst, batch, threads=None, final_posteriors=False):
    """oracle.forward_backward over the batch split into one part per host
    thread (results summed over parts in part order); prints each finished
    part.  For workloads where one serial call would run for minutes."""
    import os
    import threading
    n = batch.size
    threads = max(1, min(threads or min(os.cpu_count() or 1, 16), n))
    cuts = [round(n * j / threads) for j in range(threads + 1)]
    parts = [(cuts[j], cuts[j + 1]) for j in range(threads) if cuts[j + 1] > cuts[j]]
    res = [None] * len(parts)

    def run(j, lo, hi):
        o = batch.offsets
        sub = synth.Batch((o[lo:hi + 1] - o[lo]).copy(), batch.tokens[int(o[lo]):int(o[hi])].copy())
        res[j] = oracle.forward_backward(fst, sub, final_posteriors=final_posteriors)
        say(f"  oracle part {j + 1}/{len(parts)} done")

    ths = [threading.Thread(target=run, args=(j, lo, hi)) for j, (lo, hi) in enumerate(parts)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    lz = np.concatenate([r[0] for r in res])
    st = np.concatenate([r[3] for r in res])
    post = sum(r[1] for r in res)
    fpost = sum(r[2] for r in res) if final_posteriors else None
    return lz, post, fpost, st
