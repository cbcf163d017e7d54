#!/usr/bin/env python3
"""Throughput of the whole hot path on one MI355X.

Workload: the trigram HMM tagger written as a WFST (45 tags, 2071 tag-pair
states, vocabulary 50k, ~172M arcs) with a batch of 4096 sentences of
lognormal length (mean 25, clipped to [5, 60]) drawn Zipf(1.1) over the
vocabulary; synthetic and seeded (synth.config(2)).

One step = the whole path over the batch:
  1. wfst_fst_set_scores: new arc scores scattered into both layouts (the
     per-update part of the layout row),
  2. wfst_viterbi: batched Viterbi with on-device backtrace,
  3. wfst_forward: batched forward pass and log Z,
  4. wfst_backward: batched backward pass and expected counts (= gradient of
     sum log Z), written densely over all arcs.
value = input symbols per second = (sum of sentence lengths) / step time.

Also reported: per-kernel times (HIP events on the call stream) with the
method's bytes per launch and their fraction of the HBM peak (and of a live
1 GiB copy's bandwidth), the plain per-sentence form (the same kernels called
with one sentence per call), the training step on the 1024-sentence batch of
the same FST through torch.autograd, the bigram tagger (vocabulary 200k,
16384 sentences of length 1..200) batched against per-sentence, the
training step on the 1M-state power-law WFST (state vectors in global
memory, counts in fixed point), and the CPU
oracle on a bounded sample of the batch on this host, on one thread and on
all of them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input symbols/sec (Viterbi, fwd-bwd) batched vs per-sentence; % HBM roofline"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_sha():
    h = hashlib.sha256()
    for f in ("sweeps.hip", "prims.hip", "wfst_api.hip", "kernels.h", "layout.cpp", "layout.h"):
        with open(os.path.join(ROOT, "paper_1701_03038_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(fst_dev, batch, Q=None):
    """Bytes the method moves per launch (one batch), per input symbol (b, t)
    with label a (A_a arcs, D_a destination segments, D'_a source segments):
      Viterbi   8 A_a + 8 D_a + 4 D_a  (arcs {state, score}, segment (dst, end), back-pointer write)
      forward   8 A_a + 8 D_a          (arcs, segment table)
      backward  8 A_a + 8 D'_a         (the same over the reverse layout)
      counts    16 A_a per label the batch reads ({src, dst, score} + gradient write)
      score update 24 per arc (two layouts: arc id, score gather, score write)
      gradient fill 4 per arc (on the record path the backward sweep does
                    it, and its row then carries these bytes).
    With Q given (state vectors too large for on-chip memory) every pass also
    gathers 4 A_a and writes 4 D_a (4 D'_a) per symbol and the counts stream
    alpha and beta, 8 Q per visit."""
    import numpy as np
    arcs, dseg, rseg = (x.astype(np.int64) for x in fst_dev.label_stats())
    tokens = batch.tokens
    A_tot = int(arcs.sum())
    read = np.bincount(tokens, minlength=arcs.size) > 0
    out = {
        "viterbi": float((8 * arcs[tokens] + 12 * dseg[tokens]).sum()),
        "forward": float((8 * arcs[tokens] + 8 * dseg[tokens]).sum()),
        "backward": float((8 * arcs[tokens] + 8 * rseg[tokens]).sum()),
        "counts": float(16 * arcs[read].sum()),
        "scores": float(24 * A_tot),
        "grad_fill": float(4 * A_tot),
    }
    if Q is not None:
        out["viterbi"] += float((4 * arcs[tokens] + 4 * dseg[tokens]).sum())
        out["forward"] += float((4 * arcs[tokens] + 4 * dseg[tokens]).sum())
        out["backward"] += float((4 * arcs[tokens] + 4 * rseg[tokens]).sum())
        out["counts"] += float(8 * Q * tokens.size)
    return out


def lattice_bytes(fst_dev, Q, n_nodes, labels):
    """Bytes the method moves in one lattice pass: per labelled lattice arc
    the label's arcs and segments (8 A_a + 8 D_a, as a string step), per
    lattice arc (epsilon included) its source node's vector (4 Q), per node
    its vector written once (4 Q)."""
    import numpy as np
    arcs, dseg, _ = (x.astype(np.int64) for x in fst_dev.label_stats())
    lab = labels[labels >= 0]
    return float((8 * arcs[lab] + 8 * dseg[lab]).sum() + 4 * Q * labels.size + 4 * Q * n_nodes)


def kernel_table(prof, bytes_per, steps, traffic=None, fused_counts=False):
    """Per kernel kind: ms per pass over the batch (HIP events on the call
    stream, summed over the pass's launches), the method's bytes per pass,
    their rate and its fraction of the HBM peak; measured HBM bytes per pass
    from the committed counter summary when it is current.
    A checkpointed backward pass is one launch per block of steps and comes
    with a second forward pass (the blocks' recompute); with fused_counts the
    expected counts are taken inside the backward sweep, whose row then
    carries the count bytes too (the counts row is the conversion pass).
    With no gradient-fill launches the backward sweep zero-filled the
    gradient itself, and its row carries those bytes."""
    launches = {k: n for k, (ms, n) in prof.items()}
    blocks = max(1, round(launches.get("backward", 0) / max(steps, 1)))
    passes = {k: n / max(steps, 1) for k, n in launches.items()}
    if blocks > 1:
        passes["backward"] = 1
        passes["forward"] = 2
    by = dict(bytes_per)
    if launches.get("grad_fill", 0) == 0 and launches.get("backward", 0) > 0 and "grad_fill" in by:
        by["backward"] = by["backward"] + by["grad_fill"]
        by["grad_fill"] = 0.0
    if fused_counts:
        by["backward"] = by["backward"] + by["counts"]
        by["counts"] = 0.0
    kernels = {}
    for k, (ms, n) in prof.items():
        if n == 0 or k not in by:
            continue
        npass = passes[k] * steps
        avg = ms / npass
        gbs = by[k] / (avg * 1e-3) / 1e9
        row = {"ms_per_pass": round(avg, 4), "passes": npass, "launches": n, "alg_bytes_per_pass": by[k],
               "alg_GBps": round(gbs, 1), "alg_frac": round(gbs / PEAK_HBM_GBS, 4)}
        t = (traffic or {}).get(k)
        if t:
            row["dram_bytes_per_pass"] = t
            row["dram_GBps"] = round(t / (avg * 1e-3) / 1e9, 1)
        kernels[k] = row
    return kernels


def step_bytes(kernels, steps):
    return sum(v["alg_bytes_per_pass"] * v["passes"] for v in kernels.values()) / max(steps, 1)


def roofline_of(kernels):
    """The kernel kind with the most time per step, its rate and its fraction of peak."""
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_pass"] * kernels[k]["passes"])
    dk = kernels[dom]
    return {"bound": "hbm", "kernel": dom, "achieved": dk["alg_GBps"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(dk["alg_GBps"] / PEAK_HBM_GBS, 4), "traffic": dk.get("dram_bytes_per_pass")}


def load_traffic(name="traffic_trigram_4096.json"):
    """Measured HBM bytes per launch per kernel from a committed PMC summary,
    when it was taken on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_sha") != source_sha():
        return None
    return {k: v.get("bytes_per_pass", v.get("bytes_per_launch")) for k, v in t.get("kernels", {}).items()}


def _sub_batch(batch, lo, hi):
    import synth
    o = batch.offsets
    return synth.Batch((o[lo:hi + 1] - o[lo]).copy(), batch.tokens[int(o[lo]):int(o[hi])].copy())


def cpu_baseline(fst, batch, sample, threads=1):
    """The C oracle (Viterbi FP32 + forward-backward FP64) on the first `sample`
    sentences of the batch, split into `threads` contiguous parts run on as
    many host threads (the oracle call releases the interpreter lock)."""
    import threading
    import oracle
    syms = int(batch.offsets[sample])
    cuts = [round(sample * j / threads) for j in range(threads + 1)]
    parts = [_sub_batch(batch, cuts[j], cuts[j + 1]) for j in range(threads) if cuts[j + 1] > cuts[j]]
    tv = tf = 0.0
    for fn in (oracle.viterbi, oracle.forward_backward):
        ths = [threading.Thread(target=fn, args=(fst, p)) for p in parts]
        t0 = time.perf_counter()
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        dt = time.perf_counter() - t0
        if fn is oracle.viterbi:
            tv = dt
        else:
            tf = dt
    word = "one thread" if len(parts) == 1 else f"{len(parts)} threads"
    return {"value": syms / (tv + tf), "unit": "symbols/s", "cores": len(parts), "kind": "oracle",
            "sample": f"first {sample} of {batch.size} sentences ({syms} symbols): oracle Viterbi "
                      f"{tv:.2f} s + forward-backward with counts {tf:.2f} s, {word}",
            "host": host_cpu()}


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs)"
    except OSError:
        pass
    return f"{os.cpu_count()} logical CPUs"


def time_steps(step, steps, warmup, fst_dev=None):
    """Warm up, then time `steps` calls of step() between two events on the
    current stream (synchronised on both sides); ms per step and the library's
    per-kernel timings (HIP events on the call stream) over the timed region."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if fst_dev is not None:
        if fst_dev.health() != 0:
            raise SystemExit(f"kernel health flags {fst_dev.health():#x}")
        fst_dev.profile(True)
        fst_dev.profile_read(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(steps, 1)
    prof = None
    if fst_dev is not None:
        prof = fst_dev.profile_read(reset=True)
        fst_dev.profile(False)
    return ms, prof


def copy_bandwidth(dev, reps=5):
    """GB/s of a 1 GiB device-to-device copy (read + write bytes), median of reps."""
    import torch
    a = torch.ones(2**28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        out.append(2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    return sorted(out)[len(out) // 2]


def per_sentence_rates(wf, d, batch, off_dev, tok_dev, P):
    """The plain per-sentence form: the same entry points called with one
    sentence per call, on the first P sentences."""
    import torch
    dev = off_dev.device
    offs1 = [torch.tensor([0, int(batch.offsets[b + 1] - batch.offsets[b])], dtype=torch.int32, device=dev)
             for b in range(P)]
    toks1 = [tok_dev[int(batch.offsets[b]):int(batch.offsets[b + 1])] for b in range(P)]
    syms = int(batch.offsets[P])
    for b in range(min(P, 8)):  # warm the workspace
        wf.viterbi(d, offs1[b], toks1[b])
        wf.forward_backward(d, offs1[b], toks1[b])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for b in range(P):
        wf.viterbi(d, offs1[b], toks1[b])
    torch.cuda.synchronize()
    tv = time.perf_counter() - t
    t = time.perf_counter()
    for b in range(P):
        _, _, tape = wf.forward(d, offs1[b], toks1[b])
        wf.backward(d, tape)
        tape.free()
    torch.cuda.synchronize()
    tf = time.perf_counter() - t
    return {"sentences": P, "symbols": syms, "viterbi_symbols_per_s": round(syms / tv, 1),
            "fwd_bwd_symbols_per_s": round(syms / tf, 1),
            "viterbi_plus_fwd_bwd_symbols_per_s": round(syms / (tv + tf), 1)}


def batched_rates(wf, d, batch, off, tok, steps, warmup):
    """Batched Viterbi and batched forward + backward (expected counts), timed
    separately: symbols/s of each and per-kernel timings."""
    n = int(batch.offsets[-1])
    ms_v, _ = time_steps(lambda: wf.viterbi(d, off, tok), steps, warmup, d)

    def fb():
        _, _, tape = wf.forward(d, off, tok)
        wf.backward(d, tape)
        tape.free()
    ms_f, prof = time_steps(fb, steps, warmup, d)
    return {"viterbi_symbols_per_s": round(n / (ms_v * 1e-3), 1), "viterbi_ms": round(ms_v, 4),
            "fwd_bwd_symbols_per_s": round(n / (ms_f * 1e-3), 1), "fwd_bwd_ms": round(ms_f, 4)}, prof


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--per-sentence", type=int, default=512,
                    help="sentences run one per call for the per-sentence form (0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=1024, help="sentences timed on the CPU oracle (0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the multi-threaded oracle timing (0: the host's CPUs, at most 16)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick workgroup size and count path with wfst_fst_autotune on this batch (untimed)")
    ap.add_argument("--threads", type=int, default=0,
                    help="workgroup size per sentence of the sweeps (64..1024; 0: library default)")
    ap.add_argument("--powerlaw-steps", type=int, default=2,
                    help="timed training steps on the 1M-state power-law workload (0: skip)")
    ap.add_argument("--workloads", default="main,training,lattice,bigram,powerlaw",
                    help="comma-separated lines to run besides the main step (training, lattice, bigram, "
                         "powerlaw); "
                         "the main workload always runs (for profiler runs: --workloads main)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}); the multi-GPU form of "
              "this path is a design note only.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1701_03038_amd as wf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wf.load_library()
    dev = torch.device("cuda", 0)

    def to_dev(batch):
        return (torch.as_tensor(batch.offsets.astype(np.int32), device=dev),
                torch.as_tensor(batch.tokens, device=dev))

    log("generating the trigram tagger WFST and 4096 sentences")
    t = time.time()
    fst, batch = synth.config(2)
    log(f"  {fst.num_states} states, {fst.num_arcs} arcs, {batch.size} sentences, "
        f"{int(batch.offsets[-1])} symbols ({time.time() - t:.1f} s)")
    log("building the device layouts")
    t = time.time()
    d = wf.Fst.from_synth(fst, threads_per_sentence=args.threads)
    info = d.info()
    log(f"  done in {time.time() - t:.1f} s, {info['device_bytes'] / 2**30:.2f} GiB on device")

    off, tok = to_dev(batch)
    theta = torch.as_tensor(fst.arc_score, device=dev)
    n_sym = int(batch.offsets[-1])
    tuned = None
    if args.autotune:
        d.set_scores(theta)
        tuned = d.autotune(off, tok)
        log(f"autotune: {tuned['threads_per_sentence']} threads per sentence, {tuned['count_path']} counts; "
            f"{tuned['best_ms']} ms per pass")
        tuned = {k: v for k, v in tuned.items() if k != "times"}

    def step():
        d.set_scores(theta)
        wf.viterbi(d, off, tok)
        _, _, tape = wf.forward(d, off, tok)
        wf.backward(d, tape)
        tape.free()

    log(f"timing {args.steps} steps after {args.warmup} warmup steps")
    ms_step, prof = time_steps(step, args.steps, args.warmup, d)
    health = d.health()
    traffic = load_traffic()
    kernels = kernel_table(prof, algorithmic_bytes(d, batch), args.steps, traffic)
    roofline = roofline_of(kernels)
    copy_gbs = copy_bandwidth(dev)
    roofline["copy_GBps"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4)

    per_sentence = None
    want = set(args.workloads.split(","))
    if args.per_sentence > 0 and "main" in want:
        P = min(args.per_sentence, batch.size)
        log(f"per-sentence form on {P} sentences (one call per sentence)")
        per_sentence = per_sentence_rates(wf, d, batch, off, tok, P)

    training = None
    if "training" in want:
        log("training step on the 1024-sentence batch (LogPartition forward + backward)")
        _, b3 = synth.config(3)
        off3, tok3 = to_dev(b3)
        th3 = torch.tensor(fst.arc_score, device=dev, requires_grad=True)
        d.set_scores(th3.detach())
        tune3 = d.autotune(off3, tok3)
        log(f"  autotune: {tune3['threads_per_sentence']} threads per sentence, {tune3['count_path']} counts; "
            f"{tune3['best_ms']} ms per pass")
        tune3 = {k: v for k, v in tune3.items() if k != "times"}

        def train_step():
            th3.grad = None
            lz, _ = wf.log_partition(th3, d, off3, tok3)
            lz.sum().backward()
        ms3, prof3 = time_steps(train_step, args.steps, args.warmup, d)
        k3 = kernel_table(prof3, algorithmic_bytes(d, b3), args.steps)
        n3 = int(b3.offsets[-1])
        total_alg = step_bytes(k3, args.steps)
        training = {"workload": f"trigram tagger WFST ({fst.num_arcs} arcs), {b3.size} sentences, {n3} symbols "
                                "(lognormal lengths mean 25 in [5,60]); loss = sum of log Z; "
                                "step = set_scores + forward + backward with expected counts through "
                                "torch.autograd (LogPartition)",
                    "autotune": tune3,
                    "symbols_per_s": round(n3 / (ms3 * 1e-3), 1), "ms_per_step": round(ms3, 4),
                    "alg_bytes_per_step": total_alg,
                    "step_frac": round(total_alg / (ms3 * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                    "roofline": roofline_of(k3), "kernels": k3}
        del b3, off3, tok3, th3

    lattice = None
    if "lattice" in want:
        log("input lattices: confusion networks around the 4096 sentences, trigram tagger WFST")
        t = time.time()
        nets = [synth.confusion_network(1000 + b, batch.sentence(b), fst.num_ilabels, alternatives=3)
                for b in range(batch.size)]
        flat = wf.lattices_from_lists(nets)
        del nets
        noff_l, aoff_l, fr_l, to_l, lab_l, w_l = (torch.as_tensor(x, device=dev) for x in flat)
        n_nodes, n_larcs = int(flat[0][-1]), int(flat[1][-1])
        log(f"  {n_nodes} nodes, {n_larcs} lattice arcs ({int((flat[4] < 0).sum())} epsilon), "
            f"built in {time.time() - t:.1f} s")
        d.set_scores(theta)
        ms_l, prof_l = time_steps(lambda: wf.lattice_forward(d, noff_l, aoff_l, fr_l, to_l, lab_l, w_l),
                                  args.steps, args.warmup, d)
        _, st_l = wf.lattice_forward(d, noff_l, aoff_l, fr_l, to_l, lab_l, w_l)
        ok_l = int((st_l == wf.STATUS_OK).sum().item())
        k_l = kernel_table(prof_l, {"lattice": lattice_bytes(d, fst.num_states, n_nodes, flat[4])}, args.steps,
                           traffic)
        lattice = {"workload": f"trigram tagger WFST ({fst.num_arcs} arcs); {batch.size} confusion networks "
                               f"around the main batch's sentences: {n_nodes} nodes, {n_larcs} arcs (token + 3 "
                               "Zipf(1.1) competitors per slot, epsilon with probability 0.1, Dirichlet(1) "
                               "slot weights); pass = log Z of the FST composed with every lattice",
                   "lattice_arcs_per_s": round(n_larcs / (ms_l * 1e-3), 1),
                   "slots_per_s": round(n_sym / (ms_l * 1e-3), 1), "ms_per_pass": round(ms_l, 4),
                   "lattices_ok": ok_l, "roofline": roofline_of(k_l), "kernels": k_l}
        del noff_l, aoff_l, fr_l, to_l, lab_l, w_l, flat

    bigram = None
    if "bigram" in want:
        log("bigram tagger (vocabulary 200k), 16384 sentences of length 1..200")
        f4, b4 = synth.config(4)
        d4 = wf.Fst.from_synth(f4)
        off4, tok4 = to_dev(b4)
        tune4 = d4.autotune(off4, tok4, tune_chunk=True)
        log(f"  autotune: chunk {tune4['chunk_arcs']}, {tune4['threads_per_sentence']} threads per sentence, "
            f"{tune4['count_path']} counts; {tune4['best_ms']} ms per pass ({tune4['tried']} timed)")
        tune4 = {k: v for k, v in tune4.items() if k != "times"}
        rates4, prof4 = batched_rates(wf, d4, b4, off4, tok4, args.steps, args.warmup)
        k4 = kernel_table(prof4, algorithmic_bytes(d4, b4), args.steps)
        P4 = min(max(args.per_sentence, 1), b4.size)
        log(f"  per-sentence form on {P4} sentences")
        ps4 = per_sentence_rates(wf, d4, b4, off4, tok4, P4)
        log("  graphs: the batched pass as one replay, and one graph per sentence")
        n4 = int(b4.offsets[-1])
        g4 = wf.Graph(d4, off4, tok4)
        ms_g4, _ = time_steps(g4.replay, args.steps, args.warmup)
        g4.close()
        tg1 = {}
        for kind in ("viterbi", "viterbi_plus_fwd_bwd"):
            graphs1 = []
            for b in range(P4):
                o1 = torch.tensor([0, int(b4.offsets[b + 1] - b4.offsets[b])], dtype=torch.int32, device=dev)
                graphs1.append(wf.Graph(d4, o1, tok4[int(b4.offsets[b]):int(b4.offsets[b + 1])],
                                        forward_backward=kind != "viterbi"))
            torch.cuda.synchronize()
            t = time.perf_counter()
            for g1 in graphs1:
                g1.replay()
            torch.cuda.synchronize()
            tg1[kind] = time.perf_counter() - t
            for g1 in graphs1:
                g1.close()
            del graphs1
        log("  one 200-token sentence: sequential forward sweep vs time-parallel scan (latency)")
        lens4 = b4.lengths()
        b200 = int(np.nonzero(lens4 == 200)[0][0])
        o200 = torch.tensor([0, 200], dtype=torch.int32, device=dev)
        t200 = tok4[int(b4.offsets[b200]):int(b4.offsets[b200]) + 200]
        lat = {}
        for name, fn in (("forward_sweep", lambda: wf.forward(d4, o200, t200)[2].free()),
                         ("scan", lambda: wf.forward_scan(d4, o200, t200))):
            for _ in range(3):
                fn()
            ts = []
            for _ in range(20):
                torch.cuda.synchronize()
                t = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            lat[name + "_us"] = round(sorted(ts)[len(ts) // 2] * 1e6, 1)
        graph4 = {"batched_viterbi_plus_fwd_bwd_symbols_per_s": round(n4 / (ms_g4 * 1e-3), 1),
                  "batched_ms_per_replay": round(ms_g4, 4),
                  "per_sentence_graph_viterbi_symbols_per_s": round(ps4["symbols"] / tg1["viterbi"], 1),
                  "per_sentence_graph_viterbi_plus_fwd_bwd_symbols_per_s":
                      round(ps4["symbols"] / tg1["viterbi_plus_fwd_bwd"], 1),
                  "note": "graphs take fixed-point counts where the eager calls take per-visit records"}
        bigram = {"workload": f"bigram tagger WFST: 45 tags, 46 states, vocab 200000, {f4.num_arcs} arcs; "
                              f"{b4.size} sentences, {int(b4.offsets[-1])} symbols (lengths uniform 1..200)",
                  "autotune": tune4,
                  "batched": rates4, "per_sentence": ps4, "graphs": graph4,
                  "latency_one_sentence_T200": lat,
                  "batched_over_per_sentence": {
                      "viterbi": round(rates4["viterbi_symbols_per_s"] / ps4["viterbi_symbols_per_s"], 1),
                      "fwd_bwd": round(rates4["fwd_bwd_symbols_per_s"] / ps4["fwd_bwd_symbols_per_s"], 1)},
                  "roofline": roofline_of(k4), "kernels": k4}
        d4.close()
        del f4, b4, d4

    powerlaw = None
    if "powerlaw" in want and args.powerlaw_steps > 0:
        log("power-law WFST: 1M states, 50M arcs, 1024 random-walk strings of 100")
        t = time.time()
        f5, b5 = synth.config(5)
        log(f"  generated in {time.time() - t:.1f} s")
        t = time.time()
        d5 = wf.Fst.from_synth(f5)
        log(f"  device layouts in {time.time() - t:.1f} s, {d5.info()['device_bytes'] / 2**30:.2f} GiB")
        off5, tok5 = to_dev(b5)
        th5 = torch.tensor(f5.arc_score, device=dev, requires_grad=True)

        def train5():
            th5.grad = None
            lz, _ = wf.log_partition(th5, d5, off5, tok5)
            lz.sum().backward()
        ms5, prof5 = time_steps(train5, args.powerlaw_steps, 1, d5)
        k5 = kernel_table(prof5, algorithmic_bytes(d5, b5, Q=f5.num_states), args.powerlaw_steps,
                          load_traffic("traffic_powerlaw_1m.json"), fused_counts=True)
        n5 = int(b5.offsets[-1])
        total5 = step_bytes(k5, args.powerlaw_steps)
        powerlaw = {"workload": f"power-law WFST: {f5.num_states} states, {f5.num_arcs} arcs, out-degree "
                                "~d^-2.1 on [10,5000], labels Zipf(1.0) over 10k, scores -Exp(1); "
                                f"{b5.size} random-walk strings of 100 ({n5} symbols); CRF training step = "
                                "LogPartition forward + backward (expected counts = gradient)",
                    "steps": args.powerlaw_steps, "symbols_per_s": round(n5 / (ms5 * 1e-3), 1),
                    "ms_per_step": round(ms5, 3), "alg_bytes_per_step": total5,
                    "step_frac": round(total5 / (ms5 * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                    "roofline": roofline_of(k5), "kernels": k5}
        d5.close()
        del f5, b5, d5, th5

    if args.copy_calibration:
        log("1 GiB device copy (HBM counter reference)")
        a = torch.empty(2**28, dtype=torch.float32, device=dev)
        b2 = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b2.copy_(a)
        torch.cuda.synchronize()

    cpu = cpu_mt = None
    if args.cpu_sample > 0:
        sample = min(args.cpu_sample, batch.size)
        log(f"CPU oracle on {sample} sentences, one thread")
        cpu = cpu_baseline(fst, batch, sample)
        if "main" in want:
            nth = args.cpu_threads or min(os.cpu_count() or 1, 16)
            log(f"CPU oracle on {sample} sentences, {nth} threads")
            cpu_mt = cpu_baseline(fst, batch, sample, threads=nth)

    out = {
        "metric": METRIC,
        "value": round(n_sym / (ms_step * 1e-3), 1),
        "unit": "symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "trigram HMM tagger WFST: 45 tags, 2071 states, vocab 50000, "
                               f"{fst.num_arcs} arcs; {batch.size} sentences, {n_sym} symbols "
                               "(lognormal lengths mean 25 in [5,60], Zipf(1.1) tokens), seed 0",
                   "step": "set_scores + batched Viterbi with backtrace + batched forward (log Z) + "
                           "batched backward with expected counts over all arcs",
                   "parallelism": "single GPU",
                   "threads_per_sentence": tuned["threads_per_sentence"] if tuned else (args.threads or 256),
                   "autotune": tuned},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "batched_viterbi_symbols_per_s": round(n_sym / (kernels["viterbi"]["ms_per_pass"] * 1e-3), 1),
        "per_sentence": per_sentence,
        "training_1024": training,
        "lattice_4096": lattice,
        "bigram_16384": bigram,
        "powerlaw_1m": powerlaw,
        "cpu_oracle_threads": cpu_mt,
        "health": health,
        "source_sha": source_sha(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
