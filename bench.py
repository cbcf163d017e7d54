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

Also reported: per-kernel times (HIP events on the call stream), the HBM
roofline of the dominant kernel, the plain per-sentence form (the same
kernels called with one sentence per call) and the CPU oracle on a bounded
sample of the batch, on this host.
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


def live_arcs(fst, batch):
    """Per token (b, t) with label a and previous label p (the start state at
    t = 1): L = number of arcs with input a leaving a state p can reach, i.e.
    the arcs whose source alpha_{t-1} can occupy.  Cached per (p, a)."""
    import numpy as np
    il = fst.ilabel
    if np.all(il[1:] >= il[:-1]):
        order = None
        start = np.searchsorted(il, np.arange(fst.num_ilabels + 1))
    else:
        order = np.argsort(il, kind="stable")
        start = np.searchsorted(il[order], np.arange(fst.num_ilabels + 1))

    def arcs_of(a):
        sl = slice(start[a], start[a + 1])
        return sl if order is None else order[sl]

    dsts, cache = {}, {}
    L = np.zeros(batch.tokens.size, np.int64)
    offs = batch.offsets
    for bi in range(batch.size):
        for i in range(int(offs[bi]), int(offs[bi + 1])):
            a = int(batch.tokens[i])
            p = int(batch.tokens[i - 1]) if i > offs[bi] else -1
            key = (p, a)
            if key not in cache:
                if p not in dsts:
                    dsts[p] = np.array([fst.start]) if p < 0 else np.unique(fst.dst[arcs_of(p)])
                cache[key] = int(np.isin(fst.src[arcs_of(a)], dsts[p], assume_unique=False).sum())
            L[i] = cache[key]
    return L


def algorithmic_bytes(fst_dev, fst, batch):
    """Bytes each kernel must move per launch (one batch).  A, D, D' are the
    arcs, destination segments and source segments of a label; L the arcs of
    the token's label leaving states the previous step can reach; p the
    previous token's label.
      Viterbi 8A + 12D (arcs {state, score}, segment table, back-pointer),
      forward 8A + 8D (arcs, segment table, tape write), per token;
      backward 4D'(a) + 8L + 8D(p) per token (source keys of the label, the
        arcs of the marked segments, keys and tape of the states computed);
      counts 8A + 4D' per work item (arc ids and gradient writes, source keys)
        plus 8D(p) + 8D(a) + 8L per visit (alpha, beta and their keys, live arcs);
      score scatter 24 per arc (two layouts: arc id, score read, score write),
      gradient fill 4 per arc."""
    import numpy as np
    arcs, dseg, rseg = (x.astype(np.int64) for x in fst_dev.label_stats())
    tokens = batch.tokens
    A_tot = int(arcs.sum())
    first = np.zeros(tokens.size, bool)
    first[batch.offsets[:-1][batch.lengths() > 0]] = True
    prev = np.roll(tokens, 1)
    d_prev = np.where(first, 1, dseg[prev])
    L = live_arcs(fst, batch)
    n_vis = np.bincount(tokens, minlength=arcs.size)
    n_items = (n_vis + 63) // 64
    return {
        "viterbi": float((8 * arcs[tokens] + 12 * dseg[tokens]).sum()),
        "forward": float((8 * arcs[tokens] + 8 * dseg[tokens]).sum()),
        "backward": float((4 * rseg[tokens] + 8 * L + 8 * d_prev).sum()),
        "counts": float((n_items * (8 * arcs + 4 * rseg)).sum() + (8 * d_prev + 8 * dseg[tokens] + 8 * L).sum()),
        "scores": float(24 * A_tot),
        "grad_fill": float(4 * A_tot),
    }


def load_traffic(kernel):
    """Measured HBM bytes per launch from the committed PMC summary, when it was
    taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic_trigram_4096.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_sha") != source_sha() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel].get("bytes_per_launch")


def cpu_baseline(fst, batch, sample):
    """The C oracle (Viterbi FP32 + forward-backward FP64), single thread, on the
    first `sample` sentences of the batch."""
    import numpy as np
    import oracle
    import synth
    sub = synth.Batch(batch.offsets[:sample + 1].copy(), batch.tokens[:int(batch.offsets[sample])].copy())
    syms = int(sub.offsets[-1])
    t0 = time.perf_counter()
    oracle.viterbi(fst, sub)
    t1 = time.perf_counter()
    oracle.forward_backward(fst, sub)
    t2 = time.perf_counter()
    return {"value": syms / (t2 - t0), "unit": "symbols/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample} of {batch.size} sentences ({syms} symbols): oracle Viterbi "
                      f"{t1 - t0:.2f} s + forward-backward with counts {t2 - t1:.2f} s, one thread",
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--per-sentence", type=int, default=512,
                    help="sentences run one per call for the per-sentence form (0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=1024, help="sentences timed on the CPU oracle (0: skip)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the workgroup size per sentence with wfst_fst_autotune on this batch (untimed)")
    ap.add_argument("--threads", type=int, default=0,
                    help="workgroup size per sentence of the sweeps (64..1024; 0: library default)")
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

    dev = torch.device("cuda", 0)
    off = torch.as_tensor(batch.offsets.astype(np.int32), device=dev)
    tok = torch.as_tensor(batch.tokens, device=dev)
    theta = torch.as_tensor(fst.arc_score, device=dev)
    n_sym = int(batch.offsets[-1])
    tuned = None
    if args.autotune:
        d.set_scores(theta)
        chosen, times = d.autotune(off, tok)
        tuned = {"threads_per_sentence": chosen, "ms_per_pass": times}
        log(f"autotune: {chosen} threads per sentence; ms per pass {times}")

    def step():
        d.set_scores(theta)
        wf.viterbi(d, off, tok)
        _, _, tape = wf.forward(d, off, tok)
        wf.backward(d, tape)
        tape.free()

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if d.health() != 0:
        raise SystemExit(f"kernel health flags {d.health():#x}")

    log(f"timing {args.steps} steps")
    d.profile(True)
    d.profile_read(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / max(args.steps, 1)
    prof = d.profile_read(reset=True)
    d.profile(False)
    health = d.health()

    bytes_per = algorithmic_bytes(d, fst, batch)
    kernels = {}
    for k, (ms, n) in prof.items():
        if n == 0:
            continue
        avg = ms / n
        gbs = bytes_per[k] / (avg * 1e-3) / 1e9
        kernels[k] = {"ms_per_launch": round(avg, 4), "launches": n, "alg_bytes_per_launch": bytes_per[k],
                      "alg_GBps": round(gbs, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_launch"] * kernels[k]["launches"])
    dk = kernels[dom]
    traffic = load_traffic(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["alg_GBps"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(dk["alg_GBps"] / PEAK_HBM_GBS, 4), "traffic": traffic}

    per_sentence = None
    if args.per_sentence > 0:
        P = min(args.per_sentence, batch.size)
        log(f"per-sentence form on {P} sentences (one call per sentence)")
        offs1 = [torch.tensor([0, int(batch.offsets[b + 1] - batch.offsets[b])], dtype=torch.int32, device=dev)
                 for b in range(P)]
        toks1 = [tok[int(batch.offsets[b]):int(batch.offsets[b + 1])] for b in range(P)]
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
        per_sentence = {"sentences": P, "symbols": syms,
                        "viterbi_symbols_per_s": round(syms / tv, 1),
                        "fwd_bwd_symbols_per_s": round(syms / tf, 1),
                        "viterbi_plus_fwd_bwd_symbols_per_s": round(syms / (tv + tf), 1)}

    if args.copy_calibration:
        log("1 GiB device copy (HBM counter reference)")
        a = torch.empty(2**28, dtype=torch.float32, device=dev)
        b2 = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b2.copy_(a)
        torch.cuda.synchronize()

    cpu = None
    if args.cpu_sample > 0:
        log(f"CPU oracle on {args.cpu_sample} sentences")
        cpu = cpu_baseline(fst, batch, min(args.cpu_sample, batch.size))

    batched_parts = {k: kernels[k]["ms_per_launch"] for k in kernels}
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
                   "threads_per_sentence": tuned["threads_per_sentence"] if tuned else (args.threads or 256)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "batched_viterbi_symbols_per_s": round(n_sym / (batched_parts.get("viterbi", float("nan")) * 1e-3), 1),
        "per_sentence": per_sentence,
        "health": health,
        "source_sha": source_sha(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
