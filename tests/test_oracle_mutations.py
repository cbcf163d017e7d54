"""The oracle pins must catch plausible mistakes.

Each case plants one mistake in a copy of the C oracle's source (a swapped
index, a dropped term, a reversed tie rule ...), builds that copy with gcc on
the CPU, and checks that at least one pin fails against it.  The pins are the
independent references of test_oracle_pins: brute-force enumeration, the
paper's worked example, and the forward-backward invariants.
"""
import ctypes
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from conftest import fig1_fst

SRC = os.path.join(os.path.dirname(oracle.__file__), "wfst_oracle.c")

MUTATIONS = {
    "forward_gathers_dst": ("const double x = prev[src[k]] + (double)arc_score[k];",
                            "const double x = prev[dst[k]] + (double)arc_score[k];"),
    "backward_reduces_by_dst": ("if (x > mx[src[k]]) mx[src[k]] = x;",
                                "if (x > mx[dst[k]]) mx[dst[k]] = x;"),
    "backward_gathers_src": ("const double x = (double)arc_score[k] + nxt[dst[k]];",
                             "const double x = (double)arc_score[k] + nxt[src[k]];"),
    "log_z_drops_final": ("const double x = la_n[q] + (double)final_score[q];",
                          "const double x = la_n[q];"),
    "posterior_drops_score": ("al[src[k]] + (double)arc_score[k] + be[dst[k]] - lz",
                              "al[src[k]] + be[dst[k]] - lz"),
    "posterior_beta_at_t_minus_1": ("const double *be = lb + (size_t)t * Q;",
                                    "const double *be = lb + (size_t)(t - 1) * Q;"),
    "lse_drops_log": ("mx[q] + log(acc[q])", "mx[q] + acc[q]"),
    "viterbi_tie_highest_id": ("(v == alpha_next[d] && k < bpt[d])",
                               "(v == alpha_next[d] && k > bpt[d]) || v >= alpha_next[d]"),
    "viterbi_final_tie_highest_state": ("if (qbest < 0 || v > best) {", "if (qbest < 0 || v >= best) {"),
    "viterbi_drops_final": ("volatile float v = alpha[q] + final_score[q];", "volatile float v = alpha[q];"),
    "viterbi_start_score": ("alpha[start] = 0.0f;", "alpha[start] = -0.5f;"),
    "viterbi_in_double": ("volatile float v = from + arc_score[k]; /* one binary32 RNE addition */",
                          "volatile float v = (float)((double)from + (double)arc_score[k] + 1e-7);"),
    "backtrace_uses_dst": ("q = src[k];\n        }", "q = dst[k];\n        }"),
}


def _build_mutant(name, tmpdir):
    before, after = MUTATIONS[name]
    code = open(SRC).read()
    assert code.count(before) >= 1, f"mutation anchor for {name} not found"
    code = code.replace(before, after)
    c = os.path.join(tmpdir, f"{name}.c")
    so = os.path.join(tmpdir, f"{name}.so")
    open(c, "w").write(code)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                    "-o", so, c, "-lm"], check=True, capture_output=True)
    return so


def _pins_pass():
    """Run a compact set of pins; return True if all of them hold."""
    try:
        g, fst, batch = fig1_fst()
        score, arcs, status = oracle.viterbi(fst, batch)
        if arcs.tolist() != g["expected"]["viterbi_arcs"]:
            return False
        if score[0] != np.float32(np.log(0.48)):
            return False
        lz, post, _, _ = oracle.forward_backward(fst, batch)
        if abs(lz[0] - math.log(0.56)) > 1e-7 or np.abs(post - g["expected"]["posteriors"]).max() > 1e-7:
            return False
        tie = synth.Fst(3, 1, 0, np.array([0, 0, 0, 0], np.int32), np.array([2, 2, 1, 1], np.int32),
                        np.zeros(4, np.int32), np.zeros(4, np.int32), np.full(4, -1, np.float32),
                        np.array([-np.inf, 0, 0], np.float32))
        _, arcs, _ = oracle.viterbi(tie, synth.Batch(np.array([0, 1]), np.array([0], np.int32)))
        if arcs.tolist() != [2]:
            return False
        for seed in range(60):
            tf = synth.tiny_random_fst(seed, 4, 2, 10, integer_scores=seed % 2 == 0)
            toks = np.random.default_rng(seed).integers(0, 2, 1 + seed % 5).astype(np.int32)
            b = synth.Batch(np.array([0, toks.size], np.int64), toks)
            s, a, st_ = oracle.viterbi(tf, b)
            best, argmaxes = brute.brute_viterbi(tf, toks)
            if s[0].view(np.uint32) != np.float32(best).view(np.uint32):
                return False
            if best != -np.inf and tuple(int(k) for k in a) not in argmaxes:
                return False
            lz, post, _, _ = oracle.forward_backward(tf, b)
            blz, bpost, _ = brute.brute_forward_backward(tf, toks)
            if not (lz[0] == blz == -math.inf) and abs(lz[0] - blz) > 1e-12 * max(1, abs(blz)):
                return False
            if np.abs(post - bpost).max() > 1e-10:
                return False
        return True
    except (ValueError, IndexError, AssertionError):
        return False


def test_unmutated_oracle_passes_pins():
    assert _pins_pass()


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, monkeypatch):
    with tempfile.TemporaryDirectory() as d:
        so = _build_mutant(name, d)
        real = oracle._load()
        lib = ctypes.CDLL(so)
        for fn in ("oracle_viterbi", "oracle_forward_backward", "oracle_fb_tables"):
            getattr(lib, fn).argtypes = getattr(real, fn).argtypes
            getattr(lib, fn).restype = getattr(real, fn).restype
        monkeypatch.setattr(oracle, "_lib", lib)
        assert not _pins_pass(), f"pins did not detect mutation {name}"
