"""The AT&T / OpenFST text reader (wfst_att_parse, host only): the paper's
Figure 1 transducer written in that format parses to the arrays of its
Figure 2, decodes (on the CPU oracle) to the figure's best output string, a
random FST survives a write/read round trip bit for bit, and malformed input
is refused with the line named."""
import numpy as np
import pytest

import oracle
import synth
import paper_1701_03038_amd as wf
from conftest import fig1_fst, load_golden


def fig1_att():
    """Figure 1 as AT&T text: arcs in the order of Figure 2 (arc id = line),
    weights as costs -log p, state 5 final, symbol tables for both sides."""
    g = load_golden("fig1.json")
    lab = []
    for a in range(len(g["R"]) - 1):
        lab += [g["input_symbols"][a]] * (g["R"][a + 1] - g["R"][a])
    lines = [f"{s}\t{t}\t{i}\t{o}\t{float(-np.log(np.float64(p)))!r}"
             for s, t, i, o, p in zip(g["S"], g["T"], lab, g["O"], g["P"])]
    lines += ["5"]
    isyms = "\n".join(f"{s} {i}" for i, s in enumerate(g["input_symbols"]))
    osyms = "\n".join(f"{s} {i}" for i, s in enumerate(g["output_symbols"]))
    return "\n".join(lines) + "\n", isyms, osyms


def test_fig1_arrays():
    g, ref, batch = fig1_fst()
    text, isyms, osyms = fig1_att()
    f = wf.read_att(text, isyms, osyms)
    assert (f.num_states, f.num_ilabels, f.start, f.num_arcs) == (6, 3, 0, 6)
    for name in ("src", "dst", "ilabel", "olabel"):
        np.testing.assert_array_equal(getattr(f, name), getattr(ref, name), err_msg=name)
    # cost -log p read back as score log p, rounded once to FP32
    np.testing.assert_array_equal(f.arc_score, np.float32(-np.float64(-np.log(np.array(g["P"], np.float64)))))
    np.testing.assert_array_equal(f.final_score, ref.final_score)


def test_fig1_decodes_to_its_output_string():
    text, isyms, osyms = fig1_att()
    f = wf.read_att(text, isyms, osyms)
    toks = f.encode(["le", "chat", "</s>"])
    batch = synth.Batch(np.array([0, 3], np.int64), toks)
    score, arcs, status = oracle.viterbi(f, batch)
    assert status[0] == oracle.ST_OK and list(arcs) == [0, 2, 4]
    assert f.output_strings(f.olabel[arcs], batch.offsets) == [["the", "cat", "</s>"]]
    assert f.output_strings(np.array([-1, -1, -1]), batch.offsets) == [None]


@pytest.mark.parametrize("seed", range(5))
def test_round_trip(seed):
    fst = synth.tiny_random_fst(seed, 3 + seed, 2 + seed % 3, 20, final_prob=0.5)
    fst.src[0] = fst.start  # the first line's source is the start state
    lines = [f"{s} {d} {i} {o} {float(-np.float64(x))!r}"
             for s, d, i, o, x in zip(fst.src, fst.dst, fst.ilabel, fst.olabel, fst.arc_score)]
    lines += [f"{q} {float(-np.float64(x))!r}" if np.isfinite(x) else f"{q} inf"
              for q, x in enumerate(fst.final_score)]
    f = wf.read_att("\n".join(lines))
    assert f.start == fst.start and f.num_arcs == fst.num_arcs
    for name in ("src", "dst", "ilabel", "olabel"):
        np.testing.assert_array_equal(getattr(f, name), getattr(fst, name))
    assert f.arc_score.tobytes() == fst.arc_score.tobytes()
    assert f.final_score.tobytes() == fst.final_score[:f.num_states].tobytes()


@pytest.mark.parametrize("text,kw,code,needle", [
    ("0 1 2\n", {}, -1, "line 1"),
    ("0 1 x 0\n", {}, -1, "unknown input label"),
    ("0 1 0 0\n", {"epsilon_zero": True}, -4, "epsilon"),
    ("0 1 1 1 nan\n", {}, -1, "finite"),
    ("0 1 1 1 inf\n", {}, -1, "finite"),
    ("0 1 1 1\n-2\n", {}, -1, "line 2"),
    ("\n\n", {}, -1, "no arc"),
])
def test_refusals(text, kw, code, needle):
    with pytest.raises(wf.WfstError) as e:
        wf.read_att(text, **kw)
    assert e.value.code == code and needle in str(e.value)
