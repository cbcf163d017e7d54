import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running (full-size workload)")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def fig1_fst():
    """The FST of the paper's Figure 1 / Figure 2 as a synth.Fst."""
    import synth

    g = load_golden("fig1.json")
    Q = g["num_states"]
    n = len(g["S"])
    ilab = np.empty(n, np.int32)
    for a in range(len(g["R"]) - 1):
        ilab[g["R"][a]:g["R"][a + 1]] = a
    olab = np.array([g["output_symbols"].index(o) for o in g["O"]], np.int32)
    sc = np.log(np.array(g["P"], np.float64)).astype(np.float32)
    fin = np.full(Q, -np.inf, np.float32)
    for q, p in g["final_states"].items():
        fin[int(q)] = np.float32(np.log(p))
    fst = synth.Fst(Q, len(g["input_symbols"]), g["start"], np.array(g["S"], np.int32),
                    np.array(g["T"], np.int32), ilab, olab, sc, fin, meta={"kind": "fig1"})
    toks = np.array([g["input_symbols"].index(s) for s in g["input"]], np.int32)
    batch = synth.Batch(np.array([0, toks.size], np.int64), toks)
    return g, fst, batch
