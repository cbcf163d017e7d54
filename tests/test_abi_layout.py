"""CPU tests of the C ABI library: it loads, exports every declared symbol, and
its host layout builder produces well-formed sliced layouts."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
import paper_1701_03038_amd as wf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "wfst.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*(wfst_\w+)\(", text, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("wfst_fst_create", "wfst_viterbi", "wfst_forward", "wfst_backward",
                 "wfst_forward_backward", "wfst_fst_set_scores", "wfst_fst_destroy",
                 "wfst_tape_free", "wfst_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(wf.library_path)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(wf.EXPORTS) >= set(_declared())


def test_error_path_without_gpu_work():
    lib = wf.load_library()
    h = ctypes.c_void_p()
    rc = lib.wfst_fst_create(0, 1, 0, 0, None, None, None, None, None, None, None, None, ctypes.byref(h))
    assert rc == wf.WFST_EINVAL
    assert b"num_states" in lib.wfst_last_error()


def _check_layout(f, direction, chunk):
    lay = wf.layout_host(f.num_states, f.num_ilabels, f.src, f.dst, f.ilabel, direction, chunk)
    key = f.dst if direction == 0 else f.src
    other = f.src if direction == 0 else f.dst
    arc = lay["elem_arc"]
    real = arc >= 0
    # every arc exactly once
    assert np.array_equal(np.sort(arc[real]), np.arange(f.num_arcs))
    assert np.all(lay["elem_other"][~real] == f.num_states)
    assert np.array_equal(lay["elem_other"][real], other[arc[real]])
    si = lay["slice_info"]
    seg = lay["seg_info"]
    for a in range(f.num_ilabels):
        s0, s1 = lay["label_slice"][a], lay["label_slice"][a + 1]
        g0, g1 = lay["label_seg"][a], lay["label_seg"][a + 1]
        n_arcs = int((f.ilabel == a).sum())
        assert (g1 - g0 == 0) == (n_arcs == 0)
        # chunks: lane l of slice s is chunk 64*(s-s0)+l; rebuild each segment's arcs in order
        chunks = []
        for s in range(s0, s1):
            base, h, w, lab = si[s]
            assert lab == a and 1 <= w <= 64 and 1 <= h <= chunk
            for lane in range(w):
                col = arc[base + np.arange(h) * w + lane]
                # padding only at the end of a chunk
                k = int((col >= 0).sum())
                assert np.all(col[:k] >= 0) and np.all(col[k:] < 0) and k >= 1
                chunks.append(col[:k])
        lens = []
        for g in range(g0, g1):
            kst, first, cnt, lab = seg[g]
            assert lab == a
            arcs = np.concatenate(chunks[first:first + cnt])
            assert np.all(np.diff(arcs) > 0), "arcs of a segment in increasing id"
            assert np.all(key[arcs] == kst) and np.all(f.ilabel[arcs] == a)
            assert np.all([len(c) == chunk for c in chunks[first:first + cnt - 1]])
            lens.append((len(arcs), kst))
        # segments ordered by decreasing length, then key; keys distinct within the label
        assert lens == sorted(lens, key=lambda x: (-x[0], x[1]))
        assert len({k for _, k in lens}) == len(lens)
        # multi-chunk segments first
        multi = [n > chunk for n, _ in lens]
        assert multi == sorted(multi, reverse=True)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("chunk", [1, 3, 16])
def test_layout_tiny(direction, chunk):
    for seed in range(20):
        f = synth.tiny_random_fst(seed, 5, 3, 30)
        _check_layout(f, direction, chunk)


@pytest.mark.parametrize("direction", [0, 1])
def test_layout_trigram_small(direction):
    f, _ = synth.config(2, n_tags=6, vocab=40, batch=1)
    _check_layout(f, direction, 16)
    _check_layout(f, direction, 4)


def test_layout_config1():
    f, _ = synth.config(1)
    _check_layout(f, 0, 16)
    _check_layout(f, 1, 8)
