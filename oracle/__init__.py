"""CPU oracle for Viterbi and forward-backward over weighted FSTs.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the GPU library.

``oracle.viterbi`` / ``oracle.forward_backward`` call the serial C oracle
(``wfst_oracle.c``, Algorithm 1 / Algorithm 2 of the paper in log-domain
scores).  ``oracle.brute`` holds the pure-Python path enumerator and a dense
matrix formulation of Eq. (1) used to pin the C oracle.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

ST_OK, ST_NO_PATH, ST_BAD_TOKEN = 0, 1, 2


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.oracle_viterbi.argtypes = [i32, i32, i32, i64, P, P, P, P, P, i32, P, P, P, P, P]
    lib.oracle_viterbi.restype = ctypes.c_int
    lib.oracle_forward_backward.argtypes = [i32, i32, i32, i64, P, P, P, P, P, i32, P, P, P, P, P, P, P]
    lib.oracle_forward_backward.restype = ctypes.c_int
    lib.oracle_fb_tables.argtypes = [i32, i32, i32, i64, P, P, P, P, P, i64, P, P, P]
    lib.oracle_fb_tables.restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _fst_args(fst):
    keep = []
    out = []
    for name, dt in (("src", np.int32), ("dst", np.int32), ("ilabel", np.int32),
                     ("arc_score", np.float32), ("final_score", np.float32)):
        arr, p = _c(getattr(fst, name), dt)
        keep.append(arr)
        out.append(p)
    return keep, out


def viterbi(fst, batch):
    """Returns (best_score f32[B], best_arcs i32[N], status i32[B])."""
    lib = _load()
    keep, fargs = _fst_args(fst)
    offs, po = _c(batch.offsets, np.int64)
    toks, pt = _c(batch.tokens, np.int32)
    B = offs.shape[0] - 1
    score = np.empty(B, np.float32)
    arcs = np.empty(max(int(offs[-1]), 0), np.int32)
    status = np.empty(B, np.int32)
    rc = lib.oracle_viterbi(fst.num_states, fst.num_ilabels, fst.start, fst.num_arcs, *fargs, B,
                            po, pt, score.ctypes.data_as(ctypes.c_void_p),
                            arcs.ctypes.data_as(ctypes.c_void_p),
                            status.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"oracle_viterbi failed: {rc}")
    del keep
    return score, arcs, status


def forward_backward(fst, batch, grad_log_z=None, arc_posteriors=True, final_posteriors=False):
    """Returns (log_z f64[B], arc_post f64[A] or None, final_post f64[Q] or None, status)."""
    lib = _load()
    keep, fargs = _fst_args(fst)
    offs, po = _c(batch.offsets, np.int64)
    toks, pt = _c(batch.tokens, np.int32)
    B = offs.shape[0] - 1
    g = None
    pg = None
    if grad_log_z is not None:
        g, pg = _c(grad_log_z, np.float64)
    log_z = np.empty(B, np.float64)
    post = np.empty(fst.num_arcs, np.float64) if arc_posteriors else None
    fpost = np.empty(fst.num_states, np.float64) if final_posteriors else None
    status = np.empty(B, np.int32)
    rc = lib.oracle_forward_backward(
        fst.num_states, fst.num_ilabels, fst.start, fst.num_arcs, *fargs, B, po, pt, pg,
        log_z.ctypes.data_as(ctypes.c_void_p),
        post.ctypes.data_as(ctypes.c_void_p) if post is not None else None,
        fpost.ctypes.data_as(ctypes.c_void_p) if fpost is not None else None,
        status.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"oracle_forward_backward failed: {rc}")
    del keep, g
    return log_z, post, fpost, status


def fb_tables(fst, tokens):
    """(log forward, log backward) tables of one sentence, each f64[n+1, Q]."""
    lib = _load()
    keep, fargs = _fst_args(fst)
    w, pw = _c(tokens, np.int32)
    n = w.shape[0]
    la = np.empty((n + 1, fst.num_states), np.float64)
    lb = np.empty((n + 1, fst.num_states), np.float64)
    rc = lib.oracle_fb_tables(fst.num_states, fst.num_ilabels, fst.start, fst.num_arcs, *fargs, n,
                              pw, la.ctypes.data_as(ctypes.c_void_p),
                              lb.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"oracle_fb_tables failed: {rc}")
    del keep
    return la, lb
