"""wfsthip: Viterbi and forward-backward over large sparse WFSTs on MI355X.

A thin ctypes binding over ``libwfsthip.so`` (C ABI in ``include/wfst.h``).
This module only marshals arguments: every step of decoding, forward,
backward and expected counts runs in the library's HIP kernels.  PyTorch is
used for device memory and streams; all device tensors are on the FST's GPU
and calls are queued on the current torch stream.

The library is required: importing works without it (so that the build can
import the package), but every call raises ``WfstError`` when the shared
library is missing instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "WfstError", "Fst", "Tape", "Graph", "viterbi", "viterbi_noalloc", "forward", "forward_scan", "backward",
    "forward_backward", "lattice_forward", "lattices_from_lists",
    "LogPartition", "log_partition", "em_update", "em_step", "read_att", "AttFst", "load_library", "layout_host", "library_path",
    "STATUS_OK", "STATUS_NO_PATH", "STATUS_BAD_TOKEN", "STATUS_BAD_INPUT",
]

HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(HERE, "libwfsthip.so")

STATUS_OK, STATUS_NO_PATH, STATUS_BAD_TOKEN, STATUS_BAD_INPUT = 0, 1, 2, 3
WFST_EINVAL, WFST_ENOMEM, WFST_EHIP, WFST_EUNSUPPORTED = -1, -2, -3, -4

_lib = None


class WfstError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"wfsthip error {code}: {msg}")
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("chunk_arcs", ctypes.c_int32), ("threads_per_sentence", ctypes.c_int32),
                ("checkpoint", ctypes.c_int32), ("state_memory", ctypes.c_int32),
                ("tape_budget_bytes", ctypes.c_int64), ("count_records", ctypes.c_int64)]


class _Info(ctypes.Structure):
    _fields_ = [("num_states", ctypes.c_int32), ("num_ilabels", ctypes.c_int32),
                ("start", ctypes.c_int32), ("chunk_arcs", ctypes.c_int32),
                ("num_arcs", ctypes.c_int64),
                ("fwd_elements", ctypes.c_int64), ("rev_elements", ctypes.c_int64),
                ("fwd_segments", ctypes.c_int64), ("rev_segments", ctypes.c_int64),
                ("fwd_slices", ctypes.c_int64), ("rev_slices", ctypes.c_int64),
                ("max_fwd_segments_per_label", ctypes.c_int32),
                ("max_rev_segments_per_label", ctypes.c_int32),
                ("max_fwd_slots_per_label", ctypes.c_int32),
                ("max_rev_slots_per_label", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64)]


class _GraphArgs(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("num_tokens", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("tokens", ctypes.c_void_p), ("arc_score", ctypes.c_void_p), ("best_score", ctypes.c_void_p),
                ("best_arcs", ctypes.c_void_p), ("best_olabels", ctypes.c_void_p), ("log_z", ctypes.c_void_p),
                ("grad_log_z", ctypes.c_void_p), ("grad_arc_score", ctypes.c_void_p),
                ("grad_final", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("threads_per_sentence", ctypes.c_int32), ("count_records", ctypes.c_int32),
                ("chunk_arcs", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("tried", ctypes.c_int32),
                ("best_ms", ctypes.c_float), ("chunks", ctypes.c_int32 * 4),
                ("ms", ((ctypes.c_float * 3) * 5) * 4)]


TUNE_CHUNK = 1
THREAD_SIZES = (64, 128, 256, 512, 1024)
COUNT_PATHS = {0: "records", -1: "grouped", -2: "fixed_point"}

EXPORTS = (
    "wfst_fst_create", "wfst_fst_set_scores", "wfst_fst_destroy", "wfst_fst_get_info", "wfst_fst_health",
    "wfst_fst_profile", "wfst_fst_profile_read", "wfst_fst_label_stats",
    "wfst_viterbi", "wfst_forward", "wfst_backward", "wfst_tape_free",
    "wfst_forward_backward", "wfst_last_error", "wfst_layout_host", "wfst_fst_autotune",
    "wfst_fst_score_version", "wfst_viterbi_noalloc", "wfst_graph_create", "wfst_graph_launch",
    "wfst_graph_destroy", "wfst_em_update", "wfst_att_parse", "wfst_att_last_error", "wfst_forward_scan",
    "wfst_lattice_forward", "wfst_fst_debug_team_spin",
)


def load_library(path: str | None = None):
    """Load libwfsthip.so (raises WfstError if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or library_path
    if not os.path.exists(p):
        raise WfstError(WFST_EUNSUPPORTED, f"{p} is missing: build it with __graft_entry__.build() "
                                           "or python -m paper_1701_03038_amd.build")
    lib = ctypes.CDLL(p)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.wfst_fst_create.argtypes = [i32, i32, i32, i64, P, P, P, P, P, P, P, P, ctypes.POINTER(P)]
    lib.wfst_fst_set_scores.argtypes = [P, P, P, P]
    lib.wfst_fst_destroy.argtypes = [P]
    lib.wfst_fst_destroy.restype = None
    lib.wfst_fst_get_info.argtypes = [P, ctypes.POINTER(_Info)]
    lib.wfst_fst_health.argtypes = [P, ctypes.POINTER(ctypes.c_uint32), i32, P]
    lib.wfst_fst_profile.argtypes = [P, i32]
    lib.wfst_fst_label_stats.argtypes = [P, P, P, P]
    lib.wfst_fst_profile_read.argtypes = [P, P, P, i32]
    lib.wfst_viterbi.argtypes = [P, i32, i64, P, P, P, P, P, P, P]
    lib.wfst_viterbi_noalloc.argtypes = [P, i32, i64, P, P, P, P, P, P, P]
    lib.wfst_forward.argtypes = [P, i32, i64, P, P, P, P, ctypes.POINTER(P), P]
    lib.wfst_backward.argtypes = [P, P, P, P, P, P]
    lib.wfst_tape_free.argtypes = [P]
    lib.wfst_tape_free.restype = None
    lib.wfst_forward_backward.argtypes = [P, i32, i64, P, P, P, P, P, P, P]
    lib.wfst_last_error.argtypes = []
    lib.wfst_last_error.restype = ctypes.c_char_p
    lib.wfst_layout_host.argtypes = [i32, i32, i64, P, P, P, i32, i32, P, P, P, P, P, P, P]
    lib.wfst_fst_autotune.argtypes = [P, i32, i64, P, P, ctypes.c_char_p, i32, ctypes.POINTER(_TuneResult), P]
    lib.wfst_fst_score_version.argtypes = [P, ctypes.POINTER(ctypes.c_uint64)]
    lib.wfst_graph_create.argtypes = [P, ctypes.POINTER(_GraphArgs), P, ctypes.POINTER(P)]
    lib.wfst_graph_launch.argtypes = [P, P]
    lib.wfst_graph_destroy.argtypes = [P]
    lib.wfst_graph_destroy.restype = None
    lib.wfst_em_update.argtypes = [P, P, ctypes.c_float, P, P, P]
    lib.wfst_forward_scan.argtypes = [P, i32, i64, P, P, P, P, P, P]
    lib.wfst_lattice_forward.argtypes = [P, i32, P, P, i64, i64, P, P, P, P, P, P, P, P]
    lib.wfst_fst_debug_team_spin.argtypes = [P, i32]
    lib.wfst_att_parse.argtypes = [ctypes.c_char_p, i64, ctypes.c_char_p, i64, ctypes.c_char_p, i64, i32, P,
                                   P, P, P, P, P, P]
    lib.wfst_att_parse.restype = ctypes.c_int
    lib.wfst_att_last_error.argtypes = []
    lib.wfst_att_last_error.restype = ctypes.c_char_p
    for name in ("wfst_fst_create", "wfst_fst_set_scores", "wfst_fst_get_info", "wfst_fst_health",
                 "wfst_fst_score_version", "wfst_fst_profile", "wfst_fst_profile_read",
                 "wfst_fst_label_stats", "wfst_viterbi", "wfst_viterbi_noalloc",
                 "wfst_forward", "wfst_backward", "wfst_forward_backward", "wfst_layout_host",
                 "wfst_fst_autotune", "wfst_graph_create", "wfst_graph_launch", "wfst_em_update",
                 "wfst_forward_scan", "wfst_lattice_forward", "wfst_fst_debug_team_spin"):
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise WfstError(rc, _lib.wfst_last_error().decode(errors="replace"))


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device=None):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def layout_host(num_states, num_ilabels, src, dst, ilabel, direction=0, chunk_arcs=16):
    """Build one sliced layout on the host (no GPU) and return its arrays."""
    lib = load_library()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    ilabel = np.ascontiguousarray(ilabel, np.int32)
    sizes = np.zeros(3, np.int64)
    args = (num_states, num_ilabels, src.shape[0], _np_ptr(src), _np_ptr(dst), _np_ptr(ilabel),
            direction, chunk_arcs)
    _check(lib.wfst_layout_host(*args, _np_ptr(sizes), None, None, None, None, None, None))
    E, S, G = (int(x) for x in sizes)
    out = dict(elem_other=np.empty(E, np.int32), elem_arc=np.empty(E, np.int32),
               slice_info=np.empty((S, 4), np.int32), seg_info=np.empty((G, 4), np.int32),
               label_slice=np.empty(num_ilabels + 1, np.int32),
               label_seg=np.empty(num_ilabels + 1, np.int32))
    _check(lib.wfst_layout_host(*args, _np_ptr(sizes), *(_np_ptr(out[k]) for k in (
        "elem_other", "elem_arc", "slice_info", "seg_info", "label_slice", "label_seg"))))
    return out


class Fst:
    """Device layouts of one WFST (library-owned; freed by close())."""

    def __init__(self, num_states, num_ilabels, start, src, dst, ilabel, arc_score, final_score,
                 olabel=None, chunk_arcs=0, threads_per_sentence=0, checkpoint=0, tape_budget_bytes=0,
                 count_records=0, state_memory=0):
        import torch
        lib = load_library()
        self.num_states, self.num_ilabels, self.start = int(num_states), int(num_ilabels), int(start)
        arrs = [np.ascontiguousarray(x, np.int32) for x in (src, dst, ilabel)]
        ol = None if olabel is None else np.ascontiguousarray(olabel, np.int32)
        sc = np.ascontiguousarray(arc_score, np.float32)
        fin = np.ascontiguousarray(final_score, np.float32)
        self.num_arcs = int(arrs[0].shape[0])
        opt = _Options(chunk_arcs, threads_per_sentence, checkpoint, state_memory, tape_budget_bytes,
                       count_records)
        self.device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        _check(lib.wfst_fst_create(self.num_states, self.num_ilabels, self.start, self.num_arcs,
                                   *(_np_ptr(a) for a in arrs), _np_ptr(ol), _np_ptr(sc), _np_ptr(fin),
                                   ctypes.byref(opt), _stream(), ctypes.byref(h)))
        self._h = h
        self.has_olabels = ol is not None

    @classmethod
    def from_synth(cls, f, **kw):
        return cls(f.num_states, f.num_ilabels, f.start, f.src, f.dst, f.ilabel, f.arc_score,
                   f.final_score, olabel=f.olabel, **kw)

    @property
    def handle(self):
        if self._h is None:
            raise WfstError(WFST_EINVAL, "FST is closed")
        return self._h

    def info(self) -> dict:
        inf = _Info()
        _check(_lib.wfst_fst_get_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    KERNELS = ("viterbi", "forward", "backward", "counts", "scores", "grad_fill", "scan", "lattice")

    def label_stats(self):
        """(arcs, forward segments, reverse segments) per input label, int32 numpy arrays."""
        out = [np.zeros(self.num_ilabels, np.int32) for _ in range(3)]
        _check(_lib.wfst_fst_label_stats(self.handle, *(_np_ptr(a) for a in out)))
        return tuple(out)

    def profile(self, enable: bool = True):
        """Bracket the main kernels of later calls with HIP events (for benchmarks)."""
        _check(_lib.wfst_fst_profile(self.handle, int(enable)))

    def profile_read(self, reset: bool = True) -> dict:
        """{kernel: (total ms, launches)} for the calls made while profiling."""
        ms = np.zeros(len(self.KERNELS), np.float64)
        n = np.zeros(len(self.KERNELS), np.int64)
        _check(_lib.wfst_fst_profile_read(self.handle, _np_ptr(ms), _np_ptr(n), int(reset)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNELS)}

    def health(self, clear: bool = False) -> int:
        """Sticky health bits of the FST's kernels (0 = healthy); synchronises the stream."""
        out = ctypes.c_uint32(0)
        _check(_lib.wfst_fst_health(self.handle, ctypes.byref(out), int(clear), _stream()))
        return int(out.value)

    def debug_team_spin(self, polls: int) -> None:
        """Testing hook: poll limit of the team sweep's barrier waits (0 = default)."""
        _check(_lib.wfst_fst_debug_team_spin(self.handle, int(polls)))

    def score_version(self) -> int:
        """Number of score updates so far (a tape only serves backward at the version it was made at)."""
        out = ctypes.c_uint64(0)
        _check(_lib.wfst_fst_score_version(self.handle, ctypes.byref(out)))
        return int(out.value)

    def set_scores(self, arc_score, final_score=None):
        """New scores from device float32 tensors (arc-id order), async on the current stream."""
        for t in (arc_score, final_score):
            if t is not None and (not t.is_cuda or t.dtype.itemsize != 4 or not t.is_contiguous()):
                raise WfstError(WFST_EINVAL, "scores must be contiguous float32 device tensors")
        _check(_lib.wfst_fst_set_scores(self.handle, _dptr(arc_score), _dptr(final_score), _stream()))

    def autotune(self, offsets, tokens, cache_path=None, tune_chunk=False):
        """Time batched Viterbi + forward + backward on this batch for every
        workgroup size per sentence, count path and (tune_chunk) chunk length,
        keep the fastest; cache_path: JSON file of earlier choices.  Returns a
        dict with the choice and the timings {(chunk, threads, count path): ms}."""
        off, tok, B, N = _batch(offsets, tokens)
        r = _TuneResult()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(_lib.wfst_fst_autotune(self.handle, B, N, _dptr(off), _dptr(tok), path,
                                      TUNE_CHUNK if tune_chunk else 0, ctypes.byref(r), _stream()))
        times = {}
        for c in range(4):
            if r.chunks[c] == 0:
                continue
            for k, nt in enumerate(THREAD_SIZES):
                for m, mode in enumerate((0, -1, -2)):
                    v = r.ms[c][k][m]
                    if v >= 0:
                        times[(int(r.chunks[c]), nt, COUNT_PATHS[mode])] = round(float(v), 4)
        return {"threads_per_sentence": r.threads_per_sentence, "count_path": COUNT_PATHS[r.count_records],
                "chunk_arcs": r.chunk_arcs, "from_cache": bool(r.from_cache), "tried": r.tried,
                "best_ms": round(float(r.best_ms), 4), "times": times}

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.wfst_fst_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch(offsets, tokens):
    """Device int32 offsets [B+1] and tokens [N] (marshalled from arrays or lists)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())

    def as_dev(x):
        if isinstance(x, torch.Tensor):
            return x.to(device=dev, dtype=torch.int32).contiguous()
        return torch.as_tensor(np.ascontiguousarray(x, np.int32), device=dev)

    off, tok = as_dev(offsets), as_dev(tokens)
    B = int(off.shape[0]) - 1
    N = int(tok.shape[0])
    return off, tok, B, N


def batch_from_sentences(sentences):
    """(offsets, tokens) int32 arrays from a list of token sequences."""
    lens = [len(s) for s in sentences]
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    tok = np.concatenate([np.asarray(s, np.int32) for s in sentences]) if sentences else np.zeros(0, np.int32)
    return off.astype(np.int32), tok.astype(np.int32)


def viterbi(fst: Fst, offsets, tokens, olabels: bool = False):
    """Best path per sentence: (best_score f32[B], best_arcs i32[N], status i32[B][, olabels i32[N]])."""
    import torch
    off, tok, B, N = _batch(offsets, tokens)
    dev = off.device
    score = torch.empty(B, dtype=torch.float32, device=dev)
    arcs = torch.empty(N, dtype=torch.int32, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    ol = torch.empty(N, dtype=torch.int32, device=dev) if olabels else None
    _check(_lib.wfst_viterbi(fst.handle, B, N, _dptr(off), _dptr(tok), _dptr(score), _dptr(arcs),
                             _dptr(ol), _dptr(status), _stream()))
    return (score, arcs, status, ol) if olabels else (score, arcs, status)


def viterbi_noalloc(fst: Fst, offsets, tokens, out=None, olabels: bool = False):
    """viterbi() through the entry point that allocates nothing (its scratch is
    one fixed array per GPU).  `out` may pass preallocated (score f32[B],
    arcs i32[N], status i32[B][, olabels i32[N]]) device tensors."""
    import torch
    off, tok, B, N = _batch(offsets, tokens)
    dev = off.device
    if out is None:
        out = (torch.empty(B, dtype=torch.float32, device=dev), torch.empty(N, dtype=torch.int32, device=dev),
               torch.empty(B, dtype=torch.int32, device=dev))
        if olabels:
            out = out + (torch.empty(N, dtype=torch.int32, device=dev),)
    score, arcs, status = out[:3]
    ol = out[3] if len(out) > 3 else None
    _check(_lib.wfst_viterbi_noalloc(fst.handle, B, N, _dptr(off), _dptr(tok), _dptr(score), _dptr(arcs),
                                     _dptr(ol), _dptr(status), _stream()))
    return out


class Tape:
    """Library-owned record of a forward pass (needed by backward)."""

    def __init__(self, fst, h, keep):
        self.fst, self._h, self._keep = fst, h, keep

    def free(self):
        if self._h is not None and _lib is not None:
            _lib.wfst_tape_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def forward(fst: Fst, offsets, tokens):
    """(log_z f32[B], status i32[B], Tape)."""
    import torch
    off, tok, B, N = _batch(offsets, tokens)
    log_z = torch.empty(B, dtype=torch.float32, device=off.device)
    status = torch.empty(B, dtype=torch.int32, device=off.device)
    h = ctypes.c_void_p()
    _check(_lib.wfst_forward(fst.handle, B, N, _dptr(off), _dptr(tok), _dptr(log_z), _dptr(status),
                             ctypes.byref(h), _stream()))
    return log_z, status, Tape(fst, h, (off, tok, status))


def backward(fst: Fst, tape: Tape, grad_log_z=None, final=False):
    """d(sum_b g_b log Z_b)/d arc_score as a float32 device tensor [num_arcs];
    with final=True also d(...)/d final_score [num_states]: (grad, grad_final)."""
    import torch
    if tape._h is None:
        raise WfstError(WFST_EINVAL, "tape already freed")
    dev = tape._keep[0].device
    grad = torch.empty(fst.num_arcs, dtype=torch.float32, device=dev)
    gfin = torch.empty(fst.num_states, dtype=torch.float32, device=dev) if final else None
    g = None
    if grad_log_z is not None:
        g = grad_log_z.to(dtype=torch.float32).contiguous()
    _check(_lib.wfst_backward(fst.handle, tape._h, _dptr(g), _dptr(grad), _dptr(gfin), _stream()))
    return (grad, gfin) if final else grad


def forward_scan(fst: Fst, offsets, tokens, alpha: bool = False):
    """log Z per sentence by the time-parallel scan (FSTs of at most 64 states):
    (log_z f32[B], status i32[B][, log alpha f32[N, num_states] after each token])."""
    import torch
    off, tok, B, N = _batch(offsets, tokens)
    log_z = torch.empty(B, dtype=torch.float32, device=off.device)
    status = torch.empty(B, dtype=torch.int32, device=off.device)
    al = torch.empty((N, fst.num_states), dtype=torch.float32, device=off.device) if alpha else None
    _check(_lib.wfst_forward_scan(fst.handle, B, N, _dptr(off), _dptr(tok), _dptr(log_z), _dptr(al),
                                  _dptr(status), _stream()))
    return (log_z, status, al) if alpha else (log_z, status)


def lattices_from_lists(lattices):
    """Concatenate lattices given as (num_nodes, [(from, to, label, weight), ...])
    (local node ids, label -1 = epsilon) into the flat arrays of
    lattice_forward: node_offsets, arc_offsets, from, to, label, weight.
    Arcs are stably sorted by target node."""
    n_off = [0]
    a_off = [0]
    cols = ([], [], [], [])
    for n, arcs in lattices:
        arcs = sorted(arcs, key=lambda e: e[1])
        for e in arcs:
            for c, x in zip(cols, e):
                c.append(x)
        n_off.append(n_off[-1] + int(n))
        a_off.append(a_off[-1] + len(arcs))
    return (np.asarray(n_off, np.int32), np.asarray(a_off, np.int32), np.asarray(cols[0], np.int32),
            np.asarray(cols[1], np.int32), np.asarray(cols[2], np.int32), np.asarray(cols[3], np.float32))


def lattice_forward(fst: Fst, node_offsets, arc_offsets, arc_from, arc_to, arc_label, arc_weight,
                    node_alpha: bool = False):
    """log Z of the FST composed with each input lattice (wfst_lattice_forward):
    (log_z f32[B], status i32[B][, log alpha f32[num_nodes, num_states] per node])."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())

    def as_dev(x, dt):
        if isinstance(x, torch.Tensor):
            return x.to(device=dev, dtype=dt).contiguous()
        return torch.as_tensor(np.ascontiguousarray(x), device=dev).to(dt)

    noff, aoff = as_dev(node_offsets, torch.int32), as_dev(arc_offsets, torch.int32)
    fr, to, lab = as_dev(arc_from, torch.int32), as_dev(arc_to, torch.int32), as_dev(arc_label, torch.int32)
    w = as_dev(arc_weight, torch.float32)
    B = int(noff.shape[0]) - 1
    if int(aoff.shape[0]) != B + 1:
        raise WfstError(WFST_EINVAL, "node_offsets and arc_offsets differ in length")
    E = int(fr.shape[0])
    if not (int(to.shape[0]) == int(lab.shape[0]) == int(w.shape[0]) == E):
        raise WfstError(WFST_EINVAL, "arc arrays differ in length")
    V = int(noff[-1].item()) if B >= 0 and noff.numel() else 0
    log_z = torch.empty(max(B, 0), dtype=torch.float32, device=dev)
    status = torch.empty(max(B, 0), dtype=torch.int32, device=dev)
    al = torch.empty((V, fst.num_states), dtype=torch.float32, device=dev) if node_alpha else None
    _check(_lib.wfst_lattice_forward(fst.handle, B, _dptr(noff), _dptr(aoff), V, E, _dptr(fr), _dptr(to),
                                     _dptr(lab), _dptr(w), _dptr(log_z), _dptr(al), _dptr(status), _stream()))
    return (log_z, status, al) if node_alpha else (log_z, status)


def forward_backward(fst: Fst, offsets, tokens, final_posteriors=False):
    """(log_z f32[B], arc_posterior f32[num_arcs] summed over the batch, status i32[B]);
    with final_posteriors=True, (log_z, arc_posterior, final_posterior f32[num_states], status)."""
    import torch
    off, tok, B, N = _batch(offsets, tokens)
    log_z = torch.empty(B, dtype=torch.float32, device=off.device)
    post = torch.empty(fst.num_arcs, dtype=torch.float32, device=off.device)
    fpost = torch.empty(fst.num_states, dtype=torch.float32, device=off.device) if final_posteriors else None
    status = torch.empty(B, dtype=torch.int32, device=off.device)
    _check(_lib.wfst_forward_backward(fst.handle, B, N, _dptr(off), _dptr(tok), _dptr(log_z),
                                      _dptr(post), _dptr(fpost), _dptr(status), _stream()))
    return (log_z, post, fpost, status) if final_posteriors else (log_z, post, status)


class AttFst:
    """Arrays of an FST read from AT&T / OpenFST text (wfst_att_parse), with
    its symbol tables (id -> symbol) when given; Fst.from_synth accepts it."""

    def __init__(self, num_states, num_ilabels, start, src, dst, ilabel, olabel, arc_score, final_score,
                 isyms=None, osyms=None):
        self.num_states, self.num_ilabels, self.start = num_states, num_ilabels, start
        self.src, self.dst, self.ilabel, self.olabel = src, dst, ilabel, olabel
        self.arc_score, self.final_score = arc_score, final_score
        self.isyms, self.osyms = isyms, osyms

    @property
    def num_arcs(self):
        return int(self.src.shape[0])

    def encode(self, words):
        """Token ids of a sequence of input symbols."""
        inv = {s: i for i, s in (self.isyms or {}).items()}
        return np.array([inv[w] for w in words], np.int32)

    def output_strings(self, best_olabels, offsets):
        """Output symbols of each sentence's best path (best_olabels from
        viterbi(..., olabels=True); -1 marks a sentence without a path)."""
        ol = np.asarray(best_olabels)
        off = np.asarray(offsets)
        out = []
        for b in range(off.shape[0] - 1):
            ids = ol[int(off[b]):int(off[b + 1])]
            if ids.size and ids[0] < 0:
                out.append(None)
            else:
                out.append([self.osyms[int(i)] if self.osyms else str(int(i)) for i in ids])
        return out


def _symbols(text):
    table = {}
    for line in text.splitlines():
        f = line.split()
        if len(f) == 2:
            table[int(f[1])] = f[0]
    return table


def read_att(fst_text: str, isyms: str | None = None, osyms: str | None = None, epsilon_zero: bool = False):
    """Parse an FST in AT&T / OpenFST text form (strings, not paths) with
    optional symbol tables; returns an AttFst."""
    lib = load_library()
    t = fst_text.encode()
    it = isyms.encode() if isyms is not None else None
    ot = osyms.encode() if osyms is not None else None
    args = (t, len(t), it, len(it) if it else 0, ot, len(ot) if ot else 0, int(epsilon_zero))
    counts = np.zeros(4, np.int64)

    def check(rc):
        if rc != 0:
            raise WfstError(rc, lib.wfst_att_last_error().decode(errors="replace"))
    check(lib.wfst_att_parse(*args, _np_ptr(counts), None, None, None, None, None, None))
    Q, M, A, start = (int(x) for x in counts)
    arr = [np.empty(A, np.int32) for _ in range(4)]
    sc, fin = np.empty(A, np.float32), np.empty(Q, np.float32)
    check(lib.wfst_att_parse(*args, _np_ptr(counts), *(_np_ptr(a) for a in arr), _np_ptr(sc), _np_ptr(fin)))
    return AttFst(Q, M, start, *arr, sc, fin, _symbols(isyms) if isyms else None,
                  _symbols(osyms) if osyms else None)


def em_update(fst: Fst, counts, cur_score, smoothing: float = 0.0, out=None):
    """EM M-step: new log scores from expected counts (device float32 tensors
    in arc-id order), normalised per source state (wfst_em_update)."""
    import torch
    for t in (counts, cur_score):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise WfstError(WFST_EINVAL, "counts and scores must be contiguous float32 device tensors")
    out = torch.empty_like(cur_score) if out is None else out
    _check(_lib.wfst_em_update(fst.handle, _dptr(counts), float(smoothing), _dptr(cur_score), _dptr(out),
                               _stream()))
    return out


def em_step(fst: Fst, arc_score, offsets, tokens, smoothing: float = 0.0):
    """One EM iteration on a batch: set the scores, forward-backward (expected
    counts), M-step.  Returns (new scores f32[A], sum of log Z over the
    sentences with a path under the given scores)."""
    import torch
    fst.set_scores(arc_score)
    log_z, counts, status = forward_backward(fst, offsets, tokens)
    ll = torch.where(status == STATUS_OK, log_z.double(), torch.zeros_like(log_z, dtype=torch.float64)).sum()
    return em_update(fst, counts, arc_score, smoothing), ll


class Graph:
    """A captured batched pass sequence (wfst_graph_create): optional score
    update, Viterbi, forward and backward with expected counts, for one batch
    shape.  The offsets/tokens (and arc_score / grad_log_z) tensors are bound
    into the graph; replay() reruns the sequence on their current contents
    and writes the output tensors held by this object."""

    def __init__(self, fst, offsets, tokens, viterbi=True, forward_backward=True, backward=True,
                 arc_score=None, grad_log_z=None, final=False, olabels=False):
        import torch
        off, tok, B, N = _batch(offsets, tokens)
        dev = off.device
        self.fst, self.offsets, self.tokens = fst, off, tok
        self.arc_score = None if arc_score is None else arc_score.detach().contiguous()
        self.grad_log_z = None if grad_log_z is None else grad_log_z.to(torch.float32).contiguous()
        self.status = torch.empty(B, dtype=torch.int32, device=dev)
        f32, i32 = torch.float32, torch.int32
        self.best_score = torch.empty(B, dtype=f32, device=dev) if viterbi else None
        self.best_arcs = torch.empty(N, dtype=i32, device=dev) if viterbi else None
        self.best_olabels = torch.empty(N, dtype=i32, device=dev) if viterbi and olabels else None
        self.log_z = torch.empty(B, dtype=f32, device=dev) if forward_backward else None
        self.grad = torch.empty(fst.num_arcs, dtype=f32, device=dev) if forward_backward and backward else None
        self.grad_final = (torch.empty(fst.num_states, dtype=f32, device=dev)
                           if forward_backward and backward and final else None)
        args = _GraphArgs(B, N, off.data_ptr(), tok.data_ptr(), *(
            (t.data_ptr() if t is not None else None) for t in (
                self.arc_score, self.best_score, self.best_arcs, self.best_olabels, self.log_z, self.grad_log_z,
                self.grad, self.grad_final, self.status)))
        side = torch.cuda.Stream(device=dev)  # capture needs a created stream
        side.wait_stream(torch.cuda.current_stream(dev))
        h = ctypes.c_void_p()
        with torch.cuda.stream(side):
            _check(_lib.wfst_graph_create(fst.handle, ctypes.byref(args), _stream(dev), ctypes.byref(h)))
        torch.cuda.current_stream(dev).wait_stream(side)
        self._h = h

    def replay(self):
        """Queue one replay on the current stream."""
        if self._h is None:
            raise WfstError(WFST_EINVAL, "graph destroyed")
        _check(_lib.wfst_graph_launch(self._h, _stream()))

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.wfst_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_log_partition():
    import torch

    class LogPartition(torch.autograd.Function):
        """log Z_b of every sentence as a function of the arc scores.

        forward(arc_score f32[A] (device), fst, offsets, tokens) -> log_z f32[B].
        The scores are written into the FST's layouts (set_scores); backward
        returns d loss / d arc_score = sum_b g_b E_b[count of each arc].
        The scores are saved for backward: when another call replaced the
        FST's scores in between (two log_partition calls on one FST before
        backward), backward writes the saved scores back and runs the forward
        pass again, so the counts always pair alpha with its own scores.
        """

        @staticmethod
        def forward(ctx, arc_score, fst, offsets, tokens, final_score=None):
            th = arc_score.detach().contiguous()
            fin = None if final_score is None else final_score.detach().contiguous()
            fst.set_scores(th, fin)
            log_z, status, tape = forward(fst, offsets, tokens)
            ctx.fst, ctx.tape = fst, tape
            ctx.version = fst.score_version()
            ctx.batch = (offsets, tokens)
            ctx.has_final = final_score is not None
            ctx.final = final_score is not None and final_score.requires_grad
            ctx.save_for_backward(arc_score, final_score)
            ctx.mark_non_differentiable(status)
            return log_z, status

        @staticmethod
        def backward(ctx, grad_log_z, _grad_status):
            arc_score, final_score = ctx.saved_tensors
            fst, tape = ctx.fst, ctx.tape
            if fst.score_version() != ctx.version:
                tape.free()
                fst.set_scores(arc_score.detach().contiguous(),
                               final_score.detach().contiguous() if ctx.has_final else None)
                _, _, tape = forward(fst, *ctx.batch)
            if ctx.final:
                g, gf = backward(fst, tape, grad_log_z, final=True)
            else:
                g, gf = backward(fst, tape, grad_log_z), None
            tape.free()
            ctx.tape = None
            return g, None, None, None, gf

    return LogPartition


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _make_log_partition()
        return getattr(_Lazy._cls, name)


LogPartition = _Lazy()


def log_partition(arc_score, fst, offsets, tokens, final_score=None):
    """Differentiable log Z per sentence (returns (log_z, status)); when
    final_score (f32[num_states], device) is given it is written into the FST
    too and receives the final-state posteriors as its gradient."""
    return LogPartition.apply(arc_score, fst, offsets, tokens, final_score)
