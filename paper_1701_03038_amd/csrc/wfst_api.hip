// C ABI of the library (declared in include/wfst.h): argument validation,
// device layouts, workspace and kernel launches.
//
// Memory: every FST owns its layouts plus a grow-only workspace and a pool of
// tape buffers.  A call only allocates when it needs more than any earlier
// call on the same FST (then it synchronises its stream, frees the smaller
// buffer and allocates a larger one); in steady state calls allocate nothing.
// Consequently calls on one FST must not overlap: issue them on one stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/wfst.h"
#include "kernels.h"
#include "layout.h"
#include "prims.hip"
#include "sweeps.hip"

using namespace wfst;

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_OK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return set_err(WFST_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)                       \
    do {                                \
        int rc_ = (expr);               \
        if (rc_ != WFST_OK) return rc_; \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline int grid_for(int64_t n, int nt, int cap = 65535)
{
    const int64_t g = (n + nt - 1) / nt;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// A grow-only device buffer.
struct Buf {
    void *p = nullptr;
    size_t cap = 0;
};

int ensure(Buf &b, size_t bytes, hipStream_t s)
{
    bytes = std::max<size_t>(bytes, 256);
    if (b.cap >= bytes) return WFST_OK;
    if (b.p) {
        HIP_OK(hipStreamSynchronize(s));
        HIP_OK(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    const size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return set_err(WFST_ENOMEM, "hipMalloc(" + std::to_string(want) + " bytes): " + hipGetErrorString(e));
    }
    b.cap = want;
    return WFST_OK;
}

template <class T>
int ensure_t(Buf &b, int64_t count, hipStream_t s, T **out)
{
    TRY(ensure(b, (size_t)std::max<int64_t>(count, 1) * sizeof(T), s));
    *out = reinterpret_cast<T *>(b.p);
    return WFST_OK;
}

enum WsSlot {
    W_ORDER, W_TOKOFF, W_TILES, W_COUNTERS, W_BP, W_PATH, W_BETA, W_BMAX, W_BLOG, W_LZB, W_TOKSENT,
    W_KEY0, W_KEY1, W_VAL0, W_VAL1, W_HIST, W_GRPLO, W_GRPN, W_NIP, W_ITEMBASE, W_ITEMS, W_ITEMSLOT,
    W_PARTIAL, W_SPLITE, W_SEOFF, W_VINFO, W_FROWS, W_FSUM, W_ABUF0, W_ABUF1, W_BBUF0, W_BBUF1,
    W_ILIST, W_ILOFF, W_RKEY0, W_RKEY1, W_RVAL0, W_RVAL1, W_GSCRATCH, W_FXACC, W_FXSCALE, W_EMSUM, W_SCAN0,
    W_SCAN1, W_LATNODE, W_LATSCALE, W_BSTEP, W_TVEC, W_TPMAX, W_TPZ, W_TPART, W_TBAR, W_LATFAR, W_TWORK, W_RTILE, W_NUM
};

// Global memory for the per-workgroup state of sweeps whose state vectors do
// not fit on chip: at most this many bytes (the persistent grid shrinks to fit).
constexpr int64_t kStateScratchBudget = (int64_t)16 << 30;

// Matrices of the time-parallel scan: at most this many bytes (two per token).
constexpr int64_t kScanBudgetBytes = (int64_t)32 << 30;

// small device counters kept together (one allocation)
enum Counter { C_QUEUE = 0, C_NITEMS = 1, C_SLOTS = 2, C_ITEMQ = 3, C_TOTAL = 4 /* int64 at byte 16 */,
               C_SETOTAL = 6 /* int64 at byte 24 */, C_RECS = 8 /* uint64 at byte 32 */,
               C_RTOTAL = 10 /* uint64 at byte 40 */, C_COUNT = 12 };

struct TapeBufs {
    Buf order, tok_off, alpha, a_max, a_log, log_z, tiles, total, ck_size, ck_off, blk_size, blk_base;
};

}  // namespace

struct wfst_fst {
    int device = 0;
    int32_t Q = 0, M = 0, start = 0, chunk = 16, nt = 256;
    int32_t ckpt_mode = 0;                        // wfst_options.checkpoint
    int32_t state_mem = 0;                        // wfst_options.state_memory
    bool fx_counts = false;                       // counts by fixed-point accumulation (count_records = -2)
    bool graph_mode = false;                      // capturing a graph: no host read-back, no records
    int32_t live_graphs = 0;                      // graphs made on this FST and not destroyed
    int32_t *em_order = nullptr;                  // EM: arc ids grouped by source state
    int64_t *em_start = nullptr;                  // ... group starts [Q+1]
    int32_t *em_src = nullptr;                    // ... source state of each arc
    uint64_t score_version = 0;                   // bumped by every score update
    int64_t tape_budget = (int64_t)8 << 30;       // bytes of alpha + beta tape before auto checkpointing
    int64_t A = 0;
    DevLayout fwd, rev;
    float *final_score = nullptr;
    float *final_max = nullptr;
    int32_t *olabel = nullptr;
    int2 *label_range = nullptr;  // [M] lowest and highest arc id of each label (score updates)
    bool stage_scores = false;    // score updates staged per label through LDS
    int64_t rec_cap = 0;          // record slots per backward call (0: from the batch size); grows
    int64_t rec_max = 0;          // most records a call may use before the grouped count kernel is used
    bool rec_off = false;         // grouped count kernel only
    uint32_t *health = nullptr;  // sticky health bits of the kernels (see wfst_fst_health)
    int64_t bytes = 0;
    int cu_count = 0;
    size_t max_lds = 0;
    bool coop = false;  // cooperative launches supported (team sweeps)
    int32_t team_spin = 0;  // team barrier poll limit (0: the default)
    std::vector<std::pair<void *, size_t>> allocs;  // owned device arrays and their bytes
    Buf ws[W_NUM];
    std::vector<TapeBufs *> tape_pool;
    // per-kernel timing (wfst_fst_profile): event pairs recorded around the main kernels
    std::vector<int32_t> label_arcs, label_fwd_segs, label_rev_segs;  // host copies for reporting
    bool prof = false;
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks, spare;
};

struct wfst_tape {
    const wfst_fst *fst = nullptr;
    uint64_t score_version = 0;  // the FST's scores the forward pass ran with
    int32_t B = 0;
    int64_t N = 0, total = 0;
    const int32_t *offsets = nullptr, *tokens = nullptr;
    int32_t *status = nullptr;
    TapeBufs *bufs = nullptr;
    int32_t *order = nullptr;
    int64_t *tok_off = nullptr;
    float *alpha = nullptr, *a_max = nullptr;
    double *a_log = nullptr, *log_z = nullptr;
    // checkpointed tape (ck_c > 0): alpha~ kept every ck_c steps and at the last step
    int32_t ck_c = 0, ck_K = 1;
    int64_t *ck_off = nullptr;    // [N] offset of a kept token's alpha~, -1 otherwise
    int64_t *blk_base = nullptr;  // [B] start of each sentence in a block buffer
    int64_t blk_total = 0;        // floats of one block buffer
};

struct wfst_graph {
    wfst_fst *fst = nullptr;
    wfst_graph_args args{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Buf ws[W_NUM];                   // the graph's own workspace (eager calls never resize it)
    std::vector<TapeBufs *> pool;    // ... and tape buffers
};

namespace {

template <class T>
int dev_upload(wfst_fst *f, T **dst, const T *src, int64_t count, hipStream_t s)
{
    const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    void *p = nullptr;
    HIP_OK(hipMalloc(&p, bytes));
    f->allocs.emplace_back(p, bytes);
    f->bytes += (int64_t)bytes;
    if (src && count > 0) HIP_OK(hipMemcpyAsync(p, src, (size_t)count * sizeof(T), hipMemcpyHostToDevice, s));
    *dst = reinterpret_cast<T *>(p);
    return WFST_OK;
}

int upload_layout(wfst_fst *f, const HostLayout &h, DevLayout &d, hipStream_t s)
{
    TRY(dev_upload(f, &d.other, h.other.data(), (int64_t)h.other.size(), s));
    TRY(dev_upload(f, &d.score, h.score.data(), (int64_t)h.score.size(), s));
    TRY(dev_upload(f, &d.elem_arc, h.elem_arc.data(), (int64_t)h.elem_arc.size(), s));
    TRY(dev_upload(f, &d.slice, h.slice.data(), (int64_t)h.slice.size(), s));
    TRY(dev_upload(f, &d.seg_key, h.seg_key.data(), (int64_t)h.seg_key.size(), s));
    TRY(dev_upload(f, &d.seg_chunk, h.seg_chunk.data(), (int64_t)h.seg_chunk.size(), s));
    TRY(dev_upload(f, &d.label, h.label.data(), (int64_t)h.label.size(), s));
    d.n_elem = (int64_t)h.other.size();
    d.n_slice = (int64_t)h.slice.size();
    d.n_seg = (int64_t)h.seg_key.size();
    d.max_segs = h.max_segs;
    d.max_slots = h.max_slots;
    d.max_elems = h.max_elems;
    d.max_height = h.max_height;
    d.max_slices = h.max_slices;
    return WFST_OK;
}

// Free one device array owned by the FST (nullptr-safe).
void free_owned(wfst_fst *f, void *p)
{
    if (!p) return;
    for (size_t i = 0; i < f->allocs.size(); ++i)
        if (f->allocs[i].first == p) {
            f->bytes -= (int64_t)f->allocs[i].second;
            f->allocs.erase(f->allocs.begin() + (ptrdiff_t)i);
            break;
        }
    (void)hipFree(p);
}

void free_layout(wfst_fst *f, DevLayout &d)
{
    for (void *p : {(void *)d.other, (void *)d.score, (void *)d.elem_arc, (void *)d.elem_loc, (void *)d.slice,
                    (void *)d.seg_key, (void *)d.seg_chunk, (void *)d.label})
        free_owned(f, p);
    d = DevLayout();
}

// The 2-byte label-relative arc offsets of both layouts, for score updates
// staged per label (built when the FST's labels are staged).
int build_elem_locs(wfst_fst *f, hipStream_t s)
{
    if (!f->stage_scores) return WFST_OK;
    for (DevLayout *d : {&f->fwd, &f->rev}) {
        if (d->n_elem == 0) continue;
        TRY(dev_upload<uint16_t>(f, &d->elem_loc, nullptr, d->n_elem, s));
        hipLaunchKernelGGL(build_elem_loc, dim3(grid_for(d->n_slice, 1, 65535)), dim3(256), 0, s,
                           (const SliceInfo *)d->slice, d->n_slice, (const int32_t *)d->elem_arc,
                           (const int2 *)f->label_range, d->elem_loc);
    }
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

void free_buf(Buf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

void free_fst(wfst_fst *f)
{
    if (!f) return;
    int cur = 0;
    const bool other = hipGetDevice(&cur) == hipSuccess && cur != f->device;
    if (other) (void)hipSetDevice(f->device);
    (void)hipDeviceSynchronize();
    for (auto &a : f->allocs) (void)hipFree(a.first);
    for (Buf &b : f->ws) free_buf(b);
    for (TapeBufs *t : f->tape_pool) {
        for (Buf *b : {&t->order, &t->tok_off, &t->alpha, &t->a_max, &t->a_log, &t->log_z, &t->tiles, &t->total,
                       &t->ck_size, &t->ck_off, &t->blk_size, &t->blk_base})
            free_buf(*b);
        delete t;
    }
    for (auto &m : f->marks) { (void)hipEventDestroy(m.a); (void)hipEventDestroy(m.b); }
    for (auto &m : f->spare) { (void)hipEventDestroy(m.a); (void)hipEventDestroy(m.b); }
    if (other) (void)hipSetDevice(cur);
    delete f;
}

// Brackets one main-kernel launch with timing events when profiling is on.
struct ProfScope {
    wfst_fst *f;
    hipStream_t s;
    int kind;
    wfst_fst::Mark m{};
    bool on = false;
    ProfScope(const wfst_fst *fc, hipStream_t st, int k) : f(const_cast<wfst_fst *>(fc)), s(st), kind(k)
    {
        if (!f->prof || k < 0) return;
        if (!f->spare.empty()) {
            m = f->spare.back();
            f->spare.pop_back();
        } else if (hipEventCreate(&m.a) != hipSuccess || hipEventCreate(&m.b) != hipSuccess) {
            return;
        }
        m.kind = kind;
        on = hipEventRecord(m.a, s) == hipSuccess;
    }
    ~ProfScope()
    {
        if (on && hipEventRecord(m.b, s) == hipSuccess) f->marks.push_back(m);
    }
};

// Marked segments per backward step: at most the destinations of one label.
int32_t backward_list_cap(const wfst_fst *f) { return std::max(f->fwd.max_segs, 1); }

// Bytes of each sweep's per-sentence state for this FST (LDS, or one slot of
// the global scratch when the vectors do not fit on chip).
size_t lds_viterbi(const wfst_fst *f, bool gmem)
{
    // two FP32 value vectors and their segment indices, then the chunk partials
    return (gmem ? viterbi_state_bytes<true>(f->Q) : viterbi_state_bytes<false>(f->Q)) +
           (size_t)std::max(f->fwd.max_slots, 1) * sizeof(VPart);
}
size_t lds_backward(const wfst_fst *f)
{
    // three FP32 vectors (8-byte aligned end), the segment list and its values,
    // then the 16-bit step stamps
    const size_t q1 = (size_t)f->Q + 1;
    return ((3 * q1 * sizeof(float) + 7) & ~(size_t)7) +
           (size_t)backward_list_cap(f) * (sizeof(int2) + sizeof(double)) + q1 * sizeof(uint16_t);
}
size_t lds_lse(const wfst_fst *f, const DevLayout &l)
{
    const size_t q1 = (size_t)f->Q + 1;
    return (2 * q1 + (q1 & 1)) * sizeof(float) + (size_t)std::max(l.max_segs, 1) * (sizeof(double) + sizeof(int32_t)) +
           (size_t)std::max(l.max_slots, 1) * sizeof(double);
}
size_t lds_counts(const wfst_fst *f)
{
    return (size_t)(f->Q + 1) * 2 * sizeof(CEnt) + (size_t)f->Q * sizeof(int32_t) +
           (size_t)2 * f->fwd.max_segs * sizeof(float) + (size_t)std::max(f->rev.max_slots, 1) * sizeof(int32_t);
}

template <class K>
int persistent_grid(const wfst_fst *f, K kernel, int nt, size_t lds, int64_t work, int *grid)
{
    if (lds > f->max_lds)
        return set_err(WFST_EUNSUPPORTED, "FST needs " + std::to_string(lds) +
                                              " bytes of LDS per workgroup; the device offers " +
                                              std::to_string(f->max_lds));
    if (lds > 65536)
        HIP_OK(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, lds));
    if (per_cu < 1) return set_err(WFST_EUNSUPPORTED, "kernel does not fit on a compute unit");
    *grid = (int)std::max<int64_t>(1, std::min<int64_t>(work, (int64_t)per_cu * f->cu_count));
    return WFST_OK;
}

// Where a sweep keeps its per-sentence state, and its persistent grid.
struct SweepShape {
    bool gmem = false;
    int grid = 0;
    size_t lds = 0;                      // dynamic LDS bytes
    int64_t slot = 0;                    // bytes of one workgroup's global slot (gmem)
    unsigned char *scratch = nullptr;    // grid * slot bytes (gmem)
};

// State memory of a sweep whose state takes lds_bytes on chip or slot_bytes
// in global memory: LDS unless the options ask for global memory, the state
// does not fit, or the sweep needs the wide form (need_wide).  The global
// form's grid is capped so that its slots fit kStateScratchBudget.
template <class KL, class KG>
int sweep_shape(wfst_fst *f, hipStream_t s, KL k_lds, KG k_gmem, int nt, size_t lds_bytes, size_t slot_bytes,
                bool need_wide, int64_t work, SweepShape &sh)
{
    const bool fits = lds_bytes <= f->max_lds && !need_wide;
    sh.gmem = f->state_mem >= 2 || (f->state_mem == 0 && !fits);
    if (!sh.gmem) {
        if (!fits)
            return set_err(WFST_EUNSUPPORTED, "the FST's state vectors need " + std::to_string(lds_bytes) +
                                                  " bytes of LDS per workgroup (the device offers " +
                                                  std::to_string(f->max_lds) + "); state_memory=1 forbids the "
                                                  "global-memory form");
        sh.lds = lds_bytes;
        return persistent_grid(f, k_lds, nt, lds_bytes, work, &sh.grid);
    }
    sh.slot = (int64_t)((slot_bytes + 255) / 256 * 256);
    TRY(persistent_grid(f, k_gmem, nt, 0, work, &sh.grid));
    const int64_t fit = std::max<int64_t>(1, kStateScratchBudget / sh.slot);
    sh.grid = (int)std::min<int64_t>(sh.grid, fit);
    TRY(ensure_t(f->ws[W_GSCRATCH], sh.grid * sh.slot, s, &sh.scratch));
    return WFST_OK;
}

int check_batch(const wfst_fst *f, int32_t batch, int64_t num_tokens, const void *offsets, const void *tokens)
{
    if (!f) return set_err(WFST_EINVAL, "fst is NULL");
    if (batch < 0) return set_err(WFST_EINVAL, "batch < 0");
    if (num_tokens < 0 || num_tokens >= INT32_MAX) return set_err(WFST_EINVAL, "num_tokens outside [0, 2^31-1)");
    if (batch > 0 && !offsets) return set_err(WFST_EINVAL, "offsets is NULL");
    if (num_tokens > 0 && !tokens) return set_err(WFST_EINVAL, "tokens is NULL");
    return WFST_OK;
}

// Exclusive prefix sum of src over n elements into out; the grand total is
// written to *total (device) when total != nullptr.  tiles: scratch of
// ceil(n / kScanTile) int64.
template <class OutT>
int launch_scan(hipStream_t s, ScanSource src, int64_t n, int64_t *tiles, OutT *out, int64_t *total)
{
    const int64_t ntiles = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
    if (n > 0) hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, src, n, tiles);
    else hipLaunchKernelGGL(fill_i64, dim3(1), dim3(64), 0, s, tiles, (int64_t)1, (int64_t)0);
    hipLaunchKernelGGL(scan_tiles, dim3(1), dim3(kScanThreads), 0, s, tiles, ntiles, total);
    if (n > 0) hipLaunchKernelGGL((scan_apply<OutT>), dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, src, n,
                                  (const int64_t *)tiles, out);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

inline int64_t scan_tiles_for(int64_t n) { return std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile); }

struct Plan {
    int32_t *order = nullptr;
    int64_t *tok_off = nullptr;
    int64_t total = 0;  // capacity needed for compact per-(token, segment) storage
};

// Sentence order (length buckets, longest first) and per-token offsets of the
// compact per-step storage.  The storage size is the exact total (read back,
// one synchronisation) when the cheap bound N * max_segs exceeds `bound_cap`.
int make_plan(const wfst_fst *f, hipStream_t s, int32_t B, int64_t N, const int32_t *offsets,
              const int32_t *tokens, int32_t *order, int64_t *tok_off, int64_t *tiles, int64_t *dev_total,
              int64_t bound_cap_elems, Plan &p)
{
    p.order = order;
    p.tok_off = tok_off;
    hipLaunchKernelGGL(order_by_length, dim3(1), dim3(1024), 0, s, offsets, B, order);
    ScanSource src;
    src.tokens = tokens;
    src.label = f->fwd.label;
    src.M = f->M;
    TRY(launch_scan<int64_t>(s, src, N, tiles, tok_off, dev_total));
    const int64_t bound = N * (int64_t)std::max(f->fwd.max_segs, 1);
    if (bound <= bound_cap_elems) {
        p.total = bound;
    } else if (f->graph_mode) {
        return set_err(WFST_EUNSUPPORTED, "a graph sizes its buffers by the bound tokens x largest label (" +
                                              std::to_string(bound) + " entries), which exceeds " +
                                              std::to_string(bound_cap_elems) + "; use a smaller batch");
    } else {
        int64_t t = 0;
        HIP_OK(hipMemcpyAsync(&t, dev_total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        p.total = t;
    }
    return WFST_OK;
}

constexpr int64_t kBoundCapBytes = (int64_t)2 << 30;

TapeView tape_view(const wfst_tape *t)
{
    TapeView tp;
    tp.alpha = t->alpha;
    tp.a_max = t->a_max;
    tp.a_log = t->a_log;
    tp.log_z = t->log_z;
    tp.ck_off = t->ck_c > 0 ? t->ck_off : nullptr;
    return tp;
}

// Decide whether the forward tape keeps every alpha~ or only checkpoints
// (every c = ceil(sqrt(T_max)) steps and the last step), and lay out the
// checkpointed tape and the per-sentence block buffers.  *alpha_elems gets the
// tape size.  Auto mode checkpoints when alpha + beta tapes would exceed the
// FST's budget; deciding then needs the exact sizes from the device.
int plan_checkpoints(wfst_fst *f, hipStream_t s, wfst_tape *t, int64_t *tiles, int64_t *dev_total,
                     const Plan &p, int64_t *alpha_elems)
{
    const int32_t B = t->B;
    const int64_t N = t->N;
    t->ck_c = 0;
    t->ck_K = 1;
    if (f->ckpt_mode == 2 || N == 0) return WFST_OK;
    const int64_t bytes_bound = 2 * (int64_t)sizeof(float) * p.total;
    if (f->ckpt_mode != 1 && bytes_bound <= f->tape_budget) return WFST_OK;
    if (f->graph_mode)
        return set_err(WFST_EUNSUPPORTED, "a graph keeps the whole forward tape (checkpointing plans from "
                                          "device totals); its bound exceeds the tape budget or checkpointing "
                                          "is forced");
    // exact tape size and longest sentence
    int32_t *dev_tmax = reinterpret_cast<int32_t *>(dev_total + 1);
    hipLaunchKernelGGL(batch_max_len, dim3(1), dim3(1024), 0, s, t->offsets, B, dev_tmax);
    int64_t host[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(host, dev_total, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const int64_t total = host[0];
    int32_t tmax;
    std::memcpy(&tmax, &host[1], sizeof(int32_t));
    if (f->ckpt_mode != 1 && 2 * (int64_t)sizeof(float) * total <= f->tape_budget) {
        t->total = total;
        return WFST_OK;
    }
    if (tmax <= 0) return WFST_OK;
    int32_t c = 1;
    while ((int64_t)c * c < tmax) ++c;
    t->ck_c = c;
    t->ck_K = (tmax + c - 1) / c;
    if ((int64_t)f->M * t->ck_K >= INT32_MAX)
        return set_err(WFST_EUNSUPPORTED, "labels x checkpoint blocks exceed 2^31");
    TapeBufs *tb = t->bufs;
    int64_t *size, *bsize;
    TRY(ensure_t(tb->ck_size, N, s, &size));
    TRY(ensure_t(tb->ck_off, N, s, &t->ck_off));
    TRY(ensure_t(tb->blk_size, B, s, &bsize));
    TRY(ensure_t(tb->blk_base, B, s, &t->blk_base));
    hipLaunchKernelGGL(ckpt_sizes, dim3(grid_for(B, 256)), dim3(256), 0, s, t->offsets, B, t->tokens,
                       (const LabelInfo *)f->fwd.label, f->M, c, size);
    ScanSource src;
    src.i64 = size;
    TRY(launch_scan<int64_t>(s, src, N, tiles, t->ck_off, dev_total));
    hipLaunchKernelGGL(ckpt_mark, dim3(grid_for(N, 256, 8192)), dim3(256), 0, s, (const int64_t *)size, N,
                       t->ck_off);
    hipLaunchKernelGGL(block_sizes, dim3(grid_for(B, 256)), dim3(256), 0, s, t->offsets, B, t->tokens,
                       (const LabelInfo *)f->fwd.label, f->M, (const int64_t *)t->tok_off, c, bsize);
    ScanSource bsrc;
    bsrc.i64 = bsize;
    TRY(launch_scan<int64_t>(s, bsrc, B, tiles, t->blk_base, dev_total + 1));
    HIP_OK(hipMemcpyAsync(host, dev_total, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *alpha_elems = host[0];
    t->blk_total = host[1];
    t->total = total;
    return WFST_OK;
}

template <int NT>
int launch_viterbi(const wfst_fst *fc, hipStream_t s, const BatchView &bv, int2 *bp, int32_t *path_tmp,
                   float *best_score, int32_t *best_arcs, int32_t *best_olabels, bool no_alloc = false)
{
    wfst_fst *f = const_cast<wfst_fst *>(fc);
    SweepShape sh;
    // on chip, segment indices are 16 bits (Q + 1 < 2^16); wider FSTs take the global form
    const bool wide = f->Q + 1 > 0xffff;
    if (no_alloc) {  // on-chip form only: its grid needs no memory beyond the caller's scratch
        if (wide || f->state_mem >= 2 || lds_viterbi(f, false) > f->max_lds)
            return set_err(WFST_EUNSUPPORTED, "the no-allocation Viterbi runs only the on-chip form "
                                              "(state vectors in LDS); this FST needs the global-memory form");
        sh.lds = lds_viterbi(f, false);
        TRY(persistent_grid(f, viterbi_sweep<NT, false>, NT, sh.lds, bv.B, &sh.grid));
    } else {
        TRY(sweep_shape(f, s, viterbi_sweep<NT, false>, viterbi_sweep<NT, true>, NT, lds_viterbi(f, false),
                        lds_viterbi(f, true), wide, bv.B, sh));
    }
    ProfScope prof(f, s, no_alloc ? -1 : WFST_KERNEL_VITERBI);
    if (sh.gmem)
        hipLaunchKernelGGL((viterbi_sweep<NT, true>), dim3(sh.grid), dim3(NT), 0, s, f->fwd, f->Q, f->start,
                           (const float *)f->final_score, bv, bp, path_tmp, best_score, best_arcs, best_olabels,
                           (const int32_t *)f->olabel, sh.scratch, sh.slot);
    else
        hipLaunchKernelGGL((viterbi_sweep<NT, false>), dim3(sh.grid), dim3(NT), sh.lds, s, f->fwd, f->Q, f->start,
                           (const float *)f->final_score, bv, bp, path_tmp, best_score, best_arcs, best_olabels,
                           (const int32_t *)f->olabel, nullptr, (int64_t)0);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

// The team form of the forward sweep runs when its state must be in global
// memory (auto mode) or the options ask for it, the device launches
// cooperatively, and no graph is being captured.  One team per XCD (8 on
// this device), each of all the workgroups that fit on that XCD's CUs.
constexpr int kTeamsPerDevice = 8;

bool team_forward_wanted(const wfst_fst *f)
{
    if (f->graph_mode || !f->coop) return false;
    return f->state_mem == 3 || (f->state_mem == 0 && lds_lse(f, f->fwd) > f->max_lds);
}

template <int NT>
int launch_team_forward(wfst_fst *f, hipStream_t s, const BatchView &bv, const TapeView &tp, const BlockView &bk,
                        float *log_z)
{
    int per_cu = 0;
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, team_forward_sweep<NT>, NT, 0));
    const int G = per_cu * f->cu_count / kTeamsPerDevice;
    if (G < 1) return set_err(WFST_EUNSUPPORTED, "team sweep does not fit the device");
    TeamView tv;
    tv.G = G;
    tv.n_teams = kTeamsPerDevice;
    if (f->team_spin > 0) tv.spin_limit = f->team_spin;
    tv.q1 = ((int64_t)f->Q + 1 + 63) / 64 * 64;
    unsigned int *bar = nullptr;
    TRY(ensure_t(f->ws[W_TVEC], (int64_t)tv.n_teams * 3 * tv.q1, s, &tv.vec));
    TRY(ensure_t(f->ws[W_TPMAX], (int64_t)tv.n_teams * 2 * G, s, &tv.pmax));
    TRY(ensure_t(f->ws[W_TPZ], (int64_t)tv.n_teams * 2 * G, s, &tv.pz));
    TRY(ensure_t(f->ws[W_TPART], (int64_t)tv.n_teams * std::max(f->fwd.max_slots, 1), s, &tv.part));
    TRY(ensure_t(f->ws[W_TBAR], (int64_t)tv.n_teams + 1, s, &bar));
    TRY(ensure_t(f->ws[W_TWORK], (int64_t)tv.n_teams * 2, s, &tv.work));
    tv.bar = bar;
    tv.abort = reinterpret_cast<int32_t *>(bar + tv.n_teams);
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int32_t *>(bar), (int64_t)tv.n_teams + 1, 0);
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, tv.work, (int64_t)tv.n_teams * 2, 0);
    ProfScope prof(f, s, WFST_KERNEL_FORWARD);
    DevLayout fl = f->fwd;
    int32_t Q = f->Q, start = f->start;
    const float *final_score = (const float *)f->final_score;
    BatchView bv_ = bv;
    TapeView tp_ = tp;
    BlockView bk_ = bk;
    void *args[] = {&fl, &Q, &start, &final_score, &bv_, &tp_, &bk_, &log_z, &tv};
    HIP_OK(hipLaunchCooperativeKernel((const void *)team_forward_sweep<NT>, dim3(tv.n_teams * G), dim3(NT), args, 0,
                                      s));
    return WFST_OK;
}

template <int NT>
int launch_forward(const wfst_fst *fc, hipStream_t s, const BatchView &bv, const TapeView &tp, const BlockView &bk,
                   float *log_z)
{
    wfst_fst *f = const_cast<wfst_fst *>(fc);
    if (team_forward_wanted(f)) return launch_team_forward<NT>(f, s, bv, tp, bk, log_z);
    SweepShape sh;
    const size_t bytes = lds_lse(f, f->fwd);
    TRY(sweep_shape(f, s, forward_sweep<NT, false>, forward_sweep<NT, true>, NT, bytes, bytes, false, bv.B, sh));
    ProfScope prof(f, s, WFST_KERNEL_FORWARD);
    if (sh.gmem)
        hipLaunchKernelGGL((forward_sweep<NT, true>), dim3(sh.grid), dim3(NT), 0, s, f->fwd, f->Q, f->start,
                           (const float *)f->final_score, bv, tp, bk, log_z, sh.scratch, sh.slot);
    else
        hipLaunchKernelGGL((forward_sweep<NT, false>), dim3(sh.grid), dim3(NT), sh.lds, s, f->fwd, f->Q, f->start,
                           (const float *)f->final_score, bv, tp, bk, log_z, nullptr, (int64_t)0);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

// The backward sweep keeps its state in global memory (and the counts take
// the fixed-point form) when the options say so or its state exceeds LDS.
bool backward_in_gmem(const wfst_fst *f)
{
    return f->state_mem >= 2 || (f->state_mem == 0 && lds_backward(f) > f->max_lds);
}

template <int NT>
int launch_backward(const wfst_fst *fc, hipStream_t s, const BatchView &bv, const TapeView &tp, const BlockView &bk,
                    const RecordSink &rs)
{
    wfst_fst *f = const_cast<wfst_fst *>(fc);
    SweepShape sh;
    const size_t bytes = lds_backward(f);
    TRY(sweep_shape(f, s, backward_sweep<NT, false>, backward_sweep<NT, true>, NT, bytes, bytes, false, bv.B, sh));
    if (sh.gmem && rs.key)
        return set_err(WFST_EUNSUPPORTED, "count records need the on-chip backward sweep");
    BwdStep *steps = nullptr;
    TRY(ensure_t(f->ws[W_BSTEP], std::max<int64_t>(bv.N, 1), s, &steps));
    // the sweep zero-fills the gradient only when its grid covers the device
    // (the grid is at most one workgroup per sentence); else one fill kernel
    RecordSink sink = rs;
    if (sink.fill && sh.grid < 2 * f->cu_count) {
        ProfScope prof(f, s, WFST_KERNEL_GRAD_FILL);
        hipLaunchKernelGGL(fill_f32, dim3(grid_for(sink.fill_n, 256, 8192)), dim3(256), 0, s, sink.fill, sink.fill_n,
                           0.0f);
        sink.fill = nullptr;
    }
    ProfScope prof(f, s, WFST_KERNEL_BACKWARD);
    hipLaunchKernelGGL(bwd_step_table, dim3(grid_for(bv.B, 1)), dim3(64), 0, s, f->fwd, f->rev, bv, tp, bk,
                       (int32_t)(rs.key != nullptr || rs.acc != nullptr), steps);
    if (sh.gmem)
        hipLaunchKernelGGL((backward_sweep<NT, true>), dim3(sh.grid), dim3(NT), 0, s, f->fwd, f->rev, f->Q,
                           f->start, (const float *)f->final_score, (const float *)f->final_max, bv, tp, bk,
                           backward_list_cap(f), sink, (const BwdStep *)steps, sh.scratch, sh.slot);
    else
        hipLaunchKernelGGL((backward_sweep<NT, false>), dim3(sh.grid), dim3(NT), sh.lds, s, f->fwd, f->rev, f->Q,
                           f->start, (const float *)f->final_score, (const float *)f->final_max, bv, tp, bk,
                           backward_list_cap(f), sink, (const BwdStep *)steps, nullptr, (int64_t)0);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

// Arguments of the count kernel that stay the same over its launches.
struct CountLaunch {
    const CountItem *items;
    const int32_t *n_items;
    const int32_t *list, *list_off;  // per-block item lists (checkpointing), else null
    int32_t *item_queue;
    int64_t items_bound;
    const VisitInfo *vinfo;
    float *grad, *partial;
    int32_t *item_slot, *slot_counter;
    CountCaps caps;
};

template <int NT, int CH>
int launch_counts_nt(const wfst_fst *f, hipStream_t s, const BatchView &bv, const TapeView &tp,
                     const CountLaunch &c, int32_t blk)
{
    const size_t lds = lds_counts(f);
    int grid = 0;
    TRY(persistent_grid(f, counts_kernel<NT, CH>, NT, lds, c.items_bound, &grid));
    ProfScope prof(f, s, WFST_KERNEL_COUNTS);
    hipLaunchKernelGGL((counts_kernel<NT, CH>), dim3(grid), dim3(NT), lds, s, f->fwd, f->rev, f->Q, f->start, bv,
                       tp, c.items, c.n_items, c.list, c.list_off, blk, c.item_queue, c.vinfo, c.grad, c.partial,
                       c.item_slot, c.slot_counter, c.caps);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

// Workgroup size of the count kernel: enough wavefronts for the widest label
// of the reverse layout to fit one pass (KPP slices per wavefront).
template <int CH>
int launch_counts_ch(const wfst_fst *f, hipStream_t s, const BatchView &bv, const TapeView &tp,
                     const CountLaunch &c, int32_t blk)
{
    constexpr int KPP = count_slices_per_wave(CH);
    const int waves = (f->rev.max_slices + KPP - 1) / KPP;
    if (waves > 8) return launch_counts_nt<1024, CH>(f, s, bv, tp, c, blk);
    if (waves > 4) return launch_counts_nt<512, CH>(f, s, bv, tp, c, blk);
    return launch_counts_nt<256, CH>(f, s, bv, tp, c, blk);
}

// CH = slice height bound of the reverse layout
int launch_counts(const wfst_fst *f, hipStream_t s, const BatchView &bv, const TapeView &tp, const CountLaunch &c,
                  int32_t blk)
{
    const int ch = f->rev.max_height;
    if (ch <= 4) return launch_counts_ch<4>(f, s, bv, tp, c, blk);
    if (ch <= 8) return launch_counts_ch<8>(f, s, bv, tp, c, blk);
    if (ch <= 16) return launch_counts_ch<16>(f, s, bv, tp, c, blk);
    if (ch <= 32) return launch_counts_ch<32>(f, s, bv, tp, c, blk);
    return launch_counts_ch<64>(f, s, bv, tp, c, blk);
}

#define DISPATCH_NT(rc, nt, fn, ...)                  \
    switch (nt) {                                     \
    case 64: rc = fn<64>(__VA_ARGS__); break;         \
    case 128: rc = fn<128>(__VA_ARGS__); break;       \
    case 256: rc = fn<256>(__VA_ARGS__); break;       \
    case 512: rc = fn<512>(__VA_ARGS__); break;       \
    default: rc = fn<1024>(__VA_ARGS__); break;       \
    }

BatchView make_view(const wfst_fst *f, int32_t B, int64_t N, const int32_t *offsets, const int32_t *tokens,
                    const int32_t *order, const int64_t *tok_off, int32_t *queue, int32_t *status)
{
    BatchView bv;
    bv.B = B;
    bv.M = f->M;
    bv.N = N;
    bv.offsets = offsets;
    bv.tokens = tokens;
    bv.order = order;
    bv.tok_off = tok_off;
    bv.queue = queue;
    bv.status = status;
    bv.health = f->health;
    return bv;
}

// Stable sort of token positions by label: visits[] lists positions grouped by
// label, in increasing position inside each label; skeys[] their labels.
int sort_visits(wfst_fst *f, hipStream_t s, int64_t N, const int32_t *tokens, const int32_t *offsets, int32_t B,
                int32_t c, int32_t K, int32_t **visits_out, int32_t **skeys_out, int32_t *tok_sent)
{
    int32_t *k0, *k1, *v0, *v1;
    TRY(ensure_t(f->ws[W_KEY0], N, s, &k0));
    TRY(ensure_t(f->ws[W_KEY1], N, s, &k1));
    TRY(ensure_t(f->ws[W_VAL0], N, s, &v0));
    TRY(ensure_t(f->ws[W_VAL1], N, s, &v1));
    hipLaunchKernelGGL(token_owner, dim3(grid_for(N, 256)), dim3(256), 0, s, offsets, B, N, tokens, tok_sent, k0,
                       v0, f->M, c, K);
    int bits = 1;  // keys are < M * K + 1
    while (bits < 31 && ((int64_t)1 << bits) <= (int64_t)f->M * K) ++bits;
    const int passes = (bits + 7) / 8;
    const int64_t ntiles = (N + kSortTile - 1) / kSortTile;
    int64_t *hist, *tiles;
    TRY(ensure_t(f->ws[W_HIST], 256 * ntiles, s, &hist));
    TRY(ensure_t(f->ws[W_TILES], scan_tiles_for(256 * ntiles), s, &tiles));
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(radix_hist<int32_t>, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, (const int32_t *)k0,
                           N, shift, ntiles, hist);
        ScanSource src;
        src.i64 = hist;
        TRY(launch_scan<int64_t>(s, src, 256 * ntiles, tiles, hist, nullptr));
        hipLaunchKernelGGL(radix_scatter<int32_t>, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, (const int32_t *)k0,
                           (const int32_t *)v0, N, shift, ntiles, (const int64_t *)hist, k1, v1, f->health);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    HIP_OK(hipGetLastError());
    *skeys_out = k0;
    *visits_out = v0;
    return WFST_OK;
}

// d(sum_b g_b log Z_b)/d final_score into out[Q], from the forward tape.
int final_posteriors(wfst_fst *f, const wfst_tape *tape, const float *grad_log_z, float *out, hipStream_t s)
{
    const int32_t Q = f->Q, B = tape->B;
    constexpr int32_t G = 64;
    if (B == 0) {
        hipLaunchKernelGGL(fill_f32, dim3(grid_for(Q, 256)), dim3(256), 0, s, out, (int64_t)Q, 0.0f);
        HIP_OK(hipGetLastError());
        return WFST_OK;
    }
    // sentences per block: dense rows of at most 256 MiB
    int64_t nb_max = ((int64_t)256 << 20) / ((int64_t)Q * (int64_t)sizeof(float));
    nb_max = std::max<int64_t>(G, nb_max / G * G);
    nb_max = std::min<int64_t>(nb_max, B);
    float *rows, *S;
    TRY(ensure_t(f->ws[W_FROWS], nb_max * Q, s, &rows));
    TRY(ensure_t(f->ws[W_FSUM], (nb_max + G - 1) / G * Q, s, &S));
    const TapeView tp = tape_view(tape);
    const BatchView bv = make_view(f, B, tape->N, tape->offsets, tape->tokens, tape->order, tape->tok_off, nullptr,
                                   tape->status);
    for (int64_t b0 = 0; b0 < B; b0 += nb_max) {
        const int32_t nb = (int32_t)std::min<int64_t>(nb_max, B - b0);
        const int32_t ng = (nb + G - 1) / G;
        hipLaunchKernelGGL(fill_f32, dim3(grid_for((int64_t)nb * Q, 256, 8192)), dim3(256), 0, s, rows,
                           (int64_t)nb * Q, 0.0f);
        hipLaunchKernelGGL(final_rows, dim3(grid_for(nb, 4)), dim3(256), 0, s, bv, tp, f->fwd, Q, f->start,
                           (const float *)f->final_score, grad_log_z, (int32_t)b0, nb, rows);
        hipLaunchKernelGGL(sum_row_groups, dim3(grid_for((int64_t)ng * Q, 256, 16384)), dim3(256), 0, s,
                           (const float *)rows, nb, Q, G, S);
        hipLaunchKernelGGL(sum_groups, dim3(grid_for(Q, 256)), dim3(256), 0, s, (const float *)S, ng, Q,
                           (int32_t)(b0 > 0), out);
    }
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

// Group n expected-count records by reverse-layout slot (radix sort on the
// slot part of the keys slot:position) and sum each slot's run into its arc's
// gradient as 64-bit fixed-point integers, whose sum does not depend on the
// order of the run (arcs without records keep the zero fill).
int reduce_records(wfst_fst *f, hipStream_t s, int64_t n, int64_t N, uint64_t *k0, float *v0, uint64_t *k1,
                   float *v1, float *grad, const float *grad_log_z, int32_t B)
{
    if (n == 0) return WFST_OK;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    int64_t *hist, *tiles;
    double *scale;
    TRY(ensure_t(f->ws[W_HIST], 256 * ntiles, s, &hist));
    TRY(ensure_t(f->ws[W_TILES], scan_tiles_for(256 * ntiles), s, &tiles));
    TRY(ensure_t(f->ws[W_FXSCALE], 1, s, &scale));
    hipLaunchKernelGGL(fx_scale_kernel, dim3(1), dim3(256), 0, s, grad_log_z, B, N, scale);
    // digits from the slot part (bits 32 and up) on its significant bits;
    // 2^arc_bits > every slot, so the all-ones sentinel keys sort after all records
    int arc_bits = 1;
    while (arc_bits < 32 && ((int64_t)1 << arc_bits) <= f->rev.n_elem) ++arc_bits;
    std::vector<int> shifts;
    for (int sh = 0; sh < arc_bits; sh += 8) shifts.push_back(32 + sh);
    int32_t *iv0 = reinterpret_cast<int32_t *>(v0), *iv1 = reinterpret_cast<int32_t *>(v1);
    for (int sh : shifts) {
        hipLaunchKernelGGL(radix_hist<uint64_t>, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s,
                           (const uint64_t *)k0, n, sh, ntiles, hist);
        ScanSource src;
        src.i64 = hist;
        TRY(launch_scan<int64_t>(s, src, 256 * ntiles, tiles, hist, nullptr));
        hipLaunchKernelGGL(radix_scatter<uint64_t>, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s,
                           (const uint64_t *)k0, (const int32_t *)iv0, n, sh, ntiles, (const int64_t *)hist, k1, iv1,
                           f->health);
        std::swap(k0, k1);
        std::swap(iv0, iv1);
    }
    const int64_t nrt = (n + 63) / 64;  // tiles of 64 sorted records
    RecTile *rt;
    TRY(ensure_t(f->ws[W_RTILE], nrt, s, &rt));
    hipLaunchKernelGGL(record_tiles, dim3(grid_for(nrt * 64, 256, 16384)), dim3(256), 0, s, (const uint64_t *)k0,
                       (const float *)reinterpret_cast<float *>(iv0), n, (const int32_t *)f->rev.elem_arc,
                       (const double *)scale, grad, rt, nrt);
    hipLaunchKernelGGL(record_runs, dim3(grid_for(nrt, 256, 16384)), dim3(256), 0, s, (const RecTile *)rt, nrt,
                       (const int32_t *)f->rev.elem_arc, (const double *)scale, grad);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

constexpr int64_t kRecordsMax = (int64_t)1 << 28;  // records per call before the grouped count kernel is used

}  // namespace

// Scratch of wfst_viterbi_noalloc: one array per GPU, held until the process
// ends; every call on a GPU reuses (and overwrites) that GPU's copy.  Host
// code never passes the array's name to a kernel: it is only a host-side
// stand-in; the device address comes from hipGetSymbolAddress, per device.
constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<unsigned char *> g_scratch_ptr;  // device address of `scratch`, per device (null: not looked up)

// The current device's address of `scratch` (looked up once per device, with
// that device current).
int static_scratch(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[(size_t)dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_err(WFST_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[(size_t)dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[(size_t)dev];
    return WFST_OK;
}

// Count path of later calls: 0 records (with fallbacks), -1 label-grouped
// kernel, -2 fixed-point accumulation.
void set_count_mode(wfst_fst *f, int32_t mode)
{
    f->rec_off = mode < 0;
    f->fx_counts = mode == -2;
}

int32_t count_mode(const wfst_fst *f) { return f->fx_counts ? -2 : (f->rec_off ? -1 : 0); }

// The FST's arcs in id order (label, source, destination, current score),
// read back from the forward layout: its slot (row r, lane l) of slice s
// holds chunk s*64 + l of its label, whose segment's key is the destination.
// Synchronises the stream.
int read_arcs(wfst_fst *f, hipStream_t s, std::vector<int32_t> &src, std::vector<int32_t> &dst,
              std::vector<int32_t> &ilabel, std::vector<float> &sc)
{
    const DevLayout &d = f->fwd;
    HIP_OK(hipStreamSynchronize(s));
    std::vector<int32_t> other((size_t)d.n_elem), earc((size_t)d.n_elem), seg_key((size_t)d.n_seg);
    std::vector<float> score((size_t)d.n_elem);
    std::vector<SliceInfo> slice((size_t)d.n_slice);
    std::vector<SegChunk> seg_chunk((size_t)d.n_seg);
    std::vector<LabelInfo> label((size_t)f->M);
    HIP_OK(hipMemcpy(other.data(), d.other, other.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(earc.data(), d.elem_arc, earc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(score.data(), d.score, score.size() * sizeof(float), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(seg_key.data(), d.seg_key, seg_key.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(slice.data(), d.slice, slice.size() * sizeof(SliceInfo), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(seg_chunk.data(), d.seg_chunk, seg_chunk.size() * sizeof(SegChunk), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(label.data(), d.label, label.size() * sizeof(LabelInfo), hipMemcpyDeviceToHost));
    src.assign((size_t)f->A, 0);
    dst.assign((size_t)f->A, 0);
    ilabel.assign((size_t)f->A, 0);
    sc.assign((size_t)f->A, 0.0f);
    std::vector<int32_t> chunk_seg;
    for (int32_t a = 0; a < f->M; ++a) {
        const LabelInfo &li = label[(size_t)a];
        chunk_seg.assign((size_t)std::max(li.n_slots, 1), 0);
        for (int32_t j = 0; j < li.n_multi; ++j) {
            const SegChunk &c = seg_chunk[(size_t)(li.seg_first + j)];
            for (int32_t p = 0; p < c.count; ++p) chunk_seg[(size_t)(c.first + p)] = j;
        }
        for (int32_t sl = 0; sl < li.n_slices; ++sl) {
            const SliceInfo &si = slice[(size_t)(li.slice_first + sl)];
            for (int32_t l = 0; l < si.width; ++l) {
                const int32_t c = sl * 64 + l;
                const int32_t j = c < li.n_slots ? chunk_seg[(size_t)c] : li.n_multi + (c - li.n_slots);
                const int32_t key = seg_key[(size_t)(li.seg_first + j)];
                for (int32_t r = 0; r < si.height; ++r) {
                    const int64_t e = (int64_t)si.base + (int64_t)r * si.width + l;
                    const int32_t k = earc[(size_t)e];
                    if (k < 0) continue;
                    src[(size_t)k] = other[(size_t)e];
                    dst[(size_t)k] = key;
                    ilabel[(size_t)k] = a;
                    sc[(size_t)k] = score[(size_t)e];
                }
            }
        }
    }
    return WFST_OK;
}

// Rebuild both layouts with another chunk length from the arcs read back
// from the forward layout (with their current scores), so the FST keeps no
// host copy of its arcs.  Synchronises the stream.
int rebuild_layouts(wfst_fst *f, int32_t chunk, hipStream_t s)
{
    if (chunk == f->chunk) return WFST_OK;
    if (chunk < 1 || chunk > 64) return set_err(WFST_EINVAL, "chunk_arcs must be in [1, 64]");
    if (f->live_graphs > 0)
        return set_err(WFST_EINVAL, "the FST has graphs that point at its layouts; destroy them before a rebuild");
    std::vector<int32_t> src, dst, ilabel;
    std::vector<float> sc;
    TRY(read_arcs(f, s, src, dst, ilabel, sc));
    std::string err;
    HostLayout hf, hr;
    int rc = build_layout(f->Q, f->M, f->A, src.data(), dst.data(), ilabel.data(), sc.data(), 0, chunk, hf, err);
    if (rc == WFST_OK)
        rc = build_layout(f->Q, f->M, f->A, src.data(), dst.data(), ilabel.data(), sc.data(), 1, chunk, hr, err);
    if (rc != WFST_OK) return set_err(rc, err);
    free_layout(f, f->fwd);
    free_layout(f, f->rev);
    TRY(upload_layout(f, hf, f->fwd, s));
    TRY(upload_layout(f, hr, f->rev, s));
    TRY(build_elem_locs(f, s));
    HIP_OK(hipStreamSynchronize(s));
    f->chunk = chunk;
    f->score_version += 1;  // tapes made on the old layouts are not used again
    return WFST_OK;
}

// By-source index of the arcs for the EM M-step (built once per FST): arc
// ids grouped by source state (increasing id inside a state), the group
// starts, and each arc's source.
int ensure_source_index(wfst_fst *f, hipStream_t s)
{
    if (f->em_src) return WFST_OK;
    std::vector<int32_t> src, dst, ilabel;
    std::vector<float> sc;
    TRY(read_arcs(f, s, src, dst, ilabel, sc));
    std::vector<int64_t> start((size_t)f->Q + 1, 0);
    for (int64_t k = 0; k < f->A; ++k) start[(size_t)src[(size_t)k] + 1] += 1;
    for (int32_t q = 0; q < f->Q; ++q) start[(size_t)q + 1] += start[(size_t)q];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    std::vector<int32_t> order((size_t)std::max<int64_t>(f->A, 1));
    for (int64_t k = 0; k < f->A; ++k) order[(size_t)fill[(size_t)src[(size_t)k]]++] = (int32_t)k;
    TRY(dev_upload(f, &f->em_order, order.data(), f->A, s));
    TRY(dev_upload(f, &f->em_start, start.data(), (int64_t)start.size(), s));
    TRY(dev_upload(f, &f->em_src, src.data(), f->A, s));
    HIP_OK(hipStreamSynchronize(s));
    return WFST_OK;
}

// Autotune cache: one JSON object, one entry per line,
//   "key": {"threads_per_sentence": 64, "count_records": -2, "chunk_arcs": 16, "ms": 4.5},
struct TuneEntry {
    int32_t nt = 0, mode = 0, chunk = 0;
    float ms = -1.0f;
};

std::vector<std::pair<std::string, TuneEntry>> read_tune_cache(const char *path)
{
    std::vector<std::pair<std::string, TuneEntry>> out;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        if (q1 == std::string::npos) continue;
        TuneEntry e;
        if (std::sscanf(line.c_str() + q1 + 1,
                        ": {\"threads_per_sentence\": %d, \"count_records\": %d, \"chunk_arcs\": %d, \"ms\": %f",
                        &e.nt, &e.mode, &e.chunk, &e.ms) == 4)
            out.emplace_back(line.substr(q0 + 1, q1 - q0 - 1), e);
    }
    return out;
}

int write_tune_cache(const char *path, const std::vector<std::pair<std::string, TuneEntry>> &entries)
{
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) return set_err(WFST_EINVAL, std::string("can not write the autotune cache ") + path);
        o << "{\n";
        for (size_t i = 0; i < entries.size(); ++i) {
            const TuneEntry &e = entries[i].second;
            char buf[160];
            std::snprintf(buf, sizeof(buf),
                          ": {\"threads_per_sentence\": %d, \"count_records\": %d, \"chunk_arcs\": %d, \"ms\": %.4f}",
                          e.nt, e.mode, e.chunk, e.ms);
            o << "\"" << entries[i].first << "\"" << buf << (i + 1 < entries.size() ? ",\n" : "\n");
        }
        o << "}\n";
        if (!o) return set_err(WFST_EINVAL, std::string("can not write the autotune cache ") + path);
    }
    if (std::rename(tmp.c_str(), path) != 0)
        return set_err(WFST_EINVAL, std::string("can not replace the autotune cache ") + path);
    return WFST_OK;
}

// Cache key: device architecture, FST shape and the batch's shape (sentences,
// tokens, mean arcs per token, log2 histogram of sentence lengths).
int tune_key(const wfst_fst *f, int32_t B, int64_t N, const int32_t *offsets, const int32_t *tokens,
             int32_t flags, hipStream_t s, std::string &key)
{
    std::vector<int32_t> off((size_t)B + 1), tok((size_t)std::max<int64_t>(N, 1));
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(off.data(), offsets, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (N > 0) HIP_OK(hipMemcpy(tok.data(), tokens, (size_t)N * sizeof(int32_t), hipMemcpyDeviceToHost));
    int hist[12] = {0};
    for (int32_t b = 0; b < B; ++b) {
        const int32_t T = off[(size_t)b + 1] - off[(size_t)b];
        int k = 0;
        while (k < 11 && (1 << k) <= T) ++k;
        hist[k] += 1;
    }
    double arcs = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        const int32_t a = tok[(size_t)i];
        if (a >= 0 && a < f->M) arcs += f->label_arcs[(size_t)a];
    }
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, f->device));
    std::ostringstream k;
    k << prop.gcnArchName << " Q=" << f->Q << " M=" << f->M << " A=" << f->A << " B=" << B << " N=" << N
      << " Aw=" << (int64_t)std::llround(N > 0 ? arcs / (double)N : 0.0) << " len=";
    for (int i = 0; i < 12; ++i) k << (i ? "," : "") << hist[i];
    k << " chunks=" << ((flags & WFST_TUNE_CHUNK) ? "tuned" : std::to_string(f->chunk));
    key = k.str();
    for (char &c : key)
        if (c == '"' || c == '\\') c = '_';
    return WFST_OK;
}

}  // namespace

extern "C" {

const char *wfst_last_error(void) { return g_err.c_str(); }

int wfst_layout_host(int32_t num_states, int32_t num_ilabels, int64_t num_arcs, const int32_t *src,
                     const int32_t *dst, const int32_t *ilabel, int32_t direction, int32_t chunk_arcs,
                     int64_t *sizes, int32_t *elem_other, int32_t *elem_arc, int32_t *slice_info,
                     int32_t *seg_info, int32_t *label_slice, int32_t *label_seg)
{
    try {
        if (num_states <= 0 || num_ilabels <= 0 || num_arcs < 0 || num_arcs >= INT32_MAX || !sizes)
            return set_err(WFST_EINVAL, "bad sizes");
        if (num_arcs > 0 && (!src || !dst || !ilabel)) return set_err(WFST_EINVAL, "NULL arc array");
        if (direction != 0 && direction != 1) return set_err(WFST_EINVAL, "direction must be 0 or 1");
        for (int64_t k = 0; k < num_arcs; ++k)
            if (src[k] < 0 || src[k] >= num_states || dst[k] < 0 || dst[k] >= num_states || ilabel[k] < 0 ||
                ilabel[k] >= num_ilabels)
                return set_err(WFST_EINVAL, "arc " + std::to_string(k) + " out of range");
        HostLayout h;
        std::string err;
        const int32_t L = chunk_arcs > 0 ? chunk_arcs : auto_chunk(num_states, num_ilabels, num_arcs);
        int rc = build_layout(num_states, num_ilabels, num_arcs, src, dst, ilabel, nullptr, direction, L, h, err);
        if (rc != WFST_OK) return set_err(rc, err);
        sizes[0] = (int64_t)h.other.size();
        sizes[1] = (int64_t)h.slice.size();
        sizes[2] = (int64_t)h.seg_key.size();
        if (elem_other)
            std::memcpy(elem_other, h.other.data(), h.other.size() * sizeof(int32_t));
        if (elem_arc) std::memcpy(elem_arc, h.elem_arc.data(), h.elem_arc.size() * sizeof(int32_t));
        if (slice_info)
            for (size_t x = 0; x < h.slice.size(); ++x) {
                slice_info[4 * x + 0] = h.slice[x].base;
                slice_info[4 * x + 1] = h.slice[x].height;
                slice_info[4 * x + 2] = h.slice[x].width;
                slice_info[4 * x + 3] = h.slice[x].label;
            }
        if (seg_info || label_slice || label_seg) {
            for (int32_t a = 0; a < num_ilabels; ++a) {
                const LabelInfo &li = h.label[(size_t)a];
                if (label_slice) label_slice[a] = li.slice_first;
                if (label_seg) label_seg[a] = li.seg_first;
                if (seg_info)
                    for (int32_t j = 0; j < li.n_segs; ++j) {
                        const size_t g = (size_t)li.seg_first + j;
                        seg_info[4 * g + 0] = h.seg_key[g];
                        seg_info[4 * g + 1] = h.seg_chunk[g].first;
                        seg_info[4 * g + 2] = h.seg_chunk[g].count;
                        seg_info[4 * g + 3] = a;
                    }
            }
            if (label_slice) label_slice[num_ilabels] = (int32_t)h.slice.size();
            if (label_seg) label_seg[num_ilabels] = (int32_t)h.seg_key.size();
        }
        return WFST_OK;
    } catch (const std::bad_alloc &) {
        return set_err(WFST_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return set_err(WFST_EINVAL, e.what());
    }
}

int wfst_fst_create(int32_t num_states, int32_t num_ilabels, int32_t start, int64_t num_arcs,
                    const int32_t *src, const int32_t *dst, const int32_t *ilabel, const int32_t *olabel,
                    const float *arc_score, const float *final_score, const wfst_options *options,
                    void *stream, wfst_fst **out)
{
    if (!out) return set_err(WFST_EINVAL, "out is NULL");
    *out = nullptr;
    try {
        if (num_states <= 0 || num_states >= INT32_MAX - 1) return set_err(WFST_EINVAL, "num_states out of range");
        if (num_ilabels <= 0) return set_err(WFST_EINVAL, "num_ilabels must be positive");
        if (start < 0 || start >= num_states) return set_err(WFST_EINVAL, "start out of range");
        if (num_arcs < 0 || num_arcs >= INT32_MAX) return set_err(WFST_EUNSUPPORTED, "num_arcs must be < 2^31-1");
        if (num_arcs > 0 && (!src || !dst || !ilabel || !arc_score)) return set_err(WFST_EINVAL, "NULL arc array");
        if (!final_score) return set_err(WFST_EINVAL, "final_score is NULL");
        for (int64_t k = 0; k < num_arcs; ++k) {
            if (src[k] < 0 || src[k] >= num_states || dst[k] < 0 || dst[k] >= num_states)
                return set_err(WFST_EINVAL, "arc " + std::to_string(k) + ": state out of range");
            if (ilabel[k] < 0 || ilabel[k] >= num_ilabels)
                return set_err(WFST_EINVAL, "arc " + std::to_string(k) + ": ilabel out of range");
            if (!std::isfinite(arc_score[k]))
                return set_err(WFST_EINVAL, "arc " + std::to_string(k) + ": score is not finite");
        }
        for (int32_t q = 0; q < num_states; ++q)
            if (std::isnan(final_score[q]) || final_score[q] == INFINITY)
                return set_err(WFST_EINVAL, "final_score[" + std::to_string(q) + "] is NaN or +inf");
        wfst_options opt{};
        if (options) opt = *options;
        int32_t L = opt.chunk_arcs > 0 ? opt.chunk_arcs : auto_chunk(num_states, num_ilabels, num_arcs);
        if (L > 64) return set_err(WFST_EINVAL, "chunk_arcs must be <= 64");
        int nt = opt.threads_per_sentence > 0 ? opt.threads_per_sentence : 256;
        if (nt != 64 && nt != 128 && nt != 256 && nt != 512 && nt != 1024)
            return set_err(WFST_EINVAL, "threads_per_sentence must be 64, 128, 256, 512 or 1024");
        if (opt.checkpoint < -1 || opt.checkpoint > 2) return set_err(WFST_EINVAL, "checkpoint must be -1, 0, 1 or 2");
        if (opt.tape_budget_bytes < 0) return set_err(WFST_EINVAL, "tape_budget_bytes must be >= 0");
        if (opt.count_records < -2) return set_err(WFST_EINVAL, "count_records must be >= -2");
        if (opt.state_memory < 0 || opt.state_memory > 3)
            return set_err(WFST_EINVAL, "state_memory must be 0, 1, 2 or 3");

        hipStream_t s = as_stream(stream);
        wfst_fst *f = new wfst_fst();
        f->Q = num_states;
        f->M = num_ilabels;
        f->start = start;
        f->A = num_arcs;
        f->chunk = L;
        f->nt = nt;
        f->ckpt_mode = opt.checkpoint;
        f->rec_off = opt.count_records < 0;
        f->fx_counts = opt.count_records == -2;
        f->state_mem = opt.state_memory;
        f->rec_max = opt.count_records > 0 ? opt.count_records : kRecordsMax;
        if (opt.tape_budget_bytes > 0) f->tape_budget = opt.tape_budget_bytes;
        if (hipGetDevice(&f->device) != hipSuccess) {
            delete f;
            return set_err(WFST_EHIP, "hipGetDevice failed");
        }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, f->device) != hipSuccess) {
            delete f;
            return set_err(WFST_EHIP, "hipGetDeviceProperties failed");
        }
        f->cu_count = prop.multiProcessorCount;
        f->max_lds = prop.sharedMemPerBlock;
        f->coop = prop.cooperativeLaunch != 0;
        std::string err;
        int rc;
        {
            HostLayout h;
            rc = build_layout(num_states, num_ilabels, num_arcs, src, dst, ilabel, arc_score, 0, L, h, err);
            if (rc != WFST_OK) rc = set_err(rc, err);
            if (rc == WFST_OK) {
                f->label_arcs.assign((size_t)num_ilabels, 0);
                f->label_fwd_segs.resize((size_t)num_ilabels);
                for (int32_t a = 0; a < num_ilabels; ++a) f->label_fwd_segs[(size_t)a] = h.label[(size_t)a].n_segs;
                for (int64_t k = 0; k < num_arcs; ++k) f->label_arcs[(size_t)ilabel[k]] += 1;
            }
            if (rc == WFST_OK) rc = upload_layout(f, h, f->fwd, s);
            if (rc == WFST_OK && hipStreamSynchronize(s) != hipSuccess) rc = set_err(WFST_EHIP, "upload failed");
        }
        if (rc == WFST_OK) {
            HostLayout h;
            rc = build_layout(num_states, num_ilabels, num_arcs, src, dst, ilabel, arc_score, 1, L, h, err);
            if (rc != WFST_OK) rc = set_err(rc, err);
            if (rc == WFST_OK) {
                f->label_rev_segs.resize((size_t)num_ilabels);
                for (int32_t a = 0; a < num_ilabels; ++a) f->label_rev_segs[(size_t)a] = h.label[(size_t)a].n_segs;
            }
            if (rc == WFST_OK) rc = upload_layout(f, h, f->rev, s);
            if (rc == WFST_OK && hipStreamSynchronize(s) != hipSuccess) rc = set_err(WFST_EHIP, "upload failed");
        }
        if (rc == WFST_OK) rc = dev_upload(f, &f->final_score, final_score, num_states, s);
        if (rc == WFST_OK) rc = dev_upload<float>(f, &f->final_max, nullptr, 1, s);
        if (rc == WFST_OK) rc = dev_upload<uint32_t>(f, &f->health, nullptr, 1, s);
        if (rc == WFST_OK)
            hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int32_t *>(f->health), (int64_t)1, 0);
        if (rc == WFST_OK && olabel) rc = dev_upload(f, &f->olabel, olabel, num_arcs, s);
        if (rc == WFST_OK) {
            // arc-id range per label; labels with many arcs in a compact range get
            // their score updates staged through LDS
            std::vector<int2> range((size_t)num_ilabels, make_int2(INT32_MAX, -1));
            for (int64_t k = 0; k < num_arcs; ++k) {
                int2 &r = range[(size_t)ilabel[k]];
                r.x = std::min(r.x, (int32_t)k);
                r.y = std::max(r.y, (int32_t)k);
            }
            int64_t staged_arcs = 0;
            for (int32_t a = 0; a < num_ilabels; ++a) {
                const int2 r = range[(size_t)a];
                if (r.y >= r.x && (int64_t)r.y - r.x < kScoreStage) staged_arcs += f->label_arcs[(size_t)a];
            }
            f->stage_scores = num_arcs > 0 && num_arcs / num_ilabels >= 256 && 2 * staged_arcs >= num_arcs;
            rc = dev_upload(f, &f->label_range, range.data(), num_ilabels, s);
            if (rc == WFST_OK) rc = build_elem_locs(f, s);
        }
        if (rc == WFST_OK) {
            hipLaunchKernelGGL(final_max_kernel, dim3(1), dim3(1024), 0, s, (const float *)f->final_score, f->Q,
                               f->final_max);
            if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
                rc = set_err(WFST_EHIP, "final_max kernel failed");
        }
        if (rc != WFST_OK) {
            free_fst(f);
            return rc;
        }
        *out = f;
        return WFST_OK;
    } catch (const std::bad_alloc &) {
        return set_err(WFST_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return set_err(WFST_EINVAL, e.what());
    }
}

int wfst_fst_set_scores(wfst_fst *f, const float *arc_score_dev, const float *final_score_dev, void *stream)
{
    if (!f) return set_err(WFST_EINVAL, "fst is NULL");
    hipStream_t s = as_stream(stream);
    if (arc_score_dev || final_score_dev) f->score_version += 1;
    if (arc_score_dev && f->A > 0) {
        ProfScope prof(f, s, WFST_KERNEL_SCORES);
        const int64_t quads = (f->fwd.n_elem + 3) / 4 + (f->rev.n_elem + 3) / 4;
        int64_t tiles = (quads + 255) / 256;
        tiles = (tiles + kXcds - 1) / kXcds * kXcds;
        if (tiles > INT32_MAX) return set_err(WFST_EUNSUPPORTED, "too many arc slots for one score update");
        if (f->stage_scores) {
            hipLaunchKernelGGL(scatter_scores_by_label, dim3((unsigned)f->M), dim3(kScoreThreads),
                               kScoreStage * sizeof(float), s, (const LabelInfo *)f->fwd.label,
                               (const LabelInfo *)f->rev.label, (const int2 *)f->label_range, f->fwd.score,
                               (const int32_t *)f->fwd.elem_arc, (const uint16_t *)f->fwd.elem_loc, f->rev.score,
                               (const int32_t *)f->rev.elem_arc, (const uint16_t *)f->rev.elem_loc, arc_score_dev);
        } else {
            hipLaunchKernelGGL(scatter_scores, dim3((unsigned)tiles), dim3(256), 0, s, f->fwd.score,
                               (const int32_t *)f->fwd.elem_arc, f->fwd.n_elem, f->rev.score,
                               (const int32_t *)f->rev.elem_arc, f->rev.n_elem, arc_score_dev);
        }
    }
    if (final_score_dev) {
        hipLaunchKernelGGL(copy_f32, dim3(grid_for(f->Q, 256)), dim3(256), 0, s, f->final_score, final_score_dev,
                           (int64_t)f->Q);
        hipLaunchKernelGGL(final_max_kernel, dim3(1), dim3(1024), 0, s, (const float *)f->final_score, f->Q,
                           f->final_max);
    }
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

void wfst_fst_destroy(wfst_fst *f) { free_fst(f); }

int wfst_fst_label_stats(const wfst_fst *f, int32_t *arcs, int32_t *fwd_segments, int32_t *rev_segments)
{
    if (!f) return set_err(WFST_EINVAL, "fst is NULL");
    const size_t n = (size_t)f->M * sizeof(int32_t);
    if (arcs) std::memcpy(arcs, f->label_arcs.data(), n);
    if (fwd_segments) std::memcpy(fwd_segments, f->label_fwd_segs.data(), n);
    if (rev_segments) std::memcpy(rev_segments, f->label_rev_segs.data(), n);
    return WFST_OK;
}

int wfst_fst_profile(wfst_fst *f, int32_t enable)
{
    if (!f) return set_err(WFST_EINVAL, "fst is NULL");
    f->prof = enable != 0;
    return WFST_OK;
}

int wfst_fst_profile_read(wfst_fst *f, double *ms, int64_t *launches, int32_t reset)
{
    if (!f || !ms || !launches) return set_err(WFST_EINVAL, "NULL argument");
    for (int k = 0; k < WFST_KERNEL_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &m : f->marks) {
        HIP_OK(hipEventSynchronize(m.b));
        float t = 0.0f;
        HIP_OK(hipEventElapsedTime(&t, m.a, m.b));
        if (m.kind >= 0 && m.kind < WFST_KERNEL_COUNT) {
            ms[m.kind] += t;
            launches[m.kind] += 1;
        }
    }
    if (reset) {
        for (auto &m : f->marks) f->spare.push_back(m);
        f->marks.clear();
    }
    return WFST_OK;
}

int wfst_fst_debug_team_spin(wfst_fst *f, int32_t polls)
{
    if (!f) return set_err(WFST_EINVAL, "fst is NULL");
    if (polls < 0) return set_err(WFST_EINVAL, "polls must be >= 0");
    f->team_spin = polls;
    return WFST_OK;
}

int wfst_fst_health(const wfst_fst *f, uint32_t *flags, int32_t clear, void *stream)
{
    if (!f || !flags) return set_err(WFST_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    HIP_OK(hipMemcpyAsync(flags, f->health, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (clear) {
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int32_t *>(f->health), (int64_t)1, 0);
        HIP_OK(hipGetLastError());
    }
    return WFST_OK;
}

int wfst_fst_score_version(const wfst_fst *f, uint64_t *version)
{
    if (!f || !version) return set_err(WFST_EINVAL, "NULL argument");
    *version = f->score_version;
    return WFST_OK;
}

int wfst_fst_get_info(const wfst_fst *f, wfst_fst_info *info)
{
    if (!f || !info) return set_err(WFST_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->num_states = f->Q;
    info->num_ilabels = f->M;
    info->start = f->start;
    info->chunk_arcs = f->chunk;
    info->num_arcs = f->A;
    info->fwd_elements = f->fwd.n_elem;
    info->rev_elements = f->rev.n_elem;
    info->fwd_segments = f->fwd.n_seg;
    info->rev_segments = f->rev.n_seg;
    info->fwd_slices = f->fwd.n_slice;
    info->rev_slices = f->rev.n_slice;
    info->max_fwd_segments_per_label = f->fwd.max_segs;
    info->max_rev_segments_per_label = f->rev.max_segs;
    info->max_fwd_slots_per_label = f->fwd.max_slots;
    info->max_rev_slots_per_label = f->rev.max_slots;
    info->device_bytes = f->bytes;
    return WFST_OK;
}

int wfst_viterbi(const wfst_fst *fc, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                 const int32_t *tokens, float *best_score, int32_t *best_arcs, int32_t *best_olabels,
                 int32_t *status, void *stream)
{
    TRY(check_batch(fc, batch, num_tokens, offsets, tokens));
    if (batch == 0) return WFST_OK;
    if (!best_score || !status || (num_tokens > 0 && !best_arcs)) return set_err(WFST_EINVAL, "NULL output");
    if (best_olabels && !fc->olabel) return set_err(WFST_EINVAL, "FST was created without olabels");
    wfst_fst *f = const_cast<wfst_fst *>(fc);  // the workspace is mutable state of the FST
    hipStream_t s = as_stream(stream);
    const int64_t N = num_tokens;
    int32_t *order, *counters, *path_tmp;
    int64_t *tok_off, *tiles;
    TRY(ensure_t(f->ws[W_ORDER], batch, s, &order));
    TRY(ensure_t(f->ws[W_TOKOFF], N, s, &tok_off));
    TRY(ensure_t(f->ws[W_TILES], scan_tiles_for(N), s, &tiles));
    TRY(ensure_t(f->ws[W_COUNTERS], C_COUNT, s, &counters));
    TRY(ensure_t(f->ws[W_PATH], N, s, &path_tmp));
    int64_t *dev_total = reinterpret_cast<int64_t *>(counters + C_TOTAL);
    Plan p;
    TRY(make_plan(f, s, batch, N, offsets, tokens, order, tok_off, tiles, dev_total, kBoundCapBytes / 8, p));
    int2 *bp;
    TRY(ensure_t(f->ws[W_BP], p.total, s, &bp));
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters + C_QUEUE, (int64_t)1, 0);
    const BatchView bv = make_view(f, batch, N, offsets, tokens, order, tok_off, counters + C_QUEUE, status);
    int rc;
    DISPATCH_NT(rc, f->nt, launch_viterbi, f, s, bv, bp, path_tmp, best_score, best_arcs, best_olabels)
    return rc;
}

int wfst_viterbi_noalloc(const wfst_fst *fc, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                         const int32_t *tokens, float *best_score, int32_t *best_arcs, int32_t *best_olabels,
                         int32_t *status, void *stream)
{
    TRY(check_batch(fc, batch, num_tokens, offsets, tokens));
    if (batch == 0) return WFST_OK;
    if (!best_score || !status || (num_tokens > 0 && !best_arcs)) return set_err(WFST_EINVAL, "NULL output");
    if (best_olabels && !fc->olabel) return set_err(WFST_EINVAL, "FST was created without olabels");
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != fc->device) return set_err(WFST_EINVAL, "the FST's device must be the current device");
    unsigned char *base = nullptr;
    TRY(static_scratch(dev, &base));
    hipStream_t s = as_stream(stream);
    const int64_t N = num_tokens;
    // carve the scratch: counters | order | tok_off | scan tiles | path | back-pointers (bound: N x max segments)
    const int64_t segs = std::max(fc->fwd.max_segs, 1);
    size_t at = 0;
    auto carve = [&](size_t bytes) {
        const size_t here = at;
        at += (bytes + 255) / 256 * 256;
        return here;
    };
    const size_t o_cnt = carve(C_COUNT * sizeof(int32_t));
    const size_t o_order = carve((size_t)batch * sizeof(int32_t));
    const size_t o_tok = carve((size_t)std::max<int64_t>(N, 1) * sizeof(int64_t));
    const size_t o_tiles = carve((size_t)scan_tiles_for(N) * sizeof(int64_t));
    const size_t o_path = carve((size_t)std::max<int64_t>(N, 1) * sizeof(int32_t));
    if ((double)N * (double)segs * sizeof(int2) > (double)kStaticScratchBytes)
        return set_err(WFST_EUNSUPPORTED, "batch too large for the no-allocation Viterbi: " + std::to_string(N) +
                                              " tokens x " + std::to_string(segs) +
                                              " segments per label need more than its " +
                                              std::to_string(kStaticScratchBytes >> 20) + " MiB of scratch");
    const size_t o_bp = carve((size_t)N * (size_t)segs * sizeof(int2));
    if (at > kStaticScratchBytes)
        return set_err(WFST_EUNSUPPORTED, "batch too large for the no-allocation Viterbi: needs " +
                                              std::to_string(at) + " bytes of its " +
                                              std::to_string(kStaticScratchBytes) + "-byte scratch");
    int32_t *counters = reinterpret_cast<int32_t *>(base + o_cnt);
    int32_t *order = reinterpret_cast<int32_t *>(base + o_order);
    int64_t *tok_off = reinterpret_cast<int64_t *>(base + o_tok);
    int64_t *tiles = reinterpret_cast<int64_t *>(base + o_tiles);
    int32_t *path_tmp = reinterpret_cast<int32_t *>(base + o_path);
    int2 *bp = reinterpret_cast<int2 *>(base + o_bp);
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters, (int64_t)C_COUNT, 0);
    Plan p;
    // the bound N x max segments always fits here, so the plan reads nothing back
    TRY(make_plan(fc, s, batch, N, offsets, tokens, order, tok_off, tiles,
                  reinterpret_cast<int64_t *>(counters + C_TOTAL), INT64_MAX, p));
    const BatchView bv = make_view(fc, batch, N, offsets, tokens, order, tok_off, counters + C_QUEUE, status);
    int rc;
    DISPATCH_NT(rc, fc->nt, launch_viterbi, fc, s, bv, bp, path_tmp, best_score, best_arcs, best_olabels, true)
    return rc;
}

int wfst_forward(const wfst_fst *fc, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                 const int32_t *tokens, float *log_z, int32_t *status, wfst_tape **tape_out, void *stream)
{
    TRY(check_batch(fc, batch, num_tokens, offsets, tokens));
    if (!tape_out) return set_err(WFST_EINVAL, "tape_out is NULL");
    *tape_out = nullptr;
    if (batch > 0 && (!log_z || !status)) return set_err(WFST_EINVAL, "NULL output");
    wfst_fst *f = const_cast<wfst_fst *>(fc);
    hipStream_t s = as_stream(stream);
    const int64_t N = num_tokens;
    TapeBufs *tb;
    if (!f->tape_pool.empty()) {
        tb = f->tape_pool.back();
        f->tape_pool.pop_back();
    } else {
        tb = new TapeBufs();
    }
    wfst_tape *t = new wfst_tape();
    t->fst = f;
    t->score_version = f->score_version;
    t->B = batch;
    t->N = N;
    t->offsets = offsets;
    t->tokens = tokens;
    t->status = status;
    t->bufs = tb;
    int rc = WFST_OK;
    if (batch > 0) {
        int32_t *counters;
        int64_t *tiles, *dev_total;
        rc = ensure_t(tb->order, batch, s, &t->order);
        if (rc == WFST_OK) rc = ensure_t(tb->tok_off, N, s, &t->tok_off);
        if (rc == WFST_OK) rc = ensure_t(tb->tiles, scan_tiles_for(std::max<int64_t>(N, batch)), s, &tiles);
        if (rc == WFST_OK) rc = ensure_t(tb->total, 2, s, &dev_total);
        if (rc == WFST_OK) rc = ensure_t(f->ws[W_COUNTERS], C_COUNT, s, &counters);
        Plan p;
        if (rc == WFST_OK)
            rc = make_plan(f, s, batch, N, offsets, tokens, t->order, t->tok_off, tiles, dev_total,
                           kBoundCapBytes / 4, p);
        int64_t alpha_elems = p.total;
        if (rc == WFST_OK) {
            t->total = p.total;
            rc = plan_checkpoints(f, s, t, tiles, dev_total, p, &alpha_elems);
        }
        if (rc == WFST_OK) rc = ensure_t(tb->alpha, std::max<int64_t>(alpha_elems, 1), s, &t->alpha);
        if (rc == WFST_OK) rc = ensure_t(tb->a_max, N, s, &t->a_max);
        if (rc == WFST_OK) rc = ensure_t(tb->a_log, N, s, &t->a_log);
        if (rc == WFST_OK) rc = ensure_t(tb->log_z, batch, s, &t->log_z);
        if (rc == WFST_OK) {
            hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters + C_QUEUE, (int64_t)1, 0);
            const BatchView bv =
                make_view(f, batch, N, offsets, tokens, t->order, t->tok_off, counters + C_QUEUE, status);
            const TapeView tp = tape_view(t);
            DISPATCH_NT(rc, f->nt, launch_forward, f, s, bv, tp, BlockView(), log_z)
        }
    }
    if (rc != WFST_OK) {
        wfst_tape_free(t);
        return rc;
    }
    *tape_out = t;
    return WFST_OK;
}

void wfst_tape_free(wfst_tape *t)
{
    if (!t) return;
    if (t->fst && t->bufs) const_cast<wfst_fst *>(t->fst)->tape_pool.push_back(t->bufs);
    delete t;
}

int wfst_backward(const wfst_fst *fc, const wfst_tape *tape, const float *grad_log_z, float *grad_arc_score,
                  float *grad_final, void *stream)
{
    if (!fc || !tape) return set_err(WFST_EINVAL, "NULL fst or tape");
    if (tape->fst != fc) return set_err(WFST_EINVAL, "tape belongs to another FST");
    if (!grad_arc_score && fc->A > 0) return set_err(WFST_EINVAL, "grad_arc_score is NULL");
    if (tape->score_version != fc->score_version)
        return set_err(WFST_EINVAL, "the FST's scores changed after the forward pass of this tape "
                                    "(wfst_fst_set_scores); run the forward pass again");
    wfst_fst *f = const_cast<wfst_fst *>(fc);
    hipStream_t s = as_stream(stream);
    if (grad_final) TRY(final_posteriors(f, tape, grad_log_z, grad_final, s));
    const int32_t B = tape->B;
    const int64_t N = tape->N;
    // expected counts by fixed-point accumulation in the backward sweep: asked
    // for, or forced by a backward state too large for LDS
    // (a graph takes fixed-point counts where the records would need a read-back)
    const bool fx = f->A > 0 && B > 0 && N > 0 &&
                    (f->fx_counts || backward_in_gmem(f) || (f->graph_mode && !f->rec_off));
    // on the record path the backward sweep zero-fills the gradient itself
    // (bandwidth it leaves unused); else one fill kernel first
    const bool fill_in_sweep = f->A > 0 && !fx && !f->rec_off && B > 0 && N > 0 &&
                               ((uintptr_t)grad_arc_score & 15) == 0;
    if (f->A > 0 && !fx && !fill_in_sweep) {
        ProfScope prof(f, s, WFST_KERNEL_GRAD_FILL);
        hipLaunchKernelGGL(fill_f32, dim3(grid_for(f->A, 256, 8192)), dim3(256), 0, s, grad_arc_score, f->A, 0.0f);
    }
    if (B == 0 || N == 0) {
        HIP_OK(hipGetLastError());
        return WFST_OK;
    }
    TapeView tp = tape_view(tape);
    const int32_t K = tape->ck_c > 0 ? tape->ck_K : 1;
    BlockView bk;  // c = 0: the whole tape is resident
    int32_t *counters;
    if (tape->ck_c > 0) {
        bk.c = tape->ck_c;
        bk.base = tape->blk_base;
        const int64_t nb = std::max<int64_t>(tape->blk_total, 1);
        TRY(ensure_t(f->ws[W_ABUF0], nb, s, &bk.abuf[0]));
        TRY(ensure_t(f->ws[W_ABUF1], nb, s, &bk.abuf[1]));
        TRY(ensure_t(f->ws[W_BBUF0], nb, s, &bk.bbuf[0]));
        TRY(ensure_t(f->ws[W_BBUF1], nb, s, &bk.bbuf[1]));
    } else {
        TRY(ensure_t(f->ws[W_BETA], tape->total, s, &tp.beta));
    }
    TRY(ensure_t(f->ws[W_BMAX], N, s, &tp.b_max));
    TRY(ensure_t(f->ws[W_BLOG], N, s, &tp.b_log));
    TRY(ensure_t(f->ws[W_LZB], B, s, &tp.log_z_bwd));
    TRY(ensure_t(f->ws[W_COUNTERS], C_COUNT, s, &counters));
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters, (int64_t)C_COUNT, 0);
    const BatchView bv = make_view(f, B, N, tape->offsets, tape->tokens, tape->order, tape->tok_off,
                                   counters + C_QUEUE, tape->status);
    int rc;
    // Expected counts as records of the backward pass (sorted and summed per
    // arc) when there are at most rec_max of them; otherwise the grouped count
    // kernel below.  The choice depends only on the number of records; when
    // their slots (records plus unused chunk tails) overflow the buffer, the
    // buffer grows and the pass runs again.
    auto backward_pass = [&](const RecordSink &sink) -> int {
        int r = WFST_OK;
        if (bk.c == 0) {
            DISPATCH_NT(r, f->nt, launch_backward, f, s, bv, tp, bk, sink)
            return r;
        }
        for (int32_t k = K - 1; k >= 0; --k) {  // blocks from the end: recompute alpha~, then beta
            bk.k = k;
            hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters + C_QUEUE, (int64_t)1, 0);
            DISPATCH_NT(r, f->nt, launch_forward, f, s, bv, tp, bk, nullptr)
            if (r != WFST_OK) return r;
            hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters + C_QUEUE, (int64_t)1, 0);
            RecordSink sk = sink;
            if (k != K - 1) sk.fill = nullptr;  // the first launch zero-fills the gradient
            DISPATCH_NT(r, f->nt, launch_backward, f, s, bv, tp, bk, sk)
            if (r != WFST_OK) return r;
        }
        return WFST_OK;
    };
    // Fixed-point counts: each posterior is added to its arc's 64-bit integer
    // accumulator (indexed by the arc's reverse-layout slot) during the
    // backward sweep; one conversion pass writes the gradient.  Integer sums do
    // not depend on the order of the additions.
    auto fixed_point_counts = [&]() -> int {
        unsigned long long *acc;
        double *scale;
        const int64_t n_slots = f->rev.n_elem;
        TRY(ensure_t(f->ws[W_FXACC], n_slots, s, &acc));
        TRY(ensure_t(f->ws[W_FXSCALE], 1, s, &scale));
        {
            ProfScope prof(f, s, WFST_KERNEL_GRAD_FILL);
            hipLaunchKernelGGL(fill_i64, dim3(grid_for(n_slots, 256, 8192)), dim3(256), 0, s,
                               reinterpret_cast<int64_t *>(acc), n_slots, (int64_t)0);
        }
        hipLaunchKernelGGL(fx_scale_kernel, dim3(1), dim3(256), 0, s, grad_log_z, B, N, scale);
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters, (int64_t)C_COUNT, 0);
        RecordSink rs;
        rs.acc = acc;
        rs.fx_scale = scale;
        rs.grad_log_z = grad_log_z;
        TRY(backward_pass(rs));
        {
            ProfScope prof(f, s, WFST_KERNEL_COUNTS);
            hipLaunchKernelGGL(fx_to_grad, dim3(grid_for(n_slots, 256, 8192)), dim3(256), 0, s,
                               (const unsigned long long *)acc, (const int32_t *)f->rev.elem_arc, n_slots,
                               (const double *)scale, grad_arc_score);
        }
        HIP_OK(hipGetLastError());
        return WFST_OK;
    };
    if (fx) return fixed_point_counts();
    bool beta_done = false;  // the beta tape of the resident-tape pass is written
    if (f->A > 0 && !f->rec_off) {
        RecordSink rs;
        rs.count = reinterpret_cast<unsigned long long *>(counters + C_RECS);
        rs.total = reinterpret_cast<unsigned long long *>(counters + C_RTOTAL);
        rs.grad_log_z = grad_log_z;
        if (fill_in_sweep) {
            rs.fill = grad_arc_score;
            rs.fill_n = f->A;
        }
        int64_t cap = std::min(kRecordsMax, f->rec_cap > 0 ? f->rec_cap : 16 * N + 4096);
        for (int attempt = 0; attempt < 2; ++attempt) {
            TRY(ensure_t(f->ws[W_RKEY0], cap, s, &rs.key));
            TRY(ensure_t(f->ws[W_RVAL0], cap, s, &rs.val));
            rs.cap = cap;
            if (attempt > 0) hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters, (int64_t)C_COUNT, 0);
            TRY(backward_pass(rs));
            beta_done = true;
            unsigned long long got[2] = {0, 0};  // slots, records
            HIP_OK(hipMemcpyAsync(got, rs.count, sizeof(got), hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            if ((int64_t)got[1] > f->rec_max) {  // too many records: grouped count kernel, or fixed point
                if (lds_counts(f) > f->max_lds) return fixed_point_counts();
                break;
            }
            if ((int64_t)got[0] <= cap) {
                ProfScope prof(f, s, WFST_KERNEL_COUNTS);
                uint64_t *k1;
                float *v1;
                TRY(ensure_t(f->ws[W_RKEY1], std::max<int64_t>((int64_t)got[0], 1), s, &k1));
                TRY(ensure_t(f->ws[W_RVAL1], std::max<int64_t>((int64_t)got[0], 1), s, &v1));
                return reduce_records(f, s, (int64_t)got[0], N, rs.key, rs.val, k1, v1, grad_arc_score, grad_log_z, B);
            }
            // slots overflowed: grow to a bound no schedule can pass and run again.  A
            // chunk holds kRecChunk slots and is left with a tail under kRecStage;
            // there are at most records / kRecChunk chunks plus one per workgroup
            // and launch.
            const int64_t launches = bk.c > 0 ? K : 1;
            cap = 3 * (int64_t)got[1] + (int64_t)kRecStage * B * launches + 4096;
            f->rec_cap = std::max<int64_t>(f->rec_cap, std::min(kRecordsMax, (int64_t)got[0] + (int64_t)got[0] / 4));
        }
        // the grouped count kernel needs the beta tape of a pass without records
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters, (int64_t)C_COUNT, 0);
    }
    if (bk.c == 0 && !beta_done) TRY(backward_pass(RecordSink()));
    RecordSink no_records;

    // group the visits (token positions) by (input label, checkpoint block), stable in position
    const int32_t V = 64;
    const int32_t MK = f->M * K;
    int32_t *tok_sent, *visits, *skeys, *grp_lo, *grp_n, *nip, *item_base, *item_slot;
    TRY(ensure_t(f->ws[W_TOKSENT], N, s, &tok_sent));
    TRY(sort_visits(f, s, N, tape->tokens, tape->offsets, B, tape->ck_c, K, &visits, &skeys, tok_sent));
    TRY(ensure_t(f->ws[W_GRPLO], MK, s, &grp_lo));
    TRY(ensure_t(f->ws[W_GRPN], MK, s, &grp_n));
    TRY(ensure_t(f->ws[W_NIP], MK, s, &nip));
    TRY(ensure_t(f->ws[W_ITEMBASE], MK, s, &item_base));
    const int64_t items_bound = N / V + std::min<int64_t>(MK, N) + 1;
    CountItem *items;
    TRY(ensure_t(f->ws[W_ITEMS], items_bound, s, &items));
    TRY(ensure_t(f->ws[W_ITEMSLOT], items_bound, s, &item_slot));
    const int64_t split_bound = 2 * (N / V) + 2;
    float *partial;
    TRY(ensure_t(f->ws[W_PARTIAL], split_bound * (int64_t)std::max(f->rev.max_elems, 1), s, &partial));
    int64_t *tiles;
    TRY(ensure_t(f->ws[W_TILES], scan_tiles_for(std::max<int64_t>(MK, 256 * ((N + kSortTile - 1) / kSortTile))),
                 s, &tiles));
    hipLaunchKernelGGL(label_groups, dim3(grid_for(MK, 256)), dim3(256), 0, s, (const int32_t *)skeys, N, MK, V,
                       grp_lo, grp_n, nip);
    ScanSource src;
    src.i32 = nip;
    TRY(launch_scan<int32_t>(s, src, MK, tiles, item_base, nullptr));
    hipLaunchKernelGGL(label_items, dim3(grid_for(MK, 256)), dim3(256), 0, s, (const int32_t *)grp_lo,
                       (const int32_t *)grp_n, (const int32_t *)nip, (const int32_t *)item_base, MK, K, V, items,
                       counters + C_NITEMS, (int32_t)items_bound, f->health);
    CountCaps caps;
    caps.items_cap = (int32_t)items_bound;
    caps.slot_cap = (int32_t)split_bound;
    caps.V = V;
    int32_t *list = nullptr, *list_off = nullptr;
    if (bk.c > 0) {
        TRY(ensure_t(f->ws[W_ILIST], items_bound, s, &list));
        TRY(ensure_t(f->ws[W_ILOFF], K + 1, s, &list_off));
        hipLaunchKernelGGL(items_by_block, dim3(1), dim3(1024), 2 * K * sizeof(int32_t), s, (const CountItem *)items,
                           (const int32_t *)(counters + C_NITEMS), K, (int32_t)items_bound, list, list_off,
                           f->health);
    }
    VisitInfo *vinfo;
    TRY(ensure_t(f->ws[W_VINFO], N, s, &vinfo));
    // per-visit records read the backward normalisers: built after the beta sweep (of each block)
    auto build_visits = [&]() {
        hipLaunchKernelGGL(visit_table, dim3(grid_for(N, 256)), dim3(256), 0, s, bv, tp, bk,
                           (const int32_t *)visits, (const int32_t *)tok_sent, grad_log_z, vinfo);
    };
    int32_t *split_e;
    int64_t *se_off;
    TRY(ensure_t(f->ws[W_SPLITE], MK, s, &split_e));
    TRY(ensure_t(f->ws[W_SEOFF], MK, s, &se_off));
    int64_t *se_total = reinterpret_cast<int64_t *>(counters + C_SETOTAL);
    const CountLaunch cl{items, counters + C_NITEMS, list, list_off, counters + C_ITEMQ, items_bound, vinfo,
                         grad_arc_score, partial, item_slot, counters + C_SLOTS, caps};
    // one block of steps (all of them without checkpointing): counts, then the
    // groups split over several items
    auto counts_block = [&](int32_t blk) -> int {
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters + C_ITEMQ, (int64_t)1, 0);
        TRY(launch_counts(f, s, bv, tp, cl, blk));
        hipLaunchKernelGGL(split_group_elems, dim3(grid_for(MK, 256)), dim3(256), 0, s,
                           (const LabelInfo *)f->rev.label, (const int32_t *)nip, MK, K, bk.c > 0 ? blk : -1,
                           split_e);
        ScanSource ssrc;
        ssrc.i32 = split_e;
        TRY(launch_scan<int64_t>(s, ssrc, MK, tiles, se_off, se_total));
        const int64_t fix_bound = std::min<int64_t>(split_bound, MK) * (int64_t)std::max(f->rev.max_elems, 1);
        hipLaunchKernelGGL((counts_fixup<256>), dim3(grid_for(fix_bound, 256, 16384)), dim3(256), 0, s, f->rev,
                           (const CountItem *)items, (const int32_t *)item_base, (const int32_t *)nip,
                           (const int64_t *)se_off, (const int64_t *)se_total, (const int32_t *)item_slot,
                           (const float *)partial, grad_arc_score, caps, MK, K, f->health);
        return WFST_OK;
    };
    if (bk.c == 0) {
        build_visits();
        TRY(counts_block(0));
    } else {
        for (int32_t k = K - 1; k >= 0; --k) {  // blocks from the end: recompute alpha~, beta sweep, counts
            bk.k = k;
            hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters + C_QUEUE, (int64_t)1, 0);
            DISPATCH_NT(rc, f->nt, launch_forward, f, s, bv, tp, bk, nullptr)
            if (rc != WFST_OK) return rc;
            hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters + C_QUEUE, (int64_t)1, 0);
            DISPATCH_NT(rc, f->nt, launch_backward, f, s, bv, tp, bk, no_records)
            if (rc != WFST_OK) return rc;
            build_visits();
            TRY(counts_block(k));
        }
    }
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

int wfst_forward_backward(const wfst_fst *f, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                          const int32_t *tokens, float *log_z, float *arc_posterior, float *final_posterior,
                          int32_t *status, void *stream)
{
    wfst_tape *t = nullptr;
    TRY(wfst_forward(f, batch, num_tokens, offsets, tokens, log_z, status, &t, stream));
    int rc = wfst_backward(f, t, nullptr, arc_posterior, final_posterior, stream);
    wfst_tape_free(t);
    return rc;
}

int wfst_fst_autotune(wfst_fst *f, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                      const int32_t *tokens, const char *cache_path, int32_t flags, wfst_autotune_result *res,
                      void *stream)
{
    if (!f) return set_err(WFST_EINVAL, "fst is NULL");
    TRY(check_batch(f, batch, num_tokens, offsets, tokens));
    static const int32_t sizes[5] = {64, 128, 256, 512, 1024};
    static const int32_t modes[3] = {0, -1, -2};
    hipStream_t s = as_stream(stream);
    wfst_autotune_result r;
    std::memset(&r, 0, sizeof(r));
    for (int c = 0; c < 4; ++c)
        for (int k = 0; k < 5; ++k)
            for (int m = 0; m < 3; ++m) r.ms[c][k][m] = -1.0f;
    const int32_t keep_nt = f->nt, keep_mode = count_mode(f), keep_chunk = f->chunk;
    r.threads_per_sentence = keep_nt;
    r.count_records = keep_mode;
    r.chunk_arcs = keep_chunk;
    r.best_ms = -1.0f;
    if (batch == 0) {
        if (res) *res = r;
        return WFST_OK;
    }
    std::string key;
    std::vector<std::pair<std::string, TuneEntry>> cache;
    if (cache_path && *cache_path) {
        TRY(tune_key(f, batch, num_tokens, offsets, tokens, flags, s, key));
        cache = read_tune_cache(cache_path);
        for (auto &e : cache)
            if (e.first == key) {  // known workload: apply without timing
                TRY(rebuild_layouts(f, e.second.chunk, s));
                f->nt = e.second.nt;
                set_count_mode(f, e.second.mode);
                r.threads_per_sentence = f->nt;
                r.count_records = e.second.mode;
                r.chunk_arcs = f->chunk;
                r.best_ms = e.second.ms;
                r.from_cache = 1;
                if (res) *res = r;
                return WFST_OK;
            }
    }
    // scratch outputs of the timed passes
    const int64_t N = num_tokens;
    const size_t bytes = (size_t)batch * (2 * sizeof(float) + sizeof(int32_t)) + (size_t)N * sizeof(int32_t) +
                         (size_t)std::max<int64_t>(f->A, 1) * sizeof(float);
    void *scratch_out = nullptr;
    if (hipMalloc(&scratch_out, bytes) != hipSuccess) return set_err(WFST_ENOMEM, "autotune scratch");
    float *score = static_cast<float *>(scratch_out);
    float *log_z = score + batch;
    int32_t *status = reinterpret_cast<int32_t *>(log_z + batch);
    int32_t *arcs = status + batch;
    float *grad = reinterpret_cast<float *>(arcs + N);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = WFST_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = set_err(WFST_EHIP, "event");
    auto pass = [&]() -> int {
        TRY(wfst_viterbi(f, batch, N, offsets, tokens, score, arcs, nullptr, status, s));
        wfst_tape *t = nullptr;
        TRY(wfst_forward(f, batch, N, offsets, tokens, log_z, status, &t, s));
        const int rb = wfst_backward(f, t, nullptr, grad, nullptr, s);
        wfst_tape_free(t);
        return rb;
    };
    std::vector<int32_t> chunks;
    if (flags & WFST_TUNE_CHUNK) chunks = {4, 8, 16, 32};
    else chunks = {keep_chunk};
    int bc = -1, bk = -1, bm = -1;
    for (size_t c = 0; c < chunks.size() && rc == WFST_OK; ++c) {
        r.chunks[c] = chunks[c];
        if ((rc = rebuild_layouts(f, chunks[c], s)) != WFST_OK) break;
        for (int k = 0; k < 5 && rc == WFST_OK; ++k) {
            for (int m = 0; m < 3 && rc == WFST_OK; ++m) {
                f->nt = sizes[k];
                // records and the grouped kernel need the on-chip backward sweep, the
                // grouped kernel its own state in LDS too
                if (modes[m] != -2 && backward_in_gmem(f)) continue;
                if (modes[m] == -1 && lds_counts(f) > f->max_lds) continue;
                set_count_mode(f, modes[m]);
                int p = pass();  // untimed: grows workspaces, loads code
                if (p == WFST_EUNSUPPORTED) continue;  // this size does not fit the FST's needs
                if (p != WFST_OK) {
                    rc = p;
                    break;
                }
                if (hipEventRecord(e0, s) != hipSuccess) {
                    rc = set_err(WFST_EHIP, "event");
                    break;
                }
                if ((p = pass()) != WFST_OK) {
                    rc = p;
                    break;
                }
                float ms = 0.0f;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = set_err(WFST_EHIP, "event timing");
                    break;
                }
                r.ms[c][k][m] = ms;
                r.tried += 1;
                if (bc < 0 || ms < r.ms[bc][bk][bm]) {
                    bc = (int)c;
                    bk = k;
                    bm = m;
                }
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(scratch_out);
    if (rc == WFST_OK && bc < 0) rc = set_err(WFST_EUNSUPPORTED, "no configuration fits this FST");
    const int32_t chunk = rc == WFST_OK ? chunks[(size_t)bc] : keep_chunk;
    const int rr = rebuild_layouts(f, chunk, s);
    if (rc == WFST_OK) rc = rr;
    f->nt = rc == WFST_OK ? sizes[bk] : keep_nt;
    set_count_mode(f, rc == WFST_OK ? modes[bm] : keep_mode);
    if (rc != WFST_OK) return rc;
    r.threads_per_sentence = f->nt;
    r.count_records = modes[bm];
    r.chunk_arcs = f->chunk;
    r.best_ms = r.ms[bc][bk][bm];
    if (!key.empty()) {
        TuneEntry e;
        e.nt = f->nt;
        e.mode = modes[bm];
        e.chunk = f->chunk;
        e.ms = r.best_ms;
        cache.emplace_back(key, e);
        TRY(write_tune_cache(cache_path, cache));
    }
    if (res) *res = r;
    return WFST_OK;
}

int wfst_forward_scan(const wfst_fst *fc, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                      const int32_t *tokens, float *log_z, float *alpha, int32_t *status, void *stream)
{
    TRY(check_batch(fc, batch, num_tokens, offsets, tokens));
    if (batch == 0) return WFST_OK;
    if (!log_z || !status) return set_err(WFST_EINVAL, "NULL output");
    wfst_fst *f = const_cast<wfst_fst *>(fc);
    if (f->Q > kScanMaxQ)
        return set_err(WFST_EUNSUPPORTED, "the scan keeps dense state x state matrices: num_states must be <= " +
                                              std::to_string(kScanMaxQ));
    hipStream_t s = as_stream(stream);
    const int64_t N = num_tokens, QQ = (int64_t)f->Q * f->Q;
    if ((double)N * (double)QQ * 2.0 * sizeof(float) > (double)kScanBudgetBytes)
        return set_err(WFST_EUNSUPPORTED, "the scan needs two state x state matrices per token: " +
                                              std::to_string(N) + " tokens exceed its " +
                                              std::to_string(kScanBudgetBytes >> 30) + " GiB");
    int32_t *counters = nullptr, *first = nullptr;
    float *p0 = nullptr, *p1 = nullptr;
    TRY(ensure_t(f->ws[W_COUNTERS], C_COUNT, s, &counters));
    int32_t tmax = 0;
    if (N > 0) {
        TRY(ensure_t(f->ws[W_TOKSENT], N, s, &first));
        TRY(ensure_t(f->ws[W_SCAN0], N * QQ, s, &p0));
        TRY(ensure_t(f->ws[W_SCAN1], N * QQ, s, &p1));
        // longest sentence: the number of levels (one read-back; the scan is the latency path)
        hipLaunchKernelGGL(batch_max_len, dim3(1), dim3(1024), 0, s, offsets, batch, counters + C_TOTAL);
        HIP_OK(hipMemcpyAsync(&tmax, counters + C_TOTAL, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    ProfScope prof(f, s, WFST_KERNEL_SCAN);
    if (N > 0) {
        hipLaunchKernelGGL(token_first, dim3(grid_for(N, 256)), dim3(256), 0, s, offsets, batch, N, first);
        const unsigned g = (unsigned)std::min<int64_t>(N, 65535);
        hipLaunchKernelGGL(scan_leaves, dim3(g), dim3(kScanThreadsPerMat), 0, s, f->fwd, f->Q, tokens, N, f->M, p0);
        for (int64_t stride = 1; stride < tmax; stride *= 2) {
            hipLaunchKernelGGL(scan_level, dim3(g), dim3(kScanThreadsPerMat), 0, s, (const float *)p0, p1,
                               (const int32_t *)first, N, f->Q, (int32_t)stride);
            std::swap(p0, p1);
        }
    }
    hipLaunchKernelGGL(scan_finish, dim3(grid_for(batch, 4)), dim3(256), 0, s, (const float *)p0, offsets, tokens,
                       batch, N, f->M, f->Q, f->start, (const float *)f->final_score, log_z, alpha, status);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

size_t lds_lattice(const wfst_fst *f)
{
    return ((size_t)f->Q + 1 + (size_t)std::max(f->fwd.max_segs, 1) + (size_t)std::max(f->fwd.max_slots, 1)) *
               sizeof(double) +
           (size_t)std::max(f->fwd.max_segs, 1) * sizeof(int32_t) + ((size_t)f->Q + 1) * sizeof(float);
}

int wfst_lattice_forward(const wfst_fst *fc, int32_t batch, const int32_t *node_offsets, const int32_t *arc_offsets,
                         int64_t num_nodes, int64_t num_arcs, const int32_t *arc_from, const int32_t *arc_to,
                         const int32_t *arc_label, const float *arc_weight, float *log_z, float *node_log_alpha,
                         int32_t *status, void *stream)
{
    if (!fc) return set_err(WFST_EINVAL, "fst is NULL");
    if (batch < 0 || num_nodes < 0 || num_arcs < 0) return set_err(WFST_EINVAL, "negative size");
    if (num_nodes > INT32_MAX || num_arcs > INT32_MAX) return set_err(WFST_EINVAL, "lattice ids are int32");
    if (batch == 0) return WFST_OK;
    if (!node_offsets || !arc_offsets || !log_z || !status) return set_err(WFST_EINVAL, "NULL offsets or output");
    if (num_arcs > 0 && (!arc_from || !arc_to || !arc_label || !arc_weight))
        return set_err(WFST_EINVAL, "NULL arc array");
    wfst_fst *f = const_cast<wfst_fst *>(fc);
    hipStream_t s = as_stream(stream);
    constexpr int NT = 256;
    const size_t lds = lds_lattice(f);
    int grid = 0;
    TRY(persistent_grid(f, lattice_forward<NT>, NT, lds, batch, &grid));
    int32_t *counters = nullptr;
    float *nodes = nullptr;
    double *scale = nullptr;
    const int64_t Q1 = (int64_t)f->Q + 1;
    TRY(ensure_t(f->ws[W_COUNTERS], C_COUNT, s, &counters));
    TRY(ensure_t(f->ws[W_LATNODE], std::max<int64_t>(num_nodes, 1) * Q1, s, &nodes));
    TRY(ensure_t(f->ws[W_LATSCALE], std::max<int64_t>(num_nodes, 1), s, &scale));
    int32_t *far = nullptr;
    TRY(ensure_t(f->ws[W_LATFAR], std::max<int64_t>(num_nodes, 1), s, &far));
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, counters, (int64_t)C_COUNT, 0);
    hipLaunchKernelGGL(fill_i32, dim3(grid_for(std::max<int64_t>(num_nodes, 1), 256, 8192)), dim3(256), 0, s, far,
                       std::max<int64_t>(num_nodes, 1), 0);
    LatticeView lv;
    lv.B = batch;
    lv.n_nodes = num_nodes;
    lv.n_arcs = num_arcs;
    lv.node_off = node_offsets;
    lv.arc_off = arc_offsets;
    lv.from = arc_from;
    lv.to = arc_to;
    lv.label = arc_label;
    lv.weight = arc_weight;
    lv.nodes = nodes;
    lv.scale = scale;
    lv.far = far;
    lv.queue = counters + C_QUEUE;
    lv.offs_bad = counters + C_NITEMS;
    hipLaunchKernelGGL(lattice_offsets_check, dim3(grid_for((int64_t)batch + 1, 256)), dim3(256), 0, s, node_offsets,
                       arc_offsets, batch, num_nodes, num_arcs, counters + C_NITEMS);
    ProfScope prof(f, s, WFST_KERNEL_LATTICE);
    hipLaunchKernelGGL((lattice_forward<NT>), dim3(grid), dim3(NT), lds, s, f->fwd, f->Q, f->start, f->M,
                       (const float *)f->final_score, lv, log_z, node_log_alpha, status, f->health);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

int wfst_em_update(wfst_fst *f, const float *counts, float smoothing, const float *cur_score, float *new_score,
                   void *stream)
{
    if (!f) return set_err(WFST_EINVAL, "fst is NULL");
    if (f->A > 0 && (!counts || !cur_score || !new_score)) return set_err(WFST_EINVAL, "NULL argument");
    if (!(smoothing >= 0.0f) || std::isinf(smoothing)) return set_err(WFST_EINVAL, "smoothing must be finite and >= 0");
    if (f->A == 0) return WFST_OK;
    hipStream_t s = as_stream(stream);
    TRY(ensure_source_index(f, s));
    double *sums;
    TRY(ensure_t(f->ws[W_EMSUM], f->Q, s, &sums));
    hipLaunchKernelGGL(em_source_sums, dim3(grid_for((int64_t)f->Q * 64, 256, 65535)), dim3(256), 0, s,
                       (const int32_t *)f->em_order, (const int64_t *)f->em_start, f->Q, counts, smoothing, sums);
    hipLaunchKernelGGL(em_normalize, dim3(grid_for(f->A, 256, 16384)), dim3(256), 0, s, (const int32_t *)f->em_src,
                       f->A, counts, smoothing, (const double *)sums, cur_score, new_score);
    HIP_OK(hipGetLastError());
    return WFST_OK;
}

// One pass sequence of a graph (scores, Viterbi, forward, backward), as the
// eager entry points queue it.
static int graph_sequence(wfst_fst *f, const wfst_graph_args &a, void *stream)
{
    if (a.arc_score) TRY(wfst_fst_set_scores(f, a.arc_score, nullptr, stream));
    if (a.best_score)
        TRY(wfst_viterbi(f, a.batch, a.num_tokens, a.offsets, a.tokens, a.best_score, a.best_arcs, a.best_olabels,
                         a.status, stream));
    if (a.log_z) {
        wfst_tape *t = nullptr;
        TRY(wfst_forward(f, a.batch, a.num_tokens, a.offsets, a.tokens, a.log_z, a.status, &t, stream));
        const int r = a.grad_arc_score ? wfst_backward(f, t, a.grad_log_z, a.grad_arc_score, a.grad_final, stream)
                                       : WFST_OK;
        wfst_tape_free(t);
        TRY(r);
    }
    return WFST_OK;
}

static void graph_free(wfst_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (Buf &b : g->ws) free_buf(b);
    for (TapeBufs *t : g->pool) {
        for (Buf *b : {&t->order, &t->tok_off, &t->alpha, &t->a_max, &t->a_log, &t->log_z, &t->tiles, &t->total,
                       &t->ck_size, &t->ck_off, &t->blk_size, &t->blk_base})
            free_buf(*b);
        delete t;
    }
    delete g;
}

int wfst_graph_create(wfst_fst *f, const wfst_graph_args *args, void *stream, wfst_graph **out)
{
    if (!out) return set_err(WFST_EINVAL, "out is NULL");
    *out = nullptr;
    if (!f || !args) return set_err(WFST_EINVAL, "NULL fst or args");
    const wfst_graph_args &a = *args;
    TRY(check_batch(f, a.batch, a.num_tokens, a.offsets, a.tokens));
    if (!a.best_score && !a.log_z) return set_err(WFST_EINVAL, "a graph needs Viterbi or forward outputs");
    if (!a.status) return set_err(WFST_EINVAL, "status is NULL");
    if (a.grad_final && !a.grad_arc_score) return set_err(WFST_EINVAL, "grad_final needs grad_arc_score");
    hipStream_t s = as_stream(stream);
    if (s == nullptr) return set_err(WFST_EINVAL, "graphs are captured on a created stream, not the null stream");
    wfst_graph *g = new wfst_graph();
    g->fst = f;
    g->args = a;
    const bool prof = f->prof;
    auto enter = [&]() {
        for (int i = 0; i < W_NUM; ++i) std::swap(f->ws[i], g->ws[i]);
        std::swap(f->tape_pool, g->pool);
        f->prof = false;
        f->graph_mode = true;
    };
    auto leave = [&]() {
        for (int i = 0; i < W_NUM; ++i) std::swap(f->ws[i], g->ws[i]);
        std::swap(f->tape_pool, g->pool);
        f->prof = prof;
        f->graph_mode = false;
    };
    enter();
    // eager run: sizes the graph's buffers (nothing grows during capture) and checks the arguments
    int rc = graph_sequence(f, a, stream);
    if (rc == WFST_OK && hipStreamSynchronize(s) != hipSuccess) rc = set_err(WFST_EHIP, "eager pass of the graph");
    if (rc == WFST_OK) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            rc = set_err(WFST_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        } else {
            rc = graph_sequence(f, a, stream);
            e = hipStreamEndCapture(s, &g->graph);
            if (rc == WFST_OK && e != hipSuccess)
                rc = set_err(WFST_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        }
    }
    leave();
    if (rc == WFST_OK) {
        const hipError_t e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = set_err(WFST_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (rc != WFST_OK) {
        (void)hipStreamSynchronize(s);
        graph_free(g);
        return rc;
    }
    f->live_graphs += 1;
    *out = g;
    return WFST_OK;
}

int wfst_graph_launch(wfst_graph *g, void *stream)
{
    if (!g || !g->exec) return set_err(WFST_EINVAL, "graph is NULL");
    HIP_OK(hipGraphLaunch(g->exec, as_stream(stream)));
    if (g->args.arc_score) g->fst->score_version += 1;  // the replay replaced the scores
    return WFST_OK;
}

void wfst_graph_destroy(wfst_graph *g)
{
    if (!g) return;
    int cur = 0;
    const int dev = g->fst->device;
    const bool other = hipGetDevice(&cur) == hipSuccess && cur != dev;
    if (other) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    g->fst->live_graphs -= 1;
    graph_free(g);
    if (other) (void)hipSetDevice(cur);
}

}  // extern "C"
