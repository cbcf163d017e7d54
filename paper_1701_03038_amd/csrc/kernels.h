// Device-side views of the sliced layouts and the per-call batch state.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.h"

namespace wfst {

struct DevLayout {
    int32_t *other = nullptr;      // padded, slice-interleaved arc slots: other end state
    float *score = nullptr;        // ... and arc score
    int32_t *elem_arc = nullptr;   // arc id per slot (-1 padding)
    uint16_t *elem_loc = nullptr;  // arc id - its label's lowest arc id (0xffff: padding or too far), for
                                   // score updates staged per label; null when they are not staged
    SliceInfo *slice = nullptr;
    int32_t *seg_key = nullptr;
    SegChunk *seg_chunk = nullptr;
    LabelInfo *label = nullptr;
    int64_t n_elem = 0, n_slice = 0, n_seg = 0;
    int32_t max_segs = 0, max_slots = 0, max_elems = 0, max_height = 0, max_slices = 0;
};

// What every batched sweep needs about the batch.
struct BatchView {
    int32_t B = 0;
    int32_t M = 0;
    int64_t N = 0;
    const int32_t *offsets = nullptr;  // [B+1]
    const int32_t *tokens = nullptr;   // [N]
    const int32_t *order = nullptr;    // [B] processing order (longest first)
    const int64_t *tok_off = nullptr;  // [N] compact per-step storage offsets (prefix of segment counts)
    int32_t *queue = nullptr;          // work-queue head
    int32_t *status = nullptr;         // [B]
    uint32_t *health = nullptr;        // sticky WFST_HEALTH_* bits (see below)
};

// Health bits: a kernel that finds device data outside what its loops may
// trust stops that piece of work and records why, instead of running away.
enum HealthBit : uint32_t {
    H_QUEUE = 1u,      // a persistent workgroup popped more items than exist
    H_ITEM = 2u,       // a count work item or the item count is out of range
    H_VISIT = 4u,      // a visit, token or sentence index is out of range
    H_SLOT = 8u,       // a split-label partial slot is beyond its buffer
    H_SCATTER = 16u,   // a sort scatter position is out of range
    H_GROUP = 32u,     // label grouping produced more items than reserved
    H_TEAM = 64u,      // a team sweep's barrier timed out (the team stopped; results invalid)
};

// Capacities the count kernels check their device-side inputs against.
struct CountCaps {
    int32_t items_cap = 0, slot_cap = 0, V = 0;
};

// The forward-backward tape (compact: one value per (token, forward segment)).
struct TapeView {
    float *alpha = nullptr;    // alpha~_t on the destinations of w_t
    float *beta = nullptr;     // beta~_t on the destinations of w_t
    float *a_max = nullptr;    // [N] c_t: per-step normaliser of alpha~_t
    double *a_log = nullptr;   // [N] C_t: log scale, true log alpha_t = alpha~_t - c_t + C_t
    float *b_max = nullptr;    // [N]
    double *b_log = nullptr;   // [N]
    double *log_z = nullptr;   // [B]
    double *log_z_bwd = nullptr;  // [B] log Z recomputed from beta_0[start]
    const int64_t *ck_off = nullptr;  // checkpointed tape: alpha~ offset per token (-1: not kept); null = all kept
};

// Checkpointed forward-backward: alpha~ is kept only every c steps (and at
// the last step); the backward pass walks blocks of c steps from the end,
// recomputing each block's alpha~ from its checkpoint.  A block's alpha~ and
// beta~ live in double buffers chosen by block parity, at a per-sentence base
// plus the token's offset inside its block.
struct BlockView {
    int32_t c = 0;  // checkpoint interval; 0 = the whole tape is resident
    int32_t k = 0;  // block being processed: steps k*c+1 .. (k+1)*c
    float *abuf[2] = {nullptr, nullptr};
    float *bbuf[2] = {nullptr, nullptr};
    const int64_t *base = nullptr;  // [B]
};

// Offset of token i (sentence b starting at o0) inside its block buffer.
__device__ __forceinline__ int64_t block_rel(const BlockView &bk, const BatchView &bv, int b, int o0, int i,
                                             int &blk)
{
    blk = (i - o0) / bk.c;  // step i - o0 + 1 lies in block (step - 1) / c
    return bk.base[b] + (bv.tok_off[i] - bv.tok_off[o0 + blk * bk.c]);
}

// alpha~ of token i: the full tape, a checkpoint, or the block buffer of the
// token's block (recomputed by the current block's forward pass)
__device__ __forceinline__ const float *alpha_slot(const TapeView &tp, const BlockView &bk, const BatchView &bv,
                                                   int b, int o0, int i)
{
    if (bk.c == 0) return tp.alpha + bv.tok_off[i];
    if (tp.ck_off[i] >= 0) return tp.alpha + tp.ck_off[i];
    int blk;
    const int64_t r = block_rel(bk, bv, b, o0, i, blk);
    return bk.abuf[blk & 1] + r;
}

// Expected-count records written by the backward pass: one per (arc, visit)
// with a nonzero posterior, key = (e << 32) | token position, where e is the
// arc's slot in the reverse layout (one slot per arc; elem_arc maps it back).
// count may pass cap: records beyond cap are dropped and the caller falls back.
//
// Alternatively (acc != null) each posterior is added at once to its arc's
// fixed-point accumulator, also indexed by reverse-layout slot: acc[e] +=
// round(value * 2^S), an integer atomic, so the sum does not depend on the
// order of the additions (no records, no sort; used when records could not
// fit, or when asked for).  A step's additions then fall in its label's
// slices instead of all over the arc ids.
struct RecordSink {
    uint64_t *key = nullptr;  // null: no records
    float *val = nullptr;
    unsigned long long *count = nullptr;  // record slots taken (records + unused chunk tails)
    unsigned long long *total = nullptr;  // records (independent of scheduling)
    int64_t cap = 0;
    const float *grad_log_z = nullptr;  // g_b (null = 1)
    unsigned long long *acc = nullptr;  // [reverse slots] fixed-point sums (two's complement)
    const double *fx_scale = nullptr;   // device scalar 2^S
    // The gradient the records are later summed into, zero-filled by the sweep
    // itself, a slab per workgroup and step (null: the caller fills it).
    float *fill = nullptr;
    int64_t fill_n = 0;
};

// beta~ of token i: the full tape, or the block buffer of the token's block
__device__ __forceinline__ float *beta_slot(const TapeView &tp, const BlockView &bk, const BatchView &bv, int b,
                                            int o0, int i)
{
    if (bk.c == 0) return tp.beta + bv.tok_off[i];
    int blk;
    const int64_t r = block_rel(bk, bv, b, o0, i, blk);
    return bk.bbuf[blk & 1] + r;
}

}  // namespace wfst
