// HIP kernels for gfx950: the per-input-symbol semiring sparse matrix-vector
// step (paper, section 5) run as persistent batched sweeps.
//
// One workgroup owns one sentence at a time, popped from a length-ordered
// work queue; the state vector alpha_t (or beta_t) lives in LDS for the whole
// sentence.  A step over input symbol a streams the sliced arc blocks of a
// (coalesced 8-byte {state, score} loads, one chunk of a (label, key) segment
// per lane), gathers the previous vector from LDS, reduces each chunk
// serially, then combines multi-chunk segments in chunk order.  Every
// reduction has a fixed order: there are no floating-point atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "kernels.h"

namespace wfst {

#define WFST_NINF (-__builtin_huge_valf())

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// e^x through the hardware base-2 exponential (v_exp_f32).
__device__ __forceinline__ float exp_e(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
// ln(x) through the hardware base-2 logarithm (v_log_f32).
__device__ __forceinline__ float log_e(float x) { return __builtin_amdgcn_logf(x) * kLn2; }

// Order-preserving map of a float onto uint32 (valid for every non-NaN value).
__device__ __forceinline__ uint32_t ord_f32(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t k)
{
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
// A pointer read from memory is generic to the compiler, and generic (flat)
// accesses also count against the LDS wait counter, so every LDS wait would
// wait for them too; tape pointers read from tables are global memory.
typedef __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ gfloat *to_global(float *p) { return (gfloat *)p; }
__device__ __forceinline__ const gfloat *to_global(const float *p) { return (const gfloat *)p; }

__device__ __forceinline__ float wave_max_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// log-sum-exp accumulator (m, s): the set's LSE is m + ln s.  Merging is
// written symmetrically so that merge(a, b) and merge(b, a) round the same.
struct Lse {
    float m, s;
};
__device__ __forceinline__ Lse lse_merge(Lse a, Lse b)
{
    if (a.m == WFST_NINF) return b;
    if (b.m == WFST_NINF) return a;
    const float big = fmaxf(a.m, b.m);
    const float sbig = a.m >= b.m ? a.s : b.s;
    const float ssmall = a.m >= b.m ? b.s : a.s;
    const float small = fminf(a.m, b.m);
    if (a.m == b.m) return Lse{big, a.s + b.s};
    return Lse{big, sbig + ssmall * exp_e(small - big)};
}
// Online update with one finite value x: one exponential per value.
__device__ __forceinline__ void lse_push(Lse &acc, float x)
{
    const float d = x - acc.m;  // +inf while acc is empty
    const float e = exp_e(-fabsf(d));
    if (d > 0.0f) {
        acc.s = acc.s * e + 1.0f;
        acc.m = x;
    } else {
        acc.s = acc.s + e;
    }
}
__device__ __forceinline__ float lse_value(Lse a) { return a.s > 0.0f ? a.m + log_e(a.s) : WFST_NINF; }

__device__ __forceinline__ Lse wave_lse(Lse v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Lse w{__shfl_xor(v.m, o, 64), __shfl_xor(v.s, o, 64)};
        v = lse_merge(v, w);
    }
    return v;
}

// Log-sum-exp with the running max in FP64: terms are alpha^ + theta (exact in
// FP64), only the shifted exponent and the sum are FP32.  The per-sentence state
// is kept normalised (the step max subtracted, the scale in FP64), so FP32
// rounding does not accumulate along a long sentence.
struct LseD {
    double m;
    float s;
};
__device__ __forceinline__ void lse_push_d(LseD &acc, double x)
{
    const double d = x - acc.m;  // +inf while acc is empty
    const float e = exp_e((float)(-fabs(d)));
    if (d > 0.0) {
        acc.s = acc.s * e + 1.0f;
        acc.m = x;
    } else {
        acc.s = acc.s + e;
    }
}
__device__ __forceinline__ LseD lse_merge_d(LseD a, LseD b)
{
    if (b.m == -__builtin_huge_val()) return a;
    if (a.m == -__builtin_huge_val()) return b;
    if (b.m > a.m) return LseD{b.m, a.s * exp_e((float)(a.m - b.m)) + b.s};
    return LseD{a.m, a.s + b.s * exp_e((float)(b.m - a.m))};
}
__device__ __forceinline__ double lse_value_d(LseD a)
{
    return a.s > 0.0f ? a.m + (double)log_e(a.s) : -__builtin_huge_val();
}
__device__ __forceinline__ uint64_t ord_f64(double d)
{
    const uint64_t u = (uint64_t)__double_as_longlong(d);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord_f64(uint64_t k)
{
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffull) : ~k));
}
// block max of FP64 values into an LDS cell (ordered uint64); caller syncs
__device__ __forceinline__ void block_max_d(double v, unsigned long long *cell, int lane)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (lane == 0) atomicMax(cell, (unsigned long long)ord_f64(v));
}
// Fold a batch of terms (-inf = none) into acc: the batch max by a pairwise
// tree, the shifted exponentials independent of each other, one merge; the
// dependency chain is a few FP64 ops per batch instead of per term.
template <int RB>
__device__ __forceinline__ void lse_push_batch(LseD &acc, const double (&x)[RB])
{
    double t[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) t[u] = x[u];
#pragma unroll
    for (int w = RB / 2; w >= 1; w /= 2)
#pragma unroll
        for (int u = 0; u < w; ++u) t[u] = fmax(t[u], t[u + w]);
    const double m = t[0];
    if (m == -__builtin_huge_val()) return;
    float sum = 0.0f;
#pragma unroll
    for (int u = 0; u < RB; ++u) sum += exp_e((float)(x[u] - m));
    acc = lse_merge_d(acc, LseD{m, sum});
}

// The same for terms g[u] + e[u].score formed in FP64 on the fly (no FP64
// copy of the batch: the first tree level is built from the FP32 operands and
// each term is re-formed for its exponential).
template <int RB>
__device__ __forceinline__ void lse_push_terms(LseD &acc, const float (&g)[RB], const Elem (&e)[RB])
{
    static_assert(RB >= 2 && (RB & (RB - 1)) == 0, "row batch must be a power of two");
    double t[RB / 2];
#pragma unroll
    for (int u = 0; u < RB / 2; ++u)
        t[u] = fmax((double)g[u] + (double)e[u].score, (double)g[u + RB / 2] + (double)e[u + RB / 2].score);
#pragma unroll
    for (int w = RB / 4; w >= 1; w /= 2)
#pragma unroll
        for (int u = 0; u < w; ++u) t[u] = fmax(t[u], t[u + w]);
    const double m = t[0];
    if (m == -__builtin_huge_val()) return;
    float sum = 0.0f;
#pragma unroll
    for (int u = 0; u < RB; ++u) sum += exp_e((float)(((double)g[u] + (double)e[u].score) - m));
    acc = lse_merge_d(acc, LseD{m, sum});
}

// Move a label header loaded ahead into scalar registers where this is cheap
// (its load long done), so that a later wait on vector memory -- which also
// counts the stores issued in between -- is not needed for it.
__device__ __forceinline__ LabelInfo uniform_label(LabelInfo l)
{
    l.slice_first = wave_uniform(l.slice_first);
    l.n_slices = wave_uniform(l.n_slices);
    l.seg_first = wave_uniform(l.seg_first);
    l.n_segs = wave_uniform(l.n_segs);
    l.n_multi = wave_uniform(l.n_multi);
    l.n_slots = wave_uniform(l.n_slots);
    l.elem_first = wave_uniform(l.elem_first);
    l.n_elems = wave_uniform(l.n_elems);
    return l;
}

// A segment's value before normalisation, and its key state.
struct SegVal {
    double v;
    int32_t key;
};

// Rows of a lane's chunk loaded together before they are reduced: enough
// independent 8-byte loads in flight per wavefront to cover HBM latency.
// Rows past the slice height read the dead state (index Q, value -inf).
constexpr int kRowBatch = 16;

__device__ __forceinline__ void load_rows(const int32_t *op, const float *sp, int width, int height, int r0,
                                          int32_t dead, Elem (&e)[kRowBatch])
{
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {  // no branches: rows past the height re-read the last row
        const int at = min(r0 + u, height - 1) * width;
        const int32_t o = op[at];
        const float sc = sp[at];
        e[u] = r0 + u < height ? Elem{o, sc} : Elem{dead, 0.0f};
    }
}

// Validates the sentence's offsets and tokens; returns a WFST_STATUS_* code.
template <int NT>
__device__ int check_sentence(const BatchView &bv, int b, int &o0, int &o1)
{
    o0 = bv.offsets[b];
    o1 = bv.offsets[b + 1];
    if (o0 < 0 || o1 < o0 || (int64_t)o1 > bv.N) return WFST_STATUS_BAD_INPUT;
    int bad = 0;
    for (int i = o0 + (int)threadIdx.x; i < o1; i += NT) {
        const int a = bv.tokens[i];
        bad |= (a < 0 || a >= bv.M);
    }
    return __syncthreads_or(bad) ? WFST_STATUS_BAD_TOKEN : WFST_STATUS_OK;
}

// =====================================================================
// Viterbi (max-plus with back-pointers, paper section 5.1)
// =====================================================================

struct VPart {
    float v;
    int32_t pos;   // winning element
    int32_t pred;  // segment index of the winner's source at the previous step
};

// Bytes of the per-sentence state of the Viterbi sweep: two value vectors and
// two segment-index vectors over Q + 1 states (16-bit indices on chip, 32-bit
// in global memory), then the chunk partials of multi-chunk segments.
template <bool GMEM>
__host__ __device__ constexpr size_t viterbi_state_bytes(int32_t Q)
{
    return (size_t)(Q + 1) * 2 * (sizeof(float) + (GMEM ? sizeof(int32_t) : sizeof(uint16_t)));
}

// The per-sentence state of a persistent workgroup: LDS, or (GMEM) the
// workgroup's slot of a global scratch buffer when the state vectors of the
// FST do not fit on chip.  Each workgroup owns its slot for the whole launch.
template <bool GMEM>
__device__ __forceinline__ unsigned char *state_base(unsigned char *lds, unsigned char *gscratch, int64_t slot_bytes)
{
    if constexpr (GMEM) return gscratch + (size_t)blockIdx.x * (size_t)slot_bytes;
    else return lds;
}

template <int NT, bool GMEM>
__global__ void __launch_bounds__(NT)
viterbi_sweep(DevLayout fl, int32_t Q, int32_t start, const float *__restrict__ final_score,
              BatchView bv, int2 *__restrict__ bp, int32_t *__restrict__ path_tmp,
              float *__restrict__ best_score, int32_t *__restrict__ best_arcs,
              int32_t *__restrict__ best_olabels, const int32_t *__restrict__ olabel,
              unsigned char *__restrict__ gscratch, int64_t slot_bytes)
{
    constexpr int NW = NT / 64;
    // segment index of a state's value at step t (to chain back-pointers); a
    // segment index is below Q + 1, which the host keeps under 2^16 on chip
    using Idx = std::conditional_t<GMEM, int32_t, uint16_t>;
    constexpr Idx kNoIdx = GMEM ? Idx(-1) : Idx(0xffff);
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *smem = state_base<GMEM>(lds, gscratch, slot_bytes);
    float *val0 = reinterpret_cast<float *>(smem);
    float *val1 = val0 + (Q + 1);
    Idx *idx0 = reinterpret_cast<Idx *>(val1 + (Q + 1));
    Idx *idx1 = idx0 + (Q + 1);
    VPart *part = reinterpret_cast<VPart *>(smem + viterbi_state_bytes<GMEM>(Q));
    __shared__ int s_item;
    __shared__ unsigned long long s_best[NW];
    constexpr int kBtChunk = 256;          // backtrace steps per LDS load of their offsets
    __shared__ int64_t s_toff[kBtChunk];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);

    for (int pops = 0;; ++pops) {
        if (tid == 0) s_item = atomicAdd(bv.queue, 1);
        __syncthreads();
        const int item = wave_uniform(s_item);  // uniform: the sentence's loads go through the scalar unit
        __syncthreads();
        if (item >= bv.B) break;
        if (item < 0 || pops > bv.B) {
            if (tid == 0) atomicOr(bv.health, H_QUEUE);
            break;
        }
        const int b = bv.order[item];
        int o0, o1;
        const int st = check_sentence<NT>(bv, b, o0, o1);
        if (st != WFST_STATUS_OK) {
            if (tid == 0) {
                bv.status[b] = st;
                best_score[b] = WFST_NINF;
            }
            if (st == WFST_STATUS_BAD_TOKEN)
                for (int i = o0 + tid; i < o1; i += NT) {
                    best_arcs[i] = -1;
                    if (best_olabels) best_olabels[i] = -1;
                }
            continue;
        }
        const int T = o1 - o0;
        for (int q = tid; q <= Q; q += NT) {
            val0[q] = WFST_NINF;
            val1[q] = WFST_NINF;
            idx0[q] = kNoIdx;
            idx1[q] = kNoIdx;
        }
        __syncthreads();
        if (tid == 0) {
            val0[start] = 0.0f;
            idx0[start] = 0;
        }
        __syncthreads();

        LabelInfo li_next = T > 0 ? fl.label[bv.tokens[o0]] : LabelInfo{};
        LabelInfo lp{};  // label of the previous step (its support is reset)
        for (int t = 1; t <= T; ++t) {
            float *prev = (t & 1) ? val0 : val1;
            float *cur = (t & 1) ? val1 : val0;
            const Idx *prev_idx = (t & 1) ? idx0 : idx1;
            Idx *cur_idx = (t & 1) ? idx1 : idx0;
            const LabelInfo li = li_next;
            if (t < T) li_next = fl.label[bv.tokens[o0 + t]];  // in flight during this step
            const int64_t toff = bv.tok_off[o0 + t - 1];
            // phase 1: one chunk per lane
            for (int s = wave; s < li.n_slices; s += NW) {
                const SliceInfo si = fl.slice[li.slice_first + s];
                if (lane < si.width) {
                    const int32_t *op = fl.other + si.base + lane;
                    const float *sp = fl.score + si.base + lane;
                    const int c = s * 64 + lane;
                    const int dk = c >= li.n_slots ? fl.seg_key[li.seg_first + li.n_multi + (c - li.n_slots)] : 0;
                    float best = WFST_NINF;
                    int bpos = -1, bsrc = 0;
                    for (int r0 = 0; r0 < si.height; r0 += kRowBatch) {
                        Elem e[kRowBatch];
                        load_rows(op, sp, si.width, si.height, r0, Q, e);
#pragma unroll
                        for (int u = 0; u < kRowBatch; ++u) {
                            const float v = prev[e[u].other] + e[u].score;
                            if (v > best) {
                                best = v;
                                bpos = si.base + (r0 + u) * si.width + lane;
                                bsrc = e[u].other;
                            }
                        }
                    }
                    const int pred = bpos >= 0 ? (int)prev_idx[bsrc] : -1;
                    if (c < li.n_slots) {
                        part[c] = VPart{best, bpos, pred};
                    } else {
                        const int j = li.n_multi + (c - li.n_slots);
                        const int d = dk;
                        if (bpos >= 0) {
                            cur[d] = best;
                            cur_idx[d] = (Idx)j;
                        }
                        bp[toff + j] = make_int2(bpos, pred);
                    }
                }
            }
            __syncthreads();
            // phase 2: multi-chunk segments, chunks in order (lowest arc id wins ties)
            for (int j = tid; j < li.n_multi; j += NT) {
                const SegChunk sc = fl.seg_chunk[li.seg_first + j];
                const int d = fl.seg_key[li.seg_first + j];
                VPart w = part[sc.first];
                for (int p = 1; p < sc.count; ++p) {
                    const VPart x = part[sc.first + p];
                    if (x.v > w.v) w = x;
                }
                if (w.pos >= 0) {
                    cur[d] = w.v;
                    cur_idx[d] = (Idx)j;
                }
                bp[toff + j] = make_int2(w.pos, w.pred);
            }
            // clear alpha_{t-1}: its buffer receives alpha_{t+1}
            if (t == 1) {
                if (tid == 0) prev[start] = WFST_NINF;
            } else {
                for (int j = tid; j < lp.n_segs; j += NT) prev[fl.seg_key[lp.seg_first + j]] = WFST_NINF;
            }
            lp = li;
            __syncthreads();
        }

        // final state: max of alpha_T[q] + f[q]; lowest state id on ties
        const float *fin = (T & 1) ? val1 : val0;
        const Idx *fin_idx = (T & 1) ? idx1 : idx0;
        unsigned long long key = 0ull;
        if (T == 0) {
            if (tid == 0) {
                const float f = final_score[start];
                const float v = 0.0f + f;
                if (f != WFST_NINF && v != WFST_NINF)
                    key = ((unsigned long long)ord_f32(v) << 32) | (0xffffffffu - (uint32_t)start);
            }
        } else {
            const LabelInfo li = fl.label[bv.tokens[o1 - 1]];
            for (int j = tid; j < li.n_segs; j += NT) {
                const int d = fl.seg_key[li.seg_first + j];
                const float x = fin[d];
                const float f = final_score[d];
                if (x == WFST_NINF || f == WFST_NINF) continue;
                const float v = x + f;
                if (v == WFST_NINF) continue;
                const unsigned long long k = ((unsigned long long)ord_f32(v) << 32) | (0xffffffffu - (uint32_t)d);
                key = k > key ? k : key;
            }
        }
        key = wave_max_u64(key);
        if (lane == 0) s_best[wave] = key;
        __syncthreads();
        unsigned long long best = 0ull;
#pragma unroll
        for (int w = 0; w < NW; ++w) best = s_best[w] > best ? s_best[w] : best;
        if (best == 0ull) {
            if (tid == 0) {
                bv.status[b] = WFST_STATUS_NO_PATH;
                best_score[b] = WFST_NINF;
            }
            for (int i = o0 + tid; i < o1; i += NT) {
                best_arcs[i] = -1;
                if (best_olabels) best_olabels[i] = -1;
            }
            __syncthreads();
            continue;
        }
        // backtrace (serial, on device: paper section 5.1), kBtChunk steps at a
        // time: the steps' back-pointer offsets are first loaded into LDS by all
        // threads, so that thread 0's chain waits on one load per step
        int j = 0;
        if (tid == 0) {
            bv.status[b] = WFST_STATUS_OK;
            best_score[b] = unord_f32((uint32_t)(best >> 32));
            const int qT = (int)(0xffffffffu - (uint32_t)(best & 0xffffffffull));
            j = T > 0 ? (int)fin_idx[qT] : 0;
        }
        for (int hi = T; hi >= 1; hi -= kBtChunk) {
            const int lo = max(1, hi - kBtChunk + 1);
            for (int t = lo + tid; t <= hi; t += NT) s_toff[t - lo] = bv.tok_off[o0 + t - 1];
            __syncthreads();
            if (tid == 0)
                for (int t = hi; t >= lo; --t) {
                    const int2 e = bp[s_toff[t - lo] + j];
                    path_tmp[o0 + t - 1] = e.x;
                    j = e.y;
                }
            __syncthreads();
        }
        for (int i = o0 + tid; i < o1; i += NT) {
            const int arc = fl.elem_arc[path_tmp[i]];
            best_arcs[i] = arc;
            if (best_olabels) best_olabels[i] = olabel[arc];
        }
        __syncthreads();
    }
}

// =====================================================================
// Forward / backward (log semiring, paper section 5.2, Algorithm 2)
// =====================================================================

// Phase 1 + 2 of one log-semiring step over a sliced layout.  prev holds the
// previous vector normalised (alpha^); the value of every segment j of the
// label goes to vbuf[j] with its key, unnormalised, in FP64.  Returns this
// thread's max over what it wrote.
// A lane reduces its chunk's rows in row order, RB rows at a time.  The rows
// of a batch are loaded without branches (rows past the slice's height re-read
// its last row and are then replaced by a dead element), so that all RB loads
// are in flight together.
template <int NT, int RB>
__device__ __forceinline__ double lse_step(const DevLayout &L, const LabelInfo &li, const float *prev, double *part,
                                           double *vval, int32_t *vkey, int lane, int wave, int32_t dead)
{
    constexpr int NW = NT / 64;
    double my_max = -__builtin_huge_val();
    for (int s = wave; s < li.n_slices; s += NW) {
        const SliceInfo si = L.slice[li.slice_first + s];
        const bool on = lane < si.width;
        const int c = s * 64 + lane;
        // key state of a single-chunk segment, loaded with the first rows
        const int dkey = on && c >= li.n_slots ? L.seg_key[li.seg_first + li.n_multi + (c - li.n_slots)] : 0;
        const int col = si.base + min(lane, si.width - 1);
        LseD acc{-__builtin_huge_val(), 0.0f};
        for (int r0 = 0; r0 < si.height; r0 += RB) {
            Elem f[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int at = col + min(r0 + u, si.height - 1) * si.width;
                const int32_t o = L.other[at];
                const float sc = L.score[at];
                f[u] = on && r0 + u < si.height ? Elem{o, sc} : Elem{dead, 0.0f};
            }
            float g[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) g[u] = prev[f[u].other];
            lse_push_terms<RB>(acc, g, f);
        }
        if (on) {
            const double v = lse_value_d(acc);
            if (c < li.n_slots) {
                part[c] = v;  // a chunk of a multi-chunk segment, in log form
            } else {
                const int j = li.n_multi + (c - li.n_slots);
                vval[j] = v;
                vkey[j] = dkey;
                my_max = fmax(my_max, v);
            }
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < li.n_multi; j += NT) {
        const SegChunk sc = L.seg_chunk[li.seg_first + j];
        LseD acc{-__builtin_huge_val(), 0.0f};
        for (int p = 0; p < sc.count; ++p) {  // chunks in order
            const double x = part[sc.first + p];
            if (x != -__builtin_huge_val()) lse_push_d(acc, x);
        }
        const double v = lse_value_d(acc);
        vval[j] = v;
        vkey[j] = L.seg_key[li.seg_first + j];
        my_max = fmax(my_max, v);
    }
    return my_max;
}

// Reduce the per-thread maxima into cell (LDS, ordered uint); caller syncs.
__device__ __forceinline__ void block_max_into(float v, uint32_t *cell, int lane)
{
    v = wave_max_f(v);
    if (lane == 0) atomicMax(cell, ord_f32(v));
}

template <int NT, bool GMEM>
__global__ void __launch_bounds__(NT)
forward_sweep(DevLayout fl, int32_t Q, int32_t start, const float *__restrict__ final_score,
              BatchView bv, TapeView tp, BlockView bk, float *__restrict__ log_z_out,
              unsigned char *__restrict__ gscratch, int64_t slot_bytes)
{
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *smem = state_base<GMEM>(lds, gscratch, slot_bytes);
    float *val0 = reinterpret_cast<float *>(smem);
    float *val1 = val0 + (Q + 1);
    double *vval = reinterpret_cast<double *>(val1 + (Q + 1) + ((Q + 1) & 1));  // [max_segs] step values
    double *part = vval + fl.max_segs;                                          // [max_slots] chunk values
    int32_t *vkey = reinterpret_cast<int32_t *>(part + max(fl.max_slots, 1));   // [max_segs] their keys
    __shared__ int s_item;
    __shared__ unsigned long long s_cmax[3];
    __shared__ double s_rm[NW];
    __shared__ float s_rs[NW];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);

    for (int pops = 0;; ++pops) {
        if (tid == 0) s_item = atomicAdd(bv.queue, 1);
        __syncthreads();
        const int item = wave_uniform(s_item);  // uniform: the sentence's loads go through the scalar unit
        __syncthreads();
        if (item >= bv.B) break;
        if (item < 0 || pops > bv.B) {
            if (tid == 0) atomicOr(bv.health, H_QUEUE);
            break;
        }
        const int b = bv.order[item];
        int o0, o1;
        int t0 = 0, t1 = 0;  // steps t0+1 .. t1
        if (bk.c == 0) {
            const int st = check_sentence<NT>(bv, b, o0, o1);
            if (st != WFST_STATUS_OK) {
                if (tid == 0) {
                    bv.status[b] = st;
                    log_z_out[b] = WFST_NINF;
                    tp.log_z[b] = -__builtin_huge_val();
                }
                continue;
            }
            t1 = o1 - o0;
        } else {  // recompute one block of alpha^ from its checkpoint
            if (bv.status[b] != WFST_STATUS_OK) continue;
            o0 = bv.offsets[b];
            o1 = bv.offsets[b + 1];
            t0 = bk.k * bk.c;
            t1 = min(o1 - o0, t0 + bk.c);
            if (t1 <= t0) continue;
        }
        const int T = o1 - o0;
        for (int q = tid; q <= Q; q += NT) {
            val0[q] = WFST_NINF;
            val1[q] = WFST_NINF;
        }
        if (tid < 3) s_cmax[tid] = 0ull;
        __syncthreads();
        {
            float *first = ((t0 + 1) & 1) ? val0 : val1;
            if (t0 == 0) {
                if (tid == 0) first[start] = 0.0f;
            } else {  // the checkpoint holds the normalised state of step t0
                const int ic = o0 + t0 - 1;
                const LabelInfo lc = fl.label[bv.tokens[ic]];
                const float *ta = tp.alpha + tp.ck_off[ic];
                for (int j = tid; j < lc.n_segs; j += NT) first[fl.seg_key[lc.seg_first + j]] = ta[j];
            }
        }
        __syncthreads();
        double C = 0.0;  // log scale: log alpha_t = alpha^_t + C_t
        LabelInfo li_next = t1 > t0 ? fl.label[bv.tokens[o0 + t0]] : LabelInfo{};
        LabelInfo lp = t0 > 0 ? fl.label[bv.tokens[o0 + t0 - 1]] : LabelInfo{};
        for (int t = t0 + 1; t <= t1; ++t) {
            float *prev = (t & 1) ? val0 : val1;
            float *cur = (t & 1) ? val1 : val0;
            const int i = o0 + t - 1;
            const LabelInfo li = li_next;
            if (t < t1) li_next = fl.label[bv.tokens[i + 1]];  // in flight during this step
            float *tape;
            if (bk.c > 0) {
                int blk;
                tape = bk.abuf[bk.k & 1] + block_rel(bk, bv, b, o0, i, blk);
            } else if (tp.ck_off) {
                tape = tp.ck_off[i] >= 0 ? tp.alpha + tp.ck_off[i] : nullptr;
            } else {
                tape = tp.alpha + bv.tok_off[i];
            }
            // 8-row batches: 83 VGPRs, five workgroups per CU (16 rows: 105, four)
            const double mx = lse_step<NT, 8>(fl, li, prev, part, vval, vkey, lane, wave, Q);
            if (t == 1) {
                if (tid == 0) prev[start] = WFST_NINF;
            } else {
                for (int j = tid; j < lp.n_segs; j += NT) prev[fl.seg_key[lp.seg_first + j]] = WFST_NINF;
            }
            lp = li;
            if (tid == 0) s_cmax[(t + 1) % 3] = 0ull;
            block_max_d(mx, &s_cmax[t % 3], lane);
            __syncthreads();
            double c = unord_f64(s_cmax[t % 3]);
            if (!(c > -__builtin_huge_val())) c = 0.0;
            C += c;
            li_next = uniform_label(li_next);  // before the tape stores below
            // normalised state and tape: alpha^_t = alpha_t - c_t
            for (int j = tid; j < li.n_segs; j += NT) {
                const double v = vval[j];
                const float x = v == -__builtin_huge_val() ? WFST_NINF : (float)(v - c);
                cur[vkey[j]] = x;
                if (tape) tape[j] = x;
            }
            if (tid == 0 && bk.c == 0) {
                tp.a_max[i] = 0.0f;  // the tape is already normalised
                tp.a_log[i] = C;
            }
            __syncthreads();
        }
        if (bk.c > 0) continue;
        // log Z = C_T + LSE_q(alpha^_T[q] + f[q])
        LseD acc{-__builtin_huge_val(), 0.0f};
        if (T == 0) {
            if (tid == 0) {
                const float f = final_score[start];
                if (f != WFST_NINF) acc = LseD{(double)f, 1.0f};
            }
        } else {
            const float *fin = (T & 1) ? val1 : val0;
            const LabelInfo li = fl.label[bv.tokens[o1 - 1]];
            for (int j = tid; j < li.n_segs; j += NT) {
                const int d = fl.seg_key[li.seg_first + j];
                const float x = fin[d], f = final_score[d];
                if (x == WFST_NINF || f == WFST_NINF) continue;
                lse_push_d(acc, (double)x + (double)f);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc = lse_merge_d(acc, LseD{__shfl_xor(acc.m, o, 64), __shfl_xor(acc.s, o, 64)});
        if (lane == 0) {
            s_rm[wave] = acc.m;
            s_rs[wave] = acc.s;
        }
        __syncthreads();
        if (tid == 0) {
            LseD tot{s_rm[0], s_rs[0]};
            for (int w = 1; w < NW; ++w) tot = lse_merge_d(tot, LseD{s_rm[w], s_rs[w]});
            const double lzr = lse_value_d(tot);
            if (lzr == -__builtin_huge_val()) {
                bv.status[b] = WFST_STATUS_NO_PATH;
                log_z_out[b] = WFST_NINF;
                tp.log_z[b] = -__builtin_huge_val();
            } else {
                const double lz = C + lzr;
                bv.status[b] = WFST_STATUS_OK;
                log_z_out[b] = (float)lz;
                tp.log_z[b] = lz;
            }
        }
        __syncthreads();
    }
}

// =====================================================================
// Team forward sweep, for state vectors in global memory.  The workgroups of
// a team run one sentence together: each step's slices are shared out among
// the members, which meet at a barrier after the step.  The team's state
// vector is then gathered by many compute units within the same step, so its
// lines are reused from L2/MALL instead of each random gather fetching a line
// from HBM for one value.  Same arithmetic as the forward sweep, except that
// the stored state is alpha_t - C_{t-1} (the step max is known only after the
// barrier) and the step's normaliser is subtracted when it is read.
// =====================================================================
constexpr int kTeamSpin = 1 << 24;  // default polls per barrier wait before the team gives up

struct TeamView {
    int32_t G = 0;                  // workgroups per team (grid = G * n_teams)
    int32_t n_teams = 0;
    int64_t q1 = 0;                 // Q + 1 rounded up to 64 (vector stride)
    float *vec = nullptr;           // [n_teams][3][q1] rotating state vectors
    double *pmax = nullptr;         // [n_teams][2][G] members' step maxima, by step parity
    double *pz = nullptr;           // [n_teams][G][2] members' partial log Z (max, sum)
    double *part = nullptr;         // [n_teams][max_slots] chunk values of multi-chunk segments (rank 0)
    unsigned int *bar = nullptr;    // [n_teams] barrier counters, zero at launch
    int32_t *abort = nullptr;       // set when a member times out; every member then stops
    int32_t spin_limit = kTeamSpin; // polls per barrier wait before the team gives up
    int32_t *work = nullptr;        // [n_teams][2] slice-group counters, by step parity
};

// Team barrier number k (counted from 1): thread 0 of each member announces
// its arrival and polls until all G members have arrived.  Device-scope
// fences on both sides make the members' global writes visible to each other.
// Returns false when the team has been stopped (timeout anywhere).
__device__ __forceinline__ bool team_sync(const TeamView &tv, int team, unsigned int k, uint32_t *health)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(&tv.bar[team], 1u);
        const unsigned int target = k * (unsigned int)tv.G;
        int ok = 1;
        for (int spin = 0;; ++spin) {
            if (__hip_atomic_load(&tv.bar[team], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (__hip_atomic_load(tv.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if (spin >= tv.spin_limit) {
                atomicOr(health, H_TEAM);
                atomicExch(tv.abort, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// LSE of one chunk (a lane's column of a slice), terms u[src] - cprev + score
// in FP64 (u: the previous step's stored state), rows in layout order.
template <int RB>
__device__ __forceinline__ double team_chunk(const DevLayout &L, const SliceInfo &si, int lane, const float *u,
                                             double cprev, int32_t dead)
{
    const int col = si.base + lane;
    LseD acc{-__builtin_huge_val(), 0.0f};
    for (int r0 = 0; r0 < si.height; r0 += RB) {
        int32_t o[RB];
        float sc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {  // rows past the height re-read the last row, then count as dead
            const int at = col + min(r0 + r, si.height - 1) * si.width;
            o[r] = L.other[at];
            sc[r] = L.score[at];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int src = r0 + r < si.height ? o[r] : dead;
            const float x = u[src];
            if (x != WFST_NINF) lse_push_d(acc, ((double)x - cprev) + (double)sc[r]);
        }
    }
    return lse_value_d(acc);
}

// Set v[key_j] = -inf for the keys j = first0, first0 + stride, ... < n of a
// label's segments, four keys in flight at a time.
__device__ __forceinline__ void team_clear(float *v, const int32_t *keys, int j0, int n, int stride)
{
    for (int j = j0; j < n; j += 4 * stride) {
        int k[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) k[u] = j + u * stride < n ? keys[j + u * stride] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k[u] >= 0) v[k[u]] = WFST_NINF;
    }
}

// K chunks at once (the lane's columns of K slices; on[k] false = no column):
// all K chunks' row loads, then all their gathers, are in flight together.
template <int K, int RB>
__device__ __forceinline__ void team_chunks(const DevLayout &L, const SliceInfo (&sl)[K], const bool (&on)[K],
                                            int lane, const float *u, double cprev, int32_t dead, double (&v)[K])
{
    LseD acc[K];
    int h[K], hmax = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[k] = LseD{-__builtin_huge_val(), 0.0f};
        h[k] = on[k] ? sl[k].height : 0;
        hmax = max(hmax, h[k]);
    }
    for (int r0 = 0; r0 < hmax; r0 += RB) {
        int32_t o[K][RB];
        float sc[K][RB];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int at = sl[k].base + lane + (r0 + r) * sl[k].width;
                o[k][r] = r0 + r < h[k] ? L.other[at] : dead;
                sc[k][r] = r0 + r < h[k] ? L.score[at] : 0.0f;
            }
        float x[K][RB];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int r = 0; r < RB; ++r) x[k][r] = u[o[k][r]];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (x[k][r] != WFST_NINF) lse_push_d(acc[k], ((double)x[k][r] - cprev) + (double)sc[k][r]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = on[k] ? lse_value_d(acc[k]) : -__builtin_huge_val();
}

template <int NT>
__global__ void __launch_bounds__(NT)
team_forward_sweep(DevLayout fl, int32_t Q, int32_t start, const float *__restrict__ final_score, BatchView bv,
                   TapeView tp, BlockView bk, float *__restrict__ log_z_out, TeamView tv)
{
    constexpr int NW = NT / 64;
    constexpr int RB = 8;
    __shared__ unsigned long long s_cmax;
    __shared__ double s_rm[NW];
    __shared__ float s_rs[NW];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);
    // members of a team sit on one XCD when workgroups are dealt round-robin over the 8 XCDs
    const int team = (int)(blockIdx.x % 8u) + 8 * (int)((blockIdx.x / 8u) / (unsigned)tv.G);
    const int rank = (int)((blockIdx.x / 8u) % (unsigned)tv.G);
    const int G = tv.G;
    float *vbase = tv.vec + (int64_t)team * 3 * tv.q1;
    double *pmax = tv.pmax + (int64_t)team * 2 * G;
    double *pz = tv.pz + (int64_t)team * 2 * G;
    double *part = tv.part + (int64_t)team * max(fl.max_slots, 1);
    unsigned int nbar = 0;
    // all three vectors -inf (the invariant between sentences)
    for (int64_t x = (int64_t)rank * NT + tid; x < 3 * tv.q1; x += (int64_t)G * NT) vbase[x] = WFST_NINF;
    if (!team_sync(tv, team, ++nbar, bv.health)) return;

    for (int item = team; item < bv.B; item += tv.n_teams) {
        const int b = bv.order[item];
        int o0, o1, t0 = 0, t1 = 0;
        if (bk.c == 0) {
            const int st = check_sentence<NT>(bv, b, o0, o1);  // the same verdict in every member
            if (st != WFST_STATUS_OK) {
                if (rank == 0 && tid == 0) {
                    bv.status[b] = st;
                    log_z_out[b] = WFST_NINF;
                    tp.log_z[b] = -__builtin_huge_val();
                }
                continue;
            }
            t1 = o1 - o0;
        } else {
            if (bv.status[b] != WFST_STATUS_OK) continue;
            o0 = bv.offsets[b];
            o1 = bv.offsets[b + 1];
            t0 = bk.k * bk.c;
            t1 = min(o1 - o0, t0 + bk.c);
            if (t1 <= t0) continue;
        }
        const int T = o1 - o0;
        // initial state in vector t0 % 3 (already normalised: its step max is 0)
        float *v0 = vbase + (int64_t)(t0 % 3) * tv.q1;
        int lc_first = 0, lc_n = 0;  // segments of the checkpoint's label (block mode)
        if (t0 == 0) {
            if (rank == 0 && tid == 0) v0[start] = 0.0f;
        } else {
            const int ic = o0 + t0 - 1;
            const LabelInfo lc = fl.label[bv.tokens[ic]];
            lc_first = lc.seg_first;
            lc_n = lc.n_segs;
            const float *ta = tp.alpha + tp.ck_off[ic];
            for (int j = rank * NT + tid; j < lc_n; j += G * NT) v0[fl.seg_key[lc_first + j]] = ta[j];
        }
        if (rank == 0 && tid < 2) tv.work[2 * team + tid] = 0;
        if (!team_sync(tv, team, ++nbar, bv.health)) return;
        double C = 0.0, cprev = 0.0;
        for (int t = t0 + 1; t <= t1; ++t) {
            const float *prev = vbase + (int64_t)((t - 1) % 3) * tv.q1;
            float *cur = vbase + (int64_t)(t % 3) * tv.q1;
            float *old = vbase + (int64_t)((t + 1) % 3) * tv.q1;
            const int i = o0 + t - 1;
            const LabelInfo li = uniform_label(fl.label[bv.tokens[i]]);
            // clear the support of alpha_{t-2} (read by everyone at step t-1, before the last barrier)
            if (t - 2 == 0) {
                if (rank == 0 && tid == 0) old[start] = WFST_NINF;
            } else if (t - 2 >= t0) {
                int o_first = lc_first, o_n = lc_n;
                if (t - 2 > t0) {
                    const LabelInfo lo = fl.label[bv.tokens[i - 2]];
                    o_first = lo.seg_first;
                    o_n = lo.n_segs;
                }
                team_clear(old, fl.seg_key + o_first, rank * NT + tid, o_n, G * NT);
            }
            if (tid == 0) s_cmax = 0ull;
            __syncthreads();
            double my_max = -__builtin_huge_val();
            // slices holding chunks of multi-chunk segments: member 0; the rest dealt out
            const int n_ms = (li.n_slots + 63) / 64;
            if (rank == 0)
                for (int s = wave; s < n_ms; s += NW) {
                    const SliceInfo si = fl.slice[li.slice_first + s];
                    const int c = s * 64 + lane;
                    if (lane < si.width) {
                        const double v = team_chunk<RB>(fl, si, lane, prev, cprev, Q);
                        if (c < li.n_slots) {
                            part[c] = v;
                        } else {
                            const int d = fl.seg_key[li.seg_first + li.n_multi + (c - li.n_slots)];
                            if (v != -__builtin_huge_val()) cur[d] = (float)v;
                            my_max = fmax(my_max, v);
                        }
                    }
                }
            // the other slices, in groups of KS taken from the team's counter by each
            // wavefront (dynamic, so that members finish together); a group's row
            // loads and gathers are in flight together
            constexpr int KS = 4;
            if (rank == 0 && tid == 0) tv.work[2 * team + ((t + 1) & 1)] = 0;  // the counter of step t+1
            for (;;) {
                int grp = 0;
                if (lane == 0) grp = atomicAdd(&tv.work[2 * team + (t & 1)], 1);
                grp = __shfl(grp, 0, 64);
                const int s0 = n_ms + grp * KS;
                if (s0 >= li.n_slices) break;
                SliceInfo sl[KS];
                bool on[KS];
                int d[KS];
                double v[KS];
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const int sk = s0 + k;
                    sl[k] = sk < li.n_slices ? fl.slice[li.slice_first + sk] : SliceInfo{0, 0, 0, 0};
                }
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    on[k] = lane < sl[k].width;
                    const int c = (s0 + k) * 64 + lane;
                    d[k] = on[k] ? fl.seg_key[li.seg_first + li.n_multi + (c - li.n_slots)] : 0;
                }
                team_chunks<KS, 4>(fl, sl, on, lane, prev, cprev, Q, v);
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    if (v[k] != -__builtin_huge_val()) cur[d[k]] = (float)v[k];
                    my_max = fmax(my_max, v[k]);
                }
            }
            if (rank == 0) {
                __syncthreads();  // part[] complete (this member's own writes)
                for (int j = tid; j < li.n_multi; j += NT) {
                    const SegChunk sc = fl.seg_chunk[li.seg_first + j];
                    LseD acc{-__builtin_huge_val(), 0.0f};
                    for (int p = 0; p < sc.count; ++p) {  // chunks in order
                        const double x = part[sc.first + p];
                        if (x != -__builtin_huge_val()) lse_push_d(acc, x);
                    }
                    const double v = lse_value_d(acc);
                    if (v != -__builtin_huge_val()) cur[fl.seg_key[li.seg_first + j]] = (float)v;
                    my_max = fmax(my_max, v);
                }
            }
            block_max_d(my_max, &s_cmax, lane);
            __syncthreads();
            if (tid == 0) pmax[(t & 1) * G + rank] = unord_f64(s_cmax);
            if (!team_sync(tv, team, ++nbar, bv.health)) return;
            // the step max over all members (same order in every member)
            double c = -__builtin_huge_val();
            for (int r = 0; r < G; ++r) c = fmax(c, pmax[(t & 1) * G + r]);
            if (!(c > -__builtin_huge_val())) c = 0.0;
            C += c;
            // normalised tape: alpha^_t = stored - c_t on the destinations of w_t
            float *tape;
            if (bk.c > 0) {
                int blk;
                tape = ((bk.k & 1) ? bk.abuf[1] : bk.abuf[0]) + block_rel(bk, bv, b, o0, i, blk);
            } else if (tp.ck_off) {
                tape = tp.ck_off[i] >= 0 ? tp.alpha + tp.ck_off[i] : nullptr;
            } else {
                tape = tp.alpha + bv.tok_off[i];
            }
            if (tape) {
                const int stride = G * NT;
                for (int j = rank * NT + tid; j < li.n_segs; j += 4 * stride) {  // four in flight
                    int k[4];
                    float x[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) k[u] = j + u * stride < li.n_segs ? fl.seg_key[li.seg_first + j + u * stride] : Q;
#pragma unroll
                    for (int u = 0; u < 4; ++u) x[u] = cur[k[u]];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (j + u * stride < li.n_segs)
                            to_global(tape)[j + u * stride] = x[u] == WFST_NINF ? WFST_NINF : (float)((double)x[u] - c);
                }
            }
            if (rank == 0 && tid == 0 && bk.c == 0) {
                tp.a_max[i] = 0.0f;
                tp.a_log[i] = C;
            }
            cprev = c;
        }
        // log Z = C_T + LSE_q(alpha^_T[q] + f[q]) (members' partial sums combined in member order)
        if (bk.c == 0) {
            LseD acc{-__builtin_huge_val(), 0.0f};
            LabelInfo lf{};
            const float *fin = vbase + (int64_t)(t1 % 3) * tv.q1;
            if (T == 0) {
                if (rank == 0 && tid == 0) {
                    const float f = final_score[start];
                    if (f != WFST_NINF) acc = LseD{(double)f, 1.0f};
                }
            } else {
                lf = fl.label[bv.tokens[o1 - 1]];
                for (int j = rank * NT + tid; j < lf.n_segs; j += G * NT) {
                    const int d = fl.seg_key[lf.seg_first + j];
                    const float x = fin[d], f = final_score[d];
                    if (x == WFST_NINF || f == WFST_NINF) continue;
                    lse_push_d(acc, ((double)x - cprev) + (double)f);
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc = lse_merge_d(acc, LseD{__shfl_xor(acc.m, o, 64), __shfl_xor(acc.s, o, 64)});
            if (lane == 0) {
                s_rm[wave] = acc.m;
                s_rs[wave] = acc.s;
            }
            __syncthreads();
            if (tid == 0) {
                LseD tot{s_rm[0], s_rs[0]};
                for (int w = 1; w < NW; ++w) tot = lse_merge_d(tot, LseD{s_rm[w], s_rs[w]});
                pz[2 * rank] = tot.m;
                pz[2 * rank + 1] = (double)tot.s;
            }
            if (!team_sync(tv, team, ++nbar, bv.health)) return;
            if (rank == 0 && tid == 0) {
                LseD tot{pz[0], (float)pz[1]};
                for (int r = 1; r < G; ++r) tot = lse_merge_d(tot, LseD{pz[2 * r], (float)pz[2 * r + 1]});
                const double lzr = lse_value_d(tot);
                if (lzr == -__builtin_huge_val()) {
                    bv.status[b] = WFST_STATUS_NO_PATH;
                    log_z_out[b] = WFST_NINF;
                    tp.log_z[b] = -__builtin_huge_val();
                } else {
                    const double lz = C + lzr;
                    bv.status[b] = WFST_STATUS_OK;
                    log_z_out[b] = (float)lz;
                    tp.log_z[b] = lz;
                }
            }
        }
        // restore the invariant: clear the supports of alpha_{t1-1} and alpha_{t1}
        for (int back = 0; back < 2; ++back) {
            const int tt = t1 - back;
            if (tt < t0) break;
            float *v = vbase + (int64_t)(tt % 3) * tv.q1;
            if (tt == 0) {
                if (rank == 0 && tid == 0) v[start] = WFST_NINF;
            } else {
                int t_first = lc_first, t_n = lc_n;
                if (tt > t0) {
                    const LabelInfo lt = fl.label[bv.tokens[o0 + tt - 1]];
                    t_first = lt.seg_first;
                    t_n = lt.n_segs;
                }
                team_clear(v, fl.seg_key + t_first, rank * NT + tid, t_n, G * NT);
            }
        }
        if (!team_sync(tv, team, ++nbar, bv.health)) return;
    }
}

// Backward pass (paper, Algorithm 2 second loop, with the index typos fixed):
// beta_{t-1}[s] = LSE over the arcs k with input w_t leaving s of
// theta_k + beta_t[dst_k].  beta_{t-1} is only ever read on the states
// alpha_{t-1} can occupy -- the destinations of w_{t-1} (the start state at
// t = 1): the expected counts pair it with alpha_{t-1}, and step t-1 reads
// beta_{t-1} only at destinations of w_{t-1}.  So each step marks those
// states, scans the reverse segments of w_t (one per source state) for marked
// sources, and reduces just those segments, one thread per segment with its
// arcs in layout order.  The values on the marked states are the sums a full
// sweep computes; only the per-step normaliser (the max over the computed
// states) is taken over fewer states.  The next step's labels and segment keys
// are loaded while the current step runs.
constexpr int kSliceCache = 32;  // slice headers of the step's label staged in LDS

constexpr int rev_key_prefetch(int nt) { return nt >= 1024 ? 3 : nt >= 512 ? 5 : 9; }
// What a backward step needs besides its keys, staged in LDS for kBwdWin
// steps at a time (a ring indexed by step): the loads of a step's keys and
// alpha values then wait on no other global load.
constexpr int kBwdWin = 8;
// Reserve `mine` consecutive slots per lane at an LDS counter with one atomic
// per wavefront: returns the lane's first slot.  Called by the lanes active at
// that point (inactive lanes take no slots); the lowest active lane does the
// atomic.  mine < 16.
__device__ __forceinline__ int wave_append(int mine, int *counter, int lane)
{
    int pre = 0, total = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {  // exclusive prefix of mine over the lower lanes, bit by bit
        const uint64_t m = __ballot((mine >> k) & 1);
        pre += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << k;
        total += __popcll(m) << k;
    }
    const int leader = __builtin_ctzll(__ballot(1));
    int base = 0;
    if (lane == leader && total > 0) base = atomicAdd(counter, total);
    return __shfl(base, leader, 64) + pre;
}
static_assert(sizeof(SliceInfo) == sizeof(int4), "slice headers move as int4");
typedef int v4i __attribute__((ext_vector_type(4)));
struct BwdStep {
    int32_t slice_first, n_slices, seg_first, n_segs, n_multi, n_slots;  // reverse label of w_t
    int32_t f_seg_first, f_n_segs;  // forward label of w_{t-1} (none at t = 1)
    const float *ap;                // alpha~ of token i-1 (with records)
    float *bp;                      // beta tape slot of token i
    double aC;                      // log scale of alpha_{t-1}
    float cm;                       // c_{t-1}
    int32_t pad;
};
__device__ __forceinline__ int32_t uniform_i(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
template <class T>
__device__ __forceinline__ T *uniform_p(T *p)
{
    const uint64_t u = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}
constexpr int kTapeKeyPrefetch = 2;
// Expected-count records: a step's records are staged in LDS, then copied to a
// chunk of the record array the workgroup owns; chunks come from one global
// counter, and a chunk's unused tail is filled with sentinel keys (sorted last,
// skipped when summing).
constexpr int kRecStage = 64;
constexpr int kRecChunk = 256;
static_assert(kRecStage <= kRecChunk, "one step's staged records fit a chunk");
constexpr uint64_t kRecSentinel = ~0ull;
// Zero-fill of the gradient inside the sweep: workgroup w writes slabs w,
// w + G, w + 2G, ... (G workgroups) of 8 floats per thread, one slab at the
// end of each step (stores issued after the step's loads, so no load waits on
// them), the rest when its queue is empty.  rs.fill is 16-byte aligned;
// streaming stores, so that the fill does not evict layout lines from L2.
constexpr int kFillPerThread = 8;
__device__ __forceinline__ void fill_gradient_slab(const RecordSink &rs, int64_t slab_first, int tid)
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    const int64_t x = slab_first + kFillPerThread * (int64_t)tid;
    if (x + kFillPerThread <= rs.fill_n) {
        v4f *q = reinterpret_cast<v4f *>(rs.fill + x);
        __builtin_nontemporal_store((v4f){0.0f, 0.0f, 0.0f, 0.0f}, q);
        __builtin_nontemporal_store((v4f){0.0f, 0.0f, 0.0f, 0.0f}, q + 1);
    } else {
        for (int64_t y = x; y < rs.fill_n; ++y) __builtin_nontemporal_store(0.0f, rs.fill + y);
    }
}

// The step table of a backward launch: entry i describes the step of token i
// (step t = i - o0 + 1 of its sentence).  Built in parallel over the tokens
// just before the sweep, after the forward pass wrote the alpha scales; in a
// checkpointed pass only the launch's block is filled (its tape slots).
__global__ void bwd_step_table(DevLayout fl, DevLayout rl, BatchView bv, TapeView tp, BlockView bk, int32_t rec,
                               BwdStep *__restrict__ out)
{
    for (int b = blockIdx.x; b < bv.B; b += gridDim.x) {
        if (bv.status[b] != WFST_STATUS_OK) continue;  // offsets and tokens checked by the forward pass
        const int o0 = bv.offsets[b], T = bv.offsets[b + 1] - o0;
        int lo = 0, hi = T;
        if (bk.c > 0) {
            lo = bk.k * bk.c;
            hi = min(T, lo + bk.c);
        }
        for (int ts = lo + 1 + (int)threadIdx.x; ts <= hi; ts += blockDim.x) {
            const int is = o0 + ts - 1;
            const LabelInfo r = rl.label[bv.tokens[is]];
            BwdStep e;
            e.slice_first = r.slice_first;
            e.n_slices = r.n_slices;
            e.seg_first = r.seg_first;
            e.n_segs = r.n_segs;
            e.n_multi = r.n_multi;
            e.n_slots = r.n_slots;
            e.f_seg_first = e.f_n_segs = e.pad = 0;
            e.ap = nullptr;
            e.bp = beta_slot(tp, bk, bv, b, o0, is);
            e.aC = 0.0;
            e.cm = 0.0f;
            if (ts >= 2) {
                const LabelInfo f = fl.label[bv.tokens[is - 1]];
                e.f_seg_first = f.seg_first;
                e.f_n_segs = f.n_segs;
                if (rec) {
                    e.ap = alpha_slot(tp, bk, bv, b, o0, is - 1);
                    e.cm = tp.a_max[is - 1];
                    e.aC = tp.a_log[is - 1];
                }
            }
            out[is] = e;
        }
    }
}

// Copy the records placed at the end of the previous step (and sentinels into
// a chunk tail left behind) from the LDS stage to the record array.
__device__ __forceinline__ void copy_staged_records(const RecordSink &rs, const uint64_t *stage_key,
                                                    const float *stage_val, int n, unsigned long long base,
                                                    int tail_n, unsigned long long tail_base, int tid, int nt)
{
    for (int x = tid; x < n; x += nt) {
        const unsigned long long g = base + x;
        if (g < (unsigned long long)rs.cap) {
            rs.key[g] = stage_key[x];
            rs.val[g] = stage_val[x];
        }
    }
    for (int x = tid; x < tail_n; x += nt) {
        const unsigned long long g = tail_base + x;
        if (g < (unsigned long long)rs.cap) rs.key[g] = kRecSentinel;
    }
}

template <int NT, bool GMEM>
__global__ void __launch_bounds__(NT, GMEM ? 1 : 4)  // on chip: at most 128 VGPRs, four wavefronts per SIMD
backward_sweep(DevLayout fl, DevLayout rl, int32_t Q, int32_t start,
               const float *__restrict__ final_score, const float *__restrict__ final_max,
               BatchView bv, TapeView tp, BlockView bk, int32_t list_cap, RecordSink rs,
               const BwdStep *__restrict__ steps, unsigned char *__restrict__ gscratch, int64_t slot_bytes)
{
    constexpr int RPF = rev_key_prefetch(NT);
    constexpr int TPF = kTapeKeyPrefetch;
    constexpr int RB = 4;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *smem = state_base<GMEM>(lds, gscratch, slot_bytes);
    __shared__ __align__(16) SliceInfo scache[kSliceCache];            // slice headers of the step's label
    __shared__ BwdStep s_win[kBwdWin];                                 // step metadata ring
    float *val0 = reinterpret_cast<float *>(smem);                     // [Q+1]
    float *val1 = val0 + (Q + 1);                                      // [Q+1]
    float *aval = val1 + (Q + 1);                                      // [Q+1] alpha~_{t-1} - c_{t-1} there
    int2 *list = reinterpret_cast<int2 *>(smem + ((12 * (int64_t)(Q + 1) + 7) & ~(int64_t)7));  // [list_cap] {segment, key}
    double *lval = reinterpret_cast<double *>(list + list_cap);        // [list_cap] unnormalised value
    uint16_t *mark = reinterpret_cast<uint16_t *>(lval + list_cap);    // [Q+1] step stamp of states to compute
    __shared__ int s_item, s_count;
    __shared__ unsigned long long s_cmax[3];
    __shared__ uint64_t s_rkey[kRecStage];
    __shared__ float s_rval[kRecStage];
    __shared__ int s_rn, s_rflush, s_cused, s_csize, s_tailn;
    __shared__ unsigned long long s_cbase, s_fbase, s_tailb, s_rtotal;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const float fmax0 = *final_max;
    // raw buffer view of the reverse slice headers (word 3: 32-bit data format, the gfx9 encoding)
    const __amdgpu_buffer_rsrc_t slice_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)rl.slice, (short)0, (int)min<int64_t>(rl.n_slice * (int64_t)sizeof(SliceInfo), INT32_MAX), 0x00020000);
    const double fx = rs.acc ? *rs.fx_scale : 0.0;  // fixed-point scale of the accumulators
    const int64_t fill_slab = (int64_t)kFillPerThread * NT;  // floats per gradient slab (rs.fill)
    int64_t fill_at = (int64_t)blockIdx.x * fill_slab;       // next slab of this workgroup
    const int64_t fill_stride = (int64_t)gridDim.x * fill_slab;
    if (tid == 0) {
        s_rn = 0;
        s_cbase = 0;
        s_rtotal = 0;
        s_rflush = s_tailn = 0;  // nothing staged to copy
        s_cused = s_csize = 0;   // no chunk yet
    }

    for (int pops = 0;; ++pops) {
        if (tid == 0) s_item = atomicAdd(bv.queue, 1);
        __syncthreads();
        const int item = wave_uniform(s_item);  // uniform: the sentence's loads go through the scalar unit
        __syncthreads();
        if (item >= bv.B) break;
        if (item < 0 || pops > bv.B) {
            if (tid == 0) atomicOr(bv.health, H_QUEUE);
            break;
        }
        const int b = bv.order[item];
        if (bv.status[b] != WFST_STATUS_OK) continue;
        const int o0 = bv.offsets[b], o1 = bv.offsets[b + 1];
        const int T = o1 - o0;
        if (T == 0) {
            if (tid == 0 && bk.k == 0) tp.log_z_bwd[b] = (double)final_score[start];
            continue;
        }
        int t0 = 0, t1 = T;  // steps t1 down to t0+1
        if (bk.c > 0) {
            t0 = bk.k * bk.c;
            t1 = min(T, t0 + bk.c);
            if (t1 <= t0) continue;
        }
        float *vT = (t1 & 1) ? val1 : val0;
        float *vO = (t1 & 1) ? val0 : val1;
        for (int q = tid; q <= Q; q += NT) {  // beta^_T = f - max f, with C = max f
            const float f = q < Q ? final_score[q] : WFST_NINF;
            vT[q] = (t1 == T && f != WFST_NINF) ? f - fmax0 : WFST_NINF;
            vO[q] = WFST_NINF;
            mark[q] = 0;  // no step's stamp
        }
        __syncthreads();
        double C;  // log scale: log beta_t = beta^_t + C_t
        if (t1 == T) {
            // beta^_T on the destinations of w_T, for the expected counts
            const LabelInfo lf = fl.label[bv.tokens[o1 - 1]];
            gfloat *tape = to_global(beta_slot(tp, bk, bv, b, o0, o1 - 1));
            for (int j = tid; j < lf.n_segs; j += NT) tape[j] = vT[fl.seg_key[lf.seg_first + j]];
            if (tid == 0) {
                tp.b_max[o1 - 1] = 0.0f;
                tp.b_log[o1 - 1] = (double)fmax0;
            }
            C = (double)fmax0;
        } else {  // resume from beta^_{t1} kept by the previous (later) block
            const int i1 = o0 + t1 - 1;
            const LabelInfo lf = fl.label[bv.tokens[i1]];
            const gfloat *tape = to_global(beta_slot(tp, bk, bv, b, o0, i1));
            for (int j = tid; j < lf.n_segs; j += NT) vT[fl.seg_key[lf.seg_first + j]] = tape[j];
            C = tp.b_log[i1];
        }
        if (tid < 3) s_cmax[tid] = 0u;
        const bool rec = rs.key != nullptr || rs.acc != nullptr;  // posteriors of the visits wanted
        const bool stage = rs.key != nullptr;                       // ... as records
        const float gb = rs.grad_log_z ? rs.grad_log_z[b] : 1.0f;
        const double lz = tp.log_z[b];

        // metadata of steps t1, t1-1, ... staged in LDS; keys, alpha values
        // and slice headers of a step loaded one step ahead
        auto fill_window = [&](int thi) {  // entries of steps thi, thi-1, ... (one load each)
            if (tid < kBwdWin && thi - tid > t0) s_win[(thi - tid) & (kBwdWin - 1)] = steps[o0 + thi - tid - 1];
        };
        fill_window(t1);
        int w_lo = max(t0 + 1, t1 - kBwdWin + 1);  // lowest step in the ring
        __syncthreads();
        LabelInfo li{};  // reverse label of w_t
        int lf_first, lf_n;   // forward label of w_{t-1}: the states to compute
        const gfloat *ap;     // alpha~_{t-1} (records)
        gfloat *bp;           // beta tape slot of token i
        float cm;             // c_{t-1}
        double aC;            // log scale of alpha_{t-1}
        {
            const BwdStep &e = s_win[t1 & (kBwdWin - 1)];
            li.slice_first = uniform_i(e.slice_first);
            li.n_slices = uniform_i(e.n_slices);
            li.seg_first = uniform_i(e.seg_first);
            li.n_segs = uniform_i(e.n_segs);
            li.n_multi = uniform_i(e.n_multi);
            li.n_slots = uniform_i(e.n_slots);
            lf_first = uniform_i(e.f_seg_first);
            lf_n = uniform_i(e.f_n_segs);
            ap = to_global(uniform_p(e.ap));
            bp = to_global(uniform_p(e.bp));
            cm = e.cm;
            aC = e.aC;
        }
        int rk[RPF];  // segment keys of li (source states)
        int tk[TPF];  // keys of lf
        float ta[TPF];  // alpha~_{t-1} on them (records only; normaliser cm subtracted at use)
        int4 sl = make_int4(0, 0, 0, 0);  // slice header tid of li (a SliceInfo)
#pragma unroll
        for (int u = 0; u < RPF; ++u) {
            const int j = tid + u * NT;
            rk[u] = j < li.n_segs ? rl.seg_key[li.seg_first + j] : -1;
        }
#pragma unroll
        for (int u = 0; u < TPF; ++u) {
            const int j = tid + u * NT;
            tk[u] = j < lf_n ? fl.seg_key[lf_first + j] : -1;
            ta[u] = rec && j < lf_n ? ap[j] : WFST_NINF;
        }
        if (tid < min(li.n_slices, kSliceCache)) sl = reinterpret_cast<const int4 *>(rl.slice)[li.slice_first + tid];
        int lfp_first = 0, lfp_n = 0;  // forward label of w_t: support of beta~_t, reset after the step
        int tk_prev[TPF];
#pragma unroll
        for (int u = 0; u < TPF; ++u) tk_prev[u] = -1;

        for (int t = t1; t > t0; --t) {
            float *prev = (t & 1) ? val1 : val0;  // beta~_t
            float *cur = (t & 1) ? val0 : val1;   // beta~_{t-1}
            const int i = o0 + t - 1;
            // A: mark the states of step t-1 (with alpha~_{t-1} for the records),
            // stage the slice headers of w_t.  Stamps are 16-bit, (t - 1) % 65535 + 1:
            // every step t divisible by 65535 first clears them all, so no stamp of a
            // step 65535 or more later survives to look like this step's.
            const uint16_t stamp = (uint16_t)((t - 1) % 65535 + 1);
            if (t % 65535 == 0) {  // uniform (t is)
                for (int q = tid; q <= Q; q += NT) mark[q] = 0;
                __syncthreads();
            }
            if (t >= 2) {
#pragma unroll
                for (int u = 0; u < TPF; ++u)
                    if (tk[u] >= 0) {
                        mark[tk[u]] = stamp;
                        aval[tk[u]] = ta[u] - cm;
                    }
                for (int j = tid + TPF * NT; j < lf_n; j += NT) {
                    const int q = fl.seg_key[lf_first + j];
                    mark[q] = stamp;
                    aval[q] = rec ? ap[j] - cm : WFST_NINF;
                }
            } else if (tid == 0) {
                mark[start] = stamp;
                aval[start] = 0.0f;  // alpha~_0 = 0 at the start state, no normaliser
            }
            const float o = rec ? (float)((t >= 2 ? aC : 0.0) + C - lz) : 0.0f;  // C = log scale of beta_t
            if (tid < min(li.n_slices, kSliceCache)) reinterpret_cast<int4 *>(scache)[tid] = sl;
            if (tid == 0) s_count = 0;
            __syncthreads();
            // B, first half: which reverse segments of w_t have a marked source
            // (before the next step's loads are issued: waiting for rk must not
            // wait for them)
            uint32_t hits = 0;
#pragma unroll
            for (int u = 0; u < RPF; ++u)
                if (rk[u] >= 0 && mark[rk[u]] == stamp) hits |= 1u << u;
            if (stage) copy_staged_records(rs, s_rkey, s_rval, s_rflush, s_fbase, s_tailn, s_tailb, tid, NT);
            if (t < t1) {  // tape of beta^_t (this step's input), normalised at the end of step t+1
#pragma unroll
                for (int u = 0; u < TPF; ++u)
                    if (tk_prev[u] >= 0) bp[tid + u * NT] = prev[tk_prev[u]];
                for (int j = tid + TPF * NT; j < lfp_n; j += NT) bp[j] = prev[fl.seg_key[lfp_first + j]];
            }
            // next step's metadata from the ring (refilled every kBwdWin steps;
            // every thread read the entries it replaces before this step's
            // barrier), its keys, alpha values and slice headers in flight
            // during this step
            if (t - 1 > t0 && t - 1 < w_lo) {
                fill_window(t - 1);
                w_lo = max(t0 + 1, t - kBwdWin);
                __syncthreads();
            }
            LabelInfo li_n{};
            int lf_first_n = 0, lf_n_n = 0;
            const gfloat *ap_n = nullptr;
            gfloat *bp_n = nullptr;
            float cm_n = 0.0f;
            double aC_n = 0.0;
            int rk_n[RPF], tk_n[TPF];
            float ta_n[TPF];
            int4 sl_n = make_int4(0, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < RPF; ++u) rk_n[u] = -1;
#pragma unroll
            for (int u = 0; u < TPF; ++u) {
                tk_n[u] = -1;
                ta_n[u] = WFST_NINF;
            }
            if (t - 1 > t0) {
                const BwdStep &e = s_win[(t - 1) & (kBwdWin - 1)];
                li_n.slice_first = uniform_i(e.slice_first);
                li_n.n_slices = uniform_i(e.n_slices);
                li_n.seg_first = uniform_i(e.seg_first);
                li_n.n_segs = uniform_i(e.n_segs);
                li_n.n_multi = uniform_i(e.n_multi);
                li_n.n_slots = uniform_i(e.n_slots);
                lf_first_n = uniform_i(e.f_seg_first);
                lf_n_n = uniform_i(e.f_n_segs);
                ap_n = to_global(uniform_p(e.ap));
                bp_n = to_global(uniform_p(e.bp));
                cm_n = e.cm;
                aC_n = e.aC;
#pragma unroll
                for (int u = 0; u < RPF; ++u) {
                    const int j = tid + u * NT;
                    if (j < li_n.n_segs) rk_n[u] = rl.seg_key[li_n.seg_first + j];
                }
#pragma unroll
                for (int u = 0; u < TPF; ++u) {
                    const int j = tid + u * NT;
                    if (j < lf_n_n) {
                        tk_n[u] = fl.seg_key[lf_first_n + j];
                        if (rec) ta_n[u] = ap_n[j];
                    }
                }
                if (tid < min(li_n.n_slices, kSliceCache))
                    sl_n = reinterpret_cast<const int4 *>(rl.slice)[li_n.slice_first + tid];
            }
            // B, second half: the marked segments compacted with one LDS atomic
            // per wavefront (list order does not matter: each entry is reduced
            // on its own)
            {
                const int mine = __popc(hits);
                const int pos0 = wave_append(mine, &s_count, lane);
                int pos = pos0;
#pragma unroll
                for (int u = 0; u < RPF; ++u)
                    if (hits >> u & 1u) {
                        if (pos < list_cap) list[pos] = make_int2(tid + u * NT, rk[u]);
                        ++pos;
                    }
            }
            for (int j = tid + RPF * NT; j < li.n_segs; j += NT) {
                const int key = rl.seg_key[li.seg_first + j];
                if (mark[key] == stamp) {
                    const int pos = atomicAdd(&s_count, 1);
                    if (pos < list_cap) list[pos] = make_int2(j, key);
                }
            }
            __syncthreads();
            int n = s_count;
            if (n > list_cap) {
                if (tid == 0) atomicOr(bv.health, H_GROUP);
                n = list_cap;
            }
            // C: one thread per marked segment, its chunks and rows in layout order
            double my_max = -__builtin_huge_val();
            for (int x = tid; x < n; x += NT) {
                const int2 jk = list[x];
                const int j = jk.x;
                int c0, nc;
                if (j < li.n_multi) {
                    const SegChunk sc = rl.seg_chunk[li.seg_first + j];
                    c0 = sc.first;
                    nc = sc.count;
                } else {
                    c0 = li.n_slots + (j - li.n_multi);
                    nc = 1;
                }
                const float a = rec ? aval[jk.y] : WFST_NINF;  // alpha^_{t-1} at the source
                LseD acc{-__builtin_huge_val(), 0.0f};
                for (int c = c0; c < c0 + nc; ++c) {
                    const int s = c >> 6, l = c & 63;
                    // the slice header: from the LDS cache, else by a buffer load (a plain
                    // global load here would be merged with the LDS read into a generic one)
                    v4i sv;
                    if (s < kSliceCache)
                        sv = reinterpret_cast<const v4i *>(scache)[s];
                    else
                        sv = __builtin_amdgcn_raw_buffer_load_b128(slice_rsrc, (li.slice_first + s) * (int)sizeof(SliceInfo),
                                                                  0, 0);
                    const SliceInfo si{sv.x, sv.y, sv.z, sv.w};
                    for (int r0 = 0; r0 < si.height; r0 += RB) {
                        Elem e[RB];
                        int32_t slot_of[RB];  // reverse-layout slots, for the posteriors
#pragma unroll
                        for (int u = 0; u < RB; ++u) {  // no branches: all RB loads in flight together
                            const int pos = si.base + min(r0 + u, si.height - 1) * si.width + l;
                            const int32_t o = rl.other[pos];
                            const float sc = rl.score[pos];
                            slot_of[u] = pos;
                            e[u] = r0 + u < si.height ? Elem{o, sc} : Elem{Q, 0.0f};
                        }
                        float g[RB];
#pragma unroll
                        for (int u = 0; u < RB; ++u) g[u] = prev[e[u].other];
                        lse_push_terms<RB>(acc, g, e);
                        if (a != WFST_NINF) {
                            // posterior of each arc at this visit, as the count kernel forms it
                            float v[RB];
                            int nrec = 0;
#pragma unroll
                            for (int u = 0; u < RB; ++u) {
                                v[u] = 0.0f;
                                if (g[u] != WFST_NINF) v[u] = gb * exp_e((a + e[u].score) + (g[u] + o));
                                nrec += v[u] != 0.0f;
                            }
                            if (nrec > 0 && !stage) {
#pragma unroll
                                for (int u = 0; u < RB; ++u) {
                                    // posteriors that round to 0 at the accumulators' scale add nothing
                                    const long long q = __double2ll_rn((double)v[u] * fx);
                                    if (q == 0) continue;
                                    atomicAdd(&rs.acc[slot_of[u]], (unsigned long long)q);
                                }
                            } else if (nrec > 0) {
                                int at = wave_append(nrec, &s_rn, lane);
#pragma unroll
                                for (int u = 0; u < RB; ++u) {
                                    if (v[u] == 0.0f) continue;
                                    const uint64_t key = ((uint64_t)(uint32_t)slot_of[u] << 32) | (uint32_t)i;
                                    if (at < kRecStage) {
                                        s_rkey[at] = key;
                                        s_rval[at] = v[u];
                                    } else {  // more than the stage holds: straight to the record array
                                        const unsigned long long g = atomicAdd(rs.count, 1ull);
                                        if (g < (unsigned long long)rs.cap) {
                                            rs.key[g] = key;
                                            rs.val[g] = v[u];
                                        }
                                    }
                                    ++at;
                                }
                            }
                        }
                    }
                }
                const double v = lse_value_d(acc);
                lval[x] = v;
                my_max = fmax(my_max, v);
            }
            if (tid == 0) s_cmax[(t + 1) % 3] = 0ull;
            block_max_d(my_max, &s_cmax[t % 3], lane);
            __syncthreads();
            double c = unord_f64(s_cmax[t % 3]);
            if (!(c > -__builtin_huge_val())) c = 0.0;
            // beta^_{t-1} = beta_{t-1} - c (read by the next step after its first barrier)
            for (int x = tid; x < n; x += NT) {
                const double v = lval[x];
                cur[list[x].y] = v == -__builtin_huge_val() ? WFST_NINF : (float)(v - c);
                if (t == 1 && list[x].y == start)
                    tp.log_z_bwd[b] = v == -__builtin_huge_val() ? -__builtin_huge_val() : C + v;
            }
            C += c;
            if (stage && tid == 0) {  // place the step's staged records in the workgroup's chunk (copied next step)
                const int n = min(s_rn, kRecStage);
                s_rtotal += (unsigned long long)s_rn;
                s_rflush = n;
                s_tailn = 0;
                if (n > 0) {
                    if (s_cused + n > s_csize) {  // new chunk; the old one's unused tail gets sentinels
                        s_tailb = s_cbase + s_cused;
                        s_tailn = s_csize - s_cused;
                        s_cbase = atomicAdd(rs.count, (unsigned long long)kRecChunk);
                        s_csize = kRecChunk;
                        s_cused = 0;
                    }
                    s_fbase = s_cbase + s_cused;
                    s_cused += n;
                }
                s_rn = 0;
            }
            // no thread reads beta~_t any more: clear its support (everything at
            // the first step); the buffer is written again after the next step's
            // first barrier
            if (t == t1) {
                for (int q = tid; q < Q; q += NT) prev[q] = WFST_NINF;
            } else {
#pragma unroll
                for (int u = 0; u < TPF; ++u)
                    if (tk_prev[u] >= 0) prev[tk_prev[u]] = WFST_NINF;
                for (int j = tid + TPF * NT; j < lfp_n; j += NT) prev[fl.seg_key[lfp_first + j]] = WFST_NINF;
            }
            if (rs.fill && fill_at < rs.fill_n) {  // this workgroup's next gradient slab
                fill_gradient_slab(rs, fill_at, tid);
                fill_at += fill_stride;
            }
            if (t >= 2 && tid == 0) {
                tp.b_max[i - 1] = 0.0f;  // the tape is normalised
                tp.b_log[i - 1] = C;
            }
            lfp_first = lf_first;
            lfp_n = lf_n;
#pragma unroll
            for (int u = 0; u < TPF; ++u) tk_prev[u] = tk[u];
            li = li_n;
            lf_first = lf_first_n;
            lf_n = lf_n_n;
            ap = ap_n;
            bp = bp_n;
            aC = aC_n;
            cm = cm_n;
            sl = sl_n;
#pragma unroll
            for (int u = 0; u < RPF; ++u) rk[u] = rk_n[u];
#pragma unroll
            for (int u = 0; u < TPF; ++u) {
                tk[u] = tk_n[u];
                ta[u] = ta_n[u];
            }
        }
        __syncthreads();
        if (t0 >= 1) {  // tape of beta^_{t0}, the last step's output (a block boundary)
            float *fin = ((t0 + 1) & 1) ? val0 : val1;
            gfloat *tape = to_global(beta_slot(tp, bk, bv, b, o0, o0 + t0 - 1));
#pragma unroll
            for (int u = 0; u < TPF; ++u)
                if (tk_prev[u] >= 0) tape[tid + u * NT] = fin[tk_prev[u]];
            for (int j = tid + TPF * NT; j < lfp_n; j += NT) tape[j] = fin[fl.seg_key[lfp_first + j]];
        }
        __syncthreads();
    }
    // the rest of the gradient fill; the records staged by the last step, the
    // unused tail of the last chunk, and the workgroup's record count
    __syncthreads();
    if (rs.fill)
        for (; fill_at < rs.fill_n; fill_at += fill_stride) fill_gradient_slab(rs, fill_at, tid);
    if (rs.key != nullptr) {
        copy_staged_records(rs, s_rkey, s_rval, s_rflush, s_fbase, s_tailn, s_tailb, tid, NT);
        for (int x = s_cused + tid; x < s_csize; x += NT) {
            const unsigned long long g = s_cbase + x;
            if (g < (unsigned long long)rs.cap) rs.key[g] = kRecSentinel;
        }
        if (tid == 0 && s_rtotal > 0) atomicAdd(rs.total, s_rtotal);
    }
}

// =====================================================================
// Expected counts (paper, Algorithm 2 last loop): grouped by input label so
// that each arc's sum over the visits of its label is taken in a fixed
// order, without atomics.
// =====================================================================

struct CEnt {
    float v;
    int32_t stamp;
};

struct CountItem {
    int32_t first, last;  // range in the label-sorted visit list
    int32_t label;
    int32_t split;        // 1 when its group (label, block) has several items: partial sums + fixup
    int32_t block;        // checkpoint block of its visits (0 without checkpointing)
    int32_t carry;        // 1 when the label had items in a block processed earlier: sums continue from grad
};

// Everything the count kernel needs about one visit (sentence b, step t,
// token i), in one record: posterior of arc k at this visit is
//   g * exp((alpha~_{t-1}[src_k] - cm) + score_k + (beta~_t[dst_k] - bm) + o).
struct VisitInfo {
    const float *a_ptr;  // compact alpha~ of step t-1 (token i-1)
    const float *b_ptr;  // compact beta~ of step t (token i)
    int32_t prev_label;  // label of token i-1, -1 at t = 1 (alpha_0 = start)
    int32_t live;        // 0: sentence without a path (or invalid): skip
    float o, cm, bm, g;
};

// One thread per visit position of the label-sorted list.
__global__ void visit_table(BatchView bv, TapeView tp, BlockView bk, const int32_t *__restrict__ visits,
                            const int32_t *__restrict__ tok_sent, const float *__restrict__ grad_log_z,
                            VisitInfo *__restrict__ out)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < bv.N; v += (int64_t)gridDim.x * blockDim.x) {
        VisitInfo vi{};
        vi.prev_label = -1;
        const int i = visits[v];
        bool ok = i >= 0 && (int64_t)i < bv.N;
        const int b = ok ? tok_sent[i] : 0;
        ok = ok && b >= 0 && b < bv.B;
        int o0 = 0;
        if (ok) {
            o0 = bv.offsets[b];
            ok = i >= o0 && i < bv.offsets[b + 1];
        }
        if (!ok) atomicOr(bv.health, H_VISIT);
        if (ok && bv.status[b] == WFST_STATUS_OK) {
            const int t = i - o0 + 1;
            const double aC = t > 1 ? tp.a_log[i - 1] : 0.0;
            vi.o = (float)(aC + tp.b_log[i] - tp.log_z[b]);
            vi.cm = t > 1 ? tp.a_max[i - 1] : 0.0f;
            vi.bm = tp.b_max[i];
            vi.g = grad_log_z ? grad_log_z[b] : 1.0f;
            vi.a_ptr = t > 1 ? alpha_slot(tp, bk, bv, b, o0, i - 1) : nullptr;
            vi.b_ptr = beta_slot(tp, bk, bv, b, o0, i);
            vi.prev_label = t > 1 ? bv.tokens[i - 1] : -1;
            vi.live = 1;
        }
        out[v] = vi;
    }
}

// Expected counts (paper, Algorithm 2 last loop), grouped by input label so
// that each arc's sum over the visits of its label is taken in a fixed order,
// without atomics.  A work item is one label and up to V of its visits;
// workgroups pop items from a queue (heaviest labels come first).  The
// label's arcs are walked in the reverse layout: every lane chunk belongs to
// one source state, so one lookup of alpha_{t-1} at that source decides
// whether any of the chunk's arcs has a nonzero posterior at this visit; a
// slice whose 64 sources are all dead is skipped after one ballot.  Arcs
// skipped this way would add exactly +0, so the sums equal the dense ones.
// Per visit, alpha_{t-1} is scattered into a stamped dense LDS vector and
// beta_t (with its normaliser and the visit's scale offset folded in) into an
// LDS vector over the label's destinations; both are loaded one visit ahead.
// CH bounds the slice height; each lane keeps KPP * CH <= 64 accumulators in
// registers, so one pass covers KPP slices per wavefront and labels with more
// slices take several passes over their visits.
constexpr int count_slices_per_wave(int ch) { return 64 / ch < 8 ? 64 / ch : 8; }
// alpha and beta entries per thread carried to the next visit (512 threads
// cover the destinations of a trigram tagger's label in one round)
constexpr int count_prefetch(int nt) { return nt >= 512 ? 1 : 2; }

template <int PF>
struct VisitVals {
    int key[PF];    // alpha_{t-1}: state (-1: none)
    float aval[PF];
    float bval[PF]; // (beta~_t[j] - b_max) + offset for j = tid + u * NT
};

template <int NT, int PF = count_prefetch(NT)>
__device__ __forceinline__ void fetch_visit(const DevLayout &fl, const TapeView &tp, const VisitInfo &vi,
                                            int32_t start, int n_dst, int tid, VisitVals<PF> &x)
{
    constexpr int kPrefetch = PF;
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) x.key[u] = -1;
    if (!vi.live) return;
    const gfloat *tb = to_global(vi.b_ptr);
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
        const int j = tid + u * NT;
        if (j < n_dst) x.bval[u] = (tb[j] - vi.bm) + vi.o;
    }
    if (vi.prev_label < 0) {
        if (tid == 0) {
            x.key[0] = start;
            x.aval[0] = 0.0f;
        }
        return;
    }
    const LabelInfo lp = fl.label[vi.prev_label];
    const gfloat *ta = to_global(vi.a_ptr);
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
        const int j = tid + u * NT;
        if (j < lp.n_segs) {
            x.key[u] = fl.seg_key[lp.seg_first + j];
            x.aval[u] = ta[j] - vi.cm;
        }
    }
}

template <int NT, int CH>
__global__ void __launch_bounds__(NT)
counts_kernel(DevLayout fl, DevLayout rl, int32_t Q, int32_t start, BatchView bv, TapeView tp,
              const CountItem *__restrict__ items, const int32_t *__restrict__ n_items,
              const int32_t *__restrict__ item_list, const int32_t *__restrict__ list_off, int32_t blk,
              int32_t *__restrict__ item_queue, const VisitInfo *__restrict__ vinfo,
              float *__restrict__ grad, float *__restrict__ partial, int32_t *__restrict__ item_slot,
              int32_t *__restrict__ slot_counter, CountCaps caps)
{
    constexpr int NW = NT / 64;
    constexpr int KPP = count_slices_per_wave(CH);
    constexpr int MAXR = KPP * CH;
    constexpr int kPrefetch = count_prefetch(NT);
    extern __shared__ __align__(16) unsigned char smem[];
    CEnt *den0 = reinterpret_cast<CEnt *>(smem);
    CEnt *den1 = den0 + (Q + 1);
    int32_t *fmap = reinterpret_cast<int32_t *>(den1 + (Q + 1));  // [Q] state -> forward segment of the label
    float *bden = reinterpret_cast<float *>(fmap + Q);              // [2][max forward segments]
    int32_t *chunk_seg = reinterpret_cast<int32_t *>(bden + 2 * fl.max_segs);  // reverse chunk -> segment
    __shared__ int s_item, s_slot;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);
    for (int q = tid; q <= Q; q += NT) {
        den0[q] = CEnt{WFST_NINF, -1};
        den1[q] = CEnt{WFST_NINF, -1};
    }
    int nit = *n_items, lo = 0;  // items [lo, lo + nit) of the list (or of all items)
    if (item_list) {
        lo = list_off[blk];
        int hi = list_off[blk + 1];
        if (lo < 0 || hi < lo || hi > nit) {
            if (blockIdx.x == 0 && tid == 0) atomicOr(bv.health, H_ITEM);
            lo = hi = 0;
        }
        nit = hi - lo;
    }
    if (nit < 0 || nit > caps.items_cap) {
        if (blockIdx.x == 0 && tid == 0) atomicOr(bv.health, H_ITEM);
        nit = 0;
    }
    for (int pops = 0;; ++pops) {
        if (tid == 0) s_item = atomicAdd(item_queue, 1);
        __syncthreads();
        const int idx = wave_uniform(s_item);
        __syncthreads();
        if (idx >= nit) break;
        if (idx < 0 || pops > nit) {
            if (tid == 0) atomicOr(bv.health, H_QUEUE);
            break;
        }
        const int it = item_list ? item_list[lo + idx] : idx;
        if (it < 0 || it >= caps.items_cap) {
            if (tid == 0) atomicOr(bv.health, H_ITEM);
            continue;
        }
        const CountItem ci = items[it];
        if (ci.first < 0 || ci.last < ci.first || (int64_t)ci.last > bv.N || ci.last - ci.first > caps.V ||
            ci.label < 0 || ci.label >= bv.M) {
            if (tid == 0) atomicOr(bv.health, H_ITEM);
            continue;
        }
        const LabelInfo li = rl.label[ci.label];
        const LabelInfo lf = fl.label[ci.label];
        if (lf.n_segs > fl.max_segs) {
            if (tid == 0) atomicOr(bv.health, H_ITEM);
            continue;
        }
        for (int j = tid; j < lf.n_segs; j += NT) fmap[fl.seg_key[lf.seg_first + j]] = j;
        for (int j = tid; j < li.n_multi; j += NT) {
            const SegChunk sc = rl.seg_chunk[li.seg_first + j];
            for (int p = 0; p < sc.count; ++p) chunk_seg[sc.first + p] = j;
        }
        if (ci.split && tid == 0) {
            s_slot = atomicAdd(slot_counter, 1);
            item_slot[it] = s_slot;
        }
        __syncthreads();
        int slot = ci.split ? s_slot : -1;
        if (ci.split && (slot < 0 || slot >= caps.slot_cap)) {
            if (tid == 0) atomicOr(bv.health, H_SLOT);
            slot = -2;  // compute, write nothing
        }
        const int passes = (li.n_slices + NW * KPP - 1) / (NW * KPP);
        for (int pass = 0; pass < passes; ++pass) {
            __syncthreads();  // the previous pass may still read the LDS vectors
            float acc[MAXR];
#pragma unroll
            for (int r = 0; r < MAXR; ++r) acc[r] = 0.0f;
            if (ci.carry && !ci.split) {  // continue the label's sums from the blocks already done
#pragma unroll
                for (int k = 0; k < KPP; ++k) {
                    const int s = (pass * KPP + k) * NW + wave;
                    if (s < li.n_slices) {
                        const SliceInfo si = rl.slice[li.slice_first + s];
                        if (lane < si.width) {
#pragma unroll
                            for (int r = 0; r < CH; ++r) {
                                if (r < si.height) {
                                    const int arc = rl.elem_arc[si.base + r * si.width + lane];
                                    if (arc >= 0) acc[k * CH + r] = grad[arc];
                                }
                            }
                        }
                    }
                }
            }
            int src[KPP];  // source state of this lane's chunk in each slice of the pass (-1: none)
#pragma unroll
            for (int k = 0; k < KPP; ++k) {
                const int s = (pass * KPP + k) * NW + wave;
                src[k] = -1;
                if (s < li.n_slices) {
                    const SliceInfo si = rl.slice[li.slice_first + s];
                    if (lane < si.width) {
                        const int c = s * 64 + lane;
                        const int j = c < li.n_slots ? chunk_seg[c] : li.n_multi + (c - li.n_slots);
                        src[k] = rl.seg_key[li.seg_first + j];
                    }
                }
            }
            VisitInfo vi = vinfo[ci.first];
            VisitVals<kPrefetch> nx;
            fetch_visit<NT>(fl, tp, vi, start, lf.n_segs, tid, nx);
            for (int v = ci.first; v < ci.last; ++v) {
                CEnt *den = (v & 1) ? den1 : den0;
                float *bd = bden + (v & 1) * fl.max_segs;
                if (vi.live) {
#pragma unroll
                    for (int u = 0; u < kPrefetch; ++u) {
                        if (nx.key[u] >= 0) den[nx.key[u]] = CEnt{nx.aval[u], v};
                        if (tid + u * NT < lf.n_segs) bd[tid + u * NT] = nx.bval[u];
                    }
                    // rare: more entries than NT * kPrefetch
                    for (int j = tid + kPrefetch * NT; j < lf.n_segs; j += NT)
                        bd[j] = (to_global(vi.b_ptr)[j] - vi.bm) + vi.o;
                    if (vi.prev_label >= 0) {
                        const LabelInfo lp = fl.label[vi.prev_label];
                        for (int j = tid + kPrefetch * NT; j < lp.n_segs; j += NT)
                            den[fl.seg_key[lp.seg_first + j]] = CEnt{to_global(vi.a_ptr)[j] - vi.cm, v};
                    }
                }
                const VisitInfo cur = vi;
                if (v + 1 < ci.last) {  // next visit's record, alpha and beta, in flight during this one
                    vi = vinfo[v + 1];
                    fetch_visit<NT>(fl, tp, vi, start, lf.n_segs, tid, nx);
                }
                __syncthreads();
                if (!cur.live) continue;
#pragma unroll
                for (int k = 0; k < KPP; ++k) {
                    float a = WFST_NINF;
                    if (src[k] >= 0) {
                        const CEnt ae = den[src[k]];
                        if (ae.stamp == v) a = ae.v;
                    }
                    const bool live = a != WFST_NINF;
                    if (__ballot(live) != 0ull && live) {
                        const SliceInfo si = rl.slice[li.slice_first + (pass * KPP + k) * NW + wave];
                        const int32_t *op = rl.other + si.base + lane;
                        const float *sp = rl.score + si.base + lane;
#pragma unroll
                        for (int r = 0; r < CH; ++r) {
                            if (r < si.height) {
                                const Elem e{op[r * si.width], sp[r * si.width]};
                                if (e.other < Q) {
                                    const float x = (a + e.score) + bd[fmap[e.other]];
                                    acc[k * CH + r] += cur.g * exp_e(x);
                                }
                            }
                        }
                    }
                }
            }
            // write this pass's arcs
#pragma unroll
            for (int k = 0; k < KPP; ++k) {
                const int s = (pass * KPP + k) * NW + wave;
                const SliceInfo si = s < li.n_slices ? rl.slice[li.slice_first + s] : SliceInfo{0, 0, 0, 0};
                if (lane < si.width) {
#pragma unroll
                    for (int r = 0; r < CH; ++r) {
                        if (r < si.height) {
                            const int pos = si.base + r * si.width + lane;
                            const float val2 = acc[k * CH + r];
                            if (slot == -1) {
                                const int arc = rl.elem_arc[pos];
                                if (arc >= 0) grad[arc] = val2;
                            } else if (slot >= 0) {
                                partial[(int64_t)slot * rl.max_elems + (pos - li.elem_first)] = val2;
                            }
                        }
                    }
                }
            }
        }
    }
}

// Sums the partial counts of groups (label, block) whose visits span several
// work items: one thread per (group, element), partials added in item order,
// starting from the gradient when the label's sums carry over from earlier
// blocks.
template <int NT>
__global__ void __launch_bounds__(NT)
counts_fixup(DevLayout rl, const CountItem *__restrict__ items, const int32_t *__restrict__ item_base,
             const int32_t *__restrict__ n_items_key, const int64_t *__restrict__ se_off,
             const int64_t *__restrict__ se_total, const int32_t *__restrict__ item_slot,
             const float *__restrict__ partial, float *__restrict__ grad, CountCaps caps, int32_t MK, int32_t K,
             uint32_t *health)
{
    const int64_t W = *se_total;
    for (int64_t w = blockIdx.x * (int64_t)NT + threadIdx.x; w < W; w += (int64_t)gridDim.x * NT) {
        int lo = 0, hi = MK;  // last group with se_off <= w
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (se_off[mid] <= w) lo = mid; else hi = mid;
        }
        const int key = lo;
        const LabelInfo li = rl.label[key / K];
        const int64_t e = w - se_off[key];
        const int first = item_base[key], k = n_items_key[key];
        if (e >= li.n_elems || k < 2 || first < 0 || first + k > caps.items_cap) {
            atomicOr(health, H_ITEM);
            continue;
        }
        const int arc = rl.elem_arc[li.elem_first + e];
        float s = (items[first].carry && arc >= 0) ? grad[arc] : 0.0f;
        bool ok = true;
        int x = 0;
        for (; x + 4 <= k; x += 4) {
            int sl[4];
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                sl[u] = item_slot[first + x + u];
                ok = ok && sl[u] >= 0 && sl[u] < caps.slot_cap;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = ok ? partial[(int64_t)sl[u] * rl.max_elems + e] : 0.0f;
#pragma unroll
            for (int u = 0; u < 4; ++u) s += v[u];
        }
        for (; x < k; ++x) {
            const int sl = item_slot[first + x];
            ok = ok && sl >= 0 && sl < caps.slot_cap;
            if (ok) s += partial[(int64_t)sl * rl.max_elems + e];
        }
        if (!ok) {
            atomicOr(health, H_SLOT);
            continue;
        }
        if (arc >= 0) grad[arc] = s;
    }
}

// element count of every group (label, block) of block blk (all blocks when
// blk < 0) whose visits span several count work items
__global__ void split_group_elems(const LabelInfo *__restrict__ label, const int32_t *__restrict__ n_items_key,
                                  int32_t MK, int32_t K, int32_t blk, int32_t *__restrict__ out)
{
    for (int key = blockIdx.x * blockDim.x + threadIdx.x; key < MK; key += gridDim.x * blockDim.x) {
        const bool mine = blk < 0 || K - 1 - key % K == blk;
        out[key] = (mine && n_items_key[key] > 1) ? label[key / K].n_elems : 0;
    }
}

// Gradient from the expected-count records grouped by reverse slot (sorted),
// summed per slot as 64-bit integers round(value * 2^S) (2^S from
// fx_scale_kernel: no sum can overflow, and integer sums do not depend on the
// order of the additions).  record_tiles: one wavefront per tile of 64
// records sums every run piece in the tile by a segmented scan over the
// lanes; a run that begins and ends inside the tile is written at once, the
// pieces that cross a tile edge are kept in its RecTile.  record_runs: the
// tile where such a run begins adds the tiles it spans and writes it.
struct RecTile {
    long long head;      // sum of the tile's first piece when its run began in an earlier tile (else 0)
    long long tail;      // sum of the tile's last piece when its run begins here and goes on (else 0)
    uint32_t tail_slot;  // slot of that run (0xffffffff: none)
    int32_t full;        // 1: the tile is one piece of a run that began earlier and goes on
};
constexpr uint32_t kNoSlot = 0xffffffffu;  // the slot part of the sentinel keys

__global__ void record_tiles(const uint64_t *__restrict__ key, const float *__restrict__ val, int64_t n,
                             const int32_t *__restrict__ elem_arc, const double *__restrict__ scale,
                             float *__restrict__ grad, RecTile *__restrict__ tiles, int64_t ntiles)
{
    const int lane = threadIdx.x & 63;
    const double sc = *scale, inv = 1.0 / sc;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t tile = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; tile < ntiles; tile += nw) {
        const int64_t j = tile * 64 + lane;
        const uint64_t k = j < n ? key[j] : kRecSentinel;
        const uint32_t slot = (uint32_t)(k >> 32);
        long long q = k != kRecSentinel ? __double2ll_rn((double)val[j] * sc) : 0;
        const uint32_t before = tile > 0 ? (uint32_t)(key[tile * 64 - 1] >> 32) : kNoSlot;
        const uint32_t after = (tile + 1) * 64 < n ? (uint32_t)(key[(tile + 1) * 64] >> 32) : kNoSlot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {  // inclusive scan within runs (a run's lanes are contiguous)
            const long long qo = __shfl_up(q, o, 64);
            const uint32_t so = __shfl_up(slot, o, 64);
            if (lane >= o && so == slot) q += qo;
        }
        const uint32_t slot0 = __shfl(slot, 0, 64), slot63 = __shfl(slot, 63, 64);
        const uint32_t next = __shfl_down(slot, 1, 64);
        const bool last = lane == 63 || next != slot;  // last lane of its piece
        const bool from_before = slot == slot0 && before == slot;
        const bool to_after = lane == 63 && after == slot;
        if (last && slot != kNoSlot && !from_before && !to_after) {  // a whole run inside the tile
            const int32_t a = elem_arc[slot];
            if (a >= 0) grad[a] = (float)((double)q * inv);
        }
        const uint64_t other = __ballot(slot != slot0);
        const int l0 = other ? __builtin_ctzll(other) - 1 : 63;  // last lane of the first piece
        const bool head = slot0 != kNoSlot && before == slot0;
        const long long head_sum = __shfl(q, l0, 64), tail_sum = __shfl(q, 63, 64);
        const bool full = head && l0 == 63 && after == slot0;
        const bool owner = slot63 != kNoSlot && after == slot63 && !(head && l0 == 63);
        if (lane == 0) {
            RecTile rt;
            rt.head = head ? head_sum : 0;
            rt.tail = owner ? tail_sum : 0;
            rt.tail_slot = owner ? slot63 : kNoSlot;
            rt.full = full ? 1 : 0;
            tiles[tile] = rt;
        }
    }
}

__global__ void record_runs(const RecTile *__restrict__ tiles, int64_t ntiles, const int32_t *__restrict__ elem_arc,
                            const double *__restrict__ scale, float *__restrict__ grad)
{
    const double inv = 1.0 / *scale;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
        const RecTile rt = tiles[t];
        if (rt.tail_slot == kNoSlot) continue;
        long long sum = rt.tail;
        for (int64_t u = t + 1; u < ntiles; ++u) {  // the tiles the run spans, up to the one where it ends
            const RecTile ru = tiles[u];
            sum += ru.head;
            if (!ru.full) break;
        }
        const int32_t a = elem_arc[rt.tail_slot];
        if (a >= 0) grad[a] = (float)((double)sum * inv);
    }
}

// Final-state posteriors (gradient of log Z with respect to the final scores,
// the f-vector of Eq. 1): P_b(path ends in q) = alpha_T[q] f[q] / Z_b.  Each
// sentence of a block writes its nonzero terms into its own dense row (one
// wavefront per sentence, rows zero-filled beforehand); rows are summed per
// state in sentence order, in groups and then over groups.
__global__ void final_rows(BatchView bv, TapeView tp, DevLayout fl, int32_t Q, int32_t start,
                           const float *__restrict__ final_score, const float *__restrict__ grad_log_z,
                           int32_t b0, int32_t nb, float *__restrict__ rows)
{
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x / 64;
    for (int bb = blockIdx.x * wpb + (threadIdx.x >> 6); bb < nb; bb += gridDim.x * wpb) {
        const int b = b0 + bb;
        if (bv.status[b] != WFST_STATUS_OK) continue;
        const int o0 = bv.offsets[b], o1 = bv.offsets[b + 1];
        if (o0 < 0 || o1 < o0 || (int64_t)o1 > bv.N) {
            if (lane == 0) atomicOr(bv.health, H_VISIT);
            continue;
        }
        const float g = grad_log_z ? grad_log_z[b] : 1.0f;
        float *row = rows + (int64_t)bb * Q;
        if (o1 == o0) {  // empty sentence: the path ends where it starts
            if (lane == 0) {
                const float f = final_score[start];
                if (f != WFST_NINF) row[start] = g * exp_e((0.0f + f) + (float)(0.0 - tp.log_z[b]));
            }
            continue;
        }
        const int i = o1 - 1;
        const int a = bv.tokens[i];
        if (a < 0 || a >= bv.M) {
            if (lane == 0) atomicOr(bv.health, H_VISIT);
            continue;
        }
        const LabelInfo lf = fl.label[a];
        const float *ta = tp.alpha + (tp.ck_off ? tp.ck_off[i] : bv.tok_off[i]);
        const float c = tp.a_max[i];
        const float o = (float)(tp.a_log[i] - tp.log_z[b]);
        for (int j = lane; j < lf.n_segs; j += 64) {
            const int q = fl.seg_key[lf.seg_first + j];
            const float x = ta[j], f = final_score[q];
            if (x == WFST_NINF || f == WFST_NINF) continue;
            row[q] = g * exp_e(((x - c) + f) + o);
        }
    }
}

// S[g][q] = sum of rows[b][q] over the G rows of group g, in row order
__global__ void sum_row_groups(const float *__restrict__ rows, int32_t nb, int32_t Q, int32_t G,
                               float *__restrict__ S)
{
    const int32_t ng = (nb + G - 1) / G;
    const int64_t n = (int64_t)ng * Q;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(w / Q), q = (int)(w % Q);
        const int b1 = min(nb, (g + 1) * G);
        float s = 0.0f;
        for (int b = g * G; b < b1; ++b) s += rows[(int64_t)b * Q + q];
        S[w] = s;
    }
}

// out[q] (+)= sum over groups g of S[g][q], in group order
__global__ void sum_groups(const float *__restrict__ S, int32_t ng, int32_t Q, int32_t accumulate,
                           float *__restrict__ out)
{
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < Q; q += gridDim.x * blockDim.x) {
        float s = accumulate ? out[q] : 0.0f;
        for (int g = 0; g < ng; ++g) s += S[(int64_t)g * Q + q];
        out[q] = s;
    }
}

// ---- checkpoint planning -------------------------------------------------

// longest sentence of the batch (one workgroup)
__global__ void __launch_bounds__(1024) batch_max_len(const int32_t *__restrict__ offsets, int32_t B,
                                                      int32_t *__restrict__ out)
{
    __shared__ int32_t m;
    if (threadIdx.x == 0) m = 0;
    __syncthreads();
    int32_t x = 0;
    for (int b = threadIdx.x; b < B; b += blockDim.x) x = max(x, offsets[b + 1] - offsets[b]);
    atomicMax(&m, x);
    __syncthreads();
    if (threadIdx.x == 0) *out = m;
}

// per token: size of its kept alpha~ (steps divisible by c and the last step)
__global__ void ckpt_sizes(const int32_t *__restrict__ offsets, int32_t B, const int32_t *__restrict__ tokens,
                           const LabelInfo *__restrict__ label, int32_t M, int32_t c, int64_t *__restrict__ size)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        const int o0 = offsets[b], T = offsets[b + 1] - o0;
        for (int t = 1; t <= T; ++t) {
            const int a = tokens[o0 + t - 1];
            const bool keep = (t % c == 0 || t == T) && a >= 0 && a < M;
            size[o0 + t - 1] = keep ? label[a].n_segs : 0;
        }
    }
}

// ck_off[i] = -1 for tokens whose alpha~ is not kept
__global__ void ckpt_mark(const int64_t *__restrict__ size, int64_t N, int64_t *__restrict__ ck_off)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        if (size[i] == 0) ck_off[i] = -1;
}

// per sentence: the largest block of c steps, in compact tape entries
__global__ void block_sizes(const int32_t *__restrict__ offsets, int32_t B, const int32_t *__restrict__ tokens,
                            const LabelInfo *__restrict__ label, int32_t M, const int64_t *__restrict__ tok_off,
                            int32_t c, int64_t *__restrict__ out)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        const int o0 = offsets[b], T = offsets[b + 1] - o0;
        int64_t m = 0;
        for (int t0 = 0; t0 < T; t0 += c) {
            const int t1 = min(T, t0 + c);
            const int a = tokens[o0 + t1 - 1];
            const int64_t end = tok_off[o0 + t1 - 1] + ((a >= 0 && a < M) ? label[a].n_segs : 0);
            m = max(m, end - tok_off[o0 + t0]);
        }
        out[b] = m;
    }
}

__global__ void fill_f32(float *__restrict__ p, int64_t n, float v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_i64(int64_t *__restrict__ p, int64_t n, int64_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void copy_f32(float *__restrict__ dst, const float *__restrict__ src, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// per-token segment count of the forward layout (0 for an invalid token)
__global__ void token_segments(const int32_t *__restrict__ tokens, int64_t N, const LabelInfo *__restrict__ label,
                               int32_t M, int64_t *__restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int a = tokens[i];
        out[i] = (a >= 0 && a < M) ? label[a].n_segs : 0;
    }
}

// token -> sentence, and visit keys for grouping: the label, refined by the
// checkpoint block (later blocks first) when c > 0: key = label * K + (K-1-block)
__global__ void token_owner(const int32_t *__restrict__ offsets, int32_t B, int64_t N,
                            const int32_t *__restrict__ tokens, int32_t *__restrict__ tok_sent,
                            int32_t *__restrict__ vis_key, int32_t *__restrict__ vis_idx, int32_t M, int32_t c,
                            int32_t K)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = B;  // last b with offsets[b] <= i
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (offsets[mid] <= i) lo = mid; else hi = mid;
        }
        tok_sent[i] = lo;
        const int a = tokens[i];
        int key = (a >= 0 && a < M) ? a * K : M * K;  // invalid tokens sort last
        if (c > 0 && key < M * K) key += K - 1 - min(K - 1, (int)(i - offsets[lo]) / c);
        vis_key[i] = key;
        vis_idx[i] = (int)i;
    }
}

// one thread per label: visit range in the sorted list and its item count
__global__ void label_groups(const int32_t *__restrict__ skeys, int64_t N, int32_t M, int32_t V,
                             int32_t *__restrict__ grp_lo, int32_t *__restrict__ grp_n,
                             int32_t *__restrict__ n_items_per_label)
{
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < M; a += gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = N;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (skeys[mid] < a) lo = mid + 1; else hi = mid;
        }
        int64_t lo2 = lo, hi2 = N;
        while (lo2 < hi2) {
            const int64_t mid = (lo2 + hi2) >> 1;
            if (skeys[mid] <= a) lo2 = mid + 1; else hi2 = mid;
        }
        const int n = (int)(lo2 - lo);
        grp_lo[a] = (int)lo;
        grp_n[a] = n;
        n_items_per_label[a] = (n + V - 1) / V;
    }
}

// items of every key group (key = label * K + K-1-block); a label is split
// when its items over all blocks number more than one
__global__ void label_items(const int32_t *__restrict__ grp_lo, const int32_t *__restrict__ grp_n,
                            const int32_t *__restrict__ n_items_per_key, const int32_t *__restrict__ item_base,
                            int32_t MK, int32_t K, int32_t V,
                            CountItem *__restrict__ items, int32_t *__restrict__ n_items, int32_t items_cap,
                            uint32_t *__restrict__ health)
{
    for (int key = blockIdx.x * blockDim.x + threadIdx.x; key < MK; key += gridDim.x * blockDim.x) {
        const int k = n_items_per_key[key];
        const int base = item_base[key];
        if (base < 0 || k < 0 || base + k > items_cap) {
            atomicOr(health, H_GROUP);
            continue;
        }
        const int a = key / K;
        const int split = k > 1 ? 1 : 0;
        int carry = 0;  // keys of a label are processed in increasing order (later blocks first)
        for (int r = a * K; r < key; ++r) carry |= n_items_per_key[r] > 0;
        for (int x = 0; x < k; ++x) {
            const int f = grp_lo[key] + x * V;
            const int l = min(grp_lo[key] + grp_n[key], f + V);
            items[base + x] = CountItem{f, l, a, split, K - 1 - key % K, carry};
        }
        if (key == MK - 1) *n_items = base + k;
    }
}

// Item indices listed per checkpoint block (one workgroup): list_off[K+1]
// offsets, list[] indices.  The order inside a block does not affect results.
__global__ void __launch_bounds__(1024) items_by_block(const CountItem *__restrict__ items,
                                                       const int32_t *__restrict__ n_items, int32_t K,
                                                       int32_t items_cap, int32_t *__restrict__ list,
                                                       int32_t *__restrict__ list_off, uint32_t *__restrict__ health)
{
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t *cnt = reinterpret_cast<int32_t *>(smem);  // [K] counts, then [K] cursors
    int32_t *cur = cnt + K;
    const int n = min(max(*n_items, 0), items_cap);
    for (int k = threadIdx.x; k < K; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    for (int it = threadIdx.x; it < n; it += blockDim.x) {
        const int k = items[it].block;
        if (k >= 0 && k < K) atomicAdd(&cnt[k], 1);
        else atomicOr(health, H_ITEM);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < K; ++k) {
            list_off[k] = run;
            cur[k] = run;
            run += cnt[k];
        }
        list_off[K] = run;
    }
    __syncthreads();
    for (int it = threadIdx.x; it < n; it += blockDim.x) {
        const int k = items[it].block;
        if (k >= 0 && k < K) list[atomicAdd(&cur[k], 1)] = it;
    }
}

// New scores into both layouts through their element -> arc maps.  Each
// thread writes four consecutive elements; the layouts are concatenated in
// one index space.  Workgroups are dispatched round-robin over the 8 XCDs:
// workgroup g is given tile (g % 8) * (tiles / 8) + g / 8, so each XCD walks
// its own contiguous eighth of the elements and the scores it gathers (arcs of
// the same labels) stay in its L2.
constexpr int kXcds = 8;

__device__ __forceinline__ float scatter_one(int arc, const float *__restrict__ score)
{
    if (arc < 0) return 0.0f;  // padding keeps score 0
    const float s = score[arc];
    return s == 0.0f ? 0.0f : s;
}

__device__ __forceinline__ void scatter_range(float *__restrict__ out, const int32_t *__restrict__ elem_arc,
                                              int64_t n, int64_t e4, const float *__restrict__ score)
{
    const int64_t e = 4 * e4;
    if (e + 4 <= n) {
        const int4 a = reinterpret_cast<const int4 *>(elem_arc)[e4];
        float4 v;
        v.x = scatter_one(a.x, score);
        v.y = scatter_one(a.y, score);
        v.z = scatter_one(a.z, score);
        v.w = scatter_one(a.w, score);
        reinterpret_cast<float4 *>(out)[e4] = v;
    } else {
        for (int64_t x = e; x < n; ++x) out[x] = scatter_one(elem_arc[x], score);
    }
}

// tiles of 256 threads x 4 elements; n4a / n4b = quads of layout a / b (rounded up)
__global__ void __launch_bounds__(256) scatter_scores(float *__restrict__ out_a, const int32_t *__restrict__ arc_a,
                                                      int64_t n_a, float *__restrict__ out_b,
                                                      const int32_t *__restrict__ arc_b, int64_t n_b,
                                                      const float *__restrict__ score)
{
    const int64_t tiles = gridDim.x;  // a multiple of kXcds
    const int64_t g = blockIdx.x;
    const int64_t tile = (g % kXcds) * (tiles / kXcds) + g / kXcds;
    const int64_t q = tile * 256 + threadIdx.x;
    const int64_t n4a = (n_a + 3) / 4, n4b = (n_b + 3) / 4;
    if (q < n4a) scatter_range(out_a, arc_a, n_a, q, score);
    else if (q - n4a < n4b) scatter_range(out_b, arc_b, n_b, q - n4a, score);
}

// Score update by label (FSTs whose labels have many arcs in compact arc-id
// ranges): one workgroup per label copies the label's scores into LDS once,
// then writes both layouts' slots of the label from there, so every score is
// read from HBM once.  A label whose range exceeds the stage reads directly.
constexpr int kScoreThreads = 512;
constexpr int kScoreStage = 10112;  // floats (39.5 KiB of LDS: four workgroups per CU)

constexpr int kScoreUnroll = 8;  // elements per thread in flight

// elem_loc of a layout: for every slot of a slice, its arc's offset from the
// lowest arc id of the slice's label (0xffff for padding, or when a label's
// arcs span 0xffff ids or more: such labels are never staged).
__global__ void build_elem_loc(const SliceInfo *__restrict__ slice, int64_t n_slice, const int32_t *__restrict__ elem_arc,
                               const int2 *__restrict__ range, uint16_t *__restrict__ loc)
{
    for (int64_t s = blockIdx.x; s < n_slice; s += gridDim.x) {
        const SliceInfo si = slice[s];
        const int lo = range[si.label].x;
        const int n = si.height * si.width;
        for (int x = threadIdx.x; x < n; x += blockDim.x) {
            const int arc = elem_arc[si.base + x];
            const int d = arc - lo;
            loc[si.base + x] = (uint16_t)(arc >= 0 && d >= 0 && d < 0xffff ? d : 0xffff);
        }
    }
}

template <bool STAGED>  // scores from the LDS stage, else from global memory (kept apart: no generic loads)
__device__ __forceinline__ void scatter_label_layout(const LabelInfo &li, float *__restrict__ out,
                                                     const int32_t *__restrict__ elem_arc,
                                                     const uint16_t *__restrict__ elem_loc, const float *stage,
                                                     const float *__restrict__ score)
{
    const int32_t *ea = elem_arc + li.elem_first;
    const uint16_t *el = elem_loc + li.elem_first;
    float *o = out + li.elem_first;
    for (int e0 = threadIdx.x; e0 < li.n_elems; e0 += kScoreUnroll * kScoreThreads) {
        float v[kScoreUnroll];
        if constexpr (STAGED) {  // 2-byte offsets into the label's staged scores
            int loc[kScoreUnroll];
#pragma unroll
            for (int u = 0; u < kScoreUnroll; ++u) {
                const int e = e0 + u * kScoreThreads;
                loc[u] = e < li.n_elems ? (int)el[e] : 0xffff;
            }
#pragma unroll
            for (int u = 0; u < kScoreUnroll; ++u) v[u] = loc[u] != 0xffff ? stage[loc[u]] : 0.0f;  // padding: 0
        } else {
            int arc[kScoreUnroll];
#pragma unroll
            for (int u = 0; u < kScoreUnroll; ++u) {
                const int e = e0 + u * kScoreThreads;
                arc[u] = e < li.n_elems ? ea[e] : -1;
            }
#pragma unroll
            for (int u = 0; u < kScoreUnroll; ++u) v[u] = arc[u] >= 0 ? score[arc[u]] : 0.0f;  // padding: 0
        }
#pragma unroll
        for (int u = 0; u < kScoreUnroll; ++u) {
            const int e = e0 + u * kScoreThreads;
            if (e < li.n_elems) o[e] = v[u] == 0.0f ? 0.0f : v[u];
        }
    }
}

__global__ void __launch_bounds__(kScoreThreads)
scatter_scores_by_label(const LabelInfo *__restrict__ fl, const LabelInfo *__restrict__ rl,
                        const int2 *__restrict__ range, float *__restrict__ out_f, const int32_t *__restrict__ arc_f,
                        const uint16_t *__restrict__ loc_f, float *__restrict__ out_r,
                        const int32_t *__restrict__ arc_r, const uint16_t *__restrict__ loc_r,
                        const float *__restrict__ score)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float *stage = reinterpret_cast<float *>(smem);
    const int a = blockIdx.x;
    const int2 r = range[a];
    const int n = r.y - r.x + 1;  // <= 0 for a label without arcs
    const bool staged = n > 0 && n <= kScoreStage;
    if (staged) {
        for (int j0 = threadIdx.x; j0 < n; j0 += kScoreUnroll * kScoreThreads) {
            float x[kScoreUnroll];
#pragma unroll
            for (int u = 0; u < kScoreUnroll; ++u) {
                const int j = j0 + u * kScoreThreads;
                x[u] = j < n ? score[r.x + j] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kScoreUnroll; ++u) {
                const int j = j0 + u * kScoreThreads;
                if (j < n) stage[j] = x[u];
            }
        }
    }
    __syncthreads();
    if (staged) {
        scatter_label_layout<true>(fl[a], out_f, arc_f, loc_f, stage, score);
        scatter_label_layout<true>(rl[a], out_r, arc_r, loc_r, stage, score);
    } else {
        scatter_label_layout<false>(fl[a], out_f, arc_f, loc_f, stage, score);
        scatter_label_layout<false>(rl[a], out_r, arc_r, loc_r, stage, score);
    }
}

// Scale of the fixed-point count accumulators: 2^S with S the largest integer
// for which N * max(1, max_b |g_b|) * 2^S stays below 2^62, so no sum of
// posteriors (each at most |g_b|, at most N of them per arc) can overflow.
// One workgroup.
__global__ void __launch_bounds__(256) fx_scale_kernel(const float *__restrict__ g, int32_t B, int64_t N,
                                                       double *__restrict__ scale)
{
    __shared__ float red[256];
    float m = 1.0f;
    if (g)
        for (int b = threadIdx.x; b < B; b += 256) m = fmaxf(m, fabsf(g[b]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double bound = (double)red[0] * (double)(N > 0 ? N : 1);
        const int S = 61 - ilogb(bound);  // bound < 2^(ilogb + 1), so sums stay below 2^62
        *scale = ldexp(1.0, S);
    }
}

// grad[elem_arc[e]] = acc[e] / 2^S over the reverse slots e (each arc has one
// slot; padding slots have no arc)
__global__ void fx_to_grad(const unsigned long long *__restrict__ acc, const int32_t *__restrict__ elem_arc, int64_t n,
                           const double *__restrict__ scale, float *__restrict__ grad)
{
    const double inv = 1.0 / *scale;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = elem_arc[e];
        if (k >= 0) grad[k] = (float)((double)(long long)acc[e] * inv);
    }
}

// =====================================================================
// Time-parallel scan of the forward pass over the per-token transition
// matrices (Eq. 1 as a product of delta[w_t], evaluated as a parallel
// prefix; for FSTs with at most kScanMaxQ states).  Dense |Q| x |Q| matrices
// in the log semiring, -inf for no arc, row = source, column = destination.
// =====================================================================
constexpr int kScanMaxQ = 64;
constexpr int kScanThreadsPerMat = 256;

// log(e^a + e^b), exact for -inf operands
__device__ __forceinline__ float log_add(float a, float b)
{
    const float m = fmaxf(a, b);
    if (m == WFST_NINF) return WFST_NINF;
    return m + log_e(exp_e(a - m) + exp_e(b - m));
}

// first token index of the sentence of every token
__global__ void token_first(const int32_t *__restrict__ offsets, int32_t B, int64_t N, int32_t *__restrict__ first)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = B;  // last b with offsets[b] <= i
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (offsets[mid] <= i) lo = mid; else hi = mid;
        }
        first[i] = offsets[lo];
    }
}

// The matrix of every token's label: one workgroup per token; a thread owns
// whole destination segments (columns), so parallel arcs of one (source,
// destination) pair are log-added by one thread in arc-id order.
__global__ void __launch_bounds__(kScanThreadsPerMat)
scan_leaves(DevLayout fl, int32_t Q, const int32_t *__restrict__ tokens, int64_t N, int32_t M, float *__restrict__ P)
{
    const int64_t QQ = (int64_t)Q * Q;
    for (int64_t i = blockIdx.x; i < N; i += gridDim.x) {
        float *m = P + i * QQ;
        for (int64_t e = threadIdx.x; e < QQ; e += blockDim.x) m[e] = WFST_NINF;
        __syncthreads();
        const int a = tokens[i];
        if (a >= 0 && a < M) {
            const LabelInfo li = fl.label[a];
            for (int j = threadIdx.x; j < li.n_segs; j += blockDim.x) {
                const int d = fl.seg_key[li.seg_first + j];
                int c0 = li.n_slots + (j - li.n_multi), nc = 1;
                if (j < li.n_multi) {
                    const SegChunk sc = fl.seg_chunk[li.seg_first + j];
                    c0 = sc.first;
                    nc = sc.count;
                }
                for (int c = c0; c < c0 + nc; ++c) {
                    const SliceInfo si = fl.slice[li.slice_first + (c >> 6)];
                    for (int r = 0; r < si.height; ++r) {
                        const int e = si.base + r * si.width + (c & 63);
                        const int sq = fl.other[e];
                        if (sq >= Q) continue;  // padding
                        float &x = m[(int64_t)sq * Q + d];
                        x = log_add(x, fl.score[e]);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// One level of the inclusive scan: out[i] = in[i - stride] (x) in[i] when
// token i is at least `stride` tokens into its sentence, else in[i].  One
// workgroup per token; both operands staged in LDS; every output element is
// a two-pass log-sum-exp over k in increasing order.
__global__ void __launch_bounds__(kScanThreadsPerMat)
scan_level(const float *__restrict__ in, float *__restrict__ out, const int32_t *__restrict__ first, int64_t N,
           int32_t Q, int32_t stride)
{
    __shared__ float A[kScanMaxQ * kScanMaxQ], Bm[kScanMaxQ * kScanMaxQ];
    const int QQ = Q * Q;
    for (int64_t i = blockIdx.x; i < N; i += gridDim.x) {
        const float *b = in + i * (int64_t)QQ;
        float *o = out + i * (int64_t)QQ;
        if (i - first[i] < stride) {
            for (int e = threadIdx.x; e < QQ; e += blockDim.x) o[e] = b[e];
            continue;
        }
        const float *a = in + (i - stride) * (int64_t)QQ;
        __syncthreads();  // the previous token's products are done reading A, Bm
        for (int e = threadIdx.x; e < QQ; e += blockDim.x) {
            A[e] = a[e];
            Bm[e] = b[e];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < QQ; e += blockDim.x) {
            const int r = e / Q, c = e - r * Q;
            float m = WFST_NINF;
            for (int k = 0; k < Q; ++k) m = fmaxf(m, A[r * Q + k] + Bm[k * Q + c]);
            float v = WFST_NINF;
            if (m != WFST_NINF) {
                float sum = 0.0f;
                for (int k = 0; k < Q; ++k) sum += exp_e((A[r * Q + k] + Bm[k * Q + c]) - m);
                v = m + log_e(sum);
            }
            o[e] = v;
        }
    }
}

// Per sentence (one wavefront): status, log Z = LSE_q(P_T[start][q] + f[q])
// (FP64 accumulation), and optionally log alpha_t = row `start` of each
// prefix product (the start vector is one-hot).
__global__ void scan_finish(const float *__restrict__ P, const int32_t *__restrict__ offsets,
                           const int32_t *__restrict__ tokens, int32_t B, int64_t N, int32_t M, int32_t Q,
                           int32_t start, const float *__restrict__ final_score, float *__restrict__ log_z,
                           float *__restrict__ alpha, int32_t *__restrict__ status)
{
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x / 64;
    const int64_t QQ = (int64_t)Q * Q;
    for (int b = blockIdx.x * wpb + (threadIdx.x >> 6); b < B; b += gridDim.x * wpb) {
        const int o0 = offsets[b], o1 = offsets[b + 1];
        if (o0 < 0 || o1 < o0 || (int64_t)o1 > N) {
            if (lane == 0) {
                status[b] = WFST_STATUS_BAD_INPUT;
                log_z[b] = WFST_NINF;
            }
            continue;
        }
        int bad = 0;
        for (int i = o0 + lane; i < o1; i += 64) bad |= tokens[i] < 0 || tokens[i] >= M;
        if (__any(bad)) {
            if (lane == 0) {
                status[b] = WFST_STATUS_BAD_TOKEN;
                log_z[b] = WFST_NINF;
            }
            continue;
        }
        if (alpha)
            for (int64_t x = lane; x < (int64_t)(o1 - o0) * Q; x += 64) {
                const int64_t i = o0 + x / Q;
                const int q = (int)(x % Q);
                alpha[i * Q + q] = P[i * QQ + (int64_t)start * Q + q];
            }
        double m = -__builtin_huge_val();
        double v[2] = {-__builtin_huge_val(), -__builtin_huge_val()};
        for (int u = 0; u < 2; ++u) {
            const int q = lane + 64 * u;
            if (q < Q) {
                const float x = o1 > o0 ? P[(int64_t)(o1 - 1) * QQ + (int64_t)start * Q + q] : (q == start ? 0.0f : WFST_NINF);
                const float f = final_score[q];
                if (x != WFST_NINF && f != WFST_NINF) v[u] = (double)x + (double)f;
            }
            m = fmax(m, v[u]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        double sum = 0.0;
        if (m != -__builtin_huge_val())
            for (int u = 0; u < 2; ++u)
                if (v[u] != -__builtin_huge_val()) sum += exp(v[u] - m);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (lane == 0) {
            const bool ok = m != -__builtin_huge_val();
            status[b] = ok ? WFST_STATUS_OK : WFST_STATUS_NO_PATH;
            log_z[b] = ok ? (float)(m + log(sum)) : WFST_NINF;
        }
    }
}

// =====================================================================
// Forward pass over input lattices (the input as an acyclic weighted
// acceptor instead of a string; epsilon lattice arcs read no symbol).
// Node v's vector is the log-sum over its incoming arcs (u, v, a, w), in
// their order, of (A_u x delta[a]) + w, or A_u + w for epsilon; vectors are
// kept normalised in FP32 with an FP64 scale per node.
// =====================================================================
__device__ __forceinline__ double log_add_d(double a, double b)
{
    if (a == -__builtin_huge_val()) return b;  // the first contribution: nothing to add
    if (b == -__builtin_huge_val()) return a;
    const double m = fmax(a, b);
    return m + log1p(exp(fmin(a, b) - m));
}

struct LatticeView {
    int32_t B = 0;
    int64_t n_nodes = 0, n_arcs = 0;
    const int32_t *node_off = nullptr, *arc_off = nullptr;  // [B+1] each
    const int32_t *from = nullptr, *to = nullptr, *label = nullptr;
    const float *weight = nullptr;
    float *nodes = nullptr;   // [n_nodes * (Q+1)] normalised vectors (entry Q = -inf)
    double *scale = nullptr;  // [n_nodes]
    int32_t *far = nullptr;   // [n_nodes] zero at launch; 1: an arc leaves the node for a node beyond the next
    int32_t *queue = nullptr;
    const int32_t *offs_bad = nullptr;  // set by lattice_offsets_check
};

// Non-monotone offsets anywhere would let two lattices share node rows: one
// flag for the whole batch, which every lattice then reports as BAD_INPUT.
__global__ void lattice_offsets_check(const int32_t *__restrict__ node_off, const int32_t *__restrict__ arc_off,
                                      int32_t B, int64_t n_nodes, int64_t n_arcs, int32_t *__restrict__ flag)
{
    bool bad = false;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b <= B; b += (int64_t)gridDim.x * blockDim.x) {
        bad |= node_off[b] < 0 || (int64_t)node_off[b] > n_nodes || arc_off[b] < 0 || (int64_t)arc_off[b] > n_arcs;
        if (b < B) bad |= node_off[b + 1] <= node_off[b] || arc_off[b + 1] < arc_off[b];
    }
    if (bad) atomicOr(flag, 1);
}

template <int NT>
__global__ void __launch_bounds__(NT)
lattice_forward(DevLayout fl, int32_t Q, int32_t start, int32_t M, const float *__restrict__ final_score,
                LatticeView lv, float *__restrict__ log_z, float *__restrict__ node_alpha,
                int32_t *__restrict__ status, uint32_t *__restrict__ health)
{
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    double *acc = reinterpret_cast<double *>(smem);         // [Q+1] node being built
    double *vval = acc + (Q + 1);                             // [max_segs]
    double *part = vval + max(fl.max_segs, 1);                // [max_slots]
    int32_t *vkey = reinterpret_cast<int32_t *>(part + max(fl.max_slots, 1));  // [max_segs]
    float *pvec = reinterpret_cast<float *>(vkey + max(fl.max_segs, 1));      // [Q+1] the previous node, normalised
    __shared__ int s_item;
    __shared__ unsigned long long s_cmax;
    __shared__ double s_pscale;  // the previous node's scale
    __shared__ double s_rm[NW];
    __shared__ float s_rs[NW];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);
    const int64_t Q1 = (int64_t)Q + 1;

    for (int pops = 0;; ++pops) {
        if (tid == 0) s_item = atomicAdd(lv.queue, 1);
        __syncthreads();
        const int b = wave_uniform(s_item);
        __syncthreads();
        if (b >= lv.B) break;
        if (b < 0 || pops > lv.B) {
            if (tid == 0) atomicOr(health, H_QUEUE);
            break;
        }
        const int n0 = lv.node_off[b], n1 = lv.node_off[b + 1];
        const int a0 = lv.arc_off[b], a1 = lv.arc_off[b + 1];
        const int n = n1 - n0;
        int bad = (*lv.offs_bad || n0 < 0 || n < 1 || (int64_t)n1 > lv.n_nodes || a0 < 0 || a1 < a0 ||
                   (int64_t)a1 > lv.n_arcs) ? 1 : 0;
        int badtok = 0;
        if (!bad)
            for (int e = a0 + tid; e < a1; e += NT) {
                const int u = lv.from[e], v = lv.to[e], a = lv.label[e];
                const float w = lv.weight[e];
                bad |= u < 0 || v <= u || v >= n || (e > a0 && lv.to[e - 1] > v) || isnan(w) || w == -WFST_NINF;
                badtok |= a < -1 || a >= M;
            }
        bad = __syncthreads_or(bad);
        badtok = __syncthreads_or(badtok);
        if (bad || badtok) {
            if (tid == 0) {
                status[b] = bad ? WFST_STATUS_BAD_INPUT : WFST_STATUS_BAD_TOKEN;
                log_z[b] = WFST_NINF;
            }
            continue;
        }
        // Node vectors stay on chip while only the next node reads them; a node that
        // an arc leaves for a node further ahead is also kept in HBM.
        for (int e = a0 + tid; e < a1; e += NT)
            if (lv.to[e] > lv.from[e] + 1) lv.far[n0 + lv.from[e]] = 1;
        for (int64_t q = tid; q < Q1; q += NT) {
            const float x = q == start ? 0.0f : WFST_NINF;
            pvec[q] = x;
            if (node_alpha && q < Q) node_alpha[(int64_t)n0 * Q + q] = x;
        }
        if (tid == 0) s_pscale = 0.0;
        __syncthreads();
        if (lv.far[n0]) {
            for (int64_t q = tid; q < Q1; q += NT) lv.nodes[(int64_t)n0 * Q1 + q] = pvec[q];
            if (tid == 0) lv.scale[n0] = 0.0;
        }
        // one incoming arc merged into acc: epsilon (log-add of the source vector) or
        // a log-semiring step of the label's forward layout; prev is on chip or in HBM
        auto merge_arc = [&](const float *prev, double cu, int a) {
            if (a < 0) {
                for (int q = tid; q < Q; q += NT) {
                    const float x = prev[q];
                    if (x != WFST_NINF) acc[q] = log_add_d(acc[q], (double)x + cu);
                }
            } else {
                const LabelInfo li = uniform_label(fl.label[a]);
                (void)lse_step<NT, 8>(fl, li, prev, part, vval, vkey, lane, wave, Q);
                __syncthreads();
                for (int j = tid; j < li.n_segs; j += NT) {  // distinct keys: no two threads share one
                    const double x = vval[j];
                    if (x != -__builtin_huge_val()) acc[vkey[j]] = log_add_d(acc[vkey[j]], x + cu);
                }
            }
        };
        int e = a0;
        for (int v = 1; v < n; ++v) {
            for (int64_t q = tid; q < Q1; q += NT) acc[q] = -__builtin_huge_val();
            if (tid == 0) s_cmax = 0ull;
            __syncthreads();
            for (; e < a1 && lv.to[e] == v; ++e) {  // incoming arcs, in their order
                const int u = lv.from[e], a = lv.label[e];
                const double w = (double)lv.weight[e];
                if (u == v - 1)
                    merge_arc(pvec, s_pscale + w, a);
                else
                    merge_arc(lv.nodes + (int64_t)(n0 + u) * Q1, lv.scale[n0 + u] + w, a);
                __syncthreads();
            }
            double mx = -__builtin_huge_val();
            for (int64_t q = tid; q < Q; q += NT) mx = fmax(mx, acc[q]);
            block_max_d(mx, &s_cmax, lane);
            __syncthreads();
            double c = unord_f64(s_cmax);
            if (!(c > -__builtin_huge_val())) c = 0.0;
            const bool keep = lv.far[n0 + v] != 0;
            float *node = lv.nodes + (int64_t)(n0 + v) * Q1;
            for (int64_t q = tid; q < Q1; q += NT) {
                const double y = acc[q];
                const float x = y == -__builtin_huge_val() ? WFST_NINF : (float)(y - c);
                pvec[q] = x;
                if (keep) node[q] = x;
                if (node_alpha && q < Q) node_alpha[(int64_t)(n0 + v) * Q + q] = y == -__builtin_huge_val() ? WFST_NINF : (float)y;
            }
            if (tid == 0) {
                s_pscale = c;
                if (keep) lv.scale[n0 + v] = c;
            }
            __syncthreads();
        }
        // log Z = C_end + LSE_q(A^_end[q] + f[q]) (the last node is on chip)
        LseD z{-__builtin_huge_val(), 0.0f};
        for (int q = tid; q < Q; q += NT) {
            const float x = pvec[q], f = final_score[q];
            if (x == WFST_NINF || f == WFST_NINF) continue;
            lse_push_d(z, (double)x + (double)f);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) z = lse_merge_d(z, LseD{__shfl_xor(z.m, o, 64), __shfl_xor(z.s, o, 64)});
        if (lane == 0) {
            s_rm[wave] = z.m;
            s_rs[wave] = z.s;
        }
        __syncthreads();
        if (tid == 0) {
            LseD tot{s_rm[0], s_rs[0]};
            for (int w2 = 1; w2 < NW; ++w2) tot = lse_merge_d(tot, LseD{s_rm[w2], s_rs[w2]});
            const double lzr = lse_value_d(tot);
            const bool ok = lzr != -__builtin_huge_val();
            status[b] = ok ? WFST_STATUS_OK : WFST_STATUS_NO_PATH;
            log_z[b] = ok ? (float)(s_pscale + lzr) : WFST_NINF;
        }
        __syncthreads();
    }
}

// EM M-step, per-state totals: one wavefront per source state; lane l sums
// the state's arcs l, l + 64, ... in order in FP64, then a fixed butterfly
// combines the lanes, so the total has the same bits on every call.
__global__ void em_source_sums(const int32_t *__restrict__ order, const int64_t *__restrict__ start, int32_t Q,
                               const float *__restrict__ counts, float smoothing, double *__restrict__ sums)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = wave; q < Q; q += waves) {
        double acc = 0.0;
        for (int64_t i = start[q] + lane; i < start[q + 1]; i += 64) acc += (double)counts[order[i]] + (double)smoothing;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) sums[q] = acc;
    }
}

// EM M-step, new scores: log(c_k + s) - log(total of the source state); a
// state with zero total keeps its scores.  new_score may alias cur_score.
__global__ void em_normalize(const int32_t *__restrict__ src, int64_t A, const float *__restrict__ counts,
                             float smoothing, const double *__restrict__ sums, const float *cur_score,
                             float *new_score)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < A; k += (int64_t)gridDim.x * blockDim.x) {
        const double tot = sums[src[k]];
        const double c = (double)counts[k] + (double)smoothing;
        new_score[k] = tot > 0.0 ? (float)(log(c) - log(tot)) : cur_score[k];
    }
}

__global__ void final_max_kernel(const float *__restrict__ fin, int32_t Q, float *__restrict__ out)
{
    __shared__ float red[1024];
    float m = WFST_NINF;
    for (int q = threadIdx.x; q < Q; q += blockDim.x) m = fmaxf(m, fin[q]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] > WFST_NINF ? red[0] : 0.0f;
}

}  // namespace wfst
