// Batch bookkeeping kernels: prefix sums, the length-bucketed sentence order,
// and a stable radix sort of token positions by input label.  All of them are
// deterministic (the sentence order inside one length bucket is the only
// exception, and it changes scheduling, never results).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace wfst {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;                          // per thread
constexpr int kScanTile = kScanThreads * kScanItems;  // elements per block

// In-block exclusive scan of one value per thread (kScanThreads threads).
template <class T>
__device__ T block_exclusive_scan(T v, T *s_buf, T &total)
{
    const int tid = threadIdx.x;
    s_buf[tid] = v;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const T add = tid >= o ? s_buf[tid - o] : T(0);
        __syncthreads();
        s_buf[tid] += add;
        __syncthreads();
    }
    total = s_buf[kScanThreads - 1];
    const T incl = s_buf[tid];
    __syncthreads();
    return incl - v;
}

// Value of element i for the scans: either a plain array or the segment
// count of token i's label in a layout.
struct ScanSource {
    const int64_t *i64 = nullptr;
    const int32_t *i32 = nullptr;
    const int32_t *tokens = nullptr;  // with label: n_segs of tokens[i]
    const LabelInfo *label = nullptr;
    int32_t M = 0;
    __device__ int64_t get(int64_t i) const
    {
        if (tokens) {
            const int a = tokens[i];
            return (a >= 0 && a < M) ? label[a].n_segs : 0;
        }
        return i64 ? i64[i] : (int64_t)i32[i];
    }
};

// phase 1: per-tile sums
__global__ void __launch_bounds__(kScanThreads) scan_tile_sums(ScanSource src, int64_t n, int64_t *tile_sum)
{
    __shared__ int64_t s_buf[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t v = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) v += src.get(i);
    }
    int64_t tot;
    (void)block_exclusive_scan<int64_t>(v, s_buf, tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// phase 2: exclusive scan of the tile sums in one block; total -> *total
__global__ void __launch_bounds__(kScanThreads) scan_tiles(int64_t *tile_sum, int64_t ntiles, int64_t *total)
{
    __shared__ int64_t s_buf[kScanThreads];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < ntiles; b0 += kScanThreads) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < ntiles ? tile_sum[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan<int64_t>(v, s_buf, tot);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// phase 3: exclusive scan inside each tile plus the tile's offset
template <class OutT>
__global__ void __launch_bounds__(kScanThreads) scan_apply(ScanSource src, int64_t n, const int64_t *tile_sum,
                                                          OutT *out)
{
    __shared__ int64_t s_buf[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t vals[kScanItems];
    int64_t v = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        vals[k] = i < n ? src.get(i) : 0;
        v += vals[k];
    }
    int64_t tot;
    int64_t run = block_exclusive_scan<int64_t>(v, s_buf, tot) + tile_sum[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) out[i] = (OutT)run;
        run += vals[k];
    }
}

// Sentence order for the persistent sweeps: longest first, in length buckets
// min(T, 1023).  One block of 1024 threads.
__global__ void __launch_bounds__(1024) order_by_length(const int32_t *__restrict__ offsets, int32_t B,
                                                        int32_t *__restrict__ order)
{
    __shared__ int hist[1024];
    __shared__ int s_buf[1024];
    const int tid = threadIdx.x;
    hist[tid] = 0;
    __syncthreads();
    for (int b = tid; b < B; b += 1024) {
        int n = offsets[b + 1] - offsets[b];
        n = n < 0 ? 0 : (n > 1023 ? 1023 : n);
        atomicAdd(&hist[1023 - n], 1);
    }
    __syncthreads();
    // exclusive scan of hist (1024 bins, one per thread)
    s_buf[tid] = hist[tid];
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int add = tid >= o ? s_buf[tid - o] : 0;
        __syncthreads();
        s_buf[tid] += add;
        __syncthreads();
    }
    hist[tid] = s_buf[tid] - hist[tid];
    __syncthreads();
    for (int b = tid; b < B; b += 1024) {
        int n = offsets[b + 1] - offsets[b];
        n = n < 0 ? 0 : (n > 1023 ? 1023 : n);
        order[atomicAdd(&hist[1023 - n], 1)] = b;
    }
}

// ---------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs (int32 or uint64 keys, int32
// values), 8 bits per pass.
// Tile = 1024 elements per block of 256 threads; each wavefront scatters a
// contiguous quarter of it.
// ---------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;

__device__ __forceinline__ int digit_of(int32_t key, int shift) { return ((uint32_t)key >> shift) & 0xff; }
__device__ __forceinline__ int digit_of(uint64_t key, int shift) { return (int)((key >> shift) & 0xff); }

// hist[d * ntiles + tile] = occurrences of digit d in the tile
template <class K>
__global__ void __launch_bounds__(kSortThreads) radix_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                           int64_t ntiles, int64_t *__restrict__ hist)
{
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + (int64_t)k * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Scatter with the scanned histogram (digit-major, tile-minor).  Wave w of a
// tile owns elements [64 I w, 64 I (w+1)) (I = kSortItems) in I rounds of 64
// consecutive elements; a lane's rank among equal digits before it comes from matching
// its digit against the wave with 8 ballots, so every pass is stable.
template <class K>
__global__ void __launch_bounds__(kSortThreads) radix_scatter(const K *__restrict__ keys_in,
                                                              const int32_t *__restrict__ vals_in, int64_t n,
                                                              int shift, int64_t ntiles,
                                                              const int64_t *__restrict__ offs,
                                                              K *__restrict__ keys_out,
                                                              int32_t *__restrict__ vals_out,
                                                              uint32_t *__restrict__ health)
{
    constexpr int NW = kSortThreads / 64;
    __shared__ int wcnt[NW][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = 0; j < 4; ++j) wcnt[wave][lane + 64 * j] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)wave * 64 * kSortItems;
    const unsigned long long lt = (1ull << lane) - 1ull;
    int dg[kSortItems], rank[kSortItems];
    K kv[kSortItems];
    int32_t vv[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {  // every round's loads in flight before the ranking
        const int64_t i = base + k * 64 + lane;
        kv[k] = i < n ? keys_in[i] : K(0);
        vv[k] = i < n ? vals_in[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + k * 64 + lane;
        const bool valid = i < n;
        const int d = valid ? digit_of(kv[k], shift) : 0;
        unsigned long long m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const unsigned long long bb = __ballot(valid && ((d >> b) & 1));
            m &= ((d >> b) & 1) ? bb : ~bb;
        }
        dg[k] = valid ? d : -1;
        rank[k] = 0;
        if (valid) rank[k] = wcnt[wave][d] + __popcll(m & lt);
        const bool leader = valid && (m >> lane) == 1ull;
        __builtin_amdgcn_wave_barrier();
        if (leader) wcnt[wave][d] += __popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        int run = 0;  // thread tid owns digit tid: exclusive prefix over waves
        for (int w = 0; w < NW; ++w) {
            const int c = wcnt[w][tid];
            wcnt[w][tid] = run;
            run += c;
        }
    }
    __syncthreads();
    int64_t pos[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k)  // the digits' tile offsets, all in flight
        pos[k] = dg[k] < 0 ? -1 : offs[(int64_t)dg[k] * ntiles + blockIdx.x] + wcnt[wave][dg[k]] + rank[k];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        if (dg[k] < 0) continue;
        if (pos[k] < 0 || pos[k] >= n) {
            atomicOr(health, H_SCATTER);
            continue;
        }
        keys_out[pos[k]] = kv[k];
        vals_out[pos[k]] = vv[k];
    }
}

}  // namespace wfst
