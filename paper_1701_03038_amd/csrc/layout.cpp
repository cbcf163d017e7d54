// Host construction of the sliced per-label arc layouts (see layout.h).
#include "layout.h"

#include <algorithm>
#include <numeric>
#include <thread>

#include "../../include/wfst.h"

namespace wfst {
namespace {

int host_threads()
{
    unsigned n = std::thread::hardware_concurrency();
    if (n == 0) n = 1;
    return (int)std::min(n, 16u);
}

// Run f(begin, end, thread) over [0, n) split into contiguous ranges.
template <class F>
void parallel_ranges(int64_t n, int nthreads, F f)
{
    if (nthreads <= 1 || n < 65536) {
        f((int64_t)0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    const int64_t per = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        const int64_t b = std::min<int64_t>(n, (int64_t)t * per);
        const int64_t e = std::min<int64_t>(n, b + per);
        th.emplace_back(f, b, e, t);
    }
    for (auto &x : th) x.join();
}

// Stable counting sort of the ids in `in` by key[id] into `out`; bucket
// starts (nkeys + 1 entries) are written to starts when non-null.
void counting_sort(const int32_t *key, int32_t nkeys, const int32_t *in, int32_t *out, int64_t n,
                   std::vector<int64_t> *starts)
{
    int T = host_threads();
    if (n < 65536) T = 1;
    std::vector<std::vector<int64_t>> hist(T, std::vector<int64_t>((size_t)nkeys, 0));
    const int64_t per = (n + T - 1) / T;
    parallel_ranges(n, T, [&](int64_t b, int64_t e, int t) {
        auto &h = hist[t];
        for (int64_t i = b; i < e; ++i) h[key[in[i]]] += 1;
    });
    int64_t run = 0;
    if (starts) starts->assign((size_t)nkeys + 1, 0);
    for (int32_t k = 0; k < nkeys; ++k) {
        if (starts) (*starts)[k] = run;
        for (int t = 0; t < T; ++t) {
            const int64_t c = hist[t][k];
            hist[t][k] = run;
            run += c;
        }
    }
    if (starts) (*starts)[nkeys] = run;
    (void)per;
    parallel_ranges(n, T, [&](int64_t b, int64_t e, int t) {
        auto &h = hist[t];
        for (int64_t i = b; i < e; ++i) out[h[key[in[i]]]++] = in[i];
    });
}

struct Seg {
    int64_t start;  // position in the sorted id order
    int32_t len;
    int32_t key;
};

// Segments of one label in layout order: decreasing length, then key.
void label_segments(const int32_t *order, int64_t lo, int64_t hi, const int32_t *key,
                    std::vector<Seg> &segs)
{
    segs.clear();
    int64_t i = lo;
    while (i < hi) {
        const int32_t k = key[order[i]];
        int64_t j = i + 1;
        while (j < hi && key[order[j]] == k) ++j;
        segs.push_back(Seg{i, (int32_t)(j - i), k});
        i = j;
    }
    // runs are found in increasing key order, so a stable sort by length keeps key order on ties
    std::stable_sort(segs.begin(), segs.end(), [](const Seg &a, const Seg &b) { return a.len > b.len; });
}

struct LabelCounts {
    int64_t elems = 0;
    int32_t slices = 0, segs = 0, n_multi = 0, n_slots = 0, max_h = 0;
};

}  // namespace

int32_t auto_chunk(int32_t, int32_t, int64_t) { return 16; }

int build_layout(int32_t Q, int32_t M, int64_t A, const int32_t *src, const int32_t *dst,
                 const int32_t *ilabel, const float *score, int direction, int32_t L,
                 HostLayout &out, std::string &err)
{
    if (L < 1 || L > 64) {
        err = "chunk_arcs must be in [1, 64]";
        return WFST_EINVAL;
    }
    const int32_t *key = direction == 0 ? dst : src;
    const int32_t *other = direction == 0 ? src : dst;

    // arc ids sorted by (label, key, id): stable sort by key, then stable by label
    std::vector<int32_t> ids((size_t)A), tmp((size_t)A);
    std::iota(ids.begin(), ids.end(), 0);
    std::vector<int64_t> lstart;
    counting_sort(key, Q, ids.data(), tmp.data(), A, nullptr);
    counting_sort(ilabel, M, tmp.data(), ids.data(), A, &lstart);
    std::vector<int32_t>().swap(tmp);
    const int32_t *order = ids.data();

    const int T = host_threads();
    std::vector<LabelCounts> cnt((size_t)M);
    // pass 1: sizes per label
    parallel_ranges(M, T, [&](int64_t a0, int64_t a1, int) {
        std::vector<Seg> segs;
        std::vector<int32_t> clen;
        for (int64_t a = a0; a < a1; ++a) {
            LabelCounts &c = cnt[(size_t)a];
            label_segments(order, lstart[a], lstart[a + 1], key, segs);
            c.segs = (int32_t)segs.size();
            clen.clear();
            for (const Seg &s : segs) {
                const int32_t nch = (s.len + L - 1) / L;
                if (nch > 1) {
                    c.n_multi += 1;
                    c.n_slots += nch;
                }
                for (int32_t p = 0; p < nch; ++p) clen.push_back(std::min(L, s.len - p * L));
            }
            const int64_t C = (int64_t)clen.size();
            c.slices = (int32_t)((C + 63) / 64);
            for (int64_t s = 0; s < c.slices; ++s) {
                const int64_t c0 = s * 64, c1 = std::min<int64_t>(C, c0 + 64);
                int32_t h = 0;
                for (int64_t x = c0; x < c1; ++x) h = std::max(h, clen[(size_t)x]);
                c.elems += (int64_t)h * (c1 - c0);
                c.max_h = std::max(c.max_h, h);
            }
        }
    });

    // bases
    out = HostLayout();
    out.num_states = Q;
    out.num_ilabels = M;
    out.chunk = L;
    out.label.resize((size_t)M);
    int64_t e_run = 0, s_run = 0, g_run = 0;
    for (int32_t a = 0; a < M; ++a) {
        const LabelCounts &c = cnt[(size_t)a];
        LabelInfo &li = out.label[(size_t)a];
        if (e_run > INT32_MAX || s_run > INT32_MAX || g_run > INT32_MAX) break;
        li.slice_first = (int32_t)s_run;
        li.n_slices = c.slices;
        li.seg_first = (int32_t)g_run;
        li.n_segs = c.segs;
        li.n_multi = c.n_multi;
        li.n_slots = c.n_slots;
        li.elem_first = (int32_t)e_run;
        li.n_elems = (int32_t)c.elems;
        e_run += c.elems;
        s_run += c.slices;
        g_run += c.segs;
        out.max_segs = std::max(out.max_segs, c.segs);
        out.max_slots = std::max(out.max_slots, c.n_slots);
        out.max_elems = (int32_t)std::min<int64_t>(INT32_MAX, std::max<int64_t>(out.max_elems, c.elems));
        out.max_height = std::max(out.max_height, c.max_h);
        out.max_slices = std::max(out.max_slices, c.slices);
    }
    if (e_run >= INT32_MAX || s_run >= INT32_MAX || g_run >= INT32_MAX) {
        err = "layout exceeds 2^31-1 elements, slices or segments";
        return WFST_EUNSUPPORTED;
    }
    out.other.resize((size_t)e_run);
    out.score.resize((size_t)e_run);
    out.elem_arc.resize((size_t)e_run);
    out.slice.resize((size_t)s_run);
    out.seg_key.resize((size_t)g_run);
    out.seg_chunk.resize((size_t)g_run);

    // pass 2: fill
    parallel_ranges(M, T, [&](int64_t a0, int64_t a1, int) {
        std::vector<Seg> segs;
        std::vector<int32_t> cseg, cpart, clen;
        for (int64_t a = a0; a < a1; ++a) {
            const LabelInfo &li = out.label[(size_t)a];
            label_segments(order, lstart[a], lstart[a + 1], key, segs);
            cseg.clear();
            cpart.clear();
            clen.clear();
            for (size_t j = 0; j < segs.size(); ++j) {
                const Seg &s = segs[j];
                const int32_t nch = (s.len + L - 1) / L;
                out.seg_key[(size_t)li.seg_first + j] = s.key;
                out.seg_chunk[(size_t)li.seg_first + j] = SegChunk{(int32_t)cseg.size(), nch};
                for (int32_t p = 0; p < nch; ++p) {
                    cseg.push_back((int32_t)j);
                    cpart.push_back(p);
                    clen.push_back(std::min(L, s.len - p * L));
                }
            }
            const int64_t C = (int64_t)cseg.size();
            int64_t base = li.elem_first;
            for (int32_t s = 0; s < li.n_slices; ++s) {
                const int64_t c0 = (int64_t)s * 64, c1 = std::min<int64_t>(C, c0 + 64);
                const int32_t w = (int32_t)(c1 - c0);
                int32_t h = 0;
                for (int64_t x = c0; x < c1; ++x) h = std::max(h, clen[(size_t)x]);
                out.slice[(size_t)li.slice_first + s] = SliceInfo{(int32_t)base, h, w, (int32_t)a};
                for (int32_t r = 0; r < h; ++r) {
                    for (int32_t l = 0; l < w; ++l) {
                        const int64_t c = c0 + l;
                        const int64_t e = base + (int64_t)r * w + l;
                        if (r < clen[(size_t)c]) {
                            const Seg &sg = segs[(size_t)cseg[(size_t)c]];
                            const int32_t arc = order[sg.start + (int64_t)cpart[(size_t)c] * L + r];
                            const float sc = score ? (score[arc] == 0.0f ? 0.0f : score[arc]) : 0.0f;
                            out.other[(size_t)e] = other[arc];
                            out.score[(size_t)e] = sc;
                            out.elem_arc[(size_t)e] = arc;
                        } else {
                            out.other[(size_t)e] = Q;
                            out.score[(size_t)e] = 0.0f;
                            out.elem_arc[(size_t)e] = -1;
                        }
                    }
                }
                base += (int64_t)h * w;
            }
        }
    });
    return WFST_OK;
}

}  // namespace wfst
