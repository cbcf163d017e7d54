// Host-side sliced arc layouts shared by the C ABI and the kernels.
//
// A layout groups the arcs of the FST by input label (the per-symbol blocks
// R[a]..R[a+1]-1 of the paper's section 4), then within a label by a key
// state: the destination for the forward layout (each step reduces into a
// destination, the CSC order the paper mentions at the end of section 4) and
// the source for the reverse layout (backward steps reduce into a source).
//
// Each (label, key) group of arcs is a *segment*; its arcs are in increasing
// arc id.  Segments are cut into *chunks* of at most `chunk` arcs; one GPU lane
// reduces one chunk serially.  Chunks of a label are packed 64 at a time into
// *slices* (one wavefront): slice element (r, l) -- row r of the chunk held by
// lane l -- lives at base + r * width + l, so a wavefront reading row r loads
// `width` consecutive entries of each element array (other state, score).
// Chunks shorter than the slice height are padded with a dead element (other
// state = num_states, score 0).  Scores are an array of their own so that a
// score update writes whole cache lines.
//
// Within a label, segments are ordered by decreasing arc count, then by key
// state.  Segments with more than `chunk` arcs ("multi-chunk") therefore come
// first and own the label's first `n_slots` chunks; every later segment is a
// single chunk, and chunk c >= n_slots belongs to segment
// n_multi + (c - n_slots).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace wfst {

// One element as a kernel holds it in registers (stored as two arrays).
struct Elem {
    int32_t other;  // the non-key end state of the arc (num_states = padding)
    float score;    // arc score (log domain)
};

struct SliceInfo {
    int32_t base;   // first element
    int32_t height; // rows (max chunk length in the slice)
    int32_t width;  // chunks (lanes) in the slice, 1..64
    int32_t label;
};

struct LabelInfo {
    int32_t slice_first, n_slices;  // global slice range
    int32_t seg_first, n_segs;      // global segment range
    int32_t n_multi, n_slots;       // multi-chunk segments and the chunks they own
    int32_t elem_first, n_elems;    // element range of the label
};

struct SegChunk {
    int32_t first;  // first chunk, relative to the label
    int32_t count;  // number of chunks
};

struct HostLayout {
    int32_t num_states = 0, num_ilabels = 0, chunk = 0;
    std::vector<int32_t> other;      // non-key end state per element (num_states for padding)
    std::vector<float> score;        // arc score per element (0 for padding)
    std::vector<int32_t> elem_arc;   // arc id per element, -1 for padding
    std::vector<SliceInfo> slice;
    std::vector<int32_t> seg_key;    // key state per segment
    std::vector<SegChunk> seg_chunk;
    std::vector<LabelInfo> label;    // num_ilabels entries
    int32_t max_segs = 0, max_slots = 0, max_elems = 0, max_height = 0, max_slices = 0;
};

// direction 0: key = dst, other = src (forward); 1: key = src, other = dst.
// Returns 0 or a negative WFST_E* code with a message in err.
int build_layout(int32_t num_states, int32_t num_ilabels, int64_t num_arcs, const int32_t *src,
                 const int32_t *dst, const int32_t *ilabel, const float *score, int direction,
                 int32_t chunk, HostLayout &out, std::string &err);

// Pick a chunk size for a label-arc profile (used when options ask for auto).
int32_t auto_chunk(int32_t num_states, int32_t num_ilabels, int64_t num_arcs);

}  // namespace wfst
