/*
 * wfst.h -- C ABI of the MI355X (gfx950) library for Viterbi decoding and
 * forward-backward over large sparse nondeterministic weighted finite-state
 * transducers, after Argueta & Chiang, "Decoding with Finite-State Transducers
 * on GPUs" (EACL 2017).
 *
 * Problem statement (paper, section 3): a WFST is (Q, Sigma, s, F, delta):
 * states 0..num_states-1, input symbols 0..num_ilabels-1, one start state s,
 * a final weight f[q] per state, and for every input symbol a a sparse
 * |Q|x|Q| transition matrix delta[a].  There are no epsilon arcs.  The weight
 * of an input string w_1..w_n is s^T (prod_t delta[w_t]) f (Eq. 1).
 *
 * Scores are log-domain FP32: arc_score = log p (higher is better; a cost
 * c maps to score -c), final_score[q] = log f[q] with -inf for a non-final
 * state.  Arcs are given as a flat list; the index of an arc in that list is
 * its arc id.  Arc ids are what paths report, what breaks Viterbi ties (the
 * lowest id wins) and what indexes posteriors and gradients.
 *
 * Viterbi evaluates Eq. 1 in the max-plus semiring with back-pointers (the
 * pair semiring of section 3 on log scores; section 5.1 for the packed
 * max and the on-device backtrace).  Forward-backward evaluates Eq. 1 in the
 * log semiring (section 5.2) and returns log Z and the expected arc counts of
 * Algorithm 2, which are also d(log Z)/d(arc_score).
 *
 * Conventions for every entry point
 *   - Return value 0 = success; a negative value is a call-level error
 *     (WFST_E*), with a message from wfst_last_error() on the calling thread.
 *     No C++ exception crosses this ABI.
 *   - Per-sentence outcomes go to a caller-owned status[] array (WFST_STATUS_*).
 *   - "device" pointers are HIP device memory on the FST's device, written or
 *     read asynchronously on `stream` (a hipStream_t; NULL = the null stream).
 *     Results are valid once the stream has reached the end of the call.
 *   - A batch is `batch` sentences: tokens[offsets[b] .. offsets[b+1]-1] is
 *     sentence b; offsets has batch+1 entries, offsets[0] = 0, non-decreasing,
 *     offsets[batch] = num_tokens (passed by value so that no device read is
 *     needed to size work); num_tokens < 2^31.
 *   - An FST owns one workspace that every call on it reuses: calls on one
 *     FST must be issued on one stream (or otherwise ordered); calls on
 *     different FSTs may overlap.
 */
#ifndef WFST_H
#define WFST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* call-level return codes */
#define WFST_OK 0
#define WFST_EINVAL (-1)       /* bad argument (range, NaN/inf score, null pointer, ...) */
#define WFST_ENOMEM (-2)       /* host or device allocation failed */
#define WFST_EHIP (-3)         /* a HIP runtime call failed; message carries its string */
#define WFST_EUNSUPPORTED (-4) /* size or option outside what this build supports */

/* per-sentence status codes */
#define WFST_STATUS_OK 0
#define WFST_STATUS_NO_PATH 1   /* no accepting path: score / log Z = -inf */
#define WFST_STATUS_BAD_TOKEN 2 /* a token outside [0, num_ilabels) */
#define WFST_STATUS_BAD_INPUT 3 /* offsets not non-decreasing or inconsistent with num_tokens */

typedef struct wfst_fst wfst_fst;   /* library-owned device layouts of one FST */
typedef struct wfst_tape wfst_tape; /* library-owned forward pass state for a backward call */

/* Optional creation parameters; pass NULL for defaults.  Zero fields mean "auto". */
typedef struct wfst_options {
    int32_t chunk_arcs;         /* arcs per lane chunk in the sliced layouts (1..64); 0 = auto */
    int32_t threads_per_sentence; /* workgroup size per sentence (64,128,256,512,1024); 0 = auto */
    int32_t checkpoint;         /* forward tape: -1/0 = auto, 1 = force sqrt(T) checkpointing, 2 = never */
    int32_t state_memory;       /* per-sentence state vectors of the sweeps: 0 = auto (LDS when they fit,
                                   else global memory: the forward sweep then runs as a team sweep, below,
                                   the other sweeps with a slot of global memory per workgroup),
                                   1 = LDS only (larger FSTs are refused), 2 = always global memory, one
                                   slot per workgroup, 3 = always global memory with the team forward
                                   sweep.  Team sweep: the workgroups on one XCD form a team that runs one
                                   sentence at a time, sharing out each step's slices and meeting at a
                                   device-scope barrier after the step (a cooperative launch; not used
                                   inside graphs, nor where the device cannot launch cooperatively, which
                                   fall back to per-workgroup slots).  A barrier wait is bounded: on a
                                   timeout the team stops and wfst_fst_health reports bit 64. */
    int64_t tape_budget_bytes;  /* auto mode checkpoints when the full tape exceeds this; 0 = 8 GiB */
    int64_t count_records;      /* expected counts: 0 = auto (per-visit records of the backward pass, grouped
                                   by arc and summed as 64-bit integers of scale 2^S as below (the same
                                   bits as -2), while they fit; else the label-grouped count kernel
                                   when its state fits LDS, else fixed-point accumulation),
                                   -1 = always the grouped count kernel,
                                   -2 = always fixed-point accumulation (each posterior added to its arc
                                   as a 64-bit integer of scale 2^S, S = 61 - floor(log2(num_tokens *
                                   max(1, max |grad_log_z|))): the sum does not depend on the order),
                                   > 0 = record capacity per call.  A backward sweep whose state is in
                                   global memory always uses fixed-point accumulation. */
} wfst_options;

/* Layout statistics (for tuning and reporting). */
typedef struct wfst_fst_info {
    int32_t num_states, num_ilabels, start, chunk_arcs;
    int64_t num_arcs;
    int64_t fwd_elements, rev_elements;   /* padded arc slots in each sliced layout */
    int64_t fwd_segments, rev_segments;   /* (label, dst) and (label, src) segments */
    int64_t fwd_slices, rev_slices;
    int32_t max_fwd_segments_per_label, max_rev_segments_per_label;
    int32_t max_fwd_slots_per_label, max_rev_slots_per_label;
    int64_t device_bytes;                 /* device memory held by the FST */
} wfst_fst_info;

/*
 * Build the device layouts of an FST (paper, section 4: arcs grouped per
 * input symbol; here further grouped by destination state for the forward and
 * Viterbi passes and by source state for the backward pass, and sliced for
 * 64-wide wavefronts).
 *   src, dst, ilabel: host int32[num_arcs], ranges [0,num_states) / [0,num_ilabels).
 *   olabel: host int32[num_arcs] or NULL (then best_olabels can not be asked for).
 *   arc_score: host float[num_arcs], finite (NaN/inf -> WFST_EINVAL); -0 is
 *     stored as +0.
 *   final_score: host float[num_states], finite or -inf (NaN/+inf -> EINVAL).
 *   start: the start state.  num_arcs < 2^31.
 * The passes keep per-sentence state vectors in LDS when they fit (Viterbi
 * also needs num_states < 65535 there); otherwise each persistent workgroup
 * keeps them in its own slot of global memory (at most 16 GiB of slots;
 * fewer sentences then run at once), unless options->state_memory = 1.
 * The caller keeps ownership of its arrays (they may be freed on return).
 * The library owns *out until wfst_fst_destroy.  Work is queued on `stream`
 * and the call returns after the uploads finished.
 */
int wfst_fst_create(int32_t num_states, int32_t num_ilabels, int32_t start, int64_t num_arcs,
                    const int32_t *src, const int32_t *dst, const int32_t *ilabel,
                    const int32_t *olabel, const float *arc_score, const float *final_score,
                    const wfst_options *options, void *stream, wfst_fst **out);

/* Replace the scores: the parameter update of training, where the expected
 * counts of Algorithm 2 feed expectation-maximisation or a gradient step
 * (paper, section 4).  arc_score_dev is a DEVICE float[num_arcs] in arc-id
 * order, scattered into both layouts through the stored permutation;
 * final_score_dev (nullable) a DEVICE float[num_states].  Values are not
 * validated (a NaN propagates).  Asynchronous on stream.  Every call bumps
 * the FST's score version (wfst_fst_score_version): a tape made before the
 * update can no longer be used by wfst_backward. */
int wfst_fst_set_scores(wfst_fst *fst, const float *arc_score_dev, const float *final_score_dev,
                        void *stream);

/* *version (host) receives the FST's score version: 0 after creation, plus one
 * per wfst_fst_set_scores call. */
int wfst_fst_score_version(const wfst_fst *fst, uint64_t *version);

/* Free the device layouts built by wfst_fst_create (the arrays of section 4 /
 * Figure 2 in their sliced form) and the FST's workspace.  Synchronises the
 * FST's device; every tape of the FST must have been freed first.  NULL-safe. */
void wfst_fst_destroy(wfst_fst *fst);

int wfst_fst_get_info(const wfst_fst *fst, wfst_fst_info *info);

/* Per input label (host int32[num_ilabels] each, any may be NULL): number of
 * arcs, of (label, destination) segments and of (label, source) segments. */
int wfst_fst_label_stats(const wfst_fst *fst, int32_t *arcs, int32_t *fwd_segments, int32_t *rev_segments);

/* Per-kernel timing for benchmarks.  While enabled, every launch of the
 * library's main kernels is bracketed by HIP events on the call's stream.
 * wfst_fst_profile_read waits for the recorded events and returns, per kernel
 * kind (WFST_KERNEL_*), the summed elapsed milliseconds and the number of
 * launches (host arrays of WFST_KERNEL_COUNT); reset != 0 forgets them. */
#define WFST_KERNEL_VITERBI 0    /* Viterbi sweep incl. final state and backtrace */
#define WFST_KERNEL_FORWARD 1    /* forward (alpha) sweep incl. log Z */
#define WFST_KERNEL_BACKWARD 2   /* backward (beta) sweep */
#define WFST_KERNEL_COUNTS 3     /* expected counts by label group */
#define WFST_KERNEL_SCORES 4     /* score scatter of wfst_fst_set_scores (both layouts) */
#define WFST_KERNEL_GRAD_FILL 5  /* zero fill of the gradient */
#define WFST_KERNEL_SCAN 6       /* time-parallel scan (all its launches) */
#define WFST_KERNEL_LATTICE 7    /* forward pass over input lattices */
#define WFST_KERNEL_COUNT 8
int wfst_fst_profile(wfst_fst *fst, int32_t enable);
int wfst_fst_profile_read(wfst_fst *fst, double *ms, int64_t *launches, int32_t reset);

/* Health bits of the FST's kernels (failure detection).  Every loop whose
 * bound comes from device memory is checked; on inconsistent data a kernel
 * stops that piece of work and sets a bit instead of running away:
 *   1 queue overrun, 2 count work item out of range, 4 visit / token /
 *   sentence index out of range, 8 partial-count slot out of range,
 *   16 sort scatter out of range, 32 label grouping overflow, 64 a team
 *   sweep's barrier timed out (its results are invalid).
 * Bits are sticky across calls.  *flags (host) receives the word after the
 * FST's work queued on `stream` has finished (the call synchronises the
 * stream); clear != 0 resets the word afterwards.  0 means healthy. */
int wfst_fst_health(const wfst_fst *fst, uint32_t *flags, int32_t clear, void *stream);

/* Testing hook for failure handling: the number of polls a team sweep's
 * barrier wait makes before the team stops (health bit 64); 0 restores the
 * default (2^24).  A small limit makes a team stop at its first barrier that
 * is not passed at once, so that the timeout path can be exercised without
 * any wait that does not end. */
int wfst_fst_debug_team_spin(wfst_fst *fst, int32_t polls);

/*
 * Viterbi decoding of a batch (paper, Algorithm 1 + section 5.1).
 * Outputs (caller-owned DEVICE memory):
 *   best_score float[batch]: FP32 score of the best accepting path, equal bit
 *     for bit to a serial evaluation that adds one arc score at a time
 *     (binary32, round to nearest even) and keeps the first of equal
 *     candidates in arc-id order; -inf when there is no path.
 *   best_arcs int32[num_tokens]: arc ids of that path, in input order
 *     (-1 for a sentence without a path).  Ties: lowest arc id per state and
 *     step, lowest state id among final states.
 *   best_olabels int32[num_tokens] or NULL: olabel of each path arc.
 *   status int32[batch].
 * An empty sentence scores final_score[start] with an empty path.
 */
int wfst_viterbi(const wfst_fst *fst, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                 const int32_t *tokens, float *best_score, int32_t *best_arcs,
                 int32_t *best_olabels, int32_t *status, void *stream);

/*
 * wfst_viterbi for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, outputs and results (bit for bit) as wfst_viterbi, but no
 * allocation of any kind and no host read-back.  Its scratch (queue counter,
 * sentence order, per-token offsets, scan tiles, back-pointers, path) lives in
 * one 256 MiB array per GPU, held until the process ends.  Limits:
 *   - num_tokens * (largest number of destination segments of one label)
 *     * 8 bytes, plus about 16 bytes per token and 4 per sentence, must fit
 *     256 MiB, else WFST_EUNSUPPORTED (before any work is queued);
 *   - only the on-chip form (state vectors in LDS): an FST that needs the
 *     global-memory form gives WFST_EUNSUPPORTED;
 *   - the FST's device must be the current device (else WFST_EINVAL).
 * Every call on one GPU uses the same scratch: calls that overlap on one GPU
 * (other streams, other threads, other FSTs) race and must be serialised by
 * the caller.
 */
int wfst_viterbi_noalloc(const wfst_fst *fst, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                         const int32_t *tokens, float *best_score, int32_t *best_arcs,
                         int32_t *best_olabels, int32_t *status, void *stream);

/*
 * Forward pass (paper, Algorithm 2 first loop, log semiring): log_z float[batch]
 * (DEVICE), status int32[batch] (DEVICE).  *tape_out receives a library-owned
 * record of the pass for wfst_backward; free it with wfst_tape_free.  The tape
 * keeps pointers to offsets/tokens: they must stay valid and unchanged until
 * the tape is freed.  log Z is the log of Eq. 1's value, -inf without a path.
 */
int wfst_forward(const wfst_fst *fst, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                 const int32_t *tokens, float *log_z, int32_t *status, wfst_tape **tape_out,
                 void *stream);

/*
 * Backward pass and expected counts (paper, Algorithm 2 second and last loops).
 *   grad_log_z: DEVICE float[batch] g_b, or NULL for all ones.
 *   grad_arc_score: DEVICE float[num_arcs], OVERWRITTEN with
 *     sum_b g_b * E_b[number of uses of arc k] = d(sum_b g_b log Z_b)/d score_k.
 *   grad_final: DEVICE float[num_states] or NULL, overwritten with
 *     sum_b g_b * P_b(path ends in q).
 * Sentences without a path (or with a bad token) contribute zero.  The sums
 * over b and over visits are taken in a fixed order, or (per-visit records,
 * fixed-point accumulation) as 64-bit integers whose sum does not depend on
 * the order: results are bitwise reproducible for a given FST, batch and
 * library configuration, and the records give the same bits as fixed-point
 * accumulation.
 * Returns WFST_EINVAL when the FST's scores were replaced (set_scores) after
 * the forward pass that made the tape: the counts would pair the old alpha
 * with the new scores.
 */
int wfst_backward(const wfst_fst *fst, const wfst_tape *tape, const float *grad_log_z,
                  float *grad_arc_score, float *grad_final, void *stream);

/* Return a tape's buffers (the stored forward variables of Algorithm 2, or
 * their checkpoints) to its FST's pool.  NULL-safe; the FST must still exist. */
void wfst_tape_free(wfst_tape *tape);

/* The whole of Algorithm 2 (forward loop, backward loop, expected counts) with
 * g_b = 1: log_z float[batch], arc_posterior float[num_arcs] = sum_b
 * E_b[count_k] (for batch = 1 each value is in [0, n] and they sum to n),
 * final_posterior float[num_states] or NULL, status int32[batch].  DEVICE
 * memory, overwritten; errors as wfst_forward and wfst_backward. */
int wfst_forward_backward(const wfst_fst *fst, int32_t batch, int64_t num_tokens,
                          const int32_t *offsets, const int32_t *tokens, float *log_z,
                          float *arc_posterior, float *final_posterior, int32_t *status,
                          void *stream);

/*
 * Autotuner for batched decoding and training (the batching step of the
 * method: persistent workgroups popping sentences longest first; section 5
 * launches one kernel per symbol, and section 7.5 reports that its launch
 * overhead dominated small FSTs, which is why every launch parameter here is
 * measured rather than fixed).  On the given batch (offsets/tokens DEVICE, as
 * in wfst_viterbi) it times one batched Viterbi + forward + backward pass,
 * after one untimed pass, for each
 *   - workgroup size per sentence in {64, 128, 256, 512, 1024},
 *   - count path: 0 per-visit records, -1 label-grouped kernel, -2 fixed-point
 *     accumulation (those the FST's state sizes allow), and
 *   - with flags & WFST_TUNE_CHUNK: arcs per lane chunk in {4, 8, 16, 32},
 *     rebuilding both layouts from the device layout for each (arcs and their
 *     current scores are read back; the FST keeps no host copy),
 * and keeps the fastest for later calls on this FST.  Sentences are always
 * processed longest first in exact-length order (the finest length buckets),
 * so there are no bucket edges to tune.  Results of every configuration stay
 * exact (Viterbi bit-exact, forward-backward within its stated accuracy); only
 * speed changes.  A rebuild makes earlier tapes of the FST unusable
 * (wfst_backward refuses them).
 *   cache_path: NULL, or a JSON file of earlier choices keyed by device
 *     architecture, FST size (states, labels, arcs) and batch shape
 *     (sentences, tokens, mean arcs per token, log2 histogram of lengths); a
 *     hit applies the stored choice without timing, a miss tunes and adds the
 *     entry (the file is rewritten through a temporary file).
 *   result: HOST, or NULL.
 * Allocates and frees scratch outputs (one float per arc among them) and
 * synchronises the stream: call it off the hot path.  On error the FST keeps
 * its previous configuration.
 */
#define WFST_TUNE_CHUNK 1

typedef struct wfst_autotune_result {
    int32_t threads_per_sentence;  /* chosen configuration */
    int32_t count_records;         /* chosen count path (0, -1 or -2, as wfst_options.count_records) */
    int32_t chunk_arcs;
    int32_t from_cache;            /* 1: taken from the cache file, nothing timed */
    int32_t tried;                 /* configurations timed */
    float best_ms;                 /* ms of one pass with the chosen configuration (as timed or stored) */
    int32_t chunks[4];             /* chunk length of each row of ms (0 = row unused) */
    float ms[4][5][3];             /* ms per pass [chunk row][workgroup size][count path]; -1 = not run */
} wfst_autotune_result;

int wfst_fst_autotune(wfst_fst *fst, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                      const int32_t *tokens, const char *cache_path, int32_t flags,
                      wfst_autotune_result *result, void *stream);

/*
 * Forward pass as a time-parallel scan (paper, section 6.1: the product of
 * Eq. 1 is associative, so a parallel prefix computes it in log T depth;
 * the paper leaves this to future work).  For FSTs with at most 64 states:
 * every token's delta[w_t] becomes a dense |Q| x |Q| log-semiring matrix
 * (parallel arcs log-added in arc-id order), and an inclusive scan over each
 * sentence's matrices (ceil(log2 T_max) levels, each a matrix product per
 * token, every entry a log-sum-exp over the inner index in increasing order)
 * gives the prefix products P_t = delta[w_1] ... delta[w_t].  With the
 * one-hot start vector, log alpha_t = row `start` of P_t and
 * log Z = log sum_q exp(P_T[start][q] + final[q]) (FP64 accumulation).
 * This is the latency path: depth log T instead of T, at |Q|^3 work per
 * product and two matrices per token (at most 32 GiB); the sweeps of
 * wfst_forward are the throughput path.
 *   log_z float[batch], status int32[batch]: as wfst_forward (DEVICE).
 *   alpha: NULL or DEVICE float[num_tokens * num_states]: row i = log alpha
 *     after token i (unnormalised, natural log).
 * Errors: WFST_EUNSUPPORTED for num_states > 64 or a batch beyond the matrix
 * budget.  Reads back the longest sentence length (synchronises the stream).
 */
int wfst_forward_scan(const wfst_fst *fst, int32_t batch, int64_t num_tokens, const int32_t *offsets,
                      const int32_t *tokens, float *log_z, float *alpha, int32_t *status, void *stream);

/*
 * Forward pass over input lattices: the FST composed with an acyclic weighted
 * acceptor over input labels instead of a string (paper, section 6.1 names
 * input lattices as the case the prefix-sum scan does not cover; section 3
 * rules out epsilon transitions in the FST, which stays so: epsilon here is
 * on lattice arcs only).  Lattice b has nodes node_offsets[b] ..
 * node_offsets[b+1]-1 (local ids 0..n_b-1, in topological order; local 0 is
 * the start node, n_b-1 the end node) and arcs arc_offsets[b] ..
 * arc_offsets[b+1]-1, each (from, to, label, weight) with local node ids,
 * from < to, label in [0, num_input_labels) or -1 for epsilon, weight a
 * natural-log score (-inf = disabled arc), and the arcs of a lattice sorted by
 * `to` (stable order among equal `to` is the summation order).  With A_0 the
 * one-hot vector of the FST's start state and, for node v, in arc order,
 *   A_v = log-sum over incoming arcs (u, v, a, w) of
 *         (A_u (x) delta[a]) + w   (Eq. 1 in the log semiring), or A_u + w for epsilon,
 *   log Z_b = log sum_q exp(A_{n_b-1}[q] + final[q]).
 * A string w_1..w_T is the chain lattice 0 -w_1-> 1 ... -w_T-> T with zero
 * weights, for which this equals wfst_forward.  One persistent workgroup per
 * lattice; the node vectors are kept normalised (FP32 with an FP64 scale per
 * node) and incoming contributions are log-added in FP64 on chip.
 *   node_offsets, arc_offsets: DEVICE int32[batch + 1], non-decreasing, every
 *     lattice with at least one node.
 *   arc_from, arc_to, arc_label: DEVICE int32[num_arcs]; arc_weight DEVICE float[num_arcs].
 *   log_z: DEVICE float[batch]; status: DEVICE int32[batch] (WFST_STATUS_*:
 *     BAD_INPUT for a malformed lattice or non-monotone offsets anywhere in
 *     the batch, BAD_TOKEN for a label out of range, NO_PATH when nothing
 *     reaches a final state; log_z = -inf in all of these).
 *   node_log_alpha: NULL or DEVICE float[num_nodes * num_states]: A_v per node
 *     (natural log, unnormalised).
 * Errors: WFST_EINVAL for negative sizes or NULL buffers; WFST_EUNSUPPORTED
 * when the FST's state vector and its largest label's segments do not fit
 * the on-chip accumulator.  Does not synchronise the stream.
 */
int wfst_lattice_forward(const wfst_fst *fst, int32_t batch, const int32_t *node_offsets,
                         const int32_t *arc_offsets, int64_t num_nodes, int64_t num_arcs, const int32_t *arc_from,
                         const int32_t *arc_to, const int32_t *arc_label, const float *arc_weight, float *log_z,
                         float *node_log_alpha, int32_t *status, void *stream);

/*
 * EM M-step (paper, section 4: the expected counts of Algorithm 2 serve
 * expectation-maximisation of the transducer's weights).  The FST is read as
 * a locally normalised model p(arc | source state) with fixed final weights:
 *   new_score[k] = log(counts[k] + smoothing)
 *                  - log(sum over arcs j leaving src_k of (counts[j] + smoothing)),
 * and the arcs of a state whose total is 0 keep cur_score.  With smoothing 0
 * and counts from wfst_backward (grad_log_z = ones) under cur_score, this is
 * one EM iteration, which cannot lower sum_b log Z_b.
 *   counts, cur_score: DEVICE float[num_arcs] (arc-id order).
 *   new_score: DEVICE float[num_arcs], may be cur_score; apply it with
 *     wfst_fst_set_scores.
 *   smoothing: finite, >= 0 (else WFST_EINVAL).
 * Per-state totals are summed in FP64 in a fixed order: results are bitwise
 * reproducible.  The first call on an FST builds an index of its arcs by
 * source state (read back from the device layout; synchronises the stream;
 * 8 bytes per arc of device memory).
 */
int wfst_em_update(wfst_fst *fst, const float *counts, float smoothing, const float *cur_score,
                   float *new_score, void *stream);

/*
 * HIP graphs of a whole batched pass sequence (the batching step of the
 * method: section 5 launches one kernel per input symbol, and section 7.5
 * finds launch overhead dominating small FSTs; here a pass is a few
 * persistent launches, and a graph replays all of them, with the plan and
 * count kernels around them, as one submission).
 *
 * wfst_graph_create captures, for one batch shape and one set of argument
 * pointers (all DEVICE memory, bound into the graph):
 *   1. when arc_score != NULL: wfst_fst_set_scores(fst, arc_score, NULL),
 *   2. when best_score != NULL: wfst_viterbi into best_score / best_arcs /
 *      best_olabels (nullable) / status,
 *   3. when log_z != NULL: wfst_forward into log_z / status, then, when
 *      grad_arc_score != NULL, wfst_backward with grad_log_z (nullable =
 *      ones) into grad_arc_score and grad_final (nullable).
 * A replay (wfst_graph_launch) computes the same as those calls on whatever
 * the bound input buffers hold at that time (same batch and token counts),
 * bit for bit, except that counts the eager call would take from per-visit
 * records are taken in fixed point (equal to an eager call with
 * count_records = -2 bit for bit, and so to the records).  The graph has its own
 * workspace and tape buffers, so eager calls on the FST between replays are
 * allowed (on the same stream).  Inside a graph nothing is read back to the
 * host, so:
 *   - buffers are sized by the bound num_tokens x (largest destination-
 *     segment count of a label); bounds above 2 GiB give WFST_EUNSUPPORTED;
 *   - the forward tape is kept whole (checkpointing needs device totals):
 *     a bound above the tape budget, or checkpoint = 1, gives EUNSUPPORTED;
 *   - counts that would take per-visit records take the fixed-point path.
 * Creation runs the sequence once eagerly (its outputs are written), then
 * captures it on `stream`, which must be a created stream (not the null
 * stream); it synchronises the stream.  Layout rebuilds by the autotuner are
 * refused while graphs of the FST exist.  Destroy graphs before the FST.
 * A replay with arc_score counts as a score update for earlier tapes.
 */
typedef struct wfst_graph wfst_graph;

typedef struct wfst_graph_args {
    int32_t batch;
    int64_t num_tokens;
    const int32_t *offsets;        /* [batch+1] */
    const int32_t *tokens;         /* [num_tokens] */
    const float *arc_score;        /* [num_arcs] or NULL: scores set at the start of every replay */
    float *best_score;             /* [batch] or NULL: no Viterbi */
    int32_t *best_arcs;            /* [num_tokens] (with best_score) */
    int32_t *best_olabels;         /* [num_tokens] or NULL */
    float *log_z;                  /* [batch] or NULL: no forward-backward */
    const float *grad_log_z;       /* [batch] or NULL (ones) */
    float *grad_arc_score;         /* [num_arcs] or NULL: forward only */
    float *grad_final;             /* [num_states] or NULL */
    int32_t *status;               /* [batch], required */
} wfst_graph_args;

int wfst_graph_create(wfst_fst *fst, const wfst_graph_args *args, void *stream, wfst_graph **out);
int wfst_graph_launch(wfst_graph *graph, void *stream);
/* Synchronises the graph's device, then frees it.  NULL-safe. */
void wfst_graph_destroy(wfst_graph *graph);

/*
 * Reader for the AT&T / OpenFST text format (paper, section 7.2: the FSTs are
 * read from OpenFST's text form; section 5.1: output symbols of the best path
 * are looked up in O).  Host only, no GPU.
 *   fst_text[fst_len]: lines "src dst ilabel olabel [weight]" (an arc) or
 *     "state [weight]" (a final state), blank/tab separated.  The source of
 *     the first line is the start state.  Weights are costs (-log p): the
 *     score is -weight, a missing weight is 0; a final weight "inf" /
 *     "Infinity" marks a non-final state.  Arc weights must be finite.
 *   isyms_text / osyms_text (nullable, with lengths): symbol tables, lines
 *     "symbol id"; labels that are not in the table must be non-negative
 *     integers.
 *   epsilon_zero != 0: label id 0 is epsilon, and an epsilon input label is
 *     refused with WFST_EUNSUPPORTED (the method has no epsilon transitions,
 *     section 3).
 * First call with all arrays NULL: counts[4] (HOST) receives {num_states =
 * largest state id + 1, num_ilabels = largest input id (of the arcs or the
 * input table) + 1, num_arcs, start}.  Second call: HOST arrays src, dst,
 * ilabel, olabel (nullable), arc_score [num_arcs] and final_score
 * [num_states] (-inf for non-final states), arcs in file order (arc id =
 * line order), ready for wfst_fst_create.  Errors name the line; the message
 * comes from wfst_att_last_error().
 */
int wfst_att_parse(const char *fst_text, int64_t fst_len, const char *isyms_text, int64_t isyms_len,
                   const char *osyms_text, int64_t osyms_len, int32_t epsilon_zero, int64_t *counts,
                   int32_t *src, int32_t *dst, int32_t *ilabel, int32_t *olabel, float *arc_score,
                   float *final_score);
const char *wfst_att_last_error(void);

/* Message for the last nonzero return on this thread ("" if none). */
const char *wfst_last_error(void);

/*
 * Host-only layout query for tests (no GPU needed).  Builds the forward
 * (direction 0: grouped by label then destination) or reverse (direction 1:
 * by label then source) sliced layout into caller-allocated host arrays.
 * Call first with all output pointers NULL to get the sizes in *sizes:
 *   sizes[0] = elements, sizes[1] = slices, sizes[2] = segments.
 * elem_other int32[elements]: the other end state of each slot (num_states
 *   for a padding slot); elem_arc int32[elements]: arc id (-1 padding);
 * slice_info int32[4*slices] {base, height, width, label};
 * seg_info int32[4*segments] {key state, first chunk, chunks, label};
 * label_slice int32[num_ilabels+1], label_seg int32[num_ilabels+1].
 */
int wfst_layout_host(int32_t num_states, int32_t num_ilabels, int64_t num_arcs,
                     const int32_t *src, const int32_t *dst, const int32_t *ilabel,
                     int32_t direction, int32_t chunk_arcs, int64_t *sizes,
                     int32_t *elem_other, int32_t *elem_arc, int32_t *slice_info,
                     int32_t *seg_info, int32_t *label_slice, int32_t *label_seg);

#ifdef __cplusplus
}
#endif

#endif /* WFST_H */
