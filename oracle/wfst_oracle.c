/*
 * Serial CPU oracle for Viterbi and forward-backward over a weighted FST.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code,
 * header or table with the GPU library; it is slow and plain on purpose so
 * that it can be checked against the paper by eye.
 *
 * The problem (paper, section 3): a WFST M = (Q, Sigma, s, F, delta) with a
 * single start state s, final weights f and, for every input symbol a, a
 * sparse |Q|x|Q| transition matrix delta[a]; no epsilon arcs.  The weight of
 * a string w_1..w_n is s^T (prod_t delta[w_t]) f (Eq. 1), evaluated in a
 * semiring.  Arcs are a flat list; the index of an arc in that list is its id.
 *
 * Scores are log-domain (score = log p, higher is better), so
 *   - Viterbi is Eq. 1 in the max-plus semiring with back-pointers
 *     (the pair semiring of section 3, written on log scores), and
 *   - forward-backward is Eq. 1 in the log semiring (section 5.2 works in
 *     log-probabilities), plus the expected arc counts of Algorithm 2.
 *
 * Arcs are grouped per input label as in the CSR/COO arrays of section 4
 * (Figure 2): R[a]..R[a+1]-1 index the arcs carrying input label a, in
 * increasing arc id.
 *
 * Readings taken where the paper is silent or inconsistent:
 *   - Ties in Viterbi go to the LOWEST arc id (the paper's "otherwise" branch
 *     and its packed atomicMax would keep the highest); final-state ties go
 *     to the lowest state id.
 *   - Viterbi works on FP32 log scores: each candidate is one IEEE binary32
 *     round-to-nearest-even addition alpha[src] + score (no FMA, no flush to
 *     zero).  Candidates whose source score is -inf are skipped.
 *   - Algorithm 2's backward and count loops are read with backward[t+1] and
 *     delta[w_{t+1}] (the printed indices are off by one), counts are kept
 *     per arc rather than per state pair, and every forward/backward cell
 *     starts at the semiring zero.
 *   - Forward-backward runs in FP64; log-sum-exp is max-shifted,
 *     LSE(x) = m + log(sum exp(x_i - m)), and an empty or all -inf set gives
 *     -inf.
 *   - A sentence with no accepting path has score / log Z = -inf, status
 *     NO_PATH and contributes zero to the posteriors.  A token outside
 *     [0, num_ilabels) gives status BAD_TOKEN.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define ST_OK 0
#define ST_NO_PATH 1
#define ST_BAD_TOKEN 2

/* R (label offsets, M+1 entries) and K (arc ids grouped by label, ascending
 * id within each label): a stable counting sort of the arc list by label. */
static int label_index(int32_t M, int64_t A, const int32_t *ilabel, int64_t **R_out, int64_t **K_out)
{
    int64_t *R = (int64_t *)calloc((size_t)M + 1, sizeof(int64_t));
    int64_t *K = (int64_t *)malloc((size_t)(A > 0 ? A : 1) * sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc(((size_t)M + 1) * sizeof(int64_t));
    if (!R || !K || !fill) {
        free(R); free(K); free(fill);
        return OR_ENOMEM;
    }
    for (int64_t k = 0; k < A; ++k) R[ilabel[k] + 1] += 1;
    for (int32_t a = 0; a < M; ++a) R[a + 1] += R[a];
    memcpy(fill, R, ((size_t)M + 1) * sizeof(int64_t));
    for (int64_t k = 0; k < A; ++k) K[fill[ilabel[k]]++] = k;
    free(fill);
    *R_out = R;
    *K_out = K;
    return OR_OK;
}

static int check_fst(int32_t Q, int32_t M, int32_t start, int64_t A, const int32_t *src,
                     const int32_t *dst, const int32_t *ilabel)
{
    if (Q <= 0 || M <= 0 || start < 0 || start >= Q || A < 0) return OR_EINVAL;
    for (int64_t k = 0; k < A; ++k) {
        if (src[k] < 0 || src[k] >= Q || dst[k] < 0 || dst[k] >= Q) return OR_EINVAL;
        if (ilabel[k] < 0 || ilabel[k] >= M) return OR_EINVAL;
    }
    return OR_OK;
}

static int64_t max_len(int32_t B, const int64_t *offsets)
{
    int64_t m = 0;
    for (int32_t b = 0; b < B; ++b) {
        int64_t n = offsets[b + 1] - offsets[b];
        if (n > m) m = n;
    }
    return m;
}

static int bad_tokens(int32_t M, int64_t n, const int32_t *w)
{
    for (int64_t t = 0; t < n; ++t)
        if (w[t] < 0 || w[t] >= M) return 1;
    return 0;
}

/*
 * Viterbi (Algorithm 1 in the max-plus semiring with back-pointers, and the
 * serial backtrace of section 5.1).
 *
 * best_score[b]: FP32 score of the best accepting path (-inf if none).
 * best_arcs[offsets[b] .. offsets[b+1]-1]: its arc ids in input order (-1 if
 * none).  status[b]: ST_OK / ST_NO_PATH / ST_BAD_TOKEN.
 */
int oracle_viterbi(int32_t Q, int32_t M, int32_t start, int64_t A, const int32_t *src,
                   const int32_t *dst, const int32_t *ilabel, const float *arc_score,
                   const float *final_score, int32_t B, const int64_t *offsets,
                   const int32_t *tokens, float *best_score, int32_t *best_arcs, int32_t *status)
{
    if (check_fst(Q, M, start, A, src, dst, ilabel) != OR_OK || B < 0) return OR_EINVAL;
    int64_t *R, *K;
    if (label_index(M, A, ilabel, &R, &K) != OR_OK) return OR_ENOMEM;
    int64_t Tmax = max_len(B, offsets);
    float *alpha = (float *)malloc((size_t)Q * sizeof(float));
    float *alpha_next = (float *)malloc((size_t)Q * sizeof(float));
    int64_t *bp = (int64_t *)malloc((size_t)(Tmax > 0 ? Tmax : 1) * (size_t)Q * sizeof(int64_t));
    if (!alpha || !alpha_next || !bp) {
        free(alpha); free(alpha_next); free(bp); free(R); free(K);
        return OR_ENOMEM;
    }
    for (int32_t b = 0; b < B; ++b) {
        const int64_t n = offsets[b + 1] - offsets[b];
        const int32_t *w = tokens + offsets[b];
        int32_t *path = best_arcs + offsets[b];
        for (int64_t t = 0; t < n; ++t) path[t] = -1;
        if (bad_tokens(M, n, w)) {
            best_score[b] = -INFINITY;
            status[b] = ST_BAD_TOKEN;
            continue;
        }
        /* alpha[0] = the start vector: score 0 (probability 1) at s, -inf elsewhere */
        for (int32_t q = 0; q < Q; ++q) alpha[q] = -INFINITY;
        alpha[start] = 0.0f;
        for (int64_t t = 1; t <= n; ++t) {
            const int32_t a = w[t - 1];
            int64_t *bpt = bp + (size_t)(t - 1) * (size_t)Q;
            for (int32_t q = 0; q < Q; ++q) {
                alpha_next[q] = -INFINITY;
                bpt[q] = -1;
            }
            for (int64_t i = R[a]; i < R[a + 1]; ++i) {
                const int64_t k = K[i];
                const float from = alpha[src[k]];
                if (from == -INFINITY) continue;
                volatile float v = from + arc_score[k]; /* one binary32 RNE addition */
                const int32_t d = dst[k];
                if (v == -INFINITY) continue;
                if (bpt[d] < 0 || v > alpha_next[d] || (v == alpha_next[d] && k < bpt[d])) {
                    alpha_next[d] = v;
                    bpt[d] = k;
                }
            }
            float *tmp = alpha;
            alpha = alpha_next;
            alpha_next = tmp;
        }
        /* final: the best state under alpha[n][q] + f[q]; lowest q wins ties */
        int32_t qbest = -1;
        float best = -INFINITY;
        for (int32_t q = 0; q < Q; ++q) {
            if (alpha[q] == -INFINITY || final_score[q] == -INFINITY) continue;
            volatile float v = alpha[q] + final_score[q];
            if (v == -INFINITY) continue;
            if (qbest < 0 || v > best) {
                best = v;
                qbest = q;
            }
        }
        if (qbest < 0) {
            best_score[b] = -INFINITY;
            status[b] = ST_NO_PATH;
            continue;
        }
        best_score[b] = best;
        status[b] = ST_OK;
        int32_t q = qbest;
        for (int64_t t = n; t >= 1; --t) {
            const int64_t k = bp[(size_t)(t - 1) * (size_t)Q + (size_t)q];
            path[t - 1] = (int32_t)k;
            q = src[k];
        }
    }
    free(alpha); free(alpha_next); free(bp); free(R); free(K);
    return OR_OK;
}

/* forward and backward tables of one sentence, FP64 log domain.
 * la[t*Q + q] = log forward[t][q], lb[t*Q + q] = log backward[t][q], t = 0..n. */
static void fb_tables(int32_t Q, int32_t start, const int32_t *src, const int32_t *dst,
                      const float *arc_score, const float *final_score, const int64_t *R,
                      const int64_t *K, int64_t n, const int32_t *w, double *la, double *lb,
                      double *mx, double *acc)
{
    /* forward: la[0] = start vector, then la[t][q'] = LSE over arcs (label w_t, dst q') */
    for (int32_t q = 0; q < Q; ++q) la[q] = -INFINITY;
    la[start] = 0.0;
    for (int64_t t = 1; t <= n; ++t) {
        const int32_t a = w[t - 1];
        const double *prev = la + (size_t)(t - 1) * Q;
        double *cur = la + (size_t)t * Q;
        for (int32_t q = 0; q < Q; ++q) { mx[q] = -INFINITY; acc[q] = 0.0; }
        for (int64_t i = R[a]; i < R[a + 1]; ++i) {
            const int64_t k = K[i];
            const double x = prev[src[k]] + (double)arc_score[k];
            if (x > mx[dst[k]]) mx[dst[k]] = x;
        }
        for (int64_t i = R[a]; i < R[a + 1]; ++i) {
            const int64_t k = K[i];
            const double x = prev[src[k]] + (double)arc_score[k];
            if (x == -INFINITY) continue;
            acc[dst[k]] += exp(x - mx[dst[k]]);
        }
        for (int32_t q = 0; q < Q; ++q) cur[q] = (mx[q] == -INFINITY) ? -INFINITY : mx[q] + log(acc[q]);
    }
    /* backward: lb[n] = f, then lb[t-1][q] = LSE over arcs (label w_t, src q) */
    double *last = lb + (size_t)n * Q;
    for (int32_t q = 0; q < Q; ++q) last[q] = (double)final_score[q];
    for (int64_t t = n; t >= 1; --t) {
        const int32_t a = w[t - 1];
        const double *nxt = lb + (size_t)t * Q;
        double *cur = lb + (size_t)(t - 1) * Q;
        for (int32_t q = 0; q < Q; ++q) { mx[q] = -INFINITY; acc[q] = 0.0; }
        for (int64_t i = R[a]; i < R[a + 1]; ++i) {
            const int64_t k = K[i];
            const double x = (double)arc_score[k] + nxt[dst[k]];
            if (x > mx[src[k]]) mx[src[k]] = x;
        }
        for (int64_t i = R[a]; i < R[a + 1]; ++i) {
            const int64_t k = K[i];
            const double x = (double)arc_score[k] + nxt[dst[k]];
            if (x == -INFINITY) continue;
            acc[src[k]] += exp(x - mx[src[k]]);
        }
        for (int32_t q = 0; q < Q; ++q) cur[q] = (mx[q] == -INFINITY) ? -INFINITY : mx[q] + log(acc[q]);
    }
}

static double log_z_of(int32_t Q, const double *la_n, const float *final_score)
{
    double m = -INFINITY, s = 0.0;
    for (int32_t q = 0; q < Q; ++q) {
        const double x = la_n[q] + (double)final_score[q];
        if (x > m) m = x;
    }
    if (m == -INFINITY) return -INFINITY;
    for (int32_t q = 0; q < Q; ++q) {
        const double x = la_n[q] + (double)final_score[q];
        if (x == -INFINITY) continue;
        s += exp(x - m);
    }
    return m + log(s);
}

/*
 * Forward-backward with expected counts (Algorithm 2, log domain, FP64).
 *
 * log_z[b]: log of the total weight of sentence b (Eq. 1, log semiring).
 * arc_post[k] (nullable) = sum_b g_b * E_b[number of uses of arc k], where
 *   E_b[.] = sum_t [ilabel_k = w_t] exp(la[t-1][src_k] + score_k + lb[t][dst_k] - log Z_b)
 *   and g_b = grad_log_z[b] (1 when grad_log_z is NULL).
 * final_post[q] (nullable) = sum_b g_b exp(la[n][q] + f[q] - log Z_b).
 * Both outputs are overwritten.  NO_PATH and BAD_TOKEN sentences contribute 0.
 */
int oracle_forward_backward(int32_t Q, int32_t M, int32_t start, int64_t A, const int32_t *src,
                            const int32_t *dst, const int32_t *ilabel, const float *arc_score,
                            const float *final_score, int32_t B, const int64_t *offsets,
                            const int32_t *tokens, const double *grad_log_z, double *log_z,
                            double *arc_post, double *final_post, int32_t *status)
{
    if (check_fst(Q, M, start, A, src, dst, ilabel) != OR_OK || B < 0) return OR_EINVAL;
    int64_t *R, *K;
    if (label_index(M, A, ilabel, &R, &K) != OR_OK) return OR_ENOMEM;
    const int64_t Tmax = max_len(B, offsets);
    const size_t cells = (size_t)(Tmax + 1) * (size_t)Q;
    double *la = (double *)malloc(cells * sizeof(double));
    double *lb = (double *)malloc(cells * sizeof(double));
    double *mx = (double *)malloc((size_t)Q * sizeof(double));
    double *acc = (double *)malloc((size_t)Q * sizeof(double));
    if (!la || !lb || !mx || !acc) {
        free(la); free(lb); free(mx); free(acc); free(R); free(K);
        return OR_ENOMEM;
    }
    if (arc_post)
        for (int64_t k = 0; k < A; ++k) arc_post[k] = 0.0;
    if (final_post)
        for (int32_t q = 0; q < Q; ++q) final_post[q] = 0.0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t n = offsets[b + 1] - offsets[b];
        const int32_t *w = tokens + offsets[b];
        if (bad_tokens(M, n, w)) {
            log_z[b] = -INFINITY;
            status[b] = ST_BAD_TOKEN;
            continue;
        }
        fb_tables(Q, start, src, dst, arc_score, final_score, R, K, n, w, la, lb, mx, acc);
        const double lz = log_z_of(Q, la + (size_t)n * Q, final_score);
        log_z[b] = lz;
        if (lz == -INFINITY) {
            status[b] = ST_NO_PATH;
            continue;
        }
        status[b] = ST_OK;
        const double g = grad_log_z ? grad_log_z[b] : 1.0;
        if (arc_post) {
            for (int64_t t = 1; t <= n; ++t) {
                const int32_t a = w[t - 1];
                const double *al = la + (size_t)(t - 1) * Q;
                const double *be = lb + (size_t)t * Q;
                for (int64_t i = R[a]; i < R[a + 1]; ++i) {
                    const int64_t k = K[i];
                    const double x = al[src[k]] + (double)arc_score[k] + be[dst[k]] - lz;
                    if (x == -INFINITY) continue;
                    arc_post[k] += g * exp(x);
                }
            }
        }
        if (final_post) {
            const double *al = la + (size_t)n * Q;
            for (int32_t q = 0; q < Q; ++q) {
                const double x = al[q] + (double)final_score[q] - lz;
                if (x == -INFINITY) continue;
                final_post[q] += g * exp(x);
            }
        }
    }
    free(la); free(lb); free(mx); free(acc); free(R); free(K);
    return OR_OK;
}

/* The forward and backward tables of ONE sentence (for invariant checks):
 * la and lb each hold (n+1)*Q doubles, row t = time step t. */
int oracle_fb_tables(int32_t Q, int32_t M, int32_t start, int64_t A, const int32_t *src,
                     const int32_t *dst, const int32_t *ilabel, const float *arc_score,
                     const float *final_score, int64_t n, const int32_t *w, double *la, double *lb)
{
    if (check_fst(Q, M, start, A, src, dst, ilabel) != OR_OK || n < 0) return OR_EINVAL;
    if (bad_tokens(M, n, w)) return OR_EINVAL;
    int64_t *R, *K;
    if (label_index(M, A, ilabel, &R, &K) != OR_OK) return OR_ENOMEM;
    double *mx = (double *)malloc((size_t)Q * sizeof(double));
    double *acc = (double *)malloc((size_t)Q * sizeof(double));
    if (!mx || !acc) {
        free(mx); free(acc); free(R); free(K);
        return OR_ENOMEM;
    }
    fb_tables(Q, start, src, dst, arc_score, final_score, R, K, n, w, la, lb, mx, acc);
    free(mx); free(acc); free(R); free(K);
    return OR_OK;
}
