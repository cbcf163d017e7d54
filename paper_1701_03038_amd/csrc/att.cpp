// Reader for the AT&T / OpenFST text format of weighted transducers (the
// format the paper's FSTs are given in, section 7.2), host code.
//
// Lines: "src dst ilabel olabel [weight]" for an arc, "state [weight]" for a
// final state; fields separated by blanks or tabs; empty lines are skipped.
// The source of the first arc (or the state of the first line) is the start
// state.  Weights are costs (-log p, as OpenFST's tropical and log semirings
// store them): the score is -weight, a missing weight is 0.  A final weight
// of infinity ("inf", "Infinity") marks a non-final state.  Labels are
// non-negative integers, or symbols resolved through a symbol table ("symbol
// id" per line).  With epsilon_zero, id 0 is epsilon, which the method does
// not have on the input side (section 3: no epsilon transitions).
#include <cerrno>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/wfst.h"

namespace {

thread_local std::string g_att_err;

int att_err(int code, const std::string &msg)
{
    g_att_err = msg;
    return code;
}

// Fields of one line (blank/tab separated), without the newline.
void split_fields(const char *b, const char *e, std::vector<std::string> &out)
{
    out.clear();
    const char *p = b;
    while (p < e) {
        while (p < e && (*p == ' ' || *p == '\t' || *p == '\r')) ++p;
        const char *q = p;
        while (q < e && *q != ' ' && *q != '\t' && *q != '\r') ++q;
        if (q > p) out.emplace_back(p, (size_t)(q - p));
        p = q;
    }
}

bool parse_int(const std::string &s, int64_t &v)
{
    if (s.empty()) return false;
    char *end = nullptr;
    errno = 0;
    const long long x = std::strtoll(s.c_str(), &end, 10);
    if (errno != 0 || *end != '\0') return false;
    v = x;
    return true;
}

bool parse_weight(const std::string &s, double &w)
{
    if (s == "inf" || s == "Infinity" || s == "INF" || s == "infinity") {
        w = std::numeric_limits<double>::infinity();
        return true;
    }
    char *end = nullptr;
    errno = 0;
    w = std::strtod(s.c_str(), &end);
    return errno == 0 && *end == '\0' && !std::isnan(w);
}

// symbol table text -> map; returns the largest id (or -1)
int read_symbols(const char *text, int64_t len, std::unordered_map<std::string, int64_t> &map, int64_t &max_id,
                 const char *what)
{
    max_id = -1;
    if (!text) return WFST_OK;
    std::vector<std::string> f;
    const char *p = text, *end = text + len;
    int64_t line = 0;
    while (p < end) {
        const char *nl = static_cast<const char *>(std::memchr(p, '\n', (size_t)(end - p)));
        const char *le = nl ? nl : end;
        ++line;
        split_fields(p, le, f);
        p = nl ? nl + 1 : end;
        if (f.empty()) continue;
        int64_t id;
        if (f.size() != 2 || !parse_int(f[1], id) || id < 0 || id >= INT32_MAX)
            return att_err(WFST_EINVAL, std::string(what) + " symbol table line " + std::to_string(line) +
                                            ": expected \"symbol id\"");
        map[f[0]] = id;
        if (id > max_id) max_id = id;
    }
    return WFST_OK;
}

int label_of(const std::string &s, const std::unordered_map<std::string, int64_t> *map, int64_t &v)
{
    if (map) {
        auto it = map->find(s);
        if (it != map->end()) {
            v = it->second;
            return WFST_OK;
        }
    }
    if (parse_int(s, v) && v >= 0 && v < INT32_MAX) return WFST_OK;
    return WFST_EINVAL;
}

}  // namespace

extern "C" {

const char *wfst_att_last_error(void) { return g_att_err.c_str(); }

int wfst_att_parse(const char *fst_text, int64_t fst_len, const char *isyms_text, int64_t isyms_len,
                   const char *osyms_text, int64_t osyms_len, int32_t epsilon_zero, int64_t *counts,
                   int32_t *src, int32_t *dst, int32_t *ilabel, int32_t *olabel, float *arc_score,
                   float *final_score)
{
    try {
        if (!fst_text || fst_len < 0 || !counts) return att_err(WFST_EINVAL, "NULL text or counts");
        std::unordered_map<std::string, int64_t> imap, omap;
        int64_t imax = -1, omax = -1;
        int rc = read_symbols(isyms_text, isyms_len, imap, imax, "input");
        if (rc == WFST_OK) rc = read_symbols(osyms_text, osyms_len, omap, omax, "output");
        if (rc != WFST_OK) return rc;
        struct Arc {
            int32_t s, d, i, o;
            float score;
        };
        std::vector<Arc> arcs;
        std::vector<std::pair<int32_t, float>> finals;
        int64_t max_state = -1, max_ilabel = imax, start = -1;
        std::vector<std::string> f;
        const char *p = fst_text, *end = fst_text + fst_len;
        int64_t line = 0;
        while (p < end) {
            const char *nl = static_cast<const char *>(std::memchr(p, '\n', (size_t)(end - p)));
            const char *le = nl ? nl : end;
            ++line;
            split_fields(p, le, f);
            p = nl ? nl + 1 : end;
            if (f.empty()) continue;
            const std::string where = "line " + std::to_string(line);
            if (f.size() == 4 || f.size() == 5) {
                int64_t s, d, i, o;
                double w = 0.0;
                if (!parse_int(f[0], s) || !parse_int(f[1], d) || s < 0 || d < 0 || s >= INT32_MAX - 1 ||
                    d >= INT32_MAX - 1)
                    return att_err(WFST_EINVAL, where + ": states must be non-negative integers");
                if (label_of(f[2], isyms_text ? &imap : nullptr, i) != WFST_OK)
                    return att_err(WFST_EINVAL, where + ": unknown input label \"" + f[2] + "\"");
                if (label_of(f[3], osyms_text ? &omap : nullptr, o) != WFST_OK)
                    return att_err(WFST_EINVAL, where + ": unknown output label \"" + f[3] + "\"");
                if (f.size() == 5 && (!parse_weight(f[4], w) || std::isinf(w)))
                    return att_err(WFST_EINVAL, where + ": arc weight must be a finite number");
                if (epsilon_zero && i == 0)
                    return att_err(WFST_EUNSUPPORTED, where + ": epsilon input label (no epsilon transitions)");
                if (start < 0) start = s;
                arcs.push_back(Arc{(int32_t)s, (int32_t)d, (int32_t)i, (int32_t)o, (float)(-w)});
                max_state = std::max(max_state, std::max(s, d));
                max_ilabel = std::max(max_ilabel, i);
            } else if (f.size() == 1 || f.size() == 2) {
                int64_t q;
                double w = 0.0;
                if (!parse_int(f[0], q) || q < 0 || q >= INT32_MAX - 1)
                    return att_err(WFST_EINVAL, where + ": final state must be a non-negative integer");
                if (f.size() == 2 && !parse_weight(f[1], w))
                    return att_err(WFST_EINVAL, where + ": final weight must be a number or inf");
                if (start < 0) start = q;
                finals.emplace_back((int32_t)q, std::isinf(w) && w > 0 ? -INFINITY : (float)(-w));
                max_state = std::max(max_state, q);
            } else {
                return att_err(WFST_EINVAL, where + ": expected 4 or 5 fields (arc) or 1 or 2 (final state)");
            }
        }
        if (start < 0) return att_err(WFST_EINVAL, "no arc or final state");
        if ((int64_t)arcs.size() >= INT32_MAX) return att_err(WFST_EUNSUPPORTED, "more than 2^31-1 arcs");
        counts[0] = max_state + 1;
        counts[1] = std::max<int64_t>(max_ilabel + 1, 1);
        counts[2] = (int64_t)arcs.size();
        counts[3] = start;
        if (!src && !dst && !ilabel && !olabel && !arc_score && !final_score) return WFST_OK;
        if (!src || !dst || !ilabel || !arc_score || !final_score)
            return att_err(WFST_EINVAL, "output arrays: all of src, dst, ilabel, arc_score, final_score");
        for (size_t k = 0; k < arcs.size(); ++k) {
            src[k] = arcs[k].s;
            dst[k] = arcs[k].d;
            ilabel[k] = arcs[k].i;
            if (olabel) olabel[k] = arcs[k].o;
            arc_score[k] = arcs[k].score == 0.0f ? 0.0f : arcs[k].score;
        }
        for (int64_t q = 0; q <= max_state; ++q) final_score[q] = -INFINITY;
        for (auto &fq : finals) final_score[fq.first] = fq.second == 0.0f ? 0.0f : fq.second;
        return WFST_OK;
    } catch (const std::bad_alloc &) {
        return att_err(WFST_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return att_err(WFST_EINVAL, e.what());
    }
}

}  // extern "C"
