// Host-side parts of libcsrc: status strings, CSR -> CSRC conversion,
// quantisation, greedy colouring and the selector's structural features.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "internal.h"

namespace csrc {
static thread_local int g_last_hip = 0;
int hip_status(int e)
{
    if (e == 0) return CSRC_OK;
    g_last_hip = e;
    return CSRC_ERR_HIP;
}
}  // namespace csrc

extern "C" int32_t csrc_last_hip_error(void) { return csrc::g_last_hip; }
extern "C" const char *csrc_last_hip_error_string(void)
{
    return hipGetErrorName(static_cast<hipError_t>(csrc::g_last_hip));
}

extern "C" const char *csrc_status_string(int s)
{
    switch (s) {
    case CSRC_OK: return "ok";
    case CSRC_ERR_ARG: return "invalid argument";
    case CSRC_ERR_NOT_STRUCT_SYM: return "pattern is not structurally symmetric";
    case CSRC_ERR_DUPLICATE: return "duplicate entry";
    case CSRC_ERR_INDEX_RANGE: return "column index out of range";
    case CSRC_ERR_TOO_LARGE: return "size exceeds 32-bit indexing";
    case CSRC_ERR_ALIAS: return "destination overlaps source";
    case CSRC_ERR_WORKSPACE: return "workspace missing or too small";
    case CSRC_ERR_HIP: return "HIP runtime error";
    case CSRC_ERR_UNSUPPORTED: return "variant unsupported for this matrix";
    case CSRC_ERR_PLAN: return "plan does not match the call";
    case CSRC_ERR_NOMEM: return "host allocation failed";
    case CSRC_ERR_NO_MODEL: return "no trained selector model";
    default: return "unknown status";
    }
}

extern "C" int32_t csrc_version(void) { return 10000; }

namespace {

// Sorted, validated copy of a CSR pattern (optionally with values), plus its
// transpose built by a counting sort.  Column lists of both are ascending.
struct SortedCsr {
    int32_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

int sort_rows(int32_t n, const int64_t *rp, const int32_t *col, const double *val,
              SortedCsr &out)
{
    if (n < 0 || !rp) return CSRC_ERR_ARG;
    if (rp[0] != 0) return CSRC_ERR_ARG;
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return CSRC_ERR_ARG;
    int64_t nnz = rp[n];
    if (nnz > 0 && !col) return CSRC_ERR_ARG;
    out.n = n;
    out.ptr.assign(rp, rp + n + 1);
    out.col.resize(nnz);
    if (val) out.val.resize(nnz);
    std::vector<std::pair<int32_t, double>> tmp;
    for (int32_t i = 0; i < n; ++i) {
        int64_t a = rp[i], b = rp[i + 1];
        tmp.resize(b - a);
        for (int64_t q = a; q < b; ++q) {
            int32_t c = col[q];
            if (c < 0 || c >= n) return CSRC_ERR_INDEX_RANGE;
            tmp[q - a] = {c, val ? val[q] : 0.0};
        }
        std::stable_sort(tmp.begin(), tmp.end(),
                         [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                             return x.first < y.first;
                         });
        for (int64_t q = a; q < b; ++q) {
            if (q > a && tmp[q - a].first == tmp[q - a - 1].first) return CSRC_ERR_DUPLICATE;
            out.col[q] = tmp[q - a].first;
            if (val) out.val[q] = tmp[q - a].second;
        }
    }
    return CSRC_OK;
}

// Transpose by counting sort: rows of the result are ascending because the
// source rows are visited in ascending order.
void transpose(const SortedCsr &a, SortedCsr &t)
{
    int32_t n = a.n;
    t.n = n;
    t.ptr.assign(n + 1, 0);
    for (int32_t c : a.col) t.ptr[c + 1] += 1;
    for (int32_t i = 0; i < n; ++i) t.ptr[i + 1] += t.ptr[i];
    t.col.resize(a.col.size());
    bool hv = !a.val.empty();
    if (hv) t.val.resize(a.val.size());
    std::vector<int64_t> fill(t.ptr.begin(), t.ptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t q = a.ptr[i]; q < a.ptr[i + 1]; ++q) {
            int64_t p = fill[a.col[q]]++;
            t.col[p] = i;
            if (hv) t.val[p] = a.val[q];
        }
}

// Build the symmetric pattern: either check that A and A^T agree, or form
// their union with zeros where only the mirror is stored.  Result in `s`
// (sorted, values of A where stored, 0 otherwise).
int symmetric_pattern(int32_t n, const int64_t *rp, const int32_t *col, const double *val,
                      int32_t flags, SortedCsr &s)
{
    SortedCsr a, t;
    int st = sort_rows(n, rp, col, val, a);
    if (st) return st;
    transpose(a, t);
    bool same = a.col == t.col;
    if (same) {
        s = std::move(a);
        return CSRC_OK;
    }
    if (!(flags & CSRC_PAD_PATTERN)) return CSRC_ERR_NOT_STRUCT_SYM;
    s.n = n;
    s.ptr.assign(n + 1, 0);
    s.col.clear();
    s.val.clear();
    bool hv = !a.val.empty();
    for (int32_t i = 0; i < n; ++i) {
        int64_t p = a.ptr[i], pe = a.ptr[i + 1], q = t.ptr[i], qe = t.ptr[i + 1];
        while (p < pe || q < qe) {
            int32_t ca = p < pe ? a.col[p] : INT32_MAX;
            int32_t ct = q < qe ? t.col[q] : INT32_MAX;
            if (ca <= ct) {
                s.col.push_back(ca);
                s.val.push_back(hv ? a.val[p] : 0.0);
                ++p;
                if (ca == ct) ++q;
            } else {
                s.col.push_back(ct);
                s.val.push_back(0.0);
                ++q;
            }
        }
        s.ptr[i + 1] = (int64_t)s.col.size();
    }
    return CSRC_OK;
}

}  // namespace

extern "C" int csrc_count(int32_t n, const int64_t *row_ptr, const int32_t *col,
                          int32_t flags, int64_t *k_out)
{
    if (!k_out || n < 0 || (n > 0 && !row_ptr)) return CSRC_ERR_ARG;
    try {
        if (n == 0) { *k_out = 0; return CSRC_OK; }
        SortedCsr s;
        int st = symmetric_pattern(n, row_ptr, col, nullptr, flags, s);
        if (st) return st;
        int64_t k = 0;
        for (int32_t i = 0; i < n; ++i)
            for (int64_t q = s.ptr[i]; q < s.ptr[i + 1] && s.col[q] < i; ++q) ++k;
        if (k >= (int64_t(1) << 31)) return CSRC_ERR_TOO_LARGE;
        *k_out = k;
        return CSRC_OK;
    } catch (const std::bad_alloc &) {
        return CSRC_ERR_NOMEM;
    }
}

// Rectangular matrices (Sec. 2.1): the entries of columns < n form A_S, the
// others A_R; both keep each row's input order.
static int rect_check(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col)
{
    if (n < 0 || m < n || (n > 0 && !row_ptr)) return CSRC_ERR_ARG;
    if (n == 0) return CSRC_OK;
    if (row_ptr[0] != 0) return CSRC_ERR_ARG;
    for (int32_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return CSRC_ERR_ARG;
    if (row_ptr[n] > 0 && !col) return CSRC_ERR_ARG;
    for (int64_t q = 0; q < row_ptr[n]; ++q)
        if (col[q] < 0 || col[q] >= m) return CSRC_ERR_INDEX_RANGE;
    return CSRC_OK;
}

extern "C" int csrc_rect_count(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col, int64_t *nnz_s,
                               int64_t *nnz_r)
{
    if (!nnz_s || !nnz_r) return CSRC_ERR_ARG;
    int st = rect_check(n, m, row_ptr, col);
    if (st) return st;
    int64_t s = 0, r = 0;
    for (int64_t q = 0; n > 0 && q < row_ptr[n]; ++q) (col[q] < n ? s : r) += 1;
    if (r >= (int64_t(1) << 31)) return CSRC_ERR_TOO_LARGE;
    *nnz_s = s;
    *nnz_r = r;
    return CSRC_OK;
}

extern "C" int csrc_rect_split(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
                               int64_t *s_row_ptr, int32_t *s_col, double *s_val, int32_t *iar, int32_t *jar,
                               double *ar)
{
    if (!s_row_ptr || !iar) return CSRC_ERR_ARG;
    int st = rect_check(n, m, row_ptr, col);
    if (st) return st;
    s_row_ptr[0] = 0;
    iar[0] = 0;
    if (n == 0) return CSRC_OK;
    if (row_ptr[n] > 0 && !val) return CSRC_ERR_ARG;
    int64_t s = 0, r = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
            if (col[q] < n) {
                if (!s_col || !s_val) return CSRC_ERR_ARG;
                s_col[s] = col[q];
                s_val[s++] = val[q];
            } else {
                if (!jar || !ar) return CSRC_ERR_ARG;
                if (r >= (int64_t(1) << 31) - 1) return CSRC_ERR_TOO_LARGE;
                jar[r] = col[q];
                ar[r++] = val[q];
            }
        }
        s_row_ptr[i + 1] = s;
        iar[i + 1] = (int32_t)r;
    }
    return CSRC_OK;
}

extern "C" int csrc_from_csr(int32_t n, const int64_t *row_ptr, const int32_t *col,
                             const double *val, int32_t flags, int32_t *ia, int32_t *ja,
                             double *ad, double *al, double *au)
{
    if (n < 0 || !ia || (n > 0 && (!row_ptr || !ad))) return CSRC_ERR_ARG;
    try {
        if (n == 0) { ia[0] = 0; return CSRC_OK; }
        if (row_ptr[n] > 0 && !val) return CSRC_ERR_ARG;
        SortedCsr s, t;
        int st = symmetric_pattern(n, row_ptr, col, val, flags, s);
        if (st) return st;
        // The transpose's row i lists column i of A: entries (j, a_ji) with j
        // ascending; its part j < i is the upper mirror of row i's lower part.
        transpose(s, t);
        int64_t k = 0;
        ia[0] = 0;
        for (int32_t i = 0; i < n; ++i) {
            ad[i] = 0.0;
            int64_t q = s.ptr[i], p = t.ptr[i];
            for (; q < s.ptr[i + 1] && s.col[q] < i; ++q, ++p) {
                if (k >= (int64_t(1) << 31) - 1) return CSRC_ERR_TOO_LARGE;
                ja[k] = s.col[q];
                al[k] = s.val[q];
                au[k] = t.val[p];     // t.col[p] == s.col[q] by symmetry
                ++k;
            }
            if (q < s.ptr[i + 1] && s.col[q] == i) ad[i] = s.val[q];
            ia[i + 1] = (int32_t)k;
        }
        return CSRC_OK;
    } catch (const std::bad_alloc &) {
        return CSRC_ERR_NOMEM;
    }
}

static inline uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu))
        return (uint16_t)((u >> 16) | 0x40);              // quiet NaN
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

extern "C" int csrc_quantize(int64_t count, const double *src, int32_t dtype, void *dst)
{
    if (count < 0 || (count > 0 && (!src || !dst))) return CSRC_ERR_ARG;
    switch (dtype) {
    case CSRC_F64:
        if (count) std::memcpy(dst, src, sizeof(double) * (size_t)count);
        return CSRC_OK;
    case CSRC_F32: {
        float *d = static_cast<float *>(dst);
        for (int64_t i = 0; i < count; ++i) d[i] = (float)src[i];
        return CSRC_OK;
    }
    case CSRC_BF16: {
        uint16_t *d = static_cast<uint16_t *>(dst);
        for (int64_t i = 0; i < count; ++i) d[i] = f32_to_bf16_rne((float)src[i]);
        return CSRC_OK;
    }
    default:
        return CSRC_ERR_ARG;
    }
}

namespace csrc {

// Greedy first-fit colouring in ascending row order.  For the write-set
// criterion every y entry t keeps the colours already given to rows writing
// t; a row is barred from the colours stored at each entry it writes.  For
// the distance-two criterion the barred colours are those of the row's
// neighbours and of their neighbours.
int color_rows(int32_t n, const int32_t *ia, const int32_t *ja, int32_t criterion,
               int32_t *color, int32_t *ncolors)
{
    if (n < 0 || !ncolors || (n > 0 && (!ia || !color || (ia[n] > 0 && !ja)))) return CSRC_ERR_ARG;
    if (criterion != CSRC_COLOR_WRITE_SET && criterion != CSRC_COLOR_DISTANCE2) return CSRC_ERR_ARG;
    try {
        *ncolors = 0;
        if (n == 0) return CSRC_OK;
        std::vector<int32_t> barred(n + 1, -1);
        int32_t used = 0;
        if (criterion == CSRC_COLOR_WRITE_SET) {
            // capacity at entry t: 1 (row t itself) + number of rows storing t
            std::vector<int64_t> cap(n + 1, 0);
            for (int32_t t = 0; t < n; ++t) cap[t + 1] = 1;
            for (int64_t q = 0; q < ia[n]; ++q) cap[ja[q] + 1] += 1;
            for (int32_t t = 0; t < n; ++t) cap[t + 1] += cap[t];
            std::vector<int32_t> held(cap[n]);
            std::vector<int32_t> cnt(n, 0);
            for (int32_t i = 0; i < n; ++i) {
                for (int32_t c : {i}) {
                    for (int32_t s = 0; s < cnt[c]; ++s) barred[held[cap[c] + s]] = i;
                }
                for (int32_t q = ia[i]; q < ia[i + 1]; ++q) {
                    int32_t t = ja[q];
                    for (int32_t s = 0; s < cnt[t]; ++s) barred[held[cap[t] + s]] = i;
                }
                int32_t c = 0;
                while (barred[c] == i) ++c;
                color[i] = c;
                used = std::max(used, c + 1);
                held[cap[i] + cnt[i]++] = c;
                for (int32_t q = ia[i]; q < ia[i + 1]; ++q) {
                    int32_t t = ja[q];
                    held[cap[t] + cnt[t]++] = c;
                }
            }
        } else {
            std::vector<int64_t> p(n + 1, 0);
            for (int32_t i = 0; i < n; ++i)
                for (int32_t q = ia[i]; q < ia[i + 1]; ++q) { p[i + 1]++; p[ja[q] + 1]++; }
            for (int32_t i = 0; i < n; ++i) p[i + 1] += p[i];
            std::vector<int32_t> nb(p[n]);
            std::vector<int64_t> f(p.begin(), p.end() - 1);
            for (int32_t i = 0; i < n; ++i)
                for (int32_t q = ia[i]; q < ia[i + 1]; ++q) { nb[f[i]++] = ja[q]; nb[f[ja[q]]++] = i; }
            for (int32_t i = 0; i < n; ++i) color[i] = -1;
            for (int32_t i = 0; i < n; ++i) {
                for (int64_t a = p[i]; a < p[i + 1]; ++a) {
                    int32_t v = nb[a];
                    if (color[v] >= 0) barred[color[v]] = i;
                    for (int64_t b = p[v]; b < p[v + 1]; ++b) {
                        int32_t w = nb[b];
                        if (w != i && color[w] >= 0) barred[color[w]] = i;
                    }
                }
                int32_t c = 0;
                while (barred[c] == i) ++c;
                color[i] = c;
                used = std::max(used, c + 1);
            }
        }
        *ncolors = used;
        return CSRC_OK;
    } catch (const std::bad_alloc &) {
        return CSRC_ERR_NOMEM;
    }
}

}  // namespace csrc

extern "C" int csrc_color(int32_t n, const int32_t *ia, const int32_t *ja, int32_t criterion,
                          int32_t *color, int32_t *ncolors)
{
    return csrc::color_rows(n, ia, ja, criterion, color, ncolors);
}

extern "C" int csrc_features(int32_t n, const int32_t *ia, const int32_t *ja, int32_t vdtype,
                             int32_t ncolors, float *f)
{
    if (n < 0 || !f || (n > 0 && (!ia || (ia[n] > 0 && !ja)))) return CSRC_ERR_ARG;
    try {
        for (int q = 0; q < CSRC_NFEATURES; ++q) f[q] = 0.f;
        if (n == 0) return CSRC_OK;
        int64_t k = ia[n];
        double nnz = 2.0 * (double)k + n;
        // row lengths of the full pattern (diagonal counted once)
        std::vector<int32_t> len(n, 1);
        std::vector<int32_t> writers(n, 1);
        int64_t near = 0;
        double sum_dist = 0.0;
        int64_t bw = 0;
        for (int32_t i = 0; i < n; ++i) {
            for (int32_t q = ia[i]; q < ia[i + 1]; ++q) {
                int32_t j = ja[q];
                len[i] += 1;
                len[j] += 1;
                writers[j] += 1;
                int64_t d = (int64_t)i - j;
                sum_dist += (double)d;
                bw = std::max(bw, d);
                if (d < 64) ++near;
            }
        }
        double mean = nnz / n;
        double var = 0.0;
        int32_t maxlen = 0, maxw = 0;
        for (int32_t i = 0; i < n; ++i) {
            double d = len[i] - mean;
            var += d * d;
            maxlen = std::max(maxlen, len[i]);
            maxw = std::max(maxw, writers[i]);
        }
        var /= n;
        if (ncolors < 0) {
            std::vector<int32_t> col(n);
            int st = csrc::color_rows(n, ia, ja, CSRC_COLOR_WRITE_SET, col.data(), &ncolors);
            if (st) return st;
        }
        // 3x3 block structure: rows come in triples with identical column
        // blocks (checked on the lower pattern of the first row of each triple)
        bool block3 = (n % 3 == 0) && n >= 3;
        for (int32_t b = 0; block3 && b + 2 < n; b += 3) {
            int32_t l0 = ia[b + 1] - ia[b], l1 = ia[b + 2] - ia[b + 1], l2 = ia[b + 3] - ia[b + 2];
            if (l1 != l0 + 1 || l2 != l0 + 2 || l0 % 3 != 0) block3 = false;
        }
        double vb = csrc::value_bytes(vdtype), xb = vdtype == CSRC_F64 ? 8 : 4;
        double ws = 4.0 * (n + 1) + k * (4 + 2 * vb) + n * vb + n * 2 * xb;
        f[0] = (float)std::log2(n + 1.0);
        f[1] = (float)std::log2(nnz + 1.0);
        f[2] = (float)mean;
        f[3] = (float)var;
        f[4] = (float)(maxlen / mean);
        f[5] = (float)((double)bw / n);
        f[6] = (float)(k ? sum_dist / k / n : 0.0);
        f[7] = (float)(k ? (double)near / k : 1.0);
        f[8] = (float)std::log2(1.0 + maxw);
        f[9] = (float)(ncolors / 32.0);
        f[10] = (float)std::log2(ws / (256.0 * 1024 * 1024));
        f[11] = block3 ? 1.f : 0.f;
        return CSRC_OK;
    } catch (const std::bad_alloc &) {
        return CSRC_ERR_NOMEM;
    }
}

extern "C" int csrc_select(int32_t n, const int32_t *ia, const int32_t *ja, int32_t vdtype,
                           int32_t hidden, int32_t classes, const float *params, const float *mean,
                           const float *scale, int32_t *candidate)
{
    if (!candidate) return CSRC_ERR_ARG;
    if (!params) return CSRC_ERR_NO_MODEL;
    // every argument is checked before the features, which colour the rows
    // (seconds on a large matrix)
    if (!mean || !scale || csrc_mlp_param_count(hidden, classes) < 0) return CSRC_ERR_ARG;
    float f[CSRC_NFEATURES];
    const int st = csrc_features(n, ia, ja, vdtype, -1, f);
    if (st != CSRC_OK) return st;
    return csrc_mlp_predict_host(hidden, classes, params, mean, scale, f, candidate);
}
