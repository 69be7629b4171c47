// Host-side entry points of libcsrc under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py with
// g++, together with the library's host sources only).
//
// Every host call of the C ABI runs on seeded random structurally symmetric
// patterns and on edge cases (n = 0, empty rows, missing diagonals, padded
// patterns, rejected inputs), with basic invariants of the outputs checked
// here.  The three HIP runtime functions the host sources reference are
// stubs below that report failure: no device work happens in this process.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <utility>
#include <vector>

#include "csrc.h"

extern "C" const char *hipGetErrorName(hipError_t) { return "stub"; }
extern "C" hipError_t hipMemcpyAsync(void *, const void *, size_t, hipMemcpyKind, hipStream_t)
{
    return hipErrorNotSupported;
}
extern "C" hipError_t hipStreamSynchronize(hipStream_t) { return hipErrorNotSupported; }

namespace {

int g_fail = 0;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed) {}
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    int below(int m) { return (int)(next() % (uint64_t)m); }
};

struct Csr {
    int32_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<double> val;
};

// Symmetric pattern: each row i links to up to `deg` random rows j < i
// (within `band` when band > 0); diagonal stored with probability pdiag.
Csr random_sym(Rng &g, int32_t n, int deg, int band, double pdiag)
{
    std::vector<std::set<int32_t>> rows((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        if (g.unit() < pdiag) rows[i].insert(i);
        for (int d = 0; d < deg && i > 0; ++d) {
            int32_t lo = band > 0 ? std::max(0, i - band) : 0;
            int32_t j = lo + g.below(i - lo);
            rows[i].insert(j);
            rows[j].insert(i);
        }
    }
    Csr a;
    a.n = n;
    a.rp.assign((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        // columns in scrambled order: the split must sort them itself
        std::vector<int32_t> c(rows[i].begin(), rows[i].end());
        for (size_t k = c.size(); k > 1; --k) std::swap(c[k - 1], c[(size_t)g.below((int)k)]);
        for (int32_t j : c) {
            a.col.push_back(j);
            a.val.push_back(2.0 * g.unit() - 1.0);
        }
        a.rp[i + 1] = (int64_t)a.col.size();
    }
    return a;
}

struct Split {
    int64_t k = 0;
    std::vector<int32_t> ia, ja;
    std::vector<double> ad, al, au;
};

int split(const Csr &a, int flags, Split &s)
{
    int st = csrc_count(a.n, a.rp.data(), a.col.data(), flags, &s.k);
    if (st) return st;
    s.ia.assign((size_t)a.n + 1, -1);
    s.ja.assign((size_t)s.k, -1);
    s.ad.assign((size_t)a.n, 0.0);
    s.al.assign((size_t)s.k, 0.0);
    s.au.assign((size_t)s.k, 0.0);
    return csrc_from_csr(a.n, a.rp.data(), a.col.data(), a.val.data(), flags, s.ia.data(), s.ja.data(),
                         s.ad.data(), s.al.data(), s.au.data());
}

void check_split(const Split &s, int32_t n)
{
    CHECK(s.ia[0] == 0 && s.ia[n] == s.k);
    for (int32_t i = 0; i < n; ++i) {
        CHECK(s.ia[i] <= s.ia[i + 1]);
        for (int32_t q = s.ia[i]; q < s.ia[i + 1]; ++q) {
            CHECK(s.ja[q] >= 0 && s.ja[q] < i);
            if (q > s.ia[i]) CHECK(s.ja[q - 1] < s.ja[q]);
        }
    }
}

void exercise_plans(const Split &s, int32_t n)
{
    const int32_t tile_works[] = {0, 1, 64, 4096};
    for (int v = 0; v < CSRC_V_COUNT; ++v)
        for (int32_t tw : tile_works)
            for (int rhs : {1, 4})
                for (int am = 0; am < 2; ++am) {
                    if (am && v != CSRC_V_PRIVATE) continue;
                    if (rhs > 1 && (v == CSRC_V_TILE_COLOR || am)) continue;
                    for (int32_t vd : {CSRC_F64, CSRC_BF16}) {
                        csrc_plan_opts o;
                        CHECK(csrc_plan_opts_default(v, &o) == CSRC_OK);
                        o.tile_work = tw;
                        o.max_rhs = rhs;
                        o.atomic_merge = am;
                        csrc_plan *p = nullptr;
                        int st = csrc_plan_create(n, s.ia.data(), s.ja.data(), vd, &o, &p);
                        CHECK(st == CSRC_OK || st == CSRC_ERR_UNSUPPORTED);
                        if (st) continue;
                        csrc_plan_info info;
                        CHECK(csrc_plan_get_info(p, &info) == CSRC_OK);
                        CHECK(csrc_plan_workspace_bytes(p) >= 0);
                        for (int what = 0; what < 3; ++what) {
                            int64_t need = -1;
                            int st2 = csrc_plan_export(p, what, nullptr, 0, &need);
                            if (st2 == CSRC_OK && need > 0) {
                                std::vector<int32_t> buf((size_t)need, 0);
                                CHECK(csrc_plan_export(p, what, buf.data(), need, &need) == CSRC_OK);
                            }
                        }
                        if (v == CSRC_V_PRIVATE && info.workspace_bytes > 0) {
                            // the upload reaches the (stub) HIP runtime and fails cleanly
                            std::vector<char> ws((size_t)info.workspace_bytes);
                            CHECK(csrc_plan_upload(p, ws.data(), info.workspace_bytes, nullptr) == CSRC_ERR_HIP);
                        }
                        CHECK(csrc_plan_destroy(p) == CSRC_OK);
                    }
                }
}

void exercise_matrix(Rng &g, const Csr &a)
{
    Split s;
    CHECK(split(a, 0, s) == CSRC_OK);
    check_split(s, a.n);
    for (int32_t crit : {CSRC_COLOR_WRITE_SET, CSRC_COLOR_DISTANCE2}) {
        std::vector<int32_t> color((size_t)a.n, -1);
        int32_t nc = -1;
        CHECK(csrc_color(a.n, s.ia.data(), s.ja.data(), crit, color.data(), &nc) == CSRC_OK);
        for (int32_t i = 0; i < a.n; ++i) CHECK(color[i] >= 0 && color[i] < nc);
    }
    std::vector<float> f(CSRC_NFEATURES, 0.f);
    CHECK(csrc_features(a.n, s.ia.data(), s.ja.data(), CSRC_F64, -1, f.data()) == CSRC_OK);
    // a small random network through csrc_select and csrc_mlp_predict_host
    const int H = 4, K = 3;
    const int64_t P = csrc_mlp_param_count(H, K);
    CHECK(P > 0);
    std::vector<float> params((size_t)P), mean(CSRC_NFEATURES, 0.f), scale(CSRC_NFEATURES, 1.f);
    for (auto &w : params) w = (float)(2.0 * g.unit() - 1.0);
    int32_t c1 = -1, c2 = -2;
    CHECK(csrc_select(a.n, s.ia.data(), s.ja.data(), CSRC_F64, H, K, params.data(), mean.data(), scale.data(),
                      &c1) == CSRC_OK);
    CHECK(csrc_mlp_predict_host(H, K, params.data(), mean.data(), scale.data(), f.data(), &c2) == CSRC_OK);
    CHECK(c1 == c2 && c1 >= 0 && c1 < K);
    CHECK(csrc_select(a.n, s.ia.data(), s.ja.data(), CSRC_F64, H, K, nullptr, mean.data(), scale.data(), &c1) ==
          CSRC_ERR_NO_MODEL);
    CHECK(csrc_select(a.n, s.ia.data(), s.ja.data(), CSRC_F64, 0, K, params.data(), mean.data(), scale.data(),
                      &c1) == CSRC_ERR_ARG);
    // storage types
    for (int32_t dt : {CSRC_F64, CSRC_F32, CSRC_BF16}) {
        std::vector<char> out((size_t)std::max<int64_t>(1, s.k) * 8);
        CHECK(csrc_quantize(s.k, s.al.data(), dt, out.data()) == CSRC_OK);
    }
    exercise_plans(s, a.n);
}

void exercise_errors()
{
    // duplicate entry, index out of range, unsymmetric pattern (then padded)
    std::vector<int64_t> rp = {0, 2, 3};
    std::vector<int32_t> dup = {0, 0, 1};
    int64_t k = 0;
    CHECK(csrc_count(2, rp.data(), dup.data(), 0, &k) == CSRC_ERR_DUPLICATE);
    std::vector<int32_t> oor = {0, 5, 1};
    CHECK(csrc_count(2, rp.data(), oor.data(), 0, &k) == CSRC_ERR_INDEX_RANGE);
    std::vector<int64_t> rp2 = {0, 2, 3};
    std::vector<int32_t> uns = {0, 1, 1};      // (0,1) stored, (1,0) missing
    CHECK(csrc_count(2, rp2.data(), uns.data(), 0, &k) == CSRC_ERR_NOT_STRUCT_SYM);
    CHECK(csrc_count(2, rp2.data(), uns.data(), CSRC_PAD_PATTERN, &k) == CSRC_OK && k == 1);
    std::vector<double> v = {1.0, 2.0, 3.0};
    std::vector<int32_t> ia(3), ja(1);
    std::vector<double> ad(2), al(1), au(1);
    CHECK(csrc_from_csr(2, rp2.data(), uns.data(), v.data(), CSRC_PAD_PATTERN, ia.data(), ja.data(), ad.data(),
                        al.data(), au.data()) == CSRC_OK);
    CHECK(ia[0] == 0 && ia[1] == 0 && ia[2] == 1 && ja[0] == 0 && ad[0] == 1.0 && ad[1] == 3.0 && al[0] == 0.0 &&
          au[0] == 2.0);
    CHECK(csrc_count(-1, rp.data(), dup.data(), 0, &k) == CSRC_ERR_ARG);
    CHECK(csrc_count(2, nullptr, dup.data(), 0, &k) == CSRC_ERR_ARG);
    csrc_plan_opts o;
    CHECK(csrc_plan_opts_default(CSRC_V_COUNT, &o) == CSRC_ERR_ARG);
    CHECK(csrc_plan_opts_default(CSRC_V_PRIVATE, &o) == CSRC_OK);
    o.block = 96;
    csrc_plan *p = nullptr;
    std::vector<int32_t> ia0 = {0};
    CHECK(csrc_plan_create(0, ia0.data(), nullptr, CSRC_F64, &o, &p) == CSRC_ERR_ARG);
    CHECK(csrc_mlp_param_count(0, 3) < 0 && csrc_mlp_param_count(4, 65) < 0);
    for (int s = -14; s <= 1; ++s) CHECK(csrc_status_string(s) != nullptr);
}

void exercise_rect(Rng &g)
{
    // n x m with m = n + 7: the square part symmetric, extra columns random
    const int32_t n = 40, m = 47;
    Csr sq = random_sym(g, n, 3, 0, 0.8);
    std::vector<int64_t> rp((size_t)n + 1, 0);
    std::vector<int32_t> col;
    std::vector<double> val;
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t q = sq.rp[i]; q < sq.rp[i + 1]; ++q) {
            col.push_back(sq.col[q]);
            val.push_back(sq.val[q]);
        }
        if (g.unit() < 0.5) {
            col.push_back(n + g.below(m - n));
            val.push_back(g.unit());
        }
        rp[i + 1] = (int64_t)col.size();
    }
    int64_t ns = -1, nr = -1;
    CHECK(csrc_rect_count(n, m, rp.data(), col.data(), &ns, &nr) == CSRC_OK);
    CHECK(ns + nr == (int64_t)col.size());
    std::vector<int64_t> srp((size_t)n + 1);
    std::vector<int32_t> scol((size_t)ns), iar((size_t)n + 1), jar((size_t)std::max<int64_t>(1, nr));
    std::vector<double> sval((size_t)ns), ar((size_t)std::max<int64_t>(1, nr));
    CHECK(csrc_rect_split(n, m, rp.data(), col.data(), val.data(), srp.data(), scol.data(), sval.data(), iar.data(),
                          jar.data(), ar.data()) == CSRC_OK);
    for (int64_t q = 0; q < nr; ++q) CHECK(jar[q] >= n && jar[q] < m);
}

void exercise_batch(Rng &g)
{
    std::vector<Csr> mats;
    std::vector<Split> sp;
    for (int m = 0; m < 5; ++m) mats.push_back(random_sym(g, 50 + 70 * m, 4, 30, 1.0));
    sp.resize(mats.size());
    std::vector<int32_t> n, r;
    std::vector<const int32_t *> ia, ja;
    for (size_t m = 0; m < mats.size(); ++m) {
        CHECK(split(mats[m], 0, sp[m]) == CSRC_OK);
        n.push_back(mats[m].n);
        r.push_back(1 + (int32_t)(m * 7 % 32));
        ia.push_back(sp[m].ia.data());
        ja.push_back(sp[m].ja.data());
    }
    for (int32_t vd : {CSRC_F64, CSRC_F32}) {
        csrc_batch_opts o = {0, 0, 0, CSRC_F32};
        csrc_batch_plan *b = nullptr;
        int st = csrc_batch_plan_create((int32_t)mats.size(), n.data(), ia.data(), ja.data(), r.data(), vd, &o, &b);
        CHECK(st == CSRC_OK);
        if (st) continue;
        CHECK(csrc_batch_workspace_bytes(b) > 0);
        CHECK(csrc_batch_plan_destroy(b) == CSRC_OK);
    }
}

}  // namespace

int main()
{
    Rng g(20260101);
    exercise_errors();
    // edge cases: empty matrix, one row, no diagonal, diagonal only
    {
        Csr e;
        e.rp = {0};
        exercise_matrix(g, e);
    }
    exercise_matrix(g, random_sym(g, 1, 0, 0, 1.0));
    exercise_matrix(g, random_sym(g, 17, 0, 0, 0.5));
    exercise_matrix(g, random_sym(g, 33, 3, 0, 0.0));
    for (int t = 0; t < 6; ++t) {
        const int32_t n = 64 + g.below(1500);
        exercise_matrix(g, random_sym(g, n, 1 + g.below(8), g.below(2) ? 40 : 0, 0.9));
    }
    exercise_rect(g);
    exercise_batch(g);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("sanitize ok\n");
    return 0;
}
