// qtamd_tune.cpp -- autotuner decision table and its JSON persistence.
//
// The measuring itself happens where the kernels are (qt_me_plan_autotune times the fused
// SpMV-stage kernel of a plan for every candidate shape; the dense kernel is timed over a short
// step budget for each built wave count).  This file keeps the decisions: per size bucket, the
// fastest shape measured so far, consulted by every plan and server created afterwards.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "qt_dense.h"
#include "qt_host.h"
#include "qt_tune.h"

namespace qt {

namespace {
std::mutex g_mu;
std::map<std::string, CsrShape> g_csr;
std::map<std::string, int> g_dense;
}  // namespace

std::string csr_tune_key(int32_t prec, int64_t rows, double mean_row)
{
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= rows) ++lg;
    char b[96];
    std::snprintf(b, sizeof b, "csr:%s:n%d:r%d", prec == QT_F64 ? "f64" : "mixed", lg, (int)std::lround(mean_row));
    return b;
}

std::string dense_tune_key(int32_t prec, int np)
{
    char b[64];
    std::snprintf(b, sizeof b, "dense:%s:np%d:waves", prec == QT_F64 ? "f64" : "mixed", np);
    return b;
}

bool tune_lookup_csr(const std::string &key, CsrShape *out)
{
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_csr.find(key);
    if (it == g_csr.end()) return false;
    *out = it->second;
    return true;
}

void tune_store_csr(const std::string &key, CsrShape s)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_csr[key] = s;
}

bool tune_lookup_dense(const std::string &key, int *waves)
{
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_dense.find(key);
    if (it == g_dense.end()) return false;
    *waves = it->second;
    return true;
}

void tune_store_dense(const std::string &key, int waves)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_dense[key] = waves;
}

CsrShape csr_default_shape(int64_t rows, double mean_row)
{
    CsrShape s;
    s.lpr = mean_row <= 8.0 ? 4 : (mean_row <= 40.0 ? 8 : 16);
    // small problems: one row per group keeps enough workgroups in flight to fill 256 CUs
    s.rg = rows >= (int64_t(1) << 19) ? 2 : 1;
    s.xcd = 0;
    // the matrix through the caches, in 16-byte runs of 4 entries where the shape is built so
    s.keep = csr_shape_supported(s.lpr, s.rg, 2) ? 2 : 1;
    return s;
}

// FP64: one wave per tile row; FP32: two waves per SIMD where the padded size has more than 4 tiles
int dense_default_waves(int np, int32_t prec)
{
    const int nt = np / 16;
    if (prec == QT_F64) return nt;
    return nt * nt > 4 ? 8 : nt * nt <= 1 ? 2 : 4;
}

int csr_candidates(CsrShape *out, int max, bool single)
{
    static const int lprs[] = {4, 8, 16}, rgs[] = {1, 2, 4};
    int n = 0;
    for (int k = 0; k < 3; ++k)
        for (int x = 0; x < (single ? 2 : 1); ++x)
            for (int l : lprs)
                for (int r : rgs)
                    if (r <= l && n < max && csr_shape_supported(l, r, k)) out[n++] = CsrShape{l, r, x, k};
    return n;
}

// a stored wave count is taken only for a key of the current form and a count the solver is built with
static bool dense_key_accepts(const char *key, int waves)
{
    int np = 0, end = 0;
    char prec[16];
    if (std::sscanf(key, "dense:%15[^:]:np%d:waves%n", prec, &np, &end) != 2 || end == 0 || key[end] != 0)
        return false;
    return dense_waves_allowed(np, std::strcmp(prec, "f64") == 0 ? QT_F64 : QT_MIXED, waves);
}

}  // namespace qt

using namespace qt;

extern "C" {

qt_status qt_tune_save(const char *path)
{
    if (!path) return set_error(QT_EINVAL, "qt_tune_save: null path");
    FILE *f = std::fopen(path, "w");
    if (!f) return set_error(QT_EINVAL, std::string("qt_tune_save: cannot open ") + path);
    std::lock_guard<std::mutex> g(g_mu);
    std::fprintf(f, "{\n");
    size_t k = 0, n = g_csr.size() + g_dense.size();
    for (auto &kv : g_csr)
        std::fprintf(f, "  \"%s\": [%d, %d, %d, %d]%s\n", kv.first.c_str(), kv.second.lpr, kv.second.rg,
                     kv.second.xcd, kv.second.keep, ++k < n ? "," : "");
    for (auto &kv : g_dense)
        std::fprintf(f, "  \"%s\": [%d]%s\n", kv.first.c_str(), kv.second, ++k < n ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    return QT_OK;
}

qt_status qt_tune_load(const char *path)
{
    if (!path) return set_error(QT_EINVAL, "qt_tune_load: null path");
    FILE *f = std::fopen(path, "r");
    if (!f) return set_error(QT_EINVAL, std::string("qt_tune_load: cannot open ") + path);
    char line[256];
    int loaded = 0;
    while (std::fgets(line, sizeof line, f)) {
        char key[128];
        int a = 0, b = 0, c = 0, e = 0;
        const int m = std::sscanf(line, " \"%127[^\"]\": [%d, %d, %d, %d]", key, &a, &b, &c, &e);
        if (m >= 3 && std::strncmp(key, "csr:", 4) == 0 && csr_shape_supported(a, b, e) && (c == 0 || c == 1)) {
            tune_store_csr(key, CsrShape{a, b, c, e});
            ++loaded;
        } else if (m >= 2 && std::strncmp(key, "dense:", 6) == 0 && dense_key_accepts(key, a)) {
            tune_store_dense(key, a);
            ++loaded;
        }
    }
    std::fclose(f);
    return QT_OK;
}

}  // extern "C"
