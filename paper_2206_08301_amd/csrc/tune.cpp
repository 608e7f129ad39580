// tune.cpp -- the plan cache behind the autotuner (deinsum_tune_*).
//
// Keys name the path (per-call kernel or batched job), the problem's order,
// free mode, precision, rank and dims.  The file format is one entry per line:
//   <key> <nt> <ni> <mt> <xnt> <split> <order> <xcd> <microseconds>
// with '#' starting a comment line.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "internal.h"
#include "tune.h"

namespace deinsum {

namespace {

std::mutex g_mu;
std::map<std::string, TuneChoice> g_cache;
bool g_env_loaded = false;

deinsum_status load_file(const char *path, bool must_exist)
{
    std::ifstream f(path);
    if (!f) return must_exist ? fail(DEINSUM_ERR_INVALID_ARG, std::string("tune_load: cannot open ") + path) : DEINSUM_OK;
    std::string line;
    int lineno = 0;
    while (std::getline(f, line)) {
        ++lineno;
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string key;
        TuneChoice c;
        if (!(is >> key >> c.nt >> c.ni >> c.mt >> c.xnt >> c.split >> c.order >> c.xcd >> c.us) || c.nt < 1 ||
            c.ni < 1 || c.mt < 1 || c.xnt < 0 || c.xnt > 1 || c.split < 0 || c.order < 0 || c.order > kTuneKout || c.xcd < 0 ||
            c.xcd > 1)
            return fail(DEINSUM_ERR_PARSE, std::string("tune_load: bad entry at line ") + std::to_string(lineno));
        g_cache[key] = c;
    }
    return DEINSUM_OK;
}

deinsum_status save_file(const char *path)
{
    std::ofstream f(path, std::ios::trunc);
    if (!f) return fail(DEINSUM_ERR_INVALID_ARG, std::string("tune_save: cannot write ") + path);
    f << "# deinsum MTTKRP plan cache: key nt ni mt xnt split order xcd microseconds\n";
    for (const auto &kv : g_cache) {
        const TuneChoice &c = kv.second;
        f << kv.first << ' ' << c.nt << ' ' << c.ni << ' ' << c.mt << ' ' << c.xnt << ' ' << c.split << ' ' << c.order
          << ' ' << c.xcd << ' ' << c.us << '\n';
    }
    return f ? DEINSUM_OK : fail(DEINSUM_ERR_INVALID_ARG, std::string("tune_save: write failed for ") + path);
}

void load_env_locked()
{
    if (g_env_loaded) return;
    g_env_loaded = true;
    if (const char *p = std::getenv("DEINSUM_TUNE_CACHE")) (void)load_file(p, false);
}

}  // namespace

std::string tune_key(int path, const MttkrpProblem &pb)
{
    std::string k = path == TUNE_BATCH ? "b" : "s";
    k += ":N" + std::to_string(pb.N) + ":n" + std::to_string(pb.n) + ":p" + std::to_string(pb.prec) + ":R" +
         std::to_string(pb.R) + ":";
    for (int m = 0; m < pb.N; ++m) k += (m ? "x" : "") + std::to_string(pb.dims[m]);
    return k;
}

bool tune_lookup(const std::string &key, TuneChoice *out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string &key, const TuneChoice &c)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    g_cache[key] = c;
    if (const char *p = std::getenv("DEINSUM_TUNE_CACHE")) (void)save_file(p);
}

int tune_splits(int64_t c0, int64_t O, int out[8])
{
    const int64_t cand[5] = {c0, c0 / 2, c0 * 2, c0 / 4, c0 * 4};
    int n = 0;
    for (int64_t v : cand) {
        v = std::max<int64_t>(1, std::min<int64_t>(v, O));
        if (v > (int64_t(1) << 30)) continue;
        bool dup = false;
        for (int i = 0; i < n; ++i) dup |= out[i] == v;
        if (!dup) out[n++] = static_cast<int>(v);
    }
    return n;
}

}  // namespace deinsum

using namespace deinsum;

extern "C" {

deinsum_status deinsum_tune_load(const char *path)
{
    if (!path) return fail(DEINSUM_ERR_INVALID_ARG, "tune_load: null path");
    std::lock_guard<std::mutex> lk(g_mu);
    g_env_loaded = true;
    if (deinsum_status st = load_file(path, true)) return st;
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_tune_save(const char *path)
{
    if (!path) return fail(DEINSUM_ERR_INVALID_ARG, "tune_save: null path");
    std::lock_guard<std::mutex> lk(g_mu);
    if (deinsum_status st = save_file(path)) return st;
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
    g_env_loaded = true;
    return DEINSUM_OK;
}

deinsum_status deinsum_tune_entries(int64_t *entries)
{
    if (!entries) return fail(DEINSUM_ERR_INVALID_ARG, "tune_entries: null argument");
    std::lock_guard<std::mutex> lk(g_mu);
    *entries = static_cast<int64_t>(g_cache.size());
    return DEINSUM_OK;
}

}  // extern "C"
