// autotune.cpp -- picks the storage layout, lanes per chain, threads per
// block and threshold-table placement of a configuration by timing short
// runs of every compiled candidate on the device.
//
// Every candidate runs the same chains (same seed, same sweeps) from the
// same initial state; its merged histogram, final spins and bins are hashed
// and compared with the first candidate's.  A candidate whose results differ
// is rejected (and reported), so the choice can never change the physics.
// Results are cached in a small JSON file (MUCA_AUTOTUNE_CACHE) keyed by the
// device architecture and the problem shape.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "muca_internal.h"
#include "runtime_internal.h"

using namespace muca;

namespace {

uint64_t fnv1a(uint64_t h, const void *p, size_t n)
{
    const uint8_t *b = (const uint8_t *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_key(const muca_config *c, const char *arch)
{
    std::ostringstream k;
    k << arch << "/m" << c->model << "/L" << c->L << "/q" << c->q << "/C" << c->n_chains << "/lay" << c->layout
      << "/N" << c->n_beads;
    return k.str();
}

} // namespace

// The cache is a flat JSON object {"key": [values], ...}, one entry per line.
bool muca_cache_lookup(const std::string &path, const std::string &key, std::string &values)
{
    std::ifstream f(path);
    if (!f)
        return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    const std::string pat = "\"" + key + "\": [";
    const size_t p = s.find(pat);
    if (p == std::string::npos)
        return false;
    const size_t e = s.find(']', p + pat.size());
    if (e == std::string::npos)
        return false;
    values = s.substr(p + pat.size(), e - p - pat.size());
    return true;
}

void muca_cache_store(const std::string &path, const std::string &key, const std::string &values)
{
    std::string body;
    {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            body = ss.str();
        }
    }
    std::vector<std::string> lines;
    std::istringstream in(body);
    std::string line;
    while (std::getline(in, line)) {
        if (line.find("\": [") == std::string::npos || line.find("\"" + key + "\"") != std::string::npos)
            continue;
        while (!line.empty() && (line.back() == ',' || line.back() == ' '))
            line.pop_back();
        lines.push_back(line);
    }
    lines.push_back("  \"" + key + "\": [" + values + "]");
    std::ofstream o(path);
    o << "{\n";
    for (size_t i = 0; i < lines.size(); ++i)
        o << lines[i] << (i + 1 < lines.size() ? ",\n" : "\n");
    o << "}\n";
}

namespace {

bool cache_lookup(const std::string &path, const std::string &key, int v[4])
{
    std::string t;
    return muca_cache_lookup(path, key, t) && std::sscanf(t.c_str(), "%d, %d, %d, %d", &v[0], &v[1], &v[2], &v[3]) == 4;
}

void cache_store(const std::string &path, const std::string &key, const int v[4])
{
    char buf[128];
    std::snprintf(buf, sizeof buf, "%d, %d, %d, %d", v[0], v[1], v[2], v[3]);
    muca_cache_store(path, key, buf);
}

} // namespace

extern "C" int muca_autotune(const muca_config *cfg, void *d_ws, uint64_t ws_bytes, int64_t sweeps, void *stream,
                             muca_config *best, double *best_ms_per_sweep)
try {
    if (!cfg || !best || sweeps < 1)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return muca_fail(MUCA_E_HIP, "no device");
    const char *env = std::getenv("MUCA_AUTOTUNE_CACHE");
    const std::string key = cache_key(cfg, prop.gcnArchName);
    if (env && *env) {
        int v[4];
        if (cache_lookup(env, key, v)) {
            *best = *cfg;
            best->layout = v[0];
            best->lanes_per_chain = v[1];
            best->chains_per_block = v[2];
            best->table_in_lds = v[3];
            if (best_ms_per_sweep)
                *best_ms_per_sweep = -1.0;
            return MUCA_OK;
        }
    }
    std::vector<muca_config> cands;
    const bool lattice = cfg->model != kPolymer;
    if (lattice) {
        std::vector<int> layouts;
        if (cfg->model == kPotts)
            layouts = {MUCA_LAYOUT_BYTE};
        else if (cfg->layout != MUCA_LAYOUT_AUTO)
            layouts = {cfg->layout};
        else
            layouts = {MUCA_LAYOUT_BIT, MUCA_LAYOUT_BYTE};
        for (int lay : layouts)
            for (int lpc : {1, 2, 4, 16})
                for (int threads : {64, 256, 512})
                    for (int tl : {0, 1}) {
                        muca_config c = *cfg;
                        c.layout = lay;
                        c.lanes_per_chain = lpc;
                        c.chains_per_block = threads / lpc > 0 ? threads / lpc : 1;
                        if (c.chains_per_block * lpc != threads || (threads > 256 && tl == 0))
                            continue;
                        c.table_in_lds = tl;
                        cands.push_back(c);
                    }
    } else {
        for (int cpb : {1, 2, 4}) {
            muca_config c = *cfg;
            c.chains_per_block = cpb;
            cands.push_back(c);
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return muca_fail(MUCA_E_HIP, "event create failed");
    bool have_ref = false, have_best = false;
    uint64_t ref = 0;
    double best_ms = 0.0;
    int rejected = 0;
    std::vector<float> pos;
    if (!lattice) {
        // a polymer candidate needs initial positions: a straight chain with unit bonds along x
        pos.assign((size_t)cfg->n_chains * cfg->n_beads * 3, 0.0f);
        for (int c = 0; c < cfg->n_chains; ++c)
            for (int j = 0; j < cfg->n_beads; ++j)
                pos[((size_t)c * cfg->n_beads + j) * 3] = (float)j;
    }
    for (const muca_config &c : cands) {
        uint64_t need = 0;
        if (muca_workspace_bytes(&c, &need) != MUCA_OK || need > ws_bytes)
            continue;
        muca_run *r = nullptr;
        if (muca_init(&c, d_ws, ws_bytes, lattice ? nullptr : pos.data(), stream, &r) != MUCA_OK)
            continue;
        if (lattice && c.table_in_lds == 1 && !r->g.table_in_lds) {
            muca_free(r);
            continue;
        }
        // one untimed launch loads the code, then the timed one
        int rc = muca_thermalize(r, 1, stream);
        (void)hipEventRecord(e0, s);
        if (rc == MUCA_OK)
            rc = muca_run_iteration(r, sweeps, stream);
        (void)hipEventRecord(e1, s);
        muca_iter_stats st;
        if (rc == MUCA_OK)
            rc = muca_merge_update(r, &st);
        float ms = 0.0f;
        if (rc == MUCA_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = MUCA_E_HIP;
        if (rc != MUCA_OK) {
            muca_free(r);
            continue;
        }
        const int C = c.n_chains;
        std::vector<int32_t> bins(C);
        std::vector<double> en(C);
        std::vector<uint8_t> state(lattice ? (size_t)C * r->g.n_sites : (size_t)C * c.n_beads * 12);
        rc = muca_get_chain_state(r, 0, C, state.data(), bins.data(), lattice ? nullptr : en.data());
        uint64_t h = 1469598103934665603ull;
        h = fnv1a(h, r->H_last.data(), r->H_last.size() * 8);
        h = fnv1a(h, state.data(), state.size());
        h = fnv1a(h, bins.data(), bins.size() * 4);
        muca_free(r);
        if (rc != MUCA_OK)
            continue;
        if (!have_ref) {
            ref = h;
            have_ref = true;
        } else if (h != ref) {
            ++rejected;
            std::fprintf(stderr, "muca_autotune: candidate layout %d lpc %d cpb %d lds %d changed the results; "
                                 "rejected\n",
                         c.layout, c.lanes_per_chain, c.chains_per_block, c.table_in_lds);
            continue;
        }
        const double per = (double)ms / (double)sweeps;
        if (!have_best || per < best_ms) {
            best_ms = per;
            *best = c;
            have_best = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!have_best)
        return muca_fail(MUCA_E_NOMEM, "no candidate fits the workspace");
    if (best_ms_per_sweep)
        *best_ms_per_sweep = best_ms;
    if (env && *env) {
        const int v[4] = {best->layout, best->lanes_per_chain, best->chains_per_block, best->table_in_lds};
        cache_store(env, key, v);
    }
    return rejected ? muca_fail(MUCA_OK, "%d candidates rejected", rejected) : MUCA_OK;
}
MUCA_ABI_CATCH
