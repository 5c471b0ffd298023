// runtime.cpp -- host side of the C ABI (include/muca.h).
//
// Owns the per-run host state of the multicanonical iteration
// (arXiv:1312.2213, parallel-scheme paragraph and Fig. 1 caption):
//   * the log weights lnW and, for the recursion that uses the statistics of
//     all earlier iterations (paragraph after Eq. 2), the log weight ratios
//     lnR of neighbouring bins and their accumulated statistical weights P;
//   * the flatness test that ends the iteration;
//   * the integer acceptance thresholds uploaded for the kernels;
//   * reweighting to canonical averages (Eq. 2).
// All FP64 arithmetic here runs in a fixed order (no FMA contraction), so
// the weights and thresholds are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/muca.h"
#include "muca_internal.h"
#include "runtime_internal.h"

using namespace muca;

// fixed storage: reporting an error never allocates
static thread_local char g_last_error[512];

int muca_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::memcpy(g_last_error, buf, sizeof buf);
    return code;
}

const char *muca_last_error(void) { return g_last_error; }

RoctxRange::RoctxRange(const char *name) { roctxRangePushA(name); }
RoctxRange::~RoctxRange() { roctxRangePop(); }

static double wall_seconds()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static std::atomic<int64_t> g_run_ids{0};
static std::mutex g_log_mutex;

void muca_log_iteration(const muca_run *r, const muca_iter_stats &s, double seconds, double attempts)
{
    const char *path = std::getenv("MUCA_ITER_LOG");
    if (!path || !*path)
        return;
    static const char *names[] = {"ising", "potts", "muma", "polymer"};
    std::lock_guard<std::mutex> lock(g_log_mutex);
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f,
                 "{\"run\": %lld, \"model\": \"%s\", \"L\": %d, \"q\": %d, \"n_beads\": %d, \"chains\": %d, "
                 "\"seed\": %llu, \"iteration\": %lld, \"sweeps\": %lld, \"samples\": %lld, \"flatness\": %.17g, "
                 "\"flat\": %d, \"lo_visited\": %d, \"hi_visited\": %d, \"accept_rate\": %.17g, "
                 "\"seconds\": %.6f, \"attempts_per_s\": %.6g}\n",
                 (long long)r->log_id, names[r->g.model & 3], r->cfg.L, r->cfg.q, r->cfg.n_beads, r->cfg.n_chains,
                 (unsigned long long)r->cfg.seed, (long long)s.iteration, (long long)s.sweeps, (long long)s.samples,
                 s.flatness, s.flat, s.lo_visited, s.hi_visited, s.accept_rate, seconds,
                 seconds > 0.0 ? attempts / seconds : 0.0);
    std::fclose(f);
}

static size_t align256(size_t x) { return (x + 255u) & ~(size_t)255u; }

// ---------------------------------------------------------------------------
// Geometry of a configuration
// ---------------------------------------------------------------------------
static int bin_step(int model) { return model == kIsing ? 4 : (model == kPotts ? 1 : 2); }

static int n_cols_of(int model) { return model == kIsing ? 5 : (model == kPotts ? 9 : 10); }

int muca_geometry(const muca_config *c, Geometry *g)
{
    if (!c || !g)
        return muca_fail(MUCA_E_ARG, "null argument");
    if (c->abi_version != MUCA_ABI_VERSION)
        return muca_fail(MUCA_E_ARG, "abi_version %u, library has %u", c->abi_version, MUCA_ABI_VERSION);
    if (c->n_chains < 1)
        return muca_fail(MUCA_E_ARG, "n_chains must be >= 1");
    if (c->chain0 < 0 || (int64_t)c->chain0 + c->n_chains > 0x7FFFFFFFll)
        return muca_fail(MUCA_E_ARG, "chain0 %d with %d chains outside the 31-bit chain numbering", c->chain0,
                         c->n_chains);
    std::memset(g, 0, sizeof *g);
    g->model = c->model;
    g->c_pad = (c->n_chains + 63) / 64 * 64;
    if (c->model == kPolymer)
        return muca_polymer_geometry(c, g);
    if (c->model != kIsing && c->model != kPotts && c->model != kMuma)
        return muca_fail(MUCA_E_ARG, "unknown model %d", c->model);
    if (c->moves != 0)
        return muca_fail(MUCA_E_ARG, "moves %d: the move set is a polymer option", c->moves);
    if (!lattice_size_supported(c->L))
        return muca_fail(MUCA_E_ARG, "L = %d not compiled (4, 8, 16, 24, 32, 48, 64)", c->L);
    const int N = c->L * c->L;
    g->L = c->L;
    g->n_sites = N;
    g->step = bin_step(c->model);
    g->n_cols = n_cols_of(c->model);
    if (c->model == kPotts) {
        if (c->q < 2 || c->q > 255)
            return muca_fail(MUCA_E_ARG, "q = %d outside 2..255", c->q);
        if (c->lo < 0 || c->hi > 2 * N || c->lo > c->hi)
            return muca_fail(MUCA_E_ARG, "Potts range [%d, %d] outside [0, %d]", c->lo, c->hi, 2 * N);
        g->layout = kLayoutByte;
    } else {
        const int emin = c->model == kIsing ? -2 * N : -N;
        const int emax = -emin;
        if (c->lo < emin || c->hi > emax || c->lo > c->hi || (c->lo - emin) % g->step ||
            (c->hi - emin) % g->step)
            return muca_fail(MUCA_E_ARG, "range [%d, %d] not on the grid %d + %d k within [%d, %d]",
                             c->lo, c->hi, emin, g->step, emin, emax);
        g->layout = c->layout == MUCA_LAYOUT_BYTE ? kLayoutByte : kLayoutBit;
    }
    if (c->layout != MUCA_LAYOUT_AUTO && c->layout != MUCA_LAYOUT_BIT && c->layout != MUCA_LAYOUT_BYTE)
        return muca_fail(MUCA_E_ARG, "unknown layout %d", c->layout);
    if (c->model == kPotts && c->layout == MUCA_LAYOUT_BIT)
        return muca_fail(MUCA_E_ARG, "Potts has no bit layout");
    g->n_bins = (c->hi - c->lo) / g->step + 1;
    g->wpr = words_per_row(c->L, g->layout);
    int lpc = c->lanes_per_chain;
    if (lpc == 0) {
        // enough lanes to give every SIMD of the chip a wavefront, at most 16;
        // Potts splits each row over the lanes (L / lpc sites per lane), so
        // 16 lanes need L a multiple of 16
        lpc = (c->model == kPotts && c->L % 16) ? 4 : 16;
        while (lpc > 1 && (long)g->c_pad * lpc > 65536L)
            lpc /= lpc == 16 ? 4 : 2;
    }
    if (lpc != 1 && lpc != 2 && lpc != 4 && lpc != 16)
        return muca_fail(MUCA_E_ARG, "lanes_per_chain %d not in {1, 2, 4, 16}", lpc);
    g->lpc = lpc;
    // default: 256-thread blocks, so a block that stages the threshold table
    // in LDS (one block per CU) still carries four wavefronts of work; at
    // init, 512 where that table leaves room for one block per CU and the
    // launch fills every CU with such blocks
    int cpb = c->chains_per_block ? c->chains_per_block * lpc : 256;
    if (c->chains_per_block && (c->chains_per_block < 1 || cpb > 512 || cpb % 64 || (cpb & (cpb - 1))))
        return muca_fail(MUCA_E_ARG, "chains_per_block %d x lanes_per_chain %d must be 64, 128, 256 or 512 threads",
                         c->chains_per_block, lpc);
    while (((long)g->c_pad * lpc) % cpb)
        cpb /= 2;
    g->cpb = cpb;
    // LDS of one block: the packed 16-bit histogram, plus the staged table
    // (Potts stages 8 of its 9 columns)
    const size_t hist_lds = (size_t)lds_hist_words(g->n_bins) * 4u;
    const size_t stage_lds = (size_t)g->n_bins * lds_table_cols(g->model) * 4u;
    const size_t tab_lds = (size_t)g->n_bins * g->n_cols * 4u;
    g->lds_bytes = hist_lds + stage_lds;
    if (c->table_in_lds == 1 && g->lds_bytes > 160u * 1024u)
        return muca_fail(MUCA_E_ARG, "threshold table of %zu bytes does not fit in LDS", stage_lds);
    if (hist_lds > 64u * 1024u)
        return muca_fail(MUCA_E_ARG, "%d bins exceed the LDS histogram", g->n_bins);
    g->table_in_lds = c->table_in_lds == 1 || (c->table_in_lds < 0 && g->lds_bytes <= 160u * 1024u);
    if (g->cpb > 256 && !g->table_in_lds)
        return muca_fail(MUCA_E_ARG, "blocks of %d threads need the threshold table staged in LDS", g->cpb);
    // workspace carve
    size_t off = 0;
    g->off_words = off;
    off = align256(off + (size_t)c->L * g->wpr * g->c_pad * 4u);
    g->off_bins = off;
    off = align256(off + (size_t)g->c_pad * 4u);
    g->off_values = off;
    off = align256(off + (size_t)g->c_pad * 4u);
    g->off_table = off;
    off = align256(off + tab_lds);
    g->off_hist = off; // histogram, then the count of accepted moves
    off = align256(off + (size_t)(g->n_bins + 1) * 8u);
    g->ws_bytes = off;
    return MUCA_OK;
}





// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int muca_config_default(int32_t model, int32_t L, int32_t q, int32_t n_chains, uint64_t seed,
                                   muca_config *c)
try {
    if (!c)
        return muca_fail(MUCA_E_ARG, "null config");
    std::memset(c, 0, sizeof *c);
    c->abi_version = MUCA_ABI_VERSION;
    c->model = model;
    c->L = L;
    c->q = model == kPotts ? q : 2;
    c->n_chains = n_chains;
    c->layout = MUCA_LAYOUT_AUTO;
    c->seed = seed;
    c->flat_threshold = 0.5;
    c->chains_per_block = 0;
    c->table_in_lds = -1;
    const int N = L * L;
    if (model == kIsing) {
        c->lo = -2 * N;
        c->hi = 2 * N;
    } else if (model == kPotts) {
        c->lo = 0;
        c->hi = 2 * N;
    } else if (model == kMuma) {
        c->lo = -N;
        c->hi = N;
        c->beta = 0.5;
    }
    c->n_beads = 40;
    c->n_bins = 2500;
    c->x_lo = -200.0;
    c->x_hi = 50.0;
    c->lj_eps = 1.0;
    c->lj_sigma = 1.0;
    c->lj_rcut = 2.5;
    c->fene_k = 40.0;
    c->fene_r0 = 1.0;
    c->fene_R = 0.5;
    c->step = 0.3f;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_workspace_bytes(const muca_config *c, uint64_t *bytes)
try {
    Geometry g;
    int rc = muca_geometry(c, &g);
    if (rc)
        return rc;
    if (!bytes)
        return muca_fail(MUCA_E_ARG, "null bytes");
    *bytes = g.ws_bytes;
    return MUCA_OK;
}
MUCA_ABI_CATCH

static int check_run(const muca_run *r)
{
    if (!r)
        return muca_fail(MUCA_E_ARG, "null run");
    if (r->poisoned)
        return muca_fail(MUCA_E_STATE, "run poisoned by an earlier HIP error");
    if (r->merge_begun)
        return muca_fail(MUCA_E_STATE, "a merge was begun and not finished (muca_merge_finish)");
    return MUCA_OK;
}

muca_run::~muca_run()
{
    if (merge_ev)
        (void)hipEventDestroy(merge_ev);
    if (h_hist)
        (void)hipHostFree(h_hist);
}

// The table goes out from its pinned host mirror without a wait: the next
// launch on the run's stream is ordered after the copy, a switch to another
// stream waits for it, and every caller synchronised the stream before it
// rewrote the mirror, so no earlier copy still reads it.
int muca_upload_thresholds(muca_run *r)
{
    HIP_OR_POISON(r, hipMemcpyAsync(r->d_table, r->T.data(), r->T.size() * 4u, hipMemcpyHostToDevice, r->stream));
    return MUCA_OK;
}

int muca_rebuild_thresholds(muca_run *r)
{
    if (r->g.model == kPolymer)
        muca_polymer_build(r);
    else
        muca_lattice_thresholds(r->g.model, r->cfg.beta, r->g.n_bins, r->g.n_cols, r->lnW.data(), r->T.data());
    return muca_upload_thresholds(r);
}

extern "C" int muca_init(const muca_config *c, void *d_ws, uint64_t ws_bytes, const float *h_pos,
                         void *stream, muca_run **out)
try {
    if (!out)
        return muca_fail(MUCA_E_ARG, "null out");
    *out = nullptr;
    Geometry g;
    int rc = muca_geometry(c, &g);
    if (rc)
        return rc;
    if (!d_ws || ((uintptr_t)d_ws & 255u))
        return muca_fail(MUCA_E_ARG, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < g.ws_bytes)
        return muca_fail(MUCA_E_NOMEM, "workspace of %llu bytes, need %llu", (unsigned long long)ws_bytes,
                         (unsigned long long)g.ws_bytes);
    if (g.model != kPolymer && g.table_in_lds) {
        // stage the table in LDS only if the device grants that much per block
        int dev = 0, lim = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) {
            const size_t need = g.lds_bytes;
            if (need > (size_t)lim) {
                if (c->table_in_lds == 1 || g.cpb > 256)
                    return muca_fail(MUCA_E_ARG, "LDS request of %zu bytes above the device limit %d", need, lim);
                g.table_in_lds = false;
            }
        }
    }
    if (g.model != kPolymer && c->chains_per_block == 0 && g.table_in_lds) {
        // a staged table too large for two blocks of 256 per CU leaves one
        // wavefront per SIMD; a block of 512 puts two there, once the launch
        // has such a block for every CU
        int dev = 0, cus = 0, lds_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess) {
            const long lanes = (long)g.c_pad * g.lpc;
            if (2 * g.lds_bytes > (size_t)lds_cu && g.lds_bytes <= (size_t)lds_cu && cus > 0 &&
                lanes >= 512L * cus && lanes % 512 == 0)
                g.cpb = 512;
        }
    }
    RoctxRange range("muca_init");
    muca_run *r = new muca_run();
    r->log_id = ++g_run_ids;
    r->t_last = wall_seconds();
    r->cfg = *c;
    r->g = g;
    r->stream = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)d_ws;
    r->ws = ws;
    r->d_words = (uint32_t *)(ws + g.off_words);
    r->d_bins = (int32_t *)(ws + g.off_bins);
    r->d_values = (int32_t *)(ws + g.off_values);
    r->d_table = (uint32_t *)(ws + g.off_table);
    r->d_hist = (unsigned long long *)(ws + g.off_hist);
    r->lnW.assign(g.n_bins, 0.0);
    r->lnR.assign(g.n_bins, 0.0);
    r->P.assign(g.n_bins, 0.0);
    r->H_last.assign(g.n_bins, 0u);
    r->lnW_last.assign(g.n_bins, 0.0);
    if (g.model != kPolymer) {
        // coherent: the merge's drain kernel writes it directly
        hipError_t e = hipHostMalloc((void **)&r->h_hist, (size_t)(g.n_bins + 1) * 8u,
                                     hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess)
            e = hipHostGetDevicePointer((void **)&r->h_hist_dev, r->h_hist, 0);
        if (e != hipSuccess) {
            delete r;
            return muca_fail(MUCA_E_HIP, "init: pinned staging: %s", hipGetErrorString(e));
        }
    }
    if (g.model == kPolymer) {
        rc = muca_polymer_init(r, h_pos);
        if (rc) {
            delete r;
            return rc;
        }
        *out = r;
        return MUCA_OK;
    }
    r->mask.assign(g.n_bins, 1);
    muca_reachable_mask(g.model, c->q, c->lo, g.step, g.n_sites, g.n_bins, r->mask.data());
    try {
        r->T.assign((size_t)g.n_bins * g.n_cols, 0u);
    } catch (const std::bad_alloc &) {
        delete r;
        return muca_fail(MUCA_E_NOMEM, "init: pinned host memory for the threshold table");
    }
    LatticeInitArgs a{};
    a.words = r->d_words;
    a.bins = r->d_bins;
    a.values = r->d_values;
    a.k0 = (uint32_t)(c->seed & 0xffffffffu);
    a.k1 = (uint32_t)(c->seed >> 32);
    a.c_pad = g.c_pad;
    a.L = c->L;
    a.q = c->q;
    a.lo = c->lo;
    a.step = g.step;
    a.model = g.model;
    a.layout = g.layout;
    a.chain0 = c->chain0;
    hipError_t e = launch_lattice_init(a, r->stream);
    if (e == hipSuccess)
        e = launch_fill_u64(r->d_hist, g.n_bins + 1, r->stream);
    std::vector<int32_t> bins(g.c_pad);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bins.data(), r->d_bins, bins.size() * 4u, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) {
        delete r;
        return muca_fail(MUCA_E_HIP, "init: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < g.c_pad; ++i) {
        if (bins[i] < 0 || bins[i] >= g.n_bins) {
            delete r;
            return muca_fail(MUCA_E_RANGE, "chain %d starts in bin %d outside [0, %d)", i, bins[i],
                             g.n_bins);
        }
    }
    rc = muca_rebuild_thresholds(r);
    if (rc) {
        delete r;
        return rc;
    }
    *out = r;
    return MUCA_OK;
}
MUCA_ABI_CATCH

int muca_enqueue_sweeps(muca_run *r, int64_t sweeps, bool record, hipStream_t s, unsigned long long *em,
                        unsigned long long *hist_blocks)
{
    if (r->g.model == kPolymer)
        return muca_polymer_enqueue(r, sweeps, record, s);
    const Geometry &g = r->g;
    // the sweep count of one launch is a 32-bit argument
    const int64_t max_chunk = 1 << 30;
    const int64_t n_launch = (sweeps + max_chunk - 1) / max_chunk;
    int64_t done = 0;
    for (int64_t k = 0; k < n_launch; ++k) {
        const int64_t n = (sweeps * (k + 1)) / n_launch - done;
        LatticeArgs a{};
        a.words = r->d_words;
        a.bins = r->d_bins;
        a.thresholds = r->d_table;
        a.hist = r->d_hist;
        a.k0 = (uint32_t)(r->cfg.seed & 0xffffffffu);
        a.k1 = (uint32_t)(r->cfg.seed >> 32);
        a.g0 = r->sweep;
        a.n_sweeps = (int32_t)n;
        a.n_chains = r->cfg.n_chains;
        a.c_pad = g.c_pad;
        a.n_bins = g.n_bins;
        a.q = r->cfg.q;
        a.record = record ? 1 : 0;
        a.table_in_lds = g.table_in_lds ? 1 : 0;
        a.chain0 = r->cfg.chain0;
        a.em = em;
        a.accepts = r->d_hist + g.n_bins;
        a.hist_blocks = hist_blocks;
        HIP_OR_POISON(r, launch_lattice_sweeps(g.model, g.L, g.layout, g.lpc, g.cpb, a, s));
        r->sweep += (uint32_t)n;
        done += n;
    }
    return MUCA_OK;
}

int muca_use_stream(muca_run *r, hipStream_t s)
{
    if (r->stream != s)
        HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    r->stream = s;
    return MUCA_OK;
}

extern "C" int muca_run_iteration(muca_run *r, int64_t sweeps, void *stream)
try {
    RoctxRange range("muca_run_iteration");
    int rc = check_run(r);
    if (rc)
        return rc;
    if (sweeps < 1)
        return muca_fail(MUCA_E_ARG, "sweeps must be >= 1");
    rc = muca_use_stream(r, (hipStream_t)stream);
    if (rc)
        return rc;
    rc = muca_enqueue_sweeps(r, sweeps, true, r->stream);
    if (rc)
        return rc;
    r->pending += sweeps;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_em_shape(const muca_run *r, int32_t *n_e, int32_t *n_m)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (r->g.model != kMuma)
        return muca_fail(MUCA_E_ARG, "joint (E, M) histogram: multimagnetic runs only");
    if (n_e)
        *n_e = r->g.n_sites + 1;
    if (n_m)
        *n_m = r->g.n_bins;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_run_iteration_em(muca_run *r, int64_t sweeps, uint64_t *d_em, void *stream)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (r->g.model != kMuma)
        return muca_fail(MUCA_E_ARG, "joint (E, M) histogram: multimagnetic runs only");
    if (!d_em)
        return muca_fail(MUCA_E_ARG, "null joint histogram");
    if (sweeps < 1)
        return muca_fail(MUCA_E_ARG, "sweeps must be >= 1");
    rc = muca_use_stream(r, (hipStream_t)stream);
    if (rc)
        return rc;
    rc = muca_enqueue_sweeps(r, sweeps, true, r->stream, (unsigned long long *)d_em);
    if (rc)
        return rc;
    r->pending += sweeps;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_blocks_shape(const muca_run *r, int32_t *n_blocks, int32_t *chains_per_block)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    const Geometry &g = r->g;
    if (g.model == kPolymer)
        return muca_fail(MUCA_E_ARG, "per-block histograms: lattice runs only");
    if (n_blocks)
        *n_blocks = (int32_t)(((int64_t)g.c_pad * g.lpc) / g.cpb);
    if (chains_per_block)
        *chains_per_block = g.cpb / g.lpc;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_run_iteration_blocks(muca_run *r, int64_t sweeps, uint64_t *d_blocks, void *stream)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (r->g.model == kPolymer)
        return muca_fail(MUCA_E_ARG, "per-block histograms: lattice runs only");
    if (!d_blocks)
        return muca_fail(MUCA_E_ARG, "null block histograms");
    if (sweeps < 1)
        return muca_fail(MUCA_E_ARG, "sweeps must be >= 1");
    rc = muca_use_stream(r, (hipStream_t)stream);
    if (rc)
        return rc;
    rc = muca_enqueue_sweeps(r, sweeps, true, r->stream, nullptr, (unsigned long long *)d_blocks);
    if (rc)
        return rc;
    r->pending += sweeps;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_thermalize(muca_run *r, int64_t sweeps, void *stream)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (sweeps < 0)
        return muca_fail(MUCA_E_ARG, "sweeps must be >= 0");
    rc = muca_use_stream(r, (hipStream_t)stream);
    if (rc)
        return rc;
    return sweeps ? muca_enqueue_sweeps(r, sweeps, false, r->stream) : MUCA_OK;
}
MUCA_ABI_CATCH

int muca_finish_iteration(muca_run *r, const uint64_t *H, uint64_t accepted, muca_iter_stats *st)
{
    const Geometry &g = r->g;
    const int B = g.n_bins;
    r->lnW_last = r->lnW;
    r->H_last.assign(H, H + B);
    muca_iter_stats s{};
    s.iteration = r->iteration;
    s.sweeps = r->pending;
    // attempts per chain and sweep: every site (bead); the polymer's full
    // move set adds a rotation per bead and one double bridging
    const double per_sweep = g.model == kPolymer && r->cfg.moves ? 2.0 * g.n_sites + 1.0 : (double)g.n_sites;
    s.accept_rate = (double)accepted / ((double)r->pending * (double)r->cfg.n_chains * per_sweep);
    s.lo_visited = -1;
    s.hi_visited = -1;
    for (int b = 0; b < B; ++b) {
        s.samples += (int64_t)H[b];
        if (H[b]) {
            if (s.lo_visited < 0)
                s.lo_visited = b;
            s.hi_visited = b;
        }
    }
    if (g.model == kPolymer) {
        for (int b = 0; b < B; ++b)
            if (H[b])
                r->mask[b] = 1; // flatness over the bins visited so far
        s.flatness = muca_flatness(B, r->mask.data(), H);
        std::vector<uint8_t> all(B, 1);
        muca_recursion(B, all.data(), H, r->lnR.data(), r->P.data(), r->lnW.data());
    } else {
        s.flatness = muca_flatness(B, r->mask.data(), H);
        muca_recursion(B, r->mask.data(), H, r->lnR.data(), r->P.data(), r->lnW.data());
    }
    s.flat = s.flatness > r->cfg.flat_threshold ? 1 : 0;
    const double now = wall_seconds();
    muca_log_iteration(r, s, now - r->t_last, (double)r->pending * (double)r->cfg.n_chains * per_sweep);
    r->t_last = now;
    r->iteration += 1;
    r->pending = 0;
    r->have_last = true;
    if (st)
        *st = s;
    // every merge path has waited for the work queued before the read-back,
    // the last upload from the pinned threshold mirror included
    return muca_rebuild_thresholds(r);
}

extern "C" int muca_merge_begin(muca_run *r)
try {
    RoctxRange range("muca_merge_begin");
    int rc = check_run(r);
    if (rc)
        return rc;
    if (r->pending <= 0)
        return muca_fail(MUCA_E_STATE, "merge without sweeps since the last merge");
    if (r->h_hist) {
        // the histogram and the accepted-move count behind it are written to
        // pinned host memory and cleared by one kernel queued behind the
        // sweeps; the event behind it is all that muca_merge_finish waits for
        if (!r->merge_ev)
            HIP_OR_POISON(r, hipEventCreateWithFlags(&r->merge_ev, hipEventDisableTiming));
        HIP_OR_POISON(r, launch_drain_u64(r->d_hist, r->h_hist_dev, r->g.n_bins + 1, r->stream));
        HIP_OR_POISON(r, hipEventRecord(r->merge_ev, r->stream));
    }
    r->merge_begun = true;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_merge_finish(muca_run *r, muca_iter_stats *st)
try {
    RoctxRange range("muca_merge_finish");
    if (!r)
        return muca_fail(MUCA_E_ARG, "null run");
    if (r->poisoned)
        return muca_fail(MUCA_E_STATE, "run poisoned by an earlier HIP error");
    if (!r->merge_begun)
        return muca_fail(MUCA_E_STATE, "muca_merge_finish without muca_merge_begin");
    r->merge_begun = false;
    const int B = r->g.n_bins;
    if (r->h_hist) {
        // the read-back is behind the sweeps and behind the last threshold
        // upload, so the pinned mirror may be rewritten once it has completed
        HIP_OR_POISON(r, hipEventSynchronize(r->merge_ev));
        return muca_finish_iteration(r, r->h_hist, r->h_hist[B], st);
    }
    std::vector<uint64_t> H(B + 1); // the histogram and the accepted-move count behind it
    HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    HIP_OR_POISON(r, hipMemcpy(H.data(), r->d_hist, (size_t)(B + 1) * 8u, hipMemcpyDeviceToHost));
    HIP_OR_POISON(r, launch_fill_u64(r->d_hist, B + 1, r->stream));
    return muca_finish_iteration(r, H.data(), H[B], st);
}
MUCA_ABI_CATCH

extern "C" int muca_merge_update(muca_run *r, muca_iter_stats *st)
try {
    int rc = muca_merge_begin(r);
    return rc ? rc : muca_merge_finish(r, st);
}
MUCA_ABI_CATCH

extern "C" int muca_get_pending_hist(const muca_run *r_, uint64_t *h, int64_t n)
try {
    muca_run *r = const_cast<muca_run *>(r_);
    int rc = check_run(r);
    if (rc)
        return rc;
    if (!h || n != r->g.n_bins)
        return muca_fail(MUCA_E_ARG, "need a host array of n_bins = %d entries", r->g.n_bins);
    if (r->pending <= 0)
        return muca_fail(MUCA_E_STATE, "no sweeps since the last merge");
    HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    HIP_OR_POISON(r, hipMemcpy(h, r->d_hist, (size_t)n * 8u, hipMemcpyDeviceToHost));
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_merge_update_hist(muca_run *r, const uint64_t *h, int64_t n, muca_iter_stats *st)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (!h || n != r->g.n_bins)
        return muca_fail(MUCA_E_ARG, "need a merged histogram of n_bins = %d entries", r->g.n_bins);
    if (r->pending <= 0)
        return muca_fail(MUCA_E_STATE, "merge_update without sweeps since the last merge");
    uint64_t accepted = 0;
    HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    HIP_OR_POISON(r, hipMemcpy(&accepted, r->d_hist + r->g.n_bins, 8u, hipMemcpyDeviceToHost));
    HIP_OR_POISON(r, launch_fill_u64(r->d_hist, r->g.n_bins + 1, r->stream));
    return muca_finish_iteration(r, h, accepted, st);
}
MUCA_ABI_CATCH

extern "C" int muca_reweight(const muca_run *r, const double *betas, int32_t n, double *out)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (!r->have_last)
        return muca_fail(MUCA_E_STATE, "no merged histogram yet");
    if (n < 1 || !out)
        return muca_fail(MUCA_E_ARG, "need n >= 1 and an output array");
    const Geometry &g = r->g;
    if (g.model != kMuma && !betas)
        return muca_fail(MUCA_E_ARG, "null betas");
    std::vector<double> val(g.n_bins);
    for (int b = 0; b < g.n_bins; ++b) {
        if (g.model == kIsing || g.model == kMuma)
            val[b] = (double)(r->cfg.lo + g.step * b);
        else if (g.model == kPotts)
            val[b] = (double)(r->cfg.lo + b) - 2.0 * g.n_sites;
        else
            val[b] = r->cfg.x_lo + ((r->cfg.x_hi - r->cfg.x_lo) / (double)g.n_bins) * ((double)b + 0.5);
    }
    for (int k = 0; k < n; ++k) {
        const bool muma = g.model == kMuma;
        const double beta = muma ? r->cfg.beta : betas[k];
        muca_reweight_bins(g.n_bins, r->H_last.data(), r->lnW_last.data(), val.data(), g.n_sites, muma,
                           beta, out + 4 * k);
    }
    return MUCA_OK;
}
MUCA_ABI_CATCH


extern "C" int muca_reweight_em(const muca_run *r, const uint64_t *h_em, int64_t n_em, const double *betas,
                                int32_t n, double *out)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    const Geometry &g = r->g;
    if (g.model != kMuma)
        return muca_fail(MUCA_E_ARG, "joint (E, M) histogram: multimagnetic runs only");
    if (!r->have_last)
        return muca_fail(MUCA_E_STATE, "no merged histogram yet");
    const int NE = g.n_sites + 1, B = g.n_bins;
    if (!h_em || n_em != (int64_t)NE * B)
        return muca_fail(MUCA_E_ARG, "joint histogram of %lld entries, expected %d x %d", (long long)n_em, NE, B);
    if (n < 1 || !betas || !out)
        return muca_fail(MUCA_E_ARG, "need n >= 1, betas and an output array");
    for (int k = 0; k < n; ++k)
        muca_reweight_joint(NE, B, h_em, r->lnW_last.data(), r->cfg.lo, g.step, g.n_sites, r->cfg.beta, betas[k],
                       out + 6 * k);
    return MUCA_OK;
}
MUCA_ABI_CATCH

// Values of the binned quantity per bin (energy; MUMA: magnetisation; Potts
// E_unsat - 2N; polymer bin centres), as muca_reweight reports them.
static std::vector<double> bin_values(const muca_run *r)
{
    const Geometry &g = r->g;
    std::vector<double> val(g.n_bins);
    for (int b = 0; b < g.n_bins; ++b) {
        if (g.model == kIsing || g.model == kMuma)
            val[b] = (double)(r->cfg.lo + g.step * b);
        else if (g.model == kPotts)
            val[b] = (double)(r->cfg.lo + b) - 2.0 * g.n_sites;
        else
            val[b] = r->cfg.x_lo + ((r->cfg.x_hi - r->cfg.x_lo) / (double)g.n_bins) * ((double)b + 0.5);
    }
    return val;
}

extern "C" int muca_reweight_jackknife(const muca_run *r, const uint64_t *h_blocks, int32_t n_blocks,
                                       const double *betas, int32_t n, double *out, double *err)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (!r->have_last)
        return muca_fail(MUCA_E_STATE, "no merged histogram yet");
    const Geometry &g = r->g;
    const bool muma = g.model == kMuma;
    if (!h_blocks || n_blocks < 1 || n < 1 || !out || !err || (!muma && !betas))
        return muca_fail(MUCA_E_ARG, "need block histograms, n >= 1, betas and output arrays");
    const int B = g.n_bins;
    // the blocks that saw any chain, and their sum
    std::vector<int> used;
    std::vector<uint64_t> H(B, 0), Hk(B);
    for (int k = 0; k < n_blocks; ++k) {
        uint64_t tot = 0;
        for (int b = 0; b < B; ++b) {
            H[b] += h_blocks[(size_t)k * B + b];
            tot += h_blocks[(size_t)k * B + b];
        }
        if (tot)
            used.push_back(k);
    }
    if (used.size() < 2)
        return muca_fail(MUCA_E_ARG, "jackknife needs at least two non-empty blocks");
    const std::vector<double> val = bin_values(r);
    const double m = (double)used.size();
    std::vector<double> v(4 * used.size());
    for (int q = 0; q < n; ++q) {
        const double beta = muma ? r->cfg.beta : betas[q];
        muca_reweight_bins(B, H.data(), r->lnW_last.data(), val.data(), g.n_sites, muma, beta, out + 4 * q);
        for (size_t u = 0; u < used.size(); ++u) { // leave block used[u] out
            const uint64_t *hk = h_blocks + (size_t)used[u] * B;
            for (int b = 0; b < B; ++b)
                Hk[b] = H[b] - hk[b];
            muca_reweight_bins(B, Hk.data(), r->lnW_last.data(), val.data(), g.n_sites, muma, beta,
                               v.data() + 4 * u);
        }
        for (int c = 0; c < 4; ++c) {
            double mean = 0.0;
            for (size_t u = 0; u < used.size(); ++u)
                mean += v[4 * u + c];
            mean /= m;
            double ss = 0.0;
            for (size_t u = 0; u < used.size(); ++u) {
                const double d = v[4 * u + c] - mean;
                ss += d * d;
            }
            err[4 * q + c] = std::sqrt((m - 1.0) / m * ss);
        }
    }
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_sizes(const muca_run *r, int32_t *n_bins, int32_t *n_cols, int32_t *n_sites)
try {
    if (!r)
        return muca_fail(MUCA_E_ARG, "null run");
    if (n_bins)
        *n_bins = r->g.n_bins;
    if (n_cols)
        *n_cols = r->g.n_cols;
    if (n_sites)
        *n_sites = r->g.n_sites;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_get_lnw(const muca_run *r, double *h, int32_t n)
try {
    if (!r || !h || n != r->g.n_bins)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    std::memcpy(h, r->lnW.data(), (size_t)n * 8u);
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_get_last_hist(const muca_run *r, uint64_t *h, int32_t n)
try {
    if (!r || !h || n != r->g.n_bins)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    std::memcpy(h, r->H_last.data(), (size_t)n * 8u);
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_get_thresholds(const muca_run *r, uint32_t *h, int64_t count)
try {
    if (!r || !h || count != (int64_t)r->T.size())
        return muca_fail(MUCA_E_ARG, "bad arguments");
    std::memcpy(h, r->T.data(), (size_t)count * 4u);
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_set_lnw(muca_run *r, const double *h, int32_t n)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (!h || n != r->g.n_bins)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    r->lnW.assign(h, h + n);
    return muca_rebuild_thresholds(r);
}
MUCA_ABI_CATCH

extern "C" int muca_set_thresholds(muca_run *r, const uint32_t *h, int64_t count)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (!h || count != (int64_t)r->T.size())
        return muca_fail(MUCA_E_ARG, "bad arguments");
    HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    std::memcpy(r->T.data(), h, (size_t)count * 4u);
    return muca_upload_thresholds(r);
}
MUCA_ABI_CATCH

extern "C" int muca_get_chain_state(const muca_run *r_, int32_t chain0, int32_t count, void *state,
                                    int32_t *bins, double *energy)
try {
    muca_run *r = const_cast<muca_run *>(r_);
    int rc = check_run(r);
    if (rc)
        return rc;
    if (chain0 < 0 || count < 0 || chain0 + count > r->cfg.n_chains)
        return muca_fail(MUCA_E_ARG, "chain range [%d, %d) outside [0, %d)", chain0, chain0 + count,
                         r->cfg.n_chains);
    if (r->g.model == kPolymer)
        return muca_polymer_state(r, chain0, count, (float *)state, bins, energy);
    const Geometry &g = r->g;
    HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    if (bins && count)
        HIP_OR_POISON(r, hipMemcpy(bins, r->d_bins + chain0, (size_t)count * 4u, hipMemcpyDeviceToHost));
    if (state && count) {
        const int rows = g.L * g.wpr;
        std::vector<uint32_t> w((size_t)rows * count);
        HIP_OR_POISON(r, hipMemcpy2D(w.data(), (size_t)count * 4u, r->d_words + chain0, (size_t)g.c_pad * 4u,
                                     (size_t)count * 4u, rows, hipMemcpyDeviceToHost));
        int8_t *out = (int8_t *)state;
        const int spw = g.layout == kLayoutBit ? 32 : 4;
        for (int k = 0; k < count; ++k) {
            for (int y = 0; y < g.L; ++y) {
                for (int x = 0; x < g.L; ++x) {
                    const uint32_t word = w[((size_t)y * g.wpr + x / spw) * count + k];
                    int8_t v;
                    if (g.layout == kLayoutBit)
                        v = ((word >> (x % spw)) & 1u) ? 1 : -1;
                    else
                        v = (int8_t)((word >> ((x % spw) * 8)) & 0xFFu);
                    out[(size_t)k * g.n_sites + y * g.L + x] = v;
                }
            }
        }
    }
    if (energy && count) {
        std::vector<int32_t> b(count);
        HIP_OR_POISON(r, hipMemcpy(b.data(), r->d_bins + chain0, (size_t)count * 4u, hipMemcpyDeviceToHost));
        for (int k = 0; k < count; ++k)
            energy[k] = (double)(r->cfg.lo + g.step * b[k]);
    }
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" void muca_free(muca_run *r)
{
    if (!r)
        return;
    if (!r->poisoned && r->stream)
        (void)hipStreamSynchronize(r->stream);
    delete r;
}

// ---------------------------------------------------------------------------
// Checkpoint / restore: host state plus a byte copy of the device workspace.
// ---------------------------------------------------------------------------
namespace {
const uint32_t kCkptMagic = 0x4d554341u; // "MUCA"

template <class V>
void put_vec(std::vector<uint8_t> &o, const V &v)
{
    const uint64_t n = v.size();
    const uint8_t *p = (const uint8_t *)&n;
    o.insert(o.end(), p, p + 8);
    const uint8_t *d = (const uint8_t *)v.data();
    o.insert(o.end(), d, d + n * sizeof(typename V::value_type));
}

template <class T>
void put_pod(std::vector<uint8_t> &o, const T &v)
{
    const uint8_t *p = (const uint8_t *)&v;
    o.insert(o.end(), p, p + sizeof(T));
}

struct Reader {
    const uint8_t *p;
    uint64_t left;
    template <class T>
    bool pod(T &v)
    {
        if (left < sizeof(T))
            return false;
        std::memcpy(&v, p, sizeof(T));
        p += sizeof(T);
        left -= sizeof(T);
        return true;
    }
    template <class T>
    bool vec(std::vector<T> &v, uint64_t expect)
    {
        uint64_t n;
        if (!pod(n) || n != expect || left < n * sizeof(T))
            return false;
        v.resize(n);
        std::memcpy(v.data(), p, n * sizeof(T));
        p += n * sizeof(T);
        left -= n * sizeof(T);
        return true;
    }
};
} // namespace

extern "C" int muca_checkpoint(const muca_run *r_, void *h_buf, uint64_t *bytes)
try {
    muca_run *r = const_cast<muca_run *>(r_);
    int rc = check_run(r);
    if (rc)
        return rc;
    if (!bytes)
        return muca_fail(MUCA_E_ARG, "null bytes");
    std::vector<uint8_t> o;
    put_pod(o, kCkptMagic);
    put_pod(o, r->cfg);
    put_pod(o, r->sweep);
    put_pod(o, r->iteration);
    put_pod(o, r->pending);
    put_pod(o, (int32_t)r->have_last);
    put_vec(o, r->lnW);
    put_vec(o, r->lnR);
    put_vec(o, r->P);
    put_vec(o, r->mask);
    put_vec(o, r->T);
    put_vec(o, r->H_last);
    put_vec(o, r->lnW_last);
    const uint64_t ws = r->g.ws_bytes;
    const uint64_t total = o.size() + 8 + ws;
    if (!h_buf) {
        *bytes = total;
        return MUCA_OK;
    }
    if (*bytes < total)
        return muca_fail(MUCA_E_NOMEM, "checkpoint buffer of %llu bytes, need %llu",
                         (unsigned long long)*bytes, (unsigned long long)total);
    HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    uint8_t *dst = (uint8_t *)h_buf;
    std::memcpy(dst, o.data(), o.size());
    std::memcpy(dst + o.size(), &ws, 8);
    HIP_OR_POISON(r, hipMemcpy(dst + o.size() + 8, r->ws, ws, hipMemcpyDeviceToHost));
    *bytes = total;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" int muca_restore(muca_run *r, const void *h_buf, uint64_t bytes)
try {
    int rc = check_run(r);
    if (rc)
        return rc;
    if (!h_buf)
        return muca_fail(MUCA_E_ARG, "null buffer");
    Reader rd{(const uint8_t *)h_buf, bytes};
    uint32_t magic;
    muca_config cfg;
    if (!rd.pod(magic) || magic != kCkptMagic || !rd.pod(cfg))
        return muca_fail(MUCA_E_ARG, "not a checkpoint");
    if (std::memcmp(&cfg, &r->cfg, sizeof cfg) != 0)
        return muca_fail(MUCA_E_ARG, "checkpoint of a different configuration");
    uint32_t sweep;
    int64_t iteration, pending;
    int32_t have_last;
    std::vector<double> lnW, lnR, P, lnW_last;
    std::vector<uint8_t> mask;
    std::vector<uint32_t> T;
    std::vector<uint64_t> H_last;
    const uint64_t B = r->g.n_bins;
    bool ok = rd.pod(sweep) && rd.pod(iteration) && rd.pod(pending) && rd.pod(have_last) &&
              rd.vec(lnW, B) && rd.vec(lnR, B) && rd.vec(P, B) && rd.vec(mask, r->mask.size()) &&
              rd.vec(T, r->T.size()) && rd.vec(H_last, B) && rd.vec(lnW_last, B);
    uint64_t ws = 0;
    ok = ok && rd.pod(ws) && ws == r->g.ws_bytes && rd.left == ws;
    if (!ok)
        return muca_fail(MUCA_E_ARG, "truncated or mismatched checkpoint");
    HIP_OR_POISON(r, hipStreamSynchronize(r->stream));
    HIP_OR_POISON(r, hipMemcpy(r->ws, rd.p, ws, hipMemcpyHostToDevice));
    r->sweep = sweep;
    r->iteration = iteration;
    r->pending = pending;
    r->have_last = have_last != 0;
    r->lnW = lnW;
    r->lnR = lnR;
    r->P = P;
    r->mask = mask;
    std::copy(T.begin(), T.end(), r->T.begin());
    r->H_last = H_last;
    r->lnW_last = lnW_last;
    return MUCA_OK;
}
MUCA_ABI_CATCH
