// batch.hip -- one persistent launch advancing many multicanonical runs
// (mixed models, lattice sizes, q, ensembles) by one iteration each.
//
// The runs' chains are cut into work items of 256 / LPC chains (one
// 256-thread workgroup each).  Items are ordered longest first (sites x
// sweeps x per-site cost) and handed out by an atomic counter to a grid
// sized to fill the chip once; a workgroup stages the item's threshold
// table in LDS when it fits, runs the item's sweeps with the same sweep
// code as the plain launch, adds its LDS histogram to the run's histogram,
// and takes the next item until the queue is empty.  Chains never interact,
// so every run's histogram and chains are bit-identical to a plain launch.
//
// The host side captures [descriptor upload, counter reset, persistent
// kernel] once in a hipGraph and relaunches it every round after rewriting
// the pinned descriptor buffer (sweep counters and sweeps change per round).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "lattice_impl.h"
#include "runtime_internal.h"

namespace muca {

struct BatchDesc {
    LatticeArgs a;
    int32_t variant;
    int32_t pad[3];
};

struct BatchItem {
    int32_t inst;
    int32_t c_first;
};

struct BatchHeader {
    int32_t n_items;
    int32_t pad[63]; // keep the descriptors 256-byte aligned
};

constexpr int kBatchLs[6] = {8, 16, 24, 32, 48, 64};
constexpr int kNumVariants = 5 * 6 * 2 * 2; // {Ising bit, Ising byte, MUMA bit, MUMA byte, Potts} x L x LDS x LPC

__host__ __device__ constexpr int variant_index(int kind, int li, int tlds, int lpc16)
{
    return ((kind * 6 + li) * 2 + tlds) * 2 + lpc16;
}

// The descriptor's values are the same for the whole workgroup, but inside a
// non-inlined function the compiler cannot know it: read them through
// readfirstlane, so that the sweep loop, the key schedule and the addresses
// stay on the scalar unit as in the plain kernel.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
template <class T>
__device__ __forceinline__ T *uni(T *p)
{
    const uint64_t v = (uint64_t)p;
    return (T *)(((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v));
}

template <int V>
__device__ __noinline__ void run_variant(const BatchDesc *d, int c_first)
{
    extern __shared__ uint32_t smem[];
    constexpr int lpc16 = V % 2;
    constexpr bool TLDS = (V / 2) % 2;
    constexpr int li = (V / 4) % 6;
    constexpr int kind = V / 24;
    constexpr int L = kBatchLs[li];
    constexpr int MODEL = kind <= 1 ? kIsing : (kind <= 3 ? kMuma : kPotts);
    constexpr int LAYOUT = (kind == 0 || kind == 2) ? kLayoutBit : kLayoutByte;
    constexpr int LPC = lpc16 ? 16 : 4;
    const LatticeArgs v = d->a;
    LatticeArgs a;
    a.words = uni(v.words);
    a.bins = uni(v.bins);
    a.thresholds = uni(v.thresholds);
    a.hist = uni(v.hist);
    a.k0 = uni(v.k0), a.k1 = uni(v.k1), a.g0 = uni(v.g0);
    a.n_sweeps = uni(v.n_sweeps), a.n_chains = uni(v.n_chains), a.c_pad = uni(v.c_pad);
    a.n_bins = uni(v.n_bins), a.q = uni(v.q), a.record = uni(v.record), a.table_in_lds = uni(v.table_in_lds);
    a.chain0 = uni(v.chain0);
    a.em = uni(v.em);
    a.accepts = uni(v.accepts);
    a.hist_blocks = uni(v.hist_blocks);
    sweep_block<MODEL, L, LAYOUT, TLDS, LPC>(a, uni(c_first), smem);
}

template <int... V>
__device__ __forceinline__ void dispatch(int v, const BatchDesc *d, int c_first, std::integer_sequence<int, V...>)
{
    (void)((v == V ? (run_variant<V>(d, c_first), true) : false) || ...);
}

__global__ __launch_bounds__(256) void batch_persistent(const BatchHeader *hdr, int *counter,
                                                        const BatchDesc *descs, const BatchItem *items)
{
    __shared__ int s_item;
    const int n = hdr->n_items;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n)
            break; // uniform: every workgroup leaves once the queue is empty
        const BatchItem item = items[it];
        const BatchDesc *d = descs + item.inst;
        dispatch(d->variant, d, item.c_first, std::make_integer_sequence<int, kNumVariants>{});
        __syncthreads(); // the next item reuses the LDS
    }
}

__global__ void batch_reset(int *counter) { *counter = 0; }

} // namespace muca

using namespace muca;

// One of the two staging areas of a batch handle: rounds alternate between
// them, so a round's descriptors are written while the previous round may
// still run; `done` is recorded behind the kernel that read the area.
struct BatchSlot {
    uint8_t *h_buf = nullptr; // pinned staging of header + descriptors + items
    int *d_counter = nullptr;
    BatchHeader *d_hdr = nullptr;
    BatchDesc *d_desc = nullptr;
    BatchItem *d_items = nullptr;
    hipEvent_t done = nullptr;
    bool used = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
    int graph_grid = 0;
    size_t graph_lds = 0;
};

struct muca_batch {
    int max_runs = 0, max_items = 0, lpc = 4;
    bool use_graph = false;
    uint8_t *d_ws = nullptr;
    size_t stage_bytes = 0;
    BatchSlot slot[2];
    int next = 0;
    int n_cus = 0, lds_limit = 0;
    bool poisoned = false;
};

static size_t a256(size_t x) { return (x + 255u) & ~(size_t)255u; }

static size_t stage_size(int max_runs, int max_items)
{
    return a256(sizeof(BatchHeader)) + a256((size_t)max_runs * sizeof(BatchDesc)) +
           a256((size_t)max_items * sizeof(BatchItem));
}

// Where a round's header, descriptors and work items sit, for a staging area
// sized for (max_runs, max_items): [header | descriptors | items].
struct StageLayout {
    size_t desc_off, items_off, bytes;
};

static StageLayout stage_layout(int max_runs, int max_items)
{
    StageLayout l;
    l.desc_off = a256(sizeof(BatchHeader));
    l.items_off = l.desc_off + a256((size_t)max_runs * sizeof(BatchDesc));
    l.bytes = l.items_off + a256((size_t)max_items * sizeof(BatchItem));
    return l;
}

extern "C" int muca_batch_workspace_bytes(int32_t max_runs, int32_t max_items, uint64_t *bytes)
try {
    if (max_runs < 1 || max_items < 1 || !bytes)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    *bytes = 2 * (256 + stage_size(max_runs, max_items)); // two staging areas
    return MUCA_OK;
}
MUCA_ABI_CATCH

static void drop_graph(BatchSlot &sl)
{
    if (sl.exec)
        (void)hipGraphExecDestroy(sl.exec);
    if (sl.graph)
        (void)hipGraphDestroy(sl.graph);
    sl.exec = nullptr;
    sl.graph = nullptr;
}

static void release(muca_batch *b)
{
    for (BatchSlot &sl : b->slot) {
        if (sl.used && sl.done)
            (void)hipEventSynchronize(sl.done); // the pinned staging may still be read
        drop_graph(sl);
        if (sl.done)
            (void)hipEventDestroy(sl.done);
        if (sl.h_buf)
            (void)hipHostFree(sl.h_buf);
    }
    delete b;
}

extern "C" int muca_batch_create(int32_t max_runs, int32_t max_items, int32_t lanes_per_chain, int32_t use_graph,
                                 void *d_ws, uint64_t ws_bytes, muca_batch **out)
try {
    if (!out)
        return muca_fail(MUCA_E_ARG, "null out");
    *out = nullptr;
    uint64_t need = 0;
    int rc = muca_batch_workspace_bytes(max_runs, max_items, &need);
    if (rc)
        return rc;
    if (!d_ws || ((uintptr_t)d_ws & 255u))
        return muca_fail(MUCA_E_ARG, "batch workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < need)
        return muca_fail(MUCA_E_NOMEM, "batch workspace of %llu bytes, need %llu", (unsigned long long)ws_bytes,
                         (unsigned long long)need);
    if (lanes_per_chain != 0 && lanes_per_chain != 4 && lanes_per_chain != 16)
        return muca_fail(MUCA_E_ARG, "batched launches use 4 or 16 lanes per chain (0: chosen per run)");
    muca_batch *b = new muca_batch();
    b->max_runs = max_runs;
    b->max_items = max_items;
    b->lpc = lanes_per_chain;
    b->use_graph = use_graph != 0;
    b->d_ws = (uint8_t *)d_ws;
    b->stage_bytes = stage_size(max_runs, max_items);
    const StageLayout sl = stage_layout(max_runs, max_items);
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        BatchSlot &t = b->slot[k];
        uint8_t *p = b->d_ws + (size_t)k * (256 + b->stage_bytes);
        t.d_counter = (int *)p;
        t.d_hdr = (BatchHeader *)(p + 256);
        t.d_desc = (BatchDesc *)(p + 256 + sl.desc_off);
        t.d_items = (BatchItem *)(p + 256 + sl.items_off);
        e = hipHostMalloc((void **)&t.h_buf, b->stage_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&t.done, hipEventDisableTiming);
    }
    int dev = 0;
    if (e == hipSuccess)
        e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&b->n_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&b->lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) {
        release(b);
        return muca_fail(MUCA_E_HIP, "batch create: %s", hipGetErrorString(e));
    }
    *out = b;
    return MUCA_OK;
}
MUCA_ABI_CATCH

extern "C" void muca_batch_free(muca_batch *b)
{
    if (b)
        release(b);
}

static int kind_of(const muca_run *r)
{
    const int m = r->g.model, lay = r->g.layout;
    if (m == kIsing)
        return lay == kLayoutBit ? 0 : 1;
    if (m == kMuma)
        return lay == kLayoutBit ? 2 : 3;
    if (m == kPotts)
        return 4;
    return -1;
}

static int l_index(int L)
{
    for (int i = 0; i < 6; ++i)
        if (kBatchLs[i] == L)
            return i;
    return -1;
}

struct RoundPlan {
    int grid = 0;
    size_t lds = 0;
    int n_items = 0;
};

// The descriptor of run r for `sweeps` sweeps from its current sweep counter.
static void fill_desc(BatchDesc &d, const muca_run *r, int64_t sweeps, bool tlds, int lpc)
{
    std::memset(&d, 0, sizeof d);
    d.a.words = r->d_words;
    d.a.bins = r->d_bins;
    d.a.thresholds = r->d_table;
    d.a.hist = r->d_hist;
    d.a.k0 = (uint32_t)(r->cfg.seed & 0xffffffffu);
    d.a.k1 = (uint32_t)(r->cfg.seed >> 32);
    d.a.g0 = r->sweep;
    d.a.n_sweeps = (int32_t)sweeps;
    d.a.n_chains = r->cfg.n_chains;
    d.a.c_pad = r->g.c_pad;
    d.a.n_bins = r->g.n_bins;
    d.a.q = r->cfg.q;
    d.a.record = 1;
    d.a.table_in_lds = tlds ? 1 : 0;
    d.a.chain0 = r->cfg.chain0;
    d.a.accepts = r->d_hist + r->g.n_bins;
    d.variant = variant_index(kind_of(r), l_index(r->g.L), tlds ? 1 : 0, lpc == 16 ? 1 : 0);
}

// Lanes per chain, table placement and item cost of every run of a round,
// from the runs' measured item times (muca_batch_tune).  The chip is taken
// as n_cus slots, each running one work item at a time, and the round's
// length is estimated as max(longest item, total item time / slots): every
// run starts at the choice of least total item time, then the run with the
// longest item moves to the choice with the shorter item while that lowers
// the estimate.  Returns false if some run is not tuned.
static bool plan_tuned(muca_run *const *runs, int n, const int64_t *sweeps, int n_cus, int max_items, int *lpc,
                       int *tlds, double *cost)
{
    for (int i = 0; i < n; ++i)
        if (!runs[i]->batch_tuned)
            return false;
    auto items_of = [&](int i, int o) { return (double)((runs[i]->cfg.n_chains + 256 / (o ? 16 : 4) - 1) /
                                                        (256 / (o ? 16 : 4))); };
    // per-item time of option o (0: 4 lanes, 1: 16 lanes) at the faster table placement
    auto item_t = [&](int i, int o, int *tl) {
        const double g = runs[i]->batch_us[o][0], l = runs[i]->batch_us[o][1];
        double best = -1.0;
        int t = 0;
        if (g >= 0.0)
            best = g, t = 0;
        if (l >= 0.0 && (best < 0.0 || l < best))
            best = l, t = 1;
        if (tl)
            *tl = t;
        return best < 0.0 ? -1.0 : best * (double)sweeps[i];
    };
    double total = 0.0, items = 0.0;
    for (int i = 0; i < n; ++i) {
        const double w4 = item_t(i, 0, nullptr), w16 = item_t(i, 1, nullptr);
        int o = 0;
        if (w4 < 0.0 || (w16 >= 0.0 && items_of(i, 1) * w16 < items_of(i, 0) * w4))
            o = 1;
        if (item_t(i, o, nullptr) < 0.0)
            return false;
        lpc[i] = o ? 16 : 4;
        total += items_of(i, o) * item_t(i, o, nullptr);
        items += items_of(i, o);
    }
    auto estimate = [&](double tot) {
        double longest = 0.0;
        for (int i = 0; i < n; ++i)
            longest = std::max(longest, item_t(i, lpc[i] == 16, nullptr));
        return std::max(longest, tot / (double)n_cus);
    };
    double est = estimate(total);
    for (int step = 0; step < n; ++step) {
        int k = 0;
        for (int i = 1; i < n; ++i)
            if (item_t(i, lpc[i] == 16, nullptr) > item_t(k, lpc[k] == 16, nullptr))
                k = i;
        const int o = lpc[k] == 16, alt = 1 - o;
        const double now = item_t(k, o, nullptr), other = item_t(k, alt, nullptr);
        if (other < 0.0 || other >= now)
            break;
        const double tot2 = total - items_of(k, o) * now + items_of(k, alt) * other;
        const double items2 = items - items_of(k, o) + items_of(k, alt);
        lpc[k] = alt ? 16 : 4;
        const double est2 = estimate(tot2);
        if (est2 >= est || items2 > (double)max_items) {
            lpc[k] = o ? 16 : 4;
            break;
        }
        est = est2, total = tot2, items = items2;
    }
    for (int i = 0; i < n; ++i)
        cost[i] = item_t(i, lpc[i] == 16, &tlds[i]);
    return true;
}

// Plans one batched round: checks the runs, moves each to stream s, chooses
// lanes per chain (lpc_fixed, or per run when 0: from the measured item
// times when every run is tuned, else by the rule below) and the table
// placement, and writes the header, one descriptor per run and the work
// items (longest first) into the host staging area `stage`.  `lpc`, `tlds`,
// `order` and `cost` are caller-owned work arrays of n entries; nothing is
// allocated here, so the entry point that must not allocate can use it.
// Returns a muca_status.
static int plan_round(muca_run *const *runs, int n, const int64_t *sweeps, int lpc_fixed, int max_runs, int max_items,
                      int n_cus, int lds_limit, uint8_t *stage, int *lpc, int *tlds, int *order, double *cost,
                      hipStream_t s, RoundPlan *out)
{
    if (n > max_runs)
        return muca_fail(MUCA_E_ARG, "%d runs exceed the batch capacity %d", n, max_runs);
    for (int i = 0; i < n; ++i) {
        muca_run *r = runs[i];
        if (!r || r->poisoned)
            return muca_fail(MUCA_E_STATE, "run %d is null or poisoned", i);
        if (r->merge_begun)
            return muca_fail(MUCA_E_STATE, "run %d: a merge was begun and not finished", i);
        if (kind_of(r) < 0 || l_index(r->g.L) < 0)
            return muca_fail(MUCA_E_ARG, "run %d (model %d, L %d) has no batched variant", i, r->g.model, r->g.L);
        if (sweeps[i] < 1 || sweeps[i] > (int64_t)INT32_MAX)
            return muca_fail(MUCA_E_ARG, "run %d: sweeps %lld out of range", i, (long long)sweeps[i]);
        for (int k = 0; k < i; ++k)
            if (runs[k] == r)
                return muca_fail(MUCA_E_ARG, "run %d appears twice", i);
    }
    const size_t lds_budget = (size_t)std::min(lds_limit, 160 * 1024) - 256; // static LDS of the kernel
    auto items_of = [&](int i, int l) { return (long)((runs[i]->cfg.n_chains + 256 / l - 1) / (256 / l)); };
    // untuned rule: the per-site cost of Potts counted twice that of Ising
    auto work = [&](int i) {
        return (runs[i]->g.model == kPotts ? 2.0 : 1.0) * (double)runs[i]->g.n_sites * (double)sweeps[i];
    };
    for (int i = 0; i < n; ++i) {
        lpc[i] = lpc_fixed ? lpc_fixed : 4;
        tlds[i] = runs[i]->g.table_in_lds && runs[i]->g.lds_bytes <= lds_budget;
        cost[i] = work(i);
    }
    if (lpc_fixed == 0 && plan_tuned(runs, n, sweeps, n_cus, max_items, lpc, tlds, cost)) {
        for (int i = 0; i < n; ++i) // a measured LDS placement must still fit this device
            tlds[i] = tlds[i] && runs[i]->g.table_in_lds && runs[i]->g.lds_bytes <= lds_budget;
    } else if (lpc_fixed == 0) {
        // every run starts at 4 lanes per chain; runs are raised to 16 in
        // order of decreasing per-chain work (the critical path of the
        // launch) while all lanes still fit one resident 256-thread
        // workgroup per CU and the item list its capacity
        long lanes = 0, n_items = 0;
        for (int i = 0; i < n; ++i) {
            order[i] = i;
            lanes += items_of(i, 4) * 256;
            n_items += items_of(i, 4);
        }
        std::sort(order, order + n, [&](int x, int y) {
            const double wx = work(x), wy = work(y);
            return wx != wy ? wx > wy : x < y;
        });
        const long cap = (long)n_cus * 256;
        for (int k = 0; k < n; ++k) {
            const int i = order[k];
            if (runs[i]->g.model == kPotts && runs[i]->g.L % 16)
                continue; // Potts rows split over the lanes: 16 lanes need L a multiple of 16
            const long extra_items = items_of(i, 16) - items_of(i, 4), extra = extra_items * 256;
            if (lanes + extra > cap || n_items + extra_items > max_items)
                break;
            lanes += extra;
            n_items += extra_items;
            lpc[i] = 16;
        }
    }
    // Work items cover the run's chains only: items made of padding chains
    // alone are not launched (padding chains are never histogrammed or read).
    long total_items = 0;
    for (int i = 0; i < n; ++i)
        total_items += items_of(i, lpc[i]);
    if (total_items > max_items)
        return muca_fail(MUCA_E_ARG, "%ld work items exceed the batch capacity %d", total_items, max_items);
    const StageLayout sl = stage_layout(max_runs, max_items);
    BatchHeader *hdr = (BatchHeader *)stage;
    BatchDesc *desc = (BatchDesc *)(stage + sl.desc_off);
    BatchItem *hitems = (BatchItem *)(stage + sl.items_off);
    size_t lds = 0;
    int n_items = 0;
    for (int i = 0; i < n; ++i) {
        muca_run *r = runs[i];
        if (int rc = muca_use_stream(r, s))
            return rc; // the run's last threshold upload may still be queued elsewhere
        const int cpi = 256 / lpc[i]; // chains per item
        const size_t hist = (size_t)lds_hist_words(r->g.n_bins) * 4u;
        lds = std::max(lds, tlds[i] ? r->g.lds_bytes : hist);
        fill_desc(desc[i], r, sweeps[i], tlds[i] != 0, lpc[i]);
        for (int c0 = 0; c0 < r->cfg.n_chains; c0 += cpi)
            hitems[n_items++] = BatchItem{i, c0};
    }
    // longest first (per-item cost); equal costs keep the run and chain order
    std::sort(hitems, hitems + n_items, [&](const BatchItem &x, const BatchItem &y) {
        const double cx = cost[x.inst], cy = cost[y.inst];
        if (cx != cy)
            return cx > cy;
        return x.inst != y.inst ? x.inst < y.inst : x.c_first < y.c_first;
    });
    std::memset(hdr, 0, sizeof *hdr);
    hdr->n_items = n_items;
    // one resident workgroup per CU when the LDS staging is large, two otherwise
    const int per_cu = lds > 80u * 1024u ? 1 : 2;
    out->grid = std::max(1, std::min(n_items, n_cus * per_cu));
    out->lds = lds;
    out->n_items = n_items;
    return MUCA_OK;
}

static hipError_t set_lds(size_t lds)
{
    if (lds > 65536u)
        return hipFuncSetAttribute((const void *)batch_persistent, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

static hipError_t enqueue_batch(muca_batch *b, const BatchSlot &sl, int grid, size_t lds, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(sl.d_hdr, sl.h_buf, b->stage_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(1), 0, s, sl.d_counter);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(batch_persistent, dim3(grid), dim3(256), lds, s, sl.d_hdr, sl.d_counter, sl.d_desc,
                       sl.d_items);
    return hipGetLastError();
}

static void advance_runs(muca_run *const *runs, int n, const int64_t *sweeps)
{
    for (int i = 0; i < n; ++i) {
        runs[i]->sweep += (uint32_t)sweeps[i];
        runs[i]->pending += sweeps[i];
    }
}

extern "C" int muca_batch_run_iteration(muca_batch *b, muca_run *const *runs, int32_t n, const int64_t *sweeps,
                                        void *stream)
try {
    RoctxRange range("muca_batch_round");
    if (!b || !runs || !sweeps || n < 1)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    if (b->poisoned)
        return muca_fail(MUCA_E_STATE, "batch poisoned by an earlier HIP error");
    hipStream_t s = (hipStream_t)stream;
    BatchSlot &sl = b->slot[b->next];
    // this staging area was last read by the round before the previous one
    hipError_t e = sl.used ? hipEventSynchronize(sl.done) : hipSuccess;
    if (e != hipSuccess) {
        b->poisoned = true;
        return muca_fail(MUCA_E_HIP, "batched launch: %s", hipGetErrorString(e));
    }
    std::vector<int> lpc(n), tlds(n), order(n);
    std::vector<double> cost(n);
    RoundPlan plan;
    if (int rc = plan_round(runs, n, sweeps, b->lpc, b->max_runs, b->max_items, b->n_cus, b->lds_limit, sl.h_buf,
                            lpc.data(), tlds.data(), order.data(), cost.data(), s, &plan))
        return rc;
    const int grid = plan.grid;
    const size_t lds = plan.lds;
    e = set_lds(lds);
    if (e == hipSuccess && b->use_graph) {
        if (!sl.exec || sl.graph_stream != s || sl.graph_grid != grid || sl.graph_lds != lds) {
            drop_graph(sl);
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = enqueue_batch(b, sl, grid, lds, s);
                e = hipStreamEndCapture(s, &sl.graph);
                if (e == hipSuccess)
                    e = e2;
            }
            if (e == hipSuccess)
                e = hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0);
            sl.graph_stream = s;
            sl.graph_grid = grid;
            sl.graph_lds = lds;
        }
        if (e == hipSuccess)
            e = hipGraphLaunch(sl.exec, s);
    } else if (e == hipSuccess) {
        e = enqueue_batch(b, sl, grid, lds, s);
    }
    if (e == hipSuccess)
        e = hipEventRecord(sl.done, s);
    if (e != hipSuccess) {
        b->poisoned = true;
        for (int i = 0; i < n; ++i)
            runs[i]->poisoned = true;
        return muca_fail(MUCA_E_HIP, "batched launch: %s", hipGetErrorString(e));
    }
    sl.used = true;
    b->next ^= 1;
    advance_runs(runs, n, sweeps);
    return MUCA_OK;
}
MUCA_ABI_CATCH

// ---------------------------------------------------------------------------
// The batched launch without a batch handle: its work queue lives in a
// file-scope device array instead of a caller's workspace, for callers that
// cannot allocate device memory.
// ---------------------------------------------------------------------------
namespace muca {
constexpr int kScratchRuns = MUCA_NOALLOC_MAX_RUNS;
constexpr int kScratchItems = MUCA_NOALLOC_MAX_ITEMS;
constexpr size_t kScratchStage = 256 + // header
                                 ((kScratchRuns * sizeof(BatchDesc) + 255) / 256) * 256 +
                                 ((kScratchItems * sizeof(BatchItem) + 255) / 256) * 256;
constexpr size_t kScratchBytes = 256 /* work counter */ + kScratchStage;
constexpr int kMaxDevices = 64;
} // namespace muca

// [work counter | header | descriptors | items]; every GPU the library runs
// on holds its own copy until the process ends.
static __device__ __align__(256) uint8_t scratch[muca::kScratchBytes];

static std::mutex g_scratch_mutex;
static uint8_t *g_scratch[muca::kMaxDevices]; // device address of `scratch` per device

// The device address of the current device's `scratch`, looked up once per
// device (with that device current) on the first call there.
static int scratch_address(uint8_t **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return muca_fail(MUCA_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= muca::kMaxDevices)
        return muca_fail(MUCA_E_ARG, "device %d beyond the %d supported", dev, muca::kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return muca_fail(MUCA_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch[dev] = (uint8_t *)p;
    }
    *out = g_scratch[dev];
    return MUCA_OK;
}

extern "C" int muca_batch_run_iteration_noalloc(muca_run *const *runs, int32_t n, const int64_t *sweeps,
                                                int32_t lanes_per_chain, void *stream)
try {
    RoctxRange range("muca_batch_round_noalloc");
    if (!runs || !sweeps || n < 1)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    if (n > kScratchRuns)
        return muca_fail(MUCA_E_ARG, "%d runs exceed the no-allocation launch's maximum of %d", n, kScratchRuns);
    if (lanes_per_chain != 0 && lanes_per_chain != 4 && lanes_per_chain != 16)
        return muca_fail(MUCA_E_ARG, "batched launches use 4 or 16 lanes per chain (0: chosen per run)");
    uint8_t *d_scratch = nullptr;
    if (int rc = scratch_address(&d_scratch))
        return rc;
    int dev = 0, n_cus = 0, lds_limit = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&n_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return muca_fail(MUCA_E_HIP, "device attributes: %s", hipGetErrorString(e));
    for (int i = 0; i < n; ++i) {
        if (!runs[i])
            return muca_fail(MUCA_E_STATE, "run %d is null", i);
        hipPointerAttribute_t pa;
        if (hipPointerGetAttributes(&pa, runs[i]->ws) != hipSuccess || pa.device != dev)
            return muca_fail(MUCA_E_ARG, "run %d's workspace is not on the current device %d", i, dev);
    }
    // host staging on the stack: the copy below is complete before return
    alignas(256) uint8_t stage[kScratchStage];
    int lpc[kScratchRuns], tlds[kScratchRuns], order[kScratchRuns];
    double cost[kScratchRuns];
    RoundPlan plan;
    hipStream_t s = (hipStream_t)stream;
    if (int rc = plan_round(runs, n, sweeps, lanes_per_chain, kScratchRuns, kScratchItems, n_cus, lds_limit, stage, lpc,
                            tlds, order, cost, s, &plan))
        return rc;
    const StageLayout sl = stage_layout(kScratchRuns, kScratchItems);
    if (sl.bytes > kScratchStage)
        return muca_fail(MUCA_E_STATE, "no-allocation staging of %zu bytes exceeds its array", sl.bytes);
    int *d_counter = (int *)d_scratch;
    uint8_t *d_stage = d_scratch + 256;
    const size_t used = sl.items_off + (size_t)plan.n_items * sizeof(BatchItem);
    e = set_lds(plan.lds);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_stage, stage, used, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_reset, dim3(1), dim3(1), 0, s, d_counter); // the queue starts at 0
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_persistent, dim3(plan.grid), dim3(256), plan.lds, s, (const BatchHeader *)d_stage,
                           d_counter, (const BatchDesc *)(d_stage + sl.desc_off),
                           (const BatchItem *)(d_stage + sl.items_off));
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s); // the staging is on this stack frame; the next call rewrites `scratch`
    if (e != hipSuccess) {
        for (int i = 0; i < n; ++i)
            runs[i]->poisoned = true;
        return muca_fail(MUCA_E_HIP, "batched launch (no allocation): %s", hipGetErrorString(e));
    }
    advance_runs(runs, n, sweeps);
    return MUCA_OK;
}
MUCA_ABI_CATCH

// ---------------------------------------------------------------------------
// Autotuner of the batched launch: the time of one work item of a run's
// class (model, layout, L, q) for every candidate (4 or 16 lanes per chain,
// threshold table in LDS or in global memory), measured on probe launches of
// the run's first work item that are undone afterwards.
// ---------------------------------------------------------------------------
static std::string batch_cache_key(const muca_run *r, const char *arch)
{
    char buf[160];
    std::snprintf(buf, sizeof buf, "batch/%s/m%d/lay%d/L%d/q%d", arch, r->g.model, r->g.layout, r->g.L, r->cfg.q);
    return buf;
}

// One work item (the run's chains [0, 256 / lpc)) of `sweeps` sweeps alone
// on the device, timed by events around the kernel.
static hipError_t probe_item(muca_run *r, uint8_t *d_scratch, int lpc, bool tlds, int64_t sweeps, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1, float *ms)
{
    const StageLayout sl = stage_layout(1, 1);
    alignas(256) uint8_t stage[768];
    static_assert(sizeof(BatchDesc) <= 256 && sizeof(BatchItem) <= 256, "probe staging layout");
    std::memset(stage, 0, sizeof stage);
    ((BatchHeader *)stage)->n_items = 1;
    fill_desc(*(BatchDesc *)(stage + sl.desc_off), r, sweeps, tlds, lpc);
    *(BatchItem *)(stage + sl.items_off) = BatchItem{0, 0};
    const size_t lds = tlds ? r->g.lds_bytes : (size_t)lds_hist_words(r->g.n_bins) * 4u;
    uint8_t *d_stage = d_scratch + 256;
    hipError_t e = set_lds(lds);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_stage, stage, sl.bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_reset, dim3(1), dim3(1), 0, s, (int *)d_scratch);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_persistent, dim3(1), dim3(256), lds, s, (const BatchHeader *)d_stage,
                           (int *)d_scratch, (const BatchDesc *)(d_stage + sl.desc_off),
                           (const BatchItem *)(d_stage + sl.items_off));
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e1, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s); // the staging is on this stack frame
    if (e == hipSuccess && ms)
        e = hipEventElapsedTime(ms, e0, e1);
    return e;
}

static uint64_t fnv1a64(uint64_t h, const void *p, size_t n)
{
    const uint8_t *b = (const uint8_t *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

extern "C" int muca_batch_tune(muca_run *r, int64_t probe_sweeps, void *stream, muca_batch_tuning *out)
try {
    RoctxRange range("muca_batch_tune");
    if (!r || r->poisoned)
        return muca_fail(MUCA_E_STATE, "null or poisoned run");
    if (r->merge_begun)
        return muca_fail(MUCA_E_STATE, "a merge was begun and not finished");
    if (kind_of(r) < 0 || l_index(r->g.L) < 0)
        return muca_fail(MUCA_E_ARG, "model %d, L %d has no batched variant", r->g.model, r->g.L);
    if (probe_sweeps < 0 || probe_sweeps > (int64_t)INT32_MAX)
        return muca_fail(MUCA_E_ARG, "probe sweeps %lld out of range", (long long)probe_sweeps);
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, lds_limit = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return muca_fail(MUCA_E_HIP, "no device");
    muca_batch_tuning t;
    std::memset(&t, 0, sizeof t);
    for (auto &row : t.us_per_sweep)
        row[0] = row[1] = -1.0;
    const char *env = std::getenv("MUCA_AUTOTUNE_CACHE");
    const std::string key = batch_cache_key(r, prop.gcnArchName);
    std::string cached;
    if (env && *env && muca_cache_lookup(env, key, cached) &&
        std::sscanf(cached.c_str(), "%lf, %lf, %lf, %lf", &t.us_per_sweep[0][0], &t.us_per_sweep[0][1],
                    &t.us_per_sweep[1][0], &t.us_per_sweep[1][1]) == 4) {
        t.from_cache = 1;
    } else {
        if (int rc = muca_use_stream(r, s))
            return rc;
        uint8_t *d_scratch = nullptr;
        if (int rc = scratch_address(&d_scratch))
            return rc;
        const int64_t sw = probe_sweeps ? probe_sweeps : std::max<int64_t>(1, (50000 + r->g.n_sites - 1) / r->g.n_sites);
        const size_t lds_budget = (size_t)std::min(lds_limit, 160 * 1024) - 256;
        const bool lds_fits = r->g.table_in_lds && r->g.lds_bytes <= lds_budget;
        // the probes change the run's device state (the first item's chains,
        // bins, histogram, accepted-move count): saved here, restored after each
        std::vector<uint8_t> saved(r->g.ws_bytes);
        HIP_OR_POISON(r, hipStreamSynchronize(s));
        HIP_OR_POISON(r, hipMemcpy(saved.data(), r->ws, saved.size(), hipMemcpyDeviceToHost));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess)
            e = hipEventCreate(&e1);
        const int nc = std::min(16, r->cfg.n_chains);
        std::vector<uint8_t> state((size_t)nc * r->g.n_sites);
        std::vector<int32_t> bins(nc);
        bool have_ref = false;
        uint64_t ref = 0;
        if (e == hipSuccess) // loads the code and warms the caches: untimed
            e = probe_item(r, d_scratch, 16, lds_fits, sw, s, e0, e1, nullptr);
        for (int o = 0; o < 2 && e == hipSuccess; ++o)
            for (int tl = 1; tl >= 0 && e == hipSuccess; --tl) {
                if (tl && !lds_fits)
                    continue;
                e = hipMemcpy(r->ws, saved.data(), saved.size(), hipMemcpyHostToDevice);
                float ms = 0.0f;
                if (e == hipSuccess)
                    e = probe_item(r, d_scratch, o ? 16 : 4, tl != 0, sw, s, e0, e1, &ms);
                if (e != hipSuccess)
                    break;
                if (int rc = muca_get_chain_state(r, 0, nc, state.data(), bins.data(), nullptr)) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return rc;
                }
                uint64_t h = fnv1a64(1469598103934665603ull, state.data(), state.size());
                h = fnv1a64(h, bins.data(), bins.size() * 4);
                if (!have_ref) {
                    ref = h;
                    have_ref = true;
                } else if (h != ref) {
                    ++t.rejected;
                    std::fprintf(stderr, "muca_batch_tune: %d lanes per chain, table %s changed the chains; "
                                         "rejected\n", o ? 16 : 4, tl ? "in LDS" : "global");
                    continue;
                }
                t.us_per_sweep[o][tl] = (double)ms * 1e3 / (double)sw;
            }
        if (e == hipSuccess)
            e = hipMemcpy(r->ws, saved.data(), saved.size(), hipMemcpyHostToDevice);
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        if (e != hipSuccess) {
            r->poisoned = true;
            return muca_fail(MUCA_E_HIP, "batch tuning: %s", hipGetErrorString(e));
        }
        if (env && *env && t.rejected == 0) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "%.6g, %.6g, %.6g, %.6g", t.us_per_sweep[0][0], t.us_per_sweep[0][1],
                          t.us_per_sweep[1][0], t.us_per_sweep[1][1]);
            muca_cache_store(env, key, buf);
        }
    }
    double best = -1.0;
    for (int o = 0; o < 2; ++o)
        for (int tl = 0; tl < 2; ++tl)
            if (t.us_per_sweep[o][tl] >= 0.0 && (best < 0.0 || t.us_per_sweep[o][tl] < best)) {
                best = t.us_per_sweep[o][tl];
                t.lanes_per_chain = o ? 16 : 4;
                t.table_in_lds = tl;
            }
    if (best < 0.0)
        return muca_fail(MUCA_E_STATE, "no batched candidate kept its results");
    std::memcpy(r->batch_us, t.us_per_sweep, sizeof r->batch_us);
    r->batch_tuned = true;
    if (out)
        *out = t;
    return MUCA_OK;
}
MUCA_ABI_CATCH
