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
#include <cstring>
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

struct muca_batch {
    int max_runs = 0, max_items = 0, lpc = 4;
    bool use_graph = false;
    uint8_t *d_ws = nullptr;
    BatchHeader *d_hdr = nullptr;
    int *d_counter = nullptr;
    BatchDesc *d_desc = nullptr;
    BatchItem *d_items = nullptr;
    uint8_t *h_buf = nullptr; // pinned staging of header + descriptors + items
    size_t stage_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
    int graph_grid = 0;
    size_t graph_lds = 0;
    int n_cus = 0, lds_limit = 0;
    bool poisoned = false;
};

static size_t a256(size_t x) { return (x + 255u) & ~(size_t)255u; }

static size_t stage_size(int max_runs, int max_items)
{
    return a256(sizeof(BatchHeader)) + a256((size_t)max_runs * sizeof(BatchDesc)) +
           a256((size_t)max_items * sizeof(BatchItem));
}

extern "C" int muca_batch_workspace_bytes(int32_t max_runs, int32_t max_items, uint64_t *bytes)
try {
    if (max_runs < 1 || max_items < 1 || !bytes)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    *bytes = 256 + stage_size(max_runs, max_items);
    return MUCA_OK;
}
MUCA_ABI_CATCH

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
    b->d_counter = (int *)b->d_ws;
    uint8_t *p = b->d_ws + 256;
    b->d_hdr = (BatchHeader *)p;
    b->d_desc = (BatchDesc *)(p + a256(sizeof(BatchHeader)));
    b->d_items = (BatchItem *)(p + a256(sizeof(BatchHeader)) + a256((size_t)max_runs * sizeof(BatchDesc)));
    b->stage_bytes = stage_size(max_runs, max_items);
    hipError_t e = hipHostMalloc((void **)&b->h_buf, b->stage_bytes, hipHostMallocDefault);
    int dev = 0;
    if (e == hipSuccess)
        e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&b->n_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&b->lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) {
        if (b->h_buf)
            (void)hipHostFree(b->h_buf);
        delete b;
        return muca_fail(MUCA_E_HIP, "batch create: %s", hipGetErrorString(e));
    }
    *out = b;
    return MUCA_OK;
}
MUCA_ABI_CATCH

static void drop_graph(muca_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

extern "C" void muca_batch_free(muca_batch *b)
{
    if (!b)
        return;
    drop_graph(b);
    if (b->h_buf)
        (void)hipHostFree(b->h_buf);
    delete b;
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

static hipError_t enqueue_batch(muca_batch *b, int grid, size_t lds, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(b->d_hdr, b->h_buf, b->stage_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(1), 0, s, b->d_counter);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(batch_persistent, dim3(grid), dim3(256), lds, s, b->d_hdr, b->d_counter, b->d_desc,
                       b->d_items);
    return hipGetLastError();
}

extern "C" int muca_batch_run_iteration(muca_batch *b, muca_run *const *runs, int32_t n, const int64_t *sweeps,
                                        void *stream)
try {
    if (!b || !runs || !sweeps || n < 1)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    if (b->poisoned)
        return muca_fail(MUCA_E_STATE, "batch poisoned by an earlier HIP error");
    if (n > b->max_runs)
        return muca_fail(MUCA_E_ARG, "%d runs exceed the batch capacity %d", n, b->max_runs);
    hipStream_t s = (hipStream_t)stream;
    // lanes per chain of each run.  Automatic choice: every run starts at 4;
    // runs are raised to 16 in order of decreasing per-chain work (the
    // critical path of the launch) while all lanes still fit one resident
    // 256-thread workgroup per CU and the item list its capacity.
    // Work items cover the run's chains only: items made of padding chains
    // alone are not launched (padding chains are never histogrammed or read).
    auto items_of = [&](int i, int l) { return (long)((runs[i]->cfg.n_chains + 256 / l - 1) / (256 / l)); };
    std::vector<int> lpc(n, b->lpc ? b->lpc : 4);
    if (b->lpc == 0) {
        std::vector<int> order(n);
        long lanes = 0, n_items = 0;
        for (int i = 0; i < n; ++i) {
            order[i] = i;
            if (runs[i]) {
                lanes += items_of(i, 4) * 256;
                n_items += items_of(i, 4);
            }
        }
        auto work = [&](int i) {
            return (runs[i]->g.model == kPotts ? 2.0 : 1.0) * (double)runs[i]->g.n_sites * (double)sweeps[i];
        };
        for (int i = 0; i < n; ++i)
            if (!runs[i])
                return muca_fail(MUCA_E_STATE, "run %d is null", i);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
        const long cap = (long)b->n_cus * 256;
        for (int i : order) {
            if (runs[i]->g.model == kPotts && runs[i]->g.L % 16)
                continue; // Potts rows split over the lanes: 16 lanes need L a multiple of 16
            const long extra_items = items_of(i, 16) - items_of(i, 4), extra = extra_items * 256;
            if (lanes + extra > cap || n_items + extra_items > b->max_items)
                break;
            lanes += extra;
            n_items += extra_items;
            lpc[i] = 16;
        }
    }
    struct Item {
        double cost;
        int inst, c_first;
    };
    std::vector<Item> items;
    BatchHeader *hdr = (BatchHeader *)b->h_buf;
    BatchDesc *desc = (BatchDesc *)(b->h_buf + a256(sizeof(BatchHeader)));
    BatchItem *hitems = (BatchItem *)(b->h_buf + a256(sizeof(BatchHeader)) + a256((size_t)b->max_runs * sizeof(BatchDesc)));
    size_t lds = 0;
    const size_t lds_budget = (size_t)std::min(b->lds_limit, 160 * 1024) - 256; // static LDS of the kernel
    for (int i = 0; i < n; ++i) {
        muca_run *r = runs[i];
        if (!r || r->poisoned)
            return muca_fail(MUCA_E_STATE, "run %d is null or poisoned", i);
        if (int rc = muca_use_stream(r, s))
            return rc; // the run's last threshold upload may still be queued elsewhere
        const int kind = kind_of(r), li = l_index(r->g.L);
        if (kind < 0 || li < 0)
            return muca_fail(MUCA_E_ARG, "run %d (model %d, L %d) has no batched variant", i, r->g.model, r->g.L);
        const int cpi = 256 / lpc[i]; // chains per item
        if (sweeps[i] < 1 || sweeps[i] > (int64_t)INT32_MAX)
            return muca_fail(MUCA_E_ARG, "run %d: sweeps %lld out of range", i, (long long)sweeps[i]);
        for (int k = 0; k < i; ++k)
            if (runs[k] == r)
                return muca_fail(MUCA_E_ARG, "run %d appears twice", i);
        const size_t hist = (size_t)lds_hist_words(r->g.n_bins) * 4u;
        const bool tlds = r->g.table_in_lds && r->g.lds_bytes <= lds_budget;
        lds = std::max(lds, tlds ? r->g.lds_bytes : hist);
        BatchDesc &d = desc[i];
        std::memset(&d, 0, sizeof d);
        d.a.words = r->d_words;
        d.a.bins = r->d_bins;
        d.a.thresholds = r->d_table;
        d.a.hist = r->d_hist;
        d.a.k0 = (uint32_t)(r->cfg.seed & 0xffffffffu);
        d.a.k1 = (uint32_t)(r->cfg.seed >> 32);
        d.a.g0 = r->sweep;
        d.a.n_sweeps = (int32_t)sweeps[i];
        d.a.n_chains = r->cfg.n_chains;
        d.a.c_pad = r->g.c_pad;
        d.a.n_bins = r->g.n_bins;
        d.a.q = r->cfg.q;
        d.a.record = 1;
        d.a.table_in_lds = tlds ? 1 : 0;
        d.a.chain0 = r->cfg.chain0;
        d.a.accepts = r->d_hist + r->g.n_bins;
        d.variant = variant_index(kind, li, tlds ? 1 : 0, lpc[i] == 16 ? 1 : 0);
        const double per_site = r->g.model == kPotts ? 2.0 : 1.0;
        const double cost = per_site * (double)r->g.n_sites * (double)sweeps[i];
        for (int c0 = 0; c0 < r->cfg.n_chains; c0 += cpi)
            items.push_back({cost, i, c0});
    }
    if ((int)items.size() > b->max_items)
        return muca_fail(MUCA_E_ARG, "%zu work items exceed the batch capacity %d", items.size(), b->max_items);
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
    std::memset(hdr, 0, sizeof *hdr);
    hdr->n_items = (int32_t)items.size();
    for (size_t k = 0; k < items.size(); ++k) {
        hitems[k].inst = items[k].inst;
        hitems[k].c_first = items[k].c_first;
    }
    // one resident workgroup per CU when the LDS staging is large, two otherwise
    const int per_cu = lds > 80u * 1024u ? 1 : 2;
    const int grid = std::max(1, std::min((int)items.size(), b->n_cus * per_cu));
    hipError_t e = hipSuccess;
    if (lds > 65536u)
        e = hipFuncSetAttribute((const void *)batch_persistent, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess && b->use_graph) {
        if (!b->exec || b->graph_stream != s || b->graph_grid != grid || b->graph_lds != lds) {
            drop_graph(b);
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = enqueue_batch(b, grid, lds, s);
                e = hipStreamEndCapture(s, &b->graph);
                if (e == hipSuccess)
                    e = e2;
            }
            if (e == hipSuccess)
                e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
            b->graph_stream = s;
            b->graph_grid = grid;
            b->graph_lds = lds;
        }
        if (e == hipSuccess)
            e = hipGraphLaunch(b->exec, s);
    } else if (e == hipSuccess) {
        e = enqueue_batch(b, grid, lds, s);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s); // the pinned descriptors are rewritten by the next call
    if (e != hipSuccess) {
        b->poisoned = true;
        for (int i = 0; i < n; ++i)
            runs[i]->poisoned = true;
        return muca_fail(MUCA_E_HIP, "batched launch: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < n; ++i) {
        runs[i]->sweep += (uint32_t)sweeps[i];
        runs[i]->pending += sweeps[i];
    }
    return MUCA_OK;
}
MUCA_ABI_CATCH
