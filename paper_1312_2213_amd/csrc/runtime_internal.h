// runtime_internal.h -- host-side run state shared by the runtime sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/muca.h"
#include "host_math.h"

namespace muca {

struct Geometry {
    int model;
    int L, n_sites;      // lattice size / polymer beads
    int step;            // bin width of the binned quantity (lattice)
    int n_bins, n_cols;  // threshold table is n_bins x n_cols (polymer: n_bins x n_bins)
    int layout, wpr;     // lattice storage
    int c_pad;           // chains rounded up to a multiple of 64
    int cpb;             // threads per block
    int lpc;             // lanes per chain
    bool table_in_lds;
    size_t lds_bytes;    // LDS of one lattice block with the table staged
    size_t off_words, off_bins, off_values, off_table, off_hist, off_energy;
    size_t ws_bytes;
};

} // namespace muca

// Page-locked host memory for std::vector: the host mirror of a threshold
// table is the source of its asynchronous upload (a pageable source would be
// staged by the runtime, synchronously).  Throws std::bad_alloc on failure.
template <class V>
struct PinnedAllocator {
    using value_type = V;
    PinnedAllocator() = default;
    template <class U>
    PinnedAllocator(const PinnedAllocator<U> &) {}
    V *allocate(size_t n)
    {
        void *p = nullptr;
        if (hipHostMalloc(&p, n * sizeof(V), hipHostMallocDefault) != hipSuccess || !p)
            throw std::bad_alloc();
        return (V *)p;
    }
    void deallocate(V *p, size_t) { (void)hipHostFree(p); }
    template <class U>
    bool operator==(const PinnedAllocator<U> &) const { return true; }
    template <class U>
    bool operator!=(const PinnedAllocator<U> &) const { return false; }
};

struct muca_run {
    muca_config cfg;
    muca::Geometry g;
    hipStream_t stream = nullptr;
    uint8_t *ws = nullptr;
    uint32_t *d_words = nullptr;   // lattice words / polymer positions (as float)
    int32_t *d_bins = nullptr;
    int32_t *d_values = nullptr;
    uint32_t *d_table = nullptr;
    unsigned long long *d_hist = nullptr;
    double *d_energy = nullptr;    // polymer running energies
    std::vector<double> lnW, lnR, P;
    std::vector<uint8_t> mask;     // bins linked by the recursion / measured for flatness
    // host mirror of the thresholds, the source of their asynchronous upload:
    // rewritten only after the run's stream was synchronised
    std::vector<uint32_t, PinnedAllocator<uint32_t>> T;
    std::vector<uint64_t> H_last;  // last merged histogram H^(n)
    std::vector<double> lnW_last;  // lnW^(n) that produced H_last
    uint32_t sweep = 0;            // global sweep counter (Philox counter word 1)
    int64_t iteration = 0;
    int64_t pending = 0;           // recorded sweeps since the last merge
    bool have_last = false;
    bool poisoned = false;
    // pinned host staging (lattice runs): the histogram and accepted-move
    // count read back at a merge, and its device-side address
    uint64_t *h_hist = nullptr;
    unsigned long long *h_hist_dev = nullptr;
    // measured time of one batched work item per sweep (microseconds), by
    // [4 / 16 lanes per chain][table in global memory / in LDS]; < 0: not
    // measured or not a candidate (muca_batch_tune)
    double batch_us[2][2] = {{-1.0, -1.0}, {-1.0, -1.0}};
    bool batch_tuned = false;
    // a merge split into muca_merge_begin / muca_merge_finish: the event
    // recorded behind the histogram read-back, and whether one is under way
    hipEvent_t merge_ev = nullptr;
    bool merge_begun = false;
    // per-iteration log: this run's number and the wall clock of its last merge
    int64_t log_id = 0;
    double t_last = 0.0;
    ~muca_run();
};

int muca_fail(int code, const char *fmt, ...);

// A named range on the roctx timeline of a profiler (rocprofv3
// --marker-trace): init, iterations, merges and batched rounds show up
// beside the kernels.  Costs a function call when no profiler listens.
struct RoctxRange {
    explicit RoctxRange(const char *name);
    ~RoctxRange();
    RoctxRange(const RoctxRange &) = delete;
    RoctxRange &operator=(const RoctxRange &) = delete;
};

// One JSON line per merged iteration, appended to the file named by the
// environment variable MUCA_ITER_LOG (nothing when it is unset).
void muca_log_iteration(const muca_run *r, const muca_iter_stats &s, double seconds, double attempts);

// A HIP call whose failure poisons the run and returns MUCA_E_HIP.
#define HIP_OR_POISON(run, expr)                                                                   \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            (run)->poisoned = true;                                                                \
            return muca_fail(MUCA_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));                  \
        }                                                                                          \
    } while (0)

// The autotuners' JSON cache (MUCA_AUTOTUNE_CACHE): `values` is the text
// between the brackets of the entry `key`.
bool muca_cache_lookup(const std::string &path, const std::string &key, std::string &values);
void muca_cache_store(const std::string &path, const std::string &key, const std::string &values);

// Handlers of a C entry point's function-try-block: no exception crosses the
// ABI (host allocations are the only source: std::bad_alloc).
#define MUCA_ABI_CATCH                                                                                 \
    catch (const std::bad_alloc &)                                                                     \
    {                                                                                                  \
        return muca_fail(MUCA_E_NOMEM, "out of host memory");                                          \
    }                                                                                                  \
    catch (...)                                                                                        \
    {                                                                                                  \
        return muca_fail(MUCA_E_STATE, "unexpected exception in the library");                       \
    }
int muca_geometry(const muca_config *c, muca::Geometry *g);
// Rebuilds the threshold table from lnW and queues its upload on the run's
// stream; the caller has synchronised that stream.
int muca_rebuild_thresholds(muca_run *r);
// Moves the run to stream s; work still queued on its previous stream (the
// last threshold upload included) is waited for first.
int muca_use_stream(muca_run *r, hipStream_t s);
int muca_enqueue_sweeps(muca_run *r, int64_t sweeps, bool record, hipStream_t s,
                        unsigned long long *em = nullptr, unsigned long long *hist_blocks = nullptr);
int muca_finish_iteration(muca_run *r, const uint64_t *H, uint64_t accepted, muca_iter_stats *st);

// polymer.cpp
int muca_polymer_geometry(const muca_config *c, muca::Geometry *g);
int muca_polymer_init(muca_run *r, const float *h_pos);
void muca_polymer_build(muca_run *r);
// queues the upload of the host threshold mirror on the run's stream
int muca_upload_thresholds(muca_run *r);
int muca_polymer_enqueue(muca_run *r, int64_t sweeps, bool record, hipStream_t s);
int muca_polymer_state(muca_run *r, int32_t chain0, int32_t count, float *pos, int32_t *bins,
                       double *energy);
