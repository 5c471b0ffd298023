/*
 * muca.h -- C ABI of the MI355X (gfx950) parallel multicanonical library.
 *
 * Method: Zierenberg, Marenz, Janke, "Scaling Properties of Parallelized
 * Multicanonical Simulations" (arXiv:1312.2213).  p independent Markov
 * chains share one weight function W; after each iteration their histograms
 * are merged into H^(n) and the next weights W^(n+1) are computed from all
 * statistics gathered so far (parallel-scheme paragraph, Fig. 1 caption).
 *
 * Conventions for every entry point:
 *  - Return value: MUCA_OK (0) on success, a negative muca_status otherwise;
 *    no exception crosses the ABI.  muca_last_error() returns a thread-local
 *    message for the last failure on the calling thread.
 *  - On MUCA_E_ARG / MUCA_E_RANGE the run is left unchanged.  MUCA_E_NOMEM
 *    reports a workspace that is too small (run unchanged) or host memory
 *    (pageable or pinned) that could not be allocated; after the latter the
 *    run may hold a partial update and should be freed.
 *    On MUCA_E_HIP the run is poisoned and later calls return MUCA_E_STATE.
 *  - Pointers named d_* are device (HBM) pointers, h_* are host pointers.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    A run's device work (sweeps, the threshold upload that follows every
 *    merge) is ordered on the stream of its last call; a call on another
 *    stream first waits for the previous stream, so runs may move between
 *    streams freely.  Calls that overlap on one run are not allowed.
 *  - The library never allocates or frees device memory: the caller passes a
 *    device workspace of muca_workspace_bytes() bytes (256-byte aligned) and
 *    keeps it, and the stream, alive until muca_free().  Host-side state
 *    (log weights, accumulated statistics, a mirror of the thresholds) is
 *    owned by the run handle; the threshold mirror and the histogram
 *    read-back buffer are page-locked host memory, so that their copies are
 *    asynchronous on the run's stream.
 *  - A run is used from one thread at a time; distinct runs are independent.
 */
#ifndef MUCA_H
#define MUCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MUCA_ABI_VERSION 3u

typedef enum muca_status {
    MUCA_OK = 0,
    MUCA_E_ARG = -1,   /* invalid argument or configuration              */
    MUCA_E_NOMEM = -2, /* workspace too small, or host memory exhausted  */
    MUCA_E_HIP = -3,   /* a HIP runtime call failed (run poisoned)       */
    MUCA_E_STATE = -4, /* call out of order, or run poisoned             */
    MUCA_E_RANGE = -5  /* a chain is outside the binned range            */
} muca_status;

/* Models (paper: Ising and Potts paragraphs, Eq. 3 for MUMA, Eq. 7 for the
 * polymer). */
typedef enum muca_model {
    MUCA_ISING = 0,  /* 2D Ising, H = -sum s_i s_j (J = 1); bins over E       */
    MUCA_POTTS = 1,  /* 2D q-state Potts; bins over E_unsat (unsatisfied bonds) */
    MUCA_MUMA = 2,   /* 2D Ising at fixed beta, weight W(M) (Eq. 3); bins over M */
    MUCA_POLYMER = 3 /* bead-spring homopolymer, LJ + FENE (Eq. 7); bins over E */
} muca_model;

/* Lattice storage in HBM; results never depend on it. */
typedef enum muca_layout {
    MUCA_LAYOUT_AUTO = 0,
    MUCA_LAYOUT_BIT = 1, /* Ising/MUMA: one bit per spin                     */
    MUCA_LAYOUT_BYTE = 2 /* Ising/MUMA: int8 +-1; Potts: uint8 colour       */
} muca_layout;

typedef struct muca_config {
    uint32_t abi_version;   /* must be MUCA_ABI_VERSION                        */
    int32_t model;          /* muca_model                                      */
    int32_t L;              /* lattice: periodic L x L, L in {4,8,16,24,32,48,64} */
    int32_t q;              /* Potts: 2..255                                   */
    int32_t n_chains;       /* p, number of independent realisations (>= 1)   */
    int32_t layout;         /* muca_layout                                     */
    uint64_t seed;          /* Philox key                                      */
    int32_t lo, hi;         /* lattice: inclusive binned range, in units of the
                               binned quantity (Ising E step 4, Potts E_unsat
                               step 1, MUMA M step 2)                          */
    double beta;            /* MUMA: fixed inverse temperature                 */
    double flat_threshold;  /* flat iff min(H)/mean(H) over the flatness set > this */
    int32_t chains_per_block; /* 0 = auto; chains_per_block x lanes_per_chain
                                 must be 64, 128, 256 or 512 threads; 512
                                 only with the table staged in LDS         */
    int32_t table_in_lds;   /* -1 auto, 0 thresholds read from global memory, 1 staged in LDS */
    /* polymer */
    int32_t n_beads;        /* 2..128                                          */
    int32_t n_bins;         /* energy bins on [x_lo, x_hi)                     */
    double x_lo, x_hi;
    double lj_eps, lj_sigma, lj_rcut;
    double fene_k, fene_r0, fene_R; /* FENE -(K/2) R^2 ln(1-((r-r0)/R)^2)     */
    float step;             /* side of the displacement cube                   */
    int32_t lanes_per_chain; /* lattice: 0 = auto, else 1, 2, 4 or 16 lanes share
                                one chain's random-number work                 */
    int32_t chain0;         /* global index of the run's first chain: its chains
                               are numbered chain0 .. chain0 + n_chains - 1 in the
                               random-number counters, so a run of C chains can
                               be split into shards of consecutive chains (one
                               per device) that together give the unsplit run;
                               0 for a standalone run, >= 0                    */
    int32_t moves;          /* polymer: 0 = single-bead shifts; 1 = the paper's
                               move set (polymer paragraph): per sweep N shifts,
                               N spherical rotations (bead i about the line
                               through beads i-1 and i+1; an end bead about a
                               coordinate axis through its neighbour) and one
                               double bridging (bonds (i,i+1), (j,j+1) replaced
                               by (i,j), (i+1,j+1), beads i+1..j renumbered in
                               reverse).  0 for lattice runs.                 */
} muca_config;

typedef struct muca_iter_stats {
    int64_t iteration;  /* n of the merged histogram H^(n), from 0             */
    int64_t sweeps;     /* sweeps per chain that went into H^(n)               */
    int64_t samples;    /* sum of H^(n)                                        */
    double flatness;    /* min/mean of H^(n) over the flatness set             */
    int32_t flat;       /* flatness > flat_threshold                           */
    int32_t lo_visited; /* lowest / highest bin with H^(n) > 0, -1 if none     */
    int32_t hi_visited;
    int32_t reserved;
    double accept_rate; /* accepted / attempted moves over the sweeps of H^(n)
                           (lattice: N attempts per chain and sweep; polymer:
                           N, or 2N + 1 with the full move set); a sharded
                           run reports its own chains                        */
} muca_iter_stats;

typedef struct muca_run muca_run;

/* Fills *cfg with defaults for the model: full binned range, layout AUTO,
 * flat_threshold 0.5, polymer parameters of the bead-spring workload (LJ
 * eps = sigma = 1 cut at 2.5 and shifted; FENE K = 40, r0 = 1, R = 0.5;
 * 2500 bins on [-200, 50); step 0.3). */
int muca_config_default(int32_t model, int32_t L, int32_t q, int32_t n_chains, uint64_t seed,
                        muca_config *cfg);

/* Device workspace needed by muca_init for this configuration. */
int muca_workspace_bytes(const muca_config *cfg, uint64_t *bytes);

/* Initialises p realisations with the same weights lnW = 0 (parallel-scheme
 * paragraph).  Lattices: spins drawn on the device from the Philox stream
 * (chain, 0, site/4, INIT); then E, M and the bins.  Polymer:
 * h_positions = [n_chains][n_beads][3] float conformations (host), copied.
 * Enqueued on `stream` and synchronised before returning.  MUCA_E_RANGE if a
 * chain starts outside the binned range. */
int muca_init(const muca_config *cfg, void *d_workspace, uint64_t workspace_bytes,
              const float *h_positions, void *stream, muca_run **out);

/* One iteration's sampling step (parallel-scheme paragraph and Fig. 1
 * caption: every realisation runs M sweeps with the same weights W^(n) and
 * fills its own histogram; Eq. 1 gives the multicanonical weight, Eq. 3 the
 * multimagnetic one).  Enqueues `sweeps` (>= 1) sweeps of every chain with
 * the current thresholds, accumulating into the device histogram; returns
 * without waiting.  Repeated calls before muca_merge_update extend the same
 * iteration (bit-identical to one call with the summed sweeps).  A sweep
 * visits the sites in row-major order (polymer: beads 0..N-1); after each
 * sweep every chain adds one entry to H.  Metropolis acceptance
 * min(1, W(E')/W(E)) (MUMA: min(1, exp(-beta dE) W(M')/W(M))) by integer
 * thresholds.  The chains, spins, bins and histogram stay in the run's
 * device workspace.  MUCA_E_ARG for sweeps < 1 (run unchanged); MUCA_E_HIP
 * if the launch fails (run poisoned). */
int muca_run_iteration(muca_run *run, int64_t sweeps, void *stream);

/* Same, but the sweeps are not histogrammed (thermalisation). */
int muca_thermalize(muca_run *run, int64_t sweeps, void *stream);

/* Ends iteration n (parallel-scheme paragraph and Fig. 1 caption: the
 * realisations' histograms are merged into H^(n), which decides flatness and
 * gives the next weights W^(n+1) for all of them; the weights follow the
 * accumulated-statistics recursion named in the paragraph after Eq. 2, which
 * reduces to W^(n+1) = W^(n) / H^(n) on its first step).  Waits for the run's
 * stream, reads the merged H^(n) (B x uint64, summed over all chains on the
 * device), evaluates flatness (min / mean over the reachable bins), applies
 * the recursion in FP64 to obtain lnW^(n+1), builds the new thresholds and
 * enqueues their upload on the run's stream, and clears H.  `out` (may be
 * NULL) receives the iteration's statistics.  MUCA_E_STATE if no sweeps were
 * enqueued since the last merge; MUCA_E_HIP if a copy fails (run poisoned). */
int muca_merge_update(muca_run *run, muca_iter_stats *out);

/* muca_merge_update in two halves, so that the host part of a merge can
 * overlap device work queued after it on the same stream (the serving loop
 * launches the next batched round between them):
 *   muca_merge_begin: enqueues the read-back of the merged histogram H^(n)
 *     (and its clear) on the run's stream behind its sweeps and records an
 *     event behind it; returns at once.  MUCA_E_STATE if no sweeps were
 *     enqueued since the last merge.  Until muca_merge_finish, every other
 *     call on the run except muca_free returns MUCA_E_STATE.
 *   muca_merge_finish: waits for that event only (not for work queued on
 *     the stream after muca_merge_begin), then flatness, recursion and the
 *     new thresholds exactly as muca_merge_update, whose upload is enqueued
 *     on the run's stream behind whatever is queued there.  MUCA_E_STATE
 *     without a preceding muca_merge_begin.
 * begin + finish with nothing in between is muca_merge_update. */
int muca_merge_begin(muca_run *run);
int muca_merge_finish(muca_run *run, muca_iter_stats *out);

/* Sharded runs (one run per device, each a consecutive range of the global
 * chains, all with the same seed and weights; parallel-scheme paragraph:
 * the histograms of all realisations are merged and every part continues
 * with the same new weights).
 *   muca_get_pending_hist: copies the histogram accumulated by
 *     muca_run_iteration since the last merge (n = number of bins) to
 *     host memory h, after waiting for the run's stream; the run is unchanged.
 *     MUCA_E_STATE without sweeps since the last merge.
 *   muca_merge_update_hist: muca_merge_update with a caller-supplied merged
 *     histogram (the sum of every shard's pending histogram, e.g. from an
 *     all-reduce); the run's own pending histogram is discarded.  Every shard
 *     calling it with the same h gets the same weights and thresholds, so the
 *     shards stay the unsplit run bit for bit.  Errors as muca_merge_update;
 *     MUCA_E_ARG if n differs from the number of bins. */
int muca_get_pending_hist(const muca_run *run, uint64_t *h, int64_t n);
int muca_merge_update_hist(muca_run *run, const uint64_t *h, int64_t n, muca_iter_stats *out);

/* Reweighting (Eq. 2) of the last merged pair (H^(n), lnW^(n)).
 * Energy ensembles: for each beta[k], out[4k..4k+3] = { <E>/N, beta^2
 * Var(E)/N, <E>, ln sum_b H_b W_b^-1 e^(-beta E_b) } with N sites (beads).
 * MUMA (canonical at the run's beta; pass n = 1, betas may be NULL):
 * out = { <|M|>/N, <M^2>/N^2, <M>/N, ln sum_b H_b W_b^-1 }.
 * Potts energies are E_unsat - 2N; polymer bins use their centres. */
int muca_reweight(const muca_run *run, const double *betas, int32_t n, double *out);

/* Joint (E, M) histogram of a multimagnetic run, for reweighting in the
 * temperature (multimagnetic paragraph: the run flattens M at a fixed beta;
 * with E recorded beside M, Eq. 2 with the weight exp(-beta E) W(M) of Eq. 3
 * in place of W(E) gives canonical averages at any beta' near beta).
 *   muca_em_shape: n_e = N + 1 energy rows (row e holds E = -2N + 4e), n_m =
 *     the number of magnetisation bins.  MUCA_E_ARG if the run is not MUMA.
 *   muca_run_iteration_em: muca_run_iteration that also adds, for every
 *     chain and sweep, one count to d_em[e * n_m + b], e and b those of the
 *     configuration the sweep left.  d_em: device memory of n_e * n_m
 *     uint64, owned by the caller, accumulated into and never cleared.  The
 *     chains, the histogram H and the sweep counter are those of
 *     muca_run_iteration.  MUCA_E_ARG for a run that is not MUMA, a null
 *     d_em or sweeps < 1.
 *   muca_reweight_em: for each betas[k], out[6k..6k+5] = { <E>/N,
 *     beta'^2 Var(E)/N, <|M|>/N, <M^2>/N^2, beta' (<M^2> - <|M|>^2)/N,
 *     ln sum_{e,b} h W_b^-1 e^(-(beta' - beta) E_e) } over the host copy
 *     h_em (n_em = n_e * n_m entries) of a joint histogram recorded with the
 *     weights of the last merged iteration (the lnW^(n) of muca_reweight).
 *     MUCA_E_STATE before the first merge, MUCA_E_ARG for a size mismatch,
 *     null pointers or n < 1. */
/* Per-block histograms and jackknife errors of the reweighted observables
 * (Eq. 2 over the merged histogram; the blocks are independent groups of
 * chains, so leaving one out at a time gives the statistical error of any
 * reweighted average).  Lattice runs.
 *   muca_blocks_shape: n_blocks = the number of chain blocks (workgroups of
 *     the run's plain launch) and chains_per_block; block k holds chains
 *     [k * chains_per_block, (k + 1) * chains_per_block), padding chains
 *     (>= n_chains) never counted.  MUCA_E_ARG for a polymer run.
 *   muca_run_iteration_blocks: muca_run_iteration that also adds each
 *     block's histogram to d_blocks[k * n_bins + b] (device memory, n_blocks
 *     * n_bins uint64, owned by the caller, accumulated into, never
 *     cleared).  The chains and H are those of muca_run_iteration.
 *   muca_reweight_jackknife: from the host copy h_blocks of block
 *     histograms recorded with the weights of the last merged iteration,
 *     out[4q..4q+3] = muca_reweight's values over their sum and
 *     err[4q..4q+3] = their jackknife errors sqrt((m-1)/m sum_k (v_k -
 *     mean)^2) over the m non-empty blocks, v_k the values without block k.
 *     MUCA_E_STATE before the first merge; MUCA_E_ARG for null pointers,
 *     n < 1 or fewer than two non-empty blocks. */
int muca_blocks_shape(const muca_run *run, int32_t *n_blocks, int32_t *chains_per_block);
int muca_run_iteration_blocks(muca_run *run, int64_t sweeps, uint64_t *d_blocks, void *stream);
int muca_reweight_jackknife(const muca_run *run, const uint64_t *h_blocks, int32_t n_blocks, const double *betas,
                            int32_t n, double *out, double *err);

int muca_em_shape(const muca_run *run, int32_t *n_e, int32_t *n_m);
int muca_run_iteration_em(muca_run *run, int64_t sweeps, uint64_t *d_em, void *stream);
int muca_reweight_em(const muca_run *run, const uint64_t *h_em, int64_t n_em, const double *betas, int32_t n,
                     double *out);

/* Batched iterations (one persistent launch for several lattice runs of
 * mixed model, L, q, ensemble and layout).  The runs' chains are cut into
 * work items of 256 / lanes_per_chain chains that a grid sized to the chip
 * takes longest first from an atomic queue; each work item runs exactly the
 * sweep code of muca_run_iteration, so every run's histogram and chains are
 * bit-identical to plain launches.
 *   muca_batch_workspace_bytes: device bytes for up to max_runs runs and
 *     max_items work items (two staging areas, used by alternate rounds).
 *   muca_batch_create: lanes_per_chain 4 or 16 for every run, or 0 to
 *     choose per launch: runs start at 4 and, longest per-chain work first,
 *     move to 16 while all lanes fit one 256-thread workgroup per compute
 *     unit and the items fit max_items (see muca_batch_tune for runs whose
 *     item times were measured).  use_graph != 0 captures [descriptor
 *     upload, queue reset, persistent kernel] in a hipGraph once per staging
 *     area and relaunches it (requires a non-null stream).  d_ws is
 *     caller-owned (256-byte aligned); the handle owns two small pinned host
 *     buffers.
 *   muca_batch_run_iteration: equivalent to muca_run_iteration(runs[i],
 *     sweeps[i]) for every i; returns once the launch is enqueued.  Rounds
 *     alternate between two staging areas, each fenced by an event, so the
 *     next call can plan its round while this one runs (it waits only for
 *     the round before this one).  MUCA_E_ARG for polymer runs, L outside
 *     {8,16,24,32,48,64}, a run given twice, or capacity exceeded;
 *     MUCA_E_STATE for a run whose merge was begun and not finished.
 *     muca_batch_free waits for the rounds still reading its buffers. */
typedef struct muca_batch muca_batch;
int muca_batch_workspace_bytes(int32_t max_runs, int32_t max_items, uint64_t *bytes);
int muca_batch_create(int32_t max_runs, int32_t max_items, int32_t lanes_per_chain, int32_t use_graph,
                      void *d_ws, uint64_t ws_bytes, muca_batch **out);
int muca_batch_run_iteration(muca_batch *batch, muca_run *const *runs, int32_t n_runs, const int64_t *sweeps,
                             void *stream);
void muca_batch_free(muca_batch *batch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * batched iteration of muca_batch_run_iteration without a batch handle or
 * workspace.  Its work queue (counter, descriptors, work items) lives in a
 * file-scope device array of the library, one per GPU, held until the
 * process ends; the call allocates no device or pinned host memory.  Limits:
 * at most MUCA_NOALLOC_MAX_RUNS runs and MUCA_NOALLOC_MAX_ITEMS work items
 * (256 / lanes_per_chain chains each) per call, else MUCA_E_ARG with the run
 * unchanged.  lanes_per_chain: 4, 16, or 0 to choose per run as
 * muca_batch_create does.  The runs must live on the current device
 * (MUCA_E_ARG otherwise).  No graph capture of this call; it returns after
 * the launch has completed.  All calls on one GPU share that array: calls
 * that overlap on one GPU (from several threads) race and are not allowed.
 * Results are bit-identical to muca_batch_run_iteration and to plain
 * launches.  Other errors as muca_batch_run_iteration. */
#define MUCA_NOALLOC_MAX_RUNS 64
#define MUCA_NOALLOC_MAX_ITEMS 4096
int muca_batch_run_iteration_noalloc(muca_run *const *runs, int32_t n_runs, const int64_t *sweeps,
                                     int32_t lanes_per_chain, void *stream);

/* Autotuner of the batched launch (the batching pattern's chains per
 * workgroup and table placement, per class of run).  Measures the time of
 * one work item of the run's class (model, layout, L, q) for every candidate:
 * 4 or 16 lanes per chain (64 or 16 chains per 256-thread work item), and
 * the threshold table staged in LDS (where it fits) or read from global
 * memory.  Each probe runs the run's first work item for probe_sweeps sweeps
 * (0: about 5e4 site updates per chain) alone on the device; the run's
 * device state is saved before and restored after, so its results do not
 * change.  A candidate whose first 16 chains end in a different state than
 * the first candidate's is rejected (counted in `rejected`).  Results are
 * read from / written to the JSON file named by MUCA_AUTOTUNE_CACHE (key:
 * architecture and class; an item's time does not depend on the number of
 * chains).  The run keeps the measurement: a batched launch with
 * lanes_per_chain 0 (muca_batch_create, muca_batch_run_iteration_noalloc)
 * whose runs are all tuned takes per run the table placement of the faster
 * item and the lanes per chain that minimise the estimated length of the
 * round, max(longest item, total item time / compute units), starting from
 * the choice of least total item time; items are ordered by their measured
 * time.  The probes use the library's device array of
 * muca_batch_run_iteration_noalloc: they must not overlap with such a call
 * on the same GPU.  Returns after the probes have completed.  MUCA_E_ARG for
 * a run without a batched variant; MUCA_E_HIP if a probe fails (run
 * poisoned). */
typedef struct muca_batch_tuning {
    double us_per_sweep[2][2]; /* one item's time per sweep (microseconds):
                                  [4 / 16 lanes per chain][table global / in LDS];
                                  -1: not a candidate */
    int32_t lanes_per_chain;   /* the candidate with the shortest item */
    int32_t table_in_lds;
    int32_t from_cache;        /* 1: read from MUCA_AUTOTUNE_CACHE */
    int32_t rejected;          /* candidates that changed the chains */
} muca_batch_tuning;
int muca_batch_tune(muca_run *run, int64_t probe_sweeps, void *stream, muca_batch_tuning *out);

/* Autotuner: times `sweeps` sweeps of every compiled variant of cfg (layout,
 * lanes per chain, chains per block, threshold table in LDS or global) in
 * the caller's workspace d_ws and returns the fastest in *best (time per
 * sweep in *best_ms_per_sweep, -1 when taken from the cache).  A candidate
 * whose histogram, spins or bins differ from the first candidate's is
 * rejected.  With MUCA_AUTOTUNE_CACHE set to a file path, results are read
 * from / written to that JSON file, keyed by GPU architecture and shape.
 * The workspace must hold the largest candidate (layout BYTE for Ising). */
int muca_autotune(const muca_config *cfg, void *d_ws, uint64_t ws_bytes, int64_t sweeps, void *stream,
                  muca_config *best, double *best_ms_per_sweep);

/* Accessors (host copies; synchronise the run's stream). */
int muca_sizes(const muca_run *run, int32_t *n_bins, int32_t *n_cols, int32_t *n_sites);
int muca_get_lnw(const muca_run *run, double *h_lnw, int32_t n_bins);
int muca_get_last_hist(const muca_run *run, uint64_t *h_hist, int32_t n_bins);
int muca_get_thresholds(const muca_run *run, uint32_t *h_t, int64_t count);
/* Lattice: spins[count][N] bytes (Ising/MUMA int8 +-1, Potts uint8 colour 0..q-1), bins[count].
 * Polymer: positions[count][n_beads][3] float into `state`, energies[count]
 * double into `energy`.  Either output may be NULL. */
int muca_get_chain_state(const muca_run *run, int32_t chain0, int32_t count, void *state,
                         int32_t *bins, double *energy);

/* Test hooks: replace lnW (thresholds rebuilt) or the thresholds themselves
 * (count = n_bins * n_cols; polymer n_bins^2). */
int muca_set_lnw(muca_run *run, const double *h_lnw, int32_t n_bins);
int muca_set_thresholds(muca_run *run, const uint32_t *h_t, int64_t count);

/* Checkpoint / restore of the complete run state (chains, sweep counter,
 * weights, accumulated statistics).  muca_checkpoint with h_buf = NULL
 * returns the size in *bytes. */
int muca_checkpoint(const muca_run *run, void *h_buf, uint64_t *bytes);
int muca_restore(muca_run *run, const void *h_buf, uint64_t bytes);

void muca_free(muca_run *run);
const char *muca_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MUCA_H */
