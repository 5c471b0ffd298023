// muca_internal.h -- structures shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

enum Model : int32_t { kIsing = 0, kPotts = 1, kMuma = 2, kPolymer = 3 };
enum Layout : int32_t { kLayoutBit = 1, kLayoutByte = 2 };

// Arguments of one lattice sweep launch.  Lattice words are interleaved
// across chains: word w of row y of chain c lives at
// words[(y * wpr + w) * c_pad + c], so a wavefront's 64 lanes touch 64
// consecutive 32-bit words.
struct LatticeArgs {
    uint32_t *words;            // [L * wpr][c_pad]
    int32_t *bins;              // [c_pad] current bin of each chain
    const uint32_t *thresholds; // [n_bins * n_cols]
    unsigned long long *hist;   // [n_bins]
    uint32_t k0, k1;            // Philox key (seed)
    uint32_t g0;                // global sweep id of the first sweep
    int32_t n_sweeps;
    int32_t n_chains;           // chains >= n_chains are padding: never histogrammed
    int32_t c_pad;
    int32_t n_bins;
    int32_t q;
    int32_t record;             // histogram the sweeps
    int32_t table_in_lds;
    int32_t chain0;             // global index of the first chain handled
    // MUMA only, or null: joint histogram [(N + 1) * n_bins] of the energy
    // row e = (E + 2N) / 4 and the magnetisation bin after each recorded sweep
    unsigned long long *em;
    unsigned long long *accepts; // accepted moves of the recorded sweeps, or null
    // or null: one histogram [n_bins] per block of chains (the plain launch's
    // workgroups, chains [k * cpb, (k + 1) * cpb)), for jackknife errors
    unsigned long long *hist_blocks;
};

struct LatticeInitArgs {
    uint32_t *words;
    int32_t *bins;
    int32_t *values; // [c_pad] E (Ising/Potts E_unsat) or M (MUMA) after init
    uint32_t k0, k1;
    int32_t c_pad;
    int32_t L, q, lo, step;
    int32_t model, layout;
    int32_t chain0; // global index of chain 0 in the random-number counters
};

// Arguments of one polymer sweep launch (one chain per wavefront).
struct PolymerArgs {
    float4 *pos;                // [c_pad][64] bead positions (w unused)
    double *bond;               // [c_pad][64] energy of bond (j, j + 1)
    double *energy;             // [c_pad] running energy
    int32_t *bins;              // [c_pad]
    const uint32_t *thresholds; // [n_bins][n_bins]
    unsigned long long *hist;   // [n_bins]
    uint32_t k0, k1, g0;
    int32_t n_sweeps, n_chains, c_pad, n_bins, n_beads, record, chains_per_block;
    int32_t chain0;             // global index of chain 0 in the random-number counters
    float step;
    int32_t moves;              // 1: spherical rotations and double bridging after the shifts
    unsigned long long *accepts; // accepted moves of the recorded sweeps, or null
};

// Potential constants, each evaluated on the host once in a fixed order.
struct PolymerConsts {
    double lj_eps, lj_sigma, lj_rcut, lj_shift, fene_pref, fene_r0, fene_R, x_lo, x_hi, scale;
};

hipError_t launch_polymer_sweeps(const PolymerArgs &a, const PolymerConsts &k, hipStream_t s);

// LDS staging of one block: the threshold table (Potts keeps 8 of its 9
// columns: the dE = 0 column always accepts) and a histogram of 16-bit
// counters packed two per word.  A block adds its counters to the global
// histogram every kMaxBlockCount / (chains per block) sweeps, so no counter
// can carry into its neighbour.
__host__ __device__ inline int lds_table_cols(int model) { return model == kIsing ? 5 : (model == kPotts ? 8 : 10); }
__host__ __device__ inline int lds_hist_words(int n_bins) { return (n_bins + 1) / 2; }
constexpr int kMaxBlockCount = 65535; // chains per block x sweeps per launch

// Number of 32-bit words per lattice row.
__host__ __device__ inline int words_per_row(int L, int layout) { return layout == kLayoutBit ? (L + 31) / 32 : (L + 3) / 4; }

// Launchers (lattice.hip).
hipError_t launch_lattice_init(const LatticeInitArgs &a, hipStream_t s);
// threads per block in {64, 128, 256}; lpc lanes per chain in {1, 2, 4, 16}
hipError_t launch_lattice_sweeps(int model, int L, int layout, int lpc, int threads, const LatticeArgs &a,
                                 hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t s);
// host: device address of page-locked host memory (hipHostGetDevicePointer)
hipError_t launch_drain_u64(unsigned long long *p, unsigned long long *host, int64_t n, hipStream_t s);
bool lattice_size_supported(int L);

} // namespace muca
