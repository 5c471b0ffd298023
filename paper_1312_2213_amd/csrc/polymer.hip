// polymer.hip -- multicanonical single-monomer shift moves of many
// bead-spring homopolymers (gfx950).
//
// Model (arXiv:1312.2213, Eq. 7): Lennard-Jones between beads |i-j| >= 2,
// cut at r_c and shifted to zero there, plus FENE bonds
// -(K/2) R^2 ln(1 - ((r - r0)/R)^2) between neighbours along the chain.
// A sweep moves beads 0..N-1 in order; bead i of chain c in sweep g draws
// Philox(c, g, i, SWEEP): words 0..2 give the displacement
// ((w >> 8) 2^-24 - 1/2) * step per axis (float), word 3 the acceptance.
//
// Mapping: one chain per wavefront, lane j holds bead j (N <= 64) and the
// energy of bond (j, j+1).  At the start of a sweep lane j computes bead j's
// proposal and the FENE energies of its new bonds (the backward one for both
// outcomes of the previous bead's move).  For a move of bead i every lane
// computes its pair term new - old in FP64 (the two bonded partners take the
// precomputed bond energies); the terms are summed by a fixed binary tree
// (lane k += lane k + s for s = 32, 16, ..., 1) built from lane permutes and
// DPP moves, so the sum is the same number on every run.  The acceptance
// threshold T[b][b'] of the bin change is one load from the B x B matrix.
#include <utility>

#include "muca_internal.h"
#include "philox.h"

namespace muca {

struct PolyParams {
    double lj_eps4;     // 4 eps
    double sig2;        // sigma^2
    double rc2;         // r_c^2
    double lj_shift;    // 4 eps ((sigma/r_c)^12 - (sigma/r_c)^6)
    double fene_pref;   // (K/2) R^2, evaluated as ((0.5 K) R) R
    double fene_r0, fene_R;
    double x_lo, x_hi, scale; // bins: floor((E - x_lo) * scale) on [x_lo, x_hi)
};

__device__ __forceinline__ double lj_energy(const PolyParams &p, double r2)
{
    if (!(r2 < p.rc2))
        return 0.0;
    const double sr2 = p.sig2 / r2;
    const double sr6 = sr2 * sr2 * sr2;
    return p.lj_eps4 * (sr6 * sr6 - sr6) - p.lj_shift;
}

// FENE energy; sets *broken when the bond leaves (r0 - R, r0 + R)
__device__ __forceinline__ double fene_energy(const PolyParams &p, double r2, bool *broken)
{
    const double r = __builtin_sqrt(r2);
    const double t = (r - p.fene_r0) / p.fene_R;
    const double arg = 1.0 - t * t;
    if (!(arg > 0.0)) {
        *broken = true;
        return 0.0;
    }
    return -p.fene_pref * log(arg);
}

__device__ __forceinline__ double dist2(float ax, float ay, float az, float bx, float by, float bz)
{
    const double dx = (double)ax - (double)bx;
    const double dy = (double)ay - (double)by;
    const double dz = (double)az - (double)bz;
    return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float readlane_f32(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Value of the next / previous lane of the wave (0 past either end); used
// once per sweep.
__device__ __forceinline__ float lane_above(float v)
{
    const int lane = (int)__lane_id();
    const float r = __int_as_float(__builtin_amdgcn_ds_bpermute(((lane + 1) & 63) * 4, __float_as_int(v)));
    return lane < 63 ? r : 0.0f;
}

__device__ __forceinline__ float lane_below(float v)
{
    const int lane = (int)__lane_id();
    const float r = __int_as_float(__builtin_amdgcn_ds_bpermute(((lane + 63) & 63) * 4, __float_as_int(v)));
    return lane > 0 ? r : 0.0f;
}

// Lane k receives lane k + S (S = 32, 16, ..., 1) for every lane k < S; the
// other lanes receive values that are never read.  S = 32 and 16 cross rows
// of 16 lanes: v_permlane32_swap / v_permlane16_swap (the second result holds
// rows 2-3 / odd rows moved down); S <= 8 stays inside a row: DPP row_shl.
template <int S>
__device__ __forceinline__ uint32_t from_lane_above_u32(uint32_t v)
{
    if constexpr (S == 32)
        return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
    else if constexpr (S == 16)
        return __builtin_amdgcn_permlane16_swap(v, v, false, false)[1];
    else
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + S, 0xF, 0xF, true); // row_shl:S
}

template <int S>
__device__ __forceinline__ double from_lane_above(double v)
{
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = from_lane_above_u32<S>((uint32_t)u);
    const uint32_t hi = from_lane_above_u32<S>((uint32_t)(u >> 32));
    return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

// The fixed summation tree over 64 slots: slot k += slot k + s for
// s = 32, 16, ..., 1; the sum ends in lane 0.
__device__ __forceinline__ double tree_sum(double t)
{
    t = t + from_lane_above<32>(t);
    t = t + from_lane_above<16>(t);
    t = t + from_lane_above<8>(t);
    t = t + from_lane_above<4>(t);
    t = t + from_lane_above<2>(t);
    t = t + from_lane_above<1>(t);
    return t;
}

__device__ __forceinline__ int32_t energy_bin(const PolyParams &p, double E, int32_t nb)
{
    if (!(E >= p.x_lo) || !(E < p.x_hi))
        return -1;
    const double f = floor((E - p.x_lo) * p.scale);
    if (f < 0.0 || f >= (double)nb)
        return -1;
    return (int32_t)f;
}

__global__ __launch_bounds__(256) void polymer_sweeps(PolymerArgs a, PolyParams p)
{
    extern __shared__ uint32_t lhist[];
    for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x)
        lhist[i] = 0u;
    __syncthreads();

    const int j = (int)(threadIdx.x & 63u);
    const int c = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int N = a.n_beads;
    const bool bead = j < N;
    float4 *pos = a.pos + (size_t)c * 64;
    double *bond = a.bond + (size_t)c * 64;
    float4 x = bead ? pos[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    double ub = (j < N - 1) ? bond[j] : 0.0; // energy of bond (j, j + 1)
    double E = a.energy[c];
    int32_t b = a.bins[c];
    const uint32_t chain = (uint32_t)(a.chain0 + c);
    const bool counts = a.record && c < a.n_chains && j == 0;
    const uint32_t B = (uint32_t)a.n_bins;

    for (int s = 0; s < a.n_sweeps; ++s) {
        const uint32_t g = a.g0 + (uint32_t)s;
        const Words4 w = philox4x32_10(chain, g, (uint32_t)j, kTagSweep, a.k0, a.k1);
        // Bead j's proposal: no earlier move of the sweep changes bead j.
        const float pnx = x.x + ((float)(w.w[0] >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
        const float pny = x.y + ((float)(w.w[1] >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
        const float pnz = x.z + ((float)(w.w[2] >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
        const uint32_t racc = min(w.w[3], 0xFFFFFFFEu); // accept iff racc < T
        // The new bond energies of bead j's move, all known now: bead j + 1
        // has not moved when bead j moves, and bead j - 1 sits either where
        // the sweep found it (its move rejected) or at its proposal
        // (accepted).  Bonds whose stretch leaves the FENE domain are flagged.
        const float rx = lane_above(x.x), ry = lane_above(x.y), rz = lane_above(x.z);
        const float lx = lane_below(x.x), ly = lane_below(x.y), lz = lane_below(x.z);
        const float qx = lane_below(pnx), qy = lane_below(pny), qz = lane_below(pnz);
        double f_fwd = 0.0, f_rej = 0.0, f_acc = 0.0;
        uint32_t flags = 0u; // bit 0: forward broken, 1: back broken (rejected), 2: back broken (accepted)
        if (j + 1 < N) {
            bool br = false;
            f_fwd = fene_energy(p, dist2(rx, ry, rz, pnx, pny, pnz), &br);
            flags |= br ? 1u : 0u;
        }
        if (j >= 1 && bead) {
            bool br = false, ba = false;
            f_rej = fene_energy(p, dist2(lx, ly, lz, pnx, pny, pnz), &br);
            f_acc = fene_energy(p, dist2(qx, qy, qz, pnx, pny, pnz), &ba);
            flags |= (br ? 2u : 0u) | (ba ? 4u : 0u);
        }
        bool prev_acc = false;
        for (int i = 0; i < N; ++i) {
            const float nx = readlane_f32(pnx, i), ny = readlane_f32(pny, i), nz = readlane_f32(pnz, i);
            const float xi = readlane_f32(x.x, i), yi = readlane_f32(x.y, i), zi = readlane_f32(x.z, i);
            const uint32_t w3 = __builtin_amdgcn_readlane(racc, i);
            const uint32_t fl = __builtin_amdgcn_readlane(flags, i);
            const double fb_i = readlane_f64(prev_acc ? f_acc : f_rej, i); // new bond (i - 1, i)
            const double ff_i = readlane_f64(f_fwd, i);                     // new bond (i, i + 1)
            const double ub_i = readlane_f64(ub, i);                        // bond (i, i + 1), before
            const int sep = j > i ? j - i : i - j;
            double t = 0.0;
            if (bead && sep >= 2) {
                const double r2n = dist2(x.x, x.y, x.z, nx, ny, nz);
                const double r2o = dist2(x.x, x.y, x.z, xi, yi, zi);
                t = lj_energy(p, r2n) - lj_energy(p, r2o);
            }
            if (j == i + 1)
                t = ff_i - ub_i;
            if (j == i - 1)
                t = fb_i - ub;
            const double dE = readlane_f64(tree_sum(t), 0);
            const bool any_broken = (i + 1 < N && (fl & 1u)) || (i >= 1 && (fl & (prev_acc ? 4u : 2u)));
            const double En = E + dE;
            const int32_t bn = energy_bin(p, En, a.n_bins);
            bool acc = false;
            if (!any_broken && bn >= 0) {
                const uint32_t T = a.thresholds[(size_t)b * B + (uint32_t)bn];
                acc = w3 < T;
            }
            if (acc) {
                if (j == i) {
                    x.x = nx;
                    x.y = ny;
                    x.z = nz;
                    if (i + 1 < N)
                        ub = ff_i;
                }
                if (j == i - 1)
                    ub = fb_i;
                E = En;
                b = bn;
            }
            prev_acc = acc;
        }
        if (counts)
            atomicAdd(&lhist[b], 1u);
    }
    if (bead)
        pos[j] = x;
    if (j < N - 1)
        bond[j] = ub;
    if (j == 0) {
        a.energy[c] = E;
        a.bins[c] = b;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x) {
        const uint32_t v = lhist[i];
        if (v)
            atomicAdd(&a.hist[i], (unsigned long long)v);
    }
}

hipError_t launch_polymer_sweeps(const PolymerArgs &a, const PolymerConsts &k, hipStream_t s)
{
    PolyParams p;
    p.lj_eps4 = 4.0 * k.lj_eps;
    p.sig2 = k.lj_sigma * k.lj_sigma;
    p.rc2 = k.lj_rcut * k.lj_rcut;
    p.lj_shift = k.lj_shift;
    p.fene_pref = k.fene_pref;
    p.fene_r0 = k.fene_r0;
    p.fene_R = k.fene_R;
    p.x_lo = k.x_lo;
    p.x_hi = k.x_hi;
    p.scale = k.scale;
    const int chains_per_block = a.chains_per_block;
    if (chains_per_block < 1 || chains_per_block > 4 || a.c_pad % chains_per_block)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)(a.c_pad / chains_per_block)), block((unsigned)(64 * chains_per_block));
    hipLaunchKernelGGL(polymer_sweeps, grid, block, (size_t)a.n_bins * 4u, s, a, p);
    return hipGetLastError();
}

} // namespace muca
