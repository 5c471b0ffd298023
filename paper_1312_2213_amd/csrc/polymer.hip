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
// energy of bond (j, j+1).  For a move of bead i every lane computes its
// pair term new - old in FP64; the terms are summed by a fixed binary tree
// (lane k += lane k + s for s = 32, 16, ..., 1), so the sum is the same
// number on every run.  The acceptance threshold T[b][b'] of the bin change
// is one scalar load from the B x B matrix.
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

// lane k receives lane k + s (s = 32, 16, ..., 1); lanes whose partner is
// outside the wave get 0 (their sums are never read)
__device__ __forceinline__ double from_lane_above(double v, int s)
{
    const int lane = (int)__lane_id();
    const int src = lane + s;
    const uint64_t u = __double_as_longlong(v);
    const int idx = (src < 64 ? src : lane) * 4;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(idx, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(idx, (int)(uint32_t)(u >> 32));
    return src < 64 ? __longlong_as_double(((uint64_t)hi << 32) | lo) : 0.0;
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
    const uint32_t chain = (uint32_t)c;
    const bool counts = a.record && c < a.n_chains && j == 0;
    const uint32_t B = (uint32_t)a.n_bins;

    for (int s = 0; s < a.n_sweeps; ++s) {
        const uint32_t g = a.g0 + (uint32_t)s;
        const Words4 w = philox4x32_10(chain, g, (uint32_t)j, kTagSweep, a.k0, a.k1);
        for (int i = 0; i < N; ++i) {
            const uint32_t w0 = __builtin_amdgcn_readlane(w.w[0], i);
            const uint32_t w1 = __builtin_amdgcn_readlane(w.w[1], i);
            const uint32_t w2 = __builtin_amdgcn_readlane(w.w[2], i);
            const uint32_t w3 = __builtin_amdgcn_readlane(w.w[3], i);
            const float xi = readlane_f32(x.x, i), yi = readlane_f32(x.y, i), zi = readlane_f32(x.z, i);
            const float nx = xi + ((float)(w0 >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
            const float ny = yi + ((float)(w1 >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
            const float nz = zi + ((float)(w2 >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
            const double ub_i = readlane_f64(ub, i); // bond (i, i + 1), before the move
            const int sep = j > i ? j - i : i - j;
            bool broken = false;
            double en = 0.0, t = 0.0;
            if (bead && sep != 0) {
                const double r2n = dist2(x.x, x.y, x.z, nx, ny, nz);
                if (sep == 1) {
                    en = fene_energy(p, r2n, &broken);
                    const double eo = j < i ? ub : ub_i;
                    t = en - eo;
                } else {
                    const double r2o = dist2(x.x, x.y, x.z, xi, yi, zi);
                    t = lj_energy(p, r2n) - lj_energy(p, r2o);
                }
            }
#pragma unroll
            for (int st = 32; st >= 1; st >>= 1)
                t = t + from_lane_above(t, st);
            const double dE = readlane_f64(t, 0);
            const bool any_broken = __builtin_amdgcn_ballot_w64(broken) != 0ull;
            const double En = E + dE;
            const int32_t bn = energy_bin(p, En, a.n_bins);
            bool acc = false;
            if (!any_broken && bn >= 0) {
                const uint32_t T = a.thresholds[(size_t)b * B + (uint32_t)bn];
                acc = min(w3, 0xFFFFFFFEu) < T;
            }
            if (acc) {
                const double en_right = readlane_f64(en, i + 1 < N ? i + 1 : i); // new bond (i, i + 1)
                if (j == i) {
                    x.x = nx;
                    x.y = ny;
                    x.z = nz;
                    if (i + 1 < N)
                        ub = en_right;
                }
                if (j == i - 1)
                    ub = en; // new bond (i - 1, i)
                E = En;
                b = bn;
            }
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
