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
// Mapping: one chain per wavefront, lane j holds bead j and the energy of
// bond (j, j+1), and for 64 < N <= 128 also bead j + 64 and its bond.  At the start of a sweep lane j computes bead j's
// proposal and the FENE energies of its new bonds (the backward one for both
// outcomes of the previous bead's move).  For a move of bead i every lane
// computes its pair term new - old in FP64 (the two bonded partners take the
// precomputed bond energies); the terms are summed by a fixed binary tree
// (lane k += lane k + s for s = 32, 16, ..., 1) built from lane permutes and
// DPP moves, so the sum is the same number on every run.  The acceptance
// threshold T[b][b'] of the bin change is one load from the B x B matrix.
//
// With the paper's move set (moves = 1) each sweep continues with a
// spherical rotation of every bead (an inner bead about the line through its
// neighbours, an end bead about a coordinate axis through its neighbour,
// both by the quaternion (tau, axis) with tau symmetric about zero: only +,
// -, *, / in FP64, so the proposal is bit-identical everywhere) and one
// double bridging (two bonds swapped for two new ones, the beads between
// renumbered in reverse by one lane permute); the energy change of a
// rotation is the same lane-parallel tree sum as for a shift.
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

// The same squared distance with the first position already in FP64 (a
// float converts to double exactly).
__device__ __forceinline__ double dist2d(double ax, double ay, double az, float bx, float by, float bz)
{
    const double dx = ax - (double)bx;
    const double dy = ay - (double)by;
    const double dz = az - (double)bz;
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

// One level of the tree across rows (S = 32 or 16) in place: the swap moves
// rows 2-3 (S = 32) or the odd rows (S = 16) of its first operand into the
// second, whose own values are never read, and leaves the lanes below S of
// the first operand as they were; the sum is valid in the lanes below S.
template <int S>
__device__ __forceinline__ double tree_level_swap(double t)
{
    const uint64_t u = __double_as_longlong(t);
    uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    const uint32_t junk_lo = __builtin_nondeterministic_value(lo), junk_hi = __builtin_nondeterministic_value(hi);
    uint32_t plo, phi;
    if constexpr (S == 32) {
        const auto rl = __builtin_amdgcn_permlane32_swap(lo, junk_lo, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(hi, junk_hi, false, false);
        lo = rl[0], plo = rl[1], hi = rh[0], phi = rh[1];
    } else {
        const auto rl = __builtin_amdgcn_permlane16_swap(lo, junk_lo, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(hi, junk_hi, false, false);
        lo = rl[0], plo = rl[1], hi = rh[0], phi = rh[1];
    }
    return __longlong_as_double(((uint64_t)hi << 32) | lo) + __longlong_as_double(((uint64_t)phi << 32) | plo);
}

// The fixed summation tree over 64 slots: slot k += slot k + s for
// s = 32, 16, ..., 1; the sum ends in lane 0.
__device__ __forceinline__ double tree_sum(double t)
{
    t = tree_level_swap<32>(t);
    t = tree_level_swap<16>(t);
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

// Value of lane `src` of the wave (once per sweep).
__device__ __forceinline__ float from_lane(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src * 4, __float_as_int(v)));
}

__device__ __forceinline__ uint32_t from_lane_u32(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src * 4, (int)v);
}

__device__ __forceinline__ double from_lane_f64(double v, int src)
{
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = from_lane_u32((uint32_t)u, src), hi = from_lane_u32((uint32_t)(u >> 32), src);
    return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

// Rotation parameter of a 24-bit word: u = (k - (2^23 - 1/2)) / 2^23 in
// (-1, 1), tau = u / (1 - |u|); the mirrored word gives -tau.
__device__ __forceinline__ double rot_tau(uint32_t w)
{
    const double u = ((double)(w >> 8) - 8388607.5) / 8388608.0;
    return u / (1.0 - __builtin_fabs(u));
}

// v' = R v for the quaternion (w, a) (not normalised): |q|^2 R applied to v,
// divided by |q|^2; every product and sum in the order written.
__device__ __forceinline__ void quat_rotate(double w, double x, double y, double z, double vx, double vy, double vz,
                                            double &ox, double &oy, double &oz)
{
    const double ww = w * w, xx = x * x, yy = y * y, zz = z * z;
    const double n2 = ((ww + xx) + yy) + zz;
    const double m00 = ((ww + xx) - yy) - zz, m11 = ((ww - xx) + yy) - zz, m22 = ((ww - xx) - yy) + zz;
    const double m01 = 2.0 * (x * y - w * z), m02 = 2.0 * (x * z + w * y);
    const double m10 = 2.0 * (x * y + w * z), m12 = 2.0 * (y * z - w * x);
    const double m20 = 2.0 * (x * z - w * y), m21 = 2.0 * (y * z + w * x);
    ox = ((m00 * vx + m01 * vy) + m02 * vz) / n2;
    oy = ((m10 * vx + m11 * vy) + m12 * vz) / n2;
    oz = ((m20 * vx + m21 * vy) + m22 * vz) / n2;
}

// Pair-term cache (CACHE): the Lennard-Jones energy of every pair (a, b),
// a < b, of the wave's chain at the current positions, in LDS at slot
// f(a) + b with f(a) = a N - a (a + 1) / 2 - a - 1 (the upper triangle row
// by row).  A value depends only on the two positions and the pair's
// squared distance is the same number whichever bead is the moving one, so
// a cached term equals a recomputed one bit for bit.
__host__ __device__ inline int pair_row(int a, int N) { return a * N - a * (a + 1) / 2 - a - 1; }
__host__ __device__ inline int pair_slots(int N) { return N * (N - 1) / 2; }

// One chain per wavefront.  Lane j holds bead j and, with TWO (64 < N <= 128),
// bead j + 64 (register set 1).  A pair sum slot is lane j's term plus, with
// TWO, the term of bead j + 64.  MOVES: the paper's full move set (a
// separate variant, so the shift-only kernel carries none of its registers).
// CACHE (N <= 64 only): a shift or rotation reads the old pair term from the
// cache instead of recomputing it, and an accepted move writes the new ones;
// an accepted double bridging renumbers beads and refills the cache.
template <bool TWO, bool MOVES, bool CACHE>
__global__ __launch_bounds__(256) void polymer_sweeps(PolymerArgs a, PolyParams p)
{
    static_assert(!CACHE || !TWO, "the pair cache serves N <= 64");
    extern __shared__ uint32_t lhist[];
    for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x)
        lhist[i] = 0u;
    __syncthreads();

    constexpr int NS = TWO ? 2 : 1; // beads per lane
    constexpr int SLOTS = 64 * NS;  // bead slots per chain in memory
    const int j = (int)(threadIdx.x & 63u);
    const int c = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int N = a.n_beads;
    float4 *pos = a.pos + (size_t)c * SLOTS;
    double *bond = a.bond + (size_t)c * SLOTS;
    float4 x[NS];
    // the shift-only kernel for N <= 64 also keeps x in FP64 for the pair
    // distances (the other variants have no registers to spare for it)
    constexpr bool XD = !TWO && !MOVES;
    double xd[NS], yd[NS], zd[NS];
    auto own_d2 = [&](int s, float bx, float by, float bz) {
        if constexpr (XD)
            return dist2d(xd[s], yd[s], zd[s], bx, by, bz);
        else
            return dist2(x[s].x, x[s].y, x[s].z, bx, by, bz);
    };
    auto set_xd = [&](int s) {
        if constexpr (XD)
            xd[s] = x[s].x, yd[s] = x[s].y, zd[s] = x[s].z;
    };
    double ub[NS]; // energy of bond (bead, bead + 1)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int bd = j + 64 * s;
        x[s] = bd < N ? pos[bd] : make_float4(0.f, 0.f, 0.f, 0.f);
        set_xd(s);
        ub[s] = bd < N - 1 ? bond[bd] : 0.0;
    }
    double E = a.energy[c];
    int32_t b = a.bins[c];
    const uint32_t chain = (uint32_t)(a.chain0 + c);
    const bool counts = a.record && c < a.n_chains && j == 0;
    const uint32_t B = (uint32_t)a.n_bins;
    const int up_l = (j + 1) & 63, dn_l = (j + 63) & 63;
    uint64_t nacc = 0u; // accepted moves of the recorded sweeps (wave-uniform)
    // CACHE: the wave's pair terms; lane j's slot for the moving bead i is
    // f(j) + i when j < i and f(i) + j when j > i
    double *cache = nullptr;
    int c_lo = 0;
    // every pair term at the current positions; the lanes of one wave
    // exchange terms through LDS, whose accesses from one wave complete in
    // order: the fence only keeps the compiler from moving them
    auto fill_cache = [&]() {
        for (int k = 0; k + 2 < N; ++k) {
            const float kx = readlane_f32(x[0].x, k), ky = readlane_f32(x[0].y, k), kz = readlane_f32(x[0].z, k);
            if (j >= k + 2 && j < N)
                cache[pair_row(k, N) + j] = lj_energy(p, own_d2(0, kx, ky, kz));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    if constexpr (CACHE) {
        cache = (double *)(lhist + ((a.n_bins + 1) & ~1)) + (size_t)(threadIdx.x >> 6) * pair_slots(N);
        c_lo = pair_row(j, N);
        fill_cache();
    }

    for (int s_ = 0; s_ < a.n_sweeps; ++s_) {
        const uint32_t g = a.g0 + (uint32_t)s_;
        float pnx[NS], pny[NS], pnz[NS];
        uint32_t racc[NS], flags[NS];
        double f_fwd[NS], f_rej[NS], f_acc[NS];
        // Each bead's proposal: no earlier move of the sweep changes the bead.
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const Words4 w = philox4x32_10(chain, g, (uint32_t)(j + 64 * s), kTagSweep, a.k0, a.k1);
            pnx[s] = x[s].x + ((float)(w.w[0] >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
            pny[s] = x[s].y + ((float)(w.w[1] >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
            pnz[s] = x[s].z + ((float)(w.w[2] >> 8) * 5.9604644775390625e-08f - 0.5f) * a.step;
            racc[s] = min(w.w[3], 0xFFFFFFFEu); // accept iff racc < T
        }
        // The new bond energies of each bead's move, all known now: bead + 1
        // has not moved when the bead moves, and bead - 1 sits either where
        // the sweep found it (its move rejected) or at its proposal
        // (accepted).  Bonds whose stretch leaves the FENE domain are flagged.
        float rx[NS], ry[NS], rz[NS], lx[NS], ly[NS], lz[NS], qx[NS], qy[NS], qz[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            rx[s] = from_lane(x[s].x, up_l), ry[s] = from_lane(x[s].y, up_l), rz[s] = from_lane(x[s].z, up_l);
            lx[s] = from_lane(x[s].x, dn_l), ly[s] = from_lane(x[s].y, dn_l), lz[s] = from_lane(x[s].z, dn_l);
            qx[s] = from_lane(pnx[s], dn_l), qy[s] = from_lane(pny[s], dn_l), qz[s] = from_lane(pnz[s], dn_l);
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int bd = j + 64 * s;
            // bead + 1 is in the next lane of the same set, or lane 0 of the next set
            const int rs = (j == 63) ? s + 1 : s;
            // bead - 1 is in the previous lane of the same set, or lane 63 of the previous set
            const int ls = (j == 0) ? s - 1 : s;
            f_fwd[s] = f_rej[s] = f_acc[s] = 0.0;
            flags[s] = 0u; // bit 0: forward broken, 1: back broken (rejected), 2: back broken (accepted)
            if (bd + 1 < N && rs < NS) {
                bool br = false;
                const float ax = rs == s ? rx[s] : rx[NS - 1], ay = rs == s ? ry[s] : ry[NS - 1],
                            az = rs == s ? rz[s] : rz[NS - 1];
                f_fwd[s] = fene_energy(p, dist2(ax, ay, az, pnx[s], pny[s], pnz[s]), &br);
                flags[s] |= br ? 1u : 0u;
            }
            if (bd >= 1 && bd < N && ls >= 0) {
                bool br = false, ba = false;
                const float ax = ls == s ? lx[s] : lx[0], ay = ls == s ? ly[s] : ly[0], az = ls == s ? lz[s] : lz[0];
                const float bx = ls == s ? qx[s] : qx[0], by = ls == s ? qy[s] : qy[0], bz = ls == s ? qz[s] : qz[0];
                f_rej[s] = fene_energy(p, dist2(ax, ay, az, pnx[s], pny[s], pnz[s]), &br);
                f_acc[s] = fene_energy(p, dist2(bx, by, bz, pnx[s], pny[s], pnz[s]), &ba);
                flags[s] |= (br ? 2u : 0u) | (ba ? 4u : 0u);
            }
        }
        bool prev_acc = false;
        for (int i = 0; i < N; ++i) {
            const int li = i & 63;
            const bool hi = TWO && i >= 64; // the moving bead's register set
            auto pick = [&](auto v0, auto v1) { return hi ? v1 : v0; };
            const float nx = readlane_f32(pick(pnx[0], pnx[NS - 1]), li);
            const float ny = readlane_f32(pick(pny[0], pny[NS - 1]), li);
            const float nz = readlane_f32(pick(pnz[0], pnz[NS - 1]), li);
            const float xi = readlane_f32(pick(x[0].x, x[NS - 1].x), li);
            const float yi = readlane_f32(pick(x[0].y, x[NS - 1].y), li);
            const float zi = readlane_f32(pick(x[0].z, x[NS - 1].z), li);
            const uint32_t w3 = __builtin_amdgcn_readlane(pick(racc[0], racc[NS - 1]), li);
            const uint32_t fl = __builtin_amdgcn_readlane(pick(flags[0], flags[NS - 1]), li);
            const double fb_i = readlane_f64(prev_acc ? pick(f_acc[0], f_acc[NS - 1]) : pick(f_rej[0], f_rej[NS - 1]),
                                             li);                       // new bond (i - 1, i)
            const double ff_i = readlane_f64(pick(f_fwd[0], f_fwd[NS - 1]), li); // new bond (i, i + 1)
            const double ub_i = readlane_f64(pick(ub[0], ub[NS - 1]), li);       // bond (i, i + 1), before
            double t = 0.0;
            double lnew = 0.0; // CACHE: this lane's new pair term
            int slot = 0;
            const bool paired = j < N && (j > i + 1 || j + 1 < i);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int bd = j + 64 * s;
                const int sep = bd > i ? bd - i : i - bd;
                double ts = 0.0;
                if (bd < N && sep >= 2) {
                    if constexpr (CACHE) {
                        slot = bd < i ? c_lo + i : pair_row(i, N) + bd;
                        const double old = cache[slot];
                        lnew = lj_energy(p, own_d2(s, nx, ny, nz));
                        // the read first, its latency covered by the new term
                        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                        __builtin_amdgcn_sched_group_barrier(0x2, 200, 0);
                        ts = lnew - old;
                    } else {
                        const double r2n = own_d2(s, nx, ny, nz);
                        const double r2o = own_d2(s, xi, yi, zi);
                        ts = lj_energy(p, r2n) - lj_energy(p, r2o);
                    }
                }
                if (bd == i + 1)
                    ts = ff_i - ub_i;
                if (bd == i - 1)
                    ts = fb_i - ub[s];
                t = s == 0 ? ts : t + ts;
            }
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
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int bd = j + 64 * s;
                    if (bd == i) {
                        x[s].x = nx;
                        x[s].y = ny;
                        x[s].z = nz;
                        set_xd(s);
                        if (i + 1 < N)
                            ub[s] = ff_i;
                    }
                    if (bd == i - 1)
                        ub[s] = fb_i;
                }
                if constexpr (CACHE) {
                    if (paired)
                        cache[slot] = lnew;
                }
                E = En;
                b = bn;
                nacc += a.record ? 1u : 0u;
            }
            if constexpr (CACHE)
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            prev_acc = acc;
        }
        if constexpr (MOVES) {
            // position of bead k, the same in every lane
            auto bead = [&](int k, float &px, float &py, float &pz) {
                const int l = k & 63;
                const bool h = TWO && k >= 64;
                px = readlane_f32(h ? x[NS - 1].x : x[0].x, l);
                py = readlane_f32(h ? x[NS - 1].y : x[0].y, l);
                pz = readlane_f32(h ? x[NS - 1].z : x[0].z, l);
            };
            auto bond_of = [&](int k) { return readlane_f64((TWO && k >= 64) ? ub[NS - 1] : ub[0], k & 63); };
            // spherical rotations, beads 0..N-1 in order
            for (int i = 0; i < N; ++i) {
                const Words4 w = philox4x32_10(chain, g, (uint32_t)i, kTagRotate, a.k0, a.k1);
                float xi, yi, zi, lx = 0.f, ly = 0.f, lz = 0.f, rx = 0.f, ry = 0.f, rz = 0.f;
                bead(i, xi, yi, zi);
                if (i >= 1)
                    bead(i - 1, lx, ly, lz);
                if (i + 1 < N)
                    bead(i + 1, rx, ry, rz);
                double ax, ay, az, cx, cy, cz;
                if (i > 0 && i < N - 1) { // about the line through both neighbours
                    ax = (double)rx - (double)lx;
                    ay = (double)ry - (double)ly;
                    az = (double)rz - (double)lz;
                    cx = lx, cy = ly, cz = lz;
                } else { // an end bead: about a coordinate axis through its neighbour
                    const uint32_t axis = (uint32_t)(((uint64_t)w.w[1] * 3u) >> 32);
                    ax = axis == 0u ? 1.0 : 0.0;
                    ay = axis == 1u ? 1.0 : 0.0;
                    az = axis == 2u ? 1.0 : 0.0;
                    cx = i == 0 ? rx : lx, cy = i == 0 ? ry : ly, cz = i == 0 ? rz : lz;
                }
                double ox, oy, oz;
                quat_rotate(rot_tau(w.w[0]), ax, ay, az, (double)xi - cx, (double)yi - cy, (double)zi - cz, ox, oy,
                            oz);
                const float nx = (float)(cx + ox), ny = (float)(cy + oy), nz = (float)(cz + oz);
                bool brl = false, brr = false;
                const double fl = i >= 1 ? fene_energy(p, dist2(lx, ly, lz, nx, ny, nz), &brl) : 0.0;
                const double fr = i + 1 < N ? fene_energy(p, dist2(rx, ry, rz, nx, ny, nz), &brr) : 0.0;
                const double ub_i = bond_of(i);
                double t = 0.0;
                double lnew = 0.0; // CACHE: this lane's new pair term
                int slot = 0;
                const bool paired = j < N && (j > i + 1 || j + 1 < i);
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int bd = j + 64 * s;
                    const int sep = bd > i ? bd - i : i - bd;
                    double ts = 0.0;
                    if (bd < N && sep >= 2) {
                        if constexpr (CACHE) {
                            slot = bd < i ? c_lo + i : pair_row(i, N) + bd;
                            const double old = cache[slot];
                            lnew = lj_energy(p, own_d2(s, nx, ny, nz));
                            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                            __builtin_amdgcn_sched_group_barrier(0x2, 200, 0);
                            ts = lnew - old;
                        } else {
                            const double r2n = own_d2(s, nx, ny, nz);
                            const double r2o = own_d2(s, xi, yi, zi);
                            ts = lj_energy(p, r2n) - lj_energy(p, r2o);
                        }
                    }
                    if (bd == i + 1)
                        ts = fr - ub_i;
                    if (bd == i - 1)
                        ts = fl - ub[s];
                    t = s == 0 ? ts : t + ts;
                }
                const double dE = readlane_f64(tree_sum(t), 0);
                const double En = E + dE;
                const int32_t bn = energy_bin(p, En, a.n_bins);
                bool acc = false;
                if (!brl && !brr && bn >= 0)
                    acc = min(w.w[3], 0xFFFFFFFEu) < a.thresholds[(size_t)b * B + (uint32_t)bn];
                if (acc) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        const int bd = j + 64 * s;
                        if (bd == i) {
                            x[s].x = nx;
                            x[s].y = ny;
                            x[s].z = nz;
                            set_xd(s);
                            if (i + 1 < N)
                                ub[s] = fr;
                        }
                        if (bd == i - 1)
                            ub[s] = fl;
                    }
                    if constexpr (CACHE) {
                        if (paired)
                            cache[slot] = lnew;
                    }
                    E = En;
                    b = bn;
                    nacc += a.record ? 1u : 0u;
                }
                if constexpr (CACHE)
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
            // one double bridging: bonds (bi, bi+1), (bj, bj+1) -> (bi, bj), (bi+1, bj+1)
            const Words4 w = philox4x32_10(chain, g, 0u, kTagBridge, a.k0, a.k1);
            int bi = (int)(((uint64_t)w.w[0] * (uint64_t)(N - 1)) >> 32);
            int bj = (int)(((uint64_t)w.w[1] * (uint64_t)(N - 1)) >> 32);
            if (bi > bj) {
                const int tmp = bi;
                bi = bj;
                bj = tmp;
            }
            if (N >= 4 && bj - bi >= 2) {
                float ix, iy, iz, kx, ky, kz, jx, jy, jz, mx, my, mz; // beads bi, bi+1, bj, bj+1
                bead(bi, ix, iy, iz);
                bead(bi + 1, kx, ky, kz);
                bead(bj, jx, jy, jz);
                bead(bj + 1, mx, my, mz);
                bool br = false;
                const double fij = fene_energy(p, dist2(ix, iy, iz, jx, jy, jz), &br);
                const double fkl = fene_energy(p, dist2(kx, ky, kz, mx, my, mz), &br);
                if (!br) {
                    const double fik = bond_of(bi), fjl = bond_of(bj);
                    const double lij = lj_energy(p, dist2(ix, iy, iz, jx, jy, jz));
                    const double lkl = lj_energy(p, dist2(kx, ky, kz, mx, my, mz));
                    const double lik = lj_energy(p, dist2(ix, iy, iz, kx, ky, kz));
                    const double ljl = lj_energy(p, dist2(jx, jy, jz, mx, my, mz));
                    const double dF = ((fij + fkl) - fik) - fjl;
                    const double dL = ((lik + ljl) - lij) - lkl;
                    const double En = E + (dF + dL);
                    const int32_t bn = energy_bin(p, En, a.n_bins);
                    if (bn >= 0 && min(w.w[3], 0xFFFFFFFEu) < a.thresholds[(size_t)b * B + (uint32_t)bn]) {
                        // beads bi+1 .. bj in reverse order; the bonds between them reversed
                        float4 nxs[NS];
                        double nub[NS];
#pragma unroll
                        for (int s = 0; s < NS; ++s) {
                            const int bd = j + 64 * s;
                            const int sx = (bd > bi && bd <= bj) ? bi + 1 + bj - bd : bd;
                            const int su = (bd > bi && bd < bj) ? bi + bj - bd : bd;
                            float4 v0, v1 = make_float4(0.f, 0.f, 0.f, 0.f);
                            v0.x = from_lane(x[0].x, sx & 63), v0.y = from_lane(x[0].y, sx & 63);
                            v0.z = from_lane(x[0].z, sx & 63), v0.w = 0.f;
                            double u0 = from_lane_f64(ub[0], su & 63), u1 = 0.0;
                            if constexpr (TWO) {
                                v1.x = from_lane(x[NS - 1].x, sx & 63), v1.y = from_lane(x[NS - 1].y, sx & 63);
                                v1.z = from_lane(x[NS - 1].z, sx & 63);
                                u1 = from_lane_f64(ub[NS - 1], su & 63);
                            }
                            nxs[s] = sx >= 64 ? v1 : v0;
                            nub[s] = su >= 64 ? u1 : u0;
                            if (bd == bi)
                                nub[s] = fij;
                            if (bd == bj)
                                nub[s] = fkl;
                        }
#pragma unroll
                        for (int s = 0; s < NS; ++s) {
                            x[s] = nxs[s];
                            set_xd(s);
                            ub[s] = nub[s];
                        }
                        if constexpr (CACHE)
                            fill_cache(); // the pair terms under the new numbering
                        E = En;
                        b = bn;
                        nacc += a.record ? 1u : 0u;
                    }
                }
            }
        }
        if (counts)
            atomicAdd(&lhist[b], 1u);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int bd = j + 64 * s;
        if (bd < N)
            pos[bd] = x[s];
        if (bd < N - 1)
            bond[bd] = ub[s];
    }
    if (j == 0) {
        a.energy[c] = E;
        a.bins[c] = b;
        if (counts && a.accepts && nacc)
            atomicAdd(a.accepts, (unsigned long long)nacc);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.n_bins; i += blockDim.x) {
        const uint32_t v = lhist[i];
        if (v)
            atomicAdd(&a.hist[i], (unsigned long long)v);
    }
}

// The cache is used when four blocks of it still fit one CU's 160 KB of
// LDS: the occupancy the kernel without it reaches at one chain per wave
// and four waves per SIMD.
static bool polymer_pair_cache_fits(size_t lds_bytes) { return lds_bytes * 4u <= 160u * 1024u; }

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
    const size_t lds = (size_t)a.n_bins * 4u;
    const size_t lds_cached = (size_t)((a.n_bins + 1) & ~1) * 4u + (size_t)chains_per_block * pair_slots(a.n_beads) * 8u;
    if (a.n_beads > 64) {
        if (a.moves)
            hipLaunchKernelGGL((polymer_sweeps<true, true, false>), grid, block, lds, s, a, p);
        else
            hipLaunchKernelGGL((polymer_sweeps<true, false, false>), grid, block, lds, s, a, p);
    } else if (a.moves) {
        if (polymer_pair_cache_fits(lds_cached))
            hipLaunchKernelGGL((polymer_sweeps<false, true, true>), grid, block, lds_cached, s, a, p);
        else
            hipLaunchKernelGGL((polymer_sweeps<false, true, false>), grid, block, lds, s, a, p);
    } else if (polymer_pair_cache_fits(lds_cached)) {
        hipLaunchKernelGGL((polymer_sweeps<false, false, true>), grid, block, lds_cached, s, a, p);
    } else {
        hipLaunchKernelGGL((polymer_sweeps<false, false, false>), grid, block, lds, s, a, p);
    }
    return hipGetLastError();
}

} // namespace muca
