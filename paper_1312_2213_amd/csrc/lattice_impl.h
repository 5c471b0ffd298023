// lattice_impl.h -- Metropolis sweeps of many independent 2D lattice chains that
// share one multicanonical weight table (gfx950).
//
// Method (arXiv:1312.2213): every realisation runs single-site updates with
// the weight W(E) of Eq. 1 (Ising H = -sum s_i s_j, Potts
// H = -sum delta(s_i, s_j)) or, for the multimagnetic ensemble of Eq. 3, the
// weight exp(-beta E) W(M); after each sweep the chain's bin is added to the
// histogram that is merged over all chains (parallel-scheme paragraph).
//
// Mapping to the hardware:
//  * one chain per lane; a wavefront runs 64 chains in lockstep on the same
//    site, so the lattice words of 64 chains are 64 consecutive dwords;
//  * a sweep streams the lattice row by row through registers: rows y-1, y,
//    y+1 are held in VGPRs and row y+3 is prefetched while y is processed;
//    every site update works on registers with compile-time bit positions;
//  * Metropolis acceptance is one integer compare against a threshold
//    T[bin][column] (staged in LDS when it fits), so no exp() is evaluated;
//  * the per-block histogram lives in LDS (u32) and is added to the global
//    u64 histogram with atomics once per launch.
#pragma once
#include <utility>

#include "muca_internal.h"
#include "philox.h"

namespace muca {

template <int L, int LAYOUT>
struct Geom {
    static constexpr int kBits = LAYOUT == kLayoutBit ? 1 : 8;
    static constexpr int kSpw = 32 / kBits;
    static constexpr int kWpr = (L + kSpw - 1) / kSpw;
};

template <int MODEL>
struct Cols {
    static constexpr int value = MODEL == kIsing ? 5 : (MODEL == kPotts ? 9 : 10);
};

// Spin code of site x of a row: BIT layout -> the bit (1 = +1); BYTE layout
// (int8 +-1) -> the sign bit (1 = -1).  Equal codes <=> equal spins.
template <int L, int LAYOUT, int W>
__device__ __forceinline__ uint32_t spin_code(const uint32_t (&R)[W], int x)
{
    using G = Geom<L, LAYOUT>;
    if (LAYOUT == kLayoutBit)
        return (R[x / G::kSpw] >> (x % G::kSpw)) & 1u;
    return (R[x / G::kSpw] >> ((x % G::kSpw) * 8 + 7)) & 1u;
}

template <int L, int W>
__device__ __forceinline__ uint32_t colour(const uint32_t (&R)[W], int x)
{
    return (R[x / 4] >> ((x % 4) * 8)) & 0xFFu;
}

// ---------------------------------------------------------------------------
// Random words of one row.  With LPC lanes per chain, lane j of a chain's
// group computes the Philox calls j, j + LPC, ... of the row and every site
// reads its word from the owning lane by a DPP broadcast (quad_perm within
// quads, row_newbcast within rows of 16).  The counters, and so the words,
// are those of the one-lane-per-chain order.
// ---------------------------------------------------------------------------
template <int L, int LPC, int WPS>
struct RowRng {
    static constexpr int kSpc = 4 / WPS;                       // sites per Philox call
    static constexpr int kCalls = L / kSpc;                    // calls per row
    static constexpr int kPerLane = (kCalls + LPC - 1) / LPC;  // calls per lane
    uint32_t w[kPerLane * 4];

    __device__ __forceinline__ void fill(uint32_t chain, uint32_t g, int y, uint32_t j, uint32_t k0, uint32_t k1)
    {
#pragma unroll
        for (int m = 0; m < kPerLane; ++m) {
            uint32_t call = j + (uint32_t)(LPC * m);
            if (kCalls % LPC)
                call = call < (uint32_t)kCalls ? call : (uint32_t)kCalls - 1u; // surplus lanes: any valid call
            const Words4 r = philox4x32_10(chain, g, (uint32_t)(y * kCalls) + call, kTagSweep, k0, k1);
            // acceptance words are clamped to 2^32 - 2 once here, so that
            // "accept iff T == 2^32 - 1 or r < T" is the single compare r < T
#pragma unroll
            for (int t = 0; t < 4; ++t)
                w[4 * m + t] = (WPS == 1 || (t & 1)) ? min(r.w[t], 0xFFFFFFFEu) : r.w[t];
        }
    }

    // word WI (0..WPS-1) of site X of the row
    template <int X, int WI>
    __device__ __forceinline__ uint32_t get() const
    {
        constexpr int call = X / kSpc;
        constexpr int src = call % LPC;
        constexpr int reg = (call / LPC) * 4 + (X % kSpc) * WPS + WI;
        if constexpr (LPC == 1) {
            return w[reg];
        } else if constexpr (LPC == 2) {
            constexpr int pat = src | (src << 2) | ((2 + src) << 4) | ((2 + src) << 6);
            return (uint32_t)__builtin_amdgcn_mov_dpp((int)w[reg], pat, 0xF, 0xF, false);
        } else if constexpr (LPC == 4) {
            return (uint32_t)__builtin_amdgcn_mov_dpp((int)w[reg], src * 0x55, 0xF, 0xF, false);
        } else {
            static_assert(LPC == 16, "lanes per chain: 1, 2, 4 or 16");
            return (uint32_t)__builtin_amdgcn_mov_dpp((int)w[reg], 0x150 + src, 0xF, 0xF, false);
        }
    }
};

// value of lane O of the chain's lane group
template <int LPC, int O>
__device__ __forceinline__ uint32_t group_bcast(uint32_t v)
{
    if constexpr (LPC == 4)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, O * 0x55, 0xF, 0xF, false);
    else
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x150 + O, 0xF, 0xF, false);
}

// value of the previous / next lane of the group, cyclic
template <int LPC>
__device__ __forceinline__ uint32_t group_prev(uint32_t v)
{
    if constexpr (LPC == 4)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x93, 0xF, 0xF, false); // quad_perm [3,0,1,2]
    else
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x121, 0xF, 0xF, false); // row_ror:1
}

template <int LPC>
__device__ __forceinline__ uint32_t group_next(uint32_t v)
{
    if constexpr (LPC == 4)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x39, 0xF, 0xF, false); // quad_perm [1,2,3,0]
    else
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x12F, 0xF, 0xF, false); // row_ror:15
}

// ---------------------------------------------------------------------------
// Ising / MUMA.  Rows are held bit-packed in registers whatever the storage
// layout (bit 1 = spin +1, W1 = ceil(L/32) words, unused high bits zero).
// Before the sites of a word are visited, the misalignment of every site
// with its right, up and down neighbours is counted bit-parallel into two bit
// planes (s0 = parity, s1 = majority), and with its left neighbour into ML.
// None of these neighbours changes before the site's own attempt, except the
// left one (the previous site), whose flip f is folded in per site; and, for
// a row of one word, the right neighbour of the last site (site 0 of the
// same row), which is read from the current word.
// ---------------------------------------------------------------------------
template <int L>
struct Row1 {
    static constexpr int W = (L + 31) / 32;
};

// Four times the number of misaligned neighbours of site K of word WI,
// given the flip f of the previous site of the word (K > 0).  For a row of
// one word, the last site's right neighbour is site 0 of the same word, read
// from its current value.
// f4 is the previous site's flip times 4 (0 or 4).
template <int L, int WI, int K>
__device__ __forceinline__ int32_t misaligned4(uint32_t S, uint32_t F, uint32_t s0, uint32_t s1, uint32_t ML,
                                               uint32_t MU, uint32_t MD, uint32_t f4)
{
    constexpr int X = 32 * WI + K;
    uint32_t ml4 = ((ML >> K) & 1u) << 2;
    if constexpr (K > 0)
        ml4 ^= f4;
    if constexpr (Row1<L>::W == 1 && X == L - 1 && L > 1) {
        const uint32_t mr = ((S >> K) & 1u) ^ ((S ^ F) & 1u);
        return (int32_t)(((mr + ((MU >> K) & 1u) + ((MD >> K) & 1u)) << 2) + ml4);
    } else {
        return (int32_t)((((((s1 >> K) & 1u) << 1) + ((s0 >> K) & 1u)) << 2) + ml4);
    }
}

// Threshold address of a site with nmis4 = 4 x misaligned neighbours,
// relative to the current bin's row origin `rowb` (bytes):
//   Ising: column 4 - nmis (aligned neighbours); origin = column 4.
//   MUMA:  column 2 (4 - nmis) + plus;         origin = column 8.
template <int MODEL>
__device__ __forceinline__ int32_t col_addr(int32_t rowb, int32_t nmis4, uint32_t plus)
{
    if constexpr (MODEL == kIsing)
        return rowb - nmis4;
    else
        return rowb + (int32_t)(plus << 2) - 2 * nmis4;
}

template <int MODEL>
constexpr int32_t row_origin() { return MODEL == kIsing ? 4 : 8; }

typedef __attribute__((address_space(3))) const uint32_t lds_u32;

// Lattice words, bins and global threshold tables are global memory.  Typed
// as such, their loads and stores are global (not flat) operations also where
// the sweep runs inside a non-inlined function (the batched launch), whose
// pointer arguments the compiler cannot place: a flat operation counts
// against the LDS wait counter, which the site loop waits on for its
// threshold reads.
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) int32_t gi32;
typedef __attribute__((address_space(1))) uint8_t gu8;
typedef __attribute__((address_space(1))) unsigned long long gu64;

// Relaxed device-scope add to a global 64-bit counter.
__device__ __forceinline__ void gadd(gu64 *p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Threshold at `addr`: an absolute LDS byte address when the table is staged
// in LDS, else a byte offset from the global table.
template <bool TLDS>
__device__ __forceinline__ uint32_t load_t(const uint32_t *__restrict__ T, int32_t addr)
{
    if constexpr (TLDS)
        return *(lds_u32 *)(uintptr_t)(uint32_t)addr;
    else
        return *(const gu32 *)((uintptr_t)T + (intptr_t)addr);
}

// Byte shift of the row origin when a site with nmis4 = 4 x misaligned
// neighbours flips: Ising dE = 4 (n_al - 2), one bin per 4; MUMA M changes by
// -2 s_i, one bin per 2.
template <int MODEL>
__device__ __forceinline__ int32_t bin_step(int32_t nmis4, uint32_t plus)
{
    constexpr int NC = Cols<MODEL>::value;
    if constexpr (MODEL == kIsing)
        return nmis4 * (-NC) + 8 * NC;
    else
        return plus ? -4 * NC : 4 * NC;
}

// Site K of word WI.  `addr` (threshold address) and `dstep` (row-origin
// shift on acceptance) of this site were selected when the previous site was
// decided.  While this site's threshold read is in flight, both candidates
// for the next site (this site rejected / accepted) are computed from the bit
// planes, so after the compare a single select yields the next address: the
// loop-carried chain is LDS read -> compare -> select.
template <int MODEL, int L, int LPC, bool TLDS, int WI, int K>
__device__ __forceinline__ void ising_site(uint32_t &F, int32_t &rowb, int32_t &addr, int32_t &dstep,
                                           const RowRng<L, LPC, 1> &rng, uint32_t S, uint32_t s0, uint32_t s1,
                                           uint32_t ML, uint32_t MU, uint32_t MD, const uint32_t *__restrict__ T)
{
    constexpr int X = 32 * WI + K;
    constexpr int NB = (L - 32 * WI) < 32 ? (L - 32 * WI) : 32;
    const uint32_t t = load_t<TLDS>(T, addr);
    const uint32_t r = rng.template get<X, 0>(); // clamped: accept iff r < T
    const int32_t rowb_acc = rowb + dstep;
    int32_t addr0 = 0, addr1 = 0, dstep0 = 0, dstep1 = 0;
    if constexpr (K + 1 < NB) {
        const uint32_t plus1 = (S >> (K + 1)) & 1u;
        const int32_t n0 = misaligned4<L, WI, K + 1>(S, F, s0, s1, ML, MU, MD, 0u);
        const int32_t n1 = misaligned4<L, WI, K + 1>(S, F, s0, s1, ML, MU, MD, 4u);
        addr0 = col_addr<MODEL>(rowb, n0, plus1);
        addr1 = col_addr<MODEL>(rowb_acc, n1, plus1);
        dstep0 = bin_step<MODEL>(n0, plus1);
        dstep1 = bin_step<MODEL>(n1, plus1);
    }
    const bool acc = r < t;
    F |= (acc ? 1u : 0u) << K;
    rowb = acc ? rowb_acc : rowb;
    if constexpr (K + 1 < NB) {
        addr = acc ? addr1 : addr0;
        dstep = acc ? dstep1 : dstep0;
    }
}

template <int MODEL, int L, int LPC, bool TLDS, int WI, int... K>
__device__ __forceinline__ void ising_word(const uint32_t (&up)[Row1<L>::W], uint32_t (&cur)[Row1<L>::W],
                                           const uint32_t (&dn)[Row1<L>::W], int32_t &rowb,
                                           const RowRng<L, LPC, 1> &rng, const uint32_t *__restrict__ T,
                                           std::integer_sequence<int, K...>)
{
    constexpr int W = Row1<L>::W;
    constexpr int NB = (L - 32 * WI) < 32 ? (L - 32 * WI) : 32; // sites in this word
    const uint32_t S = cur[WI];
    const uint32_t nextbit = (WI + 1 < W) ? (cur[WI + 1] & 1u) : (cur[0] & 1u);
    const uint32_t prevbit = (WI > 0) ? (cur[WI > 0 ? WI - 1 : 0] >> 31) : ((cur[W - 1] >> ((L - 1) % 32)) & 1u);
    const uint32_t Rn = (S >> 1) | (nextbit << (NB - 1));
    const uint32_t Ln = (S << 1) | prevbit;
    const uint32_t MR = S ^ Rn, MU = S ^ up[WI], MD = S ^ dn[WI], ML = S ^ Ln;
    const uint32_t s0 = MR ^ MU ^ MD;
    const uint32_t s1 = (MR & MU) | (MR & MD) | (MU & MD);
    uint32_t F = 0u;
    const int32_t n = misaligned4<L, WI, 0>(S, 0u, s0, s1, ML, MU, MD, 0u);
    int32_t addr = col_addr<MODEL>(rowb, n, S & 1u);
    int32_t dstep = bin_step<MODEL>(n, S & 1u);
    (ising_site<MODEL, L, LPC, TLDS, WI, K>(F, rowb, addr, dstep, rng, S, s0, s1, ML, MU, MD, T), ...);
    cur[WI] = S ^ F;
}

template <int MODEL, int L, int LPC, bool TLDS, int... WI>
__device__ __forceinline__ void ising_row(const uint32_t (&up)[Row1<L>::W], uint32_t (&cur)[Row1<L>::W],
                                          const uint32_t (&dn)[Row1<L>::W], int32_t &rowb,
                                          const uint32_t *__restrict__ T, uint32_t chain, uint32_t g, int y,
                                          uint32_t j, uint32_t k0, uint32_t k1, std::integer_sequence<int, WI...>)
{
    RowRng<L, LPC, 1> rng;
    rng.fill(chain, g, y, j, k0, k1);
    (ising_word<MODEL, L, LPC, TLDS, WI>(up, cur, dn, rowb, rng, T,
                                         std::make_integer_sequence<int, ((L - 32 * WI) < 32 ? (L - 32 * WI) : 32)>{}),
     ...);
}

// ---------------------------------------------------------------------------
// Ising / MUMA with the per-site candidate work split over the lanes of a
// chain (4 or 16 lanes).  The lane that draws a site's Philox word (site X:
// call X / 4, lane (X / 4) % LPC) also builds, from bit planes of the row as
// it was when the row started, the site's descriptor: for both outcomes of
// the left neighbour's attempt, the site's bin step, and the next site's
// threshold offset for both outcomes of this site's own attempt (signed
// bytes).  The right, up and down neighbours of a site do not change before
// its attempt, except for the row's last site, whose right neighbour is site
// 0: the descriptors that involve it (sites L - 2 and L - 1) have a second
// variant for site 0 flipped.  The descriptor travels with the site's
// acceptance word in one 64-bit DPP broadcast, so a site costs: two selects
// of the bin rows (this site's and, if it flips, the next site's), two
// addresses and two reads of the next site's candidate thresholds, one
// broadcast, and select + compare of its own threshold, read one site
// earlier.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t sbyte(uint32_t v) { return (int32_t)(int8_t)(uint8_t)v; }

// value of lane O of the chain's lane group, 64 bits (one v_mov_b64 DPP with
// row_newbcast; two 32-bit quad permutes for groups of 4)
template <int LPC, int O>
__device__ __forceinline__ uint64_t group_bcast64(uint64_t v)
{
    if constexpr (LPC == 16)
        return __builtin_amdgcn_mov_dpp(v, 0x150 + O, 0xF, 0xF, false);
    else
        return (uint64_t)group_bcast<LPC, O>((uint32_t)v) | ((uint64_t)group_bcast<LPC, O>((uint32_t)(v >> 32)) << 32);
}

// two signed bytes: f(nA) | f(nB) << 8, for the site's misalignment count
// without (nA) and with (nB) the left neighbour's flip
template <int MODEL>
__device__ __forceinline__ uint32_t ilp_off2(uint32_t nA, uint32_t nB, uint32_t plus)
{
    const int32_t a = col_addr<MODEL>(0, (int32_t)(4u * nA), plus), b = col_addr<MODEL>(0, (int32_t)(4u * nB), plus);
    return ((uint32_t)a & 0xFFu) | (((uint32_t)b & 0xFFu) << 8);
}

template <int MODEL>
__device__ __forceinline__ uint32_t ilp_ds2(uint32_t nA, uint32_t nB, uint32_t plus)
{
    const int32_t a = bin_step<MODEL>((int32_t)(4u * nA), plus), b = bin_step<MODEL>((int32_t)(4u * nB), plus);
    return ((uint32_t)a & 0xFFu) | (((uint32_t)b & 0xFFu) << 8);
}

// (v << 1) | (this lane's bit of mask): one add with carry-in.  The mask is
// the lane mask written by a vector compare; inside the site loop that
// compare is a scheduling region (four or more instructions) back, after the
// loop it may be the previous instruction, hence there the two wait states
// of an SGPR written by one VALU instruction and read by the next.
template <bool NEAR>
__device__ __forceinline__ uint32_t shift_in(uint32_t v, uint64_t mask)
{
    uint32_t out;
    if constexpr (NEAR)
        asm("s_nop 1\n\tv_addc_co_u32 %0, vcc, %1, %1, %2" : "=v"(out) : "v"(v), "s"(mask) : "vcc");
    else
        asm("v_addc_co_u32 %0, vcc, %1, %1, %2" : "=v"(out) : "v"(v), "s"(mask) : "vcc");
    return out;
}

// (descriptor, acceptance word) of site X as every lane of the chain sees it
template <int L, int LPC, int X>
__device__ __forceinline__ uint64_t ilp_get(const uint64_t (&pk)[RowRng<L, LPC, 1>::kPerLane * 4], uint32_t dv2,
                                            uint32_t dv1, bool f0)
{
    constexpr int call = X / 4, O = call % LPC, R = (call / LPC) * 4 + X % 4;
    uint64_t v = group_bcast64<LPC, O>(pk[R]);
    if constexpr (X == L - 2 || X == L - 1) {
        const uint32_t alt = group_bcast<LPC, O>(X == L - 2 ? dv2 : dv1); // site 0 flipped
        v = f0 ? ((v & 0xFFFFFFFF00000000ull) | alt) : v;
    }
    return v;
}

// Site X.  On entry: B = bin row (byte origin) before the site's attempt if
// the previous site was rejected, Bf = the same if it was accepted, prev =
// that outcome, (t0, t1) = the site's threshold in either case (read one
// site earlier), cur = the site's (descriptor, word).
template <int MODEL, int L, int LPC, bool TLDS, int X>
__device__ __forceinline__ void ilp_site(const uint64_t (&pk)[RowRng<L, LPC, 1>::kPerLane * 4], uint32_t dv2,
                                         uint32_t dv1, int32_t &B, int32_t &Bf, uint64_t &cur, bool &prev, bool &f0,
                                         uint64_t &pm, uint32_t &t0, uint32_t &t1, uint32_t (&F)[Row1<L>::W],
                                         const uint32_t *__restrict__ T)
{
    const uint32_t D = (uint32_t)cur, r = (uint32_t)(cur >> 32); // r clamped: accept iff r < T
    const int32_t x0 = B + sbyte(D >> 16), x1 = Bf + sbyte(D >> 24);
    B = prev ? Bf : B;   // this site's bin row
    Bf = prev ? x1 : x0; // the next site's, if this one flips
    uint32_t n_t0 = 0u, n_t1 = 0u;
    if constexpr (X + 1 < L) {
        n_t0 = load_t<TLDS>(T, B + sbyte(D));
        n_t1 = load_t<TLDS>(T, Bf + sbyte(D >> 8));
    }
    // the previous site's flip record, while the reads are in flight: not
    // between the threshold select and the compare
    if constexpr (X > 0)
        F[(X - 1) / 32] = shift_in<false>(F[(X - 1) / 32], pm);
    // selected only now, after the next reads were issued (the barrier keeps
    // the wait for this site's reads one site behind them)
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t t = prev ? t1 : t0;
    t0 = n_t0;
    t1 = n_t1;
    // the next site's descriptor, broadcast beside the compare (this site's
    // descriptor is dead by now, and the reads above are a few instructions back)
    if constexpr (X + 1 < L)
        cur = ilp_get<L, LPC, X + 1>(pk, dv2, dv1, f0);
    const bool acc = r < t;
    if constexpr (X == 0)
        f0 = acc;
    pm = __builtin_amdgcn_ballot_w64(acc);
    prev = acc;
    __builtin_amdgcn_sched_barrier(0);
}

template <int MODEL, int L, int LPC, bool TLDS, int... X>
__device__ __forceinline__ void ilp_sites(const uint64_t (&pk)[RowRng<L, LPC, 1>::kPerLane * 4], uint32_t dv2,
                                          uint32_t dv1, uint32_t first, int32_t &rowb, uint32_t (&F)[Row1<L>::W],
                                          const uint32_t *__restrict__ T, std::integer_sequence<int, X...>)
{
    uint64_t cur = ilp_get<L, LPC, 0>(pk, dv2, dv1, false);
    uint32_t t0 = load_t<TLDS>(T, rowb + sbyte(group_bcast<LPC, 0>(first))), t1 = t0;
    int32_t B = rowb, Bf = rowb;
    bool prev = false, f0 = false;
    uint64_t pm = 0u;
    (ilp_site<MODEL, L, LPC, TLDS, X>(pk, dv2, dv1, B, Bf, cur, prev, f0, pm, t0, t1, F, T), ...);
    F[(L - 1) / 32] = shift_in<true>(F[(L - 1) / 32], pm);
    rowb = prev ? Bf : B;
}

template <int MODEL, int L, int LPC, bool TLDS>
__device__ __forceinline__ void ising_lp_row(const uint32_t (&up)[Row1<L>::W], uint32_t (&cur)[Row1<L>::W],
                                             const uint32_t (&dn)[Row1<L>::W], int32_t &rowb,
                                             const uint32_t *__restrict__ T, uint32_t chain, uint32_t g, int y,
                                             uint32_t j, uint32_t k0, uint32_t k1, uint32_t &nacc)
{
    static_assert(L % 4 == 0 && L >= 4, "rows of whole Philox calls");
    constexpr int W = Row1<L>::W;
    using R = RowRng<L, LPC, 1>;
    R rng;
    rng.fill(chain, g, y, j, k0, k1);
    // bit planes of the row as it started: misalignment with the right, up
    // and down neighbours (parity s0, majority s1), with the right one alone
    // (MR) and with the left one (ML); the spins themselves (S)
    uint32_t s0[W], s1[W], MR[W], ML[W];
#pragma unroll
    for (int wi = 0; wi < W; ++wi) {
        const int nb = (L - 32 * wi) < 32 ? (L - 32 * wi) : 32;
        const uint32_t S = cur[wi];
        const uint32_t nextbit = (wi + 1 < W) ? (cur[wi + 1 < W ? wi + 1 : 0] & 1u) : (cur[0] & 1u);
        const uint32_t prevbit = (wi > 0) ? (cur[wi > 0 ? wi - 1 : 0] >> 31) : ((cur[W - 1] >> ((L - 1) % 32)) & 1u);
        const uint32_t Rn = (S >> 1) | (nextbit << (nb - 1));
        const uint32_t Ln = (S << 1) | prevbit;
        const uint32_t mr = S ^ Rn, mu = S ^ up[wi], md = S ^ dn[wi];
        MR[wi] = mr;
        ML[wi] = S ^ Ln;
        s0[wi] = mr ^ mu ^ md;
        s1[wi] = (mr & mu) | (mr & md) | (mu & md);
    }
    // the five sites 4 call .. 4 call + 4 of each of this lane's calls: a
    // window of every plane starting at the call's first site
    auto window = [&](const uint32_t (&P)[W], uint32_t call) -> uint32_t {
        if constexpr (W == 1)
            return P[0] >> (4u * call);
        else
            return (uint32_t)((((uint64_t)P[1] << 32) | P[0]) >> (4u * call));
    };
    uint64_t pk[R::kPerLane * 4];
    uint32_t dv2 = 0u, dv1 = 0u, first = 0u;
#pragma unroll
    for (int m = 0; m < R::kPerLane; ++m) {
        uint32_t call = j + (uint32_t)(LPC * m);
        if (R::kCalls % LPC)
            call = call < (uint32_t)R::kCalls ? call : (uint32_t)R::kCalls - 1u;
        const uint32_t w0 = window(s0, call), w1 = window(s1, call), wl = window(ML, call), wr = window(MR, call),
                       ws = window(cur, call);
        const bool last = call == (uint32_t)R::kCalls - 1u;
        if constexpr (MODEL == kIsing || MODEL == kMuma) {
            // The offset and bin step of a site depend only on its
            // misalignment count n = 0..4 (Ising: -4n and 40 - 20n bytes) or
            // on n and its own spin (MUMA: 4 s - 8n and -40 / +40 for s = 1 /
            // 0), so the four sites of the call are done bytewise (byte k =
            // site k): table lookups by byte permutes, or byte arithmetic with
            // a bias of 0x80 per byte so that no byte borrows
            auto spread4 = [](uint32_t w) { return ((w & 0xFu) * 0x00204081u) & 0x01010101u; };
            const uint32_t b0 = spread4(w0), b1 = spread4(w1), bl = spread4(wl);
            const uint32_t cnt = b0 + (b1 << 1);
            const uint32_t nA = cnt + bl;
            // site 0's left neighbour (site L - 1) is not yet visited: no flip
            const uint32_t nB = cnt + (bl ^ (call == 0u ? 0x01010100u : 0x01010101u));
            uint32_t OA, OB, SA, SB;
            if constexpr (MODEL == kIsing) {
                // byte n of {hi, lo}: offsets 0, -4, ..., -16; steps 40, 20, ..., -40
                OA = __builtin_amdgcn_perm(0x000000F0u, 0xF4F8FC00u, nA);
                OB = __builtin_amdgcn_perm(0x000000F0u, 0xF4F8FC00u, nB);
                SA = __builtin_amdgcn_perm(0x000000D8u, 0xEC001428u, nA);
                SB = __builtin_amdgcn_perm(0x000000D8u, 0xEC001428u, nB);
            } else {
                const uint32_t bp = spread4(ws); // 1 in the bytes of +1 spins
                const uint32_t base = (bp << 2) + 0x80808080u;
                OA = (base - (nA << 3)) ^ 0x80808080u;
                OB = (base - (nB << 3)) ^ 0x80808080u;
                SA = SB = __builtin_amdgcn_perm(0u, 0x0000D828u, bp);
            }
            // site 4 of the window (the next call's first site): its offsets
            const uint32_t c4 = ((w1 >> 4) & 1u) * 2u + ((w0 >> 4) & 1u), l4 = (wl >> 4) & 1u;
            uint32_t E4;
            if constexpr (MODEL == kIsing)
                E4 = last ? 0u : ((uint32_t)(-4 * (int32_t)(c4 + l4)) & 0xFFu) |
                                     (((uint32_t)(-4 * (int32_t)(c4 + (l4 ^ 1u))) & 0xFFu) << 8);
            else
                E4 = last ? 0u : ilp_off2<MODEL>(c4 + l4, c4 + (l4 ^ 1u), (ws >> 4) & 1u);
            const uint32_t X0 = __builtin_amdgcn_perm(OB, OA, 0x06020501u);  // OA1 OB1 OA2 OB2
            const uint32_t X3 = __builtin_amdgcn_perm(OB, OA, 0x0C0C0703u);  // OA3 OB3
            const uint32_t X1 = __builtin_amdgcn_perm(E4, X3, 0x05040100u);  // OA3 OB3 OA4 OB4
            const uint32_t Y0 = __builtin_amdgcn_perm(SB, SA, 0x05010400u);  // SA0 SB0 SA1 SB1
            const uint32_t Y1 = __builtin_amdgcn_perm(SB, SA, 0x07030602u);  // SA2 SB2 SA3 SB3
            const uint32_t D[4] = {__builtin_amdgcn_perm(Y0, X0, 0x05040100u), __builtin_amdgcn_perm(Y0, X0, 0x07060302u),
                                   __builtin_amdgcn_perm(Y1, X1, 0x05040100u), __builtin_amdgcn_perm(Y1, X1, 0x07060302u)};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                pk[4 * m + k] = (uint64_t)D[k] | ((uint64_t)rng.w[4 * m + k] << 32);
            if (m == 0)
                first = __builtin_amdgcn_perm(OB, OA, 0x0C0C0400u); // OA0 OB0
            if (m == (R::kCalls - 1) / LPC) {
                // the row's last site (site 3 of the last call) with site 0 flipped
                const uint32_t c3 = ((w1 >> 3) & 1u) * 2u + ((w0 >> 3) & 1u), l3 = (wl >> 3) & 1u;
                const uint32_t c2 = ((wr >> 3) & 1u) ? c3 - 1u : c3 + 1u;
                const uint32_t p3 = MODEL == kIsing ? 0u : (ws >> 3) & 1u; // the Ising columns ignore the spin
                const uint32_t hoffv = ilp_off2<MODEL>(c2 + l3, c2 + (l3 ^ 1u), p3);
                const uint32_t hdsv = ilp_ds2<MODEL>(c2 + l3, c2 + (l3 ^ 1u), p3);
                dv2 = __builtin_amdgcn_perm(Y1, hoffv, 0x05040100u); // site L - 2: the last site's offsets
                dv1 = hdsv << 16;                                     // site L - 1: its own bin steps
            }
            continue;
        }
        // per site k of the window: both offsets (Hoff) and both bin steps (Hds)
        uint32_t hoff[5], hds[4], hoffv = 0u, hdsv = 0u;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const uint32_t cnt = ((w1 >> k) & 1u) * 2u + ((w0 >> k) & 1u); // misaligned of right, up, down
            const uint32_t ml = (wl >> k) & 1u, plus = (ws >> k) & 1u;
            const uint32_t nA = cnt + ml;
            // site 0's left neighbour (site L - 1) is not yet visited: no flip
            const uint32_t nB = (k == 0 && call == 0u) ? nA : cnt + (ml ^ 1u);
            hoff[k] = ilp_off2<MODEL>(nA, nB, plus);
            if (k < 4)
                hds[k] = ilp_ds2<MODEL>(nA, nB, plus);
            if (k == 3) {
                // the last site with site 0 flipped: its right neighbour toggles
                const uint32_t c2 = ((wr >> k) & 1u) ? cnt - 1u : cnt + 1u;
                hoffv = ilp_off2<MODEL>(c2 + ml, c2 + (ml ^ 1u), plus);
                hdsv = ilp_ds2<MODEL>(c2 + ml, c2 + (ml ^ 1u), plus);
            }
        }
        if (m == 0)
            first = hoff[0];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // site 4 call + 3 of the last call is the row's last site: no next site
            const uint32_t nextoff = (k == 3 && last) ? 0u : hoff[k + 1];
            const uint32_t D = nextoff | (hds[k] << 16);
            pk[4 * m + k] = (uint64_t)D | ((uint64_t)rng.w[4 * m + k] << 32);
        }
        if (m == (R::kCalls - 1) / LPC) {
            dv2 = hoffv | (hds[2] << 16); // site L - 2: the last site's offsets
            dv1 = hdsv << 16;             // site L - 1: its own bin steps
        }
    }
    uint32_t F[W];
#pragma unroll
    for (int wi = 0; wi < W; ++wi)
        F[wi] = 0u;
    ilp_sites<MODEL, L, LPC, TLDS>(pk, dv2, dv1, first, rowb, F, T, std::make_integer_sequence<int, L>{});
#pragma unroll
    for (int wi = 0; wi < W; ++wi)
        nacc += (uint32_t)__builtin_popcount(F[wi]);
    // the flips were shifted in from the low end, first site highest
#pragma unroll
    for (int wi = 0; wi < W; ++wi) {
        const int nb = (L - 32 * wi) < 32 ? (L - 32 * wi) : 32;
        cur[wi] ^= __builtin_bitreverse32(F[wi]) >> (32 - nb);
    }
}

// Unsatisfied bonds of bit-packed rows: horizontal bonds of one row
// (periodic), vertical bonds between two rows.
template <int L>
__device__ __forceinline__ uint32_t row_mis(const uint32_t (&R)[Row1<L>::W])
{
    constexpr int W = Row1<L>::W;
    uint32_t n = 0u;
#pragma unroll
    for (int wi = 0; wi < W; ++wi) {
        const int nb = (L - 32 * wi) < 32 ? (L - 32 * wi) : 32;
        const uint32_t nextbit = (wi + 1 < W) ? (R[wi + 1 < W ? wi + 1 : 0] & 1u) : (R[0] & 1u);
        n += (uint32_t)__builtin_popcount(R[wi] ^ ((R[wi] >> 1) | (nextbit << (nb - 1))));
    }
    return n;
}

template <int L>
__device__ __forceinline__ uint32_t pair_mis(const uint32_t (&A)[Row1<L>::W], const uint32_t (&B)[Row1<L>::W])
{
    uint32_t n = 0u;
#pragma unroll
    for (int wi = 0; wi < Row1<L>::W; ++wi)
        n += (uint32_t)__builtin_popcount(A[wi] ^ B[wi]);
    return n;
}

// Storage <-> packed row.  BYTE storage holds int8 +1 (0x01) / -1 (0xFF),
// four sites per word; bit 1 of a byte is set exactly for -1.
template <int L, int LAYOUT>
__device__ __forceinline__ void load_row(const gu32 *base, size_t stride, int y, uint32_t (&R)[Row1<L>::W])
{
    constexpr int W = Row1<L>::W;
    if constexpr (LAYOUT == kLayoutBit) {
#pragma unroll
        for (int w = 0; w < W; ++w)
            R[w] = base[((size_t)y * W + w) * stride];
    } else {
        constexpr int W8 = L / 4;
#pragma unroll
        for (int w = 0; w < W; ++w)
            R[w] = 0u;
#pragma unroll
        for (int m = 0; m < W8; ++m) {
            const uint32_t v = (base[((size_t)y * W8 + m) * stride] >> 1) & 0x01010101u; // -1 flags
            const uint32_t nib = ((v * 0x00204081u) >> 21) & 0xFu;
            R[(4 * m) / 32] |= (nib ^ 0xFu) << ((4 * m) % 32);
        }
    }
}

template <int L, int LAYOUT>
__device__ __forceinline__ void store_row(gu32 *base, size_t stride, int y, const uint32_t (&R)[Row1<L>::W])
{
    constexpr int W = Row1<L>::W;
    if constexpr (LAYOUT == kLayoutBit) {
#pragma unroll
        for (int w = 0; w < W; ++w)
            base[((size_t)y * W + w) * stride] = R[w];
    } else {
        constexpr int W8 = L / 4;
#pragma unroll
        for (int m = 0; m < W8; ++m) {
            const uint32_t nib = (R[(4 * m) / 32] >> ((4 * m) % 32)) & 0xFu;
            const uint32_t up1 = (nib * 0x00204081u) & 0x01010101u; // 1 in the bytes of +1 spins
            base[((size_t)y * W8 + m) * stride] = 0xFFFFFFFFu ^ (up1 * 0xFEu); // 0x01 or 0xFF
        }
    }
}

// One q-state Potts site update: proposal among the q-1 other colours,
// dE = (neighbours equal to old) - (neighbours equal to new) unsatisfied bonds.
// The four neighbour colours are gathered one per byte (v_perm); a byte of
// nb ^ rep is zero exactly where the neighbour has colour rep, and the high
// bit of each byte of ((x & 0x7F..) + 0x7F..) | x is set exactly for the
// non-zero bytes, so both counts are population counts.  c = dE + 4 indexes
// the threshold row: 9 columns in global memory; in LDS 8 columns, c = 8 in
// column 4 and c = 4 (dE = 0, always accepted) not stored.  rowb is the byte
// address of the current bin's row (LDS) or its byte offset (global).
template <int L, int LPC, bool TLDS, int W, int X>
__device__ __forceinline__ void potts_site(const uint32_t (&up)[W], uint32_t (&cur)[W],
                                           const uint32_t (&dn)[W], int32_t &rowb, const RowRng<L, LPC, 2> &rng,
                                           const uint32_t *__restrict__ T, uint32_t q)
{
    constexpr int w = X / 4, k = X % 4;
    constexpr int wl = ((X + L - 1) % L) / 4, wr = ((X + 1) % L) / 4;
    const uint32_t wp = rng.template get<X, 0>();
    const uint32_t r = rng.template get<X, 1>(); // clamped in RowRng::fill
    // byte 0 = down, byte 1 = up neighbour (bytes 2, 3 replaced below)
    const uint32_t vert = __builtin_amdgcn_perm(up[w], dn[w], (uint32_t)k | ((uint32_t)(4 + k) << 8));
    uint32_t nb;
    if constexpr (k == 1 || k == 2) {
        nb = __builtin_amdgcn_perm(vert, cur[w], 4u | (5u << 8) | ((uint32_t)(k - 1) << 16) | ((uint32_t)(k + 1) << 24));
    } else if constexpr (k == 0) { // left = byte 3 of the previous word (site L-1 for X = 0)
        const uint32_t h = __builtin_amdgcn_perm(cur[wl], cur[w], 1u | (7u << 8));
        nb = __builtin_amdgcn_perm(vert, h, 0u | (1u << 8) | (4u << 16) | (5u << 24));
    } else { // right = byte 0 of the next word (site 0, already updated, for X = L-1)
        const uint32_t h = __builtin_amdgcn_perm(cur[wr], cur[w], 2u | (4u << 8));
        nb = __builtin_amdgcn_perm(vert, h, 0u | (1u << 8) | (4u << 16) | (5u << 24));
    }
    const uint32_t oldrep = __builtin_amdgcn_perm(0u, cur[w], (uint32_t)k * 0x01010101u);
    const uint32_t old = oldrep & 0xFFu;
    uint32_t nw = old + 1u + __umulhi(wp, q - 1u);
    nw = min(nw, nw - q); // nw - q wraps above nw when nw < q
    const uint32_t newrep = __builtin_amdgcn_perm(0u, nw, 0u); // byte 0 of nw in every byte
    const uint32_t xo = nb ^ oldrep, xn = nb ^ newrep;
    const uint32_t eq_old = ~(((xo & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | xo) & 0x80808080u;
    const uint32_t ne_new = (((xn & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | xn) & 0x80808080u;
    const uint32_t c = (uint32_t)__builtin_popcount(ne_new) + (uint32_t)__builtin_popcount(eq_old); // dE + 4
    uint32_t t;
    int32_t dstep;
    if constexpr (TLDS) {
        const uint32_t col = (c ^ ((c >> 1) & 4u)) & 7u; // 0..3 -> 0..3, 8 -> 4, 5..7 -> 5..7
        t = load_t<true>(T, rowb + 4 * (int32_t)col);
        dstep = (int32_t)(c << 5) - 128;
    } else {
        t = load_t<false>(T, rowb + 4 * (int32_t)c);
        dstep = (int32_t)c * 36 - 144;
    }
    const bool acc = (r < t) | (c == 4u);
    const uint32_t delta = (oldrep ^ newrep) & (0xFFu << (8 * k));
    cur[w] ^= acc ? delta : 0u;
    rowb += acc ? dstep : 0;
}

template <int L, int LPC, bool TLDS, int W, int... X>
__device__ __forceinline__ void potts_row(const uint32_t (&up)[W], uint32_t (&cur)[W],
                                          const uint32_t (&dn)[W], int32_t &rowb,
                                          const uint32_t *__restrict__ T, uint32_t chain,
                                          uint32_t g, int y, uint32_t j, uint32_t k0, uint32_t k1, uint32_t q,
                                          std::integer_sequence<int, X...>)
{
    RowRng<L, LPC, 2> rng;
    rng.fill(chain, g, y, j, k0, k1);
    (potts_site<L, LPC, TLDS, W, X>(up, cur, dn, rowb, rng, T, q), ...);
}

// Adds the block's packed LDS counters to the global histogram and clears
// them.  Called by every thread of the block between two barriers.
__device__ __forceinline__ void flush_hist(uint32_t *lhist, int hw, unsigned long long *hist_,
                                           gu64 *blk = nullptr)
{
    gu64 *hist = (gu64 *)hist_;
    for (int i = threadIdx.x; i < hw; i += blockDim.x) {
        const uint32_t v = lhist[i];
        if (v) {
            lhist[i] = 0u;
            if (v & 0xFFFFu)
                gadd(&hist[2 * i], (unsigned long long)(v & 0xFFFFu));
            if (v >> 16)
                gadd(&hist[2 * i + 1], (unsigned long long)(v >> 16));
            if (blk) { // this block's own histogram, for jackknife errors
                if (v & 0xFFFFu)
                    gadd(&blk[2 * i], (unsigned long long)(v & 0xFFFFu));
                if (v >> 16)
                    gadd(&blk[2 * i + 1], (unsigned long long)(v >> 16));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Potts with the per-site work split over the lanes of a chain.  Lane j of
// the chain's LPC lanes owns the S = L / LPC consecutive sites [S j, S j + S)
// of every row: it keeps only its segment of rows y-1, y, y+1 (bytes 0..S-1
// of its segment words), draws the Philox words of its sites, and computes
// for each of them the threshold column for both outcomes of the left
// neighbour's attempt.  The right, up and down neighbours do not change
// before a site's own attempt, except the right neighbour of the row's last
// site (site 0, decided first), for which both variants are kept.  The
// attempts then run through the row on all lanes of the chain in lockstep:
// each takes its site's descriptor from the owning lane (DPP), selects by the
// previous outcome, reads the threshold and compares.  At the end of the row
// every lane applies the accepted proposals to its own segment and stores it
// (byte stores when segments are not word-aligned); a lane only reads back
// bytes it wrote itself.
// ---------------------------------------------------------------------------
// Adds a lane's count of accepted moves (recorded sweeps of a real chain,
// leader lane) to the run's counter and clears it; the counts stay below
// 2^32 between two flushes (at most N per sweep, flushed with the 16-bit
// LDS histogram).
__device__ __forceinline__ void flush_accepts(const LatticeArgs &a, bool counts, uint32_t &nacc)
{
    if (counts && a.accepts && nacc)
        gadd((gu64 *)a.accepts, (unsigned long long)nacc);
    nacc = 0u;
}

// Sites of a row that changed: bits of bit-packed rows, bytes of byte rows.
template <int W>
__device__ __forceinline__ uint32_t changed_bits(const uint32_t (&a)[W], const uint32_t (&b)[W])
{
    uint32_t n = 0u;
#pragma unroll
    for (int w = 0; w < W; ++w)
        n += (uint32_t)__builtin_popcount(a[w] ^ b[w]);
    return n;
}

template <int W>
__device__ __forceinline__ uint32_t changed_bytes(const uint32_t (&a)[W], const uint32_t (&b)[W])
{
    uint32_t n = 0u;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t x = a[w] ^ b[w];
        n += (uint32_t)__builtin_popcount((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u);
    }
    return n;
}

template <int L, int LPC>
struct PottsLP {
    static constexpr bool ok = (LPC == 4 || LPC == 16) && L % LPC == 0;
    static constexpr int S = L / LPC;       // sites per lane
    static constexpr int SW = (S + 3) / 4;  // words of a lane's segment
    // Philox calls (two sites each) that cover the segment: S / 2 when S is
    // even (segments start on even sites), else S / 2 + 1 (either parity)
    static constexpr int NCALL = S % 2 == 0 ? S / 2 : S / 2 + 1;
};

// Segment of row y owned by lane j: sites [S j, S j + S) in bytes 0..S-1.
template <int L, int LPC>
__device__ __forceinline__ void lp_load(const gu32 *base, size_t stride, int y, uint32_t j,
                                        uint32_t (&seg)[PottsLP<L, LPC>::SW])
{
    constexpr int S = PottsLP<L, LPC>::S, SW = PottsLP<L, LPC>::SW, W = L / 4;
    const uint32_t b0 = (uint32_t)S * j, w0 = b0 >> 2;
    if constexpr (S % 4 == 0) {
#pragma unroll
        for (int k = 0; k < SW; ++k)
            seg[k] = base[((size_t)y * W + w0 + k) * stride];
    } else {
        uint32_t raw[SW + 1];
#pragma unroll
        for (int k = 0; k <= SW; ++k) {
            const uint32_t w = w0 + (uint32_t)k < (uint32_t)W ? w0 + (uint32_t)k : (uint32_t)W - 1u;
            raw[k] = base[((size_t)y * W + w) * stride];
        }
#pragma unroll
        for (int k = 0; k < SW; ++k)
            seg[k] = __builtin_amdgcn_alignbyte(raw[k + 1], raw[k], b0 & 3u);
    }
}

template <int L, int LPC>
__device__ __forceinline__ void lp_store(gu32 *base, size_t stride, int y, uint32_t j,
                                         const uint32_t (&seg)[PottsLP<L, LPC>::SW])
{
    constexpr int S = PottsLP<L, LPC>::S, SW = PottsLP<L, LPC>::SW, W = L / 4;
    const uint32_t b0 = (uint32_t)S * j;
    if constexpr (S % 4 == 0) {
#pragma unroll
        for (int k = 0; k < SW; ++k)
            base[((size_t)y * W + (b0 >> 2) + k) * stride] = seg[k];
    } else {
#pragma unroll
        for (int m = 0; m < S; ++m) {
            const uint32_t bb = b0 + (uint32_t)m;
            gu8 *p = (gu8 *)(base + ((size_t)y * W + (bb >> 2)) * stride) + (bb & 3u);
            *p = (uint8_t)(seg[m / 4] >> (8 * (m % 4)));
        }
    }
}

// Column offset (bytes) of the code c = dE + 4 in a bin's threshold row: 8
// staged columns in LDS (c = 8 in column 4; c = 4 is never read), 9 columns
// in global memory.
template <bool TLDS>
__device__ __forceinline__ uint32_t lp_off(uint32_t c)
{
    return TLDS ? ((c ^ ((c >> 1) & 4u)) & 7u) << 2 : c << 2;
}

// Shift (bytes) of the bin row origin when a move with code c is accepted.
template <bool TLDS>
__device__ __forceinline__ int32_t lp_ds(uint32_t c)
{
    return ((int32_t)c - 4) * (TLDS ? 32 : 36);
}

// Acceptance word of a candidate, accept iff word <= T: r + 1 (r clamped to
// 2^32 - 2, so r + 1 <= T iff r < T) when the move changes the energy, 0 for
// dE = 0, which is accepted whatever threshold is read for it.
__device__ __forceinline__ uint32_t lp_word(uint32_t c, uint32_t r) { return c == 4u ? 0u : r + 1u; }

// c = dE + 4 for the colours of a site: old, proposal nw, the fixed
// neighbours (down, up, right or filler) packed with a 0xFF filler byte in
// nb, and the left neighbour lft.
__device__ __forceinline__ uint32_t lp_code(uint32_t nb, uint32_t old, uint32_t nw, uint32_t lft)
{
    const uint32_t oldrep = __builtin_amdgcn_perm(0u, old, 0u), newrep = __builtin_amdgcn_perm(0u, nw, 0u);
    const uint32_t xo = nb ^ oldrep, xn = nb ^ newrep;
    const uint32_t eq_old = ~(((xo & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | xo) & 0x80808080u;
    const uint32_t ne_new = (((xn & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | xn) & 0x80808080u;
    // the filler byte counts once as "not the new colour"; the left
    // neighbour adds [lft == old] + [lft != nw] - 1
    return (uint32_t)__builtin_popcount(ne_new) + (uint32_t)__builtin_popcount(eq_old) + (lft == old ? 1u : 0u) -
           (lft == nw ? 1u : 0u);
}

// Descriptors of site X from its owning lane, two 64-bit broadcasts:
//   geo: bytes 0, 1 = the next site's column offsets (this site rejected /
//        accepted); high dword = this site's bin shifts as two int16 (left
//        neighbour rejected / accepted);
//   acw: the site's acceptance words (left neighbour rejected / accepted).
// Sites L - 2 and L - 1 switch to their variants when site 0 was accepted
// (it is the right neighbour of site L - 1).
template <int L, int LPC, int X>
__device__ __forceinline__ void lp_get(const uint64_t (&geo)[PottsLP<L, LPC>::S],
                                       const uint64_t (&acw)[PottsLP<L, LPC>::S], uint64_t gv2, uint64_t gv1,
                                       uint64_t av1, bool f0, uint64_t &g, uint64_t &w)
{
    constexpr int S = PottsLP<L, LPC>::S, O = X / S, R = X % S;
    g = group_bcast64<LPC, O>(geo[R]);
    w = group_bcast64<LPC, O>(acw[R]);
    if constexpr (X == L - 2) {
        const uint64_t v = group_bcast64<LPC, O>(gv2);
        g = f0 ? v : g;
    }
    if constexpr (X == L - 1) {
        const uint64_t v = group_bcast64<LPC, O>(gv1), u = group_bcast64<LPC, O>(av1);
        g = f0 ? v : g;
        w = f0 ? u : w;
    }
}

// Site X.  On entry: B / Bf = the bin row origin before this site's attempt
// if the previous site was rejected / accepted, prev = that outcome, (t0, t1)
// = this site's threshold in either case (read one site earlier), (g, w) =
// its descriptors.  The next site's two candidate thresholds are read before
// this site's compare, so each read has a whole site to complete and the
// loop-carried chain is select -> compare.
template <int L, int LPC, bool TLDS, int X>
__device__ __forceinline__ void lp_site(const uint64_t (&geo)[PottsLP<L, LPC>::S],
                                        const uint64_t (&acw)[PottsLP<L, LPC>::S], uint64_t gv2, uint64_t gv1,
                                        uint64_t av1, int32_t &B, int32_t &Bf, uint64_t &g, uint64_t &w, bool &prev,
                                        bool &f0, uint64_t &pm, uint32_t &t0, uint32_t &t1, uint32_t (&F)[2],
                                        const uint32_t *__restrict__ T)
{
    const uint32_t glo = (uint32_t)g, ghi = (uint32_t)(g >> 32);
    const int32_t x0 = B + (int32_t)(int16_t)(ghi & 0xFFFFu), x1 = Bf + ((int32_t)ghi >> 16);
    B = prev ? Bf : B;   // this site's bin row
    Bf = prev ? x1 : x0; // the next site's, if this one is accepted
    const uint32_t word = prev ? (uint32_t)(w >> 32) : (uint32_t)w;
    uint32_t n_t0 = 0u, n_t1 = 0u;
    uint64_t ng = 0u, nw = 0u;
    if constexpr (X + 1 < L) {
        n_t0 = load_t<TLDS>(T, B + sbyte(glo));
        n_t1 = load_t<TLDS>(T, Bf + sbyte(glo >> 8));
        lp_get<L, LPC, X + 1>(geo, acw, gv2, gv1, av1, f0, ng, nw);
    }
    // the previous site's flip record, while the reads are in flight: not
    // between the threshold select and the compare
    if constexpr (X > 0)
        F[(X - 1) / 32] = shift_in<false>(F[(X - 1) / 32], pm);
    // selected only now, after the next reads were issued (the barrier keeps
    // the wait for this site's reads one site behind them)
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t t = prev ? t1 : t0;
    t0 = n_t0;
    t1 = n_t1;
    g = ng;
    w = nw;
    const bool acc = word <= t;
    if constexpr (X == 0)
        f0 = acc;
    pm = __builtin_amdgcn_ballot_w64(acc);
    prev = acc;
    __builtin_amdgcn_sched_barrier(0);
}

template <int L, int LPC, bool TLDS, int... X>
__device__ __forceinline__ void lp_row(const uint64_t (&geo)[PottsLP<L, LPC>::S],
                                       const uint64_t (&acw)[PottsLP<L, LPC>::S], uint64_t gv2, uint64_t gv1,
                                       uint64_t av1, uint32_t first, int32_t &rowb, uint32_t (&F)[2],
                                       const uint32_t *__restrict__ T, std::integer_sequence<int, X...>)
{
    uint64_t g, w;
    lp_get<L, LPC, 0>(geo, acw, gv2, gv1, av1, false, g, w);
    // site 0: its left neighbour (site L - 1) is not yet visited, one candidate
    uint32_t t0 = load_t<TLDS>(T, rowb + sbyte(group_bcast<LPC, 0>(first))), t1 = t0;
    int32_t B = rowb, Bf = rowb;
    bool prev = false, f0 = false;
    uint64_t pm = 0u;
    (lp_site<L, LPC, TLDS, X>(geo, acw, gv2, gv1, av1, B, Bf, g, w, prev, f0, pm, t0, t1, F, T), ...);
    F[(L - 1) / 32] = shift_in<true>(F[(L - 1) / 32], pm);
    rowb = prev ? Bf : B;
}

// The sweeps of one chain (per lane: its segment), with the histogram
// bookkeeping of sweep_block.
template <int L, int LPC, bool TLDS>
__device__ __forceinline__ int32_t potts_lp_sweeps(const LatticeArgs &a, gu32 *base, size_t stride,
                                                   uint32_t chain, uint32_t j, bool counts, int32_t b,
                                                   const uint32_t *__restrict__ T, int32_t tbase, uint32_t *lhist,
                                                   int hw, int flush_every, gu64 *blk)
{
    using P = PottsLP<L, LPC>;
    constexpr int S = P::S, SW = P::SW, NCALL = P::NCALL, KC = L / 2; // Philox calls per row
    const uint32_t q = (uint32_t)a.q;
    uint32_t up[SW], cur[SW], dn[SW], nx[SW];
    lp_load<L, LPC>(base, stride, L - 1, j, up);
    lp_load<L, LPC>(base, stride, 0, j, cur);
    lp_load<L, LPC>(base, stride, 1 % L, j, dn);
    lp_load<L, LPC>(base, stride, 2 % L, j, nx);
    int32_t rowb = TLDS ? tbase + 32 * b : 36 * b;
    auto bin_of = [&](int32_t rb) { return TLDS ? (rb - tbase) >> 5 : rb / 36; };
    const uint32_t first_call = ((uint32_t)S * j) >> 1, par = ((uint32_t)S * j) & 1u;
    const bool lane0 = j == 0u, lanel = j == (uint32_t)(LPC - 1);
    int until_flush = flush_every;
    uint32_t nacc = 0u; // accepted moves since the last flush (the same in every lane)
    for (int s = 0; s < a.n_sweeps; ++s) {
        const uint32_t g = a.g0 + (uint32_t)s;
        for (int y = 0; y < L; ++y) {
            // Philox words of the segment's sites: site i uses words
            // 2 (i & 1) (proposal) and 2 (i & 1) + 1 (acceptance) of call i / 2
            uint32_t w[NCALL][4];
#pragma unroll
            for (int k = 0; k < NCALL; ++k) {
                const uint32_t call =
                    first_call + (uint32_t)k < (uint32_t)KC ? first_call + (uint32_t)k : (uint32_t)KC - 1u;
                const Words4 r = philox4x32_10(chain, g, (uint32_t)(y * KC) + call, kTagSweep, a.k0, a.k1);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    w[k][t] = r.w[t];
            }
            uint32_t old[S], nw[S], ra[S];
#pragma unroll
            for (int m = 0; m < S; ++m) {
                uint32_t wp, wa;
                if constexpr (S % 2 == 0) {
                    wp = w[m / 2][2 * (m & 1)];
                    wa = w[m / 2][2 * (m & 1) + 1];
                } else { // the segment starts on an odd site when par = 1
                    // a bitwise select: a conditional here becomes a dynamic
                    // index into w (scratch)
                    const uint32_t mk = 0u - par;
                    wp = (w[(m + 1) / 2][2 * ((m + 1) & 1)] & mk) | (w[m / 2][2 * (m & 1)] & ~mk);
                    wa = (w[(m + 1) / 2][2 * ((m + 1) & 1) + 1] & mk) | (w[m / 2][2 * (m & 1) + 1] & ~mk);
                }
                ra[m] = min(wa, 0xFFFFFFFEu);
                old[m] = (cur[m / 4] >> (8 * (m % 4))) & 0xFFu;
                const uint32_t n = old[m] + 1u + __umulhi(wp, q - 1u);
                nw[m] = min(n, n - q); // n - q wraps above n when n < q
            }
            // neighbours across segment ends
            const uint32_t lh_old = group_prev<LPC>(old[S - 1]), lh_nw = group_prev<LPC>(nw[S - 1]);
            const uint32_t rh_old = group_next<LPC>(old[0]), rh_nw = group_next<LPC>(nw[0]);
            // the left neighbour of site 0 is site L - 1, not yet visited
            const uint32_t l0_acc = lane0 ? lh_old : lh_nw;
            // the right neighbour of the row's last site is site 0, visited first
            const uint32_t rr_acc = lanel ? rh_nw : rh_old;
            // per site: both candidates' offsets, bin shifts and acceptance words
            uint32_t offp[S], dsp[S];
            uint64_t acw[S];
            uint32_t offv = 0u, dsv = 0u;
            uint64_t av1 = 0u;
#pragma unroll
            for (int m = 0; m < S; ++m) {
                // bytes: down, up (same column), right, filler
                const uint32_t vert = __builtin_amdgcn_perm(up[m / 4], dn[m / 4],
                                                            (uint32_t)(m % 4) | ((uint32_t)(4 + m % 4) << 8));
                // (m is a constant of the unrolled loop: the branches fold)
                const int mr = (m + 1) / 4 < SW ? (m + 1) / 4 : SW - 1;
                uint32_t nb;
                if (m + 1 < S)
                    nb = __builtin_amdgcn_perm(vert, cur[mr],
                                               4u | (5u << 8) | ((uint32_t)((m + 1) % 4) << 16) | (0x0Du << 24));
                else
                    nb = __builtin_amdgcn_perm(vert, rh_old, 4u | (5u << 8) | (0u << 16) | (0x0Du << 24));
                const uint32_t l_rej = m > 0 ? old[m > 0 ? m - 1 : 0] : lh_old;
                const uint32_t l_acc = m > 0 ? nw[m > 0 ? m - 1 : 0] : l0_acc;
                const uint32_t c0 = lp_code(nb, old[m], nw[m], l_rej), c1 = lp_code(nb, old[m], nw[m], l_acc);
                offp[m] = lp_off<TLDS>(c0) | (lp_off<TLDS>(c1) << 8);
                dsp[m] = ((uint32_t)lp_ds<TLDS>(c0) & 0xFFFFu) | ((uint32_t)lp_ds<TLDS>(c1) << 16);
                acw[m] = (uint64_t)lp_word(c0, ra[m]) | ((uint64_t)lp_word(c1, ra[m]) << 32);
                if (m + 1 == S) {
                    // the row's last site (lane LPC - 1) with site 0 accepted
                    const uint32_t nb2 = __builtin_amdgcn_perm(vert, rr_acc, 4u | (5u << 8) | (0x0Du << 24));
                    const uint32_t v0 = lp_code(nb2, old[m], nw[m], l_rej), v1 = lp_code(nb2, old[m], nw[m], l_acc);
                    offv = lp_off<TLDS>(v0) | (lp_off<TLDS>(v1) << 8);
                    dsv = ((uint32_t)lp_ds<TLDS>(v0) & 0xFFFFu) | ((uint32_t)lp_ds<TLDS>(v1) << 16);
                    av1 = (uint64_t)lp_word(v0, ra[m]) | ((uint64_t)lp_word(v1, ra[m]) << 32);
                }
            }
            // the next site's offsets: the lane's own, or site 0 of the next
            // lane's segment for its last site (none after the row's last site)
            const uint32_t next0 = group_next<LPC>(offp[0]), nextv = group_next<LPC>(offv);
            uint64_t geo[S];
#pragma unroll
            for (int m = 0; m < S; ++m) {
                const uint32_t nxo = m + 1 < S ? offp[m + 1 < S ? m + 1 : 0] : (lanel ? 0u : next0);
                geo[m] = (uint64_t)nxo | ((uint64_t)dsp[m] << 32);
            }
            // site L - 2 with site 0 accepted: the last site's offsets change
            const uint64_t gv2 =
                (uint64_t)(S >= 2 ? offv : nextv) | ((uint64_t)dsp[S >= 2 ? S - 2 : 0] << 32);
            const uint64_t gv1 = (uint64_t)dsv << 32;
            uint32_t F[2] = {0u, 0u};
            lp_row<L, LPC, TLDS>(geo, acw, gv2, gv1, av1, offp[0], rowb, F, T, std::make_integer_sequence<int, L>{});
            // flips were shifted in from the low end, first site highest
            nacc += (uint32_t)__builtin_popcount(F[0]) + (uint32_t)__builtin_popcount(F[1]);
            const uint32_t F0 = __builtin_bitreverse32(F[0]) >> (32 - (L < 32 ? L : 32));
            const uint32_t F1 = L > 32 ? __builtin_bitreverse32(F[1]) >> (32 - (L > 32 ? L - 32 : 32)) : 0u;
            // this lane's accepted proposals: bits S j .. S j + S - 1 of F
            const uint32_t fj = (uint32_t)((((uint64_t)F1 << 32) | F0) >> (S * j));
#pragma unroll
            for (int m = 0; m < S; ++m)
                cur[m / 4] ^= ((fj >> m) & 1u) ? (old[m] ^ nw[m]) << (8 * (m % 4)) : 0u;
            lp_store<L, LPC>(base, stride, y, j, cur);
#pragma unroll
            for (int k = 0; k < SW; ++k) {
                up[k] = cur[k];
                cur[k] = dn[k];
                dn[k] = nx[k];
            }
            lp_load<L, LPC>(base, stride, (y + 3) % L, j, nx);
        }
        if (counts) {
            const int32_t bb = bin_of(rowb);
            atomicAdd(&lhist[bb >> 1], 1u << ((bb & 1) << 4));
        }
        if (--until_flush == 0 && s + 1 < a.n_sweeps) {
            until_flush = flush_every;
            flush_accepts(a, counts, nacc);
            __syncthreads();
            flush_hist(lhist, hw, a.hist, blk);
            __syncthreads();
        }
    }
    flush_accepts(a, counts, nacc);
    return bin_of(rowb);
}

// ---------------------------------------------------------------------------
// One block of chains: threads [0, blockDim) handle chains
// [c_first, c_first + blockDim / LPC) of the instance described by `a`.
// The threshold table is staged into LDS (TLDS) and the block's histogram is
// accumulated in LDS, then added to the instance's global histogram.
// Used by the plain kernel (one launch per instance) and by the persistent
// batched kernel (one block per work item).
// ---------------------------------------------------------------------------
template <int MODEL, int L, int LAYOUT, bool TLDS, int LPC>
__device__ __forceinline__ void sweep_block(const LatticeArgs &a, int c_first, uint32_t *smem)
{
    constexpr int NC = Cols<MODEL>::value;
    // LDS: [threshold table (staged) | packed 16-bit histogram]
    constexpr int NCL = MODEL == kPotts ? 8 : NC;
    uint32_t *lhist = TLDS ? smem + a.n_bins * NCL : smem;
    const int tid = threadIdx.x;
    const int hw = lds_hist_words(a.n_bins);
    for (int i = tid; i < hw; i += blockDim.x)
        lhist[i] = 0u;
    const uint32_t *T = a.thresholds;
    if constexpr (TLDS) {
        for (int i = tid; i < a.n_bins * NCL; i += blockDim.x) {
            int src = i;
            if constexpr (MODEL == kPotts) { // dE = 0 not stored; dE = +4 in column 4
                const int bb = i >> 3, cc = i & 7;
                src = bb * 9 + (cc == 4 ? 8 : cc);
            }
            smem[i] = ((const gu32 *)a.thresholds)[src];
        }
        T = smem;
    }
    __syncthreads();

    const int c = c_first + tid / LPC;       // chain of this lane
    const uint32_t j = (uint32_t)(tid % LPC); // rank within the chain's lane group
    const bool leader = j == 0u;
    gu32 *base = (gu32 *)a.words + c;
    const size_t stride = (size_t)a.c_pad;
    const uint32_t chain = (uint32_t)(a.chain0 + c);
    const bool counts = a.record && c < a.n_chains && leader;
    int32_t b = ((const gi32 *)a.bins)[c];
    // sweeps between two flushes of the 16-bit LDS counters
    const int flush_every = kMaxBlockCount / (int)(blockDim.x / LPC);
    int until_flush = flush_every;
    // this block's histogram (plain launches with per-block histograms)
    gu64 *blk = a.hist_blocks ? (gu64 *)a.hist_blocks + (size_t)(c_first / (int)(blockDim.x / LPC)) * (size_t)a.n_bins
                              : nullptr;

    if constexpr (MODEL == kPotts && PottsLP<L, LPC>::ok) {
        int32_t tbase = 0;
        if constexpr (TLDS)
            tbase = (int32_t)(uint32_t)(uintptr_t)(lds_u32 *)smem;
        b = potts_lp_sweeps<L, LPC, TLDS>(a, base, stride, chain, j, counts, b, T, tbase, lhist, hw, flush_every,
                                          blk);
    } else if constexpr (MODEL == kPotts) {
        constexpr int W = Geom<L, LAYOUT>::kWpr;
        const uint32_t q = (uint32_t)a.q;
        uint32_t up[W], cur[W], dn[W], nx[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            up[w] = base[((L - 1) * W + w) * stride];
            cur[w] = base[(0 * W + w) * stride];
            dn[w] = base[((1 % L) * W + w) * stride];
            nx[w] = base[((2 % L) * W + w) * stride];
        }
        // the current bin's threshold row: LDS byte address of an 8-column
        // row, or byte offset of a 9-column row in global memory
        int32_t tbase = 0;
        if constexpr (TLDS)
            tbase = (int32_t)(uint32_t)(uintptr_t)(lds_u32 *)smem;
        int32_t rowb = TLDS ? tbase + 32 * b : 36 * b;
        auto bin_of = [&](int32_t rb) { return TLDS ? (rb - tbase) >> 5 : rb / 36; };
        uint32_t nacc = 0u;
        for (int s = 0; s < a.n_sweeps; ++s) {
            const uint32_t g = a.g0 + (uint32_t)s;
            for (int y = 0; y < L; ++y) {
                uint32_t before[W];
#pragma unroll
                for (int w = 0; w < W; ++w)
                    before[w] = cur[w];
                potts_row<L, LPC, TLDS, W>(up, cur, dn, rowb, T, chain, g, y, j, a.k0, a.k1, q,
                                           std::make_integer_sequence<int, L>{});
                nacc += changed_bytes<W>(before, cur); // an accepted proposal changes the colour
                const int yn = (y + 3) % L;
                if (leader) {
#pragma unroll
                    for (int w = 0; w < W; ++w)
                        base[(y * W + w) * stride] = cur[w];
                }
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    up[w] = cur[w];
                    cur[w] = dn[w];
                    dn[w] = nx[w];
                    nx[w] = base[(yn * W + w) * stride];
                }
            }
            if (counts) {
                const int32_t bb = bin_of(rowb);
                atomicAdd(&lhist[bb >> 1], 1u << ((bb & 1) << 4));
            }
            if (--until_flush == 0 && s + 1 < a.n_sweeps) {
                until_flush = flush_every;
                flush_accepts(a, counts, nacc);
                __syncthreads();
                flush_hist(lhist, hw, a.hist, blk);
                __syncthreads();
            }
        }
        flush_accepts(a, counts, nacc);
        b = bin_of(rowb);
    } else {
        constexpr int W = Row1<L>::W;
        uint32_t up[W], cur[W], dn[W], nx[W];
        load_row<L, LAYOUT>(base, stride, L - 1, up);
        load_row<L, LAYOUT>(base, stride, 0, cur);
        load_row<L, LAYOUT>(base, stride, 1 % L, dn);
        load_row<L, LAYOUT>(base, stride, 2 % L, nx);
        // the current bin's row origin in the threshold table: an absolute LDS
        // byte address when the table is staged, else a byte offset
        int32_t tbase = 0;
        if constexpr (TLDS)
            tbase = (int32_t)(uint32_t)(uintptr_t)(lds_u32 *)smem;
        int32_t rowb = tbase + 4 * (b * NC + row_origin<MODEL>());
        // MUMA with the joint (E, M) histogram: unsatisfied bonds of the
        // sweep's final configuration, counted row by row once a row and the
        // one above it are final (the bond between rows L - 1 and 0 last)
        const bool em = MODEL == kMuma && a.em != nullptr;
        uint32_t nmis = 0u, nacc = 0u;
        for (int s = 0; s < a.n_sweeps; ++s) {
            const uint32_t g = a.g0 + (uint32_t)s;
            for (int y = 0; y < L; ++y) {
                if constexpr (LPC >= 4) {
                    ising_lp_row<MODEL, L, LPC, TLDS>(up, cur, dn, rowb, T, chain, g, y, j, a.k0, a.k1, nacc);
                } else {
                    uint32_t before[W];
#pragma unroll
                    for (int w = 0; w < W; ++w)
                        before[w] = cur[w];
                    ising_row<MODEL, L, LPC, TLDS>(up, cur, dn, rowb, T, chain, g, y, j, a.k0, a.k1,
                                                   std::make_integer_sequence<int, W>{});
                    nacc += changed_bits<W>(before, cur);
                }
                if constexpr (MODEL == kMuma) {
                    if (em) {
                        nmis += row_mis<L>(cur) + (y > 0 ? pair_mis<L>(up, cur) : 0u);
                        if (y == L - 1)
                            nmis += pair_mis<L>(cur, dn); // dn: row 0 as this sweep left it
                    }
                }
                if (leader)
                    store_row<L, LAYOUT>(base, stride, y, cur);
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    up[w] = cur[w];
                    cur[w] = dn[w];
                    dn[w] = nx[w];
                }
                load_row<L, LAYOUT>(base, stride, (y + 3) % L, nx);
            }
            if (counts) {
                const int32_t bb = (((rowb - tbase) >> 2) - row_origin<MODEL>()) / NC;
                atomicAdd(&lhist[bb >> 1], 1u << ((bb & 1) << 4));
                if constexpr (MODEL == kMuma) {
                    if (em) { // E = -2N + 2 nmis = -2N + 4 e, e <= N
                        const uint32_t e = min(nmis >> 1, (uint32_t)(L * L));
                        gadd((gu64 *)a.em + (size_t)e * (size_t)a.n_bins + (size_t)bb, 1ull);
                    }
                }
            }
            if constexpr (MODEL == kMuma)
                nmis = 0u;
            if (--until_flush == 0 && s + 1 < a.n_sweeps) {
                until_flush = flush_every;
                flush_accepts(a, counts, nacc);
                __syncthreads();
                flush_hist(lhist, hw, a.hist, blk);
                __syncthreads();
            }
        }
        flush_accepts(a, counts, nacc);
        b = (((rowb - tbase) >> 2) - row_origin<MODEL>()) / NC;
    }
    if (leader)
        ((gi32 *)a.bins)[c] = b;
    __syncthreads();
    flush_hist(lhist, hw, a.hist, blk);
}

template <int MODEL, int L, int LAYOUT, bool TLDS, int LPC>
__global__ __launch_bounds__(256) void lattice_sweeps(LatticeArgs a)
{
    extern __shared__ uint32_t smem[];
    sweep_block<MODEL, L, LAYOUT, TLDS, LPC>(a, (int)(blockIdx.x * (blockDim.x / LPC)), smem);
}

// The same with blocks of 512 threads and the table staged in LDS: where
// the staged table leaves room for one block per CU, a block of 512 puts two
// wavefronts on every SIMD, so that one wave's instructions fill the other's
// wait for its threshold reads.  A kernel of its own, so that the register
// budget of two waves per SIMD does not touch the 256-thread code.
template <int MODEL, int L, int LAYOUT, int LPC>
__global__ __launch_bounds__(512) void lattice_sweeps_wide(LatticeArgs a)
{
    extern __shared__ uint32_t smem[];
    sweep_block<MODEL, L, LAYOUT, true, LPC>(a, (int)(blockIdx.x * (blockDim.x / LPC)), smem);
}

// ---------------------------------------------------------------------------
// Launch of one compiled variant.  `threads` per block (64..256, or 512
// with the table in LDS); LPC lanes per chain, so a block holds
// threads / LPC chains.
// ---------------------------------------------------------------------------
template <int MODEL, int L, int LAYOUT, int LPC>
static hipError_t launch_variant(int threads, const LatticeArgs &a, hipStream_t s)
{
    const long lanes = (long)a.c_pad * LPC;
    const bool wide = threads == 512 && a.table_in_lds;
    if (threads < 64 || (threads > 256 && !wide) || lanes % threads)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)(lanes / threads)), block(threads);
    size_t lds = (size_t)lds_hist_words(a.n_bins) * 4u;
    if (a.table_in_lds) {
        lds += (size_t)a.n_bins * lds_table_cols(MODEL) * 4u;
        auto k = wide ? lattice_sweeps_wide<MODEL, L, LAYOUT, LPC> : lattice_sweeps<MODEL, L, LAYOUT, true, LPC>;
        if (lds > 65536u) {
            hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(k, grid, block, lds, s, a);
    } else {
        auto k = lattice_sweeps<MODEL, L, LAYOUT, false, LPC>;
        hipLaunchKernelGGL(k, grid, block, lds, s, a);
    }
    return hipGetLastError();
}

template <int MODEL, int L, int LAYOUT>
static hipError_t launch_lpc(int lpc, int threads, const LatticeArgs &a, hipStream_t s)
{
    switch (lpc) {
    case 1: return launch_variant<MODEL, L, LAYOUT, 1>(threads, a, s);
    case 2: return launch_variant<MODEL, L, LAYOUT, 2>(threads, a, s);
    case 4: return launch_variant<MODEL, L, LAYOUT, 4>(threads, a, s);
    case 16: return launch_variant<MODEL, L, LAYOUT, 16>(threads, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int MODEL, int LAYOUT>
static hipError_t launch_model(int L, int lpc, int threads, const LatticeArgs &a, hipStream_t s)
{
    switch (L) {
    case 4: return launch_lpc<MODEL, 4, LAYOUT>(lpc, threads, a, s);
    case 8: return launch_lpc<MODEL, 8, LAYOUT>(lpc, threads, a, s);
    case 16: return launch_lpc<MODEL, 16, LAYOUT>(lpc, threads, a, s);
    case 24: return launch_lpc<MODEL, 24, LAYOUT>(lpc, threads, a, s);
    case 32: return launch_lpc<MODEL, 32, LAYOUT>(lpc, threads, a, s);
    case 48: return launch_lpc<MODEL, 48, LAYOUT>(lpc, threads, a, s);
    case 64: return launch_lpc<MODEL, 64, LAYOUT>(lpc, threads, a, s);
    default: return hipErrorInvalidValue;
    }
}

} // namespace muca
