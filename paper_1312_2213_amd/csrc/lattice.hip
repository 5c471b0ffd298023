// lattice.hip -- Metropolis sweeps of many independent 2D lattice chains that
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

// One Ising / MUMA site update at compile-time column x of row y.
template <int MODEL, int L, int LAYOUT, int W, int X>
__device__ __forceinline__ void ising_site(const uint32_t (&up)[W], uint32_t (&cur)[W],
                                           const uint32_t (&dn)[W], int32_t &b, Words4 &rw,
                                           const uint32_t *__restrict__ T, uint32_t chain,
                                           uint32_t g, int y, uint32_t k0, uint32_t k1)
{
    using G = Geom<L, LAYOUT>;
    constexpr int NC = Cols<MODEL>::value;
    if ((X & 3) == 0)
        rw = philox4x32_10(chain, g, (uint32_t)(y * (L / 4) + X / 4), kTagSweep, k0, k1);
    const uint32_t r = min(rw.w[X & 3], 0xFFFFFFFEu); // accept iff r < T (T = ~0: always)
    const uint32_t s = spin_code<L, LAYOUT>(cur, X);
    const uint32_t nl = spin_code<L, LAYOUT>(cur, (X + L - 1) % L);
    const uint32_t nr = spin_code<L, LAYOUT>(cur, (X + 1) % L);
    const uint32_t nu = spin_code<L, LAYOUT>(up, X);
    const uint32_t nd = spin_code<L, LAYOUT>(dn, X);
    const int32_t n_al = 4 - (int32_t)((s ^ nl) + (s ^ nr) + (s ^ nu) + (s ^ nd));
    int32_t col, delta;
    if (MODEL == kIsing) {
        col = n_al;
        delta = n_al - 2; // dE = 4 n_al - 8, one bin per 4
    } else {
        const int32_t plus = LAYOUT == kLayoutBit ? (int32_t)s : (int32_t)(s ^ 1u);
        col = 2 * n_al + plus;
        delta = plus ? -1 : 1; // M changes by -2 s_i
    }
    const uint32_t t = T[b * NC + col];
    const bool acc = r < t;
    constexpr uint32_t fm = LAYOUT == kLayoutBit ? (1u << (X % G::kSpw)) : (0xFEu << ((X % G::kSpw) * 8));
    cur[X / G::kSpw] ^= acc ? fm : 0u;
    b += acc ? delta : 0;
}

template <int MODEL, int L, int LAYOUT, int W, int... X>
__device__ __forceinline__ void ising_row(const uint32_t (&up)[W], uint32_t (&cur)[W],
                                          const uint32_t (&dn)[W], int32_t &b,
                                          const uint32_t *__restrict__ T, uint32_t chain,
                                          uint32_t g, int y, uint32_t k0, uint32_t k1,
                                          std::integer_sequence<int, X...>)
{
    Words4 rw;
    (ising_site<MODEL, L, LAYOUT, W, X>(up, cur, dn, b, rw, T, chain, g, y, k0, k1), ...);
}

// One q-state Potts site update: proposal among the q-1 other colours,
// dE = (neighbours equal to old) - (neighbours equal to new) unsatisfied bonds.
template <int L, int W, int X>
__device__ __forceinline__ void potts_site(const uint32_t (&up)[W], uint32_t (&cur)[W],
                                           const uint32_t (&dn)[W], int32_t &b, Words4 &rw,
                                           const uint32_t *__restrict__ T, uint32_t chain,
                                           uint32_t g, int y, uint32_t k0, uint32_t k1, uint32_t q)
{
    if ((X & 1) == 0)
        rw = philox4x32_10(chain, g, (uint32_t)(y * (L / 2) + X / 2), kTagSweep, k0, k1);
    const uint32_t wp = rw.w[2 * (X & 1)];
    const uint32_t r = min(rw.w[2 * (X & 1) + 1], 0xFFFFFFFEu);
    const uint32_t old = colour<L>(cur, X);
    uint32_t nw = old + 1u + __umulhi(wp, q - 1u);
    nw = nw >= q ? nw - q : nw;
    const uint32_t cl = colour<L>(cur, (X + L - 1) % L);
    const uint32_t cr = colour<L>(cur, (X + 1) % L);
    const uint32_t cu = colour<L>(up, X);
    const uint32_t cd = colour<L>(dn, X);
    const int32_t n_old = (cl == old) + (cr == old) + (cu == old) + (cd == old);
    const int32_t n_new = (cl == nw) + (cr == nw) + (cu == nw) + (cd == nw);
    const int32_t dE = n_old - n_new;
    const uint32_t t = T[b * 9 + dE + 4];
    const bool acc = r < t;
    cur[X / 4] ^= acc ? ((old ^ nw) << ((X % 4) * 8)) : 0u;
    b += acc ? dE : 0;
}

template <int L, int W, int... X>
__device__ __forceinline__ void potts_row(const uint32_t (&up)[W], uint32_t (&cur)[W],
                                          const uint32_t (&dn)[W], int32_t &b,
                                          const uint32_t *__restrict__ T, uint32_t chain,
                                          uint32_t g, int y, uint32_t k0, uint32_t k1, uint32_t q,
                                          std::integer_sequence<int, X...>)
{
    Words4 rw;
    (potts_site<L, W, X>(up, cur, dn, b, rw, T, chain, g, y, k0, k1, q), ...);
}

template <int MODEL, int L, int LAYOUT, bool TLDS>
__global__ __launch_bounds__(256) void lattice_sweeps(LatticeArgs a)
{
    constexpr int W = Geom<L, LAYOUT>::kWpr;
    constexpr int NC = Cols<MODEL>::value;
    extern __shared__ uint32_t smem[];
    uint32_t *lhist = smem;
    const int tid = threadIdx.x;
    for (int i = tid; i < a.n_bins; i += blockDim.x)
        lhist[i] = 0u;
    const uint32_t *T = a.thresholds;
    if (TLDS) {
        uint32_t *ltab = smem + a.n_bins;
        for (int i = tid; i < a.n_bins * NC; i += blockDim.x)
            ltab[i] = a.thresholds[i];
        T = ltab;
    }
    __syncthreads();

    const int c = blockIdx.x * blockDim.x + tid;
    uint32_t *base = a.words + c;
    const size_t stride = (size_t)a.c_pad;
    uint32_t up[W], cur[W], dn[W], nx[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        up[w] = base[((L - 1) * W + w) * stride];
        cur[w] = base[(0 * W + w) * stride];
        dn[w] = base[((1 % L) * W + w) * stride];
        nx[w] = base[((2 % L) * W + w) * stride];
    }
    int32_t b = a.bins[c];
    const uint32_t chain = (uint32_t)(a.chain0 + c);
    const bool counts = a.record && c < a.n_chains;
    const uint32_t q = (uint32_t)a.q;

    for (int s = 0; s < a.n_sweeps; ++s) {
        const uint32_t g = a.g0 + (uint32_t)s;
        for (int y = 0; y < L; ++y) {
            if (MODEL == kPotts)
                potts_row<L, W>(up, cur, dn, b, T, chain, g, y, a.k0, a.k1, q,
                                std::make_integer_sequence<int, L>{});
            else
                ising_row<MODEL, L, LAYOUT, W>(up, cur, dn, b, T, chain, g, y, a.k0, a.k1,
                                               std::make_integer_sequence<int, L>{});
            const int yn = (y + 3) % L;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                base[(y * W + w) * stride] = cur[w];
                up[w] = cur[w];
                cur[w] = dn[w];
                dn[w] = nx[w];
                nx[w] = base[(yn * W + w) * stride];
            }
        }
        if (counts)
            atomicAdd(&lhist[b], 1u);
    }
    a.bins[c] = b;
    __syncthreads();
    for (int i = tid; i < a.n_bins; i += blockDim.x) {
        const uint32_t v = lhist[i];
        if (v)
            atomicAdd(&a.hist[i], (unsigned long long)v);
    }
}

// ---------------------------------------------------------------------------
// Initialisation: spin of site i of chain c from word (i & 3) of
// Philox(c, 0, i >> 2, INIT): Ising/MUMA +1 iff the top bit is set; Potts
// colour (word * q) >> 32.  Then the energy (each bond once: right, down) and
// the magnetisation, and the bin of the binned quantity.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t get_site(const uint32_t *base, size_t stride, int L, int wpr,
                                             int layout, int y, int x)
{
    const int spw = layout == kLayoutBit ? 32 : 4;
    const uint32_t word = base[((size_t)y * wpr + x / spw) * stride];
    if (layout == kLayoutBit)
        return (word >> (x % spw)) & 1u;
    return (word >> ((x % spw) * 8)) & 0xFFu;
}

__global__ void lattice_init(LatticeInitArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.c_pad)
        return;
    const int L = a.L;
    const int wpr = words_per_row(L, a.layout);
    const int spw = a.layout == kLayoutBit ? 32 : 4;
    uint32_t *base = a.words + c;
    const size_t stride = (size_t)a.c_pad;
    for (int y = 0; y < L; ++y) {
        for (int w = 0; w < wpr; ++w) {
            uint32_t word = 0u;
            for (int k = 0; k < spw; ++k) {
                const int x = w * spw + k;
                if (x >= L)
                    break;
                const int i = y * L + x;
                const Words4 r = philox4x32_10((uint32_t)c, 0u, (uint32_t)(i >> 2), kTagInit, a.k0, a.k1);
                const uint32_t v = r.w[i & 3];
                uint32_t code;
                if (a.model == kPotts)
                    code = __umulhi(v, (uint32_t)a.q);
                else if (a.layout == kLayoutBit)
                    code = v >> 31;
                else
                    code = (v >> 31) ? 0x01u : 0xFFu;
                word |= code << (a.layout == kLayoutBit ? k : 8 * k);
            }
            base[((size_t)y * wpr + w) * stride] = word;
        }
    }
    int32_t e = 0, m = 0;
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            const uint32_t s = get_site(base, stride, L, wpr, a.layout, y, x);
            const uint32_t sr = get_site(base, stride, L, wpr, a.layout, y, (x + 1) % L);
            const uint32_t sd = get_site(base, stride, L, wpr, a.layout, (y + 1) % L, x);
            if (a.model == kPotts) {
                e += (s != sr) + (s != sd);
            } else {
                e += (s == sr ? -1 : 1) + (s == sd ? -1 : 1);
                const bool plus = a.layout == kLayoutBit ? (s == 1u) : (s == 0x01u);
                m += plus ? 1 : -1;
            }
        }
    }
    const int32_t v = a.model == kMuma ? m : e;
    a.values[c] = v;
    const int32_t d = v - a.lo;
    a.bins[c] = d >= 0 ? d / a.step : -1;
}

__global__ void fill_u64(unsigned long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Dispatch over the compiled lattice sizes and layouts.
// ---------------------------------------------------------------------------
bool lattice_size_supported(int L)
{
    return L == 4 || L == 8 || L == 16 || L == 24 || L == 32 || L == 48 || L == 64;
}

template <int MODEL, int L, int LAYOUT>
static hipError_t launch_one(int cpb, const LatticeArgs &a, hipStream_t s)
{
    constexpr int NC = Cols<MODEL>::value;
    const dim3 grid(a.c_pad / cpb), block(cpb);
    size_t lds = (size_t)a.n_bins * 4u;
    if (a.table_in_lds) {
        lds += (size_t)a.n_bins * NC * 4u;
        auto k = lattice_sweeps<MODEL, L, LAYOUT, true>;
        if (lds > 65536u) {
            hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(k, grid, block, lds, s, a);
    } else {
        auto k = lattice_sweeps<MODEL, L, LAYOUT, false>;
        hipLaunchKernelGGL(k, grid, block, lds, s, a);
    }
    return hipGetLastError();
}

template <int MODEL, int LAYOUT>
static hipError_t launch_L(int L, int cpb, const LatticeArgs &a, hipStream_t s)
{
    switch (L) {
    case 4: return launch_one<MODEL, 4, LAYOUT>(cpb, a, s);
    case 8: return launch_one<MODEL, 8, LAYOUT>(cpb, a, s);
    case 16: return launch_one<MODEL, 16, LAYOUT>(cpb, a, s);
    case 24: return launch_one<MODEL, 24, LAYOUT>(cpb, a, s);
    case 32: return launch_one<MODEL, 32, LAYOUT>(cpb, a, s);
    case 48: return launch_one<MODEL, 48, LAYOUT>(cpb, a, s);
    case 64: return launch_one<MODEL, 64, LAYOUT>(cpb, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lattice_sweeps(int model, int L, int layout, int cpb, int n_cols,
                                 const LatticeArgs &a, hipStream_t s)
{
    (void)n_cols;
    if (model == kPotts)
        return launch_L<kPotts, kLayoutByte>(L, cpb, a, s);
    if (model == kIsing)
        return layout == kLayoutBit ? launch_L<kIsing, kLayoutBit>(L, cpb, a, s)
                                    : launch_L<kIsing, kLayoutByte>(L, cpb, a, s);
    if (model == kMuma)
        return layout == kLayoutBit ? launch_L<kMuma, kLayoutBit>(L, cpb, a, s)
                                    : launch_L<kMuma, kLayoutByte>(L, cpb, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_lattice_init(const LatticeInitArgs &a, hipStream_t s)
{
    const int block = 64;
    hipLaunchKernelGGL(lattice_init, dim3((a.c_pad + block - 1) / block), dim3(block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int block = 256;
    hipLaunchKernelGGL(fill_u64, dim3((unsigned)((n + block - 1) / block)), dim3(block), 0, s, p, n);
    return hipGetLastError();
}

} // namespace muca
