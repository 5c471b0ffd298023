// lattice_common.hip -- lattice initialisation, histogram clearing and the
// dispatch to the compiled sweep variants.
#include "muca_internal.h"
#include "philox.h"

namespace muca {

hipError_t launch_ising(int L, int layout, int lpc, int threads, const LatticeArgs &a, hipStream_t s);
hipError_t launch_muma(int L, int layout, int lpc, int threads, const LatticeArgs &a, hipStream_t s);
hipError_t launch_potts(int L, int lpc, int threads, const LatticeArgs &a, hipStream_t s);

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
                const Words4 r = philox4x32_10((uint32_t)(a.chain0 + c), 0u, (uint32_t)(i >> 2), kTagInit, a.k0, a.k1);
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

// Moves n counters to (page-locked, device-visible) host memory and clears
// them: a merge's read-back and reset in one dispatch.
__global__ void drain_u64(unsigned long long *p, unsigned long long *host, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        host[i] = p[i];
        p[i] = 0ull;
    }
}


bool lattice_size_supported(int L)
{
    return L == 4 || L == 8 || L == 16 || L == 24 || L == 32 || L == 48 || L == 64;
}

hipError_t launch_lattice_sweeps(int model, int L, int layout, int lpc, int threads, const LatticeArgs &a,
                                 hipStream_t s)
{
    if (model == kIsing)
        return launch_ising(L, layout, lpc, threads, a, s);
    if (model == kMuma)
        return launch_muma(L, layout, lpc, threads, a, s);
    if (model == kPotts)
        return launch_potts(L, lpc, threads, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_lattice_init(const LatticeInitArgs &a, hipStream_t s)
{
    const int block = 64;
    hipLaunchKernelGGL(lattice_init, dim3((a.c_pad + block - 1) / block), dim3(block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_drain_u64(unsigned long long *p, unsigned long long *host, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int block = 256;
    hipLaunchKernelGGL(drain_u64, dim3((unsigned)((n + block - 1) / block)), dim3(block), 0, s, p, host, n);
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
