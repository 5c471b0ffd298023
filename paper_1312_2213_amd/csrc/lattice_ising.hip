// lattice_ising.hip -- compiled Ising (MUCA over E) sweep variants.
#include "lattice_impl.h"

namespace muca {
hipError_t launch_ising(int L, int layout, int lpc, int threads, const LatticeArgs &a, hipStream_t s)
{
    return layout == kLayoutBit ? launch_model<kIsing, kLayoutBit>(L, lpc, threads, a, s)
                                : launch_model<kIsing, kLayoutByte>(L, lpc, threads, a, s);
}
} // namespace muca
