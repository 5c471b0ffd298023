// lattice_muma.hip -- compiled multimagnetic (Ising at fixed beta, W(M)) sweep variants.
#include "lattice_impl.h"

namespace muca {
hipError_t launch_muma(int L, int layout, int lpc, int threads, const LatticeArgs &a, hipStream_t s)
{
    return layout == kLayoutBit ? launch_model<kMuma, kLayoutBit>(L, lpc, threads, a, s)
                                : launch_model<kMuma, kLayoutByte>(L, lpc, threads, a, s);
}
} // namespace muca
