// lattice_potts.hip -- compiled q-state Potts (MUCA over E_unsat) sweep variants.
#include "lattice_impl.h"

namespace muca {
hipError_t launch_potts(int L, int lpc, int threads, const LatticeArgs &a, hipStream_t s)
{
    return launch_model<kPotts, kLayoutByte>(L, lpc, threads, a, s);
}
} // namespace muca
