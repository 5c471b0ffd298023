// polymer_host.cpp -- bead-spring polymer runs (placeholder until the polymer
// kernel lands; every entry point reports the model as unavailable).
#include "runtime_internal.h"

int muca_polymer_geometry(const muca_config *, muca::Geometry *)
{
    return muca_fail(MUCA_E_ARG, "polymer model not available in this build");
}
int muca_polymer_init(muca_run *, const float *) { return muca_fail(MUCA_E_ARG, "polymer model not available"); }
int muca_polymer_upload(muca_run *) { return muca_fail(MUCA_E_ARG, "polymer model not available"); }
int muca_polymer_enqueue(muca_run *, int64_t, bool, hipStream_t)
{
    return muca_fail(MUCA_E_ARG, "polymer model not available");
}
int muca_polymer_state(muca_run *, int32_t, int32_t, float *, int32_t *, double *)
{
    return muca_fail(MUCA_E_ARG, "polymer model not available");
}
