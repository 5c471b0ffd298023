// batch.cpp -- several runs advanced by one call (first version: one launch
// per run on the same stream; the persistent kernel replaces it).
#include <cstring>

#include "runtime_internal.h"

extern "C" int muca_batch_workspace_bytes(int32_t n_runs, uint64_t *bytes)
{
    if (n_runs < 1 || !bytes)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    *bytes = 256u * (uint64_t)n_runs;
    return MUCA_OK;
}

extern "C" int muca_batch_run_iteration(muca_run *const *runs, int32_t n, const int64_t *sweeps,
                                        void *d_ws, uint64_t ws_bytes, int32_t graph, void *stream)
{
    (void)d_ws;
    (void)ws_bytes;
    (void)graph;
    if (!runs || !sweeps || n < 1)
        return muca_fail(MUCA_E_ARG, "bad arguments");
    for (int i = 0; i < n; ++i) {
        int rc = muca_run_iteration(runs[i], sweeps[i], stream);
        if (rc)
            return rc;
    }
    return MUCA_OK;
}
