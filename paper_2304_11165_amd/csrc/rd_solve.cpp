// rd_solve.cpp -- steady state (conjugate gradients), adjoint and batches.
#include <hip/hip_runtime.h>

#include "rd_host.h"
#include "rd_sim.h"

extern "C" rd_status rd_sim_steady_state(rd_sim *sim, int, double, int64_t, double *, double *,
                                         int64_t *)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    return rd_fail(RD_ERR_STATE, "steady state not available yet");
}

extern "C" rd_status rd_sim_adjoint(rd_sim *sim, const float *, int64_t, double, int, double *,
                                    double *, double *)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    return rd_fail(RD_ERR_STATE, "adjoint not available yet");
}

struct rd_batch {
    int n = 0;
};

extern "C" rd_status rd_batch_create(const rd_geometry *const *, int, rd_storage, rd_batch **out)
{
    if (out) *out = nullptr;
    return rd_fail(RD_ERR_STATE, "batches not available yet");
}
extern "C" rd_status rd_batch_workspace_bytes(const rd_batch *, size_t *)
{
    return rd_fail(RD_ERR_STATE, "batches not available yet");
}
extern "C" rd_status rd_batch_bind(rd_batch *, void *, size_t, void *)
{
    return rd_fail(RD_ERR_STATE, "batches not available yet");
}
extern "C" rd_status rd_batch_tortuosity(rd_batch *, int, double, int64_t, double *, double *,
                                         int64_t *)
{
    return rd_fail(RD_ERR_STATE, "batches not available yet");
}
extern "C" void rd_batch_destroy(rd_batch *b) { delete b; }
