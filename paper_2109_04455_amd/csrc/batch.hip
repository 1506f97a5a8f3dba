// Batched sweep (placeholder until the tile-table kernels land).
#include "ctx.hpp"

struct lbf_batch_s {
    int dummy;
};

extern "C" {
lbf_status lbf_batch_create(int, const lbf_params *, lbf_batch *out)
{
    if (out) *out = nullptr;
    return LBF_EINVAL;
}
lbf_status lbf_batch_workspace_bytes(lbf_batch, size_t *) { return LBF_EINVAL; }
lbf_status lbf_batch_bind(lbf_batch, void *, size_t, void *) { return LBF_EINVAL; }
lbf_status lbf_batch_set_geometry(lbf_batch, const uint8_t *, const double *) { return LBF_EINVAL; }
lbf_status lbf_batch_flow(lbf_batch, long, int, double) { return LBF_EINVAL; }
lbf_status lbf_batch_run(lbf_batch, long, int, double, double *, double *, long *) { return LBF_EINVAL; }
lbf_status lbf_batch_get_concentration(lbf_batch, int, int, void *) { return LBF_EINVAL; }
lbf_status lbf_batch_time_steps(lbf_batch, long, double *) { return LBF_EINVAL; }
const char *lbf_batch_last_error(lbf_batch) { return "batch not implemented yet"; }
void lbf_batch_destroy(lbf_batch) {}
}
