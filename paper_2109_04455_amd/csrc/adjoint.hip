// Adjoint of the ADR step (placeholder until the reverse kernels land).
#include "ctx.hpp"

namespace lbf {
void adjoint_release(Ctx *) {}
}  // namespace lbf

extern "C" {
lbf_status lbf_adjoint_workspace_bytes(lbf_ctx c, long, int, int, size_t *)
{
    return lbf::fail(c, LBF_EINVAL, "adjoint not implemented yet");
}
lbf_status lbf_adr_adjoint(lbf_ctx c, long, int, int, void *, size_t, double *, double *)
{
    return lbf::fail(c, LBF_EINVAL, "adjoint not implemented yet");
}
}
