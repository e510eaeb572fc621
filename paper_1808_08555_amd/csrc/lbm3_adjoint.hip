// Adjoint of the FP64 step (reverse sweep with checkpointed recomputation).
#include "lbm3_handle.h"

namespace tcg {
void adjoint_release(lbm3* h)
{
    for (void* p : h->ckpt)
        if (p) (void)hipFree(p);
    h->ckpt.clear();
    if (h->adj_ws) (void)hipFree(h->adj_ws);
    h->adj_ws = nullptr;
    h->adj_ws_bytes = 0;
    h->tape_valid = false;
}
}  // namespace tcg

using namespace tcg;

extern "C" {
int lbm3_adjoint_record(lbm3_t* h, int64_t nsteps, int32_t ckpt_every)
{
    (void)h; (void)nsteps; (void)ckpt_every;
    set_error("adjoint not built yet");
    return LBM3_EUNSUPPORTED;
}
int lbm3_adjoint(lbm3_t* h, const double* drho1_T, double dsigma[3], double* drho0)
{
    (void)h; (void)drho1_T; (void)dsigma; (void)drho0;
    set_error("adjoint not built yet");
    return LBM3_EUNSUPPORTED;
}
}
