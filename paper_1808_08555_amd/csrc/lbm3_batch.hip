// Batched form: many independent lattices in one arena, advanced by graph launches.
#include "lbm3_handle.h"

using namespace tcg;

extern "C" {
int lbm3_batch_create(const lbm3_params* p, int32_t count, void* s, lbm3_batch_t** out)
{
    (void)p; (void)count; (void)s;
    if (out) *out = nullptr;
    set_error("batch not built yet");
    return LBM3_EUNSUPPORTED;
}
int lbm3_batch_init_fields(lbm3_batch_t* b, int32_t idx, const double* rho, const double* u)
{
    (void)b; (void)idx; (void)rho; (void)u;
    return LBM3_EUNSUPPORTED;
}
int lbm3_batch_step(lbm3_batch_t* b, int64_t n) { (void)b; (void)n; return LBM3_EUNSUPPORTED; }
int lbm3_batch_observables(lbm3_batch_t* b, int32_t idx, lbm3_obs* out, double* rho_out)
{
    (void)b; (void)idx; (void)out; (void)rho_out;
    return LBM3_EUNSUPPORTED;
}
int lbm3_batch_set_tile(lbm3_batch_t* b, int32_t side, int32_t threads, int32_t rows)
{
    (void)b; (void)side; (void)threads; (void)rows;
    return LBM3_EUNSUPPORTED;
}
int lbm3_batch_destroy(lbm3_batch_t* b) { (void)b; return LBM3_OK; }
}
