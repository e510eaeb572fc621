// Instantiations of the fused step (lbm3_step_impl.h) for storage double, compute double.
#include "lbm3_step_impl.h"

namespace tcg {

hipError_t tiles_f64(Fmt in, Fmt out, bool obs, const void* fin, void* fout, const Instance* inst,
                    const Tile* tiles, int ntiles, int threads, uint32_t salt, int filter,
                    double* partials, double* rho_out, hipStream_t stream)
{
    return tiles_any<double, double>(in, out, obs, fin, fout, inst, tiles, ntiles, threads, salt, filter,
                                partials, rho_out, stream);
}

int tiles_f64_occupancy(int threads) { return tiles_occupancy<double, double>(threads); }

}  // namespace tcg
