// Instantiations of the fused step (lbm3_step_impl.h) for storage float, compute double.
#include "lbm3_step_impl.h"

namespace tcg {

hipError_t tiles_f32s(Fmt in, Fmt out, bool obs, bool pt, const void* fin, void* fout, const Instance* inst,
                    const Tile* tiles, int ntiles, int threads, uint32_t salt, const int64_t* step_dev,
                    int filter, double* partials, double* rho_out, hipStream_t stream)
{
    return tiles_any<float, double>(in, out, obs, pt, fin, fout, inst, tiles, ntiles, threads, salt, step_dev,
                                filter, partials, rho_out, stream);
}

int tiles_f32s_occupancy(int threads) { return tiles_occupancy<float, double>(threads); }

hipError_t tiles_f32s_pair(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                           int threads, uint32_t salt_a, uint32_t salt_b, const int64_t* step_dev, bool pt,
                           hipStream_t stream)
{
    return tiles_pair_any<float, double>(fin, fout, inst, tiles, ntiles, threads, salt_a, salt_b, step_dev, pt,
                                          stream);
}

int tiles_f32s_pair_occupancy(int threads) { return pair_occupancy<float, double>(threads); }

hipError_t tiles_f32s_block(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                               uint32_t salt, const int64_t* step_dev, bool pt, hipStream_t stream)
{
    return tiles_block_any<float, double>(fin, fout, inst, tiles, ntiles, salt, step_dev, pt, stream);
}

}  // namespace tcg
