// Instantiations of the fused step (lbm3_step_impl.h) for storage double, compute double.
#include "lbm3_step_impl.h"

namespace tcg {

hipError_t tiles_f64(Fmt in, Fmt out, bool obs, bool pt, const void* fin, void* fout, const Instance* inst,
                    const Tile* tiles, int ntiles, int threads, uint32_t salt, const int64_t* step_dev,
                    int filter, double* partials, double* rho_out, hipStream_t stream)
{
    return tiles_any<double, double>(in, out, obs, pt, fin, fout, inst, tiles, ntiles, threads, salt, step_dev,
                                filter, partials, rho_out, stream);
}

int tiles_f64_occupancy(int threads) { return tiles_occupancy<double, double>(threads); }

hipError_t tiles_f64_tape(Fmt in, const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                          int ntiles, int threads, double* tape, hipStream_t stream)
{
    switch (threads) {
        case 64: return tiles_tape_nt<64>(in, fin, fout, inst, tiles, ntiles, tape, stream);
        case 128: return tiles_tape_nt<128>(in, fin, fout, inst, tiles, ntiles, tape, stream);
        case 256: return tiles_tape_nt<256>(in, fin, fout, inst, tiles, ntiles, tape, stream);
        case 512: return tiles_tape_nt<512>(in, fin, fout, inst, tiles, ntiles, tape, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t tiles_f64_pair(const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                          int ntiles, int threads, bool pt, hipStream_t stream)
{
    return tiles_pair_any<double, double>(fin, fout, inst, tiles, ntiles, threads, 0u, 0u, nullptr, pt, stream);
}

int tiles_f64_pair_occupancy(int threads) { return pair_occupancy<double, double>(threads); }

hipError_t tiles_f64_block_tape(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                                double* tape, hipStream_t stream)
{
    return tiles_block_tape(fin, fout, inst, tiles, ntiles, tape, stream);
}

hipError_t tiles_f64_block(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                              uint32_t salt, const int64_t* step_dev, bool pt, hipStream_t stream)
{
    return tiles_block_any<double, double>(fin, fout, inst, tiles, ntiles, salt, step_dev, pt, stream);
}

}  // namespace tcg
