// Internal declarations shared by the HIP sources of liblbm3.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "lbm3.h"

namespace tcg {

// Per-lattice constants of the step, precomputed on the host in FP64.
// Pair index p: 0 = (red, green), 1 = (red, blue), 2 = (green, blue).
struct KParams {
    int32_t nx, ny;
    int64_t plane;      // elements between the same node in consecutive planes
    int64_t pitch;      // row pitch of the 27-population layout (27 planes, rows interleaved)
    int64_t fpitch;     // row pitch of the factored layout (16 planes, rows interleaved)
    int64_t span;       // elements of one state buffer (room for 27 planes)
    double sigma[3];    // sigma_kl per pair
    double g[3];        // g_kl of the segregation law: beta_kl = beta0 (1 + s g_kl)
    double beta0;       // reference segregation parameter, Eq. (19)
    double ct_coef;     // s = min(ct_coef rho_r rho_g rho_b / rho^3, 1): 35 (Eqs. 16, 19), 27 (Eq. 15)
    double inv_nu[3];   // 1/nu_k, nu_k = (tau_k - 1/2)/3
    double cfac[3];     // 1e6 / (rho0_k rho0_l) per pair, Eq. (6)
    double guard;       // |G_kl| at or below which n_kl = 0 and the stress is 0
};

// One workgroup's share of a lattice: output columns [x0, x0 + cols) (cols <= threads - 6)
// and output rows [y0, y0 + rows) of instance `inst`.
struct Tile {
    int32_t inst;
    int32_t x0, y0, rows, cols;
    int32_t pad[3];
};

// Where one instance of a batch lives in the arena.
struct Instance {
    KParams kp;
    int64_t offset;  // element offset of plane 0 in each of the two arenas
    int32_t fmt;     // Fmt of the instance's current state (read when a launch filters by it)
    int32_t pad;
};

// Observables partials: 3 masses, 2 momenta, kinetic energy, max|u|, nonfinite flag.
constexpr int kObsFields = 8;

// Wavefront reductions (butterfly of lane exchanges across the 64 lanes of a wave, no LDS
// storage); afterwards every lane holds the wave's result.  The max lets a NaN win.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = (o > v || o != o) ? o : v;
    }
    return v;
}

enum class Prec { F64, F32S, F32 };

// State formats.  F27: the 27 recoloured populations f_ddag_{i,k} of every node, before
// streaming.  FAC: the same state factored per node as f_dag_i (9), c_k (3), V_0 and V_1 (4),
// from which f_ddag_{i,k} = c_k f_dag_i + w_i V_k . e_i is rebuilt exactly where it is pulled;
// V_2 = -(V_0 + V_1) (the three sum to zero), formed the same way by every path.
enum class Fmt : int32_t { F27 = 0, FAC = 1 };
constexpr int kFacPlanes = 16;

// Launchers (lbm3_step.hip).  All asynchronous on `stream`.  One fused step from a state in
// format `in` to one in format `out` (F27 -> FAC or FAC -> FAC); with
// filter != 0 a workgroup whose instance is not in format `in` does nothing.  pt selects the
// perturbation operator of Eqs. (4)-(5) in place of the force and Guo's term.  With FP32
// storage the stochastic rounding is salted by the step number: `step`, or, when step_dev
// is given, the value it points to on the device when the launch runs (a graph replays the
// same launches at later steps).
hipError_t launch_tiles(Prec prec, Fmt in, Fmt out, const void* fin, void* fout, const Instance* inst,
                        const Tile* tiles, int ntiles, int threads, int64_t step, int filter,
                        hipStream_t stream, bool pt = false, const int64_t* step_dev = nullptr);
// Adds n to the device step counter *step_dev (one thread), stream-ordered.
hipError_t launch_advance_step(int64_t* step_dev, int64_t n, hipStream_t stream);
hipError_t launch_observe_tiles(Prec prec, Fmt in, const void* fin, const Instance* inst,
                                const Tile* tiles, int ntiles, int threads, double* partials,
                                double* rho_out, hipStream_t stream, bool pt = false);
hipError_t launch_reduce_obs(const double* partials, int nblocks, double* out, hipStream_t stream);
hipError_t launch_init(Prec prec, const double* rho, const double* u, void* fout,
                       const KParams& kp, hipStream_t stream);
hipError_t launch_import(Prec prec, const double* f, void* fout, const KParams& kp,
                         hipStream_t stream);
hipError_t launch_export(Prec prec, Fmt in, const void* fin, double* f, const KParams& kp,
                         hipStream_t stream);
hipError_t launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t stream);
int blocks_per_cu(Prec prec, int threads);

// Tile plans (lbm3_plan.hip).
// Tiles of one lattice in locality order (row of tiles after row of tiles): strips of at
// most threads - 2 halo columns spread evenly over nx (line-aligned when nx allows), segments of
// about `rows` rows spread evenly over ny.
// halo: columns (and half the warm-up rows) beyond the strip that one pass needs: 3 for the
// single step, 6 for the two-step pass.
void plan_lattice(int inst, int nx, int ny, int threads, int rows, int elem_bytes,
                  std::vector<Tile>& out, int halo = 3);
// Reorders a locality-ordered list so that each XCD (workgroups are dealt to the XCDs in turn)
// receives one contiguous run of it, keeping neighbouring tiles, and the halos they share, in
// the same L2.
std::vector<Tile> xcd_order(const std::vector<Tile>& L, int nxcd);
// Blocks of one lattice: at most cmax x rmax nodes each (kBlockCols x kBlockRows for
// launch_block), sizes spread evenly over nx and ny, row of blocks after row of blocks.
void plan_blocks(int inst, int nx, int ny, int cmax, int rmax, std::vector<Tile>& out);
// The two state buffers of a step (read one, write the other) in one allocation, the second
// an odd number of MiB after the first (see lbm3_plan.hip); buf[1] is not freed on its own.
hipError_t alloc_state_pair(size_t bytes, void* buf[2]);
void free_state_pair(void* buf[2]);
// Rows per segment that fit the tile count to the resident workgroup slots.
int auto_rows(int nx, int ny, int threads, int slots, int elem_bytes, int halo = 3);
int device_slots(Prec prec, int threads);
// resident slots of the two-step pass (0 where it does not exist: FP32 storage, 512 threads)
int device_slots_pair(Prec prec, int threads);

size_t elem_bytes(Prec p);
// Salt of the stochastic rounding of step `step` (FP32 storage), the same on host and device.
__host__ __device__ inline uint32_t step_salt(int64_t step)
{
    uint32_t x = (uint32_t)step ^ (uint32_t)(step >> 32) * 0x9E3779B9U;
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Per-precision instantiations of the fused step (lbm3_tiles_*.hip).
#define LBM3_TILES_DECL(NAME)                                                                    \
    hipError_t NAME(Fmt in, Fmt out, bool obs, bool pt, const void* fin, void* fout,             \
                    const Instance* inst,                                                         \
                    const Tile* tiles, int ntiles, int threads, uint32_t salt,                    \
                    const int64_t* step_dev, int filter, double* partials, double* rho_out,       \
                    hipStream_t stream);                                                          \
    int NAME##_occupancy(int threads);
LBM3_TILES_DECL(tiles_f64)
LBM3_TILES_DECL(tiles_f32s)
LBM3_TILES_DECL(tiles_f32)
#undef LBM3_TILES_DECL
// One FP64 step (F27 or FAC in, FAC out) that also records, for every node, the pulled
// densities, totals, concentration gradients and the force in tape[20][ny][nx] (for the
// adjoint).
hipError_t tiles_f64_tape(Fmt in, const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                          int ntiles, int threads, double* tape, hipStream_t stream);
constexpr int kTapeFields = 20;
// Two steps per launch (factored state in and out) over a plan with cols <= threads - 12
// (threads 64, 128 or 256); bitwise the same as two single steps.  pt as for launch_tiles.
// FP32 storage takes the stochastic-rounding salts of the two steps, or their step number
// from step_dev as launch_tiles does.
hipError_t tiles_f64_pair(const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                          int ntiles, int threads, bool pt, hipStream_t stream);
hipError_t tiles_f32_pair(const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                          int ntiles, int threads, bool pt, hipStream_t stream);
hipError_t tiles_f32s_pair(const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                           int ntiles, int threads, uint32_t salt_a, uint32_t salt_b,
                           const int64_t* step_dev, bool pt, hipStream_t stream);
int tiles_f64_pair_occupancy(int threads);
int tiles_f32_pair_occupancy(int threads);
int tiles_f32s_pair_occupancy(int threads);
// Two steps per launch of any precision from `step` (factored state).
hipError_t launch_pair(Prec prec, const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                       int ntiles, int threads, int64_t step, hipStream_t stream, bool pt = false,
                       const int64_t* step_dev = nullptr);
// One step (factored state in and out) on two-dimensional blocks: tiles from plan_blocks,
// workgroups of kBlockThreads lanes; bitwise the same as the march's step.  pt, step and
// step_dev as for launch_tiles.
constexpr int kBlockCols = 28, kBlockRows = 12, kBlockThreads = 512;
hipError_t tiles_f64_block(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                           uint32_t salt, const int64_t* step_dev, bool pt, hipStream_t stream);
hipError_t tiles_f32_block(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                           uint32_t salt, const int64_t* step_dev, bool pt, hipStream_t stream);
hipError_t tiles_f32s_block(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                            uint32_t salt, const int64_t* step_dev, bool pt, hipStream_t stream);
// The FP64 block step (factored state in) that also writes the adjoint's tape, as
// tiles_f64_tape does.
hipError_t tiles_f64_block_tape(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                                double* tape, hipStream_t stream);
hipError_t launch_block(Prec prec, const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                        int ntiles, int64_t step, hipStream_t stream, bool pt = false,
                        const int64_t* step_dev = nullptr);

// Host-side helpers (lbm3_api.hip).
void set_error(const char* fmt, ...);
int validate_params(const lbm3_params* p);
void derive(const lbm3_params* p, KParams* kp, double X[3], double g[3], double nu[3]);

}  // namespace tcg
