// Internal declarations shared by the HIP sources of liblbm3.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lbm3.h"

namespace tcg {

// Per-lattice constants of the step, precomputed on the host in FP64.
// Pair index p: 0 = (red, green), 1 = (red, blue), 2 = (green, blue).
struct KParams {
    int32_t nx, ny;
    int64_t plane;      // elements between consecutive population planes
    double sigma[3];    // sigma_kl per pair
    double g[3];        // g(X_kl) of the segregation law, Eq. (20)
    double beta0;       // reference segregation parameter, Eq. (19)
    double inv_nu[3];   // 1/nu_k, nu_k = (tau_k - 1/2)/3
    double cfac[3];     // 1e6 / (rho0_k rho0_l) per pair, Eq. (6)
    double guard;       // |G_kl| at or below which n_kl = 0 and the stress is 0
};

// One workgroup's share of a lattice: a strip of output columns [x0, x0 + width)
// and output rows [y0, y0 + rows).
struct Tile {
    int32_t inst;  // instance number (batched form), 0 otherwise
    int32_t x0, y0, rows;
};

// Where one instance of a batch lives in the arena.
struct Instance {
    KParams kp;
    int64_t offset;  // element offset of plane 0 in each of the two arenas
};

// Observables partials: 3 masses, 2 momenta, kinetic energy, max|u|, nonfinite flag.
constexpr int kObsFields = 8;

enum class Prec { F64, F32S, F32 };

// Launchers (lbm3_step.hip).  All asynchronous on `stream`.
hipError_t launch_step(Prec prec, const void* fin, void* fout, const KParams& kp, int threads,
                       int rows, hipStream_t stream);
hipError_t launch_observe(Prec prec, const void* fin, const KParams& kp, int threads, int rows,
                          double* partials, int* nblocks, double* rho_out, hipStream_t stream);
hipError_t launch_reduce_obs(const double* partials, int nblocks, double* out, hipStream_t stream);
hipError_t launch_init(Prec prec, const double* rho, const double* u, void* fout,
                       const KParams& kp, hipStream_t stream);
hipError_t launch_import(Prec prec, const double* f, void* fout, const KParams& kp,
                         hipStream_t stream);
hipError_t launch_export(Prec prec, const void* fin, double* f, const KParams& kp,
                         hipStream_t stream);
hipError_t launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t stream);
hipError_t launch_step_batch(Prec prec, const void* fin, void* fout, const Instance* inst,
                             const Tile* tiles, int ntiles, int threads, hipStream_t stream);
int step_blocks(const KParams& kp, int threads, int rows);

size_t elem_bytes(Prec p);

// Host-side helpers (lbm3_api.hip).
void set_error(const char* fmt, ...);
int validate_params(const lbm3_params* p);
void derive(const lbm3_params* p, KParams* kp, double X[3], double g[3], double nu[3]);

}  // namespace tcg
