// Internal declarations shared by the HIP sources of liblbm3.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/lbm3.h"

namespace tcg {

// Per-lattice constants of the step, precomputed on the host in FP64.
// Pair index p: 0 = (red, green), 1 = (red, blue), 2 = (green, blue).
struct KParams {
    int32_t nx, ny;
    int64_t plane;      // elements between the same node in consecutive population planes
    int64_t pitch;      // elements between consecutive rows of one plane
    int64_t span;       // elements of one population buffer (27 planes)
    double sigma[3];    // sigma_kl per pair
    double g[3];        // g(X_kl) of the segregation law, Eq. (20)
    double beta0;       // reference segregation parameter, Eq. (19)
    double inv_nu[3];   // 1/nu_k, nu_k = (tau_k - 1/2)/3
    double cfac[3];     // 1e6 / (rho0_k rho0_l) per pair, Eq. (6)
    double guard;       // |G_kl| at or below which n_kl = 0 and the stress is 0
};

// One workgroup's share of a lattice: output columns [x0, x0 + cols) (cols <= threads - 4)
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
};

// Observables partials: 3 masses, 2 momenta, kinetic energy, max|u|, nonfinite flag.
constexpr int kObsFields = 8;

enum class Prec { F64, F32S, F32 };

// Launchers (lbm3_step.hip).  All asynchronous on `stream`.
hipError_t launch_tiles(Prec prec, const void* fin, void* fout, const Instance* inst,
                        const Tile* tiles, int ntiles, int threads, int64_t step, hipStream_t stream);
hipError_t launch_observe_tiles(Prec prec, const void* fin, const Instance* inst, const Tile* tiles,
                                int ntiles, int threads, double* partials, double* rho_out,
                                hipStream_t stream);
hipError_t launch_reduce_obs(const double* partials, int nblocks, double* out, hipStream_t stream);
hipError_t launch_init(Prec prec, const double* rho, const double* u, void* fout,
                       const KParams& kp, hipStream_t stream);
hipError_t launch_import(Prec prec, const double* f, void* fout, const KParams& kp,
                         hipStream_t stream);
hipError_t launch_export(Prec prec, const void* fin, double* f, const KParams& kp,
                         hipStream_t stream);
hipError_t launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t stream);
int blocks_per_cu(Prec prec, int threads);

// Tile plans (lbm3_plan.hip).
// Tiles of one lattice in locality order (strip by strip, rows upward): strips of at most
// threads-4 columns spread evenly over nx (line-aligned when nx allows), segments of about
// `rows` rows spread evenly over ny.
void plan_lattice(int inst, int nx, int ny, int threads, int rows, int elem_bytes,
                  std::vector<Tile>& out);
// Reorders a locality-ordered list so that each XCD (workgroups are dealt to the XCDs in turn)
// receives one contiguous run of it, keeping neighbouring tiles, and their shared halos, in
// the same L2.
std::vector<Tile> xcd_order(const std::vector<Tile>& L, int nxcd);
// Rows per segment that fit the tile count to the resident workgroup slots.
int auto_rows(int nx, int ny, int threads, int slots, int elem_bytes);
int device_slots(Prec prec, int threads);

size_t elem_bytes(Prec p);

// Host-side helpers (lbm3_api.hip).
void set_error(const char* fmt, ...);
int validate_params(const lbm3_params* p);
void derive(const lbm3_params* p, KParams* kp, double X[3], double g[3], double nu[3]);

}  // namespace tcg
