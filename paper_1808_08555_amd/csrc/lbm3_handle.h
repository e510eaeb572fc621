// The handle behind lbm3_t and helpers shared by the host sources.
#pragma once

#include <vector>

#include "lbm3_internal.h"

struct lbm3 {
    lbm3_params p;
    tcg::KParams kp;
    tcg::Prec prec;
    hipStream_t stream = nullptr;
    int device = 0;
    void* buf[2] = {nullptr, nullptr};  // population buffers (pull scheme, ping-pong)
    int cur = 0;                        // buffer holding the current state
    tcg::Fmt fmt = tcg::Fmt::F27;       // its format: F27 after init / set_state, FAC after a step
    int64_t step = 0;
    bool ready = false;
    bool init_at_rest = false;          // state came from init_fields with u == NULL
    int threads = 256, rows = 64;       // launch shape: threads per workgroup, rows per segment
    int rows_request = 0;               // rows asked for (0 = fitted to the resident slots)
    tcg::Instance* dinst = nullptr;     // device copy of the one-instance table
    tcg::Tile* dtiles = nullptr;        // device tile list (XCD-aware order)
    int ntiles = 0;
    tcg::Tile* dtiles2 = nullptr;       // tile list of the two-step pass (null: not used)
    int ntiles2 = 0;
    int threads2 = 0;                   // its threads per workgroup
    tcg::Tile* dtilesb = nullptr;       // block list of the one-step block kernel (null: not used)
    int ntilesb = 0;
    int pass_mode = 0;                  // steps per launch: 0 automatic, 1 one, 2 two
    bool tile_set = false;              // launch shape chosen by lbm3_set_tile
    double* staging = nullptr;          // device FP64 staging for host transfers
    size_t staging_cap = 0;
    double* partials = nullptr;         // per-workgroup observables partials
    int partials_cap = 0;
    double* obs_dev = nullptr;
    double* obs_host = nullptr;         // pinned
    // adjoint tape (lbm3_adjoint.hip)
    bool tape_valid = false;
    int64_t tape_steps = 0;
    int32_t tape_every = 0;
    std::vector<void*> ckpt;            // checkpoint states (post-streaming buffer layout)
    void* adj_ws = nullptr;             // adjoint workspace
    size_t adj_ws_bytes = 0;
    hipStream_t adj_stream = nullptr;   // the reverse sweep's own stream (graph capture)
    hipStream_t adj_stream2 = nullptr;  // the segment recompute, beside the reverse steps
    hipEvent_t adj_event = nullptr;
};

namespace tcg {
int hip_fail(hipError_t e, const char* what);
const char* last_error();
Prec prec_of(int precision);
void default_tile(const KParams& kp, Prec prec, int* threads, int* rows);
int check_rho_fields(const double* rho, const double* u, int64_t n);
int upload_plan(lbm3* h);
void adjoint_release(lbm3* h);
void adjoint_destroy(lbm3* h);  // adjoint_release plus the adjoint stream and event
// Enqueues n steps; factored = false keeps the 27-population format (the adjoint's tape).
int step_handle(lbm3* h, int64_t n);
}  // namespace tcg
