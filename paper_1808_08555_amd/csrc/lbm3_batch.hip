// Batched form: many independent lattices (instances of different sizes and parameters,
// one precision) in one device arena.  One launch of the fused step covers the tiles of
// every instance (a flat tile list, dealt to the XCDs in contiguous runs); a captured
// hipGraph of kGraphSteps such launches advances all instances with one graph launch.
// Instances hold the factored state after their first step (FP64 and FP32; FP32 storage
// keeps the 27 populations); a step that finds some instances freshly initialised
// (27-population format) runs as two launches over the same list, each skipping the
// instances of the other format.  Once every instance holds the factored state, pairs of
// steps can run as one launch of the two-step pass over its own tile list (six-column
// halo), also inside the graph.
#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <vector>

#include "lbm3_handle.h"

namespace {
constexpr int kGraphSteps = 20;  // steps per captured graph (a multiple of 4: parity kept with pairs)
}

struct lbm3_batch {
    int count = 0;
    tcg::Prec prec = tcg::Prec::F64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<tcg::Instance> inst;
    tcg::Instance* dinst = nullptr;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t step = 0;
    int threads = 256;
    bool tile_set = false;  // threads chosen by lbm3_batch_set_tile (then also the two-step width)
    bool pt = false;        // every instance uses the perturbation operator of Eqs. (4)-(5)
    std::map<int, int> rows_by_side;  // rows per segment for instances with nx == side
    tcg::Tile* dtiles = nullptr;      // step list, XCD-ordered
    int ntiles = 0;
    int pair_mode = 0;                // steps per launch: 0 = by size, 1 = one, 2 = two
    tcg::Tile* dtiles2 = nullptr;     // two-step list (empty: pairs run as single steps)
    int ntiles2 = 0;
    int threads2 = 0;
    int rows2 = 0;
    tcg::Tile* dobs = nullptr;        // observation list, instance by instance
    std::vector<int> obs_first, obs_count;
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // one graph per starting buffer parity
    double* staging = nullptr;
    size_t staging_cap = 0;
    double* partials = nullptr;
    int partials_cap = 0;
    double* obs_dev = nullptr;
    double* obs_host = nullptr;
    std::vector<char> ready;
    std::vector<tcg::Fmt> fmt;  // per instance: F27 after init_fields, FAC after a step
    // FP32 storage: the step number on the device (equal to `step` once the stream has run),
    // which salts the stochastic rounding of every launch, graph replays included
    int64_t* dstep = nullptr;
};

using namespace tcg;

static void drop_graphs(lbm3_batch* b)
{
    for (auto& g : b->exec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

static int batch_plan(lbm3_batch* b)
{
    std::vector<Tile> all;
    std::vector<Tile> obs;
    b->obs_first.assign(b->count, 0);
    b->obs_count.assign(b->count, 0);
    const int eb = (int)elem_bytes(b->prec);
    // default rows per segment: one value for all instances, chosen (like auto_rows) so that
    // the whole launch takes the fewest rounds of resident workgroups, then the fewest rows
    const int slots = std::max(1, device_slots(b->prec, b->threads));
    int auto_r = 64;
    double best = 1e300;
    for (int r : {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512}) {
        long tiles = 0;
        for (int i = 0; i < b->count; ++i) {
            std::vector<Tile> L;
            plan_lattice(i, b->inst[i].kp.nx, b->inst[i].kp.ny, b->threads, r, eb, L);
            tiles += (long)L.size();
        }
        const double cost = (double)((tiles + slots - 1) / slots) * (r + 6);
        if (cost < best) {
            best = cost;
            auto_r = r;
        }
    }
    for (int i = 0; i < b->count; ++i) {
        const KParams& kp = b->inst[i].kp;
        auto it = b->rows_by_side.find(kp.nx);
        int rows = it != b->rows_by_side.end() ? it->second : 0;
        if (rows <= 0) rows = auto_r;
        std::vector<Tile> L;
        plan_lattice(i, kp.nx, kp.ny, b->threads, rows, eb, L);
        b->obs_first[i] = (int)obs.size();
        b->obs_count[i] = (int)L.size();
        obs.insert(obs.end(), L.begin(), L.end());
        all.insert(all.end(), L.begin(), L.end());
    }
    // the two-step list: its own width (as for a single lattice) and one rows value for all
    // instances, fitted like the single step's but with the twelve warm-up rows
    std::vector<Tile> all2;
    b->rows2 = 0;
    int64_t nodes = 0;
    for (int i = 0; i < b->count; ++i) nodes += (int64_t)b->inst[i].kp.nx * b->inst[i].kp.ny;
    const bool want2 = b->pair_mode == 2 || (b->pair_mode == 0 && nodes >= ((int64_t)1 << 20));
    // two-step width: 128 columns unless the instances are wide (a 256-wide workgroup leaves
    // half its lanes idle on a 128-wide instance; measured on the 64-instance sweep with sides
    // 128-512: 27.7k MLUPS at 128 against 26.2k at 256, and never slower per size class)
    int max_side = 0;
    for (int i = 0; i < b->count; ++i) max_side = std::max(max_side, b->inst[i].kp.nx);
    const int t2 = std::min(b->tile_set ? 256 : (max_side >= 768 ? 256 : 128), b->threads);
    const int slots2 = want2 ? device_slots_pair(b->prec, t2) : 0;
    if (slots2 > 0) {
        double best2 = 1e300;
        for (int r : {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512}) {
            long tiles = 0;
            for (int i = 0; i < b->count; ++i) {
                std::vector<Tile> L;
                plan_lattice(i, b->inst[i].kp.nx, b->inst[i].kp.ny, t2, r, eb, L, 6);
                tiles += (long)L.size();
            }
            const double cost = (double)((tiles + slots2 - 1) / slots2) * (r + 12);
            if (cost < best2) {
                best2 = cost;
                b->rows2 = r;
            }
        }
        for (int i = 0; i < b->count; ++i)
            plan_lattice(i, b->inst[i].kp.nx, b->inst[i].kp.ny, t2, b->rows2, eb, all2, 6);
    }
    b->threads2 = t2;
    std::vector<Tile> T = xcd_order(all, 8), T2 = xcd_order(all2, 8);
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->dtiles) (void)hipFree(b->dtiles);
    if (b->dtiles2) (void)hipFree(b->dtiles2);
    if (b->dobs) (void)hipFree(b->dobs);
    b->dtiles = b->dtiles2 = nullptr;
    b->dobs = nullptr;
    b->ntiles = b->ntiles2 = 0;
    hipError_t e = hipMalloc((void**)&b->dtiles, T.size() * sizeof(Tile));
    if (e == hipSuccess) e = hipMalloc((void**)&b->dobs, obs.size() * sizeof(Tile));
    if (e == hipSuccess && !T2.empty()) e = hipMalloc((void**)&b->dtiles2, T2.size() * sizeof(Tile));
    if (e == hipSuccess) e = hipMemcpy(b->dtiles, T.data(), T.size() * sizeof(Tile), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->dobs, obs.data(), obs.size() * sizeof(Tile), hipMemcpyHostToDevice);
    if (e == hipSuccess && !T2.empty())
        e = hipMemcpy(b->dtiles2, T2.data(), T2.size() * sizeof(Tile), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch tile plan upload");
    b->ntiles = (int)T.size();
    b->ntiles2 = (int)T2.size();
    return LBM3_OK;
}

static int ensure_batch_staging(lbm3_batch* b, size_t doubles)
{
    if (b->staging_cap >= doubles) return LBM3_OK;
    if (b->staging) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipFree(b->staging);
        b->staging = nullptr;
        b->staging_cap = 0;
    }
    hipError_t e = hipMalloc((void**)&b->staging, doubles * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(batch staging)");
    b->staging_cap = doubles;
    return LBM3_OK;
}

// One launch from buffer c of the steady-state step (one step) or of the two-step pass
// (two steps); either way the result is in buffer c ^ 1.  With FP32 storage the launch takes
// its rounding salt from the device step counter and is followed by the counter's advance,
// so that a captured graph rounds every replay with the salts of the absolute steps it runs
// (the same as a lattice stepped alone).
static hipError_t launch_steady(lbm3_batch* b, int c, bool two, int64_t step)
{
    hipError_t e;
    if (two)
        e = launch_pair(b->prec, b->buf[c], b->buf[c ^ 1], b->dinst, b->dtiles2, b->ntiles2, b->threads2, step,
                        b->stream, b->pt, b->dstep);
    else
        e = launch_tiles(b->prec, Fmt::FAC, Fmt::FAC, b->buf[c], b->buf[c ^ 1], b->dinst, b->dtiles, b->ntiles,
                         b->threads, step, 0, b->stream, b->pt, b->dstep);
    if (e == hipSuccess && b->dstep) e = launch_advance_step(b->dstep, two ? 2 : 1, b->stream);
    return e;
}

// Captures launches worth kGraphSteps steps starting from buffer `parity` (an even number
// of launches either way, so the graph ends on the buffer it started from).
static int build_graph(lbm3_batch* b, int parity)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int c = parity;
    hipError_t le = hipSuccess;
    const bool two = b->ntiles2 > 0;
    for (int s = 0; s < kGraphSteps && le == hipSuccess; s += two ? 2 : 1) {
        le = launch_steady(b, c, two, s);
        c ^= 1;
    }
    e = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "fused-step launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->exec[parity] = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return LBM3_OK;
}

extern "C" {

int lbm3_batch_destroy(lbm3_batch_t* b)
{
    if (!b) return LBM3_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    free_state_pair(b->buf);
    if (b->dinst) (void)hipFree(b->dinst);
    if (b->dtiles) (void)hipFree(b->dtiles);
    if (b->dtiles2) (void)hipFree(b->dtiles2);
    if (b->dobs) (void)hipFree(b->dobs);
    if (b->staging) (void)hipFree(b->staging);
    if (b->partials) (void)hipFree(b->partials);
    if (b->obs_dev) (void)hipFree(b->obs_dev);
    if (b->obs_host) (void)hipHostFree(b->obs_host);
    if (b->dstep) (void)hipFree(b->dstep);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LBM3_OK;
}

int lbm3_batch_create(const lbm3_params* p, int32_t count, void* hip_stream, lbm3_batch_t** out)
{
    if (!out) {
        set_error("out is NULL");
        return LBM3_EINVAL;
    }
    *out = nullptr;
    if (!p || count < 1) {
        set_error("batch needs count >= 1 parameter sets");
        return LBM3_EINVAL;
    }
    for (int i = 0; i < count; ++i) {
        int rc = validate_params(&p[i]);
        if (rc) return rc;
        if (p[i].precision != p[0].precision) {
            set_error("all instances of a batch must have the same precision");
            return LBM3_EINVAL;
        }
        if (p[i].forcing != p[0].forcing) {
            set_error("all instances of a batch must have the same forcing (instance %d)", i);
            return LBM3_EINVAL;
        }
    }
    lbm3_batch* b = new (std::nothrow) lbm3_batch();
    if (!b) {
        set_error("host allocation failed");
        return LBM3_ENOMEM;
    }
    b->count = count;
    b->prec = prec_of(p[0].precision);
    b->pt = p[0].forcing == LBM3_FORCING_PERTURBATION;
    b->inst.resize(count);
    b->ready.assign(count, 0);
    b->fmt.assign(count, Fmt::F27);
    int64_t total = 0;
    int max_side = 0;
    for (int i = 0; i < count; ++i) {
        derive(&p[i], &b->inst[i].kp, nullptr, nullptr, nullptr);
        b->inst[i].offset = total;
        total += (b->inst[i].kp.span + 255) / 256 * 256;
        max_side = std::max(max_side, std::max(p[i].nx, p[i].ny));
    }
    b->threads = max_side >= 2000 ? 512 : (max_side >= 500 ? 256 : (max_side >= 124 ? 128 : 64));
    hipError_t e = hipSuccess;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        // graph capture needs a stream other than the null stream
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        b->own_stream = e == hipSuccess;
    }
    const size_t bytes = (size_t)total * elem_bytes(b->prec);
    if (e == hipSuccess) e = alloc_state_pair(bytes, b->buf);
    if (e == hipSuccess) e = hipMalloc((void**)&b->dinst, count * sizeof(Instance));
    if (e == hipSuccess)
        e = hipMemcpy(b->dinst, b->inst.data(), count * sizeof(Instance), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&b->obs_dev, kObsFields * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->obs_host, kObsFields * sizeof(double));
    if (e == hipSuccess && b->prec == Prec::F32S) {
        const int64_t zero = 0;
        e = hipMalloc((void**)&b->dstep, sizeof(int64_t));
        if (e == hipSuccess) e = hipMemcpy(b->dstep, &zero, sizeof zero, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        int rc = hip_fail(e, "batch allocation");
        lbm3_batch_destroy(b);
        return rc;
    }
    int rc = batch_plan(b);
    if (rc) {
        lbm3_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM3_OK;
}

int lbm3_batch_set_tile(lbm3_batch_t* b, int32_t side, int32_t threads, int32_t rows)
{
    if (!b) {
        set_error("batch is NULL");
        return LBM3_EINVAL;
    }
    if (!(threads == 64 || threads == 128 || threads == 256 || threads == 512) || rows < 0 || side < 0) {
        set_error("threads must be 64, 128, 256 or 512; rows >= 0; side >= 0");
        return LBM3_EINVAL;
    }
    if (side == 0) {
        b->threads = threads;
        b->tile_set = true;
        if (rows > 0)
            for (auto& kv : b->rows_by_side) kv.second = rows;
    } else {
        if (threads != b->threads) {
            set_error("one launch covers all instances: threads must match the batch's (%d); "
                      "set it with side = 0 first", b->threads);
            return LBM3_EINVAL;
        }
        b->rows_by_side[side] = rows;
    }
    return batch_plan(b);
}

int lbm3_batch_set_steps_per_launch(lbm3_batch_t* b, int32_t mode)
{
    if (!b) {
        set_error("batch is NULL");
        return LBM3_EINVAL;
    }
    if (mode < 0 || mode > 2) {
        set_error("mode must be 0 (by size), 1 or 2");
        return LBM3_EINVAL;
    }
    b->pair_mode = mode;
    return batch_plan(b);
}

int lbm3_batch_get_pair_launch(const lbm3_batch_t* b, int32_t* steps, int32_t* threads, int32_t* rows,
                               int32_t* workgroups)
{
    if (!b) {
        set_error("batch is NULL");
        return LBM3_EINVAL;
    }
    const bool two = b->ntiles2 > 0;
    if (steps) *steps = two ? 2 : 1;
    if (threads) *threads = two ? (b->prec == Prec::F32 ? 1 : 2) * b->threads2 : 0;
    if (rows) *rows = two ? b->rows2 : 0;
    if (workgroups) *workgroups = two ? b->ntiles2 : 0;
    return LBM3_OK;
}

int lbm3_batch_init_fields(lbm3_batch_t* b, int32_t idx, const double* rho, const double* u)
{
    if (!b || idx < 0 || idx >= b->count) {
        set_error("batch is NULL or instance index out of range");
        return LBM3_EINVAL;
    }
    const KParams& kp = b->inst[idx].kp;
    const int64_t n = (int64_t)kp.nx * kp.ny;
    int rc = check_rho_fields(rho, u, n);
    if (!rc) rc = ensure_batch_staging(b, (size_t)5 * n);
    if (rc) return rc;
    const size_t eb = elem_bytes(b->prec);
    char* base = (char*)b->buf[b->cur] + (size_t)b->inst[idx].offset * eb;
    hipError_t e = hipMemcpyAsync(b->staging, rho, 3 * n * sizeof(double), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && u)
        e = hipMemcpyAsync(b->staging + 3 * n, u, 2 * n * sizeof(double), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = launch_init(b->prec, b->staging, u ? b->staging + 3 * n : nullptr, base, kp, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch init_fields");
    b->ready[idx] = 1;
    b->fmt[idx] = Fmt::F27;
    return LBM3_OK;
}

int lbm3_batch_step(lbm3_batch_t* b, int64_t n)
{
    if (!b) {
        set_error("batch is NULL");
        return LBM3_EINVAL;
    }
    if (n < 0) {
        set_error("n must be >= 0");
        return LBM3_EINVAL;
    }
    for (int i = 0; i < b->count; ++i)
        if (!b->ready[i]) {
            set_error("instance %d has not been initialised", i);
            return LBM3_ESTATE;
        }
    if (n > 0) {
        // first step of freshly initialised instances: 27-population -> factored format
        int n27 = 0;
        for (Fmt f : b->fmt) n27 += f == Fmt::F27;
        if (n27 > 0) {
            hipError_t e = hipSuccess;
            if (n27 < b->count) {
                for (int i = 0; i < b->count; ++i) b->inst[i].fmt = (int32_t)b->fmt[i];
                e = hipMemcpyAsync(b->dinst, b->inst.data(), b->count * sizeof(Instance),
                                   hipMemcpyHostToDevice, b->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
                if (e == hipSuccess)
                    e = launch_tiles(b->prec, Fmt::FAC, Fmt::FAC, b->buf[b->cur], b->buf[b->cur ^ 1],
                                     b->dinst, b->dtiles, b->ntiles, b->threads, b->step, 1, b->stream, b->pt);
            }
            if (e == hipSuccess)
                e = launch_tiles(b->prec, Fmt::F27, Fmt::FAC, b->buf[b->cur], b->buf[b->cur ^ 1],
                                 b->dinst, b->dtiles, b->ntiles, b->threads, b->step,
                                 n27 < b->count ? 1 : 0, b->stream, b->pt);
            // these launches took their salt from b->step; keep the device counter in step
            if (e == hipSuccess && b->dstep) e = launch_advance_step(b->dstep, 1, b->stream);
            if (e != hipSuccess) return hip_fail(e, "batch step launch");
            for (auto& f : b->fmt) f = Fmt::FAC;
            b->cur ^= 1;
            b->step += 1;
            n -= 1;
        }
    }
    while (n >= kGraphSteps) {
        if (!b->exec[b->cur]) {
            int rc = build_graph(b, b->cur);
            if (rc) return rc;
        }
        hipError_t e = hipGraphLaunch(b->exec[b->cur], b->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        n -= kGraphSteps;
        b->step += kGraphSteps;
    }
    while (n > 0) {
        const bool two = n >= 2 && b->ntiles2 > 0;
        hipError_t e = launch_steady(b, b->cur, two, b->step);
        if (e != hipSuccess) return hip_fail(e, "batch step launch");
        b->cur ^= 1;
        b->step += two ? 2 : 1;
        n -= two ? 2 : 1;
    }
    return LBM3_OK;
}

int lbm3_batch_observables(lbm3_batch_t* b, int32_t idx, lbm3_obs* out, double* rho_out)
{
    if (!b || idx < 0 || idx >= b->count) {
        set_error("batch is NULL or instance index out of range");
        return LBM3_EINVAL;
    }
    if (!b->ready[idx]) {
        set_error("instance %d has not been initialised", idx);
        return LBM3_ESTATE;
    }
    const KParams& kp = b->inst[idx].kp;
    const int64_t n = (int64_t)kp.nx * kp.ny;
    const int nb = b->obs_count[idx];
    if (b->partials_cap < nb) {
        (void)hipStreamSynchronize(b->stream);
        if (b->partials) (void)hipFree(b->partials);
        b->partials = nullptr;
        b->partials_cap = 0;
        hipError_t e = hipMalloc((void**)&b->partials, (size_t)nb * kObsFields * sizeof(double));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(batch partials)");
        b->partials_cap = nb;
    }
    if (rho_out) {
        int rc = ensure_batch_staging(b, (size_t)3 * n);
        if (rc) return rc;
    }
    hipError_t e = launch_observe_tiles(b->prec, b->fmt[idx], b->buf[b->cur], b->dinst,
                                        b->dobs + b->obs_first[idx], nb, b->threads, b->partials,
                                        rho_out ? b->staging : nullptr, b->stream, b->pt);
    if (e == hipSuccess) e = launch_reduce_obs(b->partials, nb, b->obs_dev, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->obs_host, b->obs_dev, kObsFields * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess && rho_out)
        e = hipMemcpyAsync(rho_out, b->staging, 3 * n * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch observables");
    const double* o = b->obs_host;
    if (out) {
        out->step = b->step;
        for (int k = 0; k < 3; ++k) out->mass[k] = o[k];
        out->momentum[0] = o[3];
        out->momentum[1] = o[4];
        out->kinetic_energy = o[5];
        out->u_max = o[6];
        out->nonfinite = o[7] != 0.0 ? 1 : 0;
    }
    if (o[7] != 0.0) {
        set_error("instance %d is not finite at step %lld", idx, (long long)b->step);
        return LBM3_ENONFINITE;
    }
    return LBM3_OK;
}

}  // extern "C"
