// Host side of the C ABI declared in include/lbm3.h: parameter validation, the FP64
// host precompute of the segregation law, device buffers and stream-ordered launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lbm3_handle.h"

namespace tcg {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

const char* last_error() { return g_err; }

int hip_fail(hipError_t e, const char* what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? LBM3_ENOMEM : LBM3_EDEVICE;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate_params(const lbm3_params* p)
{
    if (!p) {
        set_error("params is NULL");
        return LBM3_EINVAL;
    }
    if (p->nx < 1 || p->ny < 1) {
        set_error("nx and ny must be >= 1 (got %d x %d)", p->nx, p->ny);
        return LBM3_EINVAL;
    }
    // rows are grid rows of the per-node kernels (at most 65535); beyond that the limit is
    // device memory (lbm3_create then returns LBM3_ENOMEM): all element offsets are 64-bit
    if (p->nx > 65535 || p->ny > 65535) {
        set_error("nx and ny must be <= 65535 (got %d x %d)", p->nx, p->ny);
        return LBM3_EINVAL;
    }
    for (int k = 0; k < 3; ++k) {
        if (!finite_pos(p->rho0[k])) {
            set_error("rho0[%d] must be finite and > 0", k);
            return LBM3_EINVAL;
        }
        if (!finite_pos(p->sigma[k])) {
            set_error("sigma[%d] must be finite and > 0", k);
            return LBM3_EINVAL;
        }
        if (!std::isfinite(p->tau[k]) || !(p->tau[k] > 0.5)) {
            set_error("tau[%d] must be finite and > 1/2 (viscosity (tau - 1/2)/3 > 0)", k);
            return LBM3_EINVAL;
        }
    }
    if (p->beta0 != 0.0 && !finite_pos(p->beta0)) {
        set_error("beta0 must be 0 (default 0.7) or finite and > 0");
        return LBM3_EINVAL;
    }
    if (p->boundary != LBM3_PERIODIC) {
        set_error("only periodic boundaries are provided (the model has no wall treatment)");
        return LBM3_EUNSUPPORTED;
    }
    for (int k = 0; k < 3; ++k)
        if (p->wall_wettability[k] != 0.0) {
            set_error("wall wettability is reserved and must be 0");
            return LBM3_EUNSUPPORTED;
        }
    if (p->precision < LBM3_FP64 || p->precision > LBM3_FP32) {
        set_error("precision must be LBM3_FP64, LBM3_FP32_STORAGE or LBM3_FP32");
        return LBM3_EINVAL;
    }
    if (p->beta_law < LBM3_BETA_PAPER || p->beta_law > LBM3_BETA_CONSTANT) {
        set_error("beta_law must be LBM3_BETA_PAPER, _SPENCER, _LECLAIRE or _CONSTANT (got %d)", p->beta_law);
        return LBM3_EINVAL;
    }
    if (p->forcing != LBM3_FORCING_GUO && p->forcing != LBM3_FORCING_PERTURBATION) {
        set_error("forcing must be LBM3_FORCING_GUO or LBM3_FORCING_PERTURBATION (got %d)", p->forcing);
        return LBM3_EINVAL;
    }
    return LBM3_OK;
}

// Pair p of fluids (k, l) and the third fluid m; sigma index of an unordered pair.
static const int PK[3] = {0, 0, 1}, PL[3] = {1, 2, 2};
static int pair_index(int a, int b)
{
    if (a > b) {
        int t = a;
        a = b;
        b = t;
    }
    return a == 0 ? (b == 1 ? 0 : 1) : 2;
}

// g(X) of Eq. (20) with sin(arccos X) = sqrt((1 - X)(1 + X)); within 1e-12 of |X| = 1
// the limiting value is used (g = -1 at X = 1, +1 at X = -1), so that the critical
// states, where X = +-1 exactly in real arithmetic, do not depend on the rounding of X.
static double seg_g(double X)
{
    if (X >= 1.0 - 1e-12) return -1.0;
    if (X <= -1.0 + 1e-12) return 1.0;
    const double s = std::sqrt((1.0 - X) * (1.0 + X));
    return X < 0.0 ? 1.0 - s : s - 1.0;
}

// sin(phi) for the Neumann-triangle angle with cos(phi) = X (Eq. 14), X clamped to [-1, 1]
static double sin_phi(double X)
{
    const double c = std::min(1.0, std::max(-1.0, X));
    return std::sqrt((1.0 - c) * (1.0 + c));
}

// g_kl and the coefficient of s of the comparison laws (Eqs. 15-17), from X_kl = cos(phi_kl).
// A Neumann triangle exists when every |X_kl| is below 1 by more than the 1e-12 of seg_g:
// the critical states (|X| = 1, a degenerate triangle) count as having none.
static void comparison_law(int law, const double X[3], double g[3], double* ct_coef)
{
    *ct_coef = 35.0;
    for (int q = 0; q < 3; ++q) g[q] = 0.0;
    if (law == LBM3_BETA_SPENCER) {
        // as printed: beta_rb takes sin(phi_gb) and beta_gb takes sin(phi_rb); beta_rg = beta0
        g[1] = sin_phi(X[2]) - 1.0;
        g[2] = sin_phi(X[1]) - 1.0;
        *ct_coef = 27.0;
    } else if (law == LBM3_BETA_LECLAIRE) {
        bool triangle = true;
        for (int q = 0; q < 3; ++q) triangle = triangle && std::fabs(X[q]) < 1.0 - 1e-12;
        if (!triangle) return;  // beta_kl = beta0
        double phi[3];
        int qmax = 0;
        for (int q = 0; q < 3; ++q) {
            phi[q] = std::acos(X[q]);
            if (phi[q] > phi[qmax]) qmax = q;  // the first of equal maxima
        }
        for (int q = 0; q < 3; ++q)
            if (q != qmax) g[q] = std::sin(M_PI - phi[qmax] - phi[q]) - 1.0;
    }
    // LBM3_BETA_CONSTANT: all g_kl = 0
}

void derive(const lbm3_params* p, KParams* kp, double X[3], double g[3], double nu[3])
{
    double Xl[3], gl[3], nul[3], ct_coef = 35.0;
    for (int q = 0; q < 3; ++q) {
        const int k = PK[q], l = PL[q], m = 3 - k - l;
        const double smk = p->sigma[pair_index(m, k)], sml = p->sigma[pair_index(m, l)];
        const double skl = p->sigma[q];
        Xl[q] = (smk * smk + sml * sml - skl * skl) / (2.0 * smk * sml);  // Eq. (18)
        gl[q] = seg_g(Xl[q]);
        nul[q] = (p->tau[q] - 0.5) / 3.0;  // Eq. (11) with c_s^2 = 1/3
    }
    if (p->beta_law != LBM3_BETA_PAPER) comparison_law(p->beta_law, Xl, gl, &ct_coef);
    if (X)
        for (int q = 0; q < 3; ++q) X[q] = Xl[q];
    if (g)
        for (int q = 0; q < 3; ++q) g[q] = gl[q];
    if (nu)
        for (int q = 0; q < 3; ++q) nu[q] = nul[q];
    if (kp) {
        std::memset(kp, 0, sizeof *kp);
        kp->nx = p->nx;
        kp->ny = p->ny;
        // the rows of all planes in one contiguous block: the rows a workgroup reads together
        // share DRAM pages
        kp->plane = ((int64_t)p->nx + 63) / 64 * 64;
        kp->pitch = 27 * kp->plane;
        kp->fpitch = kFacPlanes * kp->plane;
        kp->span = kp->pitch * p->ny;
        for (int q = 0; q < 3; ++q) {
            kp->sigma[q] = p->sigma[q];
            kp->g[q] = gl[q];
            kp->inv_nu[q] = 1.0 / nul[q];
            kp->cfac[q] = 1e6 / (p->rho0[PK[q]] * p->rho0[PL[q]]);
        }
        kp->beta0 = p->beta0 == 0.0 ? 0.7 : p->beta0;
        kp->ct_coef = ct_coef;
        kp->guard = p->precision == LBM3_FP32 ? 1e-6 : 1e-12;
    }
}

Prec prec_of(int precision)
{
    return precision == LBM3_FP64 ? Prec::F64 : (precision == LBM3_FP32_STORAGE ? Prec::F32S : Prec::F32);
}

// Default launch shape of the single step, from sweeps on 256^2 to 4096^2 in every
// precision: 64 threads below 384 columns, 128 below 768, then 256 (two workgroups per CU);
// rows fitted to the resident slots (auto_rows).  Narrow strips win on small lattices,
// where more workgroups with short warm-ups beat wide ones (256^2: +2-4%, 512^2: +2-4%).
void default_tile(const KParams& kp, Prec prec, int* threads, int* rows)
{
    (void)prec;
    *threads = kp.nx < 384 ? 64 : (kp.nx < 768 ? 128 : 256);
    *rows = 0;
}

int check_rho_fields(const double* rho, const double* u, int64_t n)
{
    if (!rho) {
        set_error("rho is NULL");
        return LBM3_EINVAL;
    }
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double v = rho[k * n + j];
            if (!std::isfinite(v) || v < 0.0) {
                set_error("rho[%d] at node %lld must be finite and >= 0", k, (long long)j);
                return LBM3_EINVAL;
            }
            s += v;
        }
        if (!(s > 0.0)) {
            set_error("total density must be > 0 at every node (node %lld)", (long long)j);
            return LBM3_EINVAL;
        }
        if (u)
            for (int a = 0; a < 2; ++a)
                if (!std::isfinite(u[a * n + j])) {
                    set_error("u[%d] at node %lld is not finite", a, (long long)j);
                    return LBM3_EINVAL;
                }
    }
    return LBM3_OK;
}

// Builds the tile lists for the handle's launch shape (the single step's and, where the
// two-step pass exists, its own with the wider halo) and uploads them with the one-entry
// instance table.  The two-step pass exists for every precision (64 to 256 threads); rows
// requested explicitly apply to both lists.
// Lattices up to this many nodes take their single steps on the block kernel (measured
// against the row march's single step: 1.7-1.9x faster at 128^2 and 256^2, 1.4-1.5x at
// 512^2 in FP32 and FP32 storage; at 1448^2 the march, 15.2k / 20.6k / 29.4k MLUPS in
// FP64 / FP32 storage / FP32, runs below the two-step pass anyway).
constexpr int64_t kBlockMaxNodes = (int64_t)1 << 20;

int upload_plan(lbm3* h)
{
    int rows = h->rows_request;
    const int eb = (int)elem_bytes(h->prec);
    if (rows <= 0)
        rows = auto_rows(h->kp.nx, h->kp.ny, h->threads, device_slots(h->prec, h->threads), eb);
    std::vector<Tile> L, L2;
    plan_lattice(0, h->kp.nx, h->kp.ny, h->threads, rows, eb, L);
    // The two-step pass halves the traffic per step but needs a 12-row warm-up per tile:
    // it wins on large lattices.  Below, single steps on the block kernel win (measured,
    // square compound droplets, block step vs two-step pass: FP64 12.0k vs 10.2k MLUPS at
    // 512^2, 15.8k vs 16.5k at 768^2, 17.3k vs 20.8k at 1024^2; FP32 storage 17.7k vs 17.3k
    // and FP32 31.2k vs 26.7k at 1024^2).  So pairs from 2^19 nodes in FP64 and above 2^20
    // in FP32 and FP32 storage.  The pass's own default width: 64 columns below 768 (512^2
    // FP64: +6% over 256), else 256 (FP64: 512 lanes, one step per wave group);
    // lbm3_set_tile's width applies to both passes.
    const int64_t min2 = h->prec == Prec::F64 ? (int64_t)1 << 19 : ((int64_t)1 << 20) + 1;
    const bool big = (int64_t)h->kp.nx * h->kp.ny >= min2;
    const bool want2 = h->pass_mode == 2 || (h->pass_mode == 0 && big);
    int t2 = h->tile_set ? h->threads : (h->kp.nx < 768 ? 64 : 256);
    const int slots2 = want2 ? device_slots_pair(h->prec, t2) : 0;
    if (slots2 > 0) {
        int rows2 = h->rows_request;
        if (rows2 <= 0) rows2 = auto_rows(h->kp.nx, h->kp.ny, t2, slots2, eb, 6);
        plan_lattice(0, h->kp.nx, h->kp.ny, t2, rows2, eb, L2, 6);
    }
    h->threads2 = t2;
    // Single steps of a small lattice go to the block kernel (no march warm-up), unless
    // lbm3_set_tile chose a march shape or steps-per-launch mode 2 asks for pairs.
    std::vector<Tile> LB;
    if (!h->tile_set && h->pass_mode != 2 && (int64_t)h->kp.nx * h->kp.ny <= kBlockMaxNodes)
        plan_blocks(0, h->kp.nx, h->kp.ny, kBlockCols, kBlockRows, LB);
    std::vector<Tile> T = xcd_order(L, 8), T2 = xcd_order(L2, 8), TB = xcd_order(LB, 8);
    (void)hipStreamSynchronize(h->stream);
    if (h->dtiles) (void)hipFree(h->dtiles);
    if (h->dtiles2) (void)hipFree(h->dtiles2);
    if (h->dtilesb) (void)hipFree(h->dtilesb);
    h->dtiles = h->dtiles2 = h->dtilesb = nullptr;
    h->ntiles = h->ntiles2 = h->ntilesb = 0;
    hipError_t e = hipMalloc((void**)&h->dtiles, T.size() * sizeof(Tile));
    if (e == hipSuccess && !T2.empty()) e = hipMalloc((void**)&h->dtiles2, T2.size() * sizeof(Tile));
    if (e == hipSuccess && !TB.empty()) e = hipMalloc((void**)&h->dtilesb, TB.size() * sizeof(Tile));
    if (e == hipSuccess && !h->dinst) e = hipMalloc((void**)&h->dinst, sizeof(Instance));
    Instance I{};
    I.kp = h->kp;
    I.offset = 0;
    if (e == hipSuccess) e = hipMemcpy(h->dtiles, T.data(), T.size() * sizeof(Tile), hipMemcpyHostToDevice);
    if (e == hipSuccess && !T2.empty())
        e = hipMemcpy(h->dtiles2, T2.data(), T2.size() * sizeof(Tile), hipMemcpyHostToDevice);
    if (e == hipSuccess && !TB.empty())
        e = hipMemcpy(h->dtilesb, TB.data(), TB.size() * sizeof(Tile), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->dinst, &I, sizeof I, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "tile plan upload");
    h->ntiles = (int)T.size();
    h->ntiles2 = (int)T2.size();
    h->ntilesb = (int)TB.size();
    h->rows = rows;
    return LBM3_OK;
}

// Enqueues n fused steps.  A state in the 27-population format (after init_fields or
// set_state) is converted to the factored format by its first step; from the factored
// format, pairs of steps go through the two-step pass where the plan has one.
int step_handle(lbm3* h, int64_t n)
{
    while (n > 0) {
        hipError_t e;
        int done = 1;
        const bool pt = h->p.forcing == LBM3_FORCING_PERTURBATION;
        if (h->fmt == Fmt::FAC && n >= 2 && h->ntiles2 > 0) {
            e = launch_pair(h->prec, h->buf[h->cur], h->buf[h->cur ^ 1], h->dinst, h->dtiles2, h->ntiles2,
                            h->threads2, h->step, h->stream, pt);
            done = 2;
        } else if (h->fmt == Fmt::FAC && h->ntilesb > 0) {
            e = launch_block(h->prec, h->buf[h->cur], h->buf[h->cur ^ 1], h->dinst, h->dtilesb, h->ntilesb,
                             h->step, h->stream, pt);
        } else {
            e = launch_tiles(h->prec, h->fmt, Fmt::FAC, h->buf[h->cur], h->buf[h->cur ^ 1], h->dinst,
                             h->dtiles, h->ntiles, h->threads, h->step, 0, h->stream, pt);
            h->fmt = Fmt::FAC;
        }
        if (e != hipSuccess) return hip_fail(e, "step launch");
        h->cur ^= 1;
        h->step += done;
        n -= done;
    }
    h->tape_valid = false;
    return LBM3_OK;
}

}  // namespace tcg

using namespace tcg;

// Device scratch of the allocation-free observables call (lbm3_observables_noalloc): the
// per-workgroup partial sums of the observing pass (kObsFields doubles per workgroup, at most
// kNoAllocMaxTiles workgroups) followed by the reduced kObsFields values.  Every GPU the
// library runs on holds its own copy for the life of the process; in host code `scratch` is
// only a stand-in for the symbol, and its device address on each GPU is looked up once, with
// that GPU current, when the first handle on it is created.
constexpr int kNoAllocMaxTiles = 32768;
constexpr size_t kScratchDoubles = (size_t)kNoAllocMaxTiles * kObsFields + kObsFields;
static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_dev;  // by device ordinal; null until looked up

// Looks up this device's address of `scratch` (the current device must be `device`).
static int resolve_scratch(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
    if (g_scratch_dev[device]) return LBM3_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[device] = (double*)p;
    return LBM3_OK;
}

static double* scratch_of(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < (int)g_scratch_dev.size() ? g_scratch_dev[device] : nullptr;
}

// Copies the reduced observables held in h->obs_host into *out (may be NULL); ENONFINITE
// when the state was not finite.
static int finish_obs(lbm3* h, lbm3_obs* out)
{
    const double* o = h->obs_host;
    if (out) {
        out->step = h->step;
        for (int k = 0; k < 3; ++k) out->mass[k] = o[k];
        out->momentum[0] = o[3];
        out->momentum[1] = o[4];
        out->kinetic_energy = o[5];
        out->u_max = o[6];
        out->nonfinite = o[7] != 0.0 ? 1 : 0;
    }
    if (o[7] != 0.0) {
        set_error("state is not finite at step %lld", (long long)h->step);
        return LBM3_ENONFINITE;
    }
    return LBM3_OK;
}

static int ensure_staging(lbm3* h, size_t doubles)
{
    if (h->staging_cap >= doubles) return LBM3_OK;
    if (h->staging) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->staging);
        h->staging = nullptr;
        h->staging_cap = 0;
    }
    hipError_t e = hipMalloc((void**)&h->staging, doubles * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(staging)");
    h->staging_cap = doubles;
    return LBM3_OK;
}

static int ensure_partials(lbm3* h, int nblocks)
{
    if (h->partials_cap >= nblocks) return LBM3_OK;
    if (h->partials) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->partials);
        h->partials = nullptr;
        h->partials_cap = 0;
    }
    hipError_t e = hipMalloc((void**)&h->partials, (size_t)nblocks * kObsFields * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(partials)");
    h->partials_cap = nblocks;
    return LBM3_OK;
}

extern "C" {

const char* lbm3_last_error(void) { return tcg::last_error(); }

int lbm3_derived(const lbm3_params* p, double X[3], double g[3], double nu[3])
{
    int rc = validate_params(p);
    if (rc) return rc;
    derive(p, nullptr, X, g, nu);
    return LBM3_OK;
}

int lbm3_create(const lbm3_params* p, void* hip_stream, lbm3_t** out)
{
    if (!out) {
        set_error("out is NULL");
        return LBM3_EINVAL;
    }
    *out = nullptr;
    int rc = validate_params(p);
    if (rc) return rc;
    lbm3* h = new (std::nothrow) lbm3();
    if (!h) {
        set_error("host allocation failed");
        return LBM3_ENOMEM;
    }
    h->p = *p;
    derive(p, &h->kp, nullptr, nullptr, nullptr);
    h->prec = prec_of(p->precision);
    h->stream = (hipStream_t)hip_stream;
    default_tile(h->kp, h->prec, &h->threads, &h->rows);
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDevice");
    }
    rc = resolve_scratch(h->device);
    if (rc) {
        delete h;
        return rc;
    }
    const size_t bytes = (size_t)h->kp.span * elem_bytes(h->prec);
    e = alloc_state_pair(bytes, h->buf);
    if (e != hipSuccess) {
        rc = hip_fail(e, "hipMalloc(populations)");
        lbm3_destroy(h);
        return rc;
    }
    e = hipMalloc((void**)&h->obs_dev, kObsFields * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->obs_host, kObsFields * sizeof(double));
    if (e != hipSuccess) {
        rc = hip_fail(e, "allocation of observables buffers");
        lbm3_destroy(h);
        return rc;
    }
    rc = upload_plan(h);
    if (rc) {
        lbm3_destroy(h);
        return rc;
    }
    *out = h;
    return LBM3_OK;
}

int lbm3_init_fields(lbm3_t* h, const double* rho, const double* u)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    const int64_t n = (int64_t)h->kp.nx * h->kp.ny;
    int rc = check_rho_fields(rho, u, n);
    if (rc) return rc;
    rc = ensure_staging(h, (size_t)27 * n);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(h->staging, rho, 3 * n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && u)
        e = hipMemcpyAsync(h->staging + 3 * n, u, 2 * n * sizeof(double), hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess)
        e = launch_init(h->prec, h->staging, u ? h->staging + 3 * n : nullptr, h->buf[0], h->kp,
                        h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "init_fields");
    h->cur = 0;
    h->fmt = Fmt::F27;
    h->step = 0;
    h->ready = true;
    h->tape_valid = false;
    h->init_at_rest = (u == nullptr);
    return LBM3_OK;
}

int lbm3_set_state(lbm3_t* h, const double* f)
{
    if (!h || !f) {
        set_error("handle or f is NULL");
        return LBM3_EINVAL;
    }
    const int64_t n = (int64_t)h->kp.nx * h->kp.ny;
    for (int64_t j = 0; j < 27 * n; ++j)
        if (!std::isfinite(f[j])) {
            set_error("f is not finite at element %lld", (long long)j);
            return LBM3_EINVAL;
        }
    int rc = ensure_staging(h, (size_t)27 * n);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(h->staging, f, 27 * n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = launch_import(h->prec, h->staging, h->buf[0], h->kp, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "set_state");
    h->cur = 0;
    h->fmt = Fmt::F27;
    h->step = 0;
    h->ready = true;
    h->tape_valid = false;
    h->init_at_rest = false;
    return LBM3_OK;
}

int lbm3_step(lbm3_t* h, int64_t n)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    if (n < 0) {
        set_error("n must be >= 0");
        return LBM3_EINVAL;
    }
    if (!h->ready) {
        set_error("lbm3_step before lbm3_init_fields / lbm3_set_state");
        return LBM3_ESTATE;
    }
    return step_handle(h, n);
}

int lbm3_observables(lbm3_t* h, lbm3_obs* out, double* rho_out, double* f_out)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    if (!h->ready) {
        set_error("lbm3_observables before lbm3_init_fields / lbm3_set_state");
        return LBM3_ESTATE;
    }
    const int64_t n = (int64_t)h->kp.nx * h->kp.ny;
    int rc = ensure_partials(h, h->ntiles);
    if (!rc && (rho_out || f_out)) rc = ensure_staging(h, (size_t)27 * n);
    if (rc) return rc;
    hipError_t e = launch_observe_tiles(h->prec, h->fmt, h->buf[h->cur], h->dinst, h->dtiles,
                                        h->ntiles, h->threads, h->partials,
                                        rho_out ? h->staging : nullptr, h->stream,
                                        h->p.forcing == LBM3_FORCING_PERTURBATION);
    if (e == hipSuccess) e = launch_reduce_obs(h->partials, h->ntiles, h->obs_dev, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->obs_host, h->obs_dev, kObsFields * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && rho_out)
        e = hipMemcpyAsync(rho_out, h->staging, 3 * n * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream);
    if (e == hipSuccess && f_out) {
        e = launch_export(h->prec, h->fmt, h->buf[h->cur], h->staging, h->kp, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(f_out, h->staging, 27 * n * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "observables");
    return finish_obs(h, out);
}

int lbm3_observables_noalloc(lbm3_t* h, lbm3_obs* out)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    if (!h->ready) {
        set_error("lbm3_observables_noalloc before lbm3_init_fields / lbm3_set_state");
        return LBM3_ESTATE;
    }
    if (h->ntiles > kNoAllocMaxTiles) {
        set_error("lbm3_observables_noalloc: the launch plan has %d workgroups, its static scratch "
                  "holds the partial sums of at most %d (use lbm3_observables, or fewer, taller tiles "
                  "with lbm3_set_tile)", h->ntiles, kNoAllocMaxTiles);
        return LBM3_EINVAL;
    }
    double* base = scratch_of(h->device);
    if (!base) {
        set_error("lbm3_observables_noalloc: no scratch address for device %d", h->device);
        return LBM3_EDEVICE;
    }
    double* partials = base;
    double* reduced = base + (size_t)kNoAllocMaxTiles * kObsFields;
    // every workgroup writes all of its partials and the reduction all of its outputs, so
    // nothing left from an earlier call is read
    hipError_t e = launch_observe_tiles(h->prec, h->fmt, h->buf[h->cur], h->dinst, h->dtiles, h->ntiles,
                                        h->threads, partials, nullptr, h->stream,
                                        h->p.forcing == LBM3_FORCING_PERTURBATION);
    if (e == hipSuccess) e = launch_reduce_obs(partials, h->ntiles, reduced, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->obs_host, reduced, kObsFields * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "observables_noalloc");
    return finish_obs(h, out);
}

int lbm3_destroy(lbm3_t* h)
{
    if (!h) return LBM3_OK;
    (void)hipStreamSynchronize(h->stream);
    free_state_pair(h->buf);
    if (h->staging) (void)hipFree(h->staging);
    if (h->partials) (void)hipFree(h->partials);
    if (h->obs_dev) (void)hipFree(h->obs_dev);
    if (h->obs_host) (void)hipHostFree(h->obs_host);
    if (h->dtiles) (void)hipFree(h->dtiles);
    if (h->dtiles2) (void)hipFree(h->dtiles2);
    if (h->dtilesb) (void)hipFree(h->dtilesb);
    if (h->dinst) (void)hipFree(h->dinst);
    adjoint_destroy(h);
    delete h;
    return LBM3_OK;
}

int lbm3_set_tile(lbm3_t* h, int32_t threads, int32_t rows)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    if (!(threads == 64 || threads == 128 || threads == 256 || threads == 512) || rows < 0) {
        set_error("threads must be 64, 128, 256 or 512 and rows >= 0 (0 = automatic)");
        return LBM3_EINVAL;
    }
    const int old_t = h->threads, old_r = h->rows_request;
    const bool old_set = h->tile_set;
    h->threads = threads;
    h->rows_request = rows;
    h->tile_set = true;
    int rc = upload_plan(h);
    if (rc) {
        h->threads = old_t;
        h->rows_request = old_r;
        h->tile_set = old_set;
        (void)upload_plan(h);
    }
    return rc;
}

int lbm3_get_pair_launch(const lbm3_t* h, int32_t* steps, int32_t* threads, int32_t* workgroups)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    const bool two = h->ntiles2 > 0;
    if (steps) *steps = two ? 2 : 1;
    if (threads) *threads = two ? (h->prec == Prec::F32 ? 1 : 2) * h->threads2 : 0;
    if (workgroups) *workgroups = two ? h->ntiles2 : 0;
    return LBM3_OK;
}

int lbm3_set_steps_per_launch(lbm3_t* h, int32_t mode)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    if (mode < 0 || mode > 2) {
        set_error("mode must be 0 (automatic), 1 or 2");
        return LBM3_EINVAL;
    }
    const int old = h->pass_mode;
    h->pass_mode = mode;
    int rc = upload_plan(h);
    if (rc) {
        h->pass_mode = old;
        (void)upload_plan(h);
    }
    return rc;
}

int lbm3_get_tile(const lbm3_t* h, int32_t* threads, int32_t* rows)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    if (threads) *threads = h->threads;
    if (rows) *rows = h->rows;
    return LBM3_OK;
}

int lbm3_state_buffer(const lbm3_t* h, void** dev_ptr, int32_t* eb, int64_t* plane, int64_t* pitch,
                      int32_t* nplanes)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    const bool fac = h->fmt == Fmt::FAC;
    if (dev_ptr) *dev_ptr = h->buf[h->cur];
    if (eb) *eb = (int32_t)elem_bytes(h->prec);
    if (plane) *plane = h->kp.plane;
    if (pitch) *pitch = fac ? h->kp.fpitch : h->kp.pitch;
    if (nplanes) *nplanes = fac ? kFacPlanes : 27;
    return LBM3_OK;
}

int lbm3_device_copy(void* dst, const void* src, int64_t nbytes, void* hip_stream)
{
    if (!dst || !src || nbytes < 0 || nbytes % 16) {
        set_error("device_copy: non-NULL pointers and nbytes a multiple of 16 required");
        return LBM3_EINVAL;
    }
    hipError_t e = launch_copy(dst, src, nbytes, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "device_copy");
    return LBM3_OK;
}

}  // extern "C"
