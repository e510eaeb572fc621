// The three-dimensional (D3Q19) form of the ternary step: the paper's model (Sec. 2) on the
// standard D3Q19 lattice, FP64, the force of Eq. (7) with Guo's term, any segregation law.
//
// State: the recoloured populations before streaming, 57 planes B[k][i][z][y][x] (pull
// scheme: f_{i,k}(x) = B_{i,k}(x - e_i)), two buffers.  A step is three node-parallel
// kernels:
//   k3_conc     pull; concentrations c_k, densities rho_k, totals f_i -> c[25][N]
//   k3_stress   grad c_k (Eq. 12), pair normals, C_kl, stress T      -> T[6][N], n[9][N]
//   k3_collide  F = div T (Eq. 12 again), collision with Guo's term (Eqs. 1-3, 8-11),
//               recolouring (Eq. 13 with the segregation law)        -> B'[57][N]
// Bytes per update: the state read and written once (912 B) plus the intermediates (the 25
// planes of k3_conc and the 15 of k3_stress, each written and read once: 320 B; neighbour
// re-reads served by the caches).
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "lbm3_handle.h"

namespace tcg {
namespace {

// D3Q19 links: rest, six axis links, twelve edge links; link i odd and i + 1 are opposite.
// Weights 1/3, 1/18, 1/36; c_s^2 = 1/3.
constexpr int L3X[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int L3Y[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int L3Z[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__device__ __forceinline__ double w19(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
constexpr int PK3[3] = {0, 0, 1}, PL3[3] = {1, 2, 2};

struct Geo3 {
    int nx, ny, nz;
    int64_t N;
};

// The node indices of (x, y, z) and its neighbours: the wrapped coordinates at offsets -1,
// 0, +1 per axis, formed once per node (no division per neighbour).
struct Nb3 {
    int64_t zo[3], yo[3];
    int xo[3];
    __device__ __forceinline__ Nb3(const Geo3& g, int x, int y, int z)
    {
        xo[0] = x == 0 ? g.nx - 1 : x - 1, xo[1] = x, xo[2] = x == g.nx - 1 ? 0 : x + 1;
        const int y0 = y == 0 ? g.ny - 1 : y - 1, y2 = y == g.ny - 1 ? 0 : y + 1;
        const int z0 = z == 0 ? g.nz - 1 : z - 1, z2 = z == g.nz - 1 ? 0 : z + 1;
        yo[0] = (int64_t)y0 * g.nx, yo[1] = (int64_t)y * g.nx, yo[2] = (int64_t)y2 * g.nx;
        const int64_t pl = (int64_t)g.nx * g.ny;
        zo[0] = z0 * pl, zo[1] = z * pl, zo[2] = z2 * pl;
    }
    // the node at offset (dx, dy, dz), each in -1..1
    __device__ __forceinline__ int64_t at(int dx, int dy, int dz) const { return zo[dz + 1] + yo[dy + 1] + xo[dx + 1]; }
};

// The post-streaming populations of node (x, y, z): f_{i,k} = B_{i,k}(x - e_i).
__device__ __forceinline__ void pull57(const double* __restrict__ B, const Geo3& g, const Nb3& nb,
                                       double (&f)[3][19])
{
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int64_t src = nb.at(-L3X[i], -L3Y[i], -L3Z[i]);
#pragma unroll
        for (int k = 0; k < 3; ++k) f[k][i] = B[(int64_t)(k * 19 + i) * g.N + src];
    }
}

// The totals f_i and densities rho_k of the pulled populations, summed as they arrive (the
// single populations are not needed again: collision acts on f_i, recolouring on c_k).
__device__ __forceinline__ void pull_sums(const double* __restrict__ B, const Geo3& g, const Nb3& nb,
                                          double (&ft)[19], double (&rk)[3])
{
    rk[0] = rk[1] = rk[2] = 0.0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int64_t src = nb.at(-L3X[i], -L3Y[i], -L3Z[i]);
        const double a = B[(int64_t)i * g.N + src], b = B[(int64_t)(19 + i) * g.N + src],
                     c = B[(int64_t)(38 + i) * g.N + src];
        ft[i] = a + b + c;
        rk[0] += a;
        rk[1] += b;
        rk[2] += c;
    }
}

// Eq. (12) over the nine pairs of opposite links: 3 sum_i w_i e_i [phi(x + e_i) - phi(x - e_i)]
__device__ __forceinline__ void grad19(const double* __restrict__ phi, const Nb3& nb, double (&d)[3])
{
    d[0] = d[1] = d[2] = 0.0;
#pragma unroll
    for (int i = 1; i < 19; i += 2) {
        const double df = phi[nb.at(L3X[i], L3Y[i], L3Z[i])] - phi[nb.at(-L3X[i], -L3Y[i], -L3Z[i])];
        d[0] += w19(i) * L3X[i] * df;
        d[1] += w19(i) * L3Y[i] * df;
        d[2] += w19(i) * L3Z[i] * df;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] *= 3.0;
}

// Blocks of 256 consecutive nodes (x fastest, then y, then z) on a one-dimensional grid.
// Workgroups go to the eight XCDs in turn, and each XCD has its own L2; block b therefore
// takes the node range of logical block xcd_block(b), so that each XCD works through one
// contiguous run of blocks (a slab of z) and finds most of its stencil neighbours in its
// own L2.  The map is a bijection of [0, T) for any T.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t T)
{
    const int64_t x = b & 7, k = b >> 3, q = T >> 3, r = T & 7;
    return x * q + (x < r ? x : r) + k;
}

// (x, y, z) of this thread's node; false past the last node
__device__ __forceinline__ bool node3(const Geo3& g, int& x, int& y, int& z)
{
    const int64_t n = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (n >= g.N) return false;
    // N <= 2^31 (checked at creation): 32-bit division suffices
    const uint32_t n32 = (uint32_t)n, nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
    const uint32_t p = n32 / nx, zz = p / ny;
    x = (int)(n32 - p * nx), y = (int)(p - zz * ny), z = (int)zz;
    return true;
}

__global__ __launch_bounds__(256) void k3_conc(const double* __restrict__ B, Geo3 g, double* __restrict__ c)
{
    int x, y, z;
    if (!node3(g, x, y, z)) return;
    const Nb3 nb(g, x, y, z);
    double ft[19], rk[3];
    pull_sums(B, g, nb, ft, rk);
    const double ir = 1.0 / (rk[0] + rk[1] + rk[2]);
    const int64_t j = nb.at(0, 0, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c[k * g.N + j] = rk[k] * ir;
        c[(3 + k) * g.N + j] = rk[k];
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) c[(6 + i) * g.N + j] = ft[i];
}

// Stress T = sum_pairs sigma C (|G|^2 I - G G^T)/|G| (xx, xy, xz, yy, yz, zz) and the pair
// normals n_kl (zero at or below the guard), from c_k and rho_k of k3_conc.
__global__ __launch_bounds__(256) void k3_stress(const double* __restrict__ c, Geo3 g, KParams kp,
                                                 double* __restrict__ T, double* __restrict__ nrm)
{
    int x, y, z;
    if (!node3(g, x, y, z)) return;
    const Nb3 nb(g, x, y, z);
    const int64_t j = nb.at(0, 0, 0);
    double gc[3][3], cc[3], rk[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        grad19(c + k * g.N, nb, gc[k]);
        cc[k] = c[k * g.N + j];
        rk[k] = c[(3 + k) * g.N + j];
    }
    double t[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int k = PK3[p], l = PL3[p];
        double G[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) G[a] = cc[l] * gc[k][a] - cc[k] * gc[l][a];
        const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        double n[3] = {0.0, 0.0, 0.0};
        if (g2 > kp.guard * kp.guard) {
            const double m = sqrt(g2), im = 1.0 / m;
#pragma unroll
            for (int a = 0; a < 3; ++a) n[a] = G[a] * im;
            double cf = kp.cfac[p] * (rk[k] * rk[l]);
            cf = cf < 1.0 ? cf : 1.0;
            const double s = kp.sigma[p] * cf * m;  // sigma C |G| (I - n n)
            t[0] += s * (1.0 - n[0] * n[0]);
            t[1] -= s * (n[0] * n[1]);
            t[2] -= s * (n[0] * n[2]);
            t[3] += s * (1.0 - n[1] * n[1]);
            t[4] -= s * (n[1] * n[2]);
            t[5] += s * (1.0 - n[2] * n[2]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) nrm[(3 * p + a) * g.N + j] = n[a];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) T[q * g.N + j] = t[q];
}

// F_b = sum_a d_a T_ab with the symmetric T stored as (xx, xy, xz, yy, yz, zz)
__device__ __forceinline__ void force19(const double* __restrict__ T, const Geo3& g, const Nb3& nb,
                                        double (&F)[3])
{
    constexpr int Q[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    F[0] = F[1] = F[2] = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double d[3];
            grad19(T + Q[a][b] * g.N, nb, d);
            F[b] += d[a];
        }
}

template <bool OBS>
__global__ __launch_bounds__(256) void k3_collide(const double* __restrict__ C6, const double* __restrict__ T,
                                                  const double* __restrict__ nrm, Geo3 g, KParams kp,
                                                  double* __restrict__ Bout, double* __restrict__ partials)
{
    __shared__ double red[OBS ? 8 : 1][256];
    int x, y, z;
    const bool live = node3(g, x, y, z);
    const int t = threadIdx.x;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (live) {
        const Nb3 nb(g, x, y, z);
        const int64_t j = nb.at(0, 0, 0);
        // the densities and totals k3_conc pulled
        double rk[3], ft[19];
#pragma unroll
        for (int k = 0; k < 3; ++k) rk[k] = C6[(3 + k) * g.N + j];
#pragma unroll
        for (int i = 0; i < 19; ++i) ft[i] = C6[(6 + i) * g.N + j];
        const double rho = rk[0] + rk[1] + rk[2], irho = 1.0 / rho;
        double F[3];
        force19(T, g, nb, F);
        double m[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            m[0] += ft[i] * L3X[i];
            m[1] += ft[i] * L3Y[i];
            m[2] += ft[i] * L3Z[i];
        }
        double u[3], uu = 0.0, uF = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u[a] = (m[a] + 0.5 * F[a]) * irho;
            uu += u[a] * u[a];
            uF += u[a] * F[a];
        }
        if constexpr (OBS) {
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k] = rk[k];
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[3 + a] = rho * u[a];
            acc[6] = 0.5 * rho * uu;
            acc[7] = sqrt(uu);
        } else {
            // tau = 3 nu + 1/2 with rho / nu = sum_k rho_k / nu_k (Eqs. 10-11)
            const double rho_over_nu = rk[0] * kp.inv_nu[0] + rk[1] * kp.inv_nu[1] + rk[2] * kp.inv_nu[2];
            const double itau = rho_over_nu / (3.0 * rho + 0.5 * rho_over_nu);
            const double pref = 1.0 - 0.5 * itau;
            double fd[19];
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const double eu = L3X[i] * u[0] + L3Y[i] * u[1] + L3Z[i] * u[2];
                const double eF = L3X[i] * F[0] + L3Y[i] * F[1] + L3Z[i] * F[2];
                const double feq = w19(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
                const double phi = w19(i) * pref * (3.0 * (eF - uF) + 9.0 * eu * eF);
                fd[i] = ft[i] - (ft[i] - feq) * itau + phi;
            }
            // C_t and beta_kl of the segregation law; a_p = beta_p rho_k rho_l / rho
            double ct = kp.ct_coef * rk[0] * rk[1] * rk[2] * (irho * irho * irho);
            ct = ct < 1.0 ? ct : 1.0;
            double ap[3];
#pragma unroll
            for (int p = 0; p < 3; ++p) ap[p] = kp.beta0 * (1.0 + ct * kp.g[p]) * (rk[PK3[p]] * rk[PL3[p]]) * irho;
            // V_k = sum_{l != k} a_kl n_kl (n_lk = -n_kl)
            double V[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double n0 = nrm[(0 + a) * g.N + j], n1 = nrm[(3 + a) * g.N + j], n2 = nrm[(6 + a) * g.N + j];
                V[0][a] = ap[0] * n0 + ap[1] * n1;
                V[1][a] = ap[2] * n2 - ap[0] * n0;
                V[2][a] = -(ap[1] * n1 + ap[2] * n2);
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double ck = rk[k] * irho;
#pragma unroll
                for (int i = 0; i < 19; ++i) {
                    const double ve = V[k][0] * L3X[i] + V[k][1] * L3Y[i] + V[k][2] * L3Z[i];
                    Bout[(int64_t)(k * 19 + i) * g.N + j] = ck * fd[i] + w19(i) * ve;
                }
            }
        }
    }
    if constexpr (OBS) {
        // wavefront reductions, then the four wave results in order
        for (int q = 0; q < 7; ++q) acc[q] = wave_sum(acc[q]);
        acc[7] = wave_max(acc[7]);
        if ((t & 63) == 0)
            for (int q = 0; q < 8; ++q) red[q][t >> 6] = acc[q];
        __syncthreads();
        if (t < 8) {
            double v = red[t][0];
            for (int w = 1; w < 4; ++w) v = t < 7 ? v + red[t][w] : fmax(v, red[t][w]);
            partials[(int64_t)blockIdx.x * 8 + t] = v;
        }
    }
}

// B_{i,k}(y) = w_i rho_k(y + e_i): the pulled state is f_{i,k} = w_i rho_k (fluid at rest)
__global__ __launch_bounds__(256) void k3_init(const double* __restrict__ rho, Geo3 g, double* __restrict__ B)
{
    int x, y, z;
    if (!node3(g, x, y, z)) return;
    const Nb3 nb(g, x, y, z);
    const int64_t j = nb.at(0, 0, 0);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int64_t src = nb.at(L3X[i], L3Y[i], L3Z[i]);
#pragma unroll
        for (int k = 0; k < 3; ++k) B[(int64_t)(k * 19 + i) * g.N + j] = w19(i) * rho[k * g.N + src];
    }
}

// the post-streaming populations [3][19][N] and densities [3][N] of the state
__global__ __launch_bounds__(256) void k3_export(const double* __restrict__ B, Geo3 g, double* __restrict__ fout,
                                                 double* __restrict__ rho)
{
    int x, y, z;
    if (!node3(g, x, y, z)) return;
    const Nb3 nb(g, x, y, z);
    const int64_t j = nb.at(0, 0, 0);
    double f[3][19];
    pull57(B, g, nb, f);
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int i = 0; i < 19; ++i) {
            s += f[k][i];
            if (fout) fout[(int64_t)(k * 19 + i) * g.N + j] = f[k][i];
        }
        rho[k * g.N + j] = s;
    }
}

}  // namespace
}  // namespace tcg

using namespace tcg;

struct lbm3d {
    lbm3_params p{};
    KParams kp{};
    Geo3 g{};
    hipStream_t stream = nullptr;
    double* buf[2] = {nullptr, nullptr};
    double* c = nullptr;        // [25][N]: c_k, rho_k, f_i of the pulled state
    double* T = nullptr;        // [6][N]
    double* nrm = nullptr;      // [9][N]
    double* partials = nullptr; // [blocks][8]
    double* staging = nullptr;  // [57][N] for exports and uploads
    int cur = 0;
    int64_t step = 0;
    bool ready = false;
};

static dim3 grid3(const Geo3& g) { return dim3((unsigned)((g.N + 255) / 256)); }

static void release3(lbm3d* h)
{
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (double* q : {h->buf[0], h->buf[1], h->c, h->T, h->nrm, h->partials, h->staging})
        if (q) (void)hipFree(q);
}

// k3_conc and k3_stress of the current state: the fields k3_collide reads
static hipError_t fields3(lbm3d* h)
{
    const dim3 gr = grid3(h->g), bl(256);
    hipLaunchKernelGGL(k3_conc, gr, bl, 0, h->stream, (const double*)h->buf[h->cur], h->g, h->c);
    hipLaunchKernelGGL(k3_stress, gr, bl, 0, h->stream, (const double*)h->c, h->g, h->kp, h->T, h->nrm);
    return hipGetLastError();
}

extern "C" {

int lbm3d_create(const lbm3_params* p, int32_t nz, void* hip_stream, lbm3d_t** out)
{
    if (out) *out = nullptr;
    if (!out) {
        set_error("out is NULL");
        return LBM3_EINVAL;
    }
    int rc = validate_params(p);
    if (rc) return rc;
    if (nz < 1 || nz > 65535) {
        set_error("nz must be in 1..65535 (got %d)", nz);
        return LBM3_EINVAL;
    }
    if ((int64_t)p->nx * p->ny * nz > ((int64_t)1 << 31)) {
        set_error("the D3Q19 form takes at most 2^31 nodes (got %d x %d x %d)", (int)p->nx, (int)p->ny, nz);
        return LBM3_EINVAL;
    }
    if (p->precision != LBM3_FP64) {
        set_error("the D3Q19 form is provided in LBM3_FP64 only");
        return LBM3_EUNSUPPORTED;
    }
    if (p->forcing != LBM3_FORCING_GUO) {
        set_error("the D3Q19 form runs the force of Eq. (7) with Guo's term only");
        return LBM3_EUNSUPPORTED;
    }
    lbm3d* h = new (std::nothrow) lbm3d();
    if (!h) {
        set_error("host allocation failed");
        return LBM3_ENOMEM;
    }
    h->p = *p;
    derive(p, &h->kp, nullptr, nullptr, nullptr);
    h->g = Geo3{p->nx, p->ny, nz, (int64_t)p->nx * p->ny * nz};
    h->stream = (hipStream_t)hip_stream;
    const int64_t N = h->g.N;
    const dim3 gr = grid3(h->g);
    const size_t nblocks = (size_t)gr.x * gr.y * gr.z;
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMalloc(&h->buf[b], (size_t)57 * N * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&h->c, (size_t)25 * N * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&h->T, (size_t)6 * N * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&h->nrm, (size_t)9 * N * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&h->partials, nblocks * 8 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&h->staging, (size_t)57 * N * sizeof(double));
    if (e != hipSuccess) {
        rc = hip_fail(e, "hipMalloc (D3Q19 lattice)");
        release3(h);
        delete h;
        return rc;
    }
    *out = h;
    return LBM3_OK;
}

int lbm3d_init_fields(lbm3d_t* h, const double* rho)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    const int64_t N = h->g.N;
    int rc = check_rho_fields(rho, nullptr, N);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(h->staging, rho, (size_t)3 * N * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k3_init, grid3(h->g), dim3(256), 0, h->stream, (const double*)h->staging, h->g,
                           h->buf[0]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "D3Q19 init");
    h->cur = 0;
    h->step = 0;
    h->ready = true;
    return LBM3_OK;
}

int lbm3d_step(lbm3d_t* h, int64_t n)
{
    if (!h || n < 0) {
        set_error(!h ? "handle is NULL" : "n must be >= 0");
        return LBM3_EINVAL;
    }
    if (!h->ready) {
        set_error("lbm3d_step before lbm3d_init_fields");
        return LBM3_ESTATE;
    }
    for (int64_t s = 0; s < n; ++s) {
        hipError_t e = fields3(h);
        if (e == hipSuccess) {
            hipLaunchKernelGGL((k3_collide<false>), grid3(h->g), dim3(256), 0, h->stream, (const double*)h->c,
                               (const double*)h->T, (const double*)h->nrm, h->g, h->kp, h->buf[h->cur ^ 1], nullptr);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return hip_fail(e, "D3Q19 step launch");
        h->cur ^= 1;
        h->step += 1;
    }
    return LBM3_OK;
}

int lbm3d_observables(lbm3d_t* h, lbm3d_obs* out, double* rho_out, double* f_out)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    if (!h->ready) {
        set_error("lbm3d_observables before lbm3d_init_fields");
        return LBM3_ESTATE;
    }
    const dim3 gr = grid3(h->g);
    const size_t nblocks = (size_t)gr.x * gr.y * gr.z;
    const int64_t N = h->g.N;
    hipError_t e = fields3(h);
    if (e == hipSuccess) {
        hipLaunchKernelGGL((k3_collide<true>), gr, dim3(256), 0, h->stream, (const double*)h->c,
                           (const double*)h->T, (const double*)h->nrm, h->g, h->kp, (double*)nullptr, h->partials);
        e = hipGetLastError();
    }
    std::vector<double> part(nblocks * 8);
    if (e == hipSuccess)
        e = hipMemcpyAsync(part.data(), h->partials, part.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && (rho_out || f_out)) {
        // the densities go to c (rewritten by the next step's k3_conc)
        hipLaunchKernelGGL(k3_export, gr, dim3(256), 0, h->stream, (const double*)h->buf[h->cur], h->g,
                           f_out ? h->staging : nullptr, h->c);
        e = hipGetLastError();
        if (e == hipSuccess && rho_out)
            e = hipMemcpyAsync(rho_out, h->c, (size_t)3 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && f_out)
            e = hipMemcpyAsync(f_out, h->staging, (size_t)57 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "D3Q19 observables");
    lbm3d_obs o{};
    o.step = h->step;
    bool finite = true;
    for (size_t b = 0; b < nblocks; ++b) {
        for (int q = 0; q < 7; ++q) {
            const double v = part[b * 8 + q];
            if (!std::isfinite(v)) finite = false;
            if (q < 3) o.mass[q] += v;
            else if (q < 6) o.momentum[q - 3] += v;
            else o.kinetic_energy += v;
        }
        const double um = part[b * 8 + 7];
        if (!std::isfinite(um)) finite = false;
        o.u_max = std::max(o.u_max, um);
    }
    o.nonfinite = finite ? 0 : 1;
    if (out) *out = o;
    if (!finite) {
        set_error("the D3Q19 state is not finite at step %lld", (long long)h->step);
        return LBM3_ENONFINITE;
    }
    return LBM3_OK;
}

int lbm3d_destroy(lbm3d_t* h)
{
    if (!h) return LBM3_OK;
    release3(h);
    delete h;
    return LBM3_OK;
}

}  // extern "C"
