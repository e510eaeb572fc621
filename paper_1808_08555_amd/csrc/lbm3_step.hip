// The fused ternary colour-gradient LBM time step for CDNA4 (gfx950), and its
// companion kernels (initial state, import/export of post-streaming populations,
// observables, device copy).
//
// One time step (Yu, Liu, Liang, Zhang, arXiv:1808.08555, Sec. 2) at node x:
//   pull:     f_{i,k}(x) = buffer_{i,k}(x - e_i)           (streaming, Eq. 22)
//   moments:  rho_k = sum_i f_{i,k}, f_i = sum_k f_{i,k}, c_k = rho_k / rho
//   gradient: grad c_k by the isotropic difference of Eq. (12)
//   stress:   T = sum over pairs sigma_kl C_kl |G_kl| (I - n_kl n_kl)   (Eq. 7, the
//             ordered double sum with 1/2 collapsed to one term per unordered pair,
//             since G_lk = -G_kl), C_kl of Eq. (6), G_kl = c_l grad c_k - c_k grad c_l
//   force:    F = div T, again with the difference of Eq. (12)
//   collide:  local tau from the harmonic viscosity mean (Eqs. 10-11), u with the
//             half force (Eq. 9), f_eq (Eq. 3), Guo term (Eq. 8), BGK (Eqs. 1-2)
//   recolour: f_{i,k} = c_k f_dag_i + w_i V_k . e_i, V_k = sum_{l != k} beta_kl
//             (rho_k rho_l / rho) n_kl with beta_kl of Eqs. (19)-(20)       (Eq. 13)
//   store:    buffer'_{i,k}(x) = f_ddag_{i,k}(x)
//
// Layout: population q = k*9 + i of node (x, y) at element q*plane + y*pitch + x, x fastest,
// so a wavefront's 64 lanes read and write 64 consecutive values of one plane row.  The
// host chooses the strides (see derive()): rows of the 27 planes interleaved
// (plane = padded nx, pitch = 27 plane), or whole planes one after another.
//
// Work decomposition (y-marching strips).  A workgroup of NT threads owns a strip of
// NT-4 output columns and a run of `rows` output rows.  Thread t sits on column
// x0 - 2 + t and marches up the rows.  Per input row it pulls its 27 populations once
// (stage 1) and keeps only the 9 totals and 3 densities in a three-deep register
// pipeline; the concentrations go to a three-row LDS ring.  One row behind, stage 2
// forms the colour gradients, pair normals and the stress T (three-row LDS ring);
// two rows behind, stage 3 takes the divergence of T and finishes collision and
// recolouring for the output row, writing 27 values.  Every population is thus read
// from HBM once per step (plus a 2-column and 4-row halo that other workgroups also
// read) and written once; densities, gradients and stress never leave the chip.
#include "lbm3_internal.h"

#ifndef LBM3_NT_STORE
#define LBM3_NT_STORE 0
#endif

namespace tcg {
namespace {

constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// D2Q9 weights.  In FP64 the rest weight is taken as 1 - 4 w_1 - 4 w_5, the double one
// ulp above the nearest to 4/9, so that the nine weights sum to exactly 1: with the nearest
// doubles the sum is 1 - 5.55e-17 and every collision would scale the mass by that much.
template <typename C>
__device__ __forceinline__ constexpr C wgt(int i)
{
    if constexpr (sizeof(C) == 8)
        return i == 0 ? 1.0 - 4.0 * (1.0 / 9.0) - 4.0 * (1.0 / 36.0)
                      : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    else
        return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
}

// 32-bit integer mixer ("lowbias32", from Wellons' hash-prospector search): a bijection with
// low output bias, used as a counter-based generator keyed by (step, node, population).
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// FP64 -> FP32 with stochastic rounding: v plus a uniform offset in [-ulp/2, ulp/2) of the
// float grid at v, then round to nearest, so the rounding error has zero mean.  Round to
// nearest would lose the sub-ulp per-step changes of the near-uniform bulk with a sign that
// is the same at many nodes, which shows up as a steady drift of each fluid's mass.
__device__ __forceinline__ float round_stochastic(double v, uint32_t bits)
{
    const float t = (float)v;
    const uint32_t e = __float_as_uint(t) & 0x7f800000u;
    const float ulp = e > (23u << 23) ? __uint_as_float(e - (23u << 23)) : 0.0f;
    const double r = ((double)(bits >> 8) * (1.0 / 16777216.0) - 0.5) * (double)ulp;
    return (float)(v + r);
}

// Store of one population in the storage type S from the compute type C.
template <typename S, typename C>
__device__ __forceinline__ S to_storage(C v, uint32_t key)
{
    if constexpr (sizeof(S) == 4 && sizeof(C) == 8)
        return round_stochastic(v, mix32(key));
    else
        return S(v);
}

__device__ __forceinline__ int wrapi(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Row pointers that are the same in every lane are rebuilt from scalar registers in the
// global address space, opaque to the optimiser, so that they are not re-associated with
// the per-lane column offset (which would turn every access into a hoisted 64-bit
// per-lane address) and every access compiles to the scalar-base + 32-bit vector-offset
// form of the global load/store.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T ld_at(const T* base, unsigned byte_off)
{
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) T gT;
    gchar* b = (gchar*)uniform_u64(reinterpret_cast<uint64_t>(base));
    return *(gT*)(b + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_at(T* base, unsigned byte_off, T v)
{
    typedef __attribute__((address_space(1))) char gchar;
    typedef __attribute__((address_space(1))) T gT;
    gchar* b = (gchar*)uniform_u64(reinterpret_cast<uint64_t>(base));
#if LBM3_NT_STORE
    __builtin_nontemporal_store(v, (gT*)(b + byte_off));
#else
    *(gT*)(b + byte_off) = v;
#endif
}

// Isotropic difference of Eq. (12), 3 sum_i w_i phi(x + e_i) e_i, written as weighted
// differences of opposite neighbours.  The grouping keeps exact zeros for data that
// are mirror-symmetric about the node, also when the compiler fuses multiply-adds.
template <typename C>
__device__ __forceinline__ C ddx(C e, C w, C ne, C nw, C se, C sw)
{
    return C(3) * (C(1.0 / 9.0) * (e - w) + C(1.0 / 36.0) * ((ne - sw) + (se - nw)));
}
template <typename C>
__device__ __forceinline__ C ddy(C n, C s, C ne, C nw, C se, C sw)
{
    return C(3) * (C(1.0 / 9.0) * (n - s) + C(1.0 / 36.0) * ((ne - sw) + (nw - se)));
}

template <typename C>
struct StepConsts {
    C sig[3], g[3], beta0, inv_nu[3], cfac[3], guard;
    __device__ explicit StepConsts(const KParams& kp)
    {
        for (int p = 0; p < 3; ++p) {
            sig[p] = C(kp.sigma[p]);
            g[p] = C(kp.g[p]);
            inv_nu[p] = C(kp.inv_nu[p]);
            cfac[p] = C(kp.cfac[p]);
        }
        beta0 = C(kp.beta0);
        guard = C(kp.guard);
    }
};

// Collision (Eqs. 1-3, 8-11) and recolouring (Eqs. 13, 19, 20) at one node, given the
// totals f[9], densities rk[3], pair normals n[6] (pairs rg, rb, gb) and the force.
// Writes f_ddag into out[k*9 + i]; returns u and rho u for observables.
template <typename C>
__device__ __forceinline__ void collide_recolour(const C (&f)[9], const C (&rk)[3],
                                                 const C (&n)[6], C Fx, C Fy,
                                                 const StepConsts<C>& K, C (&out)[27],
                                                 C& ux, C& uy, C& mxh, C& myh)
{
    const C rho = rk[0] + rk[1] + rk[2];
    const C irho = C(1) / rho;
    // rho / nu = sum_k rho_k / nu_k ; tau = 3 nu + 1/2
    const C rho_over_nu = rk[0] * K.inv_nu[0] + rk[1] * K.inv_nu[1] + rk[2] * K.inv_nu[2];
    const C tau = C(3) * rho / rho_over_nu + C(0.5);
    const C itau = C(1) / tau;
    // rho u = sum_i f_i e_i + F/2
    const C mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const C my = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
    mxh = mx + C(0.5) * Fx;
    myh = my + C(0.5) * Fy;
    ux = mxh * irho;
    uy = myh * irho;
    const C uu = ux * ux + uy * uy;
    const C uF = ux * Fx + uy * Fy;
    const C pref = C(1) - C(0.5) * itau;
    C fd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const C eu = C(EX[i]) * ux + C(EY[i]) * uy;
        const C eF = C(EX[i]) * Fx + C(EY[i]) * Fy;
        const C feq = wgt<C>(i) * rho * (C(1) + C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu);
        const C phi = wgt<C>(i) * pref * (C(3) * (eF - uF) + C(9) * eu * eF);
        fd[i] = f[i] - (f[i] - feq) * itau + phi;
    }
    // C_t and beta_kl of Eq. (19); a_p = beta_p rho_k rho_l / rho
    C ct = C(35) * rk[0] * rk[1] * rk[2] * (irho * irho * irho);
    ct = ct < C(1) ? ct : C(1);
    const C a0 = K.beta0 * (C(1) + ct * K.g[0]) * (rk[0] * rk[1]) * irho;
    const C a1 = K.beta0 * (C(1) + ct * K.g[1]) * (rk[0] * rk[2]) * irho;
    const C a2 = K.beta0 * (C(1) + ct * K.g[2]) * (rk[1] * rk[2]) * irho;
    // V_k = sum_{l != k} a_kl n_kl with n_lk = -n_kl
    const C V[3][2] = {{a0 * n[0] + a1 * n[2], a0 * n[1] + a1 * n[3]},
                       {a2 * n[4] - a0 * n[0], a2 * n[5] - a0 * n[1]},
                       {-(a1 * n[2] + a2 * n[4]), -(a1 * n[3] + a2 * n[5])}};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const C ck = rk[k] * irho;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const C ve = C(EX[i]) * V[k][0] + C(EY[i]) * V[k][1];
            out[k * 9 + i] = ck * fd[i] + wgt<C>(i) * ve;
        }
    }
}

// The y-marching body shared by the stepping and observing kernels.  The workgroup owns
// output columns [x0, x0 + cols) (cols <= NT - 4) and output rows [y0, y0 + rows).
// Loop-carried per-thread state at the top of iteration j (input row j):
//   vn     = the 27 raw populations of row j, loaded one iteration ahead so that the loads
//            are in flight while the previous row's stages 2 and 3 compute;
//   fA, rA = totals and densities of row j-1;  fB, rB = those of row j-2;
//   nB     = pair normals of row j-2 (formed by stage 2 of the previous iteration).
// LDS rings are indexed by input row mod 3.
template <typename S, typename C, int NT, bool OBS>
__device__ __forceinline__ void march(const S* __restrict__ fin, S* __restrict__ fout,
                                      const KParams& kp, int x0, int y0, int rows, int cols,
                                      C (*cring)[3][NT], C (*tring)[3][NT], double (&acc)[kObsFields],
                                      double* __restrict__ rho_out, uint32_t salt)
{
    const int nx = kp.nx, ny = kp.ny;
    const int64_t plane = kp.plane, pitch = kp.pitch;
    const int t = threadIdx.x;
    const int xr = x0 - 2 + t;
    const int x = wrapi(xr, nx);
    // source column for e_x = -1, 0, +1 as byte offsets from a uniform row pointer
    const unsigned scol[3] = {(unsigned)wrapi(x + 1, nx) * (unsigned)sizeof(S),
                              (unsigned)x * (unsigned)sizeof(S),
                              (unsigned)wrapi(x - 1, nx) * (unsigned)sizeof(S)};
    const unsigned xoff = (unsigned)x * (unsigned)sizeof(S);
    const bool in1 = t < cols + 4;
    const bool in2 = (t >= 1) && (t <= cols + 2);
    const bool in3 = (t >= 2) && (t <= cols + 1);
    const StepConsts<C> K(kp);

    auto load_row = [&](int j, C (&v)[27]) {
        const int r = wrapi(y0 - 2 + j, ny);
        const int64_t srow[3] = {(int64_t)wrapi(r + 1, ny) * pitch, (int64_t)r * pitch,
                                 (int64_t)wrapi(r - 1, ny) * pitch};
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 9; ++i)
                v[k * 9 + i] = C(ld_at(fin + ((int64_t)(k * 9 + i) * plane + srow[EY[i] + 1]),
                                       scol[EX[i] + 1]));
    };

    C fA[9], fB[9], rA[3], rB[3], nB[6], vn[27];
#pragma unroll
    for (int i = 0; i < 9; ++i) fA[i] = fB[i] = C(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) rA[k] = rB[k] = C(1);
#pragma unroll
    for (int q = 0; q < 6; ++q) nB[q] = C(0);
#pragma unroll
    for (int q = 0; q < 27; ++q) vn[q] = C(1);
    if (in1) load_row(0, vn);

    const int J = rows + 4;
    for (int j = 0; j < J; ++j) {
        const int s0 = j % 3;        // slot of row j
        const int s1 = (j + 2) % 3;  // slot of row j-1
        const int s2 = (j + 1) % 3;  // slot of row j-2 (and j-3 + 3)
        // ---- stage 1: totals, densities, concentrations of row j; prefetch row j+1
        C f0[9], r0[3];
        {
            C v[27];
#pragma unroll
            for (int q = 0; q < 27; ++q) v[q] = vn[q];
            if (in1 && j + 1 < J) load_row(j + 1, vn);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                C sum = C(0);
#pragma unroll
                for (int i = 0; i < 9; ++i) sum += v[k * 9 + i];
                r0[k] = sum;
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) f0[i] = (v[i] + v[9 + i]) + v[18 + i];
            const C irho = C(1) / ((r0[0] + r0[1]) + r0[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k) cring[s0][k][t] = r0[k] * irho;
        }
        __syncthreads();
        // ---- stage 2: gradients, normals and stress of row j-1 (densities rA)
        C nA[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
        if (j >= 2 && in2) {
            C gx[3], gy[3], cc[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const C* N = cring[s0][k];
                const C* M = cring[s1][k];
                const C* S_ = cring[s2][k];
                gx[k] = ddx<C>(M[t + 1], M[t - 1], N[t + 1], N[t - 1], S_[t + 1], S_[t - 1]);
                gy[k] = ddy<C>(N[t], S_[t], N[t + 1], N[t - 1], S_[t + 1], S_[t - 1]);
                cc[k] = M[t];
            }
            C Txx = C(0), Txy = C(0), Tyy = C(0);
            constexpr int PK[3] = {0, 0, 1}, PL[3] = {1, 2, 2};
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int k = PK[p], l = PL[p];
                C Gx, Gy, mag;
                {
                    // The two products of G nearly cancel where a fluid is present only as a
                    // trace; unfused, their rounding matches the plain IEEE evaluation.
#pragma clang fp contract(off)
                    Gx = cc[l] * gx[k] - cc[k] * gx[l];
                    Gy = cc[l] * gy[k] - cc[k] * gy[l];
                    mag = sqrt(Gx * Gx + Gy * Gy);
                }
                if (mag > K.guard) {
                    const C inv = C(1) / mag;
                    nA[2 * p] = Gx * inv;
                    nA[2 * p + 1] = Gy * inv;
                    C cf = K.cfac[p] * (rA[k] * rA[l]);
                    cf = cf < C(1) ? cf : C(1);
                    const C coef = K.sig[p] * cf * inv;
                    Txx += coef * (Gy * Gy);
                    Txy -= coef * (Gx * Gy);
                    Tyy += coef * (Gx * Gx);
                }
            }
            tring[s1][0][t] = Txx;
            tring[s1][1][t] = Txy;
            tring[s1][2][t] = Tyy;
        }
        __syncthreads();
        // ---- stage 3: force, collision, recolouring of row j-2 (fB, rB, nB)
        if (j >= 4 && in3) {
            const int yo = y0 + j - 4;
            C d[3][2];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const C* N = tring[s1][a];  // row j-1
                const C* M = tring[s2][a];  // row j-2
                const C* S_ = tring[s0][a]; // row j-3
                d[a][0] = ddx<C>(M[t + 1], M[t - 1], N[t + 1], N[t - 1], S_[t + 1], S_[t - 1]);
                d[a][1] = ddy<C>(N[t], S_[t], N[t + 1], N[t - 1], S_[t + 1], S_[t - 1]);
            }
            const C Fx = d[0][0] + d[1][1];  // d_x T_xx + d_y T_yx
            const C Fy = d[1][0] + d[2][1];  // d_x T_xy + d_y T_yy
            C out[27], ux, uy, mxh, myh;
            collide_recolour<C>(fB, rB, nB, Fx, Fy, K, out, ux, uy, mxh, myh);
            if constexpr (!OBS) {
                const int64_t orow = (int64_t)yo * pitch;
                const uint32_t key = ((uint32_t)yo * (uint32_t)nx + (uint32_t)x) * 27u ^ salt;
#pragma unroll
                for (int q = 0; q < 27; ++q)
                    st_at(fout + ((int64_t)q * plane + orow), xoff, to_storage<S, C>(out[q], key + (uint32_t)q));
            } else {
                const double rho = double(rB[0]) + double(rB[1]) + double(rB[2]);
                acc[0] += double(rB[0]);
                acc[1] += double(rB[1]);
                acc[2] += double(rB[2]);
                acc[3] += double(mxh);
                acc[4] += double(myh);
                const double uu = double(ux) * double(ux) + double(uy) * double(uy);
                acc[5] += 0.5 * rho * uu;
                const double um = sqrt(uu);
                acc[6] = (um > acc[6] || um != um) ? um : acc[6];
                const bool fin_ok = isfinite(double(rB[0])) && isfinite(double(rB[1])) &&
                                    isfinite(double(rB[2])) && isfinite(double(mxh)) &&
                                    isfinite(double(myh));
                if (!fin_ok) acc[7] = 1.0;
                if (rho_out) {
                    const int64_t N = (int64_t)nx * ny;
                    const int64_t o = (int64_t)yo * nx + x;
                    rho_out[o] = double(rB[0]);
                    rho_out[N + o] = double(rB[1]);
                    rho_out[2 * N + o] = double(rB[2]);
                }
            }
        }
        // ---- rotate the pipeline
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            fB[i] = fA[i];
            fA[i] = f0[i];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            rB[k] = rA[k];
            rA[k] = r0[k];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) nB[q] = nA[q];
    }
}

template <int NT>
__device__ void block_reduce_obs(double (&acc)[kObsFields], double* __restrict__ partials)
{
    __shared__ double red[kObsFields][NT];
    const int t = threadIdx.x;
#pragma unroll
    for (int a = 0; a < kObsFields; ++a) red[a][t] = acc[a];
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int a = 0; a < kObsFields; ++a) {
                if (a == 6 || a == 7) {
                    const double o = red[a][t + h];
                    red[a][t] = (o > red[a][t] || o != o) ? o : red[a][t];
                } else {
                    red[a][t] += red[a][t + h];
                }
            }
        }
        __syncthreads();
    }
    if (t < kObsFields) partials[(int64_t)blockIdx.x * kObsFields + t] = red[t][0];
}

// One fused time step over a list of tiles: workgroup b takes tiles[b] of instance
// tiles[b].inst (the plain lattice is a list with one instance).  With OBS the workgroup
// instead accumulates the observables of its output nodes into partials[b].
template <typename S, typename C, int NT, bool OBS>
__global__ __launch_bounds__(NT) void k_tiles(const S* __restrict__ fin, S* __restrict__ fout,
                                              const Instance* __restrict__ inst,
                                              const Tile* __restrict__ tiles, uint32_t salt,
                                              double* __restrict__ partials,
                                              double* __restrict__ rho_out)
{
    __shared__ C cring[3][3][NT];
    __shared__ C tring[3][3][NT];
    const Tile tl = tiles[blockIdx.x];
    const KParams kp = inst[tl.inst].kp;
    const int64_t off = inst[tl.inst].offset;
    double acc[kObsFields] = {0, 0, 0, 0, 0, 0, 0, 0};
    march<S, C, NT, OBS>(fin + off, OBS ? nullptr : fout + off, kp, tl.x0, tl.y0, tl.rows, tl.cols,
                         cring, tring, acc, rho_out,
                         salt ^ mix32((uint32_t)tl.inst * 0x9E3779B9U + 0x51ed270bU));
    if constexpr (OBS) block_reduce_obs<NT>(acc, partials);
}

// Fixed-order second pass over the per-workgroup partials (deterministic).
__global__ __launch_bounds__(256) void k_reduce_obs(const double* __restrict__ partials, int n,
                                                    double* __restrict__ out)
{
    __shared__ double red[kObsFields][256];
    const int t = threadIdx.x;
    double acc[kObsFields] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = t; b < n; b += 256) {
#pragma unroll
        for (int a = 0; a < kObsFields; ++a) {
            const double v = partials[(int64_t)b * kObsFields + a];
            if (a == 6 || a == 7)
                acc[a] = (v > acc[a] || v != v) ? v : acc[a];
            else
                acc[a] += v;
        }
    }
#pragma unroll
    for (int a = 0; a < kObsFields; ++a) red[a][t] = acc[a];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int a = 0; a < kObsFields; ++a) {
                if (a == 6 || a == 7) {
                    const double o = red[a][t + h];
                    red[a][t] = (o > red[a][t] || o != o) ? o : red[a][t];
                } else {
                    red[a][t] += red[a][t + h];
                }
            }
        }
        __syncthreads();
    }
    if (t < kObsFields) out[t] = red[t][0];
}

// Initial populations: with u == null f_{i,k} = w_i rho_k, else (rho_k/rho) f_eq_i(rho, u);
// stored so that the next pull reads them back at x (buffer(x - e_i) = f(x)).
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ rho,
                                              const double* __restrict__ u, S* __restrict__ fout,
                                              KParams kp)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    const int nx = kp.nx, ny = kp.ny;
    if (x >= nx) return;
    const int64_t N = (int64_t)nx * ny, j = (int64_t)y * nx + x;
    const C rk[3] = {C(rho[j]), C(rho[N + j]), C(rho[2 * N + j])};
    const C r = (rk[0] + rk[1]) + rk[2];
    C feq[9];
    if (u) {
        const C ux = C(u[j]), uy = C(u[N + j]);
        const C uu = ux * ux + uy * uy;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const C eu = C(EX[i]) * ux + C(EY[i]) * uy;
            feq[i] = wgt<C>(i) * r * (C(1) + C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const C v = u ? (rk[k] / r) * feq[i] : wgt<C>(i) * rk[k];
            const int64_t d = (int64_t)wrapi(y - EY[i], ny) * kp.pitch + wrapi(x - EX[i], nx);
            fout[(int64_t)(k * 9 + i) * kp.plane + d] = S(v);
        }
}

template <typename S>
__global__ __launch_bounds__(256) void k_import(const double* __restrict__ f, S* __restrict__ fout,
                                                KParams kp)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    const int nx = kp.nx, ny = kp.ny;
    if (x >= nx) return;
    const int64_t N = (int64_t)nx * ny, j = (int64_t)y * nx + x;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const int i = q % 9;
        const int64_t d = (int64_t)wrapi(y - EY[i], ny) * kp.pitch + wrapi(x - EX[i], nx);
        fout[(int64_t)q * kp.plane + d] = S(f[q * N + j]);
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_export(const S* __restrict__ fin, double* __restrict__ f,
                                                KParams kp)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    const int nx = kp.nx, ny = kp.ny;
    if (x >= nx) return;
    const int64_t N = (int64_t)nx * ny, j = (int64_t)y * nx + x;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const int i = q % 9;
        const int64_t s = (int64_t)wrapi(y - EY[i], ny) * kp.pitch + wrapi(x - EX[i], nx);
        f[q * N + j] = double(fin[(int64_t)q * kp.plane + s]);
    }
}

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                              int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

template <typename S, typename C, int NT, bool OBS>
hipError_t do_tiles(const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                    int ntiles, uint32_t salt, double* partials, double* rho_out, hipStream_t st)
{
    hipLaunchKernelGGL((k_tiles<S, C, NT, OBS>), dim3(ntiles), dim3(NT), 0, st, (const S*)fin,
                       (S*)fout, inst, tiles, salt, partials, rho_out);
    return hipGetLastError();
}

template <typename S, typename C, int NT>
int occupancy_of()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles<S, C, NT, false>, NT, 0) != hipSuccess)
        return 0;
    return nb;
}

}  // namespace

size_t elem_bytes(Prec p) { return p == Prec::F64 ? 8 : 4; }

uint32_t step_salt(int64_t step)
{
    uint32_t x = (uint32_t)step ^ (uint32_t)(step >> 32) * 0x9E3779B9U;
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

#define LBM3_DISPATCH_NT(FN, S, C, OBS, ...)                          \
    switch (threads) {                                                \
        case 64: return FN<S, C, 64, OBS>(__VA_ARGS__);               \
        case 128: return FN<S, C, 128, OBS>(__VA_ARGS__);             \
        case 256: return FN<S, C, 256, OBS>(__VA_ARGS__);             \
        case 512: return FN<S, C, 512, OBS>(__VA_ARGS__);             \
        default: return hipErrorInvalidValue;                         \
    }

hipError_t launch_tiles(Prec prec, const void* fin, void* fout, const Instance* inst,
                        const Tile* tiles, int ntiles, int threads, int64_t step, hipStream_t st)
{
    const uint32_t salt = step_salt(step);
    switch (prec) {
        case Prec::F64:
            LBM3_DISPATCH_NT(do_tiles, double, double, false, fin, fout, inst, tiles, ntiles, salt,
                             nullptr, nullptr, st);
        case Prec::F32S:
            LBM3_DISPATCH_NT(do_tiles, float, double, false, fin, fout, inst, tiles, ntiles, salt,
                             nullptr, nullptr, st);
        case Prec::F32:
            LBM3_DISPATCH_NT(do_tiles, float, float, false, fin, fout, inst, tiles, ntiles, salt,
                             nullptr, nullptr, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_observe_tiles(Prec prec, const void* fin, const Instance* inst, const Tile* tiles,
                                int ntiles, int threads, double* partials, double* rho_out,
                                hipStream_t st)
{
    switch (prec) {
        case Prec::F64:
            LBM3_DISPATCH_NT(do_tiles, double, double, true, fin, nullptr, inst, tiles, ntiles, 0u,
                             partials, rho_out, st);
        case Prec::F32S:
            LBM3_DISPATCH_NT(do_tiles, float, double, true, fin, nullptr, inst, tiles, ntiles, 0u,
                             partials, rho_out, st);
        case Prec::F32:
            LBM3_DISPATCH_NT(do_tiles, float, float, true, fin, nullptr, inst, tiles, ntiles, 0u,
                             partials, rho_out, st);
    }
    return hipErrorInvalidValue;
}

int blocks_per_cu(Prec prec, int threads)
{
#define LBM3_OCC(S, C)                                         \
    switch (threads) {                                         \
        case 64: return occupancy_of<S, C, 64>();              \
        case 128: return occupancy_of<S, C, 128>();            \
        case 256: return occupancy_of<S, C, 256>();            \
        case 512: return occupancy_of<S, C, 512>();            \
        default: return 0;                                     \
    }
    switch (prec) {
        case Prec::F64: LBM3_OCC(double, double);
        case Prec::F32S: LBM3_OCC(float, double);
        case Prec::F32: LBM3_OCC(float, float);
    }
#undef LBM3_OCC
    return 0;
}

hipError_t launch_reduce_obs(const double* partials, int nblocks, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_obs, dim3(1), dim3(256), 0, st, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_init(Prec prec, const double* rho, const double* u, void* fout,
                       const KParams& kp, hipStream_t st)
{
    dim3 grid((kp.nx + 255) / 256, kp.ny);
    switch (prec) {
        case Prec::F64:
            hipLaunchKernelGGL((k_init<double, double>), grid, dim3(256), 0, st, rho, u,
                               (double*)fout, kp);
            break;
        case Prec::F32S:
            hipLaunchKernelGGL((k_init<float, double>), grid, dim3(256), 0, st, rho, u,
                               (float*)fout, kp);
            break;
        case Prec::F32:
            hipLaunchKernelGGL((k_init<float, float>), grid, dim3(256), 0, st, rho, u,
                               (float*)fout, kp);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_import(Prec prec, const double* f, void* fout, const KParams& kp, hipStream_t st)
{
    dim3 grid((kp.nx + 255) / 256, kp.ny);
    if (prec == Prec::F64)
        hipLaunchKernelGGL((k_import<double>), grid, dim3(256), 0, st, f, (double*)fout, kp);
    else
        hipLaunchKernelGGL((k_import<float>), grid, dim3(256), 0, st, f, (float*)fout, kp);
    return hipGetLastError();
}

hipError_t launch_export(Prec prec, const void* fin, double* f, const KParams& kp, hipStream_t st)
{
    dim3 grid((kp.nx + 255) / 256, kp.ny);
    if (prec == Prec::F64)
        hipLaunchKernelGGL((k_export<double>), grid, dim3(256), 0, st, (const double*)fin, f, kp);
    else
        hipLaunchKernelGGL((k_export<float>), grid, dim3(256), 0, st, (const float*)fin, f, kp);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t st)
{
    const int64_t n = nbytes / 16;
    int64_t blocks = (n + 255) / 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const uint4*)src,
                       (uint4*)dst, n);
    return hipGetLastError();
}

}  // namespace tcg
