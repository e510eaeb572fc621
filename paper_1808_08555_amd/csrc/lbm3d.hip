// The three-dimensional form of the ternary step: the paper's model (Sec. 2) on the standard
// D3Q19 or D3Q27 lattice, the force of Eq. (7) with Guo's term, any segregation law, in
// FP64, FP32, or FP32 storage with FP64 arithmetic (stochastic rounding on store).
//
// State: the recoloured populations before streaming, 3Q planes B[k][i][z][y][x] (pull
// scheme: f_{i,k}(x) = B_{i,k}(x - e_i)), two buffers.  A step is one launch of the fused
// march (k3_march): workgroups own x-y blocks of a z segment and march up z, keeping the
// concentrations and the stress of three planes in LDS rings, so that the state is read
// and written once per update (912 B for D3Q19 in FP64, 1296 B for D3Q27) and nothing else
// goes through HBM.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "lbm3_handle.h"
#include "lbm3_rounding.h"

namespace tcg {
namespace {

// Links: rest, six axis links, twelve edge links (the D3Q19 lattice ends here), eight corner
// links (D3Q27); link i odd and i + 1 are opposite.  c_s^2 = 1/3 on both.  D3Q19 weights 1/3,
// 1/18, 1/36; D3Q27 weights 8/27, 2/27, 1/54, 1/216.  In FP32 the nearest floats sum to
// 1 + 1.5e-8 (D3Q19) and 1 + 7.5e-9 (D3Q27), and every collision would scale the mass by that
// sum (the equilibrium's zeroth moment); the float weights are therefore chosen one ulp off
// where needed so that their sum is exactly 1: D3Q19 one ulp above 1/3 and one ulp below
// 1/18 and 1/36; D3Q27 one ulp below 8/27 and one ulp above 1/54.
constexpr int L3X[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int L3Y[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int L3Z[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
template <typename C, int Q>
__device__ __forceinline__ C w3(int i)
{
    static_assert(Q == 19 || Q == 27, "D3Q19 or D3Q27");
    if constexpr (Q == 19) {
        if constexpr (sizeof(C) == 8)
            return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
        else
            return i == 0 ? 0x1.555558p-2f : (i <= 6 ? 0x1.c71c70p-5f : 0x1.c71c70p-6f);
    } else {
        if constexpr (sizeof(C) == 8)
            return i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
        else
            return i == 0 ? 0x1.2f684ap-2f : (i <= 6 ? 0x1.2f684cp-4f : (i <= 18 ? 0x1.2f684ep-6f : 0x1.2f684cp-8f));
    }
}
constexpr int PK3[3] = {0, 0, 1}, PL3[3] = {1, 2, 2};

struct Geo3 {
    int nx, ny, nz;
    int64_t N;
};

// Loads and stores at a byte offset from a plane's base: with at most 2^29 nodes the
// offset of any node within a plane fits 32 bits, so the uniform base stays in scalar
// registers and each lane holds a 32-bit offset.
template <typename S>
__device__ __forceinline__ S ld_plane(const S* __restrict__ base, uint32_t byte_off)
{
    return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename S>
__device__ __forceinline__ void st_plane(S* __restrict__ base, uint32_t byte_off, S v)
{
    *reinterpret_cast<S*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

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
template <typename S, int Q>
__device__ __forceinline__ void pull3(const S* __restrict__ B, const Geo3& g, const Nb3& nb, double (&f)[3][Q])
{
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t src = nb.at(-L3X[i], -L3Y[i], -L3Z[i]);
#pragma unroll
        for (int k = 0; k < 3; ++k) f[k][i] = double(B[(int64_t)(k * Q + i) * g.N + src]);
    }
}

// e_i . (a0, a1, a2) over the nonzero components of link i (each +-1), added in x, y, z
// order.  A zero component would only add an exact zero, so this is the value of the full
// sum (up to the sign of a zero result) without the products by zero, which floating point
// cannot drop by itself.
template <typename C>
__device__ __forceinline__ C edot(int i, C a0, C a1, C a2)
{
    const int e[3] = {L3X[i], L3Y[i], L3Z[i]};
    const C a[3] = {a0, a1, a2};
    C r = C(0);
    bool any = false;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (e[c] != 0) {
            const C v = e[c] > 0 ? a[c] : -a[c];
            r = any ? r + v : v;
            any = true;
        }
    return r;
}

// Eq. (12) over the (Q - 1)/2 pairs of opposite links: 3 sum_i w_i e_i [phi(x + e_i) -
// phi(x - e_i)], phi(dx, dy, dz) the field at offset (dx, dy, dz) from the node (zero
// components of e_i skipped, as in edot)
template <typename C, int Q, typename Get>
__device__ __forceinline__ void grad3(Get phi, C (&d)[3])
{
    d[0] = d[1] = d[2] = C(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const C df = phi(L3X[i], L3Y[i], L3Z[i]) - phi(-L3X[i], -L3Y[i], -L3Z[i]);
        if (L3X[i] != 0) d[0] += w3<C, Q>(i) * C(L3X[i]) * df;
        if (L3Y[i] != 0) d[1] += w3<C, Q>(i) * C(L3Y[i]) * df;
        if (L3Z[i] != 0) d[2] += w3<C, Q>(i) * C(L3Z[i]) * df;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] *= C(3);
}

// Stress T = sum_pairs sigma C (|G|^2 I - G G^T)/|G| (xx, xy, xz, yy, yz, zz) and the pair
// normals n_kl (n[3p + a]; zero at or below the guard) of a node from its concentrations
// cc, their gradients gc and its densities rk (Eq. 7 with C_kl of Eq. 6).
template <typename C>
__device__ __forceinline__ void stress3(const C (&gc)[3][3], const C (&cc)[3], const C (&rk)[3], const KParams& kp,
                                         C (&t)[6], C (&nrm)[9])
{
#pragma unroll
    for (int q = 0; q < 6; ++q) t[q] = C(0);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int k = PK3[p], l = PL3[p];
        C G[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) G[a] = cc[l] * gc[k][a] - cc[k] * gc[l][a];
        const C g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        C n[3] = {C(0), C(0), C(0)};
        if (g2 > C(kp.guard * kp.guard)) {
            const C m = sqrt(g2), im = C(1) / m;
#pragma unroll
            for (int a = 0; a < 3; ++a) n[a] = G[a] * im;
            C cf = C(kp.cfac[p]) * (rk[k] * rk[l]);
            cf = cf < C(1) ? cf : C(1);
            const C s = C(kp.sigma[p]) * cf * m;  // sigma C |G| (I - n n)
            t[0] += s * (C(1) - n[0] * n[0]);
            t[1] -= s * (n[0] * n[1]);
            t[2] -= s * (n[0] * n[2]);
            t[3] += s * (C(1) - n[1] * n[1]);
            t[4] -= s * (n[1] * n[2]);
            t[5] += s * (C(1) - n[2] * n[2]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) nrm[3 * p + a] = n[a];
    }
}

// F_b = sum_a d_a T_ab with the symmetric T stored as (xx, xy, xz, yy, yz, zz);
// T(q, dx, dy, dz) is component q at offset (dx, dy, dz) from the node
template <typename C, int Q, typename Get>
__device__ __forceinline__ void force3(Get T, C (&F)[3])
{
    constexpr int QI[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    F[0] = F[1] = F[2] = C(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            C d[3];
            grad3<C, Q>([&](int dx, int dy, int dz) { return T(QI[a][b], dx, dy, dz); }, d);
            F[b] += d[a];
        }
}

// Collision with Guo's term (Eqs. 1-3, 8-11) and recolouring (Eq. 13 with the segregation
// law) of one node from its densities rk, totals ft, force F and pair normals nrm.  With OBS
// the node's observables go to acc (rho_k, rho u, kinetic energy, |u|); otherwise every
// recoloured population is handed to put(k, i, value).
template <typename C, int Q, bool OBS, typename Put>
__device__ __forceinline__ void collide3(const C (&rk)[3], const C (&ft)[Q], const C (&F)[3], const C (&nrm)[9],
                                         const KParams& kp, double (&acc)[8], Put put)
{
    const C rho = rk[0] + rk[1] + rk[2], irho = C(1) / rho;
    C m[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (L3X[i] != 0) m[0] += L3X[i] > 0 ? ft[i] : -ft[i];
        if (L3Y[i] != 0) m[1] += L3Y[i] > 0 ? ft[i] : -ft[i];
        if (L3Z[i] != 0) m[2] += L3Z[i] > 0 ? ft[i] : -ft[i];
    }
    C u[3], uu = C(0), uF = C(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = (m[a] + C(0.5) * F[a]) * irho;
        uu += u[a] * u[a];
        uF += u[a] * F[a];
    }
    if constexpr (OBS) {
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += double(rk[k]);
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[3 + a] += double(rho * u[a]);
        acc[6] += 0.5 * double(rho) * double(uu);
        const double um = sqrt(double(uu));
        acc[7] = (um > acc[7] || um != um) ? um : acc[7];
    } else {
        // tau = 3 nu + 1/2 with rho / nu = sum_k rho_k / nu_k (Eqs. 10-11)
        const C rho_over_nu = rk[0] * C(kp.inv_nu[0]) + rk[1] * C(kp.inv_nu[1]) + rk[2] * C(kp.inv_nu[2]);
        const C itau = rho_over_nu / (C(3) * rho + C(0.5) * rho_over_nu);
        const C pref = C(1) - C(0.5) * itau;
        // C_t and beta_kl of the segregation law; a_p = beta_p rho_k rho_l / rho
        C ct = C(kp.ct_coef) * rk[0] * rk[1] * rk[2] * (irho * irho * irho);
        ct = ct < C(1) ? ct : C(1);
        C ap[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) ap[p] = C(kp.beta0) * (C(1) + ct * C(kp.g[p])) * (rk[PK3[p]] * rk[PL3[p]]) * irho;
        // V_k = sum_{l != k} a_kl n_kl (n_lk = -n_kl)
        C V[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const C n0 = nrm[0 + a], n1 = nrm[3 + a], n2 = nrm[6 + a];
            V[0][a] = ap[0] * n0 + ap[1] * n1;
            V[1][a] = ap[2] * n2 - ap[0] * n0;
            V[2][a] = -(ap[1] * n1 + ap[2] * n2);
        }
        C ck[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) ck[k] = rk[k] * irho;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const C eu = edot<C>(i, u[0], u[1], u[2]);
            const C eF = edot<C>(i, F[0], F[1], F[2]);
            const C feq = w3<C, Q>(i) * rho * (C(1) + C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu);
            const C phi = w3<C, Q>(i) * pref * (C(3) * (eF - uF) + C(9) * eu * eF);
            const C fd = ft[i] - (ft[i] - feq) * itau + phi;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const C ve = edot<C>(i, V[k][0], V[k][1], V[k][2]);
                put(k, i, ck[k] * fd + w3<C, Q>(i) * ve);
            }
            // each link's values leave before the next link's are formed (otherwise the
            // compiler holds all 3Q for one burst of stores)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ---- the fused step: one kernel per step, marching along z
// A workgroup of TX x TY lanes (lane t at tile column t % TX, tile row t / TX; each wave is
// two whole tile rows) owns the output nodes [x0, x0 + cols) x [y0, y0 + rows) x
// [z0, z0 + depth), cols <= TX - 4 and rows <= TY - 4.  Lane (tx, ty) sits on node column
// (x0 - 2 + tx, y0 - 2 + ty) (wrapped) and marches up z.  Iteration j, three phases closed
// by barriers:
//   stage 1, plane z0 - 2 + j: pull the 3Q populations; totals f_i and densities rho_k (kept
//            in registers for two more iterations); c_k into the LDS ring (all lanes with
//            tx <= cols + 3, ty <= rows + 3);
//   stage 2, plane z0 - 3 + j: grad c_k (Eq. 12) from the ring, stress and pair normals
//            (lanes 1 .. cols + 2, 1 .. rows + 2); T into its LDS ring;
//   stage 3, plane z0 - 4 + j: F = div T from the ring, collision and recolouring of the
//            owned nodes (lanes 2 .. cols + 1, 2 .. rows + 1), stored.
// Rings hold three planes, by plane mod 3.  depth + 4 iterations output the tile's planes.
// The arithmetic of every node is that of stress3 / force3 / collide3 in a fixed order, so
// the result does not depend on the tile shape.  With FP64 arithmetic (CB = 8 bytes) D3Q19
// takes tiles of 32 x 16 lanes and D3Q27 32 x 14, so that its larger park still leaves the
// rings within the 160 KB of LDS (145 KB against 148 KB).  FP32 arithmetic halves every
// ring and fits three waves per SIMD in registers (146 and 157 VGPRs), so it takes 32 x 24
// lanes (118 and 136 KB): 560 owned columns of 768 lanes instead of 336 of 512, measured
// 7% (D3Q19) and 28% (D3Q27) faster at 128^3.
template <int Q, int CB = 8>
struct Tile3Shape {
    static constexpr int TX = 32, TY = CB == 4 ? 24 : (Q == 27 ? 14 : 16), T = TX * TY;
    static constexpr int TS = (TX - 2) * (TY - 2);  // lanes that form the stress
    static constexpr int TP = (TX - 4) * (TY - 4);  // lanes that own output nodes
};

struct Tile3 {
    int32_t x0, y0, z0, cols, rows, depth;
};

template <typename C, int Q>
struct alignas(16) March3Lds {
    using Sh = Tile3Shape<Q, sizeof(C)>;
    C c[3][3][Sh::T];    // c_k by plane mod 3
    C T[3][6][Sh::TS];   // stress by plane mod 3, on the stress lanes
    C park[Q][Sh::TP];   // per owning lane: the totals f_i of one waiting plane
};

// S: storage type, C: compute type.  With FP32 storage of FP64 arithmetic each stored value
// is rounded stochastically with the random bits of its node (key: node index and the
// step's salt), in store order.
template <typename S, typename C, bool OBS, int Q>
__global__ __launch_bounds__((Tile3Shape<Q, sizeof(C)>::T)) __attribute__((amdgpu_waves_per_eu(sizeof(C) == 4 ? 3 : 2))) void k3_march(
    const S* __restrict__ B, Geo3 g, KParams kp, const Tile3* __restrict__ tiles, S* __restrict__ Bout,
    double* __restrict__ partials, uint32_t salt)
{
    using Sh = Tile3Shape<Q, sizeof(C)>;
    constexpr int kTX = Sh::TX, kT3 = Sh::T;
    static_assert(kT3 % 64 == 0 && (2 * kTX) % 64 == 0, "each wave is whole tile rows");
    static_assert(sizeof(double) * 8 * (kT3 / 64) <= sizeof(C) * 3 * 3 * kT3, "c ring too small for the reduction");
    __shared__ March3Lds<C, Q> L;
    const Tile3 tl = tiles[blockIdx.x];
    const int t = threadIdx.x, tx = t % kTX, ty = t / kTX;
    const bool in1 = tx <= tl.cols + 3 && ty <= tl.rows + 3;
    const bool in2 = tx >= 1 && tx <= tl.cols + 2 && ty >= 1 && ty <= tl.rows + 2;
    const bool in3 = tx >= 2 && tx <= tl.cols + 1 && ty >= 2 && ty <= tl.rows + 1;
    auto wrap = [](int a, int n) {
        const int r = a % n;
        return r < 0 ? r + n : r;
    };
    const int x = wrap(tl.x0 - 2 + tx, g.nx), y = wrap(tl.y0 - 2 + ty, g.ny);
    // node offsets within a plane at x - 1, x, x + 1 and y - 1, y, y + 1 (N <= 2^29: the
    // byte offset of any node fits 32 bits)
    const uint32_t xo[3] = {(uint32_t)(x == 0 ? g.nx - 1 : x - 1), (uint32_t)x, (uint32_t)(x == g.nx - 1 ? 0 : x + 1)};
    const uint32_t yo[3] = {(uint32_t)((y == 0 ? g.ny - 1 : y - 1) * g.nx), (uint32_t)(y * g.nx),
                            (uint32_t)((y == g.ny - 1 ? 0 : y + 1) * g.nx)};
    const uint32_t pl = (uint32_t)(g.nx * g.ny);
    // the stress lanes' and owning lanes' slots in the T ring and the park
    const int tS = (ty - 1) * (kTX - 2) + (tx - 1), tP = (ty - 2) * (kTX - 4) + (tx - 2);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // The totals f_i of a plane are used two iterations after its pull, so three planes of
    // them are live at a time: the one pulled (ft), the one waiting (W) and the one collided
    // (ftB).  Each owning lane parks one of them in LDS (its own slots, so no barrier is
    // involved): after the pull, ftB comes out of the park, W goes in, and ft becomes W.
    C W[Q], rA[3], rB[3], nB[9];
#pragma unroll
    for (int i = 0; i < Q; ++i) W[i] = C(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) rA[k] = rB[k] = C(1);
#pragma unroll
    for (int q = 0; q < 9; ++q) nB[q] = C(0);
    const int J = tl.depth + 4;
    // plane offset of plane z (wrapped) and the source of link i for planes zo[]
    auto zoff = [&](int z) { return (uint32_t)wrap(z, g.nz) * pl; };
    auto src = [&](const uint32_t (&zo)[3], int i) {
        return (zo[1 - L3Z[i]] + yo[1 - L3Y[i]] + xo[1 - L3X[i]]) * (uint32_t)sizeof(S);
    };
#pragma unroll 1
    for (int j = 0; j < J; ++j) {
        const int zc = wrap(tl.z0 - 2 + j, g.nz);
        const int s0 = j % 3, s1 = (j + 2) % 3, s2 = (j + 1) % 3;  // planes zc, zc - 1, zc - 2
        // ---- stage 1: pull of plane zc
        C ft[Q], rk[3] = {C(1), C(1), C(1)};
#pragma unroll
        for (int i = 0; i < Q; ++i) ft[i] = C(0);
        if (in1) {
            const uint32_t zo[3] = {zoff(zc - 1), zoff(zc), zoff(zc + 1)};
            rk[0] = rk[1] = rk[2] = C(0);
            if constexpr (Q == 19 || sizeof(S) == 4) {
                // one memory round trip per plane: the 3Q loads are issued together, and a
                // scheduling barrier keeps the compiler from interleaving the sums with them
                // (which serialises the loads).  The values stay in the storage type until
                // summed (half the registers with FP32 storage: D3Q27 FP32 storage then fits
                // one batch, 18% faster than one per fluid).
                S v[3 * Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const uint32_t o = src(zo, i);
#pragma unroll
                    for (int k = 0; k < 3; ++k) v[k * Q + i] = ld_plane(B + (int64_t)(k * Q + i) * g.N, o);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const C a = C(v[i]), b = C(v[Q + i]), c = C(v[2 * Q + i]);
                    ft[i] = a + b + c;
                    rk[0] += a;
                    rk[1] += b;
                    rk[2] += c;
                }
            } else {
                // D3Q27 in FP64: one round trip per fluid (all 81 values of a plane would not
                // fit beside the live registers); the totals add the fluids in the same order
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    C v[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) v[i] = C(ld_plane(B + (int64_t)(k * Q + i) * g.N, src(zo, i)));
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        ft[i] = k == 0 ? v[i] : ft[i] + v[i];
                        rk[k] += v[i];
                    }
                }
            }
            const C ir = C(1) / (rk[0] + rk[1] + rk[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k) L.c[s0][k][t] = rk[k] * ir;
        }
        C ftB[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) ftB[i] = C(0);
        if (in3) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                ftB[i] = L.park[i][tP];
                L.park[i][tP] = W[i];
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) W[i] = ft[i];
        __syncthreads();
        // ---- stage 2: stress of plane zc - 1
        C nA[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) nA[q] = C(0);
        if (j >= 2 && in2) {
            const int sl[3] = {s2, s1, s0};  // by dz + 1
            C gc[3][3], cc[3], tt[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                grad3<C, Q>([&](int dx, int dy, int dz) { return L.c[sl[dz + 1]][k][t + dy * kTX + dx]; }, gc[k]);
                cc[k] = L.c[s1][k][t];
            }
            stress3<C>(gc, cc, rA, kp, tt, nA);
#pragma unroll
            for (int q = 0; q < 6; ++q) L.T[s1][q][tS] = tt[q];
        }
        __syncthreads();
        // ---- stage 3: collision and recolouring of plane zc - 2
        if (j >= 4 && in3) {
            const int sl[3] = {s0, s2, s1};  // T of planes zc - 3, zc - 2, zc - 1 by dz + 1
            C F[3];
            force3<C, Q>([&](int q, int dx, int dy, int dz) { return L.T[sl[dz + 1]][q][tS + dy * (kTX - 2) + dx]; },
                         F);
            const uint32_t node = (uint32_t)(tl.z0 - 4 + j) * pl + yo[1] + (uint32_t)x;
            const uint32_t o = node * (uint32_t)sizeof(S);
            NodeBits bits(node * (3u * Q) ^ salt);
            collide3<C, Q, OBS>(rB, ftB, F, nB, kp, acc, [&](int k, int i, C v) {
                st_plane(Bout + (int64_t)(k * Q + i) * g.N, o, to_storage<S, C>(v, bits));
            });
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            rB[k] = rA[k];
            rA[k] = rk[k];
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) nB[q] = nA[q];
    }
    if constexpr (OBS) {
        // wavefront reductions, then the eight waves' results in order (the c ring is free
        // once every lane has passed the last barrier of the march)
        __syncthreads();
        for (int q = 0; q < 7; ++q) acc[q] = wave_sum(acc[q]);
        acc[7] = wave_max(acc[7]);
        double* red = reinterpret_cast<double*>(&L.c[0][0][0]);
        constexpr int W = kT3 / 64;
        if ((t & 63) == 0)
            for (int q = 0; q < 8; ++q) red[q * W + (t >> 6)] = acc[q];
        __syncthreads();
        if (t < 8) {
            double v = red[t * W];
            for (int w = 1; w < W; ++w) {
                const double o = red[t * W + w];
                v = t < 7 ? v + o : ((o > v || o != o) ? o : v);
            }
            partials[(int64_t)blockIdx.x * 8 + t] = v;
        }
    }
}

// Node-parallel kernels (initialisation, export): blocks of 256 consecutive nodes (x
// fastest, then y, then z) on a one-dimensional grid.  Workgroups go to the eight XCDs in
// turn; block b takes the node range of logical block xcd_block(b), so that each XCD works
// through one contiguous run of blocks.  The map is a bijection of [0, T) for any T.
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
    // N <= 2^29 (checked at creation): 32-bit division suffices
    const uint32_t n32 = (uint32_t)n, nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
    const uint32_t p = n32 / nx, zz = p / ny;
    x = (int)(n32 - p * nx), y = (int)(p - zz * ny), z = (int)zz;
    return true;
}

// B_{i,k}(y) = w_i rho_k(y + e_i): the pulled state is f_{i,k} = w_i rho_k (fluid at rest)
template <typename S, typename C, int Q>
__global__ __launch_bounds__(256) void k3_init(const double* __restrict__ rho, Geo3 g, S* __restrict__ B)
{
    int x, y, z;
    if (!node3(g, x, y, z)) return;
    const Nb3 nb(g, x, y, z);
    const int64_t j = nb.at(0, 0, 0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t src = nb.at(L3X[i], L3Y[i], L3Z[i]);
#pragma unroll
        for (int k = 0; k < 3; ++k) B[(int64_t)(k * Q + i) * g.N + j] = S(w3<C, Q>(i) * C(rho[k * g.N + src]));
    }
}

// the post-streaming populations [3][Q][N] and densities [3][N] of the state
template <typename S, int Q>
__global__ __launch_bounds__(256) void k3_export(const S* __restrict__ B, Geo3 g, double* __restrict__ fout,
                                                 double* __restrict__ rho)
{
    int x, y, z;
    if (!node3(g, x, y, z)) return;
    const Nb3 nb(g, x, y, z);
    const int64_t j = nb.at(0, 0, 0);
    double f[3][Q];
    pull3<S, Q>(B, g, nb, f);
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) {
            s += f[k][i];
            if (fout) fout[(int64_t)(k * Q + i) * g.N + j] = f[k][i];
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
    Prec prec = Prec::F64;
    int q = 19;                         // links: 19 or 27
    void* buf[2] = {nullptr, nullptr};  // the state, in the storage type of prec
    Tile3* dtiles = nullptr;     // the march's tile list
    int ntiles = 0;
    double* partials = nullptr;  // [ntiles][8]
    double* staging = nullptr;   // [3q][N] for exports and uploads
    double* rho = nullptr;       // [3][N] densities for exports
    int cur = 0;
    int64_t step = 0;
    bool ready = false;
};

static dim3 grid3(const Geo3& g) { return dim3((unsigned)((g.N + 255) / 256)); }

static void release3(lbm3d* h)
{
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_state_pair(h->buf);
    for (void* q : {(void*)h->partials, (void*)h->staging, (void*)h->rho})
        if (q) (void)hipFree(q);
    if (h->dtiles) (void)hipFree(h->dtiles);
}

// n split into `parts` parts as equal as possible: part q is [start, start + len)
static void split_even(int n, int parts, int q, int& start, int& len)
{
    const int base = n / parts, extra = n % parts;
    start = q * base + (q < extra ? q : extra);
    len = base + (q < extra ? 1 : 0);
}

// The march's tiles: the x-y plane cut into at most (TX - 4) x (TY - 4) node blocks (the
// lattice's tile shape), the z axis into `nseg` segments chosen so that rounds of resident
// workgroups x (segment depth + 4 warm-up planes) is least.  Workgroups go to the XCDs in
// turn, so the list is permuted for each XCD to take a contiguous run of it (neighbouring
// blocks, whose halos it then finds in its own L2).
static std::vector<Tile3> plan3(const Geo3& g, int slots, int q, Prec prec)
{
    const bool f32 = prec == Prec::F32;
    const int TX = 32;
    const int TY = f32 ? Tile3Shape<19, 4>::TY : (q == 27 ? Tile3Shape<27>::TY : Tile3Shape<19>::TY);
    const int ntx = (g.nx + TX - 5) / (TX - 4), nty = (g.ny + TY - 5) / (TY - 4);
    const int64_t per_seg = (int64_t)ntx * nty;
    if (slots < 1) slots = 1;
    int nseg = 1;
    double best = 1e300;
    for (int s = 1; s <= g.nz; ++s) {
        const int depth = (g.nz + s - 1) / s;
        const int64_t rounds = (per_seg * s + slots - 1) / slots;
        const double cost = (double)rounds * (depth + 4) * (1.0 + 1e-9 * s);
        if (cost < best) {
            best = cost;
            nseg = s;
        }
        if (depth <= 4) break;
    }
    std::vector<Tile3> L;
    L.reserve((size_t)per_seg * nseg);
    for (int zs = 0; zs < nseg; ++zs)
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx) {
                Tile3 t{};
                split_even(g.nx, ntx, tx, t.x0, t.cols);
                split_even(g.ny, nty, ty, t.y0, t.rows);
                split_even(g.nz, nseg, zs, t.z0, t.depth);
                L.push_back(t);
            }
    const int T = (int)L.size(), nxcd = 8;
    std::vector<Tile3> out(T);
    std::vector<int> start(nxcd + 1, 0);
    for (int x = 0; x < nxcd; ++x) start[x + 1] = start[x] + (T - x + nxcd - 1) / nxcd;
    for (int b = 0; b < T; ++b) out[b] = L[start[b % nxcd] + b / nxcd];
    return out;
}

template <typename S, typename C, int Q>
static hipError_t launch_march_t(lbm3d* h, bool obs)
{
    const S* in = (const S*)h->buf[h->cur];
    const uint32_t salt = step_salt(h->step);
    constexpr int T = Tile3Shape<Q, sizeof(C)>::T;
    if (obs)
        hipLaunchKernelGGL((k3_march<S, C, true, Q>), dim3(h->ntiles), dim3(T), 0, h->stream, in, h->g, h->kp,
                           (const Tile3*)h->dtiles, (S*)nullptr, h->partials, 0u);
    else
        hipLaunchKernelGGL((k3_march<S, C, false, Q>), dim3(h->ntiles), dim3(T), 0, h->stream, in, h->g, h->kp,
                           (const Tile3*)h->dtiles, (S*)h->buf[h->cur ^ 1], (double*)nullptr, salt);
    return hipGetLastError();
}

template <int Q>
static hipError_t launch_march_q(lbm3d* h, bool obs)
{
    switch (h->prec) {
        case Prec::F64: return launch_march_t<double, double, Q>(h, obs);
        case Prec::F32S: return launch_march_t<float, double, Q>(h, obs);
        case Prec::F32: return launch_march_t<float, float, Q>(h, obs);
    }
    return hipErrorInvalidValue;
}

static hipError_t launch_march(lbm3d* h, bool obs)
{
    return h->q == 27 ? launch_march_q<27>(h, obs) : launch_march_q<19>(h, obs);
}

template <int Q>
static hipError_t march_occupancy_q(Prec prec, int* per_cu)
{
    constexpr int T = Tile3Shape<Q>::T, T4 = Tile3Shape<Q, 4>::T;
    switch (prec) {
        case Prec::F64:
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k3_march<double, double, false, Q>, T, 0);
        case Prec::F32S:
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k3_march<float, double, false, Q>, T, 0);
        case Prec::F32:
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k3_march<float, float, false, Q>, T4, 0);
    }
    return hipErrorInvalidValue;
}

static hipError_t march_occupancy(Prec prec, int q, int* per_cu)
{
    return q == 27 ? march_occupancy_q<27>(prec, per_cu) : march_occupancy_q<19>(prec, per_cu);
}

template <int Q>
static hipError_t launch_init3_q(lbm3d* h, const double* rho)
{
    const dim3 gr = grid3(h->g), bl(256);
    switch (h->prec) {
        case Prec::F64:
            hipLaunchKernelGGL((k3_init<double, double, Q>), gr, bl, 0, h->stream, rho, h->g, (double*)h->buf[0]);
            break;
        case Prec::F32S:
            hipLaunchKernelGGL((k3_init<float, double, Q>), gr, bl, 0, h->stream, rho, h->g, (float*)h->buf[0]);
            break;
        case Prec::F32:
            hipLaunchKernelGGL((k3_init<float, float, Q>), gr, bl, 0, h->stream, rho, h->g, (float*)h->buf[0]);
            break;
    }
    return hipGetLastError();
}

static hipError_t launch_init3(lbm3d* h, const double* rho)
{
    return h->q == 27 ? launch_init3_q<27>(h, rho) : launch_init3_q<19>(h, rho);
}

template <int Q>
static hipError_t launch_export3_q(lbm3d* h, double* fout, double* rho)
{
    const dim3 gr = grid3(h->g), bl(256);
    if (h->prec == Prec::F64)
        hipLaunchKernelGGL((k3_export<double, Q>), gr, bl, 0, h->stream, (const double*)h->buf[h->cur], h->g, fout,
                           rho);
    else
        hipLaunchKernelGGL((k3_export<float, Q>), gr, bl, 0, h->stream, (const float*)h->buf[h->cur], h->g, fout,
                           rho);
    return hipGetLastError();
}

static hipError_t launch_export3(lbm3d* h, double* fout, double* rho)
{
    return h->q == 27 ? launch_export3_q<27>(h, fout, rho) : launch_export3_q<19>(h, fout, rho);
}

extern "C" {

int lbm3d_create_lattice(const lbm3_params* p, int32_t nz, int32_t q, void* hip_stream, lbm3d_t** out)
{
    if (out) *out = nullptr;
    if (!out) {
        set_error("out is NULL");
        return LBM3_EINVAL;
    }
    int rc = validate_params(p);
    if (rc) return rc;
    if (q != 19 && q != 27) {
        set_error("the three-dimensional form takes the D3Q19 or the D3Q27 lattice (q = 19 or 27, got %d)", (int)q);
        return LBM3_EINVAL;
    }
    if (nz < 1 || nz > 65535) {
        set_error("nz must be in 1..65535 (got %d)", nz);
        return LBM3_EINVAL;
    }
    if ((int64_t)p->nx * p->ny * nz > ((int64_t)1 << 29)) {
        set_error("the three-dimensional form takes at most 2^29 nodes (got %d x %d x %d)", (int)p->nx, (int)p->ny,
                  nz);
        return LBM3_EINVAL;
    }
    if (p->forcing != LBM3_FORCING_GUO) {
        set_error("the three-dimensional form runs the force of Eq. (7) with Guo's term only");
        return LBM3_EUNSUPPORTED;
    }
    lbm3d* h = new (std::nothrow) lbm3d();
    if (!h) {
        set_error("host allocation failed");
        return LBM3_ENOMEM;
    }
    h->p = *p;
    h->prec = prec_of(p->precision);
    h->q = q;
    derive(p, &h->kp, nullptr, nullptr, nullptr);
    h->g = Geo3{p->nx, p->ny, nz, (int64_t)p->nx * p->ny * nz};
    h->stream = (hipStream_t)hip_stream;
    const int64_t N = h->g.N;
    hipError_t e = hipSuccess;
    int dev = 0, cus = 0, per_cu = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = march_occupancy(h->prec, q, &per_cu);
    std::vector<Tile3> tiles;
    if (e == hipSuccess) {
        tiles = plan3(h->g, per_cu * cus, q, h->prec);
        h->ntiles = (int)tiles.size();
    }
    const size_t eb = h->prec == Prec::F64 ? sizeof(double) : sizeof(float);
    if (e == hipSuccess) e = alloc_state_pair((size_t)3 * q * N * eb, h->buf);
    if (e == hipSuccess) e = hipMalloc(&h->dtiles, tiles.size() * sizeof(Tile3));
    if (e == hipSuccess)
        e = hipMemcpy(h->dtiles, tiles.data(), tiles.size() * sizeof(Tile3), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&h->partials, tiles.size() * 8 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&h->staging, (size_t)3 * q * N * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&h->rho, (size_t)3 * N * sizeof(double));
    if (e != hipSuccess) {
        rc = hip_fail(e, "hipMalloc (three-dimensional lattice)");
        release3(h);
        delete h;
        return rc;
    }
    *out = h;
    return LBM3_OK;
}

int lbm3d_create(const lbm3_params* p, int32_t nz, void* hip_stream, lbm3d_t** out)
{
    return lbm3d_create_lattice(p, nz, 19, hip_stream, out);
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
        e = launch_init3(h, (const double*)h->staging);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "three-dimensional init");
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
        hipError_t e = launch_march(h, false);
        if (e != hipSuccess) return hip_fail(e, "three-dimensional step launch");
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
    const size_t nblocks = (size_t)h->ntiles;
    const int64_t N = h->g.N;
    hipError_t e = launch_march(h, true);
    std::vector<double> part(nblocks * 8);
    if (e == hipSuccess)
        e = hipMemcpyAsync(part.data(), h->partials, part.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && (rho_out || f_out)) {
        e = launch_export3(h, f_out ? h->staging : nullptr, h->rho);
        if (e == hipSuccess && rho_out)
            e = hipMemcpyAsync(rho_out, h->rho, (size_t)3 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && f_out)
            e = hipMemcpyAsync(f_out, h->staging, (size_t)3 * h->q * N * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "three-dimensional observables");
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
        set_error("the three-dimensional state is not finite at step %lld", (long long)h->step);
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
