// Reverse-mode derivative (adjoint) of the FP64 step, with checkpointed recomputation.
//
// The forward run keeps a checkpoint every K steps.  The reverse sweep takes the segments
// last to first: it recomputes the segment's K forward steps from its checkpoint with the
// fused step in its tape mode, which records the densities, totals, concentration
// gradients and force it pulled and formed at every node (20 values per node and step),
// then takes the K reverse steps, each two kernels reading that tape: a node-parallel one
// and a row-marching one.
//
// Notation: the population buffer B holds, at node y, the recoloured populations of y
// before streaming; the post-streaming populations are f_{i,k}(x) = B_{i,k}(x - e_i).
// One step maps B to B'.  Given lam' = dL/dB' the reverse step returns lam = dL/dB and
// adds to dL/dsigma.  Per node the forward step is (Sec. 2):
//   rho_k = sum_i f_{i,k}, f_i = sum_k f_{i,k}, c_k = rho_k/rho, grad c_k = D c_k (Eq. 12)
//   G_p = c_l grad c_k - c_k grad c_l, m_p = |G_p|, n_p = G_p/m_p, C_p = min(cf_p rho_k rho_l, 1)
//   T = sum_p sigma_p C_p (m_p^2 I - G_p G_p^T)/m_p,  F = div T  (Eqs. 6, 7)
//   tau = 3 rho / sum_k(rho_k/nu_k) + 1/2, u = (sum_i f_i e_i + F/2)/rho   (Eqs. 9-11)
//   fd_i = f_i - (f_i - feq_i)/tau + Phi_i                                 (Eqs. 1-3, 8)
//   ct = min(35 rho_0 rho_1 rho_2/rho^3, 1), beta_p = beta0 (1 + ct g_p), a_p = beta_p rho_k rho_l/rho
//   B'_{i,k} = c_k fd_i + w_i V_k . e_i,  V_k = sum_{l != k} a_kl n_kl, n_lk = -n_kl   (Eqs. 13, 19)
// and the reverse pass applies the transposed chain rule to each line, right to left.
// The difference operator of Eq. (12) is antisymmetric on a periodic lattice (D^T = -D),
// so the transposes of the gradient and of the force divergence are -divergence and
// -gradient with the same stencil.  Non-smooth points take one-sided derivatives:
// d min(a, 1)/da = 1 for a < 1 and 0 otherwise; pairs with |G| at or below the guard
// (n = 0, no stress) pass no derivative; g(X) has zero derivative where |X| is snapped to 1.
#include <algorithm>
#include <cmath>
#include <vector>

#include "lbm3_handle.h"

namespace tcg {
namespace {

constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int PK[3] = {0, 0, 1}, PL[3] = {1, 2, 2};

__device__ __forceinline__ double wgt(int i)
{
    return i == 0 ? 1.0 - 4.0 * (1.0 / 9.0) - 4.0 * (1.0 / 36.0) : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

__device__ __forceinline__ int wrapi(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Workspace fields, each [components][N] in FP64 with node index y*nx + x.  rho, ftot and
// gc point into the tape of the step being reversed.
struct AdjWS {
    double* rho;    // 3   densities
    double* ftot;   // 9   total populations
    double* gc;     // 6   grad c_k (x, y per fluid)
    double* F;      // 2   force
    double* rbar;   // 3   dL/drho_k accumulated (all node-local contributions)
    double* Fbar;   // 2   dL/dF
    double* Gbar;   // 6   dL/dG_p from the recolouring normals
    double* sig;    // [max(A1 workgroups, A2+A3 tiles)][6] per-workgroup sums: beta part (3)
                    // from A1, stress part (3) from A2+A3
};

struct Geo {
    int nx, ny;
    int64_t plane, pitch;
    double sigma[3], g[3], beta0, inv_nu[3], cfac[3], guard;
};

// colour gradient, modulus, normal and concentration factor of pair p at a node
struct PairFwd {
    double Gx, Gy, m, im, nx, ny, C;  // im = 1/m where on, else 0
    bool on;  // m > guard, decided on m^2 as the step decides it
    bool unclipped;
};

__device__ __forceinline__ PairFwd pair_fwd(const Geo& g, int p, const double (&c)[3], const double (&gx)[3],
                                            const double (&gy)[3], const double (&rk)[3])
{
    const int k = PK[p], l = PL[p];
    PairFwd r;
    r.Gx = c[l] * gx[k] - c[k] * gx[l];
    r.Gy = c[l] * gy[k] - c[k] * gy[l];
    const double g2 = r.Gx * r.Gx + r.Gy * r.Gy;
    r.m = sqrt(g2);
    r.on = g2 > g.guard * g.guard;
    r.im = r.on ? 1.0 / r.m : 0.0;
    r.nx = r.Gx * r.im;
    r.ny = r.Gy * r.im;
    const double cf = g.cfac[p] * rk[k] * rk[l];
    r.unclipped = cf < 1.0;
    r.C = r.unclipped ? cf : 1.0;
    return r;
}

__device__ __forceinline__ void node_fields(const AdjWS& w, int64_t N, int64_t j, double (&rk)[3], double (&c)[3],
                                            double (&gx)[3], double (&gy)[3])
{
    for (int k = 0; k < 3; ++k) rk[k] = w.rho[k * N + j];
    const double ir = 1.0 / (rk[0] + rk[1] + rk[2]);
    for (int k = 0; k < 3; ++k) {
        c[k] = rk[k] * ir;
        gx[k] = w.gc[(2 * k) * N + j];
        gy[k] = w.gc[(2 * k + 1) * N + j];
    }
}

// ---- A1: node-local reverse of collision and recolouring
// The node-local reverse of collision and recolouring at node (x, y) (A1): dL/df_i of the
// new adjoint state (fb), the node-local part of dL/drho_k (rb), dL/dF, dL/dG of the three
// pairs and the dL/dsigma contributions of the segregation law.
struct LocalOut {
    double fb[9], rb[3], Fb[2], Gb[3][2], sigb[3];
};

__device__ __forceinline__ void adj_local_node(const double* __restrict__ lamp, const Geo& g, const AdjWS& w, int x,
                                               int y, LocalOut& o)
{
    const int64_t N = (int64_t)g.nx * g.ny, j = (int64_t)y * g.nx + x;
    double rk[3], c[3], gx[3], gy[3];
    node_fields(w, N, j, rk, c, gx, gy);
    const double rho = rk[0] + rk[1] + rk[2];
    const double irho = 1.0 / rho, irho3 = irho * irho * irho;
    double f[9];
    for (int i = 0; i < 9; ++i) f[i] = w.ftot[i * N + j];
    PairFwd pf[3];
    for (int p = 0; p < 3; ++p) pf[p] = pair_fwd(g, p, c, gx, gy, rk);
    // the force the forward step formed at this node (div T, Eq. 7 with Eq. 12)
    const double Fx = w.F[j], Fy = w.F[N + j];
    // ---- forward collision
    const double S = rk[0] * g.inv_nu[0] + rk[1] * g.inv_nu[1] + rk[2] * g.inv_nu[2];
    const double iS = 1.0 / S;
    const double tau = 3.0 * rho * iS + 0.5;
    const double itau = 1.0 / tau;
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < 9; ++i) {
        mx += f[i] * EX[i];
        my += f[i] * EY[i];
    }
    const double ux = (mx + 0.5 * Fx) * irho, uy = (my + 0.5 * Fy) * irho;
    const double uu = ux * ux + uy * uy, uF = ux * Fx + uy * Fy, pref = 1.0 - 0.5 * itau;
    double eu[9], eF[9], feq[9], phi[9], fd[9];
    for (int i = 0; i < 9; ++i) {
        eu[i] = EX[i] * ux + EY[i] * uy;
        eF[i] = EX[i] * Fx + EY[i] * Fy;
        feq[i] = wgt(i) * rho * (1.0 + 3.0 * eu[i] + 4.5 * eu[i] * eu[i] - 1.5 * uu);
        phi[i] = wgt(i) * pref * (3.0 * (eF[i] - uF) + 9.0 * eu[i] * eF[i]);
        fd[i] = f[i] - (f[i] - feq[i]) * itau + phi[i];
    }
    // ---- forward recolouring quantities
    const double q35 = 35.0 * rk[0] * rk[1] * rk[2] * irho3;
    const bool ct_free = q35 < 1.0;
    const double ct = ct_free ? q35 : 1.0;
    double beta[3], aa[3], prod[3];
    for (int p = 0; p < 3; ++p) {
        beta[p] = g.beta0 * (1.0 + ct * g.g[p]);
        prod[p] = rk[PK[p]] * rk[PL[p]];
        aa[p] = beta[p] * prod[p] * irho;
    }
    // ---- reverse of the recolouring
    // dL/dB'_{i,k}(x) = dL/df'_{i,k}(x + e_i) = fbar'_i(x + e_i) + rhobar'_k(x + e_i)
    double ob[27];
    for (int i = 0; i < 9; ++i) {
        const int64_t nb = (int64_t)wrapi(y + EY[i], g.ny) * g.nx + wrapi(x + EX[i], g.nx);
        const double fbi = lamp[i * N + nb];
        for (int k = 0; k < 3; ++k) ob[k * 9 + i] = fbi + lamp[(9 + k) * N + nb];
    }
    double fdb[9], cb[3] = {0, 0, 0}, Vb[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int i = 0; i < 9; ++i) fdb[i] = c[0] * ob[i] + c[1] * ob[9 + i] + c[2] * ob[18 + i];
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 9; ++i) {
            cb[k] += fd[i] * ob[k * 9 + i];
            Vb[k][0] += wgt(i) * EX[i] * ob[k * 9 + i];
            Vb[k][1] += wgt(i) * EY[i] * ob[k * 9 + i];
        }
    double rb[3] = {0, 0, 0}, rhob = 0.0, ctb = 0.0, Gbr[3][2];
    for (int p = 0; p < 3; ++p) {
        const int k = PK[p], l = PL[p];
        const double dVx = Vb[k][0] - Vb[l][0], dVy = Vb[k][1] - Vb[l][1];
        const double ab = dVx * pf[p].nx + dVy * pf[p].ny;
        // n_p = G/m: dL/dG = (nb - n (n . nb)) / m with nb = a_p (Vb_k - Vb_l)
        Gbr[p][0] = Gbr[p][1] = 0.0;
        if (pf[p].on) {
            const double nbx = aa[p] * dVx, nby = aa[p] * dVy;
            const double nn = pf[p].nx * nbx + pf[p].ny * nby;
            Gbr[p][0] = (nbx - pf[p].nx * nn) * pf[p].im;
            Gbr[p][1] = (nby - pf[p].ny * nn) * pf[p].im;
        }
        // a_p = beta_p rho_k rho_l / rho
        const double betab = ab * prod[p] * irho;
        rb[k] += ab * beta[p] * rk[l] * irho;
        rb[l] += ab * beta[p] * rk[k] * irho;
        rhob -= ab * aa[p] * irho;
        // beta_p = beta0 (1 + ct g_p)
        ctb += betab * g.beta0 * g.g[p];
        o.sigb[p] = betab * g.beta0 * ct;  // times g'(X_p) dX_p/dsigma on the host
    }
    if (ct_free) {
        rb[0] += ctb * 35.0 * rk[1] * rk[2] * irho3;
        rb[1] += ctb * 35.0 * rk[0] * rk[2] * irho3;
        rb[2] += ctb * 35.0 * rk[0] * rk[1] * irho3;
        rhob -= ctb * 3.0 * q35 * irho;
    }
    // ---- reverse of the collision
    double fb[9], ub[2] = {0, 0}, Fb[2] = {0, 0}, itaub = 0.0, prefb = 0.0, uub = 0.0, uFb = 0.0;
    for (int i = 0; i < 9; ++i) {
        const double feqb = fdb[i] * itau;
        fb[i] = fdb[i] * (1.0 - itau);
        itaub += fdb[i] * (feq[i] - f[i]);
        const double phib = fdb[i];
        prefb += phib * wgt(i) * (3.0 * (eF[i] - uF) + 9.0 * eu[i] * eF[i]);
        const double A = phib * wgt(i) * pref;
        const double eFb = A * (3.0 + 9.0 * eu[i]);
        double eub = 9.0 * A * eF[i];
        uFb -= 3.0 * A;
        rhob += feqb * wgt(i) * (1.0 + 3.0 * eu[i] + 4.5 * eu[i] * eu[i] - 1.5 * uu);
        const double Bf = feqb * wgt(i) * rho;
        eub += Bf * (3.0 + 9.0 * eu[i]);
        uub -= 1.5 * Bf;
        ub[0] += eub * EX[i];
        ub[1] += eub * EY[i];
        Fb[0] += eFb * EX[i];
        Fb[1] += eFb * EY[i];
    }
    ub[0] += uFb * Fx + 2.0 * uub * ux;
    ub[1] += uFb * Fy + 2.0 * uub * uy;
    Fb[0] += uFb * ux;
    Fb[1] += uFb * uy;
    itaub -= 0.5 * prefb;
    // u = (m + F/2)/rho
    const double mbx = ub[0] * irho, mby = ub[1] * irho;
    Fb[0] += 0.5 * mbx;
    Fb[1] += 0.5 * mby;
    rhob -= (ub[0] * ux + ub[1] * uy) * irho;
    for (int i = 0; i < 9; ++i) fb[i] += mbx * EX[i] + mby * EY[i];
    // itau = 1/tau, tau = 3 rho / S + 1/2, S = sum_k rho_k inv_nu_k
    const double taub = -itaub * itau * itau;
    rhob += taub * 3.0 * iS;
    const double Sb = -taub * 3.0 * rho * iS * iS;
    for (int k = 0; k < 3; ++k) rb[k] += Sb * g.inv_nu[k];
    // c_k = rho_k / rho (the node-local uses of c)
    double cr = 0.0;
    for (int k = 0; k < 3; ++k) cr += cb[k] * rk[k];
    for (int k = 0; k < 3; ++k) rb[k] += cb[k] * irho - cr * (irho * irho);
    for (int k = 0; k < 3; ++k) rb[k] += rhob;  // rho = sum_k rho_k
    for (int i = 0; i < 9; ++i) o.fb[i] = fb[i];
    for (int k = 0; k < 3; ++k) o.rb[k] = rb[k];
    o.Fb[0] = Fb[0];
    o.Fb[1] = Fb[1];
    for (int p = 0; p < 3; ++p) {
        o.Gb[p][0] = Gbr[p][0];
        o.Gb[p][1] = Gbr[p][1];
    }
}

__global__ __launch_bounds__(256) void k_adj_local(const double* __restrict__ lamp, Geo g, AdjWS w,
                                                   double* __restrict__ lamn)
{
    __shared__ double red[3][256];
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    const int t = threadIdx.x;
    double sig_beta[3] = {0.0, 0.0, 0.0};
    if (x < g.nx) {
        LocalOut o;
        adj_local_node(lamp, g, w, x, y, o);
        const int64_t N = (int64_t)g.nx * g.ny, j = (int64_t)y * g.nx + x;
        for (int i = 0; i < 9; ++i) lamn[i * N + j] = o.fb[i];
        for (int k = 0; k < 3; ++k) w.rbar[k * N + j] = o.rb[k];
        w.Fbar[j] = o.Fb[0];
        w.Fbar[N + j] = o.Fb[1];
        for (int p = 0; p < 3; ++p) {
            w.Gbar[(2 * p) * N + j] = o.Gb[p][0];
            w.Gbar[(2 * p + 1) * N + j] = o.Gb[p][1];
            sig_beta[p] = o.sigb[p];
        }
    }
    // wavefront sums, then the four wave sums in order
    for (int p = 0; p < 3; ++p) sig_beta[p] = wave_sum(sig_beta[p]);
    if ((t & 63) == 0)
        for (int p = 0; p < 3; ++p) red[p][t >> 6] = sig_beta[p];
    __syncthreads();
    if (t < 3) {
        const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        w.sig[b * 6 + t] += ((red[t][0] + red[t][1]) + red[t][2]) + red[t][3];
    }
}

// What the reverse of the stress reads at one node: dL/dF at the eight neighbours, the
// tape's densities and concentration gradients, dL/dG from A1 and, on the tile's own
// columns, the node-local part of dL/drho_k from A1.
struct SfIn {
    double Fb[2][8];  // E, W, N, S, NE, NW, SE, SW
    double rk[3], gc[6], Gb[6], rbar[3];
};

__device__ __forceinline__ void sf_load(const Geo& g, const AdjWS& w, int64_t N, int xm, int x, int xp, int y,
                                        bool own_col, SfIn& in)
{
    const int ym = wrapi(y - 1, g.ny), yp = wrapi(y + 1, g.ny);
    const int64_t r0 = (int64_t)y * g.nx, rn = (int64_t)yp * g.nx, rs = (int64_t)ym * g.nx;
    const int64_t at[8] = {r0 + xp, r0 + xm, rn + x, rs + x, rn + xp, rn + xm, rs + xp, rs + xm};
    for (int c = 0; c < 2; ++c)
        for (int q = 0; q < 8; ++q) in.Fb[c][q] = w.Fbar[c * N + at[q]];
    const int64_t jn = r0 + x;
    for (int k = 0; k < 3; ++k) in.rk[k] = w.rho[k * N + jn];
    for (int q = 0; q < 6; ++q) {
        in.gc[q] = w.gc[q * N + jn];
        in.Gb[q] = w.Gbar[q * N + jn];
    }
    for (int k = 0; k < 3; ++k) in.rbar[k] = own_col ? w.rbar[k * N + jn] : 0.0;
}

// paired-difference form of Eq. (12) from the eight neighbours of a node
__device__ __forceinline__ void grad8(const double (&v)[8], double& dx, double& dy)
{
    dx = 3.0 * ((1.0 / 9.0) * (v[0] - v[1]) + (1.0 / 36.0) * ((v[4] - v[7]) + (v[6] - v[5])));
    dy = 3.0 * ((1.0 / 9.0) * (v[2] - v[3]) + (1.0 / 36.0) * ((v[4] - v[7]) + (v[5] - v[6])));
}

// ---- A2 + A3 in one pass: the reverse of the stress and the pair quantities, whose
// result dL/d(grad c_k) then stays in LDS, and the reverse of the gradient (c-bar = -div
// of it) and of the densities.  With the totals' part written by A1 this completes the
// adjoint state of the previous step.
//
// A workgroup marches one tile: `cols` columns from x0 and `rows` rows from y0, lane t at
// column x0 - 1 + t (one halo column each side).  Iteration j first forms dL/d(grad c_k)
// on row y0 - 1 + j for every lane, halo lanes and the halo rows above and below the tile
// included, into slot j mod 4 of an LDS ring; after one barrier it completes row
// y0 + j - 2, whose rows above and below are then in the ring.  The row written next is
// never one still being read (four slots for a three-row stencil), so one barrier per row
// suffices.  The next row's inputs are loaded before the barrier, so that their latency
// overlaps the barrier and the completion.  Only the tile's own nodes add to dL/dsigma.
template <int NT>
__global__ __launch_bounds__(NT) void k_adj_sf(Geo g, AdjWS w, const Tile* __restrict__ tiles,
                                               double* __restrict__ lam)
{
    __shared__ double ring[4][6][NT];
    const Tile tl = tiles[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t N = (int64_t)g.nx * g.ny;
    const bool lane_on = t < tl.cols + 2;
    const bool own_col = t >= 1 && t <= tl.cols;
    const int x = wrapi(tl.x0 - 1 + t, g.nx);
    const int xm = wrapi(x - 1, g.nx), xp = wrapi(x + 1, g.nx);
    double sig_st[3] = {0.0, 0.0, 0.0};
    // the densities and the completed node-local part of dL/drho_k of the row that the
    // next iteration completes
    double rk_prev[3] = {0.0, 0.0, 0.0}, part_prev[3] = {0.0, 0.0, 0.0};
    SfIn in;
    if (lane_on) sf_load(g, w, N, xm, x, xp, wrapi(tl.y0 - 1, g.ny), own_col, in);
    for (int j = 0; j < tl.rows + 2; ++j) {
        double rk[3] = {0.0, 0.0, 0.0}, part[3] = {0.0, 0.0, 0.0};
        if (lane_on) {
            // T-bar = -(transpose-free form): Tb_xx = -Dx Fbx, Tb_xy = -(Dy Fbx + Dx Fby), Tb_yy = -Dy Fby
            double dFx_dx, dFx_dy, dFy_dx, dFy_dy;
            grad8(in.Fb[0], dFx_dx, dFx_dy);
            grad8(in.Fb[1], dFy_dx, dFy_dy);
            const double Tbxx = -dFx_dx, Tbxy = -(dFx_dy + dFy_dx), Tbyy = -dFy_dy;
            double c[3], gx[3], gy[3];
            for (int k = 0; k < 3; ++k) rk[k] = in.rk[k];
            const double rho = rk[0] + rk[1] + rk[2];
            const double ir = 1.0 / rho;
            for (int k = 0; k < 3; ++k) {
                c[k] = rk[k] * ir;
                gx[k] = in.gc[2 * k];
                gy[k] = in.gc[2 * k + 1];
            }
            double cb[3] = {0, 0, 0}, gcb[3][2] = {{0, 0}, {0, 0}, {0, 0}}, rb[3] = {0, 0, 0};
            const bool own = own_col && j >= 1 && j <= tl.rows;
            for (int p = 0; p < 3; ++p) {
                const int k = PK[p], l = PL[p];
                const PairFwd f = pair_fwd(g, p, c, gx, gy, rk);
                if (!f.on) continue;
                double Gbx = in.Gb[2 * p], Gby = in.Gb[2 * p + 1];
                const double Q = Tbxx * f.Gy * f.Gy - Tbxy * f.Gx * f.Gy + Tbyy * f.Gx * f.Gx;
                const double h = g.sigma[p] * f.C * f.im;
                Gbx += h * (2.0 * Tbyy * f.Gx - Tbxy * f.Gy);
                Gby += h * (2.0 * Tbxx * f.Gy - Tbxy * f.Gx);
                const double mb = -Q * g.sigma[p] * f.C * (f.im * f.im);
                Gbx += mb * f.Gx * f.im;
                Gby += mb * f.Gy * f.im;
                if (own) sig_st[p] += Q * f.C * f.im;
                if (f.unclipped) {
                    const double Cb = Q * g.sigma[p] * f.im;
                    rb[k] += Cb * g.cfac[p] * rk[l];
                    rb[l] += Cb * g.cfac[p] * rk[k];
                }
                // G = c_l grad c_k - c_k grad c_l
                cb[l] += Gbx * gx[k] + Gby * gy[k];
                cb[k] -= Gbx * gx[l] + Gby * gy[l];
                gcb[k][0] += c[l] * Gbx;
                gcb[k][1] += c[l] * Gby;
                gcb[l][0] -= c[k] * Gbx;
                gcb[l][1] -= c[k] * Gby;
            }
            for (int k = 0; k < 3; ++k) {
                ring[j & 3][2 * k][t] = gcb[k][0];
                ring[j & 3][2 * k + 1][t] = gcb[k][1];
            }
            if (own_col) {
                double cr = 0.0;
                for (int k = 0; k < 3; ++k) cr += cb[k] * rk[k];
                const double irho = 1.0 / rho;
                for (int k = 0; k < 3; ++k) part[k] = in.rbar[k] + (rb[k] + cb[k] * irho - cr * (irho * irho));
            }
            if (j + 1 < tl.rows + 2) sf_load(g, w, N, xm, x, xp, wrapi(tl.y0 + j, g.ny), own_col, in);
        }
        __syncthreads();
        if (own_col && j >= 2) {
            // row y0 + j - 2: its south, own and north rows sit in slots j - 2, j - 1, j
            const int yc = wrapi(tl.y0 + j - 2, g.ny);
            const double(*S)[NT] = ring[(j - 2) & 3];
            const double(*C)[NT] = ring[(j - 1) & 3];
            const double(*U)[NT] = ring[j & 3];
            double cb[3];
            for (int k = 0; k < 3; ++k) {
                const int qx = 2 * k, qy = 2 * k + 1;
                const double a = 3.0 * ((1.0 / 9.0) * (C[qx][t + 1] - C[qx][t - 1]) +
                                        (1.0 / 36.0) * ((U[qx][t + 1] - S[qx][t - 1]) + (S[qx][t + 1] - U[qx][t - 1])));
                const double b = 3.0 * ((1.0 / 9.0) * (U[qy][t] - S[qy][t]) +
                                        (1.0 / 36.0) * ((U[qy][t + 1] - S[qy][t - 1]) + (U[qy][t - 1] - S[qy][t + 1])));
                cb[k] = -(a + b);
            }
            const double rho = rk_prev[0] + rk_prev[1] + rk_prev[2];
            double cr = 0.0;
            for (int k = 0; k < 3; ++k) cr += cb[k] * rk_prev[k];
            const double irho = 1.0 / rho;
            const int64_t jc = (int64_t)yc * g.nx + x;
            for (int k = 0; k < 3; ++k) lam[(9 + k) * N + jc] = part_prev[k] + cb[k] * irho - cr * (irho * irho);
        }
        for (int k = 0; k < 3; ++k) {
            rk_prev[k] = rk[k];
            part_prev[k] = part[k];
        }
    }
    // per-workgroup sums of the stress part of dL/dsigma (the ring is free again)
    __syncthreads();
    double* red = &ring[0][0][0];
    for (int p = 0; p < 3; ++p) sig_st[p] = wave_sum(sig_st[p]);
    if ((t & 63) == 0)
        for (int p = 0; p < 3; ++p) red[p * NT + (t >> 6)] = sig_st[p];
    __syncthreads();
    if (t < 3) {
        double v = red[t * NT];
        for (int q = 1; q < NT / 64; ++q) v += red[t * NT + q];
        w.sig[(int64_t)blockIdx.x * 6 + 3 + t] += v;
    }
}

// A2 at one node (the reverse of the stress and the pair quantities), as the march forms it
// for a row: from dL/dF at the eight neighbours (E, W, N, S, NE, NW, SE, SW), the tape's
// densities rk and gradients gc, dL/dG (Gb) and, for an owned node, A1's node-local dL/drho_k
// (rbar): dL/d(grad c_k) (gcb), the node's part of dL/drho_k (part, owned nodes) and the
// stress part of dL/dsigma (sig_st, owned nodes).
__device__ __forceinline__ void sf_node(const Geo& g, const double (&Fb)[2][8], const double (&rkin)[3],
                                        const double (&gcin)[6], const double (&Gbin)[6], const double (&rbar)[3],
                                        bool own, double (&gcb)[3][2], double (&part)[3], double (&sig_st)[3])
{
    double dFx_dx, dFx_dy, dFy_dx, dFy_dy;
    grad8(Fb[0], dFx_dx, dFx_dy);
    grad8(Fb[1], dFy_dx, dFy_dy);
    const double Tbxx = -dFx_dx, Tbxy = -(dFx_dy + dFy_dx), Tbyy = -dFy_dy;
    double rk[3], c[3], gx[3], gy[3];
    for (int k = 0; k < 3; ++k) rk[k] = rkin[k];
    const double rho = rk[0] + rk[1] + rk[2];
    const double ir = 1.0 / rho;
    for (int k = 0; k < 3; ++k) {
        c[k] = rk[k] * ir;
        gx[k] = gcin[2 * k];
        gy[k] = gcin[2 * k + 1];
    }
    double cb[3] = {0, 0, 0}, rb[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) gcb[k][0] = gcb[k][1] = 0.0;
    for (int p = 0; p < 3; ++p) {
        const int k = PK[p], l = PL[p];
        const PairFwd f = pair_fwd(g, p, c, gx, gy, rk);
        if (!f.on) continue;
        double Gbx = Gbin[2 * p], Gby = Gbin[2 * p + 1];
        const double Q = Tbxx * f.Gy * f.Gy - Tbxy * f.Gx * f.Gy + Tbyy * f.Gx * f.Gx;
        const double h = g.sigma[p] * f.C * f.im;
        Gbx += h * (2.0 * Tbyy * f.Gx - Tbxy * f.Gy);
        Gby += h * (2.0 * Tbxx * f.Gy - Tbxy * f.Gx);
        const double mb = -Q * g.sigma[p] * f.C * (f.im * f.im);
        Gbx += mb * f.Gx * f.im;
        Gby += mb * f.Gy * f.im;
        if (own) sig_st[p] += Q * f.C * f.im;
        if (f.unclipped) {
            const double Cb = Q * g.sigma[p] * f.im;
            rb[k] += Cb * g.cfac[p] * rk[l];
            rb[l] += Cb * g.cfac[p] * rk[k];
        }
        cb[l] += Gbx * gx[k] + Gby * gy[k];
        cb[k] -= Gbx * gx[l] + Gby * gy[l];
        gcb[k][0] += c[l] * Gbx;
        gcb[k][1] += c[l] * Gby;
        gcb[l][0] -= c[k] * Gbx;
        gcb[l][1] -= c[k] * Gby;
    }
    if (own) {
        double cr = 0.0;
        for (int k = 0; k < 3; ++k) cr += cb[k] * rk[k];
        const double irho = 1.0 / rho;
        for (int k = 0; k < 3; ++k) part[k] = rbar[k] + (rb[k] + cb[k] * irho - cr * (irho * irho));
    }
}

// A3 at an owned node: dL/drho_k of the new adjoint state from dL/d(grad c_k) of the rows
// below (S), at (C) and above (U) the node, at column t, and the node's part.
template <int BX>
__device__ __forceinline__ void a3_node(const double (*S)[BX], const double (*C)[BX], const double (*U)[BX], int t,
                                        const double (&rk)[3], const double (&part)[3], double (&out)[3])
{
    double cb[3];
    for (int k = 0; k < 3; ++k) {
        const int qx = 2 * k, qy = 2 * k + 1;
        const double a = 3.0 * ((1.0 / 9.0) * (C[qx][t + 1] - C[qx][t - 1]) +
                                (1.0 / 36.0) * ((U[qx][t + 1] - S[qx][t - 1]) + (S[qx][t + 1] - U[qx][t - 1])));
        const double b = 3.0 * ((1.0 / 9.0) * (U[qy][t] - S[qy][t]) +
                                (1.0 / 36.0) * ((U[qy][t + 1] - S[qy][t - 1]) + (U[qy][t - 1] - S[qy][t + 1])));
        cb[k] = -(a + b);
    }
    const double rho = rk[0] + rk[1] + rk[2];
    double cr = 0.0;
    for (int k = 0; k < 3; ++k) cr += cb[k] * rk[k];
    const double irho = 1.0 / rho;
    for (int k = 0; k < 3; ++k) out[k] = part[k] + cb[k] * irho - cr * (irho * irho);
}

// Per-workgroup sums of six dL/dsigma parts into w.sig[blockIdx.x][0..5] (red: LDS of at
// least 6 x waves doubles, free on entry).
template <int NT>
__device__ __forceinline__ void add_sig6(const double (&v)[6], double* red, double* __restrict__ sig)
{
    constexpr int W = NT / 64;
    const int t = threadIdx.x;
    double s[6];
    for (int q = 0; q < 6; ++q) s[q] = wave_sum(v[q]);
    if ((t & 63) == 0)
        for (int q = 0; q < 6; ++q) red[q * W + (t >> 6)] = s[q];
    __syncthreads();
    if (t < 6) {
        double a = red[t * W];
        for (int k = 1; k < W; ++k) a += red[t * W + k];
        sig[(int64_t)blockIdx.x * 6 + t] += a;
    }
}

// A2 + A3 on two-dimensional blocks (small lattices, where the march's two warm-up rows
// per tile and its row-by-row round trips are most of the time): a workgroup of BX x BY
// lanes owns at most (BX - 2) x (BY - 2) nodes, lane (tx, ty) on node (x0 - 1 + tx,
// y0 - 1 + ty).  Every lane forms dL/d(grad c_k) of its node into LDS as the march does for
// a row; after one barrier the owned lanes complete their nodes.  The arithmetic of every
// node is the march's.
template <int BX, int BY>
__global__ __launch_bounds__(BX * BY) void k_adj_sf_block(Geo g, AdjWS w, const Tile* __restrict__ tiles,
                                                          double* __restrict__ lam)
{
    __shared__ double gb[BY][6][BX];
    const Tile tl = tiles[blockIdx.x];
    const int t = threadIdx.x, tx = t % BX, ty = t / BX;
    const int64_t N = (int64_t)g.nx * g.ny;
    const bool on = tx <= tl.cols + 1 && ty <= tl.rows + 1;
    const bool own = tx >= 1 && tx <= tl.cols && ty >= 1 && ty <= tl.rows;
    const int x = wrapi(tl.x0 - 1 + tx, g.nx), y = wrapi(tl.y0 - 1 + ty, g.ny);
    double sig[6] = {0, 0, 0, 0, 0, 0}, sig_st[3] = {0, 0, 0};
    double rk[3] = {0, 0, 0}, part[3] = {0, 0, 0};
    if (on) {
        SfIn in;
        sf_load(g, w, N, wrapi(x - 1, g.nx), x, wrapi(x + 1, g.nx), y, own, in);
        double gcb[3][2];
        sf_node(g, in.Fb, in.rk, in.gc, in.Gb, in.rbar, own, gcb, part, sig_st);
        for (int k = 0; k < 3; ++k) {
            rk[k] = in.rk[k];
            gb[ty][2 * k][tx] = gcb[k][0];
            gb[ty][2 * k + 1][tx] = gcb[k][1];
        }
    }
    __syncthreads();
    if (own) {
        double out[3];
        a3_node<BX>(gb[ty - 1], gb[ty], gb[ty + 1], tx, rk, part, out);
        const int64_t jc = (int64_t)y * g.nx + x;
        for (int k = 0; k < 3; ++k) lam[(9 + k) * N + jc] = out[k];
    }
    // the stress part of dL/dsigma (the LDS is free again)
    __syncthreads();
    for (int p = 0; p < 3; ++p) sig[3 + p] = sig_st[p];
    add_sig6<BX * BY>(sig, &gb[0][0][0], w.sig);
}

// One whole reverse step, A1 + A2 + A3, on two-dimensional blocks (small lattices): a
// workgroup of BX x BY lanes owns at most (BX - 4) x (BY - 4) nodes, lane (tx, ty) on node
// (x0 - 2 + tx, y0 - 2 + ty).  Every lane runs A1 at its node (adj_local_node) and puts its
// dL/dF in LDS; the lanes within one of the block run A2 (sf_node) on those and put dL/d(grad
// c_k) in LDS; the owned lanes run A3.  dL/dF, dL/dG and A1's dL/drho_k stay on chip, and a
// step is one launch instead of two.  Each node's arithmetic is that of k_adj_local and the
// march.
template <int BX, int BY>
__global__ __launch_bounds__(BX * BY) void k_adj_block(const double* __restrict__ lamp, Geo g, AdjWS w,
                                                       const Tile* __restrict__ tiles, double* __restrict__ lamn)
{
    __shared__ double Fs[BY][2][BX];
    __shared__ double gb[BY][6][BX];
    const Tile tl = tiles[blockIdx.x];
    const int t = threadIdx.x, tx = t % BX, ty = t / BX;
    const int64_t N = (int64_t)g.nx * g.ny;
    const bool in1 = tx <= tl.cols + 3 && ty <= tl.rows + 3;
    const bool in2 = tx >= 1 && tx <= tl.cols + 2 && ty >= 1 && ty <= tl.rows + 2;
    const bool own = tx >= 2 && tx <= tl.cols + 1 && ty >= 2 && ty <= tl.rows + 1;
    const int x = wrapi(tl.x0 - 2 + tx, g.nx), y = wrapi(tl.y0 - 2 + ty, g.ny);
    const int64_t j = (int64_t)y * g.nx + x;
    double sig[6] = {0, 0, 0, 0, 0, 0}, sig_st[3] = {0, 0, 0};
    LocalOut o;
    for (int p = 0; p < 3; ++p) o.Gb[p][0] = o.Gb[p][1] = o.rb[p] = 0.0;
    if (in1) {
        adj_local_node(lamp, g, w, x, y, o);
        Fs[ty][0][tx] = o.Fb[0];
        Fs[ty][1][tx] = o.Fb[1];
        if (own) {
            for (int i = 0; i < 9; ++i) lamn[i * N + j] = o.fb[i];
            for (int p = 0; p < 3; ++p) sig[p] = o.sigb[p];
        }
    }
    __syncthreads();
    double rk[3] = {0, 0, 0}, part[3] = {0, 0, 0};
    if (in2) {
        double Fb[2][8];
        for (int c = 0; c < 2; ++c) {
            Fb[c][0] = Fs[ty][c][tx + 1];
            Fb[c][1] = Fs[ty][c][tx - 1];
            Fb[c][2] = Fs[ty + 1][c][tx];
            Fb[c][3] = Fs[ty - 1][c][tx];
            Fb[c][4] = Fs[ty + 1][c][tx + 1];
            Fb[c][5] = Fs[ty + 1][c][tx - 1];
            Fb[c][6] = Fs[ty - 1][c][tx + 1];
            Fb[c][7] = Fs[ty - 1][c][tx - 1];
        }
        double gc[6], Gb[6];
        for (int k = 0; k < 3; ++k) rk[k] = w.rho[k * N + j];
        for (int q = 0; q < 6; ++q) gc[q] = w.gc[q * N + j];
        for (int p = 0; p < 3; ++p) {
            Gb[2 * p] = o.Gb[p][0];
            Gb[2 * p + 1] = o.Gb[p][1];
        }
        double gcb[3][2];
        sf_node(g, Fb, rk, gc, Gb, o.rb, own, gcb, part, sig_st);
        for (int k = 0; k < 3; ++k) {
            gb[ty][2 * k][tx] = gcb[k][0];
            gb[ty][2 * k + 1][tx] = gcb[k][1];
        }
    }
    __syncthreads();
    if (own) {
        double out[3];
        a3_node<BX>(gb[ty - 1], gb[ty], gb[ty + 1], tx, rk, part, out);
        for (int k = 0; k < 3; ++k) lamn[(9 + k) * N + j] = out[k];
    }
    __syncthreads();
    for (int p = 0; p < 3; ++p) sig[3 + p] = sig_st[p];
    add_sig6<BX * BY>(sig, &gb[0][0][0], w.sig);
}

// The adjoint state is kept factored per node as (dL/df_i, dL/drho_k), 12 values: f_{i,k}
// enters the step only through f_i = sum_k f_{i,k} and rho_k = sum_i f_{i,k}, so
// dL/df_{i,k}(x) = dL/df_i(x) + dL/drho_k(x) and dL/dB_{i,k}(x - e_i) is that sum.
// Seed: dL/drho_1(x, T) = g(x), everything else 0.
__global__ __launch_bounds__(256) void k_adj_seed(const double* __restrict__ gT, Geo g, double* __restrict__ lam)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= g.nx) return;
    const int64_t N = (int64_t)g.nx * g.ny, j = (int64_t)y * g.nx + x;
    for (int q = 0; q < 12; ++q) lam[q * N + j] = q == 9 ? gT[j] : 0.0;
}

// initial state B_{i,k}(y) = w_i rho_k(y + e_i):  dL/drho_k(x) = sum_i w_i dL/dB_{i,k}(x - e_i)
__global__ __launch_bounds__(256) void k_adj_rho0(const double* __restrict__ lam, Geo g, double* __restrict__ out)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= g.nx) return;
    const int64_t N = (int64_t)g.nx * g.ny, j = (int64_t)y * g.nx + x;
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int i = 0; i < 9; ++i) s += wgt(i) * (lam[i * N + j] + lam[(9 + k) * N + j]);
        out[k * N + j] = s;
    }
}

// Width of the fused A2 + A3 workgroup by lattice width: narrow strips keep small
// lattices' tiles numerous enough to fill the device (measured at 256^2: 64 lanes beat
// 128 by 3%; at 2048^2 256 lanes).
int sf_width(int nx) { return nx >= 1024 ? 256 : 64; }

int sf_occupancy(int nt)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (nt) {
        case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_sf<64>, 64, 0); break;
        case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj_sf<256>, 256, 0); break;
        default: break;
    }
    return e == hipSuccess ? nb : 0;
}

// The reverse steps by lattice size: up to kAdjFusedMaxNodes nodes one launch of k_adj_block
// per step (blocks of kAdjBlockX x kAdjBlockY lanes); up to kSfBlockMaxNodes k_adj_local and
// k_adj_sf_block (blocks of kSfBlockX x kSfBlockY lanes); above, or where the forward's
// one-step launches keep to the march, k_adj_local and the march.
// Measured (adjoint MLUPS, fused vs two kernels): 3.23k vs 2.64k at 256^2, 3.56k vs 3.99k
// at 512^2, 3.62k vs 3.80k at 1024^2; the fused step runs A1 on the halo ring too, which
// costs more than the launch it saves once the lattice fills the device.
constexpr int kSfBlockX = 32, kSfBlockY = 8;
constexpr int kAdjBlockX = 32, kAdjBlockY = 16;
constexpr int64_t kAdjFusedMaxNodes = (int64_t)1 << 17;
constexpr int64_t kSfBlockMaxNodes = (int64_t)1 << 20;

// nt: march width (64 or 256), or 0 for the block pass
void launch_sf(int nt, int ntiles, hipStream_t q, const Geo& g, const AdjWS& w, const Tile* tiles, double* lam)
{
    switch (nt) {
        case 0:
            hipLaunchKernelGGL((k_adj_sf_block<kSfBlockX, kSfBlockY>), dim3(ntiles), dim3(kSfBlockX * kSfBlockY), 0, q,
                               g, w, tiles, lam);
            break;
        case 64: hipLaunchKernelGGL(k_adj_sf<64>, dim3(ntiles), dim3(64), 0, q, g, w, tiles, lam); break;
        default: hipLaunchKernelGGL(k_adj_sf<256>, dim3(ntiles), dim3(256), 0, q, g, w, tiles, lam); break;
    }
}

Geo geo_of(const KParams& kp)
{
    Geo g;
    g.nx = kp.nx;
    g.ny = kp.ny;
    g.plane = kp.plane;
    g.pitch = kp.pitch;
    for (int p = 0; p < 3; ++p) {
        g.sigma[p] = kp.sigma[p];
        g.g[p] = kp.g[p];
        g.inv_nu[p] = kp.inv_nu[p];
        g.cfac[p] = kp.cfac[p];
    }
    g.beta0 = kp.beta0;
    g.guard = kp.guard;
    return g;
}

// derivative of g(X) of Eq. (20) (zero where |X| is snapped to 1 and outside [-1, 1])
double dg_dX(double X)
{
    if (X >= 1.0 - 1e-12 || X <= -1.0 + 1e-12) return 0.0;
    const double s = std::sqrt((1.0 - X) * (1.0 + X));
    return X < 0.0 ? X / s : -X / s;
}

}  // namespace

void adjoint_release(lbm3* h)
{
    if (h->adj_stream) (void)hipStreamSynchronize(h->adj_stream);
    if (h->adj_stream2) (void)hipStreamSynchronize(h->adj_stream2);
    for (void* p : h->ckpt)
        if (p) (void)hipFree(p);
    h->ckpt.clear();
    if (h->adj_ws) (void)hipFree(h->adj_ws);
    h->adj_ws = nullptr;
    h->adj_ws_bytes = 0;
    h->tape_valid = false;
}

void adjoint_destroy(lbm3* h)
{
    adjoint_release(h);
    if (h->adj_event) (void)hipEventDestroy(h->adj_event);
    if (h->adj_stream) (void)hipStreamDestroy(h->adj_stream);
    if (h->adj_stream2) (void)hipStreamDestroy(h->adj_stream2);
    h->adj_stream2 = nullptr;
    h->adj_event = nullptr;
    h->adj_stream = nullptr;
}

}  // namespace tcg

using namespace tcg;

static int ensure_ws(lbm3* h, size_t bytes)
{
    if (h->adj_ws_bytes >= bytes) return LBM3_OK;
    if (h->adj_ws) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->adj_ws);
        h->adj_ws = nullptr;
        h->adj_ws_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->adj_ws, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(adjoint workspace)");
    h->adj_ws_bytes = bytes;
    return LBM3_OK;
}

extern "C" {

int lbm3_adjoint_pipeline_slots(int64_t nodes, uint64_t ws_two_slots, uint64_t ws_held, uint64_t device_free)
{
    // The overlap pays below 2^22 nodes (measured: +47% at 256^2, +7% at 512^2, +2% at
    // 1024^2, none at 2048^2).  A held workspace is freed before a larger one is allocated,
    // so the two-slot workspace must fit in the free memory plus what is held, keeping 1/16
    // of it in reserve for the runtime.
    if (nodes >= ((int64_t)1 << 22)) return 1;
    if (ws_two_slots <= ws_held) return 2;
    const uint64_t avail = device_free + ws_held;
    return ws_two_slots <= avail - avail / 16 ? 2 : 1;
}

int lbm3_adjoint_record(lbm3_t* h, int64_t nsteps, int32_t ckpt_every)
{
    if (!h) {
        set_error("handle is NULL");
        return LBM3_EINVAL;
    }
    if (h->prec != Prec::F64) {
        set_error("the adjoint is provided for LBM3_FP64 only");
        return LBM3_EUNSUPPORTED;
    }
    if (h->p.beta_law != LBM3_BETA_PAPER || h->p.forcing != LBM3_FORCING_GUO) {
        set_error("the adjoint is provided for the paper's segregation law and forcing "
                  "(LBM3_BETA_PAPER, LBM3_FORCING_GUO) only");
        return LBM3_EUNSUPPORTED;
    }
    if (!h->ready || h->step != 0 || !h->init_at_rest) {
        set_error("lbm3_adjoint_record needs the state set by lbm3_init_fields(rho, NULL) at step 0");
        return LBM3_ESTATE;
    }
    if (nsteps < 1 || ckpt_every < 1 || nsteps % ckpt_every) {
        set_error("nsteps >= 1 must be a multiple of ckpt_every >= 1");
        return LBM3_EINVAL;
    }
    adjoint_release(h);
    // checkpoint s holds the state at step s K: the 27 populations for s = 0 (from
    // init_fields), the factored state after that
    const int64_t nseg = nsteps / ckpt_every;
    const size_t bytes27 = (size_t)h->kp.span * sizeof(double);
    const size_t bytesfac = (size_t)h->kp.fpitch * h->kp.ny * sizeof(double);
    h->ckpt.assign(nseg, nullptr);
    for (int64_t c = 0; c < nseg; ++c) {
        hipError_t e = hipMalloc(&h->ckpt[c], c == 0 ? bytes27 : bytesfac);
        if (e != hipSuccess) {
            int rc = hip_fail(e, "hipMalloc(checkpoint)");
            adjoint_release(h);
            return rc;
        }
    }
    hipError_t e = hipMemcpyAsync(h->ckpt[0], h->buf[h->cur], bytes27, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
    for (int64_t c = 1; c <= nseg; ++c) {
        int rc = step_handle(h, ckpt_every);
        if (rc) return rc;
        if (c == nseg) break;
        e = hipMemcpyAsync(h->ckpt[c], h->buf[h->cur], bytesfac, hipMemcpyDeviceToDevice, h->stream);
        if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
    }
    h->tape_steps = nsteps;
    h->tape_every = ckpt_every;
    h->tape_valid = true;
    return LBM3_OK;
}

int lbm3_adjoint(lbm3_t* h, const double* drho1_T, double dsigma[3], double* drho0)
{
    if (!h || !drho1_T) {
        set_error("handle or drho1_T is NULL");
        return LBM3_EINVAL;
    }
    if (!h->tape_valid) {
        set_error("lbm3_adjoint needs a preceding lbm3_adjoint_record (and no step since)");
        return LBM3_ESTATE;
    }
    const KParams& kp = h->kp;
    const int64_t N = (int64_t)kp.nx * kp.ny;
    for (int64_t j = 0; j < N; ++j)
        if (!std::isfinite(drho1_T[j])) {
            set_error("drho1_T is not finite at node %lld", (long long)j);
            return LBM3_EINVAL;
        }
    const Geo g = geo_of(kp);
    const dim3 grid((kp.nx + 255) / 256, kp.ny), blk(256);
    const int64_t nblocks = (int64_t)grid.x * grid.y;
    // tiles of the fused A2 + A3 pass: blocks where the forward takes its one-step blocks
    // (ntilesb > 0: at most 2^20 nodes and no march shape chosen by lbm3_set_tile or
    // lbm3_set_steps_per_launch(2)), else strips of at most sf_width - 2 columns, rows
    // fitted to the resident workgroups
    const bool sf_block = h->ntilesb > 0 && N <= kSfBlockMaxNodes;
    const bool fused = sf_block && N <= kAdjFusedMaxNodes;
    const int sfw = sf_block ? 0 : sf_width(kp.nx);
    std::vector<Tile> sf_plan;
    if (fused) {
        plan_blocks(0, kp.nx, kp.ny, kAdjBlockX - 4, kAdjBlockY - 4, sf_plan);
    } else if (sf_block) {
        plan_blocks(0, kp.nx, kp.ny, kSfBlockX - 2, kSfBlockY - 2, sf_plan);
    } else {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 1;
        const int sf_rows = auto_rows(kp.nx, kp.ny, sfw, std::max(1, sf_occupancy(sfw)) * std::max(cus, 1), 8, 1);
        plan_lattice(0, kp.nx, kp.ny, sfw, sf_rows, 8, sf_plan, 1);
    }
    const std::vector<Tile> sf_tiles = xcd_order(sf_plan, 8);
    const int sf_ntiles = (int)sf_tiles.size();
    const int64_t nsig = std::max<int64_t>(nblocks, sf_ntiles);
    const size_t sbytes = (size_t)kp.span * sizeof(double);
    const size_t fbytes = (size_t)kp.fpitch * kp.ny * sizeof(double);
    const size_t tbytes = (size_t)kTapeFields * N * sizeof(double);
    const int K = h->tape_every;
    const int64_t nseg = h->tape_steps / K;
    // workspace: 11 adjoint fields of N doubles, two factored adjoint states (12 fields), per
    // pipeline slot two forward state buffers and the tape of K steps (20 fields each), the
    // dL/dsigma partial sums, dL/drho_1(T), the fused pass's tiles
    const size_t fields = (size_t)(3 + 2 + 6) * N;
    const size_t lbytes = (size_t)12 * N * sizeof(double);
    auto need_of = [&](int slots) {
        return fields * sizeof(double) + 2 * lbytes + slots * (2 * sbytes + (size_t)K * tbytes) +
               (size_t)nsig * 6 * sizeof(double) + N * sizeof(double) + sf_tiles.size() * sizeof(Tile);
    };
    // Two pipeline slots (the recompute of the next segment beside the reverse steps of the
    // current one) on small lattices where the second slot fits; else one.
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    int nslots = lbm3_adjoint_pipeline_slots(N, need_of(2), h->adj_ws_bytes, free_b);
    int rc = ensure_ws(h, need_of(nslots));
    if (rc == LBM3_ENOMEM && nslots == 2) {
        nslots = 1;  // the second slot did not fit after all: the one-slot sweep needs half the tape
        rc = ensure_ws(h, need_of(1));
    }
    if (rc) return rc;
    const bool overlap = nslots == 2;
    double* d = (double*)h->adj_ws;
    AdjWS w;
    w.rho = w.ftot = w.gc = w.F = nullptr;  // per step: the tape of that step
    w.rbar = d;
    w.Fbar = w.rbar + 3 * N;
    w.Gbar = w.Fbar + 2 * N;
    double* lam[2];
    lam[0] = w.Gbar + 6 * N;
    lam[1] = lam[0] + 12 * N;
    // slot b: forward buffers fwd[b][0..1] and tape[b] (one slot: both names are slot 0)
    char* fbase = (char*)(lam[1] + 12 * N);
    char* fwd[2][2] = {{fbase, fbase + sbytes}, {fbase + 2 * sbytes, fbase + 3 * sbytes}};
    double* tbase = (double*)(fbase + 2 * nslots * sbytes);
    double* tape[2] = {tbase, tbase + (size_t)K * kTapeFields * N};
    if (!overlap) {
        fwd[1][0] = fwd[0][0], fwd[1][1] = fwd[0][1];
        tape[1] = tape[0];
    }
    w.sig = tbase + (size_t)nslots * K * kTapeFields * N;
    double* gT = w.sig + nsig * 6;
    Tile* dsf = (Tile*)(gT + N);
    // The reverse steps run on the handle's own adjoint stream (graph capture needs a stream
    // other than the null stream) and the segment recomputes on a second one, both ordered
    // after the work already on the handle's stream.
    hipError_t e = hipSuccess;
    if (!h->adj_stream) e = hipStreamCreateWithFlags(&h->adj_stream, hipStreamNonBlocking);
    if (e == hipSuccess && !h->adj_stream2) e = hipStreamCreateWithFlags(&h->adj_stream2, hipStreamNonBlocking);
    if (e == hipSuccess && !h->adj_event) e = hipEventCreateWithFlags(&h->adj_event, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(h->adj_event, h->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint stream set-up");
    hipStream_t st = h->adj_stream, sf2 = h->adj_stream2;
    e = hipStreamWaitEvent(st, h->adj_event, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(sf2, h->adj_event, 0);
    if (e == hipSuccess) e = hipMemsetAsync(w.sig, 0, (size_t)nsig * 6 * sizeof(double), st);
    if (e == hipSuccess) e = hipMemcpyAsync(gT, drho1_T, N * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dsf, sf_tiles.data(), sf_tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint set-up");
    int cl = 0;
    hipLaunchKernelGGL(k_adj_seed, grid, blk, 0, st, gT, g, lam[cl]);
    // The sweep takes the segments last to first.  Segment s is recomputed from its
    // checkpoint into pipeline slot s & 1 (K forward steps recording the tape) on the second
    // stream, while the reverse steps of segment s + 1 run from the other slot; events order
    // a slot's tape before its reverse steps, and its reverse steps before the slot is
    // recomputed again.  The launch arguments depend only on the slot and the adjoint
    // buffer's parity, so after the first use each sequence is captured once and replayed
    // (segment 0 starts from the 27-population state and runs eagerly).
    auto recompute = [&](hipStream_t q, Fmt in, int b) -> hipError_t {
        hipError_t r = hipSuccess;
        for (int j = 0; j < K && r == hipSuccess; ++j) {
            const Fmt fj = j == 0 ? in : Fmt::FAC;
            double* tj = tape[b] + (size_t)j * kTapeFields * N;
            // small lattices: the block step (as the forward steps took), else the march
            r = fj == Fmt::FAC && h->ntilesb > 0
                    ? tiles_f64_block_tape(fwd[b][j & 1], fwd[b][(j + 1) & 1], h->dinst, h->dtilesb, h->ntilesb, tj,
                                           q)
                    : tiles_f64_tape(fj, fwd[b][j & 1], fwd[b][(j + 1) & 1], h->dinst, h->dtiles, h->ntiles,
                                     h->threads, tj, q);
        }
        return r;
    };
    auto reverse = [&](hipStream_t q, int b, int cl0) -> hipError_t {
        hipError_t r = hipSuccess;
        int c = cl0;
        for (int j = K - 1; j >= 0 && r == hipSuccess; --j) {
            AdjWS wj = w;
            wj.rho = tape[b] + (size_t)j * kTapeFields * N;
            wj.ftot = wj.rho + 3 * N;
            wj.gc = wj.rho + 12 * N;
            wj.F = wj.rho + 18 * N;
            if (fused) {
                hipLaunchKernelGGL((k_adj_block<kAdjBlockX, kAdjBlockY>), dim3(sf_ntiles), dim3(kAdjBlockX * kAdjBlockY),
                                   0, q, (const double*)lam[c], g, wj, (const Tile*)dsf, lam[c ^ 1]);
            } else {
                hipLaunchKernelGGL(k_adj_local, grid, blk, 0, q, (const double*)lam[c], g, wj, lam[c ^ 1]);
                launch_sf(sfw, sf_ntiles, q, g, wj, dsf, lam[c ^ 1]);
            }
            c ^= 1;
            r = hipGetLastError();
        }
        return r;
    };
    hipGraphExec_t gF[2] = {nullptr, nullptr}, gR[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    auto drop = [&]() {
        for (auto& x : gF)
            if (x) (void)hipGraphExecDestroy(x);
        for (auto& row : gR)
            for (auto& x : row)
                if (x) (void)hipGraphExecDestroy(x);
        for (auto* ev : {&ready[0], &ready[1], &freed[0], &freed[1]})
            if (*ev) (void)hipEventDestroy(*ev);
    };
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipEventCreateWithFlags(&ready[b], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&freed[b], hipEventDisableTiming);
    }
    // runs `body` on stream q, from a graph captured on its first use when replays pay off
    auto run = [&](hipStream_t q, hipGraphExec_t& gx, bool graph, auto body) -> hipError_t {
        if (!graph) return body(q);
        if (!gx) {
            hipGraph_t gr = nullptr;
            hipError_t r = hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal);
            if (r != hipSuccess) return r;
            const hipError_t le = body(q);
            r = hipStreamEndCapture(q, &gr);
            if (r == hipSuccess) r = le;
            if (r == hipSuccess) r = hipGraphInstantiate(&gx, gr, nullptr, nullptr, 0);
            if (gr) (void)hipGraphDestroy(gr);
            if (r != hipSuccess) return r;
        }
        return hipGraphLaunch(gx, q);
    };
    const bool graphs = nseg >= 3;
    bool slot_used[2] = {false, false};
    hipStream_t rq = overlap ? sf2 : st;  // the recompute's stream
    // recompute segment s into its slot
    auto start_segment = [&](int64_t s) -> hipError_t {
        const int b = overlap ? (int)(s & 1) : 0;
        const Fmt in = s == 0 ? Fmt::F27 : Fmt::FAC;
        hipError_t r = slot_used[b] ? hipStreamWaitEvent(rq, freed[b], 0) : hipSuccess;
        if (r == hipSuccess)
            r = hipMemcpyAsync(fwd[b][0], h->ckpt[s], in == Fmt::F27 ? sbytes : fbytes, hipMemcpyDeviceToDevice, rq);
        if (r == hipSuccess)
            r = run(rq, gF[b], graphs && s > 0, [&](hipStream_t q) { return recompute(q, in, b); });
        if (r == hipSuccess) r = hipEventRecord(ready[b], rq);
        slot_used[b] = true;
        return r;
    };
    if (e == hipSuccess && overlap) e = start_segment(nseg - 1);
    for (int64_t s = nseg - 1; s >= 0 && e == hipSuccess; --s) {
        const int b = overlap ? (int)(s & 1) : 0;
        if (!overlap) e = start_segment(s);
        else if (s > 0) e = start_segment(s - 1);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ready[b], 0);
        if (e == hipSuccess) e = run(st, gR[b][cl], graphs, [&](hipStream_t q) { return reverse(q, b, cl); });
        if (e == hipSuccess) e = hipEventRecord(freed[b], st);
        cl ^= K & 1;
    }
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(sf2);
        (void)hipStreamSynchronize(st);
        drop();
        return hip_fail(e, "adjoint sweep");
    }
    double* r0 = (double*)fwd[0][0];  // reuse (slot 0's recompute ended before the last reverse steps)
    hipLaunchKernelGGL(k_adj_rho0, grid, blk, 0, st, (const double*)lam[cl], g, r0);
    std::vector<double> sig((size_t)nsig * 6);
    e = hipGetLastError();
    if (e == hipSuccess && drho0) e = hipMemcpyAsync(drho0, r0, 3 * N * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sig.data(), w.sig, sig.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    hipError_t es = hipStreamSynchronize(st);
    const hipError_t es2 = hipStreamSynchronize(sf2);
    if (es == hipSuccess) es = es2;
    drop();
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return hip_fail(e, "adjoint results");
    // sigma: stress part directly; segregation part through g'(X_p) dX_p/dsigma_q
    double Sb[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = 0; b < nsig; ++b)
        for (int a = 0; a < 6; ++a) Sb[a] += sig[b * 6 + a];
    double ds[3] = {Sb[3], Sb[4], Sb[5]};
    const double* sgm = h->p.sigma;
    auto pidx = [](int a, int b) { return (a > b ? (b == 0 ? (a == 1 ? 0 : 1) : 2) : (a == 0 ? (b == 1 ? 0 : 1) : 2)); };
    for (int p = 0; p < 3; ++p) {
        const int k = PK[p], l = PL[p], m = 3 - k - l;
        const int imk = pidx(m, k), iml = pidx(m, l);
        const double smk = sgm[imk], sml = sgm[iml], skl = sgm[p];
        const double X = (smk * smk + sml * sml - skl * skl) / (2.0 * smk * sml);
        const double gp = dg_dX(X) * Sb[p];
        ds[p] += gp * (-skl / (smk * sml));
        ds[imk] += gp * (1.0 / sml - X / smk);
        ds[iml] += gp * (1.0 / smk - X / sml);
    }
    if (dsigma)
        for (int p = 0; p < 3; ++p) dsigma[p] = ds[p];
    return LBM3_OK;
}

}  // extern "C"
