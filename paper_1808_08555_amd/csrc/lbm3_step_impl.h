// The fused ternary colour-gradient LBM time step for CDNA4 (gfx950): device code shared by
// the per-precision instantiations (lbm3_tiles_*.hip) and the companion kernels
// (lbm3_step.hip).
//
// One time step (Yu, Liu, Liang, Zhang, arXiv:1808.08555, Sec. 2) at node x:
//   pull:     f_{i,k}(x) = state_{i,k}(x - e_i)                              (Eq. 22)
//   moments:  rho_k = sum_i f_{i,k}, f_i = sum_k f_{i,k}, c_k = rho_k / rho
//   gradient: grad c_k by the isotropic difference of Eq. (12)
//   stress:   T = sum over pairs sigma_kl C_kl |G_kl| (I - n_kl n_kl)   (Eq. 7, the
//             ordered double sum with 1/2 collapsed to one term per unordered pair,
//             since G_lk = -G_kl), C_kl of Eq. (6), G_kl = c_l grad c_k - c_k grad c_l
//   force:    F = div T, again with the difference of Eq. (12)
//   collide:  local tau from the harmonic viscosity mean (Eqs. 10-11), u with the
//             half force (Eq. 9), f_eq (Eq. 3), Guo term (Eq. 8), BGK (Eqs. 1-2)
//   recolour: f_ddag_{i,k} = c_k f_dag_i + w_i V_k . e_i, V_k = sum_{l != k} beta_kl
//             (rho_k rho_l / rho) n_kl with beta_kl of Eqs. (19)-(20)      (Eq. 13)
//   store:    the recoloured state of x, factored (FAC): the 16 values f_dag_i(x), c_k(x),
//             V_0(x), V_1(x) (V_2 = -(V_0 + V_1): the recolouring vectors of the three
//             fluids sum to zero).  Eq. (13) makes every f_ddag_{i,k}(x) a function of
//             these, so the next step rebuilds the populations it pulls from x - e_i with
//             recon(), the arithmetic the export of the 27 populations uses.  The first step
//             reads the 27 populations (F27) that initialisation writes.  FAC moves 16/27 of
//             the bytes of F27.
//
// Layout: plane q of node (x, y) at element q*plane + y*pitch + x, x fastest, with the rows of
// all planes interleaved (pitch = 27 plane for F27, 16 plane for FAC), so one lattice row
// of the state is one contiguous block and a wavefront's 64 lanes touch 64 consecutive values
// of one plane row.  FAC planes: 0-8 f_dag_i, 9-11 c_k, 12-15 (V_kx, V_ky) for k = 0, 1.
//
// Work decomposition (y-marching strips).  A workgroup of NT threads owns a strip of
// cols <= NT-6 output columns and a run of `rows` output rows.  Thread t sits on column
// x0 - 3 + t and marches up the rows.  Per row, stage 1 obtains the 9 totals and 3
// densities of its column (F27: 27 pulled loads; FAC: 9 pulled f_dag loads plus the c_k and
// V_k of the source row, shared with the neighbouring columns through LDS) and keeps them
// in a register pipeline; the concentrations go to a three-row LDS ring.  One row behind,
// stage 2 forms the colour gradients, pair normals and the stress T (three-row LDS ring);
// two rows behind, stage 3 takes the divergence of T and finishes collision and
// recolouring for the output row.  Every stored value is read from HBM once per step (plus
// a 3-column and 4-row halo that other workgroups also read) and written once; densities,
// gradients and stress never leave the chip.
#pragma once

#include "lbm3_internal.h"
#include "lbm3_rounding.h"

namespace tcg {
namespace {

constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// D2Q9 weights, chosen so that the nine sum to exactly 1: otherwise every collision scales
// the mass by the sum (the equilibrium's zeroth moment is rho times it).  In FP64 the rest
// weight is 1 - 4 w_1 - 4 w_5, the double one ulp above the nearest to 4/9 (the nearest
// doubles sum to 1 - 5.55e-17).  In FP32 the nearest floats sum to 1 + 7.45e-9, which
// drifted the mass by 1.5e-5 over 2000 steps at tau = 1; there w_5 is the float one ulp
// below the nearest to 1/36 (0x1.c71c70p-6), and 4/9 and 1/9 are the nearest floats.
template <typename C>
__device__ __forceinline__ constexpr C wgt(int i)
{
    if constexpr (sizeof(C) == 8)
        return i == 0 ? 1.0 - 4.0 * (1.0 / 9.0) - 4.0 * (1.0 / 36.0)
                      : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    else
        return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(0x1.c71c70p-6));
}

__device__ __forceinline__ int wrapi(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Successive row indices modulo n, the same in every lane: wrapped once at the start, then
// advanced by one per row on the scalar unit.  (Integer division has no scalar instruction:
// a % n per row would move every row address of the march into vector registers.)
struct RowCursor {
    int r, n;
    __device__ RowCursor(int a, int n_) : r(__builtin_amdgcn_readfirstlane(wrapi(a, n_))), n(n_) {}
    // the current row, then advance
    __device__ int next()
    {
        const int c = r;
        r = r + 1 == n ? 0 : r + 1;
        return c;
    }
};

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
// Stores of the new state are non-temporal: nothing reads them again within the step, and
// keeping them out of the caches leaves the caches to the halo rows and columns that
// neighbouring workgroups re-read (measured: +1% at 512 threads, +19% at 256, FP64).
template <typename T>
__device__ __forceinline__ void st_at(T* base, unsigned byte_off, T v)
{
    typedef __attribute__((address_space(1))) char gchar;
    typedef __attribute__((address_space(1))) T gT;
    gchar* b = (gchar*)uniform_u64(reinterpret_cast<uint64_t>(base));
    __builtin_nontemporal_store(v, (gT*)(b + byte_off));
}

// The plane stride as a value the optimiser must take afresh at each row: left alone, it
// hoists the 18 or 27 plane offsets of a row out of the march loop and keeps them all live
// in scalar registers, which then spill to vector lanes (FP32 storage: 91 spilled scalars,
// about 190 lane moves per row).  Recomputed per row they cost a few scalar multiplies.
__device__ __forceinline__ int64_t fresh_stride(int64_t s)
{
    asm volatile("" : "+s"(s));
    return s;
}

// Isotropic difference of Eq. (12), 3 sum_i w_i phi(x + e_i) e_i, written as weighted
// differences of opposite neighbours with the factor 3 taken into the weights (3 w = 1/3 on
// the axes, 1/12 on the diagonals).  The grouping keeps exact zeros for data that are
// mirror-symmetric about the node, also when the compiler fuses multiply-adds.
template <typename C>
__device__ __forceinline__ C ddx(C e, C w, C ne, C nw, C se, C sw)
{
    return C(1.0 / 3.0) * (e - w) + C(1.0 / 12.0) * ((ne - sw) + (se - nw));
}
template <typename C>
__device__ __forceinline__ C ddy(C n, C s, C ne, C nw, C se, C sw)
{
    return C(1.0 / 3.0) * (n - s) + C(1.0 / 12.0) * ((ne - sw) + (nw - se));
}

// V . e_i for the nine lattice directions, written out (no multiplications by 0 or 1).
template <typename C>
__device__ __forceinline__ C dot_e(C vx, C vy, int i)
{
    switch (i) {
        case 1: return vx;
        case 2: return vy;
        case 3: return -vx;
        case 4: return -vy;
        case 5: return vx + vy;
        case 6: return vy - vx;
        case 7: return -(vx + vy);
        case 8: return vx - vy;
        default: return C(0);
    }
}

// One recoloured population of Eq. (13) from the factored node state: c_k f_dag_i +
// w_i V_k . e_i, as one fused multiply-add.  The F27 store and the FAC pull both call this.
template <typename C>
__device__ __forceinline__ C recon(C ck, C fdi, C vx, C vy, int i)
{
    // the rest population's product is rounded on its own, never fused into a later sum, so
    // a value rebuilt in registers equals the same value stored and loaded back
#pragma clang fp contract(off)
    if (i == 0) return ck * fdi;
    return fma(ck, fdi, wgt<C>(i) * dot_e<C>(vx, vy, i));
}

// The third fluid's recolouring vector component from the other two (they sum to zero).
template <typename C>
__device__ __forceinline__ C fac_v2(C v0, C v1)
{
    return -(v0 + v1);
}

// Densities from the 27 pulled populations v[k*9 + i], summed in a fixed order that groups
// the directions by the source row they come from (e_y = +1, 0, -1), so that the F27 pull
// and the row-by-row FAC pull add the same values in the same order.
template <typename C>
__device__ __forceinline__ C group_sum(C a, C b, C c)
{
    return (a + b) + c;
}

// 1/x for a positive normal x (densities, relaxation-time denominators): the hardware
// reciprocal estimate refined by Newton steps (two in FP64, one in FP32) to within about an
// ulp, in place of the IEEE division sequence.
template <typename C>
__device__ __forceinline__ C recip(C x)
{
    if constexpr (sizeof(C) == 8) {
        double y = __builtin_amdgcn_rcp(x);
        double e = fma(-x, y, 1.0);
        y = fma(y, e, y);
        e = fma(-x, y, 1.0);
        return fma(y, e, y);
    } else {
        const float y = __builtin_amdgcn_rcpf(x);
        return fmaf(y, fmaf(-x, y, 1.0f), y);
    }
}

// 1/sqrt(s) for a positive normal s, the same way (Newton on y = s^(-1/2)).
template <typename C>
__device__ __forceinline__ C rsqrt_nr(C s)
{
    if constexpr (sizeof(C) == 8) {
        double y = __builtin_amdgcn_rsq(s);
        double h = 0.5 * y;
        double r = fma(-s * y, h, 0.5);
        y = fma(y, r, y);
        h = 0.5 * y;
        r = fma(-s * y, h, 0.5);
        return fma(y, r, y);
    } else {
        const float y = __builtin_amdgcn_rsqf(s);
        const float h = 0.5f * y;
        return fmaf(y, fmaf(-s * y, h, 0.5f), y);
    }
}

// Densities rho_k and totals f_i of a node from its 27 pulled populations v(9k + i), added
// in a fixed order that groups the directions by source row (e_y = +1, 0, -1); every march
// that pulls the 27-population format uses it, so all of them round alike.
template <typename C, typename Get>
__device__ __forceinline__ void densities_f27(Get v, C (&r0)[3], C (&f0)[9])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const C P = group_sum<C>(v(k * 9 + 2), v(k * 9 + 5), v(k * 9 + 6));
        const C Z = group_sum<C>(v(k * 9 + 0), v(k * 9 + 1), v(k * 9 + 3));
        const C M = group_sum<C>(v(k * 9 + 4), v(k * 9 + 7), v(k * 9 + 8));
        r0[k] = (P + Z) + M;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) f0[i] = (v(i) + v(9 + i)) + v(18 + i);
}

template <typename C>
struct StepConsts {
    C sig[3], bg[3], beta0, ct_coef, inv_nu[3], cfac[3], guard2;  // bg = beta0 g_kl
    __device__ explicit StepConsts(const KParams& kp)
    {
        for (int p = 0; p < 3; ++p) {
            sig[p] = C(kp.sigma[p]);
            bg[p] = C(kp.beta0 * kp.g[p]);
            inv_nu[p] = C(kp.inv_nu[p]);
            cfac[p] = C(kp.cfac[p]);
        }
        beta0 = C(kp.beta0);
        ct_coef = C(kp.ct_coef);
        guard2 = C(kp.guard) * C(kp.guard);
    }
};

// Collision (Eqs. 1-3, 8-11) and the recolouring factors (Eqs. 13, 19, 20, or a
// comparison law of Eqs. 15-17 through g_kl and ct_coef) at one node,
// given the totals f[9], densities rk[3], pair normals n[6] (pairs rg, rb, gb) and the
// force.  Returns f_dag, c_k, V_k (V[2k], V[2k+1]) and u, rho u for observables.
//
// With PT (the perturbation operator of Eqs. 4-5 instead of the force), F = 0 and T holds
// the node's own stress T = sum_pairs sigma C (|G|^2 I - G G^T)/|G| (row order xx, xy, yy).
// Eq. (5) summed over the ordered pairs is, with A_kl = 9 sigma_kl / (2 tau) and
// M = sum_pairs sigma C |G| n n^T = tr(T) I - T (two dimensions),
//   Phi_i = 9/(2 tau) [w_i e_i . M e_i - tr(T) B_i],
// where e_i . M e_i is T_yy for e = (+-1, 0), T_xx for (0, +-1) and tr(T) - 2 e_x e_y T_xy
// on the diagonals; B_0 = -4/27, B_1-4 = 2/27, B_5-8 = 5/108.
template <typename C, bool PT = false>
__device__ __forceinline__ void collide_recolour(const C (&f)[9], const C (&rk)[3],
                                                 const C (&n)[6], C Fx, C Fy,
                                                 const StepConsts<C>& K, C (&fd)[9], C (&ck)[3],
                                                 C (&V)[6], C& ux, C& uy, C& mxh, C& myh,
                                                 const C* T = nullptr)
{
    const C rho = rk[0] + rk[1] + rk[2];
    const C irho = recip(rho);
    // rho / nu = sum_k rho_k / nu_k ; tau = 3 nu + 1/2, so 1/tau = (rho/nu) / (3 rho + (rho/nu)/2)
    const C rho_over_nu = rk[0] * K.inv_nu[0] + rk[1] * K.inv_nu[1] + rk[2] * K.inv_nu[2];
    const C itau = rho_over_nu * recip(C(3) * rho + C(0.5) * rho_over_nu);
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
    // f_dag_i = (1 - 1/tau) f_i + (1/tau) f_eq_i + Phi_i, with the per-node factors of the
    // three weight classes formed once: (1/tau) w rho and w (1 - 1/(2 tau)).  In terms of
    // e.u and 3 e.F, f_eq_i / (w rho) = (1 - 1.5 u.u) + e.u (3 + 4.5 e.u) and
    // Phi_i / (w (1 - 1/(2 tau))) = (3 e.F - 3 u.F) + (3 e.u)(3 e.F).
    const C omi = C(1) - itau;
    const C c0 = C(1) - C(1.5) * uu;
    const C tuF = C(3) * uF, tFx = C(3) * Fx, tFy = C(3) * Fy;
    const C tr = itau * rho;
    const C W1[3] = {wgt<C>(0) * tr, wgt<C>(1) * tr, wgt<C>(5) * tr};
    const C W2[3] = {wgt<C>(0) * pref, wgt<C>(1) * pref, wgt<C>(5) * pref};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int cls = i == 0 ? 0 : (i < 5 ? 1 : 2);
        const C eu = C(EX[i]) * ux + C(EY[i]) * uy;
        const C teF = C(EX[i]) * tFx + C(EY[i]) * tFy;
        const C P = fma(eu, fma(C(4.5), eu, C(3)), c0);
        const C Q = fma(C(3) * eu, teF, teF - tuF);
        fd[i] = fma(f[i], omi, fma(W1[cls], P, W2[cls] * Q));
    }
    if constexpr (PT) {
        const C a = C(4.5) * itau;
        const C tr = T[0] + T[2];
        const C d0 = tr - C(2) * T[1], d1 = tr + C(2) * T[1];
        const C B0 = C(-4.0 / 27.0), B1 = C(2.0 / 27.0), B5 = C(5.0 / 108.0);
        fd[0] += a * (-(tr * B0));
        fd[1] += a * (wgt<C>(1) * T[2] - tr * B1);
        fd[3] += a * (wgt<C>(3) * T[2] - tr * B1);
        fd[2] += a * (wgt<C>(2) * T[0] - tr * B1);
        fd[4] += a * (wgt<C>(4) * T[0] - tr * B1);
        fd[5] += a * (wgt<C>(5) * d0 - tr * B5);
        fd[7] += a * (wgt<C>(7) * d0 - tr * B5);
        fd[6] += a * (wgt<C>(6) * d1 - tr * B5);
        fd[8] += a * (wgt<C>(8) * d1 - tr * B5);
    }
    // C_t and beta_kl of Eq. (19) (or the law's own s and g_kl); a_p = beta_p rho_k rho_l / rho
    C ct = K.ct_coef * rk[0] * rk[1] * rk[2] * (irho * irho * irho);
    ct = ct < C(1) ? ct : C(1);
    // beta_p = beta0 (1 + s g_p) = beta0 + s (beta0 g_p)
    const C a0 = fma(ct, K.bg[0], K.beta0) * (rk[0] * rk[1]) * irho;
    const C a1 = fma(ct, K.bg[1], K.beta0) * (rk[0] * rk[2]) * irho;
    const C a2 = fma(ct, K.bg[2], K.beta0) * (rk[1] * rk[2]) * irho;
    // V_k = sum_{l != k} a_kl n_kl with n_lk = -n_kl; the three sum to zero, and V_2 is taken
    // as -(V_0 + V_1) here and wherever a factored state is expanded (fac_v2), so that the
    // factored state needs only V_0 and V_1 and every path rounds alike
    V[0] = a0 * n[0] + a1 * n[2];
    V[1] = a0 * n[1] + a1 * n[3];
    V[2] = a2 * n[4] - a0 * n[0];
    V[3] = a2 * n[5] - a0 * n[1];
    V[4] = fac_v2<C>(V[0], V[2]);
    V[5] = fac_v2<C>(V[1], V[3]);
#pragma unroll
    for (int k = 0; k < 3; ++k) ck[k] = rk[k] * irho;
}

// The pulls of one source row s to rows s+1, s and s-1 (FAC input), in the fixed group order:
// f_dag(i) gives the f_dag_i pulled by this lane for direction i; X holds the c_k, V_k of the
// source row by lane (fields 0-2 c_k, 3-8 V_k), read at lane t - e_x,i.  D0 = partial sums of
// row s (directions with e_y = +1 and 0 received), D1 = those of row s + 1 (e_y = +1
// received); direction groups by e_y: +1 {2, 5, 6}, 0 {0, 1, 3}, -1 {4, 7, 8}.  Completes row
// s - 1 into r0, f0.  With PULL_ONCE the nine fields of the three source lanes t - 1, t, t + 1
// are read from LDS once (27 reads; each group pulls one direction from each of those lanes,
// so reading per direction reads every field three times): measured +7% for the FP64
// two-step pass, +11% for FP32, +13% for the FP64 step at 256^2, -3% for the FP64 one-step
// kernel at 4096^2.  (The scheduling barriers keep the arithmetic of one group from being
// interleaved with the next, which would hold the pulled values of all groups in registers
// at once.)
template <typename C, int NT, bool PULL_ONCE = true, typename FD>
__device__ __forceinline__ void pull_row(FD f_dag, const C (*X)[NT], int t, C (&d0r)[3], C (&d0f)[6],
                                         C (&d1r)[3], C (&d1f)[3], C (&r0)[3], C (&f0)[9])
{
    // by e_x + 1: fields of lane t + 1 (e_x = -1), t (0), t - 1 (+1)
    C xs[3][9];
    if constexpr (PULL_ONCE) {
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int q = 0; q < 9; ++q) xs[e][q] = X[q][t + 1 - e];
    }
    auto pull = [&](int i, C (&fk)[3]) {
        const C fdi = f_dag(i);
        if constexpr (PULL_ONCE) {
            const C* xl = xs[EX[i] + 1];
#pragma unroll
            for (int k = 0; k < 3; ++k) fk[k] = recon<C>(xl[k], fdi, xl[3 + 2 * k], xl[4 + 2 * k], i);
        } else {
            const int l = t - EX[i];
#pragma unroll
            for (int k = 0; k < 3; ++k) fk[k] = recon<C>(X[k][l], fdi, X[3 + 2 * k][l], X[4 + 2 * k][l], i);
        }
    };
    auto group = [&](int a, int b, int c, C (&g)[3], C& ta, C& tb, C& tc) {
        C fa[3], fb[3], fc[3];
        pull(a, fa);
        pull(b, fb);
        pull(c, fc);
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] = group_sum<C>(fa[k], fb[k], fc[k]);
        ta = (fa[0] + fa[1]) + fa[2];
        tb = (fb[0] + fb[1]) + fb[2];
        tc = (fc[0] + fc[1]) + fc[2];
    };
    C g[3];
    // e_y = -1: completes row s - 1 as (P + Z) + M
    group(4, 7, 8, g, f0[4], f0[7], f0[8]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) r0[k] = d0r[k] + g[k];
    f0[2] = d0f[0];
    f0[5] = d0f[1];
    f0[6] = d0f[2];
    f0[0] = d0f[3];
    f0[1] = d0f[4];
    f0[3] = d0f[5];
    // e_y = 0: row s is P (from s - 1) + Z
    group(0, 1, 3, g, d0f[3], d0f[4], d0f[5]);
#pragma unroll
    for (int k = 0; k < 3; ++k) d0r[k] = d1r[k] + g[k];
    d0f[0] = d1f[0];
    d0f[1] = d1f[1];
    d0f[2] = d1f[2];
    __builtin_amdgcn_sched_barrier(0);
    // e_y = +1: row s + 1 starts with P
    group(2, 5, 6, d1r, d1f[0], d1f[1], d1f[2]);
}

// Stage 2 at lane t: colour gradients of the middle ring row (slot s1; s0 above, s2 below),
// pair normals n[6] and the stress (Txx, Txy, Tyy) from the densities rk of that row.
// on_gradients(gx, gy) sees the gradients before the pair loop (the adjoint's tape).
struct NoGradientHook {
    template <typename A>
    __device__ void operator()(const A&, const A&) const {}
};
template <typename C, int NT, typename Hook = NoGradientHook>
__device__ __forceinline__ void stress_at_lane(const C (*cring)[3][NT], int s0, int s1, int s2, int t,
                                               const C (&rk)[3], const StepConsts<C>& K, C (&n)[6],
                                               C& Txx, C& Txy, C& Tyy, Hook on_gradients = Hook())
{
    C gx[3], gy[3];
    C cc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const C* N = cring[s0][k];
        const C* M = cring[s1][k];
        const C* S_ = cring[s2][k];
        gx[k] = ddx<C>(M[t + 1], M[t - 1], N[t + 1], N[t - 1], S_[t + 1], S_[t - 1]);
        gy[k] = ddy<C>(N[t], S_[t], N[t + 1], N[t - 1], S_[t + 1], S_[t - 1]);
        cc[k] = M[t];
    }
    on_gradients(gx, gy);
    Txx = C(0);
    Txy = C(0);
    Tyy = C(0);
    constexpr int PK[3] = {0, 0, 1}, PL[3] = {1, 2, 2};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int k = PK[p], l = PL[p];
        C Gx, Gy, g2;
        {
            // The two products of G nearly cancel where a fluid is present only as a trace;
            // unfused, their rounding matches the plain IEEE evaluation.
#pragma clang fp contract(off)
            Gx = cc[l] * gx[k] - cc[k] * gx[l];
            Gy = cc[l] * gy[k] - cc[k] * gy[l];
            g2 = Gx * Gx + Gy * Gy;
        }
        // |G| > guard, and 1/|G|
        if (g2 > K.guard2) {
            const C inv = rsqrt_nr(g2);
            n[2 * p] = Gx * inv;
            n[2 * p + 1] = Gy * inv;
            C cf = K.cfac[p] * (rk[k] * rk[l]);
            cf = cf < C(1) ? cf : C(1);
            const C coef = K.sig[p] * cf * inv;
            Txx += coef * (Gy * Gy);
            Txy -= coef * (Gx * Gy);
            Tyy += coef * (Gx * Gx);
        }
    }
}

// Stage 3's force at lane t: F = div T over the stress ring (s1 above, s2 middle, s0 below).
template <typename C, int NT>
__device__ __forceinline__ void force_at_lane(const C (*tring)[3][NT], int s0, int s1, int s2, int t,
                                              C& Fx, C& Fy)
{
    C d[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const C* N = tring[s1][a];  // row above
        const C* M = tring[s2][a];  // middle row
        const C* S_ = tring[s0][a]; // row below
        d[a][0] = ddx<C>(M[t + 1], M[t - 1], N[t + 1], N[t - 1], S_[t + 1], S_[t - 1]);
        d[a][1] = ddy<C>(N[t], S_[t], N[t + 1], N[t - 1], S_[t + 1], S_[t - 1]);
    }
    Fx = d[0][0] + d[1][1];  // d_x T_xx + d_y T_yx
    Fy = d[1][0] + d[2][1];  // d_x T_xy + d_y T_yy
}

// Stage 3's input to the collision at lane t: the force (force_at_lane), or with PT no force
// and the lane's own stress from the middle ring row, all that the perturbation operator
// of Eqs. (4)-(5) needs.
template <typename C, int NT, bool PT>
__device__ __forceinline__ void force_or_stress(const C (*tring)[3][NT], int s0, int s1, int s2, int t,
                                                C& Fx, C& Fy, C (&Tn)[3])
{
    if constexpr (PT) {
        Fx = C(0);
        Fy = C(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) Tn[a] = tring[s2][a][t];
    } else {
        force_at_lane<C, NT>(tring, s0, s1, s2, t, Fx, Fy);
    }
}

// The y-marching body shared by the stepping and observing kernels.  The workgroup owns
// output columns [x0, x0 + cols) (cols <= NT - 6) and output rows [y0, y0 + rows).  Lane t
// sits on column x0 - 3 + t; lanes 1..cols+4 form densities, 2..cols+3 gradients and
// stress, 3..cols+2 outputs (FAC input: lanes 0..cols+5 also load their column's c_k, V_k
// for the neighbours).  Iteration j completes the densities of row y0 - 2 + j (stage 1),
// the stress of the row below (stage 2) and the output row y0 - 4 + j (stage 3).
// Loop-carried per-thread state: the next input prefetched one iteration ahead (so that
// the loads are in flight while stages 2 and 3 compute); fA, rA = totals and densities of
// the row below, fB, rB two rows below; nB = pair normals two rows below.  With FAC input,
// also the partial totals and densities of the two rows above (they collect the pulls of
// each source row as it arrives).  LDS rings are indexed by row mod 3.
template <typename S, typename C, int NT, bool OBS, Fmt IN, Fmt OUT, bool TAPE, bool PT = false>
__device__ __forceinline__ void march(const S* __restrict__ fin, S* __restrict__ fout,
                                      const KParams& kp, int x0, int y0, int rows, int cols,
                                      C (*cring)[3][NT], C (*tring)[3][NT], C (*xb)[9][NT],
                                      double (&acc)[kObsFields], double* __restrict__ rho_out,
                                      uint32_t salt)
{
    const int nx = kp.nx, ny = kp.ny;
    const int64_t plane = kp.plane;
    const int t = threadIdx.x;
    const int xr = x0 - 3 + t;
    const int x = wrapi(xr, nx);
    // source column for e_x = -1, 0, +1 as byte offsets from a uniform row pointer
    const unsigned scol[3] = {(unsigned)wrapi(x + 1, nx) * (unsigned)sizeof(S),
                              (unsigned)x * (unsigned)sizeof(S),
                              (unsigned)wrapi(x - 1, nx) * (unsigned)sizeof(S)};
    const unsigned xoff = (unsigned)x * (unsigned)sizeof(S);
    const bool in0 = t <= cols + 5;
    const bool in1 = (t >= 1) && (t <= cols + 4);
    const bool in2 = (t >= 2) && (t <= cols + 3);
    const bool in3 = (t >= 3) && (t <= cols + 2);
    const StepConsts<C> K(kp);
    const int J = rows + 4;

    // ---- input: F27 pulls all 27 populations of a row directly
    constexpr int NV = IN == Fmt::F27 ? 27 : kFacPlanes;
    auto load_f27 = [&](int r, C (&v)[NV]) {
        const int64_t pitch = kp.pitch;
        const int64_t srow[3] = {(int64_t)(r + 1 == ny ? 0 : r + 1) * pitch, (int64_t)r * pitch,
                                 (int64_t)(r == 0 ? ny - 1 : r - 1) * pitch};
        const int64_t pl = fresh_stride(plane);
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 9; ++i)
                v[k * 9 + i] = C(ld_at(fin + ((int64_t)(k * 9 + i) * pl + srow[EY[i] + 1]),
                                       scol[EX[i] + 1]));
    };
    // ---- input: FAC loads source row s (wrapped): v[0..8] = f_dag_i(x - e_x,i, s) (pulled
    // along x), v[9..15] = c_k, V_0, V_1 of the lane's own column
    auto load_fac = [&](int s, C (&v)[NV]) {
        const int64_t rowo = (int64_t)s * kp.fpitch;
        const int64_t pl = fresh_stride(plane);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            v[i] = C(ld_at(fin + ((int64_t)i * pl + rowo), scol[EX[i] + 1]));
#pragma unroll
        for (int q = 9; q < NV; ++q) v[q] = C(ld_at(fin + ((int64_t)q * pl + rowo), xoff));
    };
    // FAC partial sums of the rows above (see pull_row)
    C d0r[3], d0f[6], d1r[3], d1f[3];  // d0f: f_2, f_5, f_6, f_0, f_1, f_3; d1f: f_2, f_5, f_6
    // FAC: publish the c_k, V_k of this lane's column of a source row (v[9..15], and V_2) to
    // the neighbouring lanes, in exchange slot `slot` (two slots, used by alternate rows); a
    // barrier separates this from consume_fac's reads.
    auto publish = [&](const C (&v)[NV], int slot) {
        if constexpr (IN == Fmt::FAC) {
            if (in0) {
#pragma unroll
                for (int q = 0; q < 7; ++q) xb[slot][q][t] = v[9 + q];
                xb[slot][7][t] = fac_v2<C>(v[12], v[14]);
                xb[slot][8][t] = fac_v2<C>(v[13], v[15]);
            }
        }
    };
    // FAC: the pulls of source row s (f_dag in v[0..8], c_k and V_k in exchange slot `slot`)
    auto consume_fac = [&](const C (&v)[NV], int slot, C (&r0)[3], C (&f0)[9]) {
        if (!in1) return;
        pull_row<C, NT>([&](int i) { return v[i]; }, xb[slot], t, d0r, d0f, d1r, d1f, r0, f0);
    };
    // F27: densities and totals of a row from its 27 pulled populations, same order.
    auto consume_f27 = [&](const C (&v)[NV], C (&r0)[3], C (&f0)[9]) {
        densities_f27<C>([&](int q) { return v[q]; }, r0, f0);
    };

    C fA[9], fB[9], rA[3], rB[3], nB[6], vn[NV];
#pragma unroll
    for (int i = 0; i < 9; ++i) fA[i] = fB[i] = C(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) rA[k] = rB[k] = C(1);
#pragma unroll
    for (int q = 0; q < 6; ++q) nB[q] = C(0);
#pragma unroll
    for (int q = 0; q < NV; ++q) vn[q] = C(1);
#pragma unroll
    for (int k = 0; k < 3; ++k) d0r[k] = d1r[k] = C(0);
#pragma unroll
    for (int q = 0; q < 6; ++q) d0f[q] = C(0);
#pragma unroll
    for (int q = 0; q < 3; ++q) d1f[q] = C(0);

    // rows loaded in order: F27 the middle rows y0 - 2, y0 - 1, ...; FAC the source rows
    // y0 - 3, y0 - 2, ...
    RowCursor src(IN == Fmt::F27 ? y0 - 2 : y0 - 3, ny);
    if constexpr (IN == Fmt::F27) {
        const int r = src.next();
        if (in1) load_f27(r, vn);
    } else {
        // pre-roll: source rows y0 - 3 and y0 - 2 start the partial sums of row y0 - 2, and
        // source row y0 - 1 is published for the first iteration (slots alternate by row)
        {
            const int r = src.next();
            if (in0) load_fac(r, vn);
        }
#pragma unroll 1
        for (int p = 0; p < 2; ++p) {
            C v[NV], r_[3], f_[9];
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q] = vn[q];
            publish(v, p);
            const int r = src.next();
            if (in0) load_fac(r, vn);
            __syncthreads();
            consume_fac(v, p, r_, f_);
        }
        // slot 0 was last read before the barrier above (row y0 - 3); slot 1 (row y0 - 2) is
        // next written after the first iteration's first barrier
        publish(vn, 0);
        __syncthreads();
    }

#pragma unroll 1
    for (int j = 0; j < J; ++j) {
        const int s0 = j % 3;        // slot of row j
        const int s1 = (j + 2) % 3;  // slot of row j-1
        const int s2 = (j + 1) % 3;  // slot of row j-2 (and j-3 + 3)
        // ---- stage 1: totals, densities, concentrations of row j; prefetch the next input
        C f0[9], r0[3];
        {
#pragma unroll
            for (int i = 0; i < 9; ++i) f0[i] = C(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) r0[k] = C(1);
            C v[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q] = vn[q];
            const int r = src.next();
            if constexpr (IN == Fmt::F27) {
                if (in1 && j + 1 < J) load_f27(r, vn);
                consume_f27(v, r0, f0);
            } else {
                // source row y0 - 1 + j was published in slot j % 2 before the last barrier;
                // r = row y0 + j
                if (in0 && j + 1 < J) load_fac(r, vn);
                consume_fac(v, j & 1, r0, f0);
            }
            const C irho = recip((r0[0] + r0[1]) + r0[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k) cring[s0][k][t] = r0[k] * irho;
            if constexpr (TAPE) {
                // the pulled densities and totals of the tile's own nodes of this row
                const int yd = y0 - 2 + j;
                if (in3 && yd >= y0 && yd < y0 + rows) {
                    const int64_t N = (int64_t)nx * ny, o = (int64_t)yd * nx + x;
#pragma unroll
                    for (int k = 0; k < 3; ++k) rho_out[k * N + o] = double(r0[k]);
#pragma unroll
                    for (int i = 0; i < 9; ++i) rho_out[(3 + i) * N + o] = double(f0[i]);
                }
            }
        }
        __syncthreads();
        // ---- stage 2: gradients, normals and stress of row j-1 (densities rA)
        C nA[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
        if (j >= 2 && in2) {
            C Txx, Txy, Tyy;
            if constexpr (TAPE) {
                // and their concentration gradients, one row later
                const int yd = y0 - 3 + j;
                const bool own = in3 && yd >= y0 && yd < y0 + rows;
                const int64_t N = (int64_t)nx * ny, o = (int64_t)yd * nx + x;
                stress_at_lane<C, NT>(cring, s0, s1, s2, t, rA, K, nA, Txx, Txy, Tyy,
                                      [&](const C (&gx)[3], const C (&gy)[3]) {
                                          if (own) {
#pragma unroll
                                              for (int k = 0; k < 3; ++k) {
                                                  rho_out[(12 + 2 * k) * N + o] = double(gx[k]);
                                                  rho_out[(13 + 2 * k) * N + o] = double(gy[k]);
                                              }
                                          }
                                      });
            } else {
                stress_at_lane<C, NT>(cring, s0, s1, s2, t, rA, K, nA, Txx, Txy, Tyy);
            }
            tring[s1][0][t] = Txx;
            tring[s1][1][t] = Txy;
            tring[s1][2][t] = Tyy;
        }
        // the next source row (prefetched at the top of this iteration) goes to the other
        // exchange slot, last read before the previous barrier
        if constexpr (IN == Fmt::FAC) {
            if (j + 1 < J) publish(vn, (j + 1) & 1);
        }
        __syncthreads();
        // ---- stage 3: force, collision, recolouring of row j-2 (fB, rB, nB)
        if (j >= 4 && in3) {
            const int yo = y0 + j - 4;
            C Fx, Fy, Tn[3];
            force_or_stress<C, NT, PT>(tring, s0, s1, s2, t, Fx, Fy, Tn);
            if constexpr (TAPE) {
                const int64_t N = (int64_t)nx * ny, o = (int64_t)yo * nx + x;
                rho_out[18 * N + o] = double(Fx);
                rho_out[19 * N + o] = double(Fy);
            }
            C fd[9], ck[3], V[6], ux, uy, mxh, myh;
            collide_recolour<C, PT>(fB, rB, nB, Fx, Fy, K, fd, ck, V, ux, uy, mxh, myh, Tn);
            if constexpr (!OBS) {
                static_assert(OUT == Fmt::FAC, "steps store the factored format");
                NodeBits bits(((uint32_t)yo * (uint32_t)nx + (uint32_t)x) * 27u ^ salt);
                const int64_t pl = fresh_stride(plane);
                const int64_t orow = (int64_t)yo * kp.fpitch;
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    st_at(fout + ((int64_t)i * pl + orow), xoff, to_storage<S, C>(fd[i], bits));
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    st_at(fout + ((int64_t)(9 + k) * pl + orow), xoff, to_storage<S, C>(ck[k], bits));
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    st_at(fout + ((int64_t)(12 + q) * pl + orow), xoff, to_storage<S, C>(V[q], bits));
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
                                    isfinite(double(myh)) && isfinite(uu);
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

// Two fused steps per pass (factored state in and out; FP64 arithmetic, FP64 or FP32
// storage), each step on its own waves of the workgroup.  Step A (lanes 0..NT-1 of the
// workgroup) pulls its source rows from global memory as march() does; the rows it recolours
// never leave the chip: it writes them (the 16 stored values and V_2, rounded as a store
// would round them) to an LDS exchange row xB, from which step B (lanes NT..2NT-1) pulls
// them; only B's rows are stored.  HBM traffic per step is half that of march(), and the
// arithmetic is march()'s, so the result equals two single steps bit for bit.  Each wave
// holds one step's registers, so two waves fit on a SIMD where one thread carrying both
// steps would not.
//
// Lane t of either step sits on column x0 - 6 + t.  A forms densities on lanes 1..cols+10
// and recolours lanes 3..cols+8 (B's source columns); B forms densities on lanes 4..cols+7
// and outputs lanes 6..cols+5, so cols <= NT - 12.  Every iteration has three phases, each
// closed by a barrier that both steps' waves reach (the same number of times: three per
// pre-roll and three per iteration of a loop of the same length).  Both steps run the same
// stage in the same phase, so the heavy stages meet at the same barrier:
//   phase 0: densities (stage 1; B pulls the row A recoloured in the previous iteration)
//   phase 1: stress (stage 2; B stores the f_dag_i of its previous output row)
//   phase 2: force, collision and recolouring (stage 3; A into xB, B's c_k, V_k to HBM)
// A's global loads and B's stores are placed so that the three phases of the two steps
// take about as long as each other.
// Iteration j: A consumes source row y0 - 4 + j and recolours row y0 - 7 + j into xB; B
// pulls that row in iteration j + 1 and outputs row y0 - 11 + j.
template <typename C, int NT>
struct alignas(16) PairLds {
    C cA[3][3][NT];  // A: concentration ring (by row mod 3)
    C tA[3][3][NT];  // A: stress ring
    C xA[2][9][NT];  // A: c_k, V_k of the source row, double-buffered
    C cB[3][3][NT];
    C tB[3][3][NT];
    C xB[18][NT];    // A's recoloured row: f_dag (0-8), c_k (9-11), V_k (12-17)
};

template <typename S, typename C, int NT, bool PT = false>
__device__ __forceinline__ void pair_step_a(const S* __restrict__ fin, const KParams& kp, int x0, int y0,
                                            int rows, int cols, PairLds<C, NT>& L, int t, uint32_t salt)
{
    const int nx = kp.nx, ny = kp.ny;
    const int64_t plane = kp.plane;
    const int x = wrapi(x0 - 6 + t, nx);
    const unsigned scol[3] = {(unsigned)wrapi(x + 1, nx) * (unsigned)sizeof(S),
                              (unsigned)x * (unsigned)sizeof(S),
                              (unsigned)wrapi(x - 1, nx) * (unsigned)sizeof(S)};
    const unsigned xoff = (unsigned)x * (unsigned)sizeof(S);
    const bool a0 = t <= cols + 11;
    const bool a1 = (t >= 1) && (t <= cols + 10);
    const bool a2 = (t >= 2) && (t <= cols + 9);
    const bool a3 = (t >= 3) && (t <= cols + 8);
    const StepConsts<C> K(kp);
    const int JA = rows + 10;
    const int J = rows + 11;  // one more iteration for B's last row
    // A source row is loaded in two parts: its f_dag_i at this lane's pull columns (pulled by
    // this lane in the next phase 0) and its c_k, V_0, V_1 at this lane's own column (published
    // to the neighbouring lanes in phase 1).  Each part goes into its registers once their
    // previous contents were used, so no copy of a prefetched row is kept (the registers freed
    // hold the 27 exchange fields pull_row reads once): the f_dag_i at the end of phase 0,
    // after the pull, and the c_k, V_k of the row after next at the start of phase 2, after
    // the publish, a whole iteration before they are published.  Loads issued at the start
    // of phase 0 queue behind B's stores of the phase before and hold up A's pull, the
    // longest stage of its iteration (measured: A's phase 0 took 3.6k cycles with the c_k,
    // V_k loads there against B's 2.2k, and B waited that difference at every iteration).
    // The prefetched values stay in the storage type until used.
    constexpr int NC = kFacPlanes - 9;
    auto load_fd = [&](int s, S (&v)[9]) {
        const int64_t rowo = (int64_t)s * kp.fpitch;
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = ld_at(fin + ((int64_t)i * plane + rowo), scol[EX[i] + 1]);
    };
    auto load_cv = [&](int s, S (&v)[NC]) {
        const int64_t rowo = (int64_t)s * kp.fpitch;
#pragma unroll
        for (int q = 0; q < NC; ++q) v[q] = ld_at(fin + ((int64_t)(9 + q) * plane + rowo), xoff);
    };
    auto publish = [&](const S (&v)[NC], int slot) {
        if (a0) {
#pragma unroll
            for (int q = 0; q < 7; ++q) L.xA[slot][q][t] = C(v[q]);
            L.xA[slot][7][t] = fac_v2<C>(C(v[3]), C(v[5]));
            L.xA[slot][8][t] = fac_v2<C>(C(v[4]), C(v[6]));
        }
    };
    C fA[9], fB[9], rA[3], rB[3], nB[6], d0r[3], d0f[6], d1r[3], d1f[3];
    S vf[9], vc[NC];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        fA[i] = fB[i] = C(0);
        vf[i] = S(0);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        rA[k] = rB[k] = C(1);
        d0r[k] = d1r[k] = d1f[k] = C(0);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) nB[q] = d0f[q] = C(0);
#pragma unroll
    for (int q = 0; q < NC; ++q) vc[q] = S(1);
    RowCursor src(y0 - 6, ny);
    {
        const int r = src.next();
        if (a0) {
            load_cv(r, vc);
            load_fd(r, vf);
        }
    }
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
        publish(vc, p);
        const int r = src.next();
        if (a0) load_cv(r, vc);
        __syncthreads();
        C r_[3], f_[9];
        if (a1) pull_row<C, NT>([&](int i) { return C(vf[i]); }, L.xA[p], t, d0r, d0f, d1r, d1f, r_, f_);
        if (a0) load_fd(r, vf);
    }
    publish(vc, 0);
    if (a0) load_cv(src.r, vc);  // for the loop's first publish
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < J; ++j) {
        const bool live = j < JA;
        const int s0 = j % 3, s1 = (j + 2) % 3, s2 = (j + 1) % 3;
        C f0[9], r0[3];
#pragma unroll
        for (int i = 0; i < 9; ++i) f0[i] = C(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) r0[k] = C(1);
        if (live) {
            const int r = src.next();
            const bool more = a0 && j + 1 < JA;
            if (a1) pull_row<C, NT>([&](int i) { return C(vf[i]); }, L.xA[j & 1], t, d0r, d0f, d1r, d1f, r0, f0);
            if (more) load_fd(r, vf);
            const C irho = recip((r0[0] + r0[1]) + r0[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k) L.cA[s0][k][t] = r0[k] * irho;
        }
        __syncthreads();
        C nA[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
        if (live && j >= 2 && a2) {
            C Txx, Txy, Tyy;
            stress_at_lane<C, NT>(L.cA, s0, s1, s2, t, rA, K, nA, Txx, Txy, Tyy);
            L.tA[s1][0][t] = Txx;
            L.tA[s1][1][t] = Txy;
            L.tA[s1][2][t] = Tyy;
        }
        if (j + 1 < JA) publish(vc, (j + 1) & 1);
        __syncthreads();
        // the c_k, V_k of the row src.next() returns in the next iteration
        if (a0 && j + 2 < JA) load_cv(src.r, vc);
        if (live && j >= 4 && a3) {
            C Fx, Fy, fd[9], ck[3], V[6], ux, uy, mxh, myh;
            C Tn[3];
            force_or_stress<C, NT, PT>(L.tA, s0, s1, s2, t, Fx, Fy, Tn);
            collide_recolour<C, PT>(fB, rB, nB, Fx, Fy, K, fd, ck, V, ux, uy, mxh, myh, Tn);
            if constexpr (kRounds<S, C>) {
                // the row as a single step would store it: each value rounded with the key of
                // its node (row y0 - 7 + j, wrapped) and in store order, V_2 formed from the
                // rounded V_0 and V_1 as the next step's pull forms it
                const uint32_t yo = (uint32_t)wrapi(y0 - 7 + j, ny);
                NodeBits bits((yo * (uint32_t)nx + (uint32_t)x) * 27u ^ salt);
#pragma unroll
                for (int i = 0; i < 9; ++i) L.xB[i][t] = C(to_storage<S, C>(fd[i], bits));
#pragma unroll
                for (int k = 0; k < 3; ++k) L.xB[9 + k][t] = C(to_storage<S, C>(ck[k], bits));
                C v4[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    v4[q] = C(to_storage<S, C>(V[q], bits));
                    L.xB[12 + q][t] = v4[q];
                }
                L.xB[16][t] = fac_v2<C>(v4[0], v4[2]);
                L.xB[17][t] = fac_v2<C>(v4[1], v4[3]);
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) L.xB[i][t] = fd[i];
#pragma unroll
                for (int k = 0; k < 3; ++k) L.xB[9 + k][t] = ck[k];
#pragma unroll
                for (int q = 0; q < 6; ++q) L.xB[12 + q][t] = V[q];
            }
        }
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
        __syncthreads();
    }
}

// B's rows are numbered by m: its stage 1 pulls source row y0 - 1 + m (from xB) and
// completes the densities of row y0 - 2 + m (partial sums only for m = -2, -1), its stage 2
// forms the stress of row y0 - 3 + m and its stage 3 outputs row y0 - 4 + m.  Row m runs in
// iteration m + 7, one iteration after A recoloured its source row into xB.
template <typename S, typename C, int NT, bool PT = false>
__device__ __forceinline__ void pair_step_b(S* __restrict__ fout, const KParams& kp, int x0, int y0,
                                            int rows, int cols, PairLds<C, NT>& L, int t, uint32_t salt)
{
    const int nx = kp.nx;
    const int64_t plane = kp.plane;
    const int x = wrapi(x0 - 6 + t, nx);
    const unsigned xoff = (unsigned)x * (unsigned)sizeof(S);
    const bool b1 = (t >= 4) && (t <= cols + 7);
    const bool b2 = (t >= 5) && (t <= cols + 6);
    const bool b3 = (t >= 6) && (t <= cols + 5);
    const StepConsts<C> K(kp);
    const int MB = rows + 3;  // last row index m
    const int J = rows + 11;

    // The f_dag_i of an output row are stored at the end of the next iteration's phase 1, its
    // c_k, V_k at once: B's phase 2 (collision and 16 stores) is the longest phase of the pair
    // and A waits for it at every iteration (measured 3.5k cycles against A's 2.1-2.5k).
    S fdp[9];
    int64_t prow = -1;  // row offset of the f_dag_i held in fdp, or -1
    auto store_fd = [&]() {
        if (prow >= 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i) st_at(fout + ((int64_t)i * plane + prow), xoff, fdp[i]);
            prow = -1;
        }
    };
    C fA[9], fB[9], rA[3], rB[3], nB[6], d0r[3], d0f[6], d1r[3], d1f[3];
#pragma unroll
    for (int i = 0; i < 9; ++i) fA[i] = fB[i] = C(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        rA[k] = rB[k] = C(1);
        d0r[k] = d1r[k] = d1f[k] = C(0);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) nB[q] = d0f[q] = C(0);

    // A's three pre-roll barriers
#pragma unroll 1
    for (int p = 0; p < 3; ++p) __syncthreads();

#pragma unroll 1
    for (int j = 0; j < J; ++j) {
        const int m = j - 7;
        const bool live = m >= -2 && m <= MB;
        const int s0 = (m + 6) % 3, s1 = (m + 8) % 3, s2 = (m + 7) % 3;
        // phase 0: stage 1 of row m from A's row in xB
        C f0[9], r0[3];
#pragma unroll
        for (int i = 0; i < 9; ++i) f0[i] = C(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) r0[k] = C(1);
        if (live) {
            if (b1)
                pull_row<C, NT>([&](int i) { return L.xB[i][t - EX[i]]; }, L.xB + 9, t, d0r, d0f, d1r, d1f,
                                r0, f0);
            if (m >= 0) {
                const C irho = recip((r0[0] + r0[1]) + r0[2]);
#pragma unroll
                for (int k = 0; k < 3; ++k) L.cB[s0][k][t] = r0[k] * irho;
            }
        }
        __syncthreads();
        // phase 1: stage 2
        C nA[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
        if (live && m >= 2 && b2) {
            C Txx, Txy, Tyy;
            stress_at_lane<C, NT>(L.cB, s0, s1, s2, t, rA, K, nA, Txx, Txy, Tyy);
            L.tB[s1][0][t] = Txx;
            L.tB[s1][1][t] = Txy;
            L.tB[s1][2][t] = Tyy;
        }
        store_fd();
        __syncthreads();
        // phase 2: stage 3, then row m enters the pipeline
        if (live && m >= 4 && b3) {
            const int yo = y0 - 4 + m;
            C Fx, Fy, fd[9], ck[3], V[6], ux, uy, mxh, myh;
            C Tn[3];
            force_or_stress<C, NT, PT>(L.tB, s0, s1, s2, t, Fx, Fy, Tn);
            collide_recolour<C, PT>(fB, rB, nB, Fx, Fy, K, fd, ck, V, ux, uy, mxh, myh, Tn);
            const int64_t orow = (int64_t)yo * kp.fpitch;
            NodeBits bits(((uint32_t)yo * (uint32_t)nx + (uint32_t)x) * 27u ^ salt);
            // rounded in store order, the f_dag_i first
#pragma unroll
            for (int i = 0; i < 9; ++i) fdp[i] = to_storage<S, C>(fd[i], bits);
            prow = orow;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                st_at(fout + ((int64_t)(9 + k) * plane + orow), xoff, to_storage<S, C>(ck[k], bits));
#pragma unroll
            for (int q = 0; q < 4; ++q)
                st_at(fout + ((int64_t)(12 + q) * plane + orow), xoff, to_storage<S, C>(V[q], bits));
        }
        if (live && m >= 0) {
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
        __syncthreads();
    }
    store_fd();
}

// The same two-step pass with each thread carrying both steps (used for FP32, whose two
// steps fit one thread's registers at two waves per SIMD; measured 14% faster there than the
// wave-specialised form at 4096^2, while FP64 runs 46% faster wave-specialised).  Lane t sits
// on column x0 - 6 + t.  A forms densities on lanes 1..cols+10 and recolours lanes 3..cols+8 (B's
// source columns); B forms densities on lanes 4..cols+7 and outputs lanes 6..cols+5, so
// cols <= NT - 12.  A runs six rows ahead: iteration j consumes A's source row y0 - 4 + j,
// A recolours row y0 - 7 + j, B consumes that row at once and outputs row y0 - 10 + j.
template <typename C, int NT, bool PT = false>
__device__ __forceinline__ void march2(const C* __restrict__ fin, C* __restrict__ fout,
                                       const KParams& kp, int x0, int y0, int rows, int cols,
                                       C (*cA)[3][NT], C (*tA)[3][NT], C (*xA)[9][NT],
                                       C (*cB)[3][NT], C (*tB)[3][NT], C (*xB)[NT])
{
    const int nx = kp.nx, ny = kp.ny;
    const int64_t plane = kp.plane;
    const int t = threadIdx.x;
    const int x = wrapi(x0 - 6 + t, nx);
    const unsigned scol[3] = {(unsigned)wrapi(x + 1, nx) * (unsigned)sizeof(C),
                              (unsigned)x * (unsigned)sizeof(C),
                              (unsigned)wrapi(x - 1, nx) * (unsigned)sizeof(C)};
    const unsigned xoff = (unsigned)x * (unsigned)sizeof(C);
    const bool a0 = t <= cols + 11;
    const bool a1 = (t >= 1) && (t <= cols + 10);
    const bool a2 = (t >= 2) && (t <= cols + 9);
    const bool a3 = (t >= 3) && (t <= cols + 8);
    const bool b1 = (t >= 4) && (t <= cols + 7);
    const bool b2 = (t >= 5) && (t <= cols + 6);
    const bool b3 = (t >= 6) && (t <= cols + 5);
    const StepConsts<C> K(kp);
    const int JA = rows + 10;

    auto load_fac = [&](int s, C (&v)[kFacPlanes]) {
        const int64_t rowo = (int64_t)s * kp.fpitch;
        const int64_t pl = fresh_stride(plane);
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = ld_at(fin + ((int64_t)i * pl + rowo), scol[EX[i] + 1]);
#pragma unroll
        for (int q = 9; q < kFacPlanes; ++q) v[q] = ld_at(fin + ((int64_t)q * pl + rowo), xoff);
    };
    auto publish_a = [&](const C (&v)[kFacPlanes], int slot) {
        if (a0) {
#pragma unroll
            for (int q = 0; q < 7; ++q) xA[slot][q][t] = v[9 + q];
            xA[slot][7][t] = fac_v2<C>(v[12], v[14]);
            xA[slot][8][t] = fac_v2<C>(v[13], v[15]);
        }
    };

    // A: pipeline, partial sums and the prefetched next source row
    C fA_a[9], fB_a[9], rA_a[3], rB_a[3], nB_a[6], d0r_a[3], d0f_a[6], d1r_a[3], d1f_a[3], vn[kFacPlanes];
    // B: pipeline and partial sums
    C fA_b[9], fB_b[9], rA_b[3], rB_b[3], nB_b[6], d0r_b[3], d0f_b[6], d1r_b[3], d1f_b[3];
#pragma unroll
    for (int i = 0; i < 9; ++i) fA_a[i] = fB_a[i] = fA_b[i] = fB_b[i] = C(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        rA_a[k] = rB_a[k] = rA_b[k] = rB_b[k] = C(1);
        d0r_a[k] = d1r_a[k] = d0r_b[k] = d1r_b[k] = C(0);
        d1f_a[k] = d1f_b[k] = C(0);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) nB_a[q] = nB_b[q] = d0f_a[q] = d0f_b[q] = C(0);
#pragma unroll
    for (int q = 0; q < kFacPlanes; ++q) vn[q] = C(1);

    // A's pre-roll (as march() with first output row y0 - 3): source rows y0 - 6 and y0 - 5,
    // then row y0 - 4 published for the first iteration
    RowCursor src(y0 - 6, ny);  // source rows in load order: y0 - 6, y0 - 5, ...
    {
        const int r = src.next();
        if (a0) load_fac(r, vn);
    }
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
        C v[kFacPlanes], r_[3], f_[9];
#pragma unroll
        for (int q = 0; q < kFacPlanes; ++q) v[q] = vn[q];
        publish_a(v, p);
        const int r = src.next();
        if (a0) load_fac(r, vn);
        __syncthreads();
        if (a1)
            pull_row<C, NT>([&](int i) { return v[i]; }, xA[p], t, d0r_a, d0f_a, d1r_a, d1f_a, r_, f_);
    }
    publish_a(vn, 0);
    __syncthreads();

#pragma unroll 1
    for (int j = 0; j < JA; ++j) {
        const int sa0 = j % 3, sa1 = (j + 2) % 3, sa2 = (j + 1) % 3;
        const int jb = j - 6;
        const int sb0 = (jb + 6) % 3, sb1 = (jb + 8) % 3, sb2 = (jb + 7) % 3;
        // ---- A stage 1: densities of row y0 - 5 + j from source row y0 - 4 + j
        C f0a[9], r0a[3];
        {
#pragma unroll
            for (int i = 0; i < 9; ++i) f0a[i] = C(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) r0a[k] = C(1);
            C v[kFacPlanes];
#pragma unroll
            for (int q = 0; q < kFacPlanes; ++q) v[q] = vn[q];
            const int r = src.next();  // row y0 - 3 + j
            if (a0 && j + 1 < JA) load_fac(r, vn);
            if (a1)
                pull_row<C, NT>([&](int i) { return v[i]; }, xA[j & 1], t, d0r_a, d0f_a, d1r_a, d1f_a,
                                r0a, f0a);
            const C irho = recip((r0a[0] + r0a[1]) + r0a[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k) cA[sa0][k][t] = r0a[k] * irho;
        }
        __syncthreads();
        // ---- A stage 2: stress of row y0 - 6 + j; publish the next source row
        C nA_a[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
        if (j >= 2 && a2) {
            C Txx, Txy, Tyy;
            stress_at_lane<C, NT>(cA, sa0, sa1, sa2, t, rA_a, K, nA_a, Txx, Txy, Tyy);
            tA[sa1][0][t] = Txx;
            tA[sa1][1][t] = Txy;
            tA[sa1][2][t] = Tyy;
        }
        if (j + 1 < JA) publish_a(vn, (j + 1) & 1);
        __syncthreads();
        // ---- A stage 3: recolour row y0 - 7 + j into B's exchange row
        if (j >= 4 && a3) {
            C Fx, Fy, fd[9], ck[3], V[6], ux, uy, mxh, myh;
            C Tn[3];
            force_or_stress<C, NT, PT>(tA, sa0, sa1, sa2, t, Fx, Fy, Tn);
            collide_recolour<C, PT>(fB_a, rB_a, nB_a, Fx, Fy, K, fd, ck, V, ux, uy, mxh, myh, Tn);
#pragma unroll
            for (int i = 0; i < 9; ++i) xB[i][t] = fd[i];
#pragma unroll
            for (int k = 0; k < 3; ++k) xB[9 + k][t] = ck[k];
#pragma unroll
            for (int q = 0; q < 6; ++q) xB[12 + q][t] = V[q];
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            fB_a[i] = fA_a[i];
            fA_a[i] = f0a[i];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            rB_a[k] = rA_a[k];
            rA_a[k] = r0a[k];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) nB_a[q] = nA_a[q];
        __syncthreads();
        // ---- B stage 1: pulls of source row y0 - 7 + j (the pre-roll for j = 4, 5)
        C f0b[9], r0b[3];
#pragma unroll
        for (int i = 0; i < 9; ++i) f0b[i] = C(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) r0b[k] = C(1);
        if (j >= 4 && b1)
            pull_row<C, NT>([&](int i) { return xB[i][t - EX[i]]; }, xB + 9, t, d0r_b, d0f_b, d1r_b, d1f_b,
                            r0b, f0b);
        if (jb >= 0) {
            const C irho = recip((r0b[0] + r0b[1]) + r0b[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k) cB[sb0][k][t] = r0b[k] * irho;
        }
        __syncthreads();
        // ---- B stage 2
        C nA_b[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
        if (jb >= 2 && b2) {
            C Txx, Txy, Tyy;
            stress_at_lane<C, NT>(cB, sb0, sb1, sb2, t, rA_b, K, nA_b, Txx, Txy, Tyy);
            tB[sb1][0][t] = Txx;
            tB[sb1][1][t] = Txy;
            tB[sb1][2][t] = Tyy;
        }
        __syncthreads();
        // ---- B stage 3: recolour and store row y0 - 4 + jb
        if (jb >= 4 && b3) {
            const int yo = y0 - 4 + jb;
            C Fx, Fy, fd[9], ck[3], V[6], ux, uy, mxh, myh;
            C Tn[3];
            force_or_stress<C, NT, PT>(tB, sb0, sb1, sb2, t, Fx, Fy, Tn);
            collide_recolour<C, PT>(fB_b, rB_b, nB_b, Fx, Fy, K, fd, ck, V, ux, uy, mxh, myh, Tn);
            const int64_t orow = (int64_t)yo * kp.fpitch;
            const int64_t pl = fresh_stride(plane);
#pragma unroll
            for (int i = 0; i < 9; ++i) st_at(fout + ((int64_t)i * pl + orow), xoff, fd[i]);
#pragma unroll
            for (int k = 0; k < 3; ++k) st_at(fout + ((int64_t)(9 + k) * pl + orow), xoff, ck[k]);
#pragma unroll
            for (int q = 0; q < 4; ++q) st_at(fout + ((int64_t)(12 + q) * pl + orow), xoff, V[q]);
        }
        if (jb >= 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                fB_b[i] = fA_b[i];
                fA_b[i] = f0b[i];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                rB_b[k] = rA_b[k];
                rA_b[k] = r0b[k];
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) nB_b[q] = nA_b[q];
        }
    }
}

// Combination of two partials of observable field a: sums for the masses, momenta and kinetic
// energy, the maximum for max|u| and the nonfinite flag (a NaN wins).
__device__ __forceinline__ double obs_combine(int a, double x, double y)
{
    if (a == 6 || a == 7) return (y > x || y != y) ? y : x;
    return x + y;
}

// Wavefront reduction of every observables field across the 64 lanes of a wave.
__device__ __forceinline__ void wave_reduce_obs(double (&acc)[kObsFields])
{
#pragma unroll
    for (int a = 0; a < kObsFields; ++a) acc[a] = (a == 6 || a == 7) ? wave_max(acc[a]) : wave_sum(acc[a]);
}

// Workgroup reduction of the observables partials: a wavefront reduction per wave, then the
// first lanes combine the NT/64 wave results (from `red`, LDS of at least kObsFields x NT/64
// doubles) in wave order into out[0 .. kObsFields).  The caller has synchronised the workgroup
// before `red` is reused.
template <int NT>
__device__ void block_reduce_obs(double (&acc)[kObsFields], double (*red)[NT], double* __restrict__ out)
{
    const int t = threadIdx.x;
    wave_reduce_obs(acc);
    if ((t & 63) == 0) {
#pragma unroll
        for (int a = 0; a < kObsFields; ++a) red[a][t >> 6] = acc[a];
    }
    __syncthreads();
    if (t < kObsFields) {
        double v = red[t][0];
        for (int w = 1; w < NT / 64; ++w) v = obs_combine(t, v, red[t][w]);
        out[t] = v;
    }
}

template <typename C, int NT, Fmt IN>
struct ExchangeLds {
    __device__ static C (*get())[9][NT]
    {
        __shared__ C xb[2][9][NT];
        return xb;
    }
};
template <typename C, int NT>
struct ExchangeLds<C, NT, Fmt::F27> {
    __device__ static C (*get())[9][NT] { return nullptr; }
};

// One fused time step over a list of tiles: workgroup b takes tiles[b] of instance
// tiles[b].inst (the plain lattice is a list with one instance).  With OBS the workgroup
// instead accumulates the observables of its output nodes into partials[b] (and their
// densities into rho_out when given).  With TAPE the step also writes, for every node, the
// densities rho_k, totals f_i, concentration gradients and force it pulled and formed, to
// rho_out as [20][ny][nx] (rho_k, f_i, d_x c_k and d_y c_k per fluid, F_x, F_y): the
// forward quantities the adjoint needs.  With filter, a workgroup whose instance's state is not in
// format IN returns at once.  With FP32 storage the stochastic rounding takes its salt from
// step_dev (the device's step counter, read when the launch runs) when given, else `salt`.
template <typename S, typename C, int NT, bool OBS, Fmt IN, Fmt OUT, bool TAPE = false, bool PT = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_tiles(const S* __restrict__ fin, S* __restrict__ fout,
                                              const Instance* __restrict__ inst,
                                              const Tile* __restrict__ tiles, uint32_t salt,
                                              const int64_t* __restrict__ step_dev,
                                              int filter, double* __restrict__ partials,
                                              double* __restrict__ rho_out)
{
    // the two rings in one array, so that the observables reduction can reuse them
    static_assert(sizeof(C) * 18 >= sizeof(double) * kObsFields, "rings too small for the reduction");
    __shared__ alignas(16) C rings[2][3][3][NT];
    C (*cring)[3][NT] = rings[0];
    C (*tring)[3][NT] = rings[1];
    const Tile tl = tiles[blockIdx.x];
    if (filter && inst[tl.inst].fmt != (int32_t)IN) return;
    const KParams kp = inst[tl.inst].kp;
    const int64_t off = inst[tl.inst].offset;
    double acc[kObsFields] = {0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (kRounds<S, C> && !OBS) {
        if (step_dev) salt = step_salt(*step_dev);
    }
    // the key of a stored value depends on (step, node, value) only, so an instance of a batch
    // rounds exactly as the same lattice stepped alone
    march<S, C, NT, OBS, IN, OUT, TAPE, PT>(fin + off, OBS ? nullptr : fout + off, kp, tl.x0, tl.y0, tl.rows,
                                  tl.cols, cring, tring, ExchangeLds<C, NT, IN>::get(), acc, rho_out, salt);
    if constexpr (OBS) {
        __syncthreads();  // the rings are free once every lane has left the march
        block_reduce_obs<NT>(acc, reinterpret_cast<double (*)[NT]>(&rings[0][0][0][0]),
                             partials + (int64_t)blockIdx.x * kObsFields);
    }
}

template <typename S, typename C, int NT, bool OBS, Fmt IN, Fmt OUT, bool TAPE = false, bool PT = false>
hipError_t do_tiles(const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                    int ntiles, uint32_t salt, int filter, double* partials, double* rho_out,
                    hipStream_t st, const int64_t* step_dev = nullptr)
{
    hipLaunchKernelGGL((k_tiles<S, C, NT, OBS, IN, OUT, TAPE, PT>), dim3(ntiles), dim3(NT), 0, st,
                       (const S*)fin, (S*)fout, inst, tiles, salt, step_dev, filter, partials, rho_out);
    return hipGetLastError();
}

template <typename S, typename C, int NT, bool PT>
hipError_t tiles_nt_pt(Fmt in, Fmt out, bool obs, const void* fin, void* fout, const Instance* inst,
                       const Tile* tiles, int ntiles, uint32_t salt, const int64_t* step_dev, int filter,
                       double* partials, double* rho_out, hipStream_t st)
{
    if (obs && in == Fmt::F27)
        return do_tiles<S, C, NT, true, Fmt::F27, Fmt::F27, false, PT>(fin, nullptr, inst, tiles, ntiles, 0u,
                                                                      filter, partials, rho_out, st);
    if (obs && in == Fmt::FAC)
        return do_tiles<S, C, NT, true, Fmt::FAC, Fmt::FAC, false, PT>(fin, nullptr, inst, tiles, ntiles, 0u,
                                                                      filter, partials, rho_out, st);
    if (in == Fmt::FAC && out == Fmt::FAC)
        return do_tiles<S, C, NT, false, Fmt::FAC, Fmt::FAC, false, PT>(fin, fout, inst, tiles, ntiles, salt,
                                                                       filter, nullptr, nullptr, st, step_dev);
    if (in == Fmt::F27 && out == Fmt::FAC)
        return do_tiles<S, C, NT, false, Fmt::F27, Fmt::FAC, false, PT>(fin, fout, inst, tiles, ntiles, salt,
                                                                       filter, nullptr, nullptr, st, step_dev);
    return hipErrorInvalidValue;
}

// pt: the perturbation operator of Eqs. (4)-(5) in place of the force and Guo's term
template <typename S, typename C, int NT>
hipError_t tiles_nt(Fmt in, Fmt out, bool obs, bool pt, const void* fin, void* fout, const Instance* inst,
                    const Tile* tiles, int ntiles, uint32_t salt, const int64_t* step_dev, int filter,
                    double* partials, double* rho_out, hipStream_t st)
{
    if (pt)
        return tiles_nt_pt<S, C, NT, true>(in, out, obs, fin, fout, inst, tiles, ntiles, salt, step_dev, filter,
                                           partials, rho_out, st);
    return tiles_nt_pt<S, C, NT, false>(in, out, obs, fin, fout, inst, tiles, ntiles, salt, step_dev, filter,
                                        partials, rho_out, st);
}

// The FP64 step writing the adjoint's tape (rho_out as [20][ny][nx]), factored output.
template <int NT>
hipError_t tiles_tape_nt(Fmt in, const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                         int ntiles, double* tape, hipStream_t st)
{
    if (in == Fmt::F27)
        return do_tiles<double, double, NT, false, Fmt::F27, Fmt::FAC, true>(
            fin, fout, inst, tiles, ntiles, 0u, 0, nullptr, tape, st);
    return do_tiles<double, double, NT, false, Fmt::FAC, Fmt::FAC, true>(fin, fout, inst, tiles, ntiles,
                                                                        0u, 0, nullptr, tape, st);
}

template <typename S, typename C>
hipError_t tiles_any(Fmt in, Fmt out, bool obs, bool pt, const void* fin, void* fout, const Instance* inst,
                     const Tile* tiles, int ntiles, int threads, uint32_t salt, const int64_t* step_dev,
                     int filter, double* partials, double* rho_out, hipStream_t st)
{
    switch (threads) {
        case 64: return tiles_nt<S, C, 64>(in, out, obs, pt, fin, fout, inst, tiles, ntiles, salt, step_dev, filter, partials, rho_out, st);
        case 128: return tiles_nt<S, C, 128>(in, out, obs, pt, fin, fout, inst, tiles, ntiles, salt, step_dev, filter, partials, rho_out, st);
        case 256: return tiles_nt<S, C, 256>(in, out, obs, pt, fin, fout, inst, tiles, ntiles, salt, step_dev, filter, partials, rho_out, st);
        case 512: return tiles_nt<S, C, 512>(in, out, obs, pt, fin, fout, inst, tiles, ntiles, salt, step_dev, filter, partials, rho_out, st);
        default: return hipErrorInvalidValue;
    }
}

// Two fused steps over a list of tiles; tiles come from a plan with cols <= NT - 12.  The
// workgroup has 2 NT lanes: waves of lanes 0..NT-1 run step A, the others step B (the
// choice is uniform per wave).
// With FP32 storage, salt_a and salt_b salt the two steps' stochastic rounding, or, when
// step_dev is given, those of steps *step_dev and *step_dev + 1, read when the launch runs.
template <typename S, typename C, int NT, bool PT = false>
__global__ __launch_bounds__(2 * NT) __attribute__((amdgpu_waves_per_eu(2))) void k_tiles2w(
    const S* __restrict__ fin, S* __restrict__ fout, const Instance* __restrict__ inst,
    const Tile* __restrict__ tiles, uint32_t salt_a, uint32_t salt_b, const int64_t* __restrict__ step_dev)
{
    static_assert(NT % 64 == 0, "each wave must belong to one step");
    __shared__ PairLds<C, NT> lds;
    const Tile tl = tiles[blockIdx.x];
    const KParams kp = inst[tl.inst].kp;
    const int64_t off = inst[tl.inst].offset;
    if constexpr (kRounds<S, C>) {
        if (step_dev) {
            const int64_t s = *step_dev;
            salt_a = step_salt(s);
            salt_b = step_salt(s + 1);
        }
    }
    const int lane0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x);
    if (lane0 < NT)
        pair_step_a<S, C, NT, PT>(fin + off, kp, tl.x0, tl.y0, tl.rows, tl.cols, lds, (int)threadIdx.x, salt_a);
    else
        pair_step_b<S, C, NT, PT>(fout + off, kp, tl.x0, tl.y0, tl.rows, tl.cols, lds, (int)threadIdx.x - NT,
                                  salt_b);
}

// Two fused steps over a list of tiles, one thread per column carrying both (march2);
// tiles come from a plan with cols <= NT - 12.
template <typename C, int NT, bool PT = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1))) void k_tiles2f(
    const C* __restrict__ fin, C* __restrict__ fout, const Instance* __restrict__ inst,
    const Tile* __restrict__ tiles)
{
    __shared__ alignas(16) C ringsA[2][3][3][NT];
    __shared__ alignas(16) C xA[2][9][NT];
    __shared__ alignas(16) C ringsB[2][3][3][NT];
    __shared__ alignas(16) C xB[18][NT];
    const Tile tl = tiles[blockIdx.x];
    const KParams kp = inst[tl.inst].kp;
    const int64_t off = inst[tl.inst].offset;
    march2<C, NT, PT>(fin + off, fout + off, kp, tl.x0, tl.y0, tl.rows, tl.cols, ringsA[0], ringsA[1], xA,
                  ringsB[0], ringsB[1], xB);
}

// The two-step pass: FP64 arithmetic (FP64 or FP32 storage) wave-specialised (k_tiles2w,
// 2 x threads lanes), FP32 with one thread per column (k_tiles2f, threads lanes); `threads`
// is the tile width basis NT.  pt: the perturbation operator of Eqs. (4)-(5) in place of the
// force and Guo's term.
template <typename S, typename C, int NT, bool PT>
hipError_t pair_launch(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                       uint32_t salt_a, uint32_t salt_b, const int64_t* step_dev, hipStream_t st)
{
    if constexpr (sizeof(C) == 8)
        hipLaunchKernelGGL((k_tiles2w<S, C, NT, PT>), dim3(ntiles), dim3(2 * NT), 0, st, (const S*)fin, (S*)fout,
                           inst, tiles, salt_a, salt_b, step_dev);
    else
        hipLaunchKernelGGL((k_tiles2f<C, NT, PT>), dim3(ntiles), dim3(NT), 0, st, (const C*)fin, (C*)fout, inst,
                           tiles);
    return hipGetLastError();
}

template <typename S, typename C, int NT>
hipError_t pair_launch_pt(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                          uint32_t salt_a, uint32_t salt_b, const int64_t* step_dev, bool pt, hipStream_t st)
{
    return pt ? pair_launch<S, C, NT, true>(fin, fout, inst, tiles, ntiles, salt_a, salt_b, step_dev, st)
              : pair_launch<S, C, NT, false>(fin, fout, inst, tiles, ntiles, salt_a, salt_b, step_dev, st);
}

template <typename S, typename C>
hipError_t tiles_pair_any(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                          int threads, uint32_t salt_a, uint32_t salt_b, const int64_t* step_dev, bool pt,
                          hipStream_t st)
{
    switch (threads) {
        case 64: return pair_launch_pt<S, C, 64>(fin, fout, inst, tiles, ntiles, salt_a, salt_b, step_dev, pt, st);
        case 128: return pair_launch_pt<S, C, 128>(fin, fout, inst, tiles, ntiles, salt_a, salt_b, step_dev, pt, st);
        case 256: return pair_launch_pt<S, C, 256>(fin, fout, inst, tiles, ntiles, salt_a, salt_b, step_dev, pt, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename S, typename C, int NT>
int pair_occupancy_nt()
{
    int nb = 0;
    hipError_t e;
    if constexpr (sizeof(C) == 8)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles2w<S, C, NT>, 2 * NT, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles2f<C, NT>, NT, 0);
    return e == hipSuccess ? nb : 0;
}

template <typename S, typename C>
int pair_occupancy(int threads)
{
    switch (threads) {
        case 64: return pair_occupancy_nt<S, C, 64>();
        case 128: return pair_occupancy_nt<S, C, 128>();
        case 256: return pair_occupancy_nt<S, C, 256>();
        default: return 0;
    }
}

// Resident workgroups per CU of the steady-state step (factored in and out).
template <typename S, typename C, int NT>
int occupancy_nt()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles<S, C, NT, false, Fmt::FAC, Fmt::FAC>, NT, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

template <typename S, typename C>
int tiles_occupancy(int threads)
{
    switch (threads) {
        case 64: return occupancy_nt<S, C, 64>();
        case 128: return occupancy_nt<S, C, 128>();
        case 256: return occupancy_nt<S, C, 256>();
        case 512: return occupancy_nt<S, C, 512>();
        default: return 0;
    }
}

// ---- One step on two-dimensional blocks (small lattices)
// The row march pays a warm-up of six rows per segment and one barrier-separated memory
// round trip per row; on a small lattice, whose segments must be short to fill the device,
// that is most of its time.  Here a workgroup of BX x BY lanes (lane t at column t % BX,
// row t / BX) owns the output nodes [x0, x0 + cols) x [y0, y0 + rows), cols <= BX - 4 and
// rows <= BY - 4, and lane (tx, ty) sits on node (x0 - 2 + tx, y0 - 2 + ty): all rows at
// once, one load round trip, three barriers.
//   1. every lane issues the loads of its node's pull (the f_dag_i at x - e_i) and the
//      workgroup stages the c_k, V_k of the nodes within three of the block in LDS;
//   2. lanes within two of the block: densities and totals, the groups of pull_row in its
//      order (so every sum rounds as in the march); c_k to LDS;
//   3. lanes within one: gradients, pair normals and stress (stress_at_lane); T to LDS;
//   4. the owned lanes: force (force_or_stress), collision and recolouring
//      (collide_recolour), the factored store, rounded as the march rounds it.
// Factored input and output only (a state in the 27-population format takes one step of
// the march first).  With TAPE (FP64) the owned lanes also write the adjoint's tape as the
// march does: densities, totals, concentration gradients and force, tape[20][ny][nx].
constexpr int kBlockX = 32, kBlockY = 16;
static_assert(kBlockX - 4 == kBlockCols && kBlockY - 4 == kBlockRows && kBlockX * kBlockY == kBlockThreads,
              "block plan and kernel agree");

template <typename C, int BX, int BY>
struct alignas(16) BlockLds {
    C cv[BY + 2][9][BX + 2];  // c_k, V_0, V_1, V_2 of the nodes one ring beyond the lanes'
    C c[BY][3][BX];           // c_k of the lanes' nodes
    C T[BY][3][BX];           // stress of the lanes' nodes
};

template <typename S, typename C, int BX, int BY, bool PT, bool TAPE = false>
__global__ __launch_bounds__(BX * BY) __attribute__((amdgpu_waves_per_eu(2))) void k_block(
    const S* __restrict__ fin, S* __restrict__ fout, const Instance* __restrict__ inst,
    const Tile* __restrict__ tiles, uint32_t salt, const int64_t* __restrict__ step_dev,
    double* __restrict__ tape = nullptr)
{
    static_assert(BX % 64 == 0 || 64 % BX == 0, "waves are whole tile rows");
    __shared__ BlockLds<C, BX, BY> L;
    const Tile tl = tiles[blockIdx.x];
    const KParams kp = inst[tl.inst].kp;
    const int64_t off = inst[tl.inst].offset;
    fin += off;
    fout += off;
    if constexpr (kRounds<S, C>) {
        if (step_dev) salt = step_salt(*step_dev);
    }
    const int nx = kp.nx, ny = kp.ny, cols = tl.cols, rows = tl.rows;
    const int64_t plane = kp.plane, pitch = kp.fpitch;
    const int t = threadIdx.x, tx = t % BX, ty = t / BX;
    const bool in1 = tx <= cols + 3 && ty <= rows + 3;
    const bool in2 = tx >= 1 && tx <= cols + 2 && ty >= 1 && ty <= rows + 2;
    const bool in3 = tx >= 2 && tx <= cols + 1 && ty >= 2 && ty <= rows + 1;
    const int x = wrapi(tl.x0 - 2 + tx, nx), y = wrapi(tl.y0 - 2 + ty, ny);
    const StepConsts<C> K(kp);
    // 1. the pull's f_dag_i (in flight while the c_k, V_k are staged)
    S fq[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fq[i] = S(0);
    if (in1) {
        const int xs[3] = {wrapi(x + 1, nx), x, wrapi(x - 1, nx)};  // by e_x + 1
        const int64_t ys[3] = {(int64_t)wrapi(y + 1, ny) * pitch, (int64_t)y * pitch,
                               (int64_t)wrapi(y - 1, ny) * pitch};  // by e_y + 1
#pragma unroll
        for (int i = 0; i < 9; ++i) fq[i] = fin[(int64_t)i * plane + ys[EY[i] + 1] + xs[EX[i] + 1]];
    }
    // node (x0 - 3 + u, y0 - 3 + w) at cv[w][.][u]
    const int CW = cols + 6, CH = rows + 6;
    for (int e = t; e < CW * CH; e += BX * BY) {
        const int w = e / CW, u = e - w * CW;
        const int64_t o = (int64_t)wrapi(tl.y0 - 3 + w, ny) * pitch + wrapi(tl.x0 - 3 + u, nx);
        C v[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] = C(fin[(int64_t)(9 + q) * plane + o]);
#pragma unroll
        for (int q = 0; q < 7; ++q) L.cv[w][q][u] = v[q];
        L.cv[w][7][u] = fac_v2<C>(v[3], v[5]);
        L.cv[w][8][u] = fac_v2<C>(v[4], v[6]);
    }
    __syncthreads();
    // 2. densities and totals: the source rows' groups (e_y = +1, 0, -1) as pull_row adds them
    C r0[3] = {C(1), C(1), C(1)}, f0[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f0[i] = C(0);
    if (in1) {
        auto pull = [&](int i, C (&fk)[3]) {
            const int u = tx + 1 - EX[i], w = ty + 1 - EY[i];
            const C fdi = C(fq[i]);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                fk[k] = recon<C>(L.cv[w][k][u], fdi, L.cv[w][3 + 2 * k][u], L.cv[w][4 + 2 * k][u], i);
        };
        auto group = [&](int a, int b, int c, C (&g)[3]) {
            C fa[3], fb[3], fc[3];
            pull(a, fa);
            pull(b, fb);
            pull(c, fc);
#pragma unroll
            for (int k = 0; k < 3; ++k) g[k] = group_sum<C>(fa[k], fb[k], fc[k]);
            f0[a] = (fa[0] + fa[1]) + fa[2];
            f0[b] = (fb[0] + fb[1]) + fb[2];
            f0[c] = (fc[0] + fc[1]) + fc[2];
        };
        C gp[3], gz[3], gm[3];
        group(2, 5, 6, gp);
        group(0, 1, 3, gz);
        group(4, 7, 8, gm);
#pragma unroll
        for (int k = 0; k < 3; ++k) r0[k] = (gp[k] + gz[k]) + gm[k];
        const C irho = recip((r0[0] + r0[1]) + r0[2]);
#pragma unroll
        for (int k = 0; k < 3; ++k) L.c[ty][k][tx] = r0[k] * irho;
    }
    const int64_t NN = (int64_t)nx * ny, on = (int64_t)y * nx + x;  // tape index
    if constexpr (TAPE) {
        if (in3) {
#pragma unroll
            for (int k = 0; k < 3; ++k) tape[k * NN + on] = double(r0[k]);
#pragma unroll
            for (int i = 0; i < 9; ++i) tape[(3 + i) * NN + on] = double(f0[i]);
        }
    }
    __syncthreads();
    // 3. stress (rows: ty + 1 above, ty, ty - 1 below)
    C n[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
    if (in2) {
        C Txx, Txy, Tyy;
        if constexpr (TAPE) {
            stress_at_lane<C, BX>(L.c, ty + 1, ty, ty - 1, tx, r0, K, n, Txx, Txy, Tyy,
                                  [&](const C (&gx)[3], const C (&gy)[3]) {
                                      if (in3) {
#pragma unroll
                                          for (int k = 0; k < 3; ++k) {
                                              tape[(12 + 2 * k) * NN + on] = double(gx[k]);
                                              tape[(13 + 2 * k) * NN + on] = double(gy[k]);
                                          }
                                      }
                                  });
        } else {
            stress_at_lane<C, BX>(L.c, ty + 1, ty, ty - 1, tx, r0, K, n, Txx, Txy, Tyy);
        }
        L.T[ty][0][tx] = Txx;
        L.T[ty][1][tx] = Txy;
        L.T[ty][2][tx] = Tyy;
    }
    __syncthreads();
    // 4. force, collision, recolouring, store
    if (in3) {
        C Fx, Fy, Tn[3];
        force_or_stress<C, BX, PT>(L.T, ty - 1, ty + 1, ty, tx, Fx, Fy, Tn);
        if constexpr (TAPE) {
            tape[18 * NN + on] = double(Fx);
            tape[19 * NN + on] = double(Fy);
        }
        C fd[9], ck[3], V[6], ux, uy, mxh, myh;
        collide_recolour<C, PT>(f0, r0, n, Fx, Fy, K, fd, ck, V, ux, uy, mxh, myh, Tn);
        NodeBits bits(((uint32_t)y * (uint32_t)nx + (uint32_t)x) * 27u ^ salt);
        S* o = fout + (int64_t)y * pitch + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) o[(int64_t)i * plane] = to_storage<S, C>(fd[i], bits);
#pragma unroll
        for (int k = 0; k < 3; ++k) o[(int64_t)(9 + k) * plane] = to_storage<S, C>(ck[k], bits);
#pragma unroll
        for (int q = 0; q < 4; ++q) o[(int64_t)(12 + q) * plane] = to_storage<S, C>(V[q], bits);
    }
}

// The FP64 block step writing the adjoint's tape (Guo forcing).
inline hipError_t tiles_block_tape(const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                                   int ntiles, double* tape, hipStream_t st)
{
    constexpr int BX = kBlockX, BY = kBlockY;
    hipLaunchKernelGGL((k_block<double, double, BX, BY, false, true>), dim3(ntiles), dim3(BX * BY), 0, st,
                       (const double*)fin, (double*)fout, inst, tiles, 0u, (const int64_t*)nullptr, tape);
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t tiles_block_any(const void* fin, void* fout, const Instance* inst, const Tile* tiles, int ntiles,
                           uint32_t salt, const int64_t* step_dev, bool pt, hipStream_t st)
{
    constexpr int BX = kBlockX, BY = kBlockY;
    if (pt)
        hipLaunchKernelGGL((k_block<S, C, BX, BY, true>), dim3(ntiles), dim3(BX * BY), 0, st, (const S*)fin,
                           (S*)fout, inst, tiles, salt, step_dev);
    else
        hipLaunchKernelGGL((k_block<S, C, BX, BY, false>), dim3(ntiles), dim3(BX * BY), 0, st, (const S*)fin,
                           (S*)fout, inst, tiles, salt, step_dev);
    return hipGetLastError();
}

}  // namespace
}  // namespace tcg
