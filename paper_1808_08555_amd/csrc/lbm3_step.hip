// Companion kernels of the fused step (initial state, import and export of the
// post-streaming populations, observables reduction, device copy) and the launchers; the
// step itself is in lbm3_step_impl.h, instantiated per precision in lbm3_tiles_*.hip.
#include "lbm3_step_impl.h"

namespace tcg {
namespace {

// Fixed-order second pass over the per-workgroup partials (deterministic): each lane combines
// a strided share, then the workgroup reduction (wavefront reductions, then the four wave
// results in order).
__global__ __launch_bounds__(256) void k_reduce_obs(const double* __restrict__ partials, int n,
                                                    double* __restrict__ out)
{
    __shared__ double red[kObsFields][256];
    const int t = threadIdx.x;
    double acc[kObsFields] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = t; b < n; b += 256) {
#pragma unroll
        for (int a = 0; a < kObsFields; ++a) acc[a] = obs_combine(a, acc[a], partials[(int64_t)b * kObsFields + a]);
    }
    block_reduce_obs<256>(acc, red, out);
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

// The device step counter of a batch: one lane adds the steps a launch advanced.
__global__ __launch_bounds__(64) void k_advance_step(int64_t* __restrict__ step_dev, int64_t n)
{
    if (threadIdx.x == 0) *step_dev += n;
}

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                              int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}


// Post-streaming populations f_{i,k}(x) rebuilt from a factored state at x - e_i, with the
// arithmetic the step uses when it pulls them.
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_export_fac(const S* __restrict__ fin, double* __restrict__ f,
                                                    KParams kp)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    const int nx = kp.nx, ny = kp.ny;
    if (x >= nx) return;
    const int64_t N = (int64_t)nx * ny, j = (int64_t)y * nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int64_t s = (int64_t)wrapi(y - EY[i], ny) * kp.fpitch + wrapi(x - EX[i], nx);
        const C fd = C(fin[(int64_t)i * kp.plane + s]);
        C vx[3], vy[3];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            vx[k] = C(fin[(int64_t)(12 + 2 * k) * kp.plane + s]);
            vy[k] = C(fin[(int64_t)(13 + 2 * k) * kp.plane + s]);
        }
        vx[2] = fac_v2<C>(vx[0], vx[1]);
        vy[2] = fac_v2<C>(vy[0], vy[1]);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const C ck = C(fin[(int64_t)(9 + k) * kp.plane + s]);
            f[(k * 9 + i) * N + j] = double(recon<C>(ck, fd, vx[k], vy[k], i));
        }
    }
}

}  // namespace

size_t elem_bytes(Prec p) { return p == Prec::F64 ? 8 : 4; }

hipError_t launch_pair(Prec prec, const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                       int ntiles, int threads, int64_t step, hipStream_t stream, bool pt, const int64_t* step_dev)
{
    switch (prec) {
        case Prec::F64: return tiles_f64_pair(fin, fout, inst, tiles, ntiles, threads, pt, stream);
        case Prec::F32: return tiles_f32_pair(fin, fout, inst, tiles, ntiles, threads, pt, stream);
        case Prec::F32S:
            return tiles_f32s_pair(fin, fout, inst, tiles, ntiles, threads, step_salt(step), step_salt(step + 1),
                                   step_dev, pt, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tiles(Prec prec, Fmt in, Fmt out, const void* fin, void* fout, const Instance* inst,
                        const Tile* tiles, int ntiles, int threads, int64_t step, int filter,
                        hipStream_t st, bool pt, const int64_t* step_dev)
{
    const uint32_t salt = step_salt(step);
    switch (prec) {
        case Prec::F64:
            return tiles_f64(in, out, false, pt, fin, fout, inst, tiles, ntiles, threads, salt, nullptr, filter,
                             nullptr, nullptr, st);
        case Prec::F32S:
            return tiles_f32s(in, out, false, pt, fin, fout, inst, tiles, ntiles, threads, salt, step_dev, filter,
                              nullptr, nullptr, st);
        case Prec::F32:
            return tiles_f32(in, out, false, pt, fin, fout, inst, tiles, ntiles, threads, salt, nullptr, filter,
                             nullptr, nullptr, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_block(Prec prec, const void* fin, void* fout, const Instance* inst, const Tile* tiles,
                        int ntiles, int64_t step, hipStream_t st, bool pt, const int64_t* step_dev)
{
    const uint32_t salt = step_salt(step);
    switch (prec) {
        case Prec::F64: return tiles_f64_block(fin, fout, inst, tiles, ntiles, salt, nullptr, pt, st);
        case Prec::F32S: return tiles_f32s_block(fin, fout, inst, tiles, ntiles, salt, step_dev, pt, st);
        case Prec::F32: return tiles_f32_block(fin, fout, inst, tiles, ntiles, salt, nullptr, pt, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_advance_step(int64_t* step_dev, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(64), 0, st, step_dev, n);
    return hipGetLastError();
}

hipError_t launch_observe_tiles(Prec prec, Fmt in, const void* fin, const Instance* inst,
                                const Tile* tiles, int ntiles, int threads, double* partials,
                                double* rho_out, hipStream_t st, bool pt)
{
    switch (prec) {
        case Prec::F64:
            return tiles_f64(in, in, true, pt, fin, nullptr, inst, tiles, ntiles, threads, 0u, nullptr, 0,
                             partials, rho_out, st);
        case Prec::F32S:
            return tiles_f32s(in, in, true, pt, fin, nullptr, inst, tiles, ntiles, threads, 0u, nullptr, 0,
                              partials, rho_out, st);
        case Prec::F32:
            return tiles_f32(in, in, true, pt, fin, nullptr, inst, tiles, ntiles, threads, 0u, nullptr, 0,
                             partials, rho_out, st);
    }
    return hipErrorInvalidValue;
}

int blocks_per_cu(Prec prec, int threads)
{
    switch (prec) {
        case Prec::F64: return tiles_f64_occupancy(threads);
        case Prec::F32S: return tiles_f32s_occupancy(threads);
        case Prec::F32: return tiles_f32_occupancy(threads);
    }
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

hipError_t launch_export(Prec prec, Fmt in, const void* fin, double* f, const KParams& kp,
                         hipStream_t st)
{
    dim3 grid((kp.nx + 255) / 256, kp.ny);
    if (in == Fmt::F27) {
        if (prec == Prec::F64)
            hipLaunchKernelGGL((k_export<double>), grid, dim3(256), 0, st, (const double*)fin, f, kp);
        else
            hipLaunchKernelGGL((k_export<float>), grid, dim3(256), 0, st, (const float*)fin, f, kp);
    } else if (prec == Prec::F64) {
        hipLaunchKernelGGL((k_export_fac<double, double>), grid, dim3(256), 0, st, (const double*)fin, f, kp);
    } else if (prec == Prec::F32S) {
        hipLaunchKernelGGL((k_export_fac<float, double>), grid, dim3(256), 0, st, (const float*)fin, f, kp);
    } else {
        hipLaunchKernelGGL((k_export_fac<float, float>), grid, dim3(256), 0, st, (const float*)fin, f, kp);
    }
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
