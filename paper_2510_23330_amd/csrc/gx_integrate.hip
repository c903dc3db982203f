// gx_integrate.hip -- FP64 leapfrog half steps (Sec. 3.2; positions and
// velocities stay double precision, Sec. 4.3), the FP64 energy audit, and the
// Courant timestep.  All three are streaming, HBM-bound kernels: coalesced
// SoA loads, one element per lane, no LDS staging needed.
#include "gx_internal.hpp"

#include <cstring>

// With a cube table (cube != nullptr) particle i takes the step dt of its
// cube: dtk = dtk * dt_cube[cube[i]], dtd = dtd * dt_cube[cube[i]].
__global__ __launch_bounds__(256) void k_kick_drift(
    int64_t n, double dtk_, double dtd_, const int32_t* __restrict__ cube,
    const double* __restrict__ dt_cube, double* __restrict__ x, double* __restrict__ y,
    double* __restrict__ z, double* __restrict__ vx, double* __restrict__ vy,
    double* __restrict__ vz, const double* __restrict__ ax, const double* __restrict__ ay,
    const double* __restrict__ az, int64_t n_u, double* __restrict__ u,
    const double* __restrict__ dudt, double ufloor, double* __restrict__ vpred,
    double* __restrict__ upred) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double dtk = dtk_, dtd = dtd_;
    if (cube) {
        const double dc = dt_cube[cube[i]];
        dtk *= dc;
        dtd *= dc;
    }
    const double a0 = ax[i], a1 = ay[i], a2 = az[i];
    const double v0 = vx[i] + a0 * dtk, v1 = vy[i] + a1 * dtk, v2 = vz[i] + a2 * dtk;
    vx[i] = v0;
    vy[i] = v1;
    vz[i] = v2;
    if (dtd != 0.0) {
        x[i] += v0 * dtd;
        y[i] += v1 * dtd;
        z[i] += v2 * dtd;
    }
    if (vpred) {
        vpred[i] = v0 + a0 * dtk;
        vpred[n + i] = v1 + a1 * dtk;
        vpred[2 * n + i] = v2 + a2 * dtk;
    }
    if (u && i < n_u) {
        const double du = dudt[i];
        double uu = u[i] + du * dtk;
        if (ufloor > 0.0 && uu < ufloor) uu = ufloor;
        u[i] = uu;
        if (upred) {
            double up = uu + du * dtk;
            if (ufloor > 0.0 && up < ufloor) up = ufloor;
            upred[i] = up;
        }
    }
}

extern "C" int gx_kick_drift(gx_ctx* ctx, int64_t n, double dt_kick, double dt_drift, double* x,
                             double* y, double* z, double* vx, double* vy, double* vz,
                             const double* ax, const double* ay, const double* az, int64_t n_u,
                             double* u, const double* dudt, double u_floor, double* vpred_xyz,
                             double* upred) {
    if (!ctx) return GX_EINVAL;
    if (n < 0 || !x || !y || !z || !vx || !vy || !vz || !ax || !ay || !az)
        return gx_fail(ctx, GX_EINVAL, "kick_drift: null pointer or n < 0");
    if (u && (!dudt || n_u < 0 || n_u > n)) return gx_fail(ctx, GX_EINVAL, "kick_drift: bad u/dudt");
    if (n == 0) return GX_OK;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_kick_drift, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, n, dt_kick,
                       dt_drift, nullptr, nullptr, x, y, z, vx, vy, vz, ax, ay, az, u ? n_u : 0, u,
                       dudt, u_floor, vpred_xyz, upred);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

__global__ __launch_bounds__(256) void k_add_accel(int64_t n, double* __restrict__ ax,
                                                  double* __restrict__ ay,
                                                  double* __restrict__ az,
                                                  double* __restrict__ bx,
                                                  double* __restrict__ by,
                                                  double* __restrict__ bz) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        ax[i] += bx[i];
        ay[i] += by[i];
        az[i] += bz[i];
        bx[i] = 0.0;
        by[i] = 0.0;
        bz[i] = 0.0;
    }
}

extern "C" int gx_add_accel(gx_ctx* ctx, int64_t n, double* ax, double* ay, double* az,
                            double* bx, double* by, double* bz) {
    if (!ctx) return GX_EINVAL;
    if (n < 0 || !ax || !ay || !az || !bx || !by || !bz)
        return gx_fail(ctx, GX_EINVAL, "add_accel: null pointer or n < 0");
    if (n == 0) return GX_OK;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t blocks = std::min<int64_t>(gx_blocks(n, 256), 4096);
    hipLaunchKernelGGL(k_add_accel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, ax, ay, az,
                       bx, by, bz);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_kick_drift_cubes(gx_ctx* ctx, int64_t n, const int32_t* cube_id,
                                   const double* dt_cube, double f_kick, double f_drift, double* x,
                                   double* y, double* z, double* vx, double* vy, double* vz,
                                   const double* ax, const double* ay, const double* az,
                                   double* u, const double* dudt, double u_floor,
                                   double* vpred_xyz, double* upred) {
    if (!ctx) return GX_EINVAL;
    if (n < 0 || !cube_id || !dt_cube || !x || !y || !z || !vx || !vy || !vz || !ax || !ay || !az)
        return gx_fail(ctx, GX_EINVAL, "kick_drift_cubes: null pointer or n < 0");
    if (u && !dudt) return gx_fail(ctx, GX_EINVAL, "kick_drift_cubes: u without dudt");
    if (n == 0) return GX_OK;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_kick_drift, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, n, f_kick,
                       f_drift, cube_id, dt_cube, x, y, z, vx, vy, vz, ax, ay, az, u ? n : 0, u, dudt,
                       u_floor, vpred_xyz, upred);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Energy: each block reduces a fixed contiguous slice in a fixed order, the
// final block sums the block partials in index order -> deterministic.
// ---------------------------------------------------------------------------
#define EN_BLOCKS 512

__global__ __launch_bounds__(256) void k_energy_partial(
    int64_t n, const double* __restrict__ m, const double* __restrict__ vx,
    const double* __restrict__ vy, const double* __restrict__ vz, const double* __restrict__ pot,
    int64_t ng, const double* __restrict__ mg, const double* __restrict__ u,
    double* __restrict__ part) {
    __shared__ double sh[3][4];
    double k = 0, w = 0, e = 0;
    int64_t per = (n + gridDim.x - 1) / gridDim.x;
    int64_t b = blockIdx.x * per, en = min(n, b + per);
    for (int64_t i = b + threadIdx.x; i < en; i += blockDim.x) {
        double v2 = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
        k += 0.5 * m[i] * v2;
        w += 0.5 * m[i] * pot[i];
    }
    int64_t pg = (ng + gridDim.x - 1) / gridDim.x;
    int64_t bg = blockIdx.x * pg, eg = min(ng, bg + pg);
    for (int64_t i = bg + threadIdx.x; i < eg; i += blockDim.x) e += mg[i] * u[i];
    k = wave_sum(k);
    w = wave_sum(w);
    e = wave_sum(e);
    int wv = threadIdx.x / GX_WAVE;
    if (gx_lane() == 0) {
        sh[0][wv] = k;
        sh[1][wv] = w;
        sh[2][wv] = e;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0;
        for (int q = 0; q < 4; q++) s += sh[threadIdx.x][q];
        part[blockIdx.x * 3 + threadIdx.x] = s;
    }
}

__global__ void k_energy_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x >= 3) return;
    double s = 0;
    for (int b = 0; b < nb; b++) s += part[b * 3 + threadIdx.x];
    out[threadIdx.x] = s;
}

extern "C" int gx_energy(gx_ctx* ctx, const gx_particles* p, const double* pot, int64_t n_gas,
                         const double* m_gas, const double* u, double* out) {
    if (!ctx || !p || !pot || !out) return GX_EINVAL;
    if (!p->m || !p->vx || !p->vy || !p->vz || p->n < 0)
        return gx_fail(ctx, GX_EINVAL, "energy: bad particle view");
    if (n_gas > 0 && (!m_gas || !u)) return gx_fail(ctx, GX_EINVAL, "energy: gas arrays missing");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    GX_TRY(gx_reserve(ctx, ctx->partial, (EN_BLOCKS * 3 + 8) * sizeof(double)));
    double* part = (double*)ctx->partial.p;
    double* res = part + EN_BLOCKS * 3;
    hipLaunchKernelGGL(k_energy_partial, dim3(EN_BLOCKS), dim3(256), 0, ctx->stream, p->n, p->m,
                       p->vx, p->vy, p->vz, pot, n_gas > 0 ? n_gas : 0, m_gas, u, part);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, ctx->stream, part, EN_BLOCKS, res);
    GX_LAUNCH_CHECK(ctx);
    GX_HIP(ctx, hipMemcpyAsync(out, res, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Courant step: positive doubles order like their bit patterns, so a 64-bit
// integer atomicMin gives the minimum.
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Courant step per cube: the lanes of a wave that share a cube (particles of
// one cube are contiguous, so usually all of them) take the minimum by
// shuffles and one lane updates the cube's minimum (positive doubles order
// like their bit patterns).
__global__ __launch_bounds__(256) void k_cfl(int64_t n, const float* __restrict__ H,
                                             const float* __restrict__ vsig,
                                             const int32_t* __restrict__ cube, double c,
                                             unsigned long long* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool valid = false;
    double dt = INFINITY;
    int cb = -1;
    if (i < n) {
        const double v = (double)vsig[i];
        if (v > 0.0) {
            valid = true;
            dt = c * (double)H[i] / v;
            cb = cube ? cube[i] : 0;
        }
    }
    uint64_t pending = __ballot(valid);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int lc = __shfl(cb, leader, 64);
        const bool mine = valid && cb == lc;
        double m = mine ? dt : INFINITY;
        for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
        if (lane == leader) atomicMin(&out[lc], (unsigned long long)__double_as_longlong(m));
        pending &= ~__ballot(mine);
    }
}

extern "C" int gx_sph_timestep(gx_ctx* ctx, const gx_gas* g, double c_cfl, const int32_t* cube_id,
                               int n_cubes, double* dt_out) {
    if (!ctx || !g || !dt_out || !g->H || !g->vsig) return GX_EINVAL;
    if (n_cubes < 1 || (!cube_id && n_cubes != 1)) return gx_fail(ctx, GX_EINVAL, "bad n_cubes");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const double inf = INFINITY;
    unsigned long long inf_bits;
    memcpy(&inf_bits, &inf, sizeof inf_bits);
    hipLaunchKernelGGL(k_fill_u64, dim3(gx_blocks(n_cubes, 256)), dim3(256), 0, ctx->stream,
                       (unsigned long long*)dt_out, n_cubes, inf_bits);
    if (g->n > 0)
        hipLaunchKernelGGL(k_cfl, dim3(gx_blocks(g->n, 256)), dim3(256), 0, ctx->stream, g->n, g->H,
                           g->vsig, cube_id, c_cfl, (unsigned long long*)dt_out);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}
