// gx_sn.hip -- supernova-region coupling of the surrogate (Sec. 3.2 steps 2
// and 4, Sec. 3.3): pick up the gas in the (60 pc)^3 box around each SN,
// inject the explosion energy, map particles to a voxel grid by SPH kernel
// convolution with Shepard normalisation, draw particles back from a
// predicted grid (as many as went in, so mass is conserved), and replace
// particles by ID.
#include "gx_internal.hpp"

#include <mutex>
#include <vector>

#include <cmath>

#define VOX_B 4            // voxel blocks of 4^3 = 64 voxels, one per lane
#define VOX_TILE 256
#define WC4_NORM_D 4.9238032806262495  // 495 / (32 pi)

// ---------------------------------------------------------------------------
// Extraction: particles with c - h <= x < c + h in every axis.  Two passes over
// (particle chunk, cube): counts per (cube, chunk), one exclusive scan in
// cube-major order, then a fill that keeps original order within each cube.
// ---------------------------------------------------------------------------
#define EX_ITEMS 8
#define EX_CHUNK (256 * EX_ITEMS)

__device__ __forceinline__ bool in_box(double x, double y, double z, const double* c, double h) {
    return x >= c[0] - h && x < c[0] + h && y >= c[1] - h && y < c[1] + h && z >= c[2] - h &&
           z < c[2] + h;
}

__global__ __launch_bounds__(256) void k_extract_count(int64_t n, const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ z,
                                                       const double* __restrict__ centers, double h,
                                                       int nchunk, uint32_t* __restrict__ cnt) {
    const int c = blockIdx.y;
    const double cc[3] = {centers[3 * c], centers[3 * c + 1], centers[3 * c + 2]};
    uint32_t k = 0;
    const int64_t base = (int64_t)blockIdx.x * EX_CHUNK;
    for (int r = 0; r < EX_ITEMS; r++) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n && in_box(x[i], y[i], z[i], cc, h)) k++;
    }
    __shared__ uint32_t sh[4];
    uint32_t tot;
    block_excl_scan256<uint32_t>(k, sh, &tot);
    if (threadIdx.x == 0) cnt[(int64_t)c * nchunk + blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_extract_fill(int64_t n, const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ centers, double h,
                                                      int nchunk, const uint32_t* __restrict__ off,
                                                      int32_t* __restrict__ idx) {
    const int c = blockIdx.y;
    const double cc[3] = {centers[3 * c], centers[3 * c + 1], centers[3 * c + 2]};
    __shared__ uint32_t sh[4];
    uint32_t pos = off[(int64_t)c * nchunk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * EX_CHUNK;
    for (int r = 0; r < EX_ITEMS; r++) {
        const int64_t i = base + r * 256 + threadIdx.x;
        const uint32_t f = (i < n && in_box(x[i], y[i], z[i], cc, h)) ? 1u : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan256<uint32_t>(f, sh, &tot);
        if (f) idx[pos + ex] = (int32_t)i;
        pos += tot;
    }
}

__global__ void k_extract_offsets(const uint32_t* __restrict__ off, int k, int nchunk,
                                  uint32_t total, int32_t* __restrict__ offsets) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > k) return;
    offsets[c] = (int32_t)(c < k ? off[(int64_t)c * nchunk] : total);
}

extern "C" int gx_sn_extract(gx_ctx* ctx, const gx_particles* gas, const double* centers, int k,
                             double half_side, int32_t* offsets, int32_t* idx, int64_t cap,
                             int64_t* total) {
    if (!ctx || !gas || !centers || !offsets || !idx || !total || k < 1 || !(half_side > 0))
        return GX_EINVAL;
    if (!gas->x || !gas->y || !gas->z || gas->n < 0 || gas->n >= ((int64_t)1 << 31))
        return gx_fail(ctx, GX_EINVAL, "sn_extract: bad particle view");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t n = gas->n;
    const int nchunk = (int)std::max<int64_t>(1, (n + EX_CHUNK - 1) / EX_CHUNK);
    const int64_t nc = (int64_t)k * nchunk;
    GX_TRY(gx_reserve(ctx, ctx->hist, (nc + 8) * sizeof(uint32_t) * 2));
    uint32_t* cnt = (uint32_t*)ctx->hist.p;
    uint32_t* off = cnt + nc + 4;
    GX_TRY(gx_reserve(ctx, ctx->small, 64));
    uint32_t* dtot = (uint32_t*)ctx->small.p;
    hipLaunchKernelGGL(k_extract_count, dim3(nchunk, k), dim3(256), 0, st, n, gas->x, gas->y, gas->z,
                       centers, half_side, nchunk, cnt);
    GX_TRY((gx_scan<uint32_t, uint32_t>(ctx, cnt, off, nc, dtot)));
    uint32_t h = 0;
    GX_HIP(ctx, hipMemcpyAsync(&h, dtot, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GX_HIP(ctx, hipStreamSynchronize(st));
    *total = h;
    if ((int64_t)h > cap) return gx_fail(ctx, GX_EINVAL, "sn_extract: %u particles exceed cap %lld", h, (long long)cap);
    hipLaunchKernelGGL(k_extract_fill, dim3(nchunk, k), dim3(256), 0, st, n, gas->x, gas->y, gas->z,
                       centers, half_side, nchunk, off, idx);
    hipLaunchKernelGGL(k_extract_offsets, dim3(gx_blocks(k + 1, 64)), dim3(64), 0, st, off, k, nchunk,
                       h, offsets);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Injection: the k_inj members of each cube nearest its centre (ties by
// index) receive E / (their total mass) of specific internal energy.  The
// k_inj-th smallest squared distance is found by bisection on its bit
// pattern (non-negative floats order like their bits).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sn_inject(const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ z,
                                                   const double* __restrict__ m,
                                                   const int32_t* __restrict__ offsets,
                                                   const int32_t* __restrict__ idx,
                                                   const double* __restrict__ centers, int k_inj,
                                                   double energy, double* __restrict__ u) {
    const int c = blockIdx.x;
    const int b = offsets[c], e = offsets[c + 1];
    const int cnt = e - b;
    if (cnt <= 0) return;
    const double cx = centers[3 * c], cy = centers[3 * c + 1], cz = centers[3 * c + 2];
    __shared__ uint32_t sh[4];
    __shared__ double shd[4];
    auto d2bits = [&](int j) -> unsigned long long {
        const int i = idx[j];
        const double dx = x[i] - cx, dy = y[i] - cy, dz = z[i] - cz;
        return (unsigned long long)__double_as_longlong(dx * dx + dy * dy + dz * dz);
    };
    const int want = min(k_inj, cnt);
    // smallest threshold t with #(d2 <= t) >= want
    unsigned long long lo = 0, hi = 0x7ff0000000000000ull;
    while (lo < hi) {
        const unsigned long long mid = lo + (hi - lo) / 2;
        uint32_t c_le = 0;
        for (int j = b + threadIdx.x; j < e; j += 256) c_le += d2bits(j) <= mid;
        uint32_t tot;
        block_excl_scan256<uint32_t>(c_le, sh, &tot);
        if ((int)tot >= want) hi = mid;
        else lo = mid + 1;
    }
    const unsigned long long t = lo;
    // members strictly below t, then ties at t in index order until `want`
    uint32_t below = 0;
    for (int j = b + threadIdx.x; j < e; j += 256) below += d2bits(j) < t;
    uint32_t nbelow;
    block_excl_scan256<uint32_t>(below, sh, &nbelow);
    const int ties_needed = want - (int)nbelow;
    // pass 1: total mass of the chosen members
    double msum = 0.0;
    int tie_seen = 0;
    for (int j0 = b; j0 < e; j0 += 256) {
        const int j = j0 + threadIdx.x;
        const unsigned long long d = j < e ? d2bits(j) : ~0ull;
        const uint32_t is_tie = (j < e && d == t) ? 1u : 0u;
        uint32_t ntie;
        const uint32_t ex = block_excl_scan256<uint32_t>(is_tie, sh, &ntie);
        const bool chosen = j < e && (d < t || (is_tie && tie_seen + (int)ex < ties_needed));
        if (chosen) msum += m[idx[j]];
        tie_seen += (int)ntie;
    }
    msum = wave_sum(msum);
    if ((threadIdx.x & 63) == 0) shd[threadIdx.x >> 6] = msum;
    __syncthreads();
    const double M = (shd[0] + shd[1]) + (shd[2] + shd[3]);
    __syncthreads();
    const double du = energy / M;
    tie_seen = 0;
    for (int j0 = b; j0 < e; j0 += 256) {
        const int j = j0 + threadIdx.x;
        const unsigned long long d = j < e ? d2bits(j) : ~0ull;
        const uint32_t is_tie = (j < e && d == t) ? 1u : 0u;
        uint32_t ntie;
        const uint32_t ex = block_excl_scan256<uint32_t>(is_tie, sh, &ntie);
        const bool chosen = j < e && (d < t || (is_tie && tie_seen + (int)ex < ties_needed));
        if (chosen) atomicAdd(&u[idx[j]], du);  // boxes may share a chosen particle
        tie_seen += (int)ntie;
    }
}

extern "C" int gx_sn_inject(gx_ctx* ctx, const gx_particles* gas, const int32_t* offsets,
                            const int32_t* idx, const double* centers, int k, int k_inj,
                            double energy, double* u) {
    if (!ctx || !gas || !offsets || !idx || !centers || !u || k < 1 || k_inj < 1 || !(energy >= 0))
        return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_sn_inject, dim3(k), dim3(256), 0, ctx->stream, gas->x, gas->y, gas->z,
                       gas->m, offsets, idx, centers, k_inj, energy, u);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// Ambient state of each box from its members: mean density (total mass over
// the box volume), mass-weighted temperature and bulk velocity.  One block per
// box; FP64 sums in a fixed order.
__global__ __launch_bounds__(256) void k_sn_ambient(const double* __restrict__ vx,
                                                    const double* __restrict__ vy,
                                                    const double* __restrict__ vz,
                                                    const double* __restrict__ m,
                                                    const double* __restrict__ u,
                                                    const int32_t* __restrict__ offsets,
                                                    const int32_t* __restrict__ idx, double volume,
                                                    double u_to_T, float t_floor,
                                                    float* __restrict__ amb) {
    const int c = blockIdx.x;
    const int b = offsets[c], e = offsets[c + 1];
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = b + threadIdx.x; j < e; j += 256) {
        const int i = idx[j];
        const double mi = m[i];
        s[0] += mi;
        s[1] += mi * u[i];
        s[2] += mi * vx[i];
        s[3] += mi * vy[i];
        s[4] += mi * vz[i];
    }
    __shared__ double sh[4][5];
    for (int q = 0; q < 5; q++) {
        const double t = wave_sum(s[q]);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[5];
        for (int q = 0; q < 5; q++) t[q] = (sh[0][q] + sh[1][q]) + (sh[2][q] + sh[3][q]);
        float* a = amb + 5 * c;
        if (t[0] > 0.0) {
            a[0] = (float)log10(t[0] / volume);
            a[1] = (float)log10(fmax(t[1] / t[0] * u_to_T, (double)t_floor));
            a[2] = (float)(t[2] / t[0]);
            a[3] = (float)(t[3] / t[0]);
            a[4] = (float)(t[4] / t[0]);
        } else {
            a[0] = -30.0f;
            a[1] = log10f(t_floor);
            a[2] = a[3] = a[4] = 0.0f;
        }
    }
}

extern "C" int gx_sn_ambient(gx_ctx* ctx, const gx_particles* gas, const double* u,
                             const int32_t* offsets, const int32_t* idx, int k, double side,
                             double u_to_T, float* amb) {
    if (!ctx || !gas || !u || !offsets || !idx || !amb || k < 1 || !(side > 0) || !(u_to_T > 0))
        return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_sn_ambient, dim3(k), dim3(256), 0, ctx->stream, gas->vx, gas->vy, gas->vz,
                       gas->m, u, offsets, idx, side * side * side, u_to_T, 10.0f, amb);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// Pack the members of each box into a compact particle set in the box's own
// frame (the hand-over of a region to the surrogate, Sec. 3.2 step 2):
// position (x - c_k) * scale + dst_k, velocity unchanged, kernel size * scale;
// the members keep their CSR order.
__global__ void k_sn_gather(int k, const int32_t* __restrict__ offsets,
                            const int32_t* __restrict__ idx, const double* __restrict__ centers,
                            const double* __restrict__ dst, double scale,
                            const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ z, const double* __restrict__ vx,
                            const double* __restrict__ vy, const double* __restrict__ vz,
                            const double* __restrict__ m, const double* __restrict__ u,
                            const float* __restrict__ H, double* __restrict__ ox,
                            double* __restrict__ oy, double* __restrict__ oz,
                            double* __restrict__ ovx, double* __restrict__ ovy,
                            double* __restrict__ ovz, double* __restrict__ om,
                            double* __restrict__ ou, float* __restrict__ oH) {
    const int c = blockIdx.y;
    const int b = offsets[c], e = offsets[c + 1];
    const int j = b + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= e) return;
    const int i = idx[j];
    ox[j] = (x[i] - centers[3 * c]) * scale + dst[3 * c];
    oy[j] = (y[i] - centers[3 * c + 1]) * scale + dst[3 * c + 1];
    oz[j] = (z[i] - centers[3 * c + 2]) * scale + dst[3 * c + 2];
    ovx[j] = vx[i];
    ovy[j] = vy[i];
    ovz[j] = vz[i];
    om[j] = m[i];
    ou[j] = u[i];
    if (oH) oH[j] = H ? (float)(H[i] * scale) : -1.0f;
}

extern "C" int gx_sn_gather(gx_ctx* ctx, const gx_particles* gas, const double* u, const float* H,
                            const int32_t* offsets, const int32_t* idx, int k, int64_t n_max,
                            const double* centers, const double* dst, double scale, double* x,
                            double* y, double* z, double* vx, double* vy, double* vz, double* m,
                            double* uo, float* Ho) {
    if (!ctx || !gas || !u || !offsets || !idx || !centers || !dst || k < 1 || n_max < 0 ||
        !(scale > 0) || !x || !y || !z || !vx || !vy || !vz || !m || !uo)
        return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    if (n_max == 0) return GX_OK;
    const int gxb = (int)((n_max + 255) / 256);
    hipLaunchKernelGGL(k_sn_gather, dim3(gxb, k), dim3(256), 0, ctx->stream, k, offsets, idx,
                       centers, dst, scale, gas->x, gas->y, gas->z, gas->vx, gas->vy, gas->vz,
                       gas->m, u, H, x, y, z, vx, vy, vz, m, uo, Ho);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// Inverse of the gather for replacement particles: x = (x - src_k) / scale
// + c_k + v_k dt (v_k = the box's bulk velocity, columns 2..4 of amb, so the
// particles follow the region's mean motion over the hand-over delay).
__global__ void k_sn_unframe(int k, const int32_t* __restrict__ offsets,
                             const double* __restrict__ src, const double* __restrict__ centers,
                             const float* __restrict__ amb, double dt, double inv_scale,
                             double* __restrict__ x, double* __restrict__ y,
                             double* __restrict__ z) {
    const int c = blockIdx.y;
    const int b = offsets[c], e = offsets[c + 1];
    const int j = b + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= e) return;
    double s[3];
    for (int d = 0; d < 3; d++) s[d] = centers[3 * c + d] + (amb ? (double)amb[5 * c + 2 + d] * dt : 0.0);
    x[j] = (x[j] - src[3 * c]) * inv_scale + s[0];
    y[j] = (y[j] - src[3 * c + 1]) * inv_scale + s[1];
    z[j] = (z[j] - src[3 * c + 2]) * inv_scale + s[2];
}

extern "C" int gx_sn_unframe(gx_ctx* ctx, const int32_t* offsets, int k, int64_t n_max,
                             const double* src, const double* centers, const float* amb,
                             double dt, double scale, double* x, double* y, double* z) {
    if (!ctx || !offsets || !src || !centers || k < 1 || n_max < 0 || !(scale > 0) || !x || !y ||
        !z)
        return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    if (n_max == 0) return GX_OK;
    const int gxb = (int)((n_max + 255) / 256);
    hipLaunchKernelGGL(k_sn_unframe, dim3(gxb, k), dim3(256), 0, ctx->stream, k, offsets, src,
                       centers, amb, dt, 1.0 / scale, x, y, z);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Voxelisation: rho_v = sum_j m_j W(|x_v - x_j|, H_j); T_v and v_v are Shepard
// averages sum_j f_j W_j / sum_j W_j.  Voxels are grouped into 4^3 blocks (one
// voxel per lane); each block's candidate particles are the gas-tree leaves
// within reach of the block box (reach = largest kernel size in the node),
// exactly as for the SPH force.
// ---------------------------------------------------------------------------
__global__ void k_gather_h(int64_t n, const uint32_t* __restrict__ perm, const float* __restrict__ H,
                           const double* __restrict__ u, float4* __restrict__ ss) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t o = perm[s];
    ss[s] = make_float4(H[o], (float)u[o], 0.0f, 0.0f);
}

__global__ void k_vox_blocks(int k, int grid, double half, const double* __restrict__ centers,
                             NodeRec* __restrict__ recv, float* __restrict__ rad) {
    const int nbs = grid / VOX_B;
    const int64_t per = (int64_t)nbs * nbs * nbs;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= per * k) return;
    const int c = (int)(e / per);
    int64_t t = e % per;
    const int bx = (int)(t % nbs);
    t /= nbs;
    const int by = (int)(t % nbs);
    const int bz = (int)(t / nbs);
    const double dv = 2.0 * half / grid;
    const int b3[3] = {bx, by, bz};
    NodeRec r;
    for (int d = 0; d < 3; d++) {
        const double o = centers[3 * c + d] - half;
        r.lo[d] = o + (b3[d] * VOX_B + 0.5) * dv;
        r.hi[d] = o + (b3[d] * VOX_B + VOX_B - 0.5) * dv;
    }
    r.next = -1;
    r.begin = 0;
    r.end = 64;
    r.level = -1;
    r.leaf = 0;
    r.nchild = 0;
    recv[e] = r;
    rad[e] = 0.0f;
}

__global__ __launch_bounds__(64) void k_voxelize(
    int nbv, int grid, const NodeRec* __restrict__ recv, const double4* __restrict__ pos4,
    const uint32_t* __restrict__ perm, const double* __restrict__ vx,
    const double* __restrict__ vy, const double* __restrict__ vz,
    const float4* __restrict__ ss, ListView L, double u_to_T, const float* __restrict__ amb,
    const float* __restrict__ mean, const float* __restrict__ stdv, float rho_floor_frac,
    float t_floor, uint16_t* __restrict__ out_bf, int cpad, float* __restrict__ out_f32) {
    const int g = blockIdx.x;
    if (g >= nbv) return;
    __shared__ float tx[VOX_TILE], ty[VOX_TILE], tz[VOX_TILE], tm[VOX_TILE], th[VOX_TILE],
        tT[VOX_TILE], tvx[VOX_TILE], tvy[VOX_TILE], tvz[VOX_TILE];
    __shared__ int jidx[VOX_TILE], jroff[VOX_TILE], wtot[1];
    const int lane = threadIdx.x;
    const NodeRec B = recv[g];
    const double cx = (B.lo[0] + B.hi[0]) * 0.5, cy = (B.lo[1] + B.hi[1]) * 0.5,
                 cz = (B.lo[2] + B.hi[2]) * 0.5;
    const double dv = (B.hi[0] - B.lo[0]) / (VOX_B - 1);
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const float px = (float)(B.lo[0] + lx * dv - cx), py = (float)(B.lo[1] + ly * dv - cy),
                pz = (float)(B.lo[2] + lz * dv - cz);
    const GroupList GL(L, g);
    const int npp = GL.npp;
    float sr = 0, sw = 0, stt = 0, svx = 0, svy = 0, svz = 0;
    for (int t0 = 0; t0 < npp; t0 += VOX_TILE) {
        const int tn = min(VOX_TILE, npp - t0);
        __syncthreads();
        list_slots(GL, npp, t0, t0 + tn, jidx, jroff, wtot, lane, 64);
        for (int e = lane; e < tn; e += 64) {
            const int j = jidx[e];
            const double4 p = pos4[j];
            const float4 q = ss[j];
            const uint32_t o = perm[j];
            tx[e] = (float)(p.x - cx);
            ty[e] = (float)(p.y - cy);
            tz[e] = (float)(p.z - cz);
            tm[e] = (float)p.w;
            th[e] = q.x;
            tT[e] = (float)((double)q.y * u_to_T);
            tvx[e] = (float)vx[o];
            tvy[e] = (float)vy[o];
            tvz[e] = (float)vz[o];
        }
        __syncthreads();
        for (int e = 0; e < tn; e++) {
            const float dx = tx[e] - px, dy = ty[e] - py, dz = tz[e] - pz;
            const float H = th[e];
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < H * H) {
                const float q = __builtin_sqrtf(r2) / H;
                const float t = 1.0f - q, t2 = t * t;
                const float w = (float)WC4_NORM_D / (H * H * H) * t2 * t2 * t2 *
                                (1.0f + q * (6.0f + q * (35.0f / 3.0f)));
                sr += tm[e] * w;
                sw += w;
                stt += w * tT[e];
                svx += w * tvx[e];
                svy += w * tvy[e];
                svz += w * tvz[e];
            }
        }
    }
    // voxel index inside its cube
    const int nbs = grid / VOX_B;
    const int64_t per = (int64_t)nbs * nbs * nbs;
    const int c = (int)(g / per);
    int64_t t = g % per;
    const int bx = (int)(t % nbs);
    t /= nbs;
    const int by = (int)(t % nbs);
    const int bz = (int)(t / nbs);
    const int X = bx * VOX_B + lx, Y = by * VOX_B + ly, Z = bz * VOX_B + lz;
    const int64_t v = (((int64_t)c * grid + Z) * grid + Y) * grid + X;
    const float* a = amb + 5 * c;
    float ch[5];
    const float rho_floor = rho_floor_frac * powf(10.0f, a[0]);
    ch[0] = log10f(fmaxf(sr, rho_floor));
    if (sw > 0.0f) {
        ch[1] = log10f(fmaxf(stt / sw, t_floor));
        ch[2] = svx / sw;
        ch[3] = svy / sw;
        ch[4] = svz / sw;
    } else {
        ch[1] = a[1];
        ch[2] = a[2];
        ch[3] = a[3];
        ch[4] = a[4];
    }
    if (out_f32)
        for (int q = 0; q < 5; q++) out_f32[v * 5 + q] = ch[q];
    if (out_bf) {
        for (int q = 0; q < cpad; q++) {
            const float s = q < 5 ? (ch[q] - mean[q]) / stdv[q] : 0.0f;
            uint32_t ub = __float_as_uint(s);
            ub += 0x7fffu + ((ub >> 16) & 1u);
            out_bf[v * cpad + q] = (uint16_t)(ub >> 16);
        }
    }
}

extern "C" int gx_sn_voxelize(gx_ctx* ctx, const gx_particles* gas, const double* u, const float* H,
                              const double* centers, int k, double side, int grid, double u_to_T,
                              const float* amb, const float* chan_mean, const float* chan_std,
                              uint16_t* out_bf16, int cpad, float* out_f32) {
    if (!ctx || !gas || !u || !H || !centers || !amb || k < 1 || !(side > 0))
        return GX_EINVAL;
    if (grid < VOX_B || grid % VOX_B) return gx_fail(ctx, GX_EINVAL, "sn_voxelize: grid %% 4 != 0");
    if (out_bf16 && (!chan_mean || !chan_std || cpad < 5))
        return gx_fail(ctx, GX_EINVAL, "sn_voxelize: bf16 output needs mean/std and cpad >= 5");
    if (!out_bf16 && !out_f32) return GX_EINVAL;
    GX_TRY(gx_tree_check(ctx, GX_TREE_GAS, gas));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    TreeSlot& T = ctx->tree[GX_TREE_GAS];
    const int64_t n = T.n;
    GX_TRY(gx_reserve(ctx, ctx->sph_work[8], n * sizeof(float4)));
    float4* ss = (float4*)ctx->sph_work[8].p;
    hipLaunchKernelGGL(k_gather_h, dim3(gx_blocks(n, 256)), dim3(256), 0, st, n,
                       (const uint32_t*)T.val[0].p, H, u, ss);
    GX_TRY(gx_sph_node_hmax(ctx, T, ss));
    const int nbs = grid / VOX_B;
    const int64_t per = (int64_t)nbs * nbs * nbs;
    // cubes in chunks so the per-receiver list slots stay bounded
    const int kc = (int)std::max<int64_t>(1, std::min<int64_t>(k, 65536 / per));
    GX_TRY(gx_reserve(ctx, ctx->sph_work[9], kc * per * sizeof(NodeRec)));
    GX_TRY(gx_reserve(ctx, ctx->sph_work[10], kc * per * sizeof(float)));
    NodeRec* recv = (NodeRec*)ctx->sph_work[9].p;
    float* rad = (float*)ctx->sph_work[10].p;
    const int64_t nvox = (int64_t)grid * grid * grid;
    for (int c0 = 0; c0 < k; c0 += kc) {
        const int kk = std::min(kc, k - c0);
        const int64_t nbv = kk * per;
        hipLaunchKernelGGL(k_vox_blocks, dim3(gx_blocks(nbv, 256)), dim3(256), 0, st, kk, grid,
                           0.5 * side, centers + 3 * c0, recv, rad);
        GX_LAUNCH_CHECK(ctx);
        ListView view;
        int64_t pairs = 0;
        GX_TRY(gx_sph_walk(ctx, T, ctx->sph, (int)nbv, nullptr, recv, rad, 1, nullptr, &view,
                           &pairs));
        hipLaunchKernelGGL(k_voxelize, dim3((unsigned)nbv), dim3(64), 0, st, (int)nbv, grid, recv,
                           (const double4*)T.pos4.p, (const uint32_t*)T.val[0].p, gas->vx, gas->vy,
                           gas->vz, ss, view, u_to_T, amb + 5 * c0, chan_mean, chan_std, 1e-6f,
                           10.0f, out_bf16 ? out_bf16 + c0 * nvox * cpad : nullptr, cpad,
                           out_f32 ? out_f32 + c0 * nvox * 5 : nullptr);
        GX_LAUNCH_CHECK(ctx);
    }
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Resampling: N_out particles per cube, voxel drawn with probability
// proportional to its predicted density (inverse of the cumulative sum, one
// uniform each), position uniform inside the voxel (three more uniforms),
// temperature and velocity of that voxel.
// ---------------------------------------------------------------------------
// Inclusive prefix sums of the voxel weights 10^(log10 rho) of every cube, in
// three passes with a fixed order: tiles of CDF_TILE voxels (8 consecutive
// per thread, then across the block), the tile totals of each cube, and the
// tile offsets added back.
#define CDF_TILE 2048
__global__ __launch_bounds__(256) void k_cdf_tiles(const float* __restrict__ pred, int nvox,
                                                   double* __restrict__ cdf,
                                                   double* __restrict__ ttot) {
    const int c = blockIdx.y, t = blockIdx.x;
    const int ntile = (nvox + CDF_TILE - 1) / CDF_TILE;
    const float* p = pred + (int64_t)c * nvox * 5;
    double* out = cdf + (int64_t)c * nvox;
    __shared__ double sh[4];
    const int v0 = t * CDF_TILE + threadIdx.x * 8;
    double w[8], run = 0.0;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int v = v0 + q;
        run += v < nvox ? pow(10.0, (double)p[(int64_t)v * 5]) : 0.0;
        w[q] = run;
    }
    double tot;
    const double ex = block_excl_scan256<double>(run, sh, &tot);
#pragma unroll
    for (int q = 0; q < 8; q++)
        if (v0 + q < nvox) out[v0 + q] = ex + w[q];
    if (threadIdx.x == 0) ttot[(int64_t)c * ntile + t] = tot;
}

__global__ __launch_bounds__(256) void k_cdf_offsets(int nvox, double* __restrict__ ttot) {
    const int c = blockIdx.x;
    const int ntile = (nvox + CDF_TILE - 1) / CDF_TILE;
    double* tt = ttot + (int64_t)c * ntile;
    __shared__ double sh[4];
    double carry = 0.0;
    for (int b = 0; b < ntile; b += 256) {
        const int t = b + threadIdx.x;
        const double w = t < ntile ? tt[t] : 0.0;
        double tot;
        const double ex = block_excl_scan256<double>(w, sh, &tot);
        __syncthreads();
        if (t < ntile) tt[t] = carry + ex;  // exclusive offset of tile t
        carry += tot;
    }
}

__global__ __launch_bounds__(256) void k_cdf_add(int nvox, const double* __restrict__ ttot,
                                                 double* __restrict__ cdf) {
    const int c = blockIdx.y, t = blockIdx.x;
    const int ntile = (nvox + CDF_TILE - 1) / CDF_TILE;
    const double off = ttot[(int64_t)c * ntile + t];
    double* out = cdf + (int64_t)c * nvox;
    for (int v = t * CDF_TILE + threadIdx.x; v < min(nvox, (t + 1) * CDF_TILE); v += 256) out[v] += off;
}

__global__ __launch_bounds__(256) void k_resample(
    int k, int grid, double half, const double* __restrict__ centers,
    const int32_t* __restrict__ out_off, const float* __restrict__ pred,
    const double* __restrict__ cdf, const float* __restrict__ uni, double T_to_u,
    double* __restrict__ x, double* __restrict__ y, double* __restrict__ z,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
    double* __restrict__ u) {
    const int c = blockIdx.y;
    const int b = out_off[c], e = out_off[c + 1];
    const int j = b + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= e) return;
    const int nvox = grid * grid * grid;
    const double* C = cdf + (int64_t)c * nvox;
    const double target = (double)uni[4 * (int64_t)j] * C[nvox - 1];
    int lo = 0, hi = nvox - 1;  // first voxel with C[v] > target
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (C[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    const int v = lo;
    const int X = v % grid, Y = (v / grid) % grid, Z = v / (grid * grid);
    const double dv = 2.0 * half / grid;
    x[j] = centers[3 * c] - half + (X + (double)uni[4 * (int64_t)j + 1]) * dv;
    y[j] = centers[3 * c + 1] - half + (Y + (double)uni[4 * (int64_t)j + 2]) * dv;
    z[j] = centers[3 * c + 2] - half + (Z + (double)uni[4 * (int64_t)j + 3]) * dv;
    const float* p = pred + ((int64_t)c * nvox + v) * 5;
    u[j] = pow(10.0, (double)p[1]) * T_to_u;
    vx[j] = p[2];
    vy[j] = p[3];
    vz[j] = p[4];
}

extern "C" int gx_sn_resample(gx_ctx* ctx, const float* pred, int k, int grid, double side,
                              const double* centers, const int32_t* out_off, int64_t n_out_max,
                              const float* uniforms, double T_to_u, double* x, double* y, double* z,
                              double* vx, double* vy, double* vz, double* u) {
    if (!ctx || !pred || !centers || !out_off || !uniforms || !x || !y || !z || !vx || !vy || !vz ||
        !u || k < 1 || grid < 1 || !(side > 0) || n_out_max < 0)
        return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int nvox = grid * grid * grid;
    const int ntile = (nvox + CDF_TILE - 1) / CDF_TILE;
    GX_TRY(gx_reserve(ctx, ctx->sph_work[11], (size_t)k * nvox * sizeof(double)));
    GX_TRY(gx_reserve(ctx, ctx->sph_work[7], (size_t)k * ntile * sizeof(double)));
    double* cdf = (double*)ctx->sph_work[11].p;
    double* ttot = (double*)ctx->sph_work[7].p;
    hipLaunchKernelGGL(k_cdf_tiles, dim3(ntile, k), dim3(256), 0, ctx->stream, pred, nvox, cdf, ttot);
    hipLaunchKernelGGL(k_cdf_offsets, dim3(k), dim3(256), 0, ctx->stream, nvox, ttot);
    hipLaunchKernelGGL(k_cdf_add, dim3(ntile, k), dim3(256), 0, ctx->stream, nvox,
                       (const double*)ttot, cdf);
    const unsigned gxb = (unsigned)std::max<int64_t>(1, (n_out_max + 255) / 256);
    hipLaunchKernelGGL(k_resample, dim3(gxb, k), dim3(256), 0, ctx->stream, k, grid, 0.5 * side,
                       centers, out_off, pred, cdf, uniforms, T_to_u, x, y, z, vx, vy, vz, u);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Gibbs resampling: a Markov chain per particle over the voxel indices.  The
// chain starts in the voxel of the particle that entered; each sweep redraws
// the x index from the weights 10^(log10 rho) along the line through the
// current (y, z), then y given (x, z), then z given (x, y).  Every line's
// inclusive prefix sums are formed once per call, sequentially in index order
// in FP64 (one thread per line), so each draw is a bisection of 64 entries
// and takes the same decision as a sequential sum written out plainly.
// ---------------------------------------------------------------------------
// Line prefix sums along `axis` (0: x, stride 1; 1: y, stride grid; 2: z,
// stride grid^2), stored at each voxel's own index.  Grid (lines / 256, k).
__global__ __launch_bounds__(256) void k_line_cdf(const float* __restrict__ pred, int grid,
                                                  int axis, double* __restrict__ cdf) {
    const int c = blockIdx.y;
    const int L = blockIdx.x * blockDim.x + threadIdx.x;
    const int g2 = grid * grid;
    if (L >= g2) return;
    const int64_t nvox = (int64_t)g2 * grid;
    int base, stride;
    if (axis == 0) {         // L = z * grid + y
        base = L * grid;
        stride = 1;
    } else if (axis == 1) {  // L = z * grid + x
        base = (L / grid) * g2 + (L % grid);
        stride = grid;
    } else {                 // L = y * grid + x
        base = L;
        stride = g2;
    }
    const float* p = pred + (int64_t)c * nvox * 5;
    double* out = cdf + (int64_t)c * nvox;
    double run = 0.0;
    for (int i = 0; i < grid; i++) {
        const int v = base + i * stride;
        run += pow(10.0, (double)p[(int64_t)v * 5]);
        out[v] = run;
    }
}

// first index i of the line whose prefix sum exceeds u * (line total); the
// last index when none does
__device__ __forceinline__ int line_pick(const double* __restrict__ C, int base, int stride,
                                         int grid, float u) {
    const double target = (double)u * C[base + (grid - 1) * stride];
    int lo = 0, hi = grid - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (C[base + mid * stride] > target) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_gibbs(
    int grid, double half, double dv, const double* __restrict__ centers,
    const int32_t* __restrict__ out_off, const float* __restrict__ pred,
    const double* __restrict__ cx_, const double* __restrict__ cy_,
    const double* __restrict__ cz_, const double* __restrict__ x0,
    const double* __restrict__ y0, const double* __restrict__ z0, int sweeps,
    const float* __restrict__ uni, double T_to_u, double* __restrict__ x,
    double* __restrict__ y, double* __restrict__ z, double* __restrict__ vx,
    double* __restrict__ vy, double* __restrict__ vz, double* __restrict__ u) {
#pragma clang fp contract(off)
    const int c = blockIdx.y;
    const int b = out_off[c], e = out_off[c + 1];
    const int j = b + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= e) return;
    const int g2 = grid * grid;
    const int64_t nvox = (int64_t)g2 * grid;
    const int64_t cb = (int64_t)c * nvox;
    const double lx = centers[3 * c] - half, ly = centers[3 * c + 1] - half,
                 lz = centers[3 * c + 2] - half;
    // start voxel: floor((x0 - lo) / dv), clamped to the grid
    auto cell = [&](double p, double lo) {
        const double f = floor((p - lo) / dv);
        return f < 0.0 ? 0 : (f > (double)(grid - 1) ? grid - 1 : (int)f);
    };
    int X = cell(x0[j], lx), Y = cell(y0[j], ly), Z = cell(z0[j], lz);
    const int nu = 3 * sweeps + 3;
    const float* U = uni + (int64_t)j * nu;
    for (int s = 0; s < sweeps; s++) {
        X = line_pick(cx_ + cb, (Z * grid + Y) * grid, 1, grid, U[3 * s]);
        Y = line_pick(cy_ + cb, Z * g2 + X, grid, grid, U[3 * s + 1]);
        Z = line_pick(cz_ + cb, Y * grid + X, g2, grid, U[3 * s + 2]);
    }
    const int v = (Z * grid + Y) * grid + X;
    x[j] = lx + (X + (double)U[3 * sweeps]) * dv;
    y[j] = ly + (Y + (double)U[3 * sweeps + 1]) * dv;
    z[j] = lz + (Z + (double)U[3 * sweeps + 2]) * dv;
    const float* p = pred + (cb + v) * 5;
    u[j] = pow(10.0, (double)p[1]) * T_to_u;
    vx[j] = p[2];
    vy[j] = p[3];
    vz[j] = p[4];
}

extern "C" int gx_sn_resample_gibbs(gx_ctx* ctx, const float* pred, int k, int grid, double side,
                                    const double* centers, const int32_t* out_off,
                                    int64_t n_out_max, const double* x0, const double* y0,
                                    const double* z0, int sweeps, const float* uniforms,
                                    double T_to_u, double* x, double* y, double* z, double* vx,
                                    double* vy, double* vz, double* u) {
    if (!ctx) return GX_EINVAL;
    if (!pred || !centers || !out_off || !x0 || !y0 || !z0 || !uniforms || !x || !y || !z ||
        !vx || !vy || !vz || !u)
        return gx_fail(ctx, GX_EINVAL, "sn_resample_gibbs: null pointer");
    if (k < 1 || grid < 1 || grid > 1024 || !(side > 0) || n_out_max < 0 || sweeps < 0 ||
        sweeps > 1000)
        return gx_fail(ctx, GX_EINVAL, "sn_resample_gibbs: need k >= 1, 1 <= grid <= 1024, "
                                       "side > 0, n_out_max >= 0, 0 <= sweeps <= 1000");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t nvox = (int64_t)grid * grid * grid;
    GX_TRY(gx_reserve(ctx, ctx->sph_work[11], (size_t)3 * k * nvox * sizeof(double)));
    double* cdf = (double*)ctx->sph_work[11].p;
    const int lines = grid * grid;
    for (int a = 0; a < 3; a++)
        hipLaunchKernelGGL(k_line_cdf, dim3((lines + 255) / 256, k), dim3(256), 0, ctx->stream,
                           pred, grid, a, cdf + (int64_t)a * k * nvox);
    const unsigned gxb = (unsigned)std::max<int64_t>(1, (n_out_max + 255) / 256);
    hipLaunchKernelGGL(k_gibbs, dim3(gxb, k), dim3(256), 0, ctx->stream, grid, 0.5 * side,
                       side / grid, centers, out_off, pred, (const double*)cdf,
                       (const double*)(cdf + k * nvox), (const double*)(cdf + 2 * k * nvox), x0,
                       y0, z0, sweeps, uniforms, T_to_u, x, y, z, vx, vy, vz, u);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Eight-cube encoding of the network's channels: log10 rho, log10 T, then per
// velocity component log10(v0 + max(v, 0)) and log10(v0 + max(-v, 0)); the
// inverse takes v = 10^(c+) - 10^(c-).  Formed in FP64, stored in FP32.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_encode8(int64_t V, const float* __restrict__ in,
                                                 int in_stride, double v0,
                                                 float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const float* p = in + i * in_stride;
    float* o = out + i * 8;
    o[0] = p[0];
    o[1] = p[1];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double v = (double)p[2 + a];
        o[2 + 2 * a] = (float)log10(v0 + fmax(v, 0.0));
        o[3 + 2 * a] = (float)log10(v0 + fmax(-v, 0.0));
    }
}

__global__ __launch_bounds__(256) void k_decode8(int64_t V, const float* __restrict__ in,
                                                 int in_stride, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const float* p = in + i * in_stride;
    float* o = out + i * 5;
    o[0] = p[0];
    o[1] = p[1];
#pragma unroll
    for (int a = 0; a < 3; a++)
        o[2 + a] = (float)(pow(10.0, (double)p[2 + 2 * a]) - pow(10.0, (double)p[3 + 2 * a]));
}

extern "C" int gx_sn_encode8(gx_ctx* ctx, int64_t V, const float* in5, int in_stride, double v0,
                             float* out8) {
    if (!ctx) return GX_EINVAL;
    if (V < 0 || !in5 || !out8 || in_stride < 5 || !(v0 > 0))
        return gx_fail(ctx, GX_EINVAL, "sn_encode8: need V >= 0, in_stride >= 5, v0 > 0");
    if (V == 0) return GX_OK;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_encode8, dim3(gx_blocks(V, 256)), dim3(256), 0, ctx->stream, V, in5,
                       in_stride, v0, out8);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_sn_decode8(gx_ctx* ctx, int64_t V, const float* in8, int in_stride,
                             float* out5) {
    if (!ctx) return GX_EINVAL;
    if (V < 0 || !in8 || !out5 || in_stride < 8)
        return gx_fail(ctx, GX_EINVAL, "sn_decode8: need V >= 0, in_stride >= 8");
    if (V == 0) return GX_OK;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_decode8, dim3(gx_blocks(V, 256)), dim3(256), 0, ctx->stream, V, in8,
                       in_stride, out5);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Trust check of a prediction before replacement.
// ---------------------------------------------------------------------------
struct SnBounds {
    float lo[5], hi[5];
};

// Grid (blocks per region, k): region c is marked in bad[c] when any value of
// its [grid^3][5] block is not finite or outside [lo[ch], hi[ch]].
__global__ __launch_bounds__(256) void k_sn_check(const float* __restrict__ pred, int per,
                                                  SnBounds bd, uint32_t* __restrict__ bad) {
    const float* p = pred + (int64_t)blockIdx.y * per;
    bool good = true;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < per; e += gridDim.x * blockDim.x) {
        const float v = p[e];
        const int ch = e % 5;
        float lo = bd.lo[0], hi = bd.hi[0];
#pragma unroll
        for (int q = 1; q < 5; q++)
            if (ch == q) {
                lo = bd.lo[q];
                hi = bd.hi[q];
            }
        good = good && isfinite(v) && v >= lo && v <= hi;
    }
    if (!__syncthreads_and(good ? 1 : 0) && threadIdx.x == 0) atomicOr(&bad[blockIdx.y], 1u);
}

extern "C" int gx_sn_check(gx_ctx* ctx, const float* pred, int k, int grid, const double* lo,
                           const double* hi, uint8_t* ok) {
    if (!ctx || k < 0 || grid < 1 || !lo || !hi || (k > 0 && (!pred || !ok))) return GX_EINVAL;
    const int64_t per = (int64_t)grid * grid * grid * 5;
    if (per > INT32_MAX) return gx_fail(ctx, GX_EINVAL, "sn_check: grid %d too large", grid);
    if (k == 0) return GX_OK;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    SnBounds bd;
    for (int q = 0; q < 5; q++) {
        bd.lo[q] = (float)lo[q];
        bd.hi[q] = (float)hi[q];
    }
    GX_TRY(gx_reserve(ctx, ctx->sph_work[21], (size_t)k * sizeof(uint32_t)));
    uint32_t* bad = (uint32_t*)ctx->sph_work[21].p;
    GX_TRY(gx_zero(ctx, bad, (size_t)k * sizeof(uint32_t)));
    const unsigned nbx = (unsigned)std::min<int64_t>(64, (per + 255) / 256);
    hipLaunchKernelGGL(k_sn_check, dim3(nbx, k), dim3(256), 0, ctx->stream, pred, (int)per, bd, bad);
    GX_LAUNCH_CHECK(ctx);
    std::vector<uint32_t> h(k);
    GX_HIP(ctx, hipMemcpyAsync(h.data(), bad, (size_t)k * sizeof(uint32_t), hipMemcpyDeviceToHost,
                               ctx->stream));
    GX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < k; c++) ok[c] = h[c] ? 0 : 1;
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Trust check without allocation (gx_sn_check_noalloc), for callers that
// cannot allocate device memory.  Its scratch, one flag word per region, is
// the static device array `scratch` below: every device the library runs on
// holds its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory, so its device address is taken once
// per device by gx_noalloc_setup (called from gx_create with the device
// current) and only that address is handed to kernels.
// ---------------------------------------------------------------------------
#define GX_NOALLOC_MAX_DEVICES 64
static __device__ __align__(256) uint32_t scratch[GX_NOALLOC_MAX_REGIONS];
static void* g_scratch_dev[GX_NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

int gx_noalloc_setup(gx_ctx* ctx) {
    if (ctx->device < 0 || ctx->device >= GX_NOALLOC_MAX_DEVICES)
        return gx_fail(ctx, GX_EINVAL, "device %d beyond the static scratch table", ctx->device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[ctx->device]) return GX_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return gx_fail(ctx, GX_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", ctx->device,
                       hipGetErrorString(e));
    }
    g_scratch_dev[ctx->device] = p;
    return GX_OK;
}

__global__ void k_flags_clear(uint32_t* __restrict__ bad, int k) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < k) bad[c] = 0u;
}

__global__ void k_flags_to_ok(const uint32_t* __restrict__ bad, int k, uint8_t* __restrict__ ok) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < k) ok[c] = bad[c] ? 0 : 1;
}

extern "C" int gx_sn_check_noalloc(gx_ctx* ctx, const float* pred, int k, int grid,
                                   const double* lo, const double* hi, uint8_t* ok_dev) {
    if (!ctx || k < 0 || grid < 1 || !lo || !hi || (k > 0 && (!pred || !ok_dev))) return GX_EINVAL;
    if (k > GX_NOALLOC_MAX_REGIONS)
        return gx_fail(ctx, GX_EINVAL,
                       "sn_check_noalloc: %d regions exceed the static scratch of %d regions", k,
                       GX_NOALLOC_MAX_REGIONS);
    const int64_t per = (int64_t)grid * grid * grid * 5;
    if (per > INT32_MAX) return gx_fail(ctx, GX_EINVAL, "sn_check_noalloc: grid %d too large", grid);
    if (k == 0) return GX_OK;
    uint32_t* bad = (uint32_t*)g_scratch_dev[ctx->device];
    if (!bad) return gx_fail(ctx, GX_EINVAL, "sn_check_noalloc: no scratch address for device %d",
                             ctx->device);
    GX_HIP(ctx, hipSetDevice(ctx->device));
    SnBounds bd;
    for (int q = 0; q < 5; q++) {
        bd.lo[q] = (float)lo[q];
        bd.hi[q] = (float)hi[q];
    }
    hipLaunchKernelGGL(k_flags_clear, dim3(gx_blocks(k, 256)), dim3(256), 0, ctx->stream, bad, k);
    const unsigned nbx = (unsigned)std::min<int64_t>(64, (per + 255) / 256);
    hipLaunchKernelGGL(k_sn_check, dim3(nbx, k), dim3(256), 0, ctx->stream, pred, (int)per, bd, bad);
    hipLaunchKernelGGL(k_flags_to_ok, dim3(gx_blocks(k, 256)), dim3(256), 0, ctx->stream,
                       (const uint32_t*)bad, k, ok_dev);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Replacement by particle ID (Sec. 3.2 step 4).
// ---------------------------------------------------------------------------
__global__ void k_id_map(int64_t n, const int64_t* __restrict__ id, int64_t id_cap,
                         int32_t* __restrict__ map) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && id[i] >= 0 && id[i] < id_cap) map[id[i]] = (int32_t)i;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// A main index targeted by several new particles (an ID listed twice) takes
// the last of them: each new particle claims its target with atomicMax of its
// list position, and only the winner writes.
__global__ void k_replace_claim(int64_t m, const int64_t* __restrict__ nid,
                                const int32_t* __restrict__ map, int64_t id_cap,
                                int32_t* __restrict__ win) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t id = nid[k];
    const int32_t i = (id >= 0 && id < id_cap) ? map[id] : -1;
    if (i >= 0) atomicMax(&win[i], (int32_t)k);
}

__global__ void k_replace(int64_t m, const int64_t* __restrict__ nid, const double* __restrict__ nx,
                          const double* __restrict__ ny, const double* __restrict__ nz,
                          const double* __restrict__ nvx, const double* __restrict__ nvy,
                          const double* __restrict__ nvz, const double* __restrict__ nu,
                          const int32_t* __restrict__ map, int64_t id_cap, double* __restrict__ x,
                          double* __restrict__ y, double* __restrict__ z, double* __restrict__ vx,
                          double* __restrict__ vy, double* __restrict__ vz, double* __restrict__ u,
                          int64_t u_off, double* __restrict__ H64,
                          const int32_t* __restrict__ win, unsigned long long* missing) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t id = nid[k];
    const int32_t i = (id >= 0 && id < id_cap) ? map[id] : -1;
    if (i < 0) {
        atomicAdd(missing, 1ull);
        return;
    }
    if (win[i] != (int32_t)k) return;  // a later entry with the same ID wins
    x[i] = nx[k];
    y[i] = ny[k];
    z[i] = nz[k];
    vx[i] = nvx[k];
    vy[i] = nvy[k];
    vz[i] = nvz[k];
    if (u && i >= u_off) u[i - u_off] = nu[k];
    if (H64 && i >= u_off) H64[i - u_off] = -1.0;
}

extern "C" int gx_sn_replace(gx_ctx* ctx, int64_t n, const int64_t* id, int64_t id_cap, double* x,
                             double* y, double* z, double* vx, double* vy, double* vz, double* u,
                             int64_t u_offset, double* H64, int64_t m, const int64_t* new_id,
                             const double* nx, const double* ny, const double* nz,
                             const double* nvx, const double* nvy, const double* nvz,
                             const double* nu, int64_t* n_missing) {
    if (!ctx || !id || !x || !y || !z || !vx || !vy || !vz || n < 0 || m < 0 || id_cap < 1)
        return GX_EINVAL;
    if (m > 0 && (!new_id || !nx || !ny || !nz || !nvx || !nvy || !nvz || (u && !nu)))
        return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (m > INT32_MAX || n > INT32_MAX)
        return gx_fail(ctx, GX_EINVAL, "sn_replace: more than 2^31 - 1 particles");
    GX_TRY(gx_reserve(ctx, ctx->sph_work[12], id_cap * sizeof(int32_t)));
    GX_TRY(gx_reserve(ctx, ctx->sph_work[22], std::max<int64_t>(n, 1) * sizeof(int32_t)));
    GX_TRY(gx_reserve(ctx, ctx->small, 64));
    int32_t* map = (int32_t*)ctx->sph_work[12].p;
    int32_t* win = (int32_t*)ctx->sph_work[22].p;
    unsigned long long* miss = (unsigned long long*)ctx->small.p;
    GX_TRY(gx_zero(ctx, miss, 8));
    hipLaunchKernelGGL(k_fill_i32, dim3(gx_blocks(id_cap, 256)), dim3(256), 0, st, map, id_cap, -1);
    hipLaunchKernelGGL(k_id_map, dim3(gx_blocks(n, 256)), dim3(256), 0, st, n, id, id_cap, map);
    if (m > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(gx_blocks(n, 256)), dim3(256), 0, st, win, n, -1);
        hipLaunchKernelGGL(k_replace_claim, dim3(gx_blocks(m, 256)), dim3(256), 0, st, m, new_id,
                           (const int32_t*)map, id_cap, win);
        hipLaunchKernelGGL(k_replace, dim3(gx_blocks(m, 256)), dim3(256), 0, st, m, new_id, nx, ny, nz,
                           nvx, nvy, nvz, nu, map, id_cap, x, y, z, vx, vy, vz, u, u_offset, H64,
                           (const int32_t*)win, miss);
    }
    GX_LAUNCH_CHECK(ctx);
    if (n_missing) {
        unsigned long long h = 0;
        GX_HIP(ctx, hipMemcpyAsync(&h, miss, 8, hipMemcpyDeviceToHost, st));
        GX_HIP(ctx, hipStreamSynchronize(st));
        *n_missing = (int64_t)h;
    }
    return GX_OK;
}
