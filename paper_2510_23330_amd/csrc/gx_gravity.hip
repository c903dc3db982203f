// gx_gravity.hip -- tree gravity: list construction driver and the pairwise
// kernel (Eq. 1, monopole + quadrupole cells) in the mixed-precision form of
// Sec. 4.3: per receiving group, coordinates are made relative to the
// group's box centre in FP64 and rounded to FP32; pair terms are summed in
// FP32 over one LDS tile (<= 256 sources) and tiles are combined in FP64.
//
// Work layout (CDNA4, wave64): one workgroup of 256 threads per group.  A
// group holds nG <= n_group receivers; the workgroup is split into
// 256 / pad slices (pad = 64, 128 or 256 >= nG), each slice holding every
// receiver once (one per lane) and taking its own share of each source
// tile, so small groups still fill the lanes; the slices' partial sums are
// combined through LDS at the end.  Every wave lies inside one slice, so all
// lanes of a wave read the same source from LDS (a broadcast).  Sources are
// staged cooperatively: opened-leaf particle ranges are expanded into an
// index chunk in LDS, then each thread loads one source, converts it to
// group-relative FP32 and stores it into structure-of-arrays LDS tiles.
// No MFMA: the pair law is not a contraction.
#include "gx_internal.hpp"

int gx_tree_check(gx_ctx* ctx, int which, const gx_particles* p);

__global__ __launch_bounds__(128) void k_walk_grav(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes, int nn,
    const double* __restrict__ box, double theta2, int mode, uint32_t* __restrict__ pc_cnt,
    uint32_t* __restrict__ pr_cnt, uint32_t* __restrict__ pp_tot,
    unsigned long long* __restrict__ tot, const int64_t* __restrict__ pc_off,
    int32_t* __restrict__ pc_list, const int64_t* __restrict__ pr_off,
    int32_t* __restrict__ pr_begin, int32_t* __restrict__ pr_cum);
__global__ void k_direct_lists(int ng, int n, const int32_t* __restrict__ groups,
                               const NodeRec* __restrict__ nodes, int64_t* __restrict__ pc_off,
                               int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
                               int32_t* __restrict__ pr_cum, uint32_t* __restrict__ pp_tot,
                               unsigned long long* __restrict__ tot);

#define GF_THREADS 256
#define GF_TILE 256
#define GF_CH 2048

template <typename T>
__device__ __forceinline__ T pair_rsqrt(T x);
template <>
__device__ __forceinline__ float pair_rsqrt<float>(float x) {
    return __builtin_amdgcn_rsqf(x);
}
template <>
__device__ __forceinline__ double pair_rsqrt<double>(double x) {
    return 1.0 / sqrt(x);
}

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
    T x, y, z, w;
};

template <typename T, bool QUAD>
__global__ __launch_bounds__(GF_THREADS) void k_grav_force(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const MomRec* __restrict__ mom, const double4* __restrict__ pos4, const float* __restrict__ e2s,
    const uint32_t* __restrict__ perm, const int64_t* __restrict__ pc_off,
    const int32_t* __restrict__ pc_list, const int64_t* __restrict__ pr_off,
    const int32_t* __restrict__ pr_begin, const int32_t* __restrict__ pr_cum,
    const uint32_t* __restrict__ pp_tot, double G, double* __restrict__ ax, double* __restrict__ ay,
    double* __restrict__ az, double* __restrict__ pot) {
    const int g = xcd_remap(blockIdx.x, ng);
    if (g >= ng) return;
    __shared__ int32_t jidx[GF_CH];
    // source tiles: A = (x, y, z, m) group-relative; B = (eps^2, qxx, qyy, qzz);
    // C = (qxy, qxz, qyz, -)
    __shared__ V4<T> sA[GF_TILE], sB[GF_TILE];
    __shared__ V4<T> sC[QUAD ? GF_TILE : 1];
    __shared__ double red[4][GF_THREADS];

    const int tid = threadIdx.x;
    const NodeRec gn = nodes[groups[g]];
    const int gb = gn.begin, nG = gn.end - gn.begin;
    const double cx = (gn.lo[0] + gn.hi[0]) * 0.5;
    const double cy = (gn.lo[1] + gn.hi[1]) * 0.5;
    const double cz = (gn.lo[2] + gn.hi[2]) * 0.5;
    // slices: pad lanes hold the receivers once; 256 / pad slices split each tile
    int pad = 32;
    while (pad < nG && pad < GF_THREADS) pad <<= 1;
    const int nsl = GF_THREADS / pad, il = tid % pad, sl = tid / pad;
    const int npp = (int)pp_tot[g];
    const int64_t r0 = pr_off[g], r1 = pr_off[g + 1];
    const int64_t c0 = pc_off[g], c1 = pc_off[g + 1];

    for (int ic = 0; ic < nG; ic += pad) {
        const int i = ic + il;
        const bool act = i < nG;
        T xi = 0, yi = 0, zi = 0, ei = 0, mi = 0;
        if (act) {
            double4 p = pos4[gb + i];
            xi = (T)(p.x - cx);
            yi = (T)(p.y - cy);
            zi = (T)(p.z - cz);
            mi = (T)p.w;
            ei = (T)e2s[gb + i];
        }
        double AX = 0, AY = 0, AZ = 0, PT = 0;

        // ---- particle-particle part: opened leaves -------------------------
        for (int ch = 0; ch < npp; ch += GF_CH) {
            const int che = min(npp, ch + GF_CH);
            __syncthreads();
            for (int64_t r = r0 + tid; r < r1; r += GF_THREADS) {
                const int c = pr_cum[r];
                const int cn = (r + 1 < r1) ? pr_cum[r + 1] : npp;
                const int b = pr_begin[r];
                const int lo = max(c, ch), hi = min(cn, che);
                for (int k = lo; k < hi; k++) jidx[k - ch] = b + (k - c);
            }
            __syncthreads();
            for (int t0 = ch; t0 < che; t0 += GF_TILE) {
                const int tn = min(GF_TILE, che - t0);
                if (tid < tn) {
                    const int j = jidx[t0 - ch + tid];
                    const double4 p = pos4[j];
                    sA[tid] = V4<T>{(T)(p.x - cx), (T)(p.y - cy), (T)(p.z - cz), (T)p.w};
                    sB[tid].x = (T)e2s[j];
                }
                __syncthreads();
                if (act) {
                    T fx = 0, fy = 0, fz = 0, fp = 0;
                    const int per = (tn + nsl - 1) / nsl;
                    const int jb = sl * per, je = min(tn, jb + per);
#pragma unroll 4
                    for (int jj = jb; jj < je; jj++) {
                        const V4<T> a = sA[jj];
                        const T dx = a.x - xi, dy = a.y - yi, dz = a.z - zi;
                        const T r2 = dx * dx + dy * dy + dz * dz + (ei + sB[jj].x);
                        const T rinv = pair_rsqrt<T>(r2);
                        const T mr = a.w * rinv;
                        const T mr3 = mr * rinv * rinv;
                        fx += mr3 * dx;
                        fy += mr3 * dy;
                        fz += mr3 * dz;
                        fp -= mr;
                    }
                    AX += (double)fx;
                    AY += (double)fy;
                    AZ += (double)fz;
                    PT += (double)fp;
                }
                __syncthreads();
            }
        }

        // ---- particle-cell part: accepted cells -----------------------------
        for (int64_t t0 = c0; t0 < c1; t0 += GF_TILE) {
            const int tn = (int)min((int64_t)GF_TILE, c1 - t0);
            if (tid < tn) {
                const MomRec mr = mom[pc_list[t0 + tid]];
                sA[tid] = V4<T>{(T)(mr.cx - cx), (T)(mr.cy - cy), (T)(mr.cz - cz), (T)mr.M};
                if (QUAD) {
                    sB[tid] = V4<T>{(T)mr.e2, (T)mr.q[0], (T)mr.q[1], (T)mr.q[2]};
                    sC[tid] = V4<T>{(T)mr.q[3], (T)mr.q[4], (T)mr.q[5], (T)0};
                } else {
                    sB[tid].x = (T)mr.e2;
                }
            }
            __syncthreads();
            if (act) {
                T fx = 0, fy = 0, fz = 0, fp = 0;
                const int per = (tn + nsl - 1) / nsl;
                const int jb = sl * per, je = min(tn, jb + per);
#pragma unroll 2
                for (int jj = jb; jj < je; jj++) {
                    const V4<T> a = sA[jj];
                    const V4<T> b = sB[jj];
                    const T dx = a.x - xi, dy = a.y - yi, dz = a.z - zi;
                    const T R2 = dx * dx + dy * dy + dz * dz + (ei + b.x);
                    const T Rinv = pair_rsqrt<T>(R2);
                    const T Rinv2 = Rinv * Rinv;
                    const T M = a.w;
                    const T Rinv3 = Rinv * Rinv2;
                    const T MR3 = M * Rinv3;
                    if (QUAD) {
                        const V4<T> c = sC[jj];
                        const T qdx = b.y * dx + c.x * dy + c.y * dz;
                        const T qdy = c.x * dx + b.z * dy + c.z * dz;
                        const T qdz = c.y * dx + c.z * dy + b.w * dz;
                        const T dqd = dx * qdx + dy * qdy + dz * qdz;
                        const T Rinv5 = Rinv3 * Rinv2;
                        const T u5 = dqd * Rinv5;
                        const T coef = MR3 + (T)2.5 * u5 * Rinv2;
                        fx += coef * dx - Rinv5 * qdx;
                        fy += coef * dy - Rinv5 * qdy;
                        fz += coef * dz - Rinv5 * qdz;
                        fp -= M * Rinv + (T)0.5 * u5;
                    } else {
                        fx += MR3 * dx;
                        fy += MR3 * dy;
                        fz += MR3 * dz;
                        fp -= M * Rinv;
                    }
                }
                AX += (double)fx;
                AY += (double)fy;
                AZ += (double)fz;
                PT += (double)fp;
            }
            __syncthreads();
        }

        // ---- combine slices, remove the self pair's potential, write ---------
        red[0][tid] = AX;
        red[1][tid] = AY;
        red[2][tid] = AZ;
        red[3][tid] = PT;
        __syncthreads();
        if (sl == 0 && act) {
            for (int s = 1; s < nsl; s++) {
                AX += red[0][s * pad + il];
                AY += red[1][s * pad + il];
                AZ += red[2][s * pad + il];
                PT += red[3][s * pad + il];
            }
            if (npp > 0) PT += (double)(mi * pair_rsqrt<T>(ei + ei));
            const uint32_t o = perm[gb + i];
            ax[o] = G * AX;
            ay[o] = G * AY;
            az[o] = G * AZ;
            pot[o] = G * PT;
        }
        __syncthreads();
    }
}

static int read_host(gx_ctx* ctx, void* dst, const void* src, size_t bytes) {
    GX_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
    GX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GX_OK;
}

extern "C" int gx_gravity_forces(gx_ctx* ctx, const gx_particles* p, double G, double theta,
                                 int flags, double* ax, double* ay, double* az, double* pot,
                                 gx_stats* stats) {
    if (!ctx || !p || !ax || !ay || !az || !pot) return gx_fail(ctx, GX_EINVAL, "null argument");
    if (flags & ~(GX_QUAD | GX_DIRECT | GX_PREC_FP64)) return gx_fail(ctx, GX_EINVAL, "bad flags");
    if (!(flags & GX_DIRECT) && !(theta > 0.0)) return gx_fail(ctx, GX_EINVAL, "theta must be > 0");
    if (!p->eps2) return gx_fail(ctx, GX_EINVAL, "gravity needs eps2");
    GX_TRY(gx_tree_check(ctx, GX_TREE_ALL, p));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    TreeSlot& T = ctx->tree[GX_TREE_ALL];
    ListSet& Ls = ctx->grav;
    const int ng = (int)T.n_groups, nn = (int)T.n_nodes;
    if (stats) {
        *stats = gx_stats{};
        GX_HIP(ctx, hipEventRecord(ctx->ev0, st));
    }
    GX_TRY(gx_reserve(ctx, Ls.tot, 8 * sizeof(int64_t)));
    GX_TRY(gx_zero(ctx, Ls.tot.p, 8 * sizeof(int64_t)));
    GX_TRY(gx_reserve(ctx, Ls.pc_cnt, (ng + 1) * sizeof(uint32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pr_cnt, (ng + 1) * sizeof(uint32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pp_tot, (ng + 1) * sizeof(uint32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pc_off, (ng + 1) * sizeof(int64_t)));
    GX_TRY(gx_reserve(ctx, Ls.pr_off, (ng + 1) * sizeof(int64_t)));
    int64_t* tot = (int64_t*)Ls.tot.p;
    int64_t h_tot[8] = {};
    if (flags & GX_DIRECT) {
        GX_TRY(gx_reserve(ctx, Ls.pr_begin, (ng + 1) * sizeof(int32_t)));
        GX_TRY(gx_reserve(ctx, Ls.pr_cum, (ng + 1) * sizeof(int32_t)));
        GX_TRY(gx_reserve(ctx, Ls.pc_list, 64));
        hipLaunchKernelGGL(k_direct_lists, dim3(gx_blocks(ng + 1, 256)), dim3(256), 0, st, ng,
                           (int)T.n, (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                           (int64_t*)Ls.pc_off.p, (int64_t*)Ls.pr_off.p, (int32_t*)Ls.pr_begin.p,
                           (int32_t*)Ls.pr_cum.p, (uint32_t*)Ls.pp_tot.p,
                           (unsigned long long*)tot);
        GX_LAUNCH_CHECK(ctx);
        Ls.n_pc = 0;
        Ls.n_ranges = ng;
    } else {
        const double theta2 = theta * theta;
        hipLaunchKernelGGL(k_walk_grav, dim3(gx_blocks(ng, 128)), dim3(128), 0, st, ng,
                           (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p, nn,
                           (const double*)T.box.p, theta2, 0, (uint32_t*)Ls.pc_cnt.p,
                           (uint32_t*)Ls.pr_cnt.p, (uint32_t*)Ls.pp_tot.p,
                           (unsigned long long*)tot, nullptr, nullptr, nullptr, nullptr, nullptr);
        GX_LAUNCH_CHECK(ctx);
        GX_TRY((gx_scan<uint32_t, int64_t>(ctx, (const uint32_t*)Ls.pc_cnt.p, (int64_t*)Ls.pc_off.p,
                                           ng, tot + 0)));
        GX_TRY((gx_scan<uint32_t, int64_t>(ctx, (const uint32_t*)Ls.pr_cnt.p, (int64_t*)Ls.pr_off.p,
                                           ng, tot + 1)));
        // the offsets arrays carry their totals as element ng
        GX_HIP(ctx, hipMemcpyAsync((int64_t*)Ls.pc_off.p + ng, tot + 0, 8, hipMemcpyDeviceToDevice, st));
        GX_HIP(ctx, hipMemcpyAsync((int64_t*)Ls.pr_off.p + ng, tot + 1, 8, hipMemcpyDeviceToDevice, st));
        GX_TRY(read_host(ctx, h_tot, tot, 2 * sizeof(int64_t)));
        Ls.n_pc = h_tot[0];
        Ls.n_ranges = h_tot[1];
        GX_TRY(gx_reserve(ctx, Ls.pc_list, (Ls.n_pc + 1) * sizeof(int32_t)));
        GX_TRY(gx_reserve(ctx, Ls.pr_begin, (Ls.n_ranges + 1) * sizeof(int32_t)));
        GX_TRY(gx_reserve(ctx, Ls.pr_cum, (Ls.n_ranges + 1) * sizeof(int32_t)));
        hipLaunchKernelGGL(k_walk_grav, dim3(gx_blocks(ng, 128)), dim3(128), 0, st, ng,
                           (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p, nn,
                           (const double*)T.box.p, theta2, 1, nullptr, nullptr, nullptr, nullptr,
                           (const int64_t*)Ls.pc_off.p, (int32_t*)Ls.pc_list.p,
                           (const int64_t*)Ls.pr_off.p, (int32_t*)Ls.pr_begin.p,
                           (int32_t*)Ls.pr_cum.p);
        GX_LAUNCH_CHECK(ctx);
    }
    Ls.n_groups = ng;

    const bool quad = (flags & GX_QUAD) && !(flags & GX_DIRECT);
    const bool fp64 = flags & GX_PREC_FP64;
    auto args = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(xcd_grid(ng)), dim3(GF_THREADS), 0, st, ng,
                           (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                           (const MomRec*)T.mom.p, (const double4*)T.pos4.p, (const float*)T.e2s.p,
                           (const uint32_t*)T.val[0].p, (const int64_t*)Ls.pc_off.p,
                           (const int32_t*)Ls.pc_list.p, (const int64_t*)Ls.pr_off.p,
                           (const int32_t*)Ls.pr_begin.p, (const int32_t*)Ls.pr_cum.p,
                           (const uint32_t*)Ls.pp_tot.p, G, ax, ay, az, pot);
    };
    if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev2, st));
    if (fp64) {
        if (quad) args(k_grav_force<double, true>);
        else args(k_grav_force<double, false>);
    } else {
        if (quad) args(k_grav_force<float, true>);
        else args(k_grav_force<float, false>);
    }
    GX_LAUNCH_CHECK(ctx);
    if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev3, st));
    if (stats) {
        GX_HIP(ctx, hipEventRecord(ctx->ev1, st));
        GX_HIP(ctx, hipEventSynchronize(ctx->ev1));
        float ms = 0;
        GX_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        float msk = 0;
        GX_HIP(ctx, hipEventElapsedTime(&msk, ctx->ev2, ctx->ev3));
        GX_TRY(read_host(ctx, h_tot, tot, 4 * sizeof(int64_t)));
        stats->ms = ms;
        stats->ms_kernel = msk;
        stats->n_pp = h_tot[2];
        stats->n_pc = h_tot[3];
        stats->n_groups = ng;
        stats->n_nodes = nn;
    }
    return GX_OK;
}

extern "C" int gx_gravity_list_sizes(gx_ctx* ctx, int64_t* n_groups, int64_t* n_pc,
                                     int64_t* n_pp_ranges) {
    if (!ctx) return GX_EINVAL;
    if (n_groups) *n_groups = ctx->grav.n_groups;
    if (n_pc) *n_pc = ctx->grav.n_pc;
    if (n_pp_ranges) *n_pp_ranges = ctx->grav.n_ranges;
    return GX_OK;
}

extern "C" int gx_gravity_list_export(gx_ctx* ctx, int64_t* pc_off, int32_t* pc_node,
                                      int64_t* pp_off, int32_t* pp_begin, int32_t* pp_end) {
    if (!ctx) return GX_EINVAL;
    ListSet& Ls = ctx->grav;
    const int64_t ng = Ls.n_groups;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    GX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (pc_off) GX_HIP(ctx, hipMemcpy(pc_off, Ls.pc_off.p, (ng + 1) * 8, hipMemcpyDeviceToHost));
    if (pc_node && Ls.n_pc)
        GX_HIP(ctx, hipMemcpy(pc_node, Ls.pc_list.p, Ls.n_pc * 4, hipMemcpyDeviceToHost));
    if (pp_off) GX_HIP(ctx, hipMemcpy(pp_off, Ls.pr_off.p, (ng + 1) * 8, hipMemcpyDeviceToHost));
    if (pp_begin || pp_end) {
        int64_t nr = Ls.n_ranges;
        int32_t* b = (int32_t*)malloc((nr + 1) * 4);
        int32_t* c = (int32_t*)malloc((nr + 1) * 4);
        int64_t* off = (int64_t*)malloc((ng + 1) * 8);
        uint32_t* tot = (uint32_t*)malloc((ng + 1) * 4);
        if (!b || !c || !off || !tot) {
            free(b); free(c); free(off); free(tot);
            return gx_fail(ctx, GX_ENOMEM, "host malloc");
        }
        hipError_t e1 = hipMemcpy(b, Ls.pr_begin.p, nr * 4, hipMemcpyDeviceToHost);
        hipError_t e2 = hipMemcpy(c, Ls.pr_cum.p, nr * 4, hipMemcpyDeviceToHost);
        hipError_t e3 = hipMemcpy(off, Ls.pr_off.p, (ng + 1) * 8, hipMemcpyDeviceToHost);
        hipError_t e4 = hipMemcpy(tot, Ls.pp_tot.p, ng * 4, hipMemcpyDeviceToHost);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
            free(b); free(c); free(off); free(tot);
            return gx_fail(ctx, GX_EHIP, "list export copy failed");
        }
        for (int64_t g = 0; g < ng; g++)
            for (int64_t r = off[g]; r < off[g + 1]; r++) {
                int32_t cn = (r + 1 < off[g + 1]) ? c[r + 1] : (int32_t)tot[g];
                if (pp_begin) pp_begin[r] = b[r];
                if (pp_end) pp_end[r] = b[r] + (cn - c[r]);
            }
        free(b); free(c); free(off); free(tot);
    }
    return GX_OK;
}
