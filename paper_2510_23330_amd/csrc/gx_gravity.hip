// gx_gravity.hip -- tree gravity: list construction driver and the pairwise
// kernel (Eq. 1, monopole + quadrupole cells) in the mixed-precision form of
// Sec. 4.3: per receiving group, coordinates are made relative to the
// group's box centre in FP64 and rounded to FP32; pair terms are summed in
// FP32 over one LDS tile (<= 256 sources) and tiles are combined in FP64.
//
// Work layout (CDNA4, wave64): one workgroup of 512 threads per group.  A
// group holds nG <= n_group receivers; the workgroup is split into
// floor(512 / nG) slices of exactly nG lanes, each slice holding every
// receiver once (one per lane) and taking its own share of each source
// tile, so small groups still fill the lanes; the slices' partial sums are
// combined through LDS at the end.  A wave reads at most two sources per LDS
// instruction (one per slice it touches: LDS broadcasts).  Sources are
// staged cooperatively: opened-leaf particle ranges are expanded into an
// index chunk in LDS, then each thread loads one source, converts it to
// group-relative FP32 and stores it into structure-of-arrays LDS tiles.
// No MFMA: the pair law is not a contraction.
#include "gx_internal.hpp"
#include <algorithm>
#include <cstdlib>
#include <vector>

int gx_tree_check(gx_ctx* ctx, int which, const gx_particles* p);

__global__ __launch_bounds__(128) void k_walk_grav(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes, int nn,
    const double* __restrict__ box, double theta2, int mode, uint32_t* __restrict__ pc_cnt,
    uint32_t* __restrict__ pr_cnt, uint32_t* __restrict__ pp_tot,
    unsigned long long* __restrict__ tot, const int64_t* __restrict__ pc_off,
    int32_t* __restrict__ pc_list, const int64_t* __restrict__ pr_off,
    int32_t* __restrict__ pr_begin, int32_t* __restrict__ pr_cum, int cap_pc, int cap_pr);
// One-pass wave walk over the level-order arrays (launched in the walk's own
// source file): small_stack picks the 8 KB stack, else 16 KB.
int gx_walk_grav_wave(gx_ctx* ctx, TreeSlot& T, int ng, double theta2, bool small_stack,
                      uint32_t* pc_cnt, uint32_t* pr_cnt, uint32_t* pp_tot, int32_t* pc_list,
                      int32_t* pr_begin, int32_t* pr_cum, int cap_pc, int cap_pr,
                      uint8_t* gflag, int32_t* gdepth);
// Entries of the small walk stack (the context's limit when one is set).
int gx_walk_stack_small(const gx_ctx* ctx);
__global__ __launch_bounds__(256) void k_group_totals(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, const uint32_t* __restrict__ c0,
    const uint32_t* __restrict__ c1, const uint32_t* __restrict__ pp,
    const uint8_t* __restrict__ flag, const int32_t* __restrict__ depth,
    unsigned long long* __restrict__ tot);
__global__ void k_direct_lists(int ng, int n, const int32_t* __restrict__ groups,
                               const NodeRec* __restrict__ nodes, int64_t* __restrict__ pc_off,
                               int64_t* __restrict__ pr_off, uint32_t* __restrict__ pc_cnt,
                               uint32_t* __restrict__ pr_cnt, int32_t* __restrict__ pr_begin,
                               int32_t* __restrict__ pr_cum, uint32_t* __restrict__ pp_tot,
                               unsigned long long* __restrict__ tot);

// 512 threads per group: more slices per tile, so fewer lanes of the waves
// that issue sit idle when a group's size is not a multiple of 64 (e.g. 130
// receivers: 3 slices over 7 waves instead of 1 slice over 3 waves per tile)
#define GF_THREADS 512
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
// FP32: at most 80 VGPRs (six wavefronts per SIMD); left free, the compiler
// takes 116 registers and four wavefronts, which measured ~7 % slower
__global__ __launch_bounds__(GF_THREADS)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1))) void k_grav_force(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const MomRec* __restrict__ mom, const double4* __restrict__ pos4, const float* __restrict__ e2s,
    const uint32_t* __restrict__ perm, const int64_t* __restrict__ pc_off,
    const uint32_t* __restrict__ pc_cnt, int64_t pc_stride, const int32_t* __restrict__ pc_list,
    const int64_t* __restrict__ pr_off, const uint32_t* __restrict__ pr_cnt, int64_t pr_stride,
    const int32_t* __restrict__ pr_begin, const int32_t* __restrict__ pr_cum,
    const uint32_t* __restrict__ pp_tot, double G, double* __restrict__ ax, double* __restrict__ ay,
    double* __restrict__ az, double* __restrict__ pot) {
    const int g = xcd_chunk(blockIdx.x);
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
    // slices: pad = min(nG, GF_THREADS) lanes hold the receivers once and
    // floor(GF_THREADS / pad) slices split each tile, so fewer than pad lanes
    // of the block idle (the slices are combined through LDS, any width
    // works); larger groups take several passes over their receivers
    const int pad = nG < 1 ? 1 : (nG < GF_THREADS ? nG : GF_THREADS);
    const int nsl = GF_THREADS / pad, il = tid % pad, sl = tid / pad;
    const int npp = (int)pp_tot[g];
    // list of this group: fixed slots (stride > 0) or CSR offsets
    const int64_t r0 = pr_stride ? (int64_t)g * pr_stride : pr_off[g], r1 = r0 + pr_cnt[g];
    const int64_t c0 = pc_stride ? (int64_t)g * pc_stride : pc_off[g], c1 = c0 + pc_cnt[g];

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
            // each thread's source of the next tile is read into registers
            // while the current tile is evaluated
            V4<T> npa{};
            T npe = 0;
            auto fetch_src = [&](int t) {
                if (tid < GF_TILE && t < che) {
                    const int j = jidx[t - ch];
                    const double4 p = pos4[j];
                    npa = V4<T>{(T)(p.x - cx), (T)(p.y - cy), (T)(p.z - cz), (T)p.w};
                    npe = (T)e2s[j];
                }
            };
            fetch_src(ch + tid);
            for (int t0 = ch; t0 < che; t0 += GF_TILE) {
                const int tn = min(GF_TILE, che - t0);
                if (tid < tn) {
                    sA[tid] = npa;
                    sB[tid].x = npe;
                }
                __syncthreads();
                fetch_src(t0 + GF_TILE + tid);
                if (act) {
                    T fx = 0, fy = 0, fz = 0, fp = 0;
                    const int per = (tn + nsl - 1) / nsl;
                    const int jb = sl * per, je = min(tn, jb + per);
#pragma unroll 4
                    for (int jj = jb; jj < je; jj++) {
                        const V4<T> a = sA[jj];
                        const T dx = a.x - xi, dy = a.y - yi, dz = a.z - zi;
                        // softened r^2 with the softening as the first addend,
                        // so every product folds into a fused multiply-add
                        T r2 = ei + sB[jj].x;
                        r2 = fma(dx, dx, r2);
                        r2 = fma(dy, dy, r2);
                        r2 = fma(dz, dz, r2);
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
        // each thread's record of the next tile is read into registers while
        // the current tile is evaluated; entries are addressed from the
        // group's (uniform) list start with 32-bit offsets
        V4<T> na{}, nb{}, nc{};
        const int32_t* __restrict__ plist = pc_list + c0;
        const int ncell = (int)(c1 - c0);
        auto fetch_cell = [&](int t) {
            if (tid < GF_TILE && t < ncell) {
                const MomRec mr = mom[plist[t]];
                na = V4<T>{(T)(mr.cx - cx), (T)(mr.cy - cy), (T)(mr.cz - cz), (T)mr.M};
                nb = V4<T>{(T)mr.e2, (T)mr.q[0], (T)mr.q[1], (T)mr.q[2]};
                nc = V4<T>{(T)mr.q[3], (T)mr.q[4], (T)mr.q[5], (T)0};
            }
        };
        fetch_cell(tid);
        for (int t0 = 0; t0 < ncell; t0 += GF_TILE) {
            const int tn = min(GF_TILE, ncell - t0);
            if (tid < tn) {
                sA[tid] = na;
                if (QUAD) {
                    sB[tid] = nb;
                    sC[tid] = nc;
                } else {
                    sB[tid].x = nb.x;
                }
            }
            __syncthreads();
            fetch_cell(t0 + GF_TILE + tid);
            if (act) {
                T fx = 0, fy = 0, fz = 0, fp = 0;
                const int per = (tn + nsl - 1) / nsl;
                const int jb = sl * per, je = min(tn, jb + per);
#pragma unroll 2
                for (int jj = jb; jj < je; jj++) {
                    const V4<T> a = sA[jj];
                    const V4<T> b = sB[jj];
                    const T dx = a.x - xi, dy = a.y - yi, dz = a.z - zi;
                    T R2 = ei + b.x;
                    R2 = fma(dx, dx, R2);
                    R2 = fma(dy, dy, R2);
                    R2 = fma(dz, dz, R2);
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
                        const T coef = fma(u5, (T)2.5 * Rinv2, MR3);
                        // one fused update per term keeps each component at
                        // two operations
                        fx = fma(coef, dx, fx);
                        fy = fma(coef, dy, fy);
                        fz = fma(coef, dz, fz);
                        fx = fma(-Rinv5, qdx, fx);
                        fy = fma(-Rinv5, qdy, fy);
                        fz = fma(-Rinv5, qdz, fz);
                        fp = fma(-M, Rinv, fp);
                        fp = fma((T)-0.5, u5, fp);
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
    Ls.stride_pc = Ls.stride_pr = 0;
    if (flags & GX_DIRECT) {
        GX_TRY(gx_reserve(ctx, Ls.pr_begin, (ng + 1) * sizeof(int32_t)));
        GX_TRY(gx_reserve(ctx, Ls.pr_cum, (ng + 1) * sizeof(int32_t)));
        GX_TRY(gx_reserve(ctx, Ls.pc_list, 64));
        hipLaunchKernelGGL(k_direct_lists, dim3(gx_blocks(ng + 1, 256)), dim3(256), 0, st, ng,
                           (int)T.n, (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                           (int64_t*)Ls.pc_off.p, (int64_t*)Ls.pr_off.p, (uint32_t*)Ls.pc_cnt.p,
                           (uint32_t*)Ls.pr_cnt.p, (int32_t*)Ls.pr_begin.p, (int32_t*)Ls.pr_cum.p,
                           (uint32_t*)Ls.pp_tot.p, (unsigned long long*)tot);
        GX_LAUNCH_CHECK(ctx);
        Ls.n_pc = 0;
        Ls.n_ranges = ng;
    } else {
        const double theta2 = theta * theta;
        bool done = false;
        int64_t seen_pc = 0, seen_pr = 0;  // largest per-group list sizes seen in this call
        const int64_t prev_stack = Ls.last_stack;  // deepest stack of the previous call
        Ls.last_two_pass = 1;
        Ls.last_stack = 0;
        // one pass into per-group slots sized from the largest lists of the
        // previous call; a list that does not fit sends the call to the exact
        // two-pass (count, scan, fill) construction
        if (Ls.cap_pc > 0 && Ls.cap_pr > 0 && std::llabs(Ls.cap_ng - (int64_t)ng) * 10 <= ng) {
            GX_TRY(gx_reserve(ctx, Ls.pc_list, (size_t)ng * Ls.cap_pc * sizeof(int32_t)));
            GX_TRY(gx_reserve(ctx, Ls.pr_begin, (size_t)ng * Ls.cap_pr * sizeof(int32_t)));
            GX_TRY(gx_reserve(ctx, Ls.pr_cum, (size_t)ng * Ls.cap_pr * sizeof(int32_t)));
            GX_TRY(gx_reserve(ctx, Ls.aux, (size_t)ng * (1 + sizeof(int32_t)) + 64));
            uint8_t* gflag = (uint8_t*)Ls.aux.p;
            int32_t* gdepth = (int32_t*)((uint8_t*)Ls.aux.p + (((size_t)ng + 15) & ~(size_t)15));
            // the small stack when the previous call's deepest stack fits with an
            // eighth to spare; a small-stack walk that overflows only its stack
            // is repeated once with the large one
            const int64_t s_small = gx_walk_stack_small(ctx);
            bool small = ctx->walk_small_cap > 0 ||
                         (prev_stack > 0 && prev_stack + prev_stack / 8 <= s_small);
            for (int attempt = 0; attempt < 2 && !done; attempt++) {
                GX_TRY(gx_walk_grav_wave(ctx, T, ng, theta2, small, (uint32_t*)Ls.pc_cnt.p,
                                         (uint32_t*)Ls.pr_cnt.p, (uint32_t*)Ls.pp_tot.p,
                                         (int32_t*)Ls.pc_list.p, (int32_t*)Ls.pr_begin.p,
                                         (int32_t*)Ls.pr_cum.p, Ls.cap_pc, Ls.cap_pr, gflag,
                                         gdepth));
                hipLaunchKernelGGL(k_group_totals, dim3(gx_blocks(ng, 256)), dim3(256), 0, st, ng,
                                   (const int32_t*)T.groups.p, nullptr, (const NodeRec*)T.nodes.p,
                                   (const uint32_t*)Ls.pc_cnt.p, (const uint32_t*)Ls.pr_cnt.p,
                                   (const uint32_t*)Ls.pp_tot.p, gflag, gdepth,
                                   (unsigned long long*)tot);
                GX_LAUNCH_CHECK(ctx);
                GX_TRY(read_host(ctx, h_tot, tot, 8 * sizeof(int64_t)));
                seen_pc = std::max<int64_t>(seen_pc, h_tot[5]);
                seen_pr = std::max<int64_t>(seen_pr, h_tot[6]);
                Ls.last_stack = h_tot[7];
                if (h_tot[4] == 0) {
                    done = true;
                    Ls.last_two_pass = 0;
                    Ls.stride_pc = Ls.cap_pc;
                    Ls.stride_pr = Ls.cap_pr;
                    Ls.n_pc = h_tot[0];
                    Ls.n_ranges = h_tot[1];
                } else {
                    GX_TRY(gx_zero(ctx, Ls.tot.p, 8 * sizeof(int64_t)));
                    const bool stack_only = h_tot[7] > s_small && h_tot[5] <= Ls.cap_pc &&
                                            h_tot[6] <= Ls.cap_pr;
                    if (!(small && stack_only)) break;
                    small = false;
                }
            }
        }
        if (!done) {
            hipLaunchKernelGGL(k_walk_grav, dim3(gx_blocks(ng, 128)), dim3(128), 0, st, ng,
                               (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p, nn,
                               (const double*)T.box.p, theta2, 0, (uint32_t*)Ls.pc_cnt.p,
                               (uint32_t*)Ls.pr_cnt.p, (uint32_t*)Ls.pp_tot.p,
                               (unsigned long long*)tot, nullptr, nullptr, nullptr, nullptr,
                               nullptr, 0, 0);
            GX_LAUNCH_CHECK(ctx);
            GX_TRY(read_host(ctx, h_tot, tot, 8 * sizeof(int64_t)));
            GX_TRY((gx_scan<uint32_t, int64_t>(ctx, (const uint32_t*)Ls.pc_cnt.p,
                                               (int64_t*)Ls.pc_off.p, ng, tot + 0)));
            GX_TRY((gx_scan<uint32_t, int64_t>(ctx, (const uint32_t*)Ls.pr_cnt.p,
                                               (int64_t*)Ls.pr_off.p, ng, tot + 1)));
            // the offsets arrays carry their totals as element ng
            GX_HIP(ctx, hipMemcpyAsync((int64_t*)Ls.pc_off.p + ng, tot + 0, 8,
                                       hipMemcpyDeviceToDevice, st));
            GX_HIP(ctx, hipMemcpyAsync((int64_t*)Ls.pr_off.p + ng, tot + 1, 8,
                                       hipMemcpyDeviceToDevice, st));
            Ls.n_pc = h_tot[0];
            Ls.n_ranges = h_tot[1];
            GX_TRY(gx_reserve(ctx, Ls.pc_list, (Ls.n_pc + 1) * sizeof(int32_t)));
            GX_TRY(gx_reserve(ctx, Ls.pr_begin, (Ls.n_ranges + 1) * sizeof(int32_t)));
            GX_TRY(gx_reserve(ctx, Ls.pr_cum, (Ls.n_ranges + 1) * sizeof(int32_t)));
            hipLaunchKernelGGL(k_walk_grav, dim3(gx_blocks(ng, 128)), dim3(128), 0, st, ng,
                               (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p, nn,
                               (const double*)T.box.p, theta2, 1, nullptr, nullptr, nullptr,
                               nullptr, (const int64_t*)Ls.pc_off.p, (int32_t*)Ls.pc_list.p,
                               (const int64_t*)Ls.pr_off.p, (int32_t*)Ls.pr_begin.p,
                               (int32_t*)Ls.pr_cum.p, 0, 0);
            GX_LAUNCH_CHECK(ctx);
        }
        // slot sizes for the next call: largest lists seen, plus a margin,
        // unless the slots would be far larger than the lists themselves
        // (the one-pass walk does not merge contiguous leaves, so its range
        // counts can exceed the two-pass ones: keep the larger)
        seen_pc = std::max<int64_t>(seen_pc, h_tot[5]);
        seen_pr = std::max<int64_t>(seen_pr, h_tot[6]);
        const int64_t mpc = seen_pc + seen_pc / 4 + 64, mpr = seen_pr + seen_pr / 4 + 16;
        const bool fits = (double)ng * (double)(mpc + 2 * mpr) <= 8.0 * (double)(h_tot[0] + 2 * h_tot[1]) + 1e6;
        Ls.cap_pc = fits ? (int)std::min<int64_t>(mpc, INT32_MAX / 2) : 0;
        Ls.cap_pr = fits ? (int)std::min<int64_t>(mpr, INT32_MAX / 2) : 0;
        Ls.cap_ng = ng;
    }
    Ls.n_groups = ng;

    const bool quad = (flags & GX_QUAD) && !(flags & GX_DIRECT);
    const bool fp64 = flags & GX_PREC_FP64;
    auto args = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(xcd_chunk_grid(ng)), dim3(GF_THREADS), 0, st, ng,
                           (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                           (const MomRec*)T.mom.p, (const double4*)T.pos4.p, (const float*)T.e2s.p,
                           (const uint32_t*)T.val[0].p, (const int64_t*)Ls.pc_off.p,
                           (const uint32_t*)Ls.pc_cnt.p, Ls.stride_pc, (const int32_t*)Ls.pc_list.p,
                           (const int64_t*)Ls.pr_off.p, (const uint32_t*)Ls.pr_cnt.p,
                           Ls.stride_pr, (const int32_t*)Ls.pr_begin.p,
                           (const int32_t*)Ls.pr_cum.p, (const uint32_t*)Ls.pp_tot.p, G, ax, ay,
                           az, pot);
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
        // list construction: n_rewalk = 1 when it took the two-pass path,
        // n_iter_max = deepest walk stack of the one-pass walk (0: not run)
        stats->n_rewalk = Ls.last_two_pass;
        stats->n_iter_max = Ls.last_stack;
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
    // lists live either in fixed per-group slots (stride > 0) or in CSR
    // arrays; the export is CSR in both cases
    std::vector<uint32_t> pcc(ng), prc(ng), tot(ng);
    std::vector<int64_t> pcs(ng + 1), prs(ng + 1);
    if (ng > 0) {
        GX_HIP(ctx, hipMemcpy(pcc.data(), Ls.pc_cnt.p, ng * 4, hipMemcpyDeviceToHost));
        GX_HIP(ctx, hipMemcpy(prc.data(), Ls.pr_cnt.p, ng * 4, hipMemcpyDeviceToHost));
        GX_HIP(ctx, hipMemcpy(tot.data(), Ls.pp_tot.p, ng * 4, hipMemcpyDeviceToHost));
    }
    if (Ls.stride_pc > 0) {
        for (int64_t g = 0; g < ng; g++) pcs[g] = g * Ls.stride_pc;
    } else if (ng > 0) {
        GX_HIP(ctx, hipMemcpy(pcs.data(), Ls.pc_off.p, ng * 8, hipMemcpyDeviceToHost));
    }
    if (Ls.stride_pr > 0) {
        for (int64_t g = 0; g < ng; g++) prs[g] = g * Ls.stride_pr;
    } else if (ng > 0) {
        GX_HIP(ctx, hipMemcpy(prs.data(), Ls.pr_off.p, ng * 8, hipMemcpyDeviceToHost));
    }
    const int64_t span_pc = ng ? pcs[ng - 1] + pcc[ng - 1] : 0;
    const int64_t span_pr = ng ? prs[ng - 1] + prc[ng - 1] : 0;
    std::vector<int32_t> lst(span_pc), b(span_pr), c(span_pr);
    if (span_pc) GX_HIP(ctx, hipMemcpy(lst.data(), Ls.pc_list.p, span_pc * 4, hipMemcpyDeviceToHost));
    if (span_pr) {
        GX_HIP(ctx, hipMemcpy(b.data(), Ls.pr_begin.p, span_pr * 4, hipMemcpyDeviceToHost));
        GX_HIP(ctx, hipMemcpy(c.data(), Ls.pr_cum.p, span_pr * 4, hipMemcpyDeviceToHost));
    }
    int64_t opc = 0, opr = 0;
    for (int64_t g = 0; g < ng; g++) {
        if (pc_off) pc_off[g] = opc;
        if (pp_off) pp_off[g] = opr;
        for (uint32_t k = 0; k < pcc[g]; k++, opc++)
            if (pc_node) pc_node[opc] = lst[pcs[g] + k];
        for (uint32_t k = 0; k < prc[g]; k++, opr++) {
            const int64_t r = prs[g] + k;
            const int32_t cn = (k + 1 < prc[g]) ? c[r + 1] : (int32_t)tot[g];
            if (pp_begin) pp_begin[opr] = b[r];
            if (pp_end) pp_end[opr] = b[r] + (cn - c[r]);
        }
    }
    if (pc_off) pc_off[ng] = opc;
    if (pp_off) pp_off[ng] = opr;
    return GX_OK;
}
