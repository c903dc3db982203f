// gx_sph.hip -- SPH kernel size, density/pressure and hydro force (the
// "kernel size", "density and pressure" and "hydro force" items of Table 3,
// kernels of Table 4), Wendland C4 kernel, on the gas tree slot.
//
// Receivers: the gas tree's groups (maximal nodes of at most n_group
// particles; compact boxes keep candidate lists short).  One wavefront per
// group.  Groups are usually smaller than 64, so the wave is cut into
// 64 / pad slices (pad = 16, 32 or 64 >= group size): every slice holds each
// receiver once and takes its own share of the candidates; cross-slice sums
// are butterfly shuffles, which give every lane of a receiver bit-identical
// totals.  Each group's candidate list -- particles of every gas-tree leaf
// whose box comes within the search radius of the group box -- is built by
// the wave-cooperative breadth-first walk in gx_walk.hip, in one pass into a
// fixed-capacity slot per group.
//
// Density: candidates are converted once to group-relative FP32 (position,
// mass) and kept in LDS for all Newton iterations.  Each receiver runs a
// bracketed Newton iteration on N_eff(H) = (4 pi/3) H^3 rho(H) / m; a receiver
// whose kernel size would leave the radius its list was built for stops and
// flags the group, and the host re-walks only those groups with the larger
// radius.  Force: one pass over LDS tiles of candidates, pairs inside
// max(H_i, H_j), FP32 pair arithmetic, FP64 combination per tile.
#include "gx_internal.hpp"

int gx_tree_check(gx_ctx* ctx, int which, const gx_particles* p);

__global__ __launch_bounds__(128) void k_walk_sph(
    int nb, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, const MomRec* __restrict__ mom, int nn,
    const float* __restrict__ radius, int use_hmax,
    const uint8_t* __restrict__ active, int mode, int cap, uint32_t* __restrict__ pr_cnt,
    uint32_t* __restrict__ pp_tot, unsigned long long* __restrict__ tot,
    const int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum);
__global__ __launch_bounds__(64) void k_walk_sph_bfs(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ child, const MomRec* __restrict__ mom,
    const float* __restrict__ radius, int use_hmax, const uint8_t* __restrict__ active, int cap,
    uint32_t* __restrict__ pr_cnt, uint32_t* __restrict__ pp_tot,
    unsigned long long* __restrict__ tot, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum, uint8_t* __restrict__ ovf);
__global__ __launch_bounds__(256) void k_group_totals(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, const uint32_t* __restrict__ c0,
    const uint32_t* __restrict__ c1, const uint32_t* __restrict__ pp,
    const uint8_t* __restrict__ flag, const int32_t* __restrict__ depth,
    unsigned long long* __restrict__ tot);
__global__ __launch_bounds__(64) void k_walk_sph_wave(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ child,
    const MomRec* __restrict__ mom, const float* __restrict__ radius, int use_hmax,
    const uint8_t* __restrict__ active, int mode, uint32_t* __restrict__ pr_cnt,
    uint32_t* __restrict__ pp_tot, unsigned long long* __restrict__ tot,
    const int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum, uint8_t* __restrict__ sovf);

#define SPH_THREADS 64
#define SPH_DT 256         // threads of the density and force kernels (4 waves per group)
#define SPH_CAP 2048       // candidates kept in LDS by the density kernel
#define SPH_TILE 256       // force kernel source tile
#define SPH_RANGES 1024    // capacity of a block's candidate range list (single-pass walk)
#define SPH_MARGIN 1.15f   // density search radius = margin x largest kernel size

// 495 / (32 pi), (4 pi / 3) * 495 / (32 pi) = 495 / 24, 1155 / (4 pi)
#define WC4_NORM 4.9238032806262495f
#define NEFF_C 20.625f
#define GRADW_C 91.91197457030109f

enum { W_H = 0, W_RAD, W_ACT, W_FLAG, W_VEL, W_SPH, W_STAT };

static int work(gx_ctx* ctx, int k, size_t bytes, void** p) {
    GX_TRY(gx_reserve(ctx, ctx->sph_work[k], bytes));
    *p = ctx->sph_work[k].p;
    return GX_OK;
}

// Kernel-size seed: H64 when positive and finite, else from the mean density
// of the smallest tree node holding the particle and at least n_ngb
// particles (its mass over the volume of its tight bounding box).
__global__ __launch_bounds__(256) void k_sph_seed(int64_t n, const NodeRec* __restrict__ nodes,
                                                  const MomRec* __restrict__ mom,
                                                  const double4* __restrict__ pos4,
                                                  const uint32_t* __restrict__ perm,
                                                  const double* __restrict__ H64, float n_ngb,
                                                  const double* __restrict__ box,
                                                  float* __restrict__ Hs) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double h = H64 ? H64[perm[s]] : -1.0;
    if (h > 0.0 && h < INFINITY) {
        Hs[s] = (float)h;
        return;
    }
    int node = 0;
    for (;;) {
        const NodeRec nd = nodes[node];
        if (nd.leaf) break;
        int nxt = -1;
        for (int c = node + 1; c < nd.next; c = nodes[c].next) {
            const NodeRec cn = nodes[c];
            if (cn.begin <= s && s < cn.end) {
                if (cn.end - cn.begin >= (int)n_ngb) nxt = c;
                break;
            }
        }
        if (nxt < 0) break;
        node = nxt;
    }
    // volume of the node's tight bounding box (a thin disk fills only a slab
    // of its cubic cell), guarded against flat boxes
    const NodeRec& nd = nodes[node];
    double vol = 1.0;
    for (int d = 0; d < 3; d++) {
        const double w = nd.hi[d] - nd.lo[d];
        vol *= w > 0.0 ? w : 1e-30;
    }
    const double rho = mom[node].M / vol;
    Hs[s] = (float)cbrt(3.0 * (double)n_ngb * pos4[s].w / (4.0 * M_PI * rho));
}

__global__ __launch_bounds__(64) void k_group_radius(int ng, const int32_t* __restrict__ groups,
                                                     const NodeRec* __restrict__ nodes,
                                                     const float* __restrict__ Hs, float scale,
                                                     float* __restrict__ rad) {
    const int g = blockIdx.x;
    const NodeRec r = nodes[groups[g]];
    float h = 0.0f;
    for (int s = r.begin + threadIdx.x; s < r.end; s += 64) h = fmaxf(h, Hs[s]);
    h = wave_max(h);
    if (threadIdx.x == 0) rad[g] = h * scale;
}

__device__ __forceinline__ int slice_pad(int nG) {
    int pad = 16;
    while (pad < nG && pad < 64) pad <<= 1;
    return pad;
}

// Sum over the slices of a wave (lanes il, il + pad, ...): butterfly shuffles.
template <typename T>
__device__ __forceinline__ T slice_sum(T v, int pad) {
    for (int o = pad; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// First range of a group list that overlaps candidate position ch: the last
// range whose running offset is <= ch (offsets increase strictly), found by
// bisection so that expanding one chunk of a long list costs O(log R) plus
// the ranges the chunk touches.
__device__ __forceinline__ int64_t first_range(const GroupList& L, int ch) {
    int64_t lo = L.r0, hi = L.r1 - 1;
    if (hi < lo) return lo;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (L.cum[mid] <= ch) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void expand_chunk(const GroupList& L, int npp, int ch, int che,
                                             const double4* __restrict__ pos4, double cx,
                                             double cy, double cz, float4* __restrict__ cand,
                                             int tid, int nthreads) {
    for (int64_t r = first_range(L, ch); r < L.r1; r++) {
        const int c = L.cum[r];
        const int cn = (r + 1 < L.r1) ? L.cum[r + 1] : npp;
        if (cn <= ch) continue;
        if (c >= che) break;
        const int b = L.begin[r];
        const int lo = max(c, ch), hi = min(cn, che);
        for (int k = lo + tid; k < hi; k += nthreads) {
            const double4 p = pos4[b + (k - c)];
            cand[k - ch] = make_float4((float)(p.x - cx), (float)(p.y - cy), (float)(p.z - cz),
                                       (float)p.w);
        }
    }
}

// Kernel size and density: one 256-thread workgroup per group; the group's
// candidates sit once in LDS and are shared by its four waves.  The threads
// form 256 / pad slices (pad >= nG lanes each, every receiver once per
// slice); a slice sums its share of the candidates, the shares are combined
// by shuffles inside a wave and through LDS across waves (fixed order), and
// every copy of a receiver then takes the same safeguarded Newton step.
__global__ __launch_bounds__(SPH_DT) void k_sph_density(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const double4* __restrict__ pos4, const uint32_t* __restrict__ perm,
    const uint8_t* __restrict__ active, ListView L, float* __restrict__ rad, float n_ngb, float tol,
    int max_iter, float* __restrict__ Hs, uint32_t* __restrict__ flags,
    unsigned long long* __restrict__ stat, const double* __restrict__ u, float gamma,
    double* __restrict__ H64, float* __restrict__ Hout, float* __restrict__ rho_out,
    float* __restrict__ P_out, float* __restrict__ cs_out) {
    const int g = xcd_remap(blockIdx.x, ng);
    if (g >= ng) return;
    if (active && !active[g]) return;
    __shared__ float4 cand[SPH_CAP];
    __shared__ float2 red[SPH_DT / 64][64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const NodeRec B = nodes[groups[g]];
    const int nG = B.end - B.begin;
    const int pad = slice_pad(nG), nsl = SPH_DT / pad, il = tid % pad, sl = tid / pad;
    const double cx = (B.lo[0] + B.hi[0]) * 0.5;
    const double cy = (B.lo[1] + B.hi[1]) * 0.5;
    const double cz = (B.lo[2] + B.hi[2]) * 0.5;
    const GroupList GL(L, g);
    const int npp = GL.npp;
    const float Rlim = rad[g];
    const bool in_lds = npp <= SPH_CAP;
    if (in_lds) expand_chunk(GL, npp, 0, npp, pos4, cx, cy, cz, cand, tid, SPH_DT);
    __syncthreads();

    int nflag = 0, nfail = 0, worst_it = 0;
    float hmax = 0.0f;
    for (int ic = 0; ic < nG; ic += pad) {
        const int s = B.begin + ic + il;
        const bool act = ic + il < nG;
        float xi = 0, yi = 0, zi = 0, mi = 1, H = 1.0f;
        if (act) {
            const double4 p = pos4[s];
            xi = (float)(p.x - cx);
            yi = (float)(p.y - cy);
            zi = (float)(p.z - cz);
            mi = (float)p.w;
            H = Hs[s];
        }
        float lo = 0.0f, hi = INFINITY, S0 = 0.0f;
        bool done = !act, conv = false, over = false;
        int it = 0;
        for (;;) {
            const float Hinv = 1.0f / H, Hinv2 = Hinv * Hinv;
            float s0 = 0.0f, s1 = 0.0f;
            for (int ch = 0; ch < npp; ch += SPH_CAP) {
                const int che = min(npp, ch + SPH_CAP);
                if (!in_lds) {
                    __syncthreads();
                    expand_chunk(GL, npp, ch, che, pos4, cx, cy, cz, cand, tid, SPH_DT);
                    __syncthreads();
                }
                const int cnt = che - ch;
                const int per = (cnt + nsl - 1) / nsl;
                const int kb = sl * per, ke = min(cnt, kb + per);
#pragma unroll 4
                for (int k = kb; k < ke; k++) {
                    const float4 c = cand[k];
                    const float dx = c.x - xi, dy = c.y - yi, dz = c.z - zi;
                    const float q2 = (dx * dx + dy * dy + dz * dz) * Hinv2;
                    if (q2 < 1.0f) {
                        const float q = __builtin_sqrtf(q2);
                        const float t = 1.0f - q;
                        const float t2 = t * t;
                        const float t5 = t2 * t2 * t;
                        const float poly = 1.0f + q * (6.0f + q * (35.0f / 3.0f));
                        s0 += c.w * t5 * t * poly;
                        s1 += c.w * q2 * (1.0f + 5.0f * q) * t5;
                    }
                }
            }
            // slices of this wave, then the four waves in order
            s0 = slice_sum(s0, pad);
            s1 = slice_sum(s1, pad);
            if (lane < pad) red[wv][lane] = make_float2(s0, s1);
            __syncthreads();
            s0 = 0.0f;
            s1 = 0.0f;
#pragma unroll
            for (int w = 0; w < SPH_DT / 64; w++) {
                const float2 r = red[w][il];
                s0 += r.x;
                s1 += r.y;
            }
            if (!done) {
                it++;
                S0 = s0;
                const float neff = NEFF_C * s0 / mi;
                const float f = neff - n_ngb;
                if (fabsf(f) <= tol) {
                    done = true;
                    conv = true;
                } else if (it >= max_iter) {
                    done = true;
                } else {
                    const float dn = NEFF_C * (56.0f / 3.0f) * s1 / (mi * H);
                    if (f < 0.0f) lo = H;
                    else hi = H;
                    float Hn = dn > 0.0f ? H - f / dn : NAN;
                    if (!(Hn > lo && Hn < hi)) Hn = (hi < INFINITY) ? 0.5f * (lo + hi) : 2.0f * H;
                    if (Hn > Rlim) {
                        // the list only covers kernel sizes up to Rlim: redo with a larger list
                        done = true;
                        over = true;
                    }
                    H = Hn;
                }
            }
            if (!__syncthreads_or(done ? 0 : 1)) break;
        }
        if (act && sl == 0) {
            Hs[s] = H;
            hmax = fmaxf(hmax, H);
            worst_it = max(worst_it, it);
            if (over) {
                nflag++;
            } else {
                if (!conv) nfail++;
                const uint32_t o = perm[s];
                const float rho = WC4_NORM / (H * H * H) * S0;
                const double uu = u[o];
                H64[o] = (double)H;
                Hout[o] = H;
                rho_out[o] = rho;
                if (P_out) P_out[o] = (float)((double)(gamma - 1.0f) * (double)rho * uu);
                if (cs_out) cs_out[o] = (float)sqrt((double)gamma * (gamma - 1.0f) * uu);
            }
        }
    }
    if (wv == 0) {  // slice 0 (the written copies) lies in wave 0
        nflag = (int)wave_sum((unsigned)nflag);
        nfail = (int)wave_sum((unsigned)nfail);
        worst_it = wave_max(worst_it);
        hmax = wave_max(hmax);
        if (lane == 0) {
            flags[g] = nflag ? 1u : 0u;
            atomicMax(&stat[1], (unsigned long long)worst_it);
            if (nflag) {
                rad[g] = hmax * SPH_MARGIN;
                atomicAdd(&stat[3], 1ull);
            } else {  // counted once, in the group's final round
                atomicAdd(&stat[0], (unsigned long long)nfail);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Force
// ---------------------------------------------------------------------------
// Sorted per-particle state: velocity (FP64) and {H, rho, A = P / rho^2, c}
// (FP32) with P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u).
__global__ __launch_bounds__(256) void k_sph_prep(int64_t n, const uint32_t* __restrict__ perm,
                                                  const double* __restrict__ vx,
                                                  const double* __restrict__ vy,
                                                  const double* __restrict__ vz,
                                                  const double* __restrict__ u,
                                                  const float* __restrict__ H,
                                                  const float* __restrict__ rho, float gamma,
                                                  double4* __restrict__ sv,
                                                  float4* __restrict__ ss) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t o = perm[s];
    sv[s] = make_double4(vx[o], vy[o], vz[o], 0.0);
    const double uu = u[o];
    const float r = rho[o];
    const double P = (double)(gamma - 1.0f) * (double)r * uu;
    ss[s] = make_float4(H[o], r, (float)(P / ((double)r * (double)r)),
                        (float)sqrt((double)gamma * (gamma - 1.0f) * uu));
}

// Largest kernel size per node, leaves from particles, internal from children.
__global__ __launch_bounds__(256) void k_hmax_level(int cnt, const int32_t* __restrict__ ids,
                                                    const NodeRec* __restrict__ nodes,
                                                    MomRec* __restrict__ mom,
                                                    const float4* __restrict__ ss) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cnt) return;
    int id = ids[k];
    NodeRec nd = nodes[id];
    float h = 0.0f;
    if (nd.leaf) {
        for (int s = nd.begin; s < nd.end; s++) h = fmaxf(h, ss[s].x);
    } else {
        for (int c = id + 1; c < nd.next; c = nodes[c].next) h = fmaxf(h, mom[c].hmax);
    }
    mom[id].hmax = h;
}

// Largest kernel size of every node of a tree (ss[s].x = H of sorted slot s).
int gx_sph_node_hmax(gx_ctx* ctx, TreeSlot& T, const float4* ss) {
    int64_t off = 0;
    int64_t lvl_off[GX_MAX_LEVEL + 1];
    for (int l = 0; l <= GX_MAX_LEVEL; l++) {
        lvl_off[l] = off;
        off += T.lvl_hist[l];
    }
    for (int l = GX_MAX_LEVEL; l >= 0; l--) {
        int c = (int)T.lvl_hist[l];
        if (!c) continue;
        hipLaunchKernelGGL(k_hmax_level, dim3(gx_blocks(c, 256)), dim3(256), 0, ctx->stream, c,
                           (const int32_t*)T.lvl_ids.p + lvl_off[l], (const NodeRec*)T.nodes.p,
                           (MomRec*)T.mom.p, ss);
    }
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

__global__ __launch_bounds__(64) void k_group_hmax(int ng, const int32_t* __restrict__ groups,
                                                   const MomRec* __restrict__ mom,
                                                   float* __restrict__ rad) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ng) rad[g] = mom[groups[g]].hmax;
}

__global__ __launch_bounds__(SPH_DT) void k_sph_force(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const double4* __restrict__ pos4, const uint32_t* __restrict__ perm,
    const double4* __restrict__ sv, const float4* __restrict__ ss, ListView L, float alpha,
    double* __restrict__ ax, double* __restrict__ ay, double* __restrict__ az,
    double* __restrict__ dudt, float* __restrict__ vsig_out, unsigned long long* __restrict__ stat) {
    const int g = xcd_remap(blockIdx.x, ng);
    if (g >= ng) return;
    __shared__ float tx[SPH_TILE], ty[SPH_TILE], tz[SPH_TILE], tvx[SPH_TILE], tvy[SPH_TILE],
        tvz[SPH_TILE], tm[SPH_TILE], thi[SPH_TILE], th2[SPH_TILE], tcw[SPH_TILE], trho[SPH_TILE],
        tA[SPH_TILE], tc[SPH_TILE];
    __shared__ int32_t jidx[SPH_TILE];
    __shared__ double redd[4][SPH_DT / 64][64];
    __shared__ float redv[SPH_DT / 64][64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const NodeRec B = nodes[groups[g]];
    const int nG = B.end - B.begin;
    const int pad = slice_pad(nG), nsl = SPH_DT / pad, il = tid % pad, sl = tid / pad;
    const double cx = (B.lo[0] + B.hi[0]) * 0.5;
    const double cy = (B.lo[1] + B.hi[1]) * 0.5;
    const double cz = (B.lo[2] + B.hi[2]) * 0.5;
    const double4 vref = sv[B.begin];
    const GroupList GL(L, g);
    const int npp = GL.npp;
    const int64_t r0 = GL.r0, r1 = GL.r1;
    unsigned long long nin = 0;

    for (int ic = 0; ic < nG; ic += pad) {
        const int s = B.begin + ic + il;
        const bool act = ic + il < nG;
        float xi = 0, yi = 0, zi = 0, vxi = 0, vyi = 0, vzi = 0;
        float Hi = 1, Hinv = 1, cwi = 0, rhoi = 1, Ai = 0, ci = 0;
        if (act) {
            const double4 p = pos4[s];
            xi = (float)(p.x - cx);
            yi = (float)(p.y - cy);
            zi = (float)(p.z - cz);
            const double4 v = sv[s];
            vxi = (float)(v.x - vref.x);
            vyi = (float)(v.y - vref.y);
            vzi = (float)(v.z - vref.z);
            const float4 q = ss[s];
            Hi = q.x;
            Hinv = 1.0f / Hi;
            const float h2 = Hinv * Hinv;
            cwi = -GRADW_C * h2 * h2 * Hinv;
            rhoi = q.y;
            Ai = q.z;
            ci = q.w;
        }
        const float Hi2 = Hi * Hi;
        double AX = 0, AY = 0, AZ = 0, DU = 0;
        float vs = ci;
        int64_t rr = r0;  // first range that may overlap the current tile
        for (int t0 = 0; t0 < npp; t0 += SPH_TILE) {
            const int tn = min(SPH_TILE, npp - t0);
            __syncthreads();
            for (int64_t r = rr; r < r1; r++) {
                const int c = GL.cum[r];
                if (c >= t0 + tn) break;
                const int cn = (r + 1 < r1) ? GL.cum[r + 1] : npp;
                const int b = GL.begin[r];
                const int lo = max(c, t0), hi = min(cn, t0 + tn);
                for (int k = lo + tid; k < hi; k += SPH_DT) jidx[k - t0] = b + (k - c);
            }
            while (rr < r1 && ((rr + 1 < r1) ? GL.cum[rr + 1] : npp) <= t0 + tn) rr++;
            __syncthreads();
            for (int e = tid; e < tn; e += SPH_DT) {
                const int j = jidx[e];
                const double4 p = pos4[j];
                const double4 v = sv[j];
                const float4 q = ss[j];
                tx[e] = (float)(p.x - cx);
                ty[e] = (float)(p.y - cy);
                tz[e] = (float)(p.z - cz);
                tvx[e] = (float)(v.x - vref.x);
                tvy[e] = (float)(v.y - vref.y);
                tvz[e] = (float)(v.z - vref.z);
                tm[e] = (float)p.w;
                const float hinv = 1.0f / q.x;
                const float h2 = hinv * hinv;
                thi[e] = hinv;
                th2[e] = q.x * q.x;
                tcw[e] = -GRADW_C * h2 * h2 * hinv;
                trho[e] = q.y;
                tA[e] = q.z;
                tc[e] = q.w;
            }
            __syncthreads();
            if (act) {
                float fx = 0, fy = 0, fz = 0, fu = 0;
                const int per = (tn + nsl - 1) / nsl;
                const int kb = sl * per, ke = min(tn, kb + per);
                for (int k = kb; k < ke; k++) {
                    const float dx = tx[k] - xi, dy = ty[k] - yi, dz = tz[k] - zi;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const bool inside = (r2 < Hi2 || r2 < th2[k]) && r2 > 0.0f;
                    if (inside) {
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float r = r2 * rinv;
                        const float qi = r * Hinv, qj = r * thi[k];
                        float gi = 0.0f, gj = 0.0f;
                        if (qi < 1.0f) {
                            const float t = 1.0f - qi, t2 = t * t;
                            gi = cwi * (1.0f + 5.0f * qi) * t2 * t2 * t;
                        }
                        if (qj < 1.0f) {
                            const float t = 1.0f - qj, t2 = t * t;
                            gj = tcw[k] * (1.0f + 5.0f * qj) * t2 * t2 * t;
                        }
                        const float dvx = tvx[k] - vxi, dvy = tvy[k] - vyi, dvz = tvz[k] - vzi;
                        const float vr = dvx * dx + dvy * dy + dvz * dz;
                        const float w = vr * rinv;
                        const float sig = ci + tc[k] - 3.0f * fminf(w, 0.0f);
                        const float Pi = w < 0.0f ? -alpha * sig * w / (rhoi + trho[k]) : 0.0f;
                        const float gbar = 0.5f * (gi + gj);
                        const float f = tm[k] * (Ai * gi + tA[k] * gj + Pi * gbar);
                        fx += f * dx;
                        fy += f * dy;
                        fz += f * dz;
                        fu += tm[k] * (Ai * gi + 0.5f * Pi * gbar) * vr;
                        vs = fmaxf(vs, sig);
                        nin++;
                    }
                }
                AX += (double)fx;
                AY += (double)fy;
                AZ += (double)fz;
                DU += (double)fu;
            }
        }
        // slices of each wave by shuffles, then the four waves in order
        AX = slice_sum(AX, pad);
        AY = slice_sum(AY, pad);
        AZ = slice_sum(AZ, pad);
        DU = slice_sum(DU, pad);
        for (int o = pad; o < 64; o <<= 1) vs = fmaxf(vs, __shfl_xor(vs, o, 64));
        __syncthreads();
        if (lane < pad) {
            redd[0][wv][lane] = AX;
            redd[1][wv][lane] = AY;
            redd[2][wv][lane] = AZ;
            redd[3][wv][lane] = DU;
            redv[wv][lane] = vs;
        }
        __syncthreads();
        if (act && sl == 0) {
            AX = AY = AZ = DU = 0.0;
            for (int w = 0; w < SPH_DT / 64; w++) {
                AX += redd[0][w][il];
                AY += redd[1][w][il];
                AZ += redd[2][w][il];
                DU += redd[3][w][il];
                vs = fmaxf(vs, redv[w][il]);
            }
            const uint32_t o = perm[s];
            ax[o] += AX;
            ay[o] += AY;
            az[o] += AZ;
            dudt[o] = DU;
            vsig_out[o] = vs;
        }
    }
    __shared__ unsigned long long nsh[SPH_DT / 64];
    nin = wave_sum(nin);
    if (lane == 0) nsh[wv] = nin;
    __syncthreads();
    if (tid == 0) {  // one update of the shared counters per group
        unsigned long long t = 0;
        for (int w = 0; w < SPH_DT / 64; w++) t += nsh[w];
        atomicAdd(&stat[2], t);
        atomicAdd(&stat[4], (unsigned long long)nG * (unsigned long long)npp);
    }
}

// ---------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------
// Candidate lists for every (active) group: the wave walk fills fixed-
// capacity slots in one pass and flags the groups whose list or frontier did
// not fit; only those take the thread walk (count + scan + fill) into a
// second, CSR list set.
int gx_sph_walk(gx_ctx* ctx, TreeSlot& T, ListSet& Ls, int ng, const int32_t* groups,
                const NodeRec* recv, const float* rad, int use_hmax, const uint8_t* active,
                ListView* view, int64_t* list_pairs) {
    hipStream_t st = ctx->stream;
    const int nn = (int)T.n_nodes;
    GX_TRY(gx_reserve(ctx, Ls.tot, 16 * sizeof(int64_t)));
    GX_TRY(gx_reserve(ctx, Ls.pr_cnt, (2 * ng + 2) * sizeof(uint32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pp_tot, (2 * ng + 2) * sizeof(uint32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pr_off, (ng + 1) * sizeof(int64_t)));
    GX_TRY(gx_reserve(ctx, Ls.pc_cnt, ng + 16));  // per-group overflow flags
    GX_TRY(gx_reserve(ctx, Ls.pr_begin, (size_t)ng * SPH_RANGES * sizeof(int32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pr_cum, (size_t)ng * SPH_RANGES * sizeof(int32_t)));
    int64_t* tot = (int64_t*)Ls.tot.p;
    uint32_t* cnt = (uint32_t*)Ls.pr_cnt.p;
    uint32_t* cnt2 = cnt + ng + 1;
    uint32_t* ptot = (uint32_t*)Ls.pp_tot.p;
    uint32_t* ptot2 = ptot + ng + 1;
    uint8_t* ovf = (uint8_t*)Ls.pc_cnt.p;
    GX_TRY(gx_zero(ctx, tot, 16 * sizeof(int64_t)));
    hipLaunchKernelGGL(k_walk_sph_bfs, dim3(xcd_grid(ng)), dim3(64), 0, st, ng, groups, recv,
                       (const NodeRec*)T.nodes.p, (const int32_t*)T.child.p, (const MomRec*)T.mom.p, rad, use_hmax, active,
                       SPH_RANGES, cnt, ptot, (unsigned long long*)tot, (int32_t*)Ls.pr_begin.p,
                       (int32_t*)Ls.pr_cum.p, ovf);
    hipLaunchKernelGGL(k_group_totals, dim3(gx_blocks(ng, 256)), dim3(256), 0, st, ng, groups, recv,
                       (const NodeRec*)T.nodes.p, nullptr, cnt, ptot, ovf, nullptr,
                       (unsigned long long*)tot);
    GX_LAUNCH_CHECK(ctx);
    int64_t h[16];
    GX_HIP(ctx, hipMemcpyAsync(h, tot, 16 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    GX_HIP(ctx, hipStreamSynchronize(st));
    ListView v{SPH_RANGES, cnt, (const int32_t*)Ls.pr_begin.p, (const int32_t*)Ls.pr_cum.p, ptot,
               nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int64_t pairs = h[2];
    if (h[4] > 0) {
        // overflowing groups: exact CSR lists from the wave depth-first walk
        // (count, scan, fill); groups whose walk stack would overflow take
        // the thread-level walk into the same CSR arrays
        GX_TRY(gx_reserve(ctx, Ls.aux, ng + 16));
        uint8_t* sovf = (uint8_t*)Ls.aux.p;
        const NodeRec* nodes = (const NodeRec*)T.nodes.p;
        const int32_t* child = (const int32_t*)T.child.p;
        const MomRec* mom = (const MomRec*)T.mom.p;
        hipLaunchKernelGGL(k_walk_sph_wave, dim3(xcd_grid(ng)), dim3(64), 0, st, ng, groups, recv,
                           nodes, child, mom, rad, use_hmax, ovf, 0, cnt2, ptot2,
                           (unsigned long long*)tot, nullptr, nullptr, nullptr, sovf);
        GX_LAUNCH_CHECK(ctx);
        GX_HIP(ctx, hipMemcpyAsync(h, tot, 16 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GX_HIP(ctx, hipStreamSynchronize(st));
        const bool deep = h[5] > 0;
        if (deep) {
            hipLaunchKernelGGL(k_walk_sph, dim3(gx_blocks(ng, 128)), dim3(128), 0, st, ng, groups,
                               recv, nodes, mom, nn, rad, use_hmax, sovf, 3, 0, cnt2, ptot2,
                               (unsigned long long*)(tot + 8), nullptr, nullptr, nullptr);
            GX_LAUNCH_CHECK(ctx);
        }
        GX_TRY((gx_scan<uint32_t, int64_t>(ctx, cnt2, (int64_t*)Ls.pr_off.p, ng, tot + 13)));
        GX_HIP(ctx, hipMemcpyAsync(h, tot, 16 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GX_HIP(ctx, hipStreamSynchronize(st));
        const int64_t nr = h[13];
        GX_TRY(gx_reserve(ctx, Ls.pc_off, (nr + 1) * sizeof(int32_t)));
        GX_TRY(gx_reserve(ctx, Ls.pc_list, (nr + 1) * sizeof(int32_t)));
        hipLaunchKernelGGL(k_walk_sph_wave, dim3(xcd_grid(ng)), dim3(64), 0, st, ng, groups, recv,
                           nodes, child, mom, rad, use_hmax, ovf, 1, nullptr, nullptr, nullptr,
                           (const int64_t*)Ls.pr_off.p, (int32_t*)Ls.pc_off.p,
                           (int32_t*)Ls.pc_list.p, sovf);
        GX_LAUNCH_CHECK(ctx);
        if (deep) {
            hipLaunchKernelGGL(k_walk_sph, dim3(gx_blocks(ng, 128)), dim3(128), 0, st, ng, groups,
                               recv, nodes, mom, nn, rad, use_hmax, sovf, 1, 0, nullptr, nullptr,
                               nullptr, (const int64_t*)Ls.pr_off.p, (int32_t*)Ls.pc_off.p,
                               (int32_t*)Ls.pc_list.p);
            GX_LAUNCH_CHECK(ctx);
        }
        v.ovf = ovf;
        v.off2 = (const int64_t*)Ls.pr_off.p;
        v.cnt2 = cnt2;
        v.begin2 = (const int32_t*)Ls.pc_off.p;
        v.cum2 = (const int32_t*)Ls.pc_list.p;
        v.tot2 = ptot2;
        pairs += h[10];
    }
    *list_pairs += pairs;
    Ls.n_groups = ng;
    Ls.n_ranges = h[1];
    *view = v;
    return GX_OK;
}

__global__ void k_flags_to_active(int nb, const uint32_t* __restrict__ flags,
                                  uint8_t* __restrict__ active) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nb) active[g] = flags[g] ? 1 : 0;
}

extern "C" int gx_sph_density(gx_ctx* ctx, const gx_particles* gas, gx_gas* gs, double n_ngb,
                              double gamma, double tol, int max_iter, gx_stats* stats) {
    if (!ctx || !gas || !gs) return GX_EINVAL;
    if (!gs->u || !gs->H64 || !gs->H || !gs->rho || gs->n != gas->n)
        return gx_fail(ctx, GX_EINVAL, "sph_density: gas arrays missing or length mismatch");
    if (!(n_ngb > 20.7) || !(tol > 0.0) || max_iter < 1 || !(gamma > 1.0))
        return gx_fail(ctx, GX_EINVAL,
                       "sph_density: need n_ngb > 20.625, tol > 0, max_iter >= 1, gamma > 1");
    GX_TRY(gx_tree_check(ctx, GX_TREE_GAS, gas));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    TreeSlot& T = ctx->tree[GX_TREE_GAS];
    ListSet& Ls = ctx->sph;
    const int nb = (int)T.n_groups;
    const int64_t n = T.n;
    if (stats) {
        *stats = gx_stats{};
        GX_HIP(ctx, hipEventRecord(ctx->ev0, st));
    }
    float *Hs, *rad;
    uint8_t* active;
    uint32_t* flags;
    unsigned long long* stat;
    GX_TRY(work(ctx, W_H, n * sizeof(float), (void**)&Hs));
    GX_TRY(work(ctx, W_RAD, nb * sizeof(float), (void**)&rad));
    GX_TRY(work(ctx, W_ACT, nb + 16, (void**)&active));
    GX_TRY(work(ctx, W_FLAG, nb * sizeof(uint32_t), (void**)&flags));
    GX_TRY(work(ctx, W_STAT, 16 * sizeof(unsigned long long), (void**)&stat));
    GX_TRY(gx_zero(ctx, stat, 16 * sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_sph_seed, dim3(gx_blocks(n, 256)), dim3(256), 0, st, n,
                       (const NodeRec*)T.nodes.p, (const MomRec*)T.mom.p, (const double4*)T.pos4.p,
                       (const uint32_t*)T.val[0].p, gs->H64, (float)n_ngb, (const double*)T.box.p,
                       Hs);
    hipLaunchKernelGGL(k_group_radius, dim3(nb), dim3(64), 0, st, nb, (const int32_t*)T.groups.p,
                       (const NodeRec*)T.nodes.p, Hs, SPH_MARGIN, rad);
    GX_LAUNCH_CHECK(ctx);
    const uint8_t* act = nullptr;
    int rounds = 0;
    unsigned long long h_stat[8] = {};
    int64_t list_pairs = 0;
    double kernel_ms = 0.0;
    for (;;) {
        ListView view;
        GX_TRY(gx_sph_walk(ctx, T, Ls, nb, (const int32_t*)T.groups.p, nullptr, rad, 0, act, &view,
                           &list_pairs));
        if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev2, st));
        hipLaunchKernelGGL(k_sph_density, dim3(xcd_grid(nb)), dim3(SPH_DT), 0, st, nb,
                           (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                           (const double4*)T.pos4.p,
                           (const uint32_t*)T.val[0].p, act, view, rad, (float)n_ngb, (float)tol,
                           max_iter, Hs, flags, stat, gs->u, (float)gamma, gs->H64, gs->H, gs->rho,
                           gs->P, gs->cs);
        GX_LAUNCH_CHECK(ctx);
        if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev3, st));
        GX_HIP(ctx, hipMemcpyAsync(h_stat, stat, 8 * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, st));
        GX_HIP(ctx, hipStreamSynchronize(st));
        if (stats) {
            float msk = 0;
            GX_HIP(ctx, hipEventElapsedTime(&msk, ctx->ev2, ctx->ev3));
            kernel_ms += msk;
        }
        rounds++;
        if (h_stat[3] == 0) break;
        if (rounds >= 16)
            return gx_fail(ctx, GX_ENOCONV, "sph_density: search radius did not settle in %d rounds",
                           rounds);
        hipLaunchKernelGGL(k_flags_to_active, dim3(gx_blocks(nb, 256)), dim3(256), 0, st, nb, flags,
                           active);
        act = active;
        GX_TRY(gx_zero(ctx, stat + 3, sizeof(unsigned long long)));
    }
    if (stats) {
        GX_HIP(ctx, hipEventRecord(ctx->ev1, st));
        GX_HIP(ctx, hipEventSynchronize(ctx->ev1));
        float ms = 0;
        GX_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        stats->ms = ms;
        stats->ms_kernel = kernel_ms;
        stats->n_noconv = (int64_t)h_stat[0];
        stats->n_iter_max = (int64_t)h_stat[1];
        stats->n_sph_list = list_pairs;
        stats->n_rewalk = rounds - 1;
        stats->n_groups = nb;
        stats->n_nodes = T.n_nodes;
    }
    if (h_stat[0] > 0)
        return gx_fail(ctx, GX_ENOCONV, "sph_density: %llu receivers hit max_iter", h_stat[0]);
    return GX_OK;
}

extern "C" int gx_sph_forces(gx_ctx* ctx, const gx_particles* gas, gx_gas* gs, double gamma,
                             double alpha, double* ax, double* ay, double* az, gx_stats* stats) {
    if (!ctx || !gas || !gs || !ax || !ay || !az) return GX_EINVAL;
    if (!gs->u || !gs->H || !gs->rho || !gs->dudt || !gs->vsig || gs->n != gas->n)
        return gx_fail(ctx, GX_EINVAL, "sph_forces: gas arrays missing or length mismatch");
    if (!gas->vx || !gas->vy || !gas->vz)
        return gx_fail(ctx, GX_EINVAL, "sph_forces: velocities missing");
    if (!(gamma > 1.0) || !(alpha >= 0.0))
        return gx_fail(ctx, GX_EINVAL, "sph_forces: bad gamma/alpha");
    GX_TRY(gx_tree_check(ctx, GX_TREE_GAS, gas));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    TreeSlot& T = ctx->tree[GX_TREE_GAS];
    ListSet& Ls = ctx->sph;
    const int nb = (int)T.n_groups;
    const int64_t n = T.n;
    if (stats) {
        *stats = gx_stats{};
        GX_HIP(ctx, hipEventRecord(ctx->ev0, st));
    }
    double4* sv;
    float4* ss;
    float* rad;
    unsigned long long* stat;
    GX_TRY(work(ctx, W_VEL, n * sizeof(double4), (void**)&sv));
    GX_TRY(work(ctx, W_SPH, n * sizeof(float4), (void**)&ss));
    GX_TRY(work(ctx, W_RAD, nb * sizeof(float), (void**)&rad));
    GX_TRY(work(ctx, W_STAT, 16 * sizeof(unsigned long long), (void**)&stat));
    GX_TRY(gx_zero(ctx, stat, 16 * sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_sph_prep, dim3(gx_blocks(n, 256)), dim3(256), 0, st, n,
                       (const uint32_t*)T.val[0].p, gas->vx, gas->vy, gas->vz, gs->u, gs->H, gs->rho,
                       (float)gamma, sv, ss);
    GX_TRY(gx_sph_node_hmax(ctx, T, ss));
    hipLaunchKernelGGL(k_group_hmax, dim3(gx_blocks(nb, 64)), dim3(64), 0, st, nb,
                       (const int32_t*)T.groups.p, (const MomRec*)T.mom.p, rad);
    GX_LAUNCH_CHECK(ctx);
    ListView view;
    int64_t list_pairs = 0;
    GX_TRY(gx_sph_walk(ctx, T, Ls, nb, (const int32_t*)T.groups.p, nullptr, rad, 1, nullptr, &view,
                       &list_pairs));
    if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev2, st));
    hipLaunchKernelGGL(k_sph_force, dim3(xcd_grid(nb)), dim3(SPH_DT), 0, st, nb,
                       (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                       (const double4*)T.pos4.p,
                       (const uint32_t*)T.val[0].p, sv, ss, view, (float)alpha, ax, ay, az,
                       gs->dudt, gs->vsig, stat);
    GX_LAUNCH_CHECK(ctx);
    if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev3, st));
    if (stats) {
        GX_HIP(ctx, hipEventRecord(ctx->ev1, st));
        GX_HIP(ctx, hipEventSynchronize(ctx->ev1));
        float ms = 0, msk = 0;
        GX_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        GX_HIP(ctx, hipEventElapsedTime(&msk, ctx->ev2, ctx->ev3));
        unsigned long long h[8];
        GX_HIP(ctx, hipMemcpy(h, stat, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        stats->ms = ms;
        stats->ms_kernel = msk;
        stats->n_sph_ngb = (int64_t)h[2];
        stats->n_sph_list = (int64_t)h[4];
        stats->n_groups = nb;
        stats->n_nodes = T.n_nodes;
    }
    return GX_OK;
}
