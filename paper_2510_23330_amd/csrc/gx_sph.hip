// gx_sph.hip -- SPH kernel size, density/pressure and hydro force (the
// "kernel size", "density and pressure" and "hydro force" items of Table 3,
// kernels of Table 4), Wendland C4 kernel, on the gas tree slot.
//
// Work layout: one wavefront (64 lanes) per receiving group of the gas tree
// (n_group <= 64 gives one receiver per lane; larger groups loop over chunks
// of 64).  The group's candidate list -- particles of every leaf whose box
// comes within the search radius of the group box -- is built by the
// stackless walk in gx_walk.hip.
//
// Density: the candidates are converted once to group-relative FP32
// (position, mass) and kept in LDS for all Newton iterations; each lane runs
// its own bracketed Newton iteration on N_eff(H) = (4 pi/3) H^3 rho(H) / m.
// A lane whose kernel size would leave the radius its list was built for
// stops and flags the group; the host re-walks only those groups with the
// larger radius and repeats.
//
// Force: one pass over the candidates in LDS tiles, pairs inside
// max(H_i, H_j), FP32 pair arithmetic, FP64 combination per tile.
#include "gx_internal.hpp"

int gx_tree_check(gx_ctx* ctx, int which, const gx_particles* p);

__global__ __launch_bounds__(128) void k_walk_sph(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const MomRec* __restrict__ mom, int nn, const float* __restrict__ radius, int use_hmax,
    const uint8_t* __restrict__ active, int mode, uint32_t* __restrict__ pr_cnt,
    uint32_t* __restrict__ pp_tot, unsigned long long* __restrict__ tot,
    const int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum);

#define SPH_CAP 2048     // candidates kept in LDS by the density kernel
#define SPH_TILE 256     // force kernel source tile
#define SPH_MARGIN 1.25f  // density search radius = margin x largest kernel size

// 495 / (32 pi), (4 pi / 3) * 495 / (32 pi) = 495 / 24, 1155 / (4 pi)
#define WC4_NORM 4.9238032806262495f
#define NEFF_C 20.625f
#define GRADW_C 91.91197457030109f

// ---------------------------------------------------------------------------
// Work buffers (sorted order unless noted)
// ---------------------------------------------------------------------------
enum {
    W_H = 0,     // float  kernel size per sorted slot
    W_RAD,       // float  per-group search radius
    W_ACT,       // uint8  per-group active flag
    W_FLAG,      // uint32 per-group "needs a larger radius" flag + counters
    W_VEL,       // double4 sorted velocities
    W_SPH,       // float4 sorted {H, rho, A = P/rho^2, c}
    W_STAT,      // u64 counters
};

static int work(gx_ctx* ctx, int k, size_t bytes, void** p) {
    GX_TRY(gx_reserve(ctx, ctx->sph_work[k], bytes));
    *p = ctx->sph_work[k].p;
    return GX_OK;
}

// Seed / gather kernel sizes: H_s[s] = H64[perm[s]] if positive and finite,
// else a seed from the group's mean density, (3 n_ngb m_i V_G / (4 pi M_G))^(1/3).
__global__ __launch_bounds__(64) void k_sph_seed(int ng, const int32_t* __restrict__ groups,
                                                 const NodeRec* __restrict__ nodes,
                                                 const MomRec* __restrict__ mom,
                                                 const double4* __restrict__ pos4,
                                                 const uint32_t* __restrict__ perm,
                                                 const double* __restrict__ H64, float n_ngb,
                                                 const double* __restrict__ box,
                                                 float* __restrict__ Hs, float* __restrict__ rad) {
    int g = blockIdx.x;
    const NodeRec gn = nodes[groups[g]];
    const double M = mom[groups[g]].M;
    double ext[3], vol = 1.0;
    for (int d = 0; d < 3; d++) ext[d] = gn.hi[d] - gn.lo[d];
    double side = ldexp(box[3], -gn.level);
    for (int d = 0; d < 3; d++) vol *= fmax(ext[d], 1e-3 * side);
    float hmax = 0.0f;
    for (int i = gn.begin + threadIdx.x; i < gn.end; i += 64) {
        double h = H64 ? H64[perm[i]] : -1.0;
        float hf;
        if (h > 0.0 && h < INFINITY) {
            hf = (float)h;
        } else {
            double rho = M / vol;
            hf = (float)cbrt(3.0 * (double)n_ngb * pos4[i].w / (4.0 * M_PI * rho));
        }
        Hs[i] = hf;
        hmax = fmaxf(hmax, hf);
    }
    hmax = wave_max(hmax);
    if (threadIdx.x == 0) rad[g] = hmax * SPH_MARGIN;
}

// Per-lane bracketed Newton on N_eff(H) over the group's candidates.
__global__ __launch_bounds__(64) void k_sph_density(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const double4* __restrict__ pos4, const uint32_t* __restrict__ perm,
    const uint8_t* __restrict__ active, const int64_t* __restrict__ pr_off,
    const int32_t* __restrict__ pr_begin, const int32_t* __restrict__ pr_cum,
    const uint32_t* __restrict__ pp_tot, float* __restrict__ rad, float n_ngb, float tol,
    int max_iter, float* __restrict__ Hs, uint32_t* __restrict__ flags,
    unsigned long long* __restrict__ stat, const double* __restrict__ u, float gamma,
    double* __restrict__ H64, float* __restrict__ Hout, float* __restrict__ rho_out,
    float* __restrict__ P_out, float* __restrict__ cs_out) {
    const int g = xcd_remap(blockIdx.x, ng);
    if (g >= ng) return;
    if (active && !active[g]) return;
    __shared__ float4 cand[SPH_CAP];
    __shared__ int32_t jidx[SPH_TILE];
    const int lane = threadIdx.x;
    const NodeRec gn = nodes[groups[g]];
    const double cx = (gn.lo[0] + gn.hi[0]) * 0.5;
    const double cy = (gn.lo[1] + gn.hi[1]) * 0.5;
    const double cz = (gn.lo[2] + gn.hi[2]) * 0.5;
    const int npp = (int)pp_tot[g];
    const int64_t r0 = pr_off[g], r1 = pr_off[g + 1];
    const float Rlim = rad[g];
    const bool in_lds = npp <= SPH_CAP;

    // expand ranges and convert candidates (all of them when they fit in LDS)
    auto load_chunk = [&](int ch, int che) {
        for (int64_t r = r0; r < r1; r++) {
            const int c = pr_cum[r];
            const int cn = (r + 1 < r1) ? pr_cum[r + 1] : npp;
            const int b = pr_begin[r];
            const int lo = max(c, ch), hi = min(cn, che);
            for (int k = lo + lane; k < hi; k += 64) {
                const double4 p = pos4[b + (k - c)];
                cand[k - ch] = make_float4((float)(p.x - cx), (float)(p.y - cy), (float)(p.z - cz),
                                           (float)p.w);
            }
        }
    };
    if (in_lds) load_chunk(0, npp);
    __syncthreads();

    int worst_it = 0, nfail = 0, nflag = 0;
    unsigned long long ngb = 0;
    for (int ic = gn.begin; ic < gn.end; ic += 64) {
        const int s = ic + lane;
        const bool act = s < gn.end;
        float xi = 0, yi = 0, zi = 0, mi = 1;
        float H = 1.0f;
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
        while (true) {
            // uniform loop: every lane walks the candidates while any lane iterates
            if (__ballot(!done) == 0ull) break;
            const float Hinv = 1.0f / H, Hinv2 = Hinv * Hinv;
            float s0 = 0.0f, s1 = 0.0f;
            int cntin = 0;
            for (int ch = 0; ch < npp; ch += SPH_CAP) {
                const int che = min(npp, ch + SPH_CAP);
                if (!in_lds) {
                    __syncthreads();
                    load_chunk(ch, che);
                    __syncthreads();
                }
#pragma unroll 4
                for (int k = 0; k < che - ch; k++) {
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
                        cntin++;
                    }
                }
            }
            if (!done) {
                it++;
                S0 = s0;
                const float neff = NEFF_C * s0 / mi;
                const float f = neff - n_ngb;
                if (fabsf(f) <= tol) {
                    done = true;
                    conv = true;
                    ngb += (unsigned long long)cntin;
                } else if (it >= max_iter) {
                    done = true;
                    ngb += (unsigned long long)cntin;
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
                        H = Hn;
                    } else {
                        H = Hn;
                    }
                }
            }
        }
        if (act) {
            Hs[s] = H;
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
                if (P_out) P_out[o] = (float)((gamma - 1.0f) * (double)rho * uu);
                if (cs_out) cs_out[o] = (float)sqrt((double)gamma * (gamma - 1.0f) * uu);
            }
        }
    }
    // wave reductions of the per-lane counters
    nflag = (int)wave_sum((unsigned)nflag);
    nfail = (int)wave_sum((unsigned)nfail);
    worst_it = wave_max(worst_it);
    ngb = wave_sum(ngb);
    float hmax = 0.0f;
    for (int s = gn.begin + lane; s < gn.end; s += 64) hmax = fmaxf(hmax, Hs[s]);
    hmax = wave_max(hmax);
    if (lane == 0) {
        flags[g] = nflag ? 1u : 0u;
        atomicMax(&stat[1], (unsigned long long)worst_it);
        if (nflag) {
            rad[g] = hmax * SPH_MARGIN;
            atomicAdd(&stat[3], 1ull);
        } else {  // counted once, in the group's final round
            atomicAdd(&stat[0], (unsigned long long)nfail);
            atomicAdd(&stat[2], ngb);
        }
    }
}

// ---------------------------------------------------------------------------
// Force
// ---------------------------------------------------------------------------
// Sorted per-particle state for the force: velocity (FP64) and
// {H, rho, A = P / rho^2, c} (FP32) with P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u).
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

__global__ __launch_bounds__(64) void k_group_hmax(int ng, const int32_t* __restrict__ groups,
                                                   const MomRec* __restrict__ mom,
                                                   float* __restrict__ rad) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ng) rad[g] = mom[groups[g]].hmax;
}

__global__ __launch_bounds__(64) void k_sph_force(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const double4* __restrict__ pos4, const uint32_t* __restrict__ perm,
    const double4* __restrict__ sv, const float4* __restrict__ ss,
    const int64_t* __restrict__ pr_off, const int32_t* __restrict__ pr_begin,
    const int32_t* __restrict__ pr_cum, const uint32_t* __restrict__ pp_tot, float alpha,
    double* __restrict__ ax, double* __restrict__ ay, double* __restrict__ az,
    double* __restrict__ dudt, float* __restrict__ vsig_out, unsigned long long* __restrict__ stat) {
    const int g = xcd_remap(blockIdx.x, ng);
    if (g >= ng) return;
    __shared__ float tx[SPH_TILE], ty[SPH_TILE], tz[SPH_TILE], tvx[SPH_TILE], tvy[SPH_TILE],
        tvz[SPH_TILE], tm[SPH_TILE], thi[SPH_TILE], th2[SPH_TILE], tcw[SPH_TILE], trho[SPH_TILE],
        tA[SPH_TILE], tc[SPH_TILE];
    const int lane = threadIdx.x;
    const NodeRec gn = nodes[groups[g]];
    const double cx = (gn.lo[0] + gn.hi[0]) * 0.5;
    const double cy = (gn.lo[1] + gn.hi[1]) * 0.5;
    const double cz = (gn.lo[2] + gn.hi[2]) * 0.5;
    const double4 vref = sv[gn.begin];
    const int npp = (int)pp_tot[g];
    const int64_t r0 = pr_off[g], r1 = pr_off[g + 1];
    unsigned long long nin = 0;

    for (int ic = gn.begin; ic < gn.end; ic += 64) {
        const int s = ic + lane;
        const bool act = s < gn.end;
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
        for (int t0 = 0; t0 < npp; t0 += SPH_TILE) {
            const int tn = min(SPH_TILE, npp - t0);
            __syncthreads();
            // stage the tile: lane-strided over the ranges that overlap it
            for (int64_t r = r0; r < r1; r++) {
                const int c = pr_cum[r];
                const int cn = (r + 1 < r1) ? pr_cum[r + 1] : npp;
                const int lo = max(c, t0), hi = min(cn, t0 + tn);
                if (lo >= hi) {
                    if (c >= t0 + tn) break;
                    continue;
                }
                const int b = pr_begin[r];
                for (int k = lo + lane; k < hi; k += 64) {
                    const int j = b + (k - c);
                    const int e = k - t0;
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
            }
            __syncthreads();
            if (act) {
                float fx = 0, fy = 0, fz = 0, fu = 0;
#pragma unroll 2
                for (int k = 0; k < tn; k++) {
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
        if (act) {
            const uint32_t o = perm[s];
            ax[o] += AX;
            ay[o] += AY;
            az[o] += AZ;
            dudt[o] = DU;
            vsig_out[o] = vs;
        }
    }
    nin = wave_sum(nin);
    if (lane == 0) {
        atomicAdd(&stat[2], nin);
        atomicAdd(&stat[4], (unsigned long long)(gn.end - gn.begin) * (unsigned long long)npp);
    }
}

// ---------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------
static int sph_walk(gx_ctx* ctx, TreeSlot& T, ListSet& Ls, const float* rad, int use_hmax,
                    const uint8_t* active) {
    hipStream_t st = ctx->stream;
    const int ng = (int)T.n_groups, nn = (int)T.n_nodes;
    GX_TRY(gx_reserve(ctx, Ls.tot, 8 * sizeof(int64_t)));
    GX_TRY(gx_reserve(ctx, Ls.pr_cnt, (ng + 1) * sizeof(uint32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pp_tot, (ng + 1) * sizeof(uint32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pr_off, (ng + 1) * sizeof(int64_t)));
    int64_t* tot = (int64_t*)Ls.tot.p;
    GX_TRY(gx_zero(ctx, tot, 8 * sizeof(int64_t)));
    hipLaunchKernelGGL(k_walk_sph, dim3(gx_blocks(ng, 128)), dim3(128), 0, st, ng,
                       (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                       (const MomRec*)T.mom.p, nn, rad, use_hmax, active, 0, (uint32_t*)Ls.pr_cnt.p,
                       (uint32_t*)Ls.pp_tot.p, (unsigned long long*)tot, nullptr, nullptr, nullptr);
    GX_LAUNCH_CHECK(ctx);
    GX_TRY((gx_scan<uint32_t, int64_t>(ctx, (const uint32_t*)Ls.pr_cnt.p, (int64_t*)Ls.pr_off.p, ng,
                                       tot + 1)));
    GX_HIP(ctx, hipMemcpyAsync((int64_t*)Ls.pr_off.p + ng, tot + 1, 8, hipMemcpyDeviceToDevice, st));
    int64_t h[2];
    GX_HIP(ctx, hipMemcpyAsync(h, tot, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    GX_HIP(ctx, hipStreamSynchronize(st));
    Ls.n_ranges = h[1];
    GX_TRY(gx_reserve(ctx, Ls.pr_begin, (h[1] + 1) * sizeof(int32_t)));
    GX_TRY(gx_reserve(ctx, Ls.pr_cum, (h[1] + 1) * sizeof(int32_t)));
    hipLaunchKernelGGL(k_walk_sph, dim3(gx_blocks(ng, 128)), dim3(128), 0, st, ng,
                       (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                       (const MomRec*)T.mom.p, nn, rad, use_hmax, active, 1, nullptr, nullptr,
                       nullptr, (const int64_t*)Ls.pr_off.p, (int32_t*)Ls.pr_begin.p,
                       (int32_t*)Ls.pr_cum.p);
    GX_LAUNCH_CHECK(ctx);
    Ls.n_groups = ng;
    return GX_OK;
}

__global__ void k_flags_to_active(int ng, const uint32_t* __restrict__ flags,
                                  uint8_t* __restrict__ active) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ng) active[g] = flags[g] ? 1 : 0;
}

extern "C" int gx_sph_density(gx_ctx* ctx, const gx_particles* gas, gx_gas* gs, double n_ngb,
                              double gamma, double tol, int max_iter, gx_stats* stats) {
    if (!ctx || !gas || !gs) return GX_EINVAL;
    if (!gs->u || !gs->H64 || !gs->H || !gs->rho || gs->n != gas->n)
        return gx_fail(ctx, GX_EINVAL, "sph_density: gas arrays missing or length mismatch");
    if (!(n_ngb > 20.7) || !(tol > 0.0) || max_iter < 1 || !(gamma > 1.0))
        return gx_fail(ctx, GX_EINVAL, "sph_density: need n_ngb > 20.625, tol > 0, max_iter >= 1, gamma > 1");
    GX_TRY(gx_tree_check(ctx, GX_TREE_GAS, gas));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    TreeSlot& T = ctx->tree[GX_TREE_GAS];
    ListSet& Ls = ctx->sph;
    const int ng = (int)T.n_groups;
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
    GX_TRY(work(ctx, W_RAD, ng * sizeof(float), (void**)&rad));
    GX_TRY(work(ctx, W_ACT, ng + 16, (void**)&active));
    GX_TRY(work(ctx, W_FLAG, ng * sizeof(uint32_t), (void**)&flags));
    GX_TRY(work(ctx, W_STAT, 16 * sizeof(unsigned long long), (void**)&stat));
    GX_TRY(gx_zero(ctx, stat, 16 * sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_sph_seed, dim3(ng), dim3(64), 0, st, ng, (const int32_t*)T.groups.p,
                       (const NodeRec*)T.nodes.p, (const MomRec*)T.mom.p, (const double4*)T.pos4.p,
                       (const uint32_t*)T.val[0].p, gs->H64, (float)n_ngb, (const double*)T.box.p,
                       Hs, rad);
    GX_LAUNCH_CHECK(ctx);
    const uint8_t* act = nullptr;
    int rounds = 0;
    unsigned long long h_stat[8] = {};
    int64_t list_pairs = 0;
    double kernel_ms = 0.0;
    for (;;) {
        GX_TRY(sph_walk(ctx, T, Ls, rad, 0, act));
        int64_t hl[4];
        GX_HIP(ctx, hipMemcpyAsync(hl, Ls.tot.p, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev2, st));
        hipLaunchKernelGGL(k_sph_density, dim3(xcd_grid(ng)), dim3(64), 0, st, ng,
                           (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                           (const double4*)T.pos4.p, (const uint32_t*)T.val[0].p, act,
                           (const int64_t*)Ls.pr_off.p, (const int32_t*)Ls.pr_begin.p,
                           (const int32_t*)Ls.pr_cum.p, (const uint32_t*)Ls.pp_tot.p, rad,
                           (float)n_ngb, (float)tol, max_iter, Hs, flags, stat, gs->u,
                           (float)gamma, gs->H64, gs->H, gs->rho, gs->P, gs->cs);
        GX_LAUNCH_CHECK(ctx);
        if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev3, st));
        GX_HIP(ctx, hipMemcpyAsync(h_stat, stat, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        GX_HIP(ctx, hipStreamSynchronize(st));
        if (stats) {
            float msk = 0;
            GX_HIP(ctx, hipEventElapsedTime(&msk, ctx->ev2, ctx->ev3));
            kernel_ms += msk;
        }
        list_pairs += hl[2];
        rounds++;
        if (h_stat[3] == 0) break;
        if (rounds >= 12)
            return gx_fail(ctx, GX_ENOCONV, "sph_density: search radius did not settle in %d rounds", rounds);
        // next round: only the flagged groups, with their enlarged radius
        hipLaunchKernelGGL(k_flags_to_active, dim3(gx_blocks(ng, 256)), dim3(256), 0, st, ng, flags,
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
        stats->n_noconv = (int64_t)h_stat[0];
        stats->n_iter_max = (int64_t)h_stat[1];
        stats->n_sph_ngb = (int64_t)h_stat[2];
        stats->n_sph_list = list_pairs;
        stats->n_rewalk = rounds - 1;
        stats->ms_kernel = kernel_ms;
        stats->n_groups = ng;
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
    if (!gas->vx || !gas->vy || !gas->vz) return gx_fail(ctx, GX_EINVAL, "sph_forces: velocities missing");
    if (!(gamma > 1.0) || !(alpha >= 0.0)) return gx_fail(ctx, GX_EINVAL, "sph_forces: bad gamma/alpha");
    GX_TRY(gx_tree_check(ctx, GX_TREE_GAS, gas));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    TreeSlot& T = ctx->tree[GX_TREE_GAS];
    ListSet& Ls = ctx->sph;
    const int ng = (int)T.n_groups;
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
    GX_TRY(work(ctx, W_RAD, ng * sizeof(float), (void**)&rad));
    GX_TRY(work(ctx, W_STAT, 16 * sizeof(unsigned long long), (void**)&stat));
    GX_TRY(gx_zero(ctx, stat, 16 * sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_sph_prep, dim3(gx_blocks(n, 256)), dim3(256), 0, st, n,
                       (const uint32_t*)T.val[0].p, gas->vx, gas->vy, gas->vz, gs->u, gs->H, gs->rho,
                       (float)gamma, sv, ss);
    for (int l = GX_MAX_LEVEL; l >= 0; l--) {
        int c = (int)T.lvl_hist[l];
        if (!c) continue;
        int64_t off = 0;
        for (int k = 0; k < l; k++) off += T.lvl_hist[k];
        hipLaunchKernelGGL(k_hmax_level, dim3(gx_blocks(c, 256)), dim3(256), 0, st, c,
                           (const int32_t*)T.lvl_ids.p + off, (const NodeRec*)T.nodes.p,
                           (MomRec*)T.mom.p, ss);
    }
    hipLaunchKernelGGL(k_group_hmax, dim3(gx_blocks(ng, 64)), dim3(64), 0, st, ng,
                       (const int32_t*)T.groups.p, (const MomRec*)T.mom.p, rad);
    GX_LAUNCH_CHECK(ctx);
    GX_TRY(sph_walk(ctx, T, Ls, rad, 1, nullptr));
    if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev2, st));
    hipLaunchKernelGGL(k_sph_force, dim3(xcd_grid(ng)), dim3(64), 0, st, ng,
                       (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                       (const double4*)T.pos4.p, (const uint32_t*)T.val[0].p, sv, ss,
                       (const int64_t*)Ls.pr_off.p, (const int32_t*)Ls.pr_begin.p,
                       (const int32_t*)Ls.pr_cum.p, (const uint32_t*)Ls.pp_tot.p, (float)alpha, ax,
                       ay, az, gs->dudt, gs->vsig, stat);
    GX_LAUNCH_CHECK(ctx);
    if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev3, st));
    if (stats) {
        GX_HIP(ctx, hipEventRecord(ctx->ev1, st));
        GX_HIP(ctx, hipEventSynchronize(ctx->ev1));
        float ms = 0;
        GX_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        float msk = 0;
        GX_HIP(ctx, hipEventElapsedTime(&msk, ctx->ev2, ctx->ev3));
        unsigned long long h[8];
        GX_HIP(ctx, hipMemcpy(h, stat, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        stats->ms = ms;
        stats->ms_kernel = msk;
        stats->n_sph_ngb = (int64_t)h[2];
        stats->n_sph_list = (int64_t)h[4];
        stats->n_groups = ng;
        stats->n_nodes = T.n_nodes;
    }
    return GX_OK;
}
