// gx_sph.hip -- SPH kernel size, density/pressure and hydro force (the
// "kernel size", "density and pressure" and "hydro force" items of Table 3,
// kernels of Table 4), Wendland C4 kernel, on the gas tree slot.
//
// Receivers: the gas tree's groups (maximal nodes of at most n_group
// particles; compact boxes keep candidate lists short).  One 256-thread
// workgroup per group.  Groups are usually smaller than 64, so the workgroup
// is cut into floor(256 / pad) slices of pad = min(group size, 64) lanes:
// every slice holds each receiver once and takes its own share of the
// candidates; the slices' partial sums go through LDS and are added in slice
// order, which gives every lane of a receiver bit-identical totals.  Each
// group's candidate list -- particles of every gas-tree leaf
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
    const NodeRec* __restrict__ nodes, int64_t nn, const double* __restrict__ wbox,
    const int4* __restrict__ wsph, const float* __restrict__ whmax,
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
    const NodeRec* __restrict__ nodes, int64_t nn, const double* __restrict__ wbox,
    const int4* __restrict__ wsph, const float* __restrict__ whmax,
    const float* __restrict__ radius, int use_hmax,
    const uint8_t* __restrict__ active, int mode, uint32_t* __restrict__ pr_cnt,
    uint32_t* __restrict__ pp_tot, unsigned long long* __restrict__ tot,
    const int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum, uint8_t* __restrict__ sovf);

#define SPH_THREADS 64
#define SPH_DT 256         // threads of the density and force kernels (4 waves per group)
#define SPH_CAP 2048       // force kernel: candidates per workgroup of a chunked long list
// density kernel: candidates kept in LDS, longer lists chunked over several
// workgroups (1024 or 512, for more workgroups per CU, measured slower on the
// 16M disk: 6.2 and 9.0 against 5.4 ms, as more groups take the chunked path)
#define SPH_DCAP 2048
#define SPH_TILE 256       // force kernel source tile (<= 256: hit lists hold 8-bit indices)
#define SPH_RANGES 1024    // capacity of a block's candidate range list (single-pass walk)
#define SPH_MARGIN 1.15f   // density search radius = margin x largest kernel size
#define SPH_HCAP 32        // per-lane hit list entries (density; candidate indices)
#define SPH_FCAP 32        // per-lane hit list entries (force; tile indices)
#define SPH_KAPPA 1.02f    // density hit lists hold candidates within kappa x kernel size

// 495 / (32 pi), (4 pi / 3) * 495 / (32 pi) = 495 / 24, 1155 / (4 pi)
#define WC4_NORM 4.9238032806262495f
#define NEFF_C 20.625f
#define GRADW_C 91.91197457030109f

// Work slots of the SPH calls (slots 8 - 12 belong to the SN calls).
enum {
    W_H = 0, W_RAD, W_ACT, W_FLAG, W_VEL, W_SPH, W_STAT,
    // long-list groups: chunk counts, item offsets, group list, items, Newton
    // state per slot, partial sums, finished flags
    W_HV = 13, W_HOFF, W_HLIST, W_ITEM, W_HST, W_PART, W_PARTV, W_GD,
    // per-group count of density evaluations inside the kernel support
    W_NGB = 23
};
static_assert(W_GD < 21, "work slots");

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

// Lanes per receiver slice: exactly the group's size (at most 64, larger
// groups take several passes); floor(SPH_DT / pad) slices share the
// candidates, so only SPH_DT mod pad lanes of the block idle.
__device__ __forceinline__ int slice_pad(int nG) { return nG < 1 ? 1 : (nG < 64 ? nG : 64); }

// Candidates ch .. che-1 of a group's list into LDS as FP32 positions
// relative to the group centre and masses (whole block; synchronises).
__device__ __forceinline__ void expand_chunk(const GroupList& L, int npp, int ch, int che,
                                             const double4* __restrict__ pos4, double cx,
                                             double cy, double cz, float4* __restrict__ cand,
                                             int* slot, int* roff, int* wtot, int tid,
                                             int nthreads) {
    list_slots(L, npp, ch, che, slot, roff, wtot, tid, nthreads);
    for (int k = tid; k < che - ch; k += nthreads) {
        const double4 p = pos4[slot[k]];
        cand[k] = make_float4((float)(p.x - cx), (float)(p.y - cy), (float)(p.z - cz),
                              (float)p.w);
    }
}

// Kernel sums s0 = sum m W-shape and s1 = sum m q^2 (1 + 5q) (1 - q)^5 over
// the candidates of one lane's hit list, in list order.
__device__ __forceinline__ void dens_hits(const uint16_t (*hl)[SPH_DT], int nh, int tid,
                                          const float4* __restrict__ cand, float xi, float yi,
                                          float zi, float Hinv2, float& s0, float& s1,
                                          unsigned& nin) {
    for (int j = 0; j < nh; j++) {
        const float4 c = cand[hl[j][tid]];
        const float dx = c.x - xi, dy = c.y - yi, dz = c.z - zi;
        const float q2 = (dx * dx + dy * dy + dz * dz) * Hinv2;
        if (q2 < 1.0f) {
            nin++;
            const float q = __builtin_amdgcn_sqrtf(q2);
            const float t = 1.0f - q;
            const float t2 = t * t;
            const float t5 = t2 * t2 * t;
            const float poly = 1.0f + q * (6.0f + q * (35.0f / 3.0f));
            s0 += c.w * t5 * t * poly;
            s1 += c.w * q2 * (1.0f + 5.0f * q) * t5;
        }
    }
}

// One lane's pass over candidates sl, sl + nsl, ... of cand[0, n): those
// within sqrt(lim) go to its hit list (flushed into the sums whenever some
// lane of the wave is near capacity).  Returns true when a flush happened,
// i.e. the list left behind is not complete.  Every lane of the wave runs
// the same number of steps.
__device__ __forceinline__ bool dens_scan(uint16_t (*hl)[SPH_DT], int& nh, int tid, int sl, int nsl,
                                          int n, bool act, const float4* __restrict__ cand,
                                          float xi, float yi, float zi, float lim, float Hinv2,
                                          float& s0, float& s1, unsigned& nin) {
    nh = 0;
    bool flushed = false;
    const int nst = (n + nsl - 1) / nsl;
    for (int m = 0; m < nst; m += 4) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = sl + (m + u) * nsl;
            const float4 c = cand[min(k, n - 1)];
            const float dx = c.x - xi, dy = c.y - yi, dz = c.z - zi;
            const float r2 = dx * dx + dy * dy + dz * dz;
            hl[nh][tid] = (uint16_t)k;  // kept only if counted
            nh += (act && k < n && r2 < lim) ? 1 : 0;
        }
        if (__ballot(nh > SPH_HCAP - 4)) {  // wave-uniform flush
            dens_hits(hl, nh, tid, cand, xi, yi, zi, Hinv2, s0, s1, nin);
            nh = 0;
            flushed = true;
        }
    }
    return flushed;
}

// One safeguarded Newton step on N_eff(H) = n_ngb from the kernel sums at H:
// the bracket [lo, hi] shrinks to H's side, the Newton iterate is kept when
// inside it, else bisection (or doubling while no upper bound exists).
// Done on |N_eff - n_ngb| <= tol, at max_iter evaluations, or when the next
// kernel size exceeds the list radius Rlim (over: the list must be redone).
__device__ __forceinline__ void newton_step(float s0, float s1, float mi, float n_ngb, float tol,
                                            int max_iter, float Rlim, float& H, float& lo,
                                            float& hi, float& S0, int& it, bool& done, bool& conv,
                                            bool& over) {
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
            done = true;
            over = true;
        }
        H = Hn;
    }
}

// Outputs of a converged (or capped) receiver in sorted slot s.
__device__ __forceinline__ void dens_write(int s, float H, float S0, const uint32_t* __restrict__ perm,
                                           const double* __restrict__ u, float gamma,
                                           double* __restrict__ H64, float* __restrict__ Hout,
                                           float* __restrict__ rho_out, float* __restrict__ P_out,
                                           float* __restrict__ cs_out) {
    const uint32_t o = perm[s];
    const float rho = WC4_NORM / (H * H * H) * S0;
    const double uu = u[o];
    H64[o] = (double)H;
    Hout[o] = H;
    rho_out[o] = rho;
    if (P_out) P_out[o] = (float)((double)(gamma - 1.0f) * (double)rho * uu);
    if (cs_out) cs_out[o] = (float)sqrt((double)gamma * (gamma - 1.0f) * uu);
}

// Per-group results: the list-redo flag and radius, iteration maximum and
// non-converged count, evaluated pairs (one update of each shared counter).
__device__ __forceinline__ void dens_group_stats(int g, int nflag, int nfail, int worst_it,
                                                 float hmax, unsigned long long evals,
                                                 uint32_t* __restrict__ flags,
                                                 float* __restrict__ rad,
                                                 unsigned long long* __restrict__ stat) {
    flags[g] = nflag ? 1u : 0u;
    atomicMax(&stat[1], (unsigned long long)worst_it);
    atomicAdd(&stat[5], evals);
    if (nflag) {
        rad[g] = hmax * SPH_MARGIN;
        atomicAdd(&stat[3], 1ull);
    } else {  // counted once, in the group's final round
        atomicAdd(&stat[0], (unsigned long long)nfail);
    }
}

// Kernel size and density: one 256-thread workgroup per group whose
// candidate list fits in LDS (longer lists are marked in hv and take the
// chunked path below).  The group's candidates sit once in LDS and are
// shared by its four waves.  The threads form 256 / pad slices (pad >= nG
// lanes each, every receiver once per slice); slice sl takes candidates sl,
// sl + nsl, ...  A lane tests its candidates against kappa x its kernel size
// and appends the ones inside to a hit list in LDS, then evaluates the kernel
// on the list only; a complete list is reused by later Newton passes while
// the kernel size stays within kappa x the size it was built for.  The
// slices' sums are combined by shuffles inside a wave and through LDS across
// waves (fixed order), and every copy of a receiver then takes the same
// safeguarded Newton step.
__global__ __launch_bounds__(SPH_DT) void k_sph_density(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const double4* __restrict__ pos4, const uint32_t* __restrict__ perm,
    const uint8_t* __restrict__ active, ListView L, float* __restrict__ rad, float n_ngb, float tol,
    int max_iter, float* __restrict__ Hs, uint32_t* __restrict__ flags, uint32_t* __restrict__ hv,
    unsigned long long* __restrict__ stat, uint32_t* __restrict__ gngb,
    const double* __restrict__ u, float gamma,
    double* __restrict__ H64, float* __restrict__ Hout, float* __restrict__ rho_out,
    float* __restrict__ P_out, float* __restrict__ cs_out) {
    const int g = xcd_chunk(blockIdx.x);
    if (g >= ng) return;
    if (active && !active[g]) return;
    const GroupList GL(L, g);
    const int npp = GL.npp;
    const NodeRec B = nodes[groups[g]];
    const int nG = B.end - B.begin;
    if (npp > SPH_DCAP && nG <= 64) {  // long list: chunked over several workgroups
        if (threadIdx.x == 0) hv[g] = (uint32_t)((npp + SPH_DCAP - 1) / SPH_DCAP);
        return;
    }
    // (a long list of a group above 64 receivers is evaluated here chunk by chunk)
    const bool in_lds = npp <= SPH_DCAP;
    __shared__ float4 cand[SPH_DCAP];
    __shared__ float2 red[SPH_DT];
    // hit lists; the list expansion uses the same space (slot + range
    // offsets) before the lists are built
    __shared__ __align__(16) uint16_t hl[SPH_HCAP][SPH_DT];
    __shared__ int wtot[SPH_DT / 64];
    static_assert(sizeof(hl) >= 2 * SPH_DCAP * sizeof(int), "expansion scratch");
    int* const xslot = reinterpret_cast<int*>(&hl[0][0]);
    int* const xroff = xslot + SPH_DCAP;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int pad = slice_pad(nG), nsl = SPH_DT / pad, il = tid % pad, sl = tid / pad;
    const double cx = (B.lo[0] + B.hi[0]) * 0.5;
    const double cy = (B.lo[1] + B.hi[1]) * 0.5;
    const double cz = (B.lo[2] + B.hi[2]) * 0.5;
    const float Rlim = rad[g];
    if (in_lds) expand_chunk(GL, npp, 0, npp, pos4, cx, cy, cz, cand, xslot, xroff, wtot, tid, SPH_DT);
    __syncthreads();

    int nflag = 0, nfail = 0, worst_it = 0;
    float hmax = 0.0f;
    unsigned long long evals = 0;  // receiver x candidate evaluations, all passes
    unsigned nin = 0;              // this lane's evaluations inside the kernel support
    for (int ic = 0; ic < nG; ic += pad) {
        const int s = B.begin + ic + il;
        const bool act = sl < nsl && ic + il < nG;
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
        const unsigned long long pass_evals = (unsigned long long)min(pad, nG - ic) * npp;
        float Hb = 0.0f;    // kernel size this lane's hit list was built for
        int nh = 0;         // entries in this lane's hit list
        bool have = false;  // every lane of the block holds a complete list
        for (;;) {
            evals += pass_evals;
            const float Hinv = 1.0f / H, Hinv2 = Hinv * Hinv;
            float s0 = 0.0f, s1 = 0.0f;
            if (in_lds) {
                const bool stale = __syncthreads_or(act && H > SPH_KAPPA * Hb);
                if (!have || stale) {
                    Hb = H;
                    const bool flushed = dens_scan(hl, nh, tid, sl, nsl, npp, act, cand, xi, yi,
                                                   zi, (SPH_KAPPA * SPH_KAPPA) * H * H, Hinv2, s0,
                                                   s1, nin);
                    have = !__syncthreads_or(flushed);
                }
                dens_hits(hl, nh, tid, cand, xi, yi, zi, Hinv2, s0, s1, nin);
            } else {
                for (int ch = 0; ch < npp; ch += SPH_DCAP) {
                    const int che = min(npp, ch + SPH_DCAP);
                    __syncthreads();
                    expand_chunk(GL, npp, ch, che, pos4, cx, cy, cz, cand, xslot, xroff, wtot,
                                 tid, SPH_DT);
                    __syncthreads();
                    dens_scan(hl, nh, tid, sl, nsl, che - ch, act, cand, xi, yi, zi, H * H, Hinv2,
                              s0, s1, nin);
                    dens_hits(hl, nh, tid, cand, xi, yi, zi, Hinv2, s0, s1, nin);
                }
            }
            // the slices' partial sums, added in slice order (every copy of
            // a receiver gets the same sums)
            red[tid] = make_float2(s0, s1);
            __syncthreads();
            s0 = 0.0f;
            s1 = 0.0f;
            for (int q = 0; q < nsl; q++) {
                const float2 r = red[q * pad + il];
                s0 += r.x;
                s1 += r.y;
            }
            if (!done)
                newton_step(s0, s1, mi, n_ngb, tol, max_iter, Rlim, H, lo, hi, S0, it, done, conv,
                            over);
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
                dens_write(s, H, S0, perm, u, gamma, H64, Hout, rho_out, P_out, cs_out);
            }
        }
    }
    nin = wave_sum(nin);
    if (lane == 0) wtot[wv] = (int)nin;
    __syncthreads();
    if (wv == 0) {  // slice 0 (the written copies) lies in wave 0
        nflag = (int)wave_sum((unsigned)nflag);
        nfail = (int)wave_sum((unsigned)nfail);
        worst_it = wave_max(worst_it);
        hmax = wave_max(hmax);
        if (lane == 0) {
            dens_group_stats(g, nflag, nfail, worst_it, hmax, evals, flags, rad, stat);
            unsigned tin = 0;
            for (int w = 0; w < SPH_DT / 64; w++) tin += (unsigned)wtot[w];
            gngb[g] += tin;  // one workgroup per group and round: no other writer
        }
    }
}

// Sum of n counters into *out (one workgroup, fixed order per thread; the
// statistics of a call, not on its critical path).
__global__ __launch_bounds__(256) void k_sum_u32(const uint32_t* __restrict__ v, int n,
                                                 unsigned long long* __restrict__ out) {
    __shared__ unsigned long long sh[4];
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += v[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// ---------------------------------------------------------------------------
// Long candidate lists: work items (group, chunk of SPH_DCAP candidates)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_long_items(int ng, const uint32_t* __restrict__ hv,
                                                    const int64_t* __restrict__ hoff,
                                                    int2* __restrict__ items,
                                                    int32_t* __restrict__ hlist,
                                                    uint32_t* __restrict__ nh_ctr) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng || hv[g] == 0) return;
    hlist[atomicAdd(nh_ctr, 1u)] = g;
    for (uint32_t c = 0; c < hv[g]; c++) items[hoff[g] + c] = make_int2(g, (int)c);
}

// Newton state of the receivers of long-list groups, per sorted slot:
// {lo, hi, S0, it | done << 8 | conv << 9 | over << 10}.
// Launched over at least as many blocks as there are long groups (nh[0]).
__global__ __launch_bounds__(64) void k_long_init(const uint32_t* __restrict__ nh,
                                                  const int32_t* __restrict__ hlist,
                                                  const int32_t* __restrict__ groups,
                                                  const NodeRec* __restrict__ nodes,
                                                  float4* __restrict__ hst,
                                                  uint8_t* __restrict__ gdone) {
    if (blockIdx.x >= nh[0]) return;
    const int g = hlist[blockIdx.x];
    const NodeRec B = nodes[groups[g]];
    const int il = threadIdx.x;
    if (il == 0) gdone[g] = 0;
    if (il < B.end - B.begin) hst[B.begin + il] = make_float4(0.0f, INFINITY, 0.0f, 0.0f);
}

// Partial kernel sums of one chunk of a long list at the receivers' current
// kernel sizes (skipping finished receivers): same lanes, slices and hit
// lists as k_sph_density, sums combined over slices and waves in a fixed
// order and stored per (item, receiver).
__global__ __launch_bounds__(SPH_DT) void k_sph_density_part(
    const int2* __restrict__ items, const int32_t* __restrict__ groups,
    const NodeRec* __restrict__ nodes, const double4* __restrict__ pos4, ListView L,
    const float* __restrict__ Hs, const float4* __restrict__ hst,
    const uint8_t* __restrict__ gdone, float2* __restrict__ part,
    uint32_t* __restrict__ gngb) {
    const int2 item = items[blockIdx.x];
    const int g = item.x;
    if (gdone[g]) return;
    __shared__ float4 cand[SPH_DCAP];
    __shared__ float2 red[SPH_DT];
    __shared__ __align__(16) uint16_t hl[SPH_HCAP][SPH_DT];
    __shared__ int wtot[SPH_DT / 64];
    int* const xslot = reinterpret_cast<int*>(&hl[0][0]);
    int* const xroff = xslot + SPH_DCAP;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const NodeRec B = nodes[groups[g]];
    const int nG = B.end - B.begin;
    const int pad = slice_pad(nG), nsl = SPH_DT / pad, il = tid % pad, sl = tid / pad;
    const double cx = (B.lo[0] + B.hi[0]) * 0.5;
    const double cy = (B.lo[1] + B.hi[1]) * 0.5;
    const double cz = (B.lo[2] + B.hi[2]) * 0.5;
    const GroupList GL(L, g);
    const int npp = GL.npp;
    const int ch = item.y * SPH_DCAP, che = min(npp, ch + SPH_DCAP);
    expand_chunk(GL, npp, ch, che, pos4, cx, cy, cz, cand, xslot, xroff, wtot, tid, SPH_DT);
    __syncthreads();
    const int s = B.begin + il;
    bool act = sl < nsl && il < nG;
    float xi = 0, yi = 0, zi = 0, H = 1.0f;
    if (act) {
        act = (__float_as_uint(hst[s].w) & 0x100u) == 0;  // not finished
        const double4 p = pos4[s];
        xi = (float)(p.x - cx);
        yi = (float)(p.y - cy);
        zi = (float)(p.z - cz);
        H = Hs[s];
    }
    const float Hinv = 1.0f / H, Hinv2 = Hinv * Hinv;
    float s0 = 0.0f, s1 = 0.0f;
    int nh;
    unsigned nin = 0;
    dens_scan(hl, nh, tid, sl, nsl, che - ch, act, cand, xi, yi, zi, H * H, Hinv2, s0, s1, nin);
    dens_hits(hl, nh, tid, cand, xi, yi, zi, Hinv2, s0, s1, nin);
    red[tid] = make_float2(s0, s1);
    nin = wave_sum(nin);
    if (lane == 0 && nin) atomicAdd(&gngb[g], nin);
    __syncthreads();
    if (sl == 0 && il < nG) {  // the slices' partial sums in slice order
        s0 = 0.0f;
        s1 = 0.0f;
        for (int q = 0; q < nsl; q++) {
            const float2 r = red[q * pad + il];
            s0 += r.x;
            s1 += r.y;
        }
        part[(int64_t)blockIdx.x * 64 + il] = make_float2(s0, s1);
    }
}

// Newton step for the receivers of one long-list group (one wave): chunk
// sums added in chunk order, then the step of k_sph_density; a group whose
// receivers are all done writes its outputs and statistics.
__global__ __launch_bounds__(64) void k_sph_density_long_step(
    const uint32_t* __restrict__ nh, const int32_t* __restrict__ hlist,
    const int32_t* __restrict__ groups,
    const NodeRec* __restrict__ nodes, const double4* __restrict__ pos4, ListView L,
    const uint32_t* __restrict__ hv, const int64_t* __restrict__ hoff,
    const float2* __restrict__ part, float* __restrict__ rad, float n_ngb, float tol, int max_iter,
    float* __restrict__ Hs, float4* __restrict__ hst, uint8_t* __restrict__ gdone,
    uint32_t* __restrict__ flags, uint32_t* __restrict__ pending,
    unsigned long long* __restrict__ stat, const uint32_t* __restrict__ perm,
    const double* __restrict__ u, float gamma, double* __restrict__ H64,
    float* __restrict__ Hout, float* __restrict__ rho_out, float* __restrict__ P_out,
    float* __restrict__ cs_out) {
    if (blockIdx.x >= nh[0]) return;
    const int g = hlist[blockIdx.x];
    if (gdone[g]) return;
    const NodeRec B = nodes[groups[g]];
    const int nG = B.end - B.begin;
    const int il = threadIdx.x;
    const bool act = il < nG;
    const int s = B.begin + il;
    const float Rlim = rad[g];
    float H = 1.0f, lo = 0.0f, hi = INFINITY, S0 = 0.0f;
    int it = 0;
    bool done = true, conv = false, over = false;
    if (act) {
        const float4 st = hst[s];
        const uint32_t bits = __float_as_uint(st.w);
        lo = st.x;
        hi = st.y;
        S0 = st.z;
        it = (int)(bits & 0xffu);
        done = bits & 0x100u;
        conv = bits & 0x200u;
        over = bits & 0x400u;
        H = Hs[s];
        if (!done) {
            float s0 = 0.0f, s1 = 0.0f;
            const int64_t i0 = hoff[g];
            for (uint32_t c = 0; c < hv[g]; c++) {
                const float2 p = part[(i0 + c) * 64 + il];
                s0 += p.x;
                s1 += p.y;
            }
            const float mi = (float)pos4[s].w;
            newton_step(s0, s1, mi, n_ngb, tol, max_iter, Rlim, H, lo, hi, S0, it, done, conv,
                        over);
            Hs[s] = H;
            hst[s] = make_float4(lo, hi, S0,
                                 __uint_as_float((uint32_t)it | (done ? 0x100u : 0u) |
                                                 (conv ? 0x200u : 0u) | (over ? 0x400u : 0u)));
        }
    }
    const bool all_done = __ballot(!done) == 0;
    if (il == 0) {
        const GroupList GL(L, g);
        atomicAdd(&stat[5], (unsigned long long)nG * (unsigned long long)GL.npp);
    }
    if (!all_done) {
        if (il == 0) atomicAdd(pending, 1u);
        return;
    }
    int nflag = 0, nfail = 0, worst_it = 0;
    float hmax = 0.0f;
    if (act) {
        hmax = H;
        worst_it = it;
        if (over) {
            nflag = 1;
        } else {
            if (!conv) nfail = 1;
            dens_write(s, H, S0, perm, u, gamma, H64, Hout, rho_out, P_out, cs_out);
        }
    }
    nflag = (int)wave_sum((unsigned)nflag);
    nfail = (int)wave_sum((unsigned)nfail);
    worst_it = wave_max(worst_it);
    hmax = wave_max(hmax);
    if (il == 0) {
        dens_group_stats(g, nflag, nfail, worst_it, hmax, 0ull, flags, rad, stat);
        gdone[g] = 1;
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
    T.hmax_ver++;
    return GX_OK;
}

__global__ __launch_bounds__(64) void k_group_hmax(int ng, const int32_t* __restrict__ groups,
                                                   const MomRec* __restrict__ mom,
                                                   float* __restrict__ rad) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ng) rad[g] = mom[groups[g]].hmax;
}

static_assert(SPH_TILE <= 256, "force hit lists store 8-bit tile indices");
static_assert(SPH_DCAP <= 65536, "density hit lists store 16-bit candidate indices");

// Pair terms of one lane's force hit list (tile indices, list order).
struct ForceRecv {
    float x, y, z, vx, vy, vz, Hinv, cw, rho, A, c;
};

__device__ __forceinline__ void force_hits(const uint8_t (*fl)[SPH_DT], int nh, int tid,
                                           const float4* __restrict__ t0,
                                           const float4* __restrict__ t1,
                                           const float4* __restrict__ t2,
                                           const float* __restrict__ tc, const ForceRecv& R,
                                           float alpha, float& fx, float& fy, float& fz,
                                           float& fu, float& vs) {
    for (int j = 0; j < nh; j++) {
        const int k = fl[j][tid];
        const float4 a = t0[k];  // x, y, z, H^2
        const float4 b = t1[k];  // vx, vy, vz, m
        const float4 d = t2[k];  // 1/H, gradient constant, rho, A
        const float cj = tc[k];
        const float dx = a.x - R.x, dy = a.y - R.y, dz = a.z - R.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * rinv;
        const float qi = r * R.Hinv, qj = r * d.x;
        // (1 - q)^5 vanishes at the support edge: clamping t at 0 gives the
        // same terms as a branch on q < 1
        const float ti = fmaxf(1.0f - qi, 0.0f), tj = fmaxf(1.0f - qj, 0.0f);
        const float ti2 = ti * ti, tj2 = tj * tj;
        const float gi = R.cw * (1.0f + 5.0f * qi) * ti2 * ti2 * ti;
        const float gj = d.y * (1.0f + 5.0f * qj) * tj2 * tj2 * tj;
        const float dvx = b.x - R.vx, dvy = b.y - R.vy, dvz = b.z - R.vz;
        const float vr = dvx * dx + dvy * dy + dvz * dz;
        const float w = vr * rinv;
        const float sig = R.c + cj - 3.0f * fminf(w, 0.0f);
        const float Pi = w < 0.0f ? -alpha * sig * w / (R.rho + d.z) : 0.0f;
        const float gbar = 0.5f * (gi + gj);
        const float f = b.w * (R.A * gi + d.w * gj + Pi * gbar);
        fx += f * dx;
        fy += f * dy;
        fz += f * dz;
        fu += b.w * (R.A * gi + 0.5f * Pi * gbar) * vr;
        vs = fmaxf(vs, sig);
    }
}

// Hydro force: one 256-thread workgroup per group, candidates staged in LDS
// tiles of SPH_TILE.  Lanes form slices as in the density kernel (slice sl
// takes tile entries sl, sl + nsl, ...).  A lane tests its entries for
// r < max(H_i, H_j), appends the pairs inside to a hit list in LDS (flushed
// whenever some lane of the wave is near capacity) and evaluates the pair
// terms on the list only.  FP32 sums per tile, FP64 across tiles, slices
// combined by shuffles and across waves through LDS in a fixed order.
//
// PART = false: one workgroup per group over its whole list, results added
// to the outputs; groups with lists longer than SPH_CAP are only marked in
// hv (chunk counts).  PART = true: one workgroup per work item (group, chunk
// of SPH_CAP candidates), FP64 partial sums and the chunk's largest signal
// velocity stored per (item, receiver) for k_sph_force_long_sum.
template <bool PART>
// at most 96 VGPRs (five wavefronts per SIMD; the slice sums share the tile
// storage so that five workgroups fit a CU's LDS): 3.05 against 3.2 ms on the
// 16M disk at the compiler's free choice of 99 registers and four wavefronts
__global__ __launch_bounds__(SPH_DT) __attribute__((amdgpu_waves_per_eu(5))) void k_sph_force(
    int ng, const int2* __restrict__ items, const int32_t* __restrict__ groups,
    const NodeRec* __restrict__ nodes, const double4* __restrict__ pos4,
    const uint32_t* __restrict__ perm, const double4* __restrict__ sv,
    const float4* __restrict__ ss, ListView L, float alpha, double* __restrict__ ax,
    double* __restrict__ ay, double* __restrict__ az, double* __restrict__ dudt,
    float* __restrict__ vsig_out, uint32_t* __restrict__ hv, double4* __restrict__ partd,
    float* __restrict__ partv, unsigned long long* __restrict__ stat) {
    int g, pb;
    if (PART) {
        const int2 it = items[blockIdx.x];
        g = it.x;
        pb = it.y * SPH_CAP;
    } else {
        g = xcd_chunk(blockIdx.x);
        if (g >= ng) return;
        pb = 0;
    }
    const GroupList GL(L, g);
    const int npp = GL.npp;
    if (!PART && npp > SPH_CAP && nodes[groups[g]].end - nodes[groups[g]].begin <= 64) {
        if (threadIdx.x == 0) hv[g] = (uint32_t)((npp + SPH_CAP - 1) / SPH_CAP);
        return;
    }
    const int pe = PART ? min(npp, pb + SPH_CAP) : npp;
    // source tiles; after a pass's last tile the same storage holds the
    // slices' sums (FP64 accelerations and du/dt in tiles 0-1, the largest
    // signal velocities in tile 2), between barriers
    __shared__ float4 tb3[3][SPH_TILE];
    __shared__ float tc[SPH_TILE];
    __shared__ int jidx[SPH_TILE], jroff[SPH_TILE], wtot[SPH_DT / 64];
    __shared__ uint8_t fl[SPH_FCAP][SPH_DT];
    static_assert(4 * SPH_DT * sizeof(double) <= 2 * SPH_TILE * sizeof(float4) &&
                      SPH_DT * sizeof(float) <= SPH_TILE * sizeof(float4),
                  "slice sums fit in the tile storage");
    float4* const t0 = tb3[0];
    float4* const t1 = tb3[1];
    float4* const t2 = tb3[2];
    double(*const redd)[SPH_DT] = reinterpret_cast<double(*)[SPH_DT]>(&tb3[0][0]);
    float* const redv = reinterpret_cast<float*>(&tb3[2][0]);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const NodeRec B = nodes[groups[g]];
    const int nG = B.end - B.begin;
    const int pad = slice_pad(nG), nsl = SPH_DT / pad, il = tid % pad, sl = tid / pad;
    const double cx = (B.lo[0] + B.hi[0]) * 0.5;
    const double cy = (B.lo[1] + B.hi[1]) * 0.5;
    const double cz = (B.lo[2] + B.hi[2]) * 0.5;
    const double4 vref = sv[B.begin];
    unsigned long long nin = 0;

    for (int ic = 0; ic < nG; ic += pad) {
        const int s = B.begin + ic + il;
        const bool act = sl < nsl && ic + il < nG;
        ForceRecv R = {0, 0, 0, 0, 0, 0, 1, 0, 1, 0, 0};
        float Hi = 1;
        if (act) {
            const double4 p = pos4[s];
            R.x = (float)(p.x - cx);
            R.y = (float)(p.y - cy);
            R.z = (float)(p.z - cz);
            const double4 v = sv[s];
            R.vx = (float)(v.x - vref.x);
            R.vy = (float)(v.y - vref.y);
            R.vz = (float)(v.z - vref.z);
            const float4 q = ss[s];
            Hi = q.x;
            R.Hinv = 1.0f / Hi;
            const float h2 = R.Hinv * R.Hinv;
            R.cw = -GRADW_C * h2 * h2 * R.Hinv;
            R.rho = q.y;
            R.A = q.z;
            R.c = q.w;
        }
        const float Hi2 = Hi * Hi;
        double AX = 0, AY = 0, AZ = 0, DU = 0;
        float vs = R.c;
        for (int tb = pb; tb < pe; tb += SPH_TILE) {
            const int tn = min(SPH_TILE, pe - tb);
            __syncthreads();
            list_slots(GL, npp, tb, tb + tn, jidx, jroff, wtot, tid, SPH_DT);
            for (int e = tid; e < tn; e += SPH_DT) {
                const int j = jidx[e];
                const double4 p = pos4[j];
                const double4 v = sv[j];
                const float4 q = ss[j];
                const float hinv = 1.0f / q.x;
                const float h2 = hinv * hinv;
                t0[e] = make_float4((float)(p.x - cx), (float)(p.y - cy), (float)(p.z - cz),
                                    q.x * q.x);
                t1[e] = make_float4((float)(v.x - vref.x), (float)(v.y - vref.y),
                                    (float)(v.z - vref.z), (float)p.w);
                t2[e] = make_float4(hinv, -GRADW_C * h2 * h2 * hinv, q.y, q.z);
                tc[e] = q.w;
            }
            __syncthreads();
            float fx = 0, fy = 0, fz = 0, fu = 0;
            const int nst = (tn + nsl - 1) / nsl;
            int nh = 0;
            for (int m = 0; m < nst; m += 4) {
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int k = sl + (m + u) * nsl;
                    const float4 a = t0[min(k, tn - 1)];
                    const float dx = a.x - R.x, dy = a.y - R.y, dz = a.z - R.z;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    fl[nh][tid] = (uint8_t)k;  // kept only if counted
                    nh += (act && k < tn && (r2 < Hi2 || r2 < a.w) && r2 > 0.0f) ? 1 : 0;
                }
                if (__ballot(nh > SPH_FCAP - 4)) {  // wave-uniform flush
                    nin += nh;
                    force_hits(fl, nh, tid, t0, t1, t2, tc, R, alpha, fx, fy, fz, fu, vs);
                    nh = 0;
                }
            }
            nin += nh;
            force_hits(fl, nh, tid, t0, t1, t2, tc, R, alpha, fx, fy, fz, fu, vs);
            AX += (double)fx;
            AY += (double)fy;
            AZ += (double)fz;
            DU += (double)fu;
        }
        // the slices' partial sums, added in slice order
        __syncthreads();
        redd[0][tid] = AX;
        redd[1][tid] = AY;
        redd[2][tid] = AZ;
        redd[3][tid] = DU;
        redv[tid] = vs;
        __syncthreads();
        if (act && sl == 0) {
            AX = AY = AZ = DU = 0.0;
            for (int q = 0; q < nsl; q++) {
                AX += redd[0][q * pad + il];
                AY += redd[1][q * pad + il];
                AZ += redd[2][q * pad + il];
                DU += redd[3][q * pad + il];
                vs = fmaxf(vs, redv[q * pad + il]);
            }
            if (PART) {
                const int64_t q = (int64_t)blockIdx.x * 64 + ic + il;
                partd[q] = make_double4(AX, AY, AZ, DU);
                partv[q] = vs;
            } else {
                const uint32_t o = perm[s];
                ax[o] += AX;
                ay[o] += AY;
                az[o] += AZ;
                dudt[o] = DU;
                vsig_out[o] = vs;
            }
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
        atomicAdd(&stat[4], (unsigned long long)nG * (unsigned long long)(pe - pb));
    }
}

// Receivers of one long-list group (one wave): chunk partials added in chunk
// order, results added to the outputs as in k_sph_force.
__global__ __launch_bounds__(64) void k_sph_force_long_sum(
    const uint32_t* __restrict__ nh, const int32_t* __restrict__ hlist,
    const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const uint32_t* __restrict__ hv, const int64_t* __restrict__ hoff,
    const double4* __restrict__ partd, const float* __restrict__ partv,
    const uint32_t* __restrict__ perm, double* __restrict__ ax, double* __restrict__ ay,
    double* __restrict__ az, double* __restrict__ dudt, float* __restrict__ vsig_out) {
    if (blockIdx.x >= nh[0]) return;
    const int g = hlist[blockIdx.x];
    const NodeRec B = nodes[groups[g]];
    const int il = threadIdx.x;
    if (il >= B.end - B.begin) return;
    double AX = 0, AY = 0, AZ = 0, DU = 0;
    float vs = 0.0f;
    const int64_t i0 = hoff[g];
    for (uint32_t c = 0; c < hv[g]; c++) {
        const int64_t q = (i0 + c) * 64 + il;
        const double4 p = partd[q];
        AX += p.x;
        AY += p.y;
        AZ += p.z;
        DU += p.w;
        vs = fmaxf(vs, partv[q]);
    }
    const uint32_t o = perm[B.begin + il];
    ax[o] += AX;
    ay[o] += AY;
    az[o] += AZ;
    dudt[o] = DU;
    vsig_out[o] = vs;
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
    GX_TRY(gx_walk_tree_sph(ctx, T, use_hmax));
    const double* wbox = (const double*)T.wbox.p;
    const int4* wsph = (const int4*)T.wsph.p;
    const float* whmax = (const float*)T.whmax.p;
    hipLaunchKernelGGL(k_walk_sph_bfs, dim3(xcd_chunk_grid(ng)), dim3(64), 0, st, ng, groups, recv,
                       (const NodeRec*)T.nodes.p, (int64_t)nn, wbox, wsph, whmax, rad, use_hmax,
                       active, SPH_RANGES, cnt, ptot, (unsigned long long*)tot,
                       (int32_t*)Ls.pr_begin.p, (int32_t*)Ls.pr_cum.p, ovf);
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
        const MomRec* mom = (const MomRec*)T.mom.p;
        hipLaunchKernelGGL(k_walk_sph_wave, dim3(xcd_chunk_grid(ng)), dim3(64), 0, st, ng, groups, recv,
                           nodes, (int64_t)nn, wbox, wsph, whmax, rad, use_hmax, ovf, 0, cnt2,
                           ptot2, (unsigned long long*)tot, nullptr, nullptr, nullptr, sovf);
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
        hipLaunchKernelGGL(k_walk_sph_wave, dim3(xcd_chunk_grid(ng)), dim3(64), 0, st, ng, groups, recv,
                           nodes, (int64_t)nn, wbox, wsph, whmax, rad, use_hmax, ovf, 1, nullptr,
                           nullptr, nullptr, (const int64_t*)Ls.pr_off.p, (int32_t*)Ls.pc_off.p,
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

// Work items of the groups marked in hv (chunk counts): item offsets hoff,
// items (group, chunk), group list hlist with its count in ctr[0].  Returns
// the number of items in *ni (0: nothing to do).
static int long_items(gx_ctx* ctx, int nb, const uint32_t* hv, int64_t** hoff, int2** items,
                      int32_t** hlist, uint32_t** ctr, int64_t* ni) {
    hipStream_t st = ctx->stream;
    GX_TRY(work(ctx, W_HOFF, (size_t)(nb + 1) * sizeof(int64_t), (void**)hoff));
    GX_TRY(work(ctx, W_HLIST, (size_t)(nb + 4) * sizeof(int32_t), (void**)hlist));
    *ctr = (uint32_t*)(*hlist + nb);
    GX_TRY((gx_scan<uint32_t, int64_t>(ctx, hv, *hoff, nb, *hoff + nb)));
    GX_HIP(ctx, hipMemcpyAsync(ni, *hoff + nb, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    GX_HIP(ctx, hipStreamSynchronize(st));
    if (*ni == 0) return GX_OK;
    GX_TRY(work(ctx, W_ITEM, (size_t)*ni * sizeof(int2), (void**)items));
    GX_TRY(gx_zero(ctx, *ctr, 4 * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_long_items, dim3(gx_blocks(nb, 256)), dim3(256), 0, st, nb, hv, *hoff,
                       *items, *hlist, *ctr);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// Groups whose candidate lists exceed SPH_DCAP: chunk sums over many
// workgroups, then one Newton step per receiver, until every receiver is
// done (at most max_iter passes).
static int density_long(gx_ctx* ctx, TreeSlot& T, const ListView& view, int nb, float* rad,
                        float n_ngb, float tol, int max_iter, float* Hs, uint32_t* flags,
                        const uint32_t* hv, unsigned long long* stat, uint32_t* gngb, gx_gas* gs,
                        float gamma) {
    hipStream_t st = ctx->stream;
    int64_t *hoff, ni = 0;
    int2* items;
    int32_t* hlist;
    uint32_t* ctr;
    GX_TRY(long_items(ctx, nb, hv, &hoff, &items, &hlist, &ctr, &ni));
    if (ni == 0) return GX_OK;
    if (ni > INT32_MAX / 64) return gx_fail(ctx, GX_EINVAL, "sph_density: too many list chunks");
    float4* hst;
    float2* part;
    uint8_t* gdone;
    GX_TRY(work(ctx, W_HST, (size_t)T.n * sizeof(float4), (void**)&hst));
    GX_TRY(work(ctx, W_PART, (size_t)ni * 64 * sizeof(float2), (void**)&part));
    GX_TRY(work(ctx, W_GD, (size_t)nb + 16, (void**)&gdone));
    // the group kernels run over ni blocks (>= the group count) and read the count on device
    hipLaunchKernelGGL(k_long_init, dim3((unsigned)ni), dim3(64), 0, st, (const uint32_t*)ctr,
                       (const int32_t*)hlist, (const int32_t*)T.groups.p,
                       (const NodeRec*)T.nodes.p, hst, gdone);
    GX_LAUNCH_CHECK(ctx);
    uint32_t pending = 0;
    int pass = 0;
    for (; pass < max_iter; pass++) {
        GX_TRY(gx_zero(ctx, ctr + 1, sizeof(uint32_t)));
        hipLaunchKernelGGL(k_sph_density_part, dim3((unsigned)ni), dim3(SPH_DT), 0, st,
                           (const int2*)items, (const int32_t*)T.groups.p,
                           (const NodeRec*)T.nodes.p, (const double4*)T.pos4.p, view,
                           (const float*)Hs, (const float4*)hst, (const uint8_t*)gdone, part,
                           gngb);
        hipLaunchKernelGGL(k_sph_density_long_step, dim3((unsigned)ni), dim3(64), 0, st,
                           (const uint32_t*)ctr, (const int32_t*)hlist,
                           (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                           (const double4*)T.pos4.p, view, hv, (const int64_t*)hoff,
                           (const float2*)part, rad, n_ngb, tol, max_iter, Hs, hst, gdone, flags,
                           ctr + 1, stat, (const uint32_t*)T.val[0].p, gs->u, gamma, gs->H64,
                           gs->H, gs->rho, gs->P, gs->cs);
        GX_LAUNCH_CHECK(ctx);
        GX_HIP(ctx, hipMemcpyAsync(&pending, ctr + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        GX_HIP(ctx, hipStreamSynchronize(st));
        if (pending == 0) break;
    }
    if (pending != 0)
        return gx_fail(ctx, GX_EHIP, "sph_density: long-list receivers unfinished after %d passes",
                       pass);
    return GX_OK;
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
    uint32_t* hv;
    GX_TRY(work(ctx, W_HV, (size_t)(nb + 1) * sizeof(uint32_t), (void**)&hv));
    uint32_t* gngb;
    GX_TRY(work(ctx, W_NGB, (size_t)(nb + 1) * sizeof(uint32_t), (void**)&gngb));
    GX_TRY(gx_zero(ctx, gngb, (size_t)nb * sizeof(uint32_t)));
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
        GX_TRY(gx_zero(ctx, hv, (size_t)nb * sizeof(uint32_t)));
        hipLaunchKernelGGL(k_sph_density, dim3(xcd_chunk_grid(nb)), dim3(SPH_DT), 0, st, nb,
                           (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                           (const double4*)T.pos4.p,
                           (const uint32_t*)T.val[0].p, act, view, rad, (float)n_ngb, (float)tol,
                           max_iter, Hs, flags, hv, stat, gngb, gs->u, (float)gamma, gs->H64, gs->H,
                           gs->rho, gs->P, gs->cs);
        GX_LAUNCH_CHECK(ctx);
        GX_TRY(density_long(ctx, T, view, nb, rad, (float)n_ngb, (float)tol, max_iter, Hs, flags,
                            hv, stat, gngb, gs, (float)gamma));
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
        hipLaunchKernelGGL(k_sum_u32, dim3(1), dim3(256), 0, st, (const uint32_t*)gngb, nb,
                           stat + 6);
        GX_LAUNCH_CHECK(ctx);
        GX_HIP(ctx, hipMemcpyAsync(h_stat + 6, stat + 6, sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, st));
        GX_HIP(ctx, hipStreamSynchronize(st));
        float ms = 0;
        GX_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        stats->ms = ms;
        stats->ms_kernel = kernel_ms;
        stats->n_noconv = (int64_t)h_stat[0];
        stats->n_iter_max = (int64_t)h_stat[1];
        stats->n_sph_list = (int64_t)h_stat[5];
        stats->n_sph_ngb = (int64_t)h_stat[6];
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
    uint32_t* hv;
    GX_TRY(work(ctx, W_HV, (size_t)(nb + 1) * sizeof(uint32_t), (void**)&hv));
    uint32_t* gngb;
    GX_TRY(work(ctx, W_NGB, (size_t)(nb + 1) * sizeof(uint32_t), (void**)&gngb));
    GX_TRY(gx_zero(ctx, gngb, (size_t)nb * sizeof(uint32_t)));
    GX_TRY(gx_zero(ctx, hv, (size_t)nb * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_sph_force<false>, dim3(xcd_chunk_grid(nb)), dim3(SPH_DT), 0, st, nb,
                       (const int2*)nullptr, (const int32_t*)T.groups.p,
                       (const NodeRec*)T.nodes.p, (const double4*)T.pos4.p,
                       (const uint32_t*)T.val[0].p, sv, ss, view, (float)alpha, ax, ay, az,
                       gs->dudt, gs->vsig, hv, (double4*)nullptr, (float*)nullptr, stat);
    GX_LAUNCH_CHECK(ctx);
    {  // groups with long lists: chunks over many workgroups, then ordered sums
        int64_t *hoff, ni = 0;
        int2* items;
        int32_t* hlist;
        uint32_t* ctr;
        GX_TRY(long_items(ctx, nb, hv, &hoff, &items, &hlist, &ctr, &ni));
        if (ni > 0) {
            if (ni > INT32_MAX / 64)
                return gx_fail(ctx, GX_EINVAL, "sph_forces: too many list chunks");
            double4* partd;
            float* partv;
            GX_TRY(work(ctx, W_PART, (size_t)ni * 64 * sizeof(double4), (void**)&partd));
            GX_TRY(work(ctx, W_PARTV, (size_t)ni * 64 * sizeof(float), (void**)&partv));
            hipLaunchKernelGGL(k_sph_force<true>, dim3((unsigned)ni), dim3(SPH_DT), 0, st, nb,
                               (const int2*)items, (const int32_t*)T.groups.p,
                               (const NodeRec*)T.nodes.p, (const double4*)T.pos4.p,
                               (const uint32_t*)T.val[0].p, sv, ss, view, (float)alpha, ax, ay,
                               az, gs->dudt, gs->vsig, hv, partd, partv, stat);
            hipLaunchKernelGGL(k_sph_force_long_sum, dim3((unsigned)ni), dim3(64), 0, st,
                               (const uint32_t*)ctr, (const int32_t*)hlist,
                               (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p,
                               (const uint32_t*)hv, (const int64_t*)hoff, (const double4*)partd,
                               (const float*)partv, (const uint32_t*)T.val[0].p, ax, ay, az,
                               gs->dudt, gs->vsig);
            GX_LAUNCH_CHECK(ctx);
        }
    }
    if (stats) GX_HIP(ctx, hipEventRecord(ctx->ev3, st));
    if (stats) {
        GX_HIP(ctx, hipEventRecord(ctx->ev1, st));
        GX_HIP(ctx, hipEventSynchronize(ctx->ev1));
        float ms = 0, msk = 0;
        GX_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        GX_HIP(ctx, hipEventElapsedTime(&msk, ctx->ev2, ctx->ev3));
        unsigned long long h[8];
        // on the context's stream: a plain copy would also wait for the
        // legacy default stream, i.e. for other contexts' work
        GX_HIP(ctx, hipMemcpyAsync(h, stat, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                   st));
        GX_HIP(ctx, hipStreamSynchronize(st));
        stats->ms = ms;
        stats->ms_kernel = msk;
        stats->n_sph_ngb = (int64_t)h[2];
        stats->n_sph_list = (int64_t)h[4];
        stats->n_groups = nb;
        stats->n_nodes = T.n_nodes;
    }
    return GX_OK;
}
