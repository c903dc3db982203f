// gx_walk.hip -- interaction-list construction for receiving groups
// (Sec. 5.2.2: groups of particles share one list built by one tree walk).
//
// Compiled with -ffp-contract=off: the gravity opening criterion is evaluated
// as the exact IEEE sequence
//     d2  = ((t_x * t_x) + (t_y * t_y)) + (t_z * t_z),
//           t_a = max(0, max(lo_c,a - hi_G,a, lo_G,a - hi_c,a))
//     lc  = L * 2^-level
//     accept  <=>  lc * lc < theta2 * d2
// so the lists equal those of any implementation of the same definition.
//
// The walk is stackless: nodes are stored in depth-first pre-order with a
// `next` index (first node after the subtree), so "skip" is next and "open"
// is id + 1.  One thread walks one group; consecutive groups are neighbours
// in key order and follow nearly the same path, which keeps a wave coherent.
#include "gx_internal.hpp"
#include <climits>

#pragma clang fp contract(off)

__device__ __forceinline__ double box_dist2(const double* glo, const double* ghi, const double* lo,
                                            const double* hi) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        // max(0, lo - ghi, glo - hi); fmax gives the same square as the
        // compare-and-select form (boxes hold no NaN; a -0 squares to +0)
        const double t = fmax(fmax(lo[d] - ghi[d], glo[d] - hi[d]), 0.0);
        double tt = t * t;
        s = s + tt;
    }
    return s;
}

// Largest squared distance from a point of box [lo, hi] to box [glo, ghi]
// (per axis max(0, glo - lo, hi - ghi)), summed in the order of box_dist2.
// For every box inside [lo, hi] box_dist2 is <= this value in floating point
// (each operation is monotone), so a node with box_far2 < R^2 holds only
// leaves the SPH walks would accept one by one: its whole sorted range is
// emitted at once, giving the same candidate set in fewer, longer ranges.
__device__ __forceinline__ double box_far2(const double* glo, const double* ghi, const double* lo,
                                           const double* hi) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double t1 = glo[d] - lo[d];
        double t2 = hi[d] - ghi[d];
        double t = t1 > t2 ? t1 : t2;
        t = t < 0.0 ? 0.0 : t;
        double tt = t * t;
        s = s + tt;
    }
    return s;
}

// mode 0: count (pc cells, pp ranges, pp particles; interaction totals)
// mode 1: fill the CSR lists at the offsets produced from the counts
// mode 2: one pass into fixed slots of cap_pc / cap_pr entries per group
//         (entries past a slot are counted, not written; such groups are
//         counted in tot[4])
// Modes 0 and 2 also record the largest per-group counts (tot[5], tot[6]).
__global__ __launch_bounds__(128) void k_walk_grav(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes, int nn,
    const double* __restrict__ box, double theta2, int mode, uint32_t* __restrict__ pc_cnt,
    uint32_t* __restrict__ pr_cnt, uint32_t* __restrict__ pp_tot,
    unsigned long long* __restrict__ tot, const int64_t* __restrict__ pc_off,
    int32_t* __restrict__ pc_list, const int64_t* __restrict__ pr_off,
    int32_t* __restrict__ pr_begin, int32_t* __restrict__ pr_cum, int cap_pc, int cap_pr) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const NodeRec G = nodes[groups[g]];
    const double L = box[3];
    int npc = 0, npr = 0, npp = 0, last_end = -1;
    const bool write = mode != 0;
    const int64_t pco = mode == 1 ? pc_off[g] : (int64_t)g * cap_pc;
    const int64_t pro = mode == 1 ? pr_off[g] : (int64_t)g * cap_pr;
    const int lim_pc = mode == 2 ? cap_pc : INT_MAX, lim_pr = mode == 2 ? cap_pr : INT_MAX;
    for (int n = 0; n < nn;) {
        const NodeRec& nd = nodes[n];
        double lo[3] = {nd.lo[0], nd.lo[1], nd.lo[2]};
        double hi[3] = {nd.hi[0], nd.hi[1], nd.hi[2]};
        int lev = nd.level, nxt = nd.next;
        double d2 = box_dist2(G.lo, G.hi, lo, hi);
        double lc = ldexp(L, -lev);
        double lhs = lc * lc;
        double rhs = theta2 * d2;
        if (lhs < rhs) {
            if (write && npc < lim_pc) pc_list[pco + npc] = n;
            npc++;
            n = nxt;
        } else if (nd.leaf) {
            int b = nd.begin, e = nd.end;
            if (b != last_end) {
                if (write && npr < lim_pr) {
                    pr_begin[pro + npr] = b;
                    pr_cum[pro + npr] = npp;
                }
                npr++;
            }
            npp += e - b;
            last_end = e;
            n = nxt;
        } else {
            n = n + 1;
        }
    }
    if (mode != 1) {
        pc_cnt[g] = (uint32_t)npc;
        pr_cnt[g] = (uint32_t)npr;
        pp_tot[g] = (uint32_t)npp;
        unsigned long long nG = (unsigned long long)(G.end - G.begin);
        atomicAdd(&tot[2], nG * (unsigned long long)npp);
        atomicAdd(&tot[3], nG * (unsigned long long)npc);
        atomicAdd(&tot[0], (unsigned long long)npc);
        atomicAdd(&tot[1], (unsigned long long)npr);
        atomicMax(&tot[5], (unsigned long long)npc);
        atomicMax(&tot[6], (unsigned long long)npr);
        if (mode == 2 && (npc > cap_pc || npr > cap_pr)) atomicAdd(&tot[4], 1ull);
    }
}

// Level-order copy of the tree for the gravity walk.  Sorting the nodes by
// level (stable, so each level keeps pre-order) makes the children of every
// node consecutive, and the children of consecutive nodes follow one another.
// The walk then needs only a node's first child and child count, and the
// nodes one wavefront pops together (children of consecutively popped nodes)
// sit side by side in the arrays: a 64-lane load of one field touches a few
// cache lines instead of one line per lane.
__global__ __launch_bounds__(256) void k_lvl_keys(int64_t nn, const NodeRec* __restrict__ nodes,
                                                  uint64_t* __restrict__ key,
                                                  uint32_t* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    key[i] = (uint64_t)(uint16_t)nodes[i].level;
    val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_lvl_pos(int64_t nn, const uint32_t* __restrict__ order,
                                                 int32_t* __restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    pos[order[i]] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_walk_arrays(int64_t nn, const uint32_t* __restrict__ order,
                                                     const int32_t* __restrict__ pos,
                                                     const NodeRec* __restrict__ nodes,
                                                     double* __restrict__ wbox,
                                                     int4* __restrict__ wrec,
                                                     int4* __restrict__ wsph) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const int32_t p = (int32_t)order[i];
    const NodeRec nd = nodes[p];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        wbox[d * nn + i] = nd.lo[d];
        wbox[(3 + d) * nn + i] = nd.hi[d];
    }
    const uint32_t meta = (uint32_t)(uint16_t)nd.level | ((uint32_t)(uint8_t)nd.leaf << 16) |
                          ((uint32_t)(uint8_t)nd.nchild << 24);
    // the first child of an internal node follows it in pre-order
    const int32_t first = nd.nchild > 0 ? pos[p + 1] : 0;
    wrec[i] = make_int4(p, (int32_t)meta, nd.leaf ? nd.begin : first, nd.end);
    wsph[i] = make_int4(nd.begin, nd.end, first, (int32_t)meta);
}

__global__ __launch_bounds__(256) void k_walk_hmax(int64_t nn, const uint32_t* __restrict__ order,
                                                   const MomRec* __restrict__ mom,
                                                   float* __restrict__ whmax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    whmax[i] = mom[order[i]].hmax;
}

int gx_walk_tree(gx_ctx* ctx, TreeSlot& T) {
    if (T.walk_ready) return GX_OK;
    const int64_t nn = T.n_nodes;
    if (nn <= 0 || nn >= ((int64_t)1 << 31) / 8)
        return gx_fail(ctx, GX_EINVAL, "walk arrays: %lld nodes", (long long)nn);
    hipStream_t st = ctx->stream;
    for (int k = 0; k < 2; k++) {
        GX_TRY(gx_reserve(ctx, T.wkey[k], nn * sizeof(uint64_t)));
        GX_TRY(gx_reserve(ctx, T.wval[k], nn * sizeof(uint32_t)));
    }
    GX_TRY(gx_reserve(ctx, T.wbox, 6 * nn * sizeof(double)));
    GX_TRY(gx_reserve(ctx, T.wrec, nn * sizeof(int4)));
    GX_TRY(gx_reserve(ctx, T.wsph, nn * sizeof(int4)));
    GX_TRY(gx_reserve(ctx, T.whmax, nn * sizeof(float)));
    hipLaunchKernelGGL(k_lvl_keys, dim3(gx_blocks(nn, 256)), dim3(256), 0, st, nn,
                       (const NodeRec*)T.nodes.p, (uint64_t*)T.wkey[0].p, (uint32_t*)T.wval[0].p);
    GX_LAUNCH_CHECK(ctx);
    GX_TRY(gx_radix_sort_bufs(ctx, T.wkey, T.wval, nn, 8));  // levels < 256: one pass
    hipLaunchKernelGGL(k_lvl_pos, dim3(gx_blocks(nn, 256)), dim3(256), 0, st, nn,
                       (const uint32_t*)T.wval[0].p, (int32_t*)T.wval[1].p);
    hipLaunchKernelGGL(k_walk_arrays, dim3(gx_blocks(nn, 256)), dim3(256), 0, st, nn,
                       (const uint32_t*)T.wval[0].p, (const int32_t*)T.wval[1].p,
                       (const NodeRec*)T.nodes.p, (double*)T.wbox.p, (int4*)T.wrec.p,
                       (int4*)T.wsph.p);
    GX_LAUNCH_CHECK(ctx);
    T.walk_ready = 1;
    T.whmax_ver = -1;
    return GX_OK;
}

// Level-order walk arrays plus, when use_hmax, the node kernel sizes in level
// order as of the last gx_sph_node_hmax.
int gx_walk_tree_sph(gx_ctx* ctx, TreeSlot& T, int use_hmax) {
    GX_TRY(gx_walk_tree(ctx, T));
    if (use_hmax && T.whmax_ver != T.hmax_ver) {
        const int64_t nn = T.n_nodes;
        hipLaunchKernelGGL(k_walk_hmax, dim3(gx_blocks(nn, 256)), dim3(256), 0, ctx->stream, nn,
                           (const uint32_t*)T.wval[0].p, (const MomRec*)T.mom.p,
                           (float*)T.whmax.p);
        GX_LAUNCH_CHECK(ctx);
        T.whmax_ver = T.hmax_ver;
    }
    return GX_OK;
}

// Wave-cooperative gravity walk into per-group slots (the one-pass mode of
// k_walk_grav) over the level-order arrays: one wavefront per group, an LDS
// stack of pending level-order positions; each step pops up to GWALK_WK x 64
// nodes (GWALK_WK per lane, so that as many node reads are in flight per
// round trip to memory), applies the opening criterion in the same IEEE
// sequence, appends accepted cells (by pre-order id) and opened leaves to the
// slots by ballot compaction and pushes the children of opened internal
// nodes in the order the nodes were popped.  Lists come out in a different
// order than the stackless walk's (the same sets).  Per group it writes the
// list sizes, an overflow flag (slot or stack) and the deepest stack;
// k_group_totals then forms the totals (the caller builds the lists in two
// passes when any group overflowed).
// The stack is sized per launch: GWALK_STACK_S entries (8 KB of LDS, about
// twenty wavefronts per CU: the walk is latency-bound once its loads are
// coalesced) or GWALK_STACK_L (16 KB) for deeper walks.
#define GWALK_STACK_S 2048
#define GWALK_STACK_L 4096
#define GWALK_WK 2
template <int GWALK_STACK>
__global__ __launch_bounds__(64) void k_walk_grav_wave(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes, int64_t nn,
    const double* __restrict__ wbox, const int4* __restrict__ wrec,
    const double* __restrict__ box, double theta2, uint32_t* __restrict__ pc_cnt,
    uint32_t* __restrict__ pr_cnt, uint32_t* __restrict__ pp_tot, int32_t* __restrict__ pc_list,
    int32_t* __restrict__ pr_begin, int32_t* __restrict__ pr_cum, int cap_pc, int cap_pr,
    uint8_t* __restrict__ gflag, int32_t* __restrict__ gdepth, int scap) {
    // scap: entries of stk in use, 1 <= scap <= GWALK_STACK
    const int g = xcd_chunk(blockIdx.x);
    if (g >= ng) return;
    const int lane = threadIdx.x;
    const char* bx[6];
#pragma unroll
    for (int d = 0; d < 6; d++) bx[d] = reinterpret_cast<const char*>(wbox + d * nn);
    __shared__ int32_t stk[GWALK_STACK];
    const NodeRec G = nodes[groups[g]];
    const double L = box[3];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t pco = (int64_t)g * cap_pc, pro = (int64_t)g * cap_pr;
    if (lane == 0) stk[0] = 0;  // the root is alone on level 0
    int sp = 1, npc = 0, npr = 0, npp = 0, over = 0, spmax = 1;
    __syncthreads();
    while (sp > 0 && !over) {
        const int take = sp < 64 * GWALK_WK ? sp : 64 * GWALK_WK;
        const int b0 = sp - take;
        int n[GWALK_WK];
#pragma unroll
        for (int w = 0; w < GWALK_WK; w++) {
            const int q = lane + 64 * w;
            n[w] = q < take ? stk[b0 + q] : -1;
        }
        __syncthreads();
        sp = b0;
        // all loads of this step first; a row no lane uses is skipped, idle
        // lanes of a used row read the root and discard it
        double lo[GWALK_WK][3], hi[GWALK_WK][3];
        int4 rec[GWALK_WK];
#pragma unroll
        for (int w = 0; w < GWALK_WK; w++) {
            if (64 * w >= take) {  // wave-uniform
                rec[w] = make_int4(0, 0, 0, 0);
#pragma unroll
                for (int d = 0; d < 3; d++) lo[w][d] = hi[w][d] = 0.0;
                continue;
            }
            // 32-bit byte offsets from per-array bases (loads with a scalar
            // base address; the arrays are below 2 GB, checked at build)
            const uint32_t i = n[w] >= 0 ? (uint32_t)n[w] : 0u;
            const uint32_t o8 = i * 8u;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                lo[w][d] = *reinterpret_cast<const double*>(bx[d] + o8);
                hi[w][d] = *reinterpret_cast<const double*>(bx[3 + d] + o8);
            }
            rec[w] = *reinterpret_cast<const int4*>(reinterpret_cast<const char*>(wrec) + 2u * o8);
        }
        int nch[GWALK_WK], first[GWALK_WK];
#pragma unroll
        for (int w = 0; w < GWALK_WK; w++) {
            const uint32_t meta = (uint32_t)rec[w].y;
            const int level = (int)(int16_t)(meta & 0xffffu);
            const bool isleaf = ((meta >> 16) & 0xffu) != 0;
            const double d2 = box_dist2(G.lo, G.hi, lo[w], hi[w]);
            const double lc = ldexp(L, -level);
            const double lhs = lc * lc;
            const double rhs = theta2 * d2;
            const bool live = n[w] >= 0;
            const bool acc = live && lhs < rhs;
            const bool leaf = live && !acc && isleaf;
            const bool open = live && !acc && !isleaf;
            const int b = rec[w].z, e = rec[w].w;
            // accepted cells (pre-order ids)
            const uint64_t am = __ballot(acc);
            if (acc) {
                const int pos = npc + __popcll(am & lt);
                if (pos < cap_pc) pc_list[pco + pos] = rec[w].x;
            }
            npc += __popcll(am);
            // opened leaves: particle ranges
            const uint64_t lm = __ballot(leaf);
            const int sz = leaf ? e - b : 0;
            const int incl = wave_incl_scan(sz);
            if (leaf) {
                const int pos = npr + __popcll(lm & lt);
                if (pos < cap_pr) {
                    pr_begin[pro + pos] = b;
                    pr_cum[pro + pos] = npp + incl - sz;
                }
            }
            npr += __popcll(lm);
            npp += wave_last(incl);
            nch[w] = open ? (int)(meta >> 24) : 0;
            first[w] = b;
        }
        // children of opened internal nodes onto the stack in the order the
        // nodes were popped (w = 0 rows, then w = 1): a node's children are
        // the consecutive positions first .. first + nchild - 1
        int coff[GWALK_WK], ctot = 0;
#pragma unroll
        for (int w = 0; w < GWALK_WK; w++) {
            const int ci = wave_incl_scan(nch[w]);
            coff[w] = sp + ctot + ci - nch[w];
            ctot += wave_last(ci);
        }
        if (sp + ctot > scap) {
            over = 1;
        } else {
#pragma unroll
            for (int w = 0; w < GWALK_WK; w++)
#pragma unroll
                for (int k = 0; k < 8; k++)
                    if (k < nch[w]) stk[coff[w] + k] = first[w] + k;
            sp += ctot;
            spmax = sp > spmax ? sp : spmax;
        }
        __syncthreads();
    }
    if (lane == 0) {
        // per-group results only; k_group_totals forms the sums (one shared
        // counter update per block instead of several per group)
        pc_cnt[g] = (uint32_t)npc;
        pr_cnt[g] = (uint32_t)npr;
        pp_tot[g] = (uint32_t)npp;
        gflag[g] = (over || npc > cap_pc || npr > cap_pr) ? 1 : 0;
        gdepth[g] = over ? scap + 1 : spmax;
    }
}

int gx_walk_stack_small(const gx_ctx* ctx) {
    const int c = ctx->walk_small_cap;
    return (c > 0 && c < GWALK_STACK_S) ? c : GWALK_STACK_S;
}

int gx_walk_grav_wave(gx_ctx* ctx, TreeSlot& T, int ng, double theta2, bool small_stack,
                      uint32_t* pc_cnt, uint32_t* pr_cnt, uint32_t* pp_tot, int32_t* pc_list,
                      int32_t* pr_begin, int32_t* pr_cum, int cap_pc, int cap_pr,
                      uint8_t* gflag, int32_t* gdepth) {
    GX_TRY(gx_walk_tree(ctx, T));
    auto kern = small_stack ? k_walk_grav_wave<GWALK_STACK_S> : k_walk_grav_wave<GWALK_STACK_L>;
    const int scap = small_stack ? gx_walk_stack_small(ctx) : GWALK_STACK_L;
    hipLaunchKernelGGL(kern, dim3(xcd_chunk_grid(ng)), dim3(64), 0, ctx->stream, ng,
                       (const int32_t*)T.groups.p, (const NodeRec*)T.nodes.p, (int64_t)T.n_nodes,
                       (const double*)T.wbox.p, (const int4*)T.wrec.p, (const double*)T.box.p,
                       theta2, pc_cnt, pr_cnt, pp_tot, pc_list, pr_begin, pr_cum, cap_pc, cap_pr,
                       gflag, gdepth, scap);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// Totals of a set of per-group lists: tot[0] += sum c0, tot[1] += sum c1,
// tot[2] += sum nG pp, tot[3] += sum nG c0, tot[4] += sum flag, and maxima
// tot[5] = max c0, tot[6] = max c1, tot[7] = max depth (any input may be
// NULL).  nG = receiver size (groups[g] of nodes, or recv[g]).
__global__ __launch_bounds__(256) void k_group_totals(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, const uint32_t* __restrict__ c0,
    const uint32_t* __restrict__ c1, const uint32_t* __restrict__ pp,
    const uint8_t* __restrict__ flag, const int32_t* __restrict__ depth,
    unsigned long long* __restrict__ tot) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long s[5] = {0, 0, 0, 0, 0}, m[3] = {0, 0, 0};
    if (g < ng) {
        const NodeRec& G = recv ? recv[g] : nodes[groups[g]];
        const unsigned long long nG = (unsigned long long)(G.end - G.begin);
        const unsigned long long a = c0 ? c0[g] : 0, b = c1 ? c1[g] : 0, q = pp ? pp[g] : 0;
        s[0] = a;
        s[1] = b;
        s[2] = nG * q;
        s[3] = nG * a;
        s[4] = flag ? flag[g] : 0;
        m[0] = a;
        m[1] = b;
        m[2] = depth ? (unsigned long long)depth[g] : 0;
    }
    __shared__ unsigned long long sh[4][8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; k++) {
        const unsigned long long t = wave_sum(s[k]);
        if (lane == 0) sh[wv][k] = t;
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const unsigned long long t = wave_max(m[k]);
        if (lane == 0) sh[wv][5 + k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = threadIdx.x;
        unsigned long long v = sh[0][k];
        for (int w = 1; w < 4; w++) v = k < 5 ? v + sh[w][k] : (sh[w][k] > v ? sh[w][k] : v);
        if (k < 5) {
            if (v) atomicAdd(&tot[k], v);
        } else {
            atomicMax(&tot[k], v);
        }
    }
}

// Direct summation expressed as lists: every group sees the single range [0, n).
__global__ void k_direct_lists(int ng, int n, const int32_t* __restrict__ groups,
                               const NodeRec* __restrict__ nodes, int64_t* __restrict__ pc_off,
                               int64_t* __restrict__ pr_off, uint32_t* __restrict__ pc_cnt,
                               uint32_t* __restrict__ pr_cnt, int32_t* __restrict__ pr_begin,
                               int32_t* __restrict__ pr_cum, uint32_t* __restrict__ pp_tot,
                               unsigned long long* __restrict__ tot) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > ng) return;
    pc_off[g] = 0;
    pr_off[g] = g;
    if (g == ng) return;
    pc_cnt[g] = 0;
    pr_cnt[g] = 1;
    pr_begin[g] = 0;
    pr_cum[g] = 0;
    pp_tot[g] = (uint32_t)n;
    NodeRec G = nodes[groups[g]];
    atomicAdd(&tot[2], (unsigned long long)(G.end - G.begin) * (unsigned long long)n);
}

// SPH candidate lists for receiver blocks: leaves whose box lies within reach
// of the block box, reach = max(R_b, hmax_c), R_b the block's search radius
// (density: margin x its largest kernel size; force: its largest kernel size)
// and hmax_c the largest kernel size in the node (force only).
// mode 0: count; mode 1: fill at pr_off; mode 2: single pass writing at
// b * cap with per-block counts (entries past cap are counted, not written,
// and the block is reported in tot[4]); mode 3: count like mode 0 but leave
// the counts of inactive blocks untouched.
__global__ __launch_bounds__(128) void k_walk_sph(
    int nb, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, const MomRec* __restrict__ mom, int nn,
    const float* __restrict__ radius, int use_hmax,
    const uint8_t* __restrict__ active, int mode, int cap, uint32_t* __restrict__ pr_cnt,
    uint32_t* __restrict__ pp_tot, unsigned long long* __restrict__ tot,
    const int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nb) return;
    if (active && !active[g]) {
        if (mode == 0 || mode == 2) {
            pr_cnt[g] = 0;
            pp_tot[g] = 0;
        }
        return;
    }
    const NodeRec G = recv ? recv[g] : nodes[groups[g]];
    const double RG = (double)radius[g];
    int npr = 0, npp = 0, last_end = -1;
    const int64_t pro = (mode == 1) ? pr_off[g] : (mode == 2 ? (int64_t)g * cap : 0);
    const bool write = mode == 1 || mode == 2;
    for (int n = 0; n < nn;) {
        const NodeRec& nd = nodes[n];
        double lo[3] = {nd.lo[0], nd.lo[1], nd.lo[2]};
        double hi[3] = {nd.hi[0], nd.hi[1], nd.hi[2]};
        double d2 = box_dist2(G.lo, G.hi, lo, hi);
        double R = RG;
        if (use_hmax) {
            double hm = (double)mom[n].hmax;
            R = hm > R ? hm : R;
        }
        if (d2 >= R * R) {
            n = nd.next;
        } else if (nd.leaf || box_far2(G.lo, G.hi, lo, hi) < RG * RG) {
            int b = nd.begin, e = nd.end;
            if (b != last_end) {
                if (write && (mode == 1 || npr < cap)) {
                    pr_begin[pro + npr] = b;
                    pr_cum[pro + npr] = npp;
                }
                npr++;
            }
            npp += e - b;
            last_end = e;
            n = nd.next;
        } else {
            n = n + 1;
        }
    }
    if (mode != 1) {
        pr_cnt[g] = (uint32_t)npr;
        pp_tot[g] = (uint32_t)npp;
        atomicAdd(&tot[2], (unsigned long long)(G.end - G.begin) * (unsigned long long)npp);
        atomicAdd(&tot[1], (unsigned long long)npr);
        if (mode == 2 && npr > cap) atomicAdd(&tot[4], 1ull);
    }
}

// Receivers are tree groups (groups[g]) or, when recv is non-null, arbitrary
// boxes (recv[g]).
// Wave-cooperative SPH walk: one wavefront per receiving group traverses the
// tree breadth-first.  The 64 lanes test 64 frontier nodes at a time; leaves
// within reach are appended to the group's fixed-capacity range slot (ballot
// compaction, prefix sums of their sizes give the running offsets) and
// intersecting internal nodes push their children (from the child table)
// onto the next frontier in LDS.  Ranges come out level by level, not in key
// order; consumers only rely on the running offsets.  A frontier or slot
// overflow sets the group's ovf flag (the caller then builds that group's
// list with the depth-first walks).
// 512 entries (4 KB of LDS for both frontiers, many wavefronts per CU): a
// wider frontier sends fewer groups to the depth-first walk but runs far
// fewer walks at once, which measured slower on the 16M disk.
#define BFS_FMAX 512
__global__ __launch_bounds__(64) void k_walk_sph_bfs(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, int64_t nn, const double* __restrict__ wbox,
    const int4* __restrict__ wsph, const float* __restrict__ whmax,
    const float* __restrict__ radius, int use_hmax, const uint8_t* __restrict__ active, int cap,
    uint32_t* __restrict__ pr_cnt, uint32_t* __restrict__ pp_tot,
    unsigned long long* __restrict__ tot, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum, uint8_t* __restrict__ ovf) {
    const int g = xcd_chunk(blockIdx.x);
    if (g >= ng) return;
    const int lane = threadIdx.x;
    if (active && !active[g]) {
        if (lane == 0) {
            pr_cnt[g] = 0;
            pp_tot[g] = 0;
            ovf[g] = 0;
        }
        return;
    }
    __shared__ int32_t fr[2][BFS_FMAX];
    const NodeRec G = recv ? recv[g] : nodes[groups[g]];
    const double RG = (double)radius[g];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t slot = (int64_t)g * cap;
    if (lane == 0) fr[0][0] = 0;
    int cnt = 1, cur = 0, nout = 0, npp = 0, over = 0;
    __syncthreads();
    while (cnt > 0) {
        int ncnt = 0;
        for (int base = 0; base < cnt; base += 64) {
            const int idx = base + lane;
            bool inter = false, leaf = false;
            int b = 0, e = 0, first = 0, nchild = 0;
            if (idx < cnt) {
                const int64_t n = fr[cur][idx];  // level-order position
                double lo[3], hi[3];
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    lo[d] = wbox[d * nn + n];
                    hi[d] = wbox[(3 + d) * nn + n];
                }
                const int4 r = wsph[n];
                const double d2 = box_dist2(G.lo, G.hi, lo, hi);
                double R = RG;
                if (use_hmax) {
                    const double hm = (double)whmax[n];
                    R = hm > R ? hm : R;
                }
                inter = d2 < R * R;
                const bool isleaf = (((uint32_t)r.w >> 16) & 0xffu) != 0;
                leaf = isleaf || (inter && box_far2(G.lo, G.hi, lo, hi) < RG * RG);
                b = r.x;
                e = r.y;
                first = r.z;
                nchild = (int)((uint32_t)r.w >> 24);
            }
            // emit leaves (and wholly covered nodes)
            const bool emit = inter && leaf;
            const uint64_t em = __ballot(emit);
            const int sz = emit ? e - b : 0;
            const int incl = wave_incl_scan(sz);
            if (emit) {
                const int pos = nout + __popcll(em & lt);
                if (pos < cap) {
                    pr_begin[slot + pos] = b;
                    pr_cum[slot + pos] = npp + incl - sz;
                }
            }
            nout += __popcll(em);
            npp += wave_last(incl);
            // open internal nodes: children are first .. first + nchild - 1
            const int nch = (inter && !leaf) ? nchild : 0;
            const int cincl = wave_incl_scan(nch);
            const int coff = ncnt + cincl - nch;
            for (int k = 0; k < nch; k++) {
                if (coff + k < BFS_FMAX) fr[cur ^ 1][coff + k] = first + k;
            }
            ncnt += wave_last(cincl);
        }
        __syncthreads();
        if (ncnt > BFS_FMAX) {
            over = 1;
            ncnt = BFS_FMAX;
        }
        cnt = ncnt;
        cur ^= 1;
    }
    if (lane == 0) {  // totals: k_group_totals over pr_cnt, pp_tot and ovf
        const bool bad = over || nout > cap;
        ovf[g] = bad ? 1 : 0;
        pr_cnt[g] = bad ? 0u : (uint32_t)nout;
        pp_tot[g] = bad ? 0u : (uint32_t)npp;
    }
}

// Wave-cooperative depth-first walk for the groups whose lists overflow the
// fixed slots of k_walk_sph_bfs (large kernel sizes: many candidate leaves).
// One wavefront per group; an LDS stack of pending nodes: each iteration pops
// up to 64 nodes from the top, one per lane, emits the intersecting leaves
// and pushes the children of intersecting internal nodes.  Working from the
// top keeps the stack shallow (it grows with tree depth, not with the
// frontier width).  mode 0 counts ranges and list length per group; mode 1
// writes them at pr_off[g] in the same order.  A group whose stack would
// overflow is flagged in sovf (and counted in tot[5]); the caller walks those
// with the thread-level walk instead.
#define WDFS_STACK 4096  // 16 KB of LDS
__global__ __launch_bounds__(64) void k_walk_sph_wave(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ recv,
    const NodeRec* __restrict__ nodes, int64_t nn, const double* __restrict__ wbox,
    const int4* __restrict__ wsph, const float* __restrict__ whmax,
    const float* __restrict__ radius, int use_hmax,
    const uint8_t* __restrict__ active, int mode, uint32_t* __restrict__ pr_cnt,
    uint32_t* __restrict__ pp_tot, unsigned long long* __restrict__ tot,
    const int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum, uint8_t* __restrict__ sovf) {
    const int g = xcd_chunk(blockIdx.x);
    if (g >= ng) return;
    const int lane = threadIdx.x;
    if (!active[g] || (mode == 1 && sovf[g])) {
        if (mode == 0 && lane == 0) {
            pr_cnt[g] = 0;
            pp_tot[g] = 0;
            sovf[g] = 0;
        }
        return;
    }
    __shared__ int32_t stk[WDFS_STACK];
    const NodeRec G = recv ? recv[g] : nodes[groups[g]];
    const double RG = (double)radius[g];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base_out = (mode == 1) ? pr_off[g] : 0;
    if (lane == 0) stk[0] = 0;
    int sp = 1, nout = 0, npp = 0, over = 0;
    __syncthreads();
    while (sp > 0 && !over) {
        const int take = sp < 64 ? sp : 64;
        const int b0 = sp - take;
        int n = -1;
        if (lane < take) n = stk[b0 + lane];
        __syncthreads();  // every lane has read its node before pushes reuse the slots
        sp = b0;
        bool inter = false, leaf = false;
        int b = 0, e = 0, first = 0, nchild = 0;
        if (n >= 0) {  // level-order position
            double lo[3], hi[3];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                lo[d] = wbox[d * nn + n];
                hi[d] = wbox[(3 + d) * nn + n];
            }
            const int4 r = wsph[n];
            const double d2 = box_dist2(G.lo, G.hi, lo, hi);
            double R = RG;
            if (use_hmax) {
                const double hm = (double)whmax[n];
                R = hm > R ? hm : R;
            }
            inter = d2 < R * R;
            const bool isleaf = (((uint32_t)r.w >> 16) & 0xffu) != 0;
            leaf = isleaf || (inter && box_far2(G.lo, G.hi, lo, hi) < RG * RG);
            b = r.x;
            e = r.y;
            first = r.z;
            nchild = (int)((uint32_t)r.w >> 24);
        }
        const bool emit = inter && leaf;
        const uint64_t em = __ballot(emit);
        const int sz = emit ? e - b : 0;
        const int incl = wave_incl_scan(sz);
        if (emit && mode == 1) {
            const int64_t pos = base_out + nout + __popcll(em & lt);
            pr_begin[pos] = b;
            pr_cum[pos] = npp + incl - sz;
        }
        nout += __popcll(em);
        npp += wave_last(incl);
        const int nch = (inter && !leaf) ? nchild : 0;  // children first .. first + nch - 1
        const int cincl = wave_incl_scan(nch);
        const int ctot = wave_last(cincl);
        if (sp + ctot > WDFS_STACK) {
            over = 1;
        } else {
            const int coff = sp + cincl - nch;
            for (int k = 0; k < nch; k++) stk[coff + k] = first + k;
            sp += ctot;
        }
        __syncthreads();
    }
    if (lane == 0) {
        if (mode == 0) {
            sovf[g] = over ? 1 : 0;
            pr_cnt[g] = over ? 0u : (uint32_t)nout;
            pp_tot[g] = over ? 0u : (uint32_t)npp;
            if (over) {
                atomicAdd(&tot[5], 1ull);
            } else {
                atomicAdd(&tot[10], (unsigned long long)(G.end - G.begin) * (unsigned long long)npp);
                atomicAdd(&tot[9], (unsigned long long)nout);
            }
        }
    }
}
