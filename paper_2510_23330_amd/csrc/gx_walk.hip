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

#pragma clang fp contract(off)

__device__ __forceinline__ double box_dist2(const double* glo, const double* ghi, const double* lo,
                                            const double* hi) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double t1 = lo[d] - ghi[d];
        double t2 = glo[d] - hi[d];
        double t = t1 > t2 ? t1 : t2;
        t = t < 0.0 ? 0.0 : t;
        double tt = t * t;
        s = s + tt;
    }
    return s;
}

// mode 0: count (pc cells, pp ranges, pp particles; interaction totals)
// mode 1: fill the CSR lists at the offsets produced from the counts
__global__ __launch_bounds__(128) void k_walk_grav(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes, int nn,
    const double* __restrict__ box, double theta2, int mode, uint32_t* __restrict__ pc_cnt,
    uint32_t* __restrict__ pr_cnt, uint32_t* __restrict__ pp_tot,
    unsigned long long* __restrict__ tot, const int64_t* __restrict__ pc_off,
    int32_t* __restrict__ pc_list, const int64_t* __restrict__ pr_off,
    int32_t* __restrict__ pr_begin, int32_t* __restrict__ pr_cum) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const NodeRec G = nodes[groups[g]];
    const double L = box[3];
    int npc = 0, npr = 0, npp = 0, last_end = -1;
    int64_t pco = mode ? pc_off[g] : 0, pro = mode ? pr_off[g] : 0;
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
            if (mode) pc_list[pco + npc] = n;
            npc++;
            n = nxt;
        } else if (nd.leaf) {
            int b = nd.begin, e = nd.end;
            if (b != last_end) {
                if (mode) {
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
    if (!mode) {
        pc_cnt[g] = (uint32_t)npc;
        pr_cnt[g] = (uint32_t)npr;
        pp_tot[g] = (uint32_t)npp;
        unsigned long long nG = (unsigned long long)(G.end - G.begin);
        atomicAdd(&tot[2], nG * (unsigned long long)npp);
        atomicAdd(&tot[3], nG * (unsigned long long)npc);
    }
}

// Direct summation expressed as lists: every group sees the single range [0, n).
__global__ void k_direct_lists(int ng, int n, const int32_t* __restrict__ groups,
                               const NodeRec* __restrict__ nodes, int64_t* __restrict__ pc_off,
                               int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
                               int32_t* __restrict__ pr_cum, uint32_t* __restrict__ pp_tot,
                               unsigned long long* __restrict__ tot) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > ng) return;
    pc_off[g] = 0;
    pr_off[g] = g;
    if (g == ng) return;
    pr_begin[g] = 0;
    pr_cum[g] = 0;
    pp_tot[g] = (uint32_t)n;
    NodeRec G = nodes[groups[g]];
    atomicAdd(&tot[2], (unsigned long long)(G.end - G.begin) * (unsigned long long)n);
}

// SPH candidate lists: leaves whose box lies within reach of the group box.
// reach = max(R_G, hmax_c) where R_G is the group's search radius (density:
// its largest kernel size times a margin; force: its largest kernel size) and
// hmax_c the largest kernel size in the node (force only; 0 for density).
__global__ __launch_bounds__(128) void k_walk_sph(
    int ng, const int32_t* __restrict__ groups, const NodeRec* __restrict__ nodes,
    const MomRec* __restrict__ mom, int nn, const float* __restrict__ radius, int use_hmax,
    const uint8_t* __restrict__ active, int mode, uint32_t* __restrict__ pr_cnt,
    uint32_t* __restrict__ pp_tot, unsigned long long* __restrict__ tot,
    const int64_t* __restrict__ pr_off, int32_t* __restrict__ pr_begin,
    int32_t* __restrict__ pr_cum) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    if (active && !active[g]) {
        if (!mode) {
            pr_cnt[g] = 0;
            pp_tot[g] = 0;
        }
        return;
    }
    const NodeRec G = nodes[groups[g]];
    const double RG = (double)radius[g];
    int npr = 0, npp = 0, last_end = -1;
    int64_t pro = mode ? pr_off[g] : 0;
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
        } else if (nd.leaf) {
            int b = nd.begin, e = nd.end;
            if (b != last_end) {
                if (mode) {
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
    if (!mode) {
        pr_cnt[g] = (uint32_t)npr;
        pp_tot[g] = (uint32_t)npp;
        atomicAdd(&tot[2], (unsigned long long)(G.end - G.begin) * (unsigned long long)npp);
    }
}
