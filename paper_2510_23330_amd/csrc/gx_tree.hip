// gx_tree.hip -- Morton-ordered octree with receiving groups (Sec. 3.4,
// Sec. 5.2.2): root box, keys, stable sort, permutation into sorted SoA, a
// fully parallel construction of the depth-first (pre-order) node array,
// bottom-up FP64 multipoles and group selection.
//
// This file is compiled with -ffp-contract=off: the key and box arithmetic
// below must be the exact IEEE sequence the tree definition states, so that
// trees and interaction lists are bit-identical to an independent build.
//
// Node construction without per-level passes.  With keys sorted, the nodes
// containing particle i are the runs of equal key prefixes at levels
// 0..L_i, where L_i is one more than the deepest level at which i's run holds
// more than n_leaf particles (capped at 21).  A run at level m containing i
// holds more than n_leaf particles exactly when some window of n_leaf + 1
// consecutive sorted keys that contains i shares its first m digits, so L_i
// is a sliding maximum over n_leaf + 1 windows.  Particle i starts the nodes
// of the levels deeper than its common prefix with particle i - 1, which
// gives a per-particle node count; its exclusive scan numbers the nodes in
// depth-first pre-order.  A node's end is the first later key with a
// different prefix (binary search) and the node after its subtree is the
// first node started at that end particle.
#include "gx_internal.hpp"

#pragma clang fp contract(off)

// ---------------------------------------------------------------------------
// Root box
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_box_partial(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ z,
                                                     const float* __restrict__ eps2,
                                                     double* __restrict__ part) {
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double emin = INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double p[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            mn[d] = p[d] < mn[d] ? p[d] : mn[d];
            mx[d] = p[d] > mx[d] ? p[d] : mx[d];
        }
        if (eps2) emin = fmin(emin, (double)eps2[i]);
    }
    __shared__ double sh[4][7];
    double v[7] = {mn[0], mn[1], mn[2], mx[0], mx[1], mx[2], emin};
#pragma unroll
    for (int k = 0; k < 7; k++) v[k] = (k < 3 || k == 6) ? wave_min(v[k]) : wave_max(v[k]);
    int w = threadIdx.x / GX_WAVE;
    if (gx_lane() == 0)
        for (int k = 0; k < 7; k++) sh[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 7; k++) {
            double r = sh[0][k];
            for (int q = 1; q < 4; q++) r = (k < 3 || k == 6) ? fmin(r, sh[q][k]) : fmax(r, sh[q][k]);
            part[blockIdx.x * 8 + k] = r;
        }
    }
}

// One wave: lane-strided partial minima/maxima, then across the wave (exact
// in any order).
__global__ __launch_bounds__(64) void k_box_final(const double* __restrict__ part, int nb,
                                                  double* __restrict__ box) {
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double emin = INFINITY;
    for (int b = threadIdx.x; b < nb; b += 64) {
        for (int d = 0; d < 3; d++) {
            mn[d] = fmin(mn[d], part[b * 8 + d]);
            mx[d] = fmax(mx[d], part[b * 8 + 3 + d]);
        }
        emin = fmin(emin, part[b * 8 + 6]);
    }
    for (int d = 0; d < 3; d++) {
        mn[d] = wave_min(mn[d]);
        mx[d] = wave_max(mx[d]);
    }
    emin = wave_min(emin);
    if (threadIdx.x != 0) return;
    double ext = 0.0;
    for (int d = 0; d < 3; d++) {
        double e = mx[d] - mn[d];
        ext = e > ext ? e : ext;
    }
    if (ext == 0.0) ext = 1.0;
    double L = ext * (1.0 + 0x1p-40);
    box[0] = mn[0];
    box[1] = mn[1];
    box[2] = mn[2];
    box[3] = L;
    box[4] = 2097152.0 / L;
    box[5] = emin;
}

// ---------------------------------------------------------------------------
// Keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ uint64_t axis_cell(double x, double x0, double scale) {
    double t = (x - x0) * scale;
    double f = floor(t);
    f = f > 2097151.0 ? 2097151.0 : f;
    f = f < 0.0 ? 0.0 : f;
    return (uint64_t)f;
}

__global__ __launch_bounds__(256) void k_keys(int64_t n, const double* __restrict__ x,
                                              const double* __restrict__ y,
                                              const double* __restrict__ z,
                                              const double* __restrict__ box,
                                              uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = box[4];
    uint64_t ix = axis_cell(x[i], box[0], s), iy = axis_cell(y[i], box[1], s),
             iz = axis_cell(z[i], box[2], s);
    key[i] = (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
    val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_permute(int64_t n, const uint32_t* __restrict__ perm,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ z,
                                                 const double* __restrict__ m,
                                                 const float* __restrict__ eps2,
                                                 double4* __restrict__ pos4, float* __restrict__ e2s,
                                                 int32_t* __restrict__ perm_out) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t i = perm[s];
    pos4[s] = make_double4(x[i], y[i], z[i], m[i]);
    e2s[s] = eps2 ? eps2[i] : 0.0f;
    if (perm_out) perm_out[s] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// Nodes
// ---------------------------------------------------------------------------
// Number of leading 3-bit digits two 63-bit keys share (0..21).
__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b) {
    uint64_t d = a ^ b;
    if (d == 0) return GX_MAX_LEVEL;
    return (__clzll((long long)d) - 1) / 3;
}

__global__ __launch_bounds__(256) void k_window(int64_t n, const uint64_t* __restrict__ key, int n_leaf,
                                                int8_t* __restrict__ w) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j + n_leaf >= n) return;
    w[j] = (int8_t)common_digits(key[j], key[j + n_leaf]);
}

// The nodes that start at particle i (deepest first: each shallower node
// ends at or after the deeper one, so its end is searched from there,
// galloping then bisecting), written at their pre-order slots, and their ids
// appended to the per-level lists (slot = the workgroup's base + an LDS count).
__device__ __forceinline__ void emit_nodes(int64_t i, int64_t n, const uint64_t* __restrict__ key,
                                           const uint32_t* __restrict__ cnt,
                                           const uint32_t* __restrict__ base,
                                           const int8_t* __restrict__ lmax, int64_t n_nodes,
                                           NodeRec* __restrict__ nodes, uint32_t* lcnt,
                                           const uint32_t* lbase, int32_t* __restrict__ lvl_ids) {
    const uint32_t c = cnt[i];
    if (c == 0) return;
    const int Li = lmax[i];
    const int lstart = Li - (int)c + 1;
    const uint32_t bi = base[i];
    const uint64_t ki = key[i];
    int64_t lo = i + 1;
    for (int l = Li; l >= lstart; l--) {
        int64_t end;
        if (l == 0) {
            end = n;
        } else {
            const int shift = 3 * (GX_MAX_LEVEL - l);
            const uint64_t pre = ki >> shift;
            int64_t step = 1, hi = n;
            for (;;) {
                const int64_t p = lo + step - 1;
                if (p >= n) break;
                if ((key[p] >> shift) != pre) {
                    hi = p;
                    break;
                }
                lo = p + 1;
                step <<= 1;
            }
            while (lo < hi) {  // first index in [lo, hi) with a different prefix
                const int64_t mid = (lo + hi) >> 1;
                if ((key[mid] >> shift) == pre) lo = mid + 1;
                else hi = mid;
            }
            end = lo;
        }
        NodeRec r;
        r.begin = (int32_t)i;
        r.end = (int32_t)end;
        r.level = (int16_t)l;
        r.leaf = (int8_t)(l == Li);
        r.nchild = 0;
        r.next = (int32_t)(end < n ? (int64_t)base[end] : n_nodes);
        r.lo[0] = r.lo[1] = r.lo[2] = 0.0;
        r.hi[0] = r.hi[1] = r.hi[2] = 0.0;
        const int64_t id = (int64_t)bi + (l - lstart);
        nodes[id] = r;
        lvl_ids[lbase[l] + atomicAdd(&lcnt[l], 1u)] = (int32_t)id;
        lo = end;
    }
}

// The node-count and node-emit kernels give each workgroup one contiguous
// range of particles (whole chunks of 256) and keep per-workgroup level counts
// in LDS: the counts go to blkh[level][workgroup] (no global atomics, which
// serialise when tens of thousands of workgroups update the same 22 level
// counters), a per-level scan turns them into each workgroup's first slot in
// the level's id list, and the emit kernel hands out slots inside its range
// with LDS atomics (the order of ids within a level is immaterial: every
// use of the lists treats the level's nodes independently).
#define GX_TB_BLOCKS 2048
static inline int tb_blocks(int64_t n) {
    const int64_t chunks = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(chunks, GX_TB_BLOCKS));
}
// particles per workgroup (a multiple of 256) for nb workgroups
__host__ __device__ inline int64_t tb_span(int64_t n, int nb) {
    const int64_t chunks = (n + 255) / 256;
    return ((chunks + nb - 1) / nb) * 256;
}

// Per particle: L_i (deepest level of a node containing i), the number of
// nodes that start at i; per workgroup: the nodes of its range per level.
__global__ __launch_bounds__(256) void k_node_count(int64_t n, const uint64_t* __restrict__ key,
                                                    const int8_t* __restrict__ w, int n_leaf,
                                                    uint32_t* __restrict__ cnt,
                                                    int8_t* __restrict__ lmax,
                                                    uint32_t* __restrict__ blkh) {
    __shared__ uint32_t h[GX_MAX_LEVEL + 1];
    if (threadIdx.x <= GX_MAX_LEVEL) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t span = tb_span(n, gridDim.x);
    const int64_t r0 = (int64_t)blockIdx.x * span, r1 = r0 + span < n ? r0 + span : n;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        int W = -1;
        int64_t j0 = i - n_leaf > 0 ? i - n_leaf : 0;
        int64_t j1 = i < n - 1 - n_leaf ? i : n - 1 - n_leaf;
        for (int64_t j = j0; j <= j1; j++) W = w[j] > W ? w[j] : W;
        int Li = W + 1 < GX_MAX_LEVEL ? W + 1 : GX_MAX_LEVEL;
        int lstart = (i == 0) ? 0 : common_digits(key[i - 1], key[i]) + 1;
        int c = Li >= lstart ? Li - lstart + 1 : 0;
        cnt[i] = (uint32_t)c;
        lmax[i] = (int8_t)Li;
        for (int l = lstart; l <= Li; l++) atomicAdd(&h[l], 1u);
    }
    __syncthreads();
    if (threadIdx.x <= GX_MAX_LEVEL) blkh[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// One workgroup per level: exclusive scan of the level's per-workgroup counts
// (in place, in workgroup order) and the level's total.
__global__ __launch_bounds__(256) void k_level_scan(int nb, uint32_t* __restrict__ blkh,
                                                    uint32_t* __restrict__ lvl_hist) {
    __shared__ uint32_t part[256];
    uint32_t* row = blkh + (int64_t)blockIdx.x * nb;
    const int per = (nb + 255) / 256;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    uint32_t s = 0;
    for (int b = b0; b < b1; b++) s += row[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int t = 0; t < 256; t++) {
            const uint32_t v = part[t];
            part[t] = acc;
            acc += v;
        }
        lvl_hist[blockIdx.x] = acc;
    }
    __syncthreads();
    uint32_t acc = part[threadIdx.x];
    for (int b = b0; b < b1; b++) {
        const uint32_t v = row[b];
        row[b] = acc;
        acc += v;
    }
}

__global__ __launch_bounds__(256) void k_node_emit(int64_t n, const uint64_t* __restrict__ key,
                                                   const uint32_t* __restrict__ cnt,
                                                   const uint32_t* __restrict__ base,
                                                   const int8_t* __restrict__ lmax, int64_t n_nodes,
                                                   NodeRec* __restrict__ nodes,
                                                   const uint32_t* __restrict__ lvl_off,
                                                   const uint32_t* __restrict__ blkh,
                                                   int32_t* __restrict__ lvl_ids) {
    __shared__ uint32_t lcnt[GX_MAX_LEVEL + 1], lbase[GX_MAX_LEVEL + 1];
    if (threadIdx.x <= GX_MAX_LEVEL) {
        lcnt[threadIdx.x] = 0;
        lbase[threadIdx.x] = lvl_off[threadIdx.x] + blkh[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    }
    __syncthreads();
    const int64_t span = tb_span(n, gridDim.x);
    const int64_t r0 = (int64_t)blockIdx.x * span, r1 = r0 + span < n ? r0 + span : n;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x)
        emit_nodes(i, n, key, cnt, base, lmax, n_nodes, nodes, lcnt, lbase, lvl_ids);
}

// Parent of every node and the (up to 8) children of every internal node in
// key order, -1 padded (child[8 p + k]); their number goes to nodes[p].nchild.
__global__ __launch_bounds__(256) void k_node_parent(int64_t nn, NodeRec* __restrict__ nodes,
                                                     int32_t* __restrict__ parent,
                                                     int32_t* __restrict__ child) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    if (p == 0) parent[0] = -1;
    int k = 0;
    if (!nodes[p].leaf) {
        int32_t stop = nodes[p].next;
        for (int32_t c = (int32_t)p + 1; c < stop; c = nodes[c].next) {
            parent[c] = (int32_t)p;
            child[8 * p + k++] = c;
        }
    }
    nodes[p].nchild = (int8_t)k;
    for (; k < 8; k++) child[8 * p + k] = -1;
}

// Moments of one node: a leaf from its particles, an internal node from its
// children (parallel-axis shift of the quadrupoles).  Every sum runs in
// particle or child key order, whichever thread or launch computes it.
__device__ __forceinline__ void node_moments(int id, const NodeRec& nd, NodeRec* __restrict__ nodes,
                                             MomRec* __restrict__ mom, double* __restrict__ q64,
                                             const double4* __restrict__ pos4,
                                             const float* __restrict__ e2s,
                                             const int32_t* __restrict__ child) {
    double M = 0, cx = 0, cy = 0, cz = 0, e2 = 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double q[6] = {0, 0, 0, 0, 0, 0};
    if (nd.leaf) {
        // unrolled so that several particle loads are in flight at once (the
        // sums still run in particle order)
#pragma unroll 4
        for (int s = nd.begin; s < nd.end; s++) {
            double4 p = pos4[s];
            M += p.w;
            cx += p.w * p.x;
            cy += p.w * p.y;
            cz += p.w * p.z;
            e2 += p.w * (double)e2s[s];
            lo[0] = fmin(lo[0], p.x); lo[1] = fmin(lo[1], p.y); lo[2] = fmin(lo[2], p.z);
            hi[0] = fmax(hi[0], p.x); hi[1] = fmax(hi[1], p.y); hi[2] = fmax(hi[2], p.z);
        }
        cx /= M;
        cy /= M;
        cz /= M;
#pragma unroll 4
        for (int s = nd.begin; s < nd.end; s++) {
            double4 p = pos4[s];
            double dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
            double d2 = dx * dx + dy * dy + dz * dz;
            q[0] += p.w * (3 * dx * dx - d2);
            q[1] += p.w * (3 * dy * dy - d2);
            q[2] += p.w * (3 * dz * dz - d2);
            q[3] += p.w * 3 * dx * dy;
            q[4] += p.w * 3 * dx * dz;
            q[5] += p.w * 3 * dy * dz;
        }
    } else {
        // the (one to eight) children from the child rows, in key order; the
        // loads do not depend on each other (absent slots read the first
        // child and add nothing)
        const int nc = nd.nchild;
        int cid[8];
        const int4 c03 = *reinterpret_cast<const int4*>(child + 8 * (int64_t)id);
        const int4 c47 = *reinterpret_cast<const int4*>(child + 8 * (int64_t)id + 4);
        cid[0] = c03.x; cid[1] = c03.y; cid[2] = c03.z; cid[3] = c03.w;
        cid[4] = c47.x; cid[5] = c47.y; cid[6] = c47.z; cid[7] = c47.w;
#pragma unroll
        for (int j = 1; j < 8; j++) cid[j] = j < nc ? cid[j] : cid[0];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int c = cid[j];
            const MomRec mc = mom[c];
            const NodeRec nc_ = nodes[c];
            if (j < nc) {
                M += mc.M;
                cx += mc.M * mc.cx;
                cy += mc.M * mc.cy;
                cz += mc.M * mc.cz;
                e2 += mc.M * (double)mc.e2;
                for (int d = 0; d < 3; d++) {
                    lo[d] = fmin(lo[d], nc_.lo[d]);
                    hi[d] = fmax(hi[d], nc_.hi[d]);
                }
            }
        }
        cx /= M;
        cy /= M;
        cz /= M;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int c = cid[j];
            const MomRec mc = mom[c];
            const double* qc = &q64[6 * (int64_t)c];
            const double Q0 = qc[0], Q1 = qc[1], Q2 = qc[2], Q3 = qc[3], Q4 = qc[4], Q5 = qc[5];
            if (j < nc) {
                double dx = mc.cx - cx, dy = mc.cy - cy, dz = mc.cz - cz;
                double d2 = dx * dx + dy * dy + dz * dz;
                q[0] += Q0 + mc.M * (3 * dx * dx - d2);
                q[1] += Q1 + mc.M * (3 * dy * dy - d2);
                q[2] += Q2 + mc.M * (3 * dz * dz - d2);
                q[3] += Q3 + mc.M * 3 * dx * dy;
                q[4] += Q4 + mc.M * 3 * dx * dz;
                q[5] += Q5 + mc.M * 3 * dy * dz;
            }
        }
    }
    MomRec r;
    r.cx = cx;
    r.cy = cy;
    r.cz = cz;
    r.M = M;
    for (int c = 0; c < 6; c++) {
        r.q[c] = (float)q[c];
        q64[6 * (int64_t)id + c] = q[c];
    }
    r.e2 = (float)(e2 / M);
    r.hmax = 0.0f;
    mom[id] = r;
    for (int d = 0; d < 3; d++) {
        nodes[id].lo[d] = lo[d];
        nodes[id].hi[d] = hi[d];
    }
}

// Every leaf in one launch, one thread per node id: ids are in pre-order, so
// the leaves of a wavefront cover one contiguous run of particles.
__global__ __launch_bounds__(256) void k_moments_leaves(int64_t nn, NodeRec* __restrict__ nodes,
                                                        MomRec* __restrict__ mom,
                                                        double* __restrict__ q64,
                                                        const double4* __restrict__ pos4,
                                                        const float* __restrict__ e2s) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nn) return;
    const NodeRec nd = nodes[id];
    if (!nd.leaf) return;
    node_moments((int)id, nd, nodes, mom, q64, pos4, e2s, nullptr);
}

// The internal nodes of one level (their children are done: leaves by the
// leaf launch, internal children by the launch of the level below).
__global__ __launch_bounds__(256) void k_moments_level(int cnt, const int32_t* __restrict__ ids,
                                                       NodeRec* __restrict__ nodes,
                                                       MomRec* __restrict__ mom,
                                                       double* __restrict__ q64,
                                                       const int32_t* __restrict__ child) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cnt) return;
    const int id = ids[k];
    const NodeRec nd = nodes[id];
    if (nd.leaf) return;
    node_moments(id, nd, nodes, mom, q64, nullptr, nullptr, child);
}

__global__ __launch_bounds__(256) void k_group_flag(int64_t nn, const NodeRec* __restrict__ nodes,
                                                    const int32_t* __restrict__ parent, int n_group,
                                                    uint32_t* __restrict__ flag) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nn) return;
    NodeRec nd = nodes[id];
    bool small = (nd.end - nd.begin <= n_group) || nd.leaf;
    bool top = (id == 0);
    if (!top) {
        NodeRec pn = nodes[parent[id]];
        top = pn.end - pn.begin > n_group;
    }
    flag[id] = (small && top) ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_group_compact(int64_t nn, const uint32_t* __restrict__ flag,
                                                       const uint32_t* __restrict__ off,
                                                       int32_t* __restrict__ groups) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < nn && flag[id]) groups[off[id]] = (int32_t)id;
}

// SPH receiver blocks: GX_BLOCK consecutive sorted slots and their tight box
// (one wave per block).  SPH results do not depend on how receivers are
// grouped, so full blocks keep every lane busy.
__global__ __launch_bounds__(64) void k_blocks(int64_t n, const double4* __restrict__ pos4,
                                               NodeRec* __restrict__ blk) {
    const int64_t b = blockIdx.x;
    const int64_t s = b * GX_BLOCK + threadIdx.x;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (s < n) {
        double4 p = pos4[s];
        lo[0] = hi[0] = p.x;
        lo[1] = hi[1] = p.y;
        lo[2] = hi[2] = p.z;
    }
    for (int d = 0; d < 3; d++) {
        lo[d] = wave_min(lo[d]);
        hi[d] = wave_max(hi[d]);
    }
    if (threadIdx.x == 0) {
        NodeRec r;
        for (int d = 0; d < 3; d++) {
            r.lo[d] = lo[d];
            r.hi[d] = hi[d];
        }
        r.begin = (int32_t)(b * GX_BLOCK);
        r.end = (int32_t)min(n, (b + 1) * GX_BLOCK);
        r.next = -1;
        r.level = -1;
        r.leaf = 0;
        r.nchild = 0;
        blk[b] = r;
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
static bool same_view(const TreeSlot& T, const gx_particles* p) {
    return T.built && T.n == p->n && T.x == p->x && T.y == p->y && T.z == p->z;
}

int gx_tree_check(gx_ctx* ctx, int which, const gx_particles* p) {
    if (which < 0 || which > 1) return gx_fail(ctx, GX_EINVAL, "bad tree slot %d", which);
    const TreeSlot& T = ctx->tree[which];
    if (!T.built) return gx_fail(ctx, GX_ENOTBUILT, "tree slot %d not built", which);
    if (!same_view(T, p)) return gx_fail(ctx, GX_ESTALE, "particle view differs from the built tree");
    return GX_OK;
}

extern "C" int gx_tree_build(gx_ctx* ctx, const gx_particles* p, int which, int n_leaf, int n_group,
                             int32_t* perm_out, gx_stats* stats) {
    if (!ctx || !p) return GX_EINVAL;
    if (which != GX_TREE_ALL && which != GX_TREE_GAS) return gx_fail(ctx, GX_EINVAL, "bad slot");
    if (p->n <= 0 || p->n >= (int64_t)1 << 31) return gx_fail(ctx, GX_EINVAL, "n out of range");
    if (!p->x || !p->y || !p->z || !p->m) return gx_fail(ctx, GX_EINVAL, "null coordinate pointer");
    if (n_leaf < 1 || n_leaf > 64 || n_group < n_leaf || n_group > 4096)
        return gx_fail(ctx, GX_EINVAL, "need 1 <= n_leaf <= 64 and n_leaf <= n_group <= 4096");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    if (stats) {
        *stats = gx_stats{};
        GX_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    }
    TreeSlot& T = ctx->tree[which];
    T.built = 0;
    T.walk_ready = 0;
    const int64_t n = p->n;
    hipStream_t st = ctx->stream;

    // root box
    int nbb = (int)std::min<int64_t>(1024, gx_blocks(n, 256));
    GX_TRY(gx_reserve(ctx, ctx->partial, (size_t)nbb * 8 * sizeof(double)));
    GX_TRY(gx_reserve(ctx, T.box, 8 * sizeof(double)));
    hipLaunchKernelGGL(k_box_partial, dim3(nbb), dim3(256), 0, st, n, p->x, p->y, p->z, p->eps2,
                       (double*)ctx->partial.p);
    hipLaunchKernelGGL(k_box_final, dim3(1), dim3(64), 0, st, (const double*)ctx->partial.p, nbb,
                       (double*)T.box.p);

    // keys and sort
    for (int k = 0; k < 2; k++) {
        GX_TRY(gx_reserve(ctx, T.key[k], n * sizeof(uint64_t)));
        GX_TRY(gx_reserve(ctx, T.val[k], n * sizeof(uint32_t)));
    }
    hipLaunchKernelGGL(k_keys, dim3(gx_blocks(n, 256)), dim3(256), 0, st, n, p->x, p->y, p->z,
                       (const double*)T.box.p, (uint64_t*)T.key[0].p, (uint32_t*)T.val[0].p);
    GX_LAUNCH_CHECK(ctx);
    GX_TRY(gx_radix_sort(ctx, T, n, 63));

    GX_TRY(gx_reserve(ctx, T.pos4, n * sizeof(double4)));
    GX_TRY(gx_reserve(ctx, T.e2s, n * sizeof(float)));
    hipLaunchKernelGGL(k_permute, dim3(gx_blocks(n, 256)), dim3(256), 0, st, n,
                       (const uint32_t*)T.val[0].p, p->x, p->y, p->z, p->m, p->eps2,
                       (double4*)T.pos4.p, (float*)T.e2s.p, perm_out);

    // node counts
    const uint64_t* key = (const uint64_t*)T.key[0].p;
    GX_TRY(gx_reserve(ctx, T.win, n));
    GX_TRY(gx_reserve(ctx, T.cnt, (n + 1) * sizeof(uint32_t) * 2));
    GX_TRY(gx_reserve(ctx, T.lmax, n));
    GX_TRY(gx_reserve(ctx, T.lvl_fill, 2 * 32 * sizeof(uint32_t)));
    uint32_t* cnt = (uint32_t*)T.cnt.p;
    uint32_t* base = cnt + (n + 1);
    uint32_t* lvl_hist = (uint32_t*)T.lvl_fill.p;  // [0..21] histogram, [22] n_nodes
    uint32_t* lvl_aux = lvl_hist + 32;             // [0..21] level offsets
    GX_TRY(gx_zero(ctx, lvl_hist, 2 * 32 * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_window, dim3(gx_blocks(n, 256)), dim3(256), 0, st, n, key, n_leaf,
                       (int8_t*)T.win.p);
    const int tb = tb_blocks(n);
    GX_TRY(gx_reserve(ctx, T.blkh, (size_t)(GX_MAX_LEVEL + 1) * tb * sizeof(uint32_t)));
    uint32_t* blkh = (uint32_t*)T.blkh.p;
    hipLaunchKernelGGL(k_node_count, dim3(tb), dim3(256), 0, st, n, key, (const int8_t*)T.win.p,
                       n_leaf, cnt, (int8_t*)T.lmax.p, blkh);
    hipLaunchKernelGGL(k_level_scan, dim3(GX_MAX_LEVEL + 1), dim3(256), 0, st, tb, blkh, lvl_hist);
    GX_LAUNCH_CHECK(ctx);
    GX_TRY((gx_scan<uint32_t, uint32_t>(ctx, cnt, base, n, lvl_hist + 22)));

    // one synchronisation: node count and level histogram size what follows
    if (!ctx->host_small.p) {
        GX_HIP(ctx, hipHostMalloc(&ctx->host_small.p, 4096, hipHostMallocDefault));
        ctx->host_small.cap = 4096;
    }
    uint32_t* hs = (uint32_t*)ctx->host_small.p;
    GX_HIP(ctx, hipMemcpyAsync(hs, lvl_hist, 32 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GX_HIP(ctx, hipStreamSynchronize(st));
    const int64_t nn = hs[22];
    uint32_t lvl_off_h[32] = {};
    {
        uint32_t acc = 0;
        for (int l = 0; l <= GX_MAX_LEVEL; l++) {
            T.lvl_hist[l] = hs[l];
            lvl_off_h[l] = acc;
            acc += hs[l];
        }
        if ((int64_t)acc != nn) return gx_fail(ctx, GX_EINVAL, "internal: level histogram mismatch");
    }
    T.n_nodes = nn;

    GX_TRY(gx_reserve(ctx, T.nodes, nn * sizeof(NodeRec)));
    GX_TRY(gx_reserve(ctx, T.mom, nn * sizeof(MomRec)));
    GX_TRY(gx_reserve(ctx, T.q64, nn * 6 * sizeof(double)));
    GX_TRY(gx_reserve(ctx, T.parent, nn * sizeof(int32_t)));
    GX_TRY(gx_reserve(ctx, T.child, nn * 8 * sizeof(int32_t)));
    GX_TRY(gx_reserve(ctx, T.lvl_ids, nn * sizeof(int32_t)));
    GX_TRY(gx_reserve(ctx, T.flag, (nn + 1) * sizeof(uint32_t) * 2));
    // level offsets to the device
    GX_HIP(ctx, hipMemcpyAsync(lvl_aux, lvl_off_h, 32 * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_node_emit, dim3(tb), dim3(256), 0, st, n, key, cnt, base,
                       (const int8_t*)T.lmax.p, nn, (NodeRec*)T.nodes.p, lvl_aux,
                       (const uint32_t*)blkh, (int32_t*)T.lvl_ids.p);
    hipLaunchKernelGGL(k_node_parent, dim3(gx_blocks(nn, 256)), dim3(256), 0, st, nn,
                       (NodeRec*)T.nodes.p, (int32_t*)T.parent.p, (int32_t*)T.child.p);
    GX_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_moments_leaves, dim3(gx_blocks(nn, 256)), dim3(256), 0, st, nn,
                       (NodeRec*)T.nodes.p, (MomRec*)T.mom.p, (double*)T.q64.p,
                       (const double4*)T.pos4.p, (const float*)T.e2s.p);
    for (int l = GX_MAX_LEVEL; l >= 0; l--) {
        int c = (int)T.lvl_hist[l];
        if (!c) continue;
        hipLaunchKernelGGL(k_moments_level, dim3(gx_blocks(c, 256)), dim3(256), 0, st, c,
                           (const int32_t*)T.lvl_ids.p + lvl_off_h[l], (NodeRec*)T.nodes.p,
                           (MomRec*)T.mom.p, (double*)T.q64.p, (const int32_t*)T.child.p);
    }
    GX_LAUNCH_CHECK(ctx);

    // groups
    uint32_t* flag = (uint32_t*)T.flag.p;
    uint32_t* foff = flag + (nn + 1);
    hipLaunchKernelGGL(k_group_flag, dim3(gx_blocks(nn, 256)), dim3(256), 0, st, nn,
                       (const NodeRec*)T.nodes.p, (const int32_t*)T.parent.p, n_group, flag);
    GX_TRY((gx_scan<uint32_t, uint32_t>(ctx, flag, foff, nn, lvl_hist + 23)));
    GX_HIP(ctx, hipMemcpyAsync(hs + 23, lvl_hist + 23, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GX_HIP(ctx, hipStreamSynchronize(st));
    T.n_groups = hs[23];
    GX_TRY(gx_reserve(ctx, T.groups, T.n_groups * sizeof(int32_t)));
    hipLaunchKernelGGL(k_group_compact, dim3(gx_blocks(nn, 256)), dim3(256), 0, st, nn, flag, foff,
                       (int32_t*)T.groups.p);
    GX_LAUNCH_CHECK(ctx);

    T.n_blocks = (n + GX_BLOCK - 1) / GX_BLOCK;
    GX_TRY(gx_reserve(ctx, T.blocks, T.n_blocks * sizeof(NodeRec)));
    hipLaunchKernelGGL(k_blocks, dim3((unsigned)T.n_blocks), dim3(64), 0, st, n,
                       (const double4*)T.pos4.p, (NodeRec*)T.blocks.p);
    GX_LAUNCH_CHECK(ctx);

    T.built = 1;
    T.n = n;
    T.x = p->x;
    T.y = p->y;
    T.z = p->z;
    T.n_leaf = n_leaf;
    T.n_group = n_group;
    if (stats) {
        GX_HIP(ctx, hipEventRecord(ctx->ev1, st));
        GX_HIP(ctx, hipEventSynchronize(ctx->ev1));
        float ms = 0;
        GX_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        stats->ms = ms;
        stats->n_nodes = nn;
        stats->n_groups = T.n_groups;
    }
    return GX_OK;
}

extern "C" int gx_tree_counts(gx_ctx* ctx, int which, int64_t* n_nodes, int64_t* n_groups) {
    if (!ctx || which < 0 || which > 1) return GX_EINVAL;
    const TreeSlot& T = ctx->tree[which];
    if (!T.built) return gx_fail(ctx, GX_ENOTBUILT, "tree slot %d not built", which);
    if (n_nodes) *n_nodes = T.n_nodes;
    if (n_groups) *n_groups = T.n_groups;
    return GX_OK;
}

extern "C" int gx_tree_export(gx_ctx* ctx, int which, uint64_t* keys, int32_t* perm, double* box4,
                              int32_t* begin, int32_t* end, int32_t* next, int32_t* level,
                              int8_t* leaf, double* mass, double* com, float* quad, float* eps2bar,
                              double* lo, double* hi, int32_t* groups) {
    if (!ctx || which < 0 || which > 1) return GX_EINVAL;
    const TreeSlot& T = ctx->tree[which];
    if (!T.built) return gx_fail(ctx, GX_ENOTBUILT, "tree slot %d not built", which);
    GX_HIP(ctx, hipSetDevice(ctx->device));
    GX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t n = T.n, nn = T.n_nodes;
    if (keys) GX_HIP(ctx, hipMemcpy(keys, T.key[0].p, n * 8, hipMemcpyDeviceToHost));
    if (perm) GX_HIP(ctx, hipMemcpy(perm, T.val[0].p, n * 4, hipMemcpyDeviceToHost));
    if (box4) GX_HIP(ctx, hipMemcpy(box4, T.box.p, 4 * 8, hipMemcpyDeviceToHost));
    if (groups) GX_HIP(ctx, hipMemcpy(groups, T.groups.p, T.n_groups * 4, hipMemcpyDeviceToHost));
    if (begin || end || next || level || leaf || lo || hi) {
        NodeRec* h = (NodeRec*)malloc(nn * sizeof(NodeRec));
        if (!h) return gx_fail(ctx, GX_ENOMEM, "host malloc");
        hipError_t e = hipMemcpy(h, T.nodes.p, nn * sizeof(NodeRec), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            free(h);
            return gx_fail(ctx, GX_EHIP, "export nodes: %s", hipGetErrorString(e));
        }
        for (int64_t k = 0; k < nn; k++) {
            if (begin) begin[k] = h[k].begin;
            if (end) end[k] = h[k].end;
            if (next) next[k] = h[k].next;
            if (level) level[k] = h[k].level;
            if (leaf) leaf[k] = h[k].leaf;
            for (int d = 0; d < 3; d++) {
                if (lo) lo[3 * k + d] = h[k].lo[d];
                if (hi) hi[3 * k + d] = h[k].hi[d];
            }
        }
        free(h);
    }
    if (mass || com || quad || eps2bar) {
        MomRec* h = (MomRec*)malloc(nn * sizeof(MomRec));
        if (!h) return gx_fail(ctx, GX_ENOMEM, "host malloc");
        hipError_t e = hipMemcpy(h, T.mom.p, nn * sizeof(MomRec), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            free(h);
            return gx_fail(ctx, GX_EHIP, "export moments: %s", hipGetErrorString(e));
        }
        for (int64_t k = 0; k < nn; k++) {
            if (mass) mass[k] = h[k].M;
            if (com) {
                com[3 * k] = h[k].cx;
                com[3 * k + 1] = h[k].cy;
                com[3 * k + 2] = h[k].cz;
            }
            if (quad)
                for (int c = 0; c < 6; c++) quad[6 * k + c] = h[k].q[c];
            if (eps2bar) eps2bar[k] = h[k].e2;
        }
        free(h);
    }
    return GX_OK;
}
