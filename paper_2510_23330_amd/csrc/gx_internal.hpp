// gx_internal.hpp -- context, scratch buffers and device primitives shared by
// the libgx translation units (HIP C++ for gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <type_traits>

#include "gx.h"

#define GX_MAX_LEVEL 21
#define GX_BLOCK 64  // SPH receivers per block (one per lane)
#define GX_WAVE 64

// ---------------------------------------------------------------------------
// Tree records (device, 64-byte aligned so one node visit is one cache line)
// ---------------------------------------------------------------------------
struct alignas(64) NodeRec {
    double lo[3];
    double hi[3];
    int32_t next;   // pre-order id of the first node after this subtree
    int32_t begin;  // sorted-slot range [begin, end)
    int32_t end;
    int16_t level;
    int8_t leaf;
    int8_t nchild;  // number of children (internal nodes; set with the child rows)
};
static_assert(sizeof(NodeRec) == 64, "one node record per 64-byte line");

// Multipole record read by the force kernel: FP64 centre of mass and mass,
// FP32 traceless quadrupole (xx, yy, zz, xy, xz, yz) and mean eps^2.
struct alignas(64) MomRec {
    double cx, cy, cz, M;
    float q[6];
    float e2;
    float hmax;  // SPH: largest kernel size among the node's particles
};

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

struct TreeSlot {
    int built = 0;
    const double* x = nullptr;
    const double* y = nullptr;
    const double* z = nullptr;
    int64_t n = 0;
    int n_leaf = 0, n_group = 0;
    Buf key[2], val[2];  // radix sort ping-pong (u64 keys, u32 slots)
    Buf pos4;            // double4 {x, y, z, m} in sorted order
    Buf e2s;             // float eps^2 in sorted order
    Buf win, cnt, lmax;  // node-count construction scratch
    Buf blkh;            // per-workgroup node counts per level [levels][workgroups], then bases
    Buf nodes, mom, q64, parent, child, lvl_ids, lvl_fill, flag;
    Buf groups;          // int32 node id of each group (pre-order)
    Buf blocks;          // NodeRec per SPH receiver block (64 consecutive sorted slots)
    Buf box;             // double[8]: x0, y0, z0, L, 2^21/L, min eps^2
    // gravity walk copy of the tree in level order (children of a node are
    // consecutive): sort buffers, six FP64 box arrays (lo x y z, hi x y z, each
    // n_nodes long) and one int4 per node {pre-order id, level | leaf << 16 |
    // nchild << 24, first child (internal) or particle begin (leaf), end}
    // The SPH walks use wsph, one int4 per node {particle begin, end, first
    // child, level | leaf << 16 | nchild << 24}, and whmax, the node kernel
    // sizes in level order (gathered again when hmax_ver moves on).
    Buf wkey[2], wval[2], wbox, wrec, wsph, whmax;
    int walk_ready = 0;
    int64_t hmax_ver = 0, whmax_ver = -1;
    int64_t n_nodes = 0, n_groups = 0, n_blocks = 0;
    int64_t lvl_hist[GX_MAX_LEVEL + 1] = {};
    int32_t* perm() const { return (int32_t*)val[0].p; }
    const uint64_t* keys() const { return (const uint64_t*)key[0].p; }
};

struct ListSet {  // per-group interaction lists (CSR)
    Buf pc_cnt, pc_off, pc_list;
    Buf pr_cnt, pr_off, pr_begin, pr_cum, pp_tot;
    Buf aux;  // per-group flags of the second-level overflow path
    Buf tot;  // device counters: [0] n_pc entries, [1] n_ranges, [2] n_pp inter, [3] n_pc inter
    int64_t n_groups = 0, n_pc = 0, n_ranges = 0;
    // fixed-slot layout of the last gravity lists (0: CSR) and the slot sizes
    // planned for the next call (0: none yet), valid for cap_ng groups
    int64_t stride_pc = 0, stride_pr = 0;
    int cap_pc = 0, cap_pr = 0;
    int64_t cap_ng = -1;
    int64_t last_two_pass = 1, last_stack = 0;  // diagnostics of the last construction
};

struct gx_unet_state;  // saved U-Net activations and gradients (gx_unet.hip)

struct gx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    TreeSlot tree[2];
    ListSet grav, sph;
    Buf scan_tmp[3], hist, partial, small, host_small;
    Buf wpart;  // per-chunk partial weight gradients (ordered reduction)
    Buf wrel;   // 3^3 weights re-laid out chunk-major for the slab convolution
    Buf xcm, ycm;  // channel-major copies of a layer's input and output gradient
    Buf wpart2;    // group sums of the weight-gradient partials
    Buf sph_work[24];
    // > 0: the gravity walk's small stack holds only this many entries and is
    // tried first (set by gx_set_walk_stack_limit), so that its overflow and
    // the retry with the large stack can be exercised on small workloads
    int walk_small_cap = 0;
    gx_unet_state* unet = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
};

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
int gx_fail(gx_ctx* ctx, int code, const char* fmt, ...);
int gx_reserve(gx_ctx* ctx, Buf& b, size_t bytes);
// Zero `bytes` (rounded up to 4) of device memory on the context stream.
int gx_zero(gx_ctx* ctx, void* p, size_t bytes);
// Takes, once per device (device current), the device address of the static
// scratch of the no-allocation entry point (gx_sn.hip); called by gx_create.
int gx_noalloc_setup(gx_ctx* ctx);
// Releases the U-Net activations held by a context (gx_unet.hip).
void gx_unet_free(gx_ctx* ctx);

#define GX_HIP(ctx, call)                                                               \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return gx_fail((ctx), GX_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define GX_TRY(expr)              \
    do {                          \
        int r_ = (expr);          \
        if (r_ != GX_OK) return r_; \
    } while (0)

#define GX_LAUNCH_CHECK(ctx) GX_HIP(ctx, hipGetLastError())

static inline unsigned gx_blocks(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

// Exclusive scan of n elements (device), total written to device *total
// (may be NULL).  Types: uint32_t -> uint32_t, uint32_t -> int64_t.
template <typename TI, typename TO>
int gx_scan(gx_ctx* ctx, const TI* in, TO* out, int64_t n, TO* total);

// Stable LSD radix sort of (u64 key, u32 value) pairs; result in slot 0.
int gx_radix_sort(gx_ctx* ctx, TreeSlot& T, int64_t n, int key_bits);
// The same on caller buffers key[0..1], val[0..1] (input in slot 0).
int gx_radix_sort_bufs(gx_ctx* ctx, Buf* key, Buf* val, int64_t n, int key_bits);
// Level-order walk arrays of a built tree (kept until the next build).
int gx_walk_tree(gx_ctx* ctx, TreeSlot& T);
// the weight gradient takes the channel-major path (and a fused input)
bool gx_wgrad_fused_ok(int S, int Cin, int Cout);
// The same plus the level-order node kernel sizes for SPH walks with use_hmax.
int gx_walk_tree_sph(gx_ctx* ctx, TreeSlot& T, int use_hmax);

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int gx_lane() { return (int)__lane_id(); }

// Inclusive scan over the wave (all 64 lanes active).  32-bit integers use
// DPP moves (row shifts by 1, 2, 4, 8 inside each 16-lane row, then the
// broadcasts of lane 15 to rows 1 and 3 and of lane 31 to rows 2 and 3): VALU
// cross-lane reads with no LDS round trip.  Other types shuffle.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    if constexpr (std::is_integral<T>::value && sizeof(T) == 4) {
        unsigned x = (unsigned)v;
        x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
        x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
        x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
        x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
        x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
        x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
        return (T)x;
    } else {
#pragma unroll
        for (int o = 1; o < GX_WAVE; o <<= 1) {
            T t = __shfl_up(v, o, GX_WAVE);
            if (gx_lane() >= o) v += t;
        }
        return v;
    }
}

// Inclusive running maximum over the wave (all lanes active), by the same
// DPP moves as wave_incl_scan; lanes with no source keep INT_MIN.
__device__ __forceinline__ int wave_incl_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xc, 0xf, false));
    return v;
}

// v of the next lower lane (DPP wave shift right by one); lane 0 gets fill.
__device__ __forceinline__ int wave_prev(int v, int fill) {
    return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xf, 0xf, false);
}

// Value of a 32-bit integer in lane 63 (wave-uniform result).
__device__ __forceinline__ int wave_last(int v) { return __builtin_amdgcn_readlane(v, GX_WAVE - 1); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = GX_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, GX_WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = GX_WAVE / 2; o > 0; o >>= 1) {
        T t = __shfl_xor(v, o, GX_WAVE);
        v = t < v ? t : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = GX_WAVE / 2; o > 0; o >>= 1) {
        T t = __shfl_xor(v, o, GX_WAVE);
        v = t > v ? t : v;
    }
    return v;
}

// Block-wide exclusive scan for blockDim.x == 256 (4 waves).  Returns the
// exclusive prefix of v; *block_total receives the sum.  Uses 4 shared slots.
template <typename T>
__device__ __forceinline__ T block_excl_scan256(T v, T* sh4, T* block_total) {
    T inc = wave_incl_scan(v);
    int w = threadIdx.x / GX_WAVE;
    if (gx_lane() == GX_WAVE - 1) sh4[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        T s = sh4[k];
        if (k < w) off += s;
        tot += s;
    }
    __syncthreads();
    *block_total = tot;
    return off + inc - v;
}

// Map a linear block index to a work item so that each of the 8 XCDs (which
// receive blocks round-robin) works on one contiguous eighth of the items:
// neighbouring items share data (the convolution slabs' halo planes) in that
// XCD's L2.  For items of equal cost only; see xcd_chunk below otherwise.
__device__ __forceinline__ int xcd_remap(int b, int n_items) {
    int per = (n_items + 7) / 8;
    return (b % 8) * per + b / 8;
}
static inline unsigned xcd_grid(int64_t n_items) { return (unsigned)(8 * ((n_items + 7) / 8)); }

// For items of very unequal cost (tree groups: list lengths vary with the
// local density) one contiguous eighth per XCD loads the XCDs unequally (on
// the 16M disk the busiest eighth of the gravity groups holds 1.15 times the
// mean work, and the kernel lasts as long as that XCD).  Here the items are
// dealt in chunks of XCD_CH consecutive items, chunk c to XCD c mod 8: every
// XCD gets a share of every region, and neighbours within a chunk still
// share one L2.  Blocks past the last item (the last round of chunks is
// partly empty) map to indices >= n_items and must return.
#define XCD_CH 16
__device__ __forceinline__ int xcd_chunk(int b) {
    const int k = b >> 3, x = b & 7;
    return ((k / XCD_CH) * 8 + x) * XCD_CH + k % XCD_CH;
}
static inline unsigned xcd_chunk_grid(int64_t n_items) {
    const int64_t chunks = (n_items + XCD_CH - 1) / XCD_CH;
    return (unsigned)(8 * XCD_CH * ((chunks + 7) / 8));
}

// ---------------------------------------------------------------------------
// SPH-style candidate lists (used by the SPH and voxelisation kernels)
// ---------------------------------------------------------------------------
// Candidate lists of all groups: fixed-capacity slots (group g at g * cap)
// from the wave walk, and -- for the groups flagged in `ovf` whose lists did
// not fit -- CSR lists from the thread walk.
struct ListView {
    int cap;
    const uint32_t* cnt;
    const int32_t* begin;
    const int32_t* cum;
    const uint32_t* tot;
    const uint8_t* ovf;  // may be null: no overflow lists
    const int64_t* off2;
    const uint32_t* cnt2;
    const int32_t* begin2;
    const int32_t* cum2;
    const uint32_t* tot2;
};

// One group's list: ranges [r0, r1) of begin/cum, npp candidates in total.
struct GroupList {
    const int32_t* begin;
    const int32_t* cum;
    int64_t r0, r1;
    int npp;
    __device__ __forceinline__ GroupList(const ListView& L, int g) {
        if (L.ovf && L.ovf[g]) {
            begin = L.begin2;
            cum = L.cum2;
            r0 = L.off2[g];
            r1 = r0 + L.cnt2[g];
            npp = (int)L.tot2[g];
        } else {
            begin = L.begin;
            cum = L.cum;
            r0 = (int64_t)g * L.cap;
            r1 = r0 + L.cnt[g];
            npp = (int)L.tot[g];
        }
    }
};

// First range of a group list that overlaps list position ch: the last range
// whose running offset is <= ch (offsets increase strictly), by bisection.
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

// Particle slot of every position ch .. che-1 of a group's candidate list,
// computed by the whole block (every thread must call it; it synchronises).
// The ranges touching the chunk are read in parallel, one thread per range:
// each marks its first position with its range number and records its slot
// offset; a block-wide running maximum then carries the range number to every
// position it covers.  On return slot[k - ch] holds the particle slot of list
// position k.  LDS scratch: slot and roff hold che - ch ints, wtot one int
// per wave of the block.
__device__ __forceinline__ void list_slots(const GroupList& L, int npp, int ch, int che,
                                           int* slot, int* roff, int* wtot, int tid,
                                           int nthreads) {
    const int n = che - ch;
    for (int i = tid; i < n; i += nthreads) slot[i] = -1;
    __syncthreads();
    const int64_t ra = first_range(L, ch);
    for (int64_t r = ra + tid; r < L.r1; r += nthreads) {
        const int c = L.cum[r];
        if (c >= che) break;  // later ranges of this thread start later still
        const int rl = (int)(r - ra);
        if (rl < n) {  // non-empty ranges: at most one per position
            roff[rl] = L.begin[r] - c;
            atomicMax(&slot[max(c, ch) - ch], rl);
        }
    }
    __syncthreads();
    // running maximum: contiguous segments per thread, then across lanes and waves
    const int per = (n + nthreads - 1) / nthreads;
    const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
    int run = -1;
    for (int i = b0; i < b1; i++) run = max(run, slot[i]);
    const int lane = tid & 63, wv = tid >> 6;
    const int v = wave_incl_max(run);
    if (lane == 63) wtot[wv] = v;
    __syncthreads();
    int cur = wave_prev(v, -1);
    for (int w = 0; w < wv; w++) cur = max(cur, wtot[w]);
    for (int i = b0; i < b1; i++) {
        cur = max(cur, slot[i]);
        slot[i] = ch + i + roff[cur];
    }
    __syncthreads();
}

// Build candidate lists for ng receivers (tree groups `groups`, or boxes
// `recv` when non-null) on a tree slot: leaves within max(rad[g], node hmax
// when use_hmax) of the receiver box.
int gx_sph_walk(gx_ctx* ctx, TreeSlot& T, ListSet& Ls, int ng, const int32_t* groups,
                const NodeRec* recv, const float* rad, int use_hmax, const uint8_t* active,
                ListView* view, int64_t* list_pairs);
// Largest kernel size per node from sorted per-slot (H, ...) records.
int gx_sph_node_hmax(gx_ctx* ctx, TreeSlot& T, const float4* ss);
int gx_tree_check(gx_ctx* ctx, int which, const gx_particles* p);
