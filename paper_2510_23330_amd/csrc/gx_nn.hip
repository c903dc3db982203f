// gx_nn.hip -- 3-D convolutional encoder-decoder building blocks for the
// supernova surrogate (Sec. 3.3: a U-Net of 3-D convolutions trained with a
// mean-squared error and Adam): BF16 activations and weights, FP32
// accumulation on the gfx950 matrix cores.
//
// Layouts (NDHWC, channels innermost):
//   activations  x[B][S][S][S][C]            bf16 (C % 8 == 0)
//   weights      w[Cout][kvol][Cin]           bf16, kvol = 27 (3^3, pad 1) or 1
//                (row co holds the GEMM column, K index = tap * Cin + ci,
//                 tap = (dz * 3 + dy) * 3 + dx)
//   master copy  w32 in the same layout, FP32; gradients FP32.
//
// Forward convolution as an implicit GEMM: M = B S^3 output voxels, N = Cout,
// K = kvol Cin.  A workgroup (4 waves) computes a 128 x BN tile; each K step
// stages a 128 x 32 slice of the implicit im2col matrix (zero padding at the
// volume faces) and a BN x 32 slice of the weights in LDS, and each wave runs
// v_mfma_f32_16x16x32_bf16 on its 32 x BN sub-tile.  The epilogue adds the
// bias, applies LeakyReLU or, for a gradient pass, multiplies by the
// activation derivative of a stored layer output, and writes bf16 or fp32.
// Backward data is the same kernel on weights with flipped taps and swapped
// channel roles; backward weight reduces im2col^T x dOut over voxel chunks
// (transposed through LDS) into per-chunk FP32 partial gradients, which a
// second kernel adds in chunk order (deterministic).
#include "gx_internal.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define CV_BM 256
#define CV_BK 32
#define CV_APITCH 40  // bf16 per LDS row (32 + 8 padding)
#define LRELU_SLOPE 0.1f
#ifndef GX_WG_WAVES
#define GX_WG_WAVES 4096  // waves the channel-major weight gradient aims at
#endif
#ifndef GX_WG_BLOCKS
#define GX_WG_BLOCKS 512  // blocks the LDS-staged weight gradient aims at
#endif

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

struct ConvGeom {
    int B, S, Cin, Cout, kvol;
    int64_t M;  // B * S^3
    int K;      // kvol * Cin
    int lgC;    // log2(Cin): the GEMM's K channel count is a power of two
};

// Implicit-GEMM row m: its voxel index and a 27-bit mask of the taps whose
// neighbour lies inside the volume (bit (dz+1)*9 + (dy+1)*3 + (dx+1); bit 0
// alone for 1^3 kernels; 0 for rows past M).  Decomposed once per row.
struct RowTap {
    int64_t m;
    uint32_t mask;
};

__device__ __forceinline__ RowTap row_taps(const ConvGeom& g, int64_t m) {
    RowTap r{m, 0u};
    if (m >= g.M) return r;
    if (g.kvol == 1) {
        r.mask = 1u;
        return r;
    }
    const uint32_t S = (uint32_t)g.S;
    const uint32_t mm = (uint32_t)m;  // M < 2^31 (checked on the host)
    const uint32_t t = mm / S, t2 = t / S;
    const uint32_t x = mm - t * S, y = t - t2 * S, z = t2 % S;
    const uint32_t vx = (x > 0 ? 1u : 0u) | 2u | (x + 1 < S ? 4u : 0u);
    const uint32_t vy = (y > 0 ? 1u : 0u) | 2u | (y + 1 < S ? 4u : 0u);
    const uint32_t vz = (z > 0 ? 1u : 0u) | 2u | (z + 1 < S ? 4u : 0u);
    uint32_t mask = 0u;
#pragma unroll
    for (int dz = 0; dz < 3; dz++)
#pragma unroll
        for (int dy = 0; dy < 3; dy++)
            if ((vz >> dz & 1u) && (vy >> dy & 1u)) mask |= vx << (dz * 9 + dy * 3);
    r.mask = mask;
    return r;
}

// Voxel-index offset of tap t: ((dz * S) + dy) * S + dx.
__device__ __forceinline__ int64_t tap_offset(const ConvGeom& g, int tap) {
    if (g.kvol == 1) return 0;
    const int dz = tap / 9, rr = tap - dz * 9, dy = rr / 3, dx = rr - dy * 3;
    return ((int64_t)(dz - 1) * g.S + (dy - 1)) * g.S + (dx - 1);
}

// 8 consecutive K entries (one tap, 8 channels) of im2col row r, given the
// slice's tap, channel and voxel offset.
__device__ __forceinline__ uint4 im2col8t(const uint16_t* __restrict__ in, const ConvGeom& g,
                                          const RowTap& r, bool kin, int tap, int ci,
                                          int64_t off) {
    if (!kin || !(r.mask >> tap & 1u)) return make_uint4(0, 0, 0, 0);
    return *reinterpret_cast<const uint4*>(in + (r.m + off) * g.Cin + ci);
}

// epilogue modes
enum { EP_NONE = 0, EP_LRELU = 1, EP_DACT = 2 };

// Optional per-channel affine output of the generic kernel: when scale is set,
// output channels col < nc go to out_f32[m * stride + col] as
// fmaf(value, scale[col], shift[col]) and the others are dropped.
struct ConvAffine {
    const float* scale = nullptr;
    const float* shift = nullptr;
    int nc = 0, stride = 0;
};

// Block tile CV_BM (= 256) voxels x BN output channels, 4 waves, each wave
// 64 voxels x BN: per 32-wide K slice a wave issues 4 x BN/16 MFMAs from 4 A
// and BN/16 B fragments.  Two LDS stages: the next K slice is fetched into
// registers while the current one feeds the matrix cores, then stored into
// the other stage (one barrier per slice).
template <int BN>
__global__ __launch_bounds__(256) void k_conv3d(const uint16_t* __restrict__ in,
                                                const uint16_t* __restrict__ w,
                                                const float* __restrict__ bias, ConvGeom g,
                                                int mode, const uint16_t* __restrict__ yref,
                                                uint16_t* __restrict__ out_bf,
                                                float* __restrict__ out_f32, ConvAffine aff) {
    constexpr int MR = CV_BM / 64;  // A rows staged per thread and 16-row MFMA tiles per wave
    constexpr int NT = BN / 16;     // MFMA column tiles per wave
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][CV_BM * CV_APITCH];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * CV_APITCH];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * CV_BM;
    const int n0 = blockIdx.y * BN;
    f32x4 acc[MR][NT];
#pragma unroll
    for (int i = 0; i < MR; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) acc[i][j] = f32x4{0, 0, 0, 0};

    // staging roles: A rows tid/4 + 64 r (r < MR), 8-channel group tid%4;
    // B row tid/4 (output channel) for tid < 4 BN
    const int grp = tid & 3, srow = tid >> 2;
    RowTap rows[MR];
#pragma unroll
    for (int r = 0; r < MR; r++) rows[r] = row_taps(g, m0 + srow + 64 * r);
    const bool bst = tid < BN * 4;
    const uint16_t* wrow = w + (int64_t)(n0 + (bst ? srow : 0)) * g.K;
    uint4 va[MR], vb = make_uint4(0, 0, 0, 0);
    auto fetch = [&](int k0) {
        const int k = k0 + grp * 8;
        const bool kin = k < g.K;
        const int tap = k >> g.lgC, ci = k & (g.Cin - 1);
        const int64_t off = tap_offset(g, tap);
#pragma unroll
        for (int r = 0; r < MR; r++) va[r] = im2col8t(in, g, rows[r], kin, tap, ci, off);
        if (bst) vb = kin ? *reinterpret_cast<const uint4*>(wrow + k) : make_uint4(0, 0, 0, 0);
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < MR; r++)
            *reinterpret_cast<uint4*>(&sA[buf][(srow + 64 * r) * CV_APITCH + grp * 8]) = va[r];
        if (bst) *reinterpret_cast<uint4*>(&sB[buf][srow * CV_APITCH + grp * 8]) = vb;
    };
    fetch(0);
    stage(0);
    __syncthreads();
    int cur = 0;
    const int kq = (lane >> 4) * 8;
    for (int k0 = 0; k0 < g.K; k0 += CV_BK) {
        const bool more = k0 + CV_BK < g.K;
        if (more) fetch(k0 + CV_BK);
        bf16x8 a[MR], b[NT];
#pragma unroll
        for (int i = 0; i < MR; i++)
            a[i] = *reinterpret_cast<const bf16x8*>(
                &sA[cur][(wv * (16 * MR) + i * 16 + (lane & 15)) * CV_APITCH + kq]);
#pragma unroll
        for (int j = 0; j < NT; j++)
            b[j] = *reinterpret_cast<const bf16x8*>(&sB[cur][(j * 16 + (lane & 15)) * CV_APITCH + kq]);
#pragma unroll
        for (int i = 0; i < MR; i++)
#pragma unroll
            for (int j = 0; j < NT; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (more) stage(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    // epilogue: lane holds rows 4*(lane/16) + t of each 16 x 16 tile, column lane % 16.
    // A dense affine output (stride == nc, the network head) is staged in LDS
    // and written as one contiguous run per block in 16-byte pieces.
    if (aff.scale && aff.stride == aff.nc && BN == 16 && n0 == 0) {
        float* const st = reinterpret_cast<float*>(&sA[0][0]);  // CV_BM * nc floats
        static_assert(sizeof(sA) >= CV_BM * 16 * sizeof(float), "staging fits");
        const int nc = aff.nc;
        __syncthreads();  // every wave is done with the tiles
#pragma unroll
        for (int i = 0; i < MR; i++) {
            const int col = lane & 15;
            const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int ml = wv * (16 * MR) + i * 16 + (lane >> 4) * 4 + t;
                if (col < nc) st[ml * nc + col] = fmaf(acc[i][0][t] + bv, aff.scale[col], aff.shift[col]);
            }
        }
        __syncthreads();
        const int nv = (int)min((int64_t)CV_BM, g.M - m0);
        const int nf = nv * nc;
        float* const dst = out_f32 + m0 * nc;  // 16-byte aligned: CV_BM * nc * 4 is a multiple of 16
        const int n4 = nf / 4;
        for (int e = tid; e < n4; e += 256)
            *reinterpret_cast<float4*>(dst + 4 * e) = *reinterpret_cast<const float4*>(st + 4 * e);
        for (int e = 4 * n4 + tid; e < nf; e += 256) dst[e] = st[e];
        return;
    }
#pragma unroll
    for (int i = 0; i < MR; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) {
            const int col = n0 + j * 16 + (lane & 15);
            const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int64_t m = m0 + wv * (16 * MR) + i * 16 + (lane >> 4) * 4 + t;
                if (m >= g.M) continue;
                float v = acc[i][j][t] + bv;
                const int64_t o = m * g.Cout + col;
                if (mode == EP_LRELU) {
                    v = v > 0.0f ? v : LRELU_SLOPE * v;
                } else if (mode == EP_DACT) {
                    v = bf2f(yref[o]) > 0.0f ? v : LRELU_SLOPE * v;
                }
                if (aff.scale) {
                    if (col < aff.nc) out_f32[m * aff.stride + col] = fmaf(v, aff.scale[col], aff.shift[col]);
                    continue;
                }
                if (out_bf) out_bf[o] = f2bf(v);
                if (out_f32) out_f32[o] = v;
            }
        }
}

// ---------------------------------------------------------------------------
// 3^3 convolution on output bricks (the path for every 3^3 layer)
// ---------------------------------------------------------------------------
// A workgroup computes a brick of BRZ x BRY x BRX = 4 x 8 x 8 output voxels of
// one sample for BN output channels.  For each chunk of CK input channels it
// stages the brick's input with a one-voxel halo (6 x 10 x 10 voxels) in LDS
// once, and the MFMA A fragments of all 27 taps are read straight from that
// tile (tap = a fixed LDS offset), so each input voxel is fetched from memory
// once per chunk instead of once per tap.  Wave w owns brick slice z = w
// (64 voxels = 4 MFMA row tiles).  K runs chunk-major: (chunk, tap, channel),
// 32 per MFMA step (32 / CK taps per step for CK < 32); weights stay in the
// [Cout][27][Cin] layout and each lane loads its B fragment (16 bytes) from
// memory, one step ahead.
#define BRZ 4
#define BRY 8
#define BRX 8
#define HZ (BRZ + 2)
#define HY (BRY + 2)
#define HX (BRX + 2)
#define HVOX (HZ * HY * HX)

// The convolution's input may be assembled on the fly: channels [0, c1) from
// `in` and [c1, Cin) from `in2` (a channel concatenation), each read at half
// resolution when `up` is set (nearest x2 upsampling of an (S/2)^3 grid).
struct ConvSrc {
    const uint16_t* in2;
    int c1;  // channels taken from the first source (Cin when in2 is null)
    int up;  // 1: sources hold (S/2)^3 voxels
    uint16_t* pool = nullptr;  // slab kernel: 2^3 average of the bf16 output ([B][(S/2)^3][Cout])
};

template <int BN, int CK>
__global__ __launch_bounds__(256) void k_conv3d_brick(const uint16_t* __restrict__ in,
                                                      const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias, ConvGeom g,
                                                      int mode, const uint16_t* __restrict__ yref,
                                                      uint16_t* __restrict__ out_bf,
                                                      float* __restrict__ out_f32, ConvSrc src) {
    constexpr int PITCH = CK + 8;          // bf16 per halo voxel (padding against bank conflicts)
    constexpr int NT = BN / 16;
    constexpr int TPS = 32 / CK;           // taps per MFMA step
    constexpr int NSTEP = (27 + TPS - 1) / TPS;
    constexpr int GPV = CK / 8;            // 8-channel groups per voxel
    __shared__ __attribute__((aligned(16))) uint16_t hal[HVOX * PITCH];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int S = g.S;
    const int nbx = (S + BRX - 1) / BRX, nby = (S + BRY - 1) / BRY, nbz = (S + BRZ - 1) / BRZ;
    int t = blockIdx.x;
    const int bx = t % nbx;
    t /= nbx;
    const int by = t % nby;
    t /= nby;
    const int bz = t % nbz;
    const int b = t / nbz;
    const int x0 = bx * BRX, y0 = by * BRY, z0 = bz * BRZ;
    const int n0 = blockIdx.y * BN;
    const int64_t vs0 = (int64_t)b * S * S * S;  // first voxel of the sample

    f32x4 acc[4][NT];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) acc[i][j] = f32x4{0, 0, 0, 0};

    // this lane's rows: brick voxel (z = wv, y = 2 i + (lane & 15) / 8, x = lane & 7)
    int hrow[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int vy = 2 * i + ((lane & 15) >> 3), vx = lane & 7;
        hrow[i] = (wv * HY + vy) * HX + vx;  // halo voxel of tap (0, 0, 0) = offset (-1, -1, -1)
    }
    const int kg = lane >> 4;                          // k group of this lane (8 values)
    const int tsub = kg / GPV, csub = (kg % GPV) * 8;  // tap within the step, channel offset
    const uint16_t* wcol[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) wcol[j] = w + (int64_t)(n0 + j * 16 + (lane & 15)) * g.K;

    const int nchunk = g.Cin / CK;
    const int Ss = src.up ? S / 2 : S;             // source grid
    const int64_t ss0 = (int64_t)b * Ss * Ss * Ss;  // first source voxel of the sample
    for (int c = 0; c < nchunk; c++) {
        // this chunk's source tensor, its channel stride and offset
        const bool second = src.in2 && c * CK >= src.c1;
        const uint16_t* sp = second ? src.in2 : in;
        const int sc = second ? g.Cin - src.c1 : src.c1;
        const int co = second ? c * CK - src.c1 : c * CK;
        __syncthreads();  // the previous chunk's tile has been read
        for (int e = tid; e < HVOX * GPV; e += 256) {
            const int h = e / GPV, gq = e - h * GPV;
            const int hz = h / (HY * HX), hr = h - hz * (HY * HX), hy = hr / HX, hx = hr - hy * HX;
            int Z = z0 - 1 + hz, Y = y0 - 1 + hy, X = x0 - 1 + hx;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (Z >= 0 && Z < S && Y >= 0 && Y < S && X >= 0 && X < S) {
                if (src.up) {
                    Z >>= 1;
                    Y >>= 1;
                    X >>= 1;
                }
                v = *reinterpret_cast<const uint4*>(
                    sp + (ss0 + ((int64_t)Z * Ss + Y) * Ss + X) * sc + co + gq * 8);
            }
            *reinterpret_cast<uint4*>(&hal[h * PITCH + gq * 8]) = v;
        }
        __syncthreads();
        // B fragments one step ahead
        auto load_b = [&](int st, bf16x8(&bb)[NT]) {
            const int tap = st * TPS + tsub;
#pragma unroll
            for (int j = 0; j < NT; j++) {
                uint4 q = make_uint4(0, 0, 0, 0);
                if (tap < 27) q = *reinterpret_cast<const uint4*>(wcol[j] + tap * g.Cin + c * CK + csub);
                bb[j] = *reinterpret_cast<const bf16x8*>(&q);
            }
        };
        bf16x8 bcur[NT], bnext[NT];
        load_b(0, bcur);
        for (int st = 0; st < NSTEP; st++) {
            if (st + 1 < NSTEP) load_b(st + 1, bnext);
            const int tap = st * TPS + tsub;
            bf16x8 a[4];
            if (tap < 27) {
                const int dz = tap / 9, rr = tap - dz * 9, dy = rr / 3, dx = rr - dy * 3;
                const int toff = (dz * HY + dy) * HX + dx;
#pragma unroll
                for (int i = 0; i < 4; i++)
                    a[i] = *reinterpret_cast<const bf16x8*>(&hal[(hrow[i] + toff) * PITCH + csub]);
            } else {
                const uint4 z4 = make_uint4(0, 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 4; i++) a[i] = *reinterpret_cast<const bf16x8*>(&z4);
            }
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < NT; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bcur[j], acc[i][j], 0, 0, 0);
            if (st + 1 < NSTEP) {
#pragma unroll
                for (int j = 0; j < NT; j++) bcur[j] = bnext[j];
            }
        }
    }
    // epilogue: lane holds rows 4 (lane / 16) + r of each 16-row tile, column lane % 16;
    // row q of tile i is brick voxel (z = wv, y = 2 i + q / 8, x = q % 8)
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) {
            const int col = n0 + j * 16 + (lane & 15);
            const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int q = (lane >> 4) * 4 + r;
                const int Z = z0 + wv, Y = y0 + 2 * i + (q >> 3), X = x0 + (q & 7);
                if (Z >= S || Y >= S || X >= S) continue;
                const int64_t m = vs0 + ((int64_t)Z * S + Y) * S + X;
                float v = acc[i][j][r] + bv;
                const int64_t o = m * g.Cout + col;
                if (mode == EP_LRELU) {
                    v = v > 0.0f ? v : LRELU_SLOPE * v;
                } else if (mode == EP_DACT) {
                    v = bf2f(yref[o]) > 0.0f ? v : LRELU_SLOPE * v;
                }
                if (out_bf) out_bf[o] = f2bf(v);
                if (out_f32) out_f32[o] = v;
            }
        }
}

// ---------------------------------------------------------------------------
// 3^3 convolution on output slabs with weights staged in LDS
// ---------------------------------------------------------------------------
// A workgroup computes SBZ x SBY x SBX = 8 x 4 x 16 output voxels of one
// sample for BN output channels; wave w owns z slices 2w and 2w + 1, i.e.
// eight 16-row MFMA tiles, each one x-row of 16 voxels.  The reduction runs
// over chunks of 8 input channels: per chunk the slab's input with a
// one-voxel halo (10 x 6 x 18 voxels x 8 channels) and the chunk's weights
// for all 27 taps and BN outputs (27 x BN x 8) are staged in LDS once for the
// four waves, then 7 MFMA steps cover K = 27 taps x 8 channels (4 taps per
// step, lane group kg takes tap 4 st + kg; the 28th tap slot is zero).  16
// consecutive voxels or output channels of 16 bytes each fill all 64 LDS
// banks once, so both operand reads are conflict-free without padding.  The
// weights come re-laid out as [Cin / 8][27][Cout][8] (k_wrelayout) so that
// each chunk's slice is read with whole-line loads.
#define SBZ 8
#define SBY 4
#define SBX 16
#define SHZ (SBZ + 2)
#define SHY (SBY + 2)
#define SHX (SBX + 2)
#define SHVOX (SHZ * SHY * SHX)

__global__ void k_wrelayout(const uint16_t* __restrict__ w, int Cout, int Cin,
                            uint16_t* __restrict__ wr) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one 8-channel piece
    const int ncg = Cin / 8;
    const int64_t n = (int64_t)Cout * 27 * ncg;
    if (e >= n) return;
    const int cg = (int)(e % ncg);
    const int64_t t = e / ncg;
    const int tap = (int)(t % 27);
    const int co = (int)(t / 27);
    *reinterpret_cast<uint4*>(wr + (((int64_t)cg * 27 + tap) * Cout + co) * 8) =
        *reinterpret_cast<const uint4*>(w + ((int64_t)co * 27 + tap) * Cin + cg * 8);
}

// RT row tiles per wave: 8 (wave w owns z slices 2w, 2w + 1; 8-slice slabs)
// or 4 (one z slice per wave; 4-slice slabs, half the accumulators, so the
// 64-output variant also runs three workgroups per CU).
template <int BN, int RT>
__global__ __launch_bounds__(256, (BN == 32 || RT == 4) ? 3 : 2) void k_conv3d_slab(const uint16_t* __restrict__ in,
                                                        const uint16_t* __restrict__ wr,
                                                        const float* __restrict__ bias, ConvGeom g,
                                                        int mode, const uint16_t* __restrict__ yref,
                                                        uint16_t* __restrict__ out_bf,
                                                        float* __restrict__ out_f32, ConvSrc src) {
    constexpr int NT = BN / 16;
    constexpr int NSTEP = 7;  // ceil(27 / 4)
    constexpr int ZW = RT / 4;                 // z slices per wave
    constexpr int BZ = 4 * ZW, HVOX_ = (BZ + 2) * SHY * SHX;  // slab depth, halo voxels
    // one LDS block: the halo tile, then 27 taps of weights plus a zero row for
    // the padding tap slot; after the last chunk it stages the output
    constexpr int HAL_N = HVOX_ * 8, WSH_N = 28 * BN * 8;
    __shared__ __attribute__((aligned(16))) uint16_t smem[HAL_N + WSH_N];
    uint16_t* const hal = smem;
    uint16_t* const wsh = smem + HAL_N;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int S = g.S;
    const int nbx = (S + SBX - 1) / SBX, nby = (S + SBY - 1) / SBY, nbz = (S + BZ - 1) / BZ;
    // each XCD takes a contiguous run of slabs, so neighbours that share halo
    // planes run on one L2 (the grid is padded to a multiple of 8)
    const int nslab = g.B * nbz * nby * nbx;
    int t = xcd_remap(blockIdx.x, nslab);
    if (t >= nslab) return;
    const int bx = t % nbx;
    t /= nbx;
    const int by = t % nby;
    t /= nby;
    const int bz = t % nbz;
    const int b = t / nbz;
    const int x0 = bx * SBX, y0 = by * SBY, z0 = bz * BZ;
    const int n0 = blockIdx.y * BN;
    const int64_t vs0 = (int64_t)b * S * S * S;

    f32x4 acc[RT][NT];
#pragma unroll
    for (int r = 0; r < RT; r++)
#pragma unroll
        for (int j = 0; j < NT; j++) acc[r][j] = f32x4{0, 0, 0, 0};

    // row tile r of this wave: z slice ZW wv + r / 4, y row r % 4, x = lane & 15;
    // its halo voxel is hbase plus a constant per r (an immediate LDS offset)
    const int hbase = ZW * wv * SHY * SHX + (lane & 15);
    const int kg = lane >> 4;  // tap slot of this lane within a step

    const int nchunk = g.Cin / 8;
    const int Ss = src.up ? S / 2 : S;
    const int64_t ss0 = (int64_t)b * Ss * Ss * Ss;
    // A chunk's tiles are fetched into registers one chunk ahead (their loads
    // run under the previous chunk's MFMAs) and committed to LDS between two
    // barriers.
    // (with 8 row tiles the 64-output variant fetches only the halo ahead: its
    // accumulators leave no room for the weights as well)
    constexpr bool PFW = BN * RT <= 256;
    constexpr int NHV = (HVOX_ + 255) / 256, NWV = PFW ? (27 * BN + 255) / 256 : 1;
    uint4 ph[NHV], pw[NWV];
    auto fetch_w = [&](int c) {
        const uint16_t* wc = wr + (int64_t)c * 27 * g.Cout * 8;
#pragma unroll
        for (int u = 0; u < NWV; u++) {
            const int e = tid + 256 * u;
            const int tap = e / BN, n = e - tap * BN;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (e < 27 * BN) v = *reinterpret_cast<const uint4*>(wc + ((int64_t)tap * g.Cout + n0 + n) * 8);
            pw[u] = v;
        }
    };
    auto fetch = [&](int c) {
        const bool second = src.in2 && c * 8 >= src.c1;
        const uint16_t* sp = second ? src.in2 : in;
        const int sc = second ? g.Cin - src.c1 : src.c1;
        const int co = second ? c * 8 - src.c1 : c * 8;
#pragma unroll
        for (int u = 0; u < NHV; u++) {
            const int h = tid + 256 * u;
            const int hz = h / (SHY * SHX), hr = h - hz * (SHY * SHX), hy = hr / SHX,
                      hx = hr - hy * SHX;
            int Z = z0 - 1 + hz, Y = y0 - 1 + hy, X = x0 - 1 + hx;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (h < HVOX_ && Z >= 0 && Z < S && Y >= 0 && Y < S && X >= 0 && X < S) {
                if (src.up) {
                    Z >>= 1;
                    Y >>= 1;
                    X >>= 1;
                }
                v = *reinterpret_cast<const uint4*>(sp + (ss0 + ((int64_t)Z * Ss + Y) * Ss + X) * sc +
                                                    co);
            }
            ph[u] = v;
        }
        if (PFW) fetch_w(c);
    };
    if (tid < BN) *reinterpret_cast<uint4*>(&wsh[(27 * BN + tid) * 8]) = make_uint4(0, 0, 0, 0);
    fetch(0);
    for (int c = 0; c < nchunk; c++) {
        __syncthreads();  // the previous chunk's tiles have been read
#pragma unroll
        for (int u = 0; u < NHV; u++) {
            const int h = tid + 256 * u;
            if (h < HVOX_) *reinterpret_cast<uint4*>(&hal[h * 8]) = ph[u];
        }
        if (PFW) {
#pragma unroll
            for (int u = 0; u < NWV; u++) {
                const int e = tid + 256 * u;
                if (e < 27 * BN) *reinterpret_cast<uint4*>(&wsh[e * 8]) = pw[u];
            }
        } else {
            const uint16_t* wc = wr + (int64_t)c * 27 * g.Cout * 8;
            for (int e = tid; e < 27 * BN; e += 256) {
                const int tap = e / BN, n = e - tap * BN;
                *reinterpret_cast<uint4*>(&wsh[e * 8]) =
                    *reinterpret_cast<const uint4*>(wc + ((int64_t)tap * g.Cout + n0 + n) * 8);
            }
        }
        __syncthreads();
        if (c + 1 < nchunk) fetch(c + 1);
        __builtin_amdgcn_sched_barrier(0);  // issue the next chunk's loads before the MFMAs
#pragma unroll 1
        for (int st = 0; st < NSTEP; st++) {
            // the padding slot (tap 27) multiplies the tap-26 window (in
            // bounds, finite) by the zero weight row: an exact zero
            const int tap = st * 4 + kg;
            const int ta = tap < 27 ? tap : 26;
            const int dz = ta / 9, rr = ta - dz * 9, dy = rr / 3, dx = rr - dy * 3;
            const int toff = (dz * SHY + dy) * SHX + dx;
            const uint16_t* hp = &hal[(hbase + toff) * 8];
            bf16x8 a[8], bb[NT];
#pragma unroll
            for (int r = 0; r < RT; r++)
                a[r] = *reinterpret_cast<const bf16x8*>(hp + ((r >> 2) * SHY + (r & 3)) * SHX * 8);
#pragma unroll
            for (int j = 0; j < NT; j++)
                bb[j] = *reinterpret_cast<const bf16x8*>(&wsh[(tap * BN + j * 16 + (lane & 15)) * 8]);
#pragma unroll
            for (int r = 0; r < RT; r++)
#pragma unroll
                for (int j = 0; j < NT; j++)
                    acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], bb[j], acc[r][j], 0, 0, 0);
        }
    }
    // epilogue: lane holds rows 4 (lane / 16) + q of each tile, column lane % 16;
    // row x of tile r is voxel (z0 + ZW wv + r / 4, y0 + r % 4, x0 + x).
    // A bf16-only output is staged through LDS (voxel-major rows padded by 8
    // values, so the four lane groups write different banks) and stored as
    // whole 16-byte pieces, 8 channels of one voxel per lane: consecutive
    // lanes write consecutive memory instead of 2-byte values 64 bytes apart.
    if (out_bf && !out_f32 && mode != EP_DACT) {
        constexpr int RH = RT / 2, BNP = BN + 8, NCH = BN / 8;
        static_assert(4 * RH * 16 * BNP <= HAL_N + WSH_N, "output staging fits the tiles' LDS");
        static_assert((RH * 16 * NCH) % 64 == 0, "whole pieces per lane");
        uint16_t* const st = smem + wv * (RH * 16 * BNP);
        __syncthreads();  // every wave is done with the halo and weight tiles
#pragma unroll
        for (int h = 0; h < 2; h++) {
#pragma unroll
            for (int rr = 0; rr < RH; rr++) {
#pragma unroll
                for (int j = 0; j < NT; j++) {
                    const int cl = j * 16 + (lane & 15);
                    const float bv = bias ? bias[n0 + cl] : 0.0f;
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        float v = acc[h * RH + rr][j][q] + bv;
                        if (mode == EP_LRELU) v = v > 0.0f ? v : LRELU_SLOPE * v;
                        st[(rr * 16 + (lane >> 4) * 4 + q) * BNP + cl] = f2bf(v);
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < RH * 16 * NCH / 64; u++) {
                const int kk = lane + 64 * u;
                const int vv = kk / NCH, c8 = kk - vv * NCH;
                const int r = h * RH + (vv >> 4);
                const int Z = z0 + ZW * wv + (r >> 2), Y = y0 + (r & 3), X = x0 + (vv & 15);
                if (Z < S && Y < S && X < S) {
                    const int64_t m = vs0 + ((int64_t)Z * S + Y) * S + X;
                    *reinterpret_cast<uint4*>(&out_bf[m * g.Cout + n0 + c8 * 8]) =
                        *reinterpret_cast<const uint4*>(&st[vv * BNP + c8 * 8]);
                }
            }
            if (h == 0) __syncthreads();  // pieces read before the second half is staged
        }
    } else
#pragma unroll
    for (int r = 0; r < RT; r++) {
        const int Z = z0 + ZW * wv + (r >> 2), Y = y0 + (r & 3);
        if (Z >= S || Y >= S) continue;
#pragma unroll
        for (int j = 0; j < NT; j++) {
            const int col = n0 + j * 16 + (lane & 15);
            const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int X = x0 + (lane >> 4) * 4 + q;
                if (X >= S) continue;
                const int64_t m = vs0 + ((int64_t)Z * S + Y) * S + X;
                float v = acc[r][j][q] + bv;
                const int64_t o = m * g.Cout + col;
                if (mode == EP_LRELU) {
                    v = v > 0.0f ? v : LRELU_SLOPE * v;
                } else if (mode == EP_DACT) {
                    v = bf2f(yref[o]) > 0.0f ? v : LRELU_SLOPE * v;
                }
                if (out_bf) out_bf[o] = f2bf(v);
                if (out_f32) out_f32[o] = v;
            }
        }
    }
    if constexpr (RT == 8)
    if (src.pool) {
        // 2^3 average pooling of the bf16 outputs: a lane holds all eight
        // voxels of its blocks (z pair: tiles r and r + 4, y pair: tiles r and
        // r + 1, x pair: q and q + 1); summed in the order of k_avgpool2
        const int So = S / 2, Z = z0 + 2 * wv;
        if (Z < S) {
#pragma unroll
            for (int yp = 0; yp < 2; yp++) {
                const int Y = y0 + 2 * yp;
                if (Y >= S) continue;
#pragma unroll
                for (int j = 0; j < NT; j++) {
                    const int col = n0 + j * 16 + (lane & 15);
                    const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
                    for (int qp = 0; qp < 2; qp++) {
                        const int X = x0 + (lane >> 4) * 4 + 2 * qp;
                        if (X >= S) continue;
                        float sum = 0.0f;
#pragma unroll
                        for (int d = 0; d < 8; d++) {
                            const int r = (d >> 2) * 4 + 2 * yp + ((d >> 1) & 1);
                            float v = acc[r][j][2 * qp + (d & 1)] + bv;
                            if (mode == EP_LRELU) v = v > 0.0f ? v : LRELU_SLOPE * v;
                            sum += bf2f(f2bf(v));
                        }
                        const int64_t po = (((int64_t)b * So + Z / 2) * So + Y / 2) * So + X / 2;
                        src.pool[po * g.Cout + col] = f2bf(0.125f * sum);
                    }
                }
            }
        }
    }
}

// Weights for the data gradient: w'[ci][tap'][co] = w[co][26 - tap'][ci] (or
// the same tap for 1^3 kernels), so that backward data is a forward pass.
__global__ void k_wflip(const uint16_t* __restrict__ w, int Cout, int Cin, int kvol,
                        uint16_t* __restrict__ wf) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)Cout * Cin * kvol;
    if (e >= n) return;
    const int co = (int)(e % Cout);
    int64_t t = e / Cout;
    const int tap = (int)(t % kvol);
    const int ci = (int)(t / kvol);
    const int src_tap = kvol == 27 ? 26 - tap : tap;
    wf[((int64_t)ci * kvol + tap) * Cout + co] = w[((int64_t)co * kvol + src_tap) * Cin + ci];
}

// Backward weight: dW[co][k] += sum_m dOut[m][co] * A[m][k] over a chunk of
// voxels per block.  Tiles: 64 K entries x BN output channels, voxels in steps
// of 32, both operands transposed into LDS so MFMA fragments are contiguous.
// With bpart, the blocks of the first K tile also sum dOut over their voxels
// (the bias gradient) from the transposed tile already in LDS: thread t adds
// channel t % BN over its share of each step's voxels, and the shares are
// combined in order at the end.
template <int BN>
__global__ __launch_bounds__(256) void k_conv3d_wgrad(const uint16_t* __restrict__ in,
                                                      const uint16_t* __restrict__ dout,
                                                      ConvGeom g, int64_t m_per_block,
                                                      float* __restrict__ part,
                                                      float* __restrict__ bpart) {
    constexpr int BKW = 64;                  // K tile (rows of dW^T)
    __shared__ __attribute__((aligned(16))) uint16_t sAt[BKW * CV_APITCH];  // [k][m]
    __shared__ __attribute__((aligned(16))) uint16_t sBt[BN * CV_APITCH];   // [co][m]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int k0 = blockIdx.x * BKW;
    const int n0 = blockIdx.y * BN;
    const int64_t mb = (int64_t)blockIdx.z * m_per_block;
    const int64_t me = min(g.M, mb + m_per_block);
    constexpr int NT = BN / 16;
    // this thread's K columns (8 of one tap) are the same for every voxel
    const int kw = k0 + (tid & 7) * 8;
    const bool kin = kw < g.K;
    const int tap = kin ? (kw >> g.lgC) : 0, ci = kw & (g.Cin - 1);
    const int64_t off = tap_offset(g, tap);
    // wave wv owns K rows [wv * 16, +16) x all BN columns
    f32x4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) acc[j] = f32x4{0, 0, 0, 0};
    const bool do_bias = bpart != nullptr && blockIdx.x == 0;
    constexpr int BPARTS = 256 / BN, BSPAN = 32 / BPARTS;  // voxels per thread and step
    const int bc = tid % BN, bq = tid / BN;
    float bsum = 0.0f;
    for (int64_t m0 = mb; m0 < me; m0 += 32) {
        // A^T: 32 voxels x 64 K entries -> 256 loads of 8 K entries
        {
            const int mrow = tid >> 3, grp = tid & 7;
            const int64_t m = m0 + mrow;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (m < me) v = im2col8t(in, g, row_taps(g, m), kin, tap, ci, off);
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int q = 0; q < 8; q++) sAt[(grp * 8 + q) * CV_APITCH + mrow] = h[q];
        }
        // dOut^T: 32 voxels x BN channels
        for (int e = tid; e < 32 * (BN / 8); e += 256) {
            const int mrow = e / (BN / 8), grp = e % (BN / 8);
            const int64_t m = m0 + mrow;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (m < me) v = *reinterpret_cast<const uint4*>(dout + m * g.Cout + n0 + grp * 8);
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int q = 0; q < 8; q++) sBt[(grp * 8 + q) * CV_APITCH + mrow] = h[q];
        }
        __syncthreads();
        if (do_bias) {
            const uint16_t* r = &sBt[bc * CV_APITCH + bq * BSPAN];
#pragma unroll
            for (int q = 0; q < BSPAN; q++) bsum += bf2f(r[q]);
        }
        const int kq = (lane >> 4) * 8;
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sAt[(wv * 16 + (lane & 15)) * CV_APITCH + kq]);
#pragma unroll
        for (int j = 0; j < NT; j++) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sBt[(j * 16 + (lane & 15)) * CV_APITCH + kq]);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
        }
        __syncthreads();
    }
    // acc[j][t]: row (K) = wv*16 + 4*(lane/16) + t, column (co) = j*16 + lane%16;
    // each chunk of voxels owns its own partial gradient, reduced in chunk
    // order afterwards (a deterministic sum)
    float* pc = part + (int64_t)blockIdx.z * g.Cout * g.K;
#pragma unroll
    for (int j = 0; j < NT; j++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int k = k0 + wv * 16 + (lane >> 4) * 4 + t;
            const int co = n0 + j * 16 + (lane & 15);
            if (k < g.K) pc[(int64_t)co * g.K + k] = acc[j][t];
        }
    if (do_bias) {
        // the loop ended on a barrier, so the A tile's LDS is free
        float* sb = reinterpret_cast<float*>(sAt);
        sb[tid] = bsum;
        __syncthreads();
        if (tid < BN) {
            float s = 0.0f;
            for (int q = 0; q < BPARTS; q++) s += sb[q * BN + tid];
            bpart[(int64_t)blockIdx.z * g.Cout + n0 + tid] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient from channel-major operands.  dW[co][tap][ci] = sum over
// voxels m of dY[m][co] * X[m + d(tap)][ci]: a matrix product whose
// reduction runs over voxels, so each MFMA operand fragment is 8 consecutive
// voxels of one channel.  With the layer input and output gradient copied to
// channel-major order ([b][c][v]) once per layer, such a fragment is one
// aligned 16-byte load: the y and z tap offsets move it by whole rows, and
// the x offsets of -1 and +1 come from the same 8 voxels and their left and
// right neighbours by byte alignment.
// ---------------------------------------------------------------------------
// out[b][c][v] = in[b][v][c] (bf16), one block per 64 voxels of one sample
// (V = S^3 voxels per sample, lgS = log2 S).  The input may be described as
// the fused convolutions take it: channels c1 .. C - 1 from a second source
// in2 (channel concatenation; c1 = C without one), and with up = 1 both
// sources on the (S/2)^3 grid, read at the nearest-upsampled voxel.
__global__ __launch_bounds__(256) void k_to_cmajor(const uint16_t* __restrict__ in,
                                                   const uint16_t* __restrict__ in2, int c1,
                                                   int up, int lgS, int64_t V, int C,
                                                   uint16_t* __restrict__ out) {
    __shared__ uint16_t t[256 * 66];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int64_t b = v0 / V, vv = v0 - b * V;
    const int cg8 = C / 8;
    for (int e = threadIdx.x; e < 64 * cg8; e += 256) {
        const int vox = e / cg8, cg = e - vox * cg8;
        int64_t sv = v0 + vox;  // voxel of the source (same grid)
        if (up) {
            const int64_t w = vv + vox, S = (int64_t)1 << lgS, h = S >> 1;
            const int64_t z = w >> (2 * lgS), y = (w >> lgS) & (S - 1), x = w & (S - 1);
            sv = (b * h + (z >> 1)) * h * h + (y >> 1) * h + (x >> 1);
        }
        const int c = cg * 8;
        const uint16_t* src = (in2 && c >= c1) ? in2 + sv * (C - c1) + (c - c1)
                                               : in + sv * (in2 ? c1 : C) + c;
        const uint4 d = *reinterpret_cast<const uint4*>(src);
        const uint16_t* h = reinterpret_cast<const uint16_t*>(&d);
#pragma unroll
        for (int q = 0; q < 8; q++) t[(cg * 8 + q) * 66 + vox] = h[q];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < C * 8; e += 256) {
        const int c = e >> 3, seg = e & 7;
        uint4 d;
        uint16_t* h = reinterpret_cast<uint16_t*>(&d);
#pragma unroll
        for (int q = 0; q < 8; q++) h[q] = t[c * 66 + seg * 8 + q];
        *reinterpret_cast<uint4*>(out + (b * C + c) * V + vv + seg * 8) = d;
    }
}

// One wave per task: 16 input channels (ci block), one z offset of the taps
// (all 9 of its (y, x) offsets; the single tap of a 1^3 kernel), 32 output
// channels (co block), over one chunk of voxels in steps of 32.  Per step
// each lane loads its 8 voxels of two output-gradient channels and, per y
// offset, 8 voxels of its input channel plus the two neighbours, and the wave
// issues 2 MFMAs per tap.  Partial results per chunk, reduced in chunk order
// afterwards; the tasks of the first ci block and z offset also sum the
// output gradient for the bias.
template <int KS>
__global__ __launch_bounds__(256) void k_wgrad_cm(const uint16_t* __restrict__ xt,
                                                  const uint16_t* __restrict__ yt, int B, int lgS,
                                                  int Cin, int Cout, int64_t m_per_chunk,
                                                  float* __restrict__ part,
                                                  float* __restrict__ bpart) {
    constexpr int NDZ = KS == 3 ? 3 : 1, NT = KS == 3 ? 9 : 1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int S = 1 << lgS;
    const int64_t V = (int64_t)1 << (3 * lgS), M = (int64_t)B * V;
    const int ncib = (Cin + 15) / 16, ncob = (Cout + 31) / 32;
    const int task = blockIdx.y * 4 + wv;
    if (task >= ncib * NDZ * ncob) return;  // no barrier in this kernel
    const int cib = task % ncib, dzi = (task / ncib) % NDZ, cob = task / (ncib * NDZ);
    const int dz = KS == 3 ? dzi - 1 : 0;
    const int ci = cib * 16 + (lane & 15);
    const bool civ = ci < Cin;
    const int coa = cob * 32 + (lane & 15), cob2 = coa + 16;
    const bool cva = coa < Cout, cvb = cob2 < Cout;
    const bool do_bias = bpart != nullptr && cib == 0 && dzi == 0;
    f32x4 acc[NT][2];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t][0] = acc[t][1] = f32x4{0, 0, 0, 0};
    float bsa = 0.0f, bsb = 0.0f;
    const int64_t mb = (int64_t)blockIdx.x * m_per_chunk;
    const int64_t me = min(M, mb + m_per_chunk);
    for (int64_t m0 = mb; m0 < me; m0 += 32) {
        // this lane's 8 voxels: one x-row segment
        const int64_t m = m0 + (lane >> 4) * 8;
        const int64_t b = m >> (3 * lgS), v = m & (V - 1);
        const int x0 = (int)(v & (S - 1)), y = (int)((v >> lgS) & (S - 1)),
                  z = (int)(v >> (2 * lgS));
        const uint4 zero4 = make_uint4(0, 0, 0, 0);
        const uint4 ua = cva ? *reinterpret_cast<const uint4*>(yt + (b * Cout + coa) * V + v) : zero4;
        const uint4 ub = cvb ? *reinterpret_cast<const uint4*>(yt + (b * Cout + cob2) * V + v) : zero4;
        if (do_bias) {
            const uint16_t* ha = reinterpret_cast<const uint16_t*>(&ua);
            const uint16_t* hb = reinterpret_cast<const uint16_t*>(&ub);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                bsa += bf2f(ha[q]);
                bsb += bf2f(hb[q]);
            }
        }
        bf16x8 ya, yb;
        __builtin_memcpy(&ya, &ua, 16);
        __builtin_memcpy(&yb, &ub, 16);
        const int zz = z + dz;
        const bool zv = civ && zz >= 0 && zz < S;
#pragma unroll
        for (int dyi = 0; dyi < NDZ; dyi++) {
            const int dy = KS == 3 ? dyi - 1 : 0;
            const int yy = y + dy;
            uint4 c0 = zero4;
            uint32_t left = 0, right = 0;
            if (zv && yy >= 0 && yy < S) {
                const uint16_t* row = xt + (b * Cin + ci) * V + ((int64_t)zz << (2 * lgS)) +
                                      ((int64_t)yy << lgS);
                c0 = *reinterpret_cast<const uint4*>(row + x0);
                if (KS == 3) {
                    if (x0 > 0) left = row[x0 - 1];
                    if (x0 + 8 < S) right = row[x0 + 8];
                }
            }
            bf16x8 f0;
            __builtin_memcpy(&f0, &c0, 16);
            if (KS == 3) {
                // x offset +1: (e1 .. e8); x offset -1: (e-1 .. e6)
                const uint32_t a0 = __builtin_amdgcn_alignbyte(c0.y, c0.x, 2);
                const uint32_t a1 = __builtin_amdgcn_alignbyte(c0.z, c0.y, 2);
                const uint32_t a2 = __builtin_amdgcn_alignbyte(c0.w, c0.z, 2);
                const uint32_t a3 = __builtin_amdgcn_alignbyte(right, c0.w, 2);
                const uint32_t g0 = __builtin_amdgcn_alignbyte(c0.x, left << 16, 2);
                const uint4 up = make_uint4(a0, a1, a2, a3), um = make_uint4(g0, a0, a1, a2);
                bf16x8 fp, fm;
                __builtin_memcpy(&fp, &up, 16);
                __builtin_memcpy(&fm, &um, 16);
                const int tb = dyi * 3;  // tap index within this z offset: dy * 3 + dx
                acc[tb + 0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fm, ya, acc[tb + 0][0], 0, 0, 0);
                acc[tb + 0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fm, yb, acc[tb + 0][1], 0, 0, 0);
                acc[tb + 1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f0, ya, acc[tb + 1][0], 0, 0, 0);
                acc[tb + 1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f0, yb, acc[tb + 1][1], 0, 0, 0);
                acc[tb + 2][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fp, ya, acc[tb + 2][0], 0, 0, 0);
                acc[tb + 2][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fp, yb, acc[tb + 2][1], 0, 0, 0);
            } else {
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f0, ya, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f0, yb, acc[0][1], 0, 0, 0);
            }
        }
    }
    // acc[t][h][r]: ci = cib * 16 + 4 * (lane / 16) + r, co = cob * 32 + 16 h + lane % 16
    const int K = (KS == 3 ? 27 : 1) * Cin;
    float* pc = part + (int64_t)blockIdx.x * Cout * K;
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int tap = dzi * 9 * (KS == 3 ? 1 : 0) + t;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int co = cob * 32 + 16 * h + (lane & 15);
            if (co >= Cout) continue;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int c = cib * 16 + 4 * (lane >> 4) + r;
                if (c < Cin) pc[(int64_t)co * K + tap * Cin + c] = acc[t][h][r];
            }
        }
    }
    if (do_bias) {
        // lanes l, l + 16, l + 32, l + 48 hold the same channels
        bsa += __shfl_xor(bsa, 16, 64);
        bsa += __shfl_xor(bsa, 32, 64);
        bsb += __shfl_xor(bsb, 16, 64);
        bsb += __shfl_xor(bsb, 32, 64);
        if (lane < 16) {
            if (cva) bpart[(int64_t)blockIdx.x * Cout + coa] = bsa;
            if (cvb) bpart[(int64_t)blockIdx.x * Cout + cob2] = bsb;
        }
    }
}

// The same product for grids of 16^3, 32^3 and 64^3 with the operands staged
// in LDS: a block of three waves (one per z offset of the taps) takes tiles of
// 256 output voxels (R = 256 / S rows of one z plane) for one block of 16
// input and 32 output channels.  Per tile it stages the input rows the 27
// taps read (3 planes x (R + 2) rows x S voxels x 16 channels, from the
// channel-major copy, rows padded by 8 zeros on each side so the x offsets
// of -1 and +1 read zeros at the volume's edge) and the tile's output
// gradient (32 channels x 256 voxels), then runs its 8 steps of 32 voxels
// from LDS: per step and wave 3 x (one 16-byte read and two neighbours) and
// two 16-byte gradient reads feed 18 MFMAs.  Each block takes a run of
// consecutive tiles and writes one partial gradient.
template <int LGS>
__global__ __launch_bounds__(192) void k_wgrad_lds(const uint16_t* __restrict__ xt,
                                                   const uint16_t* __restrict__ yt, int B, int Cin,
                                                   int Cout, int tiles_per_block,
                                                   float* __restrict__ part,
                                                   float* __restrict__ bpart) {
    constexpr int S = 1 << LGS, R = 256 / S, XP = S + 16, YP = 256 + 8;
    constexpr int64_t V = (int64_t)S * S * S;
    __shared__ __attribute__((aligned(16))) uint16_t sx[3][R + 2][16][XP];
    __shared__ __attribute__((aligned(16))) uint16_t sy[32][YP];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ncib = (Cin + 15) / 16;
    const int cib = blockIdx.y % ncib, cob = blockIdx.y / ncib;
    const int ntiles = B * S * (S / R);
    const int t0 = blockIdx.x * tiles_per_block, t1 = min(ntiles, t0 + tiles_per_block);
    // the pads of every staged row stay zero
    for (int e = tid; e < 3 * (R + 2) * 16; e += 192) {
        uint16_t* row = &sx[0][0][0][0] + (int64_t)e * XP;
        *reinterpret_cast<uint4*>(row) = make_uint4(0, 0, 0, 0);
        *reinterpret_cast<uint4*>(row + 8 + S) = make_uint4(0, 0, 0, 0);
    }
    const int cl = lane & 15;  // this lane's input channel (A rows) and output channel (B cols)
    const int coa = cob * 32 + cl, cob2 = coa + 16;
    const bool cva = coa < Cout, cvb = cob2 < Cout;
    const bool do_bias = bpart != nullptr && cib == 0 && wv == 0;
    f32x4 acc[9][2];
#pragma unroll
    for (int t = 0; t < 9; t++) acc[t][0] = acc[t][1] = f32x4{0, 0, 0, 0};
    float bsa = 0.0f, bsb = 0.0f;
    // the next tile's input rows and output gradient are read into registers
    // while the current tile's MFMAs run, and stored to LDS between barriers
    constexpr int XCH = 3 * (R + 2) * 16 * (S / 8);  // 16-byte pieces of input rows
    constexpr int NX = (XCH + 191) / 192, NY = (32 * 32 + 191) / 192;
    uint4 px[NX], py[NY];
    auto load_tile = [&](int tile) {
        const int plane = tile / (S / R), y0 = (tile % (S / R)) * R;
        const int b = plane >> LGS, z = plane & (S - 1);
#pragma unroll
        for (int j = 0; j < NX; j++) {
            const int e = tid + 192 * j;
            const int k = e % (S / 8);
            const int c = (e / (S / 8)) % 16;
            const int r = (e / (S / 8 * 16)) % (R + 2);
            const int pz = e / (S / 8 * 16 * (R + 2));
            const int zz = z + pz - 1, yy = y0 + r - 1, ci = cib * 16 + c;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (e < XCH && zz >= 0 && zz < S && yy >= 0 && yy < S && ci < Cin)
                v = *reinterpret_cast<const uint4*>(
                    xt + ((int64_t)b * Cin + ci) * V + ((int64_t)zz << (2 * LGS)) +
                    ((int64_t)yy << LGS) + k * 8);
            px[j] = v;
        }
        const int64_t vb = ((int64_t)z << (2 * LGS)) + ((int64_t)y0 << LGS);
#pragma unroll
        for (int j = 0; j < NY; j++) {
            const int e = tid + 192 * j;
            const int k = e & 31, c = e >> 5, co = cob * 32 + c;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (e < 32 * 32 && co < Cout)
                v = *reinterpret_cast<const uint4*>(yt + ((int64_t)b * Cout + co) * V + vb + k * 8);
            py[j] = v;
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int j = 0; j < NX; j++) {
            const int e = tid + 192 * j;
            if (e < XCH) {
                const int k = e % (S / 8);
                const int c = (e / (S / 8)) % 16;
                const int r = (e / (S / 8 * 16)) % (R + 2);
                const int pz = e / (S / 8 * 16 * (R + 2));
                *reinterpret_cast<uint4*>(&sx[pz][r][c][8 + k * 8]) = px[j];
            }
        }
#pragma unroll
        for (int j = 0; j < NY; j++) {
            const int e = tid + 192 * j;
            if (e < 32 * 32) *reinterpret_cast<uint4*>(&sy[e >> 5][(e & 31) * 8]) = py[j];
        }
    };
    if (t0 < t1) load_tile(t0);
    for (int tile = t0; tile < t1; tile++) {
        __syncthreads();  // the previous tile's reads are done
        store_tile();
        __syncthreads();
        if (tile + 1 < t1) load_tile(tile + 1);
#pragma unroll 2
        for (int st = 0; st < 8; st++) {
            const int t = st * 32 + (lane >> 4) * 8;  // this lane's 8 voxels in the tile
            const int r = t >> LGS, x0 = t & (S - 1);
            uint4 ua = *reinterpret_cast<const uint4*>(&sy[cl][t]);
            uint4 ub = *reinterpret_cast<const uint4*>(&sy[cl + 16][t]);
            if (!cva) ua = make_uint4(0, 0, 0, 0);
            if (!cvb) ub = make_uint4(0, 0, 0, 0);
            if (do_bias) {
                const uint16_t* ha = reinterpret_cast<const uint16_t*>(&ua);
                const uint16_t* hb = reinterpret_cast<const uint16_t*>(&ub);
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    bsa += bf2f(ha[q]);
                    bsb += bf2f(hb[q]);
                }
            }
            bf16x8 ya, yb;
            __builtin_memcpy(&ya, &ua, 16);
            __builtin_memcpy(&yb, &ub, 16);
#pragma unroll
            for (int dyi = 0; dyi < 3; dyi++) {
                const uint16_t* row = &sx[wv][r + dyi][cl][8];
                const uint4 c0 = *reinterpret_cast<const uint4*>(row + x0);
                const uint32_t left = row[x0 - 1], right = row[x0 + 8];
                const uint32_t a0 = __builtin_amdgcn_alignbyte(c0.y, c0.x, 2);
                const uint32_t a1 = __builtin_amdgcn_alignbyte(c0.z, c0.y, 2);
                const uint32_t a2 = __builtin_amdgcn_alignbyte(c0.w, c0.z, 2);
                const uint32_t a3 = __builtin_amdgcn_alignbyte(right, c0.w, 2);
                const uint32_t g0 = __builtin_amdgcn_alignbyte(c0.x, left << 16, 2);
                const uint4 up = make_uint4(a0, a1, a2, a3), um = make_uint4(g0, a0, a1, a2);
                bf16x8 f0, fp, fm;
                __builtin_memcpy(&f0, &c0, 16);
                __builtin_memcpy(&fp, &up, 16);
                __builtin_memcpy(&fm, &um, 16);
                const int tb = dyi * 3;
                acc[tb + 0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fm, ya, acc[tb + 0][0], 0, 0, 0);
                acc[tb + 0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fm, yb, acc[tb + 0][1], 0, 0, 0);
                acc[tb + 1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f0, ya, acc[tb + 1][0], 0, 0, 0);
                acc[tb + 1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f0, yb, acc[tb + 1][1], 0, 0, 0);
                acc[tb + 2][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fp, ya, acc[tb + 2][0], 0, 0, 0);
                acc[tb + 2][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fp, yb, acc[tb + 2][1], 0, 0, 0);
            }
        }
    }
    // acc[t][h][r]: ci = cib * 16 + 4 * (lane / 16) + r, co = cob * 32 + 16 h + lane % 16,
    // tap = wv * 9 + t
    const int K = 27 * Cin;
    float* pc = part + (int64_t)blockIdx.x * Cout * K;
#pragma unroll
    for (int t = 0; t < 9; t++) {
        const int tap = wv * 9 + t;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int co = cob * 32 + 16 * h + cl;
            if (co >= Cout) continue;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int c = cib * 16 + 4 * (lane >> 4) + r;
                if (c < Cin) pc[(int64_t)co * K + tap * Cin + c] = acc[t][h][r];
            }
        }
    }
    if (do_bias) {
        bsa += __shfl_xor(bsa, 16, 64);
        bsa += __shfl_xor(bsa, 32, 64);
        bsb += __shfl_xor(bsb, 16, 64);
        bsb += __shfl_xor(bsb, 32, 64);
        if (lane < 16) {
            if (cva) bpart[(int64_t)blockIdx.x * Cout + coa] = bsa;
            if (cvb) bpart[(int64_t)blockIdx.x * Cout + cob2] = bsb;
        }
    }
}

// out[g][e] = sum over chunks c of group g (chunks gG .. gG + G - 1, in order)
// of part[c][e]: the first of two ordered levels when there are many chunks
__global__ void k_wgrad_group_sum(const float* __restrict__ part, int64_t n, int chunks, int G,
                                  float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int c0 = blockIdx.y * G, c1 = min(chunks, c0 + G);
    float s = 0.0f;
    for (int c = c0; c < c1; c++) s += part[(int64_t)c * n + e];
    out[(int64_t)blockIdx.y * n + e] = s;
}

// dw[e] += sum over chunks c (in order) of part[c][e]
__global__ void k_wgrad_reduce(const float* __restrict__ part, int64_t n, int chunks,
                               float* __restrict__ dw) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.0f;
    for (int c = 0; c < chunks; c++) s += part[(int64_t)c * n + e];
    dw[e] += s;
}

// Bias gradient from the per-chunk partials of k_conv3d_wgrad: one wave per
// channel, lane l sums chunks l, l + 64, ...; then the lanes in a fixed
// butterfly order.
__global__ __launch_bounds__(64) void k_bias_reduce(const float* __restrict__ part, int nb, int C,
                                                    float* __restrict__ db) {
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 64) s += part[(int64_t)b * C + c];
    s = wave_sum(s);
    if (threadIdx.x == 0) db[c] += s;
}

// ---------------------------------------------------------------------------
// Pooling, upsampling, concatenation (bf16, NDHWC)
// ---------------------------------------------------------------------------
__global__ void k_avgpool2(const uint16_t* __restrict__ in, int B, int S, int C,
                           uint16_t* __restrict__ out) {
    const int So = S / 2;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)B * So * So * So * C;
    if (e >= n) return;
    const int c = (int)(e % C);
    int64_t t = e / C;
    const int x = (int)(t % So);
    t /= So;
    const int y = (int)(t % So);
    t /= So;
    const int z = (int)(t % So);
    const int64_t b = t / So;
    float s = 0.0f;
    for (int d = 0; d < 8; d++) {
        const int X = 2 * x + (d & 1), Y = 2 * y + ((d >> 1) & 1), Z = 2 * z + (d >> 2);
        s += bf2f(in[(((b * S + Z) * S + Y) * S + X) * C + c]);
    }
    out[e] = f2bf(0.125f * s);
}

__global__ void k_avgpool2_bwd(const uint16_t* __restrict__ dout, int B, int S, int C,
                               uint16_t* __restrict__ din) {
    // din at fine resolution S; dout at S/2
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)B * S * S * S * C;
    if (e >= n) return;
    const int c = (int)(e % C);
    int64_t t = e / C;
    const int x = (int)(t % S);
    t /= S;
    const int y = (int)(t % S);
    t /= S;
    const int z = (int)(t % S);
    const int64_t b = t / S;
    const int So = S / 2;
    din[e] = f2bf(0.125f * bf2f(dout[(((b * So + z / 2) * So + y / 2) * So + x / 2) * C + c]));
}

__global__ void k_upsample2(const uint16_t* __restrict__ in, int B, int S, int C,
                            uint16_t* __restrict__ out) {
    // in at S, out at 2S (nearest)
    const int So = 2 * S;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)B * So * So * So * C;
    if (e >= n) return;
    const int c = (int)(e % C);
    int64_t t = e / C;
    const int x = (int)(t % So);
    t /= So;
    const int y = (int)(t % So);
    t /= So;
    const int z = (int)(t % So);
    const int64_t b = t / So;
    out[e] = in[(((b * S + z / 2) * S + y / 2) * S + x / 2) * C + c];
}

__global__ void k_upsample2_bwd(const uint16_t* __restrict__ dout, int B, int S, int C,
                                uint16_t* __restrict__ din) {
    // din at S (coarse), dout at 2S: sum of the 8 fine cells
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)B * S * S * S * C;
    if (e >= n) return;
    const int c = (int)(e % C);
    int64_t t = e / C;
    const int x = (int)(t % S);
    t /= S;
    const int y = (int)(t % S);
    t /= S;
    const int z = (int)(t % S);
    const int64_t b = t / S;
    const int Sf = 2 * S;
    float s = 0.0f;
    for (int d = 0; d < 8; d++) {
        const int X = 2 * x + (d & 1), Y = 2 * y + ((d >> 1) & 1), Z = 2 * z + (d >> 2);
        s += bf2f(dout[(((b * Sf + Z) * Sf + Y) * Sf + X) * C + c]);
    }
    din[e] = f2bf(s);
}

// out[v][0:Ca] = a[v], out[v][Ca:Ca+Cb] = b[v]; split is the reverse.
__global__ void k_concat(const uint16_t* __restrict__ a, int Ca, const uint16_t* __restrict__ b,
                         int Cb, int64_t V, uint16_t* __restrict__ out, int split) {
    const int C = Ca + Cb;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= V * C) return;
    const int64_t v = e / C;
    const int c = (int)(e % C);
    if (!split) {
        out[e] = c < Ca ? a[v * Ca + c] : b[v * Cb + (c - Ca)];
    } else {  // a and b are outputs (const cast by caller contract)
        uint16_t* aa = const_cast<uint16_t*>(a);
        uint16_t* bb = const_cast<uint16_t*>(b);
        if (c < Ca) aa[v * Ca + c] = out[e];
        else bb[v * Cb + (c - Ca)] = out[e];
    }
}

// ---------------------------------------------------------------------------
// Loss and optimiser
// ---------------------------------------------------------------------------
// Mean squared error over the first nc channels of pred[V][Cp] vs target[V][nc]
// (fp32); writes dL/dpred (bf16, padding channels zero) and per-block partial
// sums of the squared error.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ pred, int Cp,
                                             const float* __restrict__ target, int nc, int64_t V,
                                             float scale, uint16_t* __restrict__ dpred,
                                             double* __restrict__ part) {
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < V * Cp;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = e / Cp;
        const int c = (int)(e % Cp);
        float d = 0.0f;
        if (c < nc) {
            d = pred[e] - target[v * nc + c];
            s += (double)d * d;
        }
        if (dpred) dpred[e] = f2bf(2.0f * d * scale);
    }
    s = wave_sum(s);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// w -= lr * mhat / (sqrt(vhat) + eps), mhat = m / (1 - b1^t), vhat = v / (1 - b2^t).
// Also refreshes the bf16 copy of the weights.
__global__ __launch_bounds__(256) void k_adam(int64_t n, float* __restrict__ w,
                                              const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, float lr, float b1, float b2,
                                              float omb1, float omb2, float eps, float c1,
                                              float c2, uint16_t* __restrict__ wbf) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    // omb = 1 - b, rounded once from the double value (1.0f - b in FP32 would
    // lose the low bits of b2 = 0.999)
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = f2bf(wi);
}

// out = (a + b) * (y > 0 ? 1 : slope) with b and y optional (gradient routing
// at skip, pooling and upsampling junctions of the network).
__global__ void k_grad_combine(int64_t n, const uint16_t* __restrict__ a,
                               const uint16_t* __restrict__ b, const uint16_t* __restrict__ y,
                               uint16_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = bf2f(a[i]);
    if (b) v += bf2f(b[i]);
    if (y && !(bf2f(y[i]) > 0.0f)) v *= LRELU_SLOPE;
    out[i] = f2bf(v);
}

// Backward-pass fusions of the up and down paths, eight channels (16 bytes)
// per thread.  Each computes, value for value, what the separate passes it
// replaces compute (the same bf16 roundings in the same order), so the
// gradients are bit-identical to the unfused sequence.
__device__ __forceinline__ float dact(float v, uint16_t y) {
    return bf2f(y) > 0.0f ? v : v * LRELU_SLOPE;
}

// The gradient of a concatenated input [v][Ca + Cb] split into [v][Ca] and
// [v][Cb], the first part times the leaky-ReLU derivative at ya (what the
// split followed by the gradient combination with ya computes).
__global__ __launch_bounds__(256) void k_split_dact(const uint16_t* __restrict__ gc, int64_t V,
                                                    int Ca, int Cb,
                                                    const uint16_t* __restrict__ ya,
                                                    uint16_t* __restrict__ ga,
                                                    uint16_t* __restrict__ gb) {
    const int P = (Ca + Cb) / 8;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= V * P) return;
    const int64_t v = e / P;
    const int c = (int)(e - v * P) * 8;
    const uint4 g = *reinterpret_cast<const uint4*>(gc + v * (Ca + Cb) + c);
    if (c < Ca) {
        const uint4 y = *reinterpret_cast<const uint4*>(ya + v * Ca + c);
        const uint16_t* gh = reinterpret_cast<const uint16_t*>(&g);
        const uint16_t* yh = reinterpret_cast<const uint16_t*>(&y);
        uint4 o;
        uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
        for (int j = 0; j < 8; j++) oh[j] = f2bf(dact(bf2f(gh[j]), yh[j]));
        *reinterpret_cast<uint4*>(ga + v * Ca + c) = o;
    } else {
        *reinterpret_cast<uint4*>(gb + v * Cb + (c - Ca)) = g;
    }
}

// Nearest-upsampling backward (din at S: the sum of its 8 cells of dout at
// 2S, rounded to bf16) times the leaky-ReLU derivative at y.
__global__ __launch_bounds__(256) void k_upsample2_bwd_dact(const uint16_t* __restrict__ dout,
                                                            int B, int S, int C,
                                                            const uint16_t* __restrict__ y,
                                                            uint16_t* __restrict__ din) {
    const int P = C / 8;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * S * S * S * P) return;
    const int c = (int)(e % P) * 8;
    int64_t t = e / P;
    const int x = (int)(t % S);
    t /= S;
    const int yy = (int)(t % S);
    t /= S;
    const int z = (int)(t % S);
    const int64_t b = t / S;
    const int Sf = 2 * S;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int d = 0; d < 8; d++) {
        const int X = 2 * x + (d & 1), Y = 2 * yy + ((d >> 1) & 1), Z = 2 * z + (d >> 2);
        const uint4 g = *reinterpret_cast<const uint4*>(dout + (((b * Sf + Z) * Sf + Y) * Sf + X) * C + c);
        const uint16_t* gh = reinterpret_cast<const uint16_t*>(&g);
#pragma unroll
        for (int j = 0; j < 8; j++) s[j] += bf2f(gh[j]);
    }
    const int64_t o0 = (((b * S + z) * S + yy) * S + x) * C + c;
    const uint4 yv = *reinterpret_cast<const uint4*>(y + o0);
    const uint16_t* yh = reinterpret_cast<const uint16_t*>(&yv);
    uint4 o;
    uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
    for (int j = 0; j < 8; j++) oh[j] = f2bf(dact(bf2f(f2bf(s[j])), yh[j]));
    *reinterpret_cast<uint4*>(din + o0) = o;
}

// 2^3 average-pooling backward (din at S: an eighth of its coarse cell of
// dout, rounded to bf16) plus the skip gradient, times the leaky-ReLU
// derivative at y.
__global__ __launch_bounds__(256) void k_avgpool2_bwd_combine(const uint16_t* __restrict__ dout,
                                                              int B, int S, int C,
                                                              const uint16_t* __restrict__ skip,
                                                              const uint16_t* __restrict__ y,
                                                              uint16_t* __restrict__ din) {
    const int P = C / 8;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * S * S * S * P) return;
    const int c = (int)(e % P) * 8;
    int64_t t = e / P;
    const int x = (int)(t % S);
    t /= S;
    const int yy = (int)(t % S);
    t /= S;
    const int z = (int)(t % S);
    const int64_t b = t / S;
    const int So = S / 2;
    const uint4 g = *reinterpret_cast<const uint4*>(
        dout + (((b * So + z / 2) * So + yy / 2) * So + x / 2) * C + c);
    const int64_t o0 = (((b * S + z) * S + yy) * S + x) * C + c;
    const uint4 sk = *reinterpret_cast<const uint4*>(skip + o0);
    const uint4 yv = *reinterpret_cast<const uint4*>(y + o0);
    const uint16_t* gh = reinterpret_cast<const uint16_t*>(&g);
    const uint16_t* sh = reinterpret_cast<const uint16_t*>(&sk);
    const uint16_t* yh = reinterpret_cast<const uint16_t*>(&yv);
    uint4 o;
    uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
    for (int j = 0; j < 8; j++) {
        float v = bf2f(f2bf(0.125f * bf2f(gh[j])));
        v += bf2f(sh[j]);
        oh[j] = f2bf(dact(v, yh[j]));
    }
    *reinterpret_cast<uint4*>(din + o0) = o;
}

__global__ void k_f32_to_bf16(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// ---------------------------------------------------------------------------
// Host entry points
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Per-channel statistics and affine maps (standardisation of network inputs
// and targets, and its inverse on predictions)
// ---------------------------------------------------------------------------
#define ST_BLOCKS 256
#define ST_MAXC 16
// Per-block FP64 partial sums of x and x^2 of channels [0, nc) over V rows of
// stride `stride`; part[b][2*nc].
__global__ __launch_bounds__(256) void k_chan_stats(const float* __restrict__ in, int stride, int nc,
                                                    int64_t V, double* __restrict__ part) {
    __shared__ double sh[4][2 * ST_MAXC];
    double s[2 * ST_MAXC];
    for (int c = 0; c < 2 * nc; c++) s[c] = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V;
         v += (int64_t)gridDim.x * blockDim.x) {
        for (int c = 0; c < nc; c++) {
            const double x = in[v * stride + c];
            s[c] += x;
            s[nc + c] += x * x;
        }
    }
    for (int c = 0; c < 2 * nc; c++) {
        const double t = wave_sum(s[c]);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][c] = t;
    }
    __syncthreads();
    if (threadIdx.x < 2 * nc) {
        const int c = threadIdx.x;
        part[(int64_t)blockIdx.x * 2 * nc + c] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
    }
}

// sums[c] += sum over blocks of part[b][c], in block order (deterministic).
__global__ void k_chan_stats_final(const double* __restrict__ part, int nb, int m,
                                   double* __restrict__ sums) {
    const int c = threadIdx.x;
    if (c >= m) return;
    double t = 0.0;
    for (int b = 0; b < nb; b++) t += part[(int64_t)b * m + c];
    sums[c] += t;
}

// out[v][c] = in[v][c] * scale[c] + shift[c] for c < nc, written as FP32 (row
// stride out_stride) and/or BF16 (row stride bf_stride, channels nc.. zero).
__global__ void k_chan_affine(const float* __restrict__ in, int in_stride, int nc, int64_t V,
                              const float* __restrict__ scale, const float* __restrict__ shift,
                              float* __restrict__ out, int out_stride, uint16_t* __restrict__ obf,
                              int bf_stride) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    float y[ST_MAXC];
    for (int c = 0; c < nc; c++) y[c] = fmaf(in[v * in_stride + c], scale[c], shift[c]);
    if (out)
        for (int c = 0; c < nc; c++) out[v * out_stride + c] = y[c];
    if (obf)
        for (int c = 0; c < bf_stride; c++) obf[v * bf_stride + c] = c < nc ? f2bf(y[c]) : (uint16_t)0;
}

// ---------------------------------------------------------------------------
// Symmetries of the cube (training-set augmentation)
// ---------------------------------------------------------------------------
// Sample b of in[B][S^3][C] (voxel order z-major, x fastest) is mapped by the
// cube symmetry sym[b] = perm * 8 + flips (perm in [0, 6) indexes the axis
// permutations, flip bit a reverses output axis a): output axis a takes input
// axis P[a], reversed when bit a is set.  The velocity channels vc .. vc + 2
// (vx, vy, vz), when vc >= 0, are permuted the same way and negated on the
// reversed axes, so a field that is a solution of the isotropic fluid
// equations stays one.
__constant__ int c_perm6[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

__global__ void k_cube_sym(const float* __restrict__ in, int S, int C, int vc,
                           const int32_t* __restrict__ sym, float* __restrict__ out) {
    const int b = blockIdx.y;
    const int64_t V = (int64_t)S * S * S;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int sy = sym[b];
    const int* P = c_perm6[(sy >> 3) % 6];
    const int fl = sy & 7;
    int o[3];
    o[0] = (int)(v % S);
    o[1] = (int)((v / S) % S);
    o[2] = (int)(v / ((int64_t)S * S));
    int q[3];
#pragma unroll
    for (int a = 0; a < 3; a++) q[P[a]] = (fl >> a & 1) ? S - 1 - o[a] : o[a];
    const int64_t src = ((int64_t)q[2] * S + q[1]) * S + q[0];
    const float* ip = in + ((int64_t)b * V + src) * C;
    float* op = out + ((int64_t)b * V + v) * C;
    for (int c = 0; c < C; c++) op[c] = ip[c];
    if (vc >= 0) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float w = ip[vc + P[a]];
            op[vc + a] = (fl >> a & 1) ? -w : w;
        }
    }
}

static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) l++;
    return l;
}
static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// kch: the channel count that forms the GEMM's K dimension with the taps (Cin
// for forward and weight gradient, Cout for the data gradient); it must be a
// power of two >= 8 so that a K slice splits into tap and channel by shifts.
static int check_conv(gx_ctx* ctx, int B, int S, int Cin, int Cout, int ksize, int kch) {
    if (B < 1 || S < 1 || Cin < 8 || Cin % 8 || Cout < 16 || Cout % 16 || (ksize != 3 && ksize != 1))
        return gx_fail(ctx, GX_EINVAL,
                       "conv3d: need B, S >= 1, Cin % 8 == 0, Cout % 16 == 0, ksize 1 or 3");
    if (!pow2(kch))
        return gx_fail(ctx, GX_EINVAL, "conv3d: the reduced channel count must be a power of two");
    if ((int64_t)B * S * S * S >= ((int64_t)1 << 31))
        return gx_fail(ctx, GX_EINVAL, "conv3d: B S^3 must stay below 2^31 voxels");
    return GX_OK;
}

template <int BN>
static void launch_brick(gx_ctx* ctx, dim3 grid, const uint16_t* in, const uint16_t* w,
                         const float* bias, const ConvGeom& g, int mode, const uint16_t* yref,
                         uint16_t* ob, float* of, const ConvSrc& src) {
    // chunk width: the largest of 32, 16, 8 dividing both sources' channel counts
    const int c2 = g.Cin - src.c1;
    auto fits = [&](int ck) { return g.Cin % ck == 0 && src.c1 % ck == 0 && c2 % ck == 0; };
    if (fits(32))
        hipLaunchKernelGGL((k_conv3d_brick<BN, 32>), grid, dim3(256), 0, ctx->stream, in, w, bias, g,
                           mode, yref, ob, of, src);
    else if (fits(16))
        hipLaunchKernelGGL((k_conv3d_brick<BN, 16>), grid, dim3(256), 0, ctx->stream, in, w, bias, g,
                           mode, yref, ob, of, src);
    else
        hipLaunchKernelGGL((k_conv3d_brick<BN, 8>), grid, dim3(256), 0, ctx->stream, in, w, bias, g,
                           mode, yref, ob, of, src);
}

static int launch_conv(gx_ctx* ctx, const uint16_t* in, const uint16_t* w, const float* bias,
                       const ConvGeom& g, int mode, const uint16_t* yref, uint16_t* ob,
                       float* of, ConvSrc src = ConvSrc{nullptr, -1, 0},
                       ConvAffine aff = ConvAffine{}) {
    if (src.c1 < 0) src.c1 = g.Cin;
    if (g.kvol == 27 && g.Cout % 32 == 0 && g.Cin % 8 == 0 && src.c1 % 8 == 0) {
        // weights staged in LDS: re-laid out chunk-major first
        const int64_t pieces = (int64_t)g.Cout * 27 * (g.Cin / 8);
        GX_TRY(gx_reserve(ctx, ctx->wrel, (size_t)pieces * 16));
        uint16_t* wr = (uint16_t*)ctx->wrel.p;
        hipLaunchKernelGGL(k_wrelayout, dim3(gx_blocks(pieces, 256)), dim3(256), 0, ctx->stream, w,
                           g.Cout, g.Cin, wr);
        const int S = g.S;
        const int64_t nb = (int64_t)g.B * ((S + SBZ - 1) / SBZ) * ((S + SBY - 1) / SBY) *
                           ((S + SBX - 1) / SBX);
        const int64_t nb4 = (int64_t)g.B * ((S + 3) / 4) * ((S + SBY - 1) / SBY) *
                            ((S + SBX - 1) / SBX);
        if (g.Cout % 64 == 0 && !src.pool)  // one z slice per wave (pooling needs z pairs)
            hipLaunchKernelGGL((k_conv3d_slab<64, 4>), dim3(xcd_grid(nb4), (unsigned)(g.Cout / 64)),
                               dim3(256), 0, ctx->stream, in, (const uint16_t*)wr, bias, g, mode,
                               yref, ob, of, src);
        else if (g.Cout % 64 == 0)
            hipLaunchKernelGGL((k_conv3d_slab<64, 8>), dim3(xcd_grid(nb), (unsigned)(g.Cout / 64)),
                               dim3(256), 0, ctx->stream, in, (const uint16_t*)wr, bias, g, mode,
                               yref, ob, of, src);
        else  // (one z slice per wave measured slower for 32 outputs)
            hipLaunchKernelGGL((k_conv3d_slab<32, 8>), dim3(xcd_grid(nb), (unsigned)(g.Cout / 32)),
                               dim3(256), 0, ctx->stream, in, (const uint16_t*)wr, bias, g, mode,
                               yref, ob, of, src);
        GX_LAUNCH_CHECK(ctx);
        return GX_OK;
    }
    if (g.kvol == 27) {
        const int S = g.S;
        const int64_t nb = (int64_t)g.B * ((S + BRZ - 1) / BRZ) * ((S + BRY - 1) / BRY) *
                           ((S + BRX - 1) / BRX);
        const dim3 grid((unsigned)nb, (unsigned)(g.Cout / (g.Cout % 64 == 0 ? 64 : g.Cout % 32 == 0 ? 32 : 16)));
        if (g.Cout % 64 == 0) launch_brick<64>(ctx, grid, in, w, bias, g, mode, yref, ob, of, src);
        else if (g.Cout % 32 == 0) launch_brick<32>(ctx, grid, in, w, bias, g, mode, yref, ob, of, src);
        else launch_brick<16>(ctx, grid, in, w, bias, g, mode, yref, ob, of, src);
        GX_LAUNCH_CHECK(ctx);
        return GX_OK;
    }
    const unsigned gx = (unsigned)((g.M + CV_BM - 1) / CV_BM);
    if (g.Cout % 64 == 0)
        hipLaunchKernelGGL(k_conv3d<64>, dim3(gx, g.Cout / 64), dim3(256), 0, ctx->stream, in, w,
                           bias, g, mode, yref, ob, of, aff);
    else if (g.Cout % 32 == 0)
        hipLaunchKernelGGL(k_conv3d<32>, dim3(gx, g.Cout / 32), dim3(256), 0, ctx->stream, in, w,
                           bias, g, mode, yref, ob, of, aff);
    else
        hipLaunchKernelGGL(k_conv3d<16>, dim3(gx, g.Cout / 16), dim3(256), 0, ctx->stream, in, w,
                           bias, g, mode, yref, ob, of, aff);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_conv3d_fwd(gx_ctx* ctx, const uint16_t* in, int B, int S, int Cin,
                             const uint16_t* w, const float* bias, int ksize, int Cout, int act,
                             uint16_t* out_bf16, float* out_f32) {
    if (!ctx || !in || !w || (!out_bf16 && !out_f32)) return GX_EINVAL;
    GX_TRY(check_conv(ctx, B, S, Cin, Cout, ksize, Cin));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int kv = ksize == 3 ? 27 : 1;
    ConvGeom g{B, S, Cin, Cout, kv, (int64_t)B * S * S * S, kv * Cin, ilog2(Cin)};
    return launch_conv(ctx, in, w, bias, g, act ? EP_LRELU : EP_NONE, nullptr, out_bf16, out_f32);
}

extern "C" int gx_conv_head(gx_ctx* ctx, const uint16_t* in, int B, int S, int Cin,
                            const uint16_t* w, const float* bias, int Cout, int nc,
                            const float* scale, const float* shift, float* out, int out_stride) {
    if (!ctx || !in || !w || !scale || !shift || !out || nc < 1 || nc > Cout || out_stride < nc)
        return GX_EINVAL;
    GX_TRY(check_conv(ctx, B, S, Cin, Cout, 1, Cin));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    ConvGeom g{B, S, Cin, Cout, 1, (int64_t)B * S * S * S, Cin, ilog2(Cin)};
    ConvAffine aff;
    aff.scale = scale;
    aff.shift = shift;
    aff.nc = nc;
    aff.stride = out_stride;
    return launch_conv(ctx, in, w, bias, g, EP_NONE, nullptr, nullptr, out, ConvSrc{nullptr, -1, 0},
                       aff);
}

extern "C" int gx_conv3d_fwd_pool(gx_ctx* ctx, const uint16_t* in, int B, int S, int Cin,
                                  const uint16_t* w, const float* bias, int Cout, int act,
                                  uint16_t* out_bf16, uint16_t* pool_bf16) {
    if (!ctx || !in || !w || !out_bf16 || !pool_bf16) return GX_EINVAL;
    GX_TRY(check_conv(ctx, B, S, Cin, Cout, 3, Cin));
    if (S % 2 || S < 2) return gx_fail(ctx, GX_EINVAL, "conv3d_fwd_pool: S must be even");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    ConvGeom g{B, S, Cin, Cout, 27, (int64_t)B * S * S * S, 27 * Cin, ilog2(Cin)};
    const int mode = act ? EP_LRELU : EP_NONE;
    if (Cout % 32 == 0 && Cin % 8 == 0) {  // slab kernel: pooled in its epilogue
        ConvSrc src{nullptr, Cin, 0};
        src.pool = pool_bf16;
        return launch_conv(ctx, in, w, bias, g, mode, nullptr, out_bf16, nullptr, src);
    }
    GX_TRY(launch_conv(ctx, in, w, bias, g, mode, nullptr, out_bf16, nullptr));
    const int64_t n = (int64_t)B * S * S * S * Cout / 8;
    hipLaunchKernelGGL(k_avgpool2, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream,
                       (const uint16_t*)out_bf16, B, S, Cout, pool_bf16);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_conv3d_fwd_fused(gx_ctx* ctx, const uint16_t* in, int c1, const uint16_t* in2,
                                   int upsample, int B, int S, int Cin, const uint16_t* w,
                                   const float* bias, int Cout, int act, uint16_t* out_bf16,
                                   float* out_f32) {
    if (!ctx || !in || !w || (!out_bf16 && !out_f32)) return GX_EINVAL;
    GX_TRY(check_conv(ctx, B, S, Cin, Cout, 3, Cin));
    if (in2 ? (c1 < 8 || c1 % 8 || c1 >= Cin) : (c1 != Cin))
        return gx_fail(ctx, GX_EINVAL, "conv3d_fwd_fused: c1 must split Cin in multiples of 8");
    if (upsample && (S % 2 || S < 2))
        return gx_fail(ctx, GX_EINVAL, "conv3d_fwd_fused: upsampling needs an even S");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    ConvGeom g{B, S, Cin, Cout, 27, (int64_t)B * S * S * S, 27 * Cin, ilog2(Cin)};
    return launch_conv(ctx, in, w, bias, g, act ? EP_LRELU : EP_NONE, nullptr, out_bf16, out_f32,
                       ConvSrc{in2, in2 ? c1 : Cin, upsample ? 1 : 0});
}

extern "C" int gx_conv3d_bwd_data(gx_ctx* ctx, const uint16_t* dout, int B, int S, int Cin,
                                  const uint16_t* w, int ksize, int Cout, const uint16_t* y_in,
                                  uint16_t* din) {
    if (!ctx || !dout || !w || !din) return GX_EINVAL;
    GX_TRY(check_conv(ctx, B, S, Cin, Cout, ksize, Cout));
    if (Cin % 16) return gx_fail(ctx, GX_EINVAL, "conv3d_bwd_data: Cin % 16 == 0 required");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int kv = ksize == 3 ? 27 : 1;
    const int64_t nw = (int64_t)Cout * Cin * kv;
    GX_TRY(gx_reserve(ctx, ctx->scan_tmp[2], nw * sizeof(uint16_t)));
    uint16_t* wf = (uint16_t*)ctx->scan_tmp[2].p;
    hipLaunchKernelGGL(k_wflip, dim3(gx_blocks(nw, 256)), dim3(256), 0, ctx->stream, w, Cout, Cin,
                       kv, wf);
    ConvGeom g{B, S, Cout, Cin, kv, (int64_t)B * S * S * S, kv * Cout, ilog2(Cout)};
    return launch_conv(ctx, dout, wf, nullptr, g, y_in ? EP_DACT : EP_NONE, y_in, din, nullptr);
}

// Sums the per-chunk partials (in chunk order; two ordered levels beyond 64
// chunks) into dw and the bias partials into dbias.
static int wgrad_reduce_chunks(gx_ctx* ctx, const float* part, const float* bpart, int64_t nw,
                               int64_t chunks, int Cout, float* dw, float* dbias) {
    if (chunks > 64) {
        const int ngr = (int)((chunks + 31) / 32);
        GX_TRY(gx_reserve(ctx, ctx->wpart2, (size_t)ngr * nw * sizeof(float)));
        float* p2 = (float*)ctx->wpart2.p;
        hipLaunchKernelGGL(k_wgrad_group_sum, dim3(gx_blocks(nw, 256), ngr), dim3(256), 0,
                           ctx->stream, part, nw, (int)chunks, 32, p2);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(gx_blocks(nw, 256)), dim3(256), 0, ctx->stream, p2,
                           nw, ngr, dw);
    } else {
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(gx_blocks(nw, 256)), dim3(256), 0, ctx->stream, part,
                           nw, (int)chunks, dw);
    }
    if (dbias)
        hipLaunchKernelGGL(k_bias_reduce, dim3(Cout), dim3(64), 0, ctx->stream, bpart, (int)chunks,
                           Cout, dbias);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// 3^3 weight gradient on 16^3, 32^3 and 64^3 grids with LDS-staged operands
// (k_wgrad_lds); xt, yt are the channel-major copies.
static int wgrad_staged(gx_ctx* ctx, const uint16_t* xt, const uint16_t* yt, const ConvGeom& g,
                        float* dw, float* dbias) {
    const int ncib = (g.Cin + 15) / 16, ncob = (g.Cout + 31) / 32;
    const int ntiles = (int)(g.M / 256);
    // runs of consecutive tiles per block: about GX_WG_BLOCKS blocks in all
    const int pairs = ncib * ncob;
    int tpb = std::max(1, (int)((int64_t)ntiles * pairs / GX_WG_BLOCKS));
    tpb = std::min(tpb, ntiles);
    const int64_t chunks = (ntiles + tpb - 1) / tpb;
    const int64_t nw = (int64_t)g.Cout * g.K;
    GX_TRY(gx_reserve(ctx, ctx->wpart, (size_t)(chunks * nw + chunks * g.Cout) * sizeof(float)));
    float* part = (float*)ctx->wpart.p;
    float* bpart = dbias ? part + chunks * nw : nullptr;
    const dim3 grid((unsigned)chunks, (unsigned)pairs);
    if (g.S == 64)
        hipLaunchKernelGGL(k_wgrad_lds<6>, grid, dim3(192), 0, ctx->stream, xt, yt, g.B, g.Cin,
                           g.Cout, tpb, part, bpart);
    else if (g.S == 32)
        hipLaunchKernelGGL(k_wgrad_lds<5>, grid, dim3(192), 0, ctx->stream, xt, yt, g.B, g.Cin,
                           g.Cout, tpb, part, bpart);
    else
        hipLaunchKernelGGL(k_wgrad_lds<4>, grid, dim3(192), 0, ctx->stream, xt, yt, g.B, g.Cin,
                           g.Cout, tpb, part, bpart);
    GX_LAUNCH_CHECK(ctx);
    return wgrad_reduce_chunks(ctx, part, bpart, nw, chunks, g.Cout, dw, dbias);
}

// Weight and bias gradients through channel-major copies (k_wgrad_cm): the
// voxel range is split into chunks so that the tasks fill the device, each
// chunk writes its partial gradient, and the partials are added in chunk order.
static int wgrad_cmajor(gx_ctx* ctx, const uint16_t* in, const uint16_t* in2, int c1, int up,
                        const uint16_t* dout, const ConvGeom& g, float* dw, float* dbias) {
    const int64_t V = (int64_t)g.S * g.S * g.S, M = g.M;
    const int lgS = ilog2(g.S);
    GX_TRY(gx_reserve(ctx, ctx->xcm, (size_t)M * g.Cin * sizeof(uint16_t)));
    GX_TRY(gx_reserve(ctx, ctx->ycm, (size_t)M * g.Cout * sizeof(uint16_t)));
    uint16_t* xt = (uint16_t*)ctx->xcm.p;
    uint16_t* yt = (uint16_t*)ctx->ycm.p;
    hipLaunchKernelGGL(k_to_cmajor, dim3((unsigned)(M / 64)), dim3(256), 0, ctx->stream, in, in2,
                       c1, up, lgS, V, g.Cin, xt);
    hipLaunchKernelGGL(k_to_cmajor, dim3((unsigned)(M / 64)), dim3(256), 0, ctx->stream, dout,
                       (const uint16_t*)nullptr, g.Cout, 0, lgS, V, g.Cout, yt);
    if (g.kvol == 27 && (g.S == 16 || g.S == 32 || g.S == 64))
        return wgrad_staged(ctx, xt, yt, g, dw, dbias);
    const int ndz = g.kvol == 27 ? 3 : 1;
    const int tasks = ((g.Cin + 15) / 16) * ndz * ((g.Cout + 31) / 32);
    const int ty = (tasks + 3) / 4;
    // chunks of whole 32-voxel steps, aiming at ~GX_WG_WAVES waves in all
    int64_t chunks = std::min<int64_t>(4096, std::max<int64_t>(1, (GX_WG_WAVES + tasks - 1) / tasks));
    int64_t mpc = (M + chunks - 1) / chunks;
    mpc = std::max<int64_t>(32, ((mpc + 31) / 32) * 32);
    chunks = (M + mpc - 1) / mpc;
    const int64_t nw = (int64_t)g.Cout * g.K;
    GX_TRY(gx_reserve(ctx, ctx->wpart, (size_t)(chunks * nw + chunks * g.Cout) * sizeof(float)));
    float* part = (float*)ctx->wpart.p;
    float* bpart = dbias ? part + chunks * nw : nullptr;
    const dim3 grid((unsigned)chunks, (unsigned)ty);
    if (g.kvol == 27)
        hipLaunchKernelGGL(k_wgrad_cm<3>, grid, dim3(256), 0, ctx->stream, xt, yt, g.B, lgS, g.Cin,
                           g.Cout, mpc, part, bpart);
    else
        hipLaunchKernelGGL(k_wgrad_cm<1>, grid, dim3(256), 0, ctx->stream, xt, yt, g.B, lgS, g.Cin,
                           g.Cout, mpc, part, bpart);
    return wgrad_reduce_chunks(ctx, part, bpart, nw, chunks, g.Cout, dw, dbias);
}

// Shapes of the weight gradient through channel-major copies (and of its
// fused-input form).
bool gx_wgrad_fused_ok(int S, int Cin, int Cout) {
    return pow2(S) && S >= 8 && Cin <= 256 && Cout <= 256 && Cin % 8 == 0 && Cout % 8 == 0;
}

extern "C" int gx_conv3d_bwd_weight_fused(gx_ctx* ctx, const uint16_t* in, int c1,
                                          const uint16_t* in2, int upsample,
                                          const uint16_t* dout, int B, int S, int Cin, int ksize,
                                          int Cout, float* dw, float* dbias) {
    if (!ctx || !in || !dout || !dw) return GX_EINVAL;
    GX_TRY(check_conv(ctx, B, S, Cin, Cout, ksize, Cin));
    if (!gx_wgrad_fused_ok(S, Cin, Cout))
        return gx_fail(ctx, GX_EINVAL, "conv3d_bwd_weight_fused: S a power of two >= 8, Cin and "
                                       "Cout <= 256, multiples of 8");
    if (in2 ? (c1 <= 0 || c1 >= Cin || c1 % 8 != 0) : c1 != Cin)
        return gx_fail(ctx, GX_EINVAL, "conv3d_bwd_weight_fused: bad channel split");
    if (upsample != 0 && upsample != 1) return gx_fail(ctx, GX_EINVAL, "bad upsample flag");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int kv = ksize == 3 ? 27 : 1;
    ConvGeom g{B, S, Cin, Cout, kv, (int64_t)B * S * S * S, kv * Cin, ilog2(Cin)};
    return wgrad_cmajor(ctx, in, in2, c1, upsample, dout, g, dw, dbias);
}

extern "C" int gx_conv3d_bwd_weight(gx_ctx* ctx, const uint16_t* in, const uint16_t* dout, int B,
                                    int S, int Cin, int ksize, int Cout, float* dw, float* dbias) {
    if (!ctx || !in || !dout || !dw) return GX_EINVAL;
    GX_TRY(check_conv(ctx, B, S, Cin, Cout, ksize, Cin));
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int kv = ksize == 3 ? 27 : 1;
    ConvGeom g{B, S, Cin, Cout, kv, (int64_t)B * S * S * S, kv * Cin, ilog2(Cin)};
    if (gx_wgrad_fused_ok(S, Cin, Cout))
        return wgrad_cmajor(ctx, in, nullptr, Cin, 0, dout, g, dw, dbias);
    const int kt = (g.K + 63) / 64;
    const int bn = Cout % 64 == 0 ? 64 : (Cout % 32 == 0 ? 32 : 16);
    const int nt = Cout / bn;
    // split the voxel reduction into at most 64 chunks, aiming at >= ~1024
    // blocks in all
    int64_t chunks = std::min<int64_t>(64, std::max<int64_t>(1, 1024 / (kt * nt)));
    int64_t mpb = (g.M + chunks - 1) / chunks;
    mpb = ((mpb + 31) / 32) * 32;
    if (mpb < 256) mpb = 256;
    chunks = (g.M + mpb - 1) / mpb;
    dim3 grid(kt, nt, (unsigned)chunks);
    const int64_t nw = (int64_t)Cout * g.K;
    GX_TRY(gx_reserve(ctx, ctx->wpart, (size_t)(chunks * nw + chunks * Cout) * sizeof(float)));
    float* part = (float*)ctx->wpart.p;
    float* bpart = dbias ? part + chunks * nw : nullptr;
    if (bn == 64)
        hipLaunchKernelGGL(k_conv3d_wgrad<64>, grid, dim3(256), 0, ctx->stream, in, dout, g, mpb, part,
                           bpart);
    else if (bn == 32)
        hipLaunchKernelGGL(k_conv3d_wgrad<32>, grid, dim3(256), 0, ctx->stream, in, dout, g, mpb, part,
                           bpart);
    else
        hipLaunchKernelGGL(k_conv3d_wgrad<16>, grid, dim3(256), 0, ctx->stream, in, dout, g, mpb, part,
                           bpart);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(gx_blocks(nw, 256)), dim3(256), 0, ctx->stream, part, nw,
                       (int)chunks, dw);
    if (dbias)
        hipLaunchKernelGGL(k_bias_reduce, dim3(Cout), dim3(64), 0, ctx->stream, bpart, (int)chunks,
                           Cout, dbias);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_avgpool2(gx_ctx* ctx, const uint16_t* in, int B, int S, int C, uint16_t* out,
                           int backward) {
    if (!ctx || !in || !out || S % 2 || S < 2 || C < 1 || B < 1) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    int64_t n = (int64_t)B * S * S * S * C;
    if (!backward) {
        n /= 8;
        hipLaunchKernelGGL(k_avgpool2, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, in, B, S,
                           C, out);
    } else {
        hipLaunchKernelGGL(k_avgpool2_bwd, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, in, B,
                           S, C, out);
    }
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_upsample2(gx_ctx* ctx, const uint16_t* in, int B, int S, int C, uint16_t* out,
                            int backward) {
    if (!ctx || !in || !out || S < 1 || C < 1 || B < 1) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    int64_t n = (int64_t)B * S * S * S * C;
    if (!backward) {
        n *= 8;
        hipLaunchKernelGGL(k_upsample2, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, in, B,
                           S, C, out);
    } else {
        hipLaunchKernelGGL(k_upsample2_bwd, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, in,
                           B, S, C, out);
    }
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_concat(gx_ctx* ctx, uint16_t* a, int Ca, uint16_t* b, int Cb, int64_t V,
                         uint16_t* out, int split) {
    if (!ctx || !a || !b || !out || Ca < 1 || Cb < 1 || V < 0) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t n = V * (Ca + Cb);
    hipLaunchKernelGGL(k_concat, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, a, Ca, b, Cb,
                       V, out, split);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_mse(gx_ctx* ctx, const float* pred, int Cp, const float* target, int nc,
                      int64_t V, uint16_t* dpred, double* loss) {
    if (!ctx || !pred || !target || nc < 1 || Cp < nc || V < 1 || !loss) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int nb = 512;
    GX_TRY(gx_reserve(ctx, ctx->partial, (nb + 8) * sizeof(double)));
    double* part = (double*)ctx->partial.p;
    const float scale = (float)(1.0 / ((double)V * nc));
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, ctx->stream, pred, Cp, target, nc, V, scale,
                       dpred, part);
    GX_LAUNCH_CHECK(ctx);
    double h[512];
    GX_HIP(ctx, hipMemcpyAsync(h, part, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (int i = 0; i < nb; i++) s += h[i];
    *loss = s / ((double)V * nc);
    return GX_OK;
}

extern "C" int gx_adam_step(gx_ctx* ctx, int64_t n, float* w, const float* grad, float* m, float* v,
                            double lr, double b1, double b2, double eps, int64_t t,
                            uint16_t* w_bf16) {
    if (!ctx || !w || !grad || !m || !v || n < 0 || t < 1) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    hipLaunchKernelGGL(k_adam, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, n, w, grad, m, v,
                       (float)lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2),
                       (float)eps, (float)c1, (float)c2, w_bf16);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_f32_to_bf16(gx_ctx* ctx, const float* x, int64_t n, uint16_t* y) {
    if (!ctx || !x || !y || n < 0) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, x, n, y);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_grad_combine(gx_ctx* ctx, int64_t n, const uint16_t* a, const uint16_t* b,
                               const uint16_t* y, uint16_t* out) {
    if (!ctx || !a || !out || n < 0) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_grad_combine, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, n, a, b, y,
                       out);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

// Fused backward steps of the network (used by gx_unet_backward; channel
// counts multiples of 8, 16-byte aligned rows).  Each equals the unfused
// sequence named in its kernel's comment, bit for bit.
int gx_split_dact(gx_ctx* ctx, const uint16_t* gc, int64_t V, int Ca, int Cb, const uint16_t* ya,
                  uint16_t* ga, uint16_t* gb) {
    if (!ctx || !gc || !ya || !ga || !gb || V < 0 || Ca < 8 || Cb < 8 || Ca % 8 || Cb % 8)
        return gx_fail(ctx, GX_EINVAL, "split_dact: bad arguments");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t n = V * ((Ca + Cb) / 8);
    hipLaunchKernelGGL(k_split_dact, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream, gc, V, Ca,
                       Cb, ya, ga, gb);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

int gx_upsample2_bwd_dact(gx_ctx* ctx, const uint16_t* dout, int B, int S, int C,
                          const uint16_t* y, uint16_t* din) {
    if (!ctx || !dout || !y || !din || B < 1 || S < 1 || C < 8 || C % 8)
        return gx_fail(ctx, GX_EINVAL, "upsample2_bwd_dact: bad arguments");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t n = (int64_t)B * S * S * S * (C / 8);
    hipLaunchKernelGGL(k_upsample2_bwd_dact, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream,
                       dout, B, S, C, y, din);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

int gx_avgpool2_bwd_combine(gx_ctx* ctx, const uint16_t* dout, int B, int S, int C,
                            const uint16_t* skip, const uint16_t* y, uint16_t* din) {
    if (!ctx || !dout || !skip || !y || !din || B < 1 || S < 2 || S % 2 || C < 8 || C % 8)
        return gx_fail(ctx, GX_EINVAL, "avgpool2_bwd_combine: bad arguments");
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t n = (int64_t)B * S * S * S * (C / 8);
    hipLaunchKernelGGL(k_avgpool2_bwd_combine, dim3(gx_blocks(n, 256)), dim3(256), 0, ctx->stream,
                       dout, B, S, C, skip, y, din);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_chan_stats(gx_ctx* ctx, int64_t V, const float* in, int stride, int nc,
                             double* sums) {
    if (!ctx || !in || !sums || V < 0 || nc < 1 || nc > ST_MAXC || stride < nc) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    GX_TRY(gx_reserve(ctx, ctx->partial, (size_t)ST_BLOCKS * 2 * nc * sizeof(double)));
    double* part = (double*)ctx->partial.p;
    hipLaunchKernelGGL(k_chan_stats, dim3(ST_BLOCKS), dim3(256), 0, ctx->stream, in, stride, nc, V,
                       part);
    GX_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_chan_stats_final, dim3(1), dim3(64), 0, ctx->stream, part, ST_BLOCKS,
                       2 * nc, sums);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_chan_affine(gx_ctx* ctx, int64_t V, const float* in, int in_stride, int nc,
                              const float* scale, const float* shift, float* out, int out_stride,
                              uint16_t* out_bf16, int bf_stride) {
    if (!ctx || !in || !scale || !shift || V < 0 || nc < 1 || nc > ST_MAXC || in_stride < nc ||
        (!out && !out_bf16) || (out && out_stride < nc) || (out_bf16 && bf_stride < nc) ||
        (out_bf16 && bf_stride > ST_MAXC * 4))
        return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_chan_affine, dim3(gx_blocks(V, 256)), dim3(256), 0, ctx->stream, in,
                       in_stride, nc, V, scale, shift, out, out_stride, out_bf16, bf_stride);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}

extern "C" int gx_cube_sym(gx_ctx* ctx, const float* in, int B, int S, int C, int vc,
                           const int32_t* sym, float* out) {
    if (!ctx || !in || !sym || !out || B < 1 || S < 1 || C < 1 || vc > C - 3 || in == out)
        return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t V = (int64_t)S * S * S;
    hipLaunchKernelGGL(k_cube_sym, dim3(gx_blocks(V, 256), B), dim3(256), 0, ctx->stream, in, S, C,
                       vc, sym, out);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}
