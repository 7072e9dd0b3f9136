// Surrogate-network kernels for gfx950 (C ABI in include/sg.h).
//
// The 3x3x3 convolution is an implicit GEMM: rows are output voxels, columns
// output channels, the reduction runs over the 27 taps times the input
// channels.  The matrix cores take 32 x 32 x 16 BF16 products
// (v_mfma_f32_32x32x16_bf16): lane l supplies 8 BF16 values of row l % 32
// at channels 8 (l / 32) .. +7 of a 16-channel slice, and 8 BF16 weights of
// column l % 32 at the same channels.  Channels-last activations and
// weights stored as [tap][c_out][c_in] make both operands single 16-byte
// reads.  Accumulation is FP32; the epilogue adds the bias, applies the
// activation and rounds to BF16 (or stores FP32).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "sg.h"

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __bf16 bf16;

thread_local char g_err[512] = "";

sg_status fail(sg_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

#define SG_LAUNCH_CHECK()                                                                            \
    do {                                                                                             \
        hipError_t e_ = hipGetLastError();                                                           \
        if (e_ != hipSuccess) return fail(SG_EHIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

constexpr int kThreads = 256;

__device__ inline float leaky(float v, float slope) { return v > 0.f ? v : slope * v; }

// ---- convolution forward, input staged in LDS ---------------------------------
// The same implicit GEMM with the input tile kept in LDS for all 27 taps.  A
// block owns a box of BD = 4 planes x BH = 4 TH rows x TW columns of one
// sample: 16 M-tiles of 32 voxels, each a TH x TW patch of a plane
// (TW = 32, 16 or 8 by the width, TH = 32 / TW).  Wave w computes the four
// tiles of plane w and NT x 32 output channels.  Per slice of 16 input
// channels the block stages the box with a one-voxel halo,
// (BD + 2)(BH + 2)(TW + 2) voxels of 16 channels at a 48-byte pitch (eight
// consecutive voxels then cover all LDS banks, so the 16-byte operand reads
// are conflict-free), then runs 27 taps x 4 tiles x NT MFMAs from it; the
// B operand of a tap (weights, the same for every block, so L2 hits) is
// loaded once per tap and shared by the four tiles.  Halo cells outside the
// volume hold zeros (the padding).
constexpr int kHaloPitch = 24;  // bf16 per staged voxel: 16 channels + 8 padding (48 B)

template <int TW>
struct HaloBox {
    static constexpr int TH = 32 / TW;
    static constexpr int BD = 4, BH = 4 * TH;
    static constexpr int HD = BD + 2, HH = BH + 2, HW = TW + 2;
    static constexpr int NV = HD * HH * HW;          // staged voxels
    static constexpr int ITEMS = (2 * NV + kThreads - 1) / kThreads;  // 16-byte loads per thread
};

// The input may come from two tensors: channels [0, ca) from xa, at half
// resolution (nearest 2x upsampling, up_a != 0) or full, and channels
// [ca, Ci) from xb at full resolution -- the decoder's concatenation of an
// upsampled tensor and a skip connection, read without forming it.  A single
// input is xa with ca = Ci, up_a = 0.  ca is a multiple of 16, so each
// staged channel slice comes from one tensor.
template <int NT, int TW, bool CAT>
__global__ __launch_bounds__(kThreads, 2) void k_conv3d_lds(const bf16 *__restrict__ xa, int ca, int up_a,
                                                            const bf16 *__restrict__ xb,
                                                            const bf16 *__restrict__ wt,
                                                            const float *__restrict__ bias,
                                                            void *__restrict__ y, int N, int D, int H, int W,
                                                            int Ci, int Co, int n_store, int act, float slope,
                                                            int y_f32, int nbd, int nbh, int nbw)
{
    using B = HaloBox<TW>;
    __shared__ __attribute__((aligned(16))) bf16 hs[B::NV * kHaloPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // boxes in storage order; consecutive boxes on one XCD (block i runs on XCD i mod 8)
    const int64_t nbox = (int64_t)N * nbd * nbh * nbw;
    int64_t bl = blockIdx.x;
    {
        const int64_t per = (nbox + 7) / 8;
        const int64_t rem = nbox % 8 == 0 ? 8 : nbox % 8;
        const int64_t xcd = bl % 8, k = bl / 8;
        // XCDs below rem hold `per` boxes, the others per - 1
        bl = xcd < rem ? xcd * per + k : rem * per + (xcd - rem) * (per - 1) + k;
    }
    int64_t t = bl;
    const int bw = (int)(t % nbw);
    t /= nbw;
    const int bh = (int)(t % nbh);
    t /= nbh;
    const int bd = (int)(t % nbd);
    const int n = (int)(t / nbd);
    const int d0 = bd * B::BD, h0 = bh * B::BH, w0 = bw * TW;
    const int col0 = blockIdx.y * NT * 32;
    const int lr = lane & 31, kh = (lane >> 5) * 8;
    const int th = lr / TW, tw = lr % TW;

    f32x16 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j)
            for (int r = 0; r < 16; ++r) acc[m][j][r] = 0.f;

    // The box and its halo for the channel slice c0, one 16-byte load per item
    // (zeros outside the volume), into registers.
    auto load_slice = [&](int c0, bf16x8 (&tmp)[B::ITEMS]) {
        // the slice's tensor: its base, channel count and resolution shift
        // (CAT); a single input is xa with Ci channels at full resolution
        const bool from_a = !CAT || c0 < ca;
        const bf16 *base = from_a ? xa + c0 : xb + (c0 - ca);
        const int64_t cst = CAT ? (from_a ? ca : Ci - ca) : Ci;
        const int sh = CAT && from_a && up_a ? 1 : 0;
        const int Ds = D >> sh, Hs = H >> sh, Ws = W >> sh;
#pragma unroll
        for (int i = 0; i < B::ITEMS; ++i) {
            const int item = threadIdx.x + i * kThreads;
            bf16x8 v = {};
            if (item < 2 * B::NV) {
                const int half = item & 1, hv = item >> 1;
                const int hw = hv % B::HW, hh = (hv / B::HW) % B::HH, hd = hv / (B::HW * B::HH);
                const int dd = d0 - 1 + hd, yy = h0 - 1 + hh, xx = w0 - 1 + hw;
                if (dd >= 0 && dd < D && yy >= 0 && yy < H && xx >= 0 && xx < W) {
                    const int64_t vox = (((int64_t)n * Ds + (dd >> sh)) * Hs + (yy >> sh)) * Ws + (xx >> sh);
                    v = *reinterpret_cast<const bf16x8 *>(base + vox * cst + half * 8);
                }
            }
            tmp[i] = v;
        }
    };
    auto store_slice = [&](const bf16x8 (&tmp)[B::ITEMS]) {
#pragma unroll
        for (int i = 0; i < B::ITEMS; ++i) {
            const int item = threadIdx.x + i * kThreads;
            if (item < 2 * B::NV)
                *reinterpret_cast<bf16x8 *>(hs + (item >> 1) * kHaloPitch + (item & 1) * 8) = tmp[i];
        }
    };
    // 27 taps x 4 tiles x NT products of one slice from the staged box
    auto taps = [&](int c0) {
        const bf16 *wp = wt + ((int64_t)col0 + lr) * Ci + c0 + kh;
#pragma unroll 3
        for (int tap = 0; tap < 27; ++tap) {
            const int a = tap / 9, b = (tap / 3) % 3, c = tap % 3;  // offsets + 1
            bf16x8 bv[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j)
                bv[j] = *reinterpret_cast<const bf16x8 *>(wp + ((int64_t)tap * Co + j * 32) * Ci);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int hv = ((wave + a) * B::HH + m * B::TH + th + b) * B::HW + tw + c;
                const bf16x8 av = *reinterpret_cast<const bf16x8 *>(hs + hv * kHaloPitch + kh);
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    acc[m][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv[j], acc[m][j], 0, 0, 0);
            }
        }
    };

    if constexpr (NT == 1) {
        // Registers allow the next slice's loads to be in flight during this
        // slice's products (the NT = 2 kernel is at 223 VGPRs without them).
        bf16x8 tmp[B::ITEMS];
        load_slice(0, tmp);
        for (int c0 = 0; c0 < Ci; c0 += 16) {
            __syncthreads();  // the previous slice's operand reads are done
            store_slice(tmp);
            __syncthreads();
            if (c0 + 16 < Ci) load_slice(c0 + 16, tmp);
            taps(c0);
        }
    } else {
        for (int c0 = 0; c0 < Ci; c0 += 16) {
            // stage the box and its halo: all loads first, then all LDS stores
            bf16x8 tmp[B::ITEMS];
            load_slice(c0, tmp);
            __syncthreads();  // the previous slice's operand reads are done
            store_slice(tmp);
            __syncthreads();
            taps(c0);
        }
    }
    // D layout of the 32x32 tile: column l % 32, row 8 (r/4) + 4 (l/32) + r % 4
    const int dv = d0 + wave;
    if (dv >= D) return;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int col = col0 + j * 32 + lr;
        if (col >= n_store) continue;
        const float bc = bias ? bias[col] : 0.f;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int hv = h0 + m * B::TH + row / TW, wv = w0 + row % TW;
                if (hv >= H || wv >= W) continue;
                const int64_t mv = (((int64_t)n * D + dv) * H + hv) * W + wv;
                float v = acc[m][j][r] + bc;
                if (act) v = leaky(v, slope);
                if (y_f32)
                    reinterpret_cast<float *>(y)[mv * n_store + col] = v;
                else
                    reinterpret_cast<bf16 *>(y)[mv * n_store + col] = (bf16)v;
            }
        }
    }
}

__global__ void k_weight_mirror(const bf16 *__restrict__ wt, int Co, int Ci, bf16 *__restrict__ wm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)27 * Co * Ci;
    if (i >= total) return;
    const int ci = (int)(i % Ci);
    const int co = (int)((i / Ci) % Co);
    const int t = (int)(i / ((int64_t)Ci * Co));
    wm[((int64_t)(26 - t) * Ci + ci) * Co + co] = wt[i];
}

// ---- convolution weight gradient, group-major operands ------------------------------
// dw[t][co][ci] = sum_v dy[v][co] x[v + off(t)][ci] is, per tap, a GEMM whose
// reduction runs over the voxels.  The matrix-core operands need 8
// consecutive voxels of one channel per lane, so x and dy are first copied
// "group-major": each W row (rows r = (n D + d) H + h) is cut into groups of
// 8 voxels, padded with zeros to Wp = a multiple of 16, and a group stores
// all channels' 8-voxel vectors one after another,
//   xt[((r ng + g) C + c) 8 + e] = x[r][8 g + e][c],  ng = Wp / 8.
// Every operand is then one aligned 16-byte load, a wave's 64 loads cover two
// contiguous 512-byte runs (32 channels of two groups), and the w offsets -1
// and +1 of a tap are joined from the neighbouring groups by byte alignment.
// Three one-wave blocks own a 32 x 32 (co, ci) tile and a chunk of 16-voxel
// steps; wave a holds the nine taps of d offset a - 1 in registers and walks
// the chunk: per step one dy operand and, per h offset, one x group with the
// neighbouring dwords serve three taps; along h the three x rows slide, so a
// step loads one of them (see the kernel).  Block sums go to
// partial[chunk][t][co][ci] (every entry written), added over chunks in a
// fixed order afterwards.
constexpr int kBwStep = 16;          // voxels per matrix-core K step
constexpr int kBwThreads = 64;       // one wave per block (block to chunk, d offset and tile: see the kernel)
constexpr int kBw2TargetBlocks = 1024;
constexpr int kBwReduceGroup = 32;   // chunks per group of the two-level chunk sum

// xt[((r ng + g) C + c) 8 + e] = x[r][8 g + e][c] for 8 g + e < W, 0 up to the
// padded row length (one thread per row, group and channel: consecutive
// threads take consecutive channels, so reads and 16-byte writes are
// contiguous across a wave)
__global__ void k_to_group_major(const bf16 *__restrict__ x, int64_t rows, int W, int ng, int C,
                                 bf16 *__restrict__ xt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = rows * ng * C;
    if (i >= total) return;
    const int c = (int)(i % C);
    const int64_t t = i / C;  // r ng + g
    const int g = (int)(t % ng);
    const int64_t r = t / ng;
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int w = g * 8 + e;
        v[e] = w < W ? x[(r * W + w) * C + c] : (bf16)0.f;
    }
    *reinterpret_cast<bf16x8 *>(xt + i * 8) = v;
}

typedef __attribute__((ext_vector_type(4))) unsigned u32x4;

// The 8 voxels starting one before (S = -1) or after (S = +1) the aligned
// group `cur`; nb is the neighbouring dword: the last two voxels of the
// group before (S = -1) or the first two of the group after (S = +1).
template <int S>
__device__ inline bf16x8 shift_group(const bf16x8 &cur, unsigned nb)
{
    const u32x4 c = __builtin_bit_cast(u32x4, cur);
    u32x4 r;
    if constexpr (S > 0) {
        r[0] = __builtin_amdgcn_alignbyte(c[1], c[0], 2);
        r[1] = __builtin_amdgcn_alignbyte(c[2], c[1], 2);
        r[2] = __builtin_amdgcn_alignbyte(c[3], c[2], 2);
        r[3] = __builtin_amdgcn_alignbyte(nb, c[3], 2);
    } else {
        r[0] = __builtin_amdgcn_alignbyte(c[0], nb, 2);
        r[1] = __builtin_amdgcn_alignbyte(c[1], c[0], 2);
        r[2] = __builtin_amdgcn_alignbyte(c[2], c[1], 2);
        r[3] = __builtin_amdgcn_alignbyte(c[3], c[2], 2);
    }
    return __builtin_bit_cast(bf16x8, r);
}

// One x row of the wave's channel and group: the aligned group and the
// neighbouring dwords for the w offsets -1 and +1 (zeros outside the volume).
struct XRow {
    bf16x8 cur;
    unsigned prev, next;
};

__device__ inline XRow load_xrow(const bf16 *xc, int64_t xrow, int g, int ng, int64_t xgrp, bool ok)
{
    XRow r{{}, 0u, 0u};
    if (ok) {
        const bf16 *xg = xc + (xrow * ng + g) * xgrp;
        r.cur = *reinterpret_cast<const bf16x8 *>(xg);
        if (g > 0) r.prev = *reinterpret_cast<const unsigned *>(xg - xgrp + 6);
        if (g + 1 < ng) r.next = *reinterpret_cast<const unsigned *>(xg + xgrp);
    }
    return r;
}

__device__ inline void bw_taps(const bf16x8 &av, const XRow &x, f32x16 &am, f32x16 &a0, f32x16 &ap)
{
    const bf16x8 bm = shift_group<-1>(x.cur, x.prev), bp = shift_group<1>(x.cur, x.next);
    am = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bm, am, 0, 0, 0);
    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, x.cur, a0, 0, 0, 0);
    ap = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bp, ap, 0, 0, 0);
}

// Steps are ordered by the 16-voxel column ws first, then by row
// r = (n D + d) H + h, h fastest: s = ws R + r.  Along a run of consecutive h
// a wave's three x rows (h - 1, h, h + 1 at its d offset) slide by one row
// per step, so each step loads one new x row and one dy operand, and the
// next step's loads are issued before this step's products.
// Two waves per SIMD: the accumulators then live in ordinary VGPRs (about 200, no
// spills), where the default allocation took 171 VGPRs plus 144 AGPRs and
// left one wave per SIMD.
__global__ __launch_bounds__(kBwThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_conv3d_bwd_weight_gm(
    const bf16 *__restrict__ xt, const bf16 *__restrict__ dyt, int N, int D, int H, int ng, int Ci, int Co,
    int64_t steps, int64_t per, int nchunks, float *__restrict__ partial)
{
    // Block b runs on XCD b mod 8.  Each XCD takes a contiguous eighth of the
    // chunks (nchunks is a multiple of 8) and runs, per chunk, the three d
    // offsets of every (co, ci) tile back to back, so the x and dy rows of a
    // chunk are read into that XCD's L2 once for all of them.
    const int tco = Co / 32, tiles = tco * ((Ci + 31) / 32);
    const int64_t k = blockIdx.x / 8;
    const int tile = (int)(k % tiles);
    const int a = (int)((k / tiles) % 3);  // a = d offset + 1
    const int chunk = (int)(blockIdx.x % 8) * (nchunks / 8) + (int)(k / (3 * tiles));
    const int co0 = (tile % tco) * 32, ci0 = (tile / tco) * 32;
    const int lane = threadIdx.x;
    const int64_t R = (int64_t)N * D * H;
    const int lr = lane & 31, half = lane >> 5;
    const bool ci_ok = ci0 + lr < Ci;
    // element offsets of this lane's channel; group g of row r is (r ng + g) C channels further
    const bf16 *dyc = dyt + (int64_t)(co0 + lr) * 8;
    const bf16 *xc = xt + (int64_t)(ci_ok ? ci0 + lr : 0) * 8;
    const int64_t xgrp = (int64_t)Ci * 8, dgrp = (int64_t)Co * 8;  // elements per group
    f32x16 acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k)
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
    const int64_t sbeg = (int64_t)chunk * per;
    const int64_t send = sbeg + per < steps ? sbeg + per : steps;
    for (int64_t s = sbeg; s < send;) {
        const int g = (int)(s / R) * 2 + half;  // this lane's group of 8 voxels
        const int64_t row = s % R;
        const int h = (int)(row % H);
        const int d = (int)((row / H) % D);
        const int run = (int)(send - s < (int64_t)(H - h) ? send - s : (int64_t)(H - h));
        const bool dok = d + a - 1 >= 0 && d + a - 1 < D && ci_ok;
        const int64_t xr = row + (int64_t)(a - 1) * H;  // x row at (d + a - 1, h)
        XRow r0 = load_xrow(xc, xr - 1, g, ng, xgrp, dok && h >= 1);
        XRow r1 = load_xrow(xc, xr, g, ng, xgrp, dok);
        XRow r2 = load_xrow(xc, xr + 1, g, ng, xgrp, dok && h + 1 < H);
        bf16x8 av = *reinterpret_cast<const bf16x8 *>(dyc + (row * ng + g) * dgrp);
        for (int k = 0; k < run; ++k) {
            XRow r3{{}, 0u, 0u};
            bf16x8 an = {};
            if (k + 1 < run) {
                r3 = load_xrow(xc, xr + k + 2, g, ng, xgrp, dok && h + k + 2 < H);
                an = *reinterpret_cast<const bf16x8 *>(dyc + ((row + k + 1) * ng + g) * dgrp);
            }
            bw_taps(av, r0, acc[0], acc[1], acc[2]);
            bw_taps(av, r1, acc[3], acc[4], acc[5]);
            bw_taps(av, r2, acc[6], acc[7], acc[8]);
            r0 = r1;
            r1 = r2;
            r2 = r3;
            av = an;
        }
        s += run;
    }
    // D layout of the 32x32 tile: column l % 32 (ci), row 8 (r/4) + 4 (l/32) + r % 4 (co)
    if (!ci_ok) return;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int t = a * 9 + k;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int rowc = 8 * (r >> 2) + 4 * half + (r & 3);
            partial[(((int64_t)chunk * 27 + t) * Co + co0 + rowc) * Ci + ci0 + lr] = acc[k][r];
        }
    }
}

// db[co] = sum of dyt over all groups of channel co (padding zeros add
// nothing): one block per chunk of groups and channel, fixed order
__global__ __launch_bounds__(kThreads) void k_bias_grad_gm(const bf16 *__restrict__ dyt, int64_t groups, int Co,
                                                           int64_t per, float *__restrict__ partial)
{
    __shared__ float s[kThreads];
    const int chunk = blockIdx.x, co = blockIdx.y;
    const int64_t beg = (int64_t)chunk * per;
    const int64_t end = beg + per < groups ? beg + per : groups;
    float acc = 0.f;
    for (int64_t i = beg + threadIdx.x; i < end; i += kThreads) {
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(dyt + (i * Co + co) * 8);
#pragma unroll
        for (int e = 0; e < 8; ++e) acc += (float)v[e];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = kThreads / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)chunk * Co + co] = s[0];
}

__global__ void k_reduce_partials(const float *__restrict__ partial, int nchunk, int64_t stride,
                                  float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= stride) return;
    float s = 0.f;
    for (int k = 0; k < nchunk; ++k) s += partial[(int64_t)k * stride + i];
    out[i] = s;
}

// First level of a two-level fixed-order sum over chunks: group blockIdx.y
// adds chunks [g per, (g + 1) per) into out[g][i] (one thread per entry and
// group, so long sums are spread over many more threads than entries).
__global__ void k_reduce_partials_grouped(const float *__restrict__ partial, int nchunk, int per, int64_t stride,
                                          float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= stride) return;
    const int g = blockIdx.y;
    const int k1 = (g + 1) * per < nchunk ? (g + 1) * per : nchunk;
    float s = 0.f;
    for (int k = g * per; k < k1; ++k) s += partial[(int64_t)k * stride + i];
    out[(int64_t)g * stride + i] = s;
}

// ---- elementwise and resampling ----------------------------------------------------
__global__ void k_leaky_bwd(const bf16 *__restrict__ y, const bf16 *__restrict__ dy, bf16 *__restrict__ dp,
                            int64_t count, float slope)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float g = (float)dy[i];
    dp[i] = (bf16)((float)y[i] > 0.f ? g : slope * g);
}

__global__ void k_pool2_fwd(const bf16 *__restrict__ x, int N, int D, int H, int W, int C, bf16 *__restrict__ y)
{
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2;
    const int64_t total = (int64_t)N * D2 * H2 * W2 * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i % C);
    int64_t v = i / C;
    const int w = (int)(v % W2);
    v /= W2;
    const int h = (int)(v % H2);
    v /= H2;
    const int d = (int)(v % D2);
    const int n = (int)(v / D2);
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e)
                s += (float)x[((((int64_t)n * D + 2 * d + a) * H + 2 * h + b) * W + 2 * w + e) * C + c];
    y[i] = (bf16)(s * 0.125f);
}

// dx[fine] = dy[coarse] / 8 (D, H, W of the fine tensor)
__global__ void k_pool2_bwd(const bf16 *__restrict__ dy, int N, int D, int H, int W, int C, bf16 *__restrict__ dx)
{
    const int64_t total = (int64_t)N * D * H * W * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i % C);
    int64_t v = i / C;
    const int w = (int)(v % W);
    v /= W;
    const int h = (int)(v % H);
    v /= H;
    const int d = (int)(v % D);
    const int n = (int)(v / D);
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2;
    dx[i] = (bf16)((float)dy[((((int64_t)n * D2 + d / 2) * H2 + h / 2) * W2 + w / 2) * C + c] * 0.125f);
}

// y[fine] = x[coarse] (D, H, W of the coarse tensor)
__global__ void k_up2_fwd(const bf16 *__restrict__ x, int N, int D, int H, int W, int C, bf16 *__restrict__ y)
{
    const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W;
    const int64_t total = (int64_t)N * D2 * H2 * W2 * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i % C);
    int64_t v = i / C;
    const int w = (int)(v % W2);
    v /= W2;
    const int h = (int)(v % H2);
    v /= H2;
    const int d = (int)(v % D2);
    const int n = (int)(v / D2);
    y[i] = x[((((int64_t)n * D + d / 2) * H + h / 2) * W + w / 2) * C + c];
}

// dx[coarse] = sum of the 8 fine dy (D, H, W of the coarse tensor)
__global__ void k_up2_bwd(const bf16 *__restrict__ dy, int N, int D, int H, int W, int C, bf16 *__restrict__ dx)
{
    const int64_t total = (int64_t)N * D * H * W * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i % C);
    int64_t v = i / C;
    const int w = (int)(v % W);
    v /= W;
    const int h = (int)(v % H);
    v /= H;
    const int d = (int)(v % D);
    const int n = (int)(v / D);
    const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W;
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e)
                s += (float)dy[((((int64_t)n * D2 + 2 * d + a) * H2 + 2 * h + b) * W2 + 2 * w + e) * C + c];
    dx[i] = (bf16)s;
}

__global__ void k_concat(const bf16 *__restrict__ a, int ca, const bf16 *__restrict__ b, int cb, int64_t V,
                         bf16 *__restrict__ y)
{
    const int cc = ca + cb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * cc) return;
    const int64_t v = i / cc;
    const int c = (int)(i % cc);
    y[i] = c < ca ? a[v * ca + c] : b[v * cb + (c - ca)];
}

__global__ void k_split(const bf16 *__restrict__ y, int ca, int cb, int64_t V, bf16 *__restrict__ a,
                        bf16 *__restrict__ b)
{
    const int cc = ca + cb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * cc) return;
    const int64_t v = i / cc;
    const int c = (int)(i % cc);
    if (c < ca) {
        if (a) a[v * ca + c] = y[i];
    } else {
        if (b) b[v * cb + (c - ca)] = y[i];
    }
}

// ---- the same elementwise and resampling kernels on groups of 8 channels ------------
// One thread per voxel and group of 8 channels (16-byte loads and stores),
// for channel counts that are multiples of 8 and 16-byte aligned tensors;
// per element the arithmetic and its order are those of the kernels above.
struct Vox {
    int n, d, h, w;
};

__device__ inline Vox vox_of(int64_t v, int D, int H, int W)
{
    Vox r;
    r.w = (int)(v % W);
    v /= W;
    r.h = (int)(v % H);
    v /= H;
    r.d = (int)(v % D);
    r.n = (int)(v / D);
    return r;
}

__global__ void k_pool2_fwd8(const bf16x8 *__restrict__ x, int N, int D, int H, int W, int C8, bf16x8 *__restrict__ y)
{
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * D2 * H2 * W2 * C8) return;
    const int g = (int)(i % C8);
    const Vox o = vox_of(i / C8, D2, H2, W2);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) {
                const bf16x8 v = x[((((int64_t)o.n * D + 2 * o.d + a) * H + 2 * o.h + b) * W + 2 * o.w + e) * C8 + g];
#pragma unroll
                for (int k = 0; k < 8; ++k) s[k] += (float)v[k];
            }
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (bf16)(s[k] * 0.125f);
    y[i] = r;
}

__global__ void k_pool2_bwd8(const bf16x8 *__restrict__ dy, int N, int D, int H, int W, int C8, bf16x8 *__restrict__ dx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * D * H * W * C8) return;
    const int g = (int)(i % C8);
    const Vox o = vox_of(i / C8, D, H, W);
    const bf16x8 v = dy[((((int64_t)o.n * (D / 2) + o.d / 2) * (H / 2) + o.h / 2) * (W / 2) + o.w / 2) * C8 + g];
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (bf16)((float)v[k] * 0.125f);
    dx[i] = r;
}

__global__ void k_up2_fwd8(const bf16x8 *__restrict__ x, int N, int D, int H, int W, int C8, bf16x8 *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * 8 * D * H * W * C8) return;
    const int g = (int)(i % C8);
    const Vox o = vox_of(i / C8, 2 * D, 2 * H, 2 * W);
    y[i] = x[((((int64_t)o.n * D + o.d / 2) * H + o.h / 2) * W + o.w / 2) * C8 + g];
}

__global__ void k_up2_bwd8(const bf16x8 *__restrict__ dy, int N, int D, int H, int W, int C8, bf16x8 *__restrict__ dx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * D * H * W * C8) return;
    const int g = (int)(i % C8);
    const Vox o = vox_of(i / C8, D, H, W);
    const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) {
                const bf16x8 v = dy[((((int64_t)o.n * D2 + 2 * o.d + a) * H2 + 2 * o.h + b) * W2 + 2 * o.w + e) * C8 + g];
#pragma unroll
                for (int k = 0; k < 8; ++k) s[k] += (float)v[k];
            }
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (bf16)s[k];
    dx[i] = r;
}

__global__ void k_concat8(const bf16x8 *__restrict__ a, int ca8, const bf16x8 *__restrict__ b, int cb8, int64_t V,
                          bf16x8 *__restrict__ y)
{
    const int cc = ca8 + cb8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * cc) return;
    const int64_t v = i / cc;
    const int c = (int)(i % cc);
    y[i] = c < ca8 ? a[v * ca8 + c] : b[v * cb8 + (c - ca8)];
}

__global__ void k_split8(const bf16x8 *__restrict__ y, int ca8, int cb8, int64_t V, bf16x8 *__restrict__ a,
                         bf16x8 *__restrict__ b)
{
    const int cc = ca8 + cb8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * cc) return;
    const int64_t v = i / cc;
    const int c = (int)(i % cc);
    if (c < ca8) {
        if (a) a[v * ca8 + c] = y[i];
    } else {
        if (b) b[v * cb8 + (c - ca8)] = y[i];
    }
}

__global__ void k_add8(const bf16x8 *__restrict__ a, const bf16x8 *__restrict__ b, bf16x8 *__restrict__ y, int64_t n8)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const bf16x8 x = a[i], z = b[i];
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (bf16)((float)x[k] + (float)z[k]);
    y[i] = r;
}

__global__ void k_leaky_bwd8(const bf16x8 *__restrict__ y, const bf16x8 *__restrict__ dy, bf16x8 *__restrict__ dp,
                             int64_t n8, float slope)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const bf16x8 yv = y[i], g = dy[i];
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float gk = (float)g[k];
        r[k] = (bf16)((float)yv[k] > 0.f ? gk : slope * gk);
    }
    dp[i] = r;
}

// MSE: per-block partial sums (fixed order), second pass sums them
constexpr int kMseBlocks = 1024;
__global__ __launch_bounds__(kThreads) void k_mse1(const float *__restrict__ p, const float *__restrict__ t,
                                                   int64_t count, bf16 *__restrict__ g, float *__restrict__ part)
{
    __shared__ float s[kThreads];
    float acc = 0.f;
    const float scale = 2.0f / (float)count;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += (int64_t)kMseBlocks * kThreads) {
        const float d = p[i] - t[i];
        acc += d * d;
        g[i] = (bf16)(scale * d);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = kThreads / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kThreads) void k_mse2(const float *__restrict__ part, int64_t count,
                                                   float *__restrict__ loss)
{
    __shared__ float s[kThreads];
    float acc = 0.f;
    for (int i = threadIdx.x; i < kMseBlocks; i += kThreads) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = kThreads / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = s[0] / (float)count;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, bf16 *__restrict__ wt, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (wt) wt[i] = (bf16)pi;
}

__global__ void k_to_bf16(const float *__restrict__ x, bf16 *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (bf16)x[i];
}

__global__ void k_to_f32(const bf16 *__restrict__ x, float *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

__global__ void k_add(const bf16 *__restrict__ a, const bf16 *__restrict__ b, bf16 *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (bf16)((float)a[i] + (float)b[i]);
}

struct Box {
    int x0, y0, z0, bx, by, bz;
};

__device__ inline int64_t box_cell(const Box &b, int64_t v, int nx, int ny, int nz, int &yy)
{
    const int x = (int)(v % b.bx);
    const int64_t t = v / b.bx;
    const int y = (int)(t % b.by);
    const int z = (int)(t / b.by);
    const int gx = ((b.x0 + x) % nx + nx) % nx;
    const int gz = ((b.z0 + z) % nz + nz) % nz;
    yy = b.y0 + y;
    return (int64_t)gx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * gz);
}

__global__ void k_fields_to_input(const float *__restrict__ phi, const float *__restrict__ u,
                                  const float *__restrict__ p, int nx, int ny, int nz, Box b, float s0, float s1,
                                  float s2, float s3, float s4, int c_in, bf16 *__restrict__ x,
                                  float *__restrict__ state)
{
    const int64_t V = (int64_t)b.bx * b.by * b.bz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    int yy;
    const int64_t c = box_cell(b, v, nx, ny, nz, yy);
    const int64_t N = (int64_t)nx * ny * nz;
    const float f[5] = {phi[c], u[c], u[N + c], u[2 * N + c], p[c]};
    const float sc[5] = {s0, s1, s2, s3, s4};
    for (int k = 0; k < c_in; ++k) x[v * c_in + k] = (bf16)(k < 5 ? f[k] / sc[k] : 0.f);
    if (state)
        for (int k = 0; k < 5; ++k) state[v * 5 + k] = f[k];
}

__global__ void k_state_to_input(const float *__restrict__ s, int64_t V, float q0, float q1, float q2, float q3,
                                 float q4, int c_in, bf16 *__restrict__ x)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float sc[5] = {q0, q1, q2, q3, q4};
    for (int k = 0; k < c_in; ++k) x[v * c_in + k] = (bf16)(k < 5 ? s[v * 5 + k] / sc[k] : 0.f);
}

__global__ void k_make_target(const float *__restrict__ s0, const float *__restrict__ s1, int64_t V, float q0,
                              float q1, float q2, float q3, float q4, int c_out, float *__restrict__ t)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float sc[5] = {q0, q1, q2, q3, q4};
    for (int k = 0; k < c_out; ++k) t[v * c_out + k] = k < 5 ? (s1[v * 5 + k] - s0[v * 5 + k]) / sc[k] : 0.f;
}

__global__ void k_apply_prediction(const float *__restrict__ out, int c_out, float q0, float q1, float q2,
                                   float q3, float q4, const float *__restrict__ base, float *__restrict__ phi,
                                   float *__restrict__ u, float *__restrict__ p, int nx, int ny, int nz, Box b,
                                   int walls, float pmin, float pmax, int flags)
{
    const int64_t V = (int64_t)b.bx * b.by * b.bz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    int yy;
    const int64_t c = box_cell(b, v, nx, ny, nz, yy);
    if (walls && (yy == 0 || yy == ny - 1)) return;
    const int64_t N = (int64_t)nx * ny * nz;
    const float *o = out + v * c_out;
    const float f0 = base ? base[v * 5 + 0] : phi[c];
    const float f1 = base ? base[v * 5 + 1] : u[c];
    const float f2 = base ? base[v * 5 + 2] : u[N + c];
    const float f3 = base ? base[v * 5 + 3] : u[2 * N + c];
    const float f4 = base ? base[v * 5 + 4] : p[c];
    // flags & 1: velocity increments weighted by the heavy-phase fraction q
    // of the base phi (the light phase carries no momentum to speak of);
    // flags & 2: phi increments weighted by 4 q (1 - q), which vanishes in
    // both bulk phases (phi only moves at interfaces)
    const float q = fminf(fmaxf((f0 - pmin) / (pmax - pmin), 0.f), 1.f);
    const float wu = (flags & 1) ? q : 1.f;
    const float wp = (flags & 2) ? 4.f * q * (1.f - q) : 1.f;
    // flags & 4: phi is not clipped to [pmin, pmax]
    const float ph = f0 + wp * (o[0] * q0);
    phi[c] = (flags & 4) ? ph : fminf(fmaxf(ph, pmin), pmax);
    u[c] = f1 + wu * (o[1] * q1);
    u[N + c] = f2 + wu * (o[2] * q2);
    u[2 * N + c] = f3 + wu * (o[3] * q3);
    p[c] = f4 + o[4] * q4;
}

// Jump baseline on boxes of raw states (5 FP32 channels per voxel):
// phi'(x) = phi(x - K u(x)) by trilinear interpolation, the departure point
// clamped to the box; u and p copied.
__global__ void k_advect_phase(const float *__restrict__ s, int64_t count, int bx, int by, int bz, float K,
                               float *__restrict__ o)
{
    const int64_t V = (int64_t)bx * by * bz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * count) return;
    const int64_t n = i / V, v = i % V;
    const float *sb = s + n * V * 5;
    const int x = (int)(v % bx), y = (int)((v / bx) % by), z = (int)(v / ((int64_t)bx * by));
    const float *sv = sb + v * 5;
    float px = (float)x - K * sv[1], py = (float)y - K * sv[2], pz = (float)z - K * sv[3];
    px = fminf(fmaxf(px, 0.f), (float)(bx - 1));
    py = fminf(fmaxf(py, 0.f), (float)(by - 1));
    pz = fminf(fmaxf(pz, 0.f), (float)(bz - 1));
    const int x0 = (int)floorf(px), y0 = (int)floorf(py), z0 = (int)floorf(pz);
    const int x1 = x0 + 1 < bx ? x0 + 1 : x0, y1 = y0 + 1 < by ? y0 + 1 : y0, z1 = z0 + 1 < bz ? z0 + 1 : z0;
    const float fx = px - (float)x0, fy = py - (float)y0, fz = pz - (float)z0;
    auto at = [&](int xx, int yy, int zz) { return sb[(xx + (int64_t)bx * (yy + (int64_t)by * zz)) * 5]; };
    const float c00 = at(x0, y0, z0) * (1.f - fx) + at(x1, y0, z0) * fx;
    const float c10 = at(x0, y1, z0) * (1.f - fx) + at(x1, y1, z0) * fx;
    const float c01 = at(x0, y0, z1) * (1.f - fx) + at(x1, y0, z1) * fx;
    const float c11 = at(x0, y1, z1) * (1.f - fx) + at(x1, y1, z1) * fx;
    const float c0 = c00 * (1.f - fy) + c10 * fy, c1 = c01 * (1.f - fy) + c11 * fy;
    float *ov = o + n * V * 5 + v * 5;
    ov[0] = c0 * (1.f - fz) + c1 * fz;
    ov[1] = sv[1];
    ov[2] = sv[2];
    ov[3] = sv[3];
    ov[4] = sv[4];
}

// Uniform translation of box states: out(x) = s(x - d_n) for all five
// channels by trilinear interpolation, d_n = (shift[4n], shift[4n+1],
// shift[4n+2]) the displacement of box n, the departure point clamped to the
// box; the velocity channels are then multiplied by shift[4n+3].  At steady
// translation (a bubble rising at constant speed) the whole state moves with
// the bubble, so this is the jump of a co-moving frame; the factor carries a
// slowly growing flow amplitude along.
__global__ void k_shift_boxes(const float *__restrict__ s, int64_t count, int bx, int by, int bz,
                              const float *__restrict__ shift, float *__restrict__ o)
{
    const int64_t V = (int64_t)bx * by * bz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * count) return;
    const int64_t n = i / V, v = i % V;
    const float *sb = s + n * V * 5;
    const int x = (int)(v % bx), y = (int)((v / bx) % by), z = (int)(v / ((int64_t)bx * by));
    float px = (float)x - shift[4 * n], py = (float)y - shift[4 * n + 1], pz = (float)z - shift[4 * n + 2];
    const float fu = shift[4 * n + 3];
    px = fminf(fmaxf(px, 0.f), (float)(bx - 1));
    py = fminf(fmaxf(py, 0.f), (float)(by - 1));
    pz = fminf(fmaxf(pz, 0.f), (float)(bz - 1));
    const int x0 = (int)floorf(px), y0 = (int)floorf(py), z0 = (int)floorf(pz);
    const int x1 = x0 + 1 < bx ? x0 + 1 : x0, y1 = y0 + 1 < by ? y0 + 1 : y0, z1 = z0 + 1 < bz ? z0 + 1 : z0;
    const float fx = px - (float)x0, fy = py - (float)y0, fz = pz - (float)z0;
    const int64_t r00 = (int64_t)bx * (y0 + (int64_t)by * z0), r10 = (int64_t)bx * (y1 + (int64_t)by * z0);
    const int64_t r01 = (int64_t)bx * (y0 + (int64_t)by * z1), r11 = (int64_t)bx * (y1 + (int64_t)by * z1);
    float *ov = o + n * V * 5 + v * 5;
    for (int k = 0; k < 5; ++k) {
        auto at = [&](int64_t row, int xx) { return sb[(row + xx) * 5 + k]; };
        const float c00 = at(r00, x0) * (1.f - fx) + at(r00, x1) * fx;
        const float c10 = at(r10, x0) * (1.f - fx) + at(r10, x1) * fx;
        const float c01 = at(r01, x0) * (1.f - fx) + at(r01, x1) * fx;
        const float c11 = at(r11, x0) * (1.f - fx) + at(r11, x1) * fx;
        const float c0 = c00 * (1.f - fy) + c10 * fy, c1 = c01 * (1.f - fy) + c11 * fy;
        const float val = c0 * (1.f - fz) + c1 * fz;
        ov[k] = (k >= 1 && k <= 3) ? val * fu : val;
    }
}

// Gas-indicator moments of box states, one block per box: with
// chi = clamp((phi_heavy - phi) / (phi_heavy - phi_light), 0, 1),
// out[8n + 0] = sum chi, 1..3 = sum chi (x, y, z) (box coordinates),
// 4..6 = sum chi (u_x, u_y, u_z), 7 = 0; FP64, fixed-order reduction.
constexpr int kBoxThreads = 256;
__global__ __launch_bounds__(kBoxThreads) void k_box_moments(const float *__restrict__ s, int bx, int by, int bz,
                                                            float pheavy, float plight, double *__restrict__ out)
{
    __shared__ double sh[7][kBoxThreads];
    const int64_t V = (int64_t)bx * by * bz;
    const float *sb = s + (int64_t)blockIdx.x * V * 5;
    const double inv = 1.0 / ((double)pheavy - (double)plight);
    double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t v = threadIdx.x; v < V; v += kBoxThreads) {
        const float *sv = sb + v * 5;
        const double chi = fmin(fmax(((double)pheavy - (double)sv[0]) * inv, 0.0), 1.0);
        const int x = (int)(v % bx), y = (int)((v / bx) % by), z = (int)(v / ((int64_t)bx * by));
        acc[0] += chi;
        acc[1] += chi * x;
        acc[2] += chi * y;
        acc[3] += chi * z;
        acc[4] += chi * sv[1];
        acc[5] += chi * sv[2];
        acc[6] += chi * sv[3];
    }
    for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int st = kBoxThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 8) out[(int64_t)blockIdx.x * 8 + threadIdx.x] = threadIdx.x < 7 ? sh[threadIdx.x][0] : 0.0;
}

// Projective time step of field sets: s' = s + ratio (s - s_prev) per
// channel, element (i, k) at f[k cs + i vs]; phi clipped to [lo, hi];
// velocity increments weighted by the heavy-phase fraction of the current
// phi if u_by_phase; pressure stepped only if p_step.  out may alias s.
__global__ void k_projective(const float *__restrict__ s, const float *__restrict__ sp, int64_t n, int64_t cs,
                             int64_t vs, float ratio, float lo, float hi, int u_by_phase, int phi_step, int p_step,
                             float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float phi = s[i * vs], dphi = phi - sp[i * vs];
    const float q = fminf(fmaxf((phi - lo) / (hi - lo), 0.f), 1.f);
    const float wu = u_by_phase == 1 ? q : (u_by_phase == 2 ? fmaxf(10.f * q - 9.f, 0.f) : 1.f);
    float v[3], dv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = s[(k + 1) * cs + i * vs];
        dv[k] = v[k] - sp[(k + 1) * cs + i * vs];
    }
    const float p = s[4 * cs + i * vs], dp = p - sp[4 * cs + i * vs];
    out[i * vs] = fminf(fmaxf(phi_step ? phi + ratio * dphi : phi, lo), hi);
#pragma unroll
    for (int k = 0; k < 3; ++k) out[(k + 1) * cs + i * vs] = v[k] + wu * (ratio * dv[k]);
    out[4 * cs + i * vs] = p_step ? p + ratio * dp : p;
}

// Network input of a state and its recent change: channels 0-4 = s /
// scale_in, channels 5-9 = (s - s_prev) * trend_scale, each clipped to
// [-kInClip, kInClip] (the light phase's acoustic noise gives rare, very
// large trends), zeros up to c_in.
constexpr float kInClip = 16.f;
__global__ void k_pair_to_input(const float *__restrict__ s, const float *__restrict__ sp, int64_t V, float q0,
                                float q1, float q2, float q3, float q4, float t0, float t1, float t2, float t3,
                                float t4, int c_in, bf16 *__restrict__ x)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float sc[5] = {q0, q1, q2, q3, q4}, tr[5] = {t0, t1, t2, t3, t4};
    for (int k = 0; k < c_in; ++k) {
        float val = 0.f;
        if (k < 5) val = s[v * 5 + k] / sc[k];
        else if (k < 10) val = (s[v * 5 + k - 5] - sp[v * 5 + k - 5]) * tr[k - 5];
        x[v * c_in + k] = (bf16)fminf(fmaxf(val, -kInClip), kInClip);
    }
}

// Per-channel sum and sum of squares (FP64) of a (rows, C) FP32 array,
// C <= 8: fixed grid of kMomBlocks blocks with fixed-order trees, then one
// block combining the partials in order.
constexpr int kMomBlocks = 512;
__global__ __launch_bounds__(kThreads) void k_moments1(const float *__restrict__ a, int64_t rows, int C,
                                                       double *__restrict__ part)
{
    __shared__ double sh[16][kThreads];
    double acc[16];
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < rows; r += (int64_t)kMomBlocks * kThreads)
        for (int c = 0; c < C; ++c) {
            const double v = a[r * C + c];
            acc[c] += v;
            acc[8 + c] += v * v;
        }
    for (int k = 0; k < 16; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int k = 0; k < 16; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 16) part[(int64_t)blockIdx.x * 16 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_moments2(const double *__restrict__ part, double *__restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= 16) return;
    double s = 0.0;
    for (int b = 0; b < kMomBlocks; ++b) s += part[b * 16 + k];
    out[k] = s;
}

constexpr int kProjBlocks = 1024;
// Weight of a cell in the mass projection: 4 q (1 - q) with q the phase
// fraction clamped to [0, 1]; zero in both bulk phases and in wall rows.
__device__ inline double proj_weight(double f, double pmin, double inv)
{
    double q = (f - pmin) * inv;
    q = q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
    return 4.0 * q * (1.0 - q);
}

__device__ inline bool proj_wall(int64_t i, int nx, int ny, int walls_y)
{
    if (!walls_y) return false;
    const int y = (int)((i / nx) % ny);
    return y == 0 || y == ny - 1;
}

__global__ __launch_bounds__(kThreads) void k_mass_sums(const float *__restrict__ phi, int nx, int ny, int64_t n,
                                                        int walls_y, float pmin, float pmax,
                                                        double *__restrict__ part)
{
    __shared__ double s0[kThreads], s1[kThreads];
    double a = 0.0, w = 0.0;
    const double inv = 1.0 / ((double)pmax - (double)pmin);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)kProjBlocks * kThreads) {
        if (proj_wall(i, nx, ny, walls_y)) continue;
        const double f = phi[i];
        a += f;
        w += proj_weight(f, pmin, inv);
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = w;
    __syncthreads();
    for (int k = kThreads / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            s0[threadIdx.x] += s0[threadIdx.x + k];
            s1[threadIdx.x] += s1[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// sums the block partials in a fixed order (one thread), then corrects phi
__global__ void k_mass_correct(float *__restrict__ phi, int nx, int ny, int64_t n, int walls_y,
                               const double *__restrict__ part, double target, float pmin, float pmax)
{
    __shared__ double coef;
    if (threadIdx.x == 0) {
        double a = 0.0, w = 0.0;
        for (int k = 0; k < kProjBlocks; ++k) {
            a += part[2 * k];
            w += part[2 * k + 1];
        }
        coef = w > 0.0 ? (target - a) / w : 0.0;
    }
    __syncthreads();
    const double inv = 1.0 / ((double)pmax - (double)pmin);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (proj_wall(i, nx, ny, walls_y)) continue;
        const double f = phi[i];
        phi[i] = (float)(f + coef * proj_weight(f, pmin, inv));
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

sg_status check_bwd_weight_args(const void *x, const void *dy, int n, int d, int h, int w, int c_in, int c_out,
                                const float *dw)
{
    if (!x || !dy || !dw) return fail(SG_EARG, "NULL tensor");
    if (n < 1 || d < 1 || h < 1 || w < 1) return fail(SG_EARG, "bad shape");
    if (c_in < 16 || c_in % 16) return fail(SG_EARG, "c_in must be a positive multiple of 16 (got %d)", c_in);
    if (c_out < 32 || c_out % 32) return fail(SG_EARG, "c_out must be a multiple of 32 (got %d)", c_out);
    if (!aligned16(x) || !aligned16(dy)) return fail(SG_EARG, "x and dy must be 16-byte aligned");
    return SG_OK;
}

// Launch plan of the weight gradient: W rows padded to Wp voxels, K steps of
// kBwStep voxels split into `chunks` consecutive ranges of `per` steps (about
// kBw2TargetBlocks blocks over the (co, ci) tiles); the bias sums split the
// groups into nb ranges.  Scratch layout: per-chunk partial sums, bias
// partials, then the group-major copies of x and dy.
struct BwPlan {
    int Wp;
    int64_t R;       // rows N D H
    int64_t steps;   // K steps
    int chunks;
    int64_t per;
    int nb;          // bias ranges per channel
    int64_t bper;
    int rgroups;     // groups of the two-level chunk sum (1: one level)
    size_t off_part2, off_bpart, off_xt, off_dyt, bytes;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

BwPlan bw_plan(int n, int d, int h, int w, int ci, int co)
{
    BwPlan p;
    p.Wp = (w + kBwStep - 1) / kBwStep * kBwStep;
    p.R = (int64_t)n * d * h;
    p.steps = p.R * (p.Wp / kBwStep);
    const int64_t mn = (int64_t)(co / 32) * ((ci + 31) / 32);
    int64_t ch = (kBw2TargetBlocks + mn - 1) / mn;
    if (ch > p.steps) ch = p.steps;
    if (ch < 1) ch = 1;
    p.per = (p.steps + ch - 1) / ch;
    p.chunks = (int)((p.steps + p.per - 1) / p.per + 7) / 8 * 8;  // a multiple of 8 (see the kernel); extra
                                                                  // chunks are empty and write zeros
    const int64_t groups = p.R * (p.Wp / 8);
    int64_t nb = groups / 1024;
    nb = nb < 1 ? 1 : (nb > 256 ? 256 : nb);
    p.bper = (groups + nb - 1) / nb;
    p.nb = (int)((groups + p.bper - 1) / p.bper);
    p.rgroups = (p.chunks + kBwReduceGroup - 1) / kBwReduceGroup;
    p.off_part2 = align_up((size_t)p.chunks * 27 * ci * co * sizeof(float), 256);
    p.off_bpart = p.off_part2 + (p.rgroups > 1 ? align_up((size_t)p.rgroups * 27 * ci * co * sizeof(float), 256) : 0);
    p.off_xt = p.off_bpart + align_up((size_t)p.nb * co * sizeof(float), 256);
    p.off_dyt = p.off_xt + align_up((size_t)ci * groups * 8 * sizeof(bf16), 256);
    p.bytes = p.off_dyt + align_up((size_t)co * groups * 8 * sizeof(bf16), 256);
    return p;
}

// Weight and bias gradient through the scratch `ws` (every entry written
// before it is read): group-major copies of x and dy, per-chunk partial sums
// part[chunk][t][co][ci], then a fixed-order sum over chunks (in groups of
// kBwReduceGroup chunks, then over the groups).
sg_status launch_bwd_weight(const void *x, const void *dy, int n, int d, int h, int w, int c_in, int c_out,
                            float *dw, float *db, const BwPlan &p, char *ws, hipStream_t s)
{
    float *part = (float *)ws;
    float *bpart = (float *)(ws + p.off_bpart);
    bf16 *xt = (bf16 *)(ws + p.off_xt);
    bf16 *dyt = (bf16 *)(ws + p.off_dyt);
    const int ng = p.Wp / 8;
    const int64_t groups = p.R * ng;
    hipLaunchKernelGGL(k_to_group_major, dim3(blocks_for(groups * c_in)), dim3(kThreads), 0, s, (const bf16 *)x,
                       p.R, w, ng, c_in, xt);
    SG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_to_group_major, dim3(blocks_for(groups * c_out)), dim3(kThreads), 0, s, (const bf16 *)dy,
                       p.R, w, ng, c_out, dyt);
    SG_LAUNCH_CHECK();
    const int tiles = (c_out / 32) * ((c_in + 31) / 32);
    const dim3 grid((unsigned)(3 * p.chunks * tiles));
    hipLaunchKernelGGL(k_conv3d_bwd_weight_gm, grid, dim3(kBwThreads), 0, s, xt, dyt, n, d, h, ng, c_in, c_out,
                       p.steps, p.per, p.chunks, part);
    SG_LAUNCH_CHECK();
    const int64_t stride = (int64_t)27 * c_in * c_out;
    if (p.rgroups > 1) {
        float *part2 = (float *)(ws + p.off_part2);
        hipLaunchKernelGGL(k_reduce_partials_grouped, dim3(blocks_for(stride), (unsigned)p.rgroups), dim3(kThreads), 0,
                           s, part, p.chunks, kBwReduceGroup, stride, part2);
        SG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for(stride)), dim3(kThreads), 0, s, part2, p.rgroups, stride,
                           dw);
    } else {
        hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for(stride)), dim3(kThreads), 0, s, part, p.chunks, stride,
                           dw);
    }
    SG_LAUNCH_CHECK();
    if (db) {
        hipLaunchKernelGGL(k_bias_grad_gm, dim3((unsigned)p.nb, (unsigned)c_out), dim3(kThreads), 0, s, dyt,
                           groups, c_out, p.bper, bpart);
        SG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for(c_out)), dim3(kThreads), 0, s, bpart, p.nb,
                           (int64_t)c_out, db);
        SG_LAUNCH_CHECK();
    }
    return SG_OK;
}

// ---- input gradient without allocation --------------------------------------------
// The mirrored weights of the input gradient go to a fixed device array
// instead of a caller workspace.  The array's name is a host-side stand-in in
// host code, so its device address is looked up once per device (with that
// device current) and only that address is passed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

sg_status noalloc_scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SG_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SG_EARG, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !p)
            return fail(SG_EHIP, "hipGetSymbolAddress(noalloc_scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SG_OK;
}

}  // namespace

extern "C" {

// The forward launch for one input (xa, ca = c_in, up_a = 0, xb = NULL) or
// the upsampled-and-concatenated pair (arguments checked by the callers).
static sg_status conv3d_fwd_launch(const void *xa, int32_t ca, int32_t up_a, const void *xb, int32_t n,
                                   int32_t d, int32_t h, int32_t w, int32_t c_in, const void *wt, const float *bias,
                                   int32_t c_out, int32_t n_store, int32_t act, float slope, void *y, int32_t y_f32,
                                   void *stream)
{
    if (!wt || !y) return fail(SG_EARG, "NULL tensor");
    if (n < 1 || d < 1 || h < 1 || w < 1) return fail(SG_EARG, "bad shape");
    if (c_in < 16 || c_in % 16) return fail(SG_EARG, "c_in must be a positive multiple of 16 (got %d)", c_in);
    if (c_out < 32 || c_out % 32) return fail(SG_EARG, "c_out must be a positive multiple of 32 (got %d)", c_out);
    if (n_store < 1 || n_store > c_out) return fail(SG_EARG, "n_store must be in [1, c_out]");
    if (!aligned16(wt)) return fail(SG_EARG, "wt must be 16-byte aligned");
    const int tiles = c_out / 32;
    const int tw = w > 16 ? 32 : w > 8 ? 16 : 8;
    const int th = 32 / tw;
    const int nbd = (d + 3) / 4, nbh = (h + 4 * th - 1) / (4 * th), nbw = (w + tw - 1) / tw;
    const int64_t nbox = (int64_t)n * nbd * nbh * nbw;
    // 64 output channels per block where that still gives two blocks per CU
    // (256 CUs); below that, 32 per block doubles the blocks of small layers
    const int nt = tiles % 2 == 0 && nbox * (tiles / 2) >= 512 ? 2 : 1;
    if (nbox > 0x7fffffff) return fail(SG_ESIZE, "too many voxels");
    const dim3 grid((unsigned)nbox, (unsigned)(tiles / nt));
    hipStream_t s = (hipStream_t)stream;
    const bf16 *XA = (const bf16 *)xa, *XB = (const bf16 *)xb, *Wt = (const bf16 *)wt;
#define SG_CONV_LAUNCH(NT_, TW_)                                                                              \
    do {                                                                                                      \
        if (XB)                                                                                               \
            hipLaunchKernelGGL((k_conv3d_lds<NT_, TW_, true>), grid, dim3(kThreads), 0, s, XA, ca, up_a, XB, Wt, \
                               bias, y, n, d, h, w, c_in, c_out, n_store, act, slope, y_f32, nbd, nbh, nbw);    \
        else                                                                                                  \
            hipLaunchKernelGGL((k_conv3d_lds<NT_, TW_, false>), grid, dim3(kThreads), 0, s, XA, ca, up_a, XB,   \
                               Wt, bias, y, n, d, h, w, c_in, c_out, n_store, act, slope, y_f32, nbd, nbh, nbw); \
    } while (0)
    if (nt == 2) {
        if (tw == 32) SG_CONV_LAUNCH(2, 32);
        else if (tw == 16) SG_CONV_LAUNCH(2, 16);
        else SG_CONV_LAUNCH(2, 8);
    } else {
        if (tw == 32) SG_CONV_LAUNCH(1, 32);
        else if (tw == 16) SG_CONV_LAUNCH(1, 16);
        else SG_CONV_LAUNCH(1, 8);
    }
#undef SG_CONV_LAUNCH
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_conv3d_fwd(const void *x, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c_in,
                        const void *wt, const float *bias, int32_t c_out, int32_t n_store, int32_t act,
                        float slope, void *y, int32_t y_f32, void *stream)
{
    if (!x) return fail(SG_EARG, "NULL tensor");
    if (!aligned16(x)) return fail(SG_EARG, "x and wt must be 16-byte aligned");
    return conv3d_fwd_launch(x, c_in, 0, nullptr, n, d, h, w, c_in, wt, bias, c_out, n_store, act, slope, y, y_f32,
                             stream);
}

sg_status sg_conv3d_fwd_up_cat(const void *xa, int32_t ca, const void *xb, int32_t cb, int32_t n, int32_t d,
                               int32_t h, int32_t w, const void *wt, const float *bias, int32_t c_out,
                               int32_t n_store, int32_t act, float slope, void *y, int32_t y_f32, void *stream)
{
    if (!xa || !xb) return fail(SG_EARG, "NULL tensor");
    if (!aligned16(xa) || !aligned16(xb)) return fail(SG_EARG, "xa and xb must be 16-byte aligned");
    if (ca < 16 || ca % 16 || cb < 16 || cb % 16)
        return fail(SG_EARG, "ca and cb must be positive multiples of 16 (got %d, %d)", ca, cb);
    if (d % 2 || h % 2 || w % 2) return fail(SG_EARG, "d, h and w must be even (upsampling by 2)");
    return conv3d_fwd_launch(xa, ca, 1, xb, n, d, h, w, ca + cb, wt, bias, c_out, n_store, act, slope, y, y_f32,
                             stream);
}

sg_status sg_weight_mirror(const void *wt, int32_t c_out, int32_t c_in, void *wm, void *stream)
{
    if (!wt || !wm || c_out < 1 || c_in < 1) return fail(SG_EARG, "bad arguments");
    const int64_t total = (int64_t)27 * c_out * c_in;
    hipLaunchKernelGGL(k_weight_mirror, dim3(blocks_for(total)), dim3(kThreads), 0, (hipStream_t)stream,
                       (const bf16 *)wt, c_out, c_in, (bf16 *)wm);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_conv3d_bwd_data(const void *dy, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c_out,
                             const void *wt, int32_t c_in, void *dx, void *ws, size_t ws_bytes, void *stream)
{
    if (!dy || !wt || !dx || !ws) return fail(SG_EARG, "NULL tensor");
    if (c_in < 32 || c_in % 32) return fail(SG_EARG, "c_in must be a positive multiple of 32 (got %d)", c_in);
    if (c_out < 16 || c_out % 16) return fail(SG_EARG, "c_out must be a positive multiple of 16 (got %d)", c_out);
    const size_t need = (size_t)27 * c_in * c_out * sizeof(bf16);
    if (ws_bytes < need) return fail(SG_ESIZE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    if (!aligned16(ws)) return fail(SG_EARG, "workspace must be 16-byte aligned");
    sg_status st = sg_weight_mirror(wt, c_out, c_in, ws, stream);
    if (st != SG_OK) return st;
    return sg_conv3d_fwd(dy, n, d, h, w, c_out, ws, nullptr, c_in, c_in, 0, 0.f, dx, 0, stream);
}

size_t sg_bwd_weight_workspace(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c_in, int32_t c_out)
{
    if (n < 1 || d < 1 || h < 1 || w < 1 || c_in < 1 || c_out < 32) return 0;
    return bw_plan(n, d, h, w, c_in, c_out).bytes;
}

sg_status sg_conv3d_bwd_weight(const void *x, const void *dy, int32_t n, int32_t d, int32_t h, int32_t w,
                               int32_t c_in, int32_t c_out, float *dw, float *db, void *ws, size_t ws_bytes,
                               void *stream)
{
    sg_status st = check_bwd_weight_args(x, dy, n, d, h, w, c_in, c_out, dw);
    if (st != SG_OK) return st;
    if (!ws) return fail(SG_EARG, "NULL workspace");
    const size_t need = sg_bwd_weight_workspace(n, d, h, w, c_in, c_out);
    if (ws_bytes < need) return fail(SG_ESIZE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    if (!aligned16(ws)) return fail(SG_EARG, "workspace must be 16-byte aligned");
    const BwPlan p = bw_plan(n, d, h, w, c_in, c_out);
    return launch_bwd_weight(x, dy, n, d, h, w, c_in, c_out, dw, db, p, (char *)ws, (hipStream_t)stream);
}

sg_status sg_leaky_bwd(const void *y, const void *dy, void *dp, size_t count, float slope, void *stream)
{
    if (!y || !dy || !dp) return fail(SG_EARG, "NULL tensor");
    if (count % 8 == 0 && aligned16(y) && aligned16(dy) && aligned16(dp))
        hipLaunchKernelGGL(k_leaky_bwd8, dim3(blocks_for((int64_t)count / 8)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16x8 *)y, (const bf16x8 *)dy, (bf16x8 *)dp, (int64_t)count / 8, slope);
    else
        hipLaunchKernelGGL(k_leaky_bwd, dim3(blocks_for((int64_t)count)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16 *)y, (const bf16 *)dy, (bf16 *)dp, (int64_t)count, slope);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_pool2_fwd(const void *x, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, void *y, void *stream)
{
    if (!x || !y || d % 2 || h % 2 || w % 2) return fail(SG_EARG, "pool2 needs even d, h, w");
    const int64_t total = (int64_t)n * (d / 2) * (h / 2) * (w / 2) * c;
    if (c % 8 == 0 && aligned16(x) && aligned16(y))
        hipLaunchKernelGGL(k_pool2_fwd8, dim3(blocks_for(total / 8)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16x8 *)x, n, d, h, w, c / 8, (bf16x8 *)y);
    else
        hipLaunchKernelGGL(k_pool2_fwd, dim3(blocks_for(total)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16 *)x, n, d, h, w, c, (bf16 *)y);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_pool2_bwd(const void *dy, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, void *dx, void *stream)
{
    if (!dy || !dx || d % 2 || h % 2 || w % 2) return fail(SG_EARG, "pool2 needs even d, h, w");
    const int64_t total = (int64_t)n * d * h * w * c;
    if (c % 8 == 0 && aligned16(dy) && aligned16(dx))
        hipLaunchKernelGGL(k_pool2_bwd8, dim3(blocks_for(total / 8)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16x8 *)dy, n, d, h, w, c / 8, (bf16x8 *)dx);
    else
        hipLaunchKernelGGL(k_pool2_bwd, dim3(blocks_for(total)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16 *)dy, n, d, h, w, c, (bf16 *)dx);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_up2_fwd(const void *x, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, void *y, void *stream)
{
    if (!x || !y) return fail(SG_EARG, "NULL tensor");
    const int64_t total = (int64_t)n * 8 * d * h * w * c;
    if (c % 8 == 0 && aligned16(x) && aligned16(y))
        hipLaunchKernelGGL(k_up2_fwd8, dim3(blocks_for(total / 8)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16x8 *)x, n, d, h, w, c / 8, (bf16x8 *)y);
    else
        hipLaunchKernelGGL(k_up2_fwd, dim3(blocks_for(total)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16 *)x, n, d, h, w, c, (bf16 *)y);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_up2_bwd(const void *dy, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, void *dx, void *stream)
{
    if (!dy || !dx) return fail(SG_EARG, "NULL tensor");
    const int64_t total = (int64_t)n * d * h * w * c;
    if (c % 8 == 0 && aligned16(dy) && aligned16(dx))
        hipLaunchKernelGGL(k_up2_bwd8, dim3(blocks_for(total / 8)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16x8 *)dy, n, d, h, w, c / 8, (bf16x8 *)dx);
    else
        hipLaunchKernelGGL(k_up2_bwd, dim3(blocks_for(total)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16 *)dy, n, d, h, w, c, (bf16 *)dx);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_concat(const void *a, int32_t ca, const void *b, int32_t cb, int64_t V, void *y, void *stream)
{
    if (!a || !b || !y) return fail(SG_EARG, "NULL tensor");
    if (ca % 8 == 0 && cb % 8 == 0 && aligned16(a) && aligned16(b) && aligned16(y))
        hipLaunchKernelGGL(k_concat8, dim3(blocks_for(V * (ca + cb) / 8)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16x8 *)a, ca / 8, (const bf16x8 *)b, cb / 8, V, (bf16x8 *)y);
    else
        hipLaunchKernelGGL(k_concat, dim3(blocks_for(V * (ca + cb))), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16 *)a, ca, (const bf16 *)b, cb, V, (bf16 *)y);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_split(const void *y, int32_t ca, int32_t cb, int64_t V, void *a, void *b, void *stream)
{
    if (!y) return fail(SG_EARG, "NULL tensor");
    if (ca % 8 == 0 && cb % 8 == 0 && aligned16(y) && aligned16(a) && aligned16(b))
        hipLaunchKernelGGL(k_split8, dim3(blocks_for(V * (ca + cb) / 8)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16x8 *)y, ca / 8, cb / 8, V, (bf16x8 *)a, (bf16x8 *)b);
    else
        hipLaunchKernelGGL(k_split, dim3(blocks_for(V * (ca + cb))), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16 *)y, ca, cb, V, (bf16 *)a, (bf16 *)b);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_mse(const float *pred, const float *target, int64_t count, float *loss, void *grad, float *scratch,
                 void *stream)
{
    if (!pred || !target || !loss || !grad || !scratch || count < 1) return fail(SG_EARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mse1, dim3(kMseBlocks), dim3(kThreads), 0, s, pred, target, count, (bf16 *)grad, scratch);
    SG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mse2, dim3(1), dim3(kThreads), 0, s, scratch, count, loss);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_adam(float *p, const float *g, float *m, float *v, void *wt, int64_t count, float lr, float b1,
                  float b2, float eps, int32_t step, void *stream)
{
    if (!p || !g || !m || !v || count < 1 || step < 1) return fail(SG_EARG, "bad arguments");
    const float c1 = (float)(1.0 - std::pow((double)b1, step)), c2 = (float)(1.0 - std::pow((double)b2, step));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(count)), dim3(kThreads), 0, (hipStream_t)stream, p, g, m, v,
                       (bf16 *)wt, count, lr, b1, b2, eps, c1, c2);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_to_bf16(const float *x, void *y, int64_t count, void *stream)
{
    if (!x || !y) return fail(SG_EARG, "NULL tensor");
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(count)), dim3(kThreads), 0, (hipStream_t)stream, x, (bf16 *)y, count);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_to_f32(const void *x, float *y, int64_t count, void *stream)
{
    if (!x || !y) return fail(SG_EARG, "NULL tensor");
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(count)), dim3(kThreads), 0, (hipStream_t)stream, (const bf16 *)x, y, count);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_add(const void *a, const void *b, void *y, int64_t count, void *stream)
{
    if (!a || !b || !y) return fail(SG_EARG, "NULL tensor");
    if (count % 8 == 0 && aligned16(a) && aligned16(b) && aligned16(y))
        hipLaunchKernelGGL(k_add8, dim3(blocks_for(count / 8)), dim3(kThreads), 0, (hipStream_t)stream,
                           (const bf16x8 *)a, (const bf16x8 *)b, (bf16x8 *)y, count / 8);
    else
        hipLaunchKernelGGL(k_add, dim3(blocks_for(count)), dim3(kThreads), 0, (hipStream_t)stream, (const bf16 *)a,
                           (const bf16 *)b, (bf16 *)y, count);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

static sg_status read_box(const int32_t *box, int nx, int ny, int nz, Box &b)
{
    if (!box) return fail(SG_EARG, "NULL box");
    b = Box{box[0], box[1], box[2], box[3], box[4], box[5]};
    if (b.bx < 1 || b.by < 1 || b.bz < 1 || b.bx > nx || b.bz > nz) return fail(SG_EARG, "bad box size");
    if (b.y0 < 0 || b.y0 + b.by > ny) return fail(SG_EARG, "box leaves [0, ny) in y");
    return SG_OK;
}

sg_status sg_fields_to_input(const float *phi, const float *u, const float *p, int32_t nx, int32_t ny, int32_t nz,
                             const int32_t *box, const float *si, int32_t c_in, void *x, float *state, void *stream)
{
    if (!phi || !u || !p || !si || !x || c_in < 5) return fail(SG_EARG, "bad arguments");
    Box b;
    sg_status st = read_box(box, nx, ny, nz, b);
    if (st != SG_OK) return st;
    const int64_t V = (int64_t)b.bx * b.by * b.bz;
    hipLaunchKernelGGL(k_fields_to_input, dim3(blocks_for(V)), dim3(kThreads), 0, (hipStream_t)stream, phi, u, p, nx,
                       ny, nz, b, si[0], si[1], si[2], si[3], si[4], c_in, (bf16 *)x, state);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_state_to_input(const float *s, int64_t V, const float *si, int32_t c_in, void *x, void *stream)
{
    if (!s || !si || !x || c_in < 5) return fail(SG_EARG, "bad arguments");
    hipLaunchKernelGGL(k_state_to_input, dim3(blocks_for(V)), dim3(kThreads), 0, (hipStream_t)stream, s, V, si[0],
                       si[1], si[2], si[3], si[4], c_in, (bf16 *)x);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_make_target(const float *s0, const float *s1, int64_t V, const float *so, int32_t c_out, float *t,
                         void *stream)
{
    if (!s0 || !s1 || !so || !t || c_out < 5) return fail(SG_EARG, "bad arguments");
    hipLaunchKernelGGL(k_make_target, dim3(blocks_for(V)), dim3(kThreads), 0, (hipStream_t)stream, s0, s1, V, so[0],
                       so[1], so[2], so[3], so[4], c_out, t);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_apply_prediction(const float *out, int32_t c_out, const float *so, const float *base, float *phi,
                              float *u, float *p, int32_t nx, int32_t ny, int32_t nz, const int32_t *box,
                              int32_t walls_y, float pmin, float pmax, int32_t flags, void *stream)
{
    if (!out || !so || !phi || !u || !p || c_out < 5) return fail(SG_EARG, "bad arguments");
    if (!(pmax > pmin)) return fail(SG_EARG, "phi_max must exceed phi_min");
    Box b;
    sg_status st = read_box(box, nx, ny, nz, b);
    if (st != SG_OK) return st;
    const int64_t V = (int64_t)b.bx * b.by * b.bz;
    hipLaunchKernelGGL(k_apply_prediction, dim3(blocks_for(V)), dim3(kThreads), 0, (hipStream_t)stream, out, c_out,
                       so[0], so[1], so[2], so[3], so[4], base, phi, u, p, nx, ny, nz, b, walls_y, pmin, pmax,
                       flags);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_advect_phase(const float *state, int64_t count, int32_t bx, int32_t by, int32_t bz, float K,
                          float *out, void *stream)
{
    if (!state || !out || count < 1 || bx < 1 || by < 1 || bz < 1) return fail(SG_EARG, "bad arguments");
    if (state == out) return fail(SG_EARG, "sg_advect_phase cannot run in place");
    const int64_t n = count * bx * (int64_t)by * bz;
    hipLaunchKernelGGL(k_advect_phase, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, state, count,
                       bx, by, bz, K, out);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_shift_boxes(const float *state, int64_t count, int32_t bx, int32_t by, int32_t bz, const float *shift,
                         float *out, void *stream)
{
    if (!state || !shift || !out || count < 1 || bx < 1 || by < 1 || bz < 1) return fail(SG_EARG, "bad arguments");
    if (state == out) return fail(SG_EARG, "sg_shift_boxes cannot run in place");
    const int64_t n = count * bx * (int64_t)by * bz;
    hipLaunchKernelGGL(k_shift_boxes, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, state, count,
                       bx, by, bz, shift, out);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_box_moments(const float *state, int64_t count, int32_t bx, int32_t by, int32_t bz, float phi_heavy,
                         float phi_light, double *out, void *stream)
{
    if (!state || !out || count < 1 || count > INT32_MAX || bx < 1 || by < 1 || bz < 1 || !(phi_heavy != phi_light))
        return fail(SG_EARG, "bad arguments");
    hipLaunchKernelGGL(k_box_moments, dim3((unsigned)count), dim3(kBoxThreads), 0, (hipStream_t)stream, state, bx, by,
                       bz, phi_heavy, phi_light, out);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_projective_step(const float *s, const float *s_prev, int64_t n, int64_t cs, int64_t vs, float ratio,
                             float phi_lo, float phi_hi, int32_t u_by_phase, int32_t phi_step, int32_t p_step,
                             float *out, void *stream)
{
    if (!s || !s_prev || !out || n < 1 || cs < 1 || vs < 1 || !(phi_hi > phi_lo)) return fail(SG_EARG, "bad arguments");
    if (!((cs == n && vs == 1) || (cs == 1 && vs == 5))) return fail(SG_EARG, "layout must be planar or channels last");
    if (u_by_phase < 0 || u_by_phase > 2) return fail(SG_EARG, "u_by_phase must be 0, 1 or 2 (got %d)", u_by_phase);
    hipLaunchKernelGGL(k_projective, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, s, s_prev, n, cs,
                       vs, ratio, phi_lo, phi_hi, u_by_phase, phi_step, p_step, out);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_pair_to_input(const float *s, const float *s_prev, int64_t V, const float *si, const float *ts,
                           int32_t c_in, void *x, void *stream)
{
    if (!s || !s_prev || !si || !ts || !x || c_in < 10) return fail(SG_EARG, "bad arguments");
    hipLaunchKernelGGL(k_pair_to_input, dim3(blocks_for(V)), dim3(kThreads), 0, (hipStream_t)stream, s, s_prev, V,
                       si[0], si[1], si[2], si[3], si[4], ts[0], ts[1], ts[2], ts[3], ts[4], c_in, (bf16 *)x);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_channel_moments(const float *a, int64_t rows, int32_t c, double *out, double *scratch, void *stream)
{
    if (!a || !out || !scratch || rows < 1 || c < 1 || c > 8) return fail(SG_EARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_moments1, dim3(kMomBlocks), dim3(kThreads), 0, s, a, rows, c, scratch);
    SG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_moments2, dim3(1), dim3(64), 0, s, scratch, out);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_mass_project(float *phi, int32_t nx, int32_t ny, int32_t nz, int32_t walls_y, double target,
                          float pmin, float pmax, double *scratch, void *stream)
{
    if (!phi || !scratch || nx < 1 || ny < 1 || nz < 1 || !(pmax > pmin)) return fail(SG_EARG, "bad arguments");
    if (walls_y && ny < 3) return fail(SG_EARG, "walls_y needs ny >= 3");
    const int64_t n = (int64_t)nx * ny * nz;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mass_sums, dim3(kProjBlocks), dim3(kThreads), 0, s, phi, nx, ny, n, walls_y, pmin, pmax,
                       scratch);
    SG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mass_correct, dim3(4096), dim3(kThreads), 0, s, phi, nx, ny, n, walls_y, scratch, target,
                       pmin, pmax);
    SG_LAUNCH_CHECK();
    return SG_OK;
}

sg_status sg_conv3d_bwd_data_noalloc(const void *dy, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c_out,
                                     const void *wt, int32_t c_in, void *dx, void *stream)
{
    if (!dy || !wt || !dx) return fail(SG_EARG, "NULL tensor");
    if (c_in < 32 || c_in % 32) return fail(SG_EARG, "c_in must be a positive multiple of 32 (got %d)", c_in);
    if (c_out < 16 || c_out % 16) return fail(SG_EARG, "c_out must be a positive multiple of 16 (got %d)", c_out);
    const size_t need = (size_t)27 * c_in * c_out * sizeof(bf16);
    if (need > kNoAllocScratchBytes)
        return fail(SG_ESIZE, "27 * c_in * c_out BF16 weights take %zu bytes, above the %zu-byte fixed scratch",
                    need, kNoAllocScratchBytes);
    void *wm = nullptr;
    sg_status st = noalloc_scratch_ptr(&wm);
    if (st != SG_OK) return st;
    st = sg_weight_mirror(wt, c_out, c_in, wm, stream);
    if (st != SG_OK) return st;
    return sg_conv3d_fwd(dy, n, d, h, w, c_out, wm, nullptr, c_in, c_in, 0, 0.f, dx, 0, stream);
}

const char *sg_last_error(void) { return g_err; }

}  // extern "C"
