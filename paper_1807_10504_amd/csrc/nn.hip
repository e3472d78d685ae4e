// Learned warm start for the pressure solve (project addition; the paper
// uses multigrid alone). A 6-layer convolutional network with 3x3 (2D) or
// 3x3x3 (3D) taps (circular padding, channels 3 -> 32 x 5 -> 1, ReLU between)
// maps the normalised right side, inverse density and previous pressure to a
// pressure correction; multigrid starts from p0 = p_prev + s_p * y and alone
// decides the final answer.
//
// Precision: bfloat16 weights, activations and gradients in memory, float32
// accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16), float32
// master weights and Adam moments, float64 at the solver boundary.
//
// Layout: activations NDHWC / NHWC with 32 channels (the 3 input channels and
// the 1 output channel are zero-padded to 32), bfloat16 stored as 16-bit
// patterns. Weights per layer: Wl[co][tap][ci] (tap = 9 kz + 3 ky + kx
// multiplies the input at (z + kz - 1, y + ky - 1, x + kx - 1); 2D: tap =
// 3 ky + kx) and the flipped transpose Wt[ci][taps - 1 - tap][co] used by the
// input gradient, which is then the same convolution kernel.
//
// A convolution is an implicit GEMM. In 3D (k_nn_conv3_tiled) a workgroup
// keeps the layer's weights in LDS and marches a 64 x 8 pixel tile along z,
// staging each input plane once for the three output planes it touches; in
// 2D (and on 3D grids the tiles do not fit) k_nn_conv has a wave own 16
// pixels of one row and all 32 output channels and, for each tap, multiply a
// 16 x 32 (pixel x channel) slab of the shifted input by the 32 x 16 weight
// block of each half of the output channels (two MFMA per tap); the two give
// identical results. The 3D first layer, whose input has 3 channels, packs
// the 27 (ky, kx, channel) products of each kz into one 32-wide operand
// (PACK): 3 products per output block instead of 27, in both kernels, which
// again agree bit for bit; it reads the input in 8 channels (16 bytes a
// pixel) instead of 32. The weight gradient is a GEMM
// over pixels: a workgroup stages 64 pixels of the gradient and the input
// rows they touch in LDS and accumulates the (tap, co-block, ci-block)
// 16 x 16 tiles; per-workgroup partials are summed in a fixed order.
#include <cmath>
#include <type_traits>
#include <vector>

#include "common.h"

namespace ib {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kC = 32;          // padded channel count
constexpr int kLayers = 6;
// taps per convolution: 3^dim; weights per layer kC x taps x kC, + bias
__host__ __device__ constexpr int wsize(int taps) { return kC * taps * kC; }
__host__ __device__ constexpr int psize(int taps) { return wsize(taps) + kC; }
constexpr int kGradBlocks = 256;
static const int kChan[7] = {3, 32, 32, 32, 32, 32, 1};

__device__ __forceinline__ u16 f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float(((unsigned)h) << 16); }

// ---------------------------------------------------------------------------
// input normalisation: partial sums of (b h^2)^2 and p_prev^2, max of 1/rho
__global__ void k_nn_stats(const double* __restrict__ b, const double* __restrict__ H,
                           const double* __restrict__ pp, long N, double h2, double rin,
                           double rout, double* __restrict__ part) {
    __shared__ double sh[kBlock];
    double sb = 0.0, sp = 0.0, mr = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        double bh = b[c] * h2;
        sb += bh * bh;
        double p = pp ? pp[c] : 0.0;
        sp += p * p;
        mr = fmax(mr, 1.0 / (rout + (rin - rout) * H[c]));
    }
    double r = block_reduce_sum(sb, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
    r = block_reduce_sum(sp, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = r;
    sh[threadIdx.x] = mr;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[2 * gridDim.x + blockIdx.x] = sh[0];
}

// scale[0] = s_b, scale[1] = s_p, scale[2] = s_r (each 1 when zero)
__global__ void k_nn_scales(const double* __restrict__ part, int nb, long N, double* __restrict__ scale) {
    __shared__ double sh[kBlock];
    double a = 0.0, b = 0.0, m = 0.0;
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        a += part[q];
        b += part[nb + q];
        m = fmax(m, part[2 * nb + q]);
    }
    double sa = block_reduce_sum(a, sh);
    double sb = block_reduce_sum(b, sh);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double rb = sqrt(sa / (double)N), rp = sqrt(sb / (double)N);
        scale[0] = rb > 0.0 ? rb : 1.0;
        scale[1] = rp > 0.0 ? rp : 1.0;
        scale[2] = sh[0] > 0.0 ? sh[0] : 1.0;
    }
}

// one lane per 16-byte chunk of a pixel's NCH chunks (NCH = 4: the 32
// bfloat16 channels of the layer layout, a wave writing 16 whole pixels, 1 KB,
// with one store; NCH = 1: the 8-channel form the packed 3D first layer
// reads): chunk 0 holds channels 0 .. 2, the rest are zero padding
template <int NCH>
__global__ void k_nn_input(const double* __restrict__ b, const double* __restrict__ H,
                           const double* __restrict__ pp, long N, double h2, double rin, double rout,
                           const double* __restrict__ scale, u16* __restrict__ X) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NCH * N) return;
    const long c = q / NCH;
    uint4 v = {0u, 0u, 0u, 0u};
    if (q % NCH == 0) {
        float v0 = (float)(b[c] * h2 / scale[0]);
        float v1 = (float)((1.0 / (rout + (rin - rout) * H[c])) / scale[2]);
        float v2 = (float)((pp ? pp[c] : 0.0) / scale[1]);
        v.x = (unsigned)f2bf(v0) | ((unsigned)f2bf(v1) << 16);
        v.y = f2bf(v2);
    }
    reinterpret_cast<uint4*>(X)[q] = v;
}

// ---------------------------------------------------------------------------
// The first layer has 3 input channels (the rest of the 32 are zero): its 27
// in-plane products of a plane kz, (ky, kx, ci), are packed into one K = 32
// operand, k = 3 (3 ky + kx) + ci for k < 27; k = 27 .. 31 read input
// channel 3 of the centre pixel (zero) against zero weights. Three matrix
// products per output instead of 27. pack_tap gives k's offsets.
__device__ __forceinline__ void pack_tap(int k, int& ky, int& kx, int& ci) {
    if (k < 27) {
        ky = k / 9;
        kx = (k / 3) % 3;
        ci = k % 3;
    } else {
        ky = 1;
        kx = 1;
        ci = 3;
    }
}

// weight fragment of the packed first layer for plane kz, output channels
// cb 16 .. cb 16 + 15: lane (n, kg) holds W[cb 16 + n][9 kz + 3 ky + kx][ci]
// for the eight k of kg
__device__ __forceinline__ bf16x8 pack_weights(const u16* __restrict__ Wl, int kz, int cb, int n, int kg) {
    bf16x8 b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int ky, kx, ci;
        const int k = kg * 8 + e;
        pack_tap(k, ky, kx, ci);
        const u16 v = k < 27 ? Wl[((cb * 16 + n) * 27 + 9 * kz + 3 * ky + kx) * kC + ci] : (u16)0;
        b[e] = __builtin_bit_cast(__bf16, v);
    }
    return b;
}

// Epilogue of a 16-pixel block whose products took the weights as the left
// operand: this lane holds channels c0 .. c0 + 3 (a0) and 16 + c0 .. 16 + c0
// + 3 (a1) of pixel r, bv their biases. MODE 0: + bias, ReLU, bfloat16;
// MODE 1: channel 0 + bias in float32 (the lanes with c0 = 0); MODE 2:
// bfloat16 times (act > 0). Four channels of a pixel are 8 contiguous bytes,
// stored by the lane itself.
template <int MODE>
__device__ __forceinline__ void conv_out(const f32x4& a0, const f32x4& a1, long r, int c0, const float (&bv)[2][4],
                                         const u16* __restrict__ act, u16* __restrict__ Y,
                                         float* __restrict__ Yf) {
    if constexpr (MODE == 1) {
        if (c0 == 0) Yf[r] = a0[0] + bv[0][0];
        return;
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const f32x4& a = cb ? a1 : a0;
        const int c = 16 * cb + c0;
        unsigned h[4];
        if constexpr (MODE == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) h[i] = f2bf(fmaxf(a[i] + bv[cb][i], 0.f));
        } else {
            const uint2 av = *reinterpret_cast<const uint2*>(act + r * kC + c);
            const u16 g[4] = {(u16)(av.x & 0xFFFFu), (u16)(av.x >> 16), (u16)(av.y & 0xFFFFu), (u16)(av.y >> 16)};
#pragma unroll
            for (int i = 0; i < 4; ++i) h[i] = bf2f(g[i]) > 0.f ? f2bf(a[i]) : 0u;
        }
        uint2 o;
        o.x = h[0] | (h[1] << 16);
        o.y = h[2] | (h[3] << 16);
        *reinterpret_cast<uint2*>(Y + r * kC + c) = o;
    }
}

// the biases of channels c0 .. c0 + 3 and 16 + c0 .. 16 + c0 + 3 (MODE 1:
// channel 0's only; MODE 2: none)
template <int MODE>
__device__ __forceinline__ void conv_bias(const float* __restrict__ bias, int c0, float (&bv)[2][4]) {
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[cb][i] = 0.f;
    if constexpr (MODE == 1) {
        bv[0][0] = bias[0];
    } else if constexpr (MODE == 0) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const float4 q = *reinterpret_cast<const float4*>(bias + 16 * cb + c0);
            bv[cb][0] = q.x;
            bv[cb][1] = q.y;
            bv[cb][2] = q.z;
            bv[cb][3] = q.w;
        }
    }
}

// The last layer has one output channel: its weight fragment for in-plane
// tap i = 3 ky + kx carries, as rows 0, 1, 2 of the left operand, the
// weights of taps (kz, ky, kx) for kz = 0, 1, 2 (rows 3 .. 15 zero). One
// product with an input plane then gives that plane's contributions to the
// three output planes it feeds, in rows 0 .. 2 (lane (pixel, 0), elements
// 0 .. 2). Each output is the sum, in order kz = 0, 1, 2, of its three
// in-plane chains, plus the bias.
__device__ __forceinline__ bf16x8 last_weights(const u16* __restrict__ Wl, int i, int mm, int kk) {
    if (mm < 3) return *reinterpret_cast<const bf16x8*>(Wl + (9 * mm + i) * kC + kk * 8);
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = __builtin_bit_cast(__bf16, (u16)0);
    return z;
}

// ---------------------------------------------------------------------------
// convolution on the matrix cores
// MODE 0: + bias, ReLU, bfloat16 out; MODE 1: + bias, float32 out of channel 0;
// MODE 2: bfloat16 out times (act > 0) (input gradient through the ReLU below)
template <int MODE, int DIM, bool PACK = false>
__global__ __launch_bounds__(kBlock) void k_nn_conv(const u16* __restrict__ X, const u16* __restrict__ Wl,
                                                    const float* __restrict__ bias,
                                                    const u16* __restrict__ act, u16* __restrict__ Y,
                                                    float* __restrict__ Yf, int D, int H, int W) {
    static_assert(!PACK || (DIM == 3 && MODE == 0), "the packed first layer is 3D, bias + ReLU");
    constexpr int TAPS = DIM == 3 ? 27 : 9;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int y = blockIdx.y, z = blockIdx.z;
    const int x0 = blockIdx.x * 64 + wave * 16;
    const int m = lane & 15, kg = lane >> 4;
    // first pixel of this wave's 16 (row y of plane z)
    const long row0 = ((long)z * H + y) * W + x0;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    if constexpr (MODE == 1 && DIM == 3) {
        // one output channel: per input plane z + kz - 1 the chain over the
        // nine in-plane taps, row kz of the packed product (last_weights)
        float run = 0.f;
#pragma unroll
        for (int kz = 0; kz < 3; ++kz) {
            const int zz = wrap_near(z + kz - 1, D);
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int ky = i / 3, kx = i % 3;
                const int yy = wrap_near(y + ky - 1, H), xx = wrap_near(x0 + m + kx - 1, W);
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(X + (((long)zz * H + yy) * W + xx) * kC + kg * 8);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(last_weights(Wl, i, m, kg), a, c, 0, 0, 0);
            }
            run = kz == 0 ? c[0] : run + c[kz];
        }
        if (kg == 0) Yf[row0 + m] = run + bias[0];
        return;
    }
    if constexpr (PACK) {
#pragma unroll
        for (int kz = 0; kz < 3; ++kz) {
            const int zz = wrap_near(z + kz - 1, D);
            bf16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                int ky, kx, ci;
                pack_tap(kg * 8 + e, ky, kx, ci);
                const int yy = wrap_near(y + ky - 1, H), xx = wrap_near(x0 + m + kx - 1, W);
                a[e] = __builtin_bit_cast(__bf16, X[(((long)zz * H + yy) * W + xx) * 8 + ci]);
            }
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pack_weights(Wl, kz, 0, m, kg), a, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pack_weights(Wl, kz, 1, m, kg), a, acc1, 0, 0, 0);
        }
    }
#pragma unroll
    for (int tap = 0; tap < (PACK ? 0 : TAPS); ++tap) {
        // tap = 9 kz + 3 ky + kx (kz = 1 in 2D): offsets k - 1 along each axis
        const int kz = DIM == 3 ? tap / 9 : 1, ky = (tap % 9) / 3, kx = tap % 3;
        const int zz = DIM == 3 ? wrap_near(z + kz - 1, D) : 0;
        const int yy = wrap_near(y + ky - 1, H), xx = wrap_near(x0 + m + kx - 1, W);
        bf16x8 a = *reinterpret_cast<const bf16x8*>(X + (((long)zz * H + yy) * W + xx) * kC + kg * 8);
        bf16x8 b0 = *reinterpret_cast<const bf16x8*>(Wl + ((m)*TAPS + tap) * kC + kg * 8);
        bf16x8 b1 = *reinterpret_cast<const bf16x8*>(Wl + ((16 + m) * TAPS + tap) * kC + kg * 8);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0, a, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b1, a, acc1, 0, 0, 0);
    }
    // the weights are the left operand: accumulator element i of lane (m, kg)
    // is channel 4 kg + i (acc0) / 16 + 4 kg + i (acc1) of pixel m
    float bv[2][4];
    conv_bias<MODE>(bias, 4 * kg, bv);
    conv_out<MODE>(acc0, acc1, row0 + m, 4 * kg, bv, act, Y, Yf);
}

// ---------------------------------------------------------------------------
// 3D convolution, tiled: a 512-lane workgroup owns a 64 x 8 pixel tile
// (x, y) over a range of planes. The layer's weights stay in LDS for the
// whole range; each input plane (the tile with a one-pixel halo) is staged in
// LDS once and feeds the three output planes it touches (kz = 0, 1, 2), so
// every plane is read from memory once per range and every A fragment once
// per (ky, kx). Wave w owns output row w of the tile: 4 blocks of 16 pixels x
// 2 blocks of 16 output channels, for 3 output planes in flight. Every
// accumulator receives its 27 taps in increasing tap order with the same
// operands as k_nn_conv (the packed first layer its three kz products; the
// one-channel last layer its three in-plane chains, added in kz order), so
// the two kernels give identical results.
constexpr int kTX = 64, kTY = 8, kTThreads = 512;
constexpr int kTRows = kTY + 2, kTPx = kTX + 2;
constexpr int kTPxs = 68;                         // LDS pixel stride (bank spread)
constexpr int kTPlane = kTRows * 4 * kTPxs;       // 16-byte units per staged plane
constexpr int kTW = 27 * 2 * 64;                  // 16-byte weight fragments
constexpr int kTWLoads = (kTW + kTThreads - 1) / kTThreads;

// operands of one (ky, kx) step: the input fragments of the wave's 4 pixel
// blocks and the weight fragments of the three taps (kz, ky, kx)
struct Conv3Ops {
    bf16x8 a[4];
    bf16x8 b[3][2];
};

__device__ __forceinline__ void conv3_load(Conv3Ops& o, const bf16x8* __restrict__ P,
                                           const bf16x8* __restrict__ Ws, int i, int w, int m, int kg,
                                           int lane) {
    const int ky = i / 3, kx = i % 3;
#pragma unroll
    for (int j = 0; j < 4; ++j) o.a[j] = P[((w + ky) * 4 + kg) * kTPxs + 16 * j + m + kx];
#pragma unroll
    for (int kz = 0; kz < 3; ++kz)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) o.b[kz][cb] = Ws[((9 * kz + i) * 2 + cb) * 64 + lane];
}

// bit kz of mask: the output plane this input plane feeds as tap plane kz
// lies in the range (a plane at either end of the march feeds fewer). The
// full form loads the operands of step i + 1 while the matrix cores work on
// step i.
template <int MODE, int R, bool FULL>
__device__ __forceinline__ void conv3_plane(const bf16x8* __restrict__ P, const bf16x8* __restrict__ Ws,
                                            f32x4 (&acc)[3][4][2], int w, int m, int kg, int lane, int mask) {
    static_assert(MODE != 1, "the one-channel last layer has its own plane step");
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[R][j][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // (the input-gradient form keeps the plain order: its epilogue leaves
    // no registers for a second operand set)
    if (FULL && MODE != 2) {
        Conv3Ops o[2];
        conv3_load(o[0], P, Ws, 0, w, m, kg, lane);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (i + 1 < 9) conv3_load(o[(i + 1) & 1], P, Ws, i + 1, w, m, kg, lane);
            __builtin_amdgcn_sched_barrier(0);
            const Conv3Ops& c = o[i & 1];
#pragma unroll
            for (int kz = 0; kz < 3; ++kz) {
                const int S = (R - kz + 3) % 3;
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[S][j][cb] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(c.b[kz][cb], c.a[j], acc[S][j][cb], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            bf16x8 a[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = P[((w + ky) * 4 + kg) * kTPxs + 16 * j + m + kx];
            // this plane is input plane kz of the output plane held in set (R - kz) mod 3
#pragma unroll
            for (int kz = 0; kz < 3; ++kz) {
                const int S = (R - kz + 3) % 3, tap = 9 * kz + 3 * ky + kx;
                if (!((mask >> kz) & 1)) continue;
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const bf16x8 b = Ws[(tap * 2 + cb) * 64 + lane];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[S][j][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[j], acc[S][j][cb], 0, 0, 0);
                }
            }
        }
    }
}

// the packed first layer on one staged plane: one input fragment per pixel
// block gathered from channel chunk 0 (off: the lane's eight element
// offsets, in 16-bit units), one product per (kz, output block)
template <int R, bool FULL>
__device__ __forceinline__ void conv3_plane_pack(const bf16x8* __restrict__ P, const bf16x8* __restrict__ Ws,
                                                 f32x4 (&acc)[3][4][2], int w, int m, int lane,
                                                 const int (&off)[8], int mask) {
    const u16* Pu = reinterpret_cast<const u16*>(P);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[R][j][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int base = ((w * 4) * kTPxs + 16 * j + m) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) a[j][e] = __builtin_bit_cast(__bf16, Pu[base + off[e]]);
    }
#pragma unroll
    for (int kz = 0; kz < 3; ++kz) {
        if (!FULL && !((mask >> kz) & 1)) continue;
        const int S = (R - kz + 3) % 3;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const bf16x8 b = Ws[(kz * 2 + cb) * 64 + lane];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[S][j][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[j], acc[S][j][cb], 0, 0, 0);
        }
    }
}

// the 64 pixels of one output row starting at pixel row0 (conv_out per
// block of 16; the biases are read here, where few registers are live)
template <int MODE>
__device__ __forceinline__ void conv3_store(const f32x4 (&a)[4][2], long row0, const float* __restrict__ bias,
                                            const u16* __restrict__ act, u16* __restrict__ Y,
                                            float* __restrict__ Yf, int m, int kg) {
    float bv[2][4];
    conv_bias<MODE>(bias, 4 * kg, bv);
#pragma unroll
    for (int j = 0; j < 4; ++j) conv_out<MODE>(a[j][0], a[j][1], row0 + 16 * j + m, 4 * kg, bv, act, Y, Yf);
}

template <int MODE, bool PACK = false>
__global__ __launch_bounds__(kTThreads) void k_nn_conv3_tiled(const u16* __restrict__ X,
                                                              const u16* __restrict__ Wl,
                                                              const float* __restrict__ bias,
                                                              const u16* __restrict__ act,
                                                              u16* __restrict__ Y, float* __restrict__ Yf,
                                                              int D, int H, int W, int ZR) {
    __shared__ bf16x8 Ws[kTW];
    __shared__ bf16x8 Ps[2][kTPlane];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 15, kg = lane >> 4;
    const int ntx = W / kTX, nty = H / kTY, nzr = (D + ZR - 1) / ZR;
    const int nb = ntx * nty * nzr, bid = blockIdx.x;
    // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous
    // range of tiles so that neighbouring tiles share halo rows in its L2
    const int wt = (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
    const int tx = wt % ntx, ty = (wt / ntx) % nty, zr = wt / (ntx * nty);
    const int x0 = tx * kTX, y0 = ty * kTY, z0 = zr * ZR;
    const int nz = min(ZR, D - z0), nt = nz + 2;  // input planes z0 - 1 .. z0 + nz
    const long HW = (long)H * W;

    static_assert(!PACK || MODE == 0, "the packed first layer is bias + ReLU");
    // weights: LDS fragment (tap, cb, lane) = Wl[cb 16 + m][tap][8 kg .. 8 kg + 7];
    // packed first layer: fragment (kz, cb, lane) of pack_weights
    if constexpr (PACK) {
        if (tid < 6 * 64) {
            const int l = tid & 63, tc = tid >> 6;
            Ws[tid] = pack_weights(Wl, tc >> 1, tc & 1, l & 15, l >> 4);
        }
    } else if constexpr (MODE == 1) {
        // last layer: fragment (i, lane) of last_weights
        for (int q = tid; q < 9 * 64; q += kTThreads) Ws[q] = last_weights(Wl, q >> 6, q & 15, (q & 63) >> 4);
    } else {
#pragma unroll
        for (int s = 0; s < kTWLoads; ++s) {
            const int q = tid + s * kTThreads;
            if (q < kTW) {
                const int l = q & 63, tc = q >> 6;
                const int tap = tc >> 1, cb = tc & 1, mm = l & 15, kk = l >> 4;
                Ws[q] = *reinterpret_cast<const bf16x8*>(Wl + ((cb * 16 + mm) * 27 + tap) * kC + kk * 8);
            }
        }
    }
    // packed first layer: the lane's eight input offsets (16-bit units) from
    // its pixel's chunk 0 in the staged plane
    int poff[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int ky, kx, ci;
        pack_tap(kg * 8 + e, ky, kx, ci);
        poff[e] = (ky * 4 * kTPxs + kx) * 8 + ci;
    }
    // plane staging: slot q = 16 bytes (chunk c of pixel px in halo row r;
    // the packed first layer reads chunk 0, channels 0 .. 7, only); slots
    // past the plane re-read slot 0 and are not stored
    constexpr int NCH = PACK ? 1 : 4, NSLOT = kTRows * kTPx * NCH;
    // 16-bit elements per input pixel: the packed first layer reads the
    // 8-channel form of the input
    constexpr int XS = PACK ? 8 : kC;
    constexpr int NLD = (NSLOT + kTThreads - 1) / kTThreads;
    int goff[NLD], loff[NLD];
#pragma unroll
    for (int s = 0; s < NLD; ++s) {
        int q = tid + s * kTThreads;
        const bool v = q < NSLOT;
        if (!v) q = 0;
        const int c = q % NCH, px = (q / NCH) % kTPx, r = (q / NCH) / kTPx;
        goff[s] = (wrap_near(y0 - 1 + r, H) * W + wrap_near(x0 - 1 + px, W)) * XS + c * 8;
        loff[s] = v ? (r * 4 + c) * kTPxs + px : -1;
    }
    bf16x8 pre[NLD];
    auto fetch = [&](int t) {
        const u16* base = X + (long)wrap_near(z0 - 1 + t, D) * HW * XS;
#pragma unroll
        for (int s = 0; s < NLD; ++s) pre[s] = *reinterpret_cast<const bf16x8*>(base + goff[s]);
    };
    auto commit = [&](int t) {
        bf16x8* P = Ps[t & 1];
#pragma unroll
        for (int s = 0; s < NLD; ++s)
            if (loff[s] >= 0) P[loff[s]] = pre[s];
    };
    fetch(0);
    commit(0);
    __syncthreads();

    f32x4 acc[3][4][2];
    // last layer: running sums of output planes t, t - 1, t - 2 (sets as acc)
    float run[3][4];
    // output row of this wave; pixel index of (z0 + u, y0 + wave, x0) is rowz + u H W
    const long rowz = ((long)z0 * H + y0 + wave) * W + x0;
    auto step = [&](auto rc, int t) {
        constexpr int R = decltype(rc)::value;
        const bool more = t + 1 < nt;
        if (more) fetch(t + 1);
        const int mask = (t < nz ? 1 : 0) | (t >= 1 && t <= nz ? 2 : 0) | (t >= 2 ? 4 : 0);
        if constexpr (MODE == 1) {
            f32x4 c[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            const bf16x8* P = Ps[t & 1];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int ky = i / 3, kx = i % 3;
                const bf16x8 b = Ws[i * 64 + lane];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        b, P[((wave + ky) * 4 + kg) * kTPxs + 16 * j + m + kx], c[j], 0, 0, 0);
            }
            // this plane is input plane kz of the output plane in set (R - kz) mod 3
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (mask & 1) run[R][j] = c[j][0];
                if (mask & 2) run[(R + 2) % 3][j] += c[j][1];
                if (mask & 4) run[(R + 1) % 3][j] += c[j][2];
            }
            if (t >= 2 && kg == 0) {
                const float b0 = bias[0];
#pragma unroll
                for (int j = 0; j < 4; ++j) Yf[rowz + (long)(t - 2) * HW + 16 * j + m] = run[(R + 1) % 3][j] + b0;
            }
        } else if constexpr (PACK) {
            if (mask == 7)
                conv3_plane_pack<R, true>(Ps[t & 1], Ws, acc, wave, m, lane, poff, 7);
            else
                conv3_plane_pack<R, false>(Ps[t & 1], Ws, acc, wave, m, lane, poff, mask);
        } else if (mask == 7) {
            conv3_plane<MODE, R, true>(Ps[t & 1], Ws, acc, wave, m, kg, lane, 7);
        } else {
            conv3_plane<MODE, R, false>(Ps[t & 1], Ws, acc, wave, m, kg, lane, mask);
        }
        // input plane t completes output plane t - 2 (set (R + 1) mod 3)
        if (MODE != 1 && t >= 2)
            conv3_store<MODE>(acc[(R + 1) % 3], rowz + (long)(t - 2) * HW, bias, act, Y, Yf, m, kg);
        if (more) commit(t + 1);
        __syncthreads();
    };
    for (int t = 0; t < nt; t += 3) {
        step(std::integral_constant<int, 0>{}, t);
        if (t + 1 < nt) step(std::integral_constant<int, 1>{}, t + 1);
        if (t + 2 < nt) step(std::integral_constant<int, 2>{}, t + 2);
    }
}

// ---------------------------------------------------------------------------
// loss: y (float32), target t = (p - p_prev) / s_p; gradient (2/N)(y - t) into
// channel 0 of G (bfloat16), per-block partial sums of (y - t)^2
__global__ void k_nn_loss(const float* __restrict__ y, const double* __restrict__ p,
                          const double* __restrict__ pp, const double* __restrict__ scale, long N,
                          u16* __restrict__ G, double* __restrict__ part) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    const double inv_sp = 1.0 / scale[1];
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        double t = (p[c] - (pp ? pp[c] : 0.0)) * inv_sp;
        double d = (double)y[c] - t;
        acc += d * d;
        uint4 q0;
        q0.x = f2bf((float)(2.0 * d / (double)N));
        q0.y = 0u;
        q0.z = 0u;
        q0.w = 0u;
        const uint4 z = {0u, 0u, 0u, 0u};
        uint4* o = reinterpret_cast<uint4*>(G + c * kC);
        o[0] = q0;
        o[1] = z;
        o[2] = z;
        o[3] = z;
    }
    double r = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][tap][ci] = sum_p G[p][co] X[p + off(tap)][ci], db[co] = sum_p G[p][co].
// A workgroup stages 64 gradient pixels of one row and the 3 (2D) or 9 (3D)
// input rows of 66 pixels they touch; its 4 (2D) or 12 (3D) waves own 9 of
// the 4 x taps (tap, co-block, ci-block) 16 x 16 tiles each.
template <int DIM>
__global__ __launch_bounds__(DIM == 3 ? 768 : 256) void k_nn_wgrad(const u16* __restrict__ G,
                                                                   const u16* __restrict__ X, int D,
                                                                   int H, int W, float* __restrict__ part) {
    constexpr int TAPS = DIM == 3 ? 27 : 9, ROWS = DIM == 3 ? 9 : 3;
    constexpr int NT = DIM == 3 ? 768 : 256, NWV = NT / 64;
    __shared__ u16 g_s[64][kC];
    __shared__ u16 x_s[ROWS][66][kC];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 15, kg = lane >> 4;
    const int segs_per_row = W / 64;
    const long nseg = (long)D * H * segs_per_row;
    f32x4 acc[9];
    for (int q = 0; q < 9; ++q) acc[q] = {0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;
    for (long sgi = blockIdx.x; sgi < nseg; sgi += gridDim.x) {
        const long row = sgi / segs_per_row;
        const int y = (int)(row % H), z = (int)(row / H), xs = (int)(sgi % segs_per_row) * 64;
        // stage 64 gradient pixels and the ROWS x 66 input pixels they touch
        for (int q = threadIdx.x; q < 64 * 4; q += NT) {
            int px = q >> 2, part8 = (q & 3) * 8;
            *reinterpret_cast<uint4*>(&g_s[px][part8]) =
                *reinterpret_cast<const uint4*>(G + ((row * W) + xs + px) * kC + part8);
        }
        for (int q = threadIdx.x; q < ROWS * 66 * 4; q += NT) {
            int r = q / (66 * 4), rem = q % (66 * 4);
            int px = rem >> 2, part8 = (rem & 3) * 8;
            int zz = DIM == 3 ? wrap_near(z + r / 3 - 1, D) : 0;
            int yy = wrap_near(y + r % 3 - 1, H), xx = wrap_near(xs + px - 1, W);
            *reinterpret_cast<uint4*>(&x_s[r][px][part8]) =
                *reinterpret_cast<const uint4*>(X + (((long)zz * H + yy) * W + xx) * kC + part8);
        }
        __syncthreads();
        if (threadIdx.x < kC) {
            float s = 0.f;
            for (int px = 0; px < 64; ++px) s += bf2f(g_s[px][threadIdx.x]);
            dbias += s;
        }
        // tiles t = wave + NWV j, j = 0..8: tap = t / 4, co block = (t / 2) & 1, ci block = t & 1
        for (int j = 0; j < 9; ++j) {
            const int t = wave + NWV * j;
            const int tap = t >> 2, cb = (t >> 1) & 1, nb = t & 1;
            const int r = tap / 3, kx = tap % 3;  // input row (3 kz + ky) and x offset
            for (int kk = 0; kk < 2; ++kk) {
                bf16x8 a, b;
                const int p0 = kk * 32 + kg * 8;
                for (int e = 0; e < 8; ++e) {
                    u16 ga = g_s[p0 + e][cb * 16 + m];
                    u16 xb = x_s[r][p0 + e + kx][nb * 16 + m];
                    a[e] = __builtin_bit_cast(__bf16, ga);
                    b[e] = __builtin_bit_cast(__bf16, xb);
                }
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float* out = part + (long)blockIdx.x * psize(TAPS);
    for (int j = 0; j < 9; ++j) {
        const int t = wave + NWV * j;
        const int tap = t >> 2, cb = (t >> 1) & 1, nb = t & 1;
        for (int i = 0; i < 4; ++i) {
            int co = cb * 16 + 4 * kg + i, ci = nb * 16 + m;
            out[(co * TAPS + tap) * kC + ci] = acc[j][i];
        }
    }
    if (threadIdx.x < kC) out[wsize(TAPS) + threadIdx.x] = dbias;
}

// grad[q] += sum over blocks of part[b][q], in block order
__global__ void k_nn_grad_reduce(const float* __restrict__ part, int nb, int psz, float* __restrict__ grad) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= psz) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += part[(long)b * psz + q];
    grad[q] += s;
}

// Adam on the float32 master parameters of one layer; refresh the bfloat16
// copies (Wl and the flipped transpose Wt) and the float32 bias
__global__ void k_nn_adam(float* __restrict__ master, float* __restrict__ mom, float* __restrict__ vel,
                          float* __restrict__ grad, float scale, float lr, float c1, float c2,
                          u16* __restrict__ Wl, u16* __restrict__ Wt, float* __restrict__ bias,
                          int taps) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= psize(taps)) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float g = grad[q] * scale;
    float mq = b1 * mom[q] + (1.f - b1) * g;
    float vq = b2 * vel[q] + (1.f - b2) * g * g;
    mom[q] = mq;
    vel[q] = vq;
    float mh = mq / c1, vh = vq / c2;
    float w = master[q] - lr * mh / (sqrtf(vh) + eps);
    master[q] = w;
    grad[q] = 0.f;
    if (q < wsize(taps)) {
        int co = q / (taps * kC), rem = q % (taps * kC), tap = rem / kC, ci = rem % kC;
        u16 h = f2bf(w);
        Wl[q] = h;
        Wt[(ci * taps + (taps - 1 - tap)) * kC + co] = h;
    } else {
        bias[q - wsize(taps)] = w;
    }
}

// refresh the bfloat16 copies from the master parameters
__global__ void k_nn_publish(const float* __restrict__ master, u16* __restrict__ Wl,
                             u16* __restrict__ Wt, float* __restrict__ bias, int taps) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= psize(taps)) return;
    float w = master[q];
    if (q < wsize(taps)) {
        int co = q / (taps * kC), rem = q % (taps * kC), tap = rem / kC, ci = rem % kC;
        u16 h = f2bf(w);
        Wl[q] = h;
        Wt[(ci * taps + (taps - 1 - tap)) * kC + co] = h;
    } else {
        bias[q - wsize(taps)] = w;
    }
}

// p0 = p_prev + s_p * y
__global__ void k_nn_guess(const float* __restrict__ y, const double* __restrict__ pp,
                           const double* __restrict__ scale, long N, double* __restrict__ p0) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    p0[c] = (pp ? pp[c] : 0.0) + scale[1] * (double)y[c];
}

}  // namespace ib

using namespace ib;

struct ib_nn {
    int dim = 2, taps = 9;
    int D = 1, H = 0, W = 0;
    double h = 0.0;
    long N = 0;
    u16* act[kLayers] = {};   // layer inputs (act[0] = normalised input)
    u16* act0c = nullptr;     // 3D: the normalised input in 8 channels (the packed first layer)
    float* yf = nullptr;      // network output
    u16* g[2] = {};           // gradient ping-pong
    u16* Wl = nullptr;        // kLayers * wsize(taps)
    u16* Wt = nullptr;
    float* bias = nullptr;    // kLayers * kC
    float* master = nullptr;  // kLayers * psize(taps)
    float* mom = nullptr;
    float* vel = nullptr;
    float* grad = nullptr;
    float* part = nullptr;    // kGradBlocks * psize(taps)
    double* red = nullptr;    // reductions
    double* scale = nullptr;  // s_b, s_p, s_r
    double* host = nullptr;   // pinned
    int step = 0;
    int conv = IB_NN_CONV_AUTO;
};

// planes per workgroup of the tiled kernel: 64 (two planes of halo per 64),
// halved while the grid has fewer than 512 workgroups (two rounds of one
// workgroup per CU on 256 CUs; at least 4)
static int conv3_range(const ib_nn* n) {
    const long xy = (long)(n->W / kTX) * (n->H / kTY);
    int zr = 64;
    while (zr > 4 && xy * ((n->D + zr - 1) / zr) < 512) zr /= 2;
    return zr;
}

static bool conv3_tiled(const ib_nn* n) {
    return n->dim == 3 && n->conv == IB_NN_CONV_AUTO && n->W % kTX == 0 && n->H % kTY == 0;
}

// one convolution layer: MODE 0 (bias, ReLU), 1 (float32 channel 0) or 2
// (input gradient through the ReLU mask of act)
// PACK: the first layer (3 input channels) with its in-plane products packed (3D)
template <int MODE, bool PACK = false>
static void nn_conv(const ib_nn* n, const u16* X, const u16* Wl, const float* bias, const u16* act, u16* Y,
                    float* Yf, hipStream_t st) {
    if (conv3_tiled(n)) {
        const int zr = conv3_range(n);
        const int nb = (n->W / kTX) * (n->H / kTY) * ((n->D + zr - 1) / zr);
        hipLaunchKernelGGL((k_nn_conv3_tiled<MODE, PACK>), dim3(nb), dim3(kTThreads), 0, st, X, Wl, bias, act, Y,
                           Yf, n->D, n->H, n->W, zr);
        return;
    }
    dim3 grid(n->W / 64, n->H, n->D);
    if (n->dim == 3)
        hipLaunchKernelGGL((k_nn_conv<MODE, 3, PACK>), grid, dim3(kBlock), 0, st, X, Wl, bias, act, Y, Yf, n->D,
                           n->H, n->W);
    else
        hipLaunchKernelGGL((k_nn_conv<MODE, 2>), grid, dim3(kBlock), 0, st, X, Wl, bias, act, Y, Yf, n->D, n->H,
                           n->W);
}

// train: the 32-channel input is written as well (the first layer's weight
// gradient reads it; in 3D the forward reads the 8-channel form only)
static int nn_forward(ib_nn* n, const double* b, const double* H, const double* pp, double rin,
                      double rout, bool train, hipStream_t st) {
    const int nb = 1024;
    double h2 = n->h * n->h;
    hipLaunchKernelGGL(k_nn_stats, dim3(nb), dim3(kBlock), 0, st, b, H, pp, n->N, h2, rin, rout, n->red);
    hipLaunchKernelGGL(k_nn_scales, dim3(1), dim3(kBlock), 0, st, n->red, nb, n->N, n->scale);
    if (n->dim == 3)
        hipLaunchKernelGGL(k_nn_input<1>, dim3(grid_for(n->N)), dim3(kBlock), 0, st, b, H, pp, n->N, h2, rin,
                           rout, n->scale, n->act0c);
    if (n->dim == 2 || train)
        hipLaunchKernelGGL(k_nn_input<4>, dim3(grid_for(4 * n->N)), dim3(kBlock), 0, st, b, H, pp, n->N, h2,
                           rin, rout, n->scale, n->act[0]);
    const long ws = wsize(n->taps);
    for (int l = 0; l < kLayers; ++l) {
        const u16* Wl = n->Wl + (long)l * ws;
        const float* bias = n->bias + l * kC;
        if (l == kLayers - 1)
            nn_conv<1>(n, n->act[l], Wl, bias, nullptr, nullptr, n->yf, st);
        else if (l == 0 && n->dim == 3)
            nn_conv<0, true>(n, n->act0c, Wl, bias, nullptr, n->act[l + 1], nullptr, st);
        else
            nn_conv<0>(n, n->act[l], Wl, bias, nullptr, n->act[l + 1], nullptr, st);
    }
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// forward + backward of one sample, gradients added to n->grad; loss partials
// summed into *loss (syncs)
static int nn_backward(ib_nn* n, const double* b, const double* H, const double* pp, const double* p,
                       double rin, double rout, double* loss, hipStream_t st) {
    IB_TRY(nn_forward(n, b, H, pp, rin, rout, true, st));
    const int nb = 1024;
    hipLaunchKernelGGL(k_nn_loss, dim3(nb), dim3(kBlock), 0, st, n->yf, p, pp, n->scale, n->N, n->g[0],
                       n->red);
    IB_TRY(device_sum(n->red, nb, n->red + 4 * 1024, st));
    const int ps = psize(n->taps);
    const long ws = wsize(n->taps);
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        // n->g[cur] holds layer l's pre-activation gradient (bfloat16)
        if (n->dim == 3)
            hipLaunchKernelGGL((k_nn_wgrad<3>), dim3(kGradBlocks), dim3(768), 0, st, n->g[cur], n->act[l],
                               n->D, n->H, n->W, n->part);
        else
            hipLaunchKernelGGL((k_nn_wgrad<2>), dim3(kGradBlocks), dim3(256), 0, st, n->g[cur], n->act[l],
                               n->D, n->H, n->W, n->part);
        hipLaunchKernelGGL(k_nn_grad_reduce, dim3(grid_for(ps)), dim3(kBlock), 0, st, n->part,
                           kGradBlocks, ps, n->grad + (long)l * ps);
        if (l > 0)
            nn_conv<2>(n, n->g[cur], n->Wt + (long)l * ws, nullptr, n->act[l], n->g[1 - cur], nullptr, st);
        cur = 1 - cur;
    }
    IB_HIP(hipGetLastError());
    IB_HIP(hipMemcpyAsync(n->host, n->red + 4 * 1024, sizeof(double), hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    *loss = n->host[0] / (double)n->N;
    return IB_OK;
}

static void nn_free(ib_nn* n) {
    if (!n) return;
    for (int l = 0; l < kLayers; ++l) (void)hipFree(n->act[l]);
    void* ptrs[] = {n->act0c, n->yf, n->g[0], n->g[1], n->Wl, n->Wt, n->bias, n->master, n->mom,
                    n->vel, n->grad, n->part, n->red, n->scale};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (n->host) (void)hipHostFree(n->host);
    delete n;
}

extern "C" int ib_nn_param_count(int dim) {
    if (dim != 2 && dim != 3) return 0;
    const int taps = dim == 3 ? 27 : 9;
    int t = 0;
    for (int l = 0; l < kLayers; ++l) t += kChan[l + 1] * kChan[l] * taps + kChan[l + 1];
    return t;
}

extern "C" int ib_nn_create(const ib_grid* g, ib_nn** out) {
    IB_CHECK(g && out, IB_EINVAL, "ib_nn_create: null argument");
    IB_CHECK(g->dim == 2 || g->dim == 3, IB_EINVAL, "ib_nn_create: dim must be 2 or 3");
    IB_CHECK(g->n[0] % 64 == 0 && g->n[0] >= 64 && g->n[1] >= 1 && (g->dim == 2 || g->n[2] >= 1),
             IB_EINVAL, "ib_nn_create: n[0] must be a multiple of 64");
    ib_nn* n = new ib_nn();
    n->dim = g->dim;
    n->taps = g->dim == 3 ? 27 : 9;
    n->W = g->n[0];
    n->H = g->n[1];
    n->D = g->dim == 3 ? g->n[2] : 1;
    n->h = g->h;
    n->N = (long)n->W * n->H * n->D;
    bool ok = true;
    auto alloc = [&](void** p, size_t bytes) {
        if (ok && hipMalloc(p, bytes) != hipSuccess) ok = false;
    };
    for (int l = 0; l < kLayers; ++l) alloc((void**)&n->act[l], n->N * kC * sizeof(u16));
    if (n->dim == 3) alloc((void**)&n->act0c, n->N * 8 * sizeof(u16));
    alloc((void**)&n->yf, n->N * sizeof(float));
    alloc((void**)&n->g[0], n->N * kC * sizeof(u16));
    alloc((void**)&n->g[1], n->N * kC * sizeof(u16));
    const size_t WS = wsize(n->taps), PS = psize(n->taps);
    alloc((void**)&n->Wl, kLayers * WS * sizeof(u16));
    alloc((void**)&n->Wt, kLayers * WS * sizeof(u16));
    alloc((void**)&n->bias, kLayers * kC * sizeof(float));
    alloc((void**)&n->master, kLayers * PS * sizeof(float));
    alloc((void**)&n->mom, kLayers * PS * sizeof(float));
    alloc((void**)&n->vel, kLayers * PS * sizeof(float));
    alloc((void**)&n->grad, kLayers * PS * sizeof(float));
    alloc((void**)&n->part, (size_t)kGradBlocks * PS * sizeof(float));
    alloc((void**)&n->red, 8 * 1024 * sizeof(double));
    alloc((void**)&n->scale, 4 * sizeof(double));
    if (ok && hipHostMalloc((void**)&n->host, 8 * sizeof(double)) != hipSuccess) ok = false;
    if (!ok) {
        nn_free(n);
        return fail(IB_ENOMEM, "ib_nn_create: out of memory");
    }
    size_t pb = kLayers * PS * sizeof(float);
    if (hipMemset(n->master, 0, pb) != hipSuccess || hipMemset(n->mom, 0, pb) != hipSuccess ||
        hipMemset(n->vel, 0, pb) != hipSuccess || hipMemset(n->grad, 0, pb) != hipSuccess ||
        hipMemset(n->Wl, 0, kLayers * WS * sizeof(u16)) != hipSuccess ||
        hipMemset(n->Wt, 0, kLayers * WS * sizeof(u16)) != hipSuccess ||
        hipMemset(n->bias, 0, kLayers * kC * sizeof(float)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        nn_free(n);
        return fail(IB_EHIP, "ib_nn_create: initialisation failed");
    }
    *out = n;
    return IB_OK;
}

extern "C" void ib_nn_destroy(ib_nn* n) { nn_free(n); }

extern "C" int ib_nn_set_conv(ib_nn* n, int kind) {
    IB_CHECK(n, IB_EINVAL, "ib_nn_set_conv: null network");
    IB_CHECK(kind == IB_NN_CONV_AUTO || kind == IB_NN_CONV_DIRECT, IB_EINVAL, "ib_nn_set_conv: unknown kind");
    n->conv = kind;
    return IB_OK;
}

long nn_cells(const ib_nn* nn) { return nn ? nn->N : 0; }

// params: host float32, per layer W[co][ci][(kz)][ky][kx] (unpadded channel counts) then b[co]
extern "C" int ib_nn_set_params(ib_nn* n, const float* params, int count) {
    IB_CHECK(n && params, IB_EINVAL, "ib_nn_set_params: null argument");
    IB_CHECK(count == ib_nn_param_count(n->dim), IB_EINVAL, "ib_nn_set_params: wrong parameter count");
    const int taps = n->taps, PS = psize(taps), WS = wsize(taps);
    std::vector<float> pad((size_t)kLayers * PS, 0.f);
    const float* src = params;
    for (int l = 0; l < kLayers; ++l) {
        int ci_n = kChan[l], co_n = kChan[l + 1];
        float* dst = pad.data() + (size_t)l * PS;
        for (int co = 0; co < co_n; ++co)
            for (int ci = 0; ci < ci_n; ++ci)
                for (int tap = 0; tap < taps; ++tap) dst[(co * taps + tap) * kC + ci] = *src++;
        for (int co = 0; co < co_n; ++co) dst[WS + co] = *src++;
    }
    IB_HIP(hipMemcpy(n->master, pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice));
    for (int l = 0; l < kLayers; ++l)
        hipLaunchKernelGGL(k_nn_publish, dim3(grid_for(PS)), dim3(kBlock), 0, 0,
                           n->master + (long)l * PS, n->Wl + (long)l * WS, n->Wt + (long)l * WS,
                           n->bias + l * kC, taps);
    IB_HIP(hipMemset(n->mom, 0, kLayers * PS * sizeof(float)));
    IB_HIP(hipMemset(n->vel, 0, kLayers * PS * sizeof(float)));
    IB_HIP(hipDeviceSynchronize());
    n->step = 0;
    return IB_OK;
}

static int unpad(const std::vector<float>& pad, int taps, float* params) {
    const int PS = psize(taps), WS = wsize(taps);
    float* dst = params;
    for (int l = 0; l < kLayers; ++l) {
        int ci_n = kChan[l], co_n = kChan[l + 1];
        const float* src = pad.data() + (size_t)l * PS;
        for (int co = 0; co < co_n; ++co)
            for (int ci = 0; ci < ci_n; ++ci)
                for (int tap = 0; tap < taps; ++tap) *dst++ = src[(co * taps + tap) * kC + ci];
        for (int co = 0; co < co_n; ++co) *dst++ = src[WS + co];
    }
    return IB_OK;
}

extern "C" int ib_nn_get_params(ib_nn* n, float* params, int count) {
    IB_CHECK(n && params, IB_EINVAL, "ib_nn_get_params: null argument");
    IB_CHECK(count == ib_nn_param_count(n->dim), IB_EINVAL, "ib_nn_get_params: wrong parameter count");
    std::vector<float> pad((size_t)kLayers * psize(n->taps));
    IB_HIP(hipDeviceSynchronize());
    IB_HIP(hipMemcpy(pad.data(), n->master, pad.size() * sizeof(float), hipMemcpyDeviceToHost));
    return unpad(pad, n->taps, params);
}

extern "C" int ib_nn_predict(ib_nn* n, const double* b, const double* H, const double* p_prev,
                             double rho_in, double rho_out, double* p0, void* stream) {
    IB_CHECK(n && b && H && p0, IB_EINVAL, "ib_nn_predict: null argument");
    hipStream_t st = (hipStream_t)stream;
    IB_TRY(nn_forward(n, b, H, p_prev, rho_in, rho_out, false, st));
    hipLaunchKernelGGL(k_nn_guess, dim3(grid_for(n->N)), dim3(kBlock), 0, st, n->yf, p_prev, n->scale,
                       n->N, p0);
    IB_HIP(hipGetLastError());
    return IB_OK;
}

extern "C" int ib_nn_gradients(ib_nn* n, const double* b, const double* H, const double* p_prev,
                               const double* p, double rho_in, double rho_out, float* grads_host,
                               int count, double* loss, void* stream) {
    IB_CHECK(n && b && H && p && loss, IB_EINVAL, "ib_nn_gradients: null argument");
    IB_CHECK(!grads_host || count == ib_nn_param_count(n->dim), IB_EINVAL, "ib_nn_gradients: count");
    hipStream_t st = (hipStream_t)stream;
    const size_t pbytes = (size_t)kLayers * psize(n->taps) * sizeof(float);
    IB_HIP(hipMemsetAsync(n->grad, 0, pbytes, st));
    IB_TRY(nn_backward(n, b, H, p_prev, p, rho_in, rho_out, loss, st));
    if (grads_host) {
        std::vector<float> pad((size_t)kLayers * psize(n->taps));
        IB_HIP(hipMemcpyAsync(pad.data(), n->grad, pbytes, hipMemcpyDeviceToHost, st));
        IB_HIP(hipStreamSynchronize(st));
        unpad(pad, n->taps, grads_host);
    }
    IB_HIP(hipMemsetAsync(n->grad, 0, pbytes, st));
    return IB_OK;
}

extern "C" int ib_nn_train_step(ib_nn* n, int count, const double* const* b, const double* const* H,
                                const double* const* p_prev, const double* const* p, double rho_in,
                                double rho_out, float lr, double* loss, void* stream) {
    IB_CHECK(n && b && H && p && loss && count > 0, IB_EINVAL, "ib_nn_train_step: bad argument");
    hipStream_t st = (hipStream_t)stream;
    double tot = 0.0;
    for (int s = 0; s < count; ++s) {
        double l = 0.0;
        IB_TRY(nn_backward(n, b[s], H[s], p_prev ? p_prev[s] : nullptr, p[s], rho_in, rho_out, &l, st));
        tot += l;
    }
    n->step += 1;
    float c1 = 1.f - powf(0.9f, (float)n->step), c2 = 1.f - powf(0.999f, (float)n->step);
    const int PS = psize(n->taps), WS = wsize(n->taps);
    for (int l = 0; l < kLayers; ++l)
        hipLaunchKernelGGL(k_nn_adam, dim3(grid_for(PS)), dim3(kBlock), 0, st, n->master + (long)l * PS,
                           n->mom + (long)l * PS, n->vel + (long)l * PS, n->grad + (long)l * PS,
                           1.f / (float)count, lr, c1, c2, n->Wl + (long)l * WS, n->Wt + (long)l * WS,
                           n->bias + l * kC, n->taps);
    IB_HIP(hipGetLastError());
    *loss = tot / count;
    return IB_OK;
}
