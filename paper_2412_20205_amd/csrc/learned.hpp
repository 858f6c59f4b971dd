// Learned smoother: a 3-layer 3x3 convolutional network (1 -> 16 -> 16 -> 1
// channels, ReLU, zero "same" padding, no biases) applied on a level's index
// grid, y = N(D^{-1} r / sigma), x += sigma * y, replacing the first
// pre-smoothing sweep of Algorithm 2's cycle on that level.
//
// Precision: BF16 weights; layer 1 and 3 on VALU in FP32; layer 2 as a GEMM on
// v_mfma_f32_16x16x16_bf16 (BF16 operands: layer-1 activations rounded to
// BF16, FP32 accumulation).  Training kernels use the same MFMA shape for the
// weight gradient of layer 2 (reduction over pixels) and for the input
// gradient of layer 2; the layer-2 output gradient is rounded to BF16 for them.
//
// Tiles: a workgroup of 256 threads produces a 16 x 16 output tile; it holds
// the input on 22 x 22 pixels, layer-1 activations on 20 x 20 (BF16) and
// layer-2 activations on 18 x 18 (FP32) in LDS.
//
// Canonical weight layout (also the ABI layout): W1[c][tap] (16 x 9),
// W2[co][ci][tap] (16 x 16 x 9), W3[ci][tap] (16 x 9), tap = 3 dy + dx,
// concatenated (2592 values).
#pragma once

#include "common.hpp"

namespace igamg {

constexpr int kLC = 16;
constexpr int kLW1 = 144, kLW2 = 2304, kLW3 = 144;
constexpr int kLWeights = kLW1 + kLW2 + kLW3;
constexpr int kLTile = 16;
constexpr int kLThreads = 256;

typedef short __attribute__((ext_vector_type(4))) bf16x4;
typedef float __attribute__((ext_vector_type(4))) floatx4;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Device weight set of one level: canonical BF16 plus the two MFMA B-operand
// layouts of W2 ([tap][co][ci] for the forward product, [tap][ci][co] for the
// input gradient).
struct LearnedW {
    const uint16_t* w;     // canonical, kLWeights
    const uint16_t* w2f;   // [tap][co][ci]
    const uint16_t* w2b;   // [tap][ci][co]
};

// One image seen by the network: z (height x width, row-major), the level it
// belongs to (n) and the level coordinates of its pixel (0, 0).
struct LImage {
    const float* z;
    int width, height;
    int n;
    int off_i, off_j;
};

__device__ __forceinline__ bool l_inside(const LImage& im, int pj, int pi) {
    int gj = pj + im.off_j, gi = pi + im.off_i;
    return pj >= 0 && pj < im.height && pi >= 0 && pi < im.width && gj >= 0 && gj < im.n &&
           gi >= 0 && gi < im.n;
}

struct LShared {
    float z[22 * 22];
    alignas(16) uint16_t h1[20 * 20 * kLC];
    alignas(16) float h2[18 * 18 * kLC];
    alignas(16) float w1t[kLW1];  // layer-1 weights tap-major: w1t[tap * 16 + c]
    alignas(16) float w3t[kLW3];  // layer-3 weights tap-major: w3t[tap * 16 + ci]
};

// Forward pass of one 16x16 output tile with origin (tj0, ti0); zscale
// multiplies the input.  Leaves z, h1, h2 in LDS and returns y of this
// thread's output pixel (threadIdx.x = 16 oy + ox).
__device__ inline float l_forward_tile(const LImage& im, const LearnedW& W, int tj0, int ti0,
                                       float zscale, LShared& S) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int t = tid; t < kLW1; t += kLThreads) S.w1t[(t % 9) * kLC + t / 9] = bf16_to_f32(W.w[t]);
    for (int t = tid; t < kLW3; t += kLThreads)
        S.w3t[(t % 9) * kLC + t / 9] = bf16_to_f32(W.w[kLW1 + kLW2 + t]);
    for (int t = tid; t < 22 * 22; t += kLThreads) {
        int pj = tj0 - 3 + t / 22, pi = ti0 - 3 + t % 22;
        S.z[t] = l_inside(im, pj, pi) ? im.z[(size_t)pj * im.width + pi] * zscale : 0.f;
    }
    __syncthreads();
    // layer 1 (VALU): h1 on 20 x 20, 16 channels, ReLU, zero outside the domain.
    // Each channel sums its taps in tap order; weights come 4 channels per
    // 16-byte LDS read, the 16 BF16 outputs leave in two 16-byte writes.
    for (int p = tid; p < 400; p += kLThreads) {
        int py = p / 20, px = p % 20;
        bool in = l_inside(im, tj0 - 2 + py, ti0 - 2 + px);
        float zz[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) zz[tap] = S.z[(py + tap / 3) * 22 + px + tap % 3];
        float a[kLC];
#pragma unroll
        for (int c = 0; c < kLC; ++c) a[c] = 0.f;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const floatx4* wv = reinterpret_cast<const floatx4*>(&S.w1t[tap * kLC]);
#pragma unroll
            for (int q = 0; q < kLC / 4; ++q) {
                const floatx4 w = wv[q];
#pragma unroll
                for (int e = 0; e < 4; ++e) a[4 * q + e] = fmaf(w[e], zz[tap], a[4 * q + e]);
            }
        }
        uint32_t pk[kLC / 2];
#pragma unroll
        for (int c2 = 0; c2 < kLC / 2; ++c2) {
            uint32_t lo = f32_to_bf16(in ? fmaxf(a[2 * c2], 0.f) : 0.f);
            uint32_t hi = f32_to_bf16(in ? fmaxf(a[2 * c2 + 1], 0.f) : 0.f);
            pk[c2] = lo | (hi << 16);
        }
        uint4* dst = reinterpret_cast<uint4*>(&S.h1[p * kLC]);
        dst[0] = uint4{pk[0], pk[1], pk[2], pk[3]};
        dst[1] = uint4{pk[4], pk[5], pk[6], pk[7]};
    }
    __syncthreads();
    // layer 2 (MFMA 16x16x16 BF16): rows = 16 pixels of the 18 x 18 region,
    // K = (tap, ci), N = co
    bf16x4 bw[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const uint16_t* src = W.w2f + ((size_t)tap * kLC + (lane & 15)) * kLC + 4 * (lane >> 4);
        bw[tap] = bf16x4{(short)src[0], (short)src[1], (short)src[2], (short)src[3]};
    }
    for (int g = wave; g < 21; g += kLThreads / 64) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        int pa = g * 16 + (lane & 15);  // A row: pixel of the 18x18 grid
        bool va = pa < 324;
        int qy = va ? pa / 18 : 0, qx = va ? pa % 18 : 0;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            bf16x4 a = {0, 0, 0, 0};
            if (va)
                a = *reinterpret_cast<const bf16x4*>(
                    &S.h1[((qy + tap / 3) * 20 + qx + tap % 3) * kLC + 4 * (lane >> 4)]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[tap], acc, 0, 0, 0);
        }
        int co = lane & 15;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int p = g * 16 + 4 * (lane >> 4) + j;
            if (p < 324) {
                bool in = l_inside(im, tj0 - 1 + p / 18, ti0 - 1 + p % 18);
                S.h2[p * kLC + co] = in ? fmaxf(acc[j], 0.f) : 0.f;
            }
        }
    }
    __syncthreads();
    // layer 3 (VALU)
    int oy = tid >> 4, ox = tid & 15;
    float y = 0.f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const floatx4* h = reinterpret_cast<const floatx4*>(&S.h2[((oy + tap / 3) * 18 + ox + tap % 3) * kLC]);
        const floatx4* w = reinterpret_cast<const floatx4*>(&S.w3t[tap * kLC]);
#pragma unroll
        for (int q = 0; q < kLC / 4; ++q) {
            const floatx4 hv = h[q], wv = w[q];
#pragma unroll
            for (int e = 0; e < 4; ++e) y = fmaf(wv[e], hv[e], y);
        }
    }
    return y;
}

// Inference on a whole level: x_I += sigma * N(z / sigma)_I, with
// (three waves per SIMD: at most 168 VGPRs, three workgroups per CU)
// sigma = scal[0] (skipped when sigma <= 0), or y written to yout.
template <typename T>
__global__ void __launch_bounds__(kLThreads, 3) k_learned_apply(LImage im, LearnedW W,
                                                             const double* __restrict__ sigma_dev,
                                                             T* __restrict__ x,
                                                             float* __restrict__ yout) {
    __shared__ LShared S;
    double sg = sigma_dev ? *sigma_dev : 1.0;
    if (!(sg > 0.0)) return;
    int tiles = (im.width + kLTile - 1) / kLTile;
    int tj0 = (blockIdx.x / tiles) * kLTile, ti0 = (blockIdx.x % tiles) * kLTile;
    float y = l_forward_tile(im, W, tj0, ti0, (float)(1.0 / sg), S);
    int pj = tj0 + (threadIdx.x >> 4), pi = ti0 + (threadIdx.x & 15);
    if (pj < im.height && pi < im.width && l_inside(im, pj, pi)) {
        size_t I = (size_t)pj * im.width + pi;
        if (yout)
            yout[I] = y;
        else
            x[I] = x[I] + (T)(sg * (double)y);
    }
}

// ---- inference with every layer on the matrix cores -------------------------
// One workgroup per TL x TL output tile, all three layers as MFMA products in
// the transposed form D[channel or tap][pixel] = W x patch^T, 16 pixels per
// product:
//   layer 1: h1[ch][px] = sum_tap W1[ch][tap] z[px + tap]; FP32 MFMA 16x16x4
//            (K = taps, 3 products, taps 9..11 zero), ReLU, zero outside the
//            domain, rounded to BF16 into LDS ([pixel][channel]);
//   layer 2: h2[co][px] = sum_{tap,ci} W2[co][ci][tap] h1[px + tap][ci];
//            BF16 MFMA 16x16x32 (K = 16 tap + ci, 5 products, tap 9 zero),
//            FP32 accumulation, ReLU and the domain mask in registers;
//   layer 3: u[tap][px] = sum_ci W3[ci][tap] h2[ci][px] straight from those
//            registers (FP32 MFMA 16x16x4, 4 products over the channel groups),
//            then y[px] = sum_tap u[tap][px + tap] from LDS.
// Layer 1 and 3 arithmetic stays FP32 and layer 2's operands BF16, as in the
// VALU/MFMA kernel above (results agree up to FP32 summation order).
// MFMA operand layouts (lane l, g = l / 16): 16x16x4 f32: A[l%16][g],
// B[g][l%16]; 16x16x32 bf16: A[l%16][8g + e], B[8g + e][l%16], e = 0..7;
// D[4g + j][l%16], j = 0..3, for both.
//
// The weights reach the kernel as per-lane MFMA A-operand records, written
// whenever the canonical weights change: FP32 mf32[l][8] = (a1[0..2], a3[0..3],
// 0) and BF16 mfbf[l][5][8] = a2[m][e], zero where a tap is >= 9 or a row is
// no tap.  Inside a tile every load is unconditional (clamped addresses), so
// no memory wait sits on a branch, and each wave interleaves two 16-pixel
// groups so that two independent MFMA chains are in flight.
typedef __bf16 lbf16x8 __attribute__((ext_vector_type(8)));
constexpr int kLMf32 = 64 * 8;      // floats of the FP32 records
constexpr int kLMfBf = 64 * 5 * 8;  // BF16 values of the layer-2 records

// Record positions of canonical weight k (-1: none), for the writers below.
__device__ __forceinline__ void l_mf_slot(int k, int& f32_slot, int& bf_slot) {
    f32_slot = -1;
    bf_slot = -1;
    if (k < kLW1) {
        const int ch = k / 9, tap = k % 9;
        f32_slot = (ch + 16 * (tap % 4)) * 8 + tap / 4;
    } else if (k < kLW1 + kLW2) {
        const int e2 = k - kLW1, co = e2 / (kLC * 9), ci = (e2 / 9) % kLC, tap = e2 % 9;
        const int g = 2 * (tap % 2) + ci / 8;
        bf_slot = ((co + 16 * g) * 5 + tap / 2) * 8 + ci % 8;
    } else if (k < kLWeights) {
        const int e3 = k - kLW1 - kLW2, ci = e3 / 9, tap = e3 % 9;
        f32_slot = (tap + 16 * (ci / 4)) * 8 + 3 + ci % 4;
    }
}

__device__ __forceinline__ bool l_row_in(const LImage& im, int pj) {
    const int gj = pj + im.off_j;
    return pj >= 0 && pj < im.height && gj >= 0 && gj < im.n;
}
__device__ __forceinline__ bool l_col_in(const LImage& im, int pi) {
    const int gi = pi + im.off_i;
    return pi >= 0 && pi < im.width && gi >= 0 && gi < im.n;
}
// Two FP32 values to BF16 (round to nearest even), packed low | high << 16.
__device__ __forceinline__ uint32_t l_pack_bf16(float lo, float hi) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)lo) |
           ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)hi) << 16);
}

// Tile of TL x TL outputs: layer 1 on an HW x HW grid with HW = TL + 4 a
// multiple of 16, so that a 16-pixel group is one run of a grid row; layer 2
// and 3 on UW = TL + 2 rows of the same HW-wide runs (columns UW.. unused);
// z on ZW = TL + 6.  u is stored [tap][row][HW].
template <int TL>
struct LMShared {
    static constexpr int ZW = TL + 6, HW = TL + 4, UW = TL + 2, RG = HW / 16;
    static_assert(HW % 16 == 0, "layer-1 rows must be whole 16-pixel runs");
    float z[ZW * ZW];
    alignas(16) uint16_t h1[HW * HW * kLC];
    float u[9 * UW * HW];
};

template <int TL, int NT, typename T>
__global__ void __launch_bounds__(NT) k_learned_apply_mf(LImage im, const float* __restrict__ mf32,
                                                         const uint16_t* __restrict__ mfbf,
                                                         const double* __restrict__ sigma_dev,
                                                         T* __restrict__ x, float* __restrict__ yout) {
    using SH = LMShared<TL>;
    constexpr int ZW = SH::ZW, HW = SH::HW, UW = SH::UW, RG = SH::RG, NWV = NT / 64;
    constexpr int NG1 = HW * RG, NG2 = UW * RG;
    constexpr int KZ = (ZW * ZW + NT - 1) / NT, KO = (TL * TL + NT - 1) / NT;
    __shared__ SH S;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c16 = lane & 15;
    const int tiles = (im.width + TL - 1) / TL;
    const int tj0 = (blockIdx.x / tiles) * TL, ti0 = (blockIdx.x % tiles) * TL;
    // every global load of the tile (sigma, weights, the z patch and the x
    // values to update) is issued before the first wait
    const double sg = sigma_dev ? *sigma_dev : 1.0;
    T xo[KO];
    if (!yout) {
#pragma unroll
        for (int k = 0; k < KO; ++k) {
            const int o = min(tid + k * NT, TL * TL - 1);
            const int pj = min(tj0 + o / TL, im.height - 1), pi = min(ti0 + o % TL, im.width - 1);
            xo[k] = x[(size_t)pj * im.width + pi];
        }
    }
    const floatx4 r0 = *reinterpret_cast<const floatx4*>(mf32 + lane * 8);
    const floatx4 r1 = *reinterpret_cast<const floatx4*>(mf32 + lane * 8 + 4);
    lbf16x8 a2[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) a2[m] = *reinterpret_cast<const lbf16x8*>(mfbf + (lane * 5 + m) * 8);
    float zv[KZ];
    bool zin[KZ];
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
        const int t = min(tid + k * NT, ZW * ZW - 1);
        const int pj = tj0 - 3 + t / ZW, pi = ti0 - 3 + t % ZW;
        zin[k] = l_inside(im, pj, pi);
        zv[k] = im.z[(size_t)clampi(pj, 0, im.height - 1) * im.width + clampi(pi, 0, im.width - 1)];
    }
    const float a1[3] = {r0[0], r0[1], r0[2]};
    const float a3[4] = {r0[3], r1[0], r1[1], r1[2]};
    // per-lane tap offsets (taps 9.. meet zero weights: clamped to tap 8)
    int zo[3], ho[5];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int tap = min(4 * m + g, 8);
        zo[m] = (tap / 3) * ZW + tap % 3;
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const int tap = min(2 * m + (g >> 1), 8);
        ho[m] = ((tap / 3) * HW + tap % 3) * kLC + 8 * (g & 1);
    }
    // per-lane column masks of the RG runs of a row (layer 1; layers 2-3)
    bool c1[RG], c2[RG];
    int hb2[RG];
#pragma unroll
    for (int h = 0; h < RG; ++h) {
        const int px = 16 * h + c16;
        c1[h] = l_col_in(im, ti0 - 2 + px);
        c2[h] = px < UW && l_col_in(im, ti0 - 1 + px);
        hb2[h] = (px < UW ? px : 0) * kLC;
    }
    if (!(sg > 0.0)) return;  // uniform: the whole workgroup leaves
    const float zscale = (float)(1.0 / sg);
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
        const int t = tid + k * NT;
        if (t < ZW * ZW) S.z[t] = zin[k] ? zv[k] * zscale : 0.f;
    }
    __syncthreads();
    // layer 1: group gr = run h of row r; two groups per wave in flight
    auto layer1 = [&](int gr) {
        const int r = gr / RG, h = gr % RG;
        const float* zb = S.z + r * ZW + 16 * h + c16;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 3; ++m) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[m], zb[zo[m]], acc, 0, 0, 0);
        return acc;
    };
    auto store1 = [&](int gr, const floatx4& acc) {
        const int r = gr / RG, h = gr % RG;
        const bool in = c1[h] && l_row_in(im, tj0 - 2 + r);
        const uint2 v{l_pack_bf16(in ? fmaxf(acc[0], 0.f) : 0.f, in ? fmaxf(acc[1], 0.f) : 0.f),
                      l_pack_bf16(in ? fmaxf(acc[2], 0.f) : 0.f, in ? fmaxf(acc[3], 0.f) : 0.f)};
        *reinterpret_cast<uint2*>(&S.h1[(r * HW + 16 * h + c16) * kLC + 4 * g]) = v;
    };
    for (int gr = wave; gr < NG1; gr += 2 * NWV) {
        const int gb = gr + NWV;
        const floatx4 ha = layer1(gr);
        const floatx4 hb = layer1(gb < NG1 ? gb : gr);
        store1(gr, ha);
        if (gb < NG1) store1(gb, hb);
    }
    __syncthreads();
    auto layer23 = [&](int gr) {
        const int r = gr / RG, h = gr % RG;
        const uint16_t* hb = S.h1 + r * HW * kLC + hb2[h];
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 5; ++m)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[m], *reinterpret_cast<const lbf16x8*>(hb + ho[m]), acc,
                                                          0, 0, 0);
        const bool in = c2[h] && l_row_in(im, tj0 - 1 + r);
        floatx4 u = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            u = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[j], in ? fmaxf(acc[j], 0.f) : 0.f, u, 0, 0, 0);
        return u;
    };
    auto store23 = [&](int gr, const floatx4& u) {
        const int r = gr / RG, h = gr % RG;
        float* ub = S.u + r * HW + 16 * h + c16;  // columns >= UW: unused padding
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (4 * g + j < 9) ub[(4 * g + j) * UW * HW] = u[j];
    };
    for (int gr = wave; gr < NG2; gr += 2 * NWV) {
        const int gb = gr + NWV;
        const floatx4 ua = layer23(gr);
        const floatx4 ub = layer23(gb < NG2 ? gb : gr);
        store23(gr, ua);
        if (gb < NG2) store23(gb, ub);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KO; ++k) {
        const int o = tid + k * NT;
        const int oy = o / TL, ox = o % TL;
        const int pj = tj0 + oy, pi = ti0 + ox;
        if (o < TL * TL && pj < im.height && pi < im.width && l_inside(im, pj, pi)) {
            float y = 0.f;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) y += S.u[(tap * UW + oy + tap / 3) * HW + ox + tap % 3];
            const size_t I = (size_t)pj * im.width + pi;
            if (yout)
                yout[I] = y;
            else
                x[I] = xo[k] + (T)(sg * (double)y);
        }
    }
}

// sigma = sqrt(sum partial / N), one block of kLSigmaThreads.
constexpr int kLSigmaThreads = 1024;
__global__ void __launch_bounds__(kLSigmaThreads) k_learned_sigma(const double* __restrict__ partial, int np,
                                                                  long long N, double* __restrict__ sigma) {
    __shared__ double red[kLSigmaThreads / 64];
    double s = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < np; i += kLSigmaThreads) s += partial[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) sigma[0] = sqrt(s / (double)N);
}

// One training item: an image with a loss region [l0, l0 + lsize)^2 (image
// coordinates) and its target t (lsize x lsize, row-major).
struct LItem {
    LImage im;
    const float* t;
    int l0, lsize;
};

// Forward + backward of one 16x16 tile of one item; writes this block's
// partial gradient (canonical layout, FP32) and partial squared error.
// Loss = mean over loss pixels of (y - t)^2; inv_count = 1 / (number of loss
// pixels in the batch).
__global__ void __launch_bounds__(kLThreads) k_learned_train(const LItem* __restrict__ items,
                                                             int tiles_per_item, LearnedW W,
                                                             float inv_count,
                                                             float* __restrict__ gpart,
                                                             double* __restrict__ lpart) {
    __shared__ LShared S;
    __shared__ float gy[16 * 16];
    __shared__ uint16_t gh2[324 * kLC];
    __shared__ float red[kLW1 + kLW3];
    __shared__ float dw1w[4][kLW1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const LItem it = items[blockIdx.x / tiles_per_item];
    const int tile = blockIdx.x % tiles_per_item;
    const int tpr = (it.lsize + kLTile - 1) / kLTile;
    const int tj0 = it.l0 + (tile / tpr) * kLTile, ti0 = it.l0 + (tile % tpr) * kLTile;
    float y = l_forward_tile(it.im, W, tj0, ti0, 1.f, S);
    // output gradient
    int oy = tid >> 4, ox = tid & 15;
    int lj = tj0 + oy - it.l0, li = ti0 + ox - it.l0;
    bool inl = lj < it.lsize && li < it.lsize && l_inside(it.im, tj0 + oy, ti0 + ox);
    float d = inl ? y - it.t[(size_t)lj * it.lsize + li] : 0.f;
    gy[tid] = 2.f * d * inv_count;
    {
        double sq = (double)d * d;
        for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
        __shared__ double lw[4];
        if (lane == 0) lw[wave] = sq;
        __syncthreads();
        if (tid == 0) lpart[blockIdx.x] = lw[0] + lw[1] + lw[2] + lw[3];
    }
    __syncthreads();
    float* gp = gpart + (size_t)blockIdx.x * kLWeights;
    // dW3[ci][tap] = sum_pix gy * h2[pix + tap][ci]
    for (int k = tid; k < kLW3; k += kLThreads) {
        int ci = k / 9, tap = k % 9;
        float s = 0.f;
        for (int p = 0; p < 256; ++p)
            s = fmaf(gy[p], S.h2[(((p >> 4) + tap / 3) * 18 + (p & 15) + tap % 3) * kLC + ci], s);
        gp[kLW1 + kLW2 + k] = s;
    }
    // gh2[q][ci] = (h2 > 0) * sum_tap W3[ci][tap] gy[q - tap], rounded to BF16
    for (int e = tid; e < 324 * kLC; e += kLThreads) {
        int q = e / kLC, ci = e % kLC;
        int qy = q / 18, qx = q % 18;
        float s = 0.f;
        if (S.h2[e] > 0.f) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                int gyy = qy - tap / 3, gxx = qx - tap % 3;
                if (gyy >= 0 && gyy < 16 && gxx >= 0 && gxx < 16) s = fmaf(S.w3t[tap * kLC + ci], gy[gyy * 16 + gxx], s);
            }
        }
        gh2[e] = f32_to_bf16(s);
    }
    __syncthreads();
    // dW2 (MFMA): for each tap, D[co][ci] = sum_q gh2[q][co] h1[q + tap][ci],
    // K = pixels in chunks of 16; wave w takes taps w, w+4, w+8
    for (int tap = wave; tap < 9; tap += 4) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ch = 0; ch < 21; ++ch) {
            short av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int q = ch * 16 + 4 * (lane >> 4) + r;
                if (q < 324) {
                    av[r] = (short)gh2[q * kLC + (lane & 15)];
                    int qy = q / 18, qx = q % 18;
                    bv[r] = (short)S.h1[((qy + tap / 3) * 20 + qx + tap % 3) * kLC + (lane & 15)];
                } else {
                    av[r] = 0;
                    bv[r] = 0;
                }
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bf16x4{av[0], av[1], av[2], av[3]},
                                                           bf16x4{bv[0], bv[1], bv[2], bv[3]}, acc,
                                                           0, 0, 0);
        }
        int ci = lane & 15;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int co = 4 * (lane >> 4) + j;
            gp[kLW1 + (co * kLC + ci) * 9 + tap] = acc[j];
        }
    }
    // gh1 (MFMA) on the 20 x 20 grid: D[p][ci] = sum_{tap,co} gh2[p - tap][co] W2[co][ci][tap],
    // masked by h1 > 0; accumulated straight into dW1[ci][tap'] += gh1 * z[p + tap']
    bf16x4 bw[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const uint16_t* src = W.w2b + ((size_t)tap * kLC + (lane & 15)) * kLC + 4 * (lane >> 4);
        bw[tap] = bf16x4{(short)src[0], (short)src[1], (short)src[2], (short)src[3]};
    }
    float dw1[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) dw1[t] = 0.f;
    for (int g = wave; g < 25; g += 4) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        int pa = g * 16 + (lane & 15);
        int py = pa / 20, px = pa % 20;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            int qy = py - tap / 3, qx = px - tap % 3;
            bf16x4 a = {0, 0, 0, 0};
            if (qy >= 0 && qy < 18 && qx >= 0 && qx < 18) {
                const uint16_t* src = &gh2[(qy * 18 + qx) * kLC + 4 * (lane >> 4)];
                a = bf16x4{(short)src[0], (short)src[1], (short)src[2], (short)src[3]};
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[tap], acc, 0, 0, 0);
        }
        int ci = lane & 15;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int p = g * 16 + 4 * (lane >> 4) + j;
            int ry = p / 20, rx = p % 20;
            float gv = (bf16_to_f32(S.h1[p * kLC + ci]) > 0.f) ? acc[j] : 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) dw1[t] = fmaf(gv, S.z[(ry + t / 3) * 22 + rx + t % 3], dw1[t]);
        }
    }
    // reduce dW1 partials: lanes with equal ci (l, l+16, l+32, l+48), then waves
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        float v = dw1[t];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (lane < 16) dw1w[wave][lane * 9 + t] = v;
    }
    __syncthreads();
    for (int k = tid; k < kLW1; k += kLThreads) gp[k] = dw1w[0][k] + dw1w[1][k] + dw1w[2][k] + dw1w[3][k];
    (void)red;
}

// Deterministic sum of the per-block partials: g[k] = sum_b gpart[b][k].
__global__ void k_learned_reduce(const float* __restrict__ gpart, int nblocks,
                                 const double* __restrict__ lpart, float* __restrict__ grad,
                                 double* __restrict__ loss) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kLWeights) {
        float s = 0.f;
        for (int b = 0; b < nblocks; ++b) s += gpart[(size_t)b * kLWeights + k];
        grad[k] = s;
    }
    if (k == 0) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += lpart[b];
        loss[0] = s;
    }
}

// Adam on FP32 master weights, then the BF16 copies in the three layouts.
__global__ void k_learned_adam(float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                               const float* __restrict__ grad, float lr, float b1, float b2, float eps,
                               float bc1, float bc2, uint16_t* __restrict__ wc, uint16_t* __restrict__ w2f,
                               uint16_t* __restrict__ w2b, float* __restrict__ mf32,
                               uint16_t* __restrict__ mfbf) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kLWeights) return;
    float g = grad[k];
    float mk = b1 * m[k] + (1.f - b1) * g;
    float vk = b2 * v[k] + (1.f - b2) * g * g;
    m[k] = mk;
    v[k] = vk;
    float w = master[k] - lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
    master[k] = w;
    uint16_t h = f32_to_bf16(w);
    wc[k] = h;
    if (k >= kLW1 && k < kLW1 + kLW2) {
        int e = k - kLW1, co = e / (kLC * 9), ci = (e / 9) % kLC, tap = e % 9;
        w2f[((size_t)tap * kLC + co) * kLC + ci] = h;
        w2b[((size_t)tap * kLC + ci) * kLC + co] = h;
    }
    int fs, bs;
    l_mf_slot(k, fs, bs);
    if (fs >= 0) mf32[fs] = bf16_to_f32(h);
    if (bs >= 0) mfbf[bs] = h;
}

// Canonical BF16 weights -> the two W2 layouts and the MFMA records (after an
// external load; one thread per canonical weight).
__global__ void k_learned_layouts(const uint16_t* __restrict__ wc, uint16_t* __restrict__ w2f,
                                  uint16_t* __restrict__ w2b, float* __restrict__ mf32,
                                  uint16_t* __restrict__ mfbf) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kLWeights) return;
    const uint16_t h = wc[k];
    if (k >= kLW1 && k < kLW1 + kLW2) {
        int e = k - kLW1, co = e / (kLC * 9), ci = (e / 9) % kLC, tap = e % 9;
        w2f[((size_t)tap * kLC + co) * kLC + ci] = h;
        w2b[((size_t)tap * kLC + ci) * kLC + co] = h;
    }
    int fs, bs;
    l_mf_slot(k, fs, bs);
    if (fs >= 0) mf32[fs] = bf16_to_f32(h);
    if (bs >= 0) mfbf[bs] = h;
}

// e_hf = u - x - P e_c target pieces are formed with the ordinary kernels;
// this packs one level sample: out_z = z / sigma, out_t = t / sigma (FP32).
__global__ void k_learned_pack(const double* __restrict__ r, const double* __restrict__ diag,
                               const double* __restrict__ t, long long N,
                               const double* __restrict__ sigma, float* __restrict__ oz,
                               float* __restrict__ ot) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I >= N) return;
    double s = sigma[0] > 0.0 ? sigma[0] : 1.0;
    oz[I] = (float)(r[I] / diag[I] / s);
    ot[I] = (float)(t[I] / s);
}

// sum of (r / diag)^2 per block (FP64), for sigma of a training sample.
__global__ void __launch_bounds__(kBlock) k_learned_sumsq_scaled(const double* __restrict__ r,
                                                                 const double* __restrict__ diag,
                                                                 long long N,
                                                                 double* __restrict__ partial) {
    __shared__ double red[kBlock / 64];
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    double s = 0.0;
    if (I < N) {
        double v = r[I] / diag[I];
        s = v * v;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Cut one training patch: image (lsize + 6)^2 around the loss region whose
// level-grid origin is (j0, i0); zero outside the domain.
__global__ void k_learned_cut(const float* __restrict__ zl, const float* __restrict__ tl, int n,
                              int j0, int i0, int lsize, float* __restrict__ pz,
                              float* __restrict__ pt) {
    int w = lsize + 6;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < w * w) {
        int gj = j0 - 3 + t / w, gi = i0 - 3 + t % w;
        pz[t] = (gj >= 0 && gj < n && gi >= 0 && gi < n) ? zl[(size_t)gj * n + gi] : 0.f;
    }
    if (t < lsize * lsize) {
        int gj = j0 + t / lsize, gi = i0 + t % lsize;
        pt[t] = (gj < n && gi < n) ? tl[(size_t)gj * n + gi] : 0.f;
    }
}

}  // namespace igamg
