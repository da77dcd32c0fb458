// Frontier-ordering network: a multilayer perceptron 4 -> 64 -> 64 -> 1
// (ReLU) that predicts the value function from normalised cell coordinates.
// Its only use is to give every state a bucket key for the bucket-ordered
// solve (gbf_opts.order = GBF_ORDER_BUCKETS); the solver's fixed point does
// not depend on it.  Weights are held as a bfloat16 working copy (rounded to
// nearest even from an fp32 master copy); every kernel expands them exactly
// to fp32 in LDS and accumulates in fp32 with fused multiply-adds in a fixed
// order.  Training: mean squared error on labelled samples, gradients by
// the chain rule, Adam (Kingma & Ba 2015) on the fp32 master copy.
//
// Inference (k_vhat, about 8.8 kFLOP per cell) runs layers 1 and 2 on the
// matrix cores: layer 1 in fp32, layer 2 in bf16 with each hidden activation
// split into two bf16 terms, so that the keys match the fp32 network's.
// Training (k_grad, k_reduce) is a few kFLOP per sample and runs on the
// vector ALUs in fp32.
//
// Parameter vector (4545 floats): W1 [64][4], b1 [64], W2 [64][64] (W2[j][k]
// feeds h1[k] into unit j), b2 [64], W3 [64], b3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gbf.h"
#include "gbf_device.h"
#include "gbf_internal.h"

namespace gbf {
namespace mlp {

constexpr int H = 64;
constexpr int NP = GBF_MLP_NPARAMS;
constexpr int oW1 = 0, oB1 = 256, oW2 = 320, oB2 = 4416, oW3 = 4480, oB3 = 4544;
constexpr int kStride = NP + 3;  // per-block partial: gradient, loss sum, label count (+1 pad)
static_assert(oB3 + 1 == NP, "parameter layout");

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ void load_weights(const uint16_t* __restrict__ wbf, float* w) {
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = bf16_to_f32(gp(wbf)[i]);
    __syncthreads();
}

// Features of cell c of a grid with dims N: ((x0+.5-tcx)/N0, (x1+.5-tcy)/N1,
// (x2+.5)/N2, (x3+.5)/N3).
struct Grid {
    uint32_t N[4];
    float tcx, tcy;
};

__device__ __forceinline__ void cell_features(const Grid& g, uint32_t c, float f[4]) {
    const uint32_t x0 = c % g.N[0];
    c /= g.N[0];
    const uint32_t x1 = c % g.N[1];
    c /= g.N[1];
    const uint32_t x2 = c % g.N[2];
    const uint32_t x3 = c / g.N[2];
    f[0] = ((float)x0 + 0.5f - g.tcx) / (float)g.N[0];
    f[1] = ((float)x1 + 0.5f - g.tcy) / (float)g.N[1];
    f[2] = ((float)x2 + 0.5f) / (float)g.N[2];
    f[3] = ((float)x3 + 0.5f) / (float)g.N[3];
}

// Forward pass of one sample with the weights in LDS.  h1 is returned for
// the training kernel; unit j of the second layer is folded into the
// output as soon as it is formed.
__device__ __forceinline__ float forward(const float* w, const float f[4], float h1[H]) {
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float a = w[oB1 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i) a = __builtin_fmaf(w[oW1 + j * 4 + i], f[i], a);
        h1[j] = a > 0.f ? a : 0.f;
    }
    float out = w[oB3];
    for (int j = 0; j < H; ++j) {
        float a = w[oB2 + j];
#pragma unroll
        for (int k = 0; k < H; ++k) a = __builtin_fmaf(w[oW2 + j * H + k], h1[k], a);
        out = __builtin_fmaf(w[oW3 + j], a > 0.f ? a : 0.f, out);
    }
    return out;
}

// ------------------------------------------------------------------ inference
// vhat[c] = scale * out(features(c)) for every cell; per-block minimum into
// bmin.  Each wave evaluates 32 cells per step with its contractions on the
// matrix cores, in the orientation units x cells, so that every layer's
// accumulator is, as it stands, the operand of the next layer:
//   layer 1  D1 (64 units x 32 cells) = W1 (64 x 4) F^T (4 x 32) + b1, fp32:
//            per 32-unit block, two v_mfma_f32_32x32x2_f32 over the feature
//            pairs and one that adds b1 (A = b1, B = 1 in the first half,
//            A = B = 0 in the second);
//   layer 2  D2 (64 x 32) = W2 (64 x 64) relu(D1) + b2: per output block,
//            eight v_mfma_f32_32x32x16_bf16 steps, accumulator started at
//            b2.  W2 is the bf16 working copy; h1 = relu(D1) enters as the
//            two bf16 terms hi + lo of its fp32 value (relative residual
//            below 2^-16, so the keys match the fp32 network's), and the
//            sums are fp32;
//   layer 3  out = b3 + W3 . relu(D2): fp32 fmas over the 32 units a lane
//            holds, then one exchange between the two halves of the wave.
// Operand layouts (wave64, lane l, half h = l/32): v_mfma_f32_32x32x2_f32
// takes A[i = l%32][k = h] and B[k = h][j = l%32]; v_mfma_f32_32x32x16_bf16
// takes A[i = l%32][k = 8h + e] and B[k = 8h + e][j = l%32], e = 0..7; both
// leave accumulator r (0..15) of lane l at D[i = 8(r/4) + 4h + r%4][j = l%32].
// So lane l always works on cell l%32, and register r of output block b
// holds unit acc_unit(b, r, h).  The K index of layer 2 is permuted to
// follow that: step s takes registers 8(s%2)..8(s%2)+7 of D1 block s/2, and
// the W2 operand is gathered with the same permutation (k_unit).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kCellsPerWave = 32;

__device__ __forceinline__ int acc_unit(int b, int r, int h) { return 32 * b + 8 * (r >> 2) + 4 * h + (r & 3); }
__device__ __forceinline__ int k_unit(int s, int h, int e) { return acc_unit(s >> 1, 8 * (s & 1) + e, h); }

__global__ __launch_bounds__(256) void k_vhat(const uint16_t* __restrict__ wbf, Grid g, uint32_t n, float scale,
                                              float* __restrict__ vhat, float* __restrict__ bmin) {
    __shared__ float s_b2[H], s_w3[H];
    __shared__ float s_min[256 / kWave];
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        s_b2[i] = bf16_to_f32(gp(wbf)[oB2 + i]);
        s_w3[i] = bf16_to_f32(gp(wbf)[oW3 + i]);
    }
    const int lane = lane_id();
    const int h = lane >> 5, col = lane & 31;
    // loop-invariant operands in registers
    float a1w[2][2], a1b[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int t = 0; t < 2; ++t) a1w[b][t] = bf16_to_f32(gp(wbf)[oW1 + (32 * b + col) * 4 + 2 * t + h]);
        a1b[b] = h == 0 ? bf16_to_f32(gp(wbf)[oB1 + 32 * b + col]) : 0.f;
    }
    const float one_h = h == 0 ? 1.f : 0.f;
    bf16x8 a2w[2][4];
#pragma unroll
    for (int bo = 0; bo < 2; ++bo)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            s16x8 t;
#pragma unroll
            for (int e = 0; e < 8; ++e) t[e] = (short)gp(wbf)[oW2 + (32 * bo + col) * H + k_unit(st, h, e)];
            a2w[bo][st] = __builtin_bit_cast(bf16x8, t);
        }
    const float b3 = bf16_to_f32(gp(wbf)[oB3]);
    __syncthreads();
    const uint32_t wv = threadIdx.x / kWave;
    float mn = INFINITY;
    const uint32_t cstep = gridDim.x * (256 / kWave) * kCellsPerWave;
    for (uint32_t c0 = (blockIdx.x * (256 / kWave) + wv) * kCellsPerWave; c0 < n; c0 += cstep) {
        // keep b2 and W3 in LDS: without this the compiler hoists all 128
        // of them into registers and the kernel loses occupancy
        __asm__ volatile("" ::: "memory");
        const uint32_t c = c0 + (uint32_t)col;
        float f[4];
        cell_features(g, c < n ? c : n - 1, f);
        const float fa = h ? f[1] : f[0], fb = h ? f[3] : f[2];
        // layer 1
        f32x16 d1[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            f32x16 z = {};
            z = __builtin_amdgcn_mfma_f32_32x32x2f32(a1w[b][0], fa, z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_32x32x2f32(a1w[b][1], fb, z, 0, 0, 0);
            d1[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1b[b], one_h, z, 0, 0, 0);
        }
        // layer 2, accumulators started at b2
        f32x16 d2[2];
#pragma unroll
        for (int bo = 0; bo < 2; ++bo)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 v = *reinterpret_cast<const float4*>(&s_b2[32 * bo + 8 * q + 4 * h]);
                d2[bo][4 * q + 0] = v.x;
                d2[bo][4 * q + 1] = v.y;
                d2[bo][4 * q + 2] = v.z;
                d2[bo][4 * q + 3] = v.w;
            }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            // h1 = hi + lo + r with hi = bf16(h1), lo = bf16(h1 - hi) (the
            // difference is exact in fp32) and |r| <= 2^-16 |h1|; both
            // halves go through the bf16 products, whose sums are fp32
            bf16x8 xh, xl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float a = d1[st >> 1][8 * (st & 1) + e];
                const float hv = a > 0.f ? a : 0.f;  // relu leaves no NaN
                xh[e] = (__bf16)hv;                   // nearest even
                xl[e] = (__bf16)(hv - (float)xh[e]);
            }
            d2[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2w[0][st], xh, d2[0], 0, 0, 0);
            d2[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2w[1][st], xh, d2[1], 0, 0, 0);
            d2[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2w[0][st], xl, d2[0], 0, 0, 0);
            d2[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2w[1][st], xl, d2[1], 0, 0, 0);
        }
        // layer 3
        float v = 0.f;
#pragma unroll
        for (int bo = 0; bo < 2; ++bo)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 w3 = *reinterpret_cast<const float4*>(&s_w3[32 * bo + 8 * q + 4 * h]);
                const float* wq = &w3.x;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float a = d2[bo][4 * q + t];
                    v = __builtin_fmaf(wq[t], a > 0.f ? a : 0.f, v);
                }
            }
        v += __shfl_xor(v, 32, kWave);
        if (h == 0 && c < n) {
            const float val = scale * (b3 + v);
            gp(vhat)[c] = val;
            mn = fminf(mn, val);
        }
    }
    for (int d = kWave / 2; d > 0; d >>= 1) mn = fminf(mn, __shfl_xor(mn, d, kWave));
    if (lane == 0) s_min[wv] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = s_min[0];
        for (int i = 1; i < 256 / kWave; ++i) m = fminf(m, s_min[i]);
        gp(bmin)[blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(1024) void k_min(const float* __restrict__ bmin, int nb, float* __restrict__ out) {
    __shared__ float s[1024 / kWave];
    float m = INFINITY;
    for (int i = threadIdx.x; i < nb; i += 1024) m = fminf(m, gp(bmin)[i]);
    for (int d = kWave / 2; d > 0; d >>= 1) m = fminf(m, __shfl_xor(m, d, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = s[0];
        for (int i = 1; i < 1024 / kWave; ++i) r = fminf(r, s[i]);
        gp(out)[0] = r;
    }
}

// key = clamp(floor((vhat - min) / width), 0, 65535)
__global__ __launch_bounds__(256) void k_keys(const float* __restrict__ vhat, const float* __restrict__ vmin,
                                              uint32_t n, float width, uint16_t* __restrict__ key) {
    const uint32_t c = blockIdx.x * 256u + threadIdx.x;
    if (c >= n) return;
    const float q = floorf((gp(vhat)[c] - gp(vmin)[0]) / width);
    gp(key)[c] = (uint16_t)(q <= 0.f ? 0.f : (q >= 65535.f ? 65535.f : q));
}

__global__ __launch_bounds__(256) void k_forward(const uint16_t* __restrict__ wbf, const float* __restrict__ feat,
                                                 int64_t count, float* __restrict__ out) {
    __shared__ float w[NP];
    load_weights(wbf, w);
    const int64_t s = blockIdx.x * 256ll + threadIdx.x;
    if (s >= count) return;
    float f[4], h1[H];
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = gp(feat)[s * 4 + i];
    gp(out)[s] = forward(w, f, h1);
}

// Training samples: features of the listed cells and labels V(c) / scale
// (NaN where V is infinite: such samples carry no label).
template <int DT>
__global__ __launch_bounds__(256) void k_samples(Grid g, uint32_t n, const void* __restrict__ V, float scale,
                                                 const int64_t* __restrict__ cells, int64_t count,
                                                 float* __restrict__ feat, float* __restrict__ target) {
    const int64_t s = blockIdx.x * 256ll + threadIdx.x;
    if (s >= count) return;
    const int64_t cc = gp(cells)[s];
    if (cc < 0 || cc >= (int64_t)n) {
        // a cell outside the grid gives an unlabelled, all-NaN sample
#pragma unroll
        for (int i = 0; i < 4; ++i) gp(feat)[s * 4 + i] = NAN;
        if (target) gp(target)[s] = NAN;
        return;
    }
    const uint32_t c = (uint32_t)cc;
    float f[4];
    cell_features(g, c, f);
#pragma unroll
    for (int i = 0; i < 4; ++i) gp(feat)[s * 4 + i] = f[i];
    if (target) {
        float y;
        if (DT == 0) {
            const int32_t v = gp(static_cast<const int32_t*>(V))[c];
            y = v == 0x7fffffff ? NAN : (float)v / scale;
        } else {
            const float v = gp(static_cast<const float*>(V))[c];
            y = isinf(v) ? NAN : v / scale;
        }
        gp(target)[s] = y;
    }
}

// ------------------------------------------------------------------ training
// One 64-sample block per wave.  Each lane runs the forward and backward
// pass of its sample; the per-block gradient sums over the 64 samples are
// formed from activations staged in LDS ([unit][sample], odd row pitch),
// in a fixed order, and written to the block's partial slot (no atomics:
// the result is deterministic).  The gradient is that of sum (out - y)^2;
// the reduction divides by the number of labels.
constexpr int kTB = 64;
constexpr int kPitch = kTB + 1;

__global__ __launch_bounds__(kTB) void k_grad(const uint16_t* __restrict__ wbf, const float* __restrict__ feat,
                                              const float* __restrict__ target, int64_t rows,
                                              const int64_t* __restrict__ idx, int64_t count,
                                              float* __restrict__ partial) {
    __shared__ float w[NP];
    __shared__ float bufA[H * kPitch];
    __shared__ float bufB[H * kPitch];
    __shared__ float sf[4 * kTB];
    __shared__ float sdo[kTB];
    load_weights(wbf, w);
    const int l = threadIdx.x;
    const int64_t s = blockIdx.x * (int64_t)kTB + l;
    float f[4] = {0.f, 0.f, 0.f, 0.f};
    float y = NAN;
    if (s < count) {
        const int64_t q = idx ? gp(idx)[s] : s;
        if (q >= 0 && q < rows) {  // a row outside the sample set is skipped
#pragma unroll
            for (int i = 0; i < 4; ++i) f[i] = gp(feat)[q * 4 + i];
            y = gp(target)[q];
        }
    }
    const bool lab = s < count && !isnan(y) && !isnan(f[0] + f[1] + f[2] + f[3]);
    if (!lab) f[0] = f[1] = f[2] = f[3] = 0.f;
    // forward: h1 -> bufA, h2 -> bufB, ReLU masks kept as bits
    uint64_t m1 = 0, m2 = 0;
    float h1[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float a = w[oB1 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i) a = __builtin_fmaf(w[oW1 + j * 4 + i], f[i], a);
        h1[j] = a > 0.f ? a : 0.f;
        m1 |= (uint64_t)(a > 0.f) << j;
        bufA[j * kPitch + l] = h1[j];
    }
    float out = w[oB3];
    for (int j = 0; j < H; ++j) {
        float a = w[oB2 + j];
#pragma unroll
        for (int k = 0; k < H; ++k) a = __builtin_fmaf(w[oW2 + j * H + k], h1[k], a);
        const float h2 = a > 0.f ? a : 0.f;
        m2 |= (uint64_t)(a > 0.f) << j;
        bufB[j * kPitch + l] = h2;
        out = __builtin_fmaf(w[oW3 + j], h2, out);
    }
    const float r = lab ? out - y : 0.f;
    const float dout = 2.f * r;
    sdo[l] = dout;
#pragma unroll
    for (int i = 0; i < 4; ++i) sf[i * kTB + l] = f[i];
    __syncthreads();
    float* P = partial + (int64_t)blockIdx.x * kStride;
    // dW3[j] = sum_s dout_s h2_s[j]; db3 = sum_s dout_s
    {
        const int j = l;
        float acc = 0.f;
        for (int t = 0; t < kTB; ++t) acc = __builtin_fmaf(sdo[t], bufB[j * kPitch + t], acc);
        gp(P)[oW3 + j] = acc;
        if (l == 0) {
            float b = 0.f;
            for (int t = 0; t < kTB; ++t) b += sdo[t];
            gp(P)[oB3] = b;
        }
    }
    __syncthreads();
    // da2 = dout W3 relu'(a2) -> bufB; da1 accumulated in registers
    float da1[H];
#pragma unroll
    for (int k = 0; k < H; ++k) da1[k] = 0.f;
    for (int j = 0; j < H; ++j) {
        const float d = ((m2 >> j) & 1) ? dout * w[oW3 + j] : 0.f;
        bufB[j * kPitch + l] = d;
#pragma unroll
        for (int k = 0; k < H; ++k) da1[k] = __builtin_fmaf(w[oW2 + j * H + k], d, da1[k]);
    }
    __syncthreads();
    // dW2[j][k] = sum_s da2_s[j] h1_s[k]; db2[j] = sum_s da2_s[j]   (lane = j)
    {
        const int j = l;
        float acc[H];
#pragma unroll
        for (int k = 0; k < H; ++k) acc[k] = 0.f;
        float b = 0.f;
        for (int t = 0; t < kTB; ++t) {
            const float d = bufB[j * kPitch + t];
            b += d;
#pragma unroll
            for (int k = 0; k < H; ++k) acc[k] = __builtin_fmaf(d, bufA[k * kPitch + t], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < H; ++k) gp(P)[oW2 + j * H + k] = acc[k];
        gp(P)[oB2 + j] = b;
    }
    __syncthreads();
    // da1 = (W2^T da2) relu'(a1) -> bufA
#pragma unroll
    for (int k = 0; k < H; ++k) bufA[k * kPitch + l] = ((m1 >> k) & 1) ? da1[k] : 0.f;
    __syncthreads();
    // dW1[k][i] = sum_s da1_s[k] f_s[i]; db1[k] = sum_s da1_s[k]   (lane = k)
    {
        const int k = l;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, b = 0.f;
        for (int t = 0; t < kTB; ++t) {
            const float d = bufA[k * kPitch + t];
            b += d;
            a0 = __builtin_fmaf(d, sf[0 * kTB + t], a0);
            a1 = __builtin_fmaf(d, sf[1 * kTB + t], a1);
            a2 = __builtin_fmaf(d, sf[2 * kTB + t], a2);
            a3 = __builtin_fmaf(d, sf[3 * kTB + t], a3);
        }
        gp(P)[oW1 + k * 4 + 0] = a0;
        gp(P)[oW1 + k * 4 + 1] = a1;
        gp(P)[oW1 + k * 4 + 2] = a2;
        gp(P)[oW1 + k * 4 + 3] = a3;
        gp(P)[oB1 + k] = b;
    }
    // loss sum and label count of the block
    float rr = r * r, cnt = lab ? 1.f : 0.f;
    for (int d = kWave / 2; d > 0; d >>= 1) {
        rr += __shfl_xor(rr, d, kWave);
        cnt += __shfl_xor(cnt, d, kWave);
    }
    if (l == 0) {
        gp(P)[NP] = rr;
        gp(P)[NP + 1] = cnt;
    }
}

// Sum of the block partials in block order.  grad = sum / labels.  With
// `adam`, one Adam step on the fp32 master and a fresh bf16 working copy.
struct AdamArgs {
    float lr, c1, c2;  // c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
    int on;
};

__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ partial, int nb, AdamArgs A,
                                                float* __restrict__ grad, float* __restrict__ master,
                                                float* __restrict__ mom, float* __restrict__ vel,
                                                uint16_t* __restrict__ wbf, float* __restrict__ loss) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= NP + 2) return;
    float acc = 0.f;
    for (int b = 0; b < nb; ++b) acc += gp(partial)[(int64_t)b * kStride + i];
    if (i >= NP) {
        // [0] mean loss, [1] label count (both are sums in the partials)
        if (i == NP) {
            float cnt = 0.f;
            for (int b = 0; b < nb; ++b) cnt += gp(partial)[(int64_t)b * kStride + NP + 1];
            gp(loss)[0] = cnt > 0.f ? acc / cnt : 0.f;
            gp(loss)[1] = cnt;
        }
        return;
    }
    float cnt = 0.f;
    for (int b = 0; b < nb; ++b) cnt += gp(partial)[(int64_t)b * kStride + NP + 1];
    const float g = cnt > 0.f ? acc / cnt : 0.f;
    gp(grad)[i] = g;
    if (!A.on) return;
    const float m = 0.9f * gp(mom)[i] + 0.1f * g;
    const float v = 0.999f * gp(vel)[i] + 0.001f * (g * g);
    gp(mom)[i] = m;
    gp(vel)[i] = v;
    const float th = gp(master)[i] - A.lr * (m * A.c1) / (sqrtf(v * A.c2) + 1e-8f);
    gp(master)[i] = th;
    gp(wbf)[i] = f32_to_bf16(th);
}

__global__ void k_to_bf16(const float* __restrict__ master, uint16_t* __restrict__ wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NP) gp(wbf)[i] = f32_to_bf16(gp(master)[i]);
}

}  // namespace mlp
}  // namespace gbf

using namespace gbf;
using namespace gbf::mlp;

// ------------------------------------------------------------------ C ABI
struct gbf_mlp {
    hipStream_t stream = nullptr;
    float* master = nullptr;  // fp32 master weights
    float* mom = nullptr;     // Adam first moment
    float* vel = nullptr;     // Adam second moment
    uint16_t* wbf = nullptr;  // bf16 working copy
    float* grad = nullptr;    // last gradient
    float* loss = nullptr;    // [0] last mean loss, [1] label count
    float* partial = nullptr; // per-block gradient partials
    int64_t partial_blocks = 0;
    float* bmin = nullptr;    // per-block minima of vhat
    int64_t bmin_blocks = 0;
    float* scratch_v = nullptr;  // vhat when the caller passes none
    int64_t scratch_n = 0;
    float* host = nullptr;    // pinned read-back area (NP + 8 floats)
    int64_t step = 0;         // Adam step counter
    std::vector<void*> allocs;
    ~gbf_mlp() {
        for (void* p : allocs) (void)hipFree(p);
        if (host) (void)hipHostFree(host);
    }
};

namespace {
int mfail(int code, const std::string& msg) { return gbf::set_error(code, msg); }

#ifndef GBF_VHAT_BLOCKS
#define GBF_VHAT_BLOCKS 1024
#endif

#define MHIPC(expr)                                                                                    \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return mfail(GBF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int dalloc(gbf_mlp* m, void** p, size_t bytes) {
    if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) {
        *p = nullptr;
        return mfail(GBF_ENOMEM, "hipMalloc failed (" + std::to_string(bytes) + " bytes)");
    }
    m->allocs.push_back(*p);
    return GBF_OK;
}

void dfree(gbf_mlp* m, void* p) {
    for (size_t i = 0; i < m->allocs.size(); ++i)
        if (m->allocs[i] == p) {
            (void)hipFree(p);
            m->allocs.erase(m->allocs.begin() + i);
            return;
        }
}

bool valid_grid(const int32_t* dims, int64_t* n) {
    if (!dims) return false;
    int64_t p = 1;
    for (int a = 0; a < 4; ++a) {
        if (dims[a] < 1) return false;
        p *= dims[a];
        if (p > 0xffffffffll) return false;
    }
    *n = p;
    return true;
}

Grid make_grid(const int32_t* dims, float tcx, float tcy) {
    Grid g;
    for (int a = 0; a < 4; ++a) g.N[a] = (uint32_t)dims[a];
    g.tcx = tcx;
    g.tcy = tcy;
    return g;
}

int ensure_partial(gbf_mlp* m, int64_t nb) {
    if (m->partial_blocks >= nb) return GBF_OK;
    if (m->partial) dfree(m, m->partial);
    m->partial = nullptr;
    m->partial_blocks = 0;
    int rc = dalloc(m, (void**)&m->partial, (size_t)nb * kStride * sizeof(float));
    if (rc) return rc;
    m->partial_blocks = nb;
    return GBF_OK;
}

int run_grad(gbf_mlp* m, const float* feat, const float* target, int64_t rows, const int64_t* idx, int64_t count,
             const AdamArgs& A) {
    const int64_t nb = (count + kTB - 1) / kTB;
    int rc = ensure_partial(m, nb);
    if (rc) return rc;
    k_grad<<<(unsigned)nb, kTB, 0, m->stream>>>(m->wbf, feat, target, rows, idx, count, m->partial);
    MHIPC(hipGetLastError());
    k_reduce<<<(NP + 2 + 255) / 256, 256, 0, m->stream>>>(m->partial, (int)nb, A, m->grad, m->master, m->mom,
                                                          m->vel, m->wbf, m->loss);
    MHIPC(hipGetLastError());
    return GBF_OK;
}
}  // namespace

extern "C" int gbf_mlp_create(const float* params, void* hip_stream, gbf_mlp** out) {
    if (!out) return mfail(GBF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params) return mfail(GBF_EINVAL, "params is NULL");
    for (int i = 0; i < NP; ++i)
        if (!std::isfinite(params[i])) return mfail(GBF_EINVAL, "non-finite initial parameter");
    gbf_mlp* m = new gbf_mlp();
    m->stream = (hipStream_t)hip_stream;
    int rc;
    if ((rc = dalloc(m, (void**)&m->master, NP * 4)) || (rc = dalloc(m, (void**)&m->mom, NP * 4)) ||
        (rc = dalloc(m, (void**)&m->vel, NP * 4)) || (rc = dalloc(m, (void**)&m->wbf, NP * 2)) ||
        (rc = dalloc(m, (void**)&m->grad, NP * 4)) || (rc = dalloc(m, (void**)&m->loss, 64))) {
        delete m;
        return rc;
    }
    if (hipHostMalloc((void**)&m->host, (NP + 8) * sizeof(float), 0) != hipSuccess) {
        m->host = nullptr;
        delete m;
        return mfail(GBF_ENOMEM, "pinned host allocation failed");
    }
    *out = m;
    rc = gbf_mlp_set_params(m, params);
    if (rc) {
        delete m;
        *out = nullptr;
    }
    return rc;
}

extern "C" int gbf_mlp_set_params(gbf_mlp* m, const float* params) {
    if (!m || !params) return mfail(GBF_EINVAL, "NULL argument");
    std::memcpy(m->host, params, NP * sizeof(float));
    MHIPC(hipMemcpyAsync(m->master, m->host, NP * 4, hipMemcpyHostToDevice, m->stream));
    MHIPC(hipMemsetAsync(m->mom, 0, NP * 4, m->stream));
    MHIPC(hipMemsetAsync(m->vel, 0, NP * 4, m->stream));
    k_to_bf16<<<(NP + 255) / 256, 256, 0, m->stream>>>(m->master, m->wbf);
    MHIPC(hipGetLastError());
    MHIPC(hipStreamSynchronize(m->stream));
    m->step = 0;
    return GBF_OK;
}

extern "C" int gbf_mlp_get_params(gbf_mlp* m, float* master_out, uint16_t* bf16_out) {
    if (!m) return mfail(GBF_EINVAL, "NULL network");
    if (master_out) {
        MHIPC(hipMemcpyAsync(m->host, m->master, NP * 4, hipMemcpyDeviceToHost, m->stream));
        MHIPC(hipStreamSynchronize(m->stream));
        std::memcpy(master_out, m->host, NP * 4);
    }
    if (bf16_out) {
        MHIPC(hipMemcpyAsync(m->host, m->wbf, NP * 2, hipMemcpyDeviceToHost, m->stream));
        MHIPC(hipStreamSynchronize(m->stream));
        std::memcpy(bf16_out, m->host, NP * 2);
    }
    return GBF_OK;
}

extern "C" int gbf_mlp_samples(gbf_mlp* m, const int32_t dims[4], float tcx, float tcy, const void* V,
                               int32_t v_dtype, float scale, const int64_t* cells, int64_t count, float* feat_out,
                               float* target_out) {
    int64_t n;
    if (!m || !valid_grid(dims, &n)) return mfail(GBF_EINVAL, "bad network or grid");
    if (count < 0 || count > 0x7fffffffll) return mfail(GBF_EINVAL, "bad sample count");
    if (count == 0) return GBF_OK;
    if (!cells || !feat_out) return mfail(GBF_EINVAL, "NULL cells or feature output");
    if (target_out && (!V || (v_dtype != GBF_I32 && v_dtype != GBF_F32) || !(scale > 0.f)))
        return mfail(GBF_EINVAL, "labels need V, its dtype and a positive scale");
    const Grid g = make_grid(dims, tcx, tcy);
    const unsigned nb = (unsigned)((count + 255) / 256);
    if (v_dtype == GBF_F32)
        k_samples<1><<<nb, 256, 0, m->stream>>>(g, (uint32_t)n, V, scale, cells, count, feat_out, target_out);
    else
        k_samples<0><<<nb, 256, 0, m->stream>>>(g, (uint32_t)n, V, scale, cells, count, feat_out, target_out);
    MHIPC(hipGetLastError());
    MHIPC(hipStreamSynchronize(m->stream));
    return GBF_OK;
}

extern "C" int gbf_mlp_forward(gbf_mlp* m, const float* feat, int64_t count, float* out) {
    if (!m) return mfail(GBF_EINVAL, "NULL network");
    if (count < 0 || count > 0x7fffffffll) return mfail(GBF_EINVAL, "bad count");
    if (count == 0) return GBF_OK;
    if (!feat || !out) return mfail(GBF_EINVAL, "NULL features or output");
    k_forward<<<(unsigned)((count + 255) / 256), 256, 0, m->stream>>>(m->wbf, feat, count, out);
    MHIPC(hipGetLastError());
    MHIPC(hipStreamSynchronize(m->stream));
    return GBF_OK;
}

static int check_rows(int64_t rows, const int64_t* idx, int64_t count) {
    if (count <= 0 || count > 0x7fffffffll || rows <= 0) return mfail(GBF_EINVAL, "bad sample or row count");
    if (!idx && count > rows) return mfail(GBF_EINVAL, "count exceeds the rows without an index");
    return GBF_OK;
}

extern "C" int gbf_mlp_grad(gbf_mlp* m, const float* feat, const float* target, int64_t rows, const int64_t* idx,
                            int64_t count, float* grad_out, double* loss_out, int64_t* labels_out) {
    if (!m) return mfail(GBF_EINVAL, "NULL network");
    if (!feat || !target) return mfail(GBF_EINVAL, "NULL features or targets");
    int rc = check_rows(rows, idx, count);
    if (rc) return rc;
    AdamArgs A{0.f, 0.f, 0.f, 0};
    rc = run_grad(m, feat, target, rows, idx, count, A);
    if (rc) return rc;
    MHIPC(hipMemcpyAsync(m->host, m->grad, NP * 4, hipMemcpyDeviceToHost, m->stream));
    MHIPC(hipMemcpyAsync(m->host + NP, m->loss, 8, hipMemcpyDeviceToHost, m->stream));
    MHIPC(hipStreamSynchronize(m->stream));
    if (grad_out) std::memcpy(grad_out, m->host, NP * 4);
    if (loss_out) *loss_out = m->host[NP];
    if (labels_out) *labels_out = (int64_t)m->host[NP + 1];
    return GBF_OK;
}

extern "C" int gbf_mlp_train_step(gbf_mlp* m, const float* feat, const float* target, int64_t rows,
                                  const int64_t* idx, int64_t count, float lr, float* loss_out) {
    if (!m) return mfail(GBF_EINVAL, "NULL network");
    if (!feat || !target || !(lr > 0.f)) return mfail(GBF_EINVAL, "NULL features/targets or bad rate");
    if (int rc0 = check_rows(rows, idx, count)) return rc0;
    const int64_t t = m->step + 1;
    AdamArgs A;
    A.lr = lr;
    A.c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)t)));
    A.c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)t)));
    A.on = 1;
    int rc = run_grad(m, feat, target, rows, idx, count, A);
    if (rc) return rc;
    m->step = t;
    if (loss_out) {
        MHIPC(hipMemcpyAsync(m->host + NP, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
        MHIPC(hipStreamSynchronize(m->stream));
        *loss_out = m->host[NP];
    }
    return GBF_OK;
}

extern "C" int gbf_mlp_bucket_keys(gbf_mlp* m, const int32_t dims[4], float tcx, float tcy, float scale,
                                   float width, uint16_t* key_out, float* vhat_out, float* vhat_min_out) {
    int64_t n;
    if (!m || !valid_grid(dims, &n)) return mfail(GBF_EINVAL, "bad network or grid");
    if (!key_out) return mfail(GBF_EINVAL, "key_out is NULL");
    if (!(scale > 0.f) || !(width > 0.f)) return mfail(GBF_EINVAL, "scale and width must be positive");
    float* vh = vhat_out;
    if (!vh) {
        if (m->scratch_n < n) {
            if (m->scratch_v) dfree(m, m->scratch_v);
            m->scratch_v = nullptr;
            m->scratch_n = 0;
            int rc = dalloc(m, (void**)&m->scratch_v, (size_t)n * 4);
            if (rc) return rc;
            m->scratch_n = n;
        }
        vh = m->scratch_v;
    }
    // blocks of the key kernel: 4 waves x 32 cells per step, at most
    // GBF_VHAT_BLOCKS (each wave loads its weight operands once and loops)
    const int64_t nb = std::min<int64_t>((n + 127) / 128, GBF_VHAT_BLOCKS);
    if (m->bmin_blocks < nb + 1) {
        if (m->bmin) dfree(m, m->bmin);
        m->bmin = nullptr;
        m->bmin_blocks = 0;
        int rc = dalloc(m, (void**)&m->bmin, (size_t)(nb + 1) * 4);
        if (rc) return rc;
        m->bmin_blocks = nb + 1;
    }
    const Grid g = make_grid(dims, tcx, tcy);
    k_vhat<<<(unsigned)nb, 256, 0, m->stream>>>(m->wbf, g, (uint32_t)n, scale, vh, m->bmin);
    MHIPC(hipGetLastError());
    k_min<<<1, 1024, 0, m->stream>>>(m->bmin, (int)nb, m->bmin + nb);
    MHIPC(hipGetLastError());
    k_keys<<<(unsigned)((n + 255) / 256), 256, 0, m->stream>>>(vh, m->bmin + nb, (uint32_t)n, width, key_out);
    MHIPC(hipGetLastError());
    if (vhat_min_out) MHIPC(hipMemcpyAsync(m->host + NP + 4, m->bmin + nb, 4, hipMemcpyDeviceToHost, m->stream));
    MHIPC(hipStreamSynchronize(m->stream));
    if (vhat_min_out) *vhat_min_out = m->host[NP + 4];
    return GBF_OK;
}

extern "C" void gbf_mlp_free(gbf_mlp* m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    delete m;
}
