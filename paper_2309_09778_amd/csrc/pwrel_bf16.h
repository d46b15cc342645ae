// The perceptron on the matrix cores: 64 points per wave (lane l = point l),
// v_mfma_f32_32x32x16_bf16, two groups of 32 points.
//
// Operand layout of v_mfma_f32_32x32x16_bf16 (checked on the device):
//   A (32 x 16):  lane l, element e  ->  A[l % 32][8 (l / 32) + e]
//   B (16 x 32):  lane l, element e  ->  B[8 (l / 32) + e][l % 32]
//   C/D (32x32):  lane l, element e  ->  D[8 (e / 4) + 4 (l / 32) + e % 4][l % 32]
//
// Layer 1: Z^T (hidden x points) = bf16(w1) (hidden x K, K padded to 16)
//          . bf16(U)^T (K x points) + b1 (in the accumulator).
// Layer 2 with lrelu(z) = (1 - alpha) relu(z) + alpha z:
//   y = b2 + sum_j bf16((1-alpha) v_j) relu(bf16(z_j)) + bf16(alpha v_j) bf16(z_j),
//   as four chained MFMAs (K = 16 each) whose B operands are the layer-1
//   results of the same lane converted to bf16 pairs, in the order the lane
//   holds them: chunk c in {0,1} uses D1 elements 8c .. 8c+7 (relu), chunk
//   c in {2,3} the same elements without relu.  The A operands carry the
//   output weights in the matching hidden-unit order; only row 0 is nonzero,
//   so the result sits in element 0 of lanes 0..31.
// Every lane of the wave must execute these calls (the matrix cores work on
// the whole wave); lanes without a point feed zero inputs.
#pragma once

#include "pwrel_kernels.h"

namespace pwrel {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short short2v __attribute__((ext_vector_type(2)));

struct NetBf16 {
    bf16x8 a1;     // layer-1 A operand of this lane
    floatx16 c1;   // layer-1 accumulator init: b1 of the rows this lane holds
    bf16x8 a2[4];  // layer-2 A operands (chunks 0,1: (1-alpha) v; chunks 2,3: alpha v)
    float b2;
};

// hidden unit held by element e of D1 in a lane of half h
__device__ __forceinline__ int d1_row(int e, int h) { return 8 * (e / 4) + 4 * h + (e % 4); }

__device__ __forceinline__ NetBf16 make_net_bf16(const MlpW &m, int K)
{
    NetBf16 n;
    const int l = threadIdx.x & 63, h = l >> 5, i = l & 31;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * h + e;
        n.a1[e] = (__bf16)(k < K ? m.w1[i][k] : 0.0f);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e)
        n.c1[e] = m.b1[d1_row(e, h)];
    const float ar = 1.0f - m.alpha, al = m.alpha;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            // chunk c covers D1 elements 8 (c & 1) + e'; in a lane of half h
            // the K index 8 h + e maps to element 8 (c & 1) + e of that half
            const int row = d1_row(8 * (c & 1) + e, h);
            const float w = (c < 2 ? ar : al) * m.v[row];
            n.a2[c][e] = (__bf16)(i == 0 ? w : 0.0f);
        }
    }
    n.b2 = m.b2;
    return n;
}

__device__ __forceinline__ unsigned pack_bf16(float lo, float hi)
{
    const __bf16 a = (__bf16)lo, b = (__bf16)hi;
    return (unsigned)__builtin_bit_cast(unsigned short, a) |
           ((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
}

__device__ __forceinline__ unsigned relu_bf16x2(unsigned v)
{
    // a bf16 is negative iff its sign bit is set, i.e. iff it is negative as
    // an int16; max with 0 keeps positives and maps negatives (and -0) to +0
    const short2v s = __builtin_bit_cast(short2v, v);
    const short2v z = {0, 0};
    return __builtin_bit_cast(unsigned, __builtin_elementwise_max(s, z));
}

// layer 2 for one group: returns the full D2 (row 0 = y in lanes 0..31)
__device__ __forceinline__ float net_group(const NetBf16 &n, bf16x8 b1op)
{
    floatx16 d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(n.a1, b1op, n.c1, 0, 0, 0);
    unsigned raw[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        raw[q] = pack_bf16(d[2 * q], d[2 * q + 1]);
    floatx16 y = {};
    y[0] = (threadIdx.x & 63) < 32 ? n.b2 : 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned v = raw[4 * (c & 1) + q];
            w[q] = c < 2 ? relu_bf16x2(v) : v;
        }
        const bf16x8 b = __builtin_bit_cast(bf16x8, w);
        y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(n.a2[c], b, y, 0, 0, 0);
    }
    return y[0];
}

// Network output y for the point of this lane (u: K inputs as exact floats).
__device__ __forceinline__ float net_bf16(const NetBf16 &n, const float (&u)[6])
{
    const int l = threadIdx.x & 63;
    unsigned p[4];
    p[0] = pack_bf16(u[0], u[1]);
    p[1] = pack_bf16(u[2], u[3]);
    p[2] = pack_bf16(u[4], u[5]);
    p[3] = 0u;
    // group 0: points of lanes 0..31; group 1: points of lanes 32..63 (moved down)
    unsigned g0[4], g1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const unsigned other = (unsigned)__shfl_xor((int)p[q], 32, 64);
        g0[q] = l < 32 ? p[q] : 0u;
        g1[q] = l < 32 ? other : 0u;
    }
    const float y0 = net_group(n, __builtin_bit_cast(bf16x8, g0));
    const float y1 = net_group(n, __builtin_bit_cast(bf16x8, g1));
    const float y1_up = __shfl_xor(y1, 32, 64);
    return l < 32 ? y0 : y1_up;
}

// Prediction of the point of this lane with the BF16 network where every
// neighbour exists, else one-layer Lorenzo (as predict<>).  Wave-uniform call.
template <int D>
__device__ __forceinline__ long long predict_bf16(const int (&nv)[8], int amask, bool net,
                                                  const NetBf16 &n)
{
    constexpr int NO = (1 << D) - 1;
    constexpr int K = (1 << D) - 2;
    const bool use = net && amask == NO;
    float u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        u[k] = (k < K && use) ? (float)(nv[k + 2] - nv[1]) : 0.0f;
    float y = net_bf16(n, u);
    long long s = 0;
#pragma unroll
    for (int o = 1; o <= NO; ++o)
        if ((o & ~amask) == 0)
            s += (long long)lorenzo_sign(o) * (long long)nv[o];
    if (y > 0x1p30f)
        y = 0x1p30f;
    if (!(y >= -0x1p30f))
        y = -0x1p30f;
    return use ? (long long)nv[1] + (long long)__builtin_rintf(y) : s;
}

}  // namespace pwrel
