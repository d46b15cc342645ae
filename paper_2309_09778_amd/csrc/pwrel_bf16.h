// The perceptron with its first layer on the matrix cores: 64 points per
// wave (lane l = point l), v_mfma_f32_32x32x16_bf16, two groups of 32 points.
//
// Operand layout of v_mfma_f32_32x32x16_bf16 (checked on the device):
//   A (32 x 16):  lane l, element e  ->  A[l % 32][8 (l / 32) + e]
//   B (16 x 32):  lane l, element e  ->  B[8 (l / 32) + e][l % 32]
//   C/D (32x32):  lane l, element e  ->  D[8 (e / 4) + 4 (l / 32) + e % 4][l % 32]
//
// Layer 1: Z (hidden x points) = bf16(w1) (hidden x K, K padded to 16)
//          . bf16(U) (K x points) + b1 (in the FP32 accumulator).
// Layer 2 (a matrix-vector product: on the vector ALU), with
// lrelu(z) = (1 - alpha) relu(z) + alpha z:
//   y = b2 + sum_j bf16((1-alpha) v_j) relu(bf16(z_j)) + bf16(alpha v_j) bf16(z_j).
// Lane l holds 16 of the 32 hidden units of column l % 32 (half h = l / 32);
// it sums them in a fixed order with FP32 fused multiply-adds (four partial
// sums, then their sum), the two halves of a column are added, then b2.  Every point is evaluated by the
// same instruction sequence wherever it sits in the wave, so encoder and
// decoder agree bit for bit.
// Every lane of the wave must execute these calls (the matrix cores work on
// the whole wave); lanes without a point feed zero inputs.
#pragma once

#include "pwrel_kernels.h"

namespace pwrel {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

struct NetBf16 {
    bf16x8 a1;      // layer-1 A operand of this lane
    floatx16 c1;    // layer-1 accumulator init: b1 of the rows this lane holds
    float a2[16];   // bf16((1 - alpha) v) of the rows this lane holds
    float c2[16];   // bf16(alpha v) of the same rows
    float b2;
};

// hidden unit held by element e of D in a lane of half h
__device__ __forceinline__ int d1_row(int e, int h) { return 8 * (e / 4) + 4 * h + (e % 4); }

__device__ __forceinline__ float bf16_round(float f) { return (float)(__bf16)f; }

__device__ __forceinline__ NetBf16 make_net_bf16(const MlpW &m, int K)
{
    NetBf16 n;
    const int l = threadIdx.x & 63, h = l >> 5, i = l & 31;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * h + e;
        n.a1[e] = (__bf16)(k < K ? m.w1[i][k] : 0.0f);
    }
    const float ar = 1.0f - m.alpha, al = m.alpha;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int row = d1_row(e, h);
        n.c1[e] = m.b1[row];
        n.a2[e] = bf16_round(ar * m.v[row]);
        n.c2[e] = bf16_round(al * m.v[row]);
    }
    n.b2 = m.b2;
    return n;
}

// the value of lane l ^ 32 (v_permlane32_swap: lanes 32..63 of the first
// operand trade places with lanes 0..31 of the second)
__device__ __forceinline__ unsigned xor32_lanes(unsigned x)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
}

__device__ __forceinline__ unsigned pack_bf16(float lo, float hi)
{
    const __bf16 a = (__bf16)lo, b = (__bf16)hi;
    return (unsigned)__builtin_bit_cast(unsigned short, a) |
           ((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
}

// this lane's half of layer 2 for one group: sum over its 16 hidden units,
// in four partial sums (relu and linear terms of even and odd units) added
// as (s0 + s1) + (s2 + s3)
__device__ __forceinline__ float layer2_half(const float (&a2)[16], const float (&c2)[16],
                                             const floatx16 &d)
{
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const unsigned pk = pack_bf16(d[2 * q], d[2 * q + 1]);  // round to bf16 (RNE)
        const float z0 = __builtin_bit_cast(float, pk << 16);
        const float z1 = __builtin_bit_cast(float, pk & 0xffff0000u);
        s0 = __builtin_fmaf(a2[2 * q], __builtin_fmaxf(z0, 0.0f), s0);
        s1 = __builtin_fmaf(c2[2 * q], z0, s1);
        s2 = __builtin_fmaf(a2[2 * q + 1], __builtin_fmaxf(z1, 0.0f), s2);
        s3 = __builtin_fmaf(c2[2 * q + 1], z1, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

// Both groups of layer 1 (lanes 0..31 and lanes 32..63 as the 32 columns),
// then layer 2; c1, a2, c2 as in NetBf16 for this lane's half.
__device__ __forceinline__ float net_bf16_core(const bf16x8 &a1, const floatx16 &c1,
                                               const float (&a2)[16], const float (&c2)[16],
                                               float b2, const float (&u)[6])
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
        const unsigned other = xor32_lanes(p[q]);
        g0[q] = l < 32 ? p[q] : 0u;
        g1[q] = l < 32 ? other : 0u;
    }
    const floatx16 d0 =
        __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, __builtin_bit_cast(bf16x8, g0), c1, 0, 0, 0);
    const floatx16 d1 =
        __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, __builtin_bit_cast(bf16x8, g1), c1, 0, 0, 0);
    const float s0 = layer2_half(a2, c2, d0), s1 = layer2_half(a2, c2, d1);
    // lane l < 32 owns column l of group 0: halves s0 (own, h = 0) + s0 of lane l + 32;
    // lane l >= 32 owns column l - 32 of group 1: s1 of lane l - 32 (h = 0) + s1 (own)
    const float send = l < 32 ? s1 : s0;
    const float recv = __builtin_bit_cast(float, xor32_lanes(__builtin_bit_cast(unsigned, send)));
    const float lo = l < 32 ? s0 : recv, hi = l < 32 ? recv : s1;
    return (lo + hi) + b2;
}

// Network output y for the point of this lane (u: K inputs as exact floats).
__device__ __forceinline__ float net_bf16(const NetBf16 &n, const float (&u)[6])
{
    return net_bf16_core(n.a1, n.c1, n.a2, n.c2, n.b2, u);
}

// The same network with c1, a2 and c2 kept in LDS (read at each evaluation)
// instead of registers: per half h, 48 floats at t + 48 h (c1, a2, c2).
struct NetBf16Lds {
    bf16x8 a1;
    const float *t;
    float b2;
};

__device__ __forceinline__ void stage_net_bf16(float *t, const MlpW &m)
{
    const float ar = 1.0f - m.alpha, al = m.alpha;
    for (int i = threadIdx.x; i < 32; i += blockDim.x) {
        const int h = i >> 4, e = i & 15, row = d1_row(e, h);
        t[48 * h + e] = m.b1[row];
        t[48 * h + 16 + e] = bf16_round(ar * m.v[row]);
        t[48 * h + 32 + e] = bf16_round(al * m.v[row]);
    }
}

__device__ __forceinline__ NetBf16Lds make_net_bf16_lds(const MlpW &m, int K, const float *t)
{
    NetBf16Lds n;
    const int l = threadIdx.x & 63, h = l >> 5, i = l & 31;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * h + e;
        n.a1[e] = (__bf16)(k < K ? m.w1[i][k] : 0.0f);
    }
    n.t = t + 48 * h;
    n.b2 = m.b2;
    return n;
}

__device__ __forceinline__ float net_bf16(const NetBf16Lds &n, const float (&u)[6])
{
    const float4 *t4 = reinterpret_cast<const float4 *>(n.t);
    floatx16 c1;
    float a2[16], c2[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 c = t4[q], a = t4[4 + q], v = t4[8 + q];
        c1[4 * q] = c.x; c1[4 * q + 1] = c.y; c1[4 * q + 2] = c.z; c1[4 * q + 3] = c.w;
        a2[4 * q] = a.x; a2[4 * q + 1] = a.y; a2[4 * q + 2] = a.z; a2[4 * q + 3] = a.w;
        c2[4 * q] = v.x; c2[4 * q + 1] = v.y; c2[4 * q + 2] = v.z; c2[4 * q + 3] = v.w;
    }
    return net_bf16_core(n.a1, c1, a2, c2, n.b2, u);
}

// Prediction of the point of this lane with the BF16 network where every
// neighbour exists, else one-layer Lorenzo (as predict<>).  Wave-uniform call.
template <int D, class N>
__device__ __forceinline__ long long predict_bf16(const int (&nv)[8], int amask, bool net,
                                                  const N &n)
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
