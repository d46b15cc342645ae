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
// it packs its activations and the weights in bf16 pairs and sums them with
// v_dot2 (two exact bf16 products and an FP32 accumulation per instruction)
// in four partial sums in a fixed order; the two halves of a column are
// added, then b2.  Every point is evaluated by the same instruction sequence
// wherever it sits in the wave, so encoder and decoder agree bit for bit.
// Every lane of the wave must execute these calls (the matrix cores work on
// the whole wave); lanes without a point feed zero inputs.
#pragma once

#include "pwrel_kernels.h"

namespace pwrel {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

struct NetBf16 {
    bf16x8 a1;      // layer-1 A operand of this lane
    floatx16 c1;    // layer-1 accumulator init: b1 of the rows this lane holds
    unsigned a2[8]; // bf16((1 - alpha) v) of the rows this lane holds, in pairs
    unsigned c2[8]; // bf16(alpha v) of the same rows, in pairs
    float b2;
};

// hidden unit held by element e of D in a lane of half h
__device__ __forceinline__ int d1_row(int e, int h) { return 8 * (e / 4) + 4 * h + (e % 4); }

__device__ __forceinline__ float bf16_round(float f) { return (float)(__bf16)f; }

// v_permlane32_swap: lanes 32..63 of the first operand trade places with
// lanes 0..31 of the second; the builtin returns the new first and second
// operands.  (Where both results of one swap fed the two operands of one
// FP32 add, hipcc 7.2 read the first result twice; the forms used here
// compile to distinct registers.)  The value of lane l ^ 32:
__device__ __forceinline__ unsigned xor32_lanes(unsigned x)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

// two floats to bf16 (round to nearest even), lo in bits 0..15: one
// v_cvt_pk_bf16_f32
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi)
{
    const f32x2 f = {lo, hi};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2));
}

// relu of two packed bf16 values.  A bf16 value with its sign bit set
// (negative, or -0) is a negative 16-bit integer and every other one a
// non-negative one, so a signed 16-bit max with 0 clears exactly the negative
// halves (one v_pk_max_i16).  Rounding to nearest even keeps the sign, so
// relu(bf16(z)) = bf16(max(z, 0)) (up to the sign of a zero, which no sum
// below can see).
__device__ __forceinline__ unsigned relu_bf16x2(unsigned z)
{
    const i16x2 v = __builtin_bit_cast(i16x2, z);
    return __builtin_bit_cast(unsigned, __builtin_elementwise_max(v, i16x2{0, 0}));
}

// layer-2 weights of the rows of elements 2q, 2q + 1 in a lane of half h
__device__ __forceinline__ unsigned a2_pair(const MlpW &m, int q, int h)
{
    const float ar = 1.0f - m.alpha;
    return pack_bf16(ar * m.v[d1_row(2 * q, h)], ar * m.v[d1_row(2 * q + 1, h)]);
}
__device__ __forceinline__ unsigned c2_pair(const MlpW &m, int q, int h)
{
    const float al = m.alpha;
    return pack_bf16(al * m.v[d1_row(2 * q, h)], al * m.v[d1_row(2 * q + 1, h)]);
}

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
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        n.a2[q] = a2_pair(m, q, h);
        n.c2[q] = c2_pair(m, q, h);
    }
    n.b2 = m.b2;
    return n;
}

__device__ __forceinline__ float dot2_bf16(unsigned a, unsigned b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a),
                                           __builtin_bit_cast(bf16x2, b), c, false);
}

// this lane's half of layer 2 for one group: its 16 hidden units
__device__ __forceinline__ float layer2_half(const unsigned (&a2)[8], const unsigned (&c2)[8],
                                             const floatx16 &d)
{
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        // bf16(z) (round to nearest even) and relu(bf16 z)
        const unsigned z0 = pack_bf16(d[2 * q], d[2 * q + 1]);
        const unsigned r0 = relu_bf16x2(z0);
        const unsigned z1 = pack_bf16(d[2 * q + 2], d[2 * q + 3]);
        const unsigned r1 = relu_bf16x2(z1);
        s0 = dot2_bf16(a2[q], r0, s0);
        s1 = dot2_bf16(c2[q], z0, s1);
        s2 = dot2_bf16(a2[q + 1], r1, s2);
        s3 = dot2_bf16(c2[q + 1], z1, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

// Both groups of layer 1 (lanes 0..31 and lanes 32..63 as the 32 columns),
// then layer 2; c1, a2, c2 as in NetBf16 for this lane's half.
__device__ __forceinline__ float net_bf16_core(const bf16x8 &a1, const floatx16 &c1,
                                               const unsigned (&a2)[8], const unsigned (&c2)[8],
                                               float b2, const float (&u)[6])
{
    const int l = threadIdx.x & 63;
    unsigned p[3];
    p[0] = pack_bf16(u[0], u[1]);
    p[1] = pack_bf16(u[2], u[3]);
    p[2] = pack_bf16(u[4], u[5]);
    // group 0: points of lanes 0..31 (lanes 32..63 zero: B rows 8..15);
    // group 1: points of lanes 32..63 moved down.  One swap with zero gives
    // both: the first operand keeps lanes 0..31 and receives zeros above, the
    // second receives lanes 32..63 below and keeps its zeros above.
    unsigned g0[4], g1[4];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const auto r = __builtin_amdgcn_permlane32_swap(p[q], 0u, false, false);
        g0[q] = r[0];
        g1[q] = r[1];
    }
    g0[3] = 0u;
    g1[3] = 0u;
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
// instead of registers: per half h, 32 words at t + 32 h (c1 as 16 floats,
// then the 8 a2 pairs and the 8 c2 pairs).
struct NetBf16Lds {
    bf16x8 a1;
    const unsigned *t;
    float b2;
};

__device__ __forceinline__ void stage_net_bf16(unsigned *t, const MlpW &m)
{
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        const int h = i >> 5, k = i & 31;
        t[i] = k < 16   ? __builtin_bit_cast(unsigned, m.b1[d1_row(k, h)])
               : k < 24 ? a2_pair(m, k - 16, h)
                        : c2_pair(m, k - 24, h);
    }
}

__device__ __forceinline__ NetBf16Lds make_net_bf16_lds(const MlpW &m, int K, const unsigned *t)
{
    NetBf16Lds n;
    const int l = threadIdx.x & 63, h = l >> 5, i = l & 31;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * h + e;
        n.a1[e] = (__bf16)(k < K ? m.w1[i][k] : 0.0f);
    }
    n.t = t + 32 * h;
    n.b2 = m.b2;
    return n;
}

__device__ __forceinline__ float net_bf16(const NetBf16Lds &n, const float (&u)[6])
{
    const uint4 *t4 = reinterpret_cast<const uint4 *>(n.t);
    floatx16 c1;
    unsigned a2[8], c2[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 c = t4[q];
        c1[4 * q] = __builtin_bit_cast(float, c.x);
        c1[4 * q + 1] = __builtin_bit_cast(float, c.y);
        c1[4 * q + 2] = __builtin_bit_cast(float, c.z);
        c1[4 * q + 3] = __builtin_bit_cast(float, c.w);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const uint4 a = t4[4 + q], v = t4[6 + q];
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
