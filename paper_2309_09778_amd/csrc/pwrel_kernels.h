// Device helpers shared by the compression and decompression kernels.
#pragma once

#include <type_traits>

#include <algorithm>

#include "pwrel_internal.h"

namespace pwrel {

// Network weights as a kernel argument (scalar-loaded, uniform across lanes).
// Hidden units beyond `hidden` are zero: they add fma(0, 0, y) to the output,
// which leaves every rounded prediction unchanged.
struct MlpW {
    float w1[PWREL_MAX_HIDDEN][PWREL_MAX_INPUTS];
    float b1[PWREL_MAX_HIDDEN];
    float v[PWREL_MAX_HIDDEN];
    float b2;
    float alpha;
};

inline MlpW pack_mlp(const pwrel_mlp *m)
{
    MlpW w{};
    if (!m)
        return w;
    for (int j = 0; j < m->hidden; ++j) {
        for (int k = 0; k < m->inputs; ++k)
            w.w1[j][k] = m->w1[j][k];
        w.b1[j] = m->b1[j];
        w.v[j] = m->v[j];
    }
    w.b2 = m->b2;
    w.alpha = m->alpha;
    return w;
}

inline int hidden_pad(const pwrel_mlp *m)
{
    if (!m || m->hidden <= 8)
        return 8;
    return m->hidden <= 16 ? 16 : 32;
}

__device__ __forceinline__ void set_status(int *status, int code)
{
    if (code != kOk)
        atomicCAS(status, kOk, code);
}

// Network weights staged in LDS, two float4 per hidden unit:
//   [w1[j][0..3]] [w1[j][4], w1[j][5], b1[j], v[j]]
// Every lane reads the same address (a broadcast), so the 130-258 uniform
// weights neither occupy nor spill scalar registers.
constexpr int kWlds = 2 * PWREL_MAX_HIDDEN;

template <int HP>
__device__ __forceinline__ void stage_weights(float4 *wl, const MlpW &m)
{
    for (int j = threadIdx.x; j < HP; j += blockDim.x) {
        wl[2 * j] = make_float4(m.w1[j][0], m.w1[j][1], m.w1[j][2], m.w1[j][3]);
        wl[2 * j + 1] = make_float4(m.w1[j][4], m.w1[j][5], m.b1[j], m.v[j]);
    }
}

// Weight access for the prediction: from LDS (broadcast loads) or from a
// register copy made once per kernel.
struct WeightsLds {
    const float4 *wl;
    __device__ __forceinline__ float4 a(int j) const { return wl[2 * j]; }
    __device__ __forceinline__ float4 b(int j) const { return wl[2 * j + 1]; }
};

template <int HP> struct WeightsReg {
    float4 wa[HP], wb[HP];
    __device__ __forceinline__ void load(const float4 *wl)
    {
#pragma unroll
        for (int j = 0; j < HP; ++j) {
            wa[j] = wl[2 * j];
            wb[j] = wl[2 * j + 1];
        }
    }
    __device__ __forceinline__ float4 a(int j) const { return wa[j]; }
    __device__ __forceinline__ float4 b(int j) const { return wb[j]; }
};

// Prediction of one point (Sec. 4.1 / 4.2 with the data selection rule of
// Sec. 4.4.1: the inputs are grid values of the neighbours).
//   nv[o], o = 1 .. 2^D-1 : neighbour grid values; bit i of o = one step back
//                           along axis 2-i (axis 2 is the fastest).
//   amask                 : bit i set iff axis 2-i has a neighbour.
// The network applies when every neighbour exists; otherwise the one-layer
// Lorenzo predictor with missing neighbours counted as zero.  The leaky ReLU
// is max(z, alpha z), equal to (z < 0 ? alpha z : z) for 0 <= alpha <= 1.
template <int D, int HP, class W>
__device__ __forceinline__ long long predict(const int (&nv)[8], int amask, bool net,
                                             const W &wt, float b2, float alpha)
{
    constexpr int NO = (1 << D) - 1;
    constexpr int K = (1 << D) - 2;
    if (net && amask == NO) {
        float u[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            u[k] = k < K ? (float)(nv[k + 2] - nv[1]) : 0.0f;
        float y = b2;
        auto unit = [&](int j) {
            const float4 wa = wt.a(j), wb = wt.b(j);
            const float w[6] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y};
            float z = wb.z;
#pragma unroll
            for (int k = 0; k < K; ++k)
                z = __builtin_fmaf(w[k], u[k], z);
            const float h = __builtin_fmaxf(z, z * alpha);
            y = __builtin_fmaf(wb.w, h, y);
        };
        if constexpr (std::is_same<W, WeightsLds>::value) {
            // weights read from LDS four units at a time (bounded register use)
#pragma unroll 1
            for (int j0 = 0; j0 < HP; j0 += 4) {
#pragma unroll
                for (int j = j0; j < j0 + 4; ++j)
                    unit(j);
            }
        } else {
#pragma unroll
            for (int j = 0; j < HP; ++j)
                unit(j);
        }
        if (y > 0x1p30f)
            y = 0x1p30f;
        if (!(y >= -0x1p30f))
            y = -0x1p30f;
        return (long long)nv[1] + (long long)__builtin_rintf(y);
    }
    long long s = 0;
#pragma unroll
    for (int o = 1; o <= NO; ++o)
        if ((o & ~amask) == 0)
            s += (long long)lorenzo_sign(o) * (long long)nv[o];
    return s;
}

// FP32 network output (the evaluation order of predict<>)
template <int D, int HP, class W>
__device__ __forceinline__ float net_f32(const int (&nv)[8], const W &wt, float b2, float alpha)
{
    constexpr int K = (1 << D) - 2;
    float u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        u[k] = k < K ? (float)(nv[k + 2] - nv[1]) : 0.0f;
    float y = b2;
#pragma unroll 1
    for (int j0 = 0; j0 < HP; j0 += 4) {
#pragma unroll
        for (int j = j0; j < j0 + 4; ++j) {
            const float4 wa = wt.a(j), wb = wt.b(j);
            const float w[6] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y};
            float z = wb.z;
#pragma unroll
            for (int k = 0; k < K; ++k)
                z = __builtin_fmaf(w[k], u[k], z);
            const float h = __builtin_fmaxf(z, z * alpha);
            y = __builtin_fmaf(wb.w, h, y);
        }
    }
    return y;
}

// Compile-time tile shapes (points per axis, multiples of the block edge) of
// the common block sizes; ShapeOf<D, 0> means "runtime shape".
template <int D, int BB> struct ShapeOf {
    static constexpr bool known = false;
    static constexpr int T0 = 0, T1 = 0, T2 = 0;
};
#define PWREL_SHAPE(DD, BB_, A, Bv, Cv)                                                       \
    template <> struct ShapeOf<DD, BB_> {                                                     \
        static constexpr bool known = true;                                                   \
        static constexpr int T0 = A, T1 = Bv, T2 = Cv;                                        \
    };
PWREL_SHAPE(3, 4, 8, 8, 32)
PWREL_SHAPE(3, 8, 8, 8, 32)
PWREL_SHAPE(3, 16, 16, 16, 32)
PWREL_SHAPE(2, 16, 1, 16, 128)
PWREL_SHAPE(2, 32, 1, 32, 128)
PWREL_SHAPE(2, 64, 1, 64, 64)
PWREL_SHAPE(1, 256, 1, 1, 4096)
#undef PWREL_SHAPE

// Host-side copy of the same table.
inline bool known_shape(int D, int B, int *t)
{
    struct E {
        int D, B, t0, t1, t2;
    };
    static const E tab[] = {{3, 4, 8, 8, 32},    {3, 8, 8, 8, 32},     {3, 16, 16, 16, 32},
                            {2, 16, 1, 16, 128}, {2, 32, 1, 32, 128},  {2, 64, 1, 64, 64},
                            {1, 256, 1, 1, 4096}};
    for (const E &e : tab)
        if (e.D == D && e.B == B) {
            t[0] = e.t0;
            t[1] = e.t1;
            t[2] = e.t2;
            return true;
        }
    return false;
}



// Tile shapes of the batched launch: variant 0 is the shape above; variants
// 1 and 2 group the same blocks otherwise (fewer halo entries per point, or
// larger tiles at lower occupancy).  Tiles only schedule work: every variant
// writes the same stream, so the batch autotuner may pick any by time.
constexpr int kTileVariants = 3;
template <int D, int BB, int TV> struct TileOf : ShapeOf<D, BB> {};
#define PWREL_TILE(DD, BB_, V, A, Bv, Cv)                                                     \
    template <> struct TileOf<DD, BB_, V> {                                                   \
        static constexpr bool known = true;                                                   \
        static constexpr int T0 = A, T1 = Bv, T2 = Cv;                                        \
    };
PWREL_TILE(3, 8, 1, 8, 16, 16)
PWREL_TILE(3, 8, 2, 16, 16, 16)
PWREL_TILE(2, 16, 1, 1, 32, 64)
PWREL_TILE(2, 16, 2, 1, 16, 256)
#undef PWREL_TILE

// Host-side copy: the tile of variant v of the (D, B) shape.
inline bool variant_shape(int D, int B, int v, int *t)
{
    if (v == 0)
        return known_shape(D, B, t);
    struct E {
        int D, B, v, t0, t1, t2;
    };
    static const E tab[] = {{3, 8, 1, 8, 16, 16},
                            {3, 8, 2, 16, 16, 16},
                            {2, 16, 1, 1, 32, 64},
                            {2, 16, 2, 1, 16, 256}};
    for (const E &e : tab)
        if (e.D == D && e.B == B && e.v == v) {
            t[0] = e.t0;
            t[1] = e.t1;
            t[2] = e.t2;
            return true;
        }
    return false;
}

// Start of block (bz, by, bx) in the block-major stream and its extents.
struct BlockGeo {
    long long bz, by, bx;
    int ez, ey, ex;
    long long start;
};

__device__ __forceinline__ BlockGeo block_geo3(long long bz, long long by, long long bx,
                                               const long long *n, int bd0, int bd1, int bd2)
{
    BlockGeo q;
    q.bz = bz;
    q.by = by;
    q.bx = bx;
    q.ez = (int)std::min((long long)bd0, n[0] - bz * bd0);
    q.ey = (int)std::min((long long)bd1, n[1] - by * bd1);
    q.ex = (int)std::min((long long)bd2, n[2] - bx * bd2);
    q.start = bz * bd0 * n[1] * n[2] + (long long)q.ez * (by * bd1 * n[2]) +
              (long long)q.ez * q.ey * (bx * bd2);
    return q;
}

}  // namespace pwrel
