// Sorting and run counting of 16-bit keys held by a wave, on the vector ALU
// (DPP row/quad moves and the gfx950 lane swaps; the run scan shuffles
// through the LDS crossbar).  Every 32-bit element carries two keys (low and
// high half) that are sorted as two separate sequences by one bitonic network
// on packed 16-bit minima/maxima.
#pragma once

#include <hip/hip_runtime.h>

namespace pwrel {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

template <int CTRL> __device__ __forceinline__ unsigned dpp(unsigned v)
{
    return (unsigned)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

// the value of lane ^ D
template <int D> __device__ __forceinline__ unsigned lane_xor(unsigned v)
{
    const int lane = threadIdx.x & 63;
    if constexpr (D == 1) {
        return dpp<0xB1>(v);  // quad_perm [1, 0, 3, 2]
    } else if constexpr (D == 2) {
        return dpp<0x4E>(v);  // quad_perm [2, 3, 0, 1]
    } else if constexpr (D == 4) {
        const unsigned up = dpp<0x104>(v), dn = dpp<0x114>(v);  // row_shl:4 (lane + 4), row_shr:4
        return (lane & 4) ? dn : up;
    } else if constexpr (D == 8) {
        return dpp<0x128>(v);  // row_ror:8 (lane + 8 mod 16 = lane ^ 8)
    } else if constexpr (D == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
}

__device__ __forceinline__ unsigned pk_min16(unsigned a, unsigned b)
{
    return __builtin_bit_cast(unsigned, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                   __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ unsigned pk_max16(unsigned a, unsigned b)
{
    return __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                   __builtin_bit_cast(u16x2, b)));
}

// the value of lane ^ M, M in {1, 2, 3, 4, 7, 8, 15, 16, 31, 32, 63}
template <int M> __device__ __forceinline__ unsigned lane_xor_m(unsigned v)
{
    if constexpr (M == 3)
        return dpp<0x1B>(v);  // quad_perm [3, 2, 1, 0]
    else if constexpr (M == 7)
        return dpp<0x141>(v);  // row_half_mirror
    else if constexpr (M == 15)
        return dpp<0x140>(v);  // row_mirror
    else if constexpr (M == 31)
        return lane_xor<16>(dpp<0x140>(v));
    else if constexpr (M == 63)
        return lane_xor<32>(lane_xor<16>(dpp<0x140>(v)));
    else
        return lane_xor<M>(v);
}

// Sorting network over the wave's 64 EPL elements, lane-major: element
// i = lane EPL + k is register k of the lane, so pairs closer than EPL are
// compared inside a lane (no exchange, no select).  Bitonic sort in the form
// without directions: at each block size sz, compare i with its mirror
// i ^ (sz - 1) in the block, then with i ^ d for d = sz / 4 .. 1; the lower
// index keeps the minimum every time.  Both 16-bit halves of an element are
// sorted, as two separate sequences, by the same packed minima and maxima.

// pairs i, i ^ D (D < EPL: inside the lane)
template <int EPL, int D> __device__ __forceinline__ void lm_half(unsigned (&a)[EPL])
{
    if constexpr (D < EPL) {
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            if (k & D)
                continue;
            const unsigned x = a[k], y = a[k | D];
            a[k] = pk_min16(x, y);
            a[k | D] = pk_max16(x, y);
        }
    } else {
        constexpr int M = D / EPL;
        const bool up = (threadIdx.x & M) != 0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const unsigned b = lane_xor_m<M>(a[k]);
            a[k] = up ? pk_max16(a[k], b) : pk_min16(a[k], b);
        }
    }
}

// pairs i, i ^ (SZ - 1)
template <int EPL, int SZ> __device__ __forceinline__ void lm_flip(unsigned (&a)[EPL])
{
    if constexpr (SZ <= EPL) {
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int k2 = k ^ (SZ - 1);
            if (k2 < k)
                continue;
            const unsigned x = a[k], y = a[k2];
            a[k] = pk_min16(x, y);
            a[k2] = pk_max16(x, y);
        }
    } else {
        constexpr int M = SZ / EPL - 1, HB = (SZ / EPL) >> 1;
        const bool up = (threadIdx.x & HB) != 0;
        unsigned b[EPL];
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            b[k] = lane_xor_m<M>(a[k ^ (EPL - 1)]);
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            a[k] = up ? pk_max16(a[k], b[k]) : pk_min16(a[k], b[k]);
    }
}

template <int EPL, int D> __device__ __forceinline__ void lm_halves(unsigned (&a)[EPL])
{
    if constexpr (D >= 1) {
        lm_half<EPL, D>(a);
        lm_halves<EPL, D / 2>(a);
    }
}

template <int EPL, int SZ> __device__ __forceinline__ void lm_levels(unsigned (&a)[EPL])
{
    if constexpr (SZ <= 64 * EPL) {
        lm_flip<EPL, SZ>(a);
        lm_halves<EPL, SZ / 4>(a);
        lm_levels<EPL, 2 * SZ>(a);
    }
}

template <int EPL> __device__ __forceinline__ void wave_sort_lm(unsigned (&a)[EPL])
{
    lm_levels<EPL, 2>(a);
}

// Multiset scores of both halves of lane-major sorted elements:
// J_h = sum over the runs of equal keys of c q(c), c the run's length (the
// run of key 0xFFFF less `nsent` stand-ins).  A run starts where the key
// differs from its predecessor; its start is found by the lane itself or,
// for a run entering from lower lanes, by an exclusive prefix maximum of the
// lanes' last starts.  Positions are kept + 1 (0 = none) in packed halves.
template <int EPL>
__device__ __forceinline__ void wave_runs_lm(const unsigned (&a)[EPL], unsigned nsent,
                                             const long long *qtab, unsigned long long &J0,
                                             unsigned long long &J1)
{
    const int lane = threadIdx.x & 63;
    const unsigned prev = dpp<0x138>(a[EPL - 1]);  // wave_shr:1: last element of lane - 1
    const unsigned next = dpp<0x130>(a[0]);        // wave_shl:1: first element of lane + 1
    auto startmask = [&](int k) {
        const unsigned x = a[k] ^ (k > 0 ? a[k > 0 ? k - 1 : 0] : prev);
        if (k == 0 && lane == 0)
            return 0xFFFFFFFFu;
        return ((x & 0xFFFFu) ? 0xFFFFu : 0u) | ((x >> 16) ? 0xFFFF0000u : 0u);
    };
    unsigned last = 0u;
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const unsigned pos1 = (unsigned)(lane * EPL + k + 1);
        const unsigned m = startmask(k);
        last = ((pos1 | (pos1 << 16)) & m) | (last & ~m);
    }
    // exclusive prefix maximum over the lanes (packed halves)
    unsigned incl = last;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned o = (unsigned)__shfl_up((int)incl, d, 64);
        if (lane >= d)
            incl = pk_max16(incl, o);
    }
    unsigned st = (unsigned)__shfl_up((int)incl, 1, 64);
    if (lane == 0)
        st = 0u;
    unsigned long long s0 = 0ULL, s1 = 0ULL;
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const unsigned pos1 = (unsigned)(lane * EPL + k + 1);
        const unsigned m = startmask(k);
        st = ((pos1 | (pos1 << 16)) & m) | (st & ~m);
        const unsigned y = a[k] ^ (k + 1 < EPL ? a[k + 1 < EPL ? k + 1 : k] : next);
        const bool tail = k == EPL - 1 && lane == 63;
        if (tail || (y & 0xFFFFu)) {
            int c = (int)pos1 - (int)(st & 0xFFFFu) + 1;
            if ((a[k] & 0xFFFFu) == 0xFFFFu)
                c -= (int)nsent;
            if (c > 0)
                s0 += (unsigned long long)c * (unsigned long long)qtab[c];
        }
        if (tail || (y >> 16)) {
            int c = (int)pos1 - (int)(st >> 16) + 1;
            if ((a[k] >> 16) == 0xFFFFu)
                c -= (int)nsent;
            if (c > 0)
                s1 += (unsigned long long)c * (unsigned long long)qtab[c];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s0 += (unsigned long long)__shfl_xor((long long)s0, o, 64);
        s1 += (unsigned long long)__shfl_xor((long long)s1, o, 64);
    }
    J0 = s0;
    J1 = s1;
}

}  // namespace pwrel
