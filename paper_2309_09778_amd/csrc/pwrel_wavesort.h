// Sorting and run counting of 16-bit keys held by a wave, on the vector ALU
// (DPP row/quad moves and the gfx950 lane swaps; the run scan shuffles
// through the LDS crossbar; the 512-element sort moves its register layouts
// through LDS instead).  Every 32-bit element carries two keys (low and high
// half) that are sorted as two separate sequences by one bitonic network on
// packed 16-bit minima/maxima.
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

// Sorting 512 elements (8 a lane) with every compare-exchange inside a lane.
// Bitonic sort with directions: merge s (blocks of 2^s elements) runs its
// stages on index bits s - 1 .. 0, and a block whose bit s is set sorts
// descending.  Elements of descending blocks are held complemented (the
// minimum of complements is the complement of the maximum), so every stage
// keeps the minimum at the lower index and the direction costs one XOR per
// element at each change of merge.  An element index has 9 bits; three
// layouts put three of them in a lane's registers: layout 0 bits 0-2
// (element 8 lane + k, lane-major), layout 1 bits 3-5, layout 2 bits 6-8.
// Between layouts the wave moves its elements through 568 words of LDS that
// it alone uses: element i sits in word i + 8 (i >> 6), so the words that
// layouts 1 and 2 access at one register index fall in 64 different banks.
constexpr int kSortLdsWords = 568;

template <int M> __device__ __forceinline__ int ls_base(int l)
{
    if constexpr (M == 0)
        return 8 * l + 8 * (l >> 3);
    else if constexpr (M == 1)
        return (l & 7) + 72 * (l >> 3);
    else
        return l;
}
template <int M> __host__ __device__ constexpr int ls_off(int k)
{
    return M == 0 ? k : (M == 1 ? 8 * k : 72 * k);
}

// the wave's LDS accesses before this point are ordered before those after
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int FROM, int TO>
__device__ __forceinline__ void ls_move(unsigned (&a)[8], unsigned *scr, int lane)
{
    unsigned *w = scr + ls_base<FROM>(lane);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        w[ls_off<FROM>(k)] = a[k];
    wave_lds_sync();
    const unsigned *r = scr + ls_base<TO>(lane);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        a[k] = r[ls_off<TO>(k)];
    wave_lds_sync();
}

// the stage on the index bit held by register bit R: pairs k, k | 2^R
template <int R> __device__ __forceinline__ void ls_stage(unsigned (&a)[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k & (1 << R))
            continue;
        const unsigned x = a[k], y = a[k | (1 << R)];
        a[k] = pk_min16(x, y);
        a[k | (1 << R)] = pk_max16(x, y);
    }
}

// merge S >= 4, entered and left in layout 0
template <int S>
__device__ __forceinline__ void ls_merge(unsigned (&a)[8], unsigned *scr, int lane)
{
    // direction: bit S - 1 (lane bit S - 4) out, bit S (lane bit S - 3; none for S = 9) in
    const unsigned m = (((lane >> (S - 4)) ^ (lane >> (S - 3))) & 1) ? 0xFFFFFFFFu : 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        a[k] ^= m;
    if constexpr (S >= 7) {
        ls_move<0, 2>(a, scr, lane);
        if constexpr (S >= 9)
            ls_stage<2>(a);
        if constexpr (S >= 8)
            ls_stage<1>(a);
        ls_stage<0>(a);
        ls_move<2, 1>(a, scr, lane);
    } else {
        ls_move<0, 1>(a, scr, lane);
    }
    if constexpr (S >= 6)
        ls_stage<2>(a);
    if constexpr (S >= 5)
        ls_stage<1>(a);
    ls_stage<0>(a);
    ls_move<1, 0>(a, scr, lane);
    ls_stage<2>(a);
    ls_stage<1>(a);
    ls_stage<0>(a);
}

// Sorts the wave's 512 elements (8 a lane, lane-major on return), both
// 16-bit halves as separate sequences; scr: kSortLdsWords words of LDS,
// 16-byte aligned, used by this wave only.
__device__ __forceinline__ void wave_sort_lds8(unsigned (&a)[8], unsigned *scr)
{
    const int lane = threadIdx.x & 63;
    // merges 1-3 inside the lane (layout 0); merge s complements where bit s is set
    a[2] = ~a[2];
    a[3] = ~a[3];
    a[6] = ~a[6];
    a[7] = ~a[7];
    ls_stage<0>(a);
    a[2] = ~a[2];
    a[3] = ~a[3];
    a[4] = ~a[4];
    a[5] = ~a[5];
    ls_stage<1>(a);
    ls_stage<0>(a);
    {
        const unsigned m = (lane & 1) ? 0xFFFFFFFFu : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            a[k] ^= (k & 4) ? ~m : m;
    }
    ls_stage<2>(a);
    ls_stage<1>(a);
    ls_stage<0>(a);
    ls_merge<4>(a, scr, lane);
    ls_merge<5>(a, scr, lane);
    ls_merge<6>(a, scr, lane);
    ls_merge<7>(a, scr, lane);
    ls_merge<8>(a, scr, lane);
    ls_merge<9>(a, scr, lane);
}

// Multiset scores of both halves of lane-major sorted elements:
// J_h = sum over the runs of equal keys of c q(c), c the run's length (the
// run of key 0xFFFF less `nsent` stand-ins).  A run starts where the key
// differs from its predecessor; its start is found by the lane itself or,
// for a run entering from lower lanes, by an exclusive prefix maximum of the
// lanes' last starts.  Positions are kept + 1 (0 = none) in packed halves.
// (CQ: qtab[c] already holds c q(c))
template <int EPL, bool CQ = false>
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
        // a run ends here: its length (0 otherwise, which adds 0 q(0) = 0);
        // the lookups take no branch, so they are issued back to back
        const bool tail = k == EPL - 1 && lane == 63;
        int c0 = (int)pos1 - (int)(st & 0xFFFFu) + 1;
        if ((a[k] & 0xFFFFu) == 0xFFFFu)
            c0 -= (int)nsent;
        const unsigned e0 = ((tail || (y & 0xFFFFu)) && c0 > 0) ? (unsigned)c0 : 0u;
        int c1 = (int)pos1 - (int)(st >> 16) + 1;
        if ((a[k] >> 16) == 0xFFFFu)
            c1 -= (int)nsent;
        const unsigned e1 = ((tail || (y >> 16)) && c1 > 0) ? (unsigned)c1 : 0u;
        if constexpr (CQ) {
            s0 += (unsigned long long)qtab[e0];
            s1 += (unsigned long long)qtab[e1];
        } else {
            s0 += (unsigned long long)e0 * (unsigned long long)qtab[e0];
            s1 += (unsigned long long)e1 * (unsigned long long)qtab[e1];
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
