// Sorting and run counting of 16-bit keys held by a wave, on the vector ALU
// only (DPP row/quad moves and the gfx950 lane swaps: no LDS).  Every 32-bit
// element carries two keys (low and high half) that are sorted as two
// separate sequences by one bitonic network on packed 16-bit minima/maxima.
// Element i = k 64 + lane is register k of the lane, k < EPL.
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

// one compare-exchange stage at distance D < 64 (lanes) of merge size sz
template <int EPL, int D>
__device__ __forceinline__ void bitonic_lanes(unsigned (&a)[EPL], int sz)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int i = k * 64 + lane;
        const unsigned b = lane_xor<D>(a[k]);
        const bool keep_lo = ((i & D) == 0) == ((i & sz) == 0);
        a[k] = keep_lo ? pk_min16(a[k], b) : pk_max16(a[k], b);
    }
}

// Sort both halves ascending in i (bitonic network: pairs i, i ^ d, in a
// lane's registers for d >= 64, by lane exchanges below).
template <int EPL> __device__ __forceinline__ void wave_sort_pk16(unsigned (&a)[EPL])
{
    constexpr int N = EPL * 64;
#pragma unroll
    for (int sz = 2; sz <= N; sz <<= 1) {
#pragma unroll
        for (int d = sz >> 1; d > 0; d >>= 1) {
            if (d >= 64) {
                const int dk = d >> 6;
#pragma unroll
                for (int k = 0; k < EPL; ++k) {
                    if (k & dk)
                        continue;
                    const bool asc = ((k * 64) & sz) == 0;
                    const unsigned x = a[k], y = a[k | dk];
                    const unsigned lo = pk_min16(x, y), hi = pk_max16(x, y);
                    a[k] = asc ? lo : hi;
                    a[k | dk] = asc ? hi : lo;
                }
            } else if (d == 32) {
                bitonic_lanes<EPL, 32>(a, sz);
            } else if (d == 16) {
                bitonic_lanes<EPL, 16>(a, sz);
            } else if (d == 8) {
                bitonic_lanes<EPL, 8>(a, sz);
            } else if (d == 4) {
                bitonic_lanes<EPL, 4>(a, sz);
            } else if (d == 2) {
                bitonic_lanes<EPL, 2>(a, sz);
            } else {
                bitonic_lanes<EPL, 1>(a, sz);
            }
        }
    }
}

// Runs of equal keys in sorted halves: f(half, key, count) is called by the
// lane holding the last element of each run.  A run ends where the successor
// differs and starts at the last run start at or before it (the highest set
// bit of a ballot of run starts, carried across registers).
template <int EPL, class F> __device__ __forceinline__ void wave_runs_pk16(const unsigned (&a)[EPL], F f)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long lowmask = lane == 63 ? ~0ULL : ((2ULL << lane) - 1ULL);
    int carry[2] = {-1, -1};
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int i = k * 64 + lane;
        const unsigned pw = dpp<0x138>(a[k]);  // wave_shr:1: lane - 1
        const unsigned nw = dpp<0x130>(a[k]);  // wave_shl:1: lane + 1
        const unsigned lp = k > 0 ? __builtin_amdgcn_readlane(a[k > 0 ? k - 1 : 0], 63) : 0u;
        const unsigned fn = k + 1 < EPL ? __builtin_amdgcn_readlane(a[k + 1 < EPL ? k + 1 : k], 0)
                                        : 0u;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const unsigned key = (a[k] >> (16 * h)) & 0xFFFFu;
            unsigned pk = (pw >> (16 * h)) & 0xFFFFu, nk = (nw >> (16 * h)) & 0xFFFFu;
            if (lane == 0)
                pk = k > 0 ? (lp >> (16 * h)) & 0xFFFFu : key ^ 1u;
            if (lane == 63)
                nk = k + 1 < EPL ? (fn >> (16 * h)) & 0xFFFFu : key ^ 1u;
            const unsigned long long sm = __ballot(key != pk);
            const unsigned long long m = sm & lowmask;
            const int st = m ? k * 64 + 63 - __clzll((long long)m) : carry[h];
            if (sm)
                carry[h] = k * 64 + 63 - __clzll((long long)sm);
            if (key != nk)
                f(h, key, i - st + 1);
        }
    }
}

}  // namespace pwrel
