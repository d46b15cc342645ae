// Independent-block decoder with one lane per block.
//
// With independent blocks (Sec. 4.4.2: every sub-block decodes on its own,
// starting from its first point) no block reads another, so a wave decodes 64
// whole blocks at once, lane l holding block l, all lanes at the same local
// point in the same step.  Every step is then the same for the whole wave:
// the same neighbours exist, the same branch is taken, and the network's first
// layer for the wave's 64 points is one pair of matrix-core instructions with
// every lane busy (a lane whose block keeps Lorenzo by the judge takes the
// Lorenzo value).  A lane walks its block row by row along x: the codes of a
// row are one 16-byte load (8^3 blocks), the previous row of the plane stays in
// registers, row y of the previous plane comes from an LDS ring of B rows per
// lane (its row y - 1 is the one read for the row before), and x^ of the row is written as one contiguous run (64 lanes
// = 64 neighbouring blocks = one coalesced stretch of the field).
//
// Only whole blocks go here, of fields whose grid values span less than 2^27
// (prediction arithmetic in 32 bits); blocks clipped by the field's high faces
// are decoded by the workgroup-per-block kernel.  A decoded grid value must
// lie in [p_zero, p_max] (else the stream is corrupt); x^ comes from the
// table of every grid value's inverse where the decompression built one.
#include "pwrel_bf16.h"
#include "pwrel_decode.h"

namespace pwrel {

namespace {

// B codes of a block row, two per 32-bit word
template <int B> struct RowCodes {
    uint32_t w[B / 2];
    __device__ __forceinline__ void load(const uint16_t *p)
    {
        if constexpr (B == 4) {
            const uint2 v = *reinterpret_cast<const uint2 *>(p);
            w[0] = v.x;
            w[1] = v.y;
        } else {
#pragma unroll
            for (int q = 0; q < B / 8; ++q) {
                const uint4 v = reinterpret_cast<const uint4 *>(p)[q];
                w[4 * q] = v.x;
                w[4 * q + 1] = v.y;
                w[4 * q + 2] = v.z;
                w[4 * q + 3] = v.w;
            }
        }
    }
    __device__ __forceinline__ unsigned get(int k) const
    {
        return (k & 1) ? (w[k >> 1] >> 16) : (w[k >> 1] & 0xFFFFu);
    }
};

// Lorenzo prediction over the available neighbours in 32-bit arithmetic
// (wrapping sums are exact where the result fits, which it does for a valid
// stream's grid values)
template <int D>
__device__ __forceinline__ int lorenzo32(const int (&nv)[8], int amask)
{
    unsigned s = 0;
#pragma unroll
    for (int o = 1; o < (1 << D); ++o)
        if ((o & ~amask) == 0)
            s += lorenzo_sign(o) > 0 ? (unsigned)nv[o] : 0u - (unsigned)nv[o];
    return (int)s;
}

__device__ __forceinline__ int net_pred32(float y, int n1)
{
    if (y > 0x1p30f)
        y = 0x1p30f;
    if (!(y >= -0x1p30f))
        y = -0x1p30f;
    return n1 + (int)__builtin_rintf(y);
}

template <typename T, int B>
__device__ __forceinline__ void store_row(T *dst, const T (&v)[B], bool vec)
{
    if constexpr (sizeof(T) == 4) {
        if (vec) {
#pragma unroll
            for (int q = 0; q < B / 4; ++q)
                reinterpret_cast<float4 *>(dst)[q] =
                    make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
            return;
        }
    } else {
        if (vec) {
#pragma unroll
            for (int q = 0; q < B / 2; ++q)
                reinterpret_cast<double2 *>(dst)[q] = make_double2(v[2 * q], v[2 * q + 1]);
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < B; ++k)
        dst[k] = v[k];
}

}  // namespace

constexpr int kLaneWaves = 2;  // waves per workgroup

template <typename T, int D, int B, int HP, int PREC>
__global__ void __launch_bounds__(64 * kLaneWaves) k_decode_lanes(DecodeArgs a)
{
    constexpr int NO = (1 << D) - 1;
    constexpr int K = (1 << D) - 2;
    constexpr int RW = D == 3 ? B : 1;  // ring rows: the previous plane
    __shared__ int ring[kLaneWaves][RW][B][64];
    __shared__ float4 wl[PREC == 0 ? kWlds : 1];
    if constexpr (PREC == 0)
        stage_weights<HP>(wl, a.mlp);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long long nf1 = a.nf[1], nf2 = a.nf[2];
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool have = f < a.nf[0] * nf1 * nf2;
    const long long fz = have ? f / (nf1 * nf2) : 0, fy = have ? (f / nf2) % nf1 : 0,
                    fx = have ? f % nf2 : 0;
    const long long b = (fz * a.nb[1] + fy) * a.nb[2] + fx;
    const BlockGeo q = block_geo3(fz, fy, fx, a.n, a.bd[0], a.bd[1], a.bd[2]);
    int err = kOk;
    unsigned nzero = have ? a.counts[b] : 0u;
    const unsigned long long roff = have ? a.offs[b] + a.partials[b / kScanChunk] : 0ull;
    if (have && (nzero > (unsigned)(q.ez * q.ey * q.ex) || roff + nzero > a.n_raw)) {
        err = kECorrupt;
        nzero = 0;
    }
    const bool netb = have && a.use_net && (!a.judge || a.bflags[b]);
    NetBf16 n16;
    if constexpr (PREC == 1)
        n16 = make_net_bf16(a.mlp, K);
    WeightsLds wt;
    wt.wl = wl;
    const float b2 = a.mlp.b2, alpha = a.mlp.alpha;
    const T *raw = reinterpret_cast<const T *>(a.raw);
    T *xh = reinterpret_cast<T *>(a.xh);
    const long long n1 = a.n[1], n2 = a.n[2];
    const bool vec = (n2 % (16 / (int)sizeof(T))) == 0 &&
                     (reinterpret_cast<uintptr_t>(a.xh) & 15) == 0;
    const DevConsts c = a.c;
    unsigned zc = 0;
    int prev[B];  // the previous row of this plane
    int zrp[B];   // the previous plane's row y - 1 (read for the row before)
#pragma unroll
    for (int k = 0; k < B; ++k)
        prev[k] = zrp[k] = 0;
    const int nz = D == 3 ? B : 1;
    // a row's codes are loaded one row ahead, before the previous row's
    // stores: one counter tracks a wave's loads and stores in issue order, so
    // a load issued after them would make each row wait for both
    auto row_codes = [&](RowCodes<B> &rc, int r) {
        if (have && r < nz * B)
            rc.load(a.codes + q.start + (long long)r * B);
        else
#pragma unroll
            for (int k = 0; k < B / 2; ++k)
                rc.w[k] = (uint32_t)kR | ((uint32_t)kR << 16);
    };
    RowCodes<B> rc;
    row_codes(rc, 0);
    for (int lz = 0; lz < nz; ++lz) {
        for (int ly = 0; ly < B; ++ly) {
            const int r = lz * B + ly;
            RowCodes<B> rn;
            row_codes(rn, r + 1);
            // the previous plane's rows y (ring slot of row r - B, which row r
            // then takes) and y - 1 (read for the row before)
            int zr[B], zry[B];
            if (D == 3 && lz > 0) {
                const int s0 = r % RW;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    zr[k] = ring[wv][s0][k][lane];
                    zry[k] = ly > 0 ? zrp[k] : 0;
                    zrp[k] = zr[k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < B; ++k)
                    zr[k] = zry[k] = 0;
            }
            const int amask_zy = (ly > 0 ? 2 : 0) | (D == 3 && lz > 0 ? 4 : 0);
            int cur[B];
            T xv[B];
#pragma unroll
            for (int lx = 0; lx < B; ++lx) {
                const int amask = amask_zy | (lx > 0 ? 1 : 0);
                int nv[8];
                nv[0] = 0;
                nv[1] = lx > 0 ? cur[lx > 0 ? lx - 1 : 0] : 0;
                nv[2] = prev[lx];
                nv[3] = lx > 0 ? prev[lx > 0 ? lx - 1 : 0] : 0;
                nv[4] = zr[lx];
                nv[5] = lx > 0 ? zr[lx > 0 ? lx - 1 : 0] : 0;
                nv[6] = zry[lx];
                nv[7] = lx > 0 ? zry[lx > 0 ? lx - 1 : 0] : 0;
                int pred;
                if (amask == NO) {  // wave-uniform
                    if constexpr (PREC == 1) {
                        // every lane runs the matrix cores (Lorenzo lanes feed zeros)
                        float u[6];
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            u[k] = (k < K && netb) ? (float)(nv[k + 2] - nv[1]) : 0.0f;
                        const float y = net_bf16(n16, u);
                        pred = netb ? net_pred32(y, nv[1]) : lorenzo32<D>(nv, amask);
                    } else {
                        pred = netb ? net_pred32(net_f32<D, HP>(nv, wt, b2, alpha), nv[1])
                                    : lorenzo32<D>(nv, amask);
                    }
                } else {
                    pred = lorenzo32<D>(nv, amask);
                }
                const unsigned code = rc.get(lx);
                int p;
                T x;
                if (code != 0u) {
                    p = pred - ((int)code - kR);
                    if (p < c.p_zero || p > c.p_max) {
                        err = kECorrupt;
                        p = (int)c.p_zero;
                    }
                    x = inverse_of<T>(p, a);
                } else {
                    // balance point: its raw value and that value's grid value,
                    // waited for here (s_waitcnt vmcnt(0)), in this rare branch:
                    // otherwise the common path, where p merges with this load,
                    // would wait at every point for every earlier load and store
                    if (zc < nzero) {
                        p = a.praw[roff + zc];
                        x = raw[roff + zc];
                        __builtin_amdgcn_s_waitcnt(0x0F70);
                    } else {
                        err = kECorrupt;
                        p = 0;
                        x = (T)0;
                    }
                    ++zc;
                }
                cur[lx] = p;
                xv[lx] = x;
            }
            if (have)
                store_row<T, B>(xh + ((q.bz * B + lz) * n1 + q.by * B + ly) * n2 + q.bx * B, xv,
                                vec);
            if constexpr (D == 3) {
                const int sw = r % RW;
#pragma unroll
                for (int k = 0; k < B; ++k)
                    ring[wv][sw][k][lane] = cur[k];
            }
#pragma unroll
            for (int k = 0; k < B; ++k)
                prev[k] = cur[k];
            rc = rn;
        }
        if constexpr (D == 3) {
#pragma unroll
            for (int k = 0; k < B; ++k)
                prev[k] = 0;
        }
    }
    if (have && zc != nzero)
        err = kECorrupt;
    set_status(a.status, err);
}

template <typename T, int D, int B, int HP, int PREC>
static void lanes_go(const DecodeArgs &a, hipStream_t s)
{
    const long long nfull = a.nf[0] * a.nf[1] * a.nf[2];
    const unsigned grid = (unsigned)((nfull + 64 * kLaneWaves - 1) / (64 * kLaneWaves));
    hipLaunchKernelGGL((k_decode_lanes<T, D, B, HP, PREC>), dim3(grid), dim3(64 * kLaneWaves), 0,
                       s, a);
}

template <typename T, int D, int B>
static void lanes_by_hidden(int HP, const DecodeArgs &a, hipStream_t s)
{
    if (HP == 0)
        lanes_go<T, D, B, 8, 1>(a, s);
    else if (HP == 8)
        lanes_go<T, D, B, 8, 0>(a, s);
    else if (HP == 16)
        lanes_go<T, D, B, 16, 0>(a, s);
    else
        lanes_go<T, D, B, 32, 0>(a, s);
}

bool lanes_shape(int D, int B) { return (D == 3 && (B == 4 || B == 8)) || (D == 2 && B == 16); }

void launch_decode_lanes(const Geom &g, int HP, const DecodeArgs &a, hipStream_t s)
{
    if (a.nf[0] * a.nf[1] * a.nf[2] == 0)
        return;
    if (g.dtype == PWREL_F32) {
        if (g.D == 3 && g.B == 8)
            lanes_by_hidden<float, 3, 8>(HP, a, s);
        else if (g.D == 3 && g.B == 4)
            lanes_by_hidden<float, 3, 4>(HP, a, s);
        else
            lanes_by_hidden<float, 2, 16>(HP, a, s);
    } else {
        if (g.D == 3 && g.B == 8)
            lanes_by_hidden<double, 3, 8>(HP, a, s);
        else if (g.D == 3 && g.B == 4)
            lanes_by_hidden<double, 3, 4>(HP, a, s);
        else
            lanes_by_hidden<double, 2, 16>(HP, a, s);
    }
}

}  // namespace pwrel
