// Decompression kernel: one block per workgroup (gfx950).
//
// Halo grid values come from the int32 scratch field written by earlier block
// levels; the block's grid values are rebuilt hyperplane by hyperplane
// (lz + ly + lx = s): every line (lz, ly) of the block is owned by one lane,
// which decodes its point lx = s - lz - ly with the same predictor as the
// encoder.  Then x^ = inverse(grid value) for coded points and the raw value
// for balance points.  Only the block's high faces go back to the scratch
// field (later blocks read nothing else).
#include <type_traits>

#include "pwrel_bf16.h"

namespace pwrel {

struct DecodeArgs {
    long long n[3];
    int bd[3];
    long long nb[3];
    int use_net, judge, independent;
    int level;
    long long bz_lo;
    const uint8_t *bflags;
    const uint16_t *codes;
    const unsigned long long *offs;
    const unsigned long long *partials;
    const void *raw;
    unsigned long long n_raw;
    void *xh;
    int *pgrid;
    int *status;
    DevConsts c;
    MlpW mlp;
};

__device__ __forceinline__ unsigned long long raw_offset(const unsigned long long *offs,
                                                         const unsigned long long *partials,
                                                         long long b)
{
    return offs[b] + partials[b / kScanChunk];
}

template <typename T, int D, int BB, int HP, int PREC>
__global__ void __launch_bounds__(256) k_decode(DecodeArgs a)
{
    constexpr bool CT = BB > 0;
    extern __shared__ __align__(16) unsigned char smem[];
    const int NT = blockDim.x, tid = threadIdx.x;
    constexpr int h0 = D >= 3 ? 1 : 0, h1 = D >= 2 ? 1 : 0;
    const int B = CT ? BB : a.bd[2];
    const int bd0 = D >= 3 ? B : 1, bd1 = D >= 2 ? B : 1, bd2 = B;
    const int E0 = bd0 + h0, E1 = bd1 + h1, E2 = bd2 + 1;
    const int ne = E0 * E1 * E2;
    const int BV = bd0 * bd1 * bd2;
    int *ptile = reinterpret_cast<int *>(smem);
    unsigned short *cl = reinterpret_cast<unsigned short *>(ptile + ne);
    unsigned short *rk = cl + BV;
    __shared__ float4 wl[kWlds];

    long long bz, by, bx;
    if (a.independent) {
        const long long b = blockIdx.x;
        bx = b % a.nb[2];
        by = (b / a.nb[2]) % a.nb[1];
        bz = b / (a.nb[1] * a.nb[2]);
    } else {
        bz = a.bz_lo + blockIdx.x / a.nb[1];
        by = blockIdx.x % a.nb[1];
        bx = (long long)a.level - bz - by;
        if (bz >= a.nb[0] || bx < 0 || bx >= a.nb[2])
            return;  // uniform across the workgroup
    }
    const long long b = (bz * a.nb[1] + by) * a.nb[2] + bx;
    const long long n1 = a.n[1], n2 = a.n[2];
    const BlockGeo q = block_geo3(bz, by, bx, a.n, bd0, bd1, bd2);
    const int ez = q.ez, ey = q.ey, ex = q.ex;
    const int bsize = ez * ey * ex;
    const bool full = ez == bd0 && ey == bd1 && ex == bd2;
    const long long g0z = bz * bd0, g0y = by * bd1, g0x = bx * bd2;
    const T *raw = reinterpret_cast<const T *>(a.raw);
    T *xh = reinterpret_cast<T *>(a.xh);

    stage_weights<HP>(wl, a.mlp);
    const float b2 = a.mlp.b2, alpha = a.mlp.alpha;
    // codes in full-block layout (lz * bd1 + ly) * bd2 + lx
    for (int li = tid; li < bsize; li += NT) {
        int ci = li;
        if (!full) {
            const int lx = li % ex, ly = (li / ex) % ey, lz = li / (ex * ey);
            ci = (lz * bd1 + ly) * bd2 + lx;
        }
        cl[ci] = a.codes[q.start + li];
    }
    if (!a.independent) {
        // low-face halo: plane e0 = 0, rows e1 = 0, columns e2 = 0
        const int nh0 = h0 ? E1 * E2 : 0, nh1 = h1 ? bd0 * E2 : 0, nh2 = bd0 * bd1;
        for (int hq = tid; hq < nh0 + nh1 + nh2; hq += NT) {
            int e0, e1, e2;
            if (hq < nh0) {
                e0 = 0;
                e1 = hq / E2;
                e2 = hq - e1 * E2;
            } else if (hq < nh0 + nh1) {
                const int r = hq - nh0;
                e0 = h0 + r / E2;
                e1 = 0;
                e2 = r - (r / E2) * E2;
            } else {
                const int r = hq - nh0 - nh1;
                e0 = h0 + r / bd1;
                e1 = h1 + r % bd1;
                e2 = 0;
            }
            const long long gz = g0z + e0 - h0, gy = g0y + e1 - h1, gx = g0x + e2 - 1;
            if (gz >= 0 && gy >= 0 && gx >= 0 && gz < a.n[0] && gy < n1 && gx < n2)
                ptile[(e0 * E1 + e1) * E2 + e2] = a.pgrid[(gz * n1 + gy) * n2 + gx];
        }
    }
    __syncthreads();
    // in-block rank of every balance point, in stream (local raster) order
    if (tid < 64) {
        unsigned run = 0;
        const unsigned long long below = (1ULL << tid) - 1ULL;
        for (int c0 = 0; c0 < bsize; c0 += 64) {
            const int li = c0 + tid;
            int ci = li;
            if (!full && li < bsize) {
                const int lx = li % ex, ly = (li / ex) % ey, lz = li / (ex * ey);
                ci = (lz * bd1 + ly) * bd2 + lx;
            }
            const bool z = li < bsize && cl[ci] == 0;
            const unsigned long long mask = __ballot(z);
            if (z)
                rk[ci] = (unsigned short)(run + (unsigned)__popcll(mask & below));
            run += (unsigned)__popcll(mask);
        }
    }
    const unsigned long long roff = raw_offset(a.offs, a.partials, b);
    const bool net = a.use_net && (!a.judge || a.bflags[b]);
    int noff[8];
#pragma unroll
    for (int o = 0; o < 8; ++o)
        noff[o] = (o & 1) + ((o >> 1) & 1) * E2 + ((o >> 2) & 1) * E1 * E2;
    __syncthreads();

    // hyperplane sweep: lane `line` owns (lz, ly); its point at step s is lx = s - lz - ly.
    // Up to 16 hidden units the weights live in registers for the whole sweep.
    using Wt = typename std::conditional<(HP <= 16), WeightsReg<HP>, WeightsLds>::type;
    Wt wt;
    if constexpr (HP <= 16)
        wt.load(wl);
    else
        wt.wl = wl;
    NetBf16 net16;
    if constexpr (PREC == 1)
        net16 = make_net_bf16(a.mlp, (1 << D) - 2);
    int err = kOk;
    const int nlines = bd0 * bd1;
    const int nsteps = (ez - 1) + (ey - 1) + (ex - 1) + 1;
    for (int line0 = 0; line0 < nlines; line0 += NT) {
        const int line = line0 + tid;
        const int lz = line / bd1, ly = line % bd1;
        const bool lane_on = line < nlines && lz < ez && ly < ey;
        const int ebase = ((lz + h0) * E1 + (ly + h1)) * E2 + 1;
        const int cbase = line * bd2;
        const long long gz = g0z + lz, gy = g0y + ly;
        int amask_zy;
        if (a.independent)
            amask_zy = (D >= 2 && ly != 0 ? 2 : 0) | (D >= 3 && lz != 0 ? 4 : 0);
        else
            amask_zy = (D >= 2 && gy != 0 ? 2 : 0) | (D >= 3 && gz != 0 ? 4 : 0);
        for (int s = 0; s < nsteps; ++s) {
            const int lx = s - lz - ly;
            const bool on = lane_on && lx >= 0 && lx < ex;
            const int ei = ebase + lx;
            const unsigned code = on ? cl[cbase + lx] : 0u;
            int nv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int amask = 0;
            if (on && code != 0) {
#pragma unroll
                for (int o = 1; o < (1 << D); ++o)
                    nv[o] = ptile[ei - noff[o]];
                amask = amask_zy | (a.independent ? (lx != 0) : (g0x + lx != 0));
            }
            long long pred = 0;
            if constexpr (PREC == 1) {
                // block-uniform branch; inside it every lane of the wave runs
                // the matrix-core network (lanes without a coded point feed zeros)
                if (net)
                    pred = predict_bf16<D>(nv, amask, on && code != 0, net16);
                else if (on && code != 0)
                    pred = predict<D, HP>(nv, amask, false, wt, b2, alpha);
            } else {
                if (on && code != 0)
                    pred = predict<D, HP>(nv, amask, net, wt, b2, alpha);
            }
            if (on) {
                int p;
                if (code != 0) {
                    const long long pv = pred - ((long long)code - kR);
                    if (!(pv > -(long long)kGridLimit && pv < (long long)kGridLimit)) {
                        err = kECorrupt;
                        p = 0;
                    } else {
                        p = (int)pv;
                    }
                } else {
                    const unsigned long long ri = roff + rk[cbase + lx];
                    if (ri >= a.n_raw) {
                        err = kECorrupt;
                        p = 0;
                    } else {
                        p = grid_value((double)raw[ri], a.c, err);
                    }
                }
                ptile[ei] = p;
            }
            __syncthreads();
        }
    }

    // reconstruction and the faces later blocks read
    for (int ci = tid; ci < BV; ci += NT) {
        const int lx = ci % bd2, ly = (ci / bd2) % bd1, lz = ci / (bd1 * bd2);
        if (lz >= ez || ly >= ey || lx >= ex)
            continue;
        const int ei = ((lz + h0) * E1 + (ly + h1)) * E2 + lx + 1;
        const long long gi = ((g0z + lz) * n1 + g0y + ly) * n2 + g0x + lx;
        const int p = ptile[ei];
        double v;
        if (cl[ci] != 0) {
            v = grid_inverse<T>(p, a.c);
        } else {
            const unsigned long long ri = roff + rk[ci];
            v = ri < a.n_raw ? (double)raw[ri] : 0.0;
        }
        xh[gi] = (T)v;
        if (!a.independent && (lz == ez - 1 || ly == ey - 1 || lx == ex - 1))
            a.pgrid[gi] = p;
    }
    set_status(a.status, err);
}

// ---------------------------------------------------------------------------
template <typename T, int D, int BB, int HP, int PREC>
static void go(const DecodeArgs &a, unsigned grid, unsigned nt, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_decode<T, D, BB, HP, PREC>), dim3(grid), dim3(nt), lds, s, a);
}

template <typename T, int D, int BB>
static void by_hidden(int HP, const DecodeArgs &a, unsigned grid, unsigned nt, size_t lds,
                      hipStream_t s)
{
    if (HP == 0)
        go<T, D, BB, 8, 1>(a, grid, nt, lds, s);  // matrix-core network (Lorenzo blocks: HP 8)
    else if (HP == 8)
        go<T, D, BB, 8, 0>(a, grid, nt, lds, s);
    else if (HP == 16)
        go<T, D, BB, 16, 0>(a, grid, nt, lds, s);
    else
        go<T, D, BB, 32, 0>(a, grid, nt, lds, s);
}

template <typename T>
static void by_shape(int D, int B, int HP, const DecodeArgs &a, unsigned grid, unsigned nt,
                     size_t lds, hipStream_t s)
{
    if (D == 3 && B == 8)
        by_hidden<T, 3, 8>(HP, a, grid, nt, lds, s);
    else if (D == 3 && B == 4)
        by_hidden<T, 3, 4>(HP, a, grid, nt, lds, s);
    else if (D == 3 && B == 16)
        by_hidden<T, 3, 16>(HP, a, grid, nt, lds, s);
    else if (D == 2 && B == 16)
        by_hidden<T, 2, 16>(HP, a, grid, nt, lds, s);
    else if (D == 2 && B == 32)
        by_hidden<T, 2, 32>(HP, a, grid, nt, lds, s);
    else if (D == 2 && B == 64)
        by_hidden<T, 2, 64>(HP, a, grid, nt, lds, s);
    else if (D == 1 && B == 256)
        by_hidden<T, 1, 256>(HP, a, grid, nt, lds, s);
    else if (D == 3)
        by_hidden<T, 3, 0>(HP, a, grid, nt, lds, s);
    else if (D == 2)
        by_hidden<T, 2, 0>(HP, a, grid, nt, lds, s);
    else
        by_hidden<T, 1, 0>(HP, a, grid, nt, lds, s);
}

hipError_t launch_decode(const Geom &g, const DevConsts &c, const pwrel_mlp *model, int flags,
                         const uint8_t *bflags, const uint16_t *codes, const uint32_t *counts,
                         const void *raw, unsigned long long n_raw, Workspace &ws, void *xh,
                         hipStream_t s)
{
    (void)counts;
    DecodeArgs a{};
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bd[d] = g.bd[d];
        a.nb[d] = g.nb[d];
    }
    a.use_net = (flags & PWREL_HF_NET) ? 1 : 0;
    a.judge = (flags & PWREL_HF_JUDGE) ? 1 : 0;
    a.independent = (flags & PWREL_HF_INDEPENDENT) ? 1 : 0;
    a.bflags = bflags;
    a.codes = codes;
    a.offs = ws.offsets;
    a.partials = ws.partials;
    a.raw = raw;
    a.n_raw = n_raw;
    a.xh = xh;
    a.pgrid = ws.pgrid;
    a.status = ws.status;
    a.c = c;
    a.mlp = pack_mlp(a.use_net ? model : nullptr);
    const bool mfma = a.use_net && model && model->precision == 1;
    const int HP = mfma ? 0 : hidden_pad(a.use_net ? model : nullptr);
    const int h0 = g.D >= 3 ? 1 : 0, h1 = g.D >= 2 ? 1 : 0;
    const size_t ne = (size_t)(g.bd[0] + h0) * (g.bd[1] + h1) * (g.bd[2] + 1);
    const size_t bv = (size_t)g.bd[0] * g.bd[1] * g.bd[2];
    const size_t lds = ne * 4 + bv * 4;
    const long long nlines = (long long)g.bd[0] * g.bd[1];
    const unsigned nt = (unsigned)std::min(256LL, std::max(64LL, (nlines + 63) / 64 * 64));
    if (a.independent) {
        a.level = 0;
        a.bz_lo = 0;
        if (g.dtype == PWREL_F32)
            by_shape<float>(g.D, g.B, HP, a, (unsigned)g.nblocks, nt, lds, s);
        else
            by_shape<double>(g.D, g.B, HP, a, (unsigned)g.nblocks, nt, lds, s);
        return hipGetLastError();
    }
    const long long nlev = (g.nb[0] - 1) + (g.nb[1] - 1) + (g.nb[2] - 1) + 1;
    for (long long lev = 0; lev < nlev; ++lev) {
        const long long bz_lo = std::max(0LL, lev - (g.nb[1] - 1) - (g.nb[2] - 1));
        const long long bz_hi = std::min(g.nb[0] - 1, lev);
        a.level = (int)lev;
        a.bz_lo = bz_lo;
        const unsigned grid = (unsigned)((bz_hi - bz_lo + 1) * g.nb[1]);
        if (g.dtype == PWREL_F32)
            by_shape<float>(g.D, g.B, HP, a, grid, nt, lds, s);
        else
            by_shape<double>(g.D, g.B, HP, a, grid, nt, lds, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace pwrel
