// Fused compression kernel (steps: transform, prediction, quantisation,
// verification, per-block balance-point counts) for gfx950.
//
// A workgroup stages the grid values of a tile of whole blocks plus the
// one-point halo on the low side of every active axis in LDS: first the tile
// points (coalesced row loads of x, FP64 transform, FP64 verification of the
// reconstruction), then the halo points (transform only).  It then walks the
// tile in stream order (block-major, so a wave writes 64 consecutive codes),
// predicting every point independently from its neighbours' grid values (the
// data selection rule that removes the serial dependency), and counts the
// balance points of each block in LDS.  Workgroups are persistent; the
// workgroups of XCD x (= workgroup id mod 8) walk a contiguous eighth of the
// tiles so that tiles sharing halo rows meet in the same L2.
#include "pwrel_kernels.h"

namespace pwrel {

struct CompressArgs {
    const void *x;
    const int *pfield;
    long long n[3];
    int bd[3];
    long long nb[3];
    int t[3];
    long long nt[3];
    long long ntiles;
    int use_net, judge, independent;
    uint16_t *codes;
    uint32_t *counts;
    uint8_t *bflags;
    const DevConsts *consts;
    int *status;
    MlpW mlp;
};

template <typename T, int D, int BB, int HP, bool FROM_P>
__global__ void __launch_bounds__(256) k_compress(CompressArgs a)
{
    using S = ShapeOf<D, BB>;
    constexpr bool CT = S::known;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NT = 256;
    const int tid = threadIdx.x;
    constexpr int h0 = D >= 3 ? 1 : 0, h1 = D >= 2 ? 1 : 0, h2 = 1;
    const int B = CT ? BB : a.bd[2];
    const int bd0 = D >= 3 ? B : 1, bd1 = D >= 2 ? B : 1, bd2 = B;
    const int T0 = CT ? S::T0 : a.t[0], T1 = CT ? S::T1 : a.t[1], T2 = CT ? S::T2 : a.t[2];
    const int E0 = T0 + h0, E1 = T1 + h1, E2 = T2 + h2;
    const int ne = E0 * E1 * E2;
    const int ntp = T0 * T1 * T2;
    const int nbt0 = T0 / bd0, nbt1 = T1 / bd1, nbt2 = T2 / bd2;
    const int nbt = nbt0 * nbt1 * nbt2;
    const int BV = bd0 * bd1 * bd2;

    int *ptile = reinterpret_cast<int *>(smem);
    unsigned int *cnt = reinterpret_cast<unsigned int *>(ptile + ne);
    unsigned char *okb = reinterpret_cast<unsigned char *>(cnt + nbt);

    __shared__ int s_status;
    __shared__ float4 wl[kWlds];
    stage_weights<HP>(wl, a.mlp);
    const float b2 = a.mlp.b2, alpha = a.mlp.alpha;
    for (int i = tid; i < nbt; i += NT)
        cnt[i] = 0u;
    if (tid == 0)
        s_status = *a.status;
    __syncthreads();
    if (s_status != kOk)  // uniform: every thread reads the same shared value
        return;
    const DevConsts c = *a.consts;
    const T *x = reinterpret_cast<const T *>(a.x);
    const long long n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];

    // LDS offsets of the neighbours, o = 1 .. 2^D-1
    int noff[8];
#pragma unroll
    for (int o = 0; o < 8; ++o)
        noff[o] = (o & 1) + ((o >> 1) & 1) * E2 + ((o >> 2) & 1) * E1 * E2;

    int err = kOk;
    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, nslot = (G + 7 - xcd) >> 3;
    const long long chunk = (a.ntiles + 7) / 8;
    const long long tend = std::min(a.ntiles, (long long)(xcd + 1) * chunk);

    for (long long t = (long long)xcd * chunk + slot; t < tend; t += nslot) {
        const long long tz = t / (a.nt[1] * a.nt[2]);
        const long long ty = (t / a.nt[2]) % a.nt[1];
        const long long tx = t % a.nt[2];
        const long long g0z = tz * T0, g0y = ty * T1, g0x = tx * T2;

        // --- tile points: grid value and verification ----------------------
        for (int q = tid; q < ntp; q += NT) {
            const int c2 = q % T2, c1 = (q / T2) % T1, c0 = q / (T1 * T2);
            const long long gz = g0z + c0, gy = g0y + c1, gx = g0x + c2;
            int p = 0;
            unsigned char ok = 0;
            if (gz < n0 && gy < n1 && gx < n2) {
                const long long li = (gz * n1 + gy) * n2 + gx;
                if (FROM_P) {
                    p = a.pfield[li];
                    ok = 1;
                } else {
                    const double xv = (double)x[li];
                    p = grid_value(xv, c, err);
                    ok = within_bound(xv, grid_inverse<T>(p, c), c.eps) ? 1 : 0;
                }
            }
            ptile[((c0 + h0) * E1 + (c1 + h1)) * E2 + (c2 + h2)] = p;
            okb[q] = ok;
        }
        // --- halo points (low faces): grid value only --------------------------
        // enumeration: plane e0 = 0 (if the axis is active), then e1 = 0 rows,
        // then e2 = 0 columns
        const int nh0 = h0 ? E1 * E2 : 0;
        const int nh1 = h1 ? T0 * E2 : 0;
        const int nh2 = T0 * T1;
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
                e0 = h0 + r / T1;
                e1 = h1 + r % T1;
                e2 = 0;
            }
            const long long gz = g0z + e0 - h0, gy = g0y + e1 - h1, gx = g0x + e2 - h2;
            int p = 0;
            if (gz >= 0 && gy >= 0 && gx >= 0 && gz < n0 && gy < n1 && gx < n2) {
                const long long li = (gz * n1 + gy) * n2 + gx;
                p = FROM_P ? a.pfield[li] : grid_value((double)x[li], c, err);
            }
            ptile[(e0 * E1 + e1) * E2 + e2] = p;
        }
        __syncthreads();

        // --- predict, quantize, count (stream order) -------------------------
        const long long bz0 = g0z / bd0, by0 = g0y / bd1, bx0 = g0x / bd2;
        for (int q = tid; q < nbt * BV; q += NT) {
            const int bt = q / BV, li = q - bt * BV;
            const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
            const int lx = li % bd2, ly = (li / bd2) % bd1, lz = li / (bd1 * bd2);
            const int cz = btz * bd0 + lz, cy = bty * bd1 + ly, cx = btx * bd2 + lx;
            const long long gz = g0z + cz, gy = g0y + cy, gx = g0x + cx;
            if (gz >= n0 || gy >= n1 || gx >= n2)
                continue;
            const int ei = ((cz + h0) * E1 + (cy + h1)) * E2 + (cx + h2);
            int nv[8];
            nv[0] = ptile[ei];
#pragma unroll
            for (int o = 1; o < (1 << D); ++o)
                nv[o] = ptile[ei - noff[o]];
            int amask;
            if (a.independent)
                amask = (lx != 0 ? 1 : 0) | (D >= 2 && ly != 0 ? 2 : 0) |
                        (D >= 3 && lz != 0 ? 4 : 0);
            else
                amask = (gx != 0 ? 1 : 0) | (D >= 2 && gy != 0 ? 2 : 0) |
                        (D >= 3 && gz != 0 ? 4 : 0);
            const long long pred = predict<D, HP>(nv, amask, a.use_net != 0, WeightsLds{wl}, b2, alpha);
            const bool ok = okb[(cz * T1 + cy) * T2 + cx] != 0;
            const unsigned short code = make_code(pred, nv[0], ok);
            const BlockGeo bg = block_geo3(bz0 + btz, by0 + bty, bx0 + btx, a.n, bd0, bd1, bd2);
            a.codes[bg.start + ((long long)lz * bg.ey + ly) * bg.ex + lx] = code;
            if (code == 0)
                atomicAdd(&cnt[bt], 1u);
        }
        __syncthreads();

        // --- per-block balance-point counts ------------------------------------
        for (int bt = tid; bt < nbt; bt += NT) {
            const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
            const long long bz = bz0 + btz, by = by0 + bty, bx = bx0 + btx;
            if (bz < a.nb[0] && by < a.nb[1] && bx < a.nb[2]) {
                const long long b = (bz * a.nb[1] + by) * a.nb[2] + bx;
                a.counts[b] = cnt[bt];
                if (a.bflags)
                    a.bflags[b] = a.use_net ? 1 : 0;
            }
            cnt[bt] = 0u;
        }
        // the next tile's staging overwrites ptile/okb only after this barrier
        __syncthreads();
    }
    set_status(a.status, err);
}

// ---------------------------------------------------------------------------
static size_t compress_lds(const Geom &g, const int *t)
{
    const int h0 = g.D >= 3 ? 1 : 0, h1 = g.D >= 2 ? 1 : 0;
    const size_t ne = (size_t)(t[0] + h0) * (t[1] + h1) * (t[2] + 1);
    const size_t nbt = (size_t)(t[0] / g.bd[0]) * (t[1] / g.bd[1]) * (t[2] / g.bd[2]);
    const size_t ntp = (size_t)t[0] * t[1] * t[2];
    return ne * 4 + nbt * 4 + ntp;
}

bool tile_for(const Geom &g, Tile &tile)
{
    const int B = g.B;
    if (!known_shape(g.D, B, tile.t)) {
        auto mult = [](int b, int target) { return b * std::max(1, (target + b - 1) / b); };
        if (g.D == 3) {
            tile.t[0] = mult(B, 8);
            tile.t[1] = mult(B, 8);
            tile.t[2] = mult(B, 64);
        } else if (g.D == 2) {
            tile.t[0] = 1;
            tile.t[1] = mult(B, 16);
            tile.t[2] = mult(B, 128);
        } else {
            tile.t[0] = 1;
            tile.t[1] = 1;
            tile.t[2] = mult(B, 4096);
        }
        // shrink the fastest axis (then the others) until the LDS budget fits
        const size_t budget = 48 * 1024;
        while (compress_lds(g, tile.t) > budget && tile.t[2] > g.bd[2])
            tile.t[2] -= g.bd[2];
        while (compress_lds(g, tile.t) > budget && tile.t[1] > g.bd[1])
            tile.t[1] -= g.bd[1];
        while (compress_lds(g, tile.t) > budget && tile.t[0] > g.bd[0])
            tile.t[0] -= g.bd[0];
        if (compress_lds(g, tile.t) > budget)
            return false;
    }
    tile.ntiles = 1;
    for (int d = 0; d < 3; ++d) {
        tile.nt[d] = (g.n[d] + tile.t[d] - 1) / tile.t[d];
        tile.ntiles *= tile.nt[d];
    }
    return true;
}

template <typename T, int D, int BB, int HP, bool FP>
static void go(const CompressArgs &a, unsigned grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_compress<T, D, BB, HP, FP>), dim3(grid), dim3(256), lds, s, a);
}

template <typename T, int D, int BB, bool FP>
static void by_hidden(int HP, const CompressArgs &a, unsigned grid, size_t lds, hipStream_t s)
{
    if (HP == 8)
        go<T, D, BB, 8, FP>(a, grid, lds, s);
    else if (HP == 16)
        go<T, D, BB, 16, FP>(a, grid, lds, s);
    else
        go<T, D, BB, 32, FP>(a, grid, lds, s);
}

template <typename T, bool FP>
static void by_shape(int D, int B, int HP, const CompressArgs &a, unsigned grid, size_t lds,
                     hipStream_t s)
{
    if (D == 3 && B == 8)
        by_hidden<T, 3, 8, FP>(HP, a, grid, lds, s);
    else if (D == 3 && B == 4)
        by_hidden<T, 3, 4, FP>(HP, a, grid, lds, s);
    else if (D == 3 && B == 16)
        by_hidden<T, 3, 16, FP>(HP, a, grid, lds, s);
    else if (D == 2 && B == 16)
        by_hidden<T, 2, 16, FP>(HP, a, grid, lds, s);
    else if (D == 2 && B == 32)
        by_hidden<T, 2, 32, FP>(HP, a, grid, lds, s);
    else if (D == 2 && B == 64)
        by_hidden<T, 2, 64, FP>(HP, a, grid, lds, s);
    else if (D == 1 && B == 256)
        by_hidden<T, 1, 256, FP>(HP, a, grid, lds, s);
    else if (D == 3)
        by_hidden<T, 3, 0, FP>(HP, a, grid, lds, s);
    else if (D == 2)
        by_hidden<T, 2, 0, FP>(HP, a, grid, lds, s);
    else
        by_hidden<T, 1, 0, FP>(HP, a, grid, lds, s);
}

hipError_t launch_compress(const void *x, const int *pfield, const Geom &g, const Tile &tile,
                           const pwrel_mlp *model, const pwrel_options &opt, Workspace &ws,
                           uint16_t *codes, uint32_t *counts, uint8_t *bflags, int num_cus,
                           hipStream_t s)
{
    CompressArgs a{};
    a.x = x;
    a.pfield = pfield;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bd[d] = g.bd[d];
        a.nb[d] = g.nb[d];
        a.t[d] = tile.t[d];
        a.nt[d] = tile.nt[d];
    }
    a.ntiles = tile.ntiles;
    a.use_net = opt.use_net;
    a.judge = opt.judge;
    a.independent = opt.independent_blocks;
    a.codes = codes;
    a.counts = counts;
    a.bflags = bflags;
    a.consts = ws.consts;
    a.status = ws.status;
    a.mlp = pack_mlp(opt.use_net ? model : nullptr);
    const int HP = hidden_pad(opt.use_net ? model : nullptr);
    const long long gmax = (long long)std::max(num_cus, 8) * 4;
    long long grid = std::min(gmax, (tile.ntiles + 7) / 8 * 8);
    if (grid < 8)
        grid = 8;
    const size_t lds = compress_lds(g, tile.t);
    if (pfield)
        by_shape<float, true>(g.D, g.B, HP, a, (unsigned)grid, lds, s);
    else if (g.dtype == PWREL_F32)
        by_shape<float, false>(g.D, g.B, HP, a, (unsigned)grid, lds, s);
    else
        by_shape<double, false>(g.D, g.B, HP, a, (unsigned)grid, lds, s);
    return hipGetLastError();
}

}  // namespace pwrel
