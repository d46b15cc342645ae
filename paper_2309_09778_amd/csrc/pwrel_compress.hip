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
#include "pwrel_bf16.h"

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
    const long long *qtab;  // q(c) = rint(2^32 log2 c), c = 0 .. points per block (judge)
    MlpW mlp;
};

// Judge bins: code 0 (balance point) and the prediction error clamped to
// [-127, 127] (Sec. 4.3 judge reading: entropy of the clamped code).
__device__ __forceinline__ int judge_bin(unsigned code)
{
    if (code == 0)
        return 0;
    int e = (int)code - kR;
    e = e < -127 ? -127 : (e > 127 ? 127 : e);
    return e + 128;
}

template <int D>
__device__ __forceinline__ long long lorenzo_pred(const int (&nv)[8], int amask)
{
    long long s = 0;
#pragma unroll
    for (int o = 1; o < (1 << D); ++o)
        if ((o & ~amask) == 0)
            s += (long long)lorenzo_sign(o) * (long long)nv[o];
    return s;
}

template <typename T, int D, int BB, int HP, bool FROM_P, int PREC>
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

    // judge only (first, so that the 64-bit scores are 8-byte aligned):
    // per-block scores and code histograms (network count in the low 16 bits,
    // Lorenzo count in the high 16 bits; bin 0 = balance points)
    unsigned long long *jsum = reinterpret_cast<unsigned long long *>(smem);
    int *ptile = reinterpret_cast<int *>(jsum + (a.judge ? 2 * nbt : 0));
    unsigned int *cnt = reinterpret_cast<unsigned int *>(ptile + ne);
    unsigned int *jh = cnt + nbt;
    unsigned char *okb = reinterpret_cast<unsigned char *>(jh + (a.judge ? nbt * 256 : 0));

    __shared__ int s_status;
    __shared__ float4 wl[kWlds];
    stage_weights<HP>(wl, a.mlp);
    const float b2 = a.mlp.b2, alpha = a.mlp.alpha;
    NetBf16 net16;
    if constexpr (PREC == 1)
        net16 = make_net_bf16(a.mlp, (1 << D) - 2);
    for (int i = tid; i < nbt; i += NT)
        cnt[i] = 0u;
    if (a.judge) {
        for (int i = tid; i < nbt * 256; i += NT)
            jh[i] = 0u;
        for (int i = tid; i < 2 * nbt; i += NT)
            jsum[i] = 0ULL;
    }
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
        // Rounds of NT points; every lane of a wave takes part in each round
        // (the matrix-core network works on whole waves).
        const long long bz0 = g0z / bd0, by0 = g0y / bd1, bx0 = g0x / bd2;
        const int nq = nbt * BV;
        for (int q0 = 0; q0 < nq; q0 += NT) {
            const int q = q0 + tid;
            const int qq = q < nq ? q : 0;
            const int bt = qq / BV, li = qq - bt * BV;
            const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
            const int lx = li % bd2, ly = (li / bd2) % bd1, lz = li / (bd1 * bd2);
            const int cz = btz * bd0 + lz, cy = bty * bd1 + ly, cx = btx * bd2 + lx;
            const long long gz = g0z + cz, gy = g0y + cy, gx = g0x + cx;
            const bool inside = q < nq && gz < n0 && gy < n1 && gx < n2;
            int nv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int amask = 0;
            if (inside) {
                const int ei = ((cz + h0) * E1 + (cy + h1)) * E2 + (cx + h2);
                nv[0] = ptile[ei];
#pragma unroll
                for (int o = 1; o < (1 << D); ++o)
                    nv[o] = ptile[ei - noff[o]];
                if (a.independent)
                    amask = (lx != 0 ? 1 : 0) | (D >= 2 && ly != 0 ? 2 : 0) |
                            (D >= 3 && lz != 0 ? 4 : 0);
                else
                    amask = (gx != 0 ? 1 : 0) | (D >= 2 && gy != 0 ? 2 : 0) |
                            (D >= 3 && gz != 0 ? 4 : 0);
            }
            long long pred;
            if constexpr (PREC == 1)
                pred = predict_bf16<D>(nv, amask, a.use_net != 0 && inside, net16);
            else
                pred = inside ? predict<D, HP>(nv, amask, a.use_net != 0, WeightsLds{wl}, b2, alpha)
                              : 0;
            if (!inside)
                continue;
            const bool ok = okb[(cz * T1 + cy) * T2 + cx] != 0;
            const unsigned short code = make_code(pred, nv[0], ok);
            const BlockGeo bg = block_geo3(bz0 + btz, by0 + bty, bx0 + btx, a.n, bd0, bd1, bd2);
            a.codes[bg.start + ((long long)lz * bg.ey + ly) * bg.ex + lx] = code;
            if (a.judge) {
                const unsigned short lcode = make_code(lorenzo_pred<D>(nv, amask), nv[0], ok);
                atomicAdd(&jh[bt * 256 + judge_bin(code)], 1u);
                atomicAdd(&jh[bt * 256 + judge_bin(lcode)], 1u << 16);
            } else if (code == 0) {
                atomicAdd(&cnt[bt], 1u);
            }
        }
        __syncthreads();

        if (a.judge) {
            // --- per-block judge: keep the network iff the entropy of its
            //     clamped codes is strictly below Lorenzo's (fixed-point scores) ---
            for (int i = tid; i < nbt * 256; i += NT) {
                const unsigned w = jh[i];
                const unsigned c_n = w & 0xffffu, c_l = w >> 16;
                const int bt = i >> 8;
                if ((i & 255) == 0)  // bin 0 holds the balance points of both
                    cnt[bt] = w;
                if (c_n)
                    atomicAdd(&jsum[2 * bt],
                              (unsigned long long)c_n * (unsigned long long)a.qtab[c_n]);
                if (c_l)
                    atomicAdd(&jsum[2 * bt + 1],
                              (unsigned long long)c_l * (unsigned long long)a.qtab[c_l]);
                jh[i] = 0u;
            }
            __syncthreads();
            // blocks where Lorenzo wins: overwrite the network codes written above
            for (int q = tid; q < nq; q += NT) {
                const int bt = q / BV;
                if (jsum[2 * bt] > jsum[2 * bt + 1])
                    continue;
                const int li = q - bt * BV;
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
                const bool ok = okb[(cz * T1 + cy) * T2 + cx] != 0;
                const BlockGeo bg =
                    block_geo3(bz0 + btz, by0 + bty, bx0 + btx, a.n, bd0, bd1, bd2);
                a.codes[bg.start + ((long long)lz * bg.ey + ly) * bg.ex + lx] =
                    make_code(lorenzo_pred<D>(nv, amask), nv[0], ok);
            }
            for (int bt = tid; bt < nbt; bt += NT) {
                const bool use_n = jsum[2 * bt] > jsum[2 * bt + 1];
                cnt[bt] = use_n ? (cnt[bt] & 0xffffu) : (cnt[bt] >> 16);
            }
            __syncthreads();
        }

        // --- per-block balance-point counts ------------------------------------
        for (int bt = tid; bt < nbt; bt += NT) {
            const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
            const long long bz = bz0 + btz, by = by0 + bty, bx = bx0 + btx;
            if (bz < a.nb[0] && by < a.nb[1] && bx < a.nb[2]) {
                const long long b = (bz * a.nb[1] + by) * a.nb[2] + bx;
                a.counts[b] = cnt[bt];
                if (a.bflags)
                    a.bflags[b] = a.judge ? (jsum[2 * bt] > jsum[2 * bt + 1] ? 1 : 0)
                                          : (a.use_net ? 1 : 0);
            }
            cnt[bt] = 0u;
            if (a.judge)
                jsum[2 * bt] = jsum[2 * bt + 1] = 0ULL;
        }
        // the next tile's staging overwrites ptile/okb only after this barrier
        __syncthreads();
    }
    set_status(a.status, err);
}

// ---------------------------------------------------------------------------
static size_t compress_lds(const Geom &g, const int *t, bool judge = true)
{
    const int h0 = g.D >= 3 ? 1 : 0, h1 = g.D >= 2 ? 1 : 0;
    const size_t ne = (size_t)(t[0] + h0) * (t[1] + h1) * (t[2] + 1);
    const size_t nbt = (size_t)(t[0] / g.bd[0]) * (t[1] / g.bd[1]) * (t[2] / g.bd[2]);
    const size_t ntp = (size_t)t[0] * t[1] * t[2];
    size_t n = ne * 4 + nbt * 4;
    if (judge)
        n += nbt * 256 * 4 + 2 * nbt * 8;
    return n + ntp;
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

template <typename T, int D, int BB, int HP, bool FP, int PREC>
static void go(const CompressArgs &a, unsigned grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_compress<T, D, BB, HP, FP, PREC>), dim3(grid), dim3(256), lds, s, a);
}

template <typename T, int D, int BB, bool FP>
static void by_hidden(int HP, const CompressArgs &a, unsigned grid, size_t lds, hipStream_t s)
{
    if (HP == 0)
        go<T, D, BB, 8, FP, 1>(a, grid, lds, s);  // matrix-core network
    else if (HP == 8)
        go<T, D, BB, 8, FP, 0>(a, grid, lds, s);
    else if (HP == 16)
        go<T, D, BB, 16, FP, 0>(a, grid, lds, s);
    else
        go<T, D, BB, 32, FP, 0>(a, grid, lds, s);
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
    a.qtab = ws.qtab;
    a.mlp = pack_mlp(opt.use_net ? model : nullptr);
    const bool mfma = opt.use_net && model && model->precision == 1;
    const int HP = mfma ? 0 : hidden_pad(opt.use_net ? model : nullptr);
    const long long gmax = (long long)std::max(num_cus, 8) * 4;
    long long grid = std::min(gmax, (tile.ntiles + 7) / 8 * 8);
    if (grid < 8)
        grid = 8;
    const size_t lds = compress_lds(g, tile.t, opt.judge != 0);
    if (pfield)
        by_shape<float, true>(g.D, g.B, HP, a, (unsigned)grid, lds, s);
    else if (g.dtype == PWREL_F32)
        by_shape<float, false>(g.D, g.B, HP, a, (unsigned)grid, lds, s);
    else
        by_shape<double, false>(g.D, g.B, HP, a, (unsigned)grid, lds, s);
    return hipGetLastError();
}

}  // namespace pwrel
