// Decompression kernels (gfx950): one block at a time per workgroup.
//
// Per block.  Prologue (nothing here waits for another block): the block's
// codes (one 16-byte load per lane where the block is aligned) and its first
// 64 raw values (one per lane of wave 0).  Then the low-face halo grid values
// (written by earlier blocks), and wave 0 ranks the balance points, writes
// their raw values to x^ and their grid values into the tile, so that the
// sweep only handles coded points.  Sweep: hyperplane by hyperplane
// (lz + ly + lx = s), every line (lz, ly) of the block owned by one lane,
// which decodes its point lx = s - lz - ly with the same predictor as the
// encoder.  Then the block's high faces go to the scratch grid field (later
// blocks read nothing else) and x^ = inverse(grid value) for coded points.
//
// Independent blocks: one launch, one workgroup per block.  Halo mode: one
// persistent launch; workgroups take blocks from an atomic ticket counter in
// an order where every block comes after the blocks it reads (block levels
// bz + by + bx ascending), wait for those blocks' done flags, and raise their
// own flag once their faces are stored.  A block is only waited on after a
// running workgroup has taken it, so the lowest unfinished ticket can always
// proceed; the waits are bounded all the same.
#include <type_traits>

#include "pwrel_bf16.h"

namespace pwrel {

struct DecodeArgs {
    long long n[3];
    int bd[3];
    long long nb[3];
    long long nblocks;
    int use_net, judge, independent;
    const uint8_t *bflags;
    const uint16_t *codes;
    const uint32_t *counts;
    const unsigned long long *offs;
    const unsigned long long *partials;
    const void *raw;
    unsigned long long n_raw;
    void *xh;
    int *pgrid;
    int *status;
    // halo mode: block order, done flags, ticket counter, this call's flag value
    const unsigned *order;
    unsigned *done;
    unsigned *ticket;
    unsigned epoch;
    DevConsts c;
    MlpW mlp;
};

constexpr unsigned kSpinLimit = 1u << 20;  // polls of one flag before giving up

__device__ __forceinline__ unsigned long long raw_offset(const unsigned long long *offs,
                                                         const unsigned long long *partials,
                                                         long long b)
{
    return offs[b] + partials[b / kScanChunk];
}

// Cross-workgroup data of the halo-mode decoder (face grid values, done
// flags) is only ever stored and loaded as device-scope atomics: those
// accesses go to the device's point of coherence (past the per-XCD L2
// caches), so no cache-wide write-back or invalidation is needed.  The only
// ordering required is that a block's face stores are complete before its
// flag is stored: each wave waits for its outstanding memory operations.
__device__ __forceinline__ unsigned load_flag(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int load_face(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_face(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// s_waitcnt vmcnt(0): this wave's stores have been acknowledged
__device__ __forceinline__ void wait_stores()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt = 0, expcnt and lgkmcnt not waited on
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename T, int D, int BB, int HP, int PREC>
struct BlockDecoder {
    static constexpr bool CT = BB > 0;
    static constexpr int h0 = D >= 3 ? 1 : 0, h1 = D >= 2 ? 1 : 0;
    using Wt = typename std::conditional<(HP <= 16), WeightsReg<HP>, WeightsLds>::type;

    const DecodeArgs &a;
    int NT, tid;
    int B, bd0, bd1, bd2, E0, E1, E2, ne, BV;
    unsigned short *cl;  // codes, full-block layout (16-byte aligned)
    int *ptile;          // grid tile with the low-face halo
    Wt wt;
    NetBf16 net16;
    float b2, alpha;
    int noff[8];
    int err = kOk;

    // per block
    long long bz, by, bx, b, g0z, g0y, g0x;
    BlockGeo q;
    int bsize;
    bool full;
    unsigned long long roff;
    unsigned nzero;
    bool raw_ok;
    T rv;

    __device__ BlockDecoder(const DecodeArgs &args, unsigned char *smem, const float4 *wl)
        : a(args)
    {
        NT = blockDim.x;
        tid = threadIdx.x;
        B = CT ? BB : a.bd[2];
        bd0 = D >= 3 ? B : 1;
        bd1 = D >= 2 ? B : 1;
        bd2 = B;
        E0 = bd0 + h0;
        E1 = bd1 + h1;
        E2 = bd2 + 1;
        ne = E0 * E1 * E2;
        BV = bd0 * bd1 * bd2;
        cl = reinterpret_cast<unsigned short *>(smem);
        ptile = reinterpret_cast<int *>(smem + ((BV * 2 + 15) & ~15));
        if constexpr (HP <= 16)
            wt.load(wl);
        else
            wt.wl = wl;
        if constexpr (PREC == 1)
            net16 = make_net_bf16(a.mlp, (1 << D) - 2);
        b2 = a.mlp.b2;
        alpha = a.mlp.alpha;
#pragma unroll
        for (int o = 0; o < 8; ++o)
            noff[o] = (o & 1) + ((o >> 1) & 1) * E2 + ((o >> 2) & 1) * E1 * E2;
    }

    // codes, raw prefetch (no dependence on other blocks)
    __device__ void begin(long long bi)
    {
        b = bi;
        bx = b % a.nb[2];
        by = (b / a.nb[2]) % a.nb[1];
        bz = b / (a.nb[1] * a.nb[2]);
        q = block_geo3(bz, by, bx, a.n, bd0, bd1, bd2);
        bsize = q.ez * q.ey * q.ex;
        full = q.ez == bd0 && q.ey == bd1 && q.ex == bd2;
        g0z = bz * bd0;
        g0y = by * bd1;
        g0x = bx * bd2;
        roff = raw_offset(a.offs, a.partials, b);
        nzero = a.counts[b];
        if (full && BV % 8 == 0 &&
            (reinterpret_cast<uintptr_t>(a.codes + q.start) & 15) == 0) {
            const uint4 *src = reinterpret_cast<const uint4 *>(a.codes + q.start);
            uint4 *dst = reinterpret_cast<uint4 *>(cl);
            for (int i = tid; i < BV / 8; i += NT)
                dst[i] = src[i];
        } else {
            const int ex = q.ex, ey = q.ey;
            for (int li = tid; li < bsize; li += NT) {
                int ci = li;
                if (!full) {
                    const int lx = li % ex, ly = (li / ex) % ey, lz = li / (ex * ey);
                    ci = (lz * bd1 + ly) * bd2 + lx;
                }
                cl[ci] = a.codes[q.start + li];
            }
        }
        raw_ok = nzero <= (unsigned)bsize && roff + nzero <= a.n_raw;
        if (!raw_ok)
            err = kECorrupt;
        rv = (T)0;
        if (raw_ok && tid < 64 && (unsigned)tid < nzero)
            rv = reinterpret_cast<const T *>(a.raw)[roff + tid];
    }

    // low-face halo: plane e0 = 0, rows e1 = 0, columns e2 = 0
    __device__ void halo()
    {
        const long long n1 = a.n[1], n2 = a.n[2];
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
                ptile[(e0 * E1 + e1) * E2 + e2] = load_face(a.pgrid + (gz * n1 + gy) * n2 + gx);
        }
    }

    // balance points (wave 0): rank in stream (local raster) order; the raw
    // value goes to x^ and its grid value into the tile
    __device__ void balance_points()
    {
        if (tid >= 64)
            return;
        const long long n1 = a.n[1], n2 = a.n[2];
        const int ex = q.ex, ey = q.ey;
        const T *raw = reinterpret_cast<const T *>(a.raw);
        T *xh = reinterpret_cast<T *>(a.xh);
        unsigned run = 0;
        const unsigned long long below = (1ULL << tid) - 1ULL;
        for (int c0 = 0; c0 < bsize; c0 += 64) {
            const int li = c0 + tid;
            int ci = li, lx = 0, ly = 0, lz = 0;
            if (li < bsize) {
                lx = li % ex;
                ly = (li / ex) % ey;
                lz = li / (ex * ey);
                ci = (lz * bd1 + ly) * bd2 + lx;
            }
            const bool z = li < bsize && cl[ci] == 0;
            const unsigned long long mask = __ballot(z);
            const unsigned r = run + (unsigned)__popcll(mask & below);
            const T vs = __shfl(rv, (int)(r & 63u), 64);  // every lane takes part
            if (z) {
                const int ei = ((lz + h0) * E1 + (ly + h1)) * E2 + lx + 1;
                if (raw_ok && r < nzero) {
                    const T v = r < 64 ? vs : raw[roff + r];
                    ptile[ei] = grid_value((double)v, a.c, err);
                    xh[((g0z + lz) * n1 + g0y + ly) * n2 + g0x + lx] = v;
                } else {
                    err = kECorrupt;
                    ptile[ei] = 0;
                }
            }
            run += (unsigned)__popcll(mask);
        }
        if (tid == 0 && run != nzero)
            err = kECorrupt;
    }

    // hyperplane sweep over the coded points
    __device__ void sweep()
    {
        const bool net = a.use_net && (!a.judge || a.bflags[b]);
        const int ez = q.ez, ey = q.ey, ex = q.ex;
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
                const bool act = code != 0;
                int nv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                int amask = 0;
                if (act) {
#pragma unroll
                    for (int o = 1; o < (1 << D); ++o)
                        nv[o] = ptile[ei - noff[o]];
                    amask = amask_zy | (a.independent ? (lx != 0) : (g0x + lx != 0));
                }
                long long pred = 0;
                if constexpr (PREC == 1) {
                    // block-uniform branch; inside it every lane of the wave
                    // runs the matrix cores (lanes without a coded point feed zeros)
                    if (net)
                        pred = predict_bf16<D>(nv, amask, act, net16);
                    else if (act)
                        pred = predict<D, HP>(nv, amask, false, wt, b2, alpha);
                } else {
                    if (act)
                        pred = predict<D, HP>(nv, amask, net, wt, b2, alpha);
                }
                if (act) {
                    const long long pv = pred - ((long long)code - kR);
                    int p = 0;
                    if (!(pv > -(long long)kGridLimit && pv < (long long)kGridLimit))
                        err = kECorrupt;
                    else
                        p = (int)pv;
                    ptile[ei] = p;
                }
                __syncthreads();
            }
        }
    }

    // high faces of the block to the scratch grid field
    __device__ void store_faces()
    {
        const long long n1 = a.n[1], n2 = a.n[2];
        const int ez = q.ez, ey = q.ey, ex = q.ex;
        for (int ci = tid; ci < BV; ci += NT) {
            const int lx = ci % bd2, ly = (ci / bd2) % bd1, lz = ci / (bd1 * bd2);
            if (lz >= ez || ly >= ey || lx >= ex)
                continue;
            if (lz == ez - 1 || ly == ey - 1 || lx == ex - 1)
                store_face(a.pgrid + ((g0z + lz) * n1 + g0y + ly) * n2 + g0x + lx,
                           ptile[((lz + h0) * E1 + (ly + h1)) * E2 + lx + 1]);
        }
    }

    // x^ of the coded points (balance points were written with their raw value)
    __device__ void output()
    {
        const long long n1 = a.n[1], n2 = a.n[2];
        const int ez = q.ez, ey = q.ey, ex = q.ex;
        T *xh = reinterpret_cast<T *>(a.xh);
        for (int ci = tid; ci < BV; ci += NT) {
            const int lx = ci % bd2, ly = (ci / bd2) % bd1, lz = ci / (bd1 * bd2);
            if (lz >= ez || ly >= ey || lx >= ex)
                continue;
            if (cl[ci] != 0)
                xh[((g0z + lz) * n1 + g0y + ly) * n2 + g0x + lx] = (T)grid_inverse<T>(
                    ptile[((lz + h0) * E1 + (ly + h1)) * E2 + lx + 1], a.c);
        }
    }
};

// independent blocks: one workgroup per block
template <typename T, int D, int BB, int HP, int PREC>
__global__ void __launch_bounds__(256) k_decode(DecodeArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float4 wl[kWlds];
    stage_weights<HP>(wl, a.mlp);
    __syncthreads();  // the decoder copies the staged weights into registers
    BlockDecoder<T, D, BB, HP, PREC> d(a, smem, wl);
    d.begin(blockIdx.x);
    __syncthreads();
    d.balance_points();
    __syncthreads();
    d.sweep();
    d.output();
    set_status(a.status, d.err);
}

// halo mode: persistent, blocks in dependency order, flags between blocks
template <typename T, int D, int BB, int HP, int PREC>
__global__ void __launch_bounds__(256) k_decode_flow(DecodeArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float4 wl[kWlds];
    __shared__ long long s_ticket[2];
    stage_weights<HP>(wl, a.mlp);
    const int tid = threadIdx.x;
    if (tid == 0)
        s_ticket[0] = (long long)atomicAdd(a.ticket, 1u);
    __syncthreads();  // weights staged (the decoder copies them), first ticket taken
    BlockDecoder<T, D, BB, HP, PREC> d(a, smem, wl);
    for (int it = 0;; ++it) {
        const long long t = s_ticket[it & 1];
        if (t >= a.nblocks)
            break;  // uniform
        // the next ticket is taken now: its latency hides behind this block.
        // Holding it cannot block anyone: the lowest unfinished ticket is
        // always a block some workgroup is working on.
        if (tid == 0)
            s_ticket[(it + 1) & 1] = (long long)atomicAdd(a.ticket, 1u);
        d.begin((long long)a.order[t]);
        // wait for the (up to 7) blocks whose faces form this block's halo
        if (tid < 7) {
            const int o = tid + 1;
            const long long dz = (o >> 2) & 1, dy = (o >> 1) & 1, dx = o & 1;
            const bool used = (D >= 3 || dz == 0) && (D >= 2 || dy == 0);
            const long long nz = d.bz - dz, ny = d.by - dy, nx = d.bx - dx;
            if (used && nz >= 0 && ny >= 0 && nx >= 0) {
                const unsigned *f = a.done + (nz * a.nb[1] + ny) * a.nb[2] + nx;
                unsigned spins = 0;
                while (load_flag(f) != a.epoch) {
                    // a raised status (another wait gave up) ends every wait
                    if (++spins == kSpinLimit ||
                        load_flag(reinterpret_cast<unsigned *>(a.status))) {
                        d.err = kECorrupt;
                        atomicCAS(a.status, kOk, kECorrupt);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
        }
        __syncthreads();
        d.halo();
        __syncthreads();
        d.balance_points();
        __syncthreads();
        d.sweep();
        d.store_faces();
        wait_stores();  // every wave's face stores are done before the flag goes up
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(a.done + d.b, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        d.output();
        __syncthreads();  // LDS is reused by the next block
    }
    set_status(a.status, d.err);
}

// ---------------------------------------------------------------------------
template <typename T, int D, int BB, int HP, int PREC>
static void go(bool flow, const DecodeArgs &a, unsigned grid, unsigned nt, size_t lds,
               hipStream_t s)
{
    if (flow) {
        // persistent launch: as many workgroups as can be resident at once
        // (grid holds the CU count here); more would only wait for tickets
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(&k_decode_flow<T, D, BB, HP, PREC>),
                (int)nt, lds) != hipSuccess || per_cu < 1)
            per_cu = 1;
        const unsigned g =
            (unsigned)std::min<long long>(a.nblocks, (long long)per_cu * (long long)grid);
        hipLaunchKernelGGL((k_decode_flow<T, D, BB, HP, PREC>), dim3(g), dim3(nt), lds, s, a);
    } else {
        hipLaunchKernelGGL((k_decode<T, D, BB, HP, PREC>), dim3(grid), dim3(nt), lds, s, a);
    }
}

template <typename T, int D, int BB>
static void by_hidden(bool flow, int HP, const DecodeArgs &a, unsigned grid, unsigned nt,
                      size_t lds, hipStream_t s)
{
    if (HP == 0)
        go<T, D, BB, 8, 1>(flow, a, grid, nt, lds, s);  // matrix cores (Lorenzo blocks: HP 8)
    else if (HP == 8)
        go<T, D, BB, 8, 0>(flow, a, grid, nt, lds, s);
    else if (HP == 16)
        go<T, D, BB, 16, 0>(flow, a, grid, nt, lds, s);
    else
        go<T, D, BB, 32, 0>(flow, a, grid, nt, lds, s);
}

template <typename T>
static void by_shape(bool flow, int D, int B, int HP, const DecodeArgs &a, unsigned grid,
                     unsigned nt, size_t lds, hipStream_t s)
{
    if (D == 3 && B == 8)
        by_hidden<T, 3, 8>(flow, HP, a, grid, nt, lds, s);
    else if (D == 3 && B == 4)
        by_hidden<T, 3, 4>(flow, HP, a, grid, nt, lds, s);
    else if (D == 3 && B == 16)
        by_hidden<T, 3, 16>(flow, HP, a, grid, nt, lds, s);
    else if (D == 2 && B == 16)
        by_hidden<T, 2, 16>(flow, HP, a, grid, nt, lds, s);
    else if (D == 2 && B == 32)
        by_hidden<T, 2, 32>(flow, HP, a, grid, nt, lds, s);
    else if (D == 2 && B == 64)
        by_hidden<T, 2, 64>(flow, HP, a, grid, nt, lds, s);
    else if (D == 1 && B == 256)
        by_hidden<T, 1, 256>(flow, HP, a, grid, nt, lds, s);
    else if (D == 3)
        by_hidden<T, 3, 0>(flow, HP, a, grid, nt, lds, s);
    else if (D == 2)
        by_hidden<T, 2, 0>(flow, HP, a, grid, nt, lds, s);
    else
        by_hidden<T, 1, 0>(flow, HP, a, grid, nt, lds, s);
}

hipError_t launch_decode(const Geom &g, const DevConsts &c, const pwrel_mlp *model, int flags,
                         const uint8_t *bflags, const uint16_t *codes, const uint32_t *counts,
                         const void *raw, unsigned long long n_raw, Workspace &ws,
                         const unsigned *order, unsigned epoch, void *xh, int num_cus,
                         hipStream_t s)
{
    DecodeArgs a{};
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bd[d] = g.bd[d];
        a.nb[d] = g.nb[d];
    }
    a.nblocks = g.nblocks;
    a.use_net = (flags & PWREL_HF_NET) ? 1 : 0;
    a.judge = (flags & PWREL_HF_JUDGE) ? 1 : 0;
    a.independent = (flags & PWREL_HF_INDEPENDENT) ? 1 : 0;
    a.bflags = bflags;
    a.codes = codes;
    a.counts = counts;
    a.offs = ws.offsets;
    a.partials = ws.partials;
    a.raw = raw;
    a.n_raw = n_raw;
    a.xh = xh;
    a.pgrid = ws.pgrid;
    a.status = ws.status;
    a.order = order;
    a.done = ws.done;
    a.ticket = ws.ticket;
    a.epoch = epoch;
    a.c = c;
    a.mlp = pack_mlp(a.use_net ? model : nullptr);
    const bool mfma = a.use_net && model && model->precision == 1;
    const int HP = mfma ? 0 : hidden_pad(a.use_net ? model : nullptr);
    const int h0 = g.D >= 3 ? 1 : 0, h1 = g.D >= 2 ? 1 : 0;
    const size_t ne = (size_t)(g.bd[0] + h0) * (g.bd[1] + h1) * (g.bd[2] + 1);
    const size_t bv = (size_t)g.bd[0] * g.bd[1] * g.bd[2];
    const size_t lds = ((bv * 2 + 15) & ~size_t(15)) + ne * 4;
    const long long nlines = (long long)g.bd[0] * g.bd[1];
    const unsigned nt = (unsigned)std::min(256LL, std::max(64LL, (nlines + 63) / 64 * 64));
    const bool flow = !a.independent;
    const unsigned grid = flow ? (unsigned)std::max(num_cus, 1) : (unsigned)g.nblocks;
    if (g.dtype == PWREL_F32)
        by_shape<float>(flow, g.D, g.B, HP, a, grid, nt, lds, s);
    else
        by_shape<double>(flow, g.D, g.B, HP, a, grid, nt, lds, s);
    return hipGetLastError();
}

// Block order of the halo-mode decoder: block levels bz + by + bx ascending,
// (bz, by) ascending inside a level.
void block_order(const Geom &g, std::vector<unsigned> &order)
{
    order.clear();
    order.reserve((size_t)g.nblocks);
    const long long nlev = (g.nb[0] - 1) + (g.nb[1] - 1) + (g.nb[2] - 1) + 1;
    for (long long lev = 0; lev < nlev; ++lev)
        for (long long bz = std::max(0LL, lev - (g.nb[1] - 1) - (g.nb[2] - 1));
             bz <= std::min(g.nb[0] - 1, lev); ++bz)
            for (long long by = std::max(0LL, lev - bz - (g.nb[2] - 1));
                 by <= std::min(g.nb[1] - 1, lev - bz); ++by)
                order.push_back((unsigned)((bz * g.nb[1] + by) * g.nb[2] + (lev - bz - by)));
}

}  // namespace pwrel
