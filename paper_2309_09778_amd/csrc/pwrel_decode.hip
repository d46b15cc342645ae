// Decompression kernels (gfx950): one block at a time per workgroup.
//
// Before the decoder, k_raw_grid maps every raw (balance-point) value to its
// grid value, so that no decoder evaluates the log-domain map.
//
// Per block.  Prologue (nothing here waits for another block): the block's
// codes (one 16-byte load per lane where the block is aligned) and its first
// 64 raw values and their grid values (one per lane of wave 0); wave 0 ranks
// the balance points, writes their raw values to x^ and their grid values
// into the tile, so that the sweep only handles coded points.  Then the
// low-face halo grid values (written by earlier blocks).  Sweep: hyperplane
// by hyperplane (lz + ly + lx = s), every line (lz, ly) of the block owned by
// one lane, which decodes its point lx = s - lz - ly with the same predictor
// as the encoder.
//
// Independent blocks: one launch, one workgroup per block, which ends with
// x^ = inverse(grid value) for its coded points.  Halo mode: one persistent
// launch; workgroups take blocks from an atomic ticket counter in an order
// where every block comes after the blocks it reads (block levels
// bz + by + bx ascending), wait for those blocks' done flags, and raise their
// own flag once their high faces are in the scratch grid field.  A block is
// only waited on after a running workgroup has taken it, so the lowest
// unfinished ticket can always proceed; the waits are bounded all the same.
// Every grid value of the field goes to the scratch field (tagged coded or
// balance point), and k_inverse then writes x^ of the coded points: the
// exp2 of the inverse map stays out of the chain of dependent blocks.
#include <type_traits>

#include "pwrel_bf16.h"
#include "pwrel_decode.h"

namespace pwrel {



constexpr unsigned kSpinLimit = 1u << 20;  // polls of one flag before giving up
// Scratch grid field entry: 2 p + 1 for a balance point, 2 p for a coded
// point (|p| < 2^30, so the entry fits in 32 bits)
__device__ __forceinline__ int scratch_entry(int p, bool balance)
{
    return (int)(((unsigned)p << 1) | (balance ? 1u : 0u));
}
__device__ __forceinline__ int scratch_grid(int v) { return v >> 1; }

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

template <typename T, int D, int BB, int HP, int PREC, bool FLOW>
struct BlockDecoder {
    static constexpr bool CT = BB > 0;
    static constexpr int h0 = D >= 3 ? 1 : 0, h1 = D >= 2 ? 1 : 0;
    // weights stay in LDS (broadcast loads): registers set the occupancy,
    // and occupancy hides the latency of the sweep's dependent steps
    using Wt = WeightsLds;

    const DecodeArgs &a;
    int NT, tid;
    int B, bd0, bd1, bd2, E0, E1, E2, ne, BV;
    unsigned short *cl;  // codes, full-block layout (16-byte aligned)
    int *ptile;          // grid tile with the low-face halo
    Wt wt;
    NetBf16Lds net16;
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
    int rp;

    __device__ BlockDecoder(const DecodeArgs &args, unsigned char *smem, const float4 *wl,
                            const unsigned *tb)
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
        wt.wl = wl;
        if constexpr (PREC == 1)
            net16 = make_net_bf16_lds(a.mlp, (1 << D) - 2, tb);
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
        rp = 0;
        if (raw_ok && tid < 64 && (unsigned)tid < nzero) {
            rv = reinterpret_cast<const T *>(a.raw)[roff + tid];
            rp = a.praw[roff + tid];
        }
    }

    // low-face halo: plane e0 = 0, rows e1 = 0, columns e2 = 0.  Each lane
    // issues up to kHaloBatch loads before it stores any of them to LDS, so
    // that their latencies overlap.
    static constexpr int kHaloBatch = 4;

    // on a high face of the block (stored by store_faces)
    __device__ __forceinline__ bool face(int lz, int ly, int lx) const
    {
        return lz == q.ez - 1 || ly == q.ey - 1 || lx == q.ex - 1;
    }
    __device__ void halo()
    {
        const long long n1 = a.n[1], n2 = a.n[2];
        const int nh0 = h0 ? E1 * E2 : 0, nh1 = h1 ? bd0 * E2 : 0, nh2 = bd0 * bd1;
        const int nh = nh0 + nh1 + nh2;
        for (int base = 0; base < nh; base += kHaloBatch * NT) {
            int li[kHaloBatch], v[kHaloBatch];
#pragma unroll
            for (int k = 0; k < kHaloBatch; ++k) {
                const int hq = base + k * NT + tid;
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
                const bool in = hq < nh && gz >= 0 && gy >= 0 && gx >= 0 && gz < a.n[0] &&
                                gy < n1 && gx < n2;
                li[k] = in ? (e0 * E1 + e1) * E2 + e2 : -1;
                v[k] = in ? scratch_grid(load_face(a.pgrid + (gz * n1 + gy) * n2 + gx)) : 0;
            }
#pragma unroll
            for (int k = 0; k < kHaloBatch; ++k)
                if (li[k] >= 0)
                    ptile[li[k]] = v[k];
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
            const int ps = __shfl(rp, (int)(r & 63u), 64);
            if (z) {
                const int ei = ((lz + h0) * E1 + (ly + h1)) * E2 + lx + 1;
                if (raw_ok && r < nzero) {
                    const T v = r < 64 ? vs : raw[roff + r];
                    const int p = r < 64 ? ps : a.praw[roff + r];
                    const long long gi = ((g0z + lz) * n1 + g0y + ly) * n2 + g0x + lx;
                    ptile[ei] = p;
                    xh[gi] = v;
                    if (FLOW && !face(lz, ly, lx))
                        a.pgrid[gi] = scratch_entry(p, true);
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
            const long long gline = (gz * a.n[1] + gy) * a.n[2] + g0x;
            const bool zy_face = lz == ez - 1 || ly == ey - 1;
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
                    if (FLOW && !zy_face && lx != ex - 1)
                        a.pgrid[gline + lx] = scratch_entry(p, false);
                }
                __syncthreads();
            }
        }
    }

    // high faces of the block to the scratch grid field: plane lz = ez - 1,
    // then plane ly = ey - 1 and column lx = ex - 1 below it
    __device__ void store_faces()
    {
        const long long n1 = a.n[1], n2 = a.n[2];
        const int ez = q.ez, ey = q.ey, ex = q.ex;
        const int f0 = ey * ex, f1 = (ez - 1) * ex, f2 = (ez - 1) * (ey - 1);
        for (int fi = tid; fi < f0 + f1 + f2; fi += NT) {
            int lz, ly, lx;
            if (fi < f0) {
                lz = ez - 1;
                ly = fi / ex;
                lx = fi - ly * ex;
            } else if (fi < f0 + f1) {
                const int r = fi - f0;
                lz = r / ex;
                ly = ey - 1;
                lx = r - lz * ex;
            } else {
                const int r = fi - f0 - f1;
                lz = r / (ey - 1);
                ly = r - lz * (ey - 1);
                lx = ex - 1;
            }
            const int p = ptile[((lz + h0) * E1 + (ly + h1)) * E2 + lx + 1];
            const bool bal = cl[(lz * bd1 + ly) * bd2 + lx] == 0;
            store_face(a.pgrid + ((g0z + lz) * n1 + g0y + ly) * n2 + g0x + lx,
                       scratch_entry(p, bal));
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
    __shared__ unsigned tb[PREC == 1 ? 64 : 1];
    stage_weights<HP>(wl, a.mlp);
    if constexpr (PREC == 1)
        stage_net_bf16(tb, a.mlp);
    __syncthreads();
    BlockDecoder<T, D, BB, HP, PREC, false> d(a, smem, wl, tb);
    d.begin(a.partial_only ? partial_block(blockIdx.x, a) : (long long)blockIdx.x);
    __syncthreads();
    d.balance_points();
    __syncthreads();
    d.sweep();
    d.output();
    set_status(a.status, d.err);
}

// halo mode: persistent, blocks in dependency order, flags between blocks
// (the BF16 variant is held to 128 registers: four waves per SIMD; the
// others need fewer)
template <typename T, int D, int BB, int HP, int PREC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == 1 ? 4 : 1)))
k_decode_flow(DecodeArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float4 wl[kWlds];
    __shared__ unsigned tb[PREC == 1 ? 64 : 1];
    __shared__ long long s_ticket[2];
    stage_weights<HP>(wl, a.mlp);
    if constexpr (PREC == 1)
        stage_net_bf16(tb, a.mlp);
    const int tid = threadIdx.x;
    if (tid == 0)
        s_ticket[0] = (long long)atomicAdd(a.ticket, 1u);
    __syncthreads();  // weights staged, first ticket taken
    BlockDecoder<T, D, BB, HP, PREC, true> d(a, smem, wl, tb);
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
        __syncthreads();
        // balance points read only this block's own data: placed before the
        // wait, off the chain of dependent blocks
        d.balance_points();
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
        d.sweep();
        d.store_faces();
        wait_stores();  // every wave's face stores are done before the flag goes up
        __syncthreads();  // (the barrier also ends every read of LDS: the next block reuses it)
        if (tid == 0)
            __hip_atomic_store(a.done + d.b, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    set_status(a.status, d.err);
}

// ---------------------------------------------------------------------------
// Halo-mode decoder of 3-D fields with 8^3 blocks, by pencils.
//
// A pencil is the row of blocks (bz, by, bx = 0 .. nb2 - 1).  A workgroup of
// two waves decodes it.  The compute wave: lane (lz, ly) owns line (lz, ly)
// and at step s decodes its point x = s - lz - ly, the hyperplane order of
// the blocks continued across block boundaries (each point still has the
// predictor, inputs and code of the block it belongs to).  It touches global
// memory only to store faces, and never waits for memory.  The memory wave
// feeds it through LDS: halo cells, codes, judge flags and balance points
// ahead of the compute wave, and the grid values of finished blocks to the
// scratch field behind it.
//
// Grid values sit in an LDS ring of kPenRing columns: rows (tz, ty) =
// (lz + 1, ly + 1), plus the halo plane tz = 0 (z - 1) and the halo row
// ty = 0 (y - 1) from the pencils (bz - 1, .) and (bz, by - 1).  Faces travel
// as tagged words (epoch << 32 | grid value): the lanes of the last z line
// store each grid value they decode to the z-face buffer, the lanes of the
// last y line to the y-face buffer; 17 lanes of the memory wave load the 17
// halo lines in batches of kPenGroup steps, two batches ahead, and take a
// word once its tag is this call's epoch (else they poll it, bounded).  The
// loads are issued by every lane, without branches (lanes with nothing to
// fetch read a valid dummy word), so that waiting for the older batch never
// waits for the newer one.  Nothing else orders pencils: a
// pencil only polls pencils with a lower ticket, which running workgroups
// hold.
//
// The waves publish progress in LDS: `rdy` (memory wave: every halo cell and
// block the compute wave needs up to that step is in place) and `cdone`
// (compute wave: last finished step).  Each wave writes its data before its
// counter; the LDS executes one wave's operations in order.
constexpr int kPenRing = 32;  // tile columns (a power of two)
constexpr int kPenRS = 34;    // tile row stride: at most two-way LDS bank conflicts
constexpr int kPenGroup = 2;  // halo words per load batch; two batches are in flight
constexpr int kPenAhead = 8;  // halo delivered at most this many steps ahead
constexpr int kPenRows = 81;  // (tz, ty) in [0, 9)^2
constexpr unsigned kPenPollLimit = 1u << 26;  // LDS polls of one wave before giving up

__device__ __forceinline__ unsigned long long load_tagged(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_tagged(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ long long lds_get(const long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_put(long long *p, long long v)
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the data written before stays before
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename T, int HP, int PREC>
__global__ void __launch_bounds__(128) k_decode_pencil(DecodeArgs a)
{
    __shared__ int tile[kPenRows * kPenRS];
    __shared__ __align__(16) unsigned short cring[8 * 512];
    __shared__ unsigned char fring[8];
    __shared__ float4 wl[kWlds];
    __shared__ unsigned tb[PREC == 1 ? 64 : 1];
    __shared__ long long s_ticket, rdy, cdone;
    stage_weights<HP>(wl, a.mlp);
    if constexpr (PREC == 1)
        stage_net_bf16(tb, a.mlp);
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lz = lane >> 3, ly = lane & 7;
    const long long n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const long long nb0 = a.nb[0], nb1 = a.nb[1], nb2 = a.nb[2];
    const long long npen = nb0 * nb1;
    const unsigned epoch = a.epoch;
    const T *raw = reinterpret_cast<const T *>(a.raw);
    T *xh = reinterpret_cast<T *>(a.xh);
    int err = kOk;

    for (;;) {
        if (threadIdx.x == 0) {
            s_ticket = (long long)atomicAdd(a.ticket, 1u);
            rdy = -1;
            cdone = -1;
        }
        __syncthreads();
        const long long t = s_ticket;
        if (t >= npen)
            break;  // uniform
        const long long pid = (long long)a.order[t];
        const long long bz = pid / nb1, by = pid - (pid / nb1) * nb1;
        const int ez = (int)std::min(8LL, n0 - 8 * bz), ey = (int)std::min(8LL, n1 - 8 * by);
        const long long s_last = (n2 - 1) + (ez - 1) + (ey - 1);

        if (wave == 0) {
            // ------------------------------------------------------ compute wave
            WeightsLds wt;
            wt.wl = wl;
            NetBf16Lds net16;
            if constexpr (PREC == 1)
                net16 = make_net_bf16_lds(a.mlp, 6, tb);
            const float b2 = a.mlp.b2, alpha = a.mlp.alpha;
            const bool on = lz < ez && ly < ey;
            const long long gz = 8 * bz + lz, gy = 8 * by + ly;
            const int amask_zy = (gy != 0 ? 2 : 0) | (gz != 0 ? 4 : 0);
            const bool zface = on && lz == ez - 1 && bz + 1 < nb0;
            const bool yface = on && ly == ey - 1 && by + 1 < nb1;
            unsigned long long *zrow = a.zf + (bz * n1 + (on ? gy : 0)) * n2;
            unsigned long long *yrow = a.yf + (by * n0 + (on ? gz : 0)) * n2;
            const int r0 = ((lz + 1) * 9 + (ly + 1)) * kPenRS;
            const unsigned long long tag = (unsigned long long)epoch << 32;
            const bool use_net = a.use_net != 0;
            long long ready = -1;
            unsigned polls = 0;
            for (long long s = 0; s <= s_last; ++s) {
                while (ready < s) {  // uniform
                    ready = lds_get(&rdy);
                    if (ready < s) {
                        if (++polls == kPenPollLimit) {
                            err = kECorrupt;
                            ready = s_last;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                const long long x = s - lz - ly;
                const bool act = on && x >= 0 && x < n2;
                const int xs = (int)(x & (kPenRing - 1)), xs1 = (int)((x - 1) & (kPenRing - 1));
                const int bs = (int)((x >> 3) & 7);
                const int lx = (int)(x & 7);
                // every lane reads its code (the ring index is in range for any x),
                // so that the code, the flag and the neighbours below are loaded
                // together, one LDS round trip
                const unsigned cv = cring[bs * 512 + (lz * 8 + ly) * 8 + lx];
                const unsigned code = act ? cv : 0u;
                const bool flag = fring[bs] != 0;
                // neighbours read with the code (one LDS round trip); used when coded
                int nv[8];
                nv[0] = 0;
#pragma unroll
                for (int o = 1; o < 8; ++o) {
                    const int dz = (o >> 2) & 1, dy = (o >> 1) & 1, dx = o & 1;
                    nv[o] = tile[r0 - (dz * 9 + dy) * kPenRS + (dx ? xs1 : xs)];
                }
                const bool coded = code != 0;
                const int amask = amask_zy | (x > 0 ? 1 : 0);
                const bool net = use_net && coded && flag;
                const bool full_nb = amask == 7;
                // Predictions in 32-bit wrap-around arithmetic: exact wherever the
                // point is coded (then |prediction - p| < 2^15 and |p| < 2^30).
                unsigned lor = 0u;
#pragma unroll
                for (int o = 1; o < 8; ++o)
                    if ((o & ~amask) == 0)
                        lor = lorenzo_sign(o) > 0 ? lor + (unsigned)nv[o] : lor - (unsigned)nv[o];
                unsigned pred = lor;
                if constexpr (PREC == 1) {
                    if (__ballot(net) != 0ULL) {  // wave-uniform: the matrix cores take every lane
                        const bool use = net && full_nb;
                        float u[6];
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            u[k] = use ? (float)(int)((unsigned)nv[k + 2] - (unsigned)nv[1]) : 0.0f;
                        float y = net_bf16(net16, u);
                        if (y > 0x1p30f)
                            y = 0x1p30f;
                        if (!(y >= -0x1p30f))
                            y = -0x1p30f;
                        if (use)
                            pred = (unsigned)nv[1] + (unsigned)(int)__builtin_rintf(y);
                    }
                } else {
                    if (net && full_nb) {
                        float y = net_f32<3, HP>(nv, wt, b2, alpha);
                        if (y > 0x1p30f)
                            y = 0x1p30f;
                        if (!(y >= -0x1p30f))
                            y = -0x1p30f;
                        pred = (unsigned)nv[1] + (unsigned)(int)__builtin_rintf(y);
                    }
                }
                int p = 0;
                if (coded) {
                    const int pv = (int)(pred - (code - (unsigned)kR));
                    if (!(pv > -(1 << 30) && pv < (1 << 30)))
                        err = kECorrupt;
                    else
                        p = pv;
                    tile[r0 + xs] = p;
                } else if (act) {
                    p = tile[r0 + xs];  // a balance point, staged
                }
                if (act && zface)
                    store_tagged(zrow + x, tag | (unsigned)p);
                if (act && yface)
                    store_tagged(yrow + x, tag | (unsigned)p);
                if (lane == 0)
                    lds_put(&cdone, s);
            }
        } else {
            // ------------------------------------------------------- memory wave
            const long long prow = ((8 * bz + lz) * n1 + 8 * by + ly) * n2;
            const bool on = lz < ez && ly < ey;
            const int r0 = ((lz + 1) * 9 + (ly + 1)) * kPenRS;
            // halo line of lanes 0 .. 16: (tz = 0, ty = lane) or (tz = lane - 8, ty = 0)
            int hrow = 0, hoff = 0;
            const unsigned long long *hsrc = nullptr;
            if (lane < 9) {
                const int ty = lane;
                const long long y = 8 * by + ty - 1;
                hrow = ty * kPenRS;
                hoff = ty > 0 ? ty - 1 : 0;
                if (bz >= 1 && y >= 0 && ty <= ey)
                    hsrc = a.zf + ((bz - 1) * n1 + y) * n2;
            } else if (lane < 17) {
                const int tz = lane - 8;
                const long long z = 8 * bz + tz - 1;
                hrow = (tz * 9) * kPenRS;
                hoff = tz - 1;
                if (by >= 1 && tz <= ez)
                    hsrc = a.yf + ((by - 1) * n0 + z) * n2;
            }
            const unsigned long long *hbase = hsrc ? hsrc : a.zf;
            long long cd = -1;  // compute wave progress, as last read
            unsigned polls = 0;
            auto wait_compute = [&](long long need) {
                while (cd < need) {  // uniform
                    cd = lds_get(&cdone);
                    if (cd < need) {
                        if (++polls == kPenPollLimit) {
                            err = kECorrupt;
                            cd = s_last;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
            };

            // block pipeline: metadata two blocks before staging, data one block before
            auto blk = [&](long long bx) { return (bz * nb1 + by) * nb2 + bx; };
            unsigned long long m_roff = 0, d_roff = 0;
            unsigned m_nz = 0, d_nz = 0;
            uint4 d_codes = make_uint4(0, 0, 0, 0);
            T d_rv = (T)0;
            int d_rp = 0, d_flag = 0;
            auto load_meta = [&](long long bx) {
                const long long b = blk(bx);
                m_roff = raw_offset(a.offs, a.partials, b);
                m_nz = a.counts[b];
            };
            auto load_data = [&](long long bx) {
                const BlockGeo q = block_geo3(bz, by, bx, a.n, 8, 8, 8);
                d_roff = m_roff;
                d_nz = m_nz;
                const bool full = q.ez == 8 && q.ey == 8 && q.ex == 8 &&
                                  (reinterpret_cast<uintptr_t>(a.codes + q.start) & 15) == 0;
                if (full)
                    d_codes = reinterpret_cast<const uint4 *>(a.codes + q.start)[lane];
                const bool ok = d_nz <= 512u && d_roff + d_nz <= a.n_raw;
                d_rv = (T)0;
                d_rp = 0;
                if (ok && (unsigned)lane < d_nz) {
                    d_rv = raw[d_roff + lane];
                    d_rp = a.praw[d_roff + lane];
                }
                d_flag = a.judge ? (int)a.bflags[blk(bx)] : 1;
            };
            // codes into the ring, judge flag, balance points into the tile and x^
            auto stage = [&](long long bx) {
                const BlockGeo q = block_geo3(bz, by, bx, a.n, 8, 8, 8);
                unsigned short *cl = cring + (bx & 7) * 512;
                const bool full = q.ez == 8 && q.ey == 8 && q.ex == 8 &&
                                  (reinterpret_cast<uintptr_t>(a.codes + q.start) & 15) == 0;
                if (full) {
                    reinterpret_cast<uint4 *>(cl)[lane] = d_codes;
                } else {
                    for (int li = lane; li < 512; li += 64) {
                        const int lx = li & 7, lyy = (li >> 3) & 7, lzz = li >> 6;
                        unsigned short v = 0;
                        if (lzz < q.ez && lyy < q.ey && lx < q.ex)
                            v = a.codes[q.start + (lzz * q.ey + lyy) * q.ex + lx];
                        cl[li] = v;
                    }
                }
                if (lane == 0)
                    fring[bx & 7] = (unsigned char)d_flag;
                const int bsize = q.ez * q.ey * q.ex;
                const bool raw_ok = d_nz <= (unsigned)bsize && d_roff + d_nz <= a.n_raw;
                if (!raw_ok)
                    err = kECorrupt;
                if (full && d_nz == 0) {
                    // no balance point (the common case): only check that no code is 0
                    const unsigned w[4] = {d_codes.x, d_codes.y, d_codes.z, d_codes.w};
                    bool z = false;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        z = z || (w[i] & 0xffffu) == 0u || (w[i] >> 16) == 0u;
                    if (__ballot(z) != 0ULL)
                        err = kECorrupt;
                    return;
                }
                unsigned run = 0;
                const unsigned long long below = (1ULL << lane) - 1ULL;
                for (int c0 = 0; c0 < bsize; c0 += 64) {
                    const int li = c0 + lane;
                    int lx = 0, lyy = 0, lzz = 0;
                    if (li < bsize) {
                        lx = li % q.ex;
                        lyy = (li / q.ex) % q.ey;
                        lzz = li / (q.ex * q.ey);
                    }
                    const bool z = li < bsize && cl[(lzz * 8 + lyy) * 8 + lx] == 0;
                    const unsigned long long mask = __ballot(z);
                    const unsigned r = run + (unsigned)__popcll(mask & below);
                    const T vs = __shfl(d_rv, (int)(r & 63u), 64);
                    const int ps = __shfl(d_rp, (int)(r & 63u), 64);
                    if (z) {
                        if (raw_ok && r < d_nz) {
                            const T v = r < 64 ? vs : raw[d_roff + r];
                            const int pv = r < 64 ? ps : a.praw[d_roff + r];
                            const long long xg = 8 * bx + lx;
                            tile[((lzz + 1) * 9 + lyy + 1) * kPenRS +
                                 (int)(xg & (kPenRing - 1))] = pv;
                            xh[((8 * bz + lzz) * n1 + 8 * by + lyy) * n2 + xg] = v;
                        } else {
                            err = kECorrupt;
                        }
                    }
                    run += (unsigned)__popcll(mask);
                }
                if (lane == 0 && run != d_nz)
                    err = kECorrupt;
            };
            // grid values of a finished block to the scratch field
            auto flush = [&](long long bx) {
                const int ex = (int)std::min(8LL, n2 - 8 * bx);
                const unsigned short *cl = cring + (bx & 7) * 512 + (lz * 8 + ly) * 8;
                const int *tr = tile + r0 + (int)((8 * bx) & (kPenRing - 1));
                if (on) {
                    int *dst = a.pgrid + prow + 8 * bx;
                    if (ex == 8 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                        int v[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k)
                            v[k] = scratch_entry(tr[k], cl[k] == 0);
                        reinterpret_cast<int4 *>(dst)[0] = make_int4(v[0], v[1], v[2], v[3]);
                        reinterpret_cast<int4 *>(dst)[1] = make_int4(v[4], v[5], v[6], v[7]);
                    } else {
                        for (int k = 0; k < ex; ++k)
                            dst[k] = scratch_entry(tr[k], cl[k] == 0);
                    }
                }
            };

            long long hready = -1;  // halo delivered for every need-step <= hready
            long long staged = -1;  // blocks 0 .. staged are in the rings
            long long flushed = -1; // blocks 0 .. flushed are in the scratch field
            auto publish = [&]() {
                // step s needs the halo of need-steps <= s and the blocks <= s / 8
                const long long blim = staged >= nb2 - 1 ? s_last : 8 * staged + 7;
                if (lane == 0)
                    lds_put(&rdy, std::min(hready, blim));
            };
            // Stage block j when the compute wave is done with block j - 4 (whose
            // tile columns and ring slot it takes): flush j - 4 first.  Column
            // 8 (j - 4) + 7 is last read by lane (7, 7) at step 8 j - 10.
            auto try_stage = [&](bool force) {
                const long long j = staged + 1;
                if (j >= nb2)
                    return;
                const long long need = std::min(8 * j - 10, s_last);
                if (j >= 4 || force) {
                    if (force)
                        wait_compute(j >= 4 ? need : -1);
                    else if (cd < need && (cd = lds_get(&cdone)) < need)
                        return;
                }
                if (j >= 4) {
                    flush(j - 4);
                    flushed = j - 4;
                }
                stage(j);
                staged = j;
                publish();
                if (j + 1 < nb2)
                    load_data(j + 1);
                if (j + 2 < nb2)
                    load_meta(j + 2);
            };

            // pipeline start: block 0 staged, data of block 1 and metadata of block 2 in flight
            load_meta(0);
            load_data(0);
            if (nb2 > 1)
                load_meta(1);
            stage(0);
            staged = 0;
            if (nb2 > 1)
                load_data(1);
            if (nb2 > 2)
                load_meta(2);
            publish();

            auto issue = [&](unsigned long long (&h)[kPenGroup], long long tau0) {
#pragma unroll
                for (int k = 0; k < kPenGroup; ++k) {
                    long long c = tau0 + k - hoff;
                    c = c < 0 ? 0 : (c >= n2 ? n2 - 1 : c);
                    h[k] = load_tagged(hbase + (hsrc ? c : 0));
                }
            };
            // Deliver the batch h (need-steps tau0 ..); hn is the next batch, already
            // issued.  A word not yet written by the upstream pencil is polled, and
            // each poll also reloads the word of the next need-step (in h or hn):
            // the upstream pencil writes it one step later, so it is often valid
            // when the polled word lands, which saves it a round trip of its own.
            // Reloading a valid word is harmless: a word of this call only changes
            // from stale to valid.
            auto deliver = [&](unsigned long long (&h)[kPenGroup], long long tau0,
                               unsigned long long (&hn)[kPenGroup]) {
#pragma unroll
                for (int k = 0; k < kPenGroup; ++k) {
                    const long long tau = tau0 + k;
                    if (tau > s_last)
                        break;  // uniform
                    if (cd < tau - kPenAhead)
                        wait_compute(tau - kPenAhead);
                    const long long c = tau - hoff;
                    const bool need = hsrc && c >= 0 && c < n2;
                    unsigned long long v = h[k];
                    if (__ballot(need && (unsigned)(v >> 32) != epoch) != 0ULL) {
                        // not yet written by the upstream pencil: poll it
                        unsigned spins = 0;
                        while (need && (unsigned)(v >> 32) != epoch) {
                            if (++spins == kSpinLimit ||
                                load_flag(reinterpret_cast<unsigned *>(a.status))) {
                                err = kECorrupt;
                                atomicCAS(a.status, kOk, kECorrupt);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            v = load_tagged(hsrc + c);
                            const long long c1 = c + 1 < n2 ? c + 1 : n2 - 1;
                            if (k + 1 < kPenGroup)
                                h[k + 1 < kPenGroup ? k + 1 : 0] = load_tagged(hsrc + c1);
                            else
                                hn[0] = load_tagged(hsrc + c1);
                        }
                    }
                    if (need)
                        tile[hrow + (int)(c & (kPenRing - 1))] = (int)(unsigned)v;
                    hready = tau;
                    publish();
                }
            };
            unsigned long long hA[kPenGroup], hB[kPenGroup];
            issue(hA, 0);
            issue(hB, kPenGroup);
            for (long long t0 = 0; t0 <= s_last; t0 += 2 * kPenGroup) {
                deliver(hA, t0, hB);
                try_stage(8 * (staged + 1) <= t0 + 2 * kPenGroup);
                issue(hA, t0 + 2 * kPenGroup);
                deliver(hB, t0 + kPenGroup, hA);
                try_stage(8 * (staged + 1) <= t0 + 3 * kPenGroup);
                issue(hB, t0 + 3 * kPenGroup);
            }
            hready = s_last + 1;
            publish();
            // the remaining blocks
            while (staged + 1 < nb2)
                try_stage(true);
            for (long long j = flushed + 1; j < nb2; ++j) {
                wait_compute(s_last);
                flush(j);
            }
        }
        __syncthreads();  // both waves are done with the pencil (LDS is reused)
    }
    set_status(a.status, err);
}

// grid values of the raw values (Eq. 6, 7, 12), in stream order
template <typename T>
__global__ void __launch_bounds__(256) k_raw_grid(const T *raw, unsigned long long n, DevConsts c,
                                                  int *praw, int *status)
{
    int err = kOk;
    const unsigned long long stride = (unsigned long long)gridDim.x * 256ull;
    for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += stride)
        praw[i] = grid_value((double)raw[i], c, err);
    set_status(status, err);
}

// x^ of the coded points from the scratch grid field of the halo-mode
// decoder (a balance point's x^ is already written)
// x^ of every grid value in [lo, lo + n) (the decoders' lookup table)
template <typename T>
__global__ void __launch_bounds__(256) k_inv_table(DevConsts c, long long lo, long long n, T *tab)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        tab[i] = (T)grid_inverse<T>((int)(lo + i), c);
}

template <typename T>
__device__ __forceinline__ T inverse_tab(int q, const DevConsts &c, const T *tab, long long lo,
                                         long long nt)
{
    const long long k = (long long)q - lo;
    return (tab && k >= 0 && k < nt) ? tab[k] : (T)grid_inverse<T>(q, c);
}

template <typename T>
__global__ void __launch_bounds__(256) k_inverse(const int *pgrid, long long n, DevConsts c,
                                                 const T *tab, long long lo, long long nt, T *xh)
{
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) {
        const int v = pgrid[i];
        if (!(v & 1))
            xh[i] = inverse_tab<T>(scratch_grid(v), c, tab, lo, nt);
    }
}

// The same for FP32 fields with x^ 16-byte aligned: four values per thread
// (one 16-byte load, one 16-byte store where all four are coded), two groups
// of four in flight per thread; the tail n % 4 in scalar form.
__device__ __forceinline__ void inverse4(const int4 &v, const DevConsts &c, const float *tab,
                                         long long lo, long long nt, float *dst)
{
    const int e[4] = {v.x, v.y, v.z, v.w};
    float o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        o[k] = inverse_tab<float>(scratch_grid(e[k]), c, tab, lo, nt);
    if (((e[0] | e[1] | e[2] | e[3]) & 1) == 0) {
        *reinterpret_cast<float4 *>(dst) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (!(e[k] & 1))
                dst[k] = o[k];
    }
}

__global__ void __launch_bounds__(256) k_inverse_f32x4(const int *pgrid, long long n,
                                                       DevConsts c, const float *tab, long long lo,
                                                       long long nt, float *xh)
{
    const long long n4 = n >> 2;
    const int4 *p4 = reinterpret_cast<const int4 *>(pgrid);
    const long long stride = (long long)gridDim.x * 256;
    long long i = blockIdx.x * 256LL + threadIdx.x;
    for (; i + stride < n4; i += 2 * stride) {
        const int4 a = p4[i], b = p4[i + stride];
        inverse4(a, c, tab, lo, nt, xh + 4 * i);
        inverse4(b, c, tab, lo, nt, xh + 4 * (i + stride));
    }
    if (i < n4)
        inverse4(p4[i], c, tab, lo, nt, xh + 4 * i);
    const long long r = 4 * n4 + blockIdx.x * 256LL + threadIdx.x;
    if (r < n) {
        const int v = pgrid[r];
        if (!(v & 1))
            xh[r] = inverse_tab<float>(scratch_grid(v), c, tab, lo, nt);
    }
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

// pencil decoder launch: persistent, as many two-wave workgroups as fit
template <typename T, int HP, int PREC>
static void pencil_go(const DecodeArgs &a, unsigned num_cus, hipStream_t s)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_decode_pencil<T, HP, PREC>), 128, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const long long npen = a.nb[0] * a.nb[1];
    const unsigned g = (unsigned)std::min<long long>(npen, (long long)per_cu * num_cus);
    hipLaunchKernelGGL((k_decode_pencil<T, HP, PREC>), dim3(g), dim3(128), 0, s, a);
}

template <typename T>
static void pencil_by_hidden(int HP, const DecodeArgs &a, unsigned num_cus, hipStream_t s)
{
    if (HP == 0)
        pencil_go<T, 8, 1>(a, num_cus, s);
    else if (HP == 8)
        pencil_go<T, 8, 0>(a, num_cus, s);
    else if (HP == 16)
        pencil_go<T, 16, 0>(a, num_cus, s);
    else
        pencil_go<T, 32, 0>(a, num_cus, s);
}

bool pencil_mode(const Geom &g) { return g.D == 3 && g.B == 8; }

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
    a.praw = ws.praw;
    a.status = ws.status;
    a.order = order;
    a.done = ws.done;
    a.ticket = ws.ticket;
    a.epoch = epoch;
    a.zf = ws.zf;
    a.yf = ws.yf;
    a.c = c;
    a.mlp = pack_mlp(a.use_net ? model : nullptr);
    // the inverse of every grid value the field can hold, where few enough
    const long long ntab = inv_table_size(c);
    if (ntab) {
        const unsigned tg = (unsigned)((ntab + 255) / 256);
        if (g.dtype == PWREL_F32)
            hipLaunchKernelGGL(k_inv_table<float>, dim3(tg), dim3(256), 0, s, c,
                               (long long)c.p_zero, ntab, static_cast<float *>(ws.invtab));
        else
            hipLaunchKernelGGL(k_inv_table<double>, dim3(tg), dim3(256), 0, s, c,
                               (long long)c.p_zero, ntab, static_cast<double *>(ws.invtab));
        a.invtab = ws.invtab;
        a.inv_lo = c.p_zero;
        a.inv_n = ntab;
    }
    const bool mfma = a.use_net && model && model->precision == 1;
    const int HP = mfma ? 0 : hidden_pad(a.use_net ? model : nullptr);
    const int h0 = g.D >= 3 ? 1 : 0, h1 = g.D >= 2 ? 1 : 0;
    const size_t ne = (size_t)(g.bd[0] + h0) * (g.bd[1] + h1) * (g.bd[2] + 1);
    const size_t bv = (size_t)g.bd[0] * g.bd[1] * g.bd[2];
    const size_t lds = ((bv * 2 + 15) & ~size_t(15)) + ne * 4;
    const long long nlines = (long long)g.bd[0] * g.bd[1];
    const unsigned nt = (unsigned)std::min(256LL, std::max(64LL, (nlines + 63) / 64 * 64));
    const bool flow = !a.independent;
    unsigned grid = flow ? (unsigned)std::max(num_cus, 1) : (unsigned)g.nblocks;
    const bool pencils = flow && pencil_mode(g);
    if (!flow && lanes_shape(g.D, g.B) && c.w32) {
        // whole blocks one per lane; the blocks clipped by the high faces one per workgroup
        long long nfull = 1;
        for (int d = 0; d < 3; ++d) {
            a.nf[d] = g.n[d] / g.bd[d];
            nfull *= a.nf[d];
        }
        launch_decode_lanes(g, HP, a, s);
        const long long npart = g.nblocks - nfull;
        if (npart == 0)
            return hipGetLastError();
        a.partial_only = 1;
        grid = (unsigned)npart;
    }
    if (g.dtype == PWREL_F32) {
        if (pencils)
            pencil_by_hidden<float>(HP, a, grid, s);
        else
            by_shape<float>(flow, g.D, g.B, HP, a, grid, nt, lds, s);
    } else {
        if (pencils)
            pencil_by_hidden<double>(HP, a, grid, s);
        else
            by_shape<double>(flow, g.D, g.B, HP, a, grid, nt, lds, s);
    }
    return hipGetLastError();
}

// Grid values of the raw values, before the decoder.
hipError_t launch_raw_grid(const Geom &g, const DevConsts &c, const void *raw,
                           unsigned long long n_raw, Workspace &ws, hipStream_t s)
{
    if (!n_raw)
        return hipSuccess;
    const unsigned grid = (unsigned)std::min<unsigned long long>((n_raw + 255) / 256, 4096);
    if (g.dtype == PWREL_F32)
        hipLaunchKernelGGL(k_raw_grid<float>, dim3(grid), dim3(256), 0, s,
                           static_cast<const float *>(raw), n_raw, c, ws.praw, ws.status);
    else
        hipLaunchKernelGGL(k_raw_grid<double>, dim3(grid), dim3(256), 0, s,
                           static_cast<const double *>(raw), n_raw, c, ws.praw, ws.status);
    return hipGetLastError();
}

// x^ of the coded points from the scratch grid field (halo mode), after the decoder.
hipError_t launch_inverse(const Geom &g, const DevConsts &c, Workspace &ws, void *xh,
                          hipStream_t s)
{
    const unsigned grid = (unsigned)std::min<long long>((g.N + 255) / 256, 8192);
    const bool vec = (reinterpret_cast<uintptr_t>(xh) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(ws.pgrid) & 15) == 0;
    const long long nt = inv_table_size(c);
    if (g.dtype == PWREL_F32 && vec)
        hipLaunchKernelGGL(k_inverse_f32x4, dim3(std::max(1u, grid / 4)), dim3(256), 0, s,
                           ws.pgrid, g.N, c, nt ? static_cast<const float *>(ws.invtab) : nullptr,
                           (long long)c.p_zero, nt, static_cast<float *>(xh));
    else if (g.dtype == PWREL_F32)
        hipLaunchKernelGGL(k_inverse<float>, dim3(grid), dim3(256), 0, s, ws.pgrid, g.N, c,
                           nt ? static_cast<const float *>(ws.invtab) : nullptr,
                           (long long)c.p_zero, nt, static_cast<float *>(xh));
    else
        hipLaunchKernelGGL(k_inverse<double>, dim3(grid), dim3(256), 0, s, ws.pgrid, g.N, c,
                           nt ? static_cast<const double *>(ws.invtab) : nullptr,
                           (long long)c.p_zero, nt, static_cast<double *>(xh));
    return hipGetLastError();
}

// Work order of the halo-mode decoder.  Pencils (bz, by): levels bz + by
// ascending, bz ascending inside a level.  Blocks: levels bz + by + bx
// ascending, (bz, by) ascending inside a level.
void block_order(const Geom &g, std::vector<unsigned> &order)
{
    order.clear();
    if (pencil_mode(g)) {
        order.reserve((size_t)(g.nb[0] * g.nb[1]));
        for (long long lev = 0; lev <= (g.nb[0] - 1) + (g.nb[1] - 1); ++lev)
            for (long long bz = std::max(0LL, lev - (g.nb[1] - 1));
                 bz <= std::min(g.nb[0] - 1, lev); ++bz)
                order.push_back((unsigned)(bz * g.nb[1] + (lev - bz)));
        return;
    }
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
