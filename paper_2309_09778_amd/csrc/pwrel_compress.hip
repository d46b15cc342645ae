// Compression kernels (steps: transform, prediction, quantisation,
// verification, per-block balance-point counts, per-block judge) for gfx950.
//
// FP32 fields take two passes: k_grid_entries computes the grid value and
// bound check of every value once (the hardware log2 / exp2 fast paths with
// certified fallback to FP64) into an entry 2 p (+1 where the check fails),
// then the fused kernel k_compress reads entries.  FP64 fields take the fused
// kernel alone, which then computes grid values and checks itself.
//
// A workgroup of k_compress works on a tile of whole blocks plus the
// one-point halo on the low side of every active axis (the "extended tile").
// Its inputs (entries or values) are copied global -> LDS one tile ahead
// (coalesced rows), so the loads of the next tile are in flight while the
// current one is predicted.  Grid values and check bits go to LDS.  The tile is then
// walked in stream order (block-major, so a wave writes 64 consecutive
// codes), every point predicted independently from its neighbours' grid
// values (the data selection rule that removes the serial dependency), and
// the balance points of each block counted in LDS.  Workgroups are
// persistent; those of XCD x (= workgroup id mod 8) walk a contiguous eighth
// of the tiles so that tiles sharing halo rows meet in the same L2.
#include <type_traits>

#include "pwrel_bf16.h"
#include "pwrel_wavesort.h"

namespace pwrel {

struct CompressArgs {
    // batch: nfields fields (fields[], ordered by tile0; every field of the
    // same dimensionality, dtype, block and tile), ntiles over all of them;
    // else nfields = 0 and the single field below
    const FieldDesc *fields;
    int nfields;
    const void *x;
    const int *pfield;
    long long n[3];
    int bd[3];
    long long nb[3];
    int t[3];
    long long nt[3];
    long long ntiles;
    int use_net, judge, independent;
    int entries;  // grid-field input: 2 p (+1 where the bound check failed) instead of p
    uint16_t *codes;
    uint32_t *counts;
    uint8_t *bflags;
    const DevConsts *consts;
    int *status;
    const long long *qtab;  // q(c) = rint(2^32 log2 c), c = 0 .. points per block (judge)
    MlpW mlp;
};

// Per-block judge (Sec. 4.3: the codes are entropy-coded, so a block keeps the
// network only if its codes have the lower empirical entropy).  J = sum over the
// block's points of q(c), c = the number of the block's points that carry the
// same code, q(c) = rint(2^32 log2 c); n q(n) - J is 2^32 times the entropy in
// bits.  One wave per block.  Blocks of up to 1,024 points of the compiled
// shapes: the wave sorts the block's codes of each predictor (a bitonic network
// in registers and lane exchanges; for 8^3 blocks with every stage inside a
// lane, the register layouts exchanged through LDS) and reads the
// multiplicities off the runs.
// Other blocks: codes within a window of errors are counted in a histogram
// (kJudgeWin bins: bin 0 = code 0, the balance point; bin e + kJudgeHalf for
// |e| < kJudgeHalf), the others in a per-block hash table of each predictor
// (open addressing, as many slots as the block has points rounded up to a
// power of two, so it never fills).  Either way J = the sum over the distinct
// codes of c q(c).
constexpr int kJudgeHalf = 256;
constexpr int kJudgeWin = 2 * kJudgeHalf;  // bins per block

__host__ __device__ constexpr int judge_slots(int bv)
{
    int h = 1;
    while (h < bv)
        h <<= 1;
    return h;
}

// the judge sorts in registers: compiled shape with at most 1,024 points a block
__host__ __device__ constexpr bool judge_sorts(bool known, int bv) { return known && bv <= 1024; }
__host__ __device__ constexpr int judge_epl(int bv) { return bv <= 64 ? 1 : judge_slots(bv) / 64; }

// count one more of `code` (non-zero, outside the window) in a table of hc
// slots: entry = code << 16 | count, 0 = empty
__device__ __forceinline__ void judge_hash_add(unsigned *tab, int hc, unsigned code)
{
    unsigned h = (code * 2654435761u) >> 16;
    for (int probe = 0; probe < hc; ++probe) {
        h &= (unsigned)(hc - 1);
        const unsigned old = atomicCAS(&tab[h], 0u, (code << 16) | 1u);
        if (old == 0u)
            return;
        if ((old >> 16) == code) {
            atomicAdd(&tab[h], 1u);
            return;
        }
        ++h;
    }
}

// The judge's scores of one block held by a wave: each 32-bit key carries the
// network's code (low half) and Lorenzo's (high half) of one point, EPL keys
// a lane in any order; nsent of them are stand-ins (0xFFFF in both halves)
// for positions outside the field.  Returns, for each half, the sum over its
// distinct codes of c q(c), c = the code's multiplicity.  Both halves are
// sorted at once (wave_sort_lm); stand-ins sort last and are taken off the
// last run of each half.
template <int EPL>
__device__ __forceinline__ void wave_multiset_score(unsigned (&a)[EPL], unsigned nsent,
                                                    const long long *qtab,
                                                    unsigned long long &s0,
                                                    unsigned long long &s1)
{
    wave_sort_lm<EPL>(a);
    wave_runs_lm<EPL>(a, nsent, qtab, s0, s1);
}

__device__ __forceinline__ int judge_bin(unsigned code)
{
    if (code == 0)
        return 0;
    const int e = (int)code - kR;
    return (e > -kJudgeHalf && e < kJudgeHalf) ? e + kJudgeHalf : -1;
}

__device__ __forceinline__ unsigned short code32(int e, bool ok)
{
    return (ok && e > -kR && e < kR) ? (unsigned short)(e + kR) : (unsigned short)0;
}

// Prediction errors e = prediction - p in 32-bit arithmetic, for fields whose
// grid values span less than 2^27 (DevConsts::w32): then every neighbour
// difference and every error below fits.  Same values as the 64-bit path.
//   Lorenzo: with at least one axis available the coefficients of the
//   available neighbours sum to 1, so e = sum c_o (n_o - p); with none, e = -p.
template <int D>
__device__ __forceinline__ int lorenzo_err32(const int (&nv)[8], int amask)
{
    if (amask == 0)
        return -nv[0];
    int s = 0;
#pragma unroll
    for (int o = 1; o < (1 << D); ++o)
        if ((o & ~amask) == 0)
            s += lorenzo_sign(o) * (nv[o] - nv[0]);
    return s;
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

// network error in 32 bits: e = (n_1 - p) + rint(y), |rint(y)| <= 2^30
__device__ __forceinline__ int net_err32(float y, const int (&nv)[8])
{
    if (y > 0x1p30f)
        y = 0x1p30f;
    if (!(y >= -0x1p30f))
        y = -0x1p30f;
    return (nv[1] - nv[0]) + (int)__builtin_rintf(y);
}

// Workgroup barrier that orders LDS accesses only: global stores stay in
// flight across it (no thread reads global memory that another thread of the
// workgroup wrote in the same launch; the staged tile copies are waited for
// explicitly).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// s_waitcnt vmcnt(0): this wave's outstanding global loads and stores are done
__device__ __forceinline__ void wait_vmem()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt = 0, expcnt and lgkmcnt not waited on
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Occupancy bound (measured at 512^3): six waves per SIMD for the FP32 and
// Lorenzo variants, four for the BF16 one; the registers the bound takes away
// cost a few spills, far less than the latency the extra waves hide.
// W32 (compiled tiles of grid entries only): the variant for fields whose grid
// values span less than 2^27, with one branch-free prediction loop; a launch
// of the other variant pairs with it and each returns at once on the other's
// fields, so neither carries the other's code.
template <typename T, int D, int BB, int HP, bool FROM_P, int PREC, bool BATCH, int TV = 0,
          bool W32 = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == 1 ? 3 : 6)))
k_compress(CompressArgs a)
{
    static_assert(FROM_P || !std::is_same<T, float>::value,
                  "FP32 values are read as entries (k_grid_entries)");
    using S = TileOf<D, BB, TV>;
    constexpr bool CT = S::known;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NT = 256;
    constexpr bool SPLIT = CT && FROM_P && !BATCH;  // launched as a W32 / generic pair
    if constexpr (SPLIT) {
        // the pair's other kernel takes this field: return before any set-up
        // (uniform: one field, every thread reads the same constant)
        if ((a.consts->w32 != 0) != W32)
            return;
    }
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

    // LDS: [judge: per-block scores] [block stream starts] [block extents]
    // [grid tile] [balance counts] [judge: per-block histograms, both codes of
    // every point, out-of-window list counts and lists] [bound bits]
    // (the 64-bit arrays first for alignment)
    unsigned long long *jsum = reinterpret_cast<unsigned long long *>(smem);
    long long *bst = reinterpret_cast<long long *>(jsum + (a.judge ? 2 * nbt : 0));
    unsigned *bext = reinterpret_cast<unsigned *>(bst + nbt);
    int *ptile = reinterpret_cast<int *>(bext + nbt);
    unsigned int *cnt = reinterpret_cast<unsigned int *>(ptile + ne);
    using V = typename std::conditional<FROM_P, int, T>::type;
    unsigned int *jh = cnt + nbt;  // [nbt][kJudgeWin]: network count | Lorenzo count << 16
    // judge only: both codes of every tile point (network | Lorenzo << 16)
    // the judge's path (sort in registers, or window + hash tables)
    constexpr int BVc = BB * (D >= 2 ? BB : 1) * (D >= 3 ? BB : 1);  // 0: runtime shape
    constexpr bool JS = judge_sorts(CT, BVc);
    constexpr int JEPL = JS ? judge_epl(BVc) : 1;
    // 8^3 blocks: the sort whose stages all run inside a lane (layouts moved
    // through the grid tile's LDS once the tile is predicted)
    constexpr bool JL = JS && D == 3 && BB == 8;
    if constexpr (JL) {
        static_assert(JEPL == 8, "512 points a block");
        static_assert((S::T0 + 1) * (S::T1 + 1) * (S::T2 + 1) >= (NT / 64) * kSortLdsWords,
                      "the grid tile holds every wave's sort words");
        static_assert((S::T0 / 8) * (S::T1 / 8) * (S::T2 / 8) % 4 == 0,
                      "the grid tile starts 16-byte aligned (28 bytes a block before it)");
    }
    const int HC = judge_slots(BV);
    const bool jwin = a.judge && !JS;
    unsigned *jb = jh + (jwin ? nbt * kJudgeWin : 0);
    // judge: [nbt][2] code-0 counts of each predictor; window path: [nbt][2][HC]
    // hash tables of the out-of-window codes
    unsigned *jz = jb + (a.judge ? ntp : 0);
    unsigned *jht = jz + (a.judge ? 2 * nbt : 0);
    unsigned char *okb = reinterpret_cast<unsigned char *>(jht + (jwin ? 2 * nbt * HC : 0));

    __shared__ int s_status;
    __shared__ float4 wl[kWlds];
    // the judge's q-table in LDS (sorted path, blocks of up to 512 points);
    // for 8^3 blocks it holds c q(c), the term a run of c equal codes adds
    constexpr bool JQ = JS && BVc <= 512;
    __shared__ long long sq[JQ ? BVc + 1 : 1];
    if constexpr (JQ) {
        if (a.judge)
            for (int i = tid; i <= BVc; i += NT)
                sq[i] = JL ? (long long)((unsigned long long)i * (unsigned long long)a.qtab[i])
                           : a.qtab[i];
    }
    const long long *qt = JQ ? sq : a.qtab;
    stage_weights<HP>(wl, a.mlp);
    const float b2 = a.mlp.b2, alpha = a.mlp.alpha;
    NetBf16 net16;
    if constexpr (PREC == 1)
        net16 = make_net_bf16(a.mlp, (1 << D) - 2);
    for (int i = tid; i < nbt; i += NT)
        cnt[i] = 0u;
    if (a.judge) {
        if (jwin) {
            for (int i = tid; i < nbt * kJudgeWin; i += NT)
                jh[i] = 0u;
            for (int i = tid; i < 2 * nbt * HC; i += NT)
                jht[i] = 0u;
        }
        for (int i = tid; i < 2 * nbt; i += NT)
            jsum[i] = 0ULL;
    }
    if (tid == 0)
        s_status = BATCH ? kOk : *a.status;
    __syncthreads();
    if (s_status != kOk)  // uniform: every thread reads the same shared value
        return;
    // the field of a tile (batch: binary search of the fields' first tiles)
    struct Fld {
        const V *src;
        long long n[3], nb[3], nt[3], tile0;
        uint16_t *codes;
        uint32_t *counts;
        uint8_t *bflags;
        const DevConsts *consts;
        int *status;
    };
    auto field_of = [&](long long t) {
        Fld F;
        if constexpr (!BATCH) {
            F.src = FROM_P ? reinterpret_cast<const V *>(a.pfield)
                           : reinterpret_cast<const V *>(a.x);
            for (int d = 0; d < 3; ++d) {
                F.n[d] = a.n[d];
                F.nb[d] = a.nb[d];
                F.nt[d] = a.nt[d];
            }
            F.tile0 = 0;
            F.codes = a.codes;
            F.counts = a.counts;
            F.bflags = a.bflags;
            F.consts = a.consts;
            F.status = a.status;
        } else {
            int lo = 0, hi = a.nfields - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.fields[mid].tile0 <= t)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            // uniform across the workgroup: the field's words load as scalars
            const FieldDesc &d = a.fields[__builtin_amdgcn_readfirstlane(lo)];
            F.src = FROM_P ? reinterpret_cast<const V *>(d.pfield) : reinterpret_cast<const V *>(d.x);
            for (int k = 0; k < 3; ++k) {
                F.n[k] = d.n[k];
                F.nb[k] = d.nb[k];
                F.nt[k] = d.nt[k];
            }
            F.tile0 = d.tile0;
            F.codes = d.codes;
            F.counts = d.counts;
            F.bflags = d.bflags;
            F.consts = d.consts;
            F.status = d.status;
        }
        return F;
    };
    Fld F = field_of(0);
    DevConsts c = *F.consts;
    long long n0 = F.n[0], n1 = F.n[1], n2 = F.n[2];
    bool w32 = c.w32 != 0;

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

    // grid value (and bound check) of one point from its value
    const V *src = F.src;
    auto point = [&](V v, bool verify, int &p, unsigned char &ok) {
        if constexpr (FROM_P) {
            const int e = (int)v;
            p = a.entries ? (e >> 1) : e;
            ok = (a.entries && (e & 1)) ? 0 : 1;
        } else {
            // FP64 values (FP32 fields arrive as entries from k_grid_entries)
            const double xv = (double)v;
            p = grid_value(xv, c, err);
            if (verify)
                ok = within_bound(xv, grid_inverse<T>(p, c), c.eps) ? 1 : 0;
        }
    };

    // The extended tile is E0 x E1 rows of E2 entries; entry (e0, e1, e2) is
    // the point (z0 + e0 - h0, y0 + e1 - h1, x0 + e2 - h2).  Per tile: its
    // origin, the linear index of entry (0, 0, 0), and the entry ranges that
    // lie inside the field.
    struct TileRef {
        long long z0, y0, x0, base, n1, n2;
        int lo0, hi0, lo1, hi1, lo2, hi2;
    };
    // tile t (of the launch) of field G
    auto tile_ref = [&](const Fld &G, long long t) {
        TileRef r;
        const long long lt = t - G.tile0;
        r.z0 = lt / (G.nt[1] * G.nt[2]) * T0;
        r.y0 = (lt / G.nt[2]) % G.nt[1] * T1;
        r.x0 = lt % G.nt[2] * T2;
        r.lo0 = (h0 && r.z0 == 0) ? 1 : 0;
        r.lo1 = (h1 && r.y0 == 0) ? 1 : 0;
        r.lo2 = r.x0 == 0 ? 1 : 0;
        r.hi0 = (int)std::min((long long)E0, G.n[0] - r.z0 + h0);
        r.hi1 = (int)std::min((long long)E1, G.n[1] - r.y0 + h1);
        r.hi2 = (int)std::min((long long)E2, G.n[2] - r.x0 + h2);
        r.n1 = G.n[1];
        r.n2 = G.n[2];
        r.base = ((r.z0 - h0) * r.n1 + (r.y0 - h1)) * r.n2 + (r.x0 - h2);
        return r;
    };
    auto row_base = [&](const TileRef &r, int row) {
        const int e0 = row / E1, e1 = row - (row / E1) * E1;
        return r.base + ((long long)e0 * r.n1 + e1) * r.n2;
    };
    auto row_in = [&](const TileRef &r, int row) {
        const int e0 = row / E1, e1 = row - (row / E1) * E1;
        return e0 >= r.lo0 && e0 < r.hi0 && e1 >= r.lo1 && e1 < r.hi1;
    };
    const int nrows = E0 * E1;

    // Compile-time tiles of FP32 fields or grid input: the next tile's values
    // are copied global -> LDS (no registers held) while the current tile is
    // predicted, one row of the extended tile per wave instruction.  xs is an
    // LDS object of its own, so no other LDS access can alias the copies.
    constexpr bool PIPE = CT && (FROM_P || std::is_same<T, float>::value);
    constexpr int NEX = CT ? (S::T0 + h0) * (S::T1 + h1) * (S::T2 + h2) : 1;
    __shared__ unsigned xs[PIPE ? NEX : 1];
    // the wave index, provably uniform: the staging loop's row arithmetic is scalar
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    auto stage = [&](long long t) {
        const Fld G = BATCH ? field_of(t) : F;
        const unsigned *src32 = reinterpret_cast<const unsigned *>(G.src);
        const TileRef r = tile_ref(G, t);
        for (int row = wave; row < nrows; row += NT / 64) {
            if (!row_in(r, row))
                continue;  // uniform across the wave
            const long long rb = row_base(r, row);
            for (int c0 = 0; c0 < E2; c0 += 64) {
                const int e2 = c0 + lane;
                if (e2 >= r.lo2 && e2 < r.hi2)
                    __builtin_amdgcn_global_load_lds(src32 + rb + e2, xs + row * E2 + c0, 4, 0,
                                                     0);
            }
        }
    };

    // prediction units: a segment of SEG consecutive points of one block row
    const int SEG = CT ? (BB < 8 ? BB : 8) : (bd2 % 8 == 0 ? 8 : (bd2 % 4 == 0 ? 4 : 1));
    const int nseg = bd2 / SEG;
    const int nunits = nbt * bd0 * bd1 * nseg;
    // transform items: a chunk of CL entries of one extended-tile row
    constexpr int CL = 11;
    const int nch = (E2 + CL - 1) / CL;

    long long t = (long long)xcd * chunk + slot;
    if constexpr (PIPE) {
        if (t < tend)
            stage(t);
    }

    for (; t < tend; t += nslot) {
        if (BATCH && !(t >= F.tile0 && t < F.tile0 + F.nt[0] * F.nt[1] * F.nt[2])) {
            // a tile of another field: its geometry, outputs and constants
            if (err != kOk) {
                set_status(F.status, err);
                err = kOk;
            }
            F = field_of(t);
            c = *F.consts;
            n0 = F.n[0];
            n1 = F.n[1];
            n2 = F.n[2];
            w32 = c.w32 != 0;
            src = F.src;
        }
        const TileRef r = tile_ref(F, t);
        const long long g0z = r.z0, g0y = r.y0, g0x = r.x0;
        if constexpr (PIPE)
            wait_vmem();  // this wave's copies have landed
        lds_barrier();    // ... and every other wave's

        // --- grid values of the extended tile; bound check of the tile points --
        for (int it = tid; it < nrows * nch; it += NT) {
            const int row = it / nch, ch = it - (it / nch) * nch;
            const int e0 = row / E1, e1 = row - (row / E1) * E1;
            const bool rin = row_in(r, row);
            const bool rhalo = e0 < h0 || e1 < h1;
            const long long rb = row_base(r, row);
            const int okrow = ((e0 - h0) * T1 + (e1 - h1)) * T2 - h2;
            const int cend = std::min(E2, ch * CL + CL);
            for (int e2 = ch * CL; e2 < cend; ++e2) {
                const bool in = rin && e2 >= r.lo2 && e2 < r.hi2;
                const bool halo = rhalo || e2 < h2;
                int p = 0;
                unsigned char ok = 0;
                if (in) {
                    V v;
                    if constexpr (PIPE)
                        __builtin_memcpy(&v, &xs[row * E2 + e2], 4);
                    else
                        v = src[rb + e2];
                    point(v, !halo, p, ok);
                }
                ptile[row * E2 + e2] = p;
                if (!halo)
                    okb[okrow + e2] = ok;
            }
        }
        // block stream starts and extents of the tile's blocks
        const long long bz0 = g0z / bd0, by0 = g0y / bd1, bx0 = g0x / bd2;
        for (int bt = tid; bt < nbt; bt += NT) {
            const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
            const long long bz = bz0 + btz, by = by0 + bty, bx = bx0 + btx;
            if (bz < F.nb[0] && by < F.nb[1] && bx < F.nb[2]) {
                const BlockGeo bg = block_geo3(bz, by, bx, F.n, bd0, bd1, bd2);
                bst[bt] = bg.start;
                bext[bt] = (unsigned)bg.ex | ((unsigned)bg.ey << 16);
            }
        }
        lds_barrier();

        // the next tile's copies are in flight during this tile's prediction
        // (issued after the barrier: a barrier waits for outstanding copies)
        if constexpr (PIPE) {
            if (t + nslot < tend)
                stage(t + nslot);
        }

        // --- predict, quantize, count --------------------------------------
        // Unit u = ((bt * bd0 + lz) * bd1 + ly) * nseg + seg walks its segment
        // along x; units in stream order, so a wave writes consecutive codes.
        // The x - 1 neighbours come from the previous step of the same unit.
        // Every lane of a wave runs the same number of steps (the matrix-core
        // network works on whole waves).
        const int limz = (int)std::min((long long)T0, n0 - g0z);
        const int limy = (int)std::min((long long)T1, n1 - g0y);
        const int limx = (int)std::min((long long)T2, n2 - g0x);
        const int first = (g0x == 0 ? 1 : 0) | (D >= 2 && g0y == 0 ? 2 : 0) |
                          (D >= 3 && g0z == 0 ? 4 : 0);  // axes that start at the field edge
        const int edge = a.independent ? 7 : first;
        constexpr int NO = (1 << D) - 1;
        const int DZ = E1 * E2, DY = E2;
        if constexpr (W32) {
            // Branch-free loop (grid values spanning less than 2^27): a missing
            // axis zeroes its neighbours (the Lorenzo predictor counts them as
            // zero; e = sum of signed neighbours - p wraps exactly in 32 bits),
            // points outside the field are computed and dropped, codes leave
            // four at a time where a group lies in the field.
            static_assert(CT && FROM_P, "the 32-bit loop reads compiled tiles of entries");
            constexpr int S8 = BB < 8 ? BB : 8;
            const bool vec = (reinterpret_cast<uintptr_t>(F.codes) & 7) == 0;
#pragma unroll 1
            for (int u0 = 0; u0 < nunits; u0 += NT) {
                const int u = u0 + tid;
                const int uu = u < nunits ? u : 0;
                const int seg = uu % nseg, row = uu / nseg;
                const int ly = row % bd1, lz = (row / bd1) % bd0, bt = row / (bd1 * bd0);
                const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
                const int cz = btz * bd0 + lz, cy = bty * bd1 + ly, cx0 = btx * bd2 + seg * S8;
                const bool urow = u < nunits && cz < limz && cy < limy;
                const int pz = a.independent ? lz : cz, py = a.independent ? ly : cy;
                const int my = (D >= 2 && (py != 0 || !(edge & 2))) ? -1 : 0;
                const int mz = (D >= 3 && (pz != 0 || !(edge & 4))) ? -1 : 0;
                const bool yz_full = (D < 2 || my != 0) && (D < 3 || mz != 0);
                const int px0 = a.independent ? seg * S8 : cx0;
                const bool x0 = px0 != 0 || !(edge & 1);  // x - 1 of the first point available
                const int nin = urow ? limx - cx0 : 0;    // points of the segment in the field: min(nin, S8)
                const int eb = ((cz + h0) * E1 + (cy + h1)) * E2 + (cx0 + h2);
                const int ex = (int)(bext[bt] & 0xffffu), ey = (int)(bext[bt] >> 16);
                const long long pos0 = bst[bt] + (long long)((lz * ey + ly) * ex + seg * S8);
                const int okr = (cz * T1 + cy) * T2 + cx0;
                uint16_t *dst = F.codes + pos0;
                int q0 = ptile[eb - 1];
                int q2 = D >= 2 ? ptile[eb - 1 - DY] : 0;
                int q4 = D >= 3 ? ptile[eb - 1 - DZ] : 0;
                int q6 = D >= 3 ? ptile[eb - 1 - DZ - DY] : 0;
                unsigned long long cacc = 0ULL;
                unsigned nz = 0;
#pragma unroll 1
                for (int i = 0; i < S8; ++i) {
                    const bool inside = i < nin;
                    const int p = ptile[eb + i];
                    const int c2 = D >= 2 ? ptile[eb + i - DY] : 0;
                    const int c4 = D >= 3 ? ptile[eb + i - DZ] : 0;
                    const int c6 = D >= 3 ? ptile[eb + i - DZ - DY] : 0;
                    const bool xa = i > 0 || x0;
                    const int mx = xa ? -1 : 0;
                    const int n1 = q0 & mx;
                    int el;
                    if constexpr (D == 1) {
                        el = n1 - p;
                    } else if constexpr (D == 2) {
                        el = (n1 + (c2 & my)) - ((q2 & my & mx) + p);
                    } else {
                        const int n2 = c2 & my, n3 = q2 & my & mx;
                        const int n4 = c4 & mz, n5 = q4 & mz & mx;
                        const int n6 = c6 & mz & my, n7 = q6 & mz & my & mx;
                        el = ((n1 + n2) + (n4 + n7)) - ((n3 + n5) + (n6 + p));
                    }
                    const bool use = a.use_net != 0 && inside && xa && yz_full;
                    const bool okp = okb[okr + i] != 0;
                    int e = el;
                    if constexpr (PREC == 1) {
                        constexpr int K = (1 << D) - 2;
                        const int nvr[6] = {c2, q2, c4, q4, c6, q6};
                        float uin[6];
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            uin[k] = (k < K && use)
                                         ? (float)(int)((unsigned)nvr[k] - (unsigned)q0)
                                         : 0.0f;
                        const float y = net_bf16(net16, uin);  // every lane takes part
                        if (use) {
                            const int nv2[8] = {p, q0, 0, 0, 0, 0, 0, 0};
                            e = net_err32(y, nv2);
                        }
                    } else {
                        if (use) {
                            const int nv[8] = {p, q0, c2, q2, c4, q4, c6, q6};
                            e = net_err32(net_f32<D, HP>(nv, WeightsLds{wl}, b2, alpha), nv);
                        }
                    }
                    const unsigned code = code32(e, okp);
                    if (inside) {
                        nz += code == 0u ? 1u : 0u;
                        if (a.judge)
                            jb[okr + i] = code | ((unsigned)code32(el, okp) << 16);
                    }
                    cacc |= (unsigned long long)code << (16 * (i & 3));
                    if ((i & 3) == 3 || i == S8 - 1) {  // uniform: every lane is at step i
                        const int i0 = i & ~3;
                        if (vec && i0 + 3 < nin && ((pos0 + i0) & 3) == 0) {
                            *reinterpret_cast<unsigned long long *>(dst + i0) = cacc;
                        } else {
                            for (int k = 0; k <= (i & 3); ++k)
                                if (i0 + k < nin)
                                    dst[i0 + k] = (uint16_t)(cacc >> (16 * k));
                        }
                        cacc = 0ULL;
                    }
                    q0 = p;
                    q2 = c2;
                    q4 = c4;
                    q6 = c6;
                }
                if (!a.judge && nz)
                    atomicAdd(&cnt[bt], nz);
            }
        } else {
#pragma unroll 1
        for (int u0 = 0; u0 < nunits; u0 += NT) {
            const int u = u0 + tid;
            const int uu = u < nunits ? u : 0;
            const int seg = uu % nseg, row = uu / nseg;
            const int ly = row % bd1, lz = (row / bd1) % bd0, bt = row / (bd1 * bd0);
            const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
            const int cz = btz * bd0 + lz, cy = bty * bd1 + ly, cx0 = btx * bd2 + seg * SEG;
            const bool urow = u < nunits && cz < limz && cy < limy;
            // axes y, z available for this row (the x axis is decided per point)
            const int pz = a.independent ? lz : cz, py = a.independent ? ly : cy;
            const int amask_zy = (D >= 2 && (py != 0 || !(edge & 2)) ? 2 : 0) |
                                 (D >= 3 && (pz != 0 || !(edge & 4)) ? 4 : 0);
            const int eb = ((cz + h0) * E1 + (cy + h1)) * E2 + (cx0 + h2);  // entry of point 0
            const int ex = (int)(bext[bt] & 0xffffu), ey = (int)(bext[bt] >> 16);
            const long long pos0 = bst[bt] + (long long)((lz * ey + ly) * ex + seg * SEG);
            const int okr = (cz * T1 + cy) * T2 + cx0;
            // previous column (x - 1): own row, row y - 1, plane z - 1, both
            int q0 = 0, q2 = 0, q4 = 0, q6 = 0;
            if (urow) {
                q0 = ptile[eb - 1];
                if (D >= 2)
                    q2 = ptile[eb - 1 - DY];
                if (D >= 3) {
                    q4 = ptile[eb - 1 - DZ];
                    q6 = ptile[eb - 1 - DZ - DY];
                }
            }
            unsigned nzero = 0;
            for (int i = 0; i < SEG; ++i) {
                const int cx = cx0 + i;
                const bool inside = urow && cx < limx;
                int nv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                int amask = 0;
                int c0 = q0, c2 = q2, c4 = q4, c6 = q6;
                if (inside) {
                    const int ei = eb + i;
                    c0 = ptile[ei];
                    if (D >= 2)
                        c2 = ptile[ei - DY];
                    if (D >= 3) {
                        c4 = ptile[ei - DZ];
                        c6 = ptile[ei - DZ - DY];
                    }
                    nv[0] = c0;
                    nv[1] = q0;
                    nv[2] = c2;
                    nv[3] = q2;
                    nv[4] = c4;
                    nv[5] = q4;
                    nv[6] = c6;
                    nv[7] = q6;
                    const int px = a.independent ? seg * SEG + i : cx;
                    amask = amask_zy | ((px != 0 || !(edge & 1)) ? 1 : 0);
                }
                q0 = c0;
                q2 = c2;
                q4 = c4;
                q6 = c6;
                const bool full = amask == NO;
                const bool ok = inside && okb[okr + i] != 0;
                unsigned short code, lcode = 0;
                if constexpr (PREC == 1) {
                    // the network on the matrix cores (every lane takes part), Lorenzo
                    // where it does not apply; the same predictions as predict_bf16
                    constexpr int K = (1 << D) - 2;
                    const bool use = a.use_net != 0 && inside && full;
                    float u[6];
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        u[k] = (k < K && use)
                                   ? (float)(int)((unsigned)nv[k + 2] - (unsigned)nv[1])
                                   : 0.0f;
                    const float y = net_bf16(net16, u);
                    if (w32) {
                        const int el = lorenzo_err32<D>(nv, amask);
                        code = code32(use ? net_err32(y, nv) : el, ok);
                        lcode = code32(el, ok);
                    } else {
                        float yc = y;
                        if (yc > 0x1p30f)
                            yc = 0x1p30f;
                        if (!(yc >= -0x1p30f))
                            yc = -0x1p30f;
                        const long long pl = lorenzo_pred<D>(nv, amask);
                        code = make_code(use ? (long long)nv[1] + (long long)__builtin_rintf(yc)
                                             : pl,
                                         nv[0], ok);
                        lcode = make_code(pl, nv[0], ok);
                    }
                } else {
                    if (w32) {
                        const int e =
                            (a.use_net && full)
                                ? net_err32(net_f32<D, HP>(nv, WeightsLds{wl}, b2, alpha), nv)
                                : lorenzo_err32<D>(nv, amask);
                        code = code32(e, ok);
                    } else {
                        code = make_code(inside ? predict<D, HP>(nv, amask, a.use_net != 0,
                                                                 WeightsLds{wl}, b2, alpha)
                                                : 0,
                                         nv[0], ok);
                    }
                }
                if (!inside)
                    continue;
                F.codes[pos0 + i] = code;
                nzero += code == 0 ? 1u : 0u;
                if (a.judge) {
                    if constexpr (PREC != 1)
                        lcode = w32 ? code32(lorenzo_err32<D>(nv, amask), ok)
                                    : make_code(lorenzo_pred<D>(nv, amask), nv[0], ok);
                    jb[okr + i] = (unsigned)code | ((unsigned)lcode << 16);
                }
            }
            if (!a.judge && nzero)
                atomicAdd(&cnt[bt], nzero);
        }
        }
        lds_barrier();

        if (a.judge) {
            // --- per-block judge: keep the network iff the entropy of its codes
            //     is strictly below Lorenzo's (fixed-point scores), one wave per
            //     block (LDS atomics outside the prediction loop, where no
            //     memory operation is outstanding) ---
            const int lane = tid & 63;
            for (int bt = tid >> 6; bt < nbt; bt += NT / 64) {
                const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
                unsigned long long s0 = 0ULL, s1 = 0ULL;
                unsigned z0 = 0, z1 = 0;
                if constexpr (JL) {
                    // element k + 8 lane = point (lane >> 3, lane & 7, k) of the
                    // block; the sort's LDS is the wave's share of the grid
                    // tile, which nothing reads again before the next tile
                    const int cz = btz * 8 + (lane >> 3), cy = bty * 8 + (lane & 7);
                    const int cx0 = btx * 8;
                    const bool rin = cz < limz && cy < limy;
                    const unsigned *src = jb + (cz * T1 + cy) * T2 + cx0;
                    unsigned kv[8];
                    unsigned nsent = 0;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const bool pt = rin && cx0 + k < limx;
                        const unsigned v = pt ? src[k] : 0xFFFFFFFFu;
                        kv[k] = v;
                        nsent += (unsigned)__popcll(__ballot(!pt));
                        z0 += (unsigned)__popcll(__ballot(pt && (v & 0xffffu) == 0u));
                        z1 += (unsigned)__popcll(__ballot(pt && (v >> 16) == 0u));
                    }
                    unsigned *scr = reinterpret_cast<unsigned *>(ptile) +
                                    __builtin_amdgcn_readfirstlane(tid >> 6) * kSortLdsWords;
                    wave_sort_lds8(kv, static_cast<unsigned *>(__builtin_assume_aligned(scr, 16)));
                    wave_runs_lm<8, true>(kv, nsent, qt, s0, s1);
                } else if constexpr (JS) {
                    unsigned kv[JEPL];
                    unsigned nsent = 0;
#pragma unroll
                    for (int k = 0; k < JEPL; ++k) {
                        const int li = k * 64 + lane;
                        const int lx = li % bd2, ly = (li / bd2) % bd1, lz = li / (bd1 * bd2);
                        const int cz = btz * bd0 + lz, cy = bty * bd1 + ly, cx = btx * bd2 + lx;
                        const bool pt = li < BV && cz < limz && cy < limy && cx < limx;
                        const unsigned v = pt ? jb[(cz * T1 + cy) * T2 + cx] : 0xFFFFFFFFu;
                        kv[k] = v;
                        nsent += (unsigned)__popcll(__ballot(!pt));
                        z0 += (unsigned)__popcll(__ballot(pt && (v & 0xffffu) == 0u));
                        z1 += (unsigned)__popcll(__ballot(pt && (v >> 16) == 0u));
                    }
                    wave_multiset_score<JEPL>(kv, nsent, qt, s0, s1);
                } else {
                    unsigned *hb = jh + bt * kJudgeWin;
                    unsigned *t0 = jht + (2 * bt) * HC, *t1 = t0 + HC;
                    for (int q0 = 0; q0 < BV; q0 += 64) {
                        const int li = q0 + lane;
                        const int lx = li % bd2, ly = (li / bd2) % bd1, lz = li / (bd1 * bd2);
                        const int cz = btz * bd0 + lz, cy = bty * bd1 + ly, cx = btx * bd2 + lx;
                        const bool pt = li < BV && cz < limz && cy < limy && cx < limx;
                        const unsigned v = pt ? jb[(cz * T1 + cy) * T2 + cx] : 0u;
                        const unsigned c0 = v & 0xffffu, c1 = v >> 16;
                        const int b0 = judge_bin(c0), b1 = judge_bin(c1);
                        if (pt) {
                            if (b0 >= 0)
                                atomicAdd(&hb[b0], 1u);
                            else
                                judge_hash_add(t0, HC, c0);
                            if (b1 >= 0)
                                atomicAdd(&hb[b1], 1u << 16);
                            else
                                judge_hash_add(t1, HC, c1);
                        }
                        z0 += (unsigned)__popcll(__ballot(pt && c0 == 0u));
                        z1 += (unsigned)__popcll(__ballot(pt && c1 == 0u));
                    }
                    // this wave's LDS atomics above complete before its reads below
                    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
                    for (int k = lane; k < kJudgeWin; k += 64) {
                        const unsigned w = hb[k];
                        const unsigned cn = w & 0xffffu, cl = w >> 16;
                        if (cn)
                            s0 += (unsigned long long)cn * (unsigned long long)a.qtab[cn];
                        if (cl)
                            s1 += (unsigned long long)cl * (unsigned long long)a.qtab[cl];
                        hb[k] = 0u;  // cleared for the next tile
                    }
                    for (int k = lane; k < HC; k += 64) {
                        const unsigned cn = t0[k] & 0xffffu, cl = t1[k] & 0xffffu;
                        if (cn)
                            s0 += (unsigned long long)cn * (unsigned long long)a.qtab[cn];
                        if (cl)
                            s1 += (unsigned long long)cl * (unsigned long long)a.qtab[cl];
                        t0[k] = 0u;
                        t1[k] = 0u;
                    }
#pragma unroll
                    for (int d = 32; d > 0; d >>= 1) {
                        s0 += (unsigned long long)__shfl_xor((long long)s0, d, 64);
                        s1 += (unsigned long long)__shfl_xor((long long)s1, d, 64);
                    }
                }
                if (lane == 0) {
                    jsum[2 * bt] = s0;
                    jsum[2 * bt + 1] = s1;
                    jz[2 * bt] = z0;
                    jz[2 * bt + 1] = z1;
                }
            }
            lds_barrier();
            // blocks where Lorenzo wins: each thread overwrites the network codes
            // it stored in the prediction loop (the same units, so its earlier
            // stores to these addresses are ordered before these) with the
            // Lorenzo codes noted there
            for (int u0 = 0; u0 < nunits; u0 += NT) {
                const int u = u0 + tid;
                if (u >= nunits)
                    break;
                const int seg = u % nseg, row = u / nseg;
                const int ly = row % bd1, lz = (row / bd1) % bd0, bt = row / (bd1 * bd0);
                if (jsum[2 * bt] > jsum[2 * bt + 1])
                    continue;
                const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
                const int cz = btz * bd0 + lz, cy = bty * bd1 + ly, cx0 = btx * bd2 + seg * SEG;
                if (!(cz < limz && cy < limy))
                    continue;
                const int ex = (int)(bext[bt] & 0xffffu), ey = (int)(bext[bt] >> 16);
                const long long pos0 = bst[bt] + (long long)((lz * ey + ly) * ex + seg * SEG);
                const int okr = (cz * T1 + cy) * T2 + cx0;
                for (int i = 0; i < SEG; ++i)
                    if (cx0 + i < limx)
                        F.codes[pos0 + i] = (uint16_t)(jb[okr + i] >> 16);
            }
            for (int bt = tid; bt < nbt; bt += NT) {
                const bool use_n = jsum[2 * bt] > jsum[2 * bt + 1];
                cnt[bt] = use_n ? jz[2 * bt] : jz[2 * bt + 1];  // balance points of the winner
            }
            lds_barrier();
        }

        // --- per-block balance-point counts ------------------------------------
        for (int bt = tid; bt < nbt; bt += NT) {
            const int btx = bt % nbt2, bty = (bt / nbt2) % nbt1, btz = bt / (nbt1 * nbt2);
            const long long bz = bz0 + btz, by = by0 + bty, bx = bx0 + btx;
            if (bz < F.nb[0] && by < F.nb[1] && bx < F.nb[2]) {
                const long long b = (bz * F.nb[1] + by) * F.nb[2] + bx;
                F.counts[b] = cnt[bt];
                if (F.bflags)
                    F.bflags[b] = a.judge ? (jsum[2 * bt] > jsum[2 * bt + 1] ? 1 : 0)
                                          : (a.use_net ? 1 : 0);
            }
            cnt[bt] = 0u;
            if (a.judge)
                jsum[2 * bt] = jsum[2 * bt + 1] = 0ULL;
        }
        // the next tile overwrites the LDS arrays only after this barrier
        lds_barrier();
    }
    set_status(F.status, err);
}

// ---------------------------------------------------------------------------
static size_t compress_lds(const Geom &g, const int *t, bool judge = true)
{
    const int h0 = g.D >= 3 ? 1 : 0, h1 = g.D >= 2 ? 1 : 0;
    const size_t ne = (size_t)(t[0] + h0) * (t[1] + h1) * (t[2] + 1);
    const size_t nbt = (size_t)(t[0] / g.bd[0]) * (t[1] / g.bd[1]) * (t[2] / g.bd[2]);
    const size_t ntp = (size_t)t[0] * t[1] * t[2];
    size_t n = nbt * 8 + nbt * 4 + ne * 4 + nbt * 4;  // starts, extents, tile, counts
    if (judge) {  // scores, both codes per point, code-0 counts; window path: bins, tables
        const int bv = g.bd[0] * g.bd[1] * g.bd[2];
        int kt[3];
        n += 2 * nbt * 8 + ntp * 4 + 2 * nbt * 4;
        if (!judge_sorts(known_shape(g.D, g.B, kt), bv))
            n += nbt * kJudgeWin * 4 + 2 * nbt * (size_t)judge_slots(bv) * 4;
    }
    return n + ntp;  // bound bits
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

template <typename T, int D, int BB, int HP, bool FP, int PREC, bool BATCH, int TV, bool W32>
static void go_one(const CompressArgs &a, unsigned num_cus, size_t lds, hipStream_t s)
{
    // persistent grid: every workgroup that can be resident at once (a
    // multiple of 8 so that each XCD gets the same number), at most one per tile
    const void *fn =
        reinterpret_cast<const void *>(&k_compress<T, D, BB, HP, FP, PREC, BATCH, TV, W32>);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    long long grid = std::min((long long)per_cu * num_cus, (a.ntiles + 7) / 8 * 8);
    grid = std::max(8LL, grid / 8 * 8);
    hipLaunchKernelGGL((k_compress<T, D, BB, HP, FP, PREC, BATCH, TV, W32>), dim3((unsigned)grid),
                       dim3(256), lds, s, a);
}

template <typename T, int D, int BB, int HP, bool FP, int PREC, bool BATCH = false, int TV = 0>
static void go(const CompressArgs &a, unsigned num_cus, size_t lds, hipStream_t s)
{
    // compiled tiles of grid entries: the 32-bit variant and the generic one,
    // each returning at once on the other's fields
    if constexpr (ShapeOf<D, BB>::known && FP && !BATCH)
        go_one<T, D, BB, HP, FP, PREC, BATCH, TV, true>(a, num_cus, lds, s);
    go_one<T, D, BB, HP, FP, PREC, BATCH, TV, false>(a, num_cus, lds, s);
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

template <typename T, int D, int BB, int TV>
static void by_hidden_batch(int HP, const CompressArgs &a, unsigned grid, size_t lds, hipStream_t s)
{
    if (HP == 0)
        go<T, D, BB, 8, true, 1, true, TV>(a, grid, lds, s);
    else if (HP == 8)
        go<T, D, BB, 8, true, 0, true, TV>(a, grid, lds, s);
    else if (HP == 16)
        go<T, D, BB, 16, true, 0, true, TV>(a, grid, lds, s);
    else
        go<T, D, BB, 32, true, 0, true, TV>(a, grid, lds, s);
}

template <typename T, int D, int BB>
static void by_variant_batch(int TV, int HP, const CompressArgs &a, unsigned grid, size_t lds,
                             hipStream_t s)
{
    if (TV == 1)
        by_hidden_batch<T, D, BB, 1>(HP, a, grid, lds, s);
    else if (TV == 2)
        by_hidden_batch<T, D, BB, 2>(HP, a, grid, lds, s);
    else
        by_hidden_batch<T, D, BB, 0>(HP, a, grid, lds, s);
}

bool batch_shape(int D, int B) { return (D == 3 && B == 8) || (D == 2 && B == 16); }

// One persistent launch over every tile of nfields FP32 fields of one class
// (dimensionality and block): d_fields (device) in tile order, each reading
// its grid-value entries; tiles of shape variant `variant` (tile.t).
hipError_t launch_compress_batch(const FieldDesc *d_fields, int nfields, long long ntiles,
                                 const Geom &g, const Tile &tile, int variant,
                                 const pwrel_mlp *model, const pwrel_options &opt,
                                 const long long *qtab, int num_cus, hipStream_t s)
{
    int vt[3];
    if (!batch_shape(g.D, g.B) || g.dtype != PWREL_F32 || variant < 0 ||
        variant >= kTileVariants || !variant_shape(g.D, g.B, variant, vt) ||
        vt[0] != tile.t[0] || vt[1] != tile.t[1] || vt[2] != tile.t[2])
        return hipErrorInvalidValue;
    CompressArgs a{};
    a.fields = d_fields;
    a.nfields = nfields;
    for (int d = 0; d < 3; ++d) {
        a.bd[d] = g.bd[d];
        a.t[d] = tile.t[d];
    }
    a.ntiles = ntiles;
    a.use_net = opt.use_net;
    a.judge = opt.judge;
    a.independent = opt.independent_blocks;
    a.entries = 1;
    a.qtab = qtab;
    a.mlp = pack_mlp(opt.use_net ? model : nullptr);
    const bool mfma = opt.use_net && model && model->precision == 1;
    const int HP = mfma ? 0 : hidden_pad(opt.use_net ? model : nullptr);
    const size_t lds = compress_lds(g, tile.t, opt.judge != 0);
    const unsigned grid = (unsigned)std::max(num_cus, 8);
    if (g.D == 3)
        by_variant_batch<float, 3, 8>(variant, HP, a, grid, lds, s);
    else
        by_variant_batch<float, 2, 16>(variant, HP, a, grid, lds, s);
    return hipGetLastError();
}

// Grid value and bound check of every value of an FP32 field (the same
// fast paths, fallbacks and order as the fused kernel's per-point step), one
// entry per value: 2 p, plus 1 where the PW_REL bound check fails.  The fused
// kernel then reads entries instead of values, so no extended tile computes
// its halo's grid values a second time.
__device__ __forceinline__ int grid_entry(float xf, const DevConsts &c, int &err)
{
    int p;
    bool sure;
    if (!grid_value_fast(xf, c, p, sure)) {
        p = grid_value((double)xf, c, err);
        sure = false;
    }
    bool ok = true;
    if (!sure && !within_bound_fast(xf, p, c, ok))
        ok = within_bound((double)xf, grid_inverse<float>(p, c), c.eps);
    return (int)(((unsigned)p << 1) | (ok ? 0u : 1u));  // |p| < 2^30
}

__global__ void __launch_bounds__(256) k_grid_entries(const float *__restrict__ x, long long n,
                                                      const DevConsts *consts, int *status,
                                                      int *__restrict__ ent)
{
    if (*status != kOk)
        return;  // every thread reads the same word: a uniform exit
    const DevConsts c = *consts;
    int err = kOk;
    const long long stride = (long long)gridDim.x * 256;
    const long long tid = blockIdx.x * 256LL + threadIdx.x;
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    const long long n4 = vec ? n >> 2 : 0;
    for (long long i = tid; i < n4; i += stride) {
        const float4 v = reinterpret_cast<const float4 *>(x)[i];
        reinterpret_cast<int4 *>(ent)[i] = make_int4(grid_entry(v.x, c, err), grid_entry(v.y, c, err),
                                                     grid_entry(v.z, c, err), grid_entry(v.w, c, err));
    }
    for (long long i = 4 * n4 + tid; i < n; i += stride)
        ent[i] = grid_entry(x[i], c, err);
    set_status(status, err);
}

// Grid entries of a batch: workgroup k takes chunk k - chunk0 of the field
// whose chunk range holds k (binary search of the fields' first chunks).
__global__ void __launch_bounds__(256) k_grid_entries_batch(const BatchField *fields, int nf)
{
    const long long k = blockIdx.x;
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fields[mid].echunk0 <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchField &f = fields[__builtin_amdgcn_readfirstlane(lo)];
    if (*f.status != kOk)
        return;  // no barrier below: a per-thread exit is safe
    const DevConsts c = *f.consts;
    const float *x = static_cast<const float *>(f.x);
    const long long b0 = (k - f.echunk0) * kEntryChunk, b1 = std::min(f.N, b0 + kEntryChunk);
    int err = kOk;
    // four values per 16-byte load and store where the field is 16-byte
    // aligned (chunk starts are multiples of 4 values, entry rows of 64)
    const long long n4 = f.vec ? (b1 - b0) >> 2 : 0;
    const float4 *x4 = reinterpret_cast<const float4 *>(x + b0);
    int4 *e4 = reinterpret_cast<int4 *>(f.pgrid + b0);
    for (long long i = threadIdx.x; i < n4; i += 256) {
        const float4 v = x4[i];
        e4[i] = make_int4(grid_entry(v.x, c, err), grid_entry(v.y, c, err),
                          grid_entry(v.z, c, err), grid_entry(v.w, c, err));
    }
    for (long long i = b0 + 4 * n4 + threadIdx.x; i < b1; i += 256)
        f.pgrid[i] = grid_entry(x[i], c, err);
    set_status(f.status, err);
}

hipError_t launch_grid_entries_batch(const BatchField *d_fields, int nf, long long nchunks,
                                     hipStream_t s)
{
    if (nchunks > 0)
        hipLaunchKernelGGL(k_grid_entries_batch, dim3((unsigned)nchunks), dim3(256), 0, s,
                           d_fields, nf);
    return hipGetLastError();
}

hipError_t launch_grid_entries(const float *x, const Geom &g, Workspace &ws, int *ent,
                               hipStream_t s)
{
    const long long work = (g.N + 3) / 4;
    const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>((work + 255) / 256, 8192));
    hipLaunchKernelGGL(k_grid_entries, dim3(grid), dim3(256), 0, s, x, g.N, ws.consts, ws.status,
                       ent);
    return hipGetLastError();
}

hipError_t launch_compress(const void *x, const int *pfield, const Geom &g, const Tile &tile,
                           const pwrel_mlp *model, const pwrel_options &opt, Workspace &ws,
                           uint16_t *codes, uint32_t *counts, uint8_t *bflags, int num_cus,
                           hipStream_t s, bool entries)
{
    CompressArgs a{};
    a.x = x;
    a.pfield = pfield;
    a.entries = entries ? 1 : 0;
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
    const unsigned grid = (unsigned)std::max(num_cus, 8);  // CUs; go() sizes the grid
    const size_t lds = compress_lds(g, tile.t, opt.judge != 0);
    // dynamic LDS plus the kernel's static arrays (weights, status) must fit
    // in one workgroup's share
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess)
        return hipErrorInvalidDevice;
    if (lds + sizeof(float4) * kWlds + 64 > (size_t)lds_max)
        return hipErrorInvalidConfiguration;
    if (pfield)
        by_shape<float, true>(g.D, g.B, HP, a, (unsigned)grid, lds, s);
    else if (g.dtype == PWREL_F32)
        return hipErrorInvalidValue;  // FP32 fields take the two passes (entries)
    else
        by_shape<double, false>(g.D, g.B, HP, a, (unsigned)grid, lds, s);
    return hipGetLastError();
}

}  // namespace pwrel
