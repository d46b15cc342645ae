// Field statistics, constants, scan / raw scatter, stream header, histogram
// and inspection kernels of the PW_REL perceptron codec (gfx950).
//
// Compression:   reset -> stats -> consts -> compress -> scan -> scatter -> header
// Decompression: reset -> scan -> decode (per block level, or all blocks at once)
#include "pwrel_kernels.h"
#include "pwrel_wavesort.h"

namespace pwrel {

// ---------------------------------------------------------------------------
// reset: status and balance-point total (graph-safe: a kernel, not a memset)
// ---------------------------------------------------------------------------
__global__ void k_reset(int *status, unsigned long long *n_raw, unsigned *ticket)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *status = kOk;
        *n_raw = 0ULL;
        *ticket = 0u;
    }
}

// ---------------------------------------------------------------------------
// a1: statistics in two stages.  Each workgroup reduces its part of the field
// (per-lane min / max of |x| bit patterns -- order-preserving for finite
// non-negative floats -- and counts; wave shuffles, then LDS) to one record;
// the constants kernel reduces the records.  No same-address atomics.
// ---------------------------------------------------------------------------
struct Acc {
    unsigned long long mn, mx, nz, nn, nf;
};

__device__ __forceinline__ void classify(float v, Acc &a)
{
    const unsigned b = __float_as_uint(v);
    const unsigned m = b & 0x7fffffffu;
    if ((m >> 23) == 0xffu) {
        a.nf++;
    } else if (m == 0u) {
        a.nz++;
    } else {
        a.nn += (b >> 31);
        a.mn = (unsigned long long)m < a.mn ? (unsigned long long)m : a.mn;
        a.mx = (unsigned long long)m > a.mx ? (unsigned long long)m : a.mx;
    }
}

__device__ __forceinline__ void classify(double v, Acc &a)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned long long m = b & 0x7fffffffffffffffULL;
    if ((m >> 52) == 0x7ffULL) {
        a.nf++;
    } else if (m == 0ULL) {
        a.nz++;
    } else {
        a.nn += (b >> 63);
        a.mn = m < a.mn ? m : a.mn;
        a.mx = m > a.mx ? m : a.mx;
    }
}

__device__ __forceinline__ void wave_reduce(Acc &a)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long mn = __shfl_xor(a.mn, off, 64);
        const unsigned long long mx = __shfl_xor(a.mx, off, 64);
        a.mn = mn < a.mn ? mn : a.mn;
        a.mx = mx > a.mx ? mx : a.mx;
        a.nz += __shfl_xor(a.nz, off, 64);
        a.nn += __shfl_xor(a.nn, off, 64);
        a.nf += __shfl_xor(a.nf, off, 64);
    }
}

// combine the per-wave records of the workgroup into thread 0
__device__ __forceinline__ void block_reduce(Acc &a)
{
    __shared__ Acc part[4];
    wave_reduce(a);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        part[w] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
            a.mn = part[q].mn < a.mn ? part[q].mn : a.mn;
            a.mx = part[q].mx > a.mx ? part[q].mx : a.mx;
            a.nz += part[q].nz;
            a.nn += part[q].nn;
            a.nf += part[q].nf;
        }
    }
}

// FP32 values per thread in 32-bit accumulators, without branches: the same
// classes and extremes as classify(float)
struct Acc32 {
    unsigned mn, mx, nz, nn, nf;
};

__device__ __forceinline__ void classify32(float v, Acc32 &a)
{
    const unsigned b = __float_as_uint(v);
    const unsigned m = b & 0x7fffffffu;
    const bool nonfinite = m >= 0x7f800000u, zero = m == 0u;
    const bool normal = !nonfinite && !zero;
    a.nf += nonfinite ? 1u : 0u;
    a.nz += zero ? 1u : 0u;
    a.nn += normal ? (b >> 31) : 0u;
    a.mn = normal && m < a.mn ? m : a.mn;
    a.mx = normal && m > a.mx ? m : a.mx;
}

// part `part` of nparts of a field's statistics (a workgroup's share) into *out
template <typename T, typename V, int VW>
__device__ __forceinline__ void stats_part(const T *__restrict__ x, long long n, int part,
                                           int nparts, DevStats *out)
{
    Acc a{~0ULL, 0ULL, 0ULL, 0ULL, 0ULL};
    const long long tid = (long long)part * blockDim.x + threadIdx.x;
    const long long nthr = (long long)nparts * blockDim.x;
    const long long nv = n / VW;
    const V *xv = reinterpret_cast<const V *>(x);
    if constexpr (std::is_same<T, float>::value) {
        // fewer than 2^32 values per thread: the 32-bit counts cannot wrap
        Acc32 b{~0u, 0u, 0u, 0u, 0u};
        for (long long i = tid; i < nv; i += nthr) {
            const V v = xv[i];
            const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
            for (int q = 0; q < VW; ++q)
                classify32(e[q], b);
        }
        for (long long i = nv * VW + tid; i < n; i += nthr)
            classify32(x[i], b);
        a.mn = b.mn == ~0u ? ~0ULL : (unsigned long long)b.mn;
        a.mx = b.mx;
        a.nz = b.nz;
        a.nn = b.nn;
        a.nf = b.nf;
    } else {
        for (long long i = tid; i < nv; i += nthr) {
            const V v = xv[i];
            const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
            for (int q = 0; q < VW; ++q)
                classify(e[q], a);
        }
        for (long long i = nv * VW + tid; i < n; i += nthr)
            classify(x[i], a);
    }
    block_reduce(a);
    if (threadIdx.x == 0) {
        DevStats r{};
        r.min_bits = a.mn;
        r.max_bits = a.mx;
        r.n_zero = a.nz;
        r.n_neg = a.nn;
        r.n_nonfinite = a.nf;
        *out = r;
    }
}

template <typename T, typename V, int VW>
__global__ void __launch_bounds__(256) k_stats(const T *__restrict__ x, long long n,
                                               DevStats *parts)
{
    stats_part<T, V, VW>(x, n, blockIdx.x, gridDim.x, parts + blockIdx.x);
}

// ---------------------------------------------------------------------------
// a2: reduce the statistics records, then the constants (Eq. 8-12) on one
// thread; everything stays on the device.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double from_abs_bits(unsigned long long b);
template <>
__device__ __forceinline__ double from_abs_bits<float>(unsigned long long b)
{
    return (double)__uint_as_float((unsigned)b);
}
template <>
__device__ __forceinline__ double from_abs_bits<double>(unsigned long long b)
{
    return __longlong_as_double((long long)b);
}

template <typename T>
__device__ __forceinline__ void consts_reduce(const DevStats *parts, int nparts, double eps,
                                              DevConsts *c, int *status)
{
    Acc a{~0ULL, 0ULL, 0ULL, 0ULL, 0ULL};
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        const DevStats r = parts[i];
        a.mn = r.min_bits < a.mn ? r.min_bits : a.mn;
        a.mx = r.max_bits > a.mx ? r.max_bits : a.mx;
        a.nz += r.n_zero;
        a.nn += r.n_neg;
        a.nf += r.n_nonfinite;
    }
    block_reduce(a);
    if (threadIdx.x != 0)
        return;
    double amin = 1.0, amax = 1.0;
    if (a.mn != ~0ULL) {
        amin = from_abs_bits<T>(a.mn);
        amax = from_abs_bits<T>(a.mx);
    }
    DevConsts k{};
    k.abs_min = amin;
    k.abs_max = amax;
    k.n_zero = a.nz;
    k.n_neg = a.nn;
    k.n_nonfinite = a.nf;
    int err = kOk;
    if (a.nf)
        err = kENonFinite;
    const double tau = sizeof(T) == 4 ? 0x1p-126 : 0x1p-1022;
    double eps0 = amin * 0.5;
    if (tau < eps0)
        eps0 = tau;
    if (err == kOk && !(eps0 > 0.0))
        err = kERange;
    const double one_eps = 1.0 + eps;
    if (err == kOk) {
        k.eps = eps;
        k.eps0 = eps0;
        k.b_a = det_log2(one_eps);
        k.w = k.b_a + k.b_a;
        k.r = 1.0 / k.w;
        k.Lp = det_log2(amin);
        k.Ln = ((det_log2(amax + eps0) + k.Lp) + k.w) - det_log2(amin - eps0);
        k.d0 = det_log2(eps0) + k.Lp;
        const double tz = k.d0 * k.r;
        const double tb = (det_log2(amax) + k.Lp) * k.r;
        const double tn = (det_log2(amin) + k.Ln) * k.r;
        if (!(__builtin_fabs(tz) < kGridLimit) || !(__builtin_fabs(tb) < kGridLimit) ||
            !(__builtin_fabs(tn) < kGridLimit)) {
            err = kERange;
        } else {
            k.p_zero = (long long)__builtin_rint(tz);
            k.b_sign = (long long)__builtin_rint(tb);
            k.n_lo = (long long)__builtin_rint(tn);
            k.delta = k.b_sign + 1 - k.n_lo;
            if (k.delta < 0)
                k.delta = 0;
        }
        // largest grid value any point can take: positive values end at
        // b_sign, negative ones grow with |x| up to |x| = abs_max
        if (err == kOk) {
            long long qmax = k.b_sign;
            if (a.nn) {
                long long qn = (long long)__builtin_rint((det_log2(amax) + k.Ln) * k.r) + k.delta;
                qn = qn < k.b_sign + 1 ? k.b_sign + 1 : qn;
                qmax = qn > qmax ? qn : qmax;
            }
            k.w32 = (qmax - k.p_zero) < (1LL << 27) ? 1 : 0;
            k.p_max = qmax + 1;
        }
        // fast-path margins: |t_fast - t| <= (err(log2) + 2^-52 (|log2 x| + |L| + 1))
        // r + 2^-52 |t| with |log2 x| < 129 and |t| < 2^30, enlarged by 1/64
        k.fm_p = ((kFastLog2Err + 0x1p-52 * (130.0 + __builtin_fabs(k.Lp))) * k.r + 0x1p-22) *
                 (1.0 + 0x1p-6);
        k.fm_n = ((kFastLog2Err + 0x1p-52 * (130.0 + __builtin_fabs(k.Ln))) * k.r + 0x1p-22) *
                 (1.0 + 0x1p-6);
        // certified-bound margin: 2^-21 / ln(1 + eps), ln(1 + eps) = b_a ln 2
        k.vm = 0x1p-21 / (k.b_a * 0.6931471805599453);
    }
    k.status = err;
    *c = k;
    set_status(status, err);
}

template <typename T>
__global__ void __launch_bounds__(256) k_consts(const DevStats *parts, int nparts, double eps,
                                                DevConsts *c, int *status)
{
    consts_reduce<T>(parts, nparts, eps, c, status);
}

// ---------------------------------------------------------------------------
// a3 alone: grid value of every point (inspection entry point).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_transform(const T *__restrict__ x, long long n,
                                                   const DevConsts *cp, int *status,
                                                   int *__restrict__ p)
{
    if (*status != kOk)
        return;  // no barrier below: a per-thread exit is safe
    const DevConsts c = *cp;
    int err = kOk;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = grid_value((double)x[i], c, err);
    set_status(status, err);
}

// ---------------------------------------------------------------------------
// a7: exclusive scan of per-block balance-point counts (two levels).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned o = __shfl_up(v, d, 64);
        if (lane >= d)
            v += o;
    }
    return v;
}

// chunk `chunk` (kScanChunk counts) of an exclusive scan: offsets relative to
// the chunk, the chunk's total into partials[chunk]
template <typename C>
__device__ __forceinline__ void scan_chunk(const C *__restrict__ counts, long long nb, long long chunk,
                                           unsigned long long *__restrict__ offs,
                                           unsigned long long *__restrict__ partials)
{
    __shared__ unsigned wsum[4];
    constexpr int PER = kScanChunk / 256;
    const long long base = chunk * kScanChunk + threadIdx.x * PER;
    unsigned v[PER];
    unsigned s = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        v[q] = (base + q < nb) ? counts[base + q] : 0u;
        s += v[q];
    }
    const unsigned incl = wave_incl_scan(s);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63)
        wsum[w] = incl;
    __syncthreads();
    unsigned wbase = 0;
    for (int q = 0; q < w; ++q)
        wbase += wsum[q];
    unsigned run = wbase + incl - s;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        if (base + q < nb)
            offs[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 255)
        partials[chunk] = (unsigned long long)(wbase + incl);
}

template <typename C>
__global__ void __launch_bounds__(256) k_scan_local(const C *__restrict__ counts,
                                                    long long nb,
                                                    unsigned long long *__restrict__ offs,
                                                    unsigned long long *__restrict__ partials)
{
    scan_chunk<C>(counts, nb, blockIdx.x, offs, partials);
}

__device__ __forceinline__ void scan_partials(unsigned long long *partials, long long np,
                                              unsigned long long *total)
{
    __shared__ unsigned long long sh[1024];
    unsigned long long carry = 0;
    for (long long b0 = 0; b0 < np; b0 += 1024) {
        const long long i = b0 + threadIdx.x;
        const unsigned long long v = i < np ? partials[i] : 0ULL;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const unsigned long long o = threadIdx.x >= d ? sh[threadIdx.x - d] : 0ULL;
            __syncthreads();
            sh[threadIdx.x] += o;
            __syncthreads();
        }
        if (i < np)
            partials[i] = carry + sh[threadIdx.x] - v;
        const unsigned long long tot = sh[1023];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0)
        *total = carry;
}

__global__ void __launch_bounds__(1024) k_scan_partials(unsigned long long *partials,
                                                        long long np,
                                                        unsigned long long *total)
{
    scan_partials(partials, np, total);
}

// ---------------------------------------------------------------------------
// a7: raw values of balance points in stream order (one wave per block, wave
// ballot + popcount for the in-block rank).
// ---------------------------------------------------------------------------


// the raw values of block b's balance points (one wave)
template <typename T>
__device__ __forceinline__ void scatter_block(const T *__restrict__ x, const GeoArgs &g,
                                              const uint16_t *__restrict__ codes,
                                              const uint32_t *__restrict__ counts,
                                              const unsigned long long *offs,
                                              const unsigned long long *partials,
                                              T *__restrict__ raw, unsigned long long raw_cap,
                                              int *status, long long b)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    {
        const unsigned cnt = counts[b];
        if (cnt == 0)
            return;
        const long long bx = b % g.nb[2], by = (b / g.nb[2]) % g.nb[1],
                        bz = b / (g.nb[1] * g.nb[2]);
        const BlockGeo q = block_geo3(bz, by, bx, g.n, g.bd[0], g.bd[1], g.bd[2]);
        const long long bsize = (long long)q.ez * q.ey * q.ex;
        const unsigned long long base = offs[b] + partials[b / kScanChunk];
        unsigned run = 0;
        for (long long c0 = 0; c0 < bsize && run < cnt; c0 += 64) {
            const long long li = c0 + lane;
            const bool z = li < bsize && codes[q.start + li] == 0;
            const unsigned long long mask = __ballot(z);
            if (z) {
                const unsigned rank = run + (unsigned)__popcll(mask & below);
                const long long lx = li % q.ex, ly = (li / q.ex) % q.ey, lz = li / (q.ex * q.ey);
                const long long gi = ((bz * g.bd[0] + lz) * g.n[1] + by * g.bd[1] + ly) *
                                         g.n[2] + bx * g.bd[2] + lx;
                if (base + rank < raw_cap)
                    raw[base + rank] = x[gi];
                else
                    set_status(status, kENoSpc);
            }
            run += (unsigned)__popcll(mask);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_scatter(const T *__restrict__ x, GeoArgs g,
                                                 const uint16_t *__restrict__ codes,
                                                 const uint32_t *__restrict__ counts,
                                                 const unsigned long long *offs,
                                                 const unsigned long long *partials,
                                                 T *__restrict__ raw, unsigned long long raw_cap,
                                                 int *status)
{
    if (*status != kOk)
        return;  // wave-level work only: a per-thread exit is safe
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long b = wave; b < g.nblocks; b += nwaves)
        scatter_block<T>(x, g, codes, counts, offs, partials, raw, raw_cap, status, b);
}

// ---------------------------------------------------------------------------
// stream header (one thread)
// ---------------------------------------------------------------------------


// Writes the header and zeroes every alignment gap, so that equal inputs give
// byte-identical streams.
__device__ __forceinline__ void write_header(const HeaderArgs &h, const DevConsts *cp,
                                             const unsigned long long *n_raw, int *status,
                                             pwrel_header *out, unsigned long long *out_size)
{
    unsigned char *bytes = reinterpret_cast<unsigned char *>(out);
    for (int r = 0; r < kHeaderGaps; ++r)
        for (unsigned long long i = h.pad_lo[r] + threadIdx.x; i < h.pad_hi[r]; i += blockDim.x)
            bytes[i] = 0;
    if (threadIdx.x != 0)
        return;
    pwrel_header o{};
    const DevConsts c = *cp;
    o.magic = PWREL_MAGIC;
    o.version = PWREL_VERSION;
    o.dtype = h.dtype;
    o.ndim = h.ndim;
    for (int d = 0; d < 3; ++d)
        o.dims[d] = h.dims[d];
    o.block = h.block;
    o.flags = h.flags;
    o.eps = c.eps;
    o.eps0 = c.eps0;
    o.b_a = c.b_a;
    o.w = c.w;
    o.r = c.r;
    o.Lp = c.Lp;
    o.Ln = c.Ln;
    o.d0 = c.d0;
    o.p_zero = c.p_zero;
    o.b_sign = c.b_sign;
    o.n_lo = c.n_lo;
    o.delta = c.delta;
    o.n = h.n;
    o.nblocks = h.nblocks;
    o.n_raw = *n_raw;
    o.off_model = h.off_model;
    o.off_bflags = h.off_bflags;
    o.off_counts = h.off_counts;
    o.off_codes = h.off_codes;
    o.off_raw = h.off_raw;
    o.total_size = h.off_raw + o.n_raw * (unsigned long long)h.raw_size;
    o.abs_min = c.abs_min;
    o.abs_max = c.abs_max;
    o.n_zero = c.n_zero;
    o.n_neg = c.n_neg;
    o.p_max = c.p_max;
    o.off_huff = h.off_huff;
    o.off_sizes = h.off_sizes;
    o.off_bits = h.off_bits;
    o.n_bits = h.n_bits;
    o.n_sym = h.n_sym;
    o.size_bytes = h.size_bytes;
    o.esc_len = h.esc_len;
    int st = *status;
    if (st == kOk && o.total_size > h.capacity)
        st = kENoSpc;
    o.status = st;
    *out = o;
    if (out_size)
        *out_size = st == kOk ? o.total_size : 0ULL;
}

__global__ void __launch_bounds__(256) k_header(HeaderArgs h, const DevConsts *cp,
                                                const unsigned long long *n_raw, int *status,
                                                pwrel_header *out)
{
    write_header(h, cp, n_raw, status, out, nullptr);
}

// ---------------------------------------------------------------------------
// code histogram (inspection, and the Huffman stage's codebook): LDS window
// around the zero-error code, global atomics outside it, one flush per
// workgroup.
// ---------------------------------------------------------------------------
constexpr int kHistWin = 32768;  // half the code space: 128 KiB of LDS

// Per workgroup (1024 threads, one or two per CU) over its share of the codes:
// a histogram of half the code space at a time in LDS (128 KiB): first the
// central half (errors within +-2^14), then, only if the workgroup met any
// code outside it, the outer half; each pass ends with one flush of the
// non-zero bins.  No code goes to a global atomic on its own, however wide
// the errors.  Each thread counts a contiguous run of codes (16-byte loads),
// so the lanes of an atomic instruction mostly address different bins.
__global__ void __launch_bounds__(1024) k_hist(const uint16_t *__restrict__ codes, long long n,
                                               unsigned long long *hist)
{
    extern __shared__ unsigned win[];
    __shared__ int s_outer;
    const long long nth = (long long)gridDim.x * blockDim.x;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool al = (reinterpret_cast<uintptr_t>(codes) & 15) == 0;
    const long long n8 = al ? n / 8 : 0;
    constexpr unsigned lo = kR - kHistWin / 2, hi = kR + kHistWin / 2;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = threadIdx.x; i < kHistWin; i += blockDim.x)
            win[i] = 0u;
        if (threadIdx.x == 0 && pass == 0)
            s_outer = 0;
        __syncthreads();
        bool outer = false;
        // bin of a code in this pass's half, or -1
        auto bin = [&](unsigned code) -> int {
            const bool central = code >= lo && code < hi;
            if (pass == 0) {
                outer |= !central;
                return central ? (int)(code - lo) : -1;
            }
            return central ? -1 : (int)(code < lo ? code : code - kHistWin);
        };
        auto add = [&](unsigned code) {
            const int k = bin(code);
            if (k >= 0)
                atomicAdd(&win[k], 1u);
        };
        for (long long i = t; i < n8; i += nth) {
            const uint4 v = reinterpret_cast<const uint4 *>(codes)[i];
            const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                add(w[k] & 0xFFFFu);
                add(w[k] >> 16);
            }
        }
        for (long long i = 8 * n8 + t; i < n; i += nth)
            add(codes[i]);
        if (pass == 0 && outer)
            s_outer = 1;
        __syncthreads();
        for (int i = threadIdx.x; i < kHistWin; i += blockDim.x)
            if (win[i]) {
                const unsigned code = pass == 0 ? lo + i : (i < (int)lo ? i : i + kHistWin);
                atomicAdd(&hist[code], (unsigned long long)win[i]);
            }
        const bool again = s_outer != 0;
        __syncthreads();
        if (!again)
            break;  // uniform: every thread read the same shared flag
    }
}

__global__ void k_zero_u64(unsigned long long *p, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0ULL;
}

// ---------------------------------------------------------------------------
// deterministic math on the device (inspection entry point)
// ---------------------------------------------------------------------------
__global__ void k_detmath(const double *x, double *l2, double *e2, unsigned long long n)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double v = x[i];
    if (l2)
        l2[i] = v > 0.0 ? det_log2(v) : 0.0;
    if (e2)
        e2[i] = det_exp2(v);
}

// ---------------------------------------------------------------------------
// Exhaustive checks of the fast-path bounds: the largest |fast_log2(a) -
// det_log2(a)| over every normal float a > 0, and the largest relative error
// of v_exp_f32 over every float |f| <= 1/2 (reduced as ordered bit patterns
// of non-negative doubles).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void max_bits(unsigned long long *dst, double v, unsigned long long *sh)
{
    // wave maximum, then one atomic per wave
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long ob = __shfl_xor(b, o, 64);
        b = ob > b ? ob : b;
    }
    (void)sh;
    if ((threadIdx.x & 63) == 0)
        atomicMax(dst, b);
}

__global__ void __launch_bounds__(256) k_fm_log(unsigned long long *out)
{
    const unsigned lo = 0x00800000u, hi = 0x7f7fffffu;  // normal positive floats
    double worst = 0.0;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
         i <= hi - lo; i += (unsigned long long)gridDim.x * blockDim.x) {
        const float a = __uint_as_float(lo + (unsigned)i);
        const double e = __builtin_fabs(fast_log2(a) - det_log2((double)a));
        worst = e > worst ? e : worst;
    }
    max_bits(out, worst, nullptr);
}

__global__ void __launch_bounds__(256) k_fm_exp(unsigned long long *out)
{
    const unsigned hi = 0x3f000000u;  // |f| <= 0.5, both signs, subnormals included
    double worst = 0.0;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
         i < 2ULL * (hi + 1ULL); i += (unsigned long long)gridDim.x * blockDim.x) {
        const unsigned mag = (unsigned)(i >> 1);
        const float f = __uint_as_float(mag | ((unsigned)(i & 1) << 31));
        const double ref = det_exp2((double)f);
        const double e = __builtin_fabs((double)__builtin_amdgcn_exp2f(f) - ref) / ref;
        worst = e > worst ? e : worst;
    }
    max_bits(out, worst, nullptr);
}

// ===========================================================================
// launchers
// ===========================================================================
static unsigned grid_for(long long work, int per, unsigned cap)
{
    long long g = (work + per - 1) / per;
    if (g < 1)
        g = 1;
    if (g > cap)
        g = cap;
    return (unsigned)g;
}

hipError_t launch_reset(Workspace &ws, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, ws.status, ws.n_raw, ws.ticket);
    return hipGetLastError();
}

static unsigned stats_grid(const Geom &g) { return grid_for(g.N, 256 * 16, kStatParts); }

hipError_t launch_stats(const void *x, const Geom &g, Workspace &ws, hipStream_t s)
{
    const unsigned grid = stats_grid(g);
    const bool al16 = (reinterpret_cast<uintptr_t>(x) & 15u) == 0;
    if (g.dtype == PWREL_F32) {
        if (al16)
            hipLaunchKernelGGL((k_stats<float, float4, 4>), dim3(grid), dim3(256), 0, s,
                               (const float *)x, g.N, ws.stats);
        else
            hipLaunchKernelGGL((k_stats<float, float, 1>), dim3(grid), dim3(256), 0, s,
                               (const float *)x, g.N, ws.stats);
    } else {
        if (al16)
            hipLaunchKernelGGL((k_stats<double, double2, 2>), dim3(grid), dim3(256), 0, s,
                               (const double *)x, g.N, ws.stats);
        else
            hipLaunchKernelGGL((k_stats<double, double, 1>), dim3(grid), dim3(256), 0, s,
                               (const double *)x, g.N, ws.stats);
    }
    return hipGetLastError();
}

hipError_t launch_consts(const Geom &g, double eps, Workspace &ws, hipStream_t s)
{
    const int nparts = (int)stats_grid(g);
    if (g.dtype == PWREL_F32)
        hipLaunchKernelGGL(k_consts<float>, dim3(1), dim3(256), 0, s, ws.stats, nparts, eps,
                           ws.consts, ws.status);
    else
        hipLaunchKernelGGL(k_consts<double>, dim3(1), dim3(256), 0, s, ws.stats, nparts, eps,
                           ws.consts, ws.status);
    return hipGetLastError();
}

hipError_t launch_transform(const void *x, const Geom &g, Workspace &ws, int *d_p, hipStream_t s)
{
    const unsigned grid = grid_for(g.N, 256 * 8, 8192);
    if (g.dtype == PWREL_F32)
        hipLaunchKernelGGL(k_transform<float>, dim3(grid), dim3(256), 0, s, (const float *)x,
                           g.N, ws.consts, ws.status, d_p);
    else
        hipLaunchKernelGGL(k_transform<double>, dim3(grid), dim3(256), 0, s, (const double *)x,
                           g.N, ws.consts, ws.status, d_p);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *counts, const Geom &g, Workspace &ws, hipStream_t s)
{
    const long long nparts = (g.nblocks + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_local<uint32_t>, dim3((unsigned)nparts), dim3(256), 0, s, counts,
                       g.nblocks, ws.offsets, ws.partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, ws.partials, nparts,
                       ws.n_raw);
    return hipGetLastError();
}

hipError_t launch_scan_sizes(const void *sizes, int elem_bytes, long long n,
                             unsigned long long *offs, unsigned long long *partials,
                             unsigned long long *total, hipStream_t s)
{
    const long long nparts = (n + kScanChunk - 1) / kScanChunk;
    if (elem_bytes == 2)
        hipLaunchKernelGGL(k_scan_local<uint16_t>, dim3((unsigned)nparts), dim3(256), 0, s,
                           static_cast<const uint16_t *>(sizes), n, offs, partials);
    else
        hipLaunchKernelGGL(k_scan_local<uint32_t>, dim3((unsigned)nparts), dim3(256), 0, s,
                           static_cast<const uint32_t *>(sizes), n, offs, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, nparts, total);
    return hipGetLastError();
}

static GeoArgs geo_args(const Geom &g)
{
    GeoArgs a{};
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bd[d] = g.bd[d];
        a.nb[d] = g.nb[d];
    }
    a.nblocks = g.nblocks;
    return a;
}

hipError_t launch_scatter(const void *x, const Geom &g, const uint16_t *codes,
                          const uint32_t *counts, Workspace &ws, void *raw,
                          unsigned long long raw_cap, hipStream_t s)
{
    const unsigned grid = grid_for(g.nblocks, 4, 8192);
    const GeoArgs ga = geo_args(g);
    if (g.dtype == PWREL_F32)
        hipLaunchKernelGGL(k_scatter<float>, dim3(grid), dim3(256), 0, s, (const float *)x, ga,
                           codes, counts, ws.offsets, ws.partials, (float *)raw, raw_cap,
                           ws.status);
    else
        hipLaunchKernelGGL(k_scatter<double>, dim3(grid), dim3(256), 0, s, (const double *)x, ga,
                           codes, counts, ws.offsets, ws.partials, (double *)raw, raw_cap,
                           ws.status);
    return hipGetLastError();
}

HeaderArgs make_header_args(const Geom &g, int flags, const uint64_t *offs, uint64_t capacity,
                            bool stream_gaps, const HuffLayout *hl)
{
    HeaderArgs h{};
    h.dtype = g.dtype;
    h.ndim = g.D;
    h.block = g.B;
    h.flags = flags;
    for (int d = 0; d < 3; ++d)
        h.dims[d] = d < g.D ? (unsigned long long)g.n[3 - g.D + d] : 0ULL;
    h.n = g.N;
    h.nblocks = g.nblocks;
    h.off_model = offs[0];
    h.off_bflags = offs[1];
    h.off_counts = offs[2];
    h.off_codes = hl ? 0ULL : offs[3];
    h.off_raw = offs[4];
    h.capacity = capacity;
    h.raw_size = g.dtype == PWREL_F32 ? 4 : 8;
    // each section's end and the next section's start: the gap between them is zeroed
    unsigned long long ends[kHeaderGaps], nexts[kHeaderGaps];
    int ng = 0;
    auto gap = [&](unsigned long long e, unsigned long long n) {
        ends[ng] = e;
        nexts[ng] = n;
        ++ng;
    };
    gap(sizeof(pwrel_header), offs[0]);
    gap((flags & PWREL_HF_NET) ? offs[0] + sizeof(pwrel_mlp) : offs[0], offs[1]);
    gap((flags & PWREL_HF_JUDGE) ? offs[1] + (unsigned long long)g.nblocks : offs[1], offs[2]);
    if (hl) {
        h.off_huff = hl->off_huff;
        h.off_sizes = hl->off_sizes;
        h.off_bits = hl->off_bits;
        h.n_bits = hl->n_bits;
        h.n_sym = hl->n_sym;
        h.size_bytes = hl->size_bytes;
        h.esc_len = hl->esc_len;
        gap(offs[2] + 4ull * (unsigned long long)g.nblocks, hl->off_huff);
        gap(hl->off_huff + hl->table_bytes, hl->off_sizes);
        gap(hl->off_sizes + (unsigned long long)hl->size_bytes * g.nblocks, hl->off_bits);
        gap(hl->off_bits + 4ull * ((hl->n_bits + 31) / 32), offs[4]);
    } else {
        gap(offs[2] + 4ull * (unsigned long long)g.nblocks, offs[3]);
        gap(offs[3] + 2ull * (unsigned long long)g.N, offs[4]);
    }
    for (int r = 0; r < kHeaderGaps; ++r) {
        h.pad_lo[r] = r < ng ? ends[r] : 0;
        h.pad_hi[r] = r < ng ? std::max(ends[r], nexts[r]) : 0;
        if (!stream_gaps && r > 0)  // a lone header: only its own tail
            h.pad_hi[r] = h.pad_lo[r];
    }
    if (!stream_gaps)
        h.pad_hi[0] = PWREL_HEADER_BYTES;
    return h;
}

hipError_t launch_header(const Geom &g, int flags, const uint64_t *offs, Workspace &ws,
                         void *d_header, uint64_t capacity, bool stream_gaps, hipStream_t s,
                         const HuffLayout *hl)
{
    const HeaderArgs h = make_header_args(g, flags, offs, capacity, stream_gaps, hl);
    hipLaunchKernelGGL(k_header, dim3(1), dim3(256), 0, s, h, ws.consts, ws.n_raw, ws.status,
                       (pwrel_header *)d_header);
    return hipGetLastError();
}

__global__ void k_write_model(pwrel_mlp m, pwrel_mlp *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *dst = m;
}

hipError_t launch_write_model(const pwrel_mlp &m, void *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_write_model, dim3(1), dim3(64), 0, s, m, static_cast<pwrel_mlp *>(dst));
    return hipGetLastError();
}

hipError_t launch_hist(const uint16_t *codes, long long n, unsigned long long *hist,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(256), 0, s, hist, 65536LL);
    if (n > 0)
        hipLaunchKernelGGL(k_hist, dim3(grid_for(n, 1024 * 64, 256)), dim3(1024),
                           kHistWin * sizeof(unsigned), s, codes, n, hist);
    return hipGetLastError();
}

hipError_t launch_fastmath_check(unsigned long long *out2, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, out2, 2LL);
    hipLaunchKernelGGL(k_fm_log, dim3(4096), dim3(256), 0, s, out2);
    hipLaunchKernelGGL(k_fm_exp, dim3(4096), dim3(256), 0, s, out2 + 1);
    return hipGetLastError();
}

hipError_t launch_detmath(const double *x, double *l2, double *e2, uint64_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_detmath, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, l2, e2,
                       (unsigned long long)n);
    return hipGetLastError();
}

}  // namespace pwrel

// ===========================================================================
// batched compression: the per-field stages over a table of fields, one
// launch each whatever the number of fields (workgroups find their field by
// a binary search of the fields' first parts, chunks or blocks)
// ===========================================================================
namespace pwrel {

template <typename K>
__device__ __forceinline__ int batch_field_of(const BatchField *f, int nf, long long k, K key)
{
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (key(f[mid]) <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ void k_batch_reset(const BatchField *f, int nf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nf) {
        *f[i].status = kOk;
        *f[i].n_raw = 0ULL;
    }
}

// statistics: workgroup k = part k - part0 of its field
template <typename T, typename V, int VW>
__global__ void __launch_bounds__(256) k_batch_stats(const BatchField *f, int nf,
                                                     DevStats *records)
{
    const long long k = blockIdx.x;
    const int i = batch_field_of(f, nf, k, [](const BatchField &b) { return b.part0; });
    const BatchField &b = f[i];
    const T *x = static_cast<const T *>(b.x);
    if (b.vec)
        stats_part<T, V, VW>(x, b.N, (int)(k - b.part0), (int)b.nparts, records + k);
    else
        stats_part<T, T, 1>(x, b.N, (int)(k - b.part0), (int)b.nparts, records + k);
}

template <typename T>
__global__ void __launch_bounds__(256) k_batch_consts(const BatchField *f,
                                                      const DevStats *records)
{
    const BatchField &b = f[blockIdx.x];
    consts_reduce<T>(records + b.part0, (int)b.nparts, b.eps, b.consts, b.status);
}

hipError_t launch_batch_front(const BatchField *d_fields, int nf, int dtype, long long nparts,
                              DevStats *records, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3((nf + 255) / 256), dim3(256), 0, s, d_fields, nf);
    if (dtype == PWREL_F32) {
        hipLaunchKernelGGL((k_batch_stats<float, float4, 4>), dim3((unsigned)nparts), dim3(256),
                           0, s, d_fields, nf, records);
        hipLaunchKernelGGL(k_batch_consts<float>, dim3(nf), dim3(256), 0, s, d_fields, records);
    } else {
        hipLaunchKernelGGL((k_batch_stats<double, double2, 2>), dim3((unsigned)nparts),
                           dim3(256), 0, s, d_fields, nf, records);
        hipLaunchKernelGGL(k_batch_consts<double>, dim3(nf), dim3(256), 0, s, d_fields, records);
    }
    return hipGetLastError();
}

// scan: workgroup k = chunk k - chunk0 of its field; offsets and chunk
// partials at the field's own base (blk0, chunk0)
__global__ void __launch_bounds__(256) k_batch_scan_local(const BatchField *f, int nf,
                                                          unsigned long long *offs,
                                                          unsigned long long *partials)
{
    const long long k = blockIdx.x;
    const int i = batch_field_of(f, nf, k, [](const BatchField &b) { return b.chunk0; });
    const BatchField &b = f[i];
    scan_chunk<uint32_t>(b.counts, b.g.nblocks, k - b.chunk0, offs + b.blk0,
                         partials + b.chunk0);
}

__global__ void __launch_bounds__(1024) k_batch_scan_partials(const BatchField *f,
                                                              unsigned long long *partials)
{
    const BatchField &b = f[blockIdx.x];
    scan_partials(partials + b.chunk0, b.nchunks, b.n_raw);
}

// raw values: one wave per scan chunk (kScanChunk blocks) of the batch's
// chunk numbering; a chunk without balance points (its exclusive offsets
// equal the next chunk's) is skipped whole, and within a chunk only the
// blocks with a non-zero count are walked.
template <typename T>
__global__ void __launch_bounds__(256) k_batch_scatter(const BatchField *f, int nf,
                                                       long long nchunks,
                                                       const unsigned long long *offs,
                                                       const unsigned long long *partials)
{
    const long long c = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (c >= nchunks)
        return;  // wave-uniform
    const int lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane(
        batch_field_of(f, nf, c, [](const BatchField &b) { return b.chunk0; }));
    const BatchField &b = f[i];
    if (*b.status != kOk)
        return;  // wave-uniform
    const long long lc = c - b.chunk0;
    const unsigned long long hi = lc + 1 < b.nchunks ? partials[c + 1] : *b.n_raw;
    if (hi == partials[c])
        return;
    const long long b0 = lc * kScanChunk, b1 = std::min(b.g.nblocks, b0 + kScanChunk);
    for (long long k0 = b0; k0 < b1; k0 += 64) {
        const long long k = k0 + lane;
        const unsigned cnt = k < b1 ? b.counts[k] : 0u;
        unsigned long long m = __ballot(cnt != 0u);
        while (m) {
            const int j = __builtin_ctzll(m);
            m &= m - 1ULL;
            scatter_block<T>(static_cast<const T *>(b.x), b.g, b.codes, b.counts, offs + b.blk0,
                             partials + b.chunk0, static_cast<T *>(b.raw), b.raw_cap, b.status,
                             k0 + j);
        }
    }
}

// the model section of each field that carries one: the network of the
// field's dimensionality (models[ndim - 1], device)
__global__ void __launch_bounds__(256) k_batch_model(const BatchField *f, const pwrel_mlp *models)
{
    const BatchField &b = f[blockIdx.x];
    if (!b.model_dst)
        return;
    const unsigned *src = reinterpret_cast<const unsigned *>(models + (b.h.ndim - 1));
    unsigned *dst = static_cast<unsigned *>(b.model_dst);
    for (int i = threadIdx.x; i < (int)(sizeof(pwrel_mlp) / 4); i += blockDim.x)
        dst[i] = src[i];
}

__global__ void __launch_bounds__(256) k_batch_header(const BatchField *f)
{
    const BatchField &b = f[blockIdx.x];
    write_header(b.h, b.consts, b.n_raw, b.status, static_cast<pwrel_header *>(b.header),
                 b.out_size);
}

hipError_t launch_batch_back(const BatchField *d_fields, int nf, int dtype, long long nchunks,
                             long long nblocks, unsigned long long *offsets,
                             unsigned long long *partials, const pwrel_mlp *models,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_scan_local, dim3((unsigned)nchunks), dim3(256), 0, s, d_fields,
                       nf, offsets, partials);
    hipLaunchKernelGGL(k_batch_scan_partials, dim3(nf), dim3(1024), 0, s, d_fields, partials);
    (void)nblocks;
    const unsigned grid = (unsigned)((nchunks + 3) / 4);
    if (dtype == PWREL_F32)
        hipLaunchKernelGGL(k_batch_scatter<float>, dim3(grid), dim3(256), 0, s, d_fields, nf,
                           nchunks, offsets, partials);
    else
        hipLaunchKernelGGL(k_batch_scatter<double>, dim3(grid), dim3(256), 0, s, d_fields, nf,
                           nchunks, offsets, partials);
    if (models)
        hipLaunchKernelGGL(k_batch_model, dim3(nf), dim3(256), 0, s, d_fields, models);
    hipLaunchKernelGGL(k_batch_header, dim3(nf), dim3(256), 0, s, d_fields);
    return hipGetLastError();
}

}  // namespace pwrel
