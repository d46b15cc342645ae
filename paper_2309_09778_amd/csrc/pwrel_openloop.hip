// Open-loop mode: the paper's literal data selection (Sec. 4.4.1, 4.4.2),
// kept beside the codec as a measurement of why the codec predicts from
// grid-snapped values instead.  The compressor predicts every point from its
// neighbours' raw log-domain values (continuous grid coordinates), so every
// point is predicted independently; the decompressor can only predict from
// its own reconstructions, so its errors can accumulate and break the bound.
// The paper's controls against the drift: balance points (the first point of
// every block, codes outside the m-bit range, and deliberate ones after `gap`
// points of a block without one), m chosen by coverage (Sec. 4.3).
// Independent blocks: each block decodes from its own balance points.
//
// Kernels: coordinates of every value (FP64), codes of every point (one
// thread per point: prediction from raw coordinates, the coverage histogram
// of the prediction errors), the balance rule (one thread per block, in
// stream order), raw values by the codec's scan and scatter, decoding (one
// thread per block, points in stream order, reconstructed coordinates kept
// in a field-order scratch), and a check of the bound on every point.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "pwrel_internal.h"
#include "pwrel_kernels.h"

namespace pwrel {

struct OlState {
    double *T = nullptr;  // coordinates (field order): the encoder's, then the decoder's
    size_t T_cap = 0;
    unsigned long long *rep = nullptr;  // [0..17] histogram, [18] violations, [19] max rel bits
};

void ol_release(OlState *o)
{
    if (!o)
        return;
    if (o->T)
        (void)hipFree(o->T);
    if (o->rep)
        (void)hipFree(o->rep);
    delete o;
}

namespace {

constexpr int kOlRep = 24;

// continuous grid coordinate of x (the grid value before rounding)
__device__ __forceinline__ double ol_coord(double x, const DevConsts &c)
{
    if (x == 0.0)
        return (double)c.p_zero;
    if (x > 0.0)
        return (det_log2(x) + c.Lp) * c.r;
    return (det_log2(-x) + c.Ln) * c.r + (double)c.delta;
}

// zero / positive / negative by the nearest grid value, magnitude from the
// coordinate
__device__ __forceinline__ double ol_inverse(double t, const DevConsts &c)
{
    const double q = __builtin_rint(t);
    if (q <= (double)c.p_zero)
        return 0.0;
    if (q <= (double)c.b_sign)
        return det_exp2(t * c.w - c.Lp);
    return -det_exp2((t - (double)c.delta) * c.w - c.Ln);
}

struct OlArgs {
    const void *x;
    long long n[3];   // extents (leading 1 below the field's dimensionality)
    int bd[3];        // block edge per axis (1 on the missing ones)
    long long nb[3];
    long long N, nblocks;
    int D, mbits, gap, use_net;
    double eps;
    double *T;
    uint16_t *codes;
    uint32_t *counts;
    const DevConsts *consts;
    unsigned long long *rep;
    const unsigned long long *offs, *partials;
    const void *raw;
    void *xh;
    MlpW mlp;
    int H, K;
};

// FP32 network of the inputs u (fma order of the oracle: hidden units in
// order, inputs in order; output accumulated over the hidden units in order)
__device__ __forceinline__ float ol_net(const OlArgs &a, const float *u)
{
    float y = a.mlp.b2;
    for (int j = 0; j < a.H; ++j) {
        float z = a.mlp.b1[j];
        for (int k = 0; k < a.K; ++k)
            z = __builtin_fmaf(a.mlp.w1[j][k], u[k], z);
        const float h = z < 0.0f ? z * a.mlp.alpha : z;
        y = __builtin_fmaf(a.mlp.v[j], h, y);
    }
    return y;
}

// prediction of point (z, y, x) from the coordinates T of its block's
// neighbours (bit 0 of o: one step back along x, bit 1 along y, bit 2 along z)
__device__ __forceinline__ double ol_predict(const OlArgs &a, const double *T, long long z,
                                             long long y, long long x)
{
    const int no = (1 << a.D) - 1;
    double nv[8];
    int avail = 0;
    for (int o = 1; o <= no; ++o) {
        const long long qx = x - (o & 1), qy = y - ((o >> 1) & 1), qz = z - ((o >> 2) & 1);
        const bool ok = qx >= 0 && qy >= 0 && qz >= 0 && qx / a.bd[2] == x / a.bd[2] &&
                        qy / a.bd[1] == y / a.bd[1] && qz / a.bd[0] == z / a.bd[0];
        nv[o] = ok ? T[(qz * a.n[1] + qy) * a.n[2] + qx] : 0.0;
        avail |= ok ? (1 << o) : 0;
    }
    if (a.use_net && avail == (1 << (no + 1)) - 2) {
        float u[6];
        for (int k = 0; k < a.K; ++k)
            u[k] = (float)(nv[k + 2] - nv[1]);
        return nv[1] + (double)ol_net(a, u);
    }
    double s = 0.0;
    for (int o = 1; o <= no; ++o)
        if (avail & (1 << o))
            s = (__builtin_popcount((unsigned)o) & 1) ? s + nv[o] : s - nv[o];
    return s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_ol_coords(OlArgs a)
{
    const DevConsts c = *a.consts;
    const T *x = static_cast<const T *>(a.x);
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < a.N; i += (long long)gridDim.x * 256)
        a.T[i] = ol_coord((double)x[i], c);
}

// stream position of field point (z, y, x)
__device__ __forceinline__ long long ol_pos(const OlArgs &a, long long z, long long y, long long x)
{
    const BlockGeo q = block_geo3(z / a.bd[0], y / a.bd[1], x / a.bd[2], a.n, a.bd[0], a.bd[1],
                                  a.bd[2]);
    const long long lz = z - q.bz * a.bd[0], ly = y - q.by * a.bd[1], lx = x - q.bx * a.bd[2];
    return q.start + (lz * q.ey + ly) * q.ex + lx;
}

// codes before the balance rule (0 = out of the m-bit range) and the
// histogram of the bits each prediction error needs
__global__ void __launch_bounds__(256) k_ol_codes(OlArgs a)
{
    __shared__ unsigned long long hs[18];
    if (threadIdx.x < 18)
        hs[threadIdx.x] = 0ULL;
    __syncthreads();
    const double half = (double)(1 << (a.mbits - 1));
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < a.N; i += (long long)gridDim.x * 256) {
        const long long x = i % a.n[2], y = (i / a.n[2]) % a.n[1], z = i / (a.n[1] * a.n[2]);
        const double cq = __builtin_rint(ol_predict(a, a.T, z, y, x) - a.T[i]);
        const double m = __builtin_fabs(cq);
        int need = 17;
        for (int b = 1; b <= 16; ++b)
            if (m < (double)(1 << (b - 1))) {
                need = b;
                break;
            }
        atomicAdd(&hs[need], 1ULL);
        a.codes[ol_pos(a, z, y, x)] = m < half ? (uint16_t)(cq + half) : (uint16_t)0;
    }
    __syncthreads();
    if (threadIdx.x < 18 && hs[threadIdx.x])
        atomicAdd(&a.rep[threadIdx.x], hs[threadIdx.x]);
}

// balance rule of each block, in stream order: its first point, codes out of
// range, and a deliberate one after `gap` points without one; balance points
// counted per block
__global__ void __launch_bounds__(256) k_ol_balance(OlArgs a)
{
    const long long b = blockIdx.x * 256LL + threadIdx.x;
    if (b >= a.nblocks)
        return;
    const long long bx = b % a.nb[2], by = (b / a.nb[2]) % a.nb[1], bz = b / (a.nb[1] * a.nb[2]);
    const BlockGeo q = block_geo3(bz, by, bx, a.n, a.bd[0], a.bd[1], a.bd[2]);
    const long long sz = (long long)q.ez * q.ey * q.ex;
    long long since = 0;
    unsigned cnt = 0;
    for (long long k = 0; k < sz; ++k) {
        uint16_t cd = a.codes[q.start + k];
        bool bal = k == 0 || cd == 0;
        if (!bal && a.gap > 0 && since + 1 >= a.gap)
            bal = true;
        since = bal ? 0 : since + 1;
        if (bal) {
            if (cd != 0)
                a.codes[q.start + k] = 0;
            ++cnt;
        }
    }
    a.counts[b] = cnt;
}

// decoding: one thread per block, points in stream order
template <typename T>
__global__ void __launch_bounds__(256) k_ol_decode(OlArgs a)
{
    const long long b = blockIdx.x * 256LL + threadIdx.x;
    if (b >= a.nblocks)
        return;
    const DevConsts c = *a.consts;
    const double half = (double)(1 << (a.mbits - 1));
    const long long bx = b % a.nb[2], by = (b / a.nb[2]) % a.nb[1], bz = b / (a.nb[1] * a.nb[2]);
    const BlockGeo q = block_geo3(bz, by, bx, a.n, a.bd[0], a.bd[1], a.bd[2]);
    unsigned long long kr = a.offs[b] + a.partials[b / kScanChunk];
    const T *raw = static_cast<const T *>(a.raw);
    T *xh = static_cast<T *>(a.xh);
    long long pos = q.start;
    for (int lz = 0; lz < q.ez; ++lz)
        for (int ly = 0; ly < q.ey; ++ly)
            for (int lx = 0; lx < q.ex; ++lx, ++pos) {
                const long long z = bz * a.bd[0] + lz, y = by * a.bd[1] + ly,
                                x = bx * a.bd[2] + lx;
                const long long i = (z * a.n[1] + y) * a.n[2] + x;
                const uint16_t cd = a.codes[pos];
                if (cd == 0) {
                    const T v = raw[kr++];
                    xh[i] = v;
                    a.T[i] = ol_coord((double)v, c);
                } else {
                    const double t = ol_predict(a, a.T, z, y, x) - ((double)cd - half);
                    a.T[i] = t;
                    xh[i] = (T)ol_inverse(t, c);
                }
            }
}

// the bound on every point (sign and zero included) and the largest relative
// error over the non-zero values
template <typename T>
__global__ void __launch_bounds__(256) k_ol_check(OlArgs a)
{
    const T *x = static_cast<const T *>(a.x);
    const T *xh = static_cast<const T *>(a.xh);
    unsigned long long bad = 0;
    double worst = 0.0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < a.N; i += (long long)gridDim.x * 256) {
        const double v = (double)x[i], h = (double)xh[i];
        bool ok;
        if (v == 0.0) {
            ok = h == 0.0;
        } else {
            const double d = __builtin_fabs(v - h);
            ok = h != 0.0 && __builtin_signbit(v) == __builtin_signbit(h) &&
                 d <= a.eps * __builtin_fabs(v);
            const double rel = d / __builtin_fabs(v);
            worst = rel > worst ? rel : worst;  // NaN never enters
        }
        bad += ok ? 0ULL : 1ULL;
    }
    for (int o = 32; o > 0; o >>= 1) {
        bad += (unsigned long long)__shfl_xor((long long)bad, o, 64);
        const double w = __shfl_xor(worst, o, 64);
        worst = w > worst ? w : worst;
    }
    if ((threadIdx.x & 63) == 0) {
        if (bad)
            atomicAdd(&a.rep[18], bad);
        atomicMax(&a.rep[19], (unsigned long long)__double_as_longlong(worst));
    }
}

__global__ void k_ol_zero(unsigned long long *p, int n)
{
    if (threadIdx.x < n)
        p[threadIdx.x] = 0ULL;
}

struct OlDeviceGuard {
    int prev = -1;
    explicit OlDeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~OlDeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

unsigned ol_grid(long long work)
{
    return (unsigned)std::max<long long>(1, std::min<long long>((work + 255) / 256, 16384));
}

int choose_m(const unsigned long long *hist, double eps)
{
    // the oracle's rule: coverage closest to 50% below a 1.5% bound, 80% from
    // 1.5% up; ties to the smaller m
    unsigned long long n = 0;
    for (int j = 0; j < 18; ++j)
        n += hist[j];
    const double target = eps < 0.015 ? 0.5 : 0.8;
    int best = 2;
    double bestd = 1e300;
    unsigned long long cum = 0;
    for (int m = 1; m <= 16; ++m) {
        cum += hist[m];
        if (m < 2)
            continue;
        const double cov = n ? (double)cum / (double)n : 1.0;
        const double d = cov > target ? cov - target : target - cov;
        if (d < bestd) {
            bestd = d;
            best = m;
        }
    }
    return best;
}

}  // namespace
}  // namespace pwrel

using namespace pwrel;

extern "C" int pwrel_openloop(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                              int dtype, double eps, int block_size, const pwrel_mlp *model,
                              int mbits, int gap, uint16_t *d_codes, uint32_t *d_counts,
                              void *d_raw, uint64_t raw_capacity, void *d_xhat,
                              pwrel_openloop_report *report, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (pwrel_check_args(dims, ndim, dtype, eps, block_size) != PWREL_OK)
        return api_fail(ctx, PWREL_EINVAL, "bad dims/ndim/dtype/bound/block size");
    if (!d_field || !d_codes || !d_counts || !d_xhat || !report || (raw_capacity && !d_raw))
        return api_fail(ctx, PWREL_EINVAL, "NULL argument");
    if (mbits != 0 && (mbits < 2 || mbits > 16))
        return api_fail(ctx, PWREL_EINVAL, "mbits must be 2..16, or 0 (chosen by coverage)");
    if (gap < 0)
        return api_fail(ctx, PWREL_EINVAL, "gap must be >= 0");
    if (model) {
        if (const char *why = model_problem(model, ndim))
            return api_fail(ctx, PWREL_EINVAL, why);
    }
    Geom g;
    make_geom(dims, ndim, dtype, block_size, g);
    OlArgs a{};
    a.x = d_field;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bd[d] = g.bd[d];
        a.nb[d] = g.nb[d];
    }
    a.N = g.N;
    a.nblocks = g.nblocks;
    a.D = g.D;
    a.gap = gap;
    a.eps = eps;
    a.use_net = model ? 1 : 0;
    a.mlp = pack_mlp(model);
    a.H = model ? model->hidden : 0;
    a.K = model ? model->inputs : 0;
    a.codes = d_codes;
    a.counts = d_counts;
    a.raw = d_raw;
    a.xh = d_xhat;

    OlDeviceGuard guard(api_device(ctx));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    OlState *&st = api_ol_state(ctx);
    if (!st && !(st = new (std::nothrow) OlState()))
        return api_fail(ctx, PWREL_ENOMEM, "open-loop state allocation failed");
    hipError_t e = hipSuccess;
    if (st->T_cap < (size_t)g.N) {
        if (st->T)
            (void)hipFree(st->T);
        st->T = nullptr;
        st->T_cap = 0;
        if ((e = hipMalloc(reinterpret_cast<void **>(&st->T), (size_t)g.N * sizeof(double))) !=
            hipSuccess)
            return api_fail(ctx, PWREL_ENOMEM, "open-loop coordinate allocation failed");
        st->T_cap = (size_t)g.N;
    }
    if (!st->rep &&
        (e = hipMalloc(reinterpret_cast<void **>(&st->rep), kOlRep * sizeof(unsigned long long))) !=
            hipSuccess)
        return api_fail(ctx, PWREL_ENOMEM, "open-loop report allocation failed");
    int rc = api_ensure_scan(ctx, g);
    if (rc != PWREL_OK)
        return rc;
    Workspace &ws = api_ws(ctx);
    a.T = st->T;
    a.rep = st->rep;
    a.consts = ws.consts;
    a.offs = ws.offsets;
    a.partials = ws.partials;

    // statistics and constants (Eq. 8-12), then the coordinates
    if ((e = launch_reset(ws, s)) != hipSuccess || (e = launch_stats(d_field, g, ws, s)) != hipSuccess ||
        (e = launch_consts(g, eps, ws, s)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "open-loop constants");
    hipLaunchKernelGGL(k_ol_zero, dim3(1), dim3(64), 0, s, st->rep, kOlRep);
    if (dtype == PWREL_F32)
        hipLaunchKernelGGL(k_ol_coords<float>, dim3(ol_grid(g.N)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_ol_coords<double>, dim3(ol_grid(g.N)), dim3(256), 0, s, a);
    int status = PWREL_OK;
    if ((e = hipMemcpyAsync(&status, ws.status, sizeof status, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "open-loop status copy");
    if (status != PWREL_OK)
        return api_status(ctx, status);
    unsigned long long hist[kOlRep];
    a.mbits = mbits ? mbits : 16;
    hipLaunchKernelGGL(k_ol_codes, dim3(ol_grid(g.N)), dim3(256), 0, s, a);
    if (mbits == 0) {
        // m by coverage: the histogram of the prediction errors, then the codes again
        if ((e = hipMemcpyAsync(hist, st->rep, sizeof hist, hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return api_fail(ctx, PWREL_EHIP, "open-loop histogram copy");
        a.mbits = choose_m(hist, eps);
        hipLaunchKernelGGL(k_ol_zero, dim3(1), dim3(64), 0, s, st->rep, kOlRep);
        hipLaunchKernelGGL(k_ol_codes, dim3(ol_grid(g.N)), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_ol_balance, dim3((unsigned)((g.nblocks + 255) / 256)), dim3(256), 0, s, a);
    if ((e = launch_scan(d_counts, g, ws, s)) != hipSuccess ||
        (e = launch_scatter(d_field, g, d_codes, d_counts, ws, d_raw, raw_capacity, s)) !=
            hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "open-loop raw values");
    if (dtype == PWREL_F32) {
        hipLaunchKernelGGL(k_ol_decode<float>, dim3((unsigned)((g.nblocks + 255) / 256)), dim3(256),
                           0, s, a);
        hipLaunchKernelGGL(k_ol_check<float>, dim3(ol_grid(g.N)), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_ol_decode<double>, dim3((unsigned)((g.nblocks + 255) / 256)),
                           dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_ol_check<double>, dim3(ol_grid(g.N)), dim3(256), 0, s, a);
    }
    unsigned long long nr = 0;
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(hist, st->rep, sizeof hist, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&nr, ws.n_raw, sizeof nr, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&status, ws.status, sizeof status, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "open-loop report copy");
    if (status != PWREL_OK)
        return api_status(ctx, status);
    std::memset(report, 0, sizeof *report);
    report->n_raw = nr;
    report->violations = hist[18];
    double worst;
    std::memcpy(&worst, &hist[19], sizeof worst);
    report->max_rel_error = worst;
    for (int j = 0; j < 18; ++j)
        report->hist[j] = hist[j];
    report->mbits = a.mbits;
    report->gap = gap;
    return PWREL_OK;
}
