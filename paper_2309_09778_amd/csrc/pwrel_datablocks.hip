// Data blocks (Sec. 5: the stream carries factor_pos and factor_neg for its
// data block; Algorithm 1 computes them from the extreme values of its input).
//
// A 3-D FP32 field is split into data blocks, sub-volumes of edge `sub` (a
// multiple of the 8^3 prediction block; the last along an axis clipped), in
// raster order.  Each one is compressed into its own stream with its own
// statistics, factors and constants: exactly the stream pwrel_compress writes
// for that sub-volume alone.  Compression: one gather kernel copies every
// data block, contiguous in C order, into the context's staging, back to
// back; one batched compression then runs over all of them.  Decompression:
// each stream is decoded into the staging and one scatter kernel puts the
// sub-volumes back in place.
#include <algorithm>
#include <array>
#include <vector>

#include "pwrel_internal.h"

namespace pwrel {
namespace {

struct SubGeo {
    long long n[3];   // field dims
    long long ns[3];  // data blocks per axis
    int sub;          // data-block edge
};

// field index i <-> (data block, index inside its contiguous copy)
__device__ __forceinline__ long long stage_index(const SubGeo &g, long long i,
                                                 const unsigned long long *offs)
{
    const long long x = i % g.n[2], y = (i / g.n[2]) % g.n[1], z = i / (g.n[1] * g.n[2]);
    const long long bz = z / g.sub, by = y / g.sub, bx = x / g.sub;
    const long long lz = z - bz * g.sub, ly = y - by * g.sub, lx = x - bx * g.sub;
    const long long ey = min((long long)g.sub, g.n[1] - by * g.sub);
    const long long ex = min((long long)g.sub, g.n[2] - bx * g.sub);
    const long long db = (bz * g.ns[1] + by) * g.ns[2] + bx;
    return (long long)offs[db] + (lz * ey + ly) * ex + lx;
}

// consecutive threads take consecutive field values (coalesced reads of the
// gather, coalesced writes of the scatter), each a run of a data block's row
__global__ void k_gather_sub(const float *__restrict__ x, SubGeo g,
                             const unsigned long long *__restrict__ offs,
                             float *__restrict__ stage, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        stage[stage_index(g, i, offs)] = x[i];
}

__global__ void k_scatter_sub(const float *__restrict__ stage, SubGeo g,
                              const unsigned long long *__restrict__ offs, float *__restrict__ x,
                              long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = stage[stage_index(g, i, offs)];
}

// the data blocks of a field: extents and offsets in the staging (host)
struct SubPlan {
    SubGeo g{};
    std::vector<unsigned long long> offs;
    std::vector<std::array<uint64_t, 3>> dims;
    long long n = 0;
};

bool plan_of(const uint64_t *dims, int sub, SubPlan &p)
{
    if (sub < 8 || sub % 8 != 0)
        return false;
    p.g.sub = sub;
    p.n = 1;
    for (int d = 0; d < 3; ++d) {
        if (dims[d] < 1)
            return false;
        p.g.n[d] = (long long)dims[d];
        p.g.ns[d] = (p.g.n[d] + sub - 1) / sub;
        p.n *= p.g.n[d];
    }
    unsigned long long off = 0;
    for (long long bz = 0; bz < p.g.ns[0]; ++bz)
        for (long long by = 0; by < p.g.ns[1]; ++by)
            for (long long bx = 0; bx < p.g.ns[2]; ++bx) {
                const uint64_t ez = (uint64_t)std::min<long long>(sub, p.g.n[0] - bz * sub);
                const uint64_t ey = (uint64_t)std::min<long long>(sub, p.g.n[1] - by * sub);
                const uint64_t ex = (uint64_t)std::min<long long>(sub, p.g.n[2] - bx * sub);
                p.offs.push_back(off);
                p.dims.push_back({ez, ey, ex});
                off += ez * ey * ex;
            }
    return true;
}

unsigned grid_of(long long n)
{
    return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 65536));
}

struct Guard {
    int prev = -1;
    explicit Guard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~Guard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

}  // namespace
}  // namespace pwrel

using namespace pwrel;

extern "C" int pwrel_compress_datablocks(pwrel_ctx *ctx, const float *d_field,
                                         const uint64_t *dims, double rel_error_bound, int sub,
                                         const pwrel_mlp *model, const pwrel_options *opt,
                                         void *d_out, uint64_t out_stride, uint64_t *d_sizes,
                                         uint64_t *n_sub_out, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!d_field || !dims || !d_out || !d_sizes || !n_sub_out)
        return api_fail(ctx, PWREL_EINVAL, "NULL argument");
    SubPlan p;
    if (!plan_of(dims, sub, p))
        return api_fail(ctx, PWREL_EINVAL, "data-block edge must be a positive multiple of 8");
    if (out_stride % 256 != 0 || (reinterpret_cast<uintptr_t>(d_out) & 15))
        return api_fail(ctx, PWREL_EINVAL,
                        "the stream stride must be a multiple of 256 and d_out 16-byte aligned");
    const size_t nsub = p.offs.size();
    Guard guard(api_device(ctx));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *stage = nullptr;
    unsigned long long *d_offs = nullptr;
    hipError_t e = api_dstage(ctx, (size_t)p.n, nsub, &stage, &d_offs);
    if (e != hipSuccess)
        return api_fail(ctx, PWREL_ENOMEM, "data-block staging allocation failed");
    std::vector<pwrel_field_desc> f(nsub);
    unsigned char *out = static_cast<unsigned char *>(d_out);
    for (size_t i = 0; i < nsub; ++i) {
        f[i].d_field = stage + p.offs[i];
        for (int d = 0; d < 3; ++d)
            f[i].dims[d] = p.dims[i][d];
        f[i].ndim = 3;
        f[i].reserved = 0;
        f[i].d_out = out + i * out_stride;
        f[i].out_capacity = out_stride;
    }
    // the offsets go up before the gather reads them; the field table of the
    // batched call is built from host values only
    if ((e = hipMemcpyAsync(d_offs, p.offs.data(), nsub * sizeof(unsigned long long),
                            hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "data-block offsets copy");
    hipLaunchKernelGGL(k_gather_sub, dim3(grid_of(p.n)), dim3(256), 0, s, d_field, p.g, d_offs,
                       stage, p.n);
    if ((e = hipGetLastError()) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "data-block gather");
    const int block[3] = {0, 16, 8};
    const pwrel_mlp *models[3] = {nullptr, nullptr, model};
    const int st = pwrel_compress_batch(ctx, (int)nsub, f.data(), PWREL_F32, rel_error_bound,
                                        block, models, opt, d_sizes, stream);
    if (st != PWREL_OK)
        return st;
    *n_sub_out = nsub;
    return PWREL_OK;
}

extern "C" int pwrel_decompress_datablocks(pwrel_ctx *ctx, const void *d_in, uint64_t in_stride,
                                           const uint64_t *sizes, float *d_field,
                                           const uint64_t *dims, int sub, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!d_in || !sizes || !d_field || !dims)
        return api_fail(ctx, PWREL_EINVAL, "NULL argument");
    SubPlan p;
    if (!plan_of(dims, sub, p))
        return api_fail(ctx, PWREL_EINVAL, "data-block edge must be a positive multiple of 8");
    if (in_stride % 256 != 0 || (reinterpret_cast<uintptr_t>(d_in) & 15))
        return api_fail(ctx, PWREL_EINVAL,
                        "the stream stride must be a multiple of 256 and d_in 16-byte aligned");
    const size_t nsub = p.offs.size();
    Guard guard(api_device(ctx));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *stage = nullptr;
    unsigned long long *d_offs = nullptr;
    hipError_t e = api_dstage(ctx, (size_t)p.n, nsub, &stage, &d_offs);
    if (e != hipSuccess)
        return api_fail(ctx, PWREL_ENOMEM, "data-block staging allocation failed");
    if ((e = hipMemcpyAsync(d_offs, p.offs.data(), nsub * sizeof(unsigned long long),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "data-block offsets copy");
    const unsigned char *in = static_cast<const unsigned char *>(d_in);
    std::vector<float *> outs(nsub);
    std::vector<std::array<uint64_t, 3>> dd(p.dims);
    for (size_t i = 0; i < nsub; ++i)
        outs[i] = stage + p.offs[i];
    // every stream's kernels queued back to back (one header copy, one status read)
    const int st = api_decompress_many(ctx, in, in_stride, sizes, nsub, outs.data(),
                                       reinterpret_cast<const uint64_t(*)[3]>(dd.data()), s);
    if (st != PWREL_OK)
        return st;
    hipLaunchKernelGGL(k_scatter_sub, dim3(grid_of(p.n)), dim3(256), 0, s, stage, p.g, d_offs,
                       d_field, p.n);
    if ((e = hipGetLastError()) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "data-block scatter");
    return PWREL_OK;
}
