// pwrel_compress_batch: many FP32 fields compressed by one fixed sequence of
// launches, whatever their number and shapes.  Each field gets exactly the
// stream pwrel_compress would write for it (Algorithm 1 per field: its own
// statistics and constants, Eq. 8-12, its own codes, counts, raw values and
// header); only the work is pooled.  Tiles of every field of one class
// (dimensionality and block) form the work list of one persistent compression
// launch, and the per-field stages (statistics, constants, grid entries,
// scan, raw scatter, model, header) each run as one launch over a field
// table that the kernels search by their workgroup or block number.
//
// The host builds the field table once per distinct request (fields, bound,
// blocks, models, options, size array) and copies it to the device through
// pinned staging memory.  A repeated request launches kernels only: no host
// work, no allocation, no synchronisation, so such a call can be captured in
// a HIP graph and replayed.  The per-field sizes go to a device array.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pwrel_internal.h"
#include "pwrel_kernels.h"

namespace pwrel {

namespace {

template <typename P>
hipError_t grow_dev(P *&ptr, size_t &cap, size_t need)
{
    if (need <= cap && ptr)
        return hipSuccess;
    if (ptr)
        (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    const hipError_t e = hipMalloc(reinterpret_cast<void **>(&ptr), std::max<size_t>(need, 1) * sizeof(P));
    if (e == hipSuccess)
        cap = std::max<size_t>(need, 1);
    return e;
}

struct DeviceGuard_ {
    int prev = -1;
    explicit DeviceGuard_(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard_()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

constexpr size_t a256(size_t v) { return (v + 255u) & ~size_t(255u); }

// statistics records of a field: the single-field path's part count
long long stat_parts(long long N)
{
    long long g = (N + 256 * 16 - 1) / (256 * 16);
    return std::max(1LL, std::min<long long>(g, kStatParts));
}

// classes of the batch: (3-D, block 8) and (2-D, block 16)
constexpr int kClasses = 2;
int class_of(int ndim) { return ndim == 3 ? 0 : 1; }

struct Request {
    std::vector<pwrel_field_desc> fields;
    int dtype = 0;
    double eps = 0.0;
    int block[3] = {};
    pwrel_mlp models[3] = {};
    int has_model[3] = {};
    pwrel_options opt{};
    uint64_t *sizes = nullptr;
    int variant[2] = {};  // tile shape variant of each class

    bool same(const Request &o) const
    {
        if (fields.size() != o.fields.size() || dtype != o.dtype || eps != o.eps ||
            sizes != o.sizes || std::memcmp(block, o.block, sizeof block) ||
            std::memcmp(variant, o.variant, sizeof variant) ||
            std::memcmp(has_model, o.has_model, sizeof has_model) ||
            std::memcmp(&opt, &o.opt, sizeof opt))
            return false;
        for (int d = 0; d < 3; ++d)
            if (has_model[d] && std::memcmp(&models[d], &o.models[d], sizeof(pwrel_mlp)))
                return false;
        return fields.empty() ||
               std::memcmp(fields.data(), o.fields.data(),
                           fields.size() * sizeof(pwrel_field_desc)) == 0;
    }
};

}  // namespace

// Per-context state of the batched path: device workspace, the device field
// table and its pinned staging copy, and the prepared request.
struct BatchState {
    DevStats *records = nullptr;
    size_t records_cap = 0;
    DevConsts *consts = nullptr;
    size_t consts_cap = 0;
    int *status = nullptr;
    size_t status_cap = 0;
    unsigned long long *nraw = nullptr;
    size_t nraw_cap = 0;
    int *pgrid = nullptr;
    size_t pgrid_cap = 0;
    unsigned long long *offs = nullptr;
    size_t offs_cap = 0;
    unsigned long long *parts = nullptr;
    size_t parts_cap = 0;
    unsigned char *dtab = nullptr;
    size_t dtab_cap = 0;
    unsigned char *htab = nullptr;  // pinned
    size_t htab_cap = 0;
    hipEvent_t ev = nullptr;  // the last table copy
    hipStream_t prep_stream = nullptr;
    bool ready = false;
    int variant[kClasses] = {};  // tile shape variant of each class (set or tuned)
    hipEvent_t tev[kClasses][2] = {};  // around each class's compression launch (tuning)
    bool timing = false;
    Request req;
    // the prepared launches
    int nf = 0;
    long long nparts = 0, nechunks = 0, nchunks = 0, nblocks = 0;
    size_t off_fd[kClasses] = {}, off_models = 0;
    int nclass[kClasses] = {};
    long long ntiles[kClasses] = {};
    Geom geo[kClasses];
    Tile tile[kClasses];
};

void batch_release(BatchState *b)
{
    if (!b)
        return;
    void *dev[] = {b->records, b->consts, b->status, b->nraw,
                   b->pgrid,   b->offs,   b->parts,  b->dtab};
    for (void *p : dev)
        if (p)
            (void)hipFree(p);
    if (b->htab)
        (void)hipHostFree(b->htab);
    if (b->ev)
        (void)hipEventDestroy(b->ev);
    for (auto &pr : b->tev)
        for (hipEvent_t e : pr)
            if (e)
                (void)hipEventDestroy(e);
    delete b;
}

namespace {

// The request's checks (host only).  Returns PWREL_OK or an error with message.
int check_request(pwrel_ctx *ctx, const Request &r)
{
    const size_t n = r.fields.size();
    if (r.dtype != PWREL_F32)
        return api_fail(ctx, PWREL_EINVAL, "batched compression takes FP32 fields");
    if (r.opt.entropy)
        return api_fail(ctx, PWREL_EINVAL, "batched compression writes 16-bit codes (entropy = 0)");
    if (r.opt.judge && !r.opt.use_net)
        return api_fail(ctx, PWREL_EINVAL, "the per-block judge needs a network (use_net)");
    if (!r.sizes)
        return api_fail(ctx, PWREL_EINVAL, "NULL size array");
    for (size_t i = 0; i < n; ++i) {
        const pwrel_field_desc &f = r.fields[i];
        const std::string at = "field " + std::to_string(i) + ": ";
        if (f.ndim != 2 && f.ndim != 3)
            return api_fail(ctx, PWREL_EINVAL, (at + "batched fields are 2-D or 3-D").c_str());
        const int B = r.block[f.ndim - 1];
        if (!batch_shape(f.ndim, B))
            return api_fail(ctx, PWREL_EINVAL,
                            (at + "block size must be 8 (3-D) or 16 (2-D)").c_str());
        if (pwrel_check_args(f.dims, f.ndim, r.dtype, r.eps, B) != PWREL_OK)
            return api_fail(ctx, PWREL_EINVAL, (at + "bad dims or bound").c_str());
        if (!f.d_field || !f.d_out)
            return api_fail(ctx, PWREL_EINVAL, (at + "NULL field or output").c_str());
        if (reinterpret_cast<uintptr_t>(f.d_out) & 15)
            return api_fail(ctx, PWREL_EINVAL, (at + "output not 16-byte aligned").c_str());
        Geom g;
        make_geom(f.dims, f.ndim, r.dtype, B, g);
        const Layout L = layout_for(g, flags_of(r.opt));
        if (f.out_capacity < L.off[4])
            return api_fail(ctx, PWREL_ENOSPC,
                            (at + "output capacity below header + codes").c_str());
        if (r.opt.use_net) {
            if (!r.has_model[f.ndim - 1])
                return api_fail(ctx, PWREL_EINVAL, (at + "no model for its dimensionality").c_str());
            if (const char *why = model_problem(&r.models[f.ndim - 1], f.ndim))
                return api_fail(ctx, PWREL_EINVAL, (at + why).c_str());
        }
    }
    return PWREL_OK;
}

// Builds the field table of request r into the state's workspace and pinned
// staging memory and queues its copy to the device on s.
int prepare(pwrel_ctx *ctx, BatchState &b, const Request &r, hipStream_t s)
{
    const int nf = (int)r.fields.size();
    const int flags = flags_of(r.opt);
    std::vector<Geom> geo((size_t)nf);
    std::vector<Tile> til((size_t)nf);
    long long nparts = 0, nechunks = 0, nchunks = 0, nblocks = 0, ngrid = 0;
    int nclass[kClasses] = {};
    for (int i = 0; i < nf; ++i) {
        const pwrel_field_desc &f = r.fields[(size_t)i];
        make_geom(f.dims, f.ndim, r.dtype, r.block[f.ndim - 1], geo[(size_t)i]);
        const Geom &g = geo[(size_t)i];
        Tile &t = til[(size_t)i];
        if (!variant_shape(g.D, g.B, r.variant[class_of(f.ndim)], t.t))
            return api_fail(ctx, PWREL_EINVAL, "no such batched tile shape");
        t.ntiles = 1;
        for (int d = 0; d < 3; ++d) {
            t.nt[d] = (g.n[d] + t.t[d] - 1) / t.t[d];
            t.ntiles *= t.nt[d];
        }
        nparts += stat_parts(g.N);
        nechunks += (g.N + kEntryChunk - 1) / kEntryChunk;
        nchunks += (g.nblocks + kScanChunk - 1) / kScanChunk;
        nblocks += g.nblocks;
        ngrid += (g.N + 63) / 64 * 64;
        ++nclass[class_of(f.ndim)];
    }
    hipError_t e;
    if ((e = grow_dev(b.records, b.records_cap, (size_t)nparts)) != hipSuccess ||
        (e = grow_dev(b.consts, b.consts_cap, (size_t)nf)) != hipSuccess ||
        (e = grow_dev(b.status, b.status_cap, (size_t)nf)) != hipSuccess ||
        (e = grow_dev(b.nraw, b.nraw_cap, (size_t)nf)) != hipSuccess ||
        (e = grow_dev(b.pgrid, b.pgrid_cap, (size_t)ngrid)) != hipSuccess ||
        (e = grow_dev(b.offs, b.offs_cap, (size_t)nblocks)) != hipSuccess ||
        (e = grow_dev(b.parts, b.parts_cap, (size_t)nchunks)) != hipSuccess)
        return api_fail(ctx, PWREL_ENOMEM, "batch workspace allocation failed");

    // table layout: [BatchField nf] [FieldDesc of class 0] [.. class 1] [models 3]
    size_t off = a256((size_t)nf * sizeof(BatchField));
    size_t off_fd[kClasses];
    for (int k = 0; k < kClasses; ++k) {
        off_fd[k] = off;
        off = a256(off + (size_t)nclass[k] * sizeof(FieldDesc));
    }
    const size_t off_models = off;
    const size_t bytes = off + 3 * sizeof(pwrel_mlp);
    if ((e = grow_dev(b.dtab, b.dtab_cap, bytes)) != hipSuccess)
        return api_fail(ctx, PWREL_ENOMEM, "batch table allocation failed");
    // the previous table copy must be done before its staging is rewritten
    if (b.ev && (e = hipEventSynchronize(b.ev)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "batch table event");
    if (b.htab_cap < bytes) {
        if (b.htab)
            (void)hipHostFree(b.htab);
        b.htab = nullptr;
        b.htab_cap = 0;
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&b.htab), bytes, 0)) != hipSuccess)
            return api_fail(ctx, PWREL_ENOMEM, "batch staging allocation failed");
        b.htab_cap = bytes;
    }
    if (!b.ev && (e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "batch event creation failed");

    std::memset(b.htab, 0, bytes);
    BatchField *bf = reinterpret_cast<BatchField *>(b.htab);
    FieldDesc *fd[kClasses];
    for (int k = 0; k < kClasses; ++k)
        fd[k] = reinterpret_cast<FieldDesc *>(b.htab + off_fd[k]);
    pwrel_mlp *models = reinterpret_cast<pwrel_mlp *>(b.htab + off_models);
    for (int d = 0; d < 3; ++d)
        if (r.has_model[d])
            models[d] = r.models[d];

    long long part0 = 0, echunk0 = 0, chunk0 = 0, blk0 = 0, grid0 = 0;
    long long tile0[kClasses] = {};
    int ci[kClasses] = {};
    const size_t tsize = 4;
    for (int i = 0; i < nf; ++i) {
        const pwrel_field_desc &f = r.fields[(size_t)i];
        const Geom &g = geo[(size_t)i];
        const Tile &t = til[(size_t)i];
        const Layout L = layout_for(g, flags);
        unsigned char *out = static_cast<unsigned char *>(f.d_out);
        BatchField &q = bf[i];
        q.x = f.d_field;
        q.vec = (reinterpret_cast<uintptr_t>(f.d_field) & 15u) == 0 ? 1 : 0;
        for (int d = 0; d < 3; ++d) {
            q.g.n[d] = g.n[d];
            q.g.bd[d] = g.bd[d];
            q.g.nb[d] = g.nb[d];
        }
        q.g.nblocks = g.nblocks;
        q.N = g.N;
        q.eps = r.eps;
        q.part0 = part0;
        q.nparts = stat_parts(g.N);
        q.chunk0 = chunk0;
        q.nchunks = (g.nblocks + kScanChunk - 1) / kScanChunk;
        q.blk0 = blk0;
        q.echunk0 = echunk0;
        q.codes = reinterpret_cast<uint16_t *>(out + L.off[3]);
        q.counts = reinterpret_cast<uint32_t *>(out + L.off[2]);
        q.bflags = (flags & PWREL_HF_JUDGE) ? out + L.off[1] : nullptr;
        q.raw = out + L.off[4];
        q.raw_cap = (f.out_capacity - L.off[4]) / tsize;
        q.model_dst = (flags & PWREL_HF_NET) ? out + L.off[0] : nullptr;
        q.header = out;
        q.out_size = reinterpret_cast<unsigned long long *>(r.sizes + i);
        q.pgrid = b.pgrid + grid0;
        q.consts = b.consts + i;
        q.status = b.status + i;
        q.n_raw = b.nraw + i;
        q.h = make_header_args(g, flags, L.off, f.out_capacity, true, nullptr);

        const int k = class_of(f.ndim);
        FieldDesc &c = fd[k][ci[k]++];
        c.x = f.d_field;
        c.pfield = q.pgrid;
        for (int d = 0; d < 3; ++d) {
            c.n[d] = g.n[d];
            c.nb[d] = g.nb[d];
            c.nt[d] = t.nt[d];
        }
        c.tile0 = tile0[k];
        c.codes = q.codes;
        c.counts = q.counts;
        c.bflags = q.bflags;
        c.consts = q.consts;
        c.status = q.status;
        tile0[k] += t.ntiles;
        b.geo[k] = g;
        b.tile[k] = t;

        part0 += q.nparts;
        echunk0 += (g.N + kEntryChunk - 1) / kEntryChunk;
        chunk0 += q.nchunks;
        blk0 += g.nblocks;
        grid0 += (g.N + 63) / 64 * 64;
    }
    if ((e = hipMemcpyAsync(b.dtab, b.htab, bytes, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipEventRecord(b.ev, s)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "batch table copy");
    b.prep_stream = s;
    b.nf = nf;
    b.nparts = nparts;
    b.nechunks = nechunks;
    b.nchunks = nchunks;
    b.nblocks = nblocks;
    for (int k = 0; k < kClasses; ++k) {
        b.off_fd[k] = off_fd[k];
        b.nclass[k] = nclass[k];
        b.ntiles[k] = tile0[k];
    }
    b.off_models = off_models;
    b.req = r;
    b.ready = true;
    return PWREL_OK;
}

// The launches of a prepared batch (no host work beyond the launches).
hipError_t launch_prepared(const BatchState &b, const Request &r, const long long *qtab,
                           int num_cus, hipStream_t s)
{
    const BatchField *bf = reinterpret_cast<const BatchField *>(b.dtab);
    hipError_t e;
    if ((e = launch_batch_front(bf, b.nf, r.dtype, b.nparts, b.records, s)) != hipSuccess ||
        (e = launch_grid_entries_batch(bf, b.nf, b.nechunks, s)) != hipSuccess)
        return e;
    for (int k = 0; k < kClasses; ++k) {
        if (!b.nclass[k])
            continue;
        const int d = b.geo[k].D - 1;
        const FieldDesc *fd = reinterpret_cast<const FieldDesc *>(b.dtab + b.off_fd[k]);
        if (b.timing && (e = hipEventRecord(b.tev[k][0], s)) != hipSuccess)
            return e;
        if ((e = launch_compress_batch(fd, b.nclass[k], b.ntiles[k], b.geo[k], b.tile[k],
                                       r.variant[k], r.opt.use_net ? &r.models[d] : nullptr,
                                       r.opt, qtab, num_cus, s)) != hipSuccess)
            return e;
        if (b.timing && (e = hipEventRecord(b.tev[k][1], s)) != hipSuccess)
            return e;
    }
    const pwrel_mlp *models =
        r.opt.use_net ? reinterpret_cast<const pwrel_mlp *>(b.dtab + b.off_models) : nullptr;
    return launch_batch_back(bf, b.nf, r.dtype, b.nchunks, b.nblocks, b.offs, b.parts, models,
                             s);
}

}  // namespace

}  // namespace pwrel

namespace pwrel {
namespace {

// The request of a pwrel_compress_batch call (host copies of the arguments).
Request make_request(const pwrel_field_desc *fields, int n, int dtype, double eps,
                     const int *block_size, const pwrel_mlp *const *models,
                     const pwrel_options *opt_in, uint64_t *d_out_sizes)
{
    Request r;
    r.fields.assign(fields, fields + n);
    r.dtype = dtype;
    r.eps = eps;
    r.block[0] = 0;
    r.block[1] = block_size && block_size[1] ? block_size[1] : 16;
    r.block[2] = block_size && block_size[2] ? block_size[2] : 8;
    r.opt = opt_in ? *opt_in : pwrel_options{1, 0, 0, 0};
    r.sizes = d_out_sizes;
    for (int d = 1; d < 3; ++d)
        if (r.opt.use_net && models && models[d]) {
            r.models[d] = *models[d];
            r.has_model[d] = 1;
        }
    return r;
}

BatchState *state_of(pwrel_ctx *ctx)
{
    BatchState *&b = api_batch_state(ctx);
    if (!b)
        b = new (std::nothrow) BatchState();
    return b;
}

// One batched compression of request r (checked) with the context's tile
// variants: the table is built unless r repeats the prepared request.
int batch_call(pwrel_ctx *ctx, BatchState &b, Request &r, hipStream_t s)
{
    for (int k = 0; k < kClasses; ++k)
        r.variant[k] = b.variant[k];
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "stream capture query failed");
    const bool capturing = cap != hipStreamCaptureStatusNone;
    hipError_t e;
    int st;
    if (!(b.ready && b.req.same(r))) {
        if (capturing)
            return api_fail(ctx, PWREL_EINVAL,
                            "a captured batch must repeat the request of an earlier call "
                            "(the field table is built outside capture)");
        if ((st = prepare(ctx, b, r, s)) != PWREL_OK) {
            b.ready = false;
            return st;
        }
    } else if (!capturing && s != b.prep_stream &&
               (e = hipStreamWaitEvent(s, b.ev, 0)) != hipSuccess) {
        return api_fail(ctx, PWREL_EHIP, "batch table wait");
    }
    if ((e = launch_prepared(b, b.req, api_qtab(ctx), api_num_cus(ctx), s)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP,
                        (std::string("batch launch: ") + hipGetErrorString(e)).c_str());
    return PWREL_OK;
}

}  // namespace
}  // namespace pwrel

using namespace pwrel;

extern "C" int pwrel_compress_batch(pwrel_ctx *ctx, int n, const pwrel_field_desc *fields,
                                    int dtype, double rel_error_bound, const int *block_size,
                                    const pwrel_mlp *const *models, const pwrel_options *opt_in,
                                    uint64_t *d_out_sizes, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (n < 1 || !fields)
        return api_fail(ctx, PWREL_EINVAL, "no fields");
    Request r = make_request(fields, n, dtype, rel_error_bound, block_size, models, opt_in,
                             d_out_sizes);
    int st = check_request(ctx, r);
    if (st != PWREL_OK)
        return st;
    pwrel::DeviceGuard_ guard(api_device(ctx));
    BatchState *b = state_of(ctx);
    if (!b)
        return api_fail(ctx, PWREL_ENOMEM, "batch state allocation failed");
    return batch_call(ctx, *b, r, reinterpret_cast<hipStream_t>(stream));
}

extern "C" int pwrel_batch_set_tiles(pwrel_ctx *ctx, const int *variant)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!variant)
        return api_fail(ctx, PWREL_EINVAL, "NULL variant array");
    for (int k = 0; k < kClasses; ++k)
        if (variant[k] < 0 || variant[k] >= kTileVariants)
            return api_fail(ctx, PWREL_EINVAL, "tile variant out of range");
    BatchState *b = state_of(ctx);
    if (!b)
        return api_fail(ctx, PWREL_ENOMEM, "batch state allocation failed");
    for (int k = 0; k < kClasses; ++k)
        b->variant[k] = variant[k];
    return PWREL_OK;
}

extern "C" int pwrel_batch_get_tiles(pwrel_ctx *ctx, int *variant, int *shapes)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!variant)
        return api_fail(ctx, PWREL_EINVAL, "NULL variant array");
    BatchState *b = state_of(ctx);
    if (!b)
        return api_fail(ctx, PWREL_ENOMEM, "batch state allocation failed");
    static const int DB[kClasses][2] = {{3, 8}, {2, 16}};
    for (int k = 0; k < kClasses; ++k) {
        variant[k] = b->variant[k];
        if (shapes)
            variant_shape(DB[k][0], DB[k][1], b->variant[k], shapes + 3 * k);
    }
    return PWREL_OK;
}

extern "C" int pwrel_compress_batch_tune(pwrel_ctx *ctx, int n, const pwrel_field_desc *fields,
                                         int dtype, double rel_error_bound,
                                         const int *block_size, const pwrel_mlp *const *models,
                                         const pwrel_options *opt_in, uint64_t *d_out_sizes,
                                         int reps, int *variant_out, double *ms_out,
                                         void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (n < 1 || !fields)
        return api_fail(ctx, PWREL_EINVAL, "no fields");
    if (reps < 1 || reps > 1000)
        return api_fail(ctx, PWREL_EINVAL, "reps must be 1..1000");
    Request r = make_request(fields, n, dtype, rel_error_bound, block_size, models, opt_in,
                             d_out_sizes);
    int st = check_request(ctx, r);
    if (st != PWREL_OK)
        return st;
    pwrel::DeviceGuard_ guard(api_device(ctx));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
        return api_fail(ctx, PWREL_EINVAL, "tuning times launches: not under capture");
    BatchState *b = state_of(ctx);
    if (!b)
        return api_fail(ctx, PWREL_ENOMEM, "batch state allocation failed");
    hipError_t e;
    for (auto &pr : b->tev)
        for (hipEvent_t &ev : pr)
            if (!ev && (e = hipEventCreate(&ev)) != hipSuccess)
                return api_fail(ctx, PWREL_EHIP, "timing event creation failed");
    double med[kClasses][kTileVariants] = {};
    const int keep[kClasses] = {b->variant[0], b->variant[1]};
    for (int v = 0; v < kTileVariants; ++v) {
        for (int k = 0; k < kClasses; ++k)
            b->variant[k] = v;
        std::vector<double> t[kClasses];
        for (int rep = 0; rep <= reps; ++rep) {  // rep 0 builds the table and warms up
            b->timing = rep > 0;
            st = batch_call(ctx, *b, r, s);
            b->timing = false;
            if (st == PWREL_OK && (e = hipStreamSynchronize(s)) != hipSuccess)
                st = api_fail(ctx, PWREL_EHIP, "tuning synchronize");
            if (st != PWREL_OK) {
                for (int k = 0; k < kClasses; ++k)
                    b->variant[k] = keep[k];
                return st;
            }
            if (rep == 0)
                continue;
            for (int k = 0; k < kClasses; ++k) {
                float ms = 0.0f;
                if (b->nclass[k] &&
                    hipEventElapsedTime(&ms, b->tev[k][0], b->tev[k][1]) == hipSuccess)
                    t[k].push_back(ms);
            }
        }
        for (int k = 0; k < kClasses; ++k) {
            std::sort(t[k].begin(), t[k].end());
            med[k][v] = t[k].empty() ? 0.0 : t[k][t[k].size() / 2];
        }
    }
    for (int k = 0; k < kClasses; ++k) {
        int best = 0;
        for (int v = 1; v < kTileVariants; ++v)
            if (med[k][v] < med[k][best])
                best = v;
        b->variant[k] = best;
        if (variant_out)
            variant_out[k] = best;
        if (ms_out)
            for (int v = 0; v < kTileVariants; ++v)
                ms_out[k * kTileVariants + v] = med[k][v];
    }
    // leave the outputs (and the prepared table) of the chosen variants
    if ((st = batch_call(ctx, *b, r, s)) != PWREL_OK)
        return st;
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "tuning synchronize");
    return PWREL_OK;
}
