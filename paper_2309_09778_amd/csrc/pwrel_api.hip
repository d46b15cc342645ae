// C ABI of the PW_REL perceptron compressor (see include/pwrel.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <queue>
#include <string>
#include <vector>

#include "pwrel_huffman.h"
#include "pwrel_internal.h"
#include "pwrel_train.h"

using namespace pwrel;

struct pwrel_ctx {
    int device = 0;
    int num_cus = 256;
    Workspace ws;
    uint32_t *counts_scratch = nullptr;  // per-block counts for pwrel_encode_grid
    size_t counts_scratch_cap = 0;
    uint8_t *bflags_scratch = nullptr;   // per-block judge flags for pwrel_train_codebook
    size_t bflags_scratch_cap = 0;
    std::string err;
    int profiling = 0;
    hipEvent_t ev[10] = {};
    bool ev_ok = false;
    double phase_ms[PWREL_NUM_PHASES] = {};
    // learned part: chunk counts and offsets, pairs, parameters, scores
    uint32_t *chunk_cnt = nullptr;
    size_t chunk_cnt_cap = 0;
    unsigned long long *chunk_off = nullptr;
    size_t chunk_off_cap = 0;
    float *pairs = nullptr;
    size_t pairs_cap = 0;
    float *theta = nullptr;  // [1 + candidates][kMaxParams]
    MlpW *nets = nullptr;    // [1 + candidates]
    unsigned long long *vhist = nullptr;  // [1 + candidates][65536]
    size_t vhist_cap = 0;
    double *scal = nullptr;  // sigma, partial sums (256), loss
    long long *scores = nullptr;
    // halo-mode decoder: block order of the last geometry, flag epoch
    unsigned *order = nullptr;
    size_t order_cap = 0;
    long long order_nb[3] = {-1, -1, -1};
    int order_pen = -1;  // the cached order is of pencils (1) or of blocks (0)
    unsigned epoch = 0;
    void *hdr = nullptr;  // header of pwrel_compress_raw (PWREL_HEADER_BYTES)
    void *hstage = nullptr;  // pinned host staging of a caller's codebook (its upload stays async)
    float *dstage = nullptr;  // data blocks gathered contiguous (pwrel_*_datablocks)
    size_t dstage_cap = 0;
    unsigned long long *doffs = nullptr;  // their offsets in dstage
    size_t doffs_cap = 0;
    int *mstatus = nullptr;  // status of a call that decodes several streams
    size_t mstatus_cap = 0;
    pwrel::BatchState *batch = nullptr;  // pwrel_compress_batch's workspace and table
    pwrel::OlState *ol = nullptr;        // pwrel_openloop's scratch
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

int fail(pwrel_ctx *ctx, int code, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    return code;
}

int hip_fail(pwrel_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, PWREL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int check_model(pwrel_ctx *ctx, const pwrel_mlp *m, int ndim)
{
    const char *why = model_problem(m, ndim);
    return why ? fail(ctx, PWREL_EINVAL, why) : PWREL_OK;
}

template <typename P>
hipError_t grow(P *&ptr, size_t &cap, size_t need)
{
    if (need <= cap && ptr)
        return hipSuccess;
    if (ptr)
        (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    const hipError_t e = hipMalloc(reinterpret_cast<void **>(&ptr), need * sizeof(P));
    if (e == hipSuccess)
        cap = need;
    return e;
}

int ensure_scan(pwrel_ctx *ctx, const Geom &g)
{
    hipError_t e = grow(ctx->ws.offsets, ctx->ws.offsets_cap, (size_t)g.nblocks);
    if (e == hipSuccess)
        e = grow(ctx->ws.partials, ctx->ws.partials_cap,
                 (size_t)((g.nblocks + kScanChunk - 1) / kScanChunk));
    if (e != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
    return PWREL_OK;
}

// buffers of the Huffman stage: 16-bit codes (N), encoder tables, per-block
// bit offsets
int ensure_huffman(pwrel_ctx *ctx, const Geom &g)
{
    Workspace &ws = ctx->ws;
    hipError_t e = grow(ws.codes16, ws.codes16_cap, (size_t)std::max<long long>(g.N, 1));
    if (e == hipSuccess)
        e = grow(ws.boffsets, ws.boffsets_cap, (size_t)g.nblocks);
    if (e == hipSuccess)
        e = grow(ws.bpartials, ws.bpartials_cap,
                 (size_t)((g.nblocks + kScanChunk - 1) / kScanChunk));
    if (e == hipSuccess && !ws.enc_len)
        e = hipMalloc(reinterpret_cast<void **>(&ws.enc_len), 65536);
    if (e == hipSuccess && !ws.enc_code)
        e = hipMalloc(reinterpret_cast<void **>(&ws.enc_code), 65536 * sizeof(unsigned long long));
    if (e == hipSuccess && !ws.bits_total)
        e = hipMalloc(reinterpret_cast<void **>(&ws.bits_total), 256);
    if (e != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, std::string("Huffman workspace: ") + hipGetErrorString(e));
    return PWREL_OK;
}

// where the Huffman sections of a stream go (after the counts section)
HuffLayout huff_layout(const Geom &g, const Layout &L, uint64_t n_sym, uint64_t n_bits,
                       uint64_t n_raw, uint64_t tsize, uint64_t &total)
{
    HuffLayout h{};
    h.n_sym = (uint32_t)n_sym;
    h.n_bits = n_bits;
    h.size_bytes = (uint32_t)huff_size_bytes(g);
    h.table_bytes = huff_table_bytes(n_sym);
    h.off_huff = L.off[3];
    h.off_sizes = align256(h.off_huff + h.table_bytes);
    h.off_bits = align256(h.off_sizes + (uint64_t)h.size_bytes * (uint64_t)g.nblocks);
    const uint64_t off_raw = align256(h.off_bits + 4ull * ((n_bits + 31) / 32));
    total = off_raw + n_raw * tsize;
    return h;
}

int finish_status(pwrel_ctx *ctx, int st)
{
    switch (st) {
    case PWREL_OK:
        return PWREL_OK;
    case PWREL_ERANGE:
        return fail(ctx, st, "a grid value leaves +-2^30: the bound is too tight for the range");
    case PWREL_ENONFINITE:
        return fail(ctx, st, "the field holds NaN or Inf");
    case PWREL_ENOSPC:
        return fail(ctx, st, "output capacity too small");
    case PWREL_ECORRUPT:
        return fail(ctx, st, "stream is corrupt");
    default:
        return fail(ctx, st, "device reported status " + std::to_string(st));
    }
}

// Profiling marks: record event `i` on the stream when profiling is on.
void mark(pwrel_ctx *ctx, int i, hipStream_t s)
{
    if (ctx->profiling && ctx->ev_ok)
        (void)hipEventRecord(ctx->ev[i], s);
}

// After a synchronize: phase p = time from mark a to mark b.
void collect(pwrel_ctx *ctx, const int (*spans)[3], int n)
{
    if (!(ctx->profiling && ctx->ev_ok))
        return;
    for (int i = 0; i < n; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ctx->ev[spans[i][1]], ctx->ev[spans[i][2]]) == hipSuccess)
            ctx->phase_ms[spans[i][0]] = ms;
    }
}

uint64_t splitmix64(uint64_t s)
{
    uint64_t z = s + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Statistics, constants and the per-chunk pair counts of a field, then the
// exclusive offsets of the chunks (host scan, copied back to the device).
int sample_counts(pwrel_ctx *ctx, const void *d_field, const Geom &g, double eps,
                  int independent, double rho, uint64_t seed, hipStream_t s, SampleArgs &a,
                  unsigned long long &ntr, unsigned long long &nva, long long &nch)
{
    a = SampleArgs{};
    a.x = d_field;
    for (int d = 0; d < 3; ++d)
        a.n[d] = g.n[d];
    a.N = g.N;
    a.B = g.B;
    a.independent = independent ? 1 : 0;
    a.rho = rho;
    a.seed = seed;
    a.c = ctx->ws.consts;
    nch = (g.N + kSampleChunk - 1) / kSampleChunk;
    hipError_t e = grow(ctx->chunk_cnt, ctx->chunk_cnt_cap, (size_t)(2 * nch));
    if (e == hipSuccess)
        e = grow(ctx->chunk_off, ctx->chunk_off_cap, (size_t)(2 * nch));
    if (e != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, "sampling workspace allocation failed");
    if ((e = launch_reset(ctx->ws, s)) != hipSuccess ||
        (e = launch_stats(d_field, g, ctx->ws, s)) != hipSuccess ||
        (e = launch_consts(g, eps, ctx->ws, s)) != hipSuccess ||
        (e = launch_sample(true, a, g.D, g.dtype, ctx->chunk_cnt, ctx->chunk_cnt + nch, nullptr,
                           s)) != hipSuccess)
        return hip_fail(ctx, e, "sample count");
    std::vector<uint32_t> cnt((size_t)(2 * nch));
    int dst = 0;
    if ((e = hipMemcpyAsync(cnt.data(), ctx->chunk_cnt, cnt.size() * sizeof(uint32_t),
                            hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&dst, ctx->ws.status, sizeof dst, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "sample count copy");
    if (dst != PWREL_OK)
        return finish_status(ctx, dst);
    std::vector<unsigned long long> off((size_t)(2 * nch));
    ntr = nva = 0;
    for (long long i = 0; i < nch; ++i) {
        off[(size_t)i] = ntr;
        off[(size_t)(nch + i)] = nva;
        ntr += cnt[(size_t)i];
        nva += cnt[(size_t)(nch + i)];
    }
    if ((e = hipMemcpyAsync(ctx->chunk_off, off.data(), off.size() * sizeof(unsigned long long),
                            hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "sample offsets copy");
    return PWREL_OK;
}

bool train_shape_ok(int hidden, int inputs)
{
    return hidden >= 1 && hidden <= PWREL_MAX_HIDDEN && (inputs == 0 || inputs == 2 || inputs == 6);
}

}  // namespace

extern "C" {

const char *pwrel_status_string(int status)
{
    switch (status) {
    case PWREL_OK: return "ok";
    case PWREL_EINVAL: return "invalid argument";
    case PWREL_ERANGE: return "grid value out of range";
    case PWREL_ENONFINITE: return "non-finite input";
    case PWREL_ENOSPC: return "output capacity too small";
    case PWREL_ECORRUPT: return "corrupt stream";
    case PWREL_EHIP: return "HIP runtime error";
    case PWREL_ENOMEM: return "out of memory";
    default: return "unknown status";
    }
}

int pwrel_check_args(const uint64_t *dims, int ndim, int dtype, double eps, int block_size)
{
    Geom g;
    if (!make_geom(dims, ndim, dtype, block_size, g))
        return PWREL_EINVAL;
    if (!(eps > 0.0 && eps < 1.0) || !(1.0 + eps > 1.0))
        return PWREL_EINVAL;
    return PWREL_OK;
}

uint64_t pwrel_compress_bound(const uint64_t *dims, int ndim, int dtype, int block_size)
{
    Geom g;
    if (!make_geom(dims, ndim, dtype, block_size, g))
        return 0;
    const Layout L = layout_for(g, PWREL_HF_NET | PWREL_HF_JUDGE);
    // a Huffman stream holds at most 16 bits per code (else the codes are
    // stored as they are), plus its codebook and per-block sizes
    const uint64_t huff_extra = align256(huff_table_bytes(65536)) +
                                align256(4ull * (uint64_t)g.nblocks) + 256;
    return L.off[4] + huff_extra + (uint64_t)g.N * (dtype == PWREL_F32 ? 4u : 8u);
}

int pwrel_create(pwrel_ctx **out, int device)
{
    if (!out)
        return PWREL_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return PWREL_EINVAL;
    pwrel_ctx *ctx = new (std::nothrow) pwrel_ctx();
    if (!ctx)
        return PWREL_ENOMEM;
    ctx->device = device;
    DeviceGuard guard(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cus = prop.multiProcessorCount;
    Workspace &ws = ctx->ws;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&ws.stats), kStatParts * sizeof(DevStats));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ws.consts), sizeof(DevConsts));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ws.status), 256);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ws.hist), 65536 * sizeof(unsigned long long));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ws.n_raw), 256);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ws.ticket), 256);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ws.qtab), kQtab * sizeof(long long));
    if (e == hipSuccess)
        e = hipMalloc(&ws.invtab, kInvTable * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ctx->theta),
                      (PWREL_MAX_CANDIDATES + 1) * kMaxParams * sizeof(float));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ctx->nets), PWREL_MAX_CANDIDATES * sizeof(MlpW));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ctx->scal), 512 * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&ctx->scores),
                      PWREL_MAX_CANDIDATES * sizeof(long long));
    if (e == hipSuccess)
        e = launch_qtable(ws.qtab, kQtab, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = noalloc_setup(device);  // the static scratch of pwrel_compress_noalloc
    if (e != hipSuccess) {
        pwrel_destroy(ctx);
        return PWREL_ENOMEM;
    }
    *out = ctx;
    return PWREL_OK;
}

void pwrel_destroy(pwrel_ctx *ctx)
{
    if (!ctx)
        return;
    DeviceGuard guard(ctx->device);
    Workspace &ws = ctx->ws;
    void *ptrs[] = {ws.stats,       ws.consts,      ws.status,     ws.hist,        ws.n_raw,
                    ws.offsets,     ws.partials,    ws.pgrid,      ws.qtab,        ctx->counts_scratch,
                    ctx->chunk_cnt, ctx->chunk_off, ctx->pairs,    ctx->theta,     ctx->nets,
                    ctx->vhist,     ctx->scal,      ctx->scores,   ws.done,        ws.ticket,
                    ctx->order,     ws.praw,        ws.zf,         ws.yf,          ctx->hdr,
                    ws.codes16,     ws.enc_len,     ws.enc_code,   ws.boffsets,    ws.bpartials,
                    ws.bits_total,  ws.invtab,     ctx->bflags_scratch, ctx->dstage, ctx->doffs,
                    ctx->mstatus};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    if (ctx->ev_ok)
        for (hipEvent_t &e : ctx->ev)
            (void)hipEventDestroy(e);
    batch_release(ctx->batch);
    ol_release(ctx->ol);
    if (ctx->hstage)
        (void)hipHostFree(ctx->hstage);
    delete ctx;
}

const char *pwrel_last_error(const pwrel_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "no context";
}

}  // extern "C"

namespace {

bool check_compress_args(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                         int dtype, double eps, int block_size, const pwrel_mlp *model,
                         const pwrel_options &opt, Geom &g, Tile &tile, int &st)
{
    st = PWREL_OK;
    if (pwrel_check_args(dims, ndim, dtype, eps, block_size) != PWREL_OK) {
        st = fail(ctx, PWREL_EINVAL, "bad dims/ndim/dtype/bound/block size");
        return false;
    }
    if (!d_field) {
        st = fail(ctx, PWREL_EINVAL, "NULL field");
        return false;
    }
    if (opt.judge && !opt.use_net) {
        st = fail(ctx, PWREL_EINVAL, "the per-block judge needs a network (use_net)");
        return false;
    }
    if (opt.use_net && (st = check_model(ctx, model, ndim)) != PWREL_OK)
        return false;
    make_geom(dims, ndim, dtype, block_size, g);
    if (!tile_for(g, tile)) {
        st = fail(ctx, PWREL_EINVAL, "block too large for the LDS tile");
        return false;
    }
    return true;
}

}  // namespace

namespace pwrel {

bool api_check_compress(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                        int dtype, double eps, int block_size, const pwrel_mlp *model,
                        const pwrel_options &opt, Geom &g, Tile &tile, int &st)
{
    return check_compress_args(ctx, d_field, dims, ndim, dtype, eps, block_size, model, opt, g,
                               tile, st);
}

int api_fail(pwrel_ctx *ctx, int code, const char *msg) { return fail(ctx, code, msg); }
int api_status(pwrel_ctx *ctx, int device_status) { return finish_status(ctx, device_status); }
int api_device(const pwrel_ctx *ctx) { return ctx->device; }
int api_num_cus(const pwrel_ctx *ctx) { return ctx->num_cus; }
const long long *api_qtab(const pwrel_ctx *ctx) { return ctx->ws.qtab; }
BatchState *&api_batch_state(pwrel_ctx *ctx) { return ctx->batch; }
OlState *&api_ol_state(pwrel_ctx *ctx) { return ctx->ol; }
Workspace &api_ws(pwrel_ctx *ctx) { return ctx->ws; }
hipError_t api_dstage(pwrel_ctx *ctx, size_t n, size_t nsub, float **stage,
                      unsigned long long **offs)
{
    hipError_t e = grow(ctx->dstage, ctx->dstage_cap, std::max<size_t>(n, 1));
    if (e == hipSuccess)
        e = grow(ctx->doffs, ctx->doffs_cap, std::max<size_t>(nsub, 1));
    *stage = ctx->dstage;
    *offs = ctx->doffs;
    return e;
}
int api_ensure_scan(pwrel_ctx *ctx, const Geom &g) { return ensure_scan(ctx, g); }

// The compression launches (Algorithm 1): reset, statistics, constants, grid
// values and bound checks (FP32), prediction / quantisation / judge, scan,
// raw scatter, model, header.  Queued on s; nothing is synchronised or
// allocated here.  ws.pgrid must hold g.N entries for FP32 fields.
hipError_t compress_launches(Workspace &ws, int num_cus, const void *d_field, const Geom &g,
                             const Tile &tile, double eps, const pwrel_mlp *model,
                             const pwrel_options &opt, const Sections &sec, hipStream_t s,
                             void (*mark_fn)(void *, int, hipStream_t), void *mark_arg)
{
    auto mark_at = [&](int i) {
        if (mark_fn)
            mark_fn(mark_arg, i, s);
    };
    const int flags = flags_of(opt);
    const Layout L = layout_for(g, flags);
    hipError_t e;
    if ((e = launch_reset(ws, s)) != hipSuccess)
        return e;
    mark_at(0);
    if ((e = launch_stats(d_field, g, ws, s)) != hipSuccess ||
        (e = launch_consts(g, eps, ws, s)) != hipSuccess)
        return e;
    mark_at(1);
    if (g.dtype == PWREL_F32) {
        // two passes: grid values and bound checks once per value into the
        // grid scratch field, then prediction and quantisation from it
        if ((e = launch_grid_entries(static_cast<const float *>(d_field), g, ws, ws.pgrid, s)) !=
                hipSuccess ||
            (e = launch_compress(d_field, ws.pgrid, g, tile, model, opt, ws, sec.codes,
                                 sec.counts, sec.bflags, num_cus, s, true)) != hipSuccess)
            return e;
    } else if ((e = launch_compress(d_field, nullptr, g, tile, model, opt, ws, sec.codes,
                                    sec.counts, sec.bflags, num_cus, s)) != hipSuccess) {
        return e;
    }
    mark_at(2);
    if ((e = launch_scan(sec.counts, g, ws, s)) != hipSuccess ||
        (e = launch_scatter(d_field, g, sec.codes, sec.counts, ws, sec.raw, sec.raw_cap, s)) !=
            hipSuccess)
        return e;
    if (opt.use_net && sec.model && (e = launch_write_model(*model, sec.model, s)) != hipSuccess)
        return e;
    if ((e = launch_header(g, flags, L.off, ws, sec.header, sec.header_capacity,
                           sec.stream_gaps, s)) != hipSuccess)
        return e;
    mark_at(3);
    return hipSuccess;
}

}  // namespace pwrel

namespace {

void mark_cb(void *ctx, int i, hipStream_t s) { mark(static_cast<pwrel_ctx *>(ctx), i, s); }

// The end of a Huffman-stage compression whose codebook would not pay: the
// 16-bit codes (in the context's code buffer, balance-point counts scanned)
// go into the stream as pwrel_compress writes them without the stage.
int finish_codes16(pwrel_ctx *ctx, const void *d_field, const Geom &g, const pwrel_mlp *model,
                   const pwrel_options &opt, unsigned char *out, uint64_t out_capacity,
                   uint64_t *out_size, hipStream_t s)
{
    Workspace &ws = ctx->ws;
    const int pflags = flags_of(opt) & ~PWREL_HF_HUFFMAN;
    const Layout L = layout_for(g, pflags);
    const uint64_t tsize = g.dtype == PWREL_F32 ? 4u : 8u;
    const uint32_t *counts = reinterpret_cast<const uint32_t *>(out + L.off[2]);
    hipError_t e;
    if ((e = hipMemcpyAsync(out + L.off[3], ws.codes16, 2ull * (uint64_t)g.N,
                            hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = launch_scatter(d_field, g, ws.codes16, counts, ws, out + L.off[4],
                            (out_capacity - L.off[4]) / tsize, s)) != hipSuccess ||
        (opt.use_net && (e = launch_write_model(*model, out + L.off[0], s)) != hipSuccess) ||
        (e = launch_header(g, pflags, L.off, ws, out, out_capacity, true, s)) != hipSuccess)
        return hip_fail(ctx, e, "compress (16-bit codes)");
    mark(ctx, 3, s);
    pwrel_header h;
    if ((e = hipMemcpyAsync(&h, out, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "header copy");
    static const int spans16[3][3] = {{0, 0, 1}, {1, 1, 2}, {2, 2, 3}};
    collect(ctx, spans16, 3);
    if (h.status != PWREL_OK)
        return finish_status(ctx, h.status);
    *out_size = h.total_size;
    return PWREL_OK;
}

// A caller's trained codebook (Sec. 4.3) is a valid canonical table: counts
// that sum to n_sym within the Kraft bound, an escape of at most 16 bits
// that has a slot, and every listed code once.
bool codebook_ok(const pwrel_codebook &cb)
{
    uint64_t nsym = 0, kraft = 0;
    for (int l = 1; l <= kHuffMaxLen; ++l) {
        nsym += cb.count[l];
        kraft += (uint64_t)cb.count[l] << (kHuffMaxLen - l);
    }
    if (cb.count[0] != 0 || nsym == 0 || nsym > 65536 || nsym != cb.n_sym ||
        kraft > (uint64_t(1) << kHuffMaxLen) || cb.esc_len > 16 ||
        (cb.esc_len != 0 && cb.count[cb.esc_len] == 0))
        return false;
    uint64_t esc_ix = ~0ull;
    if (cb.esc_len) {
        uint64_t idx = 0;
        for (uint32_t l = 1; l <= cb.esc_len; ++l)
            idx += cb.count[l];
        esc_ix = idx - 1;
    }
    std::vector<uint64_t> seen(1024, 0);
    for (uint64_t i = 0; i < nsym; ++i) {
        if (i == esc_ix)
            continue;
        const uint32_t v = cb.syms[i];
        if (seen[v >> 6] & (1ull << (v & 63)))
            return false;
        seen[v >> 6] |= 1ull << (v & 63);
    }
    return true;
}

// The Huffman stage with a trained codebook: the table is known before any
// code is, so the per-block sizes and their scan follow the compression
// kernels directly; one small copy (balance points, status, coded bits)
// then lays the stream out.
int huffman_trained_tail(pwrel_ctx *ctx, const void *d_field, const Geom &g,
                         const pwrel_mlp *model, const pwrel_options &opt, unsigned char *out,
                         uint64_t out_capacity, uint64_t *out_size, hipStream_t s)
{
    Workspace &ws = ctx->ws;
    const pwrel_codebook &cb = *opt.codebook;
    const int flags = flags_of(opt);
    const Layout L = layout_for(g, flags);
    const uint64_t tsize = g.dtype == PWREL_F32 ? 4u : 8u;
    const uint32_t *counts = reinterpret_cast<const uint32_t *>(out + L.off[2]);
    hipError_t e;
    if ((e = launch_scan(counts, g, ws, s)) != hipSuccess)
        return hip_fail(ctx, e, "compress (scan)");
    uint64_t total = 0;
    HuffLayout hl = huff_layout(g, L, cb.n_sym, 0, 0, tsize, total);
    if (hl.off_bits > out_capacity)  // table and sizes alone outgrow the output
        return finish_codes16(ctx, d_field, g, model, opt, out, out_capacity, out_size, s);
    uint32_t *d_tab = reinterpret_cast<uint32_t *>(out + hl.off_huff);
    struct {
        unsigned long long n_raw, bits;
        int status;
    } got{};
    // the table goes through pinned staging, so its upload does not hold the
    // host while the compression kernels run (every call ends synchronised,
    // so the staging is free again at the next)
    const size_t tbytes = sizeof cb.count + 2ull * cb.n_sym;
    if (!ctx->hstage &&
        (e = hipHostMalloc(&ctx->hstage, sizeof cb.count + sizeof cb.syms, 0)) != hipSuccess) {
        ctx->hstage = nullptr;
        return fail(ctx, PWREL_ENOMEM, "codebook staging allocation failed");
    }
    std::memcpy(ctx->hstage, cb.count, sizeof cb.count);
    std::memcpy(static_cast<unsigned char *>(ctx->hstage) + sizeof cb.count, cb.syms,
                2ull * cb.n_sym);
    if ((e = hipMemcpyAsync(d_tab, ctx->hstage, tbytes, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = launch_huff_sizes(g, ws.codes16, d_tab, cb.esc_len, out + hl.off_sizes, ws, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&got.n_raw, ws.n_raw, sizeof got.n_raw, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&got.bits, ws.bits_total, sizeof got.bits, hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipMemcpyAsync(&got.status, ws.status, sizeof got.status, hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "compress (Huffman sizes)");
    if (got.status == PWREL_ECORRUPT)
        return fail(ctx, PWREL_EINVAL, "the codebook has no codeword and no escape for a code");
    if (got.status != PWREL_OK)
        return finish_status(ctx, got.status);
    hl = huff_layout(g, L, cb.n_sym, got.bits, got.n_raw, tsize, total);
    hl.esc_len = cb.esc_len;
    if (total >= L.off[4] + got.n_raw * tsize)
        return finish_codes16(ctx, d_field, g, model, opt, out, out_capacity, out_size, s);
    if (total > out_capacity)
        return fail(ctx, PWREL_ENOSPC, "output capacity too small");
    const uint64_t off_raw = align256(hl.off_bits + 4ull * ((hl.n_bits + 31) / 32));
    const uint64_t offs[5] = {L.off[0], L.off[1], L.off[2], 0, off_raw};
    if ((e = launch_scatter(d_field, g, ws.codes16, counts, ws, out + off_raw,
                            (out_capacity - off_raw) / tsize, s)) != hipSuccess ||
        (e = launch_huff_pack(g, ws.codes16, out + hl.off_sizes,
                              reinterpret_cast<uint32_t *>(out + hl.off_bits),
                              (hl.n_bits + 31) / 32, ws, s)) != hipSuccess ||
        (opt.use_net && (e = launch_write_model(*model, out + L.off[0], s)) != hipSuccess) ||
        (e = launch_header(g, flags, offs, ws, out, out_capacity, true, s, &hl)) != hipSuccess)
        return hip_fail(ctx, e, "compress (Huffman stage)");
    mark(ctx, 3, s);
    pwrel_header h;
    if ((e = hipMemcpyAsync(&h, out, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "header copy");
    static const int spans[3][3] = {{0, 0, 1}, {1, 1, 2}, {2, 2, 3}};
    collect(ctx, spans, 3);
    if (h.status != PWREL_OK)
        return finish_status(ctx, h.status);
    *out_size = h.total_size;
    return PWREL_OK;
}

// Statistics, constants, grid values, prediction and quantisation of a field
// into the context's 16-bit code buffer (block-major), per-block counts and
// judge flags into the given buffers; phase marks 0 to 2.
int codes_pass(pwrel_ctx *ctx, const void *d_field, const Geom &g, const Tile &tile, double eps,
               const pwrel_mlp *model, const pwrel_options &opt, uint32_t *counts,
               uint8_t *bflags, hipStream_t s)
{
    Workspace &ws = ctx->ws;
    hipError_t e;
    mark(ctx, 0, s);
    if ((e = launch_reset(ws, s)) != hipSuccess || (e = launch_stats(d_field, g, ws, s)) != hipSuccess ||
        (e = launch_consts(g, eps, ws, s)) != hipSuccess)
        return hip_fail(ctx, e, "compress (statistics)");
    mark(ctx, 1, s);
    if (g.dtype == PWREL_F32) {
        if ((e = launch_grid_entries(static_cast<const float *>(d_field), g, ws, ws.pgrid, s)) !=
                hipSuccess ||
            (e = launch_compress(d_field, ws.pgrid, g, tile, model, opt, ws, ws.codes16, counts,
                                 bflags, ctx->num_cus, s, true)) != hipSuccess)
            return hip_fail(ctx, e, "compress");
    } else if ((e = launch_compress(d_field, nullptr, g, tile, model, opt, ws, ws.codes16, counts,
                                    bflags, ctx->num_cus, s)) != hipSuccess) {
        return hip_fail(ctx, e, "compress");
    }
    mark(ctx, 2, s);
    return PWREL_OK;
}

// pwrel_compress with the Huffman stage (Sec. 4.1 coding stage; Algorithm 1
// writes the Huffman codes).  Pass 1 on the device: statistics, constants,
// grid values, prediction and quantisation into the context's 16-bit code
// buffer, the balance-point scan and the code histogram.  The host then
// builds the codebook from the histogram and lays the stream out (the coded
// size is sum count * length, known before any bit is written).  Pass 2:
// raw values, codebook, per-block bit sizes, packed bits, model, header.
int compress_huffman(pwrel_ctx *ctx, const void *d_field, const Geom &g, const Tile &tile,
                     double eps, const pwrel_mlp *model, const pwrel_options &opt,
                     unsigned char *out, uint64_t out_capacity, uint64_t *out_size, hipStream_t s)
{
    Workspace &ws = ctx->ws;
    int st;
    if ((st = ensure_huffman(ctx, g)) != PWREL_OK)
        return st;
    const int flags = flags_of(opt);
    const Layout L = layout_for(g, flags);
    const uint64_t tsize = g.dtype == PWREL_F32 ? 4u : 8u;
    uint32_t *counts = reinterpret_cast<uint32_t *>(out + L.off[2]);
    uint8_t *bflags = (flags & PWREL_HF_JUDGE) ? out + L.off[1] : nullptr;
    hipError_t e;
    if ((st = codes_pass(ctx, d_field, g, tile, eps, model, opt, counts, bflags, s)) != PWREL_OK)
        return st;
    if (opt.codebook)
        return huffman_trained_tail(ctx, d_field, g, model, opt, out, out_capacity, out_size, s);
    std::vector<uint64_t> hist(65536);
    unsigned long long n_raw = 0;
    int dst = 0;
    if ((e = launch_scan(counts, g, ws, s)) != hipSuccess ||
        (e = launch_hist(ws.codes16, g.N, ws.hist, s)) != hipSuccess ||
        (e = hipMemcpyAsync(hist.data(), ws.hist, 65536 * sizeof(uint64_t), hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipMemcpyAsync(&n_raw, ws.n_raw, sizeof n_raw, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&dst, ws.status, sizeof dst, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "compress (histogram)");
    if (dst != PWREL_OK)
        return finish_status(ctx, dst);
    HuffTable t;
    if (!huff_build(hist.data(), t))
        return fail(ctx, PWREL_EHIP, "internal: Huffman lengths fail the Kraft inequality");
    if (t.n_bits > 16ull * (uint64_t)g.N)
        return fail(ctx, PWREL_EHIP, "internal: Huffman code longer than the 16-bit codes");
    uint64_t total = 0;
    const HuffLayout hl = huff_layout(g, L, t.syms.size(), t.n_bits, n_raw, tsize, total);
    if (total >= L.off[4] + n_raw * tsize)
        // the codebook costs more than it saves (codes spread over many
        // values in a small field): the stream keeps the 16-bit codes
        return finish_codes16(ctx, d_field, g, model, opt, out, out_capacity, out_size, s);
    if (total > out_capacity)
        return fail(ctx, PWREL_ENOSPC, "output capacity too small");
    // codebook section: count[0..32], then the symbols in canonical order
    std::vector<uint32_t> tab((hl.table_bytes + 3) / 4, 0u);
    std::memcpy(tab.data(), t.count.data(), t.count.size() * sizeof(uint32_t));
    std::memcpy(reinterpret_cast<unsigned char *>(tab.data()) + 4 * (kHuffMaxLen + 1),
                t.syms.data(), t.syms.size() * sizeof(uint16_t));
    const uint64_t off_raw = align256(hl.off_bits + 4ull * ((hl.n_bits + 31) / 32));
    const uint64_t offs[5] = {L.off[0], L.off[1], L.off[2], 0, off_raw};
    uint32_t *d_tab = reinterpret_cast<uint32_t *>(out + hl.off_huff);
    if ((e = hipMemcpyAsync(d_tab, tab.data(), hl.table_bytes, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = launch_scatter(d_field, g, ws.codes16, counts, ws, out + off_raw,
                            (out_capacity - off_raw) / tsize, s)) != hipSuccess ||
        (e = launch_huff_encode(g, ws.codes16, d_tab, out + hl.off_sizes,
                                reinterpret_cast<uint32_t *>(out + hl.off_bits),
                                (hl.n_bits + 31) / 32, ws, s)) != hipSuccess)
        return hip_fail(ctx, e, "compress (Huffman stage)");
    if (opt.use_net && (e = launch_write_model(*model, out + L.off[0], s)) != hipSuccess)
        return hip_fail(ctx, e, "model");
    if ((e = launch_header(g, flags, offs, ws, out, out_capacity, true, s, &hl)) != hipSuccess)
        return hip_fail(ctx, e, "header");
    mark(ctx, 3, s);
    pwrel_header h;
    unsigned long long bits_dev = 0;
    if ((e = hipMemcpyAsync(&h, out, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&bits_dev, ws.bits_total, sizeof bits_dev, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "header copy");
    static const int spans[3][3] = {{0, 0, 1}, {1, 1, 2}, {2, 2, 3}};
    collect(ctx, spans, 3);
    if (h.status != PWREL_OK)
        return finish_status(ctx, h.status);
    if (bits_dev != t.n_bits)
        return fail(ctx, PWREL_EHIP, "internal: coded size differs from the codebook's");
    *out_size = h.total_size;
    return PWREL_OK;
}

}  // namespace

extern "C" {

int pwrel_compress(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                   int dtype, double eps, int block_size, const pwrel_mlp *model,
                   const pwrel_options *opt_in, void *d_out, uint64_t out_capacity,
                   uint64_t *out_size, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    pwrel_options opt{1, 0, 0, 0};
    if (opt_in)
        opt = *opt_in;
    Geom g;
    Tile tile;
    int st;
    if (!check_compress_args(ctx, d_field, dims, ndim, dtype, eps, block_size, model, opt, g,
                             tile, st))
        return st;
    if (!d_out || !out_size)
        return fail(ctx, PWREL_EINVAL, "NULL output or size pointer");
    if (reinterpret_cast<uintptr_t>(d_out) & 15)
        return fail(ctx, PWREL_EINVAL, "the output must start 16-byte aligned");
    const int flags = flags_of(opt);
    const Layout L = layout_for(g, flags);
    if (out_capacity < L.off[4])
        return fail(ctx, PWREL_ENOSPC, "output capacity below header + codes");
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((st = ensure_scan(ctx, g)) != PWREL_OK)
        return st;
    hipError_t e;
    if (g.dtype == PWREL_F32 &&
        (e = grow(ctx->ws.pgrid, ctx->ws.pgrid_cap, (size_t)g.N)) != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, "grid field allocation failed");
    unsigned char *out = static_cast<unsigned char *>(d_out);
    if (opt.entropy && opt.codebook && !codebook_ok(*opt.codebook))
        return fail(ctx, PWREL_EINVAL, "the codebook is not a valid canonical table");
    if (opt.entropy)
        return compress_huffman(ctx, d_field, g, tile, eps, model, opt, out, out_capacity,
                                out_size, s);
    const unsigned tsize = dtype == PWREL_F32 ? 4u : 8u;
    Sections sec{};
    sec.codes = reinterpret_cast<uint16_t *>(out + L.off[3]);
    sec.counts = reinterpret_cast<uint32_t *>(out + L.off[2]);
    sec.bflags = (flags & PWREL_HF_JUDGE) ? out + L.off[1] : nullptr;
    sec.raw = out + L.off[4];
    sec.raw_cap = (out_capacity - L.off[4]) / tsize;
    sec.header = out;
    sec.stream_gaps = true;
    sec.model = out + L.off[0];
    sec.header_capacity = out_capacity;
    if ((e = compress_launches(ctx->ws, ctx->num_cus, d_field, g, tile, eps, model, opt, sec, s,
                               mark_cb, ctx)) != hipSuccess)
        return hip_fail(ctx, e, "compress");
    pwrel_header h;
    if ((e = hipMemcpyAsync(&h, out, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(ctx, e, "header copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "synchronize");
    static const int spans[3][3] = {{0, 0, 1}, {1, 1, 2}, {2, 2, 3}};
    collect(ctx, spans, 3);
    if (h.status != PWREL_OK)
        return finish_status(ctx, h.status);
    *out_size = h.total_size;
    return PWREL_OK;
}

int pwrel_compress_raw(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                       int dtype, double eps, int block_size, const pwrel_mlp *model,
                       const pwrel_options *opt_in, uint16_t *d_codes, uint32_t *d_counts,
                       uint8_t *d_bflags, void *d_raw, uint64_t raw_capacity,
                       pwrel_header *header_out, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    pwrel_options opt{1, 0, 0, 0};
    if (opt_in)
        opt = *opt_in;
    Geom g;
    Tile tile;
    int st;
    if (!check_compress_args(ctx, d_field, dims, ndim, dtype, eps, block_size, model, opt, g,
                             tile, st))
        return st;
    if (!d_codes || !d_counts || !header_out || (opt.judge && !d_bflags) ||
        (raw_capacity && !d_raw))
        return fail(ctx, PWREL_EINVAL, "NULL section pointer");
    if (opt.entropy)
        return fail(ctx, PWREL_EINVAL, "compress_raw returns the 16-bit codes (entropy = 0)");
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((st = ensure_scan(ctx, g)) != PWREL_OK)
        return st;
    hipError_t e;
    if (g.dtype == PWREL_F32 &&
        (e = grow(ctx->ws.pgrid, ctx->ws.pgrid_cap, (size_t)g.N)) != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, "grid field allocation failed");
    if (!ctx->hdr && (e = hipMalloc(&ctx->hdr, PWREL_HEADER_BYTES)) != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, "header scratch allocation failed");
    const Layout L = layout_for(g, flags_of(opt));
    const unsigned tsize = dtype == PWREL_F32 ? 4u : 8u;
    Sections sec{};
    sec.codes = d_codes;
    sec.counts = d_counts;
    sec.bflags = opt.judge ? d_bflags : nullptr;
    sec.raw = d_raw;
    sec.raw_cap = raw_capacity;
    sec.header = ctx->hdr;
    sec.stream_gaps = false;
    sec.model = nullptr;
    // the header checks the stream size against this capacity: the stream
    // these sections form fits iff the raw values do
    sec.header_capacity = L.off[4] + raw_capacity * tsize;
    if ((e = compress_launches(ctx->ws, ctx->num_cus, d_field, g, tile, eps, model, opt, sec, s,
                               mark_cb, ctx)) != hipSuccess)
        return hip_fail(ctx, e, "compress_raw");
    pwrel_header h;
    if ((e = hipMemcpyAsync(&h, ctx->hdr, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "header copy");
    if (h.status != PWREL_OK)
        return finish_status(ctx, h.status);
    *header_out = h;
    return PWREL_OK;
}

// --- a trained network kept between fields (Sec. 5 retains the trained model) -----
namespace {

constexpr uint32_t kModelMagic = 0x444D5750u;  // "PWMD"
constexpr uint32_t kModelVersion = 1u;

uint64_t fnv1a64(const unsigned char *p, uint64_t n)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (uint64_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

uint64_t model_bytes(int H, int K) { return 24 + 4ull * (H * K + 2 * H + 1) + 8; }

void put32(unsigned char *&p, uint32_t v)
{
    std::memcpy(p, &v, 4);
    p += 4;
}
void putf(unsigned char *&p, float v)
{
    std::memcpy(p, &v, 4);
    p += 4;
}
uint32_t get32(const unsigned char *&p)
{
    uint32_t v;
    std::memcpy(&v, p, 4);
    p += 4;
    return v;
}
float getf(const unsigned char *&p)
{
    float v;
    std::memcpy(&v, p, 4);
    p += 4;
    return v;
}

}  // namespace

int pwrel_model_save(const pwrel_mlp *m, void *buf, uint64_t cap, uint64_t *size)
{
    if (!m || !size)
        return PWREL_EINVAL;
    if (m->inputs != 0 && m->inputs != 2 && m->inputs != 6)
        return PWREL_EINVAL;
    if (model_problem(m, m->inputs == 6 ? 3 : (m->inputs == 2 ? 2 : 1)))
        return PWREL_EINVAL;
    const int H = m->hidden, K = m->inputs;
    const uint64_t need = model_bytes(H, K);
    *size = need;
    if (!buf || cap < need)
        return PWREL_ENOSPC;
    unsigned char *p = static_cast<unsigned char *>(buf), *p0 = p;
    put32(p, kModelMagic);
    put32(p, kModelVersion);
    put32(p, (uint32_t)H);
    put32(p, (uint32_t)K);
    putf(p, m->alpha);
    put32(p, (uint32_t)m->precision);
    for (int j = 0; j < H; ++j)
        for (int k = 0; k < K; ++k)
            putf(p, m->w1[j][k]);
    for (int j = 0; j < H; ++j)
        putf(p, m->b1[j]);
    for (int j = 0; j < H; ++j)
        putf(p, m->v[j]);
    putf(p, m->b2);
    const uint64_t h = fnv1a64(p0, (uint64_t)(p - p0));
    std::memcpy(p, &h, 8);
    return PWREL_OK;
}

int pwrel_model_load(const void *buf, uint64_t size, pwrel_mlp *out)
{
    if (!buf || !out)
        return PWREL_EINVAL;
    if (size < 24)
        return PWREL_ECORRUPT;
    const unsigned char *p = static_cast<const unsigned char *>(buf), *p0 = p;
    if (get32(p) != kModelMagic || get32(p) != kModelVersion)
        return PWREL_ECORRUPT;
    const uint32_t H = get32(p), K = get32(p);
    if (H < 2 || H > PWREL_MAX_HIDDEN || (K != 0 && K != 2 && K != 6))
        return PWREL_ECORRUPT;
    const uint64_t need = model_bytes((int)H, (int)K);
    if (size != need)
        return PWREL_ECORRUPT;
    uint64_t h;
    std::memcpy(&h, p0 + need - 8, 8);
    if (h != fnv1a64(p0, need - 8))
        return PWREL_ECORRUPT;
    pwrel_mlp m;
    std::memset(&m, 0, sizeof m);
    m.hidden = (int32_t)H;
    m.inputs = (int32_t)K;
    m.alpha = getf(p);
    m.precision = (int32_t)get32(p);
    for (uint32_t j = 0; j < H; ++j)
        for (uint32_t k = 0; k < K; ++k)
            m.w1[j][k] = getf(p);
    for (uint32_t j = 0; j < H; ++j)
        m.b1[j] = getf(p);
    for (uint32_t j = 0; j < H; ++j)
        m.v[j] = getf(p);
    m.b2 = getf(p);
    if (model_problem(&m, K == 6 ? 3 : (K == 2 ? 2 : 1)))
        return PWREL_ECORRUPT;
    *out = m;
    return PWREL_OK;
}

int pwrel_stream_model(pwrel_ctx *ctx, const void *d_in, uint64_t in_size, pwrel_mlp *out,
                       void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!d_in || !out)
        return fail(ctx, PWREL_EINVAL, "NULL stream or output");
    if (in_size < PWREL_HEADER_BYTES)
        return fail(ctx, PWREL_ECORRUPT, "stream shorter than its header");
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    pwrel_header h;
    hipError_t e = hipMemcpyAsync(&h, d_in, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "header copy");
    pwrel_header v;
    if (pwrel_read_header(&h, in_size, &v) != PWREL_OK)
        return fail(ctx, PWREL_ECORRUPT, "stream header is corrupt or truncated");
    if (!(v.flags & PWREL_HF_NET))
        return fail(ctx, PWREL_EINVAL, "the stream holds no network");
    pwrel_mlp m;
    e = hipMemcpyAsync(&m, static_cast<const unsigned char *>(d_in) + v.off_model, sizeof m,
                       hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "model copy");
    if (model_problem(&m, v.ndim))
        return fail(ctx, PWREL_ECORRUPT, "stream model is invalid");
    *out = m;
    return PWREL_OK;
}

int pwrel_read_header(const void *buf, uint64_t size, pwrel_header *out)
{
    if (!buf || !out || size < sizeof(pwrel_header))
        return PWREL_ECORRUPT;
    pwrel_header h;
    std::memcpy(&h, buf, sizeof h);
    if (h.magic != PWREL_MAGIC || h.version != PWREL_VERSION)
        return PWREL_ECORRUPT;
    if (h.dtype != PWREL_F32 && h.dtype != PWREL_F64)
        return PWREL_ECORRUPT;
    Geom g;
    if (!make_geom(h.dims, h.ndim, h.dtype, h.block, g))
        return PWREL_ECORRUPT;
    if ((uint64_t)g.N != h.n || (uint64_t)g.nblocks != h.nblocks || h.status != PWREL_OK)
        return PWREL_ECORRUPT;
    if (h.flags & ~(PWREL_HF_NET | PWREL_HF_JUDGE | PWREL_HF_INDEPENDENT | PWREL_HF_HUFFMAN))
        return PWREL_ECORRUPT;
    const Layout L = layout_for(g, h.flags);
    if (h.off_model != L.off[0] || h.off_bflags != L.off[1] || h.off_counts != L.off[2])
        return PWREL_ECORRUPT;
    const uint64_t tsize = h.dtype == PWREL_F32 ? 4u : 8u;
    if (h.n_raw > h.n)
        return PWREL_ECORRUPT;
    if (h.flags & PWREL_HF_HUFFMAN) {
        if (h.off_codes != 0 || h.n_sym < 1 || h.n_sym > 65536 || h.n_bits > 16ull * h.n ||
            h.size_bytes != (uint32_t)huff_size_bytes(g) || h.esc_len > 16)
            return PWREL_ECORRUPT;
        uint64_t total = 0;
        const HuffLayout hl = huff_layout(g, L, h.n_sym, h.n_bits, h.n_raw, tsize, total);
        if (h.off_huff != hl.off_huff || h.off_sizes != hl.off_sizes ||
            h.off_bits != hl.off_bits || h.off_raw != align256(hl.off_bits + 4ull * ((h.n_bits + 31) / 32)))
            return PWREL_ECORRUPT;
    } else {
        if (h.off_codes != L.off[3] || h.off_raw != L.off[4] || h.off_huff || h.off_sizes ||
            h.off_bits || h.n_bits || h.n_sym || h.size_bytes || h.esc_len)
            return PWREL_ECORRUPT;
    }
    if (h.total_size != h.off_raw + h.n_raw * tsize || h.total_size > size)
        return PWREL_ECORRUPT;
    if (!(h.w > 0.0) || !std::isfinite(h.w) || !std::isfinite(h.Lp) || !std::isfinite(h.Ln) ||
        !(h.eps > 0.0 && h.eps < 1.0) || !(h.p_zero <= h.b_sign) || h.delta < 0 ||
        h.p_max <= h.b_sign)
        return PWREL_ECORRUPT;
    *out = h;
    return PWREL_OK;
}

}  // extern "C"

namespace {

// what a decompression reads of a stream before its kernels: the header and
// the model that may follow it
struct StreamHead {
    pwrel_header h;
    unsigned char pad[PWREL_HEADER_BYTES - sizeof(pwrel_header)];
    pwrel_mlp m;
};
static_assert(sizeof(pwrel_header) <= PWREL_HEADER_BYTES, "header too large");

// Check a stream's header (held in host memory: `want` bytes of it were
// read) against the caller's field, then queue every decoding kernel on s.
// Leaves the stream's status in ws.status and its decoded balance points in
// ws.n_raw; *hout receives the checked header.
int decompress_launch(pwrel_ctx *ctx, const StreamHead &head, uint64_t want, const void *d_in,
                      uint64_t in_size, void *d_field, const uint64_t *dims, int ndim, int dtype,
                      hipStream_t s, pwrel_header *hout)
{
    hipError_t e;
    pwrel_header h;
    if (pwrel_read_header(&head.h, in_size, &h) != PWREL_OK)
        return fail(ctx, PWREL_ECORRUPT, "stream header is corrupt or truncated");
    if (h.ndim != ndim || h.dtype != dtype)
        return fail(ctx, PWREL_EINVAL, "dims/dtype do not match the stream");
    for (int d = 0; d < ndim; ++d)
        if (h.dims[d] != dims[d])
            return fail(ctx, PWREL_EINVAL, "dims do not match the stream");
    if ((h.flags & PWREL_HF_JUDGE) && !(h.flags & PWREL_HF_NET))
        return fail(ctx, PWREL_ECORRUPT, "judge flag without a network");
    const pwrel_mlp *model = nullptr;
    if (h.flags & PWREL_HF_NET) {
        if (want < PWREL_HEADER_BYTES + sizeof(pwrel_mlp))
            return fail(ctx, PWREL_ECORRUPT, "stream too short for its model");
        model = &head.m;
        if (check_model(ctx, model, ndim) != PWREL_OK)
            return fail(ctx, PWREL_ECORRUPT, "stream model is invalid");
    }
    Geom g;
    make_geom(h.dims, h.ndim, h.dtype, h.block, g);
    int st = ensure_scan(ctx, g);
    if (st)
        return st;
    if ((e = grow(ctx->ws.praw, ctx->ws.praw_cap, (size_t)std::max<uint64_t>(h.n_raw, 1))) !=
        hipSuccess)
        return fail(ctx, PWREL_ENOMEM, "raw grid value allocation failed");
    if (!(h.flags & PWREL_HF_INDEPENDENT)) {
        if ((e = grow(ctx->ws.pgrid, ctx->ws.pgrid_cap, (size_t)g.N)) != hipSuccess)
            return fail(ctx, PWREL_ENOMEM, "grid scratch allocation failed");
        // Done flags and tagged faces: zeroed when (re)allocated; each call
        // uses a new epoch (0 is the value of a fresh word), so words of
        // earlier calls never match.  When the epoch wraps, all are cleared.
        const bool pen = pencil_mode(g);
        const size_t nzf = pen ? (size_t)(g.nb[0] * g.n[1] * g.n[2]) : 0;
        const size_t nyf = pen ? (size_t)(g.nb[1] * g.n[0] * g.n[2]) : 0;
        if (ctx->ws.done_cap < (size_t)g.nblocks) {
            if ((e = grow(ctx->ws.done, ctx->ws.done_cap, (size_t)g.nblocks)) != hipSuccess ||
                (e = hipMemsetAsync(ctx->ws.done, 0, ctx->ws.done_cap * sizeof(unsigned), s)) !=
                    hipSuccess)
                return fail(ctx, PWREL_ENOMEM, "decoder flag allocation failed");
        }
        if (pen && (ctx->ws.zf_cap < nzf || ctx->ws.yf_cap < nyf)) {
            if ((e = grow(ctx->ws.zf, ctx->ws.zf_cap, nzf)) != hipSuccess ||
                (e = hipMemsetAsync(ctx->ws.zf, 0, ctx->ws.zf_cap * 8, s)) != hipSuccess ||
                (e = grow(ctx->ws.yf, ctx->ws.yf_cap, nyf)) != hipSuccess ||
                (e = hipMemsetAsync(ctx->ws.yf, 0, ctx->ws.yf_cap * 8, s)) != hipSuccess)
                return fail(ctx, PWREL_ENOMEM, "decoder face allocation failed");
        }
        if (++ctx->epoch == 0) {
            ctx->epoch = 1;
            if ((ctx->ws.done &&
                 (e = hipMemsetAsync(ctx->ws.done, 0, ctx->ws.done_cap * sizeof(unsigned), s)) !=
                     hipSuccess) ||
                (ctx->ws.zf && (e = hipMemsetAsync(ctx->ws.zf, 0, ctx->ws.zf_cap * 8, s)) !=
                                   hipSuccess) ||
                (ctx->ws.yf && (e = hipMemsetAsync(ctx->ws.yf, 0, ctx->ws.yf_cap * 8, s)) !=
                                   hipSuccess))
                return hip_fail(ctx, e, "decoder flag reset");
        }
        if (ctx->order_nb[0] != g.nb[0] || ctx->order_nb[1] != g.nb[1] ||
            ctx->order_nb[2] != g.nb[2] || ctx->order_pen != (int)pen) {
            std::vector<unsigned> order;
            block_order(g, order);
            if ((long long)order.size() != (pen ? g.nb[0] * g.nb[1] : g.nblocks))
                return fail(ctx, PWREL_EHIP, "internal: block order incomplete");
            if ((e = grow(ctx->order, ctx->order_cap, order.size())) != hipSuccess)
                return fail(ctx, PWREL_ENOMEM, "decoder order allocation failed");
            if ((e = hipMemcpyAsync(ctx->order, order.data(), order.size() * sizeof(unsigned),
                                    hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return hip_fail(ctx, e, "decoder order copy");
            for (int d = 0; d < 3; ++d)
                ctx->order_nb[d] = g.nb[d];
            ctx->order_pen = (int)pen;
        }
    }
    DevConsts c{};
    c.eps = h.eps;
    c.eps0 = h.eps0;
    c.b_a = h.b_a;
    c.w = h.w;
    c.r = h.r;
    c.Lp = h.Lp;
    c.Ln = h.Ln;
    c.d0 = h.d0;
    c.p_zero = h.p_zero;
    c.b_sign = h.b_sign;
    c.n_lo = h.n_lo;
    c.delta = h.delta;
    c.p_max = h.p_max;
    c.w32 = (h.p_max - h.p_zero) < (1LL << 27) ? 1 : 0;
    if ((e = launch_reset(ctx->ws, s)) != hipSuccess)
        return hip_fail(ctx, e, "reset");
    mark(ctx, 4, s);
    const unsigned char *in = static_cast<const unsigned char *>(d_in);
    const uint32_t *counts = reinterpret_cast<const uint32_t *>(in + h.off_counts);
    const uint16_t *codes = reinterpret_cast<const uint16_t *>(in + h.off_codes);
    if (h.flags & PWREL_HF_HUFFMAN) {
        // the decoding kernel checks the codebook's length counts (a prefix
        // code of n_sym symbols) before it reads the table
        if ((st = ensure_huffman(ctx, g)) != PWREL_OK)
            return st;
        if ((e = launch_huff_decode(g, reinterpret_cast<const uint32_t *>(in + h.off_huff),
                                    reinterpret_cast<const uint32_t *>(in + h.off_bits),
                                    (h.n_bits + 31) / 32, in + h.off_sizes, ctx->ws.codes16,
                                    h.n_sym, h.esc_len, ctx->ws, s)) != hipSuccess)
            return hip_fail(ctx, e, "Huffman decode");
        codes = ctx->ws.codes16;
    }
    const uint8_t *bflags = (h.flags & PWREL_HF_JUDGE) ? in + h.off_bflags : nullptr;
    if ((e = launch_scan(counts, g, ctx->ws, s)) != hipSuccess)
        return hip_fail(ctx, e, "scan");
    mark(ctx, 5, s);
    if ((e = launch_raw_grid(g, c, in + h.off_raw, h.n_raw, ctx->ws, s)) != hipSuccess)
        return hip_fail(ctx, e, "raw grid values");
    mark(ctx, 6, s);
    if ((e = launch_decode(g, c, model, h.flags, bflags, codes, counts, in + h.off_raw, h.n_raw,
                           ctx->ws, ctx->order, ctx->epoch, d_field, ctx->num_cus, s)) !=
        hipSuccess)
        return hip_fail(ctx, e, "decode");
    mark(ctx, 7, s);
    if (!(h.flags & PWREL_HF_INDEPENDENT) &&
        (e = launch_inverse(g, c, ctx->ws, d_field, s)) != hipSuccess)
        return hip_fail(ctx, e, "inverse");
    mark(ctx, 8, s);
    *hout = h;
    return PWREL_OK;
}

__global__ void k_fill_i32(int *p, int n, int v)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = v;
}

// one thread: a decoded stream's status and balance-point count into the
// status of a call that decodes several streams (the first error stays)
__global__ void k_accum_status(const int *status, const unsigned long long *n_raw,
                               unsigned long long want, int *acc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0 || *acc != PWREL_OK)
        return;
    if (*status != PWREL_OK)
        *acc = *status;
    else if (*n_raw != want)
        *acc = PWREL_ECORRUPT;
}

}  // namespace

extern "C" {

int pwrel_decompress(pwrel_ctx *ctx, const void *d_in, uint64_t in_size, void *d_field,
                     const uint64_t *dims, int ndim, int dtype, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!d_in || !d_field || !dims)
        return fail(ctx, PWREL_EINVAL, "NULL stream, field or dims");
    if (reinterpret_cast<uintptr_t>(d_in) & 15)
        return fail(ctx, PWREL_EINVAL, "the stream must start 16-byte aligned");
    if (in_size < PWREL_HEADER_BYTES)
        return fail(ctx, PWREL_ECORRUPT, "stream shorter than its header");
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    StreamHead head;
    const uint64_t want = std::min<uint64_t>(in_size, sizeof head);
    std::memset(&head, 0, sizeof head);
    hipError_t e = hipMemcpyAsync(&head, d_in, want, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "header copy");
    pwrel_header h;
    int st = decompress_launch(ctx, head, want, d_in, in_size, d_field, dims, ndim, dtype, s, &h);
    if (st != PWREL_OK)
        return st;
    int dst = 0;
    unsigned long long nr = 0;
    if ((e = hipMemcpyAsync(&dst, ctx->ws.status, sizeof dst, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&nr, ctx->ws.n_raw, sizeof nr, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "status copy");
    if (dst == PWREL_OK && nr != h.n_raw)
        dst = PWREL_ECORRUPT;
    static const int spans[4][3] = {{3, 4, 5}, {5, 5, 6}, {4, 6, 7}, {6, 7, 8}};
    collect(ctx, spans, 4);
    return finish_status(ctx, dst);
}

}  // extern "C"

namespace pwrel {

// Several streams decoded in stream order with two host synchronisations in
// all: one strided copy brings every header (and model) up, the streams'
// kernels are queued one stream after the other, each stream's status and
// balance-point count folded into one word, read at the end.
int api_decompress_many(pwrel_ctx *ctx, const unsigned char *d_in, uint64_t stride,
                        const uint64_t *sizes, size_t n, float *const *outs,
                        const uint64_t (*dims)[3], hipStream_t s)
{
    DeviceGuard guard(ctx->device);
    if (n == 0)
        return PWREL_OK;
    std::vector<StreamHead> heads(n);
    std::memset(heads.data(), 0, n * sizeof(StreamHead));
    hipError_t e;
    if ((e = grow(ctx->mstatus, ctx->mstatus_cap, 1)) != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, "status allocation failed");
    const size_t want = std::min<uint64_t>(stride, sizeof(StreamHead));
    if ((e = hipMemcpy2DAsync(heads.data(), sizeof(StreamHead), d_in, stride, want, n,
                              hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "header copy");
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, ctx->mstatus, 1, PWREL_OK);
    for (size_t i = 0; i < n; ++i) {
        if (sizes[i] < PWREL_HEADER_BYTES || sizes[i] > stride)
            return fail(ctx, PWREL_ECORRUPT, "a stream's length is invalid");
        pwrel_header h;
        const int st = decompress_launch(ctx, heads[i], std::min<uint64_t>(sizes[i], want),
                                         d_in + i * stride, sizes[i], outs[i], dims[i], 3,
                                         PWREL_F32, s, &h);
        if (st != PWREL_OK)
            return st;
        hipLaunchKernelGGL(k_accum_status, dim3(1), dim3(64), 0, s, ctx->ws.status,
                           ctx->ws.n_raw, (unsigned long long)h.n_raw, ctx->mstatus);
    }
    int dst = 0;
    if ((e = hipMemcpyAsync(&dst, ctx->mstatus, sizeof dst, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "status copy");
    return finish_status(ctx, dst);
}

}  // namespace pwrel

extern "C" {

int pwrel_transform(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                    int dtype, double eps, int32_t *d_p, pwrel_header *hdr_out, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (pwrel_check_args(dims, ndim, dtype, eps, 2) != PWREL_OK || !d_field || !d_p)
        return fail(ctx, PWREL_EINVAL, "bad arguments");
    Geom g;
    make_geom(dims, ndim, dtype, 2, g);
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = launch_reset(ctx->ws, s)) != hipSuccess ||
        (e = launch_stats(d_field, g, ctx->ws, s)) != hipSuccess ||
        (e = launch_consts(g, eps, ctx->ws, s)) != hipSuccess ||
        (e = launch_transform(d_field, g, ctx->ws, d_p, s)) != hipSuccess)
        return hip_fail(ctx, e, "transform");
    DevConsts c;
    int dst = 0;
    if ((e = hipMemcpyAsync(&c, ctx->ws.consts, sizeof c, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&dst, ctx->ws.status, sizeof dst, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "constants copy");
    if (dst != PWREL_OK)
        return finish_status(ctx, dst);
    if (hdr_out) {
        pwrel_header h{};
        h.magic = PWREL_MAGIC;
        h.version = PWREL_VERSION;
        h.dtype = dtype;
        h.ndim = ndim;
        for (int d = 0; d < ndim; ++d)
            h.dims[d] = dims[d];
        h.eps = c.eps;
        h.eps0 = c.eps0;
        h.b_a = c.b_a;
        h.w = c.w;
        h.r = c.r;
        h.Lp = c.Lp;
        h.Ln = c.Ln;
        h.d0 = c.d0;
        h.p_zero = c.p_zero;
        h.b_sign = c.b_sign;
        h.n_lo = c.n_lo;
        h.delta = c.delta;
        h.n = (uint64_t)g.N;
        h.abs_min = c.abs_min;
        h.abs_max = c.abs_max;
        h.n_zero = c.n_zero;
        h.n_neg = c.n_neg;
        *hdr_out = h;
    }
    return PWREL_OK;
}

int pwrel_encode_grid(pwrel_ctx *ctx, const int32_t *d_p, const uint64_t *dims, int ndim,
                      int block_size, const pwrel_mlp *model, const pwrel_options *opt_in,
                      uint16_t *d_codes, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    pwrel_options opt{1, 0, 0, 0};
    if (opt_in)
        opt = *opt_in;
    Geom g;
    if (!make_geom(dims, ndim, PWREL_F32, block_size, g) || !d_p || !d_codes)
        return fail(ctx, PWREL_EINVAL, "bad arguments");
    if (opt.judge)
        return fail(ctx, PWREL_EINVAL, "judge is not available on grid input");
    if (opt.use_net) {
        const int st = check_model(ctx, model, ndim);
        if (st)
            return st;
    }
    Tile tile;
    if (!tile_for(g, tile))
        return fail(ctx, PWREL_EINVAL, "block too large for the LDS tile");
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = grow(ctx->counts_scratch, ctx->counts_scratch_cap, (size_t)g.nblocks);
    if (e != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, "count scratch allocation failed");
    if ((e = launch_reset(ctx->ws, s)) != hipSuccess ||
        (e = launch_compress(nullptr, d_p, g, tile, model, opt, ctx->ws, d_codes,
                             ctx->counts_scratch, nullptr, ctx->num_cus, s)) != hipSuccess)
        return hip_fail(ctx, e, "encode_grid");
    int dst = 0;
    if ((e = hipMemcpyAsync(&dst, ctx->ws.status, sizeof dst, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "status copy");
    return finish_status(ctx, dst);
}

int pwrel_detmath(pwrel_ctx *ctx, const double *d_x, double *d_log2, double *d_exp2, uint64_t n,
                  void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!d_x && n)
        return fail(ctx, PWREL_EINVAL, "NULL input");
    DeviceGuard guard(ctx->device);
    const hipError_t e =
        launch_detmath(d_x, d_log2, d_exp2, n, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PWREL_OK : hip_fail(ctx, e, "detmath");
}

int pwrel_fastmath_check(pwrel_ctx *ctx, double *log2_err, double *exp2_rel_err, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!log2_err || !exp2_rel_err)
        return fail(ctx, PWREL_EINVAL, "NULL output");
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long bits[2] = {0, 0};
    hipError_t e;
    if ((e = launch_fastmath_check(ctx->ws.hist, s)) != hipSuccess ||
        (e = hipMemcpyAsync(bits, ctx->ws.hist, sizeof bits, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "fastmath_check");
    std::memcpy(log2_err, &bits[0], sizeof(double));
    std::memcpy(exp2_rel_err, &bits[1], sizeof(double));
    return PWREL_OK;
}

int pwrel_set_profiling(pwrel_ctx *ctx, int enable)
{
    if (!ctx)
        return PWREL_EINVAL;
    DeviceGuard guard(ctx->device);
    if (enable && !ctx->ev_ok) {
        bool ok = true;
        for (hipEvent_t &e : ctx->ev)
            ok = ok && hipEventCreate(&e) == hipSuccess;
        if (!ok)
            return fail(ctx, PWREL_EHIP, "event creation failed");
        ctx->ev_ok = true;
    }
    ctx->profiling = enable ? 1 : 0;
    return PWREL_OK;
}

int pwrel_phase_times(pwrel_ctx *ctx, double *ms, int n)
{
    if (!ctx || !ms || n < 0)
        return PWREL_EINVAL;
    const int k = std::min(n, PWREL_NUM_PHASES);
    for (int i = 0; i < k; ++i)
        ms[i] = ctx->phase_ms[i];
    return k;
}

int pwrel_histogram(pwrel_ctx *ctx, const uint16_t *d_codes, uint64_t n, uint64_t *hist,
                    void *stream)
{
    if (!ctx || !hist || (!d_codes && n))
        return PWREL_EINVAL;
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_hist(d_codes, (long long)n, ctx->ws.hist, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hist, ctx->ws.hist, 65536 * sizeof(uint64_t), hipMemcpyDeviceToHost,
                           s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    return e == hipSuccess ? PWREL_OK : hip_fail(ctx, e, "histogram");
}

int pwrel_huffman_codebook(const uint64_t *hist, uint32_t *count33, uint16_t *syms,
                           uint32_t *n_sym, uint64_t *n_bits)
{
    if (!hist || !count33 || !syms || !n_sym || !n_bits)
        return PWREL_EINVAL;
    HuffTable t;
    if (!huff_build(hist, t))
        return PWREL_EHIP;
    std::memcpy(count33, t.count.data(), (kHuffMaxLen + 1) * sizeof(uint32_t));
    std::memcpy(syms, t.syms.data(), t.syms.size() * sizeof(uint16_t));
    *n_sym = (uint32_t)t.syms.size();
    *n_bits = t.n_bits;
    return PWREL_OK;
}

int pwrel_huffman_trained_codebook(const uint64_t *hist, pwrel_codebook *out)
{
    if (!hist || !out)
        return PWREL_EINVAL;
    HuffTable t;
    uint32_t esc = 0;
    if (!huff_build_trained(hist, t, esc))
        return PWREL_EHIP;
    std::memset(out, 0, sizeof *out);
    std::memcpy(out->count, t.count.data(), (kHuffMaxLen + 1) * sizeof(uint32_t));
    std::memcpy(out->syms, t.syms.data(), t.syms.size() * sizeof(uint16_t));
    out->n_sym = (uint32_t)t.syms.size();
    out->esc_len = esc;
    return PWREL_OK;
}

uint64_t pwrel_huffman_bits(const uint64_t *hist, uint32_t *max_len_out)
{
    // Huffman code lengths by repeated merging of the two lightest subtrees;
    // the coded size is sum(count * length).  A single used symbol costs one
    // bit per occurrence.
    if (!hist)
        return 0;
    struct Node {
        uint64_t w;
        int id;
    };
    auto cmp = [](const Node &a, const Node &b) { return a.w > b.w || (a.w == b.w && a.id > b.id); };
    std::priority_queue<Node, std::vector<Node>, decltype(cmp)> q(cmp);
    std::vector<int> parent;
    std::vector<int> leaf_of;
    for (int s = 0; s < 65536; ++s)
        if (hist[s]) {
            leaf_of.push_back(s);
            q.push({hist[s], (int)parent.size()});
            parent.push_back(-1);
        }
    if (parent.empty()) {
        if (max_len_out)
            *max_len_out = 0;
        return 0;
    }
    if (parent.size() == 1) {
        if (max_len_out)
            *max_len_out = 1;
        return hist[leaf_of[0]];
    }
    while (q.size() > 1) {
        const Node a = q.top();
        q.pop();
        const Node b = q.top();
        q.pop();
        const int id = (int)parent.size();
        parent.push_back(-1);
        parent[a.id] = id;
        parent[b.id] = id;
        q.push({a.w + b.w, id});
    }
    uint64_t bits = 0;
    uint32_t maxl = 0;
    std::vector<uint32_t> depth(parent.size(), 0);
    for (int i = (int)parent.size() - 2; i >= 0; --i)
        depth[i] = depth[parent[i]] + 1;
    for (size_t i = 0; i < leaf_of.size(); ++i) {
        bits += hist[leaf_of[i]] * depth[i];
        maxl = std::max(maxl, depth[i]);
    }
    if (max_len_out)
        *max_len_out = maxl;
    return bits;
}

int pwrel_sample(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim, int dtype,
                 double eps, int block_size, int independent_blocks, double rho, uint64_t seed,
                 uint64_t *d_idx, int32_t *d_u, int32_t *d_t, uint8_t *d_isval, uint64_t cap,
                 uint64_t *n_out, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (pwrel_check_args(dims, ndim, dtype, eps, block_size) != PWREL_OK || !d_field || !n_out)
        return fail(ctx, PWREL_EINVAL, "bad dims/ndim/dtype/bound/block size or NULL pointer");
    if (!(rho > 0.0 && rho <= 1.0))
        return fail(ctx, PWREL_EINVAL, "sampling rate must lie in (0, 1]");
    if (cap > 0 && (!d_idx || !d_t || !d_isval || (ndim > 1 && !d_u)))
        return fail(ctx, PWREL_EINVAL, "NULL output with a nonzero capacity");
    Geom g;
    make_geom(dims, ndim, dtype, block_size, g);
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    SampleArgs a;
    unsigned long long ntr = 0, nva = 0;
    long long nch = 0;
    int st = sample_counts(ctx, d_field, g, eps, independent_blocks, rho, seed, s, a, ntr, nva, nch);
    if (st)
        return st;
    SampleOut o{};
    o.off_tr = ctx->chunk_off;
    o.off_va = ctx->chunk_off + nch;
    if (cap > 0) {
        o.u_all = d_u;
        o.t_all = d_t;
        o.isval = d_isval;
        o.idx_all = reinterpret_cast<unsigned long long *>(d_idx);
        o.cap_all = cap;
        hipError_t e;
        if ((e = launch_sample(false, a, g.D, g.dtype, nullptr, nullptr, &o, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(ctx, e, "sample write");
    }
    *n_out = ntr + nva;
    return PWREL_OK;
}

int pwrel_loss_grad(pwrel_ctx *ctx, const float *d_theta, int hidden, int inputs, float alpha,
                    const float *d_u, const float *d_t, uint64_t n, double sigma, double lambda,
                    float *d_grad, float *loss_out, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!train_shape_ok(hidden, inputs) || n == 0 || !d_theta || !d_t || (inputs && !d_u) ||
        !d_grad || !loss_out || !(sigma > 0.0) || !(lambda >= 0.0) ||
        !(alpha >= 0.0f && alpha <= 1.0f))
        return fail(ctx, PWREL_EINVAL, "bad arguments");
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    GradArgs a{};
    a.H = hidden;
    a.theta = d_theta;
    a.u = d_u;
    a.t = d_t;
    a.n = (long long)n;
    a.sigma = sigma;
    a.lambda = lambda;
    a.alpha = alpha;
    a.grad = d_grad;
    a.loss = reinterpret_cast<float *>(ctx->scal + 300);
    hipError_t e;
    if ((e = launch_loss_grad(hidden, inputs, a, s)) != hipSuccess ||
        (e = hipMemcpyAsync(loss_out, a.loss, sizeof(float), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "loss_grad");
    return PWREL_OK;
}

int pwrel_train_pairs(pwrel_ctx *ctx, const float *d_u, const float *d_t, uint64_t n, int hidden,
                      int inputs, float alpha, double sigma, const float *d_theta0, int n_cand,
                      const double *lr, const double *lambda, int batch, int epochs,
                      float *d_theta_out, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!train_shape_ok(hidden, inputs) || !d_t || (inputs && !d_u) || !d_theta0 ||
        !d_theta_out || !lr || !lambda || n_cand < 1 || n_cand > kMaxTrained || batch < 1 ||
        batch > 256 || epochs < 1 || epochs > 64 || !(sigma > 0.0) ||
        !(alpha >= 0.0f && alpha <= 1.0f))
        return fail(ctx, PWREL_EINVAL, "bad arguments");
    TrainArgs a{};
    for (int c = 0; c < n_cand; ++c) {
        if (!(lr[c] > 0.0 && std::isfinite(lr[c])) || !(lambda[c] >= 0.0 && std::isfinite(lambda[c])))
            return fail(ctx, PWREL_EINVAL, "learning rates must be positive, L2 weights >= 0");
        a.lr[c] = lr[c];
        a.lambda[c] = lambda[c];
    }
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *d_sigma = ctx->scal + 400;
    const double sg = sigma;
    a.H = hidden;
    a.u = d_u;
    a.t = d_t;
    a.n = (long long)n;
    a.sigma = d_sigma;
    a.alpha = alpha;
    a.batch = batch;
    a.epochs = epochs;
    a.theta0 = d_theta0;
    a.theta_out = d_theta_out;
    hipError_t e;
    if ((e = hipMemcpyAsync(d_sigma, &sg, sizeof sg, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_train(hidden, inputs, a, n_cand, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "train_pairs");
    return PWREL_OK;
}

int pwrel_train(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim, int dtype,
                double eps, int block_size, const pwrel_train_options *opt,
                const pwrel_mlp *init, pwrel_mlp *out, pwrel_train_report *report, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (pwrel_check_args(dims, ndim, dtype, eps, block_size) != PWREL_OK || !d_field || !opt ||
        !out)
        return fail(ctx, PWREL_EINVAL, "bad dims/ndim/dtype/bound/block size or NULL pointer");
    const pwrel_train_options &o = *opt;
    if (!(o.rho > 0.0 && o.rho <= 1.0) || o.batch < 1 || o.batch > 256 || o.epochs < 1 ||
        o.epochs > 64 || o.n_lr < 1 || o.n_lr > 4 || o.n_lambda < 1 || o.n_lambda > 4 ||
        (o.precision != 0 && o.precision != 1))
        return fail(ctx, PWREL_EINVAL, "bad training options");
    TrainArgs ta{};
    const int ncand = o.n_lr * o.n_lambda;
    for (int c = 0; c < ncand; ++c) {
        const double l = o.lr[c / o.n_lambda], m = o.lambda[c % o.n_lambda];
        if (!(l > 0.0 && std::isfinite(l)) || !(m >= 0.0 && std::isfinite(m)))
            return fail(ctx, PWREL_EINVAL, "learning rates must be positive, L2 weights >= 0");
        ta.lr[c] = l;
        ta.lambda[c] = m;
    }
    pwrel_mlp m0;
    if (init) {
        m0 = *init;
    } else if (pwrel_mlp_init(&m0, ndim, o.hidden, o.alpha, o.seed) != PWREL_OK) {
        return fail(ctx, PWREL_EINVAL, "bad hidden width for the initial network");
    }
    int st = check_model(ctx, &m0, ndim);
    if (st)
        return st;
    const int H = m0.hidden, K = m0.inputs, P = H * K + 2 * H + 1;
    Geom g;
    make_geom(dims, ndim, dtype, block_size, g);
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t ev[4] = {};
    for (hipEvent_t &e : ev)
        if (hipEventCreate(&e) != hipSuccess)
            e = nullptr;
    auto cleanup = [&]() {
        for (hipEvent_t &e : ev)
            if (e)
                (void)hipEventDestroy(e);
    };
    auto rec = [&](int i) {
        if (ev[i])
            (void)hipEventRecord(ev[i], s);
    };
    rec(0);
    SampleArgs sa;
    unsigned long long ntr = 0, nva = 0;
    long long nch = 0;
    st = sample_counts(ctx, d_field, g, eps, o.independent_blocks, o.rho, o.seed, s, sa, ntr, nva,
                       nch);
    if (st) {
        cleanup();
        return st;
    }
    hipError_t e = grow(ctx->pairs, ctx->pairs_cap,
                        std::max<size_t>(1, (size_t)((ntr + nva) * (unsigned long long)(K + 1))));
    if (e == hipSuccess)
        e = grow(ctx->vhist, ctx->vhist_cap, (size_t)(ncand + 1) * 65536);
    if (e != hipSuccess) {
        cleanup();
        return fail(ctx, PWREL_ENOMEM, "training pair buffers");
    }
    SampleOut so{};
    so.off_tr = ctx->chunk_off;
    so.off_va = ctx->chunk_off + nch;
    so.u_tr = ctx->pairs;
    so.t_tr = so.u_tr + ntr * K;
    so.u_va = so.t_tr + ntr;
    so.t_va = so.u_va + nva * K;
    so.cap_tr = ntr;
    so.cap_va = nva;
    std::vector<float> th0((size_t)P);
    for (int j = 0; j < H; ++j) {
        for (int k = 0; k < K; ++k)
            th0[(size_t)(j * K + k)] = m0.w1[j][k];
        th0[(size_t)(H * K + j)] = m0.b1[j];
        th0[(size_t)(H * K + H + j)] = m0.v[j];
    }
    th0[(size_t)(H * K + 2 * H)] = m0.b2;
    ta.H = H;
    ta.u = so.u_tr;
    ta.t = so.t_tr;
    ta.n = (long long)ntr;
    ta.sigma = ctx->scal;
    ta.alpha = m0.alpha;
    ta.batch = o.batch;
    ta.epochs = o.epochs;
    ta.theta0 = ctx->theta;
    ta.theta_out = ctx->theta + P;
    FoldArgs fa{};
    fa.theta = ctx->theta + P;
    fa.sigma = ctx->scal;
    fa.H = H;
    fa.K = K;
    fa.ncand = ncand;
    fa.init = pack_mlp(&m0);
    fa.nets = ctx->nets;
    ValArgs va{};
    va.u = so.u_va;
    va.t = so.t_va;
    va.n = (long long)nva;
    va.nets = ctx->nets;
    va.hist = ctx->vhist;
    if ((e = launch_sample(false, sa, g.D, g.dtype, nullptr, nullptr, &so, s)) != hipSuccess) {
        cleanup();
        return hip_fail(ctx, e, "sample write");
    }
    rec(1);
    if ((e = launch_sigma(so.t_tr, (long long)ntr, ctx->scal + 1, ctx->scal, s)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->theta, th0.data(), th0.size() * sizeof(float),
                            hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_train(H, K, ta, ncand, s)) != hipSuccess) {
        cleanup();
        return hip_fail(ctx, e, "train");
    }
    rec(2);
    if ((e = launch_fold(fa, s)) != hipSuccess ||
        (e = launch_validate(g.D, hidden_pad(&m0), va, ncand + 1, ctx->scores, s)) !=
            hipSuccess) {
        cleanup();
        return hip_fail(ctx, e, "validate");
    }
    rec(3);
    std::vector<long long> sc((size_t)(ncand + 1));
    std::vector<float> th((size_t)ncand * P);
    double sigma = 1.0;
    if ((e = hipMemcpyAsync(sc.data(), ctx->scores, sc.size() * sizeof(long long),
                            hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(th.data(), ctx->theta + P, th.size() * sizeof(float),
                            hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&sigma, ctx->scal, sizeof sigma, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        cleanup();
        return hip_fail(ctx, e, "training results copy");
    }
    int best = 0;
    for (int c = 1; c <= ncand; ++c)
        if (sc[(size_t)c] > sc[(size_t)best])
            best = c;
    pwrel_mlp res = m0;
    if (best > 0) {
        // the same fold as the validation networks (FP64 then FP32)
        const float *t = th.data() + (size_t)(best - 1) * P;
        for (int j = 0; j < H; ++j) {
            for (int k = 0; k < K; ++k)
                res.w1[j][k] = (float)((double)t[j * K + k] / sigma);
            res.b1[j] = t[H * K + j];
            res.v[j] = (float)((double)t[H * K + H + j] * sigma);
        }
        res.b2 = (float)((double)t[H * K + 2 * H] * sigma);
    }
    res.precision = o.precision;
    if (report) {
        pwrel_train_report r{};
        r.n_train = ntr;
        r.n_val = nva;
        r.sigma = sigma;
        r.chosen = best;
        r.n_candidates = ncand + 1;
        for (int c = 0; c <= ncand; ++c)
            r.val_score[c] = sc[(size_t)c];
        float ms = 0.0f;
        if (ev[0] && ev[1] && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess)
            r.ms_sample = ms;
        if (ev[1] && ev[2] && hipEventElapsedTime(&ms, ev[1], ev[2]) == hipSuccess)
            r.ms_train = ms;
        if (ev[2] && ev[3] && hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess)
            r.ms_select = ms;
        *report = r;
    }
    cleanup();
    *out = res;
    return PWREL_OK;
}

int pwrel_train_codebook(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                         int dtype, double eps, int block_size, const pwrel_mlp *model,
                         const pwrel_options *opt_in, double frac, uint64_t seed,
                         pwrel_codebook *out, void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    if (!out)
        return fail(ctx, PWREL_EINVAL, "NULL codebook");
    if (!(frac > 0.0 && frac <= 1.0))
        return fail(ctx, PWREL_EINVAL, "the validation fraction must lie in (0, 1]");
    pwrel_options opt{1, 0, 0, 0, nullptr};
    if (opt_in)
        opt = *opt_in;
    Geom g;
    Tile tile;
    int st;
    if (!check_compress_args(ctx, d_field, dims, ndim, dtype, eps, block_size, model, opt, g,
                             tile, st))
        return st;
    DeviceGuard guard(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((st = ensure_scan(ctx, g)) != PWREL_OK || (st = ensure_huffman(ctx, g)) != PWREL_OK)
        return st;
    hipError_t e = hipSuccess;
    if (g.dtype == PWREL_F32)
        e = grow(ctx->ws.pgrid, ctx->ws.pgrid_cap, (size_t)g.N);
    if (e == hipSuccess)
        e = grow(ctx->counts_scratch, ctx->counts_scratch_cap, (size_t)g.nblocks);
    if (e == hipSuccess && opt.judge)
        e = grow(ctx->bflags_scratch, ctx->bflags_scratch_cap, (size_t)g.nblocks);
    if (e != hipSuccess)
        return fail(ctx, PWREL_ENOMEM, "scratch allocation failed");
    if ((st = codes_pass(ctx, d_field, g, tile, eps, model, opt, ctx->counts_scratch,
                         opt.judge ? ctx->bflags_scratch : nullptr, s)) != PWREL_OK)
        return st;
    std::vector<uint64_t> hist(65536);
    int dst = 0;
    if ((e = launch_table_hist(ctx->ws.codes16, g, frac, seed, ctx->ws.hist, s)) != hipSuccess ||
        (e = hipMemcpyAsync(hist.data(), ctx->ws.hist, 65536 * sizeof(uint64_t),
                            hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&dst, ctx->ws.status, sizeof dst, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(ctx, e, "validation block histogram");
    if (dst != PWREL_OK)
        return finish_status(ctx, dst);
    if (pwrel_huffman_trained_codebook(hist.data(), out) != PWREL_OK)
        return fail(ctx, PWREL_EHIP, "internal: trained codebook construction failed");
    return PWREL_OK;
}

int pwrel_mlp_init(pwrel_mlp *m, int ndim, int hidden, float alpha, uint64_t seed)
{
    // hidden unit 0 carries the Lorenzo combination of the neighbour
    // differences, unit 1 its negation; output weights +-1/(1+alpha) turn the
    // two leaky-ReLU halves back into the identity; the remaining units get
    // small hashed input weights and zero output weight.
    if (!m || ndim < 1 || ndim > 3 || hidden < 2 || hidden > PWREL_MAX_HIDDEN)
        return PWREL_EINVAL;
    std::memset(m, 0, sizeof *m);
    m->hidden = hidden;
    m->inputs = (1 << ndim) - 2;
    m->alpha = alpha;
    for (int k = 0; k < m->inputs; ++k) {
        const float c = (float)lorenzo_sign(k + 2);
        m->w1[0][k] = c;
        m->w1[1][k] = -c;
    }
    m->v[0] = (float)(1.0 / (1.0 + (double)alpha));
    m->v[1] = -m->v[0];
    for (int j = 2; j < hidden; ++j)
        for (int k = 0; k < m->inputs; ++k) {
            const uint64_t h = splitmix64(seed ^ (uint64_t)(j * m->inputs + k));
            const double u = (double)(h >> 11) * 0x1p-53;
            m->w1[j][k] = (float)(0.1 * (2.0 * u - 1.0));
        }
    return PWREL_OK;
}

}  // extern "C"
