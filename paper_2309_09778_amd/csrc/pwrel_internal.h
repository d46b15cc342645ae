// Internal interface between the C ABI (pwrel_api.hip) and the kernels
// (pwrel_codec.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/pwrel.h"
#include "pwrel_device.h"

namespace pwrel {

// Field geometry padded to three axes: axis 2 is the fastest.  Axes that are
// not among the last `D` have extent 1, block edge 1 and no neighbours.
struct Geom {
    int D;
    int B;
    int dtype;
    long long n[3];
    int bd[3];        // block edge per axis (B or 1)
    long long nb[3];  // blocks per axis
    long long N;
    long long nblocks;
};

// Tile of whole blocks handled by one workgroup iteration of the compressor.
struct Tile {
    int t[3];         // tile extent per axis (multiple of bd)
    long long nt[3];  // tiles per axis
    long long ntiles;
};

constexpr int kStatParts = 1024;  // per-workgroup statistics records

// Device workspace owned by a context.
struct Workspace {
    DevStats *stats = nullptr;            // kStatParts records
    DevConsts *consts = nullptr;
    int *status = nullptr;
    unsigned long long *hist = nullptr;   // 65536 bins
    unsigned long long *n_raw = nullptr;  // total balance points
    unsigned long long *offsets = nullptr;  // per-block exclusive prefix (nblocks)
    unsigned long long *partials = nullptr; // per-scan-chunk totals
    size_t offsets_cap = 0, partials_cap = 0;
    int *pgrid = nullptr;  // decoder grid-value scratch (N int32)
    size_t pgrid_cap = 0;
    int *praw = nullptr;   // decoder: grid values of the raw values (n_raw int32)
    size_t praw_cap = 0;
    long long *qtab = nullptr;  // rint(2^32 log2 c), c = 0 .. kQtab - 1 (judge scores)
    unsigned *done = nullptr;   // halo-mode decoder: per-block done flags (epoch values)
    size_t done_cap = 0;
    unsigned *ticket = nullptr; // halo-mode decoder: next block ticket
    // pencil decoder: tagged z faces (nb0 x n1 x n2) and y faces (nb1 x n0 x n2)
    unsigned long long *zf = nullptr, *yf = nullptr;
    size_t zf_cap = 0, yf_cap = 0;
    // Huffman stage: 16-bit codes between the coder and the predictor stage
    // (N), encoder tables (65,536 lengths and codewords), per-block bit
    // offsets (exclusive scan: per block and per scan chunk) and total bits
    uint16_t *codes16 = nullptr;
    size_t codes16_cap = 0;
    uint8_t *enc_len = nullptr;
    unsigned long long *enc_code = nullptr;  // codeword | length << 32; while decoding, the
                                             // decoder's lookup table
    unsigned long long *boffsets = nullptr, *bpartials = nullptr;
    size_t boffsets_cap = 0, bpartials_cap = 0;
    unsigned long long *bits_total = nullptr;
    // decoders: x^ of every grid value in [p_zero, p_max] (kInvTable entries of
    // the field's dtype at most; allocated with the context)
    void *invtab = nullptr;
};

constexpr long long kInvTable = 1 << 16;
// entries of the decoders' inverse table for these constants (0: none)
inline long long inv_table_size(const DevConsts &c)
{
    const long long n = c.p_max - c.p_zero + 1;
    return (n > 0 && n <= kInvTable) ? n : 0;
}

// Field geometry as a kernel argument.
struct GeoArgs {
    long long n[3];
    int bd[3];
    long long nb[3];
    long long nblocks;
};

// One field of a batched launch: its input, geometry, outputs and
// constants; tiles tile0 .. tile0 + ntiles - 1 of the launch are its tiles.
struct FieldDesc {
    const void *x;
    const int *pfield;
    long long n[3];
    long long nb[3];
    long long nt[3];
    long long tile0;
    uint16_t *codes;
    uint32_t *counts;
    uint8_t *bflags;
    const DevConsts *consts;
    int *status;
};

// what the header kernel writes besides the device constants (host-built)
constexpr int kHeaderGaps = 8;
struct HeaderArgs {
    int dtype, ndim, block, flags;
    unsigned long long dims[3];
    unsigned long long n, nblocks;
    unsigned long long off_model, off_bflags, off_counts, off_codes, off_raw;
    unsigned long long capacity;
    int raw_size;
    unsigned long long pad_lo[kHeaderGaps], pad_hi[kHeaderGaps];  // gaps between sections
    // Huffman sections (0 without them)
    unsigned long long off_huff, off_sizes, off_bits, n_bits;
    unsigned n_sym, size_bytes, esc_len;
};
// One field of pwrel_compress_batch for the batched statistics, constants,
// grid entries, scan, raw scatter, model and header kernels (device table).
struct BatchField {
    const void *x;
    int vec;                   // x 16-byte aligned
    int pad0;
    GeoArgs g;
    long long N;
    double eps;
    long long part0, nparts;   // statistics records of the field
    long long chunk0, nchunks; // scan chunks (kScanChunk blocks) of the field
    long long blk0;            // first block in the batch's block numbering
    long long echunk0;         // first grid-entry chunk (kEntryChunk values)
    uint16_t *codes;
    uint32_t *counts;
    uint8_t *bflags;
    void *raw;
    unsigned long long raw_cap;
    void *model_dst;           // the stream's model section, or nullptr
    void *header;
    unsigned long long *out_size;  // device: the stream's length (0 on error)
    int *pgrid;                // grid entries of an FP32 field
    DevConsts *consts;
    int *status;
    unsigned long long *n_raw;
    HeaderArgs h;
};
constexpr long long kEntryChunk = 8192;

constexpr int kQtab = 4097;

constexpr int kScanChunk = 4096;

// Kernel launchers (return the launch error, if any).
hipError_t launch_reset(Workspace &ws, hipStream_t s);
void block_order(const Geom &g, std::vector<unsigned> &order);
bool pencil_mode(const Geom &g);
hipError_t launch_stats(const void *x, const Geom &g, Workspace &ws, hipStream_t s);
hipError_t launch_consts(const Geom &g, double eps, Workspace &ws, hipStream_t s);
hipError_t launch_transform(const void *x, const Geom &g, Workspace &ws, int *d_p, hipStream_t s);
// pfield: grid field input instead of x (entries: 2 p + failed-check bit, from
// launch_grid_entries; else plain p with every check passed)
hipError_t launch_compress(const void *x, const int *pfield, const Geom &g, const Tile &tile,
                           const pwrel_mlp *model, const pwrel_options &opt, Workspace &ws,
                           uint16_t *codes, uint32_t *counts, uint8_t *bflags, int num_cus,
                           hipStream_t s, bool entries = false);
// grid value and bound check of every FP32 value, one entry each (2 p + failed-check bit)
hipError_t launch_grid_entries(const float *x, const Geom &g, Workspace &ws, int *ent,
                               hipStream_t s);
hipError_t launch_scan(const uint32_t *counts, const Geom &g, Workspace &ws, hipStream_t s);
// exclusive scan of n per-block sizes (uint16 or uint32): offsets per block
// relative to their scan chunk, chunk bases in partials, the sum in *total
hipError_t launch_scan_sizes(const void *sizes, int elem_bytes, long long n,
                             unsigned long long *offs, unsigned long long *partials,
                             unsigned long long *total, hipStream_t s);
hipError_t launch_scatter(const void *x, const Geom &g, const uint16_t *codes,
                          const uint32_t *counts, Workspace &ws, void *raw,
                          unsigned long long raw_cap, hipStream_t s);
// Placement of the Huffman sections of a stream (host-computed)
struct HuffLayout {
    uint64_t off_huff, off_sizes, off_bits, n_bits, table_bytes;
    uint32_t n_sym, size_bytes, esc_len;
};
HeaderArgs make_header_args(const Geom &g, int flags, const uint64_t *offs, uint64_t capacity,
                            bool stream_gaps, const HuffLayout *hl);
// stream_gaps: zero the alignment gaps between the sections that follow
// d_header; hl: the Huffman sections (offs[3], the codes offset, unused)
hipError_t launch_header(const Geom &g, int flags, const uint64_t *offs, Workspace &ws,
                         void *d_header, uint64_t capacity, bool stream_gaps, hipStream_t s,
                         const HuffLayout *hl = nullptr);
// the network into the stream's model section (a kernel, no host copy)
hipError_t launch_write_model(const pwrel_mlp &m, void *dst, hipStream_t s);
hipError_t launch_decode(const Geom &g, const DevConsts &c, const pwrel_mlp *model, int flags,
                         const uint8_t *bflags, const uint16_t *codes, const uint32_t *counts,
                         const void *raw, unsigned long long n_raw, Workspace &ws,
                         const unsigned *order, unsigned epoch, void *xh, int num_cus,
                         hipStream_t s);
hipError_t launch_raw_grid(const Geom &g, const DevConsts &c, const void *raw,
                           unsigned long long n_raw, Workspace &ws, hipStream_t s);
hipError_t launch_inverse(const Geom &g, const DevConsts &c, Workspace &ws, void *xh,
                          hipStream_t s);
hipError_t launch_detmath(const double *x, double *l2, double *e2, uint64_t n, hipStream_t s);
hipError_t launch_fastmath_check(unsigned long long *out2, hipStream_t s);
hipError_t launch_hist(const uint16_t *codes, long long n, unsigned long long *hist,
                       hipStream_t s);

bool tile_for(const Geom &g, Tile &tile);

// --- batched compression (pwrel_compress_batch) ------------------------------------
bool batch_shape(int D, int B);  // classes the batched compressor is compiled for
// reset, statistics (records: nparts), constants
hipError_t launch_batch_front(const BatchField *d_fields, int nf, int dtype, long long nparts,
                              DevStats *records, hipStream_t s);
hipError_t launch_grid_entries_batch(const BatchField *d_fields, int nf, long long nchunks,
                                     hipStream_t s);
hipError_t launch_compress_batch(const FieldDesc *d_fields, int nfields, long long ntiles,
                                 const Geom &g, const Tile &tile, int variant,
                                 const pwrel_mlp *model, const pwrel_options &opt,
                                 const long long *qtab, int num_cus, hipStream_t s);
// scan, raw scatter, model (models: device, [3] by ndim - 1, or nullptr),
// header of every field
hipError_t launch_batch_back(const BatchField *d_fields, int nf, int dtype, long long nchunks,
                             long long nblocks, unsigned long long *offsets,
                             unsigned long long *partials, const pwrel_mlp *models,
                             hipStream_t s);

// --- host helpers shared by the entry points --------------------------------------
constexpr uint64_t align256(uint64_t v) { return (v + 255u) & ~uint64_t(255u); }

inline int max_block(int ndim) { return ndim == 1 ? 4096 : (ndim == 2 ? 64 : 16); }

// C-order dims padded to three axes (false if the arguments are invalid)
inline bool make_geom(const uint64_t *dims, int ndim, int dtype, int B, Geom &g)
{
    if (!dims || ndim < 1 || ndim > 3 || B < 2 || B > max_block(ndim))
        return false;
    if (dtype != PWREL_F32 && dtype != PWREL_F64)
        return false;
    g.D = ndim;
    g.B = B;
    g.dtype = dtype;
    g.N = 1;
    g.nblocks = 1;
    for (int d = 0; d < 3; ++d) {
        const int src = d - (3 - ndim);
        const uint64_t nd = src >= 0 ? dims[src] : 1;
        if (nd < 1 || nd > (uint64_t(1) << 40))
            return false;
        g.n[d] = (long long)nd;
        g.bd[d] = src >= 0 ? B : 1;
        g.nb[d] = (g.n[d] + g.bd[d] - 1) / g.bd[d];
        if (g.N > (1LL << 42) / g.n[d])
            return false;
        g.N *= g.n[d];
        g.nblocks *= g.nb[d];
    }
    return true;
}

// byte offsets of the stream sections (model, bflags, counts, codes, raw)
struct Layout {
    uint64_t off[5];
};

inline Layout layout_for(const Geom &g, int flags)
{
    Layout L;
    uint64_t o = PWREL_HEADER_BYTES;
    L.off[0] = o;
    if (flags & PWREL_HF_NET)
        o = align256(o + sizeof(pwrel_mlp));
    L.off[1] = o;
    if (flags & PWREL_HF_JUDGE)
        o = align256(o + (uint64_t)g.nblocks);
    L.off[2] = o;
    o = align256(o + 4ull * (uint64_t)g.nblocks);
    L.off[3] = o;
    o = align256(o + 2ull * (uint64_t)g.N);
    L.off[4] = o;
    return L;
}

inline int flags_of(const pwrel_options &opt)
{
    return (opt.use_net ? PWREL_HF_NET : 0) | (opt.judge ? PWREL_HF_JUDGE : 0) |
           (opt.independent_blocks ? PWREL_HF_INDEPENDENT : 0) |
           (opt.entropy ? PWREL_HF_HUFFMAN : 0);
}

// why a network cannot be used on an ndim field, or nullptr
inline const char *model_problem(const pwrel_mlp *m, int ndim)
{
    if (!m)
        return "model is NULL but use_net is set";
    if (m->hidden < 2 || m->hidden > PWREL_MAX_HIDDEN)
        return "model hidden width must be 2..32";
    if (m->inputs != (1 << ndim) - 2)
        return "model inputs must equal 2^ndim - 2";
    if (m->precision != 0 && m->precision != 1)
        return "model precision must be 0 (FP32) or 1 (BF16 matrix cores)";
    if (!(m->alpha >= 0.0f && m->alpha <= 1.0f))
        return "leaky-ReLU slope must lie in [0, 1]";
    auto bad = [](float v) { return !(v == v) || v > 65536.0f || v < -65536.0f; };
    if (bad(m->b2))
        return "model weights must be finite and below 2^16";
    for (int j = 0; j < m->hidden; ++j) {
        if (bad(m->b1[j]) || bad(m->v[j]))
            return "model weights must be finite and below 2^16";
        for (int k = 0; k < m->inputs; ++k)
            if (bad(m->w1[j][k]))
                return "model weights must be finite and below 2^16";
    }
    return nullptr;
}

// Where the sections of one compression go (device pointers), and how the
// header is written.
struct Sections {
    uint16_t *codes;
    uint32_t *counts;
    uint8_t *bflags;           // judge only
    void *raw;
    uint64_t raw_cap;          // values
    void *header;              // device, PWREL_HEADER_BYTES
    bool stream_gaps;          // header is the start of a stream: zero its alignment gaps
    void *model;               // device destination of the model, or nullptr
    uint64_t header_capacity;  // stream capacity (raw overflow -> ENOSPC in the header)
};

// the compression launches of one field (pwrel_api.hip); mark_fn (optional)
// is called with phase marks 0..3 between them
hipError_t compress_launches(Workspace &ws, int num_cus, const void *d_field, const Geom &g,
                             const Tile &tile, double eps, const pwrel_mlp *model,
                             const pwrel_options &opt, const Sections &sec, hipStream_t s,
                             void (*mark_fn)(void *, int, hipStream_t), void *mark_arg);

// --- entry-point helpers (pwrel_api.hip) used by entry points in other files -----
// argument checks of pwrel_compress (the message goes to the context)
bool api_check_compress(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                        int dtype, double eps, int block_size, const pwrel_mlp *model,
                        const pwrel_options &opt, Geom &g, Tile &tile, int &st);
int api_fail(pwrel_ctx *ctx, int code, const char *msg);
int api_status(pwrel_ctx *ctx, int device_status);  // status of a finished call, with message
int api_device(const pwrel_ctx *ctx);
int api_num_cus(const pwrel_ctx *ctx);
const long long *api_qtab(const pwrel_ctx *ctx);  // the judge's q(c) table
// the context's batched-compression state (created on first use, released
// by pwrel_destroy through batch_release)
struct BatchState;
BatchState *&api_batch_state(pwrel_ctx *ctx);
void batch_release(BatchState *b);
// the context's open-loop state (coordinate scratch, report counters)
struct OlState;
OlState *&api_ol_state(pwrel_ctx *ctx);
void ol_release(OlState *o);
Workspace &api_ws(pwrel_ctx *ctx);
// n FP32 3-D streams at d_in + i * stride (lengths sizes[i], host) decoded
// into outs[i] (dims[i]) in stream order, with two host synchronisations
int api_decompress_many(pwrel_ctx *ctx, const unsigned char *d_in, uint64_t stride,
                        const uint64_t *sizes, size_t n, float *const *outs,
                        const uint64_t (*dims)[3], hipStream_t s);
// the context's data-block staging: n floats and nsub offsets (grown on demand)
hipError_t api_dstage(pwrel_ctx *ctx, size_t n, size_t nsub, float **stage,
                      unsigned long long **offs);
int api_ensure_scan(pwrel_ctx *ctx, const Geom &g);  // per-block scan buffers

// static scratch of pwrel_compress_noalloc (pwrel_noalloc.hip): set up once
// per device by pwrel_create, with that device current
hipError_t noalloc_setup(int device);

}  // namespace pwrel
