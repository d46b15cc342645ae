/*
 * pwrel -- perceptron-predicted point-wise relative (PW_REL) lossy compressor
 * for AMD Instinct MI355X (gfx950), after Chen & Li, arXiv 2309.09778.
 *
 * C ABI.  Every pointer named d_* is a device pointer on the context's GPU;
 * every other pointer is host memory.  Streams are passed as `void *` holding
 * a hipStream_t (NULL = the device's null stream).  Fields are dense C-order
 * arrays: dims[0] is the slowest axis, dims[ndim-1] the fastest.
 *
 * Error behaviour: every entry point returns PWREL_OK (0) or a negative
 * pwrel_status; nothing is thrown across the ABI.  The message of the last
 * failure on a context is available from pwrel_last_error().  On failure the
 * contents of output buffers are unspecified and *out_size is not written.
 * Argument errors are reported before any GPU work is queued.
 *
 * Ownership: the caller owns every field, stream and output buffer.  The
 * context owns its device workspace (grown on demand, freed by
 * pwrel_destroy); a context must not be used from two threads at once.
 */
#ifndef PWREL_H
#define PWREL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { PWREL_F32 = 0, PWREL_F64 = 1 } pwrel_dtype;

typedef enum {
    PWREL_OK = 0,
    PWREL_EINVAL = -1,     /* bad argument (dims, ndim, dtype, bound, block size, model) */
    PWREL_ERANGE = -2,     /* a grid value would leave +-2^30 (bound too tight for the range) */
    PWREL_ENONFINITE = -3, /* the field holds NaN or Inf */
    PWREL_ENOSPC = -4,     /* output capacity too small */
    PWREL_ECORRUPT = -5,   /* stream header or sections inconsistent */
    PWREL_EHIP = -6,       /* a HIP runtime call failed */
    PWREL_ENOMEM = -7      /* device or host allocation failed */
} pwrel_status;

#define PWREL_MAX_HIDDEN 32
#define PWREL_MAX_INPUTS 6
#define PWREL_HEADER_BYTES 512
#define PWREL_MAGIC 0x4C455750u /* "PWEL" little-endian */
#define PWREL_VERSION 1u

/*
 * The three-layer perceptron (Sec. 4.2, Fig. 3).  Inputs are the K = 2^ndim - 2
 * neighbour differences u_k = n_{k+2} - n_1 of grid values on the prediction
 * surface (n_1 = previous point along the fastest axis; neighbour o steps back
 * by one along axis ndim-1-i for every set bit i of o); hidden layer of
 * `hidden` leaky-ReLU units with slope `alpha`; one linear output y.  The
 * prediction is n_1 + rint(clamp(y, -2^30, 2^30)).
 *
 * precision 0: evaluated in FP32 on the vector ALUs in a fixed order with
 *   explicit fused multiply-adds: z_j = fma(w1[j][K-1], u_{K-1}, ... fma(w1[j][0],
 *   u_0, b1[j])), h_j = z_j < 0 ? z_j * alpha : z_j, y = fma(v[H-1], h_{H-1},
 *   ... fma(v[0], h_0, b2)).  Bit-identical to the CPU oracle.
 * precision 1: the hidden layer on the matrix cores, 64 points per wave:
 *   z = b1 + bf16(w1) bf16(u) (BF16 products, FP32 accumulation), then, using
 *   lrelu(z) = (1 - alpha) relu(z) + alpha z,
 *   y = b2 + sum_j bf16((1 - alpha) v_j) relu(bf16(z_j)) + bf16(alpha v_j) bf16(z_j)
 *   on the vector ALU (exact BF16 products, FP32 fused multiply-adds in a
 *   fixed order).  Encoder and decoder issue the same instructions on the
 *   same operands, so streams are self-consistent; the PW_REL bound is
 *   enforced by the quantizer and verification either way.
 */
typedef struct {
    int32_t hidden;    /* H, 2..32 */
    int32_t inputs;    /* K = 2^ndim - 2 */
    float alpha;       /* leaky-ReLU slope, 0 <= alpha <= 1 */
    float w1[PWREL_MAX_HIDDEN][PWREL_MAX_INPUTS];
    float b1[PWREL_MAX_HIDDEN];
    float v[PWREL_MAX_HIDDEN];
    float b2;
    int32_t precision; /* 0 = FP32 vector ALU, 1 = BF16 matrix cores */
} pwrel_mlp;

/*
 * A Huffman codebook built once by the training phase (Sec. 4.3: one table
 * from the code frequencies of the validation blocks, reused for every block
 * of the compression; Sec. 5 rebuilds it to decode).  Codes the validation
 * never produced share an escape codeword, followed in the stream by the
 * code's own 16 bits (most significant first); with an escape no codeword is
 * longer than 16 bits.  Filled by pwrel_train_codebook or
 * pwrel_huffman_trained_codebook; host memory, owned by the caller.
 */
typedef struct {
    uint32_t count[33];   /* count[l] = codewords of l bits, the escape included; count[0] = 0 */
    uint32_t n_sym;       /* entries of syms (the sum of count) */
    uint32_t esc_len;     /* bits of the escape codeword; 0 = no escape (every code listed) */
    uint16_t syms[65536]; /* the symbols in canonical order (by length, then value); the
                             escape is the last of its length and is stored as 0 */
} pwrel_codebook;

/* Compression options; pass NULL for the defaults (all zero except use_net = 1). */
typedef struct {
    int32_t use_net;            /* 0: one-layer Lorenzo everywhere; 1: network where all
                                   neighbours exist (needs a model) */
    int32_t judge;              /* 1 (needs use_net): per block keep the network only if the
                                   empirical entropy of its codes is strictly below that of
                                   Lorenzo's codes (flag per block in the stream).  Every
                                   distinct code of the block (code 0 included) is a symbol;
                                   compared as J = sum over symbols of c rint(2^32 log2 c),
                                   higher J = lower entropy (Sec. 4.3: the codes are
                                   entropy-coded) */
    int32_t independent_blocks; /* 0: the prediction surface crosses block faces (halo mode);
                                   1: neighbours outside the block count as missing, so every
                                   block decodes on its own (Sec. 4.4.2) */
    int32_t entropy;            /* 0: the stream stores 16-bit codes; 1: the codes are
                                   Huffman coded (Sec. 4.1 coding stage, Algorithm 1: optimal
                                   codeword lengths of at most 32 bits from this field's code
                                   histogram, canonical codewords); where the codebook would
                                   cost more than it saves, the stream keeps the 16-bit codes
                                   (no PWREL_HF_HUFFMAN flag).  pwrel_compress only */
    const pwrel_codebook *codebook; /* entropy = 1 only (else ignored): NULL = the codebook of
                                   this field's histogram, as above; else this trained codebook
                                   (host memory, read during the call), no histogram pass; where
                                   its coded size is not below the 16-bit codes, the stream
                                   keeps them */
} pwrel_options;

/*
 * Stream header (first PWREL_HEADER_BYTES of every stream, little-endian).
 * Sections follow at the stated byte offsets, each 256-byte aligned:
 *   model  : pwrel_mlp                      (if flags & PWREL_HF_NET)
 *   bflags : uint8  [nblocks], 1 = network  (if flags & PWREL_HF_JUDGE)
 *   counts : uint32 [nblocks]   code-0 points per block
 *   codes  : uint16 [n]         block-major: blocks in raster order, points in
 *                               local raster order; code = e + 2^15 with
 *                               e = prediction - grid value, 0 = balance point
 *   raw    : dtype  [n_raw]     input values of the code-0 points, same order
 * With PWREL_HF_HUFFMAN the codes section is replaced by three sections
 * (off_codes = 0), and raw follows them:
 *   huff   : uint32 count[33]    count[l] = codewords of l bits (count[0] = 0),
 *            uint16 syms[n_sym]  the coded symbols in canonical order (by
 *                                length, then value); codeword of the i-th
 *                                symbol of length l = first[l] + its rank among
 *                                them, first[1] = 0, first[l] = (first[l-1] +
 *                                count[l-1]) << 1 (RFC 1951 canonical code)
 *   sizes  : uint16 (size_bytes = 2) or uint32 (4) [nblocks]  bits of each block
 *   bits   : uint32 [ceil(n_bits / 32)]  the blocks' codewords in stream order,
 *                                most significant bit first, no padding between
 *                                blocks (block b starts at the sum of the sizes
 *                                before it)
 */
#define PWREL_HF_NET 1
#define PWREL_HF_JUDGE 2
#define PWREL_HF_INDEPENDENT 4
#define PWREL_HF_HUFFMAN 8
typedef struct {
    uint32_t magic, version;
    int32_t dtype, ndim;
    uint64_t dims[3];
    int32_t block, flags;
    double eps;   /* relative bound b_r */
    double eps0;  /* stand-in magnitude of zero */
    double b_a;   /* log2(1 + eps), Eq. 8 */
    double w;     /* grid step 2 b_a */
    double r;     /* 1 / w */
    double Lp;    /* log2 factor_pos, Eq. 9 */
    double Ln;    /* log2 factor_neg, Eq. 10 */
    double d0;    /* log-domain image of zero, Eq. 12 */
    int64_t p_zero, b_sign, n_lo, delta; /* grid thresholds and negative offset */
    uint64_t n, nblocks, n_raw;
    uint64_t off_model, off_bflags, off_counts, off_codes, off_raw, total_size;
    double abs_min, abs_max;
    uint64_t n_zero, n_neg;
    int32_t status; /* device-side status of the producing call (0 = ok) */
    uint32_t esc_len; /* PWREL_HF_HUFFMAN: bits of the escape codeword (0 = none), see
                         pwrel_codebook */
    /* Huffman sections (PWREL_HF_HUFFMAN; else all 0) */
    uint64_t off_huff, off_sizes, off_bits;
    uint64_t n_bits;      /* coded bits of all blocks */
    uint32_t n_sym;       /* symbols of the codebook */
    uint32_t size_bytes;  /* bytes per block bit size (2 or 4) */
    int64_t p_max;        /* bound on every grid value: b_sign, or the grid value of the
                             largest-magnitude negative, plus one step */
} pwrel_header;

typedef struct pwrel_ctx pwrel_ctx;

/* Create a context on HIP device `device` (allocates a small workspace). */
int pwrel_create(pwrel_ctx **out, int device);
void pwrel_destroy(pwrel_ctx *ctx);
const char *pwrel_last_error(const pwrel_ctx *ctx);
const char *pwrel_status_string(int status);

/* Limits on block_size: 1-D 2..4096, 2-D 2..64, 3-D 2..16. */
int pwrel_check_args(const uint64_t *dims, int ndim, int dtype, double rel_error_bound,
                     int block_size);

/* Upper bound of the stream size in bytes (0 if the arguments are invalid). */
uint64_t pwrel_compress_bound(const uint64_t *dims, int ndim, int dtype, int block_size);

/*
 * Compress (Algorithm 1 with the transform of Sec. 3.2, the predictor of
 * Sec. 4.1/4.2 fed with grid-snapped actual values per Sec. 4.4.1, and the
 * 2^16-code quantizer with balance points).  Every point of the result
 * decompresses to x^ with |x - x^| <= eps |x|, the sign of x, and x^ = 0
 * exactly where x = 0.  model may be NULL when opt->use_net = 0.  Writes the
 * stream to d_out (capacity out_capacity bytes, 16-byte aligned, as every
 * device allocation is) and its length to *out_size; synchronises `stream`
 * once to learn that length.  PWREL_EINVAL for an unaligned d_out.
 */
int pwrel_compress(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                   int dtype, double rel_error_bound, int block_size, const pwrel_mlp *model,
                   const pwrel_options *opt, void *d_out, uint64_t out_capacity,
                   uint64_t *out_size, void *stream);

/*
 * Decompress a stream (Sec. 5): blocks in dependency order (block levels in
 * halo mode, all at once with independent blocks), grid values rebuilt from the
 * same prediction, x^ = exact inverse transform rounded to dtype; code-0 points
 * take their raw value.  dims/ndim/dtype must match the header; d_in must start
 * 16-byte aligned (PWREL_EINVAL otherwise).  Synchronises `stream` to read the
 * header and, at the end, the decoders' status.
 */
int pwrel_decompress(pwrel_ctx *ctx, const void *d_in, uint64_t in_size, void *d_field,
                     const uint64_t *dims, int ndim, int dtype, void *stream);

/* Validate a header held in host memory (no GPU work). */
int pwrel_read_header(const void *buf, uint64_t size, pwrel_header *out);

/*
 * pwrel_compress_raw: the computation of pwrel_compress (Algorithm 1) with
 * the stream's sections returned in separate caller buffers instead of one
 * stream, for inspection and bit-exact checking:
 *   d_codes  uint16 [n]        block-major codes (as the stream's codes section)
 *   d_counts uint32 [nblocks]  code-0 points per block
 *   d_bflags uint8  [nblocks]  per-block predictor flag (needed iff opt->judge;
 *                              else may be NULL)
 *   d_raw    dtype  [raw_capacity] raw values of the code-0 points, stream order
 *   header_out (host)          the header the stream would carry (constants,
 *                              n_raw, section offsets, total_size, status)
 * Synchronizes `stream` once.  Errors as pwrel_compress; PWREL_ENOSPC when
 * more than raw_capacity values are unpredictable.
 */
int pwrel_compress_raw(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                       int dtype, double rel_error_bound, int block_size,
                       const pwrel_mlp *model, const pwrel_options *opt, uint16_t *d_codes,
                       uint32_t *d_counts, uint8_t *d_bflags, void *d_raw,
                       uint64_t raw_capacity, pwrel_header *header_out, void *stream);

/*
 * pwrel_compress_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels, stream and errors as pwrel_compress,
 * but every device scratch buffer (statistics records, constants, status,
 * raw counter, judge table, per-block scan, the FP32 grid-value field) lies
 * in one static device array of the library (about 24 MiB per GPU, held by
 * each GPU the library runs on until the process ends); nothing is allocated
 * or freed, and the context's own workspace is not touched.  The array's
 * address is looked up, and its constant table filled, by pwrel_create on
 * the context's device.  Limits: at most 2^22 values and 2^20 blocks per
 * field, else PWREL_EINVAL (with a message) before any GPU work.  Every call
 * on one GPU shares that GPU's array (it keeps the last call's contents;
 * each call clears what must start at zero), so calls that overlap on one
 * GPU, from any context or stream, race: the caller serialises them.
 * Synchronises `stream` once to read the stream length.
 */
int pwrel_compress_noalloc(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                           int dtype, double rel_error_bound, int block_size,
                           const pwrel_mlp *model, const pwrel_options *opt, void *d_out,
                           uint64_t out_capacity, uint64_t *out_size, void *stream);
#define PWREL_NOALLOC_MAX_VALUES (1ull << 22)
#define PWREL_NOALLOC_MAX_BLOCKS (1ull << 20)

/*
 * pwrel_compress_batch: n FP32 fields, each compressed into its own stream
 * exactly as pwrel_compress would (Algorithm 1 per field: the field's own
 * statistics and constants, Eq. 8-12, its codes, counts, raw values and
 * header; byte-identical streams), by one fixed sequence of about ten
 * launches whatever n and the shapes: one persistent compression launch per
 * class over every tile of its fields, and one launch per per-field stage
 * over a field table.  Classes: 3-D fields with block 8 and 2-D fields with
 * block 16 (the compiled batched tile shapes).
 *   fields[i]       (host) d_field (device, C order), dims/ndim (2 or 3),
 *                   reserved = 0, d_out (device, out_capacity bytes,
 *                   16-byte aligned; at least the header + codes part, else
 *                   PWREL_ENOSPC)
 *   block_size[3]   (host, or NULL) block edge by ndim - 1; 0 = default
 *                   (16 for 2-D, 8 for 3-D); others give PWREL_EINVAL
 *   models[3]       (host, or NULL) network by ndim - 1, needed for every
 *                   dimensionality present when opt->use_net; copied
 *   opt             as pwrel_compress; entropy must be 0 (16-bit codes)
 *   d_out_sizes[n]  (device) each stream's length, 0 where that field
 *                   failed; the field's status is in its stream header
 * Ordered on `stream`; no synchronisation and no device allocation once the
 * request was seen.  The context keeps the field table of the last request
 * (fields, bound, blocks, models, options, d_out_sizes): a call that repeats
 * it launches kernels only, so it may run under HIP graph capture and be
 * replayed; a new request builds the table (host work, allocation on growth,
 * one asynchronous copy) and is refused with PWREL_EINVAL under capture.
 * Calls sharing a context run in stream order; concurrent calls on one
 * context from different streams race on its workspace.
 */
typedef struct {
    const void *d_field;
    uint64_t dims[3];
    int32_t ndim;
    int32_t reserved;
    void *d_out;
    uint64_t out_capacity;
} pwrel_field_desc;

int pwrel_compress_batch(pwrel_ctx *ctx, int n, const pwrel_field_desc *fields, int dtype,
                         double rel_error_bound, const int *block_size,
                         const pwrel_mlp *const *models, const pwrel_options *opt,
                         uint64_t *d_out_sizes, void *stream);

/*
 * Data blocks (Sec. 5: a stream carries factor_pos and factor_neg for its data
 * block; Algorithm 1 computes them from the extreme values of its input).  A
 * 3-D FP32 field (dims[3], C order, device) is split into data blocks: its
 * sub-volumes of edge `sub` (a positive multiple of 8; the last along an
 * axis clipped), in raster order.  Each is compressed into its own stream
 * with its own statistics, factors and constants, byte for byte the stream
 * pwrel_compress writes for that sub-volume alone (block 8, 16-bit codes,
 * `model` and *opt as there; entropy must be 0).
 *  pwrel_compress_datablocks - stream i goes to d_out + i * out_stride
 *      (device; out_stride a multiple of 256 of at least the header + codes of
 *      a data block, d_out 16-byte aligned), its length to d_sizes[i] (device,
 *      0 for a failed data block, as pwrel_compress_batch); *n_sub_out (host)
 *      receives the number of data blocks.  One gather kernel copies the
 *      sub-volumes contiguous into the context's staging (grown to the field),
 *      then one batched compression runs; synchronises the stream once
 *      before the gather (the data-block table).
 *  pwrel_decompress_datablocks - the field back from those streams: sizes
 *      (host, the n_sub lengths), d_in / in_stride as written.  One strided
 *      copy brings every header up; each stream is checked and decoded as
 *      pwrel_decompress does, all of them queued back to back; one scatter
 *      kernel puts the sub-volumes in place; the first failing stream's
 *      status is returned (two host synchronisations in all).  Errors:
 *      PWREL_EINVAL for bad arguments, PWREL_ECORRUPT for a length outside
 *      the stride or a damaged stream.
 */
int pwrel_compress_datablocks(pwrel_ctx *ctx, const float *d_field, const uint64_t *dims,
                              double rel_error_bound, int sub, const pwrel_mlp *model,
                              const pwrel_options *opt, void *d_out, uint64_t out_stride,
                              uint64_t *d_sizes, uint64_t *n_sub_out, void *stream);
int pwrel_decompress_datablocks(pwrel_ctx *ctx, const void *d_in, uint64_t in_stride,
                                const uint64_t *sizes, float *d_field, const uint64_t *dims,
                                int sub, void *stream);

/*
 * Tile shapes of the batched compression launch.  A tile is the group of
 * whole blocks one workgroup predicts at a time; it schedules work only, so
 * every shape gives the same streams.  Each class has PWREL_BATCH_TILES
 * shapes (3-D block 8: 8x8x32, 8x16x16, 16x16x16; 2-D block 16: 16x128,
 * 32x64, 16x256), variant 0 by default; the context keeps one per class.
 *  pwrel_batch_set_tiles - variant[2] (host): 3-D class, then 2-D class;
 *      PWREL_EINVAL outside 0 .. PWREL_BATCH_TILES - 1.
 *  pwrel_batch_get_tiles - the context's variants into variant[2], and
 *      their tile extents (z, y, x) into shapes[6] unless it is NULL.
 *  pwrel_compress_batch_tune - the autotuner: runs the request (arguments
 *      as pwrel_compress_batch) with each variant, `reps` timed runs after a
 *      warm-up, times each class's compression launch with HIP events, and
 *      keeps the variant of median-fastest time per class in the context
 *      (variant_out[2], host, may be NULL; ms_out[2][PWREL_BATCH_TILES]
 *      medians, host, may be NULL; 0 for an absent class).  Ends with the
 *      request's outputs written by the chosen variants and the stream
 *      synchronised.  Not under capture (PWREL_EINVAL).
 */
/*
 * pwrel_openloop: the paper's literal data selection (Sec. 4.4.1 and 4.4.2:
 * predict from the neighbours' actual values), run as a measurement beside
 * the codec.  The compressor predicts every point from its neighbours' raw
 * log-domain values (the continuous grid coordinate (log2|x| + L) r, before
 * rounding; Eq. 6, 7); the decompressor can only predict from its own
 * reconstructions, so errors accumulate and the PW_REL bound can break.
 * The paper's controls: balance points stored raw (Sec. 4.3, Sec. 5) at the
 * first point of every block (Sec. 4.4.2), where a code leaves the m-bit
 * range, and deliberately after `gap` points of a block without one
 * (Sec. 4.4.1(b); gap 0 = none); m chosen by coverage (Sec. 4.3: closest to
 * 50% below a 1.5% bound, to 80% from 1.5% up).  Independent blocks; the
 * network (model, or NULL for Lorenzo) is evaluated in FP32 on
 * u_k = float(t_{k+2} - t_1).  Codes: c = rint(prediction - t), code
 * c + 2^(m-1) where |c| < 2^(m-1), 0 = balance point.
 *   mbits        2..16, or 0: chosen by coverage (one more pass)
 *   d_codes      uint16 [n] (device) block-major codes
 *   d_counts     uint32 [nblocks] (device) balance points per block
 *   d_raw        dtype [raw_capacity] (device) balance-point values, stream order
 *   d_xhat       dtype [n] (device) the open-loop decoder's reconstruction
 *   report       (host) n_raw, points violating the bound (sign and zero
 *                included), the largest relative error, the histogram of the
 *                bits the prediction errors need (hist[m]: first fitting m
 *                bits, 17 = none), the m and gap used
 * Synchronises `stream`.  PWREL_ENOSPC when raw_capacity is too small.
 */
typedef struct {
    uint64_t n_raw;
    uint64_t violations;
    double max_rel_error;
    uint64_t hist[18];
    int32_t mbits;
    int32_t gap;
} pwrel_openloop_report;

int pwrel_openloop(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                   int dtype, double rel_error_bound, int block_size, const pwrel_mlp *model,
                   int mbits, int gap, uint16_t *d_codes, uint32_t *d_counts, void *d_raw,
                   uint64_t raw_capacity, void *d_xhat, pwrel_openloop_report *report,
                   void *stream);

#define PWREL_BATCH_TILES 3
int pwrel_batch_set_tiles(pwrel_ctx *ctx, const int *variant);
int pwrel_batch_get_tiles(pwrel_ctx *ctx, int *variant, int *shapes);
int pwrel_compress_batch_tune(pwrel_ctx *ctx, int n, const pwrel_field_desc *fields, int dtype,
                              double rel_error_bound, const int *block_size,
                              const pwrel_mlp *const *models, const pwrel_options *opt,
                              uint64_t *d_out_sizes, int reps, int *variant_out, double *ms_out,
                              void *stream);

/*
 * A trained network kept for later fields (Sec. 5: the model trained in the
 * training phase is retained and used to compress; Sec. 4.3).  pwrel_mlp is a
 * plain value owned by the caller, so nothing is allocated or freed here.
 *  pwrel_model_save - serialise *m (host) into buf (host, cap bytes): magic
 *      "PWMD", version 1, hidden, inputs, alpha, precision, then w1 [H][K],
 *      b1 [H], v [H], b2 as little-endian FP32, then an FNV-1a 64-bit checksum
 *      of everything before it.  *size receives the byte count (also when
 *      buf is NULL or cap is too small: then PWREL_ENOSPC).  PWREL_EINVAL for
 *      an invalid network.
 *  pwrel_model_load - parse and validate such bytes into *out; PWREL_ECORRUPT
 *      if the magic, version, sizes or checksum do not match or the network
 *      is invalid.
 *  pwrel_stream_model - the network stored in a stream (device memory,
 *      in_size bytes) into *out (host); PWREL_EINVAL if the stream has none,
 *      PWREL_ECORRUPT if its header or model is invalid.  Synchronizes.
 */
int pwrel_model_save(const pwrel_mlp *m, void *buf, uint64_t cap, uint64_t *size);
int pwrel_model_load(const void *buf, uint64_t size, pwrel_mlp *out);
int pwrel_stream_model(pwrel_ctx *ctx, const void *d_in, uint64_t in_size, pwrel_mlp *out,
                       void *stream);

/*
 * Inspection entry points (same kernels as the codec):
 *  pwrel_transform   - statistics, constants and grid value of every point
 *                      (Sec. 3.2, Eq. 6-12); header constants to *hdr_out.
 *  pwrel_encode_grid - prediction and codes of a given int32 grid field with
 *                      every point taken as verified (Sec. 4.1/4.2, Algorithm 1);
 *                      codes in stream order.
 *  pwrel_detmath     - the device's deterministic log2/exp2 on n doubles.
 */
int pwrel_transform(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                    int dtype, double rel_error_bound, int32_t *d_p, pwrel_header *hdr_out,
                    void *stream);
int pwrel_encode_grid(pwrel_ctx *ctx, const int32_t *d_p, const uint64_t *dims, int ndim,
                      int block_size, const pwrel_mlp *model, const pwrel_options *opt,
                      uint16_t *d_codes, void *stream);
int pwrel_detmath(pwrel_ctx *ctx, const double *d_x, double *d_log2, double *d_exp2, uint64_t n,
                  void *stream);

/*
 * Histogram (65536 bins, host output) of n codes held on the device (e.g. the
 * codes section of a stream), and the size in bits of those codes under a
 * Huffman code built from the histogram (Sec. 4.1: the coding stage after
 * quantisation; used for the ratio report).  pwrel_histogram synchronises.
 */
int pwrel_histogram(pwrel_ctx *ctx, const uint16_t *d_codes, uint64_t n, uint64_t *hist65536,
                    void *stream);
uint64_t pwrel_huffman_bits(const uint64_t *hist65536, uint32_t *max_len_out);

/*
 * The codebook a Huffman stream stores for a code histogram (host only; Sec.
 * 4.1 Huffman stage): count33[l] = symbols given l-bit codewords (l = 0..32,
 * count33[0] = 0), syms (capacity 65,536) = the used symbols in canonical
 * order (by length, then value), *n_sym their number, *n_bits = sum over
 * symbols of count * length.  Lengths are those of an optimal prefix code
 * whenever its longest codeword has at most 32 bits (else a valid code with
 * lengths capped at 32).  Returns PWREL_OK, or PWREL_EINVAL for a NULL
 * argument.
 */
int pwrel_huffman_codebook(const uint64_t *hist65536, uint32_t *count33, uint16_t *syms,
                           uint32_t *n_sym, uint64_t *n_bits);

/*
 * The trained codebook of a validation code histogram (host only; Sec. 4.3):
 * the paper averages the counts per validation block, a common factor, so
 * the totals give the same table.  Leaves: every code with a non-zero count,
 * and, when some code has none, the escape, weighted by the number of codes
 * seen exactly once (at least 1).  Lengths: the optimal prefix code of the
 * leaves with no codeword longer than 16 bits (32 when every code was seen),
 * by package-merge; ties between equal weights go to the smaller code, the
 * escape after every code.  Returns PWREL_OK, or PWREL_EINVAL for a NULL
 * argument.
 */
int pwrel_huffman_trained_codebook(const uint64_t *hist65536, pwrel_codebook *out);

/*
 * Device time per phase of the last pwrel_compress / pwrel_decompress on this
 * context, in milliseconds, from HIP events recorded on the caller's stream
 * while profiling is enabled (off by default; enabling adds no host sync).
 * Phases: 0 statistics + constants, 1 compression kernels (FP32: grid
 * values and bound checks, then the fused prediction / quantisation kernel),
 * 2 scan + raw scatter + header (and, for Huffman streams, the histogram,
 * the host codebook and the encoder), 3 decoder scan (and Huffman decoding),
 * 4 decoder main kernel
 * (block levels, pencils or independent blocks), 5 decoder grid values of
 * the raw values, 6 decoder inverse map of the scratch grid field (halo
 * mode; 0 otherwise).  Returns the number of phases written (<= n).
 */
#define PWREL_NUM_PHASES 7
int pwrel_set_profiling(pwrel_ctx *ctx, int enable);
int pwrel_phase_times(pwrel_ctx *ctx, double *ms, int n);

/*
 * Learned part (Sec. 4.3; Fig. 4): draw training pairs from the field itself,
 * train several (learning rate, L2) candidates at once on the device (one
 * workgroup each: forward, backward and Adam in FP32), keep the candidate
 * whose validation codes have the lowest empirical entropy (the untrained
 * network, i.e. Lorenzo, is candidate 0, so the result is never worse on the
 * validation set), and return it with the scale folded in.
 *
 * Sampling: point i is drawn iff U(i) < rho, U(i) = (splitmix64(seed ^ i) >> 11)
 * 2^-53; it is a validation pair iff U(i) < 0.2 rho (8:2 split).  Only points
 * whose neighbours all exist (inside the block when independent_blocks is set)
 * and whose 2^ndim grid values (point and neighbours) lie in one sign range
 * are kept, and only if every input u_k = n_{k+2} - n_1 and the target
 * t = p - n_1 satisfy |.| < 2^15.
 * Loss per candidate: mean over each minibatch of 0.5 (y(u / s) - t / s)^2 plus
 * (lambda / 2)(|w1|^2 + |v|^2), s = max(1, RMS of the training targets);
 * minibatches in pair order, Adam (beta 0.9 / 0.999, epsilon 1e-8) from the
 * initial network's weights taken as scaled-domain parameters.
 * Selection: validation codes of each candidate's FP32 network (raw domain:
 * w1 / s, b1, v s, b2 s), score J = sum over code values of c rint(2^32 log2 c)
 * (higher J = lower entropy); the highest J wins, ties to the lower index.
 */
#define PWREL_MAX_CANDIDATES 17 /* the untrained network + up to 4 x 4 trained */
typedef struct {
    double rho;            /* sampling rate, 0 < rho <= 1 */
    uint64_t seed;
    int32_t hidden;        /* H of the trained network, 2..32 (init == NULL only) */
    int32_t epochs;        /* passes over the training pairs, 1..64 (the paper: one) */
    int32_t batch;         /* minibatch size, 1..256 */
    int32_t n_lr, n_lambda; /* 1..4 each; candidate 1 + a n_lambda + b = (lr[a], lambda[b]) */
    int32_t independent_blocks;
    double lr[4], lambda[4];
    float alpha;           /* leaky-ReLU slope in [0, 1] (init == NULL only) */
    int32_t precision;     /* precision stored in the returned network (0 or 1) */
} pwrel_train_options;

typedef struct {
    uint64_t n_train, n_val;
    double sigma;
    int32_t chosen;                           /* 0 = untrained network */
    int32_t n_candidates;                     /* 1 + n_lr n_lambda */
    int64_t val_score[PWREL_MAX_CANDIDATES];  /* J of each candidate's validation codes */
    double ms_sample, ms_train, ms_select;    /* device time per phase */
} pwrel_train_report;

/*
 * pwrel_train: d_field as for pwrel_compress (device, C order); init = the
 * starting network (host; NULL = pwrel_mlp_init(ndim, opt->hidden, opt->alpha,
 * opt->seed)); *out (host) receives the chosen network, *report (host,
 * optional) the counts, scale, scores and phase times.  Synchronizes the
 * stream.  Errors: PWREL_EINVAL for bad arguments (no pairs drawn is not an
 * error: the untrained network is returned), the field's own errors as for
 * pwrel_compress, PWREL_ENOMEM when the pair buffers cannot be allocated.
 */
int pwrel_train(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim, int dtype,
                double rel_error_bound, int block_size, const pwrel_train_options *opt,
                const pwrel_mlp *init, pwrel_mlp *out, pwrel_train_report *report, void *stream);

/*
 * The Huffman table of the training phase (Sec. 4.3: the compression is
 * simulated on the validation set, each code's frequency is averaged per
 * block, and one table built from them serves every block of the
 * compression).  The field is compressed with `model` and *opt (use_net,
 * judge, independent_blocks; entropy and codebook ignored) into the
 * context's workspace; the validation set is the blocks b (raster order of
 * the blocks) with u01(splitmix64(seed ^ b)) < frac, u01 = the top 53 bits
 * scaled to [0, 1); their codes' counts give the table as
 * pwrel_huffman_trained_codebook builds it.  frac in (0, 1]; the paper's
 * validation share is 0.02 (a 10 % sample split 8:2).  *out (host) receives
 * the table; pass it as pwrel_options.codebook, for this field or for others
 * like it.  Synchronizes the stream.  Errors as pwrel_compress, and
 * PWREL_EINVAL for a NULL out or frac outside (0, 1].
 */
int pwrel_train_codebook(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim,
                         int dtype, double rel_error_bound, int block_size, const pwrel_mlp *model,
                         const pwrel_options *opt, double frac, uint64_t seed,
                         pwrel_codebook *out, void *stream);

/*
 * Training pieces on their own (same kernels as pwrel_train), for checking.
 * Device pointers carry the d_ prefix; all calls synchronize the stream.
 *  pwrel_sample     - the pairs of a field in ascending point order: d_idx (point
 *                     index), d_u (int32 [n][K], K = 2^ndim - 2), d_t (int32),
 *                     d_isval (u8, 1 = validation); writes at most cap pairs
 *                     (any of the four may be NULL only when cap is 0) and
 *                     returns the total in *n_out.
 *  pwrel_loss_grad  - loss (host *loss_out) and gradient (d_grad, P floats) of
 *                     the scaled-domain parameters d_theta ([w1 (H x K) | b1 (H)
 *                     | v (H) | b2], FP32, P = H K + 2 H + 1) on n pairs (d_u
 *                     FP32 [n][K], d_t FP32 [n]), mean over all n pairs.
 *  pwrel_train_pairs- Adam training of n_cand (1..16) candidates from d_theta0
 *                     (P floats) on given pairs; candidate c uses lr[c] and
 *                     lambda[c] (host arrays); d_theta_out [n_cand][P].
 */
int pwrel_sample(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims, int ndim, int dtype,
                 double rel_error_bound, int block_size, int independent_blocks, double rho,
                 uint64_t seed, uint64_t *d_idx, int32_t *d_u, int32_t *d_t, uint8_t *d_isval,
                 uint64_t cap, uint64_t *n_out, void *stream);
int pwrel_loss_grad(pwrel_ctx *ctx, const float *d_theta, int hidden, int inputs, float alpha,
                    const float *d_u, const float *d_t, uint64_t n, double sigma, double lambda,
                    float *d_grad, float *loss_out, void *stream);
int pwrel_train_pairs(pwrel_ctx *ctx, const float *d_u, const float *d_t, uint64_t n, int hidden,
                      int inputs, float alpha, double sigma, const float *d_theta0, int n_cand,
                      const double *lr, const double *lambda, int batch, int epochs,
                      float *d_theta_out, void *stream);

/*
 * FP32 fields take fast paths for the transform and the bound check: the
 * hardware log2 (v_log_f32 on the significand in [sqrt(1/2), sqrt(2)), plus
 * the exponent) and exp2 (v_exp_f32 on the fraction of the exponent).  A fast
 * result is used only where these bounds prove it equal to the FP64 result:
 *   |fast_log2(a) - det_log2(a)| <= PWREL_FAST_LOG2_ERR  (every normal float a > 0)
 *   |v_exp_f32(f) - 2^f| <= PWREL_FAST_EXP2_ERR * 2^f    (every float |f| <= 1/2)
 * so the output is identical to the FP64 path's.  pwrel_fastmath_check
 * measures both maxima on the device over every such input (a few ms) and
 * writes them to the two host doubles; the bounds hold iff each is <= its
 * constant.  Synchronizes the stream.
 */
#define PWREL_FAST_LOG2_ERR 0x1p-20
#define PWREL_FAST_EXP2_ERR 0x1p-20
int pwrel_fastmath_check(pwrel_ctx *ctx, double *log2_err, double *exp2_rel_err, void *stream);

/* Network that reproduces Lorenzo exactly (end of Sec. 4.2). */
int pwrel_mlp_init(pwrel_mlp *out, int ndim, int hidden, float alpha, uint64_t seed);

#ifdef __cplusplus
}
#endif

#endif /* PWREL_H */
