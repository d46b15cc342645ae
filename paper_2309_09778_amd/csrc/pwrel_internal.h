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
};

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
hipError_t launch_scatter(const void *x, const Geom &g, const uint16_t *codes,
                          const uint32_t *counts, Workspace &ws, void *raw,
                          unsigned long long raw_cap, hipStream_t s);
hipError_t launch_header(const Geom &g, int flags, const uint64_t *offs, Workspace &ws,
                         void *d_header, uint64_t capacity, hipStream_t s);
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

}  // namespace pwrel
