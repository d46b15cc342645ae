// pwrel_compress_noalloc: compression (the kernels of pwrel_compress) with
// every device scratch buffer carved from one file-scope device array, so the
// call allocates nothing.  For callers that cannot allocate device memory
// (code under graph capture, tight serving loops).
//
// The array `scratch` is a per-device object of the code object: each GPU
// holds its own copy at its own address.  Host code never uses the array's
// name as an address; pwrel_create (once per device, with that device
// current) looks the address up with hipGetSymbolAddress and fills the
// judge's constant table in it, and the entry point uses only that address.
// Every call on a device shares the device's array: two calls that overlap
// on one GPU race.  Each call clears what must start at zero (status, raw
// counter) with its reset kernel.
#include <mutex>
#include <string>

#include "pwrel_internal.h"
#include "pwrel_train.h"

namespace pwrel {

// Limits of the static scratch
constexpr uint64_t kNoAllocMaxValues = PWREL_NOALLOC_MAX_VALUES;
constexpr uint64_t kNoAllocMaxBlocks = PWREL_NOALLOC_MAX_BLOCKS;

namespace {

constexpr uint64_t a256(uint64_t v) { return (v + 255u) & ~uint64_t(255u); }

// byte layout of the scratch array
constexpr uint64_t kOffStats = 0;
constexpr uint64_t kOffConsts = a256(kOffStats + kStatParts * sizeof(DevStats));
constexpr uint64_t kOffStatus = a256(kOffConsts + sizeof(DevConsts));
constexpr uint64_t kOffNraw = kOffStatus + 256;
constexpr uint64_t kOffTicket = kOffNraw + 256;
constexpr uint64_t kOffQtab = kOffTicket + 256;
constexpr uint64_t kOffPartials = a256(kOffQtab + kQtab * sizeof(long long));
constexpr uint64_t kOffOffsets =
    a256(kOffPartials + (kNoAllocMaxBlocks / kScanChunk + 1) * sizeof(unsigned long long));
constexpr uint64_t kOffGrid = a256(kOffOffsets + kNoAllocMaxBlocks * sizeof(unsigned long long));
constexpr uint64_t kScratchBytes = a256(kOffGrid + kNoAllocMaxValues * sizeof(int));

}  // namespace

}  // namespace pwrel

// ~24 MiB per device, zero-initialised when the code object is loaded
static __device__ __align__(256) unsigned char scratch[pwrel::kScratchBytes];

namespace pwrel {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};  // scratch address per device (from the symbol lookup)

unsigned char *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

Workspace scratch_workspace(unsigned char *base)
{
    Workspace ws;
    ws.stats = reinterpret_cast<DevStats *>(base + kOffStats);
    ws.consts = reinterpret_cast<DevConsts *>(base + kOffConsts);
    ws.status = reinterpret_cast<int *>(base + kOffStatus);
    ws.n_raw = reinterpret_cast<unsigned long long *>(base + kOffNraw);
    ws.ticket = reinterpret_cast<unsigned *>(base + kOffTicket);
    ws.qtab = reinterpret_cast<long long *>(base + kOffQtab);
    ws.partials = reinterpret_cast<unsigned long long *>(base + kOffPartials);
    ws.partials_cap = kNoAllocMaxBlocks / kScanChunk + 1;
    ws.offsets = reinterpret_cast<unsigned long long *>(base + kOffOffsets);
    ws.offsets_cap = kNoAllocMaxBlocks;
    ws.pgrid = reinterpret_cast<int *>(base + kOffGrid);
    ws.pgrid_cap = kNoAllocMaxValues;
    return ws;
}

}  // namespace

// Set-up of the scratch array on `device` (the caller has made it current):
// look up its address and fill the judge's constant table.  Once per device;
// later calls return at once.  Called by pwrel_create.
hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device])
        return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    if (!p)
        return hipErrorInvalidSymbol;
    unsigned char *base = static_cast<unsigned char *>(p);
    if ((e = launch_qtable(reinterpret_cast<long long *>(base + kOffQtab), kQtab, nullptr)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(nullptr)) != hipSuccess)
        return e;
    g_ptr[device] = base;
    return hipSuccess;
}

}  // namespace pwrel

using namespace pwrel;

extern "C" int pwrel_compress_noalloc(pwrel_ctx *ctx, const void *d_field, const uint64_t *dims,
                                      int ndim, int dtype, double eps, int block_size,
                                      const pwrel_mlp *model, const pwrel_options *opt_in,
                                      void *d_out, uint64_t out_capacity, uint64_t *out_size,
                                      void *stream)
{
    if (!ctx)
        return PWREL_EINVAL;
    pwrel_options opt{1, 0, 0, 0};
    if (opt_in)
        opt = *opt_in;
    Geom g;
    Tile tile;
    int st;
    if (!api_check_compress(ctx, d_field, dims, ndim, dtype, eps, block_size, model, opt, g, tile,
                            st))
        return st;
    if (!d_out || !out_size)
        return api_fail(ctx, PWREL_EINVAL, "NULL output or size pointer");
    if (reinterpret_cast<uintptr_t>(d_out) & 15)
        return api_fail(ctx, PWREL_EINVAL, "the output must start 16-byte aligned");
    if (opt.entropy)
        return api_fail(ctx, PWREL_EINVAL, "pwrel_compress_noalloc stores 16-bit codes (entropy = 0)");
    if ((uint64_t)g.N > kNoAllocMaxValues || (uint64_t)g.nblocks > kNoAllocMaxBlocks)
        return api_fail(ctx, PWREL_EINVAL,
                        "pwrel_compress_noalloc: the field exceeds the static scratch (at most "
                        "2^22 values and 2^20 blocks); use pwrel_compress");
    const int flags = flags_of(opt);
    const Layout L = layout_for(g, flags);
    if (out_capacity < L.off[4])
        return api_fail(ctx, PWREL_ENOSPC, "output capacity below header + codes");
    const int device = api_device(ctx);
    unsigned char *base = noalloc_scratch(device);
    if (!base)
        return api_fail(ctx, PWREL_EHIP, "static scratch was not set up on this device");
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess)
        prev = -1;
    if (prev != device && hipSetDevice(device) != hipSuccess)
        return api_fail(ctx, PWREL_EHIP, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Workspace ws = scratch_workspace(base);
    unsigned char *out = static_cast<unsigned char *>(d_out);
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
    hipError_t e = compress_launches(ws, api_num_cus(ctx), d_field, g, tile, eps, model, opt, sec,
                                     s, nullptr, nullptr);
    pwrel_header h;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&h, out, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (prev >= 0 && prev != device)
        (void)hipSetDevice(prev);
    if (e != hipSuccess)
        return api_fail(ctx, PWREL_EHIP,
                        (std::string("compress_noalloc: ") + hipGetErrorString(e)).c_str());
    if (h.status != PWREL_OK)
        return api_status(ctx, h.status);
    *out_size = h.total_size;
    return PWREL_OK;
}
