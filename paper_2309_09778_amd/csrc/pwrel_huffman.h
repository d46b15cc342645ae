// Huffman stage of the codec (pwrel_huffman.hip): host codebook, device
// encoder and decoder.  Internal; not part of the ABI.
#pragma once

#include <vector>

#include "pwrel_internal.h"

namespace pwrel {

constexpr int kHuffMaxLen = 32;  // longest codeword (bits)

// The stream's codebook section: uint32 count[kHuffMaxLen + 1] (count[l] =
// symbols of length l, count[0] = 0), then uint16 syms[n_sym] in canonical
// order (by length, then symbol value).
struct HuffTable {
    std::vector<uint32_t> count;  // kHuffMaxLen + 1 entries
    std::vector<uint16_t> syms;
    uint64_t n_bits = 0;          // sum over symbols of count * length
    uint32_t max_len = 0;
};

inline uint64_t huff_table_bytes(uint64_t n_sym) { return 4ull * (kHuffMaxLen + 1) + 2ull * n_sym; }

// optimal lengths (at most kHuffMaxLen bits) from a 65,536-bin histogram;
// false if the lengths fail the Kraft inequality (cannot happen for a valid
// histogram)
bool huff_build(const uint64_t *hist, HuffTable &t);

// bytes per block bit size in the stream (2 when every block fits 65,535 bits)
int huff_size_bytes(const Geom &g);

// encoder: per-block sizes into d_sizes, the packed words into d_bits
// (nwords words, zeroed here first); codes block-major; ws.enc_len,
// ws.enc_code, ws.boffsets, ws.bpartials, ws.bits_total are used
hipError_t launch_huff_encode(const Geom &g, const uint16_t *codes, const uint32_t *d_tab,
                              void *d_sizes, uint32_t *d_bits, unsigned long long nwords,
                              Workspace &ws, hipStream_t s);
// decoder: codes (block-major) from the table (nsym symbols), words and
// per-block sizes
hipError_t launch_huff_decode(const Geom &g, const uint32_t *d_tab, const uint32_t *d_bits,
                              unsigned long long nwords, const void *d_sizes, uint16_t *codes,
                              unsigned nsym, Workspace &ws, hipStream_t s);

}  // namespace pwrel
