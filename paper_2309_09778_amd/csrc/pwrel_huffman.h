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

// the escape symbol of a trained codebook (an index past the 16-bit codes)
constexpr uint32_t kHuffEsc = 65536;
// the trained codebook (lengths of at most 16 bits with an escape, 32
// without) from validation code counts; esc_len = the escape's length (0 =
// none); the escape is listed as 0, last among the symbols of its length
bool huff_build_trained(const uint64_t *hist, HuffTable &t, uint32_t &esc_len);

// bytes per block bit size in the stream (2 when every block fits 65,535 bits)
int huff_size_bytes(const Geom &g);

// encoder: per-block sizes into d_sizes, the packed words into d_bits
// (nwords words, zeroed here first); codes block-major; ws.enc_len,
// ws.enc_code, ws.boffsets, ws.bpartials, ws.bits_total are used
hipError_t launch_huff_encode(const Geom &g, const uint16_t *codes, const uint32_t *d_tab,
                              void *d_sizes, uint32_t *d_bits, unsigned long long nwords,
                              Workspace &ws, hipStream_t s);
// the encoder's two halves: encoder tables (esc_len: the table's escape
// length, 0 = none), per-block sizes and their scan (total in ws.bits_total);
// then the zeroed bit section and the packing
hipError_t launch_huff_sizes(const Geom &g, const uint16_t *codes, const uint32_t *d_tab,
                             unsigned esc_len, void *d_sizes, Workspace &ws, hipStream_t s);
hipError_t launch_huff_pack(const Geom &g, const uint16_t *codes, const void *d_sizes,
                            uint32_t *d_bits, unsigned long long nwords, Workspace &ws,
                            hipStream_t s);
// decoder: codes (block-major) from the table (nsym symbols, escape of
// esc_len bits or none), words and per-block sizes
hipError_t launch_huff_decode(const Geom &g, const uint32_t *d_tab, const uint32_t *d_bits,
                              unsigned long long nwords, const void *d_sizes, uint16_t *codes,
                              unsigned nsym, unsigned esc_len, Workspace &ws, hipStream_t s);

}  // namespace pwrel
