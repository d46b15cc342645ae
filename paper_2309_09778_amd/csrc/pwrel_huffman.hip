// Huffman coding of the quantisation codes (Sec. 4.1: the codes go through a
// Huffman coding stage after quantisation; Algorithm 1 writes Huffman codes to
// the stream; Sec. 5 rebuilds the Huffman tree to decompress).
//
// Codebook: optimal code lengths from the field's 65,536-bin code histogram
// (host; at most kHuffMaxLen bits), canonical codewords (shorter codes first,
// equal lengths in symbol order), stored in the stream as the number of
// symbols of each length and the symbols in canonical order.
//
// Encoder (device): per-block bit sizes (one wave per block, a wave sum of
// code lengths), an exclusive scan of the sizes, then one wave per block packs
// its codewords MSB-first into 32-bit words: each lane places its codeword at
// the wave prefix of the lengths in an LDS copy of the block's words, and the
// wave stores them (its two boundary words, shared with the neighbouring
// blocks, by atomic OR into a zeroed bit section).
//
// Decoder (device): one thread per block from its own bit offset, a 64-bit
// bit buffer refilled one word at a time; codewords of up to kLutBits bits in
// one LDS table lookup, longer ones by the canonical limits of each length.
#include <algorithm>
#include <vector>

#include "pwrel_huffman.h"
#include "pwrel_kernels.h"

namespace pwrel {

// ---------------------------------------------------------------------------
// host: code lengths and canonical order
// ---------------------------------------------------------------------------
namespace {

// Huffman lengths by merging the two lightest subtrees (two sorted queues:
// leaves by weight, then merged nodes in the order they are made, which is
// non-decreasing in weight).  Returns the largest length.
uint32_t huffman_depths(const std::vector<std::pair<uint64_t, uint32_t>> &leaves,
                        std::vector<uint32_t> &depth)
{
    const size_t n = leaves.size();
    depth.assign(n, 0);
    if (n == 1) {
        depth[0] = 1;
        return 1;
    }
    std::vector<uint64_t> iw(n - 1);
    std::vector<uint32_t> iparent(n - 1, 0), lparent(n, 0);
    size_t li = 0, ii = 0;
    for (size_t k = 0; k + 1 < n; ++k) {
        uint32_t pick[2];
        uint64_t wsum = 0;
        for (int t = 0; t < 2; ++t) {
            const bool leaf = li < n && (ii >= k || leaves[li].first <= iw[ii]);
            if (leaf) {
                wsum += leaves[li].first;
                pick[t] = (uint32_t)li++;
                lparent[pick[t]] = (uint32_t)k;
            } else {
                wsum += iw[ii];
                pick[t] = (uint32_t)(n + ii);
                iparent[ii++] = (uint32_t)k;
            }
        }
        iw[k] = wsum;
    }
    // the last merged node is the root; parents are made after their children
    std::vector<uint32_t> idepth(n - 1, 0);
    for (size_t k = n - 1; k-- > 0;)
        if (k + 2 < n)
            idepth[k] = idepth[iparent[k]] + 1;
    uint32_t mx = 0;
    for (size_t i = 0; i < n; ++i) {
        depth[i] = idepth[lparent[i]] + 1;
        mx = std::max(mx, depth[i]);
    }
    return mx;
}

// Lengths above lmax: move leaves up in pairs until the Kraft sum fits (the
// classic bit-length adjustment), then hand the lengths out again by weight
// (heaviest symbol, shortest code).  A valid prefix code, not always optimal;
// only used when the optimal code has a codeword longer than lmax.
void limit_depths(const std::vector<std::pair<uint64_t, uint32_t>> &leaves,
                  std::vector<uint32_t> &depth, uint32_t maxd, uint32_t lmax)
{
    std::vector<uint64_t> cnt(maxd + 2, 0);
    for (uint32_t d : depth)
        cnt[d]++;
    for (uint32_t i = maxd; i > lmax; --i) {
        while (cnt[i] > 0) {
            uint32_t j = i - 2;
            while (cnt[j] == 0)
                --j;
            cnt[i] -= 2;
            cnt[i - 1] += 1;
            cnt[j + 1] += 2;
            cnt[j] -= 1;
        }
    }
    // leaves are in increasing weight: the lightest take the longest codes
    size_t i = 0;
    for (uint32_t d = lmax; d >= 1 && i < depth.size(); --d)
        for (uint64_t c = 0; c < cnt[d] && i < depth.size(); ++c)
            depth[i++] = d;
}

}  // namespace

bool huff_build(const uint64_t *hist, HuffTable &t)
{
    // used symbols in increasing (count, symbol): least-significant-digit radix
    // passes of 11 bits over the counts, stable, starting from symbol order
    std::vector<std::pair<uint64_t, uint32_t>> leaves, tmp;
    uint64_t cmax = 0;
    for (uint32_t s = 0; s < 65536u; ++s)
        if (hist[s]) {
            leaves.push_back({hist[s], s});
            cmax = std::max(cmax, hist[s]);
        }
    t.count.assign(kHuffMaxLen + 1, 0);
    t.syms.clear();
    t.n_bits = 0;
    t.max_len = 0;
    if (leaves.empty())
        return true;
    tmp.resize(leaves.size());
    for (int shift = 0; shift < 64 && (cmax >> shift) != 0; shift += 11) {
        uint32_t bucket[2049] = {0};
        for (const auto &l : leaves)
            bucket[((l.first >> shift) & 2047u) + 1]++;
        for (int k = 0; k < 2048; ++k)
            bucket[k + 1] += bucket[k];
        for (const auto &l : leaves)
            tmp[bucket[(l.first >> shift) & 2047u]++] = l;
        leaves.swap(tmp);
    }
    std::vector<uint32_t> depth;
    uint32_t mx = huffman_depths(leaves, depth);
    if (mx > kHuffMaxLen) {
        limit_depths(leaves, depth, mx, kHuffMaxLen);
        mx = kHuffMaxLen;
    }
    // canonical order (length, then symbol): per symbol its length, then the
    // symbols in value order bucketed by length
    std::vector<uint8_t> len(65536, 0);
    for (size_t i = 0; i < leaves.size(); ++i) {
        len[leaves[i].second] = (uint8_t)depth[i];
        t.count[depth[i]]++;
        t.n_bits += leaves[i].first * depth[i];
    }
    uint32_t pos[kHuffMaxLen + 2] = {0};
    for (int l = 1; l <= kHuffMaxLen; ++l)
        pos[l + 1] = pos[l] + t.count[l];
    t.syms.resize(leaves.size());
    for (uint32_t s = 0; s < 65536u; ++s)
        if (len[s])
            t.syms[pos[len[s]]++] = (uint16_t)s;
    t.max_len = mx;
    // Kraft check (the canonical construction needs sum 2^-l <= 1)
    uint64_t kraft = 0;
    for (uint32_t l = 1; l <= kHuffMaxLen; ++l)
        kraft += (uint64_t)t.count[l] << (kHuffMaxLen - l);
    return kraft <= (uint64_t(1) << kHuffMaxLen);
}

// The codebook of the training phase (Sec. 4.3: one table from the
// validation set's code frequencies, reused for every block).  The leaves
// are the codes with a non-zero count and, when some code was never seen,
// the escape (alphabet index 65536, weight = the number of codes seen once,
// at least 1), which stands for every unseen code and is followed in the
// stream by the code's 16 bits.  Lengths: the optimal prefix code with no
// codeword longer than 16 bits (32 without an escape), by package-merge
// (Larmore and Hirschberg 1990).  Row r holds the leaves merged with the
// pairs of row r - 1 (a leaf goes before a pair of equal weight); the last
// row's 2n - 2 lightest items are selected, and every selected prefix of a
// row asks for twice its pairs from the row before.  Only each row's leaf
// positions are kept (a bit per item): the selected prefix of a row holds
// the lightest m_r leaves, and a leaf's length is the number of rows whose
// m_r passes it.
bool huff_build_trained(const uint64_t *hist, HuffTable &t, uint32_t &esc_len)
{
    struct Leaf {
        uint64_t w;
        uint32_t s;
    };
    std::vector<Leaf> leaves;
    uint64_t ones = 0;
    bool unseen = false;
    for (uint32_t s = 0; s < 65536u; ++s) {
        if (hist[s])
            leaves.push_back({hist[s], s});
        ones += hist[s] == 1;
        unseen |= hist[s] == 0;
    }
    if (unseen)
        leaves.push_back({std::max<uint64_t>(ones, 1), kHuffEsc});
    std::stable_sort(leaves.begin(), leaves.end(),
                     [](const Leaf &a, const Leaf &b) { return a.w < b.w; });
    const size_t n = leaves.size();
    const uint32_t lmax = unseen ? 16u : (uint32_t)kHuffMaxLen;
    std::vector<uint32_t> len(n, 0);
    if (n == 1) {
        len[0] = 1;
    } else {
        if (n > ((size_t)1 << lmax))
            return false;
        // forward: each row's item weights (to pair them into the next row)
        // and leaf flags (to count the selected leaves on the way back)
        std::vector<std::vector<uint64_t>> isleaf(lmax);
        std::vector<uint64_t> prev, cur;
        std::vector<size_t> rows(lmax);
        for (uint32_t r = 0; r < lmax; ++r) {
            const size_t np = r == 0 ? 0 : prev.size() / 2;
            cur.clear();
            cur.reserve(n + np);
            isleaf[r].assign((n + np + 63) / 64, 0ull);
            size_t i = 0, j = 0;
            while (i < n || j < np) {
                const uint64_t pw = j < np ? prev[2 * j] + prev[2 * j + 1] : 0;
                if (j >= np || (i < n && leaves[i].w <= pw)) {
                    isleaf[r][cur.size() >> 6] |= 1ull << (cur.size() & 63);
                    cur.push_back(leaves[i++].w);
                } else {
                    cur.push_back(pw);
                    ++j;
                }
            }
            rows[r] = cur.size();
            prev.swap(cur);
        }
        size_t take = 2 * n - 2;
        if (rows[lmax - 1] < take)
            return false;
        // backward: selected leaves of each row, then the pairs it takes
        std::vector<int64_t> diff(n + 1, 0);
        for (uint32_t r = lmax; r-- > 0;) {
            size_t m = 0;
            for (size_t k = 0; k < take / 64; ++k)
                m += (size_t)__builtin_popcountll(isleaf[r][k]);
            if (take & 63)
                m += (size_t)__builtin_popcountll(isleaf[r][take / 64] &
                                                  ((1ull << (take & 63)) - 1));
            diff[0] += 1;
            diff[m] -= 1;
            take = 2 * (take - m);
        }
        if (take != 0)
            return false;
        int64_t acc = 0;
        for (size_t i = 0; i < n; ++i) {
            acc += diff[i];
            len[i] = (uint32_t)acc;
        }
    }
    // canonical order: by length, then symbol (the escape last of its length)
    t.count.assign(kHuffMaxLen + 1, 0);
    t.n_bits = 0;
    t.max_len = 0;
    esc_len = 0;
    std::vector<std::pair<uint32_t, uint32_t>> ord(n);
    for (size_t i = 0; i < n; ++i) {
        if (len[i] < 1 || len[i] > lmax)
            return false;
        t.count[len[i]]++;
        t.max_len = std::max(t.max_len, len[i]);
        if (leaves[i].s == kHuffEsc)
            esc_len = len[i];
        ord[i] = {len[i], leaves[i].s};
    }
    std::sort(ord.begin(), ord.end());
    t.syms.resize(n);
    for (size_t i = 0; i < n; ++i)
        t.syms[i] = ord[i].second == kHuffEsc ? (uint16_t)0 : (uint16_t)ord[i].second;
    uint64_t kraft = 0;
    for (uint32_t l = 1; l <= (uint32_t)kHuffMaxLen; ++l)
        kraft += (uint64_t)t.count[l] << (kHuffMaxLen - l);
    return kraft <= (uint64_t(1) << kHuffMaxLen);
}

// ---------------------------------------------------------------------------
// device
// ---------------------------------------------------------------------------

// canonical first codeword and first canonical index of every length
struct Canon {
    unsigned first[kHuffMaxLen + 2];
    unsigned index[kHuffMaxLen + 2];
    unsigned count[kHuffMaxLen + 2];
};

__device__ __forceinline__ void canon_from(const uint32_t *cnt, Canon &c)
{
    unsigned code = 0, idx = 0;
    c.first[0] = 0;
    c.index[0] = 0;
    c.count[0] = 0;
    for (int l = 1; l <= kHuffMaxLen; ++l) {
        code = (code + c.count[l - 1]) << 1;
        c.count[l] = cnt[l];
        c.first[l] = code;
        c.index[l] = idx;
        idx += cnt[l];
    }
    c.count[kHuffMaxLen + 1] = 0;
}

__global__ void k_fill_u32(uint32_t *p, unsigned long long n, uint32_t v)
{
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        p[i] = v;
}

// canonical index and codeword of the escape (the last symbol of length
// esc_len); ~0u when there is none
__device__ __forceinline__ void esc_of(const uint32_t *cnt, unsigned esc_len, unsigned &ix,
                                       unsigned &code)
{
    ix = ~0u;
    code = 0;
    if (esc_len == 0 || esc_len > (unsigned)kHuffMaxLen || cnt[esc_len] == 0)
        return;
    unsigned c = 0, idx = 0, prev = 0;
    for (unsigned l = 1; l <= esc_len; ++l) {
        c = (c + prev) << 1;
        prev = cnt[l];
        idx += l < esc_len ? cnt[l] : 0u;
    }
    ix = idx + cnt[esc_len] - 1;
    code = c + cnt[esc_len] - 1;
}

// encoder table before k_huff_enc: every code unused (esc_len = 0), or
// every code the escape codeword followed by its own 16 bits
__global__ void k_huff_enc_init(const uint32_t *__restrict__ tab, unsigned esc_len,
                                uint8_t *__restrict__ enc_len,
                                unsigned long long *__restrict__ enc_code)
{
    unsigned ix, ecode;
    esc_of(tab, esc_len, ix, ecode);
    for (unsigned s = blockIdx.x * blockDim.x + threadIdx.x; s < 65536u;
         s += gridDim.x * blockDim.x) {
        const unsigned l = ix == ~0u ? 0u : esc_len + 16;
        enc_len[s] = (uint8_t)l;
        enc_code[s] = ix == ~0u ? 0ull
                                : ((unsigned long long)l << 32) | ((ecode << 16) | s);
    }
}

// encoder table: length and codeword of every symbol the table lists (the
// escape's slot excepted)
__global__ void k_huff_enc(const uint32_t *__restrict__ tab, unsigned esc_len,
                           uint8_t *__restrict__ enc_len, unsigned long long *__restrict__ enc_code)
{
    const uint32_t *cnt = tab;
    const uint16_t *syms = reinterpret_cast<const uint16_t *>(tab + kHuffMaxLen + 1);
    unsigned nsym = 0;
    for (int l = 1; l <= kHuffMaxLen; ++l)
        nsym += cnt[l];
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned eix, ecode;
    esc_of(cnt, esc_len, eix, ecode);
    if (i >= nsym || i == eix)
        return;
    unsigned code = 0, idx = 0, prev = 0;
    for (int l = 1; l <= kHuffMaxLen; ++l) {
        code = (code + prev) << 1;
        prev = cnt[l];
        if (i < idx + cnt[l]) {
            const unsigned s = syms[i];
            enc_len[s] = (uint8_t)l;
            enc_code[s] = ((unsigned long long)l << 32) | (code + (i - idx));
            return;
        }
        idx += cnt[l];
    }
}

// per-block bit sizes: one wave per block, eight codes per lane (one 16-byte
// load) where the block's codes are 16-byte aligned
template <typename S>
__global__ void __launch_bounds__(256) k_huff_sizes(const uint16_t *__restrict__ codes, GeoArgs g,
                                                    const uint8_t *__restrict__ enc_len,
                                                    S *__restrict__ sizes, int *status)
{
    const int lane = threadIdx.x & 63;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    int err = kOk;
    for (long long b = wave; b < g.nblocks; b += nwaves) {
        const long long bx = b % g.nb[2], by = (b / g.nb[2]) % g.nb[1],
                        bz = b / (g.nb[1] * g.nb[2]);
        const BlockGeo q = block_geo3(bz, by, bx, g.n, g.bd[0], g.bd[1], g.bd[2]);
        const long long bsize = (long long)q.ez * q.ey * q.ex;
        const uint16_t *src = codes + q.start;
        unsigned s = 0, zl = 0;
        long long i0 = 0;
        if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            for (; i0 + 512 <= bsize; i0 += 512) {
                const uint4 v = reinterpret_cast<const uint4 *>(src + i0)[lane];
                const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const unsigned l0 = enc_len[w[k] & 0xFFFFu], l1 = enc_len[w[k] >> 16];
                    zl |= (l0 == 0 ? 1u : 0u) | (l1 == 0 ? 1u : 0u);
                    s += l0 + l1;
                }
            }
        }
        for (long long i = i0 + lane; i < bsize; i += 64) {
            const unsigned l = enc_len[src[i]];
            zl |= l == 0 ? 1u : 0u;
            s += l;
        }
        if (zl)
            err = kECorrupt;  // a code the codebook does not hold
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1)
            s += __shfl_xor(s, d, 64);
        if (lane == 0)
            sizes[b] = (S)s;
    }
    set_status(status, err);
}

// append n codes (lengths l[], codewords c[]) at bit `pos` of the LDS words w:
// whole words by plain stores, the first and last (shared with the lanes on
// either side) by atomic OR
__device__ __forceinline__ void pack_emit(uint32_t *w, unsigned pos, const unsigned *l,
                                          const unsigned *c, int n)
{
    unsigned long long acc = 0;
    int nacc = (int)(pos & 31u);
    unsigned wp = pos >> 5;
    bool first = true;
    for (int j = 0; j < n; ++j) {
        acc |= (unsigned long long)c[j] << (64 - nacc - (int)l[j]);
        nacc += (int)l[j];
        if (nacc >= 32) {
            const uint32_t word = (uint32_t)(acc >> 32);
            if (first)
                atomicOr(&w[wp], word);
            else
                w[wp] = word;
            first = false;
            ++wp;
            acc <<= 32;
            nacc -= 32;
        }
    }
    if (nacc > 0)
        atomicOr(&w[wp], (uint32_t)(acc >> 32));
}

// Bit packing: one wave per block, the block's words assembled in LDS.  Each
// lane packs a run of consecutive codes (eight, from one 16-byte load, where
// aligned; else one) into its own bit span: whole words by plain LDS stores,
// the first and last word of its span (shared with the neighbouring lanes) by
// atomic OR.  The wave then stores the block's words, the two boundary words
// (shared with the neighbouring blocks) by atomic OR into the zeroed section.
template <typename S>
__global__ void __launch_bounds__(256) k_huff_pack(const uint16_t *__restrict__ codes, GeoArgs g,
                                                   const unsigned long long *__restrict__ enc,
                                                   const S *__restrict__ sizes,
                                                   const unsigned long long *__restrict__ boffs,
                                                   const unsigned long long *__restrict__ bparts,
                                                   uint32_t *__restrict__ bits, int wave_words,
                                                   const int *status)
{
    extern __shared__ uint32_t lw[];
    const int st0 = *status;
    const int lane = threadIdx.x & 63;
    uint32_t *w = lw + (threadIdx.x >> 6) * wave_words;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    auto emit = [&](unsigned pos, const unsigned *l, const unsigned *c, int n) {
        pack_emit(w, pos, l, c, n);
    };
    // A wave packs several blocks in turn; each block's geometry, bit offset,
    // bit size and first 16-byte load of codes are fetched while the block
    // before it is packed, so their round trips overlap that work.
    struct Ahead {
        BlockGeo q;
        unsigned long long start;
        unsigned nbits;
        uint4 v;
    };
    auto fetch = [&](long long b, Ahead &p) {
        const long long bx = b % g.nb[2], by = (b / g.nb[2]) % g.nb[1],
                        bz = b / (g.nb[1] * g.nb[2]);
        p.q = block_geo3(bz, by, bx, g.n, g.bd[0], g.bd[1], g.bd[2]);
        p.start = boffs[b] + bparts[b / kScanChunk];
        p.nbits = (unsigned)sizes[b];
        const uint16_t *src = codes + p.q.start;
        const long long bsize = (long long)p.q.ez * p.q.ey * p.q.ex;
        p.v = ((reinterpret_cast<uintptr_t>(src) & 15) == 0 && bsize >= 512)
                  ? reinterpret_cast<const uint4 *>(src)[lane]
                  : make_uint4(0u, 0u, 0u, 0u);
    };
    Ahead cur{}, nxt{};
    if (wave < g.nblocks)
        fetch(wave, cur);
    if (st0 != kOk)
        return;
    for (long long b = wave; b < g.nblocks; b += nwaves) {
        if (b + nwaves < g.nblocks)
            fetch(b + nwaves, nxt);
        const BlockGeo q = cur.q;
        const long long bsize = (long long)q.ez * q.ey * q.ex;
        const unsigned long long start = cur.start;
        const unsigned s0 = (unsigned)(start & 31u);
        const unsigned nbits = cur.nbits;
        const int nw = (int)((s0 + nbits + 31u) >> 5);
        for (int k = lane; k < nw; k += 64)
            w[k] = 0u;
        __builtin_amdgcn_wave_barrier();
        unsigned run = s0;
        const uint16_t *src = codes + q.start;
        long long i0 = 0;
        if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            for (; i0 + 512 <= bsize; i0 += 512) {
                const uint4 v = i0 == 0 ? cur.v : reinterpret_cast<const uint4 *>(src + i0)[lane];
                const unsigned cw[4] = {v.x, v.y, v.z, v.w};
                unsigned l[8], c[8], t = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const unsigned sym = (cw[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                    const unsigned long long ec = enc[sym];  // one gather per code
                    l[j] = (unsigned)(ec >> 32);
                    c[j] = (unsigned)ec;
                    t += l[j];
                }
                unsigned incl = t;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const unsigned o = __shfl_up(incl, d, 64);
                    if (lane >= d)
                        incl += o;
                }
                emit(run + incl - t, l, c, 8);
                run += __shfl(incl, 63, 64);
            }
        }
        for (long long c0 = i0; c0 < bsize; c0 += 64) {
            const long long i = c0 + lane;
            unsigned l = 0, cw = 0;
            if (i < bsize) {
                const unsigned long long ec = enc[src[i]];
                l = (unsigned)(ec >> 32);
                cw = (unsigned)ec;
            }
            unsigned incl = l;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const unsigned o = __shfl_up(incl, d, 64);
                if (lane >= d)
                    incl += o;
            }
            if (l)
                emit(run + incl - l, &l, &cw, 1);
            run += __shfl(incl, 63, 64);
        }
        // this wave's LDS writes above are complete before its reads below
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        __builtin_amdgcn_wave_barrier();
        const unsigned long long w0 = start >> 5;
        const bool part_lo = s0 != 0, part_hi = ((s0 + nbits) & 31u) != 0;
        for (int k = lane; k < nw; k += 64) {
            const bool shared = (k == 0 && part_lo) || (k == nw - 1 && part_hi);
            if (shared)
                atomicOr(&bits[w0 + k], w[k]);
            else
                bits[w0 + k] = w[k];
        }
        __builtin_amdgcn_wave_barrier();
        cur = nxt;
    }
}

// Bit packing of a 3-D field of whole 8^3 blocks (every side a multiple of
// 8; block b's 512 codes at b * 512): k_huff_pack's packing, pipelined so
// that a wave's stores never drain before its next block.  One counter tracks
// a wave's loads and stores in issue order, so a wait for a load also waits
// for every store issued before that load.  Here the loads a block waits for
// (its table gathers, issued one block ahead, from codes read two blocks
// ahead) come before the previous block's stores; every block issues the same
// vector memory instructions (its words through a buffer range that drops
// the lanes past them; offsets and sizes as scalar loads), so each wait counts
// only what came after its load.
constexpr int kWholeStoreRounds = 9;  // 64-lane rounds of a block's at most 514 words

template <typename S>
__global__ void __launch_bounds__(256) k_huff_pack_whole(const uint16_t *__restrict__ codes,
                                                         long long nblocks,
                                                         const unsigned long long *__restrict__ enc,
                                                         const S *__restrict__ sizes,
                                                         const unsigned long long *__restrict__ boffs,
                                                         const unsigned long long *__restrict__ bparts,
                                                         uint32_t *__restrict__ bits, int wave_words,
                                                         const int *status)
{
    extern __shared__ uint32_t lw[];
    if (*status != kOk)
        return;
    const int lane = threadIdx.x & 63;
    uint32_t *w = lw + (threadIdx.x >> 6) * wave_words;
    const long long wave =
        __builtin_amdgcn_readfirstlane((int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    if (wave >= nblocks)
        return;
    const long long last = nblocks - 1;
    auto codes_of = [&](long long b) {
        return reinterpret_cast<const uint4 *>(codes + b * 512)[lane];
    };
    auto gather = [&](const uint4 &v, unsigned (&l)[8], unsigned (&c)[8]) {
        const unsigned cw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const unsigned long long ec = enc[(cw[j >> 1] >> (16 * (j & 1))) & 0xFFFFu];
            l[j] = (unsigned)(ec >> 32);
            c[j] = (unsigned)ec;
        }
    };
    unsigned l[8], c[8];
    uint4 vn = codes_of(wave);
    gather(vn, l, c);
    vn = codes_of(std::min(wave + nwaves, last));
    for (long long b = wave; b < nblocks; b += nwaves) {
        // the next block's gathers (its codes arrived during this block's
        // predecessor), then the codes of the block after it
        unsigned ln[8], cn[8];
        gather(vn, ln, cn);
        vn = codes_of(std::min(b + 2 * nwaves, last));
        const unsigned long long start = boffs[b] + bparts[b / kScanChunk];
        // the block's size through a scalar load (a 16-bit size from the
        // aligned word that holds it)
        unsigned nbits;
        if constexpr (sizeof(S) == 2) {
            const unsigned sw = reinterpret_cast<const unsigned *>(sizes)[b >> 1];
            nbits = (b & 1) ? sw >> 16 : sw & 0xFFFFu;
        } else {
            nbits = (unsigned)sizes[b];
        }
        const unsigned s0 = (unsigned)(start & 31u);
        const int nw = (int)((s0 + nbits + 31u) >> 5);
        for (int k = lane; k < nw; k += 64)
            w[k] = 0u;
        __builtin_amdgcn_wave_barrier();
        unsigned t = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            t += l[j];
        unsigned incl = t;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned o = __shfl_up(incl, d, 64);
            if (lane >= d)
                incl += o;
        }
        pack_emit(w, s0 + incl - t, l, c, 8);
        // this wave's LDS writes above are complete before its reads below
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        __builtin_amdgcn_wave_barrier();
        const unsigned long long w0 = start >> 5;
        const bool part_lo = s0 != 0, part_hi = ((s0 + nbits) & 31u) != 0;
        // words shared with a neighbouring block, by atomic OR below; the
        // others by plain stores (lanes past the block's words fall outside
        // the range and store nothing)
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc(bits + w0, 0, nw * 4, 0x00020000);
#pragma unroll
        for (int q = 0; q < kWholeStoreRounds; ++q) {
            const int k = lane + 64 * q;
            const bool shared = (k == 0 && part_lo) || (k == nw - 1 && part_hi);
            const uint32_t v = w[k < wave_words ? k : 0];
            __builtin_amdgcn_raw_buffer_store_b32(v, r, (k < nw && !shared) ? 4 * k : 4 * nw, 0, 0);
        }
        if (lane == 0 && part_lo)
            atomicOr(&bits[w0], w[0]);
        if (lane == 1 && part_hi)
            atomicOr(&bits[w0 + nw - 1], w[nw - 1]);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            l[j] = ln[j];
            c[j] = cn[j];
        }
    }
}

// decoder: one thread per block
constexpr int kLutBits = 14;

// Per-block decoder, one thread per block.  Codes of up to kLutBits bits come
// from a lookup table of the next kLutBits bits (the escape flagged in it); for
// a longer code the table gives the shortest and longest length under its
// prefix, and the length is the shortest plus the canonical length limits (in
// LDS) between the two that its window reaches; its symbol sits at index
// offset[len] + the code.  The table and the
// symbols (all of them when ALL_LDS, else the first kSymsLds) live in the
// workgroup's LDS, so a step waits on no global load.  Each thread's bits
// come half a 128-byte line at a time: the half being read sits in the
// thread's own LDS slot, the next half is in flight in registers; one refill
// of 32 bits per symbol (a word read from the slot at the thread's own index)
// keeps at least 33 bits in the buffer (no codeword, escape and its 16 bits
// included, is longer than 32).  LDS: the table (64 KiB), the slots (64 bytes
// a thread) and the symbols (at most kSymsLds) fit in 160 KiB.
constexpr int kUnpackThreads = 1024;
constexpr int kSymsLds = 15360;
// lookup-table entries: symbol | length << 16 for a code of at most kLutBits
// bits (kLutEsc: the escape); kLutLong | shortest << 16 | longest << 8 for a
// prefix of longer codes; 0 for bits no codeword starts with
constexpr uint32_t kLutEsc = 0x80000000u;
constexpr uint32_t kLutLong = 0x40000000u;

// The decoder's lookup table, built once per call (kLutBits-bit windows, one
// entry per thread): a codeword of at most kLutBits bits gives its symbol and
// length (kLutEsc: the escape); a prefix of longer codes gives the shortest
// and longest length under it (kLutLong); 0 where no codeword starts.  Length
// counts that describe no prefix code of nsym symbols leave the table
// unwritten (the decoder checks them too, and stops).
__global__ void __launch_bounds__(256) k_huff_lut(const uint32_t *__restrict__ tab, unsigned nsym,
                                                  unsigned esc_len, uint32_t *__restrict__ lut)
{
    __shared__ Canon cs;
    __shared__ unsigned slim[kHuffMaxLen + 2];
    __shared__ unsigned smax, sesc;
    __shared__ int sok;
    const uint32_t *cnt = tab;
    const uint16_t *syms = reinterpret_cast<const uint16_t *>(tab + kHuffMaxLen + 1);
    if (threadIdx.x == 0) {
        unsigned long long ns = 0, kraft = 0;
        for (int l = 1; l <= kHuffMaxLen; ++l) {
            ns += cnt[l];
            kraft += (unsigned long long)cnt[l] << (kHuffMaxLen - l);
        }
        sok = cnt[0] == 0 && ns == nsym && kraft <= (1ull << kHuffMaxLen) &&
              (esc_len == 0 || (esc_len <= 16u && cnt[esc_len] != 0));
        canon_from(cnt, cs);
        unsigned mx = 0;
        for (int l = 1; l <= kHuffMaxLen; ++l) {
            const unsigned long long end = ((unsigned long long)cs.first[l] + cs.count[l])
                                           << (32 - l);
            slim[l] = end > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned)end;
            if (cs.count[l])
                mx = (unsigned)l;
        }
        smax = mx;
        unsigned ecode;
        esc_of(cnt, esc_len, sesc, ecode);
    }
    __syncthreads();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (!sok || e >= (1 << kLutBits))
        return;
    uint32_t v = 0;
    for (int l = 1; l <= kLutBits; ++l) {
        const unsigned pre = (unsigned)e >> (kLutBits - l);
        if (pre - cs.first[l] < cs.count[l]) {
            const unsigned ix = cs.index[l] + (pre - cs.first[l]);
            v = ix == sesc ? kLutEsc | ((uint32_t)l << 16) : syms[ix] | ((uint32_t)l << 16);
            break;
        }
    }
    if (v == 0 && smax > (unsigned)kLutBits) {
        // longer codes under this prefix: the lengths of its first and last
        // windows bound theirs
        const unsigned lo = (unsigned)e << (32 - kLutBits);
        const unsigned hi = lo | ((1u << (32 - kLutBits)) - 1u);
        unsigned a = kLutBits + 1, b = kLutBits + 1;
        for (unsigned qq = kLutBits + 1; qq < smax; ++qq) {
            a += lo >= slim[qq] ? 1u : 0u;
            b += hi >= slim[qq] ? 1u : 0u;
        }
        v = kLutLong | (a << 16) | (b << 8);
    }
    lut[e] = v;
}

template <typename S, bool ALL_LDS>
__global__ void __launch_bounds__(kUnpackThreads) k_huff_unpack(const uint32_t *__restrict__ tab,
                                                     const uint32_t *__restrict__ bits,
                                                     unsigned long long nwords, GeoArgs g,
                                                     const S *__restrict__ sizes,
                                                     const unsigned long long *__restrict__ boffs,
                                                     const unsigned long long *__restrict__ bparts,
                                                     uint16_t *__restrict__ codes, int *status,
                                                     unsigned nsym, unsigned esc_len,
                                                     const uint32_t *__restrict__ glut)
{
    extern __shared__ __align__(16) unsigned char hsm[];
    uint32_t *lut = reinterpret_cast<uint32_t *>(hsm);  // symbol | length << 16 (0: longer)
    // the threads' half lines: group k (16 bytes) of thread t at lines[k * blockDim.x + t]
    uint4 *lines = reinterpret_cast<uint4 *>(lut + (1 << kLutBits));
    uint16_t *ssyms = reinterpret_cast<uint16_t *>(lines + 4 * blockDim.x);
    __shared__ Canon cs;
    __shared__ int soff[kHuffMaxLen + 2];        // index[l] - first[l]
    __shared__ unsigned slim[kHuffMaxLen + 2];   // left-aligned end of the length-l codes
    __shared__ unsigned smax;                    // longest code length
    __shared__ unsigned sesc;                    // canonical index of the escape (~0u: none)
    __shared__ int sok;                          // the stream's length counts are valid
    const uint32_t *cnt = tab;
    const uint16_t *syms = reinterpret_cast<const uint16_t *>(tab + kHuffMaxLen + 1);
    const unsigned nlds = nsym < (unsigned)kSymsLds ? nsym : (unsigned)kSymsLds;
    if (threadIdx.x == 0) {
        // the length counts must describe a prefix code of the nsym stored
        // symbols (Kraft sum at most 1) whose escape, if any, has a slot;
        // checked here so no thread indexes the table before they are
        unsigned long long ns = 0, kraft = 0;
        for (int l = 1; l <= kHuffMaxLen; ++l) {
            ns += cnt[l];
            kraft += (unsigned long long)cnt[l] << (kHuffMaxLen - l);
        }
        sok = cnt[0] == 0 && ns == nsym && kraft <= (1ull << kHuffMaxLen) &&
              (esc_len == 0 || (esc_len <= 16u && cnt[esc_len] != 0));
        canon_from(cnt, cs);
        unsigned mx = 0;
        for (int l = 1; l <= kHuffMaxLen; ++l) {
            soff[l] = (int)cs.index[l] - (int)cs.first[l];
            // below the longest length the end stays under 2^32
            const unsigned long long end = ((unsigned long long)cs.first[l] + cs.count[l])
                                           << (32 - l);
            slim[l] = end > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned)end;
            if (cs.count[l])
                mx = (unsigned)l;
        }
        smax = mx;
        unsigned ecode;
        esc_of(cnt, esc_len, sesc, ecode);
    }
    for (unsigned k = threadIdx.x; k < nlds; k += blockDim.x)
        ssyms[k] = syms[k];
    __syncthreads();
    if (!sok) {
        if (threadIdx.x == 0)
            set_status(status, kECorrupt);
        return;
    }
    // the lookup table, built once per call by k_huff_lut
    for (int e = threadIdx.x; e < (1 << kLutBits) / 4; e += blockDim.x)
        reinterpret_cast<uint4 *>(lut)[e] = reinterpret_cast<const uint4 *>(glut)[e];
    const unsigned maxlen = __builtin_amdgcn_readfirstlane(smax);
    const unsigned esc_ix = __builtin_amdgcn_readfirstlane(sesc);
    __syncthreads();
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.nblocks)
        return;
    const long long bx = b % g.nb[2], by = (b / g.nb[2]) % g.nb[1], bz = b / (g.nb[1] * g.nb[2]);
    const BlockGeo q = block_geo3(bz, by, bx, g.n, g.bd[0], g.bd[1], g.bd[2]);
    const long long bsize = (long long)q.ez * q.ey * q.ex;
    const unsigned long long start = boffs[b] + bparts[b / kScanChunk];
    const unsigned nbits_block = (unsigned)sizes[b];
    int err = kOk;
    if (start + nbits_block > nwords * 32ull) {
        set_status(status, kECorrupt);
        return;
    }
    // The bit queue.  All 262,144 block streams of a 512^3 field are read at
    // once, and a stream read 16 bytes at a time would see its line leave L2
    // between two of its reads; a thread therefore fetches 64 bytes at a
    // time.  The half line in use sits in the thread's LDS slot (a word is
    // taken at the thread's own index: no register shuffling, which a wave
    // would pay whenever any of its threads needed it), the next half is in
    // flight in registers.
    // A half line holding any word of the section is read whole: the section
    // starts 256-byte aligned and the next section starts at the next 256-byte
    // boundary after it (the gap zeroed), so the half stays inside the stream;
    // halves past the section read as zeros.
    const uint4 *w4 = reinterpret_cast<const uint4 *>(bits);
    auto load_half = [&](uint4 (&d)[4], unsigned long long h) {
        if (16 * h < nwords) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                d[k] = w4[4 * h + k];
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                d[k] = make_uint4(0u, 0u, 0u, 0u);
        }
    };
    uint4 *slot = lines + threadIdx.x;
    const unsigned stride = blockDim.x;
    auto put_half = [&](const uint4 (&d)[4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            slot[k * stride] = d[k];
    };
    unsigned long long half = (start >> 5) >> 4;  // 16 words a half
    uint4 N[4];
    load_half(N, half);
    put_half(N);
    load_half(N, half + 1);
    unsigned widx = (unsigned)((start >> 5) & 15u);  // next word of the half in the slot
    unsigned long long buf = 0;
    int nb = 0;
    auto take = [&]() {
        if (widx == 16) {
            put_half(N);
            ++half;
            widx = 0;
            load_half(N, half + 1);
        }
        const unsigned w =
            reinterpret_cast<const unsigned *>(slot + (widx >> 2) * stride)[widx & 3u];
        ++widx;
        buf |= (unsigned long long)w << (32 - nb);
        nb += 32;
    };
    take();
    take();
    const unsigned sk = (unsigned)(start & 31u);
    buf <<= sk;
    nb -= (int)sk;
    unsigned used = 0;
    auto next_sym = [&]() -> unsigned {
        if (nb <= 32)
            take();
        const unsigned win = (unsigned)(buf >> 32);
        const uint32_t e = lut[win >> (32 - kLutBits)];
        unsigned l = (e >> 16) & 0xFFu, sym = e & 0xFFFFu;
        bool esc = (e & kLutEsc) != 0;
        if (e & kLutLong) {
            // a longer code: its length lies between the bounds of its prefix;
            // add the length limits between them that the window reaches
            unsigned len = l;
            const unsigned lmax = (e >> 8) & 0xFFu;
            for (unsigned qq = l; qq < lmax; ++qq)
                len += win >= slim[qq] ? 1u : 0u;
            // index[len] + (code - first[len]), in wrapping 32-bit arithmetic
            // (exact: the true index is below 2^16)
            const unsigned ix = (unsigned)soff[len] + (win >> (32 - len));
            if (len > maxlen || ix >= nsym) {
                err = kECorrupt;
                l = 1;
                sym = 0;
                esc = false;
            } else {
                l = len;
                esc = ix == esc_ix;
                if constexpr (ALL_LDS)
                    sym = ssyms[ix];
                else
                    sym = ix < nlds ? ssyms[ix] : syms[ix];
            }
        }
        if (l == 0) {  // the bits match no codeword
            err = kECorrupt;
            l = 1;
        }
        buf <<= l;
        nb -= (int)l;
        used += l;
        if (esc) {
            // the escaped code's own 16 bits follow (the escape has at most
            // 16 bits, so the buffer still holds them)
            sym = (unsigned)(buf >> 48);
            buf <<= 16;
            nb -= 16;
            used += 16;
        }
        return sym;
    };
    uint16_t *dst = codes + q.start;
    long long i = 0;
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        // eight codes per 16-byte store, two per step into a shifting word queue
        for (; i + 8 <= bsize && err == kOk; i += 8) {
            uint4 acc = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
                const unsigned lo = next_sym();
                const unsigned hi = next_sym();
                acc.x = acc.y;
                acc.y = acc.z;
                acc.z = acc.w;
                acc.w = lo | (hi << 16);
            }
            *reinterpret_cast<uint4 *>(dst + i) = acc;
        }
    }
    for (; i < bsize && err == kOk; ++i)
        dst[i] = (uint16_t)next_sym();
    if (used != nbits_block)
        err = kECorrupt;
    set_status(status, err);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

GeoArgs geo_of(const Geom &g)
{
    GeoArgs a{};
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bd[d] = g.bd[d];
        a.nb[d] = g.nb[d];
    }
    a.nblocks = g.nblocks;
    return a;
}

unsigned wave_grid(long long nblocks)
{
    const long long g = (nblocks + 3) / 4;
    return (unsigned)std::max<long long>(1, std::min<long long>(g, 16384));
}

}  // namespace

int huff_size_bytes(const Geom &g)
{
    const long long bv = (long long)g.bd[0] * g.bd[1] * g.bd[2];
    return bv * kHuffMaxLen <= 65535 ? 2 : 4;
}

hipError_t launch_huff_sizes(const Geom &g, const uint16_t *codes, const uint32_t *d_tab,
                             unsigned esc_len, void *d_sizes, Workspace &ws, hipStream_t s)
{
    const GeoArgs ga = geo_of(g);
    hipLaunchKernelGGL(k_huff_enc_init, dim3(64), dim3(256), 0, s, d_tab, esc_len, ws.enc_len,
                       ws.enc_code);
    hipLaunchKernelGGL(k_huff_enc, dim3(256), dim3(256), 0, s, d_tab, esc_len, ws.enc_len,
                       ws.enc_code);
    const unsigned grid = wave_grid(g.nblocks);
    hipError_t e;
    if (huff_size_bytes(g) == 2) {
        uint16_t *sz = static_cast<uint16_t *>(d_sizes);
        hipLaunchKernelGGL(k_huff_sizes<uint16_t>, dim3(grid), dim3(256), 0, s, codes, ga,
                           ws.enc_len, sz, ws.status);
        e = launch_scan_sizes(sz, 2, g.nblocks, ws.boffsets, ws.bpartials, ws.bits_total, s);
    } else {
        uint32_t *sz = static_cast<uint32_t *>(d_sizes);
        hipLaunchKernelGGL(k_huff_sizes<uint32_t>, dim3(grid), dim3(256), 0, s, codes, ga,
                           ws.enc_len, sz, ws.status);
        e = launch_scan_sizes(sz, 4, g.nblocks, ws.boffsets, ws.bpartials, ws.bits_total, s);
    }
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_huff_pack(const Geom &g, const uint16_t *codes, const void *d_sizes,
                            uint32_t *d_bits, unsigned long long nwords, Workspace &ws,
                            hipStream_t s)
{
    const GeoArgs ga = geo_of(g);
    const long long bv = (long long)g.bd[0] * g.bd[1] * g.bd[2];
    const int wave_words = (int)((bv * kHuffMaxLen + 31) / 32 + 2);
    // waves per workgroup of the packer: each holds its block's words in LDS
    const int wpg = (int)std::max<long long>(1, std::min<long long>(4, 65536 / (4 * wave_words)));
    const size_t lds = wpg * sizeof(uint32_t) * (size_t)wave_words;
    const unsigned pgrid =
        (unsigned)std::max<long long>(1, std::min<long long>((g.nblocks + wpg - 1) / wpg, 16384));
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<unsigned long long>(
                                       std::max<unsigned long long>(1, (nwords + 255) / 256), 8192)),
                       dim3(256), 0, s, d_bits, nwords, 0u);
    // whole 8^3 blocks (every side a multiple of 8), codes 16-byte aligned: the
    // pipelined packer
    const bool whole = g.D == 3 && g.bd[0] == 8 && g.bd[1] == 8 && g.bd[2] == 8 &&
                       g.n[0] % 8 == 0 && g.n[1] % 8 == 0 && g.n[2] % 8 == 0 &&
                       (reinterpret_cast<uintptr_t>(codes) & 15) == 0 &&
                       wave_words <= 64 * kWholeStoreRounds;
    if (whole) {
        if (huff_size_bytes(g) == 2)
            hipLaunchKernelGGL(k_huff_pack_whole<uint16_t>, dim3(pgrid), dim3(64 * wpg), lds, s,
                               codes, g.nblocks, ws.enc_code,
                               static_cast<const uint16_t *>(d_sizes), ws.boffsets, ws.bpartials,
                               d_bits, wave_words, ws.status);
        else
            hipLaunchKernelGGL(k_huff_pack_whole<uint32_t>, dim3(pgrid), dim3(64 * wpg), lds, s,
                               codes, g.nblocks, ws.enc_code,
                               static_cast<const uint32_t *>(d_sizes), ws.boffsets, ws.bpartials,
                               d_bits, wave_words, ws.status);
        return hipGetLastError();
    }
    if (huff_size_bytes(g) == 2)
        hipLaunchKernelGGL(k_huff_pack<uint16_t>, dim3(pgrid), dim3(64 * wpg), lds, s, codes, ga,
                           ws.enc_code, static_cast<const uint16_t *>(d_sizes),
                           ws.boffsets, ws.bpartials, d_bits, wave_words, ws.status);
    else
        hipLaunchKernelGGL(k_huff_pack<uint32_t>, dim3(pgrid), dim3(64 * wpg), lds, s, codes, ga,
                           ws.enc_code, static_cast<const uint32_t *>(d_sizes),
                           ws.boffsets, ws.bpartials, d_bits, wave_words, ws.status);
    return hipGetLastError();
}

hipError_t launch_huff_encode(const Geom &g, const uint16_t *codes, const uint32_t *d_tab,
                              void *d_sizes, uint32_t *d_bits, unsigned long long nwords,
                              Workspace &ws, hipStream_t s)
{
    hipError_t e = launch_huff_sizes(g, codes, d_tab, 0, d_sizes, ws, s);
    if (e != hipSuccess)
        return e;
    return launch_huff_pack(g, codes, d_sizes, d_bits, nwords, ws, s);
}

hipError_t launch_huff_decode(const Geom &g, const uint32_t *d_tab, const uint32_t *d_bits,
                              unsigned long long nwords, const void *d_sizes, uint16_t *codes,
                              unsigned nsym, unsigned esc_len, Workspace &ws, hipStream_t s)
{
    const GeoArgs ga = geo_of(g);
    // one thread per block: workgroups of 1024 threads where the blocks fill
    // every CU that way, smaller ones (down to one wave) for fewer blocks, so
    // that a small field still spreads over all CUs
    long long want = (g.nblocks + 255) / 256;
    unsigned threads = 64;
    while ((long long)threads < want && threads < (unsigned)kUnpackThreads)
        threads <<= 1;
    const unsigned grid = (unsigned)((g.nblocks + threads - 1) / threads);
    // the lookup table goes through the encoder's codeword buffer (unused
    // while decoding)
    uint32_t *glut = reinterpret_cast<uint32_t *>(ws.enc_code);
    hipLaunchKernelGGL(k_huff_lut, dim3((1 << kLutBits) / 256), dim3(256), 0, s, d_tab, nsym,
                       esc_len, glut);
    const bool all = nsym <= (unsigned)kSymsLds;
    const unsigned nlds = all ? nsym : (unsigned)kSymsLds;
    const size_t lds = (size_t)(1 << kLutBits) * sizeof(uint32_t) + (size_t)threads * 64 +
                       (size_t)nlds * sizeof(uint16_t);
    const int sb = huff_size_bytes(g);
    hipError_t e = launch_scan_sizes(d_sizes, sb, g.nblocks, ws.boffsets, ws.bpartials,
                                     ws.bits_total, s);
    if (e != hipSuccess)
        return e;
    auto go = [&](auto kern, const auto *sz) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, s, d_tab, d_bits, nwords, ga,
                           sz, ws.boffsets, ws.bpartials, codes, ws.status, nsym, esc_len, glut);
    };
    if (sb == 2) {
        const uint16_t *sz = static_cast<const uint16_t *>(d_sizes);
        if (all)
            go(k_huff_unpack<uint16_t, true>, sz);
        else
            go(k_huff_unpack<uint16_t, false>, sz);
    } else {
        const uint32_t *sz = static_cast<const uint32_t *>(d_sizes);
        if (all)
            go(k_huff_unpack<uint32_t, true>, sz);
        else
            go(k_huff_unpack<uint32_t, false>, sz);
    }
    return hipGetLastError();
}

}  // namespace pwrel
