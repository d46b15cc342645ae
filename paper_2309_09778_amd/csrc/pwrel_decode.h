// Decoder kernel arguments and the independent-block lane decoder (internal).
#pragma once

#include "pwrel_kernels.h"

namespace pwrel {

struct DecodeArgs {
    long long n[3];
    int bd[3];
    long long nb[3];
    long long nblocks;
    int use_net, judge, independent;
    const uint8_t *bflags;
    const uint16_t *codes;
    const uint32_t *counts;
    const unsigned long long *offs;
    const unsigned long long *partials;
    const void *raw;
    unsigned long long n_raw;
    void *xh;
    int *pgrid;
    const int *praw;  // grid values of the raw values
    int *status;
    // halo mode: block order, done flags, ticket counter, this call's flag value
    const unsigned *order;
    unsigned *done;
    unsigned *ticket;
    unsigned epoch;
    // pencil decoder: tagged face buffers
    unsigned long long *zf, *yf;
    DevConsts c;
    MlpW mlp;
    // independent blocks: whole blocks per axis (decoded one per lane); the
    // workgroup-per-block kernel then takes only the clipped blocks
    long long nf[3];
    int partial_only;
    // x^ of every grid value q in [inv_lo, inv_lo + inv_n) (dtype of the field),
    // or nullptr: then x^ = grid_inverse(q) per point
    const void *invtab;
    long long inv_lo, inv_n;
};

// x^ of grid value q: from the table where it holds q, else computed
template <typename T>
__device__ __forceinline__ T inverse_of(int q, const DecodeArgs &a)
{
    const long long k = (long long)q - a.inv_lo;
    if (a.invtab && k >= 0 && k < a.inv_n)
        return reinterpret_cast<const T *>(a.invtab)[k];
    return (T)grid_inverse<T>(q, a.c);
}

// The k-th block clipped by a high face of the field (blocks outside the
// nf[0] x nf[1] x nf[2] grid of whole blocks): first the clipped z planes of
// blocks, then the clipped y rows below them, then the clipped x columns.
__host__ __device__ inline long long partial_block(long long k, const DecodeArgs &a)
{
    const long long nb0 = a.nb[0], nb1 = a.nb[1], nb2 = a.nb[2];
    const long long f0 = a.nf[0], f1 = a.nf[1], f2 = a.nf[2];
    const long long c1 = (nb0 - f0) * nb1 * nb2, c2 = f0 * (nb1 - f1) * nb2;
    long long bz, by, bx;
    if (k < c1) {
        bz = f0 + k / (nb1 * nb2);
        by = (k / nb2) % nb1;
        bx = k % nb2;
    } else if (k < c1 + c2) {
        const long long r = k - c1;
        bz = r / ((nb1 - f1) * nb2);
        by = f1 + (r / nb2) % (nb1 - f1);
        bx = r % nb2;
    } else {
        const long long r = k - c1 - c2;
        bz = r / (f1 * (nb2 - f2));
        by = (r / (nb2 - f2)) % f1;
        bx = f2 + r % (nb2 - f2);
    }
    return (bz * nb1 + by) * nb2 + bx;
}

// shapes the lane decoder handles (3-D blocks of 4 or 8, 2-D blocks of 16)
bool lanes_shape(int D, int B);
// decode the whole blocks of an independent-block stream, x^ written directly;
// HP as the workgroup decoder's (0 = BF16 matrix cores)
void launch_decode_lanes(const Geom &g, int HP, const DecodeArgs &a, hipStream_t s);

}  // namespace pwrel
