// Counter-based minibatch sampler of libntc, usable on host and device.
//
// Section II-B draws, for row p of the mode being updated, B_{l,p} =
// floor(c n_p) of the row's n_p observed entries uniformly at random.  A
// fresh subset is drawn for every (sweep k, mode i, inner step l, row p):
//
//   1. Four 32-bit round keys K = Philox4x32-10(counter, key) with
//      key = (seed lo, seed hi), counter = (p, k, (i << 16) | l, 0x53414D50).
//      Philox4x32-R: Salmon, Moraes, Dror, Shaw, SC'11.
//   2. A keyed permutation of [0, 2^w), w = max(2, ceil(log2 n_p)): an
//      unbalanced Feistel network (high half ceil(w/2) bits, low half
//      floor(w/2) bits) of 8 rounds, or 24 rounds when w <= 4; round r xors
//      the high half (r even) or the low half (r odd) with
//      F(other half, K[r mod 4] ^ r*0x9E3779B9), F a multiply/xorshift mix.
//   3. Cycle walking (Black and Rogaway 2002) restricts it to [0, n_p); the
//      sample is the images of j = 0 .. B_{l,p}-1.
//
// Everything is 32-bit integer arithmetic, so host and device agree bit for
// bit, and any j can be mapped independently (one lane per sample).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define NTC_HD __host__ __device__ __forceinline__
#else
#define NTC_HD inline
#endif

namespace ntc {

constexpr uint32_t kTagSample = 0x53414D50u;  // counter word 3 of the sampler
constexpr uint32_t kTagInit = 0x494E4954u;    // counter word 3 of the default init

struct U32x4 {
    uint32_t v[4];
};

NTC_HD void mul_wide(uint32_t a, uint32_t b, uint32_t &hi, uint32_t &lo)
{
    const uint64_t p = static_cast<uint64_t>(a) * static_cast<uint64_t>(b);
    hi = static_cast<uint32_t>(p >> 32);
    lo = static_cast<uint32_t>(p);
}

// Philox4x32 with 10 rounds; bijective in the counter for a fixed key.
NTC_HD U32x4 philox4x32_10(U32x4 ctr, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint32_t hA, lA, hB, lB;
        mul_wide(0xD2511F53u, ctr.v[0], hA, lA);
        mul_wide(0xCD9E8D57u, ctr.v[2], hB, lB);
        const U32x4 nxt = {{hB ^ ctr.v[1] ^ k0, lB, hA ^ ctr.v[3] ^ k1, lA}};
        ctr = nxt;
        k0 += 0x9E3779B9u;  // Weyl key schedule
        k1 += 0xBB67AE85u;
    }
    return ctr;
}

NTC_HD U32x4 sample_keys(uint64_t seed, int64_t k, int32_t mode, int32_t l, int64_t row)
{
    const U32x4 ctr = {{static_cast<uint32_t>(row), static_cast<uint32_t>(k),
                        (static_cast<uint32_t>(mode) << 16) | (static_cast<uint32_t>(l) & 0xFFFFu), kTagSample}};
    return philox4x32_10(ctr, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
}

NTC_HD uint32_t mix32(uint32_t v, uint32_t key)
{
    uint32_t h = v ^ key;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    return h;
}

// Domain description of one row's permutation.
struct Prp {
    uint32_t n;       // row length (domain size)
    uint32_t lo_bits; // floor(w/2)
    uint32_t hi_mask; // 2^ceil(w/2) - 1
    uint32_t lo_mask; // 2^floor(w/2) - 1
    int rounds;       // 8, or 24 when w <= 4
    U32x4 key;
};

NTC_HD Prp make_prp(uint32_t n, const U32x4 &key)
{
    uint32_t w = 2;
    while ((static_cast<uint64_t>(1) << w) < n)
        ++w;
    Prp d;
    d.n = n;
    d.lo_bits = w >> 1;
    d.hi_mask = (1u << (w - (w >> 1))) - 1u;
    d.lo_mask = (1u << (w >> 1)) - 1u;
    d.rounds = (w <= 4) ? 24 : 8;
    d.key = key;
    return d;
}

NTC_HD uint32_t prp_word(const Prp &d, uint32_t x)
{
    uint32_t hi = x >> d.lo_bits;
    uint32_t lo = x & d.lo_mask;
    // rounds is a multiple of 4: one pass of this loop uses K[0..3] in order
    for (int r = 0; r < d.rounds; r += 4) {
        const uint32_t r0 = static_cast<uint32_t>(r) * 0x9E3779B9u;
        hi ^= mix32(lo, d.key.v[0] ^ r0) & d.hi_mask;
        lo ^= mix32(hi, d.key.v[1] ^ (r0 + 0x9E3779B9u)) & d.lo_mask;
        hi ^= mix32(lo, d.key.v[2] ^ (r0 + 2u * 0x9E3779B9u)) & d.hi_mask;
        lo ^= mix32(hi, d.key.v[3] ^ (r0 + 3u * 0x9E3779B9u)) & d.lo_mask;
    }
    return (hi << d.lo_bits) | lo;
}

// j-th sampled position of the row (j < n).  The walk ends: the orbit of
// j under the permutation returns to j < n.
NTC_HD uint32_t prp_index(const Prp &d, uint32_t j)
{
    uint32_t x = prp_word(d, j);
    while (x >= d.n)
        x = prp_word(d, x);
    return x;
}

// B = floor(c n) with one binary64 multiply (identical on host and device).
NTC_HD int64_t minibatch_size(double c, int64_t n)
{
    const double t = c * static_cast<double>(n);
    int64_t b = static_cast<int64_t>(t);  // t >= 0: truncation is floor
    return b;
}

}  // namespace ntc
