// Counter-based minibatch sampler of libntc, usable on host and device.
//
// Section II-B draws, for row p of the mode being updated, B_{l,p} =
// floor(c n_p) of the row's n_p observed entries uniformly at random.  A
// fresh subset is drawn for every (sweep k, mode i, inner step l, row p):
//
//   1. Four 32-bit round keys K = Philox4x32-10(counter, key) with
//      key = (seed lo, seed hi), counter = (p, k, (i << 16) | l, 0x53414D50).
//      Philox4x32-R: Salmon, Moraes, Dror, Shaw, SC'11.
//   2. A keyed permutation of the word domain Z_A x Z_B, w = max(2,
//      ceil(log2 n_p)), A = 2^ceil(w/2), B = ceil(n_p / A): a Feistel network
//      with modular addition (FFX, Bellare-Rogaway-Spies 2010) of 8 rounds,
//      24 when w <= 4; round r adds F(other part, K[r mod 4] ^ r*0x9E3779B9)
//      into the Z_A part (r even) or, scaled to [0, B), into the Z_B part.
//   3. Cycle walking (Black and Rogaway 2002) restricts it to [0, n_p); the
//      sample is the images of j = 0 .. B_{l,p}-1.  A*B - n_p < A keeps the
//      walk short, so the lanes of a wave stay together.
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

// Round function: key xor, then two rounds of xor-shift and a multiply of
// the low 24 bits by a 24-bit constant (full-rate v_mul_u32_u24 on gfx9).
NTC_HD uint32_t mix32(uint32_t v, uint32_t key)
{
    uint32_t h = v ^ key;
    h ^= h >> 16;
    h = (h & 0xFFFFFFu) * 0x9E3779u;
    h ^= h >> 13;
    h = (h & 0xFFFFFFu) * 0xC2B2AEu;
    h ^= h >> 16;
    return h;
}

// Domain description of one row's permutation: the word domain is
// Z_A x Z_B, A = 2^a, a = ceil(w/2), B = ceil(n/A), word = lo * A + hi.
struct Prp {
    uint32_t n;       // row length
    uint32_t a;       // bits of the Z_A part
    uint32_t amask;   // A - 1
    uint32_t B;       // radix of the Z_B part
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
    d.a = (w + 1) >> 1;
    d.amask = (1u << d.a) - 1u;
    d.B = static_cast<uint32_t>((static_cast<uint64_t>(n) + d.amask) >> d.a);
    d.rounds = (w <= 4) ? 24 : 8;
    d.key = key;
    return d;
}

// One pass of the FFX-style network (modular addition, alternating halves).
NTC_HD uint32_t prp_word(const Prp &d, uint32_t x)
{
    uint32_t hi = x & d.amask;
    uint32_t lo = x >> d.a;
    // rounds is a multiple of 4: one pass of this loop uses K[0..3] in order
    for (int r = 0; r < d.rounds; r += 4) {
        const uint32_t r0 = static_cast<uint32_t>(r) * 0x9E3779B9u;
        hi = (hi + mix32(lo, d.key.v[0] ^ r0)) & d.amask;
        lo += ((mix32(hi, d.key.v[1] ^ (r0 + 0x9E3779B9u)) & 0xFFFFu) * d.B) >> 16;
        lo = lo >= d.B ? lo - d.B : lo;
        hi = (hi + mix32(lo, d.key.v[2] ^ (r0 + 2u * 0x9E3779B9u))) & d.amask;
        lo += ((mix32(hi, d.key.v[3] ^ (r0 + 3u * 0x9E3779B9u)) & 0xFFFFu) * d.B) >> 16;
        lo = lo >= d.B ? lo - d.B : lo;
    }
    return (lo << d.a) | hi;
}

// j-th sampled position of the row (j < n).  The walk ends: the orbit of
// j under the permutation returns to j < n; since A*B - n < A the expected
// number of extra passes is below A / n.
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
