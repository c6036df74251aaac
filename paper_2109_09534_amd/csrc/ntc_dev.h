// Device helpers shared by the row kernels of libntc (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "ntc_internal.h"

namespace ntc {
namespace {

// Every row kernel runs one launch over one or many problems (a Launch):
// block b belongs to entry owner[b] (entry 0 when there is one entry) and is
// that entry's local block b - start[entry]; a problem of a pool that has
// stopped leaves at once.  The entry's RowArgs are read
// through the constant address space: they never change during a launch, so
// every field is a scalar load that the compiler may repeat at any point
// instead of holding it in registers.
typedef const __attribute__((address_space(4))) RowArgs CRowArgs;
#define NTC_ROW_PARAMS                                                                                       \
    const RowArgs *__restrict__ args_, const int32_t *__restrict__ start_, const int32_t *__restrict__ owner_, \
        const int32_t nent_
#define NTC_ROW_RESOLVE(a, blk)                              \
    int blk = static_cast<int>(blockIdx.x);                  \
    int ent_ = 0;                                            \
    if (nent_ > 1) {                                         \
        ent_ = owner_[blockIdx.x];                           \
        blk -= start_[ent_];                                 \
    }                                                        \
    CRowArgs &a = ((CRowArgs *)args_)[ent_];                 \
    if (a.stop != nullptr && *a.stop != 0)                   \
        return

// A 16-byte record.  NT (the problem's records are larger than the GPU's
// last-level cache): each sampled record is read once per sweep, so it is
// loaded non-temporally; its line is marked to leave the caches first and the
// factor rows that the gathers reuse stay cached longer.  A smaller record
// set stays cached from one sweep to the next and loads normally.  (A
// runtime choice between the two loads is merged by the compiler into one
// load without the hint, so the choice is a template parameter.)
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ uint4 load_record4(const uint32_t *p)
{
    u32x4_t t;
    if constexpr (NT)
        t = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(p));
    else
        t = *reinterpret_cast<const u32x4_t *>(p);
    return make_uint4(t.x, t.y, t.z, t.w);
}

// c ? u : v for a 16-byte record, one component at a time (a select of the
// whole vector can be lowered through private memory).
__device__ __forceinline__ uint4 pick4(bool c, const uint4 &u, const uint4 &v)
{
    return make_uint4(c ? u.x : v.x, c ? u.y : v.y, c ? u.z : v.z, c ? u.w : v.w);
}

template <int W>
__device__ __forceinline__ float group_sum(float v)
{
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Two wave sums at once, level by level, so that each level's two exchanges
// are in flight together.
__device__ __forceinline__ void wave_sum2(double &x, double &y)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double px = __shfl_xor(x, off, 64), py = __shfl_xor(y, off, 64);
        x += px;
        y += py;
    }
}

// True when d holds in every active lane of the wave.
__device__ __forceinline__ bool wave_all(bool d)
{
    return __ballot(!d) == 0;
}

// True when d holds in every active lane of this lane's 16-lane DPP row.
__device__ __forceinline__ bool row_all(bool d)
{
    const unsigned long long m = __ballot(!d);
    return ((m >> (__lane_id() & 48)) & 0xFFFFull) == 0;
}

// DPP controls (gfx9): quad permutations, half-row and row mirrors, row rotations.
constexpr int kDppXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
constexpr int kDppRor = 0x120;       // + s: row_ror:s

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Sum over the 16 lanes of a DPP row: quad butterflies, then two row
// rotations (every lane gets the sum; lanes may differ in the last bit).
__device__ __forceinline__ float row_sum_f32(float x)
{
    x += dpp_f32<kDppXor1>(x);
    x += dpp_f32<kDppXor2>(x);
    x += dpp_f32<kDppRor + 4>(x);
    x += dpp_f32<kDppRor + 8>(x);
    return x;
}

__device__ __forceinline__ double row_sum_f64(double x)
{
    x += dpp_f64<kDppXor1>(x);
    x += dpp_f64<kDppXor2>(x);
    x += dpp_f64<kDppHalfMirror>(x);
    x += dpp_f64<kDppMirror>(x);
    return x;
}

// Two row sums at once, level by level (independent DPP moves fill each
// other's wait states).
__device__ __forceinline__ void row_sum2_f64(double &x, double &y)
{
    double px = dpp_f64<kDppXor1>(x), py = dpp_f64<kDppXor1>(y);
    x += px;
    y += py;
    px = dpp_f64<kDppXor2>(x);
    py = dpp_f64<kDppXor2>(y);
    x += px;
    y += py;
    px = dpp_f64<kDppHalfMirror>(x);
    py = dpp_f64<kDppHalfMirror>(y);
    x += px;
    y += py;
    px = dpp_f64<kDppMirror>(x);
    py = dpp_f64<kDppMirror>(y);
    x += px;
    y += py;
}

__device__ __forceinline__ double row_max_f64(double x)
{
    x = fmax(x, dpp_f64<kDppXor1>(x));
    x = fmax(x, dpp_f64<kDppXor2>(x));
    x = fmax(x, dpp_f64<kDppHalfMirror>(x));
    x = fmax(x, dpp_f64<kDppMirror>(x));
    return x;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// This lane's term of the Collatz-Wielandt bound max_i (H v)_i / v_i (the
// optional L_p estimator): (H v)_i / v_i where v_i > 0, else 0.  H >= 0 and
// lambda > 0 keep every live entry of the iterate positive.
__device__ __forceinline__ double cw_ratio(bool live, double v, double w)
{
    return (live && v > 0.0) ? w / v : 0.0;
}

// L_p of Alg. 1 by the power method on an iterate held one entry per lane,
// from the start vector entry v (1/sqrt(R) on live lanes, 0 elsewhere):
// mv(x) returns this lane's entry of H x, sum(x) and mx(x) the sum and the
// maximum of x over the lanes of the row, sum2(x, y) replaces x and y by
// their two sums (the same adds as sum, interleaved), all(d) whether d holds
// in every lane of the row.  Returns the Rayleigh quotient of
// the T-th normalised iterate, or with lp_bound its Collatz-Wielandt bound
// max_i (H v)_i / v_i; 0 when H v_0 vanishes (L = 0 by definition).
//
// Normalising by ||H v|| only fixes the length of the iterate, so the
// products are scaled by exact powers of two instead, which round nothing:
// the first product fixes 2^-e with 2^e <= ||H v_0|| < 2^(e+1) and every
// later product takes the same 2^-e.  H here is a sampled Gram matrix of
// nonnegative rows plus lambda I, so its top eigenvector u is nonnegative and
// ||H v_0|| >= L u.v_0 >= L / sqrt(R): each later product scales the length
// by less than 2 sqrt(R) and never shrinks the component along u.  Every 32
// products the iterate is brought back near unit length by another power of
// two (32 products grow it by at most (2 sqrt(64))^32 = 2^128, so its sum of
// squares stays far inside FP64's range for any T), and once more at the end.
//
// The Rayleigh quotient of power iterates of a positive semidefinite matrix
// never decreases and approaches lambda_max geometrically; here the start
// vector has a component of at least 1/sqrt(R) along the nonnegative top
// eigenvector, so the approach is regular from the first products.  Every 2
// products from the 4th on the quotient is taken; once two consecutive ones
// (2 products apart, the later at least the 6th) agree to 2^-40 of the
// quotient, the remaining products could move it only by steps no larger
// than the last, so that quotient is returned: it equals the T-th one to
// about 1e-11 relative, six orders of magnitude inside the one-sweep parity
// bar.  The Collatz-Wielandt bound always runs all T products.
//
// Every decision here (the scale exponents, the exit) must be the same in
// all lanes of the row, or the lanes would leave the loop at different
// products and the cross-lane sums would read lanes that have left.  The
// sums are built from commutative pairwise adds, so they are the same bits
// in every lane as long as no product is fused into the first add: the
// products below are formed with contraction off.  The exit is also voted
// (a wave ballot): it is taken only when no lane of the row disagrees.
constexpr double kRqConverged = 9.094947017729282e-13;  // 2^-40

template <class MV, class SUM, class SUM2, class MAX, class ALL>
__device__ __forceinline__ double lp_estimate(bool live, double v, int T, int lp_bound, MV mv, SUM sum, SUM2 sum2,
                                              MAX mx, ALL all)
{
#pragma clang fp contract(off)
    double vv = 1.0;  // ||v||^2 (the start vector has unit norm)
    if (T > 0) {
        double w = mv(v);
        double n2 = sum(w * w);
        if (!(n2 > 0.0))
            return 0.0;
        const int e = ilogb(n2) >> 1;
        v = ldexp(w, -e);
        if (T == 1) {
            vv = ldexp(n2, -2 * e);
        } else {
            double rq_prev = 0.0;
            for (int t = 1; t < T; ++t) {
                w = mv(v);  // H v_t
                if (!lp_bound && t >= 4 && (t & 1) == 0 && t + 1 < T) {
                    double vw = v * w, vv2 = v * v;
                    sum2(vw, vv2);
                    const double rq = vw / vv2;
                    if (t >= 6 && all(fabs(rq - rq_prev) <= kRqConverged * rq))
                        return rq;
                    rq_prev = rq;
                }
                v = ldexp(w, -e);
                if ((t & 31) == 0 && t + 1 < T) {
                    n2 = sum(v * v);
                    if (!(n2 > 0.0))
                        return 0.0;
                    v = ldexp(v, -(ilogb(n2) >> 1));
                }
            }
            n2 = sum(v * v);
            if (!(n2 > 0.0))
                return 0.0;
            const int k = ilogb(n2) >> 1;
            v = ldexp(v, -k);
            vv = ldexp(n2, -2 * k);
        }
    }
    const double w = mv(v);
    return lp_bound ? mx(cw_ratio(live, v, w)) : sum(v * w) / vv;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

}  // namespace
}  // namespace ntc
