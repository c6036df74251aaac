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

// The T normalised products of the power method (Alg. 1, L_p) on an iterate
// held one entry per lane: mv(x) returns this lane's entry of H v, sum(x) the
// sum of x over the lanes of the row.  Normalising by ||H v|| only fixes the
// length of the iterate, so the products are scaled by exact powers of two
// instead, which round nothing: the first product fixes 2^-e with
// 2^e <= ||H v_0|| < 2^(e+1) and every later product takes the same 2^-e.
// H here is a sampled Gram matrix of nonnegative rows plus lambda I, so its
// top eigenvector u is nonnegative and ||H v_0|| >= L u.v_0 >= L / sqrt(R):
// each later product scales the length by less than 2 sqrt(R) and never
// shrinks the component along u.  Every 32 products the iterate is brought
// back near unit length by another power of two (32 products grow it by at
// most (2 sqrt(64))^32 = 2^128, so its sum of squares stays far inside
// FP64's range for any T), and once more at the end.  Returns false if
// H v_0 vanishes (L = 0 by definition); else v is the final iterate and
// vv = ||v||^2 exactly.
template <class MV, class SUM>
__device__ __forceinline__ bool power_iterate(double &v, double &vv, int T, MV mv, SUM sum)
{
    if (T <= 0)
        return true;
    const double w = mv(v);
    double n2 = sum(w * w);
    if (!(n2 > 0.0))
        return false;
    const int e = ilogb(n2) >> 1;
    v = ldexp(w, -e);
    if (T == 1) {
        vv = ldexp(n2, -2 * e);
        return true;
    }
    for (int t = 1; t < T; ++t) {
        v = ldexp(mv(v), -e);
        if ((t & 31) == 0 && t + 1 < T) {  // wave-uniform: T is
            n2 = sum(v * v);
            if (!(n2 > 0.0))
                return false;
            v = ldexp(v, -(ilogb(n2) >> 1));
        }
    }
    n2 = sum(v * v);
    if (!(n2 > 0.0))
        return false;
    const int k = ilogb(n2) >> 1;
    v = ldexp(v, -k);
    vv = ldexp(n2, -2 * k);
    return true;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

}  // namespace
}  // namespace ntc
