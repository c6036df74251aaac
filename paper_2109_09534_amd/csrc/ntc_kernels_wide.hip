// Row kernels of libntc for 16 < R <= 64 on gfx950 (wave64).
//
// R > 32, or N > 4: one 64-lane workgroup per work item.  The wave is split
// into G = 64/RP groups of RP lanes; lane r of a group owns column r of the
// rank dimension.  A batch of up to 64 samples is mapped one sample per lane
// for the sampler and the record fetch (one 16/32-byte record per lane),
// staged in LDS, then consumed G samples at a time: every group gathers its
// sample's N-1 factor rows (one contiguous 4R-byte segment per mode, or 2R
// bytes from the BF16 shadow), forms the Khatri-Rao row k (Hadamard product,
// increasing mode order), reduces k.y with shuffles inside the group, and
// accumulates g += (k.y - x) k in FP32 and the row Hessian H += k k^T in
// FP64.  Groups are combined at the end of the item; a whole-row item then
// runs the FP64 power method for L_p and the fused step/projection/
// extrapolation; a split item writes its partial (g, H) and the finalize
// kernel combines the partials in slot order.
#include <hip/hip_runtime.h>

#include "ntc_bf16.h"
#include "ntc_dev.h"
#include "ntc_few.h"
#include "ntc_internal.h"
#include "ntc_rng.h"

namespace ntc {
namespace {

// Power method, step, projection and extrapolation for one row (Alg. 1,
// L_p, A_{l+1}, beta, Y_{l+1}).  Called by all 64 lanes; lanes r < RP of the
// first group hold g[r] (sampled gradient without ridge) and row r of the
// sampled H (without ridge); all other lanes pass zeros.
template <int RP, bool BF16, class Args>
__device__ void finish_row(const Args &a, int row, int lane, double g, double (&h)[RP], float y, double *s_v)
{
    const int R = a.R;
    const bool live = lane < RP && lane < R;
    if (live) {
        g += a.lambda * static_cast<double>(y);
#pragma unroll
        for (int q = 0; q < RP; ++q)
            if (q == lane)
                h[q] += a.lambda;  // static register index; diagonal of row `lane`
    }
    auto matvec = [&](double x) {
        if (lane < RP)
            s_v[lane] = x;
        __syncthreads();
        double w = 0.0;
        if (lane < RP) {
#pragma unroll
            for (int q = 0; q < RP; ++q)
                w += h[q] * s_v[q];
        }
        __syncthreads();
        return w;
    };
    const double L = lp_estimate(live, live ? a.v0 : 0.0, a.power_iters, a.lp_bound, matvec,
                                 [](double x) { return wave_sum(x); }, [](double &x, double &y) { wave_sum2(x, y); },
                                 [](double x) { return wave_max(x); }, [](bool d) { return wave_all(d); });
    if (!live)
        return;
    const int64_t off = static_cast<int64_t>(row) * R + lane;
    const float a_prev = (a.l == 0) ? y : a.A[off];
    const bool more = a.l + 1 < a.max_inner;
    if (L > 0.0) {
        double an = static_cast<double>(y) - g / L;
        an = an > 0.0 ? an : 0.0;
        const double sl = sqrt(L), sm = a.sqrt_lambda;
        const double beta = (sl - sm) / (sl + sm);
        const float af = static_cast<float>(an);
        a.A[off] = af;
        if (BF16)
            a.A16[off] = f32_to_bf16(af);
        if (more)
            a.Y[off] = static_cast<float>(an + beta * (an - static_cast<double>(a_prev)));
    } else if (more && a.l == 0) {
        a.Y[off] = y;  // row skipped: Y_1 = Y_0
    }
}

template <int RP, int NM, bool BF16, bool NT>
__global__ __launch_bounds__(64) void k_row_items(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    constexpr int G = 64 / RP;
    constexpr int RED = (G > 1) ? 64 * RP : 1;
    __shared__ uint32_t s_rec[64 * 8];
    __shared__ float s_k[64];
    __shared__ double s_red[RED];
    __shared__ double s_v[RP];
    __shared__ double s_g[64];

    const int nm = (NM > 0) ? NM : a.nmodes;
    const int rw = (NM > 0) ? ((NM <= 4) ? 4 : 8) : a.rec_words;
    const Item it = a.items[blk_];
    const int lane = threadIdx.x;
    const int r = lane % RP;
    const int grp = lane / RP;
    const int R = a.R;
    const bool rlive = r < R;

    const int64_t base = a.rowptr[it.row];
    const int64_t n = a.rowptr[it.row + 1] - base;
    const Prp prp = make_prp(static_cast<uint32_t>(n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, it.row));
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const float y = rlive ? ysrc[static_cast<int64_t>(it.row) * R + r] : 0.0f;

    float gacc = 0.0f;
    double h[RP];
#pragma unroll
    for (int q = 0; q < RP; ++q)
        h[q] = 0.0;

    for (int jb = it.j0; jb < it.j1; jb += 64) {
        const int cnt = min(64, it.j1 - jb);
        if (lane < cnt) {
            const uint32_t q = prp_index(prp, static_cast<uint32_t>(jb + lane));
            const uint32_t *src = a.records + (base + q) * rw;
            const uint4 w0 = load_record4<NT>(src);
            s_rec[lane * 8 + 0] = w0.x;
            s_rec[lane * 8 + 1] = w0.y;
            s_rec[lane * 8 + 2] = w0.z;
            s_rec[lane * 8 + 3] = w0.w;
            if (rw == 8) {
                const uint4 w1 = load_record4<NT>(src + 4);
                s_rec[lane * 8 + 4] = w1.x;
                s_rec[lane * 8 + 5] = w1.y;
                s_rec[lane * 8 + 6] = w1.z;
                s_rec[lane * 8 + 7] = w1.w;
            }
        }
        __syncthreads();
        for (int t0 = 0; t0 < cnt; t0 += G) {
            const int t = t0 + grp;
            const bool valid = t < cnt;
            float kv = 0.0f, x = 0.0f;
            if (valid) {
                kv = rlive ? 1.0f : 0.0f;
                for (int mm = 0; mm < nm - 1; ++mm) {
                    const int64_t off = s_rec[t * 8 + mm];  // coordinate * R
                    float f = 0.0f;
                    if (rlive) {
                        if (BF16)
                            f = bf16_to_f32(a.gath16[mm][off + r]);
                        else
                            f = a.gath[mm][off + r];
                    }
                    kv *= f;
                }
                x = __uint_as_float(s_rec[t * 8 + nm - 1]);
            }
            const float pred = group_sum<RP>(kv * y);
            const float res = valid ? pred - x : 0.0f;
            gacc = fmaf(res, kv, gacc);
            s_k[lane] = kv;
            __syncthreads();
            const double kd = static_cast<double>(kv);
#pragma unroll
            for (int q = 0; q < RP; ++q)
                h[q] = fma(kd, static_cast<double>(s_k[grp * RP + q]), h[q]);
            __syncthreads();
        }
    }

    // combine the groups into the first group
    double g = static_cast<double>(gacc);
    if (G > 1) {
        s_g[lane] = g;
#pragma unroll
        for (int q = 0; q < RP; ++q)
            s_red[lane * RP + q] = h[q];
        __syncthreads();
        if (grp == 0) {
            for (int gg = 1; gg < G; ++gg) {
                g += s_g[gg * RP + r];
#pragma unroll
                for (int q = 0; q < RP; ++q)
                    h[q] += s_red[(gg * RP + r) * RP + q];
            }
        } else {
            g = 0.0;
#pragma unroll
            for (int q = 0; q < RP; ++q)
                h[q] = 0.0;
        }
        __syncthreads();
    }

    if (it.slot >= 0) {
        if (lane < RP) {
            double *P = a.partials + static_cast<int64_t>(it.slot) * (RP + RP * RP);
            P[lane] = g;
#pragma unroll
            for (int q = 0; q < RP; ++q)
                P[RP + lane * RP + q] = h[q];
        }
        return;
    }
    finish_row<RP, BF16>(a, it.row, lane, g, h, y, s_v);
}

template <int RP, bool BF16>
__global__ __launch_bounds__(64) void k_row_finalize(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ double s_v[RP];
    const SplitRow sr = a.split[blk_];
    const int lane = threadIdx.x;
    const int R = a.R;
    double g = 0.0;
    double h[RP];
#pragma unroll
    for (int q = 0; q < RP; ++q)
        h[q] = 0.0;
    float y = 0.0f;
    if (lane < RP) {
        for (int s = 0; s < sr.nslots; ++s) {
            const double *P = a.partials + static_cast<int64_t>(sr.slot0 + s) * (RP + RP * RP);
            g += P[lane];
#pragma unroll
            for (int q = 0; q < RP; ++q)
                h[q] += P[RP + lane * RP + q];
        }
        if (lane < R) {
            const float *ysrc = (a.l == 0) ? a.A : a.Y;
            y = ysrc[static_cast<int64_t>(sr.row) * R + lane];
        }
    }
    finish_row<RP, BF16>(a, sr.row, lane, g, h, y, s_v);
}

// ------------------------------------------------- wave-per-item (R <= 32)
//
// 17 <= R <= 32, N <= 4: one wave per work item, split into four 16-lane
// groups; lane j of a group owns columns 2j and 2j + 1.  The item's samples
// are taken 64 at a time (sampler and record fetch one per lane, staged in
// LDS) and consumed four per step, one per group: each group gathers its
// sample's N-1 factor rows (one 8-byte pair per lane: 128 contiguous bytes
// per mode, or 64 from the BF16 shadow), forms the Khatri-Rao row k, reduces
// k.y over its 16 lanes with DPP and accumulates g += (k.y - x) k in FP32.
// With the columns ordered evens first, H has three distinct 16x16 blocks
// (even-even, even-odd, odd-odd); one v_mfma_f32_16x16x4f32 per block and
// step adds the four groups' rank-1 updates (K = the four groups) in FP32,
// added into FP64 after every 32 samples.

// Sum over the 32 lanes of a group (every lane of the group gets it).
__device__ __forceinline__ float group32_sum_f32(float x)
{
    x += dpp_f32<kDppXor1>(x);
    x += dpp_f32<kDppXor2>(x);
    x += dpp_f32<kDppRor + 4>(x);
    x += dpp_f32<kDppRor + 8>(x);
    return x + __shfl_xor(x, 16, 64);
}

// x[l] + x[l ^ 16] and x[l] + x[l ^ 32] through the gfx950 lane swaps (no
// LDS round trip).  A swap of x with itself leaves the lower and the upper
// partner's value in the two results, in either order, so their sum is the
// same in every lane of the pair.
__device__ __forceinline__ double swap16_sum(double x)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    const uint32_t lo = static_cast<uint32_t>(b), hi = static_cast<uint32_t>(b >> 32);
    const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double x0 = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(ph[0]) << 32) | pl[0]));
    const double x1 = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(ph[1]) << 32) | pl[1]));
    return x0 + x1;
}

__device__ __forceinline__ double swap32_sum(double x)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    const uint32_t lo = static_cast<uint32_t>(b), hi = static_cast<uint32_t>(b >> 32);
    const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const double x0 = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(ph[0]) << 32) | pl[0]));
    const double x1 = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(ph[1]) << 32) | pl[1]));
    return x0 + x1;
}

__device__ __forceinline__ double swap16_max(double x)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    const uint32_t lo = static_cast<uint32_t>(b), hi = static_cast<uint32_t>(b >> 32);
    const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double x0 = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(ph[0]) << 32) | pl[0]));
    const double x1 = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(ph[1]) << 32) | pl[1]));
    return fmax(x0, x1);
}

__device__ __forceinline__ double group32_max_f64(double x)
{
    return swap16_max(row_max_f64(x));
}

__device__ __forceinline__ double group32_sum_f64(double x)
{
    x += dpp_f64<kDppXor1>(x);
    x += dpp_f64<kDppXor2>(x);
    x += dpp_f64<kDppHalfMirror>(x);
    x += dpp_f64<kDppMirror>(x);
    return swap16_sum(x);
}

// Two group32 sums at once, level by level.
__device__ __forceinline__ void group32_sum2_f64(double &x, double &y)
{
    row_sum2_f64(x, y);
    x = swap16_sum(x);
    y = swap16_sum(y);
}

constexpr int kSlot32 = 32 + 32 * 32;  // doubles per partial slot: g[32], row-major H[32][32]

// One entry summed over `count` consecutive partial slots of S doubles, in
// slot order; the loads of eight slots are in flight together.
template <int S>
__device__ __forceinline__ double slot_sum(const double *p, int count)
{
    double acc = 0.0;
    for (int q = 0; q < count; q += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            t[u] = q + u < count ? p[static_cast<int64_t>(q + u) * S] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (q + u < count)
                acc += t[u];
    }
    return acc;
}

// Accumulator register v of lane l of v_mfma_f32_32x32x2f32 holds
// H[(v % 4) + 8 (v / 4) + 4 (l / 32)][l % 32].
__device__ __forceinline__ int mfma32_row(int v, int l)
{
    return (v & 3) + 8 * (v >> 2) + 4 * (l >> 5);
}

// Power method, step, projection and extrapolation for a row held by the
// whole wave, with H in any symmetric ordering of the columns.  Lane l:
// i = l % 32, half = l / 32 holds hd[q] = H[i][16 half + q] of the sampled
// Hessian in that ordering, with the ridge lambda already on its diagonal
// (the callers add it where H is staged); index i stands for column `col`
// of the factor; g: sampled gradient of that column (without ridge), y its
// Y value, on every lane.
template <bool BF16, class Args>
__device__ void finish_row32(const Args &a, int row, int lane, int col, double g, double (&hd)[16], float y,
                             double *s_v)
{
    const int R = a.R;
    const int i = lane & 31, half = lane >> 5;
    const bool live = col < R;
    if (live)
        g += a.lambda * static_cast<double>(y);
    // w_i = (H v)_i: each half sums its 16 columns, then the halves combine
    auto matvec = [&](double vi) {
        if (half == 0)
            s_v[i] = vi;
        __builtin_amdgcn_wave_barrier();
        double w4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 16; ++q)
            w4[q & 3] = fma(hd[q], s_v[16 * half + q], w4[q & 3]);
        __builtin_amdgcn_wave_barrier();
        return swap32_sum((w4[0] + w4[1]) + (w4[2] + w4[3]));
    };
    const double L = lp_estimate(live, live ? a.v0 : 0.0, a.power_iters, a.lp_bound, matvec,
                                 [](double x) { return group32_sum_f64(x); },
                                 [](double &x, double &y) { group32_sum2_f64(x, y); },
                                 [](double x) { return group32_max_f64(x); }, [](bool d) { return wave_all(d); });
    if (!live || half != 0)
        return;
    const int64_t off = static_cast<int64_t>(row) * R + col;
    const float a_prev = (a.l == 0) ? y : a.A[off];
    const bool more = a.l + 1 < a.max_inner;
    if (L > 0.0) {
        double an = static_cast<double>(y) - g / L;
        an = an > 0.0 ? an : 0.0;
        const double sl = sqrt(L), sm = a.sqrt_lambda;
        const double beta = (sl - sm) / (sl + sm);
        const float af = static_cast<float>(an);
        a.A[off] = af;
        if (BF16)
            a.A16[off] = f32_to_bf16(af);
        if (more)
            a.Y[off] = static_cast<float>(an + beta * (an - static_cast<double>(a_prev)));
    } else if (more && a.l == 0) {
        a.Y[off] = y;  // row skipped: Y_1 = Y_0
    }
}

template <int NM, bool BF16, bool PAIRS, bool NT>
// Five waves per SIMD: at most 96 registers, no spills, with the 8 KB of
// LDS below that is 20 waves per CU.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_rows32(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ uint4 s_rec[2 * 64];
    __shared__ double s_h[12 * 64];  // FP64 sums of the EE, EO, OO blocks: register v of lane l at v*64 + l
    // after the sample loop the record buffers are free: the gradient
    // partials (2 x 64) and the power method's vector (32) reuse them, which
    // keeps the wave at 8 KB of LDS (20 waves per CU)
    double *const s_g = reinterpret_cast<double *>(s_rec);
    double *const s_v = s_g + 2 * 64;
    const Item it = a.items[blk_];
    const int lane = threadIdx.x;
    const int j = lane & 15;    // columns 2j (even) and 2j + 1 (odd)
    const int grp = lane >> 4;  // which of the step's four samples
    const int R = a.R;
    const int c0 = 2 * j, c1 = 2 * j + 1;
    const bool l0 = c0 < R, l1 = c1 < R;
    // PAIRS (R even): every row starts 8-byte (FP32) / 4-byte (BF16) aligned,
    // so a lane reads its two columns with one load

    const int64_t base = a.rowptr[it.row];
    const int64_t n = a.rowptr[it.row + 1] - base;
    const Prp prp = make_prp(static_cast<uint32_t>(n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, it.row));
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const int64_t roff = static_cast<int64_t>(it.row) * R;
    const float y0 = l0 ? ysrc[roff + c0] : 0.0f;
    const float y1 = l1 ? ysrc[roff + c1] : 0.0f;
#pragma unroll
    for (int v = 0; v < 12; ++v)
        s_h[v * 64 + lane] = 0.0;
    // columns past R read columns 0 and 1 of the same row (never past its
    // end: the zero row is the last row of the table) and are masked afterwards
    const uint32_t e0 = l0 ? c0 : 0, e1 = l1 ? c1 : 1;
    const uint32_t pc = l0 ? c0 : 0;  // pair offset (R even: c0 < R implies c0 + 1 < R)

    // Software pipeline over blocks of 64 samples (one record per lane,
    // double-buffered in LDS) and sub-batches of 4 steps (16 samples): the
    // records of block k+1 are in flight while block k is reduced, and the
    // gathers of sub-batch s+1 while sub-batch s is.  No load sits under a
    // branch (a record past the item's end is read from entry 0 and staged
    // as the zero record; the gathers of a missing step read the zero rows),
    // so the compiler counts the loads in flight and a wait for sub-batch s
    // leaves the loads issued after it outstanding.
    struct Sub {
        float f0[NM - 1][4], f1[NM - 1][4];
    };
    const uint4 zr = make_uint4(a.zrec[0], a.zrec[1], a.zrec[2], a.zrec[3]);
    auto fetch = [&](int jb, bool &live) {
        live = lane < it.j1 - jb;
        int64_t e = 0;
        if (live)
            e = base + prp_index(prp, static_cast<uint32_t>(jb + lane));
        return load_record4<NT>(a.records + e * 4);
    };
    // gathers of the four steps from s0 of a staged block
    auto issue = [&](const uint4 *buf, int s0, Sub &S) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            {
                const uint4 rec = buf[4 * (s0 + t) + grp];
                const uint32_t rw[3] = {rec.x, rec.y, rec.z};
#pragma unroll
                for (int mm = 0; mm < NM - 1; ++mm) {
                    if (BF16) {
                        const uint16_t *src = a.gath16[mm] + rw[mm];
                        if (PAIRS) {
                            const uint32_t w = *reinterpret_cast<const uint32_t *>(src + pc);
                            S.f0[mm][t] = __uint_as_float(w << 16);
                            S.f1[mm][t] = __uint_as_float(w & 0xFFFF0000u);
                        } else {
                            S.f0[mm][t] = bf16_to_f32(src[e0]);
                            S.f1[mm][t] = bf16_to_f32(src[e1]);
                        }
                    } else {
                        const float *src = a.gath[mm] + rw[mm];
                        if (PAIRS) {
                            const float2 w = *reinterpret_cast<const float2 *>(src + pc);
                            S.f0[mm][t] = w.x;
                            S.f1[mm][t] = w.y;
                        } else {
                            S.f0[mm][t] = src[e0];
                            S.f1[mm][t] = src[e1];
                        }
                    }
                }
            }
        }
    };
    float gf0 = 0.0f, gf1 = 0.0f;
    f32x4 ee = {0.0f}, eo = {0.0f}, oo = {0.0f};
    auto compute = [&](const uint4 *buf, int s0, int ns, const Sub &S) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < ns) {  // wave-uniform
                float k0 = S.f0[0][t], k1 = S.f1[0][t];
#pragma unroll
                for (int mm = 1; mm < NM - 1; ++mm) {
                    k0 *= S.f0[mm][t];
                    k1 *= S.f1[mm][t];
                }
                k0 = l0 ? k0 : 0.0f;
                k1 = l1 ? k1 : 0.0f;
                const uint4 rec = buf[4 * (s0 + t) + grp];
                const uint32_t xw[4] = {rec.x, rec.y, rec.z, rec.w};
                const float x = __uint_as_float(xw[NM - 1]);  // 0 for a missing sample
                const float pred = row_sum_f32(fmaf(k0, y0, k1 * y1));
                const float res = pred - x;
                gf0 = fmaf(res, k0, gf0);
                gf1 = fmaf(res, k1, gf1);
                // the four groups' samples: K = 4 of each 16x16 block of the column-permuted H
                ee = __builtin_amdgcn_mfma_f32_16x16x4f32(k0, k0, ee, 0, 0, 0);
                eo = __builtin_amdgcn_mfma_f32_16x16x4f32(k0, k1, eo, 0, 0, 0);
                oo = __builtin_amdgcn_mfma_f32_16x16x4f32(k1, k1, oo, 0, 0, 0);
            }
        }
    };
    // FP32 block sums of 32 samples go into FP64
    auto flush = [&]() {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            s_h[v * 64 + lane] += static_cast<double>(ee[v]);
            s_h[(4 + v) * 64 + lane] += static_cast<double>(eo[v]);
            s_h[(8 + v) * 64 + lane] += static_cast<double>(oo[v]);
            ee[v] = 0.0f;
            eo[v] = 0.0f;
            oo[v] = 0.0f;
        }
    };
    auto nsteps = [&](int jb, int sub) {  // valid steps of sub-batch `sub` of the block at jb
        const int steps = (min(64, it.j1 - jb) + 3) >> 2;
        return max(0, min(4, steps - 4 * sub));
    };

    Sub SA, SB;
    int buf = 0;
    {
        bool lv;
        const uint4 w = fetch(it.j0, lv);
        s_rec[lane] = pick4(lv, w, zr);
        __builtin_amdgcn_wave_barrier();
        issue(s_rec, 0, SA);
    }
    for (int jb = it.j0; jb < it.j1; jb += 64) {
        // the next block's records, in flight during this block (all zero
        // records after the last block: staged and gathered, never reduced)
        bool lvn;
        const uint4 wn = fetch(jb + 64, lvn);
        const uint4 *cur = s_rec + 64 * buf;
        issue(cur, 4, SB);
        compute(cur, 0, nsteps(jb, 0), SA);
        issue(cur, 8, SA);
        compute(cur, 4, nsteps(jb, 1), SB);
        flush();
        issue(cur, 12, SB);
        compute(cur, 8, nsteps(jb, 2), SA);
        {
            uint4 *nxt = s_rec + 64 * (buf ^ 1);
            nxt[lane] = pick4(lvn, wn, zr);
            __builtin_amdgcn_wave_barrier();
            issue(nxt, 0, SA);
        }
        compute(cur, 12, nsteps(jb, 3), SB);
        flush();
        __builtin_amdgcn_wave_barrier();  // this block's reads of s_rec come before its next staging
        buf ^= 1;
    }
    // gradient of columns 2j and 2j + 1: the four groups' partial sums in group order
    s_g[lane] = static_cast<double>(gf0);
    s_g[64 + lane] = static_cast<double>(gf1);
    __builtin_amdgcn_wave_barrier();
    // block entries: register v of lane l holds D[4 (l / 16) + v][l % 16], kept at
    // s_h[(4 b + (r & 3)) * 64 + 16 (r >> 2) + c] for entry (r, c) of block b (EE, EO, OO)
    auto gsum = [&](int c) {
        const int par = c & 1, jj = c >> 1;
        return ((s_g[64 * par + jj] + s_g[64 * par + 16 + jj]) + s_g[64 * par + 32 + jj]) + s_g[64 * par + 48 + jj];
    };

    if (it.slot >= 0) {
        // partial slot in column order: H[2i][2c] = EE[i][c], H[2i][2c+1] = EO[i][c] = H[2c+1][2i],
        // H[2i+1][2c+1] = OO[i][c]
        double *P = a.partials + static_cast<int64_t>(it.slot) * kSlot32;
        if (lane < 32)
            P[lane] = gsum(lane);
        const int cc = lane & 15;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ii = 4 * (lane >> 4) + v;
            P[32 + (2 * ii) * 32 + 2 * cc] = s_h[v * 64 + lane];
            P[32 + (2 * ii) * 32 + 2 * cc + 1] = s_h[(4 + v) * 64 + lane];
            P[32 + (2 * cc + 1) * 32 + 2 * ii] = s_h[(4 + v) * 64 + lane];
            P[32 + (2 * ii + 1) * 32 + 2 * cc + 1] = s_h[(8 + v) * 64 + lane];
        }
        return;
    }
    // the power method on the permuted order: index p < 16 is column 2p, p >= 16 is column 2(p-16)+1.
    // Lane (i, half) takes row i, columns 16 half .. 16 half + 15 of
    //   [EE EO ]
    //   [EO' OO]
    // which is a row of EE, EO or OO, or for i >= 16, half 0, a column of EO.
    const int i = lane & 31, half = lane >> 5;
    const int col = i < 16 ? 2 * i : 2 * (i - 16) + 1;
    const double g = gsum(col);
    __builtin_amdgcn_wave_barrier();  // every lane has read s_g before the record area is reused below
    // EO transposed into the record area (16 x 16, row-major): lane l holds EO[4 (l / 16) + v][l % 16]
    double *const s_t = s_g;
    {
        const int c = lane & 15, r0 = 4 * (lane >> 4);
        double2 *const dst = reinterpret_cast<double2 *>(s_t + c * 16 + r0);
        dst[0] = make_double2(s_h[4 * 64 + lane], s_h[5 * 64 + lane]);
        dst[1] = make_double2(s_h[6 * 64 + lane], s_h[7 * 64 + lane]);
    }
    // the ridge on the diagonal, by the lane that reads it: EE[i][i] (lanes 0-15), OO[i-16][i-16] (lanes 48-63)
    const int r = i & 15;
    const int b = i < 16 ? half : 2;  // block of the row read: EE, EO or OO
    const int rbase = (4 * b + (r & 3)) * 64 + 16 * (r >> 2);
    if (col < R && (i < 16) == (half == 0))
        s_h[rbase + r] += a.lambda;
    __builtin_amdgcn_wave_barrier();
    const double *const src = (i >= 16 && half == 0) ? s_t + 16 * r : s_h + rbase;
    double hd[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        hd[q] = src[q];
    __builtin_amdgcn_wave_barrier();  // the power method's vector reuses the record area
    const float y = i < 16 ? y0 : y1;  // column col of the row, already in registers
    finish_row32<BF16>(a, it.row, lane, col, g, hd, y, s_v);
}

// ------------------------------------------------- wave-per-item (R <= 64)
//
// Rows with 33 <= R <= 64 and N <= 4: one wave per item (a whole row of at
// most item_samples samples, or a chunk of a split row).  Four 16-lane
// groups take one sample each per step; lane j owns columns 4j .. 4j+3.
// With the columns ordered by c mod 4 (position 16 (c mod 4) + c / 4), H
// splits into 16x16 blocks B(q1, q2)[i][j] = sum_s k_s[4i+q1] k_s[4j+q2];
// the ten with q1 <= q2 take one v_mfma_f32_16x16x4f32 each per step (the
// step's four samples are the K = 4 of the product).  Block sums go into FP64
// (LDS) every 32 samples.  A split item writes its partial slot (g[64], H
// row-major) for the slot sums and the finalize; a whole row assembles its
// FP64 H row per lane and runs the power method and the step.
// VEC: columns a lane reads per load (4 when R % 4 == 0, 2 when R is even).
constexpr int kSlot64 = 64 + 64 * 64;

// block index of (q1, q2), q1 <= q2, in the order (0,0) (0,1) (0,2) (0,3) (1,1) ...
__device__ __forceinline__ int blk64(int q1, int q2)
{
    return q1 * 4 - (q1 * (q1 - 1)) / 2 + (q2 - q1);
}

template <int NM, bool BF16, int VEC, bool NT>
__global__ __launch_bounds__(64) void k_rows64(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ uint4 s_rec[2 * 64];
    __shared__ double s_h[40 * 64];  // block b, register v of lane l at (4 b + v) * 64 + l
    // After the sample loop the record buffers are free and hold the gradient
    // partials (column 4 j + q of group g at q * 64 + 16 g + j); the power
    // method's vector reuses the start of s_h once every lane has read its
    // row of H.  22 KB of LDS per wave: seven waves per CU instead of six.
    double *const s_g = reinterpret_cast<double *>(s_rec);
    double *const s_v = s_h;
    const Item it = a.items[blk_];
    const int lane = threadIdx.x;
    const int j = lane & 15;
    const int grp = lane >> 4;
    const int R = a.R;
    const int cb = 4 * j;
    bool live[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        live[q] = cb + q < R;

    const int64_t base = a.rowptr[it.row];
    const int64_t n = a.rowptr[it.row + 1] - base;
    const Prp prp = make_prp(static_cast<uint32_t>(n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, it.row));
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const int64_t roff = static_cast<int64_t>(it.row) * R;
    float yq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        yq[q] = live[q] ? ysrc[roff + cb + q] : 0.0f;
#pragma unroll
    for (int v = 0; v < 40; ++v)
        s_h[v * 64 + lane] = 0.0;
    // columns past R read column 0 of the same row (never past its end: the
    // zero row is the last row of the table) and are masked afterwards.
    // VEC = 4 (R % 4 == 0): cb < R implies cb + 3 < R; VEC = 2 (R even): a
    // pair starting below R ends below R.
    uint32_t off[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        off[q] = live[q] ? cb + q : 0;
    const uint32_t off4 = live[0] ? cb : 0;
    const uint32_t off2[2] = {live[0] ? cb : 0u, live[2] ? cb + 2u : 0u};

    struct Sub {
        float f[NM - 1][2][4];
    };
    // no load under a branch, so the compiler counts the loads in flight: a
    // record past the item's end is read from entry 0 and staged as the zero
    // record, and the gathers of a missing step read the zero rows
    const uint4 zr = make_uint4(a.zrec[0], a.zrec[1], a.zrec[2], a.zrec[3]);
    auto fetch = [&](int jb, bool &lv) {
        lv = lane < it.j1 - jb;
        int64_t e = 0;
        if (lv)
            e = base + prp_index(prp, static_cast<uint32_t>(jb + lane));
        return load_record4<NT>(a.records + e * 4);
    };
    // gathers of the two steps from s0 of a staged block
    auto issue = [&](const uint4 *buf, int s0, Sub &S) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            {
                const uint4 rec = buf[4 * (s0 + t) + grp];
                const uint32_t rw[3] = {rec.x, rec.y, rec.z};
#pragma unroll
                for (int mm = 0; mm < NM - 1; ++mm) {
                    float *d = S.f[mm][t];
                    if (BF16) {
                        const uint16_t *src = a.gath16[mm] + rw[mm];
                        if (VEC == 4) {
                            const uint2 w = *reinterpret_cast<const uint2 *>(src + off4);
                            d[0] = __uint_as_float(w.x << 16);
                            d[1] = __uint_as_float(w.x & 0xFFFF0000u);
                            d[2] = __uint_as_float(w.y << 16);
                            d[3] = __uint_as_float(w.y & 0xFFFF0000u);
                        } else if (VEC == 2) {
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const uint32_t w = *reinterpret_cast<const uint32_t *>(src + off2[h]);
                                d[2 * h] = __uint_as_float(w << 16);
                                d[2 * h + 1] = __uint_as_float(w & 0xFFFF0000u);
                            }
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                d[q] = bf16_to_f32(src[off[q]]);
                        }
                    } else {
                        const float *src = a.gath[mm] + rw[mm];
                        if (VEC == 4) {
                            const float4 w = *reinterpret_cast<const float4 *>(src + off4);
                            d[0] = w.x;
                            d[1] = w.y;
                            d[2] = w.z;
                            d[3] = w.w;
                        } else if (VEC == 2) {
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const float2 w = *reinterpret_cast<const float2 *>(src + off2[h]);
                                d[2 * h] = w.x;
                                d[2 * h + 1] = w.y;
                            }
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                d[q] = src[off[q]];
                        }
                    }
                }
            }
        }
    };
    float gf[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 acc[10];
#pragma unroll
    for (int b = 0; b < 10; ++b)
        acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    auto compute = [&](const uint4 *buf, int s0, int ns, const Sub &S) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (t < ns) {  // wave-uniform
                float k[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float v = S.f[0][t][q];
#pragma unroll
                    for (int mm = 1; mm < NM - 1; ++mm)
                        v *= S.f[mm][t][q];
                    k[q] = live[q] ? v : 0.0f;
                }
                const uint4 rec = buf[4 * (s0 + t) + grp];
                const uint32_t xw[4] = {rec.x, rec.y, rec.z, rec.w};
                const float x = __uint_as_float(xw[NM - 1]);  // 0 for a missing sample
                const float pred = row_sum_f32(fmaf(k[0], yq[0], fmaf(k[1], yq[1], fmaf(k[2], yq[2], k[3] * yq[3]))));
                const float res = pred - x;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    gf[q] = fmaf(res, k[q], gf[q]);
#pragma unroll
                for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
                    for (int q2 = q1; q2 < 4; ++q2)
                        acc[blk64(q1, q2)] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32(k[q1], k[q2], acc[blk64(q1, q2)], 0, 0, 0);
            }
        }
    };
    // FP32 block sums of 32 samples go into FP64
    auto flush = [&]() {
#pragma unroll
        for (int b = 0; b < 10; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                s_h[(4 * b + v) * 64 + lane] += static_cast<double>(acc[b][v]);
                acc[b][v] = 0.0f;
            }
    };
    auto nsteps = [&](int jb, int sub) {  // valid steps of sub-batch `sub` (2 steps) of the block at jb
        const int steps = (min(64, it.j1 - jb) + 3) >> 2;
        return max(0, min(2, steps - 2 * sub));
    };

    // software pipeline: records of the next block of 64 samples in flight
    // during this one, gathers of the next sub-batch during this one
    Sub SA, SB;
    int buf = 0;
    {
        bool lv;
        const uint4 w = fetch(it.j0, lv);
        s_rec[lane] = pick4(lv, w, zr);
        __builtin_amdgcn_wave_barrier();
        issue(s_rec, 0, SA);
    }
    for (int jb = it.j0; jb < it.j1; jb += 64) {
        // the next block's records (all zero records after the last block:
        // staged and gathered, never reduced)
        bool lvn;
        const uint4 wn = fetch(jb + 64, lvn);
        const uint4 *cur = s_rec + 64 * buf;
#pragma unroll
        for (int sp = 0; sp < 8; sp += 2) {
            issue(cur, 2 * (sp + 1), SB);
            compute(cur, 2 * sp, nsteps(jb, sp), SA);
            if (sp + 2 < 8) {
                issue(cur, 2 * (sp + 2), SA);
            } else {
                uint4 *nxt = s_rec + 64 * (buf ^ 1);
                nxt[lane] = pick4(lvn, wn, zr);
                __builtin_amdgcn_wave_barrier();
                issue(nxt, 0, SA);
            }
            compute(cur, 2 * (sp + 1), nsteps(jb, sp + 1), SB);
            if (sp == 2 || sp == 6)
                flush();
        }
        __builtin_amdgcn_wave_barrier();  // this block's reads of s_rec come before its next staging
        buf ^= 1;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        s_g[q * 64 + lane] = static_cast<double>(gf[q]);
    __builtin_amdgcn_wave_barrier();
    // gradient of column c: the four groups' partials in group order
    auto gsum = [&](int c) {
        const int q = c & 3, jj = c >> 2;
        return ((s_g[q * 64 + jj] + s_g[q * 64 + 16 + jj]) + s_g[q * 64 + 32 + jj]) + s_g[q * 64 + 48 + jj];
    };

    if (it.slot >= 0) {
        // partial slot, row-major: this lane's block entries D[4 (l / 16) + v][l % 16] of B(q1, q2)
        // are H[4 (4 grp + v) + q1][4 j + q2], and their transposes
        double *P = a.partials + static_cast<int64_t>(it.slot) * kSlot64;
        P[lane] = gsum(lane);
#pragma unroll
        for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
            for (int q2 = q1; q2 < 4; ++q2)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double val = s_h[(4 * blk64(q1, q2) + v) * 64 + lane];
                    const int r = 4 * (4 * grp + v) + q1, c = cb + q2;
                    P[64 + r * 64 + c] = val;
                    if (q1 != q2)
                        P[64 + c * 64 + r] = val;
                }
        return;
    }
    // whole row: lane r takes row r of H (position (q1, i) with r = 4 i + q1)
    const int r = lane, q1 = r & 3, i = r >> 2;
    double h[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) {
        const int q2 = c & 3, jj = c >> 2;
        // q1 <= q2: B(q1, q2)[i][jj]; else the transpose B(q2, q1)[jj][i]
        const int lo = q1 <= q2 ? q1 : q2, hi = q1 <= q2 ? q2 : q1;
        const int ri = q1 <= q2 ? i : jj, ci = q1 <= q2 ? jj : i;
        h[c] = s_h[(4 * blk64(lo, hi) + (ri & 3)) * 64 + 16 * (ri >> 2) + ci];
    }
    const double g = gsum(r);
    const float y = r < R ? ysrc[roff + r] : 0.0f;
    finish_row<64, BF16>(a, it.row, lane, g, h, y, s_v);
}

// Split rows with 17 <= R <= 32: a 256-thread block sums the row's partial
// slots, thread t taking entries t, t + 256, ... of the slot in slot order
// (coalesced, a fixed order per entry), then its first wave runs the power
// method and step as above.
template <bool BF16>
__global__ __launch_bounds__(256) void k_finalize32(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ double s_p[kSlot32];
    __shared__ double s_v[32];
    const SplitRow sr = a.split[blk_];
    const int tid = threadIdx.x;
    const double *src = a.partials + static_cast<int64_t>(sr.slot0) * kSlot32;
    for (int e = tid; e < kSlot32; e += 256)
        s_p[e] = slot_sum<kSlot32>(src + e, sr.nslots);
    __syncthreads();
    if (tid >= 64)
        return;
    const int lane = tid;
    const int i = lane & 31, half = lane >> 5;
    const double g = s_p[i];
    if (i < a.R && half == (i >> 4))
        s_p[32 + i * 33] += a.lambda;  // the ridge, by the lane that reads the diagonal
    double hd[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        hd[q] = s_p[32 + i * 32 + 16 * half + q];
    float y = 0.0f;
    if (i < a.R) {
        const float *ysrc = (a.l == 0) ? a.A : a.Y;
        y = ysrc[static_cast<int64_t>(sr.row) * a.R + i];
    }
    finish_row32<BF16>(a, sr.row, lane, i, g, hd, y, s_v);
}

// Second-level slot sums of rows split into many items: one 256-thread
// block per group, thread t summing entries t, t + 256, ... over the group's
// slots in slot order.
template <int RP>
__global__ __launch_bounds__(256) void k_reduce_slots(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    constexpr int S = RP + RP * RP;
    const SlotGroup gr = a.groups[blk_];
    const double *src = a.partials + static_cast<int64_t>(gr.src) * S;
    for (int e = threadIdx.x; e < S; e += 256)
        a.partials[static_cast<int64_t>(gr.dst) * S + e] = slot_sum<S>(src + e, gr.count);
}


// ------------------------------------------------- rows with few samples (17 <= R <= 32)
//
// Rows whose minibatch has at most tiny_max (16 by default) samples, four to
// a one-wave block, one sample per lane (ntc_few.h).
template <int NM, bool BF16, int W, bool NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_few32(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ FewShared sh;
    few_rows<32, NM, BF16, W, NT>(a, a.tiny, a.n_tiny, blk_, sh);
}

#define NTC_GO(KERNEL, BLOCK) \
    hipLaunchKernelGGL(KERNEL, dim3(L.blocks), dim3(BLOCK), 0, s, L.args, L.start, L.owner, L.n)

template <bool BF16, bool PAIRS, bool NT>
hipError_t go_rows32(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.nmodes == 3)
        NTC_GO((k_rows32<3, BF16, PAIRS, NT>), 64);
    else if (kc.nmodes == 4)
        NTC_GO((k_rows32<4, BF16, PAIRS, NT>), 64);
    else
        NTC_GO((k_rows32<2, BF16, PAIRS, NT>), 64);
    return hipGetLastError();
}

template <bool BF16, int VEC, bool NT>
hipError_t go_rows64(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.nmodes == 3)
        NTC_GO((k_rows64<3, BF16, VEC, NT>), 64);
    else if (kc.nmodes == 4)
        NTC_GO((k_rows64<4, BF16, VEC, NT>), 64);
    else
        NTC_GO((k_rows64<2, BF16, VEC, NT>), 64);
    return hipGetLastError();
}

template <bool BF16, bool NT>
hipError_t go_rows(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.rp == 32) {
        if (kc.nmodes > 4)
            NTC_GO((k_row_items<32, 0, BF16, NT>), 64);
        else if (kc.pairs)
            return go_rows32<BF16, true, NT>(kc, L, s);
        else
            return go_rows32<BF16, false, NT>(kc, L, s);
    } else if (kc.rp == 64) {
        if (kc.nmodes > 4)
            NTC_GO((k_row_items<64, 0, BF16, NT>), 64);
        else if (kc.pairs == 2)
            return go_rows64<BF16, 4, NT>(kc, L, s);
        else if (kc.pairs == 1)
            return go_rows64<BF16, 2, NT>(kc, L, s);
        else
            return go_rows64<BF16, 1, NT>(kc, L, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool BF16, int W, bool NT>
hipError_t go_few32(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.nmodes == 3)
        NTC_GO((k_few32<3, BF16, W, NT>), 64);
    else if (kc.nmodes == 4)
        NTC_GO((k_few32<4, BF16, W, NT>), 64);
    else
        NTC_GO((k_few32<2, BF16, W, NT>), 64);
    return hipGetLastError();
}

// load width of the few-sample kernel: FP32 four columns when R % 4 == 0, BF16
// eight when R % 8 == 0; two when R is even; else one; R = 32 without masks
template <bool BF16, bool NT>
hipError_t go_few(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.rp != 32 || kc.nmodes > 4)
        return hipErrorInvalidValue;
    const int w = kc.pairs == 4 ? 3 : BF16 ? (kc.pairs == 3 ? 2 : kc.pairs >= 1 ? 1 : 0) : (kc.pairs >= 2 ? 2 : kc.pairs);
    if (w == 3)
        return go_few32<BF16, 3, NT>(kc, L, s);
    if (w == 2)
        return go_few32<BF16, 2, NT>(kc, L, s);
    if (w == 1)
        return go_few32<BF16, 1, NT>(kc, L, s);
    return go_few32<BF16, 0, NT>(kc, L, s);
}

template <bool BF16>
hipError_t go_finalize(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.rp == 32)
        NTC_GO((k_finalize32<BF16>), 256);
    else if (kc.rp == 64)
        NTC_GO((k_row_finalize<64, BF16>), 64);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t go_reduce(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.rp == 32)
        NTC_GO((k_reduce_slots<32>), 256);
    else if (kc.rp == 64)
        NTC_GO((k_reduce_slots<64>), 256);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

#undef NTC_GO

}  // namespace

namespace {

template <bool NT>
hipError_t launch_wide(RowKernel kind, const KernelClass &kc, const Launch &L, hipStream_t s)
{
    const bool b = kc.bf16 != 0;
    switch (kind) {
    case kRows:
        return b ? go_rows<true, NT>(kc, L, s) : go_rows<false, NT>(kc, L, s);
    case kFinalize:
        return b ? go_finalize<true>(kc, L, s) : go_finalize<false>(kc, L, s);
    case kReduce:
        return go_reduce(kc, L, s);
    case kTiny:
        return b ? go_few<true, NT>(kc, L, s) : go_few<false, NT>(kc, L, s);
    case kChunks:
    case kFew:
        return hipSuccess;
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_row_kernel_wide(RowKernel kind, const KernelClass &kc, const Launch &L, hipStream_t s)
{
    return kc.nt ? launch_wide<true>(kind, kc, L, s) : launch_wide<false>(kind, kc, L, s);
}

}  // namespace ntc
