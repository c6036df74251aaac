// Rows with few samples, four to a wave (gfx950, wave64): shared by the
// R <= 16 and the 17 <= R <= 32 row kernels.
//
// A row whose minibatch has at most 16 samples is owned by one 16-lane group,
// lane s of the group by its sample s.  A lane gathers its sample's whole
// factor rows (C = 16 or 32 columns), so k, k.y and the row sum of k stay in
// the lane.  The Gram matrix G = K K^T of each row (B x B, B <= 16) comes
// from one v_mfma_f32_16x16x1f32 per column: its four output blocks are the
// four groups' rank-one updates by that column.  The column sums of the
// residual terms (the sampled gradient) are a four-level DPP reduce-scatter
// that leaves lane s with columns (C / 16) s .. (C / 16) s + C / 16 - 1.
//
// The power method of Alg. 1 on H = K^T K + lambda I runs in the span of v_0
// and the sampled rows, v = alpha v_0 + K^T u: with c = K v_0, z = G u and
// K v = alpha c + z,
//   H v = (lambda alpha) v_0 + K^T (K v + lambda u),
//   ||v||^2 = alpha^2 + u.(2 alpha c + z),   v.Hv = ||K v||^2 + lambda ||v||^2,
// so every product is one 16-entry product by G, and the iterates, the
// power-of-two scalings, the exit test and the Rayleigh quotient are those
// of the R-dimensional method in exact arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include "ntc_bf16.h"
#include "ntc_dev.h"
#include "ntc_internal.h"
#include "ntc_rng.h"

namespace ntc {
namespace {

// The first C columns of a factor row; columns >= R are zero, and a load
// past R reads the start of the same row instead (never past the row's end).
// W: 3 = R is C, four FP32 or eight BF16 columns per load; 2 = four FP32 or
// eight BF16 columns per load; 1 = two per load; 0 = one.
template <int C, int W>
__device__ __forceinline__ void few_row(const float *p, int R, float (&out)[C])
{
    if constexpr (W >= 2) {
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {
            const bool in = W == 3 || 4 * q < R;
            const float4 t = reinterpret_cast<const float4 *>(p)[in ? q : 0];
            out[4 * q] = in ? t.x : 0.0f;
            out[4 * q + 1] = in ? t.y : 0.0f;
            out[4 * q + 2] = in ? t.z : 0.0f;
            out[4 * q + 3] = in ? t.w : 0.0f;
        }
    } else if constexpr (W == 1) {
#pragma unroll
        for (int q = 0; q < C / 2; ++q) {
            const bool in = 2 * q < R;
            const float2 t = reinterpret_cast<const float2 *>(p)[in ? q : 0];
            out[2 * q] = in ? t.x : 0.0f;
            out[2 * q + 1] = in ? t.y : 0.0f;
        }
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const bool in = c < R;
            const float t = p[in ? c : 0];
            out[c] = in ? t : 0.0f;
        }
    }
}

template <int C, int W>
__device__ __forceinline__ void few_row(const uint16_t *p, int R, float (&out)[C])
{
    if constexpr (W >= 2) {
#pragma unroll
        for (int q = 0; q < C / 8; ++q) {
            const bool in = W == 3 || 8 * q < R;
            const uint4 t = reinterpret_cast<const uint4 *>(p)[in ? q : 0];
            const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                out[8 * q + 2 * h] = in ? __uint_as_float(w[h] << 16) : 0.0f;
                out[8 * q + 2 * h + 1] = in ? __uint_as_float(w[h] & 0xFFFF0000u) : 0.0f;
            }
        }
    } else if constexpr (W == 1) {
#pragma unroll
        for (int q = 0; q < C / 2; ++q) {
            const bool in = 2 * q < R;
            const uint32_t t = reinterpret_cast<const uint32_t *>(p)[in ? q : 0];
            out[2 * q] = in ? __uint_as_float(t << 16) : 0.0f;
            out[2 * q + 1] = in ? __uint_as_float(t & 0xFFFF0000u) : 0.0f;
        }
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const bool in = c < R;
            const uint16_t t = p[in ? c : 0];
            out[c] = in ? bf16_to_f32(t) : 0.0f;
        }
    }
}

// k = the elementwise product of the sample's other-mode factor rows
template <int C, int NM, bool BF16, int W, class Args>
__device__ __forceinline__ void few_k(const Args &a, const uint4 &rec, float (&k)[C])
{
    const uint32_t rw[3] = {rec.x, rec.y, rec.z};
    if (BF16)
        few_row<C, W>(a.gath16[0] + rw[0], a.R, k);
    else
        few_row<C, W>(a.gath[0] + rw[0], a.R, k);
#pragma unroll
    for (int mm = 1; mm < NM - 1; ++mm) {
        float f[C];
        if (BF16)
            few_row<C, W>(a.gath16[mm] + rw[mm], a.R, f);
        else
            few_row<C, W>(a.gath[mm] + rw[mm], a.R, f);
#pragma unroll
        for (int c = 0; c < C; ++c)
            k[c] *= f[c];
    }
}

// One level of the reduce-scatter over a 16-lane row: lane l keeps the upper
// half of its N values when `hi`, else the lower half, and adds the partner's
// copy of the half it keeps (the partner, l ^ mask with the bit of `hi`
// flipped, keeps the other half).
template <int CTRL, int N, int C>
__device__ __forceinline__ void few_rs(float (&r)[C], bool hi)
{
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
        const float keep = hi ? r[i + N / 2] : r[i];
        const float send = hi ? r[i] : r[i + N / 2];
        r[i] = keep + dpp_f32<CTRL>(send);
    }
}

// Column sums over the 16 lanes of the group: lane s gets columns
// (C / 16) s + j in r[j], j < C / 16 (partners l ^ 15, l ^ 7, l ^ 3, l ^ 1
// keep the column halves selected by bits 3, 2, 1, 0 of s).
template <int C>
__device__ __forceinline__ void few_colsum(float (&r)[C], int s)
{
    constexpr int kDppXor3 = 0x1B;  // quad_perm [3,2,1,0]
    few_rs<kDppMirror, C>(r, (s >> 3) & 1);
    few_rs<kDppHalfMirror, C / 2>(r, (s >> 2) & 1);
    few_rs<kDppXor3, C / 4>(r, (s >> 1) & 1);
    few_rs<kDppXor1, C / 8>(r, s & 1);
}

// LDS of one wave of the few-sample rows
struct FewShared {
    float4 gram[4 * 64];  // the four groups' G, column-major 16 x 16 each
    double2 u[4 * 8];     // each group's u, for the products by G
};

// Rows list[0 .. count) of one problem; this wave takes rows 4 blk .. 4 blk + 3.
template <int C, int NM, bool BF16, int W, bool NT, class Args>
__device__ __forceinline__ void few_rows(const Args &a, const RowItem *list, int count, int blk, FewShared &sh)
{
#pragma clang fp contract(off)
    constexpr int CL = C / 16;  // columns per lane after the reduce-scatter
    const int lane = threadIdx.x;
    const int grp = lane >> 4, s = lane & 15;
    const int id = blk * 4 + grp;
    const bool has = id < count;
    RowItem ri{0, 0, 0};
    if (has)
        ri = list[id];
    const int R = a.R;
    const int B = has ? static_cast<int>(minibatch_size(a.c, ri.n)) : 0;  // 1 .. 16
    // sample s: its record, or entry 0 of the records read and replaced by the zero record
    int64_t e = 0;
    if (s < B) {
        const Prp prp = make_prp(static_cast<uint32_t>(ri.n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, ri.row));
        e = ri.base + prp_index(prp, static_cast<uint32_t>(s));
    }
    const uint4 w = load_record4<NT>(a.records + e * 4);
    const uint4 rec = pick4(s < B, w, make_uint4(a.zrec[0], a.zrec[1], a.zrec[2], a.zrec[3]));
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const int64_t roff = static_cast<int64_t>(ri.row) * R;
    float y[C];
    few_row<C, W>(ysrc + roff, R, y);  // (BF16 W = 2 implies R % 4 == 0, W = 1 that R is even)
    float k[C];
    few_k<C, NM, BF16, W>(a, rec, k);

    // the residual of the sample, c_s = (K v_0)_s in FP64, and the Gram matrix
    const uint32_t xw[4] = {rec.x, rec.y, rec.z, rec.w};
    const float x = __uint_as_float(xw[NM - 1]);  // 0 for a missing sample
    float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    double c4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        p4[c & 3] = fmaf(k[c], y[c], p4[c & 3]);
        c4[c & 3] += static_cast<double>(k[c]);
    }
    const float res = ((p4[0] + p4[1]) + (p4[2] + p4[3])) - x;
    const double cs = ((c4[0] + c4[1]) + (c4[2] + c4[3])) * a.v0;
    f32x16 gacc;
#pragma unroll
    for (int v = 0; v < 16; ++v)
        gacc[v] = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (W == 3 || c < R)  // uniform
            gacc = __builtin_amdgcn_mfma_f32_16x16x1f32(k[c], k[c], gacc, 0, 0, 0);
    // register v of lane l holds block v / 4, row 4 (l / 16) + v % 4, column l % 16: four
    // consecutive rows of one column per block, stored column-major
#pragma unroll
    for (int b = 0; b < 4; ++b)
        sh.gram[b * 64 + (lane & 15) * 4 + (lane >> 4)] =
            make_float4(gacc[4 * b], gacc[4 * b + 1], gacc[4 * b + 2], gacc[4 * b + 3]);
    // the sampled gradient's column sums (FP32)
    float gk[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
        gk[c] = res * k[c];
    few_colsum<C>(gk, s);
    __builtin_amdgcn_wave_barrier();
    // row s of this group's G (column s: G is symmetric)
    double hd[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 t = sh.gram[grp * 64 + s * 4 + q];
        hd[4 * q] = static_cast<double>(t.x);
        hd[4 * q + 1] = static_cast<double>(t.y);
        hd[4 * q + 2] = static_cast<double>(t.z);
        hd[4 * q + 3] = static_cast<double>(t.w);
    }

    // the power method on (alpha, u), the decisions made exactly as in lp_estimate
    const double lam = a.lambda;
    const int T = a.power_iters;
    auto gmv = [&](double uu) {  // (G u)_s
        reinterpret_cast<double *>(sh.u)[16 * grp + s] = uu;
        __builtin_amdgcn_wave_barrier();
        const double2 *uv = sh.u + 8 * grp;
        double z4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double2 t = uv[q];
            z4[(2 * q) & 3] = fma(hd[2 * q], t.x, z4[(2 * q) & 3]);
            z4[(2 * q + 1) & 3] = fma(hd[2 * q + 1], t.y, z4[(2 * q + 1) & 3]);
        }
        __builtin_amdgcn_wave_barrier();
        return (z4[0] + z4[1]) + (z4[2] + z4[3]);
    };
    auto norm2 = [&](double al, double u, double z) {  // ||v||^2
        return al * al + row_sum_f64(u * (2.0 * al * cs + z));
    };
    double al = 1.0, u = 0.0, z = 0.0, vv = 1.0;
    double L = -1.0;  // set when the method ends early
    if (T > 0) {
        al = lam;  // v_1 = H v_0 = lambda v_0 + K^T c
        u = cs;
        z = gmv(u);
        double n2 = norm2(al, u, z);
        if (!(n2 > 0.0)) {
            L = 0.0;
        } else {
            const int e2 = ilogb(n2) >> 1;
            al = ldexp(al, -e2);
            u = ldexp(u, -e2);
            z = ldexp(z, -e2);
            if (T == 1) {
                vv = ldexp(n2, -2 * e2);
            } else {
                double rq_prev = 0.0;
                for (int t = 1; t < T; ++t) {
                    const double kv = al * cs + z;  // (K v_t)_s
                    if (!a.lp_bound && t >= 4 && (t & 1) == 0 && t + 1 < T) {
                        double s1 = kv * kv, s2 = u * (2.0 * al * cs + z);
                        row_sum2_f64(s1, s2);
                        const double nv = al * al + s2;
                        const double rq = (s1 + lam * nv) / nv;
                        if (t >= 6 && row_all(fabs(rq - rq_prev) <= kRqConverged * rq)) {
                            L = rq;
                            break;
                        }
                        rq_prev = rq;
                    }
                    al = ldexp(lam * al, -e2);
                    u = ldexp(kv + lam * u, -e2);
                    z = gmv(u);
                    if ((t & 31) == 0 && t + 1 < T) {
                        n2 = norm2(al, u, z);
                        if (!(n2 > 0.0)) {
                            L = 0.0;
                            break;
                        }
                        const int e3 = ilogb(n2) >> 1;
                        al = ldexp(al, -e3);
                        u = ldexp(u, -e3);
                        z = ldexp(z, -e3);
                    }
                }
                if (L < 0.0) {
                    n2 = norm2(al, u, z);
                    if (!(n2 > 0.0)) {
                        L = 0.0;
                    } else {
                        const int e4 = ilogb(n2) >> 1;
                        al = ldexp(al, -e4);
                        u = ldexp(u, -e4);
                        z = ldexp(z, -e4);
                        vv = ldexp(n2, -2 * e4);
                    }
                }
            }
        }
    }
    const double kv = al * cs + z;  // K v of the final iterate
    if (L < 0.0 && !a.lp_bound)
        L = (row_sum_f64(kv * kv) + lam * vv) / vv;
    const int c0 = CL * s;  // this lane's columns c0 .. c0 + CL - 1
    if (a.lp_bound) {
        // Collatz-Wielandt bound of the final iterate: v_i = alpha v0 + (K^T u)_i,
        // (H v)_i = (K^T K v)_i + lambda v_i, from the sample rows gathered again
        float kk[C];
        few_k<C, NM, BF16, W>(a, rec, kk);
        float xu[C], xk[C];
        const float uf = static_cast<float>(u), kvf = static_cast<float>(kv);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            xu[c] = kk[c] * uf;
            xk[c] = kk[c] * kvf;
        }
        few_colsum<C>(xu, s);
        few_colsum<C>(xk, s);
        double m = 0.0;
#pragma unroll
        for (int j = 0; j < CL; ++j) {
            const double vi = al * a.v0 + static_cast<double>(xu[j]);
            const double hv = static_cast<double>(xk[j]) + lam * vi;
            if (c0 + j < R && vi > 0.0)
                m = fmax(m, hv / vi);
        }
        if (L < 0.0)
            L = row_max_f64(m);
    }
    if (!has)
        return;
    const bool more = a.l + 1 < a.max_inner;
    const double sl = sqrt(L > 0.0 ? L : 0.0), sm = a.sqrt_lambda;
    const double beta = (sl - sm) / (sl + sm);
#pragma unroll
    for (int j = 0; j < CL; ++j) {
        const int col = c0 + j;
        if (col >= R)
            continue;
        const int64_t off = roff + col;
        const float yc = ysrc[off];
        const float a_prev = (a.l == 0) ? yc : a.A[off];
        if (L > 0.0) {
            const double g = static_cast<double>(gk[j]) + lam * static_cast<double>(yc);
            double an = static_cast<double>(yc) - g / L;
            an = an > 0.0 ? an : 0.0;
            const float af = static_cast<float>(an);
            a.A[off] = af;
            if (BF16)
                a.A16[off] = f32_to_bf16(af);
            if (more)
                a.Y[off] = static_cast<float>(an + beta * (an - static_cast<double>(a_prev)));
        } else if (more && a.l == 0) {
            a.Y[off] = yc;  // row skipped: Y_1 = Y_0
        }
    }
}

// ------------------------------------------------- rows with at most 4 samples, 16 to a wave
//
// R <= 16, N <= 4: quad q (lanes 4q .. 4q + 3) owns a row, lane s of the quad
// its sample s.  G = K K^T (4 x 4) comes from DPP broadcasts within the quad
// (G[s][t] = sum_c k_s[c] k_t[c], one fused multiply-add per column with
// lane t's value read through the DPP); the sampled gradient's column sums
// are a two-level reduce-scatter (lane s keeps columns 4s .. 4s + 3); the
// power method runs on (alpha, u), u in R^4, as in few_rows, its products by
// G through the same broadcasts.

template <int T>
__device__ __forceinline__ float quad_bcast_f32(float x)
{
    return dpp_f32<T * 0x55>(x);  // quad_perm [T,T,T,T]
}

template <int T>
__device__ __forceinline__ double quad_bcast_f64(double x)
{
    return dpp_f64<T * 0x55>(x);
}

__device__ __forceinline__ double quad_sum_f64(double x)
{
    x += dpp_f64<kDppXor1>(x);
    return x + dpp_f64<kDppXor2>(x);
}

__device__ __forceinline__ void quad_sum2_f64(double &x, double &y)
{
    double px = dpp_f64<kDppXor1>(x), py = dpp_f64<kDppXor1>(y);
    x += px;
    y += py;
    px = dpp_f64<kDppXor2>(x);
    py = dpp_f64<kDppXor2>(y);
    x += px;
    y += py;
}

__device__ __forceinline__ double quad_max_f64(double x)
{
    x = fmax(x, dpp_f64<kDppXor1>(x));
    return fmax(x, dpp_f64<kDppXor2>(x));
}

// True when d holds in every active lane of this lane's quad.
__device__ __forceinline__ bool quad_all(bool d)
{
    const unsigned long long m = __ballot(!d);
    return ((m >> (__lane_id() & 60)) & 0xFull) == 0;
}

// Column sums of 16 values over the quad: lane s gets columns 4s + j in r[j]
// (partners l ^ 3 and l ^ 1 keep the halves selected by bits 1 and 0 of s).
__device__ __forceinline__ void quad_colsum(float (&r)[16], int s)
{
    constexpr int kDppXor3 = 0x1B;  // quad_perm [3,2,1,0]
    few_rs<kDppXor3, 16>(r, (s >> 1) & 1);
    few_rs<kDppXor1, 8>(r, s & 1);
}

// Rows list[0 .. count) of one problem with at most 4 samples each; this wave
// takes rows 16 blk .. 16 blk + 15.
template <int NM, bool BF16, int W, bool NT, class Args>
__device__ __forceinline__ void quad_rows(const Args &a, const RowItem *list, int count, int blk)
{
#pragma clang fp contract(off)
    constexpr int C = 16;
    const int lane = threadIdx.x;
    const int grp = lane >> 2, s = lane & 3;
    const int id = blk * 16 + grp;
    const bool has = id < count;
    RowItem ri{0, 0, 0};
    if (has)
        ri = list[id];
    const int R = a.R;
    const int B = has ? static_cast<int>(minibatch_size(a.c, ri.n)) : 0;  // 1 .. 4
    int64_t e = 0;
    if (s < B) {
        const Prp prp = make_prp(static_cast<uint32_t>(ri.n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, ri.row));
        e = ri.base + prp_index(prp, static_cast<uint32_t>(s));
    }
    const uint4 w = load_record4<NT>(a.records + e * 4);
    const uint4 rec = pick4(s < B, w, make_uint4(a.zrec[0], a.zrec[1], a.zrec[2], a.zrec[3]));
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const int64_t roff = static_cast<int64_t>(ri.row) * R;
    float y[C];
    few_row<C, W>(ysrc + roff, R, y);
    float k[C];
    few_k<C, NM, BF16, W>(a, rec, k);

    const uint32_t xw[4] = {rec.x, rec.y, rec.z, rec.w};
    const float x = __uint_as_float(xw[NM - 1]);  // 0 for a missing sample
    float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    double c4[4] = {0.0, 0.0, 0.0, 0.0};
    float g4[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // row s of G
#pragma unroll
    for (int c = 0; c < C; ++c) {
        p4[c & 3] = fmaf(k[c], y[c], p4[c & 3]);
        c4[c & 3] += static_cast<double>(k[c]);
        g4[0] = fmaf(quad_bcast_f32<0>(k[c]), k[c], g4[0]);
        g4[1] = fmaf(quad_bcast_f32<1>(k[c]), k[c], g4[1]);
        g4[2] = fmaf(quad_bcast_f32<2>(k[c]), k[c], g4[2]);
        g4[3] = fmaf(quad_bcast_f32<3>(k[c]), k[c], g4[3]);
    }
    const float res = ((p4[0] + p4[1]) + (p4[2] + p4[3])) - x;
    const double cs = ((c4[0] + c4[1]) + (c4[2] + c4[3])) * a.v0;
    float gk[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
        gk[c] = res * k[c];
    quad_colsum(gk, s);
    const double hd[4] = {static_cast<double>(g4[0]), static_cast<double>(g4[1]), static_cast<double>(g4[2]),
                          static_cast<double>(g4[3])};

    const double lam = a.lambda;
    const int T = a.power_iters;
    auto gmv = [&](double uu) {  // (G u)_s
        const double z01 = fma(hd[0], quad_bcast_f64<0>(uu), hd[1] * quad_bcast_f64<1>(uu));
        const double z23 = fma(hd[2], quad_bcast_f64<2>(uu), hd[3] * quad_bcast_f64<3>(uu));
        return z01 + z23;
    };
    auto norm2 = [&](double al, double u, double z) {  // ||v||^2
        return al * al + quad_sum_f64(u * (2.0 * al * cs + z));
    };
    double al = 1.0, u = 0.0, z = 0.0, vv = 1.0;
    double L = -1.0;
    if (T > 0) {
        al = lam;
        u = cs;
        z = gmv(u);
        double n2 = norm2(al, u, z);
        if (!(n2 > 0.0)) {
            L = 0.0;
        } else {
            const int e2 = ilogb(n2) >> 1;
            al = ldexp(al, -e2);
            u = ldexp(u, -e2);
            z = ldexp(z, -e2);
            if (T == 1) {
                vv = ldexp(n2, -2 * e2);
            } else {
                double rq_prev = 0.0;
                for (int t = 1; t < T; ++t) {
                    const double kv = al * cs + z;
                    if (!a.lp_bound && t >= 4 && (t & 1) == 0 && t + 1 < T) {
                        double s1 = kv * kv, s2 = u * (2.0 * al * cs + z);
                        quad_sum2_f64(s1, s2);
                        const double nv = al * al + s2;
                        const double rq = (s1 + lam * nv) / nv;
                        if (t >= 6 && quad_all(fabs(rq - rq_prev) <= kRqConverged * rq)) {
                            L = rq;
                            break;
                        }
                        rq_prev = rq;
                    }
                    al = ldexp(lam * al, -e2);
                    u = ldexp(kv + lam * u, -e2);
                    z = gmv(u);
                    if ((t & 31) == 0 && t + 1 < T) {
                        n2 = norm2(al, u, z);
                        if (!(n2 > 0.0)) {
                            L = 0.0;
                            break;
                        }
                        const int e3 = ilogb(n2) >> 1;
                        al = ldexp(al, -e3);
                        u = ldexp(u, -e3);
                        z = ldexp(z, -e3);
                    }
                }
                if (L < 0.0) {
                    n2 = norm2(al, u, z);
                    if (!(n2 > 0.0)) {
                        L = 0.0;
                    } else {
                        const int e4 = ilogb(n2) >> 1;
                        al = ldexp(al, -e4);
                        u = ldexp(u, -e4);
                        z = ldexp(z, -e4);
                        vv = ldexp(n2, -2 * e4);
                    }
                }
            }
        }
    }
    const double kv = al * cs + z;
    if (L < 0.0 && !a.lp_bound)
        L = (quad_sum_f64(kv * kv) + lam * vv) / vv;
    const int c0 = 4 * s;  // this lane's columns c0 .. c0 + 3
    if (a.lp_bound) {
        float kk[C];
        few_k<C, NM, BF16, W>(a, rec, kk);
        float xu[C], xk[C];
        const float uf = static_cast<float>(u), kvf = static_cast<float>(kv);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            xu[c] = kk[c] * uf;
            xk[c] = kk[c] * kvf;
        }
        quad_colsum(xu, s);
        quad_colsum(xk, s);
        double m = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double vi = al * a.v0 + static_cast<double>(xu[j]);
            const double hv = static_cast<double>(xk[j]) + lam * vi;
            if (c0 + j < R && vi > 0.0)
                m = fmax(m, hv / vi);
        }
        if (L < 0.0)
            L = quad_max_f64(m);
    }
    if (!has)
        return;
    const bool more = a.l + 1 < a.max_inner;
    const double sl = sqrt(L > 0.0 ? L : 0.0), sm = a.sqrt_lambda;
    const double beta = (sl - sm) / (sl + sm);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = c0 + j;
        if (col >= R)
            continue;
        const int64_t off = roff + col;
        const float yc = ysrc[off];
        const float a_prev = (a.l == 0) ? yc : a.A[off];
        if (L > 0.0) {
            const double g = static_cast<double>(gk[j]) + lam * static_cast<double>(yc);
            double an = static_cast<double>(yc) - g / L;
            an = an > 0.0 ? an : 0.0;
            const float af = static_cast<float>(an);
            a.A[off] = af;
            if (BF16)
                a.A16[off] = f32_to_bf16(af);
            if (more)
                a.Y[off] = static_cast<float>(an + beta * (an - static_cast<double>(a_prev)));
        } else if (more && a.l == 0) {
            a.Y[off] = yc;  // row skipped: Y_1 = Y_0
        }
    }
}

}  // namespace
}  // namespace ntc
