// HIP kernels of libntc for gfx950 (wave64).
//
// Row kernel (Alg. 1, the body of the row loop): one 64-lane workgroup per
// work item.  The wave is split into G = 64/RP groups of RP lanes; lane r of
// a group owns column r of the rank dimension.  A batch of up to 64 samples
// is mapped one sample per lane for the sampler and the record fetch (one
// 16/32-byte record per lane), staged in LDS, then consumed G samples at a
// time: every group gathers its sample's N-1 factor rows (one contiguous
// 4R-byte segment per mode, or 2R bytes from the BF16 shadow), forms the
// Khatri-Rao row k (Hadamard product, increasing mode order), reduces k.y
// with shuffles inside the group, and accumulates g += (k.y - x) k in FP32
// and the row Hessian H += k k^T in FP64.  Groups are combined at the end of
// the item; a whole-row item then runs the FP64 power method for L_p and the
// fused step/projection/extrapolation; a split item writes its partial
// (g, H) and the finalize kernel combines the partials in slot order.
#include <hip/hip_runtime.h>

#include "ntc_internal.h"
#include "ntc_rng.h"

namespace ntc {
namespace {

__device__ __forceinline__ float bf16_to_f32(uint16_t b)
{
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// round-to-nearest-even FP32 -> BF16 (inputs are finite)
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
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

// Power method, step, projection and extrapolation for one row (Alg. 1,
// L_p, A_{l+1}, beta, Y_{l+1}).  Called by all 64 lanes; lanes r < RP of the
// first group hold g[r] (sampled gradient without ridge) and row r of the
// sampled H (without ridge); all other lanes pass zeros.
template <int RP, bool BF16>
__device__ void finish_row(const RowArgs &a, int row, int lane, double g, double (&h)[RP], float y, double *s_v)
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
    double v = live ? 1.0 / sqrt(static_cast<double>(R)) : 0.0;
    bool vanished = false;
    for (int t = 0; t < a.power_iters; ++t) {
        if (lane < RP)
            s_v[lane] = v;
        __syncthreads();
        double w = 0.0;
        if (lane < RP) {
#pragma unroll
            for (int q = 0; q < RP; ++q)
                w += h[q] * s_v[q];
        }
        __syncthreads();
        const double n2 = wave_sum(w * w);
        if (!(n2 > 0.0)) {
            vanished = true;
            break;
        }
        v = w / sqrt(n2);
    }
    double L = 0.0;
    if (!vanished) {
        if (lane < RP)
            s_v[lane] = v;
        __syncthreads();
        double w = 0.0;
        if (lane < RP) {
#pragma unroll
            for (int q = 0; q < RP; ++q)
                w += h[q] * s_v[q];
        }
        __syncthreads();
        L = wave_sum(v * w);
    }
    if (!live)
        return;
    const int64_t off = static_cast<int64_t>(row) * R + lane;
    const float a_prev = (a.l == 0) ? y : a.A[off];
    const bool more = a.l + 1 < a.max_inner;
    if (L > 0.0) {
        double an = static_cast<double>(y) - g / L;
        an = an > 0.0 ? an : 0.0;
        const double sl = sqrt(L), sm = sqrt(a.lambda);
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

template <int RP, int NM, bool BF16>
__global__ __launch_bounds__(64) void k_row_items(const RowArgs a)
{
    constexpr int G = 64 / RP;
    constexpr int RED = (G > 1) ? 64 * RP : 1;
    __shared__ uint32_t s_rec[64 * 8];
    __shared__ float s_k[64];
    __shared__ double s_red[RED];
    __shared__ double s_v[RP];
    __shared__ double s_g[64];

    const int nm = (NM > 0) ? NM : a.nmodes;
    const int rw = (NM > 0) ? ((NM <= 4) ? 4 : 8) : a.rec_words;
    const Item it = a.items[blockIdx.x];
    const int lane = threadIdx.x;
    const int r = lane % RP;
    const int grp = lane / RP;
    const int R = a.R;
    const bool rlive = r < R;

    const int64_t base = a.rowptr[it.row];
    const int64_t n = a.rowptr[it.row + 1] - base;
    const Prp prp = make_prp(static_cast<uint32_t>(n), sample_keys(a.seed, a.k, a.mode, a.l, it.row));
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
            const uint4 *src = reinterpret_cast<const uint4 *>(a.records + (base + q) * rw);
            const uint4 w0 = src[0];
            s_rec[lane * 8 + 0] = w0.x;
            s_rec[lane * 8 + 1] = w0.y;
            s_rec[lane * 8 + 2] = w0.z;
            s_rec[lane * 8 + 3] = w0.w;
            if (rw == 8) {
                const uint4 w1 = src[1];
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
                    const int64_t idx = s_rec[t * 8 + mm];
                    float f = 0.0f;
                    if (rlive) {
                        if (BF16)
                            f = bf16_to_f32(a.gath16[mm][idx * R + r]);
                        else
                            f = a.gath[mm][idx * R + r];
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
__global__ __launch_bounds__(64) void k_row_finalize(const RowArgs a)
{
    __shared__ double s_v[RP];
    const SplitRow sr = a.split[blockIdx.x];
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

// ------------------------------------------------------------------ loss
__device__ __forceinline__ double block_sum(double v, double *s)
{
    // fixed-shape tree: deterministic for a fixed blockDim
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (t < st)
            s[t] += s[t + st];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kLossThreads) void k_loss_partials(const LossArgs a)
{
    __shared__ double s[kLossThreads];
    const int R = a.R;
    const int nm = a.nmodes;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    // training entries, walked through the mode-0 CSR
    double sse = 0.0;
    for (int64_t e = tid; e < a.nnz; e += stride) {
        int64_t lo = 0, hi = a.I0;  // find p with rowptr[p] <= e < rowptr[p+1]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (a.rowptr0[mid] <= e)
                lo = mid;
            else
                hi = mid;
        }
        const uint32_t *rec = a.records0 + e * a.rec_words;
        double pred = 0.0;
        for (int r = 0; r < R; ++r) {
            double prod = static_cast<double>(a.U[0][lo * R + r]);
            for (int m = 1; m < nm; ++m)
                prod *= static_cast<double>(a.U[m][static_cast<int64_t>(rec[m - 1]) * R + r]);
            pred += prod;
        }
        const double res = static_cast<double>(__uint_as_float(rec[nm - 1])) - pred;
        sse += res * res;
    }
    double tse = 0.0, tsx = 0.0;
    for (int64_t e = tid; e < a.n_test; e += stride) {
        const int32_t *cc = a.test_coords + e * nm;
        double pred = 0.0;
        for (int r = 0; r < R; ++r) {
            double prod = 1.0;
            for (int m = 0; m < nm; ++m)
                prod *= static_cast<double>(a.U[m][static_cast<int64_t>(cc[m]) * R + r]);
            pred += prod;
        }
        const double x = static_cast<double>(a.test_values[e]);
        const double res = x - pred;
        tse += res * res;
        tsx += x * x;
    }
    double reg = 0.0;
    for (int m = 0; m < nm; ++m) {
        const int64_t cntm = a.dims[m] * R;
        for (int64_t t = tid; t < cntm; t += stride) {
            const double u = static_cast<double>(a.U[m][t]);
            reg += u * u;
        }
    }
    sse = block_sum(sse, s);
    tse = block_sum(tse, s);
    tsx = block_sum(tsx, s);
    reg = block_sum(reg, s);
    if (threadIdx.x == 0) {
        a.part[0 * kLossBlocks + blockIdx.x] = sse;
        a.part[1 * kLossBlocks + blockIdx.x] = tse;
        a.part[2 * kLossBlocks + blockIdx.x] = tsx;
        a.part[3 * kLossBlocks + blockIdx.x] = reg;
    }
}

__global__ __launch_bounds__(kLossThreads) void k_loss_final(const LossArgs a)
{
    __shared__ double s[kLossThreads];
    for (int q = 0; q < 4; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < kLossBlocks; b += blockDim.x)
            v += a.part[q * kLossBlocks + b];
        v = block_sum(v, s);
        if (threadIdx.x == 0)
            a.out[q] = v;
    }
}

// ------------------------------------------------------------- init, bf16
__global__ void k_init_factor(float *U, uint16_t *U16, int64_t count, int32_t mode, uint64_t seed, float scale)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= count)
        return;
    const uint64_t blk = static_cast<uint64_t>(t) >> 2;
    const U32x4 ctr = {{static_cast<uint32_t>(blk), static_cast<uint32_t>(blk >> 32), static_cast<uint32_t>(mode),
                        kTagInit}};
    const U32x4 o = philox4x32_10(ctr, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const float u = static_cast<float>(o.v[t & 3] >> 8) * 5.9604644775390625e-08f;  // 2^-24
    const float val = u * scale;
    U[t] = val;
    if (U16)
        U16[t] = f32_to_bf16(val);
}

__global__ void k_to_bf16(const float *U, uint16_t *U16, int64_t count)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < count)
        U16[t] = f32_to_bf16(U[t]);
}

__global__ void k_debug_sample(const int64_t *rowptr, int64_t row, uint64_t seed, int64_t k, int32_t mode,
                               int32_t l, double c, int32_t *pos, int32_t *count)
{
    const int64_t n = rowptr[row + 1] - rowptr[row];
    const int64_t b = minibatch_size(c, n);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *count = static_cast<int32_t>(b);
    if (b <= 0)
        return;
    const Prp prp = make_prp(static_cast<uint32_t>(n), sample_keys(seed, k, mode, l, row));
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < b;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x)
        pos[j] = static_cast<int32_t>(prp_index(prp, static_cast<uint32_t>(j)));
}

template <int RP, bool BF16>
hipError_t launch_items_rp(const RowArgs &a, hipStream_t s)
{
    if (a.nmodes == 3)
        hipLaunchKernelGGL((k_row_items<RP, 3, BF16>), dim3(a.n_items), dim3(64), 0, s, a);
    else if (a.nmodes == 4)
        hipLaunchKernelGGL((k_row_items<RP, 4, BF16>), dim3(a.n_items), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_row_items<RP, 0, BF16>), dim3(a.n_items), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <bool BF16>
hipError_t launch_items_b(const RowArgs &a, int rp, hipStream_t s)
{
    switch (rp) {
    case 8:
        return launch_items_rp<8, BF16>(a, s);
    case 16:
        return launch_items_rp<16, BF16>(a, s);
    case 32:
        return launch_items_rp<32, BF16>(a, s);
    case 64:
        return launch_items_rp<64, BF16>(a, s);
    default:
        return hipErrorInvalidValue;
    }
}

template <bool BF16>
hipError_t launch_final_b(const RowArgs &a, int rp, hipStream_t s)
{
    switch (rp) {
    case 8:
        hipLaunchKernelGGL((k_row_finalize<8, BF16>), dim3(a.n_split), dim3(64), 0, s, a);
        break;
    case 16:
        hipLaunchKernelGGL((k_row_finalize<16, BF16>), dim3(a.n_split), dim3(64), 0, s, a);
        break;
    case 32:
        hipLaunchKernelGGL((k_row_finalize<32, BF16>), dim3(a.n_split), dim3(64), 0, s, a);
        break;
    case 64:
        hipLaunchKernelGGL((k_row_finalize<64, BF16>), dim3(a.n_split), dim3(64), 0, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_row_items(const RowArgs &a, int rp, bool bf16, hipStream_t s)
{
    if (a.n_items <= 0)
        return hipSuccess;
    return bf16 ? launch_items_b<true>(a, rp, s) : launch_items_b<false>(a, rp, s);
}

hipError_t launch_row_finalize(const RowArgs &a, int rp, bool bf16, hipStream_t s)
{
    if (a.n_split <= 0)
        return hipSuccess;
    return bf16 ? launch_final_b<true>(a, rp, s) : launch_final_b<false>(a, rp, s);
}

hipError_t launch_loss(const LossArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_loss_partials, dim3(kLossBlocks), dim3(kLossThreads), 0, s, a);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kLossThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init_factor(float *U, uint16_t *U16, int64_t count, int32_t mode, uint64_t seed, float scale,
                              hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_init_factor, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, U, U16, count, mode, seed,
                       scale);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *U, uint16_t *U16, int64_t count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_to_bf16, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, U, U16, count);
    return hipGetLastError();
}

hipError_t launch_debug_sample(const int64_t *rowptr, int64_t row, uint64_t seed, int64_t k, int32_t mode,
                               int32_t l, double c, int32_t *pos_out, int32_t *count_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_sample, dim3(64), dim3(256), 0, s, rowptr, row, seed, k, mode, l, c, pos_out,
                       count_out);
    return hipGetLastError();
}

}  // namespace ntc
