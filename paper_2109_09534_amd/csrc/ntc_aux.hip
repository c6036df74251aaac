// Auxiliary kernels of libntc for gfx950: the FP64 loss of eq. (Problem_TC)
// with train/test RMSE, the default Philox initialisation, the BF16 shadow
// refresh and the device sampler probe.
#include <hip/hip_runtime.h>

#include "ntc_aux.h"
#include "ntc_bf16.h"
#include "ntc_rng.h"

namespace ntc {
namespace {

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

// Prediction sum_r prod_m U_m[i_m, r] in FP64 from row offsets off[m] = i_m * R.
template <bool VEC4>
__device__ __forceinline__ double cpd_predict(const LossArgs &a, const uint32_t *off, int nm, int R)
{
    double pred = 0.0;
    if (VEC4) {
        for (int r = 0; r < R; r += 4) {
            double p0 = 1.0, p1 = 1.0, p2 = 1.0, p3 = 1.0;
            for (int m = 0; m < nm; ++m) {
                const float4 u = *reinterpret_cast<const float4 *>(a.U[m] + off[m] + r);
                p0 *= static_cast<double>(u.x);
                p1 *= static_cast<double>(u.y);
                p2 *= static_cast<double>(u.z);
                p3 *= static_cast<double>(u.w);
            }
            pred += p0;
            pred += p1;
            pred += p2;
            pred += p3;
        }
    } else {
        for (int r = 0; r < R; ++r) {
            double prod = 1.0;
            for (int m = 0; m < nm; ++m)
                prod *= static_cast<double>(a.U[m][off[m] + r]);
            pred += prod;
        }
    }
    return pred;
}

// Training entries are walked in mode-0 CSR order; each record carries the
// other coordinates (times R) and the row (times R, in a spare record word or
// a side array), so an entry needs no search.  Fixed grid and per-thread
// order: the sums are deterministic.
template <bool VEC4>
__global__ __launch_bounds__(kLossThreads) void k_loss_partials(const LossArgs a)
{
    __shared__ double s[kLossThreads];
    const int R = a.R;
    const int nm = a.nmodes;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    double sse = 0.0;
    for (int64_t e = tid; e < a.nnz; e += stride) {
        const uint32_t *rec = a.records0 + e * a.rec_words;
        uint32_t off[kMaxModes];
        off[0] = a.row0 ? a.row0[e] : rec[a.row_word];
        for (int m = 1; m < nm; ++m)
            off[m] = rec[m - 1];
        const double pred = cpd_predict<VEC4>(a, off, nm, R);
        const double res = static_cast<double>(__uint_as_float(rec[nm - 1])) - pred;
        sse += res * res;
    }
    double tse = 0.0, tsx = 0.0;
    for (int64_t e = tid; e < a.n_test; e += stride) {
        const int32_t *cc = a.test_coords + e * nm;
        uint32_t off[kMaxModes];
        for (int m = 0; m < nm; ++m)
            off[m] = static_cast<uint32_t>(cc[m]) * static_cast<uint32_t>(R);
        const double pred = cpd_predict<VEC4>(a, off, nm, R);
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

// ---------------------------------------------------------- batched forms
typedef const __attribute__((address_space(4))) LossArgs CLossArgs;

// Held-out sums of many problems in one launch: block b belongs to entry
// owner[b] and is that entry's local block b - start[entry] of
// start[entry+1] - start[entry]; part[2b] = sum of squared test residuals,
// part[2b+1] = sum of squared test values over its strided share.
__global__ __launch_bounds__(kLossThreads) void k_test_partials_b(const LossArgs *__restrict__ args,
                                                                  const int32_t *__restrict__ start,
                                                                  const int32_t *__restrict__ owner, int32_t n,
                                                                  double *__restrict__ part)
{
    __shared__ double s[kLossThreads];
    const int j = n > 1 ? owner[blockIdx.x] : 0;
    const int b = static_cast<int>(blockIdx.x) - start[j];
    const int nb = start[j + 1] - start[j];
    CLossArgs &a = ((CLossArgs *)args)[j];
    const int R = a.R;
    const int nm = a.nmodes;
    double tse = 0.0, tsx = 0.0;
    for (int64_t e = static_cast<int64_t>(b) * blockDim.x + threadIdx.x; e < a.n_test;
         e += static_cast<int64_t>(nb) * blockDim.x) {
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
    tse = block_sum(tse, s);
    tsx = block_sum(tsx, s);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = tse;
        part[2 * blockIdx.x + 1] = tsx;
    }
}

// One block per entry: sum the entry's block partials in block order.
__global__ __launch_bounds__(kLossThreads) void k_test_final_b(const int32_t *__restrict__ start,
                                                               const double *__restrict__ part,
                                                               double *__restrict__ out)
{
    __shared__ double s[kLossThreads];
    const int j = blockIdx.x;
    for (int q = 0; q < 2; ++q) {
        double v = 0.0;
        for (int b = start[j] + threadIdx.x; b < start[j + 1]; b += blockDim.x)
            v += part[2 * b + q];
        v = block_sum(v, s);
        if (threadIdx.x == 0)
            out[2 * j + q] = v;
    }
}

__global__ void k_pool_rule(const PoolRuleArgs a)
{
    const int j = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= a.n)
        return;
    const int slot = a.slot[j];
    if (a.stop[slot] != 0)
        return;
    *a.kdev[j] += 1;
    const int64_t s = a.sweeps[slot] + 1;
    a.sweeps[slot] = s;
    bool stop = s >= a.max_sweeps;
    if (a.tidx[j] >= 0) {
        const double rmse = sqrt(a.test_out[2 * a.tidx[j]] / static_cast<double>(a.n_test[j]));
        const int W = a.window;
        double *h = a.hist + static_cast<int64_t>(slot) * (W + 1);
        const int64_t k = a.nhist[slot];  // this value is rmse after k sweeps
        h[k % (W + 1)] = rmse;
        a.nhist[slot] = k + 1;
        a.last[slot] = rmse;
        if (W > 0 && k >= W) {
            const double then = h[(k - W) % (W + 1)];
            stop = stop || !(then - rmse >= a.tol * rmse);
        }
    }
    if (stop)
        a.stop[slot] = 1;
}

}  // namespace

hipError_t launch_loss(const LossArgs &a, hipStream_t s)
{
    if (a.R % 4 == 0)
        hipLaunchKernelGGL(k_loss_partials<true>, dim3(kLossBlocks), dim3(kLossThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_loss_partials<false>, dim3(kLossBlocks), dim3(kLossThreads), 0, s, a);
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

int32_t test_blocks(int64_t n_test)
{
    const int64_t per = 16 * kLossThreads;
    const int64_t nb = (n_test + per - 1) / per;
    return static_cast<int32_t>(nb < 1 ? 1 : nb > 64 ? 64 : nb);
}

hipError_t launch_test_sums(const LossArgs *args, const int32_t *start, const int32_t *owner, int32_t n,
                            int32_t blocks, double *part, double *out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_test_partials_b, dim3(blocks), dim3(kLossThreads), 0, s, args, start, owner, n, part);
    hipLaunchKernelGGL(k_test_final_b, dim3(n), dim3(kLossThreads), 0, s, start, part, out);
    return hipGetLastError();
}

hipError_t launch_pool_rule(const PoolRuleArgs &a, hipStream_t s)
{
    if (a.n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pool_rule, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ntc
