// Auxiliary kernels of libntc for gfx950: the FP64 loss of eq. (Problem_TC)
// with train/test RMSE, the default Philox initialisation, the BF16 shadow
// refresh and the device sampler probe.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ntc_aux.h"
#include "ntc_bf16.h"
#include "ntc_dev.h"
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

// The predictions sum_r prod_m U_m[i_m, r] of UN entries in FP64, from row
// offsets off[u][m] = i_m * R, by the G lanes of their group (this lane is
// q): each lane multiplies out its columns, then the group sums by DPP.
// The UN entries' row loads are independent, so they are in flight
// together.  Every lane of the group gets the same sums.  NM > 0 fixes the
// number of modes at compile time; NM = 0 takes nm.
template <int UN, int NM, class A>
__device__ __forceinline__ void group_predict(const A &a, const uint32_t (&off)[UN][kMaxModes], int nm, int R,
                                              int G, int q, double (&pred)[UN])
{
    constexpr int MM = NM > 0 ? NM : kMaxModes;
#pragma unroll
    for (int u = 0; u < UN; ++u)
        pred[u] = 0.0;
    if (R % 4 == 0) {
        for (int c = 4 * q; c < R; c += 4 * G) {
            double p[UN][4];
#pragma unroll
            for (int m = 0; m < MM; ++m) {
                if (NM == 0 && m >= nm)
                    break;
                float4 v[UN];
#pragma unroll
                for (int u = 0; u < UN; ++u)
                    v[u] = *reinterpret_cast<const float4 *>(a.U[m] + off[u][m] + c);
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    const double x0 = v[u].x, x1 = v[u].y, x2 = v[u].z, x3 = v[u].w;
                    p[u][0] = m == 0 ? x0 : p[u][0] * x0;
                    p[u][1] = m == 0 ? x1 : p[u][1] * x1;
                    p[u][2] = m == 0 ? x2 : p[u][2] * x2;
                    p[u][3] = m == 0 ? x3 : p[u][3] * x3;
                }
            }
#pragma unroll
            for (int u = 0; u < UN; ++u)
                pred[u] += (p[u][0] + p[u][1]) + (p[u][2] + p[u][3]);
        }
    } else {
        for (int c = q; c < R; c += 16) {
            double p[UN];
#pragma unroll
            for (int m = 0; m < MM; ++m) {
                if (NM == 0 && m >= nm)
                    break;
                float v[UN];
#pragma unroll
                for (int u = 0; u < UN; ++u)
                    v[u] = a.U[m][off[u][m] + c];
#pragma unroll
                for (int u = 0; u < UN; ++u)
                    p[u] = m == 0 ? static_cast<double>(v[u]) : p[u] * static_cast<double>(v[u]);
            }
#pragma unroll
            for (int u = 0; u < UN; ++u)
                pred[u] += p[u];
        }
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
        double acc = pred[u];
        if (G >= 2)
            acc += dpp_f64<kDppXor1>(acc);
        if (G >= 4)
            acc += dpp_f64<kDppXor2>(acc);
        if (G >= 8)
            acc += dpp_f64<kDppHalfMirror>(acc);
        if (G >= 16)
            acc += dpp_f64<kDppMirror>(acc);
        pred[u] = acc;
    }
}

// Held-out sums over entries grp, grp + ngroups, ... of a test set, UN
// entries per group step; an index past the end repeats the step's first
// entry and is not counted.  The group's first lane keeps the sums.
template <int UN, int NM, class A>
__device__ __forceinline__ void test_sums(const A &a, int64_t grp, int64_t ngroups, int nm, int R, int G, int q,
                                          double &tse, double &tsx)
{
    for (int64_t e0 = grp; e0 < a.n_test; e0 += UN * ngroups) {
        uint32_t off[UN][kMaxModes];
        float x[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t e = e0 + u * ngroups < a.n_test ? e0 + u * ngroups : e0;
            const int32_t *cc = a.test_coords + e * nm;
#pragma unroll
            for (int m = 0; m < (NM > 0 ? NM : kMaxModes); ++m)
                off[u][m] = (NM > 0 || m < nm) ? static_cast<uint32_t>(cc[m]) * static_cast<uint32_t>(R) : 0u;
            x[u] = a.test_values[e];
        }
        double pred[UN];
        group_predict<UN, NM>(a, off, nm, R, G, q, pred);
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const double xv = static_cast<double>(x[u]);
            const double res = xv - pred[u];
            if (q == 0 && e0 + u * ngroups < a.n_test) {
                tse += res * res;
                tsx += xv * xv;
            }
        }
    }
}

// Training entries are walked in mode-0 CSR order; each record carries the
// other coordinates (times R) and the row (times R, in a spare record word or
// a side array), so an entry needs no search.  A group of lanes takes UN
// entries at a time (entry_lanes); the group's first lane keeps the sums.
// Fixed grid and per-thread order: the sums are deterministic.
template <int NM>
__global__ __launch_bounds__(kLossThreads) void k_loss_partials(const LossArgs a)
{
    constexpr int UN = 4;
    __shared__ double s[kLossThreads];
    const int R = a.R;
    const int nm = NM > 0 ? NM : a.nmodes;
    const int G = entry_lanes(R);
    const int q = threadIdx.x & (G - 1);
    const int64_t ngroups = static_cast<int64_t>(gridDim.x) * (blockDim.x / G);
    const int64_t grp = static_cast<int64_t>(blockIdx.x) * (blockDim.x / G) + threadIdx.x / G;
    double sse = 0.0;
    for (int64_t e0 = grp; e0 < a.nnz; e0 += UN * ngroups) {
        uint32_t off[UN][kMaxModes];
        float x[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t e = e0 + u * ngroups < a.nnz ? e0 + u * ngroups : e0;
            const uint32_t *rec = a.records0 + e * a.rec_words;
            off[u][0] = a.row0 ? a.row0[e] : rec[a.row_word];
#pragma unroll
            for (int m = 1; m < (NM > 0 ? NM : kMaxModes); ++m)
                off[u][m] = (NM > 0 || m < nm) ? rec[m - 1] : 0u;
            x[u] = __uint_as_float(rec[nm - 1]);
        }
        double pred[UN];
        group_predict<UN, NM>(a, off, nm, R, G, q, pred);
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const double res = static_cast<double>(x[u]) - pred[u];
            if (q == 0 && e0 + u * ngroups < a.nnz)
                sse += res * res;
        }
    }
    double tse = 0.0, tsx = 0.0;
    test_sums<UN, NM>(a, grp, ngroups, nm, R, G, q, tse, tsx);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
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

// ---------------------------------------------------- allocation-free loss
// Sums over two caller-held COO sets (train, held-out) and the regulariser,
// one partial per block: part[q * gridDim.x + block] for q = train SSE,
// held-out SSE, held-out sum x^2, sum U^2.
template <int NM>
__global__ __launch_bounds__(kLossThreads) void k_coo_partials(const LossArgs tr, const LossArgs te, double *part)
{
    __shared__ double s[kLossThreads];
    const int R = tr.R;
    const int nm = NM > 0 ? NM : tr.nmodes;
    const int G = entry_lanes(R);
    const int q = threadIdx.x & (G - 1);
    const int64_t ngroups = static_cast<int64_t>(gridDim.x) * (blockDim.x / G);
    const int64_t grp = static_cast<int64_t>(blockIdx.x) * (blockDim.x / G) + threadIdx.x / G;
    double sse = 0.0, sx_train = 0.0, tse = 0.0, tsx = 0.0;
    test_sums<4, NM>(tr, grp, ngroups, nm, R, G, q, sse, sx_train);
    test_sums<4, NM>(te, grp, ngroups, nm, R, G, q, tse, tsx);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    double reg = 0.0;
    for (int m = 0; m < nm; ++m) {
        const int64_t cntm = tr.dims[m] * R;
        for (int64_t t = tid; t < cntm; t += stride) {
            const double u = static_cast<double>(tr.U[m][t]);
            reg += u * u;
        }
    }
    sse = block_sum(sse, s);
    tse = block_sum(tse, s);
    tsx = block_sum(tsx, s);
    reg = block_sum(reg, s);
    if (threadIdx.x == 0) {
        const int nb = gridDim.x;
        part[0 * nb + blockIdx.x] = sse;
        part[1 * nb + blockIdx.x] = tse;
        part[2 * nb + blockIdx.x] = tsx;
        part[3 * nb + blockIdx.x] = reg;
    }
}

// The nb block partials summed in block order, then the four results of
// ntc_loss, written to the caller's device memory.
__global__ __launch_bounds__(kLossThreads) void k_coo_final(const double *part, int nb, int64_t n_train,
                                                            int64_t n_test, double lambda, double *out)
{
    __shared__ double s[kLossThreads];
    double v[4];
    for (int q = 0; q < 4; ++q) {
        double x = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            x += part[q * nb + b];
        v[q] = block_sum(x, s);
    }
    if (threadIdx.x == 0) {
        out[0] = 0.5 * v[0] + 0.5 * lambda * v[3];
        out[1] = n_train > 0 ? sqrt(v[0] / static_cast<double>(n_train)) : 0.0;
        out[2] = n_test > 0 ? sqrt(v[1] / static_cast<double>(n_test)) : 0.0;
        out[3] = (n_test > 0 && v[2] > 0.0) ? sqrt(v[1]) / sqrt(v[2]) : 0.0;
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
    const int G = entry_lanes(R);  // uniform over the block: it belongs to one entry
    const int q = threadIdx.x & (G - 1);
    const int per = blockDim.x / G;
    double tse = 0.0, tsx = 0.0;
    test_sums<2, 0>(a, static_cast<int64_t>(b) * per + threadIdx.x / G, static_cast<int64_t>(nb) * per, nm, R, G, q,
                    tse, tsx);
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
    if (a.nmodes == 3)
        hipLaunchKernelGGL(k_loss_partials<3>, dim3(kLossBlocks), dim3(kLossThreads), 0, s, a);
    else if (a.nmodes == 4)
        hipLaunchKernelGGL(k_loss_partials<4>, dim3(kLossBlocks), dim3(kLossThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_loss_partials<0>, dim3(kLossBlocks), dim3(kLossThreads), 0, s, a);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kLossThreads), 0, s, a);
    return hipGetLastError();
}

// The partial sums of launch_loss_coo_noalloc.  Host code never uses this
// name as an address: each device's copy is reached through the pointer
// hipGetSymbolAddress returns for it, taken once per device.
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The address of this device's copy of `scratch`, looked up on the first
// call made with the device current.
hipError_t scratch_ptr(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

hipError_t launch_loss_coo_noalloc(const LossArgs &train, const LossArgs &test, double lambda, double *out,
                                   hipStream_t s)
{
    double *part = nullptr;
    hipError_t e = scratch_ptr(&part);
    if (e != hipSuccess)
        return e;
    // about eight group-steps of four entries per thread over both sets
    const int64_t per = 8 * 4 * (kLossThreads / entry_lanes(train.R));
    const int64_t total = train.n_test + test.n_test;
    int64_t nb = (total + per - 1) / per;
    nb = nb < 1 ? 1 : nb > kNoallocBlocks ? kNoallocBlocks : nb;
    if (4 * nb > kNoallocScratchDoubles)
        return hipErrorInvalidValue;
    const dim3 grid(static_cast<uint32_t>(nb)), block(kLossThreads);
    if (train.nmodes == 3)
        hipLaunchKernelGGL(k_coo_partials<3>, grid, block, 0, s, train, test, part);
    else if (train.nmodes == 4)
        hipLaunchKernelGGL(k_coo_partials<4>, grid, block, 0, s, train, test, part);
    else
        hipLaunchKernelGGL(k_coo_partials<0>, grid, block, 0, s, train, test, part);
    hipLaunchKernelGGL(k_coo_final, dim3(1), block, 0, s, static_cast<const double *>(part), static_cast<int>(nb),
                       train.n_test, test.n_test, lambda, out);
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

int32_t test_blocks(int64_t n_test, int32_t rank)
{
    // about eight group-steps per thread, at most kMaxTestBlocks blocks
    const int64_t per = 8 * (kLossThreads / entry_lanes(rank));
    const int64_t nb = (n_test + per - 1) / per;
    return static_cast<int32_t>(nb < 1 ? 1 : nb > kMaxTestBlocks ? kMaxTestBlocks : nb);
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
