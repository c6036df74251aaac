// Device-side interfaces of the auxiliary kernels (loss, init, BF16 refresh,
// sampler probe).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntc_internal.h"

namespace ntc {

struct LossArgs {
    const uint32_t *records0;     // CSR records of mode 0 (coordinates * R)
    const uint32_t *row0;         // [nnz] row * R of every mode-0 record, or null
    int32_t row_word;             // record word holding row * R when row0 is null
    int64_t nnz;
    const int32_t *test_coords;
    const float *test_values;
    int64_t n_test;
    const float *U[kMaxModes];
    int64_t dims[kMaxModes];
    int32_t nmodes;
    int32_t rec_words;
    int32_t R;
    double *part;                 // [4][kLossBlocks]: train SSE, test SSE, test sum x^2, sum U^2
    double *out;                  // [4]
};

constexpr int kLossBlocks = 2048;  // 32 waves per CU: enough loads in flight
constexpr int kLossThreads = 256;
constexpr int kMaxTestBlocks = 1024;  // held-out blocks per problem in a pool launch

// Lanes that share one entry in the training and held-out sums.  With
// R % 4 == 0 a lane reads four consecutive columns of each factor row as one
// 16-byte load, and the group is the power of two >= R / 4 (at most 16);
// otherwise 16 lanes read one column each.  A group is aligned within a
// 16-lane DPP row, so it reads each factor row as one coalesced access.
__host__ __device__ inline int entry_lanes(int R)
{
    if (R % 4 != 0)
        return 16;
    int g = 1;
    while (g < 16 && 4 * g < R)
        g <<= 1;
    return g;
}

hipError_t launch_loss(const LossArgs &a, hipStream_t s);

// The loss of launch_loss over two COO sets held by the caller (train and
// held-out: test_coords/test_values/n_test of each LossArgs), with the
// partial sums in a fixed device array of kNoallocBlocks * 4 doubles (one
// per GPU, never freed) instead of an allocation: no hipMalloc, no memset,
// no copy and no synchronisation, so a caller may capture it in a graph.
// out (device, 4 doubles) receives {objective, train RMSE, test RMSE, test
// relative error}.  Calls that overlap on one GPU race on the array.
constexpr int kNoallocBlocks = 1024;
constexpr int64_t kNoallocScratchDoubles = 4 * static_cast<int64_t>(kNoallocBlocks);
hipError_t launch_loss_coo_noalloc(const LossArgs &train, const LossArgs &test, double lambda, double *out,
                                   hipStream_t s);
hipError_t launch_init_factor(float *U, uint16_t *U16, int64_t count, int32_t mode, uint64_t seed, float scale,
                              hipStream_t s);
hipError_t launch_to_bf16(const float *U, uint16_t *U16, int64_t count, hipStream_t s);
hipError_t launch_debug_sample(const int64_t *rowptr, int64_t row, uint64_t seed, int64_t k, int32_t mode,
                               int32_t l, double c, int32_t *pos_out, int32_t *count_out, hipStream_t s);

// Batched held-out sums (the pool's stop rule): entry j owns blocks
// [start[j], start[j+1]) (start has n+1 entries, owner one per block; owner
// may be null when n == 1); out[2j] = sum of squared test residuals,
// out[2j+1] = sum of squared test values.  part holds 2 doubles per block.
int32_t test_blocks(int64_t n_test, int32_t rank);
hipError_t launch_test_sums(const LossArgs *args, const int32_t *start, const int32_t *owner, int32_t n,
                            int32_t blocks, double *part, double *out, hipStream_t s);
// End of a pool sweep, per running problem j (device state indexed by slot):
// unless it has already stopped, advance its sweep counters, record the
// held-out RMSE of this sweep (test entry tidx[j] >= 0) and apply the stop
// rule: stop after sweep s >= window when rmse(s - window) - rmse(s) <
// tol * rmse(s), or when s >= max_sweeps.
struct PoolRuleArgs {
    int32_t n;                   // running problems
    const int32_t *slot;         // [n] slot of each
    int64_t *const *kdev;        // [n] the problems' sampler counters
    const int32_t *tidx;         // [n] index into test_out, or -1 (no held-out set)
    const int64_t *n_test;       // [n] held-out entries
    const double *test_out;      // [2 * test entries] held-out sums of this sweep
    int32_t *stop;               // [slots]
    int64_t *sweeps;             // [slots]
    int64_t *nhist;              // [slots] RMSE values recorded so far (the first at admission)
    double *hist;                // [slots][window + 1] ring of recent RMSE values
    double *last;                // [slots] most recent RMSE
    int32_t window;
    int32_t max_sweeps;
    double tol;
};
hipError_t launch_pool_rule(const PoolRuleArgs &a, hipStream_t s);

}  // namespace ntc
