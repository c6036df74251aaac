// Internal view of a problem handle, for the batching pool.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "ntc.h"
#include "ntc_internal.h"

namespace ntc {

// Record `msg` as the calling thread's last error and return `s`.
ntc_status set_error(ntc_status s, const std::string &msg);

// What the pool needs to launch a problem's row kernels inside a batch.
struct ProblemView {
    KernelClass kc;
    int32_t nmodes;
    int32_t rank;
    int32_t max_inner;
    const RowArgs *args_host;      // [nmodes * max_inner]: row-kernel arguments of (mode, inner step)
    int64_t *kdev;                 // device sweep counter read by the row kernels
    int32_t blocks[kMaxModes][kRowKernels];  // grid blocks per mode and RowKernel kind
    const float *U[kMaxModes];     // device factors
    int64_t n_test;                // held-out set on the device
    const int32_t *test_coords;
    const float *test_values;
    size_t bytes;                  // device bytes the handle holds
    int64_t k;                     // host sweep counter
    int64_t updates_per_sweep;
};

ntc_status problem_view(ntc_handle h, ProblemView *v);

// The pool advanced the device sweep counter by n: keep the host copy in step.
void note_sweeps(ntc_handle h, int64_t n);

// Upper bound of the temporary device bytes ntc_create_device_csr takes (and
// frees before it returns) for a problem of these sizes, allocations
// rounded up to 256 bytes.
ntc_status device_csr_temp_bytes(int32_t nmodes, const int64_t *dims, int64_t nnz, size_t *bytes);

}  // namespace ntc
