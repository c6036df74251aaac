// Internal view of a problem handle, for the batching pool.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

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

// A ROCTX range over one host API call, shown by rocprofv3's marker trace
// beside the kernels the call enqueued (a no-op with no profiler attached).
// `name` must outlive the call.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Range names of the modes of a sweep.
inline const char *mode_range_name(int mode)
{
    static const char *const names[kMaxModes] = {"ntc mode 0", "ntc mode 1", "ntc mode 2", "ntc mode 3",
                                                 "ntc mode 4", "ntc mode 5", "ntc mode 6", "ntc mode 7"};
    return names[mode];
}

// Upper bound of the temporary device bytes ntc_create_device_csr takes (and
// frees before it returns) for a problem of these sizes, allocations
// rounded up to 256 bytes.
ntc_status device_csr_temp_bytes(int32_t nmodes, const int64_t *dims, int64_t nnz, size_t *bytes);

}  // namespace ntc
