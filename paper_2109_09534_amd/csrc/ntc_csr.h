// Device-side CSR build (ntc_create_device_csr): interfaces of ntc_csr.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntc_internal.h"

namespace ntc {

struct CsrDims {
    int64_t d[kMaxModes];
};

// One mode's build: device COO in, sorted keys and ids, rowptr [I+1],
// records [nnz][rw] (and row0 [nnz] when given) out.  temp: temp_bytes of
// scratch for the radix sort (csr_sort_bytes).
struct CsrMode {
    const int32_t *coords;
    const float *values;
    int64_t nnz;
    int32_t nmodes;
    int32_t mode;
    int64_t I;
    int32_t rw;
    uint32_t R;
    int32_t own_word;
    uint32_t *keys_in, *keys_out, *ids_in, *ids_out;
    void *temp;
    size_t temp_bytes;
    int64_t *rowptr;
    uint32_t *records;
    uint32_t *row0;
};

hipError_t csr_validate(const int32_t *coords, const float *values, int64_t nnz, int32_t nmodes,
                        const CsrDims &dims, unsigned long long *first_bad, hipStream_t s);
hipError_t csr_sort_bytes(int64_t nnz, size_t *bytes);
hipError_t csr_mode(const CsrMode &c, hipStream_t s);

}  // namespace ntc
