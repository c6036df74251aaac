// Device-side CSR build of libntc (ntc_create_device_csr): the same
// mode-sorted records and row pointers as the host build, made on the GPU.
//
// Per mode m the entries are sorted by i_m with a stable radix sort (keys
// i_m, values the COO entry ids), so ties keep COO order exactly as the
// host's counting sort does; the row pointers are the lower bounds of
// 0 .. I_m in the sorted keys, and the records are gathered from the COO
// through the sorted ids.  Every step is deterministic.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "ntc_csr.h"

namespace ntc {
namespace {

// First entry whose coordinate is out of range or whose value is not finite
// (atomic minimum of the entry index; vector atomics only).
__global__ void k_validate(const int32_t *coords, const float *values, int64_t nnz, int32_t nmodes,
                           CsrDims dims, unsigned long long *first_bad)
{
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < nnz;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        bool bad = !isfinite(values[e]);
        for (int m = 0; m < nmodes; ++m) {
            const int32_t x = coords[e * nmodes + m];
            bad = bad || x < 0 || static_cast<int64_t>(x) >= dims.d[m];
        }
        if (bad)
            atomicMin(first_bad, static_cast<unsigned long long>(e));
    }
}

__global__ void k_keys(const int32_t *coords, int64_t nnz, int32_t nmodes, int32_t mode, uint32_t *keys,
                       uint32_t *ids)
{
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < nnz;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        keys[e] = static_cast<uint32_t>(coords[e * nmodes + mode]);
        ids[e] = static_cast<uint32_t>(e);
    }
}

// rowptr[i] = number of sorted keys below i, for i in [0, I]
__global__ void k_rowptr(const uint32_t *keys, int64_t nnz, int64_t I, int64_t *rowptr)
{
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i <= I;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int64_t lo = 0, hi = nnz;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (static_cast<int64_t>(keys[mid]) < i)
                lo = mid + 1;
            else
                hi = mid;
        }
        rowptr[i] = lo;
    }
}

// records[pos] = other-mode coordinates times R (increasing mode order), the
// value bits, zeros, and (own_word >= 0) the entry's own coordinate times R;
// row0[pos] = own coordinate times R when row0 is given
__global__ void k_records(const int32_t *coords, const float *values, const uint32_t *ids, int64_t nnz,
                          int32_t nmodes, int32_t mode, int32_t rw, uint32_t R, int32_t own_word, uint32_t *records,
                          uint32_t *row0)
{
    for (int64_t pos = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; pos < nnz;
         pos += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t e = ids[pos];
        const int32_t *ce = coords + e * nmodes;
        uint32_t *rec = records + pos * rw;
        int w = 0;
        for (int m = 0; m < nmodes; ++m)
            if (m != mode)
                rec[w++] = static_cast<uint32_t>(ce[m]) * R;
        rec[w++] = __float_as_uint(values[e]);
        for (; w < rw; ++w)
            rec[w] = 0u;
        const uint32_t own = static_cast<uint32_t>(ce[mode]) * R;
        if (own_word >= 0)
            rec[own_word] = own;
        if (row0)
            row0[pos] = own;
    }
}

int grid_for(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return static_cast<int>(b < 1 ? 1 : b > 65536 ? 65536 : b);
}

}  // namespace

hipError_t csr_validate(const int32_t *coords, const float *values, int64_t nnz, int32_t nmodes,
                        const CsrDims &dims, unsigned long long *first_bad, hipStream_t s)
{
    if (nnz <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3(grid_for(nnz)), dim3(256), 0, s, coords, values, nnz, nmodes, dims,
                       first_bad);
    return hipGetLastError();
}

hipError_t csr_sort_bytes(int64_t nnz, size_t *bytes)
{
    *bytes = 0;
    return rocprim::radix_sort_pairs(nullptr, *bytes, static_cast<const uint32_t *>(nullptr),
                                     static_cast<uint32_t *>(nullptr), static_cast<const uint32_t *>(nullptr),
                                     static_cast<uint32_t *>(nullptr), static_cast<size_t>(nnz), 0, 32);
}

hipError_t csr_mode(const CsrMode &c, hipStream_t s)
{
    if (c.nnz > 0) {
        hipLaunchKernelGGL(k_keys, dim3(grid_for(c.nnz)), dim3(256), 0, s, c.coords, c.nnz, c.nmodes, c.mode,
                           c.keys_in, c.ids_in);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        unsigned bits = 1;
        while (bits < 32 && (static_cast<uint64_t>(1) << bits) < static_cast<uint64_t>(c.I))
            ++bits;
        size_t bytes = c.temp_bytes;
        e = rocprim::radix_sort_pairs(c.temp, bytes, c.keys_in, c.keys_out, c.ids_in, c.ids_out,
                                      static_cast<size_t>(c.nnz), 0, bits, s);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_rowptr, dim3(grid_for(c.I + 1)), dim3(256), 0, s, c.keys_out, c.nnz, c.I, c.rowptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || c.nnz <= 0)
        return e;
    hipLaunchKernelGGL(k_records, dim3(grid_for(c.nnz)), dim3(256), 0, s, c.coords, c.values, c.ids_out, c.nnz,
                       c.nmodes, c.mode, c.rw, c.R, c.own_word, c.records, c.row0);
    return hipGetLastError();
}

}  // namespace ntc
