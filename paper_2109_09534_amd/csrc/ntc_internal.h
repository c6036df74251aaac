// Internal types of libntc shared by the host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ntc {

constexpr int kMaxModes = 8;
constexpr int kMaxRank = 64;

// One unit of row work: samples [j0, j1) of the row's minibatch.  slot < 0:
// the item covers the whole minibatch and finishes the row itself; slot >= 0:
// it writes its partial (g, H) to partial slot `slot` and a finalize pass
// combines the row's slots in slot order.
struct Item {
    int32_t row;
    int32_t j0;
    int32_t j1;
    int32_t slot;
};

// A row whose minibatch is split over `nslots` consecutive partial slots.
struct SplitRow {
    int32_t row;
    int32_t slot0;
    int32_t nslots;
    int32_t pad;
};

// Arguments of the row kernels for one (mode, inner step).
struct RowArgs {
    const int64_t *rowptr;        // [I+1] CSR of this mode
    const uint32_t *records;      // [nnz][rec_words]: other-mode coordinates * R (increasing mode), value bits
    const Item *items;
    const SplitRow *split;
    const int32_t *tiny;          // rows whose minibatch has 1..kTinyB samples (R <= 16 kernels)
    const float *gath[kMaxModes - 1];     // other modes' FP32 factors, increasing mode order
    const uint16_t *gath16[kMaxModes - 1];// their BF16 shadows (precision form)
    float *A;                     // this mode's factor (A_l in, A_{l+1} out, in place)
    float *Y;                     // extrapolated iterate buffer (MAX_INNER > 1)
    uint16_t *A16;                // this mode's BF16 shadow (or null)
    double *partials;             // [slots][RP + RP*RP]
    uint32_t zrec[8];             // record of a missing sample: the all-zero row (index I_m) of each
                                  // other mode, value 0
    uint64_t seed;
    int64_t k;
    double lambda;
    double c;
    int32_t mode;
    int32_t l;
    int32_t nmodes;
    int32_t rec_words;
    int32_t R;
    int32_t max_inner;
    int32_t power_iters;
    int32_t n_items;
    int32_t n_partial;            // (wave-per-item kernels) items [0, n_partial) write partial slots
    int32_t n_group;              // (R <= 16) items [0, n_group) are whole rows for the group kernel,
                                  // items [n_group, n_items) row chunks for the block kernel
    int32_t n_split;
    int32_t n_tiny;
};

// Rows whose minibatch has at most this many samples run one row per lane.
constexpr int kTinyB = 4;


// R <= 16: whole rows one per 16-lane group (5 <= N <= 8: also every chunk)
// R > 16: every item, one per wave
hipError_t launch_row_items(const RowArgs &a, int rp, bool bf16, hipStream_t s);
// R <= 16 and N <= 4: row chunks of rows with many samples, one per 256-thread block
hipError_t launch_row_chunks(const RowArgs &a, int rp, bool bf16, hipStream_t s);
hipError_t launch_row_finalize(const RowArgs &a, int rp, bool bf16, hipStream_t s);
hipError_t launch_row_tiny(const RowArgs &a, bool bf16, hipStream_t s);

}  // namespace ntc
