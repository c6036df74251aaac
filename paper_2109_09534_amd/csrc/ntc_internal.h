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

// A whole row for the kernels that take rows with few samples (R <= 16,
// N <= 4): its CSR offset and length ride along, so the kernel needs no
// row-pointer lookup before it can sample.  Same size as Item.
struct RowItem {
    int32_t row;
    int32_t n;
    int64_t base;
};

// A row whose minibatch is split over `nslots` consecutive partial slots.
struct SplitRow {
    int32_t row;
    int32_t slot0;
    int32_t nslots;
    int32_t pad;
};

// Rows split into many items (R > 16) first sum groups of up to kFanIn
// consecutive partial slots into one second-level slot, so no finalize has
// to walk thousands of slots: {first source slot, count, destination slot}.
struct SlotGroup {
    int32_t src;
    int32_t count;
    int32_t dst;
    int32_t pad;
};
constexpr int kFanIn = 32;

// Arguments of the row kernels for one (mode, inner step).
struct RowArgs {
    const int64_t *rowptr;        // [I+1] CSR of this mode
    const uint32_t *records;      // [nnz][rec_words]: other-mode coordinates * R (increasing mode), value bits
    const Item *items;
    const SplitRow *split;
    const SlotGroup *groups;      // (R > 16) second-level slot sums, n_groups of them
    const RowItem *tiny;          // rows whose minibatch has 1..kTinyB samples (R <= 16 kernels) or
                                  // 1..kFewB32 samples (17 <= R <= 32, N <= 4)
    const RowItem *rows;          // (R <= 16, N <= 4) items [0, n_group) stored as RowItem
    const float *gath[kMaxModes - 1];     // other modes' FP32 factors, increasing mode order
    const uint16_t *gath16[kMaxModes - 1];// their BF16 shadows (precision form)
    float *A;                     // this mode's factor (A_l in, A_{l+1} out, in place)
    float *Y;                     // extrapolated iterate buffer (MAX_INNER > 1)
    uint16_t *A16;                // this mode's BF16 shadow (or null)
    double *partials;             // [slots][RP + RP*RP]
    uint32_t zrec[8];             // record of a missing sample: the all-zero row (index I_m) of each
                                  // other mode, value 0
    uint64_t seed;
    const int64_t *kptr;          // sweep counter k of the problem (device)
    const int32_t *stop;          // pool: nonzero once the problem has stopped (device), else null
    double lambda;
    double sqrt_lambda;           // sqrt(lambda), for the extrapolation weight beta
    double v0;                    // 1 / sqrt(R): every entry of the power method's start vector
    double c;
    int32_t mode;
    int32_t l;
    int32_t nmodes;
    int32_t rec_words;
    int32_t R;
    int32_t max_inner;
    int32_t power_iters;
    int32_t lp_bound;             // 0: Rayleigh quotient; 1: Collatz-Wielandt bound of the power iterate
    int32_t n_items;
    int32_t n_partial;            // (wave-per-item kernels) items [0, n_partial) write partial slots
    int32_t n_group;              // (R <= 16) items [0, n_group) are whole rows for the group kernel,
                                  // items [n_group, n_items) row chunks for the block kernel
    int32_t n_few;                // (R <= 16, N <= 4) the last n_few whole rows, [n_group - n_few,
                                  // n_group), have at most 16 samples: the few-sample kernel takes them
    int32_t n_split;
    int32_t n_tiny;
    int32_t n_groups;
};

// Records of a problem (all modes) up to this many bytes stay in the GPU's
// last-level cache (256 MB on MI355X) from one sweep to the next; larger
// record sets are loaded non-temporally.
constexpr int64_t kCachedRecordBytes = int64_t(256) << 20;

// Rows whose minibatch has at most this many samples run one row per lane (R <= 16).
constexpr int kTinyB = 4;
// 17 <= R <= 32, N <= 4: rows with at most this many samples run four to a
// wave, one per 16-lane group and one sample per lane.
constexpr int kFewB32 = 16;
// R <= 16, N <= 4: whole rows with tiny_max < B_p <= this many samples (and at
// most group_max) run the same way instead of in the group kernel.
constexpr int kFewB16 = 16;


// One launch of a row kernel over n entries (problems).  args: [n] device
// RowArgs.  For n > 1, start: [n] first block of each entry, owner:
// [blocks] entry of each block (both device); for n == 1 both may be null.
struct Launch {
    const RowArgs *args;
    const int32_t *start;
    const int32_t *owner;
    int32_t n;
    int32_t blocks;
};

// Kernel family of a problem: padded rank (16, 32, 64), mode count, BF16
// gathers, and how wide the loads of a factor row may be: for R <= 16, 2 when
// R % 4 == 0, else 0; for R <= 32, 4 when
// R == 32, 3 when R % 8 == 0, 2 when R % 4 == 0, 1 when R is even, else 0 (R
// is even: a lane reads its column pair with one load); for R <= 64, 2 when
// R % 4 == 0, 1 when R is even, else 0.
struct KernelClass {
    int32_t rp;
    int32_t nmodes;
    int32_t bf16;
    int32_t pairs;
    int32_t nt;  // 1: records loaded non-temporally (the problem's records exceed kCachedRecordBytes)
};

// The row kernels.  R <= 16: kRows takes whole rows with B_p <= group_max, one
// per 16-lane group (for N > 4 also every chunk); kChunks takes row chunks,
// one per 256-thread block; kTiny rows with B_p <= kTinyB, one per lane (one-wave blocks);
// kFinalize combines the partial slots of split rows.  R > 16: kRows takes
// every work item, one per wave; for 17 <= R <= 32 with N <= 4, kTiny takes
// the rows with B_p <= kFewB32, four per one-wave block.  kFew (R <= 16,
// N <= 4) takes the whole rows with kTinyB < B_p <= kFewB16, four per
// one-wave block, one sample per lane.
// kReduce (R > 16) sums groups of partial slots of rows split into many items.
enum RowKernel { kRows = 0, kFinalize = 1, kTiny = 2, kChunks = 3, kReduce = 4, kFew = 5 };
constexpr int kRowKernels = 6;

// Grid blocks one problem needs for `kind`.
int32_t row_kernel_blocks(RowKernel kind, const KernelClass &kc, int32_t n_items, int32_t n_group, int32_t n_split,
                          int32_t n_tiny, int32_t n_groups, int32_t n_few);
hipError_t launch_row_kernel(RowKernel kind, const KernelClass &kc, const Launch &L, hipStream_t s);
// the R > 16 kernels (called by launch_row_kernel)
hipError_t launch_row_kernel_wide(RowKernel kind, const KernelClass &kc, const Launch &L, hipStream_t s);
// k[t] += 1 for t < n (the sweep counters, once per sweep)
hipError_t launch_advance(int64_t *k, int32_t n, hipStream_t s);

}  // namespace ntc
