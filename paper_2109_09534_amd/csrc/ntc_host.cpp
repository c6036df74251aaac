// Host side of libntc: argument checks, the CSR-per-mode build, the static
// row schedule, device memory, and the C ABI declared in include/ntc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "ntc.h"
#include "ntc_aux.h"
#include "ntc_csr.h"
#include "ntc_internal.h"
#include "ntc_problem.h"
#include "ntc_rng.h"

using ntc::Item;
using ntc::SplitRow;

namespace {

thread_local std::string g_last_error;

ntc_status fail(ntc_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

}  // namespace

ntc_status ntc::set_error(ntc_status s, const std::string &msg)
{
    return fail(s, msg);
}

namespace {

#define NTC_HIP(expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            return fail(NTC_EDEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_));         \
    } while (0)

// Lanes per rank group: R <= 16 runs the group-per-item kernels (a 16-lane
// DPP row per item); larger ranks the wave-per-item kernels.
int padded_rank(int R)
{
    return R <= 16 ? 16 : R <= 32 ? 32 : 64;
}

int record_words(int nmodes)
{
    return nmodes <= 4 ? 4 : 8;
}

// Samples per work item: R <= 16 with N <= 4, a chunk for a 256-thread block
// (rows of more than group_max samples); otherwise a fixed amount of work per
// wave (the wave consumes 64/RP samples per step).
int item_samples(int rp, int nmodes)
{
    if (rp == 16)
        return nmodes <= 4 ? 6144 : 4096;
    return 512 * (64 / rp);
}

unsigned host_threads()
{
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0)
        t = 1;
    return std::min(t, 16u);
}

template <typename F>
void parallel_for(int64_t n, F &&f)
{
    const unsigned T = host_threads();
    if (T <= 1 || n < 1 << 16) {
        f(0, 0, n);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; ++t) {
        const int64_t a = n * t / T, b = n * (t + 1) / T;
        th.emplace_back([&f, t, a, b] { f(t, a, b); });
    }
    for (auto &x : th)
        x.join();
}

// Stable counting sort of the COO entries by coordinate `mode`, done in T
// contiguous chunks so that ties keep COO order.  Writes rowptr [I+1] and,
// if given, the records [nnz][rw] (other-mode coordinates times R, in
// increasing mode order, then the value bits) and/or the permutation [nnz].
// own_word >= 0 also stores the entry's own coordinate times R in that
// (otherwise padding) word of the record, for the loss.
void csr_build(int nmodes, const int64_t *dims, int64_t nnz, const int32_t *coords, const float *values, int mode,
               int rw, std::vector<int64_t> &rowptr, uint32_t *records, int64_t *perm, uint32_t rank = 1,
               int own_word = -1)
{
    const int64_t I = dims[mode];
    const unsigned T = (nnz < (1 << 16)) ? 1u : host_threads();
    std::vector<uint32_t> cnt(static_cast<size_t>(T) * static_cast<size_t>(I), 0u);
    std::vector<std::thread> th;
    auto chunk = [&](unsigned t, int64_t &a, int64_t &b) {
        a = nnz * t / T;
        b = nnz * (t + 1) / T;
    };
    auto count = [&](unsigned t) {
        int64_t a, b;
        chunk(t, a, b);
        uint32_t *c = cnt.data() + static_cast<size_t>(t) * I;
        for (int64_t e = a; e < b; ++e)
            ++c[coords[e * nmodes + mode]];
    };
    for (unsigned t = 0; t < T; ++t)
        th.emplace_back(count, t);
    for (auto &x : th)
        x.join();
    th.clear();
    rowptr.assign(static_cast<size_t>(I) + 1, 0);
    for (int64_t p = 0; p < I; ++p) {
        int64_t run = rowptr[p];
        for (unsigned t = 0; t < T; ++t) {
            uint32_t &c = cnt[static_cast<size_t>(t) * I + p];
            const uint32_t v = c;
            c = static_cast<uint32_t>(run);
            run += v;
        }
        rowptr[p + 1] = run;
    }
    auto scatter = [&](unsigned t) {
        int64_t a, b;
        chunk(t, a, b);
        uint32_t *off = cnt.data() + static_cast<size_t>(t) * I;
        for (int64_t e = a; e < b; ++e) {
            const int32_t *ce = coords + e * nmodes;
            const uint32_t pos = off[ce[mode]]++;
            if (perm)
                perm[pos] = e;
            if (records) {
                uint32_t *rec = records + static_cast<int64_t>(pos) * rw;
                int w = 0;
                for (int m = 0; m < nmodes; ++m)
                    if (m != mode)
                        rec[w++] = static_cast<uint32_t>(ce[m]) * rank;  // element offset of the factor row
                uint32_t vb;
                std::memcpy(&vb, values + e, 4);
                rec[w++] = vb;
                for (; w < rw; ++w)
                    rec[w] = 0u;
                if (own_word >= 0)
                    rec[own_word] = static_cast<uint32_t>(ce[mode]) * rank;
            }
        }
    };
    for (unsigned t = 0; t < T; ++t)
        th.emplace_back(scatter, t);
    for (auto &x : th)
        x.join();
}

struct ModeState {
    int64_t I = 0;
    int64_t *rowptr = nullptr;
    uint32_t *records = nullptr;
    Item *items = nullptr;
    SplitRow *split = nullptr;
    ntc::SlotGroup *groups = nullptr;
    int32_t n_groups = 0;
    ntc::RowItem *tiny = nullptr;
    int32_t n_tiny = 0;
    int64_t tiny_samples = 0;
    int32_t n_items = 0;
    int32_t n_partial = 0;
    int32_t n_group = 0;
    int32_t n_few = 0;                           // the last n_few whole rows of the group kernel's list
    int64_t few_samples = 0;
    int32_t n_split = 0;
    int32_t n_slots = 0;
    int64_t samples = 0;
    int64_t active_rows = 0;
    int64_t fused_rows = 0;
    int64_t row_samples = 0, row_fused = 0;      // launched by launch_row_items
    int64_t chunk_samples = 0, chunk_fused = 0;  // launched by launch_row_chunks
    std::vector<int64_t> h_rowptr;
};

}  // namespace

struct ntc_problem {
    int N = 0, R = 0, RP = 0, rw = 0;
    int64_t dims[ntc::kMaxModes] = {};
    int64_t nnz = 0;
    double c = 0.1, lambda = 1e-3;
    int max_inner = 1, power_iters = 20, lp_bound = 0;
    uint64_t seed = 0;
    bool bf16 = false;
    int64_t k = 0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;   // second stream for the one-row-per-lane launches
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int tiny_max = ntc::kTinyB;
    int item_samples = 0;
    int group_max = 512;
    int overlap = 1;
    int device = 0;
    ntc_alloc_fn alloc = nullptr;
    ntc_free_fn dfree = nullptr;
    void *actx = nullptr;
    std::vector<void *> owned;
    float *U[ntc::kMaxModes] = {};
    uint16_t *U16[ntc::kMaxModes] = {};
    float *Y = nullptr;
    double *partials = nullptr;
    ModeState md[ntc::kMaxModes];
    int64_t n_test = 0;
    int32_t *test_coords = nullptr;
    float *test_values = nullptr;
    double *loss_part = nullptr;
    double *loss_out = nullptr;
    int64_t *kdev = nullptr;            // device copy of the sweep counter k
    ntc::RowArgs *args_dev = nullptr;  // [N][max_inner] row-kernel arguments (static after create)
    std::vector<ntc::RowArgs> args_host;  // host copy of args_dev
    size_t bytes = 0;                   // device bytes held
    uint32_t *row0 = nullptr;  // row * R per mode-0 record when the record has no spare word
    int32_t row_word = -1;     // record word of mode 0 holding row * R
    int32_t *dbg = nullptr;  // debug sampler output [max row length + 1]
    int64_t max_row = 0;

    void *dalloc(size_t bytes)
    {
        if (bytes == 0)
            bytes = 256;
        void *p = nullptr;
        if (alloc) {
            p = alloc(bytes, stream, actx);
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        if (p) {
            owned.push_back(p);
            this->bytes += bytes;
        }
        return p;
    }

    ~ntc_problem()
    {
        if (owned.empty())
            return;
        if (stream)
            (void)hipStreamSynchronize(stream);
        else
            (void)hipDeviceSynchronize();
        for (void *p : owned) {
            if (dfree)
                dfree(p, actx);
            else
                (void)hipFree(p);
        }
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
        if (ev_fork)
            (void)hipEventDestroy(ev_fork);
        if (ev_join)
            (void)hipEventDestroy(ev_join);
    }
};

namespace {

ntc_status alloc_or_fail(ntc_problem *h, void **dst, size_t bytes, const char *what)
{
    *dst = h->dalloc(bytes);
    if (!*dst)
        return fail(NTC_ENOMEM, std::string("device allocation failed: ") + what + " (" + std::to_string(bytes) +
                                    " bytes)");
    return NTC_OK;
}

#define NTC_TRY(expr)                 \
    do {                              \
        ntc_status s_ = (expr);       \
        if (s_ != NTC_OK)             \
            return s_;                \
    } while (0)

ntc::KernelClass kernel_class(const ntc_problem *h)
{
    // pairs: how wide the loads of a factor row may be (R <= 16: 2 when R % 4 == 0;
    // R <= 32: 4 when R == 32, 3 when R % 8 == 0, 2 when R % 4 == 0, 1 when R is
    // even; R <= 64: 2 when R % 4 == 0, 1 when R is even; else 0)
    int32_t pairs = 0;
    if (h->RP == 16)
        pairs = h->R % 4 == 0 ? 2 : 0;
    else if (h->RP == 32)
        pairs = h->R == 32 ? 4 : h->R % 8 == 0 ? 3 : h->R % 4 == 0 ? 2 : h->R % 2 == 0 ? 1 : 0;
    else if (h->RP == 64)
        pairs = h->R % 4 == 0 ? 2 : h->R % 2 == 0 ? 1 : 0;
    const int32_t nt = h->nnz * h->rw * 4 * h->N > ntc::kCachedRecordBytes ? 1 : 0;
    return ntc::KernelClass{h->RP, h->N, h->bf16 ? 1 : 0, pairs, nt};
}

ntc::RowArgs row_args(ntc_problem *h, int mode, int l)
{
    ntc::RowArgs a{};
    const ModeState &m = h->md[mode];
    a.rowptr = m.rowptr;
    a.records = m.records;
    a.items = m.items;
    a.split = m.split;
    a.groups = m.groups;
    a.n_groups = m.n_groups;
    a.tiny = m.tiny;
    a.rows = (h->RP == 16 && h->N <= 4) ? reinterpret_cast<const ntc::RowItem *>(m.items) : nullptr;
    a.n_tiny = m.n_tiny;
    a.c = h->c;
    int w = 0;
    for (int mm = 0; mm < h->N; ++mm) {
        if (mm == mode)
            continue;
        a.gath[w] = h->U[mm];
        a.gath16[w] = h->U16[mm];
        ++w;
    }
    {
        int z = 0;
        for (int mm = 0; mm < h->N; ++mm)
            if (mm != mode)
                a.zrec[z++] = static_cast<uint32_t>(h->dims[mm] * h->R);
        for (; z < 8; ++z)
            a.zrec[z] = 0u;  // value 0 and padding
    }
    a.A = h->U[mode];
    a.Y = h->Y;
    a.A16 = h->U16[mode];
    a.partials = h->partials;
    a.seed = h->seed;
    a.kptr = h->kdev;
    a.lambda = h->lambda;
    a.sqrt_lambda = std::sqrt(h->lambda);
    a.v0 = 1.0 / std::sqrt(static_cast<double>(h->R));
    a.mode = mode;
    a.l = l;
    a.nmodes = h->N;
    a.rec_words = h->rw;
    a.R = h->R;
    a.max_inner = h->max_inner;
    a.power_iters = h->power_iters;
    a.lp_bound = h->lp_bound;
    a.n_items = m.n_items;
    a.n_partial = m.n_partial;
    a.n_group = m.n_group;
    a.n_few = m.n_few;
    a.n_split = m.n_split;
    return a;
}

// Optional per-launch event timing (ntc_profile_sweep).
struct LaunchProbe {
    std::vector<ntc_launch_record> rec;
    std::vector<hipEvent_t> ev;  // two per launch
    bool concurrent = false;     // keep the side-stream overlap of ntc_sweep
};

ntc_status enqueue_mode(ntc_problem *h, int mode, LaunchProbe *probe = nullptr)
{
    ntc::TraceRange range(ntc::mode_range_name(mode));
    const ModeState &md = h->md[mode];
    const ntc::KernelClass kc = kernel_class(h);
    for (int l = 0; l < h->max_inner; ++l) {
        ntc::Launch L{};
        L.args = h->args_dev + mode * h->max_inner + l;
        L.n = 1;
        // With a side stream, work on disjoint rows runs concurrently
        // (fork/join through events): the one-row-per-lane rows, and for
        // R <= 16 with N <= 4 also the whole rows of the group kernel, go to
        // the side stream while the chunks and the finalize of split rows
        // (which reads only the chunks' partial slots) stay on the main
        // stream.  A serial profiled sweep runs everything on one stream.
        // overlap = 2 keeps the one-row-per-lane rows on the main stream, ahead of the chunks.
        const bool rows_aside = kc.rp == 16 && kc.nmodes <= 4;
        const bool tiny_aside = h->overlap != 2;
        const int32_t n_aside = (tiny_aside ? md.n_tiny : 0) + (rows_aside ? md.n_group - md.n_few : 0);
        const int32_t n_main = (rows_aside ? md.n_items - md.n_group + md.n_few : md.n_items) + md.n_split +
                               (tiny_aside ? 0 : md.n_tiny);
        const bool fork = (!probe || probe->concurrent) && h->side && n_aside > 0 && n_main > 0;
        if (fork) {
            NTC_HIP(hipEventRecord(h->ev_fork, h->stream));
            NTC_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
        }
        // launch order: rows, chunks, few-sample rows, rows of at most tiny_max samples, finalize
        // of split rows.  For R <= 16 the side stream runs the group rows, then the rows of at
        // most 4 samples (C1: 0.891 against 0.898 ms per sweep the other way round); the
        // rows of 5 to 16 samples stay on the main stream after the chunks.
        for (ntc::RowKernel kern : {ntc::kRows, ntc::kChunks, ntc::kFew, ntc::kTiny, ntc::kReduce, ntc::kFinalize}) {
            L.blocks = ntc::row_kernel_blocks(kern, kc, md.n_items, md.n_group, md.n_split, md.n_tiny, md.n_groups,
                                              md.n_few);
            if (L.blocks <= 0)
                continue;
            const bool aside = (kern == ntc::kTiny && tiny_aside) || (kern == ntc::kRows && rows_aside);
            hipStream_t st = (aside && fork) ? h->side : h->stream;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (probe) {
                NTC_HIP(hipEventCreate(&e0));
                NTC_HIP(hipEventCreate(&e1));
                probe->ev.push_back(e0);
                probe->ev.push_back(e1);
                NTC_HIP(hipEventRecord(e0, st));
            }
            NTC_HIP(ntc::launch_row_kernel(kern, kc, L, st));
            if (probe) {
                NTC_HIP(hipEventRecord(e1, st));
                ntc_launch_record r{};
                r.kernel = kern;
                r.mode = mode;
                r.inner = l;
                r.blocks = L.blocks;
                r.samples = kern == ntc::kRows ? md.row_samples : kern == ntc::kTiny ? md.tiny_samples
                            : kern == ntc::kChunks ? md.chunk_samples : kern == ntc::kFew ? md.few_samples : 0;
                r.rows = kern == ntc::kRows ? md.row_fused : kern == ntc::kFinalize ? md.n_split
                         : kern == ntc::kTiny ? md.n_tiny : kern == ntc::kChunks ? md.chunk_fused
                         : kern == ntc::kFew ? md.n_few : 0;
                probe->rec.push_back(r);
            }
        }
        if (fork) {
            NTC_HIP(hipEventRecord(h->ev_join, h->side));
            NTC_HIP(hipStreamWaitEvent(h->stream, h->ev_join, 0));
        }
    }
    return NTC_OK;
}

ntc_status sync(ntc_problem *h)
{
    NTC_HIP(hipStreamSynchronize(h->stream));
    return NTC_OK;
}

ntc_status check_mode(ntc_problem *h, int32_t mode)
{
    if (!h)
        return fail(NTC_EINVAL, "null handle");
    if (mode < 0 || mode >= h->N)
        return fail(NTC_EINVAL, "mode out of range");
    return NTC_OK;
}

ntc_status validate_factor(const float *src, int64_t count, int mode)
{
    for (int64_t t = 0; t < count; ++t)
        if (!(src[t] >= 0.0f) || !std::isfinite(src[t]))
            return fail(NTC_EINVAL, "factor of mode " + std::to_string(mode) +
                                        " has a negative or non-finite entry at " + std::to_string(t));
    return NTC_OK;
}

}  // namespace

// Everything ntc_create computes on the host before it touches the device:
// the validated parameters, the CSR records and row pointers of every mode,
// the row schedule, the held-out set and the initial factors.  Building one
// needs no device and no shared state, so it may run on any host thread.
struct ntc_prepared {
    int N = 0, R = 0, RP = 0, rw = 0;
    int64_t dims[ntc::kMaxModes] = {};
    int64_t nnz = 0;
    double c = 0.1, lambda = 1e-3;
    int max_inner = 1, power_iters = 20, lp_bound = 0;
    uint64_t seed = 0;
    bool bf16 = false;
    int tiny_max = ntc::kTinyB, item_samples = 0, group_max = 512;
    struct Mode {
        ModeState st;                      // counts of the schedule (device pointers unset)
        std::vector<uint32_t> rec;         // [nnz][rw]
        std::vector<ntc::RowItem> tiny;
        std::vector<Item> items;
        std::vector<SplitRow> split;
        std::vector<ntc::SlotGroup> groups;
        uint32_t *dev_rec = nullptr;       // records already built on the device (ntc_create_device_csr)
    } md[ntc::kMaxModes];
    std::vector<uint32_t> row0;            // row * R of every mode-0 record (N = 4 or 8)
    uint32_t *dev_row0 = nullptr;          // the same, built on the device
    int32_t row_word = -1;
    int32_t max_slots = 0;
    int64_t max_row = 0;
    std::vector<int32_t> test_coords;
    std::vector<float> test_values;
    std::vector<std::vector<float>> init;  // caller's factors, or empty for the default init
    float init_scale = 1.0f;
};

namespace {

// The host's check of one COO entry: coordinates in range, a finite value.
ntc_status check_entry(const int32_t *coords, const float *values, int N, const int64_t *dims, int64_t e)
{
    for (int m = 0; m < N; ++m) {
        const int32_t x = coords[e * N + m];
        if (x < 0 || x >= dims[m])
            return fail(NTC_EINVAL, "coordinate out of range at entry " + std::to_string(e));
    }
    if (!std::isfinite(values[e]))
        return fail(NTC_EINVAL, "non-finite value at entry " + std::to_string(e));
    return NTC_OK;
}

// Every check of ntc_create's arguments except the per-entry one.
ntc_status check_params(int32_t N, const int64_t *dims, int64_t nnz, const int32_t *coords, const float *values,
                        int32_t R, const ntc_params &p)
{
    if (N < 2 || N > ntc::kMaxModes)
        return fail(NTC_EINVAL, "nmodes must be in [2, 8]");
    if (R < 1 || R > ntc::kMaxRank)
        return fail(NTC_EINVAL, "rank must be in [1, 64]");
    if (!dims)
        return fail(NTC_EINVAL, "dims is null");
    if (nnz < 0 || nnz >= (int64_t(1) << 31))
        return fail(NTC_EINVAL, "nnz must be in [0, 2^31)");
    if (nnz > 0 && (!coords || !values))
        return fail(NTC_EINVAL, "coords/values are null");
    if (!(p.c > 0.0 && p.c <= 1.0))
        return fail(NTC_EINVAL, "c must be in (0, 1]");
    if (!(p.lambda >= 0.0) || !std::isfinite(p.lambda))
        return fail(NTC_EINVAL, "lambda must be finite and >= 0");
    if (p.max_inner < 1 || p.max_inner > 0xFFFF)
        return fail(NTC_EINVAL, "max_inner must be in [1, 65535]");
    if (p.power_iters < 0)
        return fail(NTC_EINVAL, "power_iters must be >= 0");
    if (p.lp_bound != 0 && p.lp_bound != 1)
        return fail(NTC_EINVAL, "lp_bound must be 0 or 1");
    if (p.tiny_max < -1 || p.tiny_max > ntc::kFewB32 || (R <= 16 && p.tiny_max > ntc::kTinyB))
        return fail(NTC_EINVAL, "tiny_max must be -1 or in [0, 4] (R <= 16), [0, 16] (R > 16)");
    if (p.item_samples < 0 || (p.item_samples > 0 && p.item_samples < 16))
        return fail(NTC_EINVAL, "item_samples must be 0 or >= 16");
    if (p.group_max < 0)
        return fail(NTC_EINVAL, "group_max must be >= 0");
    if (p.overlap < 0 || p.overlap > 2)
        return fail(NTC_EINVAL, "overlap must be 0, 1 or 2");
    if (p.n_test < 0 || (p.n_test > 0 && (!p.test_coords || !p.test_values)))
        return fail(NTC_EINVAL, "test set pointers are null");
    for (int m = 0; m < N; ++m) {
        if (dims[m] < 1 || dims[m] >= (int64_t(1) << 31))
            return fail(NTC_EINVAL, "dims[" + std::to_string(m) + "] must be in [1, 2^31)");
        if ((dims[m] + 1) * R * 4 >= (int64_t(1) << 32))
            return fail(NTC_EUNSUPPORTED, "factor of mode " + std::to_string(m) +
                                              " would exceed 4 GiB (gathers use 32-bit byte offsets)");
    }

    for (int64_t e = 0; e < p.n_test; ++e) {
        for (int m = 0; m < N; ++m) {
            const int32_t x = p.test_coords[e * N + m];
            if (x < 0 || x >= dims[m])
                return fail(NTC_EINVAL, "test coordinate out of range at entry " + std::to_string(e));
        }
        if (!std::isfinite(p.test_values[e]))
            return fail(NTC_EINVAL, "non-finite test value at entry " + std::to_string(e));
    }
    if (p.init_factors)
        for (int m = 0; m < N; ++m) {
            if (!p.init_factors[m])
                return fail(NTC_EINVAL, "init_factors[" + std::to_string(m) + "] is null");
            NTC_TRY(validate_factor(p.init_factors[m], dims[m] * R, m));
        }
    return NTC_OK;
}

// dev_rowptr (N of them): the row pointers of a CSR already built on the
// device, whose entries were checked there; the host then builds only the
// schedule.
ntc_status prepare_impl(ntc_prepared *q, int32_t N, const int64_t *dims, int64_t nnz, const int32_t *coords,
                        const float *values, int32_t R, const ntc_params &p,
                        const std::vector<int64_t> *dev_rowptr = nullptr)
{
    NTC_TRY(check_params(N, dims, nnz, coords, values, R, p));
    for (int64_t e = 0; e < (dev_rowptr ? 0 : nnz); ++e)
        NTC_TRY(check_entry(coords, values, N, dims, e));

    q->N = N;
    q->R = R;
    q->RP = padded_rank(R);
    q->rw = record_words(N);
    q->nnz = nnz;
    q->c = p.c;
    q->lambda = p.lambda;
    q->max_inner = p.max_inner;
    q->power_iters = p.power_iters;
    q->lp_bound = p.lp_bound;
    q->seed = p.seed;
    q->bf16 = p.gather_bf16 != 0;
    q->tiny_max = p.tiny_max >= 0 ? p.tiny_max : R <= 16 ? ntc::kTinyB : ntc::kFewB32;
    q->item_samples = p.item_samples;
    q->group_max = p.group_max > 0 ? p.group_max : 512;
    for (int m = 0; m < N; ++m)
        q->dims[m] = dims[m];

    // CSR per mode and the static schedule
    const int rp = q->RP;
    const int smax = q->item_samples > 0 ? q->item_samples : item_samples(rp, N);
    for (int m = 0; m < N; ++m) {
        ntc_prepared::Mode &pm = q->md[m];
        ModeState &md = pm.st;
        md.I = dims[m];
        // mode 0's records also carry the row (times R) for the loss: in the
        // padding word when there is one, else in a separate array
        const int own = (m == 0 && N < q->rw) ? N : -1;
        if (dev_rowptr) {
            md.h_rowptr = dev_rowptr[m];
        } else {
            pm.rec.assign(static_cast<size_t>(std::max<int64_t>(nnz, 1)) * q->rw, 0u);
            csr_build(N, dims, nnz, coords, values, m, q->rw, md.h_rowptr, pm.rec.data(), nullptr,
                      static_cast<uint32_t>(R), own);
        }
        if (m == 0 && own < 0 && nnz > 0 && !dev_rowptr) {
            q->row0.assign(static_cast<size_t>(nnz), 0u);
            for (int64_t r = 0; r < md.I; ++r)
                for (int64_t e = md.h_rowptr[r]; e < md.h_rowptr[r + 1]; ++e)
                    q->row0[e] = static_cast<uint32_t>(r * R);
        }
        if (m == 0)
            q->row_word = own;
        std::vector<int32_t> rows;
        std::vector<int64_t> bsz(static_cast<size_t>(md.I));
        for (int64_t r = 0; r < md.I; ++r) {
            const int64_t n = md.h_rowptr[r + 1] - md.h_rowptr[r];
            q->max_row = std::max(q->max_row, n);
            bsz[r] = ntc::minibatch_size(q->c, n);
            if (bsz[r] > 0)
                rows.push_back(static_cast<int32_t>(r));
        }
        std::stable_sort(rows.begin(), rows.end(), [&](int32_t a, int32_t b) { return bsz[a] > bsz[b]; });
        std::vector<Item> &items = pm.items;
        std::vector<Item> whole;
        std::vector<SplitRow> &split = pm.split;
        std::vector<ntc::SlotGroup> &groups = pm.groups;
        std::vector<ntc::RowItem> &tiny = pm.tiny;
        auto row_item = [&](int32_t r) {
            const int64_t b0 = md.h_rowptr[r];
            return ntc::RowItem{r, static_cast<int32_t>(md.h_rowptr[r + 1] - b0), b0};
        };
        auto as_item = [](const ntc::RowItem &ri) {
            Item it;
            static_assert(sizeof(Item) == sizeof(ntc::RowItem), "item layouts");
            std::memcpy(&it, &ri, sizeof(it));
            return it;
        };
        int32_t slot = 0;
        if (rp == 16) {
            // one row per lane / one sample per lane / one row per 16-lane group / 16 groups per row chunk
            const int64_t few_max = q->N <= 4 ? std::min<int64_t>(ntc::kFewB16, q->group_max) : 0;
            std::vector<Item> chunks;
            for (int32_t r : rows) {
                const int64_t b = bsz[r];
                md.samples += b;
                md.active_rows += 1;
                if (b <= q->tiny_max) {
                    tiny.push_back(row_item(r));
                    md.tiny_samples += b;
                } else if (b <= q->group_max) {
                    md.fused_rows += 1;
                    if (b <= few_max) {  // the tail of the list (rows come in decreasing B_p)
                        md.n_few += 1;
                        md.few_samples += b;
                    } else {
                        md.row_fused += 1;
                        md.row_samples += b;
                    }
                    // N <= 4: the group kernel reads these as RowItem
                    items.push_back(q->N <= 4 ? as_item(row_item(r)) : Item{r, 0, static_cast<int32_t>(b), -1});
                } else if (b <= smax) {
                    md.fused_rows += 1;
                    md.chunk_fused += 1;
                    md.chunk_samples += b;
                    chunks.push_back(Item{r, 0, static_cast<int32_t>(b), -1});
                } else {
                    md.chunk_samples += b;
                    const int32_t s0 = slot;
                    for (int64_t j0 = 0; j0 < b; j0 += smax)
                        chunks.push_back(Item{r, static_cast<int32_t>(j0),
                                              static_cast<int32_t>(std::min(b, j0 + smax)), slot++});
                    split.push_back(SplitRow{r, s0, slot - s0, 0});
                }
            }
            md.n_group = static_cast<int32_t>(items.size());
            items.insert(items.end(), chunks.begin(), chunks.end());
            if (q->N > 4) {  // the group kernel takes every item
                md.row_samples += md.chunk_samples;
                md.row_fused += md.chunk_fused;
                md.chunk_samples = md.chunk_fused = 0;
            }
        } else {
            // 17 <= R <= 32, N <= 4: rows of at most tiny_max samples, four per wave
            const int64_t few_max = (rp == 32 && N <= 4) ? q->tiny_max : 0;
            for (int32_t r : rows) {
                const int64_t b = bsz[r];
                md.samples += b;
                md.active_rows += 1;
                if (b <= few_max) {
                    tiny.push_back(row_item(r));
                    md.tiny_samples += b;
                    continue;
                }
                md.row_samples += b;
                if (b <= smax) {
                    md.fused_rows += 1;
                    md.row_fused += 1;
                    whole.push_back(Item{r, 0, static_cast<int32_t>(b), -1});
                } else {
                    const int32_t s0 = slot;
                    for (int64_t j0 = 0; j0 < b; j0 += smax)
                        items.push_back(Item{r, static_cast<int32_t>(j0),
                                             static_cast<int32_t>(std::min(b, j0 + smax)), slot++});
                    const int32_t ns = slot - s0;
                    if (ns > 2 * ntc::kFanIn) {
                        // second level: groups of kFanIn slots, numbered after all first-level slots
                        const int32_t g0 = static_cast<int32_t>(groups.size());
                        for (int32_t q = 0; q < ns; q += ntc::kFanIn)
                            groups.push_back(ntc::SlotGroup{s0 + q, std::min(ntc::kFanIn, ns - q), -1, 0});
                        split.push_back(SplitRow{r, -1 - g0, static_cast<int32_t>(groups.size()) - g0, 0});
                    } else {
                        split.push_back(SplitRow{r, s0, ns, 0});
                    }
                }
            }
            // second-level slots follow the first-level ones
            for (size_t q = 0; q < groups.size(); ++q)
                groups[q].dst = slot + static_cast<int32_t>(q);
            for (SplitRow &sr : split)
                if (sr.slot0 < 0)
                    sr.slot0 = groups[static_cast<size_t>(-1 - sr.slot0)].dst;
            slot += static_cast<int32_t>(groups.size());
        }
        md.n_partial = static_cast<int32_t>(items.size());
        items.insert(items.end(), whole.begin(), whole.end());
        md.n_tiny = static_cast<int32_t>(tiny.size());
        md.n_items = static_cast<int32_t>(items.size());
        md.n_split = static_cast<int32_t>(split.size());
        md.n_slots = slot;
        md.n_groups = static_cast<int32_t>(groups.size());
        q->max_slots = std::max(q->max_slots, slot);
    }

    // held-out set and initial factors
    if (p.n_test > 0) {
        q->test_coords.assign(p.test_coords, p.test_coords + p.n_test * N);
        q->test_values.assign(p.test_values, p.test_values + p.n_test);
    }
    if (p.init_factors) {
        q->init.resize(N);
        for (int m = 0; m < N; ++m)
            q->init[m].assign(p.init_factors[m], p.init_factors[m] + dims[m] * R);
    } else {
        double sum = 0.0;
        for (int64_t e = 0; e < nnz; ++e)
            sum += static_cast<double>(values[e]);
        double mean = nnz > 0 ? sum / static_cast<double>(nnz) : 0.0;
        if (!(mean > 1e-30))
            mean = 1e-30;
        q->init_scale = static_cast<float>(
            std::pow(mean / (static_cast<double>(R) * std::pow(2.0, -static_cast<double>(N))), 1.0 / static_cast<double>(N)));
    }
    return NTC_OK;
}

// Device side of ntc_create: allocations, uploads, default init.
ntc_status commit_impl(ntc_problem *h, const ntc_prepared &q, const ntc_params &p)
{
    const int N = q.N, R = q.R;
    const int64_t nnz = q.nnz;
    h->N = N;
    h->R = R;
    h->RP = q.RP;
    h->rw = q.rw;
    h->nnz = nnz;
    h->c = q.c;
    h->lambda = q.lambda;
    h->max_inner = q.max_inner;
    h->power_iters = q.power_iters;
    h->lp_bound = q.lp_bound;
    h->seed = q.seed;
    h->bf16 = q.bf16;
    h->stream = static_cast<hipStream_t>(p.stream);
    h->alloc = p.dev_alloc;
    h->dfree = p.dev_free;
    h->actx = p.alloc_ctx;
    h->tiny_max = q.tiny_max;
    h->item_samples = q.item_samples;
    h->group_max = q.group_max;
    h->max_row = q.max_row;
    h->row_word = q.row_word;
    NTC_HIP(hipGetDevice(&h->device));
    h->overlap = p.overlap;
    if (p.overlap) {
        NTC_HIP(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        NTC_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        NTC_HIP(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    }
    for (int m = 0; m < N; ++m)
        h->dims[m] = q.dims[m];

    // factors and shadows
    int64_t maxI = 0;
    // every factor has one extra all-zero row (index I_m): the gathers of a
    // missing sample read it, so its Khatri-Rao row is exactly zero
    for (int m = 0; m < N; ++m) {
        const int64_t cntm = (q.dims[m] + 1) * R;
        maxI = std::max(maxI, q.dims[m]);
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->U[m]), cntm * sizeof(float), "factor"));
        NTC_HIP(hipMemset(h->U[m], 0, cntm * sizeof(float)));
        if (h->bf16) {
            NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->U16[m]), cntm * sizeof(uint16_t), "bf16 shadow"));
            NTC_HIP(hipMemset(h->U16[m], 0, cntm * sizeof(uint16_t)));
        }
    }
    if (h->max_inner > 1)
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->Y), maxI * R * sizeof(float), "Y buffer"));
    if (q.dev_row0) {
        h->row0 = q.dev_row0;  // built on the device, already owned by h
    } else if (!q.row0.empty()) {
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->row0), static_cast<size_t>(nnz) * 4, "loss rows"));
        NTC_HIP(hipMemcpy(h->row0, q.row0.data(), static_cast<size_t>(nnz) * 4, hipMemcpyHostToDevice));
    }
    for (int m = 0; m < N; ++m) {
        const ntc_prepared::Mode &pm = q.md[m];
        ModeState &md = h->md[m];
        md = pm.st;
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&md.rowptr), (md.I + 1) * sizeof(int64_t), "rowptr"));
        NTC_HIP(hipMemcpy(md.rowptr, md.h_rowptr.data(), (md.I + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
        if (pm.dev_rec) {
            md.records = pm.dev_rec;  // built on the device, already owned by h
        } else {
            NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&md.records),
                                  static_cast<size_t>(std::max<int64_t>(nnz, 1)) * h->rw * 4, "records"));
            NTC_HIP(hipMemcpy(md.records, pm.rec.data(), static_cast<size_t>(nnz) * h->rw * 4,
                              hipMemcpyHostToDevice));
        }
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&md.tiny), pm.tiny.size() * sizeof(ntc::RowItem),
                              "tiny rows"));
        if (!pm.tiny.empty())
            NTC_HIP(hipMemcpy(md.tiny, pm.tiny.data(), pm.tiny.size() * sizeof(ntc::RowItem), hipMemcpyHostToDevice));
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&md.groups), pm.groups.size() * sizeof(ntc::SlotGroup),
                              "slot groups"));
        if (!pm.groups.empty())
            NTC_HIP(hipMemcpy(md.groups, pm.groups.data(), pm.groups.size() * sizeof(ntc::SlotGroup),
                              hipMemcpyHostToDevice));
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&md.items), pm.items.size() * sizeof(Item), "items"));
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&md.split), pm.split.size() * sizeof(SplitRow), "split"));
        if (!pm.items.empty())
            NTC_HIP(hipMemcpy(md.items, pm.items.data(), pm.items.size() * sizeof(Item), hipMemcpyHostToDevice));
        if (!pm.split.empty())
            NTC_HIP(hipMemcpy(md.split, pm.split.data(), pm.split.size() * sizeof(SplitRow), hipMemcpyHostToDevice));
    }
    const int rp = h->RP;
    NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->partials),
                          static_cast<size_t>(std::max(q.max_slots, 1)) * (rp + rp * rp) * sizeof(double), "partials"));

    // held-out set and loss buffers
    const int64_t n_test = static_cast<int64_t>(q.test_values.size());
    h->n_test = n_test;
    NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->test_coords),
                          static_cast<size_t>(std::max<int64_t>(n_test, 1)) * N * sizeof(int32_t), "test coords"));
    NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->test_values),
                          static_cast<size_t>(std::max<int64_t>(n_test, 1)) * sizeof(float), "test values"));
    if (n_test > 0) {
        NTC_HIP(hipMemcpy(h->test_coords, q.test_coords.data(), n_test * N * sizeof(int32_t), hipMemcpyHostToDevice));
        NTC_HIP(hipMemcpy(h->test_values, q.test_values.data(), n_test * sizeof(float), hipMemcpyHostToDevice));
    }
    NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->loss_part), 4 * ntc::kLossBlocks * sizeof(double),
                          "loss partials"));
    NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->loss_out), 4 * sizeof(double), "loss out"));
    NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->dbg), (h->max_row + 1) * sizeof(int32_t), "debug"));

    // device sweep counter and the row-kernel argument table of every (mode, inner step)
    NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->kdev), sizeof(int64_t), "sweep counter"));
    NTC_HIP(hipMemcpy(h->kdev, &h->k, sizeof(int64_t), hipMemcpyHostToDevice));
    {
        std::vector<ntc::RowArgs> &tab = h->args_host;
        tab.clear();
        for (int m = 0; m < N; ++m)
            for (int l = 0; l < h->max_inner; ++l)
                tab.push_back(row_args(h, m, l));
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&h->args_dev), tab.size() * sizeof(ntc::RowArgs),
                              "row arguments"));
        NTC_HIP(hipMemcpy(h->args_dev, tab.data(), tab.size() * sizeof(ntc::RowArgs), hipMemcpyHostToDevice));
    }

    // initial factors
    if (!q.init.empty()) {
        for (int m = 0; m < N; ++m) {
            NTC_HIP(hipMemcpy(h->U[m], q.init[m].data(), q.dims[m] * R * sizeof(float), hipMemcpyHostToDevice));
            if (h->bf16)
                NTC_HIP(ntc::launch_to_bf16(h->U[m], h->U16[m], q.dims[m] * R, h->stream));
        }
    } else {
        for (int m = 0; m < N; ++m)
            NTC_HIP(ntc::launch_init_factor(h->U[m], h->U16[m], q.dims[m] * R, m, h->seed, q.init_scale, h->stream));
    }
    return sync(h);
}

}  // namespace

ntc_status ntc::problem_view(ntc_handle h, ntc::ProblemView *v)
{
    if (!h || !v)
        return fail(NTC_EINVAL, "null argument");
    v->kc = kernel_class(h);
    v->nmodes = h->N;
    v->rank = h->R;
    v->max_inner = h->max_inner;
    v->args_host = h->args_host.data();
    v->kdev = h->kdev;
    for (int m = 0; m < h->N; ++m) {
        const ModeState &md = h->md[m];
        for (int kind = 0; kind < ntc::kRowKernels; ++kind)
            v->blocks[m][kind] = ntc::row_kernel_blocks(static_cast<ntc::RowKernel>(kind), v->kc, md.n_items,
                                                        md.n_group, md.n_split, md.n_tiny, md.n_groups, md.n_few);
        v->U[m] = h->U[m];
    }
    v->n_test = h->n_test;
    v->test_coords = h->test_coords;
    v->test_values = h->test_values;
    v->bytes = h->bytes;
    v->k = h->k;
    int64_t u = 0;
    for (int m = 0; m < h->N; ++m)
        u += h->md[m].samples * h->max_inner;
    v->updates_per_sweep = u;
    return NTC_OK;
}

ntc_status ntc::device_csr_temp_bytes(int32_t nmodes, const int64_t *dims, int64_t nnz, size_t *bytes)
{
    if (!bytes || !dims || nmodes < 2 || nmodes > ntc::kMaxModes || nnz < 0)
        return fail(NTC_EINVAL, "invalid argument");
    auto r = [](size_t b) { return (std::max<size_t>(b, 256) + 255) / 256 * 256; };
    const size_t n = static_cast<size_t>(std::max<int64_t>(nnz, 1));
    int64_t maxI = 0;
    for (int m = 0; m < nmodes; ++m)
        maxI = std::max(maxI, dims[m]);
    size_t sort = 0;
    NTC_HIP(ntc::csr_sort_bytes(nnz, &sort));
    *bytes = r(n * nmodes * 4) + r(n * 4) + 4 * r(n * 4) + r(sizeof(unsigned long long)) +
             r(static_cast<size_t>(maxI + 1) * 8) + r(sort);
    return NTC_OK;
}

void ntc::note_sweeps(ntc_handle h, int64_t n)
{
    h->k += n;
}

// ======================================================================= ABI
// The mode-sorted CSR of every mode built on the device (ntc_create_device_csr):
// the COO is uploaded once and checked there; per mode a stable radix sort
// by coordinate gives the same entry order as the host's counting sort.  The
// records (and mode 0's row array when the record has no spare word) are
// allocated through h and handed to commit; the row pointers come back for
// the host-side schedule.  Temporaries come from h's allocator when it has
// one (a pool's arena), else from hipMalloc, and are freed here once h's
// stream has finished with them.
struct DeviceTemps {
    ntc_problem *h;
    std::vector<void *> p;
    explicit DeviceTemps(ntc_problem *owner) : h(owner) {}
    ~DeviceTemps()
    {
        if (!p.empty())
            (void)hipStreamSynchronize(h->stream);
        for (void *x : p) {
            if (h->alloc && h->dfree)
                h->dfree(x, h->actx);
            else
                (void)hipFree(x);
        }
    }
    hipError_t get(void **dst, size_t bytes)
    {
        *dst = nullptr;
        bytes = std::max<size_t>(bytes, 256);
        if (h->alloc) {
            *dst = h->alloc(bytes, h->stream, h->actx);
            if (!*dst)
                return hipErrorOutOfMemory;
        } else {
            const hipError_t e = hipMalloc(dst, bytes);
            if (e != hipSuccess)
                return e;
        }
        p.push_back(*dst);
        return hipSuccess;
    }
};

ntc_status device_csr(ntc_problem *h, ntc_prepared &q, std::vector<int64_t> (&rowptr)[ntc::kMaxModes], int32_t N,
                      const int64_t *dims, int64_t nnz, const int32_t *coords, const float *values, int32_t R)
{
    DeviceTemps t(h);
    const hipStream_t st = h->stream;
    int32_t *d_coords = nullptr;
    float *d_values = nullptr;
    uint32_t *keys_in = nullptr, *keys_out = nullptr, *ids_in = nullptr, *ids_out = nullptr;
    unsigned long long *bad = nullptr;
    int64_t *d_rowptr = nullptr;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    int64_t maxI = 0;
    for (int m = 0; m < N; ++m)
        maxI = std::max(maxI, dims[m]);
    const size_t n = static_cast<size_t>(std::max<int64_t>(nnz, 1));
    NTC_HIP(t.get(reinterpret_cast<void **>(&d_coords), n * N * 4));
    NTC_HIP(t.get(reinterpret_cast<void **>(&d_values), n * 4));
    NTC_HIP(t.get(reinterpret_cast<void **>(&keys_in), n * 4));
    NTC_HIP(t.get(reinterpret_cast<void **>(&keys_out), n * 4));
    NTC_HIP(t.get(reinterpret_cast<void **>(&ids_in), n * 4));
    NTC_HIP(t.get(reinterpret_cast<void **>(&ids_out), n * 4));
    NTC_HIP(t.get(reinterpret_cast<void **>(&bad), sizeof(unsigned long long)));
    NTC_HIP(t.get(reinterpret_cast<void **>(&d_rowptr), static_cast<size_t>(maxI + 1) * 8));
    NTC_HIP(ntc::csr_sort_bytes(nnz, &temp_bytes));
    NTC_HIP(t.get(&temp, temp_bytes));
    if (nnz > 0) {
        NTC_HIP(hipMemcpyAsync(d_coords, coords, static_cast<size_t>(nnz) * N * 4, hipMemcpyHostToDevice, st));
        NTC_HIP(hipMemcpyAsync(d_values, values, static_cast<size_t>(nnz) * 4, hipMemcpyHostToDevice, st));
    }
    // the first bad entry, reported with the host's message for it
    const unsigned long long none = ~0ull;
    NTC_HIP(hipMemcpyAsync(bad, &none, sizeof(none), hipMemcpyHostToDevice, st));
    ntc::CsrDims cd{};
    for (int m = 0; m < N; ++m)
        cd.d[m] = dims[m];
    NTC_HIP(ntc::csr_validate(d_coords, d_values, nnz, N, cd, bad, st));
    unsigned long long first = none;
    NTC_HIP(hipMemcpyAsync(&first, bad, sizeof(first), hipMemcpyDeviceToHost, st));
    NTC_HIP(hipStreamSynchronize(st));
    if (first != none)
        return check_entry(coords, values, N, dims, static_cast<int64_t>(first));
    const int rw = record_words(N);
    for (int m = 0; m < N; ++m) {
        ntc::CsrMode c{};
        c.coords = d_coords;
        c.values = d_values;
        c.nnz = nnz;
        c.nmodes = N;
        c.mode = m;
        c.I = dims[m];
        c.rw = rw;
        c.R = static_cast<uint32_t>(R);
        c.own_word = (m == 0 && N < rw) ? N : -1;
        c.keys_in = keys_in;
        c.keys_out = keys_out;
        c.ids_in = ids_in;
        c.ids_out = ids_out;
        c.temp = temp;
        c.temp_bytes = temp_bytes;
        c.rowptr = d_rowptr;
        NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&c.records), n * rw * 4, "records"));
        if (m == 0 && c.own_word < 0 && nnz > 0) {
            NTC_TRY(alloc_or_fail(h, reinterpret_cast<void **>(&c.row0), static_cast<size_t>(nnz) * 4, "loss rows"));
            q.dev_row0 = c.row0;
        }
        NTC_HIP(ntc::csr_mode(c, st));
        rowptr[m].resize(static_cast<size_t>(dims[m]) + 1);
        NTC_HIP(hipMemcpyAsync(rowptr[m].data(), d_rowptr, (dims[m] + 1) * 8, hipMemcpyDeviceToHost, st));
        NTC_HIP(hipStreamSynchronize(st));
        q.md[m].dev_rec = c.records;
    }
    return NTC_OK;
}

extern "C" {

void ntc_params_default(ntc_params *p)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof(*p));
    p->c = 0.1;
    p->lambda = 1e-3;
    p->max_inner = 1;
    p->power_iters = 20;
    p->tiny_max = -1;
    p->overlap = 1;
}

ntc_status ntc_create(ntc_handle *out, int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *coords,
                      const float *values, int32_t rank, const ntc_params *p)
{
    ntc::TraceRange range("ntc_create");
    if (!out)
        return fail(NTC_EINVAL, "out is null");
    *out = nullptr;
    ntc_params def;
    ntc_params_default(&def);
    ntc_problem *h = new (std::nothrow) ntc_problem();
    if (!h)
        return fail(NTC_ENOMEM, "host allocation failed");
    ntc_status s;
    try {
        ntc_prepared q;
        s = prepare_impl(&q, nmodes, dims, nnz, coords, values, rank, p ? *p : def);
        if (s == NTC_OK)
            s = commit_impl(h, q, p ? *p : def);
    } catch (const std::bad_alloc &) {
        s = fail(NTC_ENOMEM, "host allocation failed");
    }
    if (s != NTC_OK) {
        delete h;
        return s;
    }
    *out = h;
    return NTC_OK;
}

ntc_status ntc_create_device_csr(ntc_handle *out, int32_t nmodes, const int64_t *dims, int64_t nnz,
                                 const int32_t *coords, const float *values, int32_t rank, const ntc_params *p)
{
    ntc::TraceRange range("ntc_create_device_csr");
    if (!out)
        return fail(NTC_EINVAL, "out is null");
    *out = nullptr;
    ntc_params def;
    ntc_params_default(&def);
    const ntc_params &pp = p ? *p : def;
    NTC_TRY(check_params(nmodes, dims, nnz, coords, values, rank, pp));
    ntc_problem *h = new (std::nothrow) ntc_problem();
    if (!h)
        return fail(NTC_ENOMEM, "host allocation failed");
    // device memory the problem keeps goes through the caller's allocator, as in commit
    h->stream = static_cast<hipStream_t>(pp.stream);
    h->alloc = pp.dev_alloc;
    h->dfree = pp.dev_free;
    h->actx = pp.alloc_ctx;
    ntc_status s;
    try {
        ntc_prepared q;
        std::vector<int64_t> rowptr[ntc::kMaxModes];
        s = device_csr(h, q, rowptr, nmodes, dims, nnz, coords, values, rank);
        if (s == NTC_OK)
            s = prepare_impl(&q, nmodes, dims, nnz, coords, values, rank, pp, rowptr);
        if (s == NTC_OK)
            s = commit_impl(h, q, pp);
    } catch (const std::bad_alloc &) {
        s = fail(NTC_ENOMEM, "host allocation failed");
    }
    if (s != NTC_OK) {
        delete h;
        return s;
    }
    *out = h;
    return NTC_OK;
}

ntc_status ntc_prepare(ntc_prepared_handle *out, int32_t nmodes, const int64_t *dims, int64_t nnz,
                       const int32_t *coords, const float *values, int32_t rank, const ntc_params *p)
{
    ntc::TraceRange range("ntc_prepare");
    if (!out)
        return fail(NTC_EINVAL, "out is null");
    *out = nullptr;
    ntc_params def;
    ntc_params_default(&def);
    ntc_prepared *q = new (std::nothrow) ntc_prepared();
    if (!q)
        return fail(NTC_ENOMEM, "host allocation failed");
    ntc_status s;
    try {
        s = prepare_impl(q, nmodes, dims, nnz, coords, values, rank, p ? *p : def);
    } catch (const std::bad_alloc &) {
        s = fail(NTC_ENOMEM, "host allocation failed");
    }
    if (s != NTC_OK) {
        delete q;
        return s;
    }
    *out = q;
    return NTC_OK;
}

ntc_status ntc_prepared_schedule(ntc_prepared_handle q, int32_t mode, int64_t counts[7], int64_t *rowptr_out,
                                 int32_t *tiny_out, int32_t *items_out, int32_t *split_out, int32_t *groups_out)
{
    if (!q || !counts)
        return fail(NTC_EINVAL, "null argument");
    if (mode < 0 || mode >= q->N)
        return fail(NTC_EINVAL, "mode out of range");
    const ntc_prepared::Mode &pm = q->md[mode];
    const ModeState &md = pm.st;
    counts[0] = static_cast<int64_t>(pm.tiny.size());
    counts[1] = static_cast<int64_t>(pm.items.size());
    counts[2] = md.n_group;
    counts[3] = static_cast<int64_t>(pm.split.size());
    counts[4] = static_cast<int64_t>(pm.groups.size());
    counts[5] = md.n_slots;
    counts[6] = md.samples;
    if (rowptr_out)
        std::memcpy(rowptr_out, md.h_rowptr.data(), md.h_rowptr.size() * sizeof(int64_t));
    static_assert(sizeof(ntc::RowItem) == 16 && sizeof(Item) == 16 && sizeof(SplitRow) == 16 &&
                      sizeof(ntc::SlotGroup) == 16,
                  "schedule entries are four 32-bit words");
    if (tiny_out && !pm.tiny.empty())
        std::memcpy(tiny_out, pm.tiny.data(), pm.tiny.size() * 16);
    if (items_out && !pm.items.empty())
        std::memcpy(items_out, pm.items.data(), pm.items.size() * 16);
    if (split_out && !pm.split.empty())
        std::memcpy(split_out, pm.split.data(), pm.split.size() * 16);
    if (groups_out && !pm.groups.empty())
        std::memcpy(groups_out, pm.groups.data(), pm.groups.size() * 16);
    return NTC_OK;
}

ntc_status ntc_prepared_bytes(ntc_prepared_handle q, size_t *bytes)
{
    if (!q || !bytes)
        return fail(NTC_EINVAL, "null argument");
    auto up = [](int64_t b) { return static_cast<size_t>((std::max<int64_t>(b, 1) + 255) / 256 * 256); };
    const int64_t N = q->N, R = q->R, rp = q->RP;
    size_t t = 0;
    int64_t maxI = 0;
    for (int m = 0; m < N; ++m) {
        const ntc_prepared::Mode &pm = q->md[m];
        maxI = std::max(maxI, q->dims[m]);
        t += up((q->dims[m] + 1) * R * 4) + (q->bf16 ? up((q->dims[m] + 1) * R * 2) : 0);
        t += up((q->dims[m] + 1) * 8) + up(std::max<int64_t>(q->nnz, 1) * q->rw * 4);
        t += up(static_cast<int64_t>(pm.tiny.size() * sizeof(ntc::RowItem)));
        t += up(static_cast<int64_t>(pm.groups.size() * sizeof(ntc::SlotGroup)));
        t += up(static_cast<int64_t>(pm.items.size() * sizeof(Item)));
        t += up(static_cast<int64_t>(pm.split.size() * sizeof(SplitRow)));
    }
    if (q->max_inner > 1)
        t += up(maxI * R * 4);
    if (!q->row0.empty())
        t += up(q->nnz * 4);
    t += up(std::max<int64_t>(q->max_slots, 1) * (rp + rp * rp) * 8);
    const int64_t nt = std::max<int64_t>(static_cast<int64_t>(q->test_values.size()), 1);
    t += up(nt * N * 4) + up(nt * 4);
    t += up(4 * ntc::kLossBlocks * 8) + up(32) + up((q->max_row + 1) * 4) + up(8);
    t += up(N * q->max_inner * static_cast<int64_t>(sizeof(ntc::RowArgs)));
    *bytes = t;
    return NTC_OK;
}

ntc_status ntc_create_prepared(ntc_handle *out, ntc_prepared_handle q, const ntc_params *p)
{
    ntc::TraceRange range("ntc_create_prepared");
    if (!out || !q)
        return fail(NTC_EINVAL, "null argument");
    *out = nullptr;
    ntc_params def;
    ntc_params_default(&def);
    ntc_problem *h = new (std::nothrow) ntc_problem();
    if (!h)
        return fail(NTC_ENOMEM, "host allocation failed");
    ntc_status s;
    try {
        s = commit_impl(h, *q, p ? *p : def);
    } catch (const std::bad_alloc &) {
        s = fail(NTC_ENOMEM, "host allocation failed");
    }
    if (s != NTC_OK) {
        delete h;
        return s;
    }
    *out = h;
    return NTC_OK;
}

ntc_status ntc_prepared_release(ntc_prepared_handle q)
{
    delete q;
    return NTC_OK;
}

ntc_status ntc_sweep(ntc_handle h, int32_t nsweeps)
{
    ntc::TraceRange range("ntc_sweep");
    if (!h)
        return fail(NTC_EINVAL, "null handle");
    if (nsweeps < 0)
        return fail(NTC_EINVAL, "nsweeps must be >= 0");
    for (int32_t s = 0; s < nsweeps; ++s) {
        for (int m = 0; m < h->N; ++m)
            NTC_TRY(enqueue_mode(h, m));
        NTC_HIP(ntc::launch_advance(h->kdev, 1, h->stream));
        h->k += 1;
    }
    return NTC_OK;
}

ntc_status ntc_update_mode(ntc_handle h, int32_t mode)
{
    ntc::TraceRange range("ntc_update_mode");
    NTC_TRY(check_mode(h, mode));
    return enqueue_mode(h, mode);
}

ntc_status ntc_loss(ntc_handle h, double out[4])
{
    ntc::TraceRange range("ntc_loss");
    if (!h || !out)
        return fail(NTC_EINVAL, "null argument");
    ntc::LossArgs a{};
    a.records0 = h->md[0].records;
    a.row0 = h->row0;
    a.row_word = h->row_word;
    a.nnz = h->nnz;
    a.test_coords = h->test_coords;
    a.test_values = h->test_values;
    a.n_test = h->n_test;
    for (int m = 0; m < h->N; ++m) {
        a.U[m] = h->U[m];
        a.dims[m] = h->dims[m];
    }
    a.nmodes = h->N;
    a.rec_words = h->rw;
    a.R = h->R;
    a.part = h->loss_part;
    a.out = h->loss_out;
    NTC_HIP(ntc::launch_loss(a, h->stream));
    double s[4];
    NTC_HIP(hipMemcpyAsync(s, h->loss_out, sizeof(s), hipMemcpyDeviceToHost, h->stream));
    NTC_TRY(sync(h));
    out[0] = 0.5 * s[0] + 0.5 * h->lambda * s[3];
    out[1] = h->nnz > 0 ? std::sqrt(s[0] / static_cast<double>(h->nnz)) : 0.0;
    out[2] = h->n_test > 0 ? std::sqrt(s[1] / static_cast<double>(h->n_test)) : 0.0;
    out[3] = (h->n_test > 0 && s[2] > 0.0) ? std::sqrt(s[1]) / std::sqrt(s[2]) : 0.0;
    for (int q = 0; q < 4; ++q)
        if (!std::isfinite(out[q]))
            return fail(NTC_ENONFINITE, "loss is not finite");
    return NTC_OK;
}

ntc_status ntc_loss_coo_noalloc(int32_t nmodes, const int64_t *dims, int32_t rank, int64_t n_train,
                                const int32_t *train_coords, const float *train_values, int64_t n_test,
                                const int32_t *test_coords, const float *test_values, const float *const *factors,
                                double lambda, double *out, void *stream)
{
    if (nmodes < 2 || nmodes > ntc::kMaxModes)
        return fail(NTC_EINVAL, "nmodes must be in [2, 8]");
    if (rank < 1 || rank > ntc::kMaxRank)
        return fail(NTC_EINVAL, "rank must be in [1, 64]");
    if (!dims || !factors || !out)
        return fail(NTC_EINVAL, "null argument");
    if (n_train < 0 || n_test < 0)
        return fail(NTC_EINVAL, "entry counts must be >= 0");
    if (n_train >= (int64_t(1) << 31) || n_test >= (int64_t(1) << 31))
        return fail(NTC_EUNSUPPORTED, "at most 2^31 - 1 entries per set");
    if ((n_train > 0 && (!train_coords || !train_values)) || (n_test > 0 && (!test_coords || !test_values)))
        return fail(NTC_EINVAL, "null entry arrays for a nonempty set");
    if (!(lambda >= 0.0) || !std::isfinite(lambda))
        return fail(NTC_EINVAL, "lambda must be finite and >= 0");
    ntc::LossArgs tr{}, te{};
    for (int m = 0; m < nmodes; ++m) {
        if (dims[m] < 1)
            return fail(NTC_EINVAL, "dims must be >= 1");
        // row offsets coordinate * R are 32-bit in the kernels
        if (dims[m] * static_cast<int64_t>(rank) > (int64_t(1) << 32) - 1)
            return fail(NTC_EUNSUPPORTED, "dims[m] * rank must be below 2^32");
        if (!factors[m])
            return fail(NTC_EINVAL, "null factor pointer");
        tr.U[m] = te.U[m] = factors[m];
        tr.dims[m] = te.dims[m] = dims[m];
    }
    tr.nmodes = te.nmodes = nmodes;
    tr.R = te.R = rank;
    tr.test_coords = train_coords;
    tr.test_values = train_values;
    tr.n_test = n_train;
    te.test_coords = test_coords;
    te.test_values = test_values;
    te.n_test = n_test;
    NTC_HIP(ntc::launch_loss_coo_noalloc(tr, te, lambda, out, static_cast<hipStream_t>(stream)));
    return NTC_OK;
}

ntc_status ntc_get_factors(ntc_handle h, int32_t mode, float *host_out)
{
    NTC_TRY(check_mode(h, mode));
    if (!host_out)
        return fail(NTC_EINVAL, "host_out is null");
    NTC_HIP(hipMemcpyAsync(host_out, h->U[mode], h->dims[mode] * h->R * sizeof(float), hipMemcpyDeviceToHost,
                           h->stream));
    return sync(h);
}

ntc_status ntc_set_factors(ntc_handle h, int32_t mode, const float *host_in)
{
    NTC_TRY(check_mode(h, mode));
    if (!host_in)
        return fail(NTC_EINVAL, "host_in is null");
    NTC_TRY(validate_factor(host_in, h->dims[mode] * h->R, mode));
    NTC_TRY(sync(h));
    NTC_HIP(hipMemcpy(h->U[mode], host_in, h->dims[mode] * h->R * sizeof(float), hipMemcpyHostToDevice));
    if (h->bf16)
        NTC_HIP(ntc::launch_to_bf16(h->U[mode], h->U16[mode], h->dims[mode] * h->R, h->stream));
    return sync(h);
}

ntc_status ntc_get_factors_device(ntc_handle h, int32_t mode, float *dev_out)
{
    NTC_TRY(check_mode(h, mode));
    if (!dev_out)
        return fail(NTC_EINVAL, "dev_out is null");
    NTC_HIP(hipMemcpyAsync(dev_out, h->U[mode], h->dims[mode] * h->R * sizeof(float), hipMemcpyDeviceToDevice,
                           h->stream));
    return NTC_OK;
}

ntc_status ntc_get_sweep(ntc_handle h, int64_t *k)
{
    if (!h || !k)
        return fail(NTC_EINVAL, "null argument");
    *k = h->k;
    return NTC_OK;
}

ntc_status ntc_set_sweep(ntc_handle h, int64_t k)
{
    if (!h)
        return fail(NTC_EINVAL, "null handle");
    if (k < 0)
        return fail(NTC_EINVAL, "k must be >= 0");
    NTC_TRY(sync(h));
    NTC_HIP(hipMemcpy(h->kdev, &k, sizeof(int64_t), hipMemcpyHostToDevice));
    h->k = k;
    return NTC_OK;
}

ntc_status ntc_get_work(ntc_handle h, int64_t *updates_per_sweep, int64_t *row_steps_per_sweep)
{
    if (!h)
        return fail(NTC_EINVAL, "null handle");
    int64_t u = 0, r = 0;
    for (int m = 0; m < h->N; ++m) {
        u += h->md[m].samples * h->max_inner;
        r += h->md[m].active_rows * h->max_inner;
    }
    if (updates_per_sweep)
        *updates_per_sweep = u;
    if (row_steps_per_sweep)
        *row_steps_per_sweep = r;
    return NTC_OK;
}

ntc_status ntc_debug_sample(ntc_handle h, int64_t k, int32_t mode, int32_t l, int64_t row, int32_t *pos_out,
                            int32_t *count)
{
    NTC_TRY(check_mode(h, mode));
    if (!pos_out || !count)
        return fail(NTC_EINVAL, "null argument");
    if (row < 0 || row >= h->dims[mode])
        return fail(NTC_EINVAL, "row out of range");
    if (l < 0 || l > 0xFFFF)
        return fail(NTC_EINVAL, "l out of range");
    NTC_HIP(ntc::launch_debug_sample(h->md[mode].rowptr, row, h->seed, k, mode, l, h->c, h->dbg + 1, h->dbg,
                                     h->stream));
    int32_t cnt = 0;
    NTC_HIP(hipMemcpyAsync(&cnt, h->dbg, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    NTC_TRY(sync(h));
    if (cnt > 0) {
        NTC_HIP(hipMemcpyAsync(pos_out, h->dbg + 1, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        NTC_TRY(sync(h));
    }
    *count = cnt;
    return NTC_OK;
}

ntc_status ntc_debug_csr(ntc_handle h, int32_t mode, int64_t *rowptr_out, uint32_t *records_out)
{
    NTC_TRY(check_mode(h, mode));
    if (!rowptr_out || (h->nnz > 0 && !records_out))
        return fail(NTC_EINVAL, "null argument");
    NTC_HIP(hipMemcpyAsync(rowptr_out, h->md[mode].rowptr, (h->dims[mode] + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToHost, h->stream));
    if (h->nnz > 0)
        NTC_HIP(hipMemcpyAsync(records_out, h->md[mode].records,
                               static_cast<size_t>(h->nnz) * h->rw * sizeof(uint32_t), hipMemcpyDeviceToHost,
                               h->stream));
    return sync(h);
}

ntc_status ntc_host_sample(uint64_t seed, int64_t k, int32_t mode, int32_t l, int64_t row, int64_t n, double c,
                           int32_t *pos_out, int64_t *count)
{
    if (!count || n < 0 || n >= (int64_t(1) << 31) || !(c > 0.0 && c <= 1.0))
        return fail(NTC_EINVAL, "invalid argument");
    const int64_t b = ntc::minibatch_size(c, n);
    if (b > 0 && !pos_out)
        return fail(NTC_EINVAL, "pos_out is null");
    if (b > 0) {
        const ntc::Prp prp = ntc::make_prp(static_cast<uint32_t>(n), ntc::sample_keys(seed, k, mode, l, row));
        for (int64_t j = 0; j < b; ++j)
            pos_out[j] = static_cast<int32_t>(ntc::prp_index(prp, static_cast<uint32_t>(j)));
    }
    *count = b;
    return NTC_OK;
}

ntc_status ntc_host_csr(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *coords, int32_t mode,
                        int64_t *rowptr_out, int64_t *perm_out)
{
    if (nmodes < 2 || nmodes > ntc::kMaxModes || !dims || mode < 0 || mode >= nmodes || nnz < 0 ||
        (nnz > 0 && !coords) || !rowptr_out)
        return fail(NTC_EINVAL, "invalid argument");
    for (int64_t e = 0; e < nnz; ++e)
        for (int m = 0; m < nmodes; ++m)
            if (coords[e * nmodes + m] < 0 || coords[e * nmodes + m] >= dims[m])
                return fail(NTC_EINVAL, "coordinate out of range");
    std::vector<int64_t> rp;
    csr_build(nmodes, dims, nnz, coords, nullptr, mode, record_words(nmodes), rp, nullptr, perm_out);
    std::memcpy(rowptr_out, rp.data(), rp.size() * sizeof(int64_t));
    return NTC_OK;
}

ntc_status ntc_synchronize(ntc_handle h)
{
    if (!h)
        return fail(NTC_EINVAL, "null handle");
    return sync(h);
}

ntc_status ntc_time_sweeps(ntc_handle h, int32_t nsweeps, double *ms)
{
    if (!h || !ms)
        return fail(NTC_EINVAL, "null argument");
    hipEvent_t e0, e1;
    NTC_HIP(hipEventCreate(&e0));
    NTC_HIP(hipEventCreate(&e1));
    NTC_HIP(hipEventRecord(e0, h->stream));
    ntc_status s = ntc_sweep(h, nsweeps);
    if (s != NTC_OK)
        return s;
    NTC_HIP(hipEventRecord(e1, h->stream));
    NTC_HIP(hipEventSynchronize(e1));
    float t = 0.0f;
    NTC_HIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t;
    return NTC_OK;
}

ntc_status ntc_profile_sweep(ntc_handle h, ntc_launch_record *out, int32_t cap, int32_t *count)
{
    return ntc_profile_sweeps(h, 1, 0, out, cap, count);
}

ntc_status ntc_profile_sweeps(ntc_handle h, int32_t nsweeps, int32_t concurrent, ntc_launch_record *out,
                              int32_t cap, int32_t *count)
{
    ntc::TraceRange range("ntc_profile_sweeps");
    if (!h || !count || (cap > 0 && !out))
        return fail(NTC_EINVAL, "null argument");
    if (nsweeps < 0)
        return fail(NTC_EINVAL, "nsweeps must be >= 0");
    LaunchProbe probe;
    probe.concurrent = concurrent != 0;
    ntc_status s = NTC_OK;
    for (int32_t k = 0; k < nsweeps && s == NTC_OK; ++k) {
        for (int m = 0; m < h->N && s == NTC_OK; ++m)
            s = enqueue_mode(h, m, &probe);
        if (s == NTC_OK) {
            if (ntc::launch_advance(h->kdev, 1, h->stream) != hipSuccess)
                s = fail(NTC_EDEVICE, "launch of the sweep-counter update failed");
            h->k += 1;
        }
    }
    hipError_t se = hipStreamSynchronize(h->stream);
    if (se == hipSuccess && h->side)
        se = hipStreamSynchronize(h->side);
    for (size_t i = 0; i < probe.rec.size(); ++i) {
        float t = 0.0f;
        if (se == hipSuccess && hipEventElapsedTime(&t, probe.ev[2 * i], probe.ev[2 * i + 1]) == hipSuccess)
            probe.rec[i].ms = t;
        if (static_cast<int32_t>(i) < cap)
            out[i] = probe.rec[i];
    }
    for (hipEvent_t e : probe.ev)
        (void)hipEventDestroy(e);
    if (s != NTC_OK)
        return s;
    NTC_HIP(se);
    *count = static_cast<int32_t>(probe.rec.size());
    return NTC_OK;
}

ntc_status ntc_estimate_bytes(int32_t nmodes, const int64_t *dims, int64_t nnz, int32_t rank, const ntc_params *p,
                              size_t *bytes)
{
    if (!dims || !bytes)
        return fail(NTC_EINVAL, "null argument");
    if (nmodes < 2 || nmodes > ntc::kMaxModes || rank < 1 || rank > ntc::kMaxRank || nnz < 0)
        return fail(NTC_EINVAL, "nmodes, rank or nnz out of range");
    ntc_params def;
    ntc_params_default(&def);
    const ntc_params &q = p ? *p : def;
    const int64_t N = nmodes, R = rank, rp = padded_rank(rank), rw = record_words(nmodes);
    const int64_t smax = q.item_samples > 0 ? q.item_samples : item_samples(static_cast<int>(rp), nmodes);
    const double c = (q.c > 0.0 && q.c <= 1.0) ? q.c : 1.0;
    const int64_t inner = std::max<int32_t>(q.max_inner, 1);
    auto up = [](int64_t b) { return static_cast<size_t>((std::max<int64_t>(b, 1) + 255) / 256 * 256); };
    // partial slots of one mode: a split row of B_p > smax samples takes
    // ceil(B_p / smax) < 2 B_p / smax of them, its slot groups fewer again
    const int64_t slots = 2 * static_cast<int64_t>(std::ceil(c * static_cast<double>(nnz) / smax)) + 1;
    size_t t = 0;
    int64_t maxI = 0;
    for (int m = 0; m < nmodes; ++m) {
        if (dims[m] < 1)
            return fail(NTC_EINVAL, "dims must be >= 1");
        maxI = std::max(maxI, dims[m]);
        t += up((dims[m] + 1) * R * 4);
        if (q.gather_bf16)
            t += up((dims[m] + 1) * R * 2);
        t += up((dims[m] + 1) * 8);                                   // rowptr
        t += up(nnz * rw * 4);                                        // records
        t += up(dims[m] * 16);                                        // rows of a few samples
        t += up((dims[m] + nnz / smax + 1) * 16);                     // work items
        t += up(dims[m] * 16);                                        // split rows
        t += up(slots * 16);                                          // slot groups
    }
    if (inner > 1)
        t += up((maxI + 1) * R * 4);
    if (N >= rw)
        t += up(nnz * 4);                                             // loss rows
    t += up(slots * (rp + rp * rp) * 8);
    const int64_t nt = std::max<int64_t>(q.n_test, 1);
    t += up(nt * N * 4) + up(nt * 4);
    t += up(4 * ntc::kLossBlocks * 8) + up(32) + up((nnz + 1) * 4) + up(8);
    t += up(N * inner * static_cast<int64_t>(sizeof(ntc::RowArgs)));
    *bytes = t;
    return NTC_OK;
}

ntc_status ntc_release(ntc_handle h)
{
    delete h;
    return NTC_OK;
}

const char *ntc_last_error(void)
{
    return g_last_error.c_str();
}

const char *ntc_version(void)
{
    return "libntc 0.1 (gfx950)";
}

}  // extern "C"
