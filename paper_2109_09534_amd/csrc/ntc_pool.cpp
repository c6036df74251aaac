// Batching and serving form of libntc: many independent problems share one
// device memory arena, and each pool sweep runs Alg. 2 once for all running
// problems with one launch per (mode, inner step, row kernel, kernel family).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "ntc.h"
#include "ntc_aux.h"
#include "ntc_internal.h"
#include "ntc_problem.h"

namespace {

ntc_status fail(ntc_status s, const std::string &msg)
{
    return ntc::set_error(s, msg);
}

#define POOL_HIP(expr)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            return fail(NTC_EDEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_));         \
    } while (0)

#define POOL_TRY(expr)              \
    do {                            \
        ntc_status s_ = (expr);     \
        if (s_ != NTC_OK)           \
            return s_;              \
    } while (0)

constexpr size_t kAlign = 256;

// First-fit allocator over one device allocation; free blocks are kept
// sorted by offset and coalesced on release.
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    std::map<size_t, size_t> free_blocks;          // offset -> size
    std::unordered_map<size_t, size_t> live;       // offset -> size

    void reset(char *b, size_t c)
    {
        base = b;
        cap = c;
        used = 0;
        free_blocks.clear();
        live.clear();
        if (c > 0)
            free_blocks[0] = c;
    }

    void *alloc(size_t bytes)
    {
        bytes = (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < bytes)
                continue;
            const size_t off = it->first, size = it->second;
            free_blocks.erase(it);
            if (size > bytes)
                free_blocks[off + bytes] = size - bytes;
            live[off] = bytes;
            used += bytes;
            return base + off;
        }
        return nullptr;
    }

    void release(void *p)
    {
        if (!p)
            return;
        const size_t off = static_cast<size_t>(static_cast<char *>(p) - base);
        auto lv = live.find(off);
        if (lv == live.end())
            return;
        size_t start = off, size = lv->second;
        live.erase(lv);
        used -= size;
        auto next = free_blocks.lower_bound(start);
        if (next != free_blocks.end() && next->first == start + size) {
            size += next->second;
            next = free_blocks.erase(next);
        }
        if (next != free_blocks.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                size += prev->second;
                free_blocks.erase(prev);
            }
        }
        free_blocks[start] = size;
    }

    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &kv : free_blocks)
            m = std::max(m, kv.second);
        return m;
    }
};

void *arena_alloc(size_t bytes, void *, void *ctx)
{
    return static_cast<Arena *>(ctx)->alloc(bytes);
}

void arena_free(void *p, void *ctx)
{
    static_cast<Arena *>(ctx)->release(p);
}

struct Slot {
    ntc_handle h = nullptr;
    int32_t state = NTC_SLOT_FREE;
    int64_t sweeps = 0;        // host copy of the device count
    double rmse = 0.0;         // last held-out RMSE (NaN without a held-out set)
    ntc::ProblemView view{};
};

struct PoolLaunch {
    ntc::RowKernel kind;
    ntc::KernelClass kc;
    ntc::Launch L;
};

}  // namespace

struct ntc_pool {
    ntc_pool_params p{};
    hipStream_t stream = nullptr;
    bool own_stream = false;  // created by the pool (graph capture needs a non-null stream)
    char *arena_mem = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    int64_t sweeps = 0;

    // launch tables of the current set of running slots (rebuilt when it changes)
    bool dirty = true;
    char *tab = nullptr;
    size_t tab_cap = 0;
    std::vector<PoolLaunch> launches;
    ntc::PoolRuleArgs rule{};
    int32_t n_run = 0;
    const ntc::LossArgs *t_args = nullptr;
    const int32_t *t_start = nullptr;
    const int32_t *t_owner = nullptr;
    int32_t n_t = 0, t_blocks = 0;
    std::vector<int32_t> t_slot;  // test entry -> slot
    double *t_part = nullptr;     // [2 * kMaxTestBlocks * max_slots]
    double *t_out = nullptr;      // [2 * max_slots]
    // device state of the stop rule, per slot, and its pinned host copy
    int32_t *st_stop = nullptr;
    int64_t *st_sweeps = nullptr;
    int64_t *st_nhist = nullptr;
    double *st_hist = nullptr;    // [slots][window + 1]
    double *st_last = nullptr;
    char *st_host = nullptr;      // sweeps | last | stop, copied back after each step

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~ntc_pool()
    {
        if (stream)
            (void)hipStreamSynchronize(stream);
        else
            (void)hipDeviceSynchronize();
        for (Slot &s : slots)
            if (s.h)
                (void)ntc_release(s.h);
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (graph)
            (void)hipGraphDestroy(graph);
        if (tab)
            (void)hipFree(tab);
        if (t_part)
            (void)hipFree(t_part);
        if (t_out)
            (void)hipFree(t_out);
        for (void *q : {static_cast<void *>(st_stop), static_cast<void *>(st_sweeps), static_cast<void *>(st_nhist),
                        static_cast<void *>(st_hist), static_cast<void *>(st_last)})
            if (q)
                (void)hipFree(q);
        if (st_host)
            (void)hipHostFree(st_host);
        if (arena_mem)
            (void)hipFree(arena_mem);
        if (own_stream && stream)
            (void)hipStreamDestroy(stream);
    }
};

namespace {

ntc_status check_slot(ntc_pool *pool, int32_t slot)
{
    if (!pool)
        return fail(NTC_EINVAL, "null pool");
    if (slot < 0 || slot >= static_cast<int32_t>(pool->slots.size()))
        return fail(NTC_EINVAL, "slot out of range");
    return NTC_OK;
}

void drop_graph(ntc_pool *pool)
{
    if (pool->exec)
        (void)hipGraphExecDestroy(pool->exec);
    if (pool->graph)
        (void)hipGraphDestroy(pool->graph);
    pool->exec = nullptr;
    pool->graph = nullptr;
}

// Host image of the device tables, appended with 256-byte alignment.
struct TableImage {
    std::vector<char> bytes;
    size_t put(const void *src, size_t n)
    {
        const size_t off = (bytes.size() + kAlign - 1) / kAlign * kAlign;
        bytes.resize(off + std::max<size_t>(n, 1));
        if (n)
            std::memcpy(bytes.data() + off, src, n);
        return off;
    }
};

bool same_class(const ntc::KernelClass &a, const ntc::KernelClass &b)
{
    return a.rp == b.rp && a.nmodes == b.nmodes && a.bf16 == b.bf16 && a.pairs == b.pairs && a.nt == b.nt;
}

// Launch tables of the running slots: per (mode, inner step), per kernel
// family, per row kernel, one Launch over every problem with work for it.
ntc_status rebuild(ntc_pool *pool)
{
    // nothing may still read the old graph or tables
    POOL_HIP(hipStreamSynchronize(pool->stream));
    drop_graph(pool);
    pool->launches.clear();
    std::vector<int32_t> run;
    for (int32_t i = 0; i < static_cast<int32_t>(pool->slots.size()); ++i)
        if (pool->slots[i].state == NTC_SLOT_RUNNING)
            run.push_back(i);
    std::vector<ntc::KernelClass> classes;
    int maxN = 0, maxL = 0;
    for (int32_t i : run) {
        const ntc::ProblemView &v = pool->slots[i].view;
        maxN = std::max(maxN, v.nmodes);
        maxL = std::max(maxL, v.max_inner);
        bool seen = false;
        for (const auto &c : classes)
            seen = seen || same_class(c, v.kc);
        if (!seen)
            classes.push_back(v.kc);
    }

    struct Pending {
        ntc::RowKernel kind;
        ntc::KernelClass kc;
        size_t args, start, owner;
        int32_t n, blocks;
    };
    std::vector<Pending> pend;
    TableImage img;
    const ntc::RowKernel order[6] = {ntc::kTiny, ntc::kFew, ntc::kChunks, ntc::kRows, ntc::kReduce, ntc::kFinalize};
    for (int m = 0; m < maxN; ++m) {
        for (int l = 0; l < maxL; ++l) {
            for (const auto &kc : classes) {
                for (ntc::RowKernel kind : order) {
                    std::vector<ntc::RowArgs> args;
                    std::vector<int32_t> start, owner;
                    int32_t blocks = 0;
                    for (int32_t i : run) {
                        const ntc::ProblemView &v = pool->slots[i].view;
                        if (!same_class(v.kc, kc) || m >= v.nmodes || l >= v.max_inner)
                            continue;
                        const int32_t b = v.blocks[m][kind];
                        if (b <= 0)
                            continue;
                        ntc::RowArgs ra = v.args_host[m * v.max_inner + l];
                        ra.stop = pool->st_stop + i;
                        args.push_back(ra);
                        start.push_back(blocks);
                        owner.insert(owner.end(), static_cast<size_t>(b), static_cast<int32_t>(args.size() - 1));
                        blocks += b;
                    }
                    if (args.empty())
                        continue;
                    Pending pd{kind, kc, 0, 0, 0, static_cast<int32_t>(args.size()), blocks};
                    pd.args = img.put(args.data(), args.size() * sizeof(ntc::RowArgs));
                    pd.start = img.put(start.data(), start.size() * sizeof(int32_t));
                    pd.owner = img.put(owner.data(), owner.size() * sizeof(int32_t));
                    pend.push_back(pd);
                }
            }
        }
    }
    // held-out sums for the stop rule, and the rule's per-problem tables
    std::vector<ntc::LossArgs> targs;
    std::vector<int32_t> tstart, towner, rslot, rtidx;
    std::vector<int64_t *> kp;
    std::vector<int64_t> rntest;
    pool->t_slot.clear();
    int32_t tb = 0;
    for (int32_t i : run) {
        const ntc::ProblemView &v = pool->slots[i].view;
        rslot.push_back(i);
        kp.push_back(v.kdev);
        rntest.push_back(v.n_test);
        if (v.n_test <= 0) {
            rtidx.push_back(-1);
            continue;
        }
        rtidx.push_back(static_cast<int32_t>(targs.size()));
        ntc::LossArgs a{};
        a.test_coords = v.test_coords;
        a.test_values = v.test_values;
        a.n_test = v.n_test;
        for (int m = 0; m < v.nmodes; ++m)
            a.U[m] = v.U[m];
        a.nmodes = v.nmodes;
        a.R = v.rank;
        targs.push_back(a);
        tstart.push_back(tb);
        const int32_t nb = ntc::test_blocks(v.n_test, v.rank);
        towner.insert(towner.end(), static_cast<size_t>(nb), static_cast<int32_t>(targs.size() - 1));
        tb += nb;
        pool->t_slot.push_back(i);
    }
    tstart.push_back(tb);
    const size_t rs_off = img.put(rslot.data(), rslot.size() * sizeof(int32_t));
    const size_t rk_off = img.put(kp.data(), kp.size() * sizeof(int64_t *));
    const size_t rt_off = img.put(rtidx.data(), rtidx.size() * sizeof(int32_t));
    const size_t rn_off = img.put(rntest.data(), rntest.size() * sizeof(int64_t));
    const size_t ta_off = img.put(targs.data(), targs.size() * sizeof(ntc::LossArgs));
    const size_t ts_off = img.put(tstart.data(), tstart.size() * sizeof(int32_t));
    const size_t to_off = img.put(towner.data(), towner.size() * sizeof(int32_t));

    if (img.bytes.size() > pool->tab_cap) {
        if (pool->tab)
            POOL_HIP(hipFree(pool->tab));
        pool->tab = nullptr;
        pool->tab_cap = 0;
        const size_t cap = std::max<size_t>(img.bytes.size() * 3 / 2, 1 << 16);
        POOL_HIP(hipMalloc(reinterpret_cast<void **>(&pool->tab), cap));
        pool->tab_cap = cap;
    }
    POOL_HIP(hipMemcpy(pool->tab, img.bytes.data(), img.bytes.size(), hipMemcpyHostToDevice));
    char *base = pool->tab;
    for (const Pending &pd : pend) {
        PoolLaunch pl{pd.kind, pd.kc, {}};
        pl.L.args = reinterpret_cast<const ntc::RowArgs *>(base + pd.args);
        pl.L.start = reinterpret_cast<const int32_t *>(base + pd.start);
        pl.L.owner = reinterpret_cast<const int32_t *>(base + pd.owner);
        pl.L.n = pd.n;
        pl.L.blocks = pd.blocks;
        pool->launches.push_back(pl);
    }
    ntc::PoolRuleArgs &r = pool->rule;
    r.n = static_cast<int32_t>(rslot.size());
    r.slot = reinterpret_cast<const int32_t *>(base + rs_off);
    r.kdev = reinterpret_cast<int64_t *const *>(base + rk_off);
    r.tidx = reinterpret_cast<const int32_t *>(base + rt_off);
    r.n_test = reinterpret_cast<const int64_t *>(base + rn_off);
    r.test_out = pool->t_out;
    r.stop = pool->st_stop;
    r.sweeps = pool->st_sweeps;
    r.nhist = pool->st_nhist;
    r.hist = pool->st_hist;
    r.last = pool->st_last;
    r.window = pool->p.window;
    r.max_sweeps = pool->p.max_sweeps;
    r.tol = pool->p.tol;
    pool->n_run = r.n;
    pool->t_args = reinterpret_cast<const ntc::LossArgs *>(base + ta_off);
    pool->t_start = reinterpret_cast<const int32_t *>(base + ts_off);
    pool->t_owner = reinterpret_cast<const int32_t *>(base + to_off);
    pool->n_t = static_cast<int32_t>(targs.size());
    pool->t_blocks = tb;
    pool->dirty = false;
    return NTC_OK;
}

// One pool sweep: every row launch in (mode, inner step) order (problems
// that have stopped leave at once), the held-out sums, then the stop rule,
// which also advances the sweep counters of the problems still running.
ntc_status enqueue_sweep(ntc_pool *pool)
{
    for (const PoolLaunch &pl : pool->launches)
        POOL_HIP(ntc::launch_row_kernel(pl.kind, pl.kc, pl.L, pool->stream));
    POOL_HIP(ntc::launch_test_sums(pool->t_args, pool->t_start, pool->t_owner, pool->n_t, pool->t_blocks,
                                   pool->t_part, pool->t_out, pool->stream));
    POOL_HIP(ntc::launch_pool_rule(pool->rule, pool->stream));
    return NTC_OK;
}

ntc_status capture(ntc_pool *pool)
{
    POOL_HIP(hipStreamBeginCapture(pool->stream, hipStreamCaptureModeThreadLocal));
    const ntc_status s = enqueue_sweep(pool);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(pool->stream, &g);
    if (s != NTC_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return s;
    }
    POOL_HIP(e);
    pool->graph = g;
    POOL_HIP(hipGraphInstantiate(&pool->exec, pool->graph, nullptr, nullptr, 0));
    return NTC_OK;
}

}  // namespace

extern "C" {

void ntc_pool_params_default(ntc_pool_params *p)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof(*p));
    p->max_slots = 1024;
    p->use_graph = 1;
    p->window = 5;
    p->max_sweeps = 500;
    p->tol = 1e-4;
}

ntc_status ntc_pool_create(ntc_pool_handle *out, const ntc_pool_params *p)
{
    if (!out)
        return fail(NTC_EINVAL, "out is null");
    *out = nullptr;
    ntc_pool_params def;
    ntc_pool_params_default(&def);
    const ntc_pool_params &q = p ? *p : def;
    if (q.max_slots < 1 || q.max_slots > 65536)
        return fail(NTC_EINVAL, "max_slots must be in [1, 65536]");
    if (q.window < 0 || q.max_sweeps < 1 || !(q.tol >= 0.0))
        return fail(NTC_EINVAL, "window >= 0, max_sweeps >= 1 and tol >= 0 are required");
    ntc_pool *pool = new (std::nothrow) ntc_pool();
    if (!pool)
        return fail(NTC_ENOMEM, "host allocation failed");
    pool->p = q;
    pool->stream = static_cast<hipStream_t>(q.stream);
    if (!pool->stream) {
        if (hipStreamCreateWithFlags(&pool->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            pool->stream = nullptr;
            delete pool;
            return fail(NTC_EDEVICE, "stream creation failed");
        }
        pool->own_stream = true;
    }
    pool->slots.resize(static_cast<size_t>(q.max_slots));
    size_t cap = q.arena_bytes;
    if (cap == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete pool;
            return fail(NTC_EDEVICE, "hipMemGetInfo failed");
        }
        cap = fr / 4 * 3;
    }
    cap = cap / kAlign * kAlign;
    if (cap < kAlign) {
        delete pool;
        return fail(NTC_EINVAL, "arena_bytes too small");
    }
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&pool->arena_mem), cap);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        pool->arena_mem = nullptr;
        delete pool;
        return fail(NTC_ENOMEM, "arena allocation of " + std::to_string(cap) + " bytes failed");
    }
    pool->arena.reset(pool->arena_mem, cap);
    const size_t ms = static_cast<size_t>(q.max_slots);
    const size_t W1 = static_cast<size_t>(q.window) + 1;
    const size_t part_bytes = ms * ntc::kMaxTestBlocks * 2 * sizeof(double);
    if (hipMalloc(reinterpret_cast<void **>(&pool->t_part), part_bytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&pool->t_out), ms * 2 * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&pool->st_stop), ms * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&pool->st_sweeps), ms * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&pool->st_nhist), ms * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&pool->st_hist), ms * W1 * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&pool->st_last), ms * sizeof(double)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&pool->st_host), ms * (4 + 8 + 8), 0) != hipSuccess) {
        (void)hipGetLastError();
        delete pool;
        return fail(NTC_ENOMEM, "pool buffers");
    }
    *out = pool;
    return NTC_OK;
}

namespace {

int32_t free_slot_of(const ntc_pool *pool)
{
    for (int32_t i = 0; i < static_cast<int32_t>(pool->slots.size()); ++i)
        if (pool->slots[i].state == NTC_SLOT_FREE)
            return i;
    return -1;
}

// Device half of an admission: the prepared problem goes into the arena and
// a free slot, with the stop-rule state of sweep 0.
ntc_status register_slot(ntc_pool *pool, ntc_handle h, int32_t free_slot, int32_t *slot);
void pool_params(ntc_pool *pool, ntc_params *q);

ntc_status admit_prepared(ntc_pool *pool, ntc_prepared_handle prep, int32_t *slot)
{
    *slot = -1;
    const int32_t free_slot = free_slot_of(pool);
    if (free_slot < 0)
        return fail(NTC_ENOMEM, "no free slot");
    size_t need = 0;
    POOL_TRY(ntc_prepared_bytes(prep, &need));
    if (need > pool->arena.largest_free())
        return fail(NTC_ENOMEM, "arena cannot hold the problem now (" + std::to_string(need) + " bytes needed, " +
                                    std::to_string(pool->arena.largest_free()) + " in the largest free block)");
    ntc_params q;
    ntc_params_default(&q);
    pool_params(pool, &q);
    ntc_handle h = nullptr;
    POOL_TRY(ntc_create_prepared(&h, prep, &q));
    return register_slot(pool, h, free_slot, slot);
}

// The pool's settings for a problem's device memory and stream.
void pool_params(ntc_pool *pool, ntc_params *q)
{
    q->stream = pool->stream;
    q->dev_alloc = arena_alloc;
    q->dev_free = arena_free;
    q->alloc_ctx = &pool->arena;
    q->overlap = 0;
}

// Put a created problem into free slot `free_slot`: its held-out RMSE at
// admission opens the stop rule's history.  On failure the problem is
// released and the slot stays free.
ntc_status register_slot(ntc_pool *pool, ntc_handle h, int32_t free_slot, int32_t *slot)
{
    Slot &s = pool->slots[free_slot];
    s = Slot{};
    s.h = h;
    ntc_status st = ntc::problem_view(h, &s.view);
    double loss[4] = {0, 0, 0, 0};
    if (st == NTC_OK && s.view.n_test > 0)
        st = ntc_loss(h, loss);
    if (st != NTC_OK) {
        (void)ntc_release(h);
        s = Slot{};
        return st;
    }
    s.rmse = s.view.n_test > 0 ? loss[2] : std::numeric_limits<double>::quiet_NaN();
    {
        const int32_t zero = 0;
        const int64_t zero64 = 0, nh = s.view.n_test > 0 ? 1 : 0;
        hipError_t e = hipMemcpy(pool->st_stop + free_slot, &zero, sizeof(zero), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pool->st_sweeps + free_slot, &zero64, sizeof(zero64), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pool->st_nhist + free_slot, &nh, sizeof(nh), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pool->st_hist + static_cast<size_t>(free_slot) * (pool->p.window + 1), &s.rmse,
                          sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pool->st_last + free_slot, &s.rmse, sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)ntc_release(h);
            s = Slot{};
            return fail(NTC_EDEVICE, std::string("pool state upload failed: ") + hipGetErrorString(e));
        }
    }
    s.state = NTC_SLOT_RUNNING;
    pool->dirty = true;
    *slot = free_slot;
    return NTC_OK;
}

}  // namespace


ntc_status ntc_pool_admit(ntc_pool_handle pool, int32_t nmodes, const int64_t *dims, int64_t nnz,
                          const int32_t *coords, const float *values, int32_t rank, const ntc_params *p,
                          int32_t *slot)
{
    ntc::TraceRange range("ntc_pool_admit");
    if (!pool || !slot)
        return fail(NTC_EINVAL, "null argument");
    *slot = -1;
    if (free_slot_of(pool) < 0)
        return fail(NTC_ENOMEM, "no free slot");
    // refuse before the host work when even the upper bound cannot fit
    ntc_params q;
    if (p)
        q = *p;
    else
        ntc_params_default(&q);
    size_t bound = 0;
    POOL_TRY(ntc_estimate_bytes(nmodes, dims, nnz, rank, &q, &bound));
    if (bound > pool->arena.largest_free())
        return fail(NTC_ENOMEM, "arena cannot hold the problem now (up to " + std::to_string(bound) +
                                    " bytes needed, " + std::to_string(pool->arena.largest_free()) +
                                    " in the largest free block)");
    ntc_prepared_handle prep = nullptr;
    POOL_TRY(ntc_prepare(&prep, nmodes, dims, nnz, coords, values, rank, &q));
    const ntc_status st = admit_prepared(pool, prep, slot);
    (void)ntc_prepared_release(prep);
    return st;
}

ntc_status ntc_pool_admit_device_csr(ntc_pool_handle pool, int32_t nmodes, const int64_t *dims, int64_t nnz,
                                     const int32_t *coords, const float *values, int32_t rank, const ntc_params *p,
                                     int32_t *slot)
{
    ntc::TraceRange range("ntc_pool_admit_device_csr");
    if (!pool || !slot)
        return fail(NTC_EINVAL, "null argument");
    *slot = -1;
    const int32_t free_slot = free_slot_of(pool);
    if (free_slot < 0)
        return fail(NTC_ENOMEM, "no free slot");
    ntc_params q;
    if (p)
        q = *p;
    else
        ntc_params_default(&q);
    size_t bound = 0, temps = 0;
    POOL_TRY(ntc_estimate_bytes(nmodes, dims, nnz, rank, &q, &bound));
    POOL_TRY(ntc::device_csr_temp_bytes(nmodes, dims, nnz, &temps));
    if (bound + temps > pool->arena.largest_free())
        return fail(NTC_ENOMEM, "arena cannot hold the problem and its CSR temporaries now (up to " +
                                    std::to_string(bound + temps) + " bytes needed, " +
                                    std::to_string(pool->arena.largest_free()) + " in the largest free block)");
    pool_params(pool, &q);
    ntc_handle h = nullptr;
    POOL_TRY(ntc_create_device_csr(&h, nmodes, dims, nnz, coords, values, rank, &q));
    return register_slot(pool, h, free_slot, slot);
}

ntc_status ntc_pool_admit_prepared(ntc_pool_handle pool, ntc_prepared_handle prepared, int32_t *slot)
{
    ntc::TraceRange range("ntc_pool_admit_prepared");
    if (!pool || !prepared || !slot)
        return fail(NTC_EINVAL, "null argument");
    return admit_prepared(pool, prepared, slot);
}

ntc_status ntc_pool_step(ntc_pool_handle pool, int32_t nsweeps)
{
    ntc::TraceRange range("ntc_pool_step");
    if (!pool)
        return fail(NTC_EINVAL, "null pool");
    if (nsweeps < 0)
        return fail(NTC_EINVAL, "nsweeps must be >= 0");
    if (nsweeps == 0)
        return NTC_OK;
    if (pool->dirty)
        POOL_TRY(rebuild(pool));
    if (pool->n_run == 0)
        return NTC_OK;  // nothing running
    // the sweeps run back to back; the stop rule is applied on the device
    // after every sweep, and a stopped problem's kernels leave at once
    for (int32_t it = 0; it < nsweeps; ++it) {
        if (pool->p.use_graph) {
            if (!pool->exec)
                POOL_TRY(capture(pool));
            POOL_HIP(hipGraphLaunch(pool->exec, pool->stream));
        } else {
            POOL_TRY(enqueue_sweep(pool));
        }
    }
    const size_t ms = pool->slots.size();
    int64_t *h_sweeps = reinterpret_cast<int64_t *>(pool->st_host);
    double *h_last = reinterpret_cast<double *>(pool->st_host + ms * 8);
    int32_t *h_stop = reinterpret_cast<int32_t *>(pool->st_host + ms * 16);
    POOL_HIP(hipMemcpyAsync(h_stop, pool->st_stop, ms * 4, hipMemcpyDeviceToHost, pool->stream));
    POOL_HIP(hipMemcpyAsync(h_sweeps, pool->st_sweeps, ms * 8, hipMemcpyDeviceToHost, pool->stream));
    POOL_HIP(hipMemcpyAsync(h_last, pool->st_last, ms * 8, hipMemcpyDeviceToHost, pool->stream));
    POOL_HIP(hipStreamSynchronize(pool->stream));
    pool->sweeps += nsweeps;
    for (size_t i = 0; i < ms; ++i) {
        Slot &s = pool->slots[i];
        if (s.state != NTC_SLOT_RUNNING)
            continue;
        ntc::note_sweeps(s.h, h_sweeps[i] - s.sweeps);
        s.sweeps = h_sweeps[i];
        if (s.view.n_test > 0)
            s.rmse = h_last[i];
        if (h_stop[i] != 0) {
            s.state = NTC_SLOT_STOPPED;
            pool->dirty = true;
        }
    }
    return NTC_OK;
}

ntc_status ntc_pool_query(ntc_pool_handle pool, int32_t slot, int32_t *state, int64_t *sweeps, double *test_rmse)
{
    POOL_TRY(check_slot(pool, slot));
    const Slot &s = pool->slots[slot];
    if (state)
        *state = s.state;
    if (sweeps)
        *sweeps = s.sweeps;
    if (test_rmse)
        *test_rmse = s.h ? s.rmse : std::numeric_limits<double>::quiet_NaN();
    return NTC_OK;
}

ntc_status ntc_pool_loss(ntc_pool_handle pool, int32_t slot, double out[4])
{
    ntc::TraceRange range("ntc_pool_loss");
    POOL_TRY(check_slot(pool, slot));
    if (!pool->slots[slot].h)
        return fail(NTC_ESTATE, "slot is free");
    return ntc_loss(pool->slots[slot].h, out);
}

ntc_status ntc_pool_get_factors(ntc_pool_handle pool, int32_t slot, int32_t mode, float *host_out)
{
    POOL_TRY(check_slot(pool, slot));
    if (!pool->slots[slot].h)
        return fail(NTC_ESTATE, "slot is free");
    return ntc_get_factors(pool->slots[slot].h, mode, host_out);
}

ntc_status ntc_pool_stopped(ntc_pool_handle pool, int32_t *slots, int32_t cap, int32_t *count)
{
    if (!pool || !count || (cap > 0 && !slots))
        return fail(NTC_EINVAL, "null argument");
    int32_t n = 0;
    for (int32_t i = 0; i < static_cast<int32_t>(pool->slots.size()); ++i)
        if (pool->slots[i].state == NTC_SLOT_STOPPED) {
            if (n < cap)
                slots[n] = i;
            ++n;
        }
    *count = n;
    return NTC_OK;
}

ntc_status ntc_pool_evict(ntc_pool_handle pool, int32_t slot)
{
    POOL_TRY(check_slot(pool, slot));
    Slot &s = pool->slots[slot];
    if (s.state == NTC_SLOT_FREE)
        return fail(NTC_ESTATE, "slot is already free");
    POOL_HIP(hipStreamSynchronize(pool->stream));
    const ntc_status st = ntc_release(s.h);
    s = Slot{};
    pool->dirty = true;
    return st;
}

ntc_status ntc_pool_info(ntc_pool_handle pool, size_t *used, size_t *free_bytes, int32_t *running, int32_t *stopped,
                         int64_t *pool_sweeps)
{
    if (!pool)
        return fail(NTC_EINVAL, "null pool");
    int32_t r = 0, st = 0;
    for (const Slot &s : pool->slots) {
        r += s.state == NTC_SLOT_RUNNING;
        st += s.state == NTC_SLOT_STOPPED;
    }
    if (used)
        *used = pool->arena.used;
    if (free_bytes)
        *free_bytes = pool->arena.cap - pool->arena.used;
    if (running)
        *running = r;
    if (stopped)
        *stopped = st;
    if (pool_sweeps)
        *pool_sweeps = pool->sweeps;
    return NTC_OK;
}

ntc_status ntc_pool_release(ntc_pool_handle pool)
{
    delete pool;
    return NTC_OK;
}

}  // extern "C"
