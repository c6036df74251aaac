// Row kernels of libntc for R <= 16 on gfx950 (wave64), the launch
// dispatch for every rank, and the sweep-counter update.
#include <hip/hip_runtime.h>

#include "ntc_bf16.h"
#include "ntc_dev.h"
#include "ntc_few.h"
#include "ntc_internal.h"
#include "ntc_rng.h"

namespace ntc {
namespace {

// ------------------------------------------------- group-per-item (R <= 16)
//
// For R <= 16 every work item is owned by one 16-lane group (one DPP row),
// so a wave advances four rows at once.  Inside a row: k.y by a four-step
// DPP butterfly; the row Hessian k k^T by one v_mfma_f32_16x16x1f32 per step,
// whose four 16x16 output blocks are the four groups' rank-1 updates (FP32
// over a batch of 16 samples, then added into FP64); the power method in a
// skewed layout (lane r keeps H[r][sigma_s(r)] for the 16 row rotations
// sigma_s, so H v is 16 FMAs against row-rotated copies of v).  A batch of
// 16 samples per group is mapped one sample per lane for the sampler and the
// record fetch, staged in LDS, and all factor gathers of the batch are
// issued before any arithmetic.

// (H v)_lane = sum_s hd[s] * v[sigma_s(lane)], as four independent FMA
// chains (s mod 4) summed at the end, so the latency of one product is four
// FMAs deep instead of sixteen.
template <int S>
__device__ __forceinline__ void skew_chain(const double (&hd)[16], double v, double &w)
{
    w = fma(hd[S], dpp_f64<kDppRor + S>(v), w);
    if constexpr (S + 4 < 16)
        skew_chain<S + 4>(hd, v, w);
}

__device__ __forceinline__ double skew_matvec(const double (&hd)[16], double v)
{
    double w0 = hd[0] * v, w1 = 0.0, w2 = 0.0, w3 = 0.0;
    skew_chain<4>(hd, v, w0);
    skew_chain<1>(hd, v, w1);
    skew_chain<2>(hd, v, w2);
    skew_chain<3>(hd, v, w3);
    return (w0 + w1) + (w2 + w3);
}

// Power method, step, projection and extrapolation for the row owned by
// this 16-lane group.  Lane r holds g[r] (sampled gradient without ridge)
// and hd[s] = H[r][sigma_s(r)] (sampled Hessian without ridge); lanes r >= R
// hold zeros.  No cross-group communication.
template <bool BF16, class Args>
__device__ void finish_row16(const Args &a, int row, int r, double g, double (&hd)[16], float y)
{
    const int R = a.R;
    const bool live = r < R;
    if (live) {
        g += a.lambda * static_cast<double>(y);
        hd[0] += a.lambda;  // sigma_0 is the identity: the diagonal
    }
    const double L = lp_estimate(live, live ? a.v0 : 0.0, a.power_iters, a.lp_bound,
                                 [&](double x) { return skew_matvec(hd, x); }, [](double x) { return row_sum_f64(x); },
                                 [](double &x, double &y) { row_sum2_f64(x, y); },
                                 [](double x) { return row_max_f64(x); }, [](bool d) { return row_all(d); });
    if (!live)
        return;
    const int64_t off = static_cast<int64_t>(row) * R + r;
    const float a_prev = (a.l == 0) ? y : a.A[off];
    const bool more = a.l + 1 < a.max_inner;
    if (L > 0.0) {
        double an = static_cast<double>(y) - g / L;
        an = an > 0.0 ? an : 0.0;
        const double sl = sqrt(L), sm = a.sqrt_lambda;
        const double beta = (sl - sm) / (sl + sm);
        const float af = static_cast<float>(an);
        a.A[off] = af;
        if (BF16)
            a.A16[off] = f32_to_bf16(af);
        if (more)
            a.Y[off] = static_cast<float>(an + beta * (an - static_cast<double>(a_prev)));
    } else if (more && a.l == 0) {
        a.Y[off] = y;  // row skipped: Y_1 = Y_0
    }
}

constexpr int kSlot16 = 16 + 16 * 16;  // doubles per partial slot: g[16], row-major H[16][16]


// Lane index within the DPP row that row_ror:s reads for this lane, for
// s = 0..15: the skewed Hessian layout uses exactly the hardware rotation.
__device__ __forceinline__ void ror_sources(int r, int (&sig)[16])
{
    sig[0] = r;
#define NTC_SIG(S) sig[S] = __builtin_amdgcn_update_dpp(0, r, kDppRor + S, 0xF, 0xF, true)
    NTC_SIG(1); NTC_SIG(2); NTC_SIG(3); NTC_SIG(4); NTC_SIG(5); NTC_SIG(6); NTC_SIG(7); NTC_SIG(8);
    NTC_SIG(9); NTC_SIG(10); NTC_SIG(11); NTC_SIG(12); NTC_SIG(13); NTC_SIG(14); NTC_SIG(15);
#undef NTC_SIG
}

// Per-group state of one work item of the group kernels.
struct GroupItem {
    Item it;
    bool has;
    int len;
    int64_t base;
    Prp prp;
};

// Whole row `id` of the group kernel (N <= 4), from its RowItem.
template <class Args>
__device__ __forceinline__ GroupItem load_row_item(const Args &a, int id)
{
    GroupItem g;
    g.has = id < a.n_group - a.n_few;
    RowItem ri{0, 1, 0};
    if (g.has)
        ri = a.rows[id];
    g.base = ri.base;
    g.len = g.has ? static_cast<int>(minibatch_size(a.c, ri.n)) : 0;
    g.it = Item{ri.row, 0, g.len, -1};
    g.prp = make_prp(static_cast<uint32_t>(ri.n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, ri.row));
    return g;
}

template <class Args>
__device__ __forceinline__ GroupItem load_group_item(const Args &a, int id)
{
    GroupItem g;
    g.has = id < a.n_items;
    g.it = Item{0, 0, 0, -1};
    if (g.has)
        g.it = a.items[id];
    g.base = 0;
    int64_t n = 1;
    if (g.has) {
        g.base = a.rowptr[g.it.row];
        n = a.rowptr[g.it.row + 1] - g.base;
    }
    g.len = g.it.j1 - g.it.j0;
    g.prp = make_prp(static_cast<uint32_t>(n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, g.it.row));
    return g;
}

// Record of sample jb + r of the item; returns whether the sample exists.
// Every lane loads, whatever the item's length: a lane past its end reads
// entry 0 of the records (in bounds whenever a row kernel runs) and
// stage_record puts the zero record in its place.  With no load under a
// branch the compiler can count the loads in flight, so a later wait for
// older loads leaves this one outstanding.
// spos: the item's sampled positions in increasing order (a whole row; see
// sort_positions), else NULL and sample j is the PRP's image of j0 + j.
template <int RW, bool NT, class Args>
__device__ __forceinline__ bool fetch_record(const Args &a, const GroupItem &g, int jb, int r, uint4 &w0,
                                             uint4 &w1, const uint16_t *spos = nullptr)
{
    const bool live = jb + r < g.len;
    int64_t e = 0;
    if (live)
        e = g.base + (spos ? static_cast<uint32_t>(spos[jb + r])
                           : prp_index(g.prp, static_cast<uint32_t>(g.it.j0 + jb + r)));
    const uint32_t *src = a.records + e * RW;
    w0 = load_record4<NT>(src);
    w1 = (RW == 8) ? load_record4<NT>(src + 4) : w0;
    return live;
}

// LDS accesses of one wave are performed in order, so staging needs only a
// compiler barrier, not a fence (a fence would also wait for the gathers in
// flight).
template <int RW, class Args>
__device__ __forceinline__ void stage_record(const Args &a, uint4 *buf, int lane, bool live, const uint4 &w0,
                                             const uint4 &w1)
{
    buf[lane * (RW / 4)] = pick4(live, w0, make_uint4(a.zrec[0], a.zrec[1], a.zrec[2], a.zrec[3]));
    if (RW == 8)
        buf[lane * (RW / 4) + 1] = pick4(live, w1, make_uint4(a.zrec[4], a.zrec[5], a.zrec[6], a.zrec[7]));
    __builtin_amdgcn_wave_barrier();
}

// Issue the factor gathers of one batch: f[mm][t] = U_mm[idx(t, mm), r].
// Branch-free: every lane loads from an in-bounds address (a missing sample
// has index 0 in LDS, a lane r >= R reads column 0) and the compute masks the
// value, so all loads of the batch issue back to back.
template <int NM, int RW, bool BF16, class Args>
__device__ __forceinline__ void gather_batch(const Args &a, const uint32_t *srec, int rr, float (&f)[NM - 1][16])
{
#pragma unroll
    for (int mm = 0; mm < NM - 1; ++mm) {
        // 32-bit byte offsets from a wave-uniform base (factors are < 4 GiB)
        const char *base = BF16 ? reinterpret_cast<const char *>(a.gath16[mm])
                                : reinterpret_cast<const char *>(a.gath[mm]);
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const uint32_t e = srec[t * RW + mm] + static_cast<uint32_t>(rr);  // coordinate * R + column
            if (BF16)
                f[mm][t] = bf16_to_f32(*reinterpret_cast<const uint16_t *>(base + e * 2u));
            else
                f[mm][t] = *reinterpret_cast<const float *>(base + e * 4u);
        }
    }
}

// Items of the group kernels with a compile-time mode count N <= 4.  The
// batch loop is software-pipelined: while batch b is reduced, the factor
// gathers of batch b+1 and the record fetches of batch b+2 are in flight
// (records double-buffered in LDS, gathered values held raw until used).
template <int NM, int RW, bool BF16, bool NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NM <= 3 ? 4 : 2))) void k_rows16(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ uint4 s_rec[2][64 * (RW / 4)];
    // FP64 sum of the MFMA blocks: register v of lane l at s_h[v * 64 + l]
    __shared__ double s_h[16 * 64];
    const int lane = threadIdx.x;
    const int r = lane & 15;
    const int grp = lane >> 4;
    // whole rows: items [0, n_group), four per wave
    const GroupItem g = load_row_item(a, blk_ * 4 + grp);
    const int R = a.R;
    const bool rlive = r < R;
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const float y = (g.has && rlive) ? ysrc[static_cast<int64_t>(g.it.row) * R + r] : 0.0f;

    // the MFMA below reads all 64 lanes: the batch loop runs the same number
    // of times in every group (the longest item of the wave); missing
    // samples enter as k = 0
    const int maxlen = max(max(__builtin_amdgcn_readlane(g.len, 0), __builtin_amdgcn_readlane(g.len, 16)),
                           max(__builtin_amdgcn_readlane(g.len, 32), __builtin_amdgcn_readlane(g.len, 48)));
    const int nb = (maxlen + 15) / 16;

    double gd = 0.0;
#pragma unroll
    for (int v = 0; v < 16; ++v)
        s_h[v * 64 + lane] = 0.0;

    const int rr = rlive ? r : 0;
    uint4 w0, w1;
    float f[NM - 1][16];  // gathered factor values of the next batch to reduce
    if (nb > 0) {
        // both batches' records in flight together; batch 1 is staged after
        // batch 0's gathers are issued (all zero records when nb == 1)
        uint4 v0, v1;
        const bool l0 = fetch_record<RW, NT>(a, g, 0, r, w0, w1);
        const bool l1 = fetch_record<RW, NT>(a, g, 16, r, v0, v1);
        stage_record<RW>(a, s_rec[0], lane, l0, w0, w1);
        gather_batch<NM, RW, BF16>(a, reinterpret_cast<const uint32_t *>(s_rec[0]) + grp * 16 * RW, rr, f);
        stage_record<RW>(a, s_rec[1], lane, l1, v0, v1);
    }
    for (int bi = 0; bi < nb; ++bi) {
        const int jb = bi * 16;
        const int tmax = min(16, maxlen - jb);
        // Khatri-Rao rows of this batch; this frees f for the next gathers
        float kc[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            float k = f[0][t];
#pragma unroll
            for (int mm = 1; mm < NM - 1; ++mm)
                k *= f[mm][t];
            kc[t] = rlive ? k : 0.0f;  // a missing sample gathered the zero rows
        }
        // issue order: records of batch b+2, then gathers of batch b+1, so
        // that staging the records later waits only for the record loads
        // (fetched in every iteration: past the end they are zero records)
        const bool lv2 = fetch_record<RW, NT>(a, g, jb + 32, r, w0, w1);
        if (bi + 1 < nb)
            gather_batch<NM, RW, BF16>(a, reinterpret_cast<const uint32_t *>(s_rec[(bi + 1) & 1]) + grp * 16 * RW,
                                       rr, f);
        const uint32_t *srec = reinterpret_cast<const uint32_t *>(s_rec[bi & 1]) + grp * 16 * RW;
        float gf = 0.0f;
        f32x16 acc = {0.0f};
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            if (t < tmax) {  // wave-uniform
                const float k = kc[t];
                const float x = __uint_as_float(srec[t * RW + NM - 1]);  // 0 for a missing sample
                const float pred = row_sum_f32(k * y);
                gf = fmaf(pred - x, k, gf);
                // four independent rank-1 updates, one per group: block b += k_b k_b^T
                acc = __builtin_amdgcn_mfma_f32_16x16x1f32(k, k, acc, 0, 0, 0);
            }
        }
        gd += static_cast<double>(gf);
#pragma unroll
        for (int v = 0; v < 16; ++v)
            s_h[v * 64 + lane] += static_cast<double>(acc[v]);
        __builtin_amdgcn_wave_barrier();  // the compute above read s_rec[bi & 1]
        if (bi + 2 < nb)
            stage_record<RW>(a, s_rec[bi & 1], lane, lv2, w0, w1);
    }

    // register v of lane l holds block v/4, row 4*(l/16) + v%4, column l%16:
    // row r of this group's block is at v = 4*grp + r%4, lanes 16*(r/4) + q
    __builtin_amdgcn_wave_barrier();
    if (!g.has)
        return;
    const double *hrow = s_h + (4 * grp + (r & 3)) * 64 + 16 * (r >> 2);
    int sig[16];
    ror_sources(r, sig);
    double hs[16];
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2)
        hs[s2] = hrow[sig[s2]];
    finish_row16<BF16>(a, g.it.row, r, gd, hs, y);
}


// A whole row of at most kSortedRowMax entries and kSortedChunkMax samples
// runs through k_chunk16 in position order when the records stream from HBM
// (NT, records past the last-level cache): its minibatch is the same set,
// and records that share a line are then loaded by one instruction.  When
// the records stay cached, the merged requests would have hit the cache
// anyway and the ordering only delays the block's first loads.
constexpr int kSortedRowMax = 65536;   // positions fit 16 bits; a 2048-word bitmap
constexpr int kSortedChunkMax = 6144;

// The positions {pi(j) : j < g.len} of a whole row of n entries, in
// increasing order, into pos[0 .. g.len): one bit per position in `bits`
// (ceil(n / 32) words), then each of the 256 threads turns a run of words
// into positions at the offset an exclusive scan of the runs' bit counts
// gives (`scan`: 256 words).  The order is the positions' own, so the result
// does not depend on the order of the atomics.  Block-wide: every thread
// calls it.
__device__ __forceinline__ void sort_positions(const GroupItem &g, int64_t n, uint32_t *bits, uint32_t *scan,
                                               uint16_t *pos, int tid)
{
    const int W = static_cast<int>((n + 31) >> 5);
    for (int w = tid; w < W; w += 256)
        bits[w] = 0u;
    __syncthreads();
    for (int j = tid; j < g.len; j += 256) {
        const uint32_t p = prp_index(g.prp, static_cast<uint32_t>(g.it.j0 + j));
        atomicOr(&bits[p >> 5], 1u << (p & 31u));
    }
    __syncthreads();
    const int per = (W + 255) >> 8;
    const int w0 = min(tid * per, W);
    const int w1 = min(w0 + per, W);
    uint32_t cnt = 0;
    for (int w = w0; w < w1; ++w)
        cnt += __popc(bits[w]);
    scan[tid] = cnt;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {  // inclusive scan (Hillis-Steele)
        const uint32_t v = tid >= d ? scan[tid - d] : 0u;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    uint32_t o = scan[tid] - cnt;
    for (int w = w0; w < w1; ++w) {
        for (uint32_t m = bits[w]; m != 0u; m &= m - 1u)
            pos[o++] = static_cast<uint16_t>(w * 32 + __builtin_ctz(m));
    }
    __syncthreads();
}

// Chunks of rows with many sampled entries: one 256-thread block (16
// groups) per chunk of up to item_samples entries of ONE row.  Batch t of
// the chunk (16 entries) goes to group t mod 16, so every group walks a
// short chain of batches.  The four groups of a wave hold samples of the
// same row, so one v_mfma_f32_16x16x4f32 per step adds all four k k^T into a
// single 16x16 block (K = the four groups); register v of lane l holds
// H[4*(l/16) + v][l%16].  The four waves' FP64 sums and the 16 groups'
// gradients are combined in LDS in a fixed order; a chunk that is the whole
// row finishes it in place, otherwise it writes a partial slot.
template <int NM, int RW, bool BF16, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NM <= 3 ? 4 : 2))) void k_chunk16(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ uint4 s_rec[4][2][64 * (RW / 4)];
    __shared__ double s_hw[4][4 * 64];  // per wave: its FP64 block sum, register v of lane l at v*64 + l
    __shared__ double s_g[16 * 16];     // per group: gradient partial of lane r
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15;
    const int grp = lane >> 4;
    const int G = wave * 4 + grp;       // group index in the block
    const Item it = a.items[a.n_group + blk_];
    const int R = a.R;
    const bool rlive = r < R;
    const int rr = rlive ? r : 0;
    const int64_t base = a.rowptr[it.row];
    const int64_t n = a.rowptr[it.row + 1] - base;
    GroupItem g;
    g.has = true;
    g.it = it;
    g.base = base;
    g.len = it.j1 - it.j0;
    g.prp = make_prp(static_cast<uint32_t>(n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, it.row));
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const float y = rlive ? ysrc[static_cast<int64_t>(it.row) * R + r] : 0.0f;
    // position order for a whole row that fits (block-uniform); the bitmap
    // and the scan reuse the buffers of the final combination
    __shared__ uint16_t s_pos[NT ? kSortedChunkMax : 1];
    const uint16_t *spos = nullptr;
    if (NT && it.slot < 0 && n <= kSortedRowMax && g.len <= kSortedChunkMax) {
        static_assert(sizeof(s_hw) >= (kSortedRowMax / 32) * 4 && sizeof(s_g) >= 256 * 4, "sort buffers");
        sort_positions(g, n, reinterpret_cast<uint32_t *>(&s_hw[0][0]), reinterpret_cast<uint32_t *>(s_g), s_pos,
                       tid);
        spos = s_pos;
    }

    const int nbatch = (g.len + 15) / 16;  // batches of the chunk
    const int nit = (nbatch + 15) / 16;    // iterations of every group (uniform in the block)
    // batch handled by group G at iteration i: G + 16 i (entries from 16 * batch)

    double gd = 0.0;
    double hd[4] = {0.0, 0.0, 0.0, 0.0};
    uint4 w0, w1;
    float f[NM - 1][16];
    uint4 *rb0 = s_rec[wave][0];
    uint4 *rb1 = s_rec[wave][1];
    if (nit > 0) {
        uint4 v0, v1;
        const bool l0 = fetch_record<RW, NT>(a, g, 16 * G, r, w0, w1, spos);
        const bool l1 = fetch_record<RW, NT>(a, g, 16 * (G + 16), r, v0, v1, spos);
        stage_record<RW>(a, rb0, lane, l0, w0, w1);
        gather_batch<NM, RW, BF16>(a, reinterpret_cast<const uint32_t *>(rb0) + grp * 16 * RW, rr, f);
        stage_record<RW>(a, rb1, lane, l1, v0, v1);
    }
    for (int i = 0; i < nit; ++i) {
        float kc[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            float k = f[0][t];
#pragma unroll
            for (int mm = 1; mm < NM - 1; ++mm)
                k *= f[mm][t];
            kc[t] = rlive ? k : 0.0f;  // a missing sample gathered the zero rows
        }
        const bool lv2 = fetch_record<RW, NT>(a, g, 16 * (G + 16 * (i + 2)), r, w0, w1, spos);
        if (i + 1 < nit)
            gather_batch<NM, RW, BF16>(a, reinterpret_cast<const uint32_t *>((i & 1) ? rb0 : rb1) + grp * 16 * RW,
                                       rr, f);
        const uint32_t *srec = reinterpret_cast<const uint32_t *>((i & 1) ? rb1 : rb0) + grp * 16 * RW;
        float gf = 0.0f;
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const float k = kc[t];
            const float x = __uint_as_float(srec[t * RW + NM - 1]);  // 0 for a missing sample
            const float pred = row_sum_f32(k * y);
            gf = fmaf(pred - x, k, gf);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(k, k, acc, 0, 0, 0);
        }
        gd += static_cast<double>(gf);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            hd[v] += static_cast<double>(acc[v]);
        __builtin_amdgcn_wave_barrier();  // the compute above read this buffer
        if (i + 2 < nit)
            stage_record<RW>(a, (i & 1) ? rb1 : rb0, lane, lv2, w0, w1);
    }

    // fixed-order combination over the four waves and the 16 groups
#pragma unroll
    for (int v = 0; v < 4; ++v)
        s_hw[wave][v * 64 + lane] = hd[v];
    s_g[G * 16 + r] = gd;
    __syncthreads();
    if (wave != 0)
        return;
    double h4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        h4[v] = ((s_hw[0][v * 64 + lane] + s_hw[1][v * 64 + lane]) + s_hw[2][v * 64 + lane]) + s_hw[3][v * 64 + lane];
    double gsum = 0.0;
    for (int q = 0; q < 16; ++q)
        gsum += s_g[q * 16 + r];
    if (it.slot >= 0) {
        double *P = a.partials + static_cast<int64_t>(it.slot) * kSlot16;
        if (grp == 0)
            P[r] = gsum;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            P[16 + (4 * grp + v) * 16 + r] = h4[v];
        return;
    }
    // whole row: row-major H in LDS (reusing wave 0's slot), then group 0 finishes
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int v = 0; v < 4; ++v)
        s_hw[0][(4 * grp + v) * 16 + r] = h4[v];
    __builtin_amdgcn_wave_barrier();
    if (grp != 0)
        return;
    int sig[16];
    ror_sources(r, sig);
    double hs[16];
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2)
        hs[s2] = s_hw[0][r * 16 + sig[s2]];
    finish_row16<BF16>(a, it.row, r, gsum, hs, y);
}

// Items of the group kernels for 5 <= N <= 8 (32-byte records): the same
// computation without the software pipeline; the Khatri-Rao product is
// accumulated over a runtime mode loop.
template <bool BF16, bool NT>
__global__ __launch_bounds__(64) void k_rows16_nm(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ uint4 s_rec[64 * 2];
    __shared__ double s_h[4 * 256];
    const int lane = threadIdx.x;
    const int r = lane & 15;
    const int grp = lane >> 4;
    const int nm = a.nmodes;
    const GroupItem g = load_group_item(a, blk_ * 4 + grp);
    const int R = a.R;
    const bool rlive = r < R;
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const float y = (g.has && rlive) ? ysrc[static_cast<int64_t>(g.it.row) * R + r] : 0.0f;
    const int maxlen = max(max(__builtin_amdgcn_readlane(g.len, 0), __builtin_amdgcn_readlane(g.len, 16)),
                           max(__builtin_amdgcn_readlane(g.len, 32), __builtin_amdgcn_readlane(g.len, 48)));
    double gd = 0.0;
    double hd[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        hd[q] = 0.0;
    for (int jb = 0; jb < maxlen; jb += 16) {
        const int cnt = min(16, max(0, g.len - jb));
        const int tmax = min(16, maxlen - jb);
        uint4 w0, w1;
        const bool lv = fetch_record<8, NT>(a, g, jb, r, w0, w1);
        stage_record<8>(a, s_rec, lane, lv, w0, w1);
        const uint32_t *srec = reinterpret_cast<const uint32_t *>(s_rec) + grp * 16 * 8;
        float kp[16];
#pragma unroll
        for (int t = 0; t < 16; ++t)
            kp[t] = (t < cnt && rlive) ? 1.0f : 0.0f;
        for (int mm = 0; mm < nm - 1; ++mm) {
            float f[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                f[t] = 0.0f;
                if (t < cnt && rlive) {
                    const int64_t off = srec[t * 8 + mm];  // coordinate * R
                    f[t] = BF16 ? bf16_to_f32(a.gath16[mm][off + r]) : a.gath[mm][off + r];
                }
            }
#pragma unroll
            for (int t = 0; t < 16; ++t)
                kp[t] *= f[t];
        }
        float gf = 0.0f;
        f32x16 acc = {0.0f};
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            if (t < tmax) {
                const float k = kp[t];
                const float x = __uint_as_float(srec[t * 8 + nm - 1]);
                const float pred = row_sum_f32(k * y);
                gf = fmaf(pred - x, k, gf);
                acc = __builtin_amdgcn_mfma_f32_16x16x1f32(k, k, acc, 0, 0, 0);
            }
        }
        gd += static_cast<double>(gf);
#pragma unroll
        for (int q = 0; q < 16; ++q)
            hd[q] += static_cast<double>(acc[q]);
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int v = 0; v < 16; ++v)
        s_h[(v >> 2) * 256 + (4 * grp + (v & 3)) * 16 + r] = hd[v];
    __builtin_amdgcn_wave_barrier();
    if (!g.has)
        return;
    const double *hrow = s_h + grp * 256 + r * 16;
    if (g.it.slot >= 0) {
        double *P = a.partials + static_cast<int64_t>(g.it.slot) * kSlot16;
        P[r] = gd;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            P[16 + r * 16 + q] = hrow[q];
        return;
    }
    int sig[16];
    ror_sources(r, sig);
    double hs[16];
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2)
        hs[s2] = hrow[sig[s2]];
    finish_row16<BF16>(a, g.it.row, r, gd, hs, y);
}

// Rows whose minibatch has at most kTinyB samples (R <= 16): one row per
// lane, no cross-lane traffic.  With K the b x R matrix of the sampled
// Khatri-Rao rows, H = K^T K + lambda I, and the T-th (unnormalised) power
// iterate from v0 is x_T = lambda^T v0 + K^T u_T with u_0 = 0 and
//     u_{t+1} = (G + lambda I) u_t + lambda^t c,   G = K K^T, c = K v0,
// because H (a v0 + K^T u) = lambda a v0 + K^T (a c + G u + lambda u).  The
// Rayleigh quotient of x_T is ||a c + G u||^2 / ||x||^2 + lambda with
// ||x||^2 = a^2 + 2 a u.c + u^T G u (||v0|| = 1).  This is the same iterate
// as T normalised products with H, evaluated in the b-dimensional span of
// the samples: O(T b^2) instead of O(T b R) operations per row.
// One factor row of up to 16 columns into registers (zeros past R).  When
// R % 4 == 0 every row starts on a 16-byte (FP32) or 8-byte (BF16) boundary
// and is read with vector loads.
// The loads are branch-free: a part past R reads the start of the same row
// again and is zeroed afterwards, so no load sits under a branch and the
// compiler's wait counts stay exact across the rows of a sample.
template <bool V4>
__device__ __forceinline__ void load_row16(const float *p, int R, float (&out)[16])
{
    if (V4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool in = q == 0 || 4 * q < R;  // R >= 4 here
            const float4 t = reinterpret_cast<const float4 *>(p)[in ? q : 0];
            out[4 * q] = in ? t.x : 0.0f;
            out[4 * q + 1] = in ? t.y : 0.0f;
            out[4 * q + 2] = in ? t.z : 0.0f;
            out[4 * q + 3] = in ? t.w : 0.0f;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const bool in = r == 0 || r < R;  // R >= 1
            const float t = p[in ? r : 0];
            out[r] = in ? t : 0.0f;
        }
    }
}

template <bool V4>
__device__ __forceinline__ void load_row16(const uint16_t *p, int R, float (&out)[16])
{
    if (V4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool in = q == 0 || 4 * q < R;
            const uint2 t = reinterpret_cast<const uint2 *>(p)[in ? q : 0];
            out[4 * q] = in ? __uint_as_float(t.x << 16) : 0.0f;
            out[4 * q + 1] = in ? __uint_as_float(t.x & 0xFFFF0000u) : 0.0f;
            out[4 * q + 2] = in ? __uint_as_float(t.y << 16) : 0.0f;
            out[4 * q + 3] = in ? __uint_as_float(t.y & 0xFFFF0000u) : 0.0f;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const bool in = r == 0 || r < R;
            const uint16_t t = p[in ? r : 0];
            out[r] = in ? bf16_to_f32(t) : 0.0f;
        }
    }
}

template <int NM, int RW, bool BF16, bool V4, bool NT>
__device__ __forceinline__ void tiny_row(CRowArgs &a, int id)
{
    const int nm = (NM > 0) ? NM : a.nmodes;
    const int R = a.R;
    const RowItem ri = a.tiny[id];
    const int row = ri.row;
    const int64_t base = ri.base;
    const int64_t n = ri.n;
    const int b = static_cast<int>(minibatch_size(a.c, n));  // 1 .. kTinyB
    const Prp prp = make_prp(static_cast<uint32_t>(n), sample_keys(a.seed, a.kptr[0], a.mode, a.l, row));
    const float *ysrc = (a.l == 0) ? a.A : a.Y;
    const int64_t roff = static_cast<int64_t>(row) * R;
    float y[16];
    load_row16<V4>(ysrc + roff, R, y);

    // the sample positions, then every record load at once (no load under
    // a branch: a missing sample reads entry 0 of the row and takes the
    // zero record, whose rows are zero and whose value is 0), then the
    // factor rows
    int64_t at[kTinyB];
#pragma unroll
    for (int j = 0; j < kTinyB; ++j) {
        at[j] = base;
        if (j < b)
            at[j] = base + prp_index(prp, static_cast<uint32_t>(j));
    }
    uint32_t rec[kTinyB][RW];
#pragma unroll
    for (int j = 0; j < kTinyB; ++j) {
        const uint32_t *src = a.records + at[j] * RW;
#pragma unroll
        for (int w4 = 0; w4 < RW / 4; ++w4) {
            const uint4 t = load_record4<NT>(src + 4 * w4);
            rec[j][4 * w4] = t.x;
            rec[j][4 * w4 + 1] = t.y;
            rec[j][4 * w4 + 2] = t.z;
            rec[j][4 * w4 + 3] = t.w;
        }
    }
#pragma unroll
    for (int j = 0; j < kTinyB; ++j)
#pragma unroll
        for (int w = 0; w < RW; ++w)
            rec[j][w] = (j < b) ? rec[j][w] : a.zrec[w];
    float kk[kTinyB][16];
    float gf[16];
#pragma unroll
    for (int r = 0; r < 16; ++r)
        gf[r] = 0.0f;
#pragma unroll
    for (int j = 0; j < kTinyB; ++j) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            kk[j][r] = 1.0f;
        for (int mm = 0; mm < nm - 1; ++mm) {
            float f[16];
            if (BF16)
                load_row16<V4>(a.gath16[mm] + rec[j][mm], R, f);  // coordinate * R
            else
                load_row16<V4>(a.gath[mm] + rec[j][mm], R, f);
#pragma unroll
            for (int r = 0; r < 16; ++r)
                kk[j][r] *= f[r];
        }
        // (columns past R are zero: load_row16 zeroes them in every row)
        // a missing sample has k = 0 (zero rows) and x = 0: it adds nothing
        const float x = __uint_as_float(rec[j][nm - 1]);
        float pred = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            pred = fmaf(kk[j][r], y[r], pred);
        const float res = pred - x;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            gf[r] = fmaf(res, kk[j][r], gf[r]);
    }

    // c = K v0 and G = K K^T in FP64 (products of FP32 values are exact)
    const double lam = a.lambda;
    const double v0 = a.v0;
    double c[kTinyB], G[kTinyB][kTinyB];
#pragma unroll
    for (int i = 0; i < kTinyB; ++i) {
        double si = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            si += static_cast<double>(kk[i][r]);
        c[i] = si * v0;
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double d = 0.0;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                d = fma(static_cast<double>(kk[i][r]), static_cast<double>(kk[j][r]), d);
            G[i][j] = d;
            G[j][i] = d;
        }
    }
    // the recurrence, rescaled every step (only the direction matters)
    double al = 1.0, u[kTinyB];
#pragma unroll
    for (int i = 0; i < kTinyB; ++i)
        u[i] = 0.0;
    for (int t = 0; t < a.power_iters; ++t) {
        double un[kTinyB];
        double mx = fabs(al * lam);
#pragma unroll
        for (int i = 0; i < kTinyB; ++i) {
            double s = fma(lam, u[i], al * c[i]);
#pragma unroll
            for (int j = 0; j < kTinyB; ++j)
                s = fma(G[i][j], u[j], s);
            un[i] = s;
            mx = fmax(mx, fabs(s));
        }
        if (!(mx > 0.0)) {
            al = 0.0;
#pragma unroll
            for (int i = 0; i < kTinyB; ++i)
                u[i] = 0.0;
            break;
        }
        // by the power of two at or below the largest magnitude: exact, no division
        const int e = ilogb(mx);
        al = ldexp(al * lam, -e);
#pragma unroll
        for (int i = 0; i < kTinyB; ++i)
            u[i] = ldexp(un[i], -e);
    }
    double x2 = al * al, kx2 = 0.0;
    double kx[kTinyB];
#pragma unroll
    for (int i = 0; i < kTinyB; ++i) {
        double gu = 0.0;
#pragma unroll
        for (int j = 0; j < kTinyB; ++j)
            gu = fma(G[i][j], u[j], gu);
        x2 = fma(u[i], fma(2.0 * al, c[i], gu), x2);   // a^2 + 2 a u.c + u^T G u
        kx[i] = fma(al, c[i], gu);                     // (K x)_i = a c_i + (G u)_i
        kx2 = fma(kx[i], kx[i], kx2);
    }
    double L = (x2 > 0.0) ? kx2 / x2 + lam : 0.0;
    if (a.lp_bound) {
        // Collatz-Wielandt bound: x_r = a v0 + (K^T u)_r, (H x)_r = (K^T K x)_r + lambda x_r
        L = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r < R) {
                double xr = al * v0, hx = 0.0;
#pragma unroll
                for (int i = 0; i < kTinyB; ++i) {
                    const double kir = static_cast<double>(kk[i][r]);
                    xr = fma(kir, u[i], xr);
                    hx = fma(kir, kx[i], hx);
                }
                hx = fma(lam, xr, hx);
                if (xr > 0.0)
                    L = fmax(L, hx / xr);
            }
        }
    }

    const bool more = a.l + 1 < a.max_inner;
    if (L > 0.0) {
        const double sl = sqrt(L), sm = a.sqrt_lambda;
        const double beta = (sl - sm) / (sl + sm);
        // A_l: the row read for y when l == 0, else the whole row in one go
        float al16[16];
        if (a.l == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                al16[r] = y[r];
        } else {
            load_row16<V4>(a.A + roff, R, al16);
        }
        // A_{l+1} = (y - g/L)_+ and Y_{l+1} = A_{l+1} + beta (A_{l+1} - A_l), four columns at a time
        auto step4 = [&](int r0, float (&an4)[4], float (&yn4)[4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = r0 + u;
                const double g = static_cast<double>(gf[r]) + lam * static_cast<double>(y[r]);
                double an = static_cast<double>(y[r]) - g / L;
                an = an > 0.0 ? an : 0.0;
                const float ap = al16[r];
                an4[u] = static_cast<float>(an);
                yn4[u] = static_cast<float>(an + beta * (an - static_cast<double>(ap)));
            }
        };
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (4 * q >= R)
                continue;
            float an4[4], yn4[4];
            step4(4 * q, an4, yn4);
            if (V4) {
                reinterpret_cast<float4 *>(a.A + roff)[q] = make_float4(an4[0], an4[1], an4[2], an4[3]);
                if (BF16)
                    reinterpret_cast<uint2 *>(a.A16 + roff)[q] =
                        make_uint2(static_cast<uint32_t>(f32_to_bf16(an4[0])) |
                                       (static_cast<uint32_t>(f32_to_bf16(an4[1])) << 16),
                                   static_cast<uint32_t>(f32_to_bf16(an4[2])) |
                                       (static_cast<uint32_t>(f32_to_bf16(an4[3])) << 16));
                if (more)
                    reinterpret_cast<float4 *>(a.Y + roff)[q] = make_float4(yn4[0], yn4[1], yn4[2], yn4[3]);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int r = 4 * q + u;
                    if (r < R) {
                        a.A[roff + r] = an4[u];
                        if (BF16)
                            a.A16[roff + r] = f32_to_bf16(an4[u]);
                        if (more)
                            a.Y[roff + r] = yn4[u];
                    }
                }
            }
        }
    } else if (more && a.l == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            if (r < R)
                a.Y[roff + r] = y[r];
    }
}

// One-wave blocks: a wave of this kernel holds a whole SIMD's registers, so
// a block of four would wait for a CU whose four SIMDs are all free, while a
// one-wave block starts on any free SIMD, beside the blocks of the launches
// running concurrently.
constexpr int kTinyBlock = 64;

template <int NM, int RW, bool BF16, bool NT>
__global__ __launch_bounds__(kTinyBlock) void k_tiny16(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    const int id = blk_ * kTinyBlock + threadIdx.x;
    if (id >= a.n_tiny)
        return;
    // R % 4 is uniform over the block (one problem per block)
    if ((a.R & 3) == 0)
        tiny_row<NM, RW, BF16, true, NT>(a, id);
    else
        tiny_row<NM, RW, BF16, false, NT>(a, id);
}

// Rows with 1 <= B_p <= tiny_max samples (N <= 4): sixteen per one-wave
// block, four lanes per row and one sample per lane (ntc_few.h).  V4: R % 4 == 0
// (the kernel class); the load width within it follows R.
template <int NM, bool BF16, bool V4, bool NT>
__global__ __launch_bounds__(64) void k_quad16(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    if constexpr (V4) {
        if (a.R == 16)
            quad_rows<NM, BF16, 3, NT>(a, a.tiny, a.n_tiny, blk_);
        else if (!BF16 || (a.R & 7) == 0)
            quad_rows<NM, BF16, 2, NT>(a, a.tiny, a.n_tiny, blk_);
        else
            quad_rows<NM, BF16, 1, NT>(a, a.tiny, a.n_tiny, blk_);
    } else {
        if ((a.R & 1) == 0)
            quad_rows<NM, BF16, 1, NT>(a, a.tiny, a.n_tiny, blk_);
        else
            quad_rows<NM, BF16, 0, NT>(a, a.tiny, a.n_tiny, blk_);
    }
}

// Whole rows with 5 <= B_p <= 16 samples (N <= 4): four per one-wave block,
// one sample per lane, the power method in the span of v_0 and the sampled
// rows (ntc_few.h).  V4: R % 4 == 0 (the kernel class); the load width
// within it follows R, which is uniform over the block (one problem per
// block).
template <int NM, bool BF16, bool V4, bool NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_few16(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ FewShared sh;
    const RowItem *list = a.rows + (a.n_group - a.n_few);
    if constexpr (V4) {
        if (a.R == 16)
            few_rows<16, NM, BF16, 3, NT>(a, list, a.n_few, blk_, sh);
        else if (!BF16 || (a.R & 7) == 0)
            few_rows<16, NM, BF16, 2, NT>(a, list, a.n_few, blk_, sh);
        else
            few_rows<16, NM, BF16, 1, NT>(a, list, a.n_few, blk_, sh);
    } else {
        if ((a.R & 1) == 0)
            few_rows<16, NM, BF16, 1, NT>(a, list, a.n_few, blk_, sh);
        else
            few_rows<16, NM, BF16, 0, NT>(a, list, a.n_few, blk_, sh);
    }
}

// Rows split over several items: one 256-thread block per row; its 16
// groups sum the row's slots with a fixed stride, a fixed-order tree in LDS
// combines them, and the first group finishes the row.
template <bool BF16>
__global__ __launch_bounds__(256) void k_finalize16(NTC_ROW_PARAMS)
{
    NTC_ROW_RESOLVE(a, blk_);
    __shared__ double s_part[16 * 16 * 17];
    const SplitRow sr = a.split[blk_];
    const int tid = threadIdx.x;
    const int r = tid & 15;
    const int grp = tid >> 4;
    double g = 0.0;
    double hd[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        hd[q] = 0.0;
    int sig[16];
    ror_sources(r, sig);
    for (int s = grp; s < sr.nslots; s += 16) {
        const double *P = a.partials + static_cast<int64_t>(sr.slot0 + s) * kSlot16;
        g += P[r];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            hd[q] += P[16 + r * 16 + sig[q]];
    }
    double *mine = s_part + (grp * 16 + r) * 17;
    mine[0] = g;
#pragma unroll
    for (int q = 0; q < 16; ++q)
        mine[1 + q] = hd[q];
    __syncthreads();
    for (int st = 8; st > 0; st >>= 1) {
        if (grp < st) {
            const double *other = s_part + ((grp + st) * 16 + r) * 17;
#pragma unroll
            for (int q = 0; q < 17; ++q)
                mine[q] += other[q];
        }
        __syncthreads();
    }
    if (grp != 0)
        return;
    g = mine[0];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        hd[q] = mine[1 + q];
    float y = 0.0f;
    if (r < a.R) {
        const float *ysrc = (a.l == 0) ? a.A : a.Y;
        y = ysrc[static_cast<int64_t>(sr.row) * a.R + r];
    }
    finish_row16<BF16>(a, sr.row, r, g, hd, y);
}

#define NTC_GO(KERNEL, BLOCK) \
    hipLaunchKernelGGL(KERNEL, dim3(L.blocks), dim3(BLOCK), 0, s, L.args, L.start, L.owner, L.n)

template <bool BF16, bool NT>
hipError_t go_rows16(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.nmodes == 3)
        NTC_GO((k_rows16<3, 4, BF16, NT>), 64);
    else if (kc.nmodes == 4)
        NTC_GO((k_rows16<4, 4, BF16, NT>), 64);
    else if (kc.nmodes == 2)
        NTC_GO((k_rows16<2, 4, BF16, NT>), 64);
    else
        NTC_GO((k_rows16_nm<BF16, NT>), 64);
    return hipGetLastError();
}

template <bool BF16, bool V4, bool NT>
hipError_t go_quad16(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.nmodes == 3)
        NTC_GO((k_quad16<3, BF16, V4, NT>), 64);
    else if (kc.nmodes == 4)
        NTC_GO((k_quad16<4, BF16, V4, NT>), 64);
    else
        NTC_GO((k_quad16<2, BF16, V4, NT>), 64);
    return hipGetLastError();
}

template <bool BF16, bool NT>
hipError_t go_tiny(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.nmodes <= 4)
        return kc.pairs ? go_quad16<BF16, true, NT>(kc, L, s) : go_quad16<BF16, false, NT>(kc, L, s);
    NTC_GO((k_tiny16<0, 8, BF16, NT>), kTinyBlock);
    return hipGetLastError();
}

template <bool BF16, bool V4, bool NT>
hipError_t go_few16v(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.nmodes == 3)
        NTC_GO((k_few16<3, BF16, V4, NT>), 64);
    else if (kc.nmodes == 4)
        NTC_GO((k_few16<4, BF16, V4, NT>), 64);
    else if (kc.nmodes == 2)
        NTC_GO((k_few16<2, BF16, V4, NT>), 64);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <bool BF16, bool NT>
hipError_t go_few16(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    return kc.pairs ? go_few16v<BF16, true, NT>(kc, L, s) : go_few16v<BF16, false, NT>(kc, L, s);
}

template <bool BF16, bool NT>
hipError_t go_chunks(const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (kc.nmodes == 3)
        NTC_GO((k_chunk16<3, 4, BF16, NT>), 256);
    else if (kc.nmodes == 4)
        NTC_GO((k_chunk16<4, 4, BF16, NT>), 256);
    else if (kc.nmodes == 2)
        NTC_GO((k_chunk16<2, 4, BF16, NT>), 256);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

#undef NTC_GO

__global__ void k_advance(int64_t *k, int32_t n)
{
    const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < n)
        k[t] += 1;
}

}  // namespace

int32_t row_kernel_blocks(RowKernel kind, const KernelClass &kc, int32_t n_items, int32_t n_group, int32_t n_split,
                          int32_t n_tiny, int32_t n_groups, int32_t n_few)
{
    const bool g16 = kc.rp == 16;
    switch (kind) {
    case kRows:
        return g16 ? (kc.nmodes > 4 ? (n_items + 3) / 4 : (n_group - n_few + 3) / 4) : n_items;
    case kFew:
        return (g16 && kc.nmodes <= 4) ? (n_few + 3) / 4 : 0;
    case kFinalize:
        return n_split;
    case kTiny:
        if (g16)
            return kc.nmodes <= 4 ? (n_tiny + 15) / 16 : (n_tiny + kTinyBlock - 1) / kTinyBlock;
        return (kc.rp == 32 && kc.nmodes <= 4) ? (n_tiny + 3) / 4 : 0;
    case kChunks:
        return (g16 && kc.nmodes <= 4) ? n_items - n_group : 0;
    case kReduce:
        return g16 ? 0 : n_groups;
    }
    return 0;
}

namespace {

template <bool NT>
hipError_t launch_row16(RowKernel kind, const KernelClass &kc, const Launch &L, hipStream_t s)
{
    const bool b = kc.bf16 != 0;
    switch (kind) {
    case kRows:
        return b ? go_rows16<true, NT>(kc, L, s) : go_rows16<false, NT>(kc, L, s);
    case kFinalize:
        hipLaunchKernelGGL(b ? k_finalize16<true> : k_finalize16<false>, dim3(L.blocks), dim3(256), 0, s, L.args,
                           L.start, L.owner, L.n);
        return hipGetLastError();
    case kTiny:
        return b ? go_tiny<true, NT>(kc, L, s) : go_tiny<false, NT>(kc, L, s);
    case kChunks:
        return b ? go_chunks<true, NT>(kc, L, s) : go_chunks<false, NT>(kc, L, s);
    case kReduce:
        return hipSuccess;
    case kFew:
        return b ? go_few16<true, NT>(kc, L, s) : go_few16<false, NT>(kc, L, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_row_kernel(RowKernel kind, const KernelClass &kc, const Launch &L, hipStream_t s)
{
    if (L.blocks <= 0 || L.n <= 0)
        return hipSuccess;
    if (kc.rp != 16)
        return launch_row_kernel_wide(kind, kc, L, s);
    return kc.nt ? launch_row16<true>(kind, kc, L, s) : launch_row16<false>(kind, kc, L, s);
}

hipError_t launch_advance(int64_t *k, int32_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_advance, dim3((n + 255) / 256), dim3(256), 0, s, k, n);
    return hipGetLastError();
}

}  // namespace ntc
