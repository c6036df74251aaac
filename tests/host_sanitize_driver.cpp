// The library's host code (argument checks, per-mode CSR build, row
// schedule, host sampler, byte counts) run with no device, for builds under
// gcc's address, undefined-behaviour and thread sanitizers.  The device
// launchers are replaced by stubs that abort: nothing called here may reach
// a device.  Every array handed to the library has exactly the size its
// declaration in ntc.h states, so a write past it is reported.
//
// Problems are seeded and synthetic (row lengths skewed like a Zipf law),
// covering the schedule's shapes: rows of a few samples, whole rows, split
// rows and slot groups; N from 2 to 8; R from 1 to 64; empty inputs.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "ntc.h"
#include "ntc_aux.h"
#include "ntc_csr.h"
#include "ntc_internal.h"

namespace ntc {
[[noreturn]] static void device_entry(const char *name)
{
    std::fprintf(stderr, "device entry %s reached from host-only code\n", name);
    std::abort();
}
hipError_t csr_validate(const int32_t *, const float *, int64_t, int32_t, const CsrDims &, unsigned long long *,
                        hipStream_t)
{
    device_entry("csr_validate");
}
hipError_t csr_sort_bytes(int64_t, size_t *) { device_entry("csr_sort_bytes"); }
hipError_t csr_mode(const CsrMode &, hipStream_t) { device_entry("csr_mode"); }
hipError_t launch_loss(const LossArgs &, hipStream_t) { device_entry("launch_loss"); }
hipError_t launch_loss_coo_noalloc(const LossArgs &, const LossArgs &, double, double *, hipStream_t)
{
    device_entry("launch_loss_coo_noalloc");
}
hipError_t launch_init_factor(float *, uint16_t *, int64_t, int32_t, uint64_t, float, hipStream_t)
{
    device_entry("launch_init_factor");
}
hipError_t launch_to_bf16(const float *, uint16_t *, int64_t, hipStream_t) { device_entry("launch_to_bf16"); }
hipError_t launch_debug_sample(const int64_t *, int64_t, uint64_t, int64_t, int32_t, int32_t, double, int32_t *,
                               int32_t *, hipStream_t)
{
    device_entry("launch_debug_sample");
}
hipError_t launch_row_kernel(RowKernel, const KernelClass &, const Launch &, hipStream_t)
{
    device_entry("launch_row_kernel");
}
hipError_t launch_advance(int64_t *, int32_t, hipStream_t) { device_entry("launch_advance"); }
int32_t row_kernel_blocks(RowKernel, const KernelClass &, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t)
{
    device_entry("row_kernel_blocks");
}
}  // namespace ntc

namespace {

int g_failures = 0;

void check(bool ok, const std::string &what)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what.c_str());
        ++g_failures;
    }
}

// splitmix64: input generator only
struct Gen {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return static_cast<double>(next() >> 11) * 0x1.0p-53; }
};

struct Coo {
    std::vector<int64_t> dims;
    std::vector<int32_t> coords;
    std::vector<float> values;
    int64_t nnz() const { return static_cast<int64_t>(values.size()); }
};

// Coordinates of mode 0 skewed like Zipf(s) by inverse-power sampling, the
// others uniform; values in (0, 1].
Coo make_coo(std::vector<int64_t> dims, int64_t nnz, double zipf_s, uint64_t seed)
{
    Coo p;
    p.dims = dims;
    Gen g{seed};
    const size_t N = dims.size();
    p.coords.resize(static_cast<size_t>(nnz) * N);
    p.values.resize(static_cast<size_t>(nnz));
    for (int64_t e = 0; e < nnz; ++e) {
        for (size_t m = 0; m < N; ++m) {
            int64_t i;
            if (m == 0 && zipf_s > 0.0) {
                const double u = g.uniform();
                i = static_cast<int64_t>(std::pow(u, 1.0 + 2.0 * zipf_s) * static_cast<double>(dims[0]));
            } else {
                i = static_cast<int64_t>(g.next() % static_cast<uint64_t>(dims[m]));
            }
            p.coords[static_cast<size_t>(e) * N + m] = static_cast<int32_t>(i < dims[m] ? i : dims[m] - 1);
        }
        p.values[static_cast<size_t>(e)] = static_cast<float>(1.0 - g.uniform());
    }
    return p;
}

int64_t samples_of(double c, int64_t n) { return static_cast<int64_t>(std::floor(c * static_cast<double>(n))); }

// Every row with B_p > 0 scheduled once, split rows covering [0, B_p) in
// order from slots in range; every row pointer in order.
void check_schedule(ntc_prepared_handle q, const Coo &p, int32_t R, const ntc_params &prm, const std::string &tag)
{
    const int32_t N = static_cast<int32_t>(p.dims.size());
    for (int32_t m = 0; m < N; ++m) {
        const std::string t = tag + " mode " + std::to_string(m);
        int64_t counts[7];
        check(ntc_prepared_schedule(q, m, counts, nullptr, nullptr, nullptr, nullptr, nullptr) == NTC_OK,
              t + ": counts");
        const int64_t I = p.dims[static_cast<size_t>(m)];
        std::vector<int64_t> rp(static_cast<size_t>(I + 1));
        std::vector<int32_t> tiny(static_cast<size_t>(counts[0] * 4)), items(static_cast<size_t>(counts[1] * 4)),
            split(static_cast<size_t>(counts[3] * 4)), groups(static_cast<size_t>(counts[4] * 4));
        check(ntc_prepared_schedule(q, m, counts, rp.data(), tiny.data(), items.data(), split.data(),
                                    groups.data()) == NTC_OK,
              t + ": tables");
        bool ordered = rp[0] == 0 && rp[static_cast<size_t>(I)] == p.nnz();
        for (int64_t i = 0; i < I; ++i)
            ordered = ordered && rp[static_cast<size_t>(i)] <= rp[static_cast<size_t>(i + 1)];
        check(ordered, t + ": row pointers");
        if (!ordered)
            continue;

        std::vector<int64_t> rowptr2(static_cast<size_t>(I + 1)), perm(static_cast<size_t>(std::max<int64_t>(p.nnz(), 1)));
        check(ntc_host_csr(N, p.dims.data(), p.nnz(), p.coords.data(), m, rowptr2.data(), perm.data()) == NTC_OK &&
                  rowptr2 == rp,
              t + ": ntc_host_csr row pointers");

        std::vector<int64_t> b(static_cast<size_t>(I));
        int64_t total = 0;
        for (int64_t i = 0; i < I; ++i) {
            b[static_cast<size_t>(i)] = samples_of(prm.c, rp[static_cast<size_t>(i + 1)] - rp[static_cast<size_t>(i)]);
            total += b[static_cast<size_t>(i)];
        }
        check(counts[6] == total, t + ": sampled entries");
        std::vector<int> claimed(static_cast<size_t>(I), 0);
        auto claim = [&](int64_t row) {
            if (row < 0 || row >= I) {
                check(false, t + ": row out of range");
                return;
            }
            ++claimed[static_cast<size_t>(row)];
        };
        for (int64_t x = 0; x < counts[0]; ++x)
            claim(tiny[static_cast<size_t>(4 * x)]);
        const bool row_items = R <= 16 && N <= 4;
        std::vector<int64_t> slot_row(static_cast<size_t>(counts[5]), -1), slot_j0(slot_row), slot_j1(slot_row);
        for (int64_t x = 0; x < counts[1]; ++x) {
            const int32_t *w = &items[static_cast<size_t>(4 * x)];
            if (row_items && x < counts[2]) {
                claim(w[0]);
                continue;
            }
            if (w[3] < 0) {
                claim(w[0]);
                continue;
            }
            const bool ok = w[3] < counts[5] && slot_row[static_cast<size_t>(w[3])] < 0 && w[0] >= 0 && w[0] < I &&
                            0 <= w[1] && w[1] < w[2] && w[2] <= b[static_cast<size_t>(w[0])];
            check(ok, t + ": partial item " + std::to_string(x));
            if (ok) {
                slot_row[static_cast<size_t>(w[3])] = w[0];
                slot_j0[static_cast<size_t>(w[3])] = w[1];
                slot_j1[static_cast<size_t>(w[3])] = w[2];
            }
        }
        std::vector<std::vector<int64_t>> group_src(static_cast<size_t>(counts[5]));
        for (int64_t x = 0; x < counts[4]; ++x) {
            const int32_t *w = &groups[static_cast<size_t>(4 * x)];
            const bool ok = w[1] >= 1 && w[0] >= 0 && int64_t(w[0]) + w[1] <= counts[5] && w[2] >= 0 &&
                            w[2] < counts[5];
            check(ok, t + ": slot group " + std::to_string(x));
            if (ok)
                for (int32_t k = 0; k < w[1]; ++k)
                    group_src[static_cast<size_t>(w[2])].push_back(w[0] + k);
        }
        std::set<int64_t> used;
        for (int64_t x = 0; x < counts[3]; ++x) {
            const int32_t *w = &split[static_cast<size_t>(4 * x)];
            if (!(w[2] >= 1 && w[1] >= 0 && int64_t(w[1]) + w[2] <= counts[5])) {
                check(false, t + ": split row slots out of range");
                continue;
            }
            std::vector<int64_t> slots;
            for (int32_t k = 0; k < w[2]; ++k) {
                const int64_t s = w[1] + k;
                if (!group_src[static_cast<size_t>(s)].empty())
                    slots.insert(slots.end(), group_src[static_cast<size_t>(s)].begin(),
                                 group_src[static_cast<size_t>(s)].end());
                else
                    slots.push_back(s);
            }
            int64_t j = 0;
            bool ok = true;
            for (int64_t s : slots) {
                ok = ok && slot_row[static_cast<size_t>(s)] == w[0] && slot_j0[static_cast<size_t>(s)] == j &&
                     used.insert(s).second;
                j = slot_j1[static_cast<size_t>(s)];
            }
            ok = ok && w[0] >= 0 && w[0] < I && j == b[static_cast<size_t>(w[0])];
            check(ok, t + ": split row " + std::to_string(w[0]));
            claim(w[0]);
        }
        bool once = true;
        for (int64_t i = 0; i < I; ++i)
            once = once && claimed[static_cast<size_t>(i)] == (b[static_cast<size_t>(i)] > 0 ? 1 : 0);
        check(once, t + ": rows with samples scheduled exactly once");

        // host sampler on the longest row and a few others: B_p distinct positions in [0, n_p)
        int64_t longest = 0;
        for (int64_t i = 1; i < I; ++i)
            if (rp[static_cast<size_t>(i + 1)] - rp[static_cast<size_t>(i)] >
                rp[static_cast<size_t>(longest + 1)] - rp[static_cast<size_t>(longest)])
                longest = i;
        for (int64_t row : {longest, I / 2, I - 1}) {
            const int64_t n = rp[static_cast<size_t>(row + 1)] - rp[static_cast<size_t>(row)];
            std::vector<int32_t> pos(static_cast<size_t>(std::max<int64_t>(samples_of(prm.c, n), 1)));
            int64_t cnt = -1;
            const bool ok = ntc_host_sample(prm.seed, 3, m, 0, row, n, prm.c, pos.data(), &cnt) == NTC_OK;
            std::set<int32_t> seen(pos.begin(), pos.begin() + std::max<int64_t>(cnt, 0));
            bool in_range = true;
            for (int64_t s = 0; s < cnt; ++s)
                in_range = in_range && pos[static_cast<size_t>(s)] >= 0 && pos[static_cast<size_t>(s)] < n;
            check(ok && cnt == samples_of(prm.c, n) && static_cast<int64_t>(seen.size()) == cnt && in_range,
                  t + ": host sampler on row " + std::to_string(row));
        }
    }
}

void run_case(const std::string &tag, const Coo &p, int32_t R, ntc_params prm, int64_t n_test = 0)
{
    const int32_t N = static_cast<int32_t>(p.dims.size());
    Coo test;
    if (n_test > 0) {
        test = make_coo(p.dims, n_test, 0.0, 0xC0FFEEull + static_cast<uint64_t>(R));
        prm.n_test = n_test;
        prm.test_coords = test.coords.data();
        prm.test_values = test.values.data();
    }
    ntc_prepared_handle q = nullptr;
    const ntc_status s = ntc_prepare(&q, N, p.dims.data(), p.nnz(), p.coords.data(), p.values.data(), R, &prm);
    check(s == NTC_OK && q, tag + ": ntc_prepare (" + ntc_last_error() + ")");
    if (s != NTC_OK)
        return;
    size_t bytes = 0, estimate = 0;
    check(ntc_prepared_bytes(q, &bytes) == NTC_OK && bytes > 0, tag + ": ntc_prepared_bytes");
    const ntc_status se = ntc_estimate_bytes(N, p.dims.data(), p.nnz(), R, &prm, &estimate);
    check(se == NTC_OK, tag + ": ntc_estimate_bytes (" + ntc_last_error() + ")");
    check(se != NTC_OK || estimate >= bytes, tag + ": ntc_estimate_bytes is an upper bound (" +
                                                 std::to_string(estimate) + " < " + std::to_string(bytes) + ")");
    check_schedule(q, p, R, prm, tag);
    check(ntc_prepared_release(q) == NTC_OK, tag + ": release");
}

// A call that must fail with `want`, leave *out NULL and set a message.
void expect_error(const std::string &tag, ntc_status want, const Coo &p, int32_t R, const ntc_params &prm,
                  int32_t nmodes = -1, int64_t nnz = -1)
{
    ntc_prepared_handle q = reinterpret_cast<ntc_prepared_handle>(&g_failures);  // overwritten with NULL
    const int32_t N = nmodes >= 0 ? nmodes : static_cast<int32_t>(p.dims.size());
    const ntc_status s = ntc_prepare(&q, N, p.dims.data(), nnz >= 0 ? nnz : p.nnz(), p.coords.data(),
                                     p.values.data(), R, &prm);
    check(s == want && q == nullptr && std::strlen(ntc_last_error()) > 0,
          tag + ": expected status " + std::to_string(want) + ", got " + std::to_string(s));
    if (s == NTC_OK)
        ntc_prepared_release(q);
}

}  // namespace

int main()
{
    ntc_params d;
    ntc_params_default(&d);

    const Coo zipf3 = make_coo({4000, 300, 40}, 120000, 1.1, 1);
    run_case("3-way R=16 default schedule", zipf3, 16, d);
    {
        ntc_params p = d;
        p.c = 0.3;
        p.item_samples = 64;
        p.group_max = 32;
        p.tiny_max = 2;
        run_case("3-way R=16 small chunks", zipf3, 16, p, 500);
    }
    {
        ntc_params p = d;
        p.tiny_max = 0;
        p.group_max = 0;
        p.gather_bf16 = 1;
        p.max_inner = 3;
        run_case("3-way R=8 no tiny rows, BF16, MAX_INNER 3", zipf3, 8, p);
    }
    const Coo zipf4 = make_coo({3000, 2000, 60, 20}, 150000, 1.05, 2);
    run_case("4-way R=32 few-sample rows", zipf4, 32, d);
    {
        ntc_params p = d;
        p.tiny_max = 5;
        p.item_samples = 16;
        p.c = 0.8;
        run_case("4-way R=24 slot groups", zipf4, 24, p, 1000);
    }
    run_case("4-way R=50", zipf4, 50, d);
    {
        ntc_params p = d;
        p.c = 1.0;
        run_case("matrix R=64 full batch", make_coo({400, 300}, 60000, 0.0, 3), 64, p);
    }
    run_case("5-way R=16", make_coo({20, 15, 12, 10, 8}, 30000, 0.0, 4), 16, d);
    run_case("8-way R=1", make_coo({5, 4, 3, 3, 3, 2, 2, 2}, 2000, 0.0, 5), 1, d);
    run_case("one row per mode", make_coo({1, 1, 1}, 50, 0.0, 6), 4, d);
    run_case("empty", make_coo({7, 5, 3}, 0, 0.0, 7), 16, d);
    run_case("rows without samples", make_coo({50000, 40, 30}, 20000, 0.0, 8), 16, d);
    {
        // caller's initial factors, all entries 0.5
        const Coo p3 = make_coo({60, 50, 40}, 8000, 0.5, 9);
        std::vector<std::vector<float>> init;
        std::vector<const float *> ptr;
        for (int64_t I : p3.dims)
            init.emplace_back(static_cast<size_t>(I) * 12, 0.5f);
        for (auto &v : init)
            ptr.push_back(v.data());
        ntc_params p = d;
        p.init_factors = ptr.data();
        run_case("caller's init factors", p3, 12, p, 200);
    }

    // invalid arguments
    const Coo small = make_coo({30, 20, 10}, 500, 0.0, 10);
    ntc_params p = d;
    expect_error("rank 0", NTC_EINVAL, small, 0, p);
    expect_error("rank 65", NTC_EINVAL, small, 65, p);
    expect_error("one mode", NTC_EINVAL, small, 8, p, 1);
    p.c = 0.0;
    expect_error("c = 0", NTC_EINVAL, small, 8, p);
    p.c = 1.5;
    expect_error("c > 1", NTC_EINVAL, small, 8, p);
    p = d;
    p.lambda = -1.0;
    expect_error("negative lambda", NTC_EINVAL, small, 8, p);
    p = d;
    p.max_inner = 0;
    expect_error("MAX_INNER 0", NTC_EINVAL, small, 8, p);
    p = d;
    p.tiny_max = 5;
    expect_error("tiny_max 5 at R = 16", NTC_EINVAL, small, 16, p);
    p = d;
    p.item_samples = 8;
    expect_error("item_samples 8", NTC_EINVAL, small, 16, p);
    {
        Coo bad = small;
        bad.coords[bad.coords.size() - 1] = static_cast<int32_t>(bad.dims[2]);
        expect_error("coordinate past the last row", NTC_EINVAL, bad, 8, d);
        bad = small;
        bad.coords[0] = -1;
        expect_error("negative coordinate", NTC_EINVAL, bad, 8, d);
        bad = small;
        bad.values[bad.values.size() / 2] = NAN;
        expect_error("NaN value", NTC_EINVAL, bad, 8, d);
        bad = small;
        bad.dims[1] = 0;
        expect_error("empty mode", NTC_EINVAL, bad, 8, d);
    }
    {
        Coo test = make_coo(small.dims, 10, 0.0, 11);
        test.coords[5] = 1000;
        p = d;
        p.n_test = 10;
        p.test_coords = test.coords.data();
        p.test_values = test.values.data();
        expect_error("held-out coordinate out of range", NTC_EINVAL, small, 8, p);
    }
    {
        std::vector<float> f0(30 * 8, 0.1f), f1(20 * 8, 0.1f), f2(10 * 8, 0.1f);
        f1[17] = -0.25f;
        const float *ptr[3] = {f0.data(), f1.data(), f2.data()};
        p = d;
        p.init_factors = ptr;
        expect_error("negative initial factor", NTC_EINVAL, small, 8, p);
    }
    check(ntc_prepared_release(nullptr) == NTC_OK, "release of NULL");
    int64_t counts[7];
    check(ntc_prepared_schedule(nullptr, 0, counts, nullptr, nullptr, nullptr, nullptr, nullptr) == NTC_EINVAL,
          "schedule of NULL");
    check(ntc_host_csr(3, small.dims.data(), small.nnz(), small.coords.data(), 3, nullptr, nullptr) == NTC_EINVAL,
          "host CSR of a mode out of range");

    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("sanitized host code: ok (%s)\n", ntc_version());
    return 0;
}
