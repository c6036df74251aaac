/*
 * Driver for the address/undefined-behaviour sanitizer run of the FP64
 * oracle (test infrastructure, built by tests/test_oracle_sanitizers.py with
 * gcc only).  It exercises every entry point of ntc_oracle.c on small
 * seeded problems: CSR build, sampler, sweeps for N = 2..5 and R = 1..64,
 * MAX_INNER > 1, lambda = 0, both L_p estimators, the BF16-gather form, the
 * row-by-row update and the loss, plus a problem with no entries and one
 * whose rows are all skipped.  Exit status 0 when every call returned.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct ora ora_t;
ora_t *ora_create(int N, const int64_t *dims, int64_t nnz, const int32_t *coords, const float *values, int R,
                  double c, double lambda, int max_inner, int power_iters, uint64_t seed, int64_t n_test,
                  const int32_t *test_coords, const float *test_values, const float *const *init);
void ora_free(ora_t *o);
void ora_sweep(ora_t *o, int nsweeps);
void ora_update_rows(const ora_t *o, int i, const int64_t *rows, int64_t nrows, double *out);
void ora_loss(const ora_t *o, double out[4]);
void ora_get_factors(const ora_t *o, int m, double *out);
void ora_set_factors(ora_t *o, int m, const double *in);
void ora_get_csr(const ora_t *o, int m, int64_t *rowptr_out, int64_t *perm_out);
void ora_set_lp_bound(ora_t *o, int bound);
void ora_set_gather_bf16(ora_t *o, int on);
int64_t ora_sample_positions(uint64_t seed, int64_t k, int32_t mode, int32_t l, int64_t row, int64_t n, double c,
                             int32_t *pos);
double ora_power_lmax(const double *H, int R, int T);
double ora_lmax_cw(const double *H, int R, int T);
int ora_set_threads(int n);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 11);
}

static int run(int N, const int64_t *dims, int64_t nnz, int R, double c, double lam, int inner, int T, int cw,
               int bf16, int ntest)
{
    int32_t *co = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1) * N);
    float *va = malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *tc = malloc(sizeof(int32_t) * (size_t)(ntest > 0 ? ntest : 1) * N);
    float *tv = malloc(sizeof(float) * (size_t)(ntest > 0 ? ntest : 1));
    for (int64_t e = 0; e < nnz; ++e) {
        for (int m = 0; m < N; ++m)
            co[e * N + m] = (int32_t)(next_u32() % (uint32_t)dims[m]);
        va[e] = (float)(next_u32() % 1000) / 250.0f;
    }
    for (int e = 0; e < ntest; ++e) {
        for (int m = 0; m < N; ++m)
            tc[e * N + m] = (int32_t)(next_u32() % (uint32_t)dims[m]);
        tv[e] = 1.0f;
    }
    ora_t *o = ora_create(N, dims, nnz, co, va, R, c, lam, inner, T, 7, ntest, tc, tv, NULL);
    if (!o)
        return 1;
    ora_set_lp_bound(o, cw);
    ora_set_gather_bf16(o, bf16);
    ora_sweep(o, 2);
    double loss[4];
    ora_loss(o, loss);
    int64_t rows[3] = {0, dims[0] / 2, dims[0] - 1};
    double *out = malloc(sizeof(double) * 3 * (size_t)R);
    ora_update_rows(o, 0, rows, 3, out);
    double *f = malloc(sizeof(double) * (size_t)dims[1] * (size_t)R);
    ora_get_factors(o, 1, f);
    ora_set_factors(o, 1, f);
    int64_t *rp = malloc(sizeof(int64_t) * (size_t)(dims[N - 1] + 1));
    int64_t *perm = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    ora_get_csr(o, N - 1, rp, perm);
    ora_free(o);
    free(co); free(va); free(tc); free(tv); free(out); free(f); free(rp); free(perm);
    return 0;
}

int main(void)
{
    ora_set_threads(2);
    int bad = 0;
    const int64_t d3[3] = {30, 20, 10}, d2[2] = {50, 40}, d4[4] = {12, 10, 8, 6}, d5[5] = {8, 7, 6, 5, 4};
    bad |= run(3, d3, 3000, 8, 0.1, 1e-3, 1, 20, 0, 0, 100);
    bad |= run(3, d3, 3000, 16, 0.5, 0.0, 2, 3, 0, 1, 100);
    bad |= run(2, d2, 1500, 1, 1.0, 1e-2, 3, 20, 1, 0, 50);
    bad |= run(4, d4, 2500, 33, 0.3, 1e-3, 1, 0, 1, 1, 60);
    bad |= run(5, d5, 2000, 64, 0.4, 1e-3, 2, 40, 0, 0, 30);
    bad |= run(3, d3, 0, 4, 0.1, 1e-3, 1, 20, 0, 0, 0);        /* no entries */
    bad |= run(3, d3, 40, 4, 0.05, 1e-3, 1, 20, 0, 0, 5);      /* every row skipped */
    int32_t pos[64];
    for (int64_t n = 0; n < 64; ++n)
        (void)ora_sample_positions(3, 5, 1, 0, n, n, 0.5, pos);
    double H[4] = {2.0, 1.0, 1.0, 3.0};
    if (!(ora_power_lmax(H, 2, 20) > 0.0) || !(ora_lmax_cw(H, 2, 0) > 0.0))
        bad = 1;
    printf(bad ? "sanitized oracle: FAILED\n" : "sanitized oracle: ok\n");
    return bad;
}
