/*
 * FP64 CPU oracle for AO accelerated stochastic nonnegative tensor completion
 * (Siaminou, Papagiannakos, Kolomvakis, Liavas, arXiv 2109.09534).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the HIP library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the library.
 *
 * What it computes, step by step, in IEEE binary64:
 *   - Section II, eq. (Problem_TC): masked least squares + ridge over
 *     nonnegative CPD factors; the per-mode subproblem (Problem_MLS) in the
 *     unfolding of eq. (Y_(i) = U^(i) K^T) is an NMC problem (matrix_NMC).
 *   - Alg. 2: Gauss-Seidel sweeps over the modes 0..N-1; mode i is updated by
 *     S_NMC with the other modes' current factors.
 *   - Alg. 1 (S_NMC): A_0 = Y_0 = A_*; for l < MAX_INNER, every row p
 *     independently (Alg. 3 runs these rows in parallel): sample B_{l,p} =
 *     floor(c * ||M(p,:)||_0) of the row's observed entries (eq. M_hat_def and
 *     the sampling rule of Section II-B; skip the row when that is 0), form
 *     the sampled gradient W + Z + lambda*Y(p,:) and the row Hessian
 *     H = B^T diag(M_hat(p,:)) B + lambda*I, take L_p = max eig(H) by the power
 *     method, step A_{l+1}(p,:) = (Y(p,:) - grad/L_p)_+, then extrapolate with
 *     beta = (sqrt(L_p) - sqrt(lambda)) / (sqrt(L_p) + sqrt(lambda)).
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - the minibatch of a row is a uniformly drawn subset without replacement,
 *     fresh for every (sweep k, mode i, inner step l, row p): a Feistel
 *     permutation of [0, n_p) keyed by one Philox4x32-10 block; the sample is
 *     the permutation's first B_{l,p} images, summed in that order;
 *   - the power method starts at 1/sqrt(R) * ones, runs T_pow normalised
 *     products and returns the Rayleigh quotient;
 *   - optional estimator (the paper leaves better L_p estimates open,
 *     Section III): the Collatz-Wielandt upper bound of the same iterate,
 *     L_p = max_i (H v)_i / v_i over the i with v_i > 0.  H is entrywise
 *     nonnegative here (a Gram matrix of nonnegative rows plus lambda I), so
 *     by the Collatz-Wielandt formula this is >= lambda_max(H) for every
 *     positive v, and it is the largest row sum of H when T_pow = 0;
 *   - optional precision form (an option of this implementation, not of the
 *     paper): the other modes' factor values enter the Khatri-Rao rows as
 *     bfloat16 copies of their FP32 values (ora_bf16); everything else,
 *     including the row's own y, stays binary64;
 *   - lambda is not scaled by c; rows with B_{l,p} = 0, or with L_p <= 0,
 *     keep A and Y unchanged;
 *   - Nesterov restarts at every S_NMC call; Y is discarded on return;
 *   - the CSR of mode m is a stable sort of the COO entries by i_m.
 *
 * Philox4x32-10 follows Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3" (SC'11).  The permutation of [0, n) is a Feistel
 * network over a mixed-radix domain Z_A x Z_B with modular addition (the
 * FFX construction of Bellare, Rogaway and Spies, 2010; 8 rounds, 24 on
 * domains of at most 16 words), restricted to [0, n) by cycle walking
 * (Black and Rogaway, "Ciphers with arbitrary finite domains", 2002).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAXN 8
#define ORA_MAXR 64

/* Counter-layout tags of the sampler and of the default initialisation. */
#define ORA_TAG_SAMPLE 0x53414D50u
#define ORA_TAG_INIT 0x494E4954u

typedef struct ora {
    int N, R;
    int64_t dims[ORA_MAXN];
    int64_t nnz;
    int32_t *coords; /* [nnz][N] train COO (copied) */
    double *vals;    /* [nnz] train values, promoted from FP32 */
    int64_t *rowptr[ORA_MAXN];
    int64_t *perm[ORA_MAXN]; /* CSR of mode m: COO entry ids, stably sorted by i_m */
    double *U[ORA_MAXN];     /* factors, row-major [I_m][R] */
    double c, lambda;
    int max_inner, power_iters;
    int lp_bound; /* 0: Rayleigh quotient of the power iterate; 1: Collatz-Wielandt bound */
    int gather_bf16; /* 1: the other modes' factor values enter the Khatri-Rao rows as BF16 copies */
    uint64_t seed;
    int64_t k; /* AO sweep counter */
    int64_t n_test;
    int32_t *tcoords;
    double *tvals;
} ora_t;

/* ------------------------------------------------------------------ Philox */
/* One Philox-4x32 round: two 32x32->64 multiplies, then the fixed word
 * permutation with the round key mixed into the high halves. */
static void philox_round(uint32_t x[4], const uint32_t key[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ key[0];
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x[3] ^ key[1];
    uint32_t y3 = lo0;
    x[0] = y0;
    x[1] = y1;
    x[2] = y2;
    x[3] = y3;
}

/* Philox4x32 with `rounds` rounds; the key is bumped by the Weyl constants
 * between rounds. */
void ora_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < rounds; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(x, k);
    }
    out[0] = x[0];
    out[1] = x[1];
    out[2] = x[2];
    out[3] = x[3];
}

/* Round keys of the row sampler for (seed, sweep k, mode i, inner l, row p). */
void ora_sample_keys(uint64_t seed, int64_t k, int32_t mode, int32_t l, int64_t row, uint32_t keys[4])
{
    uint32_t ctr[4] = {(uint32_t)row, (uint32_t)k, ((uint32_t)mode << 16) | ((uint32_t)l & 0xFFFFu),
                       ORA_TAG_SAMPLE};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    ora_philox4x32(ctr, key, 10, keys);
}

/* ----------------------------------------------------------------- Feistel */
/* Round function on 32 bits: key xor, then two rounds of xor-shift and a
 * multiply of the low 24 bits by a 24-bit odd constant (low 32 bits kept). */
static uint32_t feistel_f(uint32_t x, uint32_t key)
{
    uint32_t h = x ^ key;
    h ^= h >> 16;
    h = (h & 0xFFFFFFu) * 0x9E3779u;
    h ^= h >> 13;
    h = (h & 0xFFFFFFu) * 0xC2B2AEu;
    h ^= h >> 16;
    return h;
}

/* w = the smallest integer >= 2 with 2^w >= n. */
int ora_feistel_width(int64_t n)
{
    int w = 2;
    while (((int64_t)1 << w) < n)
        ++w;
    return w;
}

/* Number of rounds: 24 when w <= 4 (tiny domains need many rounds before
 * every subset is about equally likely), 8 otherwise. */
int ora_feistel_rounds(int w) { return w <= 4 ? 24 : 8; }

/* One pass of the Feistel network over the mixed-radix domain Z_A x Z_B,
 * A = 2^ceil(w/2), B = ceil(n / A), the word x = lo * A + hi with hi in Z_A,
 * lo in Z_B (FFX-style rounds with modular addition, Bellare, Rogaway and
 * Spies 2010).  Round r uses kappa_r = K[r mod 4] ^ (r * 0x9E3779B9); even
 * rounds set hi = (hi + F(lo, kappa_r)) mod A, odd rounds set
 * lo = (lo + ((F(hi, kappa_r) mod 2^16) * B) div 2^16) mod B.  Each round is a
 * bijection of Z_A x Z_B, so the pass permutes [0, A*B), and A*B - n < A. */
uint32_t ora_feistel_net(uint32_t x, int64_t n, const uint32_t keys[4])
{
    int w = ora_feistel_width(n);
    int a = (w + 1) / 2;
    uint32_t A = 1u << a;
    uint32_t B = (uint32_t)((n + A - 1) / A);
    uint32_t hi = x & (A - 1u), lo = x >> a;
    int rounds = ora_feistel_rounds(w);
    for (int r = 0; r < rounds; ++r) {
        uint32_t kappa = keys[r & 3] ^ (uint32_t)((uint32_t)r * 0x9E3779B9u);
        if ((r & 1) == 0) {
            hi = (hi + feistel_f(lo, kappa)) & (A - 1u);
        } else {
            uint32_t t = ((feistel_f(hi, kappa) & 0xFFFFu) * B) >> 16;
            lo = lo + t;
            if (lo >= B)
                lo -= B;
        }
    }
    return (lo << a) | hi;
}

/* pi(j): the network applied to j, re-applied while the image is >= n
 * (cycle walking, Black and Rogaway 2002). */
uint32_t ora_feistel_pos(uint32_t j, int64_t n, const uint32_t keys[4])
{
    uint32_t x = ora_feistel_net(j, n, keys);
    while ((int64_t)x >= n)
        x = ora_feistel_net(x, n, keys);
    return x;
}

/* Size A*B of the permuted word domain for a row of length n. */
int64_t ora_feistel_domain(int64_t n)
{
    int w = ora_feistel_width(n);
    int64_t A = (int64_t)1 << ((w + 1) / 2);
    return A * ((n + A - 1) / A);
}

/* B_{l,p} = floor(c * n): one binary64 multiply, then floor. */
int64_t ora_sample_size(double c, int64_t n)
{
    return (int64_t)floor(c * (double)n);
}

/* The sampled positions (within the row) of row `row` of length n. */
int64_t ora_sample_positions(uint64_t seed, int64_t k, int32_t mode, int32_t l, int64_t row, int64_t n,
                             double c, int32_t *pos_out)
{
    int64_t b = ora_sample_size(c, n);
    if (b <= 0)
        return 0;
    uint32_t keys[4];
    ora_sample_keys(seed, k, mode, l, row, keys);
    for (int64_t j = 0; j < b; ++j)
        pos_out[j] = (int32_t)ora_feistel_pos((uint32_t)j, n, keys);
    return b;
}

/* ------------------------------------------------------------ power method */
/* L = largest eigenvalue of the symmetric H (R x R, row-major), by T
 * normalised products from v = ones/sqrt(R); returns the Rayleigh quotient,
 * or 0 if H v vanishes. */
double ora_power_lmax(const double *H, int R, int T)
{
    double v[ORA_MAXR], w[ORA_MAXR];
    for (int r = 0; r < R; ++r)
        v[r] = 1.0 / sqrt((double)R);
    for (int t = 0; t < T; ++t) {
        double nrm2 = 0.0;
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
            for (int q = 0; q < R; ++q)
                s += H[r * R + q] * v[q];
            w[r] = s;
            nrm2 += s * s;
        }
        if (!(nrm2 > 0.0))
            return 0.0;
        double nrm = sqrt(nrm2);
        for (int r = 0; r < R; ++r)
            v[r] = w[r] / nrm;
    }
    double rq = 0.0;
    for (int r = 0; r < R; ++r) {
        double s = 0.0;
        for (int q = 0; q < R; ++q)
            s += H[r * R + q] * v[q];
        rq += v[r] * s;
    }
    return rq;
}

/* L as the Collatz-Wielandt upper bound max_i (H v)_i / v_i at the power
 * method's T-th normalised iterate (v_0 = ones/sqrt(R)), over the i with
 * v_i > 0; 0 if H v vanishes. */
double ora_lmax_cw(const double *H, int R, int T)
{
    double v[ORA_MAXR], w[ORA_MAXR];
    for (int r = 0; r < R; ++r)
        v[r] = 1.0 / sqrt((double)R);
    for (int t = 0; t < T; ++t) {
        double nrm2 = 0.0;
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
            for (int q = 0; q < R; ++q)
                s += H[r * R + q] * v[q];
            w[r] = s;
            nrm2 += s * s;
        }
        if (!(nrm2 > 0.0))
            return 0.0;
        double nrm = sqrt(nrm2);
        for (int r = 0; r < R; ++r)
            v[r] = w[r] / nrm;
    }
    double best = 0.0;
    for (int r = 0; r < R; ++r) {
        if (!(v[r] > 0.0))
            continue;
        double s = 0.0;
        for (int q = 0; q < R; ++q)
            s += H[r * R + q] * v[q];
        double ratio = s / v[r];
        if (ratio > best)
            best = ratio;
    }
    return best;
}

/* ----------------------------------------------------------------- set-up */
static void build_csr(ora_t *o, int m)
{
    int64_t I = o->dims[m];
    int64_t *rp = (int64_t *)calloc((size_t)I + 1, sizeof(int64_t));
    int64_t *perm = (int64_t *)malloc((size_t)(o->nnz > 0 ? o->nnz : 1) * sizeof(int64_t));
    for (int64_t e = 0; e < o->nnz; ++e)
        rp[o->coords[e * o->N + m] + 1] += 1;
    for (int64_t p = 0; p < I; ++p)
        rp[p + 1] += rp[p];
    int64_t *fill = (int64_t *)malloc((size_t)I * sizeof(int64_t));
    memcpy(fill, rp, (size_t)I * sizeof(int64_t));
    /* scanning the COO in order keeps ties in COO order (a stable sort) */
    for (int64_t e = 0; e < o->nnz; ++e) {
        int64_t p = o->coords[e * o->N + m];
        perm[fill[p]++] = e;
    }
    free(fill);
    o->rowptr[m] = rp;
    o->perm[m] = perm;
}

void ora_free(ora_t *o);

/* Returns NULL on invalid input.  `init` is NULL or N arrays of FP32 factors
 * (I_m x R row-major); otherwise factors are Philox Uniform[0,1) * s with
 * s = (mean(x) / (R * 2^-N))^(1/N) rounded to FP32. */
ora_t *ora_create(int N, const int64_t *dims, int64_t nnz, const int32_t *coords, const float *values,
                  int R, double c, double lambda, int max_inner, int power_iters, uint64_t seed,
                  int64_t n_test, const int32_t *test_coords, const float *test_values,
                  const float *const *init)
{
    if (N < 2 || N > ORA_MAXN || R < 1 || R > ORA_MAXR || nnz < 0 || !(c > 0.0 && c <= 1.0) ||
        !(lambda >= 0.0) || max_inner < 1 || power_iters < 0)
        return NULL;
    ora_t *o = (ora_t *)calloc(1, sizeof(ora_t));
    o->N = N;
    o->R = R;
    o->nnz = nnz;
    o->c = c;
    o->lambda = lambda;
    o->max_inner = max_inner;
    o->power_iters = power_iters;
    o->seed = seed;
    o->k = 0;
    for (int m = 0; m < N; ++m)
        o->dims[m] = dims[m];
    o->coords = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * N * sizeof(int32_t));
    o->vals = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    for (int64_t e = 0; e < nnz; ++e) {
        for (int m = 0; m < N; ++m) {
            int32_t ix = coords[e * N + m];
            if (ix < 0 || ix >= dims[m]) {
                ora_free(o);
                return NULL;
            }
            o->coords[e * N + m] = ix;
        }
        o->vals[e] = (double)values[e];
    }
    for (int m = 0; m < N; ++m)
        build_csr(o, m);
    o->n_test = n_test;
    o->tcoords = (int32_t *)malloc((size_t)(n_test > 0 ? n_test : 1) * N * sizeof(int32_t));
    o->tvals = (double *)malloc((size_t)(n_test > 0 ? n_test : 1) * sizeof(double));
    for (int64_t e = 0; e < n_test; ++e) {
        for (int m = 0; m < N; ++m)
            o->tcoords[e * N + m] = test_coords[e * N + m];
        o->tvals[e] = (double)test_values[e];
    }
    float s = 1.0f;
    if (!init) {
        double sum = 0.0;
        for (int64_t e = 0; e < nnz; ++e)
            sum += o->vals[e];
        double mean = nnz > 0 ? sum / (double)nnz : 0.0;
        if (!(mean > 1e-30))
            mean = 1e-30;
        s = (float)pow(mean / ((double)R * pow(2.0, -(double)N)), 1.0 / (double)N);
    }
    for (int m = 0; m < N; ++m) {
        int64_t cnt = dims[m] * R;
        o->U[m] = (double *)malloc((size_t)cnt * sizeof(double));
        if (init) {
            for (int64_t t = 0; t < cnt; ++t)
                o->U[m][t] = (double)init[m][t];
        } else {
            uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
            for (int64_t t = 0; t < cnt; ++t) {
                uint64_t blk = (uint64_t)t >> 2;
                uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), (uint32_t)m, ORA_TAG_INIT};
                uint32_t out[4];
                ora_philox4x32(ctr, key, 10, out);
                float u = (float)(out[t & 3] >> 8) * 0x1p-24f;
                o->U[m][t] = (double)(u * s);
            }
        }
    }
    return o;
}

void ora_free(ora_t *o)
{
    if (!o)
        return;
    for (int m = 0; m < ORA_MAXN; ++m) {
        free(o->rowptr[m]);
        free(o->perm[m]);
        free(o->U[m]);
    }
    free(o->coords);
    free(o->vals);
    free(o->tcoords);
    free(o->tvals);
    free(o);
}

/* ---------------------------------------------------------- BF16 copies */
/* The precision form (not the paper's: an option of this implementation)
 * keeps FP32 factors and gathers the other modes' rows from BF16 copies of
 * them.  The copy of a factor value x is defined here from the two formats:
 * x is first the FP32 factor entry (round to nearest, ties to even, as a C
 * conversion does), then the bfloat16 number nearest to it (1 sign bit,
 * 8 exponent bits, 7 fraction bits: the FP32 numbers whose low 16 bits are
 * zero), ties to the one with an even last fraction bit.  Only finite values
 * below the largest bfloat16 occur (factors are finite and >= 0). */
double ora_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    uint32_t lo_bits = u & 0xFFFF0000u;             /* the bfloat16 toward zero */
    uint32_t hi_bits = lo_bits + 0x00010000u;        /* the next one away from zero */
    float lo, hi;
    memcpy(&lo, &lo_bits, sizeof lo);
    memcpy(&hi, &hi_bits, sizeof hi);
    double dl = fabs((double)f - (double)lo), dh = fabs((double)hi - (double)f);
    if (dl < dh)
        return (double)lo;
    if (dh < dl)
        return (double)hi;
    return (lo_bits & 0x00010000u) ? (double)hi : (double)lo; /* tie: even last bit */
}

/* ------------------------------------------------------------ one row step */
/* Alg. 1 for row p of mode i at inner step l, with the other modes' factors
 * as they are now.  y, a are Y_l(p,:), A_l(p,:); writes A_{l+1}(p,:) and
 * Y_{l+1}(p,:).  Optional outputs: the sampled gradient at y (with ridge),
 * the row Hessian (with ridge), L_p and beta.  Returns the sample size used
 * (0 = row skipped). */
int64_t ora_row_step(const ora_t *o, int i, int l, int64_t p, const double *y, const double *a,
                     double *a_next, double *y_next, double *g_out, double *H_out, double *L_out,
                     double *beta_out)
{
    const int R = o->R, N = o->N;
    int64_t start = o->rowptr[i][p];
    int64_t n = o->rowptr[i][p + 1] - start;
    int64_t b = ora_sample_size(o->c, n);
    if (b <= 0) {
        memcpy(a_next, a, (size_t)R * sizeof(double));
        memcpy(y_next, y, (size_t)R * sizeof(double));
        return 0;
    }
    uint32_t keys[4];
    ora_sample_keys(o->seed, o->k, i, l, p, keys);
    double g[ORA_MAXR], H[ORA_MAXR * ORA_MAXR], ks[ORA_MAXR];
    memset(g, 0, sizeof(double) * (size_t)R);
    memset(H, 0, sizeof(double) * (size_t)R * (size_t)R);
    for (int64_t j = 0; j < b; ++j) {
        int64_t q = ora_feistel_pos((uint32_t)j, n, keys);
        int64_t e = o->perm[i][start + q];
        /* Khatri-Rao row of the sampled entry: Hadamard product of the other
         * modes' factor rows, in increasing mode order */
        for (int r = 0; r < R; ++r)
            ks[r] = 1.0;
        for (int m = 0; m < N; ++m) {
            if (m == i)
                continue;
            const double *row = o->U[m] + (int64_t)o->coords[e * N + m] * R;
            for (int r = 0; r < R; ++r)
                ks[r] *= o->gather_bf16 ? ora_bf16(row[r]) : row[r];
        }
        double pred = 0.0;
        for (int r = 0; r < R; ++r)
            pred += ks[r] * y[r];
        double res = pred - o->vals[e]; /* W + Z contribution: (k.y - x) k */
        for (int r = 0; r < R; ++r) {
            g[r] += res * ks[r];
            for (int q2 = 0; q2 < R; ++q2)
                H[r * R + q2] += ks[r] * ks[q2];
        }
    }
    for (int r = 0; r < R; ++r) {
        g[r] += o->lambda * y[r];
        H[r * R + r] += o->lambda;
    }
    double L = o->lp_bound ? ora_lmax_cw(H, R, o->power_iters) : ora_power_lmax(H, R, o->power_iters);
    double beta = 0.0;
    if (g_out)
        memcpy(g_out, g, sizeof(double) * (size_t)R);
    if (H_out)
        memcpy(H_out, H, sizeof(double) * (size_t)R * (size_t)R);
    if (L_out)
        *L_out = L;
    if (!(L > 0.0)) {
        memcpy(a_next, a, (size_t)R * sizeof(double));
        memcpy(y_next, y, (size_t)R * sizeof(double));
        if (beta_out)
            *beta_out = 0.0;
        return 0;
    }
    beta = (sqrt(L) - sqrt(o->lambda)) / (sqrt(L) + sqrt(o->lambda));
    for (int r = 0; r < R; ++r) {
        double an = y[r] - g[r] / L;
        an = an > 0.0 ? an : 0.0;
        a_next[r] = an;
        y_next[r] = an + beta * (an - a[r]);
    }
    if (beta_out)
        *beta_out = beta;
    return b;
}

/* ------------------------------------------------------------------ S_NMC */
/* Alg. 1 for mode i at the current sweep counter: MAX_INNER Jacobi passes
 * over the rows, each reading Y_l, A_l and writing Y_{l+1}, A_{l+1}. */
void ora_update_mode(ora_t *o, int i)
{
    const int R = o->R;
    const int64_t I = o->dims[i];
    size_t bytes = (size_t)I * R * sizeof(double);
    double *A = (double *)malloc(bytes), *Y = (double *)malloc(bytes);
    double *An = (double *)malloc(bytes), *Yn = (double *)malloc(bytes);
    memcpy(A, o->U[i], bytes);
    memcpy(Y, o->U[i], bytes);
    for (int l = 0; l < o->max_inner; ++l) {
        int64_t p;
#pragma omp parallel for schedule(dynamic, 16)
        for (p = 0; p < I; ++p)
            ora_row_step(o, i, l, p, Y + p * R, A + p * R, An + p * R, Yn + p * R, NULL, NULL, NULL, NULL);
        double *t = A;
        A = An;
        An = t;
        t = Y;
        Y = Yn;
        Yn = t;
    }
    memcpy(o->U[i], A, bytes);
    free(A);
    free(Y);
    free(An);
    free(Yn);
}

/* Alg. 2: `nsweeps` circular passes over the modes. */
void ora_sweep(ora_t *o, int nsweeps)
{
    for (int s = 0; s < nsweeps; ++s) {
        for (int i = 0; i < o->N; ++i)
            ora_update_mode(o, i);
        o->k += 1;
    }
}

/* Selected rows of a mode update, computed one by one from the current
 * factors without changing any state: out[t*R..] = U^(i)(rows[t],:) after
 * MAX_INNER inner steps. */
void ora_update_rows(const ora_t *o, int i, const int64_t *rows, int64_t nrows, double *out)
{
    const int R = o->R;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < nrows; ++t) {
        double a[ORA_MAXR], y[ORA_MAXR], an[ORA_MAXR], yn[ORA_MAXR];
        memcpy(a, o->U[i] + rows[t] * R, (size_t)R * sizeof(double));
        memcpy(y, a, (size_t)R * sizeof(double));
        for (int l = 0; l < o->max_inner; ++l) {
            ora_row_step(o, i, l, rows[t], y, a, an, yn, NULL, NULL, NULL, NULL);
            memcpy(a, an, (size_t)R * sizeof(double));
            memcpy(y, yn, (size_t)R * sizeof(double));
        }
        memcpy(out + t * R, a, (size_t)R * sizeof(double));
    }
}

/* ------------------------------------------------------------------- loss */
static double predict(const ora_t *o, const int32_t *cc)
{
    double s = 0.0;
    for (int r = 0; r < o->R; ++r) {
        double prod = 1.0;
        for (int m = 0; m < o->N; ++m)
            prod *= o->U[m][(int64_t)cc[m] * o->R + r];
        s += prod;
    }
    return s;
}

/* Sum of f(e) over [0, n) in fixed 4096-entry blocks, blocks summed in order
 * (independent of the thread count). */
static double sq_residual_sum(const ora_t *o, const int32_t *coords, const double *vals, int64_t n,
                              double *sq_x)
{
    int64_t nb = (n + 4095) / 4096;
    double *part = (double *)calloc((size_t)(nb > 0 ? nb : 1) * 2, sizeof(double));
    int64_t bi;
#pragma omp parallel for schedule(static)
    for (bi = 0; bi < nb; ++bi) {
        double s = 0.0, sx = 0.0;
        int64_t e1 = (bi + 1) * 4096 < n ? (bi + 1) * 4096 : n;
        for (int64_t e = bi * 4096; e < e1; ++e) {
            double r = vals[e] - predict(o, coords + e * o->N);
            s += r * r;
            sx += vals[e] * vals[e];
        }
        part[2 * bi] = s;
        part[2 * bi + 1] = sx;
    }
    double s = 0.0, sx = 0.0;
    for (bi = 0; bi < nb; ++bi) {
        s += part[2 * bi];
        sx += part[2 * bi + 1];
    }
    free(part);
    if (sq_x)
        *sq_x = sx;
    return s;
}

/* out = {objective (eq. Problem_TC), train RMSE, test RMSE, test RRE}. */
void ora_loss(const ora_t *o, double out[4])
{
    double sse = sq_residual_sum(o, o->coords, o->vals, o->nnz, NULL);
    double reg = 0.0;
    for (int m = 0; m < o->N; ++m)
        for (int64_t t = 0; t < o->dims[m] * o->R; ++t)
            reg += o->U[m][t] * o->U[m][t];
    out[0] = 0.5 * sse + 0.5 * o->lambda * reg;
    out[1] = o->nnz > 0 ? sqrt(sse / (double)o->nnz) : 0.0;
    if (o->n_test > 0) {
        double sx = 0.0;
        double tse = sq_residual_sum(o, o->tcoords, o->tvals, o->n_test, &sx);
        out[2] = sqrt(tse / (double)o->n_test);
        out[3] = sx > 0.0 ? sqrt(tse) / sqrt(sx) : 0.0;
    } else {
        out[2] = 0.0;
        out[3] = 0.0;
    }
}

/* --------------------------------------------------------------- accessors */
void ora_get_factors(const ora_t *o, int m, double *out)
{
    memcpy(out, o->U[m], (size_t)o->dims[m] * o->R * sizeof(double));
}
void ora_set_factors(ora_t *o, int m, const double *in)
{
    memcpy(o->U[m], in, (size_t)o->dims[m] * o->R * sizeof(double));
}
int64_t ora_get_sweep(const ora_t *o) { return o->k; }
void ora_set_sweep(ora_t *o, int64_t k) { o->k = k; }

/* 0: L_p is the Rayleigh quotient of the power iterate; 1: the
 * Collatz-Wielandt upper bound of the same iterate. */
void ora_set_lp_bound(ora_t *o, int bound) { o->lp_bound = bound ? 1 : 0; }
void ora_set_gather_bf16(ora_t *o, int on) { o->gather_bf16 = on ? 1 : 0; }
void ora_get_csr(const ora_t *o, int m, int64_t *rowptr_out, int64_t *perm_out)
{
    memcpy(rowptr_out, o->rowptr[m], (size_t)(o->dims[m] + 1) * sizeof(int64_t));
    memcpy(perm_out, o->perm[m], (size_t)o->nnz * sizeof(int64_t));
}
int ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
