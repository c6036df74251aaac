/*
 * ntc.h -- C ABI of libntc: AO accelerated stochastic nonnegative tensor
 * completion on one AMD MI355X (gfx950).
 *
 * Method: Siaminou, Papagiannakos, Kolomvakis, Liavas, "Accelerated
 * Stochastic Gradient for Nonnegative Tensor Completion and Parallel
 * Implementation" (arXiv 2109.09534).
 *   - Section II, eq. (Problem_TC): minimise 1/2 ||M * (X - [[U^(1..N)]])||_F^2
 *     + lambda/2 sum_i ||U^(i)||_F^2 over nonnegative factors.
 *   - Alg. 2: circular (Gauss-Seidel) updates of the modes; each mode update
 *     is the NMC problem of eq. (matrix_NMC) solved by Alg. 1.
 *   - Alg. 1: MAX_INNER row-wise steps; row p draws B_{l,p} = floor(c n_p) of
 *     its n_p observed entries (Section II-B), forms the sampled gradient and
 *     the row Hessian H_{l,p}, takes L_p = max eig(H_{l,p}) by the power
 *     method, steps A <- (Y - grad/L_p)_+ and extrapolates with
 *     beta = (sqrt(L_p) - sqrt(lambda)) / (sqrt(L_p) + sqrt(lambda)).
 *
 * Conventions for every entry point:
 *   - Every pointer argument is HOST memory owned by the caller, read or
 *     written before the call returns, unless stated otherwise.  Device memory
 *     belongs to the handle and is freed by ntc_release.
 *   - Indices are 0-based.  Factors are row-major FP32 arrays [I_m][R].
 *   - Every call returns an ntc_status; on failure ntc_last_error() gives a
 *     thread-local message.  Asynchronous device faults surface at the next
 *     synchronising call as NTC_EDEVICE.
 *   - One handle is driven by one host thread at a time; different handles
 *     are independent.  Work is enqueued on the stream given at creation.
 */
#ifndef NTC_H
#define NTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ntc_problem *ntc_handle;

typedef enum {
    NTC_OK = 0,
    NTC_EINVAL = -1,       /* invalid argument (message says which) */
    NTC_ENOMEM = -2,       /* device or host allocation failed */
    NTC_EDEVICE = -3,      /* HIP runtime error, including asynchronous faults */
    NTC_EUNSUPPORTED = -4, /* a valid request the library does not support */
    NTC_ENONFINITE = -5,   /* the loss evaluated to a non-finite value */
    NTC_ESTATE = -6        /* call not valid in the handle's current state */
} ntc_status;

/* Optional device allocator (e.g. PyTorch's caching allocator).  alloc
 * returns device memory usable on `stream`, or NULL; free releases it. */
typedef void *(*ntc_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*ntc_free_fn)(void *ptr, void *ctx);

typedef struct ntc_params {
    double c;             /* minibatch fraction, 0 < c <= 1 (Section II-B asks c < 1;
                             c == 1 makes every minibatch the whole row) */
    double lambda;        /* ridge weight >= 0 (eq. Problem_TC); not scaled by c */
    int32_t max_inner;    /* MAX_INNER of Alg. 1, >= 1 */
    int32_t power_iters;  /* normalised power-method products per row, >= 0 (default 20) */
    uint64_t seed;        /* Philox key of the minibatch sampler and the default init */
    int32_t gather_bf16;  /* 1: gather other-mode factor rows from a BF16 shadow copy
                             (FP32 master factors, FP32 accumulation) */
    int32_t tiny_max;     /* schedule: rows with 1 <= B_p <= tiny_max run several rows per
                             wave, one sample per lane: R <= 16 (four lanes per row; -1 =
                             default 4, at most 4) and 17 <= R <= 32 with nmodes <= 4 (16
                             lanes per row; -1 = default 16, at most 16); 0 = off */
    int64_t n_test;             /* optional held-out entries for ntc_loss (0 = none) */
    const int32_t *test_coords; /* [n_test][nmodes], host, copied */
    const float *test_values;   /* [n_test], host, copied */
    const float *const *init_factors; /* NULL: Philox Uniform[0,1)*s init (see ntc_create);
                                         else nmodes host arrays [I_m][R], entries >= 0 */
    void *stream;               /* hipStream_t; NULL = the null stream */
    ntc_alloc_fn dev_alloc;     /* optional; NULL = hipMalloc */
    ntc_free_fn dev_free;
    void *alloc_ctx;
    int32_t item_samples;       /* schedule: sampled entries per work item; longer minibatches
                                   are split over several items (0 = default) */
    int32_t overlap;            /* schedule: 1 = run the one-row-per-lane launch (and, for R <= 16,
                                   N <= 4, the one-row-per-group launch) on a second stream
                                   concurrently with the chunks (default); 2 = only the
                                   one-row-per-group launch on the second stream; 0 = serial */
    int32_t group_max;          /* schedule (R <= 16): rows with tiny_max < B_p <= group_max run
                                   one row per 16-lane group, longer ones as 256-thread chunks of
                                   item_samples entries (0 = default 512) */
    int32_t lp_bound;           /* L_p estimator: 0 = Rayleigh quotient of the T_pow-th power iterate
                                   (default); 1 = Collatz-Wielandt upper bound max_i (H v)_i / v_i of
                                   the same iterate (>= lambda_max for the nonnegative H here, so a
                                   shorter, safe step; with power_iters = 0 the largest row sum of H) */
} ntc_params;

/* Fill *p with defaults: c = 0.1, lambda = 1e-3, max_inner = 1,
 * power_iters = 20, seed = 0, FP32 gathers, no test set, default init,
 * null stream, hipMalloc, default schedule (tiny_max = -1, item_samples = 0,
 * overlap = 1).  The schedule changes the order of floating-point sums
 * only, never the sampled entries. */
void ntc_params_default(ntc_params *p);

/* Create a problem from the observed entries (Section II: X on Omega).
 *   nmodes in [2, 8]; dims[m] in [1, 2^31); nnz in [0, 2^31);
 *   coords [nnz][nmodes] int32, 0 <= coords < dims; values [nnz] finite FP32;
 *   rank R in [1, 64].
 * Builds one CSR per mode (entries stably sorted by i_m: the unfolding
 * X_(i), M_(i) of Section II), a static row schedule from
 * B_p = floor(c n_p), uploads everything and initialises the factors:
 * either the caller's init_factors, or Philox4x32-10 uniforms
 * u = (word >> 8) * 2^-24 times s = (mean(values) / (R 2^-N))^(1/N) rounded
 * to FP32.  The sweep counter k starts at 0.  Duplicate coordinates are
 * treated as separate observations.  On failure *out is NULL. */
ntc_status ntc_create(ntc_handle *out, int32_t nmodes, const int64_t *dims, int64_t nnz,
                      const int32_t *coords, const float *values, int32_t rank, const ntc_params *p);

/* ntc_create with the CSR built on the device: the COO entries (host
 * arrays, as for ntc_create) are copied to the GPU once and checked there,
 * and each mode's entries are sorted by i_m with a stable radix sort, so the
 * records, row pointers and every later result are bit-identical to
 * ntc_create's.  Only the row schedule is built on the host, from the row
 * pointers.  Temporaries (about 24 bytes per entry) come from hipMalloc and
 * are freed before return; what the problem keeps goes through dev_alloc as
 * in ntc_create.  Errors as ntc_create (the first bad entry is reported with
 * the same message); NTC_EDEVICE if the device build fails. */
ntc_status ntc_create_device_csr(ntc_handle *out, int32_t nmodes, const int64_t *dims, int64_t nnz,
                                 const int32_t *coords, const float *values, int32_t rank, const ntc_params *p);

/* ntc_create in two steps, for callers that build problems on other host
 * threads while the GPU works (serving):
 *   ntc_prepare      validates the arguments and does all host work (CSR of
 *                    every mode, row schedule, copies of the held-out set and
 *                    initial factors); it touches no device and no shared
 *                    state, so any host thread may call it;
 *   ntc_create_prepared  allocates, uploads and initialises, like the second
 *                    half of ntc_create; p supplies only stream, allocator and
 *                    overlap (its method parameters are those given to
 *                    ntc_prepare); the prepared problem is not consumed;
 *   ntc_prepared_bytes   the exact device bytes ntc_create_prepared allocates
 *                    (allocations rounded to 256 bytes);
 *   ntc_prepared_release frees it (NULL is accepted). */
typedef struct ntc_prepared *ntc_prepared_handle;
ntc_status ntc_prepare(ntc_prepared_handle *out, int32_t nmodes, const int64_t *dims, int64_t nnz,
                       const int32_t *coords, const float *values, int32_t rank, const ntc_params *p);
ntc_status ntc_create_prepared(ntc_handle *out, ntc_prepared_handle prepared, const ntc_params *p);
ntc_status ntc_prepared_bytes(ntc_prepared_handle prepared, size_t *bytes);
ntc_status ntc_prepared_release(ntc_prepared_handle prepared);

/* The row schedule ntc_prepare built for `mode` (host data, no device), for
 * checks of the invariants the row kernels rely on.  counts receives
 * {tiny rows, items, items that are whole rows of the group kernel (the
 * first ones), split rows, slot groups, partial slots, sampled entries}.
 * Each non-NULL array receives its entries as four 32-bit words:
 *   rowptr_out [dims[mode]+1] int64: the CSR row pointers;
 *   tiny_out   rows with 1 <= B_p <= tiny_max: {row, n_p, base lo, base hi};
 *   items_out  the first `group` items, when R <= 16 and nmodes <= 4:
 *              {row, n_p, base lo, base hi} (whole rows); every other item:
 *              {row, j0, j1, slot}, samples [j0, j1) of the row's minibatch,
 *              slot -1 for a whole row, else the partial slot it writes;
 *   split_out  {row, first slot, slot count, 0}: rows combined from slots;
 *   groups_out {first source slot, count, destination slot, 0}: R > 16 rows
 *              of many items, whose slots are first summed in groups.
 * Samples of a row are B_p = floor(c n_p) (Section II-B). */
ntc_status ntc_prepared_schedule(ntc_prepared_handle prepared, int32_t mode, int64_t counts[7], int64_t *rowptr_out,
                                 int32_t *tiny_out, int32_t *items_out, int32_t *split_out, int32_t *groups_out);

/* Enqueue `nsweeps` iterations of Alg. 2 (each: modes 0..N-1 in order, each
 * mode one S_NMC call of Alg. 1 with MAX_INNER inner steps), advancing k by
 * one per sweep.  Asynchronous: returns once the work is enqueued. */
ntc_status ntc_sweep(ntc_handle h, int32_t nsweeps);

/* Enqueue one S_NMC call (Alg. 1) for `mode` at the current k without
 * advancing k: the body of Alg. 2's inner loop for one i. */
ntc_status ntc_update_mode(ntc_handle h, int32_t mode);

/* Synchronise and evaluate, in FP64 on the device with a deterministic
 * two-stage reduction: out[0] = objective of eq. (Problem_TC) on the
 * training entries, out[1] = train RMSE, out[2] = test RMSE,
 * out[3] = test relative error ||x - x_hat|| / ||x|| (0 without a test set).
 * Returns NTC_ENONFINITE if any of them is not finite. */
ntc_status ntc_loss(ntc_handle h, double out[4]);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The loss of
 * ntc_loss (eq. Problem_TC, FP64, deterministic two-stage reduction) on
 * caller-held DEVICE arrays, with no handle:
 *   nmodes in [2, 8]; dims [nmodes] host; rank in [1, 64];
 *   train_coords [n_train][nmodes] int32 and train_values [n_train] FP32,
 *   test_coords [n_test][nmodes] and test_values [n_test]: device, 0-based
 *   coordinates that MUST lie in [0, dims[m]) (they are not checked: the
 *   call does not read device memory back);
 *   factors: host array of nmodes device pointers, FP32 [dims[m]][rank];
 *   out: DEVICE memory for 4 doubles, written on `stream` with
 *   {objective on the train set, train RMSE, test RMSE, test relative error}
 *   as ntc_loss defines them (non-finite values are written as they are).
 * Enqueued on `stream` (hipStream_t, NULL = the null stream); nothing is
 * allocated, set or copied by the host and nothing is synchronised.  Partial
 * sums live in a fixed device array of 1024 x 4 doubles (32 KiB per GPU,
 * held until the process ends); the call uses at most that, so calls that
 * overlap on one GPU (other streams, other threads) race on it and must be
 * ordered by the caller.  Errors: NTC_EINVAL (arguments), NTC_EUNSUPPORTED
 * (n_train or n_test >= 2^31, or dims[m] * rank >= 2^32), NTC_EDEVICE
 * (launch failure). */
ntc_status ntc_loss_coo_noalloc(int32_t nmodes, const int64_t *dims, int32_t rank, int64_t n_train,
                                const int32_t *train_coords, const float *train_values, int64_t n_test,
                                const int32_t *test_coords, const float *test_values, const float *const *factors,
                                double lambda, double *out, void *stream);

/* Synchronise and copy mode `mode`'s FP32 factor [I_m][R] to host_out. */
ntc_status ntc_get_factors(ntc_handle h, int32_t mode, float *host_out);

/* Copy a host FP32 factor [I_m][R] (entries >= 0, finite) into the handle
 * (also refreshes the BF16 shadow). */
ntc_status ntc_set_factors(ntc_handle h, int32_t mode, const float *host_in);

/* Copy mode `mode`'s factor into caller-owned DEVICE memory dev_out
 * (I_m * R floats), ordered on the handle's stream. */
ntc_status ntc_get_factors_device(ntc_handle h, int32_t mode, float *dev_out);

/* Sweep counter k (the Philox counter word of the sampler).  With the
 * factors it is the whole state: resuming from (factors, k) reproduces an
 * uninterrupted run bit-exactly. */
ntc_status ntc_get_sweep(ntc_handle h, int64_t *k);
ntc_status ntc_set_sweep(ntc_handle h, int64_t k);

/* Problem facts: the number of sampled entries one sweep consumes
 * (sum over modes and inner steps of sum_p B_p) and the number of rows that
 * take a step per sweep. */
ntc_status ntc_get_work(ntc_handle h, int64_t *updates_per_sweep, int64_t *row_steps_per_sweep);

/* Positions (within the row, in [0, n_p)) of the minibatch that row `row` of
 * `mode` draws at sweep k and inner step l, computed BY THE DEVICE sampler
 * (Section II-B: B_p = floor(c n_p) entries, uniformly, without
 * replacement).  pos_out holds >= n_p int32; *count receives B_p.
 * Synchronising. */
ntc_status ntc_debug_sample(ntc_handle h, int64_t k, int32_t mode, int32_t l, int64_t row,
                            int32_t *pos_out, int32_t *count);

/* The CSR of mode `mode` (the unfolding X_(i), M_(i) of Section II) exactly
 * as the handle holds it on the device, whichever build made it:
 * rowptr_out [dims[mode]+1] int64 (entries of row p are positions
 * [rowptr[p], rowptr[p+1]) in the stable order by coordinate `mode`, ties in
 * COO order); records_out [nnz][W] uint32 with W = 4 for nmodes <= 4 and 8
 * otherwise: the other modes' coordinates times R in increasing mode order,
 * the FP32 value bits, then zeros, except that for mode 0 with nmodes < W
 * word nmodes holds the entry's own coordinate times R.  Synchronising. */
ntc_status ntc_debug_csr(ntc_handle h, int32_t mode, int64_t *rowptr_out, uint32_t *records_out);

/* The same positions computed by the library's HOST copy of the sampler for
 * a row of length n (no device, no handle).  pos_out holds >= floor(c n)
 * int32; returns the count through *count. */
ntc_status ntc_host_sample(uint64_t seed, int64_t k, int32_t mode, int32_t l, int64_t row, int64_t n,
                           double c, int32_t *pos_out, int64_t *count);

/* The library's host CSR build for one mode, without a device: rowptr_out
 * [dims[mode]+1] int64 and perm_out [nnz] int64 (COO entry ids, stably
 * sorted by coordinate `mode`). */
ntc_status ntc_host_csr(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *coords,
                        int32_t mode, int64_t *rowptr_out, int64_t *perm_out);

/* Block until all work enqueued on h's stream has finished. */
ntc_status ntc_synchronize(ntc_handle h);

/* Enqueue `nsweeps` sweeps (as ntc_sweep) between two HIP events recorded on
 * h's stream, synchronise, and return the elapsed device time in *ms. */
ntc_status ntc_time_sweeps(ntc_handle h, int32_t nsweeps, double *ms);

/* One launch of a sweep as seen by ntc_profile_sweep. */
typedef struct ntc_launch_record {
    int32_t kernel;  /* 0: rows held by one work item (sample, gather, gradient,
                        Hessian, power method, step), one per 16-lane group for
                        R <= 16, one per wave otherwise;
                        1: finalize of rows split over several work items;
                        2: rows with at most 4 sampled entries, one per lane;
                        3: chunks of rows with many samples, one per 256-thread
                        block (R <= 16);
                        4: second-level sums of the partial slots of rows split
                        into many items (R > 16) */
    int32_t mode;    /* mode being updated */
    int32_t inner;   /* inner step l of Alg. 1 */
    int32_t blocks;  /* workgroups launched */
    int64_t samples; /* sampled entries the launch consumes */
    int64_t rows;    /* rows whose step (L_p, projection, extrapolation) it performs */
    double ms;       /* duration between HIP events around the launch */
} ntc_launch_record;

/* Run ONE sweep exactly as ntc_sweep does (k advances), recording HIP
 * events around every kernel launch; writes up to `cap` records in launch
 * order and the number of launches to *count.  Synchronising. */
ntc_status ntc_profile_sweep(ntc_handle h, ntc_launch_record *out, int32_t cap, int32_t *count);

/* Run `nsweeps` sweeps exactly as ntc_sweep does, recording HIP events
 * around every kernel launch on the stream that launch runs on.
 * concurrent = 1 keeps ntc_sweep's side-stream overlap, so a duration
 * includes sharing the GPU with the launches beside it (as a kernel trace
 * shows it); 0 runs every launch on h's stream, one after another
 * (ntc_profile_sweep is this with nsweeps = 1).  Writes up to `cap`
 * records, in launch order sweep after sweep, and the number of launches to
 * *count.  Synchronising.  Errors: NTC_EINVAL for a null handle or count,
 * out == NULL with cap > 0, or nsweeps < 0. */
ntc_status ntc_profile_sweeps(ntc_handle h, int32_t nsweeps, int32_t concurrent, ntc_launch_record *out,
                              int32_t cap, int32_t *count);

/* Upper bound of the device bytes ntc_create would allocate for this
 * problem (factors, BF16 shadows, CSR records and row pointers, the row
 * schedule, partial slots, held-out set, argument tables), computed on the
 * host from the sizes alone.  Used for admission by free memory. */
ntc_status ntc_estimate_bytes(int32_t nmodes, const int64_t *dims, int64_t nnz, int32_t rank,
                              const ntc_params *p, size_t *bytes);

/* Release all device and host memory of h (NULL is accepted). */
ntc_status ntc_release(ntc_handle h);

/* ------------------------------------------------------------------------
 * Batching and serving: many independent problems on one GPU.
 *
 * A pool owns one device memory arena and up to max_slots problems.  Each
 * admitted problem is a full ntc_create problem (own data, factors, seed
 * and sweep counter) whose device memory comes from the arena.  A pool
 * sweep runs Alg. 2 once for every running problem: per (mode, inner step)
 * one launch of each row kernel covers all running problems of the same
 * kernel family (padded rank, mode count, BF16 gathers), so a problem's
 * rows take exactly the code path and arithmetic they take alone; a
 * problem's factors after s pool sweeps are bit-identical to s ntc_sweep
 * calls on it alone.  The launches of one sweep are captured once as a HIP
 * graph and replayed until the set of running problems changes.
 *
 * Stop rule (evaluated on the device after every sweep, per problem with a
 * held-out set): stop after sweep s >= window when RMSE_test(s - window) -
 * RMSE_test(s) < tol * RMSE_test(s), or at max_sweeps (problems without a
 * held-out set stop only there).  A stopped problem keeps its slot and
 * memory (for queries) until ntc_pool_evict.
 * ---------------------------------------------------------------------- */
typedef struct ntc_pool *ntc_pool_handle;

typedef struct ntc_pool_params {
    size_t arena_bytes;       /* device memory for all problems (0 = 3/4 of free memory) */
    int32_t max_slots;        /* concurrent problems, 1..65536 (default 1024) */
    int32_t use_graph;        /* 1 = replay sweeps as a captured HIP graph (default), 0 = eager */
    int32_t window;           /* stop rule window (default 5) */
    int32_t max_sweeps;       /* stop after this many sweeps (default 500) */
    double tol;               /* stop rule relative tolerance (default 1e-4) */
    void *stream;             /* hipStream_t; NULL = the null stream */
} ntc_pool_params;

typedef enum { NTC_SLOT_FREE = 0, NTC_SLOT_RUNNING = 1, NTC_SLOT_STOPPED = 2 } ntc_slot_state;

void ntc_pool_params_default(ntc_pool_params *p);
ntc_status ntc_pool_create(ntc_pool_handle *out, const ntc_pool_params *p);

/* Admit a problem (arguments as ntc_create; p->stream, the allocator and
 * the overlap setting are replaced by the pool's).  Returns NTC_ENOMEM, with
 * nothing changed, when no slot is free or the arena cannot hold it now;
 * *slot receives the slot index on success. */
ntc_status ntc_pool_admit(ntc_pool_handle pool, int32_t nmodes, const int64_t *dims, int64_t nnz,
                          const int32_t *coords, const float *values, int32_t rank, const ntc_params *p,
                          int32_t *slot);

/* Admit a problem built by ntc_prepare (on any thread): only the device
 * work happens here.  Same results and errors as ntc_pool_admit. */
ntc_status ntc_pool_admit_prepared(ntc_pool_handle pool, ntc_prepared_handle prepared, int32_t *slot);

/* Admit a problem whose CSR is built on the device, as ntc_create_device_csr
 * builds it (bit-identical to ntc_pool_admit's problem): the COO upload, the
 * checks, the per-mode sort and the records run on the pool's stream, and
 * the temporaries come from the arena and return to it before the call
 * does.  NTC_ENOMEM, with nothing changed, when no slot is free or the arena
 * cannot hold the problem plus its temporaries now; other errors as
 * ntc_create_device_csr.  Synchronising. */
ntc_status ntc_pool_admit_device_csr(ntc_pool_handle pool, int32_t nmodes, const int64_t *dims, int64_t nnz,
                                     const int32_t *coords, const float *values, int32_t rank, const ntc_params *p,
                                     int32_t *slot);

/* Enqueue `nsweeps` pool sweeps over the running problems back to back and
 * wait for them.  The stop rule is applied on the device after every sweep;
 * a problem that stops mid-way is not touched by the remaining sweeps, so
 * its factors are those of the sweep at which it stopped whatever nsweeps
 * is.  Synchronising. */
ntc_status ntc_pool_step(ntc_pool_handle pool, int32_t nsweeps);

/* State of a slot: *state (ntc_slot_state), sweeps run, and the last
 * held-out RMSE of the stop rule (NaN before the first check). */
ntc_status ntc_pool_query(ntc_pool_handle pool, int32_t slot, int32_t *state, int64_t *sweeps, double *test_rmse);

/* Full loss (as ntc_loss) and factors of a running or stopped slot. */
ntc_status ntc_pool_loss(ntc_pool_handle pool, int32_t slot, double out[4]);
ntc_status ntc_pool_get_factors(ntc_pool_handle pool, int32_t slot, int32_t mode, float *host_out);

/* Slots that have stopped and are not yet evicted: up to cap indices into
 * slots, the total through *count. */
ntc_status ntc_pool_stopped(ntc_pool_handle pool, int32_t *slots, int32_t cap, int32_t *count);

/* Free a slot and return its memory to the arena. */
ntc_status ntc_pool_evict(ntc_pool_handle pool, int32_t slot);

/* Arena bytes in use and free, running and stopped slot counts, sweeps run. */
ntc_status ntc_pool_info(ntc_pool_handle pool, size_t *used, size_t *free_bytes, int32_t *running,
                         int32_t *stopped, int64_t *pool_sweeps);

ntc_status ntc_pool_release(ntc_pool_handle pool);

/* Thread-local message of the last failing call on this thread. */
const char *ntc_last_error(void);

/* Version string of the library build. */
const char *ntc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NTC_H */
