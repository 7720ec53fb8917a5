/*
 * hperm: exact permanents of sparse non-negative integer matrices on an AMD Instinct
 * MI355X (gfx950), after Wang, Liang, Bai and Huo, "A load balancing strategy for
 * parallel computation of sparse permanents" (arXiv 1112.6072).
 *
 * The path behind these calls:
 *   1. validation, bounds and arithmetic mode (host);
 *   2. expansion (2) of the paper, applied as in Algorithm H_per (Section 2.1) and the
 *      pre-expansion of Algorithm PH (Section 2.2), splits per(A) into sub-matrix jobs
 *      (host, C++);
 *   3. each job's 0-1 pattern gets a KKLLL estimate (Section 2.3) on the GPU (FP32; the
 *      estimate only orders jobs and never enters a result);
 *   4. jobs are sorted by non-increasing estimate (the improved Step 3 of Algorithm PH,
 *      Section 3.3) and cut into work items of a device queue;
 *   5. every job is evaluated exactly by R-NW (Ryser's formula in Nijenhuis-Wilf form,
 *      Introduction) in Gray-code order by HIP kernels, in modular or wrap-around integer
 *      arithmetic chosen so that the result is exact;
 *   6. per-job values are normalised and summed (Step 4 of Algorithm PH) into per(A).
 *
 * Conventions for every call: pointers are host pointers unless a parameter says
 * "device"; inputs are only read during the call and may be freed when it returns;
 * every call returns an hperm_status and writes outputs only on HPERM_OK (poll/wait
 * also on HPERM_NOT_READY, leaving the output untouched); no exception crosses the ABI.
 * A context is used by one thread at a time, except hperm_submit/poll/wait/cancel,
 * which are internally synchronised.
 */
#ifndef HPERM_H
#define HPERM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hperm_status {
    HPERM_OK = 0,
    HPERM_NOT_READY = 1,     /* poll: the request is still running */
    HPERM_E_INVALID = -1,    /* bad argument: sizes, ordering, null pointers, option ranges */
    HPERM_E_RANGE = -2,      /* the exact result or an expanded entry does not fit the
                                supported integer range (see hperm_permanent_csr) */
    HPERM_E_DEVICE = -3,     /* a HIP call failed; hperm_last_error names it */
    HPERM_E_NOMEM = -4,      /* host or device memory (or the caller's arena) is too small */
    HPERM_E_BUSY = -5,       /* serving: no free request slot */
    HPERM_E_CANCELLED = -6,  /* serving: the request was cancelled */
    HPERM_E_TIMEOUT = -7,    /* serving: wait timed out (the request keeps running) */
    HPERM_E_INTERNAL = -8,   /* an integrity check failed (a job value not divisible by
                                2^(m-1), a residue check mismatch); never returned silently */
    HPERM_E_TOOBIG = -9      /* serving: the request's estimated work exceeds the serving
                                limit (opts.serve_limit_ms) */
} hperm_status;

/* Job order of the device queue (Step 3 of Algorithm PH and its improved form). */
typedef enum hperm_order {
    HPERM_ORDER_ESTIMATE = 0,    /* non-increasing KKLLL estimate (the paper's strategy) */
    HPERM_ORDER_NATURAL = 1,     /* expansion (depth-first) order (the original PH Step 3) */
    HPERM_ORDER_RANDOM = 2,      /* seeded shuffle */
    HPERM_ORDER_EXACT_COST = 3   /* non-increasing subset-term count 2^(m-1), then estimate */
} hperm_order;

/* Exact arithmetic of the R-NW kernels. AUTO picks per job from a proven bound. */
typedef enum hperm_arith {
    HPERM_ARITH_AUTO = 0,
    HPERM_ARITH_W64 = 1,    /* integers mod 2^64 (exact when per * 2^(m-1) < 2^63) */
    HPERM_ARITH_W128 = 2,   /* integers mod 2^128 (exact when per * 2^(m-1) < 2^127) */
    HPERM_ARITH_RES = 3     /* residues mod three primes near 2^61, host CRT (per < ~2^182) */
} hperm_arith;

typedef struct hperm_opts {
    int32_t m_cut;        /* expand while the order exceeds m_cut (1..40; default 20) */
    int32_t m_cap;        /* largest job order (m_cut..40; default 36) */
    int32_t s_leaf;       /* a node whose sparsest line has >= s_leaf nonzeros and whose order
                             is <= m_cap becomes a job (Algorithm H_per uses 5; default 5) */
    int32_t arith;        /* hperm_arith (default AUTO) */
    int32_t order;        /* hperm_order (default ESTIMATE) */
    int32_t trials;       /* KKLLL trials per job (1..4096; default 32) */
    uint64_t seed;        /* seed of the KKLLL draws and of ORDER_RANDOM (default 1) */
    int32_t chunk_log2;   /* Gray indices per lane = 2^chunk_log2 (0..12); 0 = default table */
    int32_t persistent;   /* 1: one persistent launch over the queue (default);
                             0: one launch per job (the plain comparator) */
    int32_t host_threads; /* expansion threads (0 = hardware threads, at most 64) */
    int32_t max_table_mib;/* host job-table limit per expansion call in MiB (0 = 4096): an
                             expansion that would outgrow it stops with HPERM_E_NOMEM instead
                             of exhausting host memory (raise m_cut to get fewer jobs) */
    int32_t time_jobs;    /* 1: persistent runs of hperm_run_jobs record each job's work time
                             (hperm_jobs_cycles; the scheduling study of the paper's load
                             balancing section); 0: off (default). Ignored while serving. */
    int32_t split_order;  /* t in [7, 23] (default 12): persistent runs continue Algorithm H_per
                             (Section 2.1) on the device for every mod-2^64 job of order t+1..24,
                             splitting it by expansion (2) down to order t, and evaluate the
                             leaves by R-NW inside the same kernel (one wave per job); other jobs
                             take the R-NW queue. Results are unchanged (the expansion is an
                             identity). 0: off, every job by R-NW. Ignored when s_leaf > 5 and by
                             one-launch-per-job runs. */
    int32_t device_expand;/* T in [0, 24] (default 22): when T exceeds the split order in
                             effect, the blocking calls (hperm_permanent_csr / _dense / _batch_csr)
                             expand every problem of order n > T whose proven bound is below
                             2^102 on the device instead of the host: expansion (2) with Algorithm
                             H_per's line rule (Section 2.1) level by level down to sub-matrices
                             of order T, which the device continuation of H_per finishes; the
                             whole tree stays on the GPU in bounded memory; problems of one
                             order share one expansion (their results then report the group's
                             job and subset-term counts and times). Other problems take the
                             host path; the serving loop sends requests above order T to its
                             device lane (hperm_serve_start). Results are the same integers.
                             0 (or T <= split order): off. */
    int32_t device_expand_mib; /* device memory for the expansion's level buffers in MiB
                             (0 = 8192); more memory means fewer, larger launches */
    int32_t use_graphs;   /* 1: the device part of a persistent run on a job table (clears,
                             every launch group, the recombination and the result download) is
                             captured once as a HIP graph and replayed by later runs with the
                             same table, buffers, launch groups and tuning (the queue upload stays
                             outside, so the job order may change between replays); per-launch
                             times are then not available (the run's whole span is reported in
                             its first launch record). Not for runs with per-job results or job
                             timing. 0: every launch issued (default). */
    int32_t serve_limit_ms;/* serving admission by work: a request whose estimated GPU time
                             (hperm_tree_estimate with 64 descents, at the device path's leaf
                             rate of about 2e8 leaves/s) exceeds this many milliseconds
                             completes with HPERM_E_TOOBIG without device work. 0: no limit
                             (default). */
} hperm_opts;

/* Result of one permanent. The value is non-negative: magnitude limbs, little-endian. */
typedef struct hperm_result {
    uint64_t limb[8];       /* per(A) = sum_k limb[k] * 2^(64k) */
    int32_t nlimb;          /* limbs in use (0 means per(A) = 0) */
    int32_t n_jobs;         /* sub-matrix jobs evaluated on the GPU */
    int32_t max_m;          /* largest job order */
    int32_t arith_mask;     /* bit (1 << hperm_arith) set for every mode used */
    uint64_t subset_terms;  /* sum over jobs of 2^(m-1): the R-NW Gray-code terms */
    double t_expand_s;      /* host expansion + job packing */
    double t_estimate_s;    /* KKLLL kernel */
    double t_rnw_s;         /* R-NW kernels (HIP events on the library stream) */
    double t_total_s;       /* the whole call */
} hperm_result;

typedef struct hperm_ctx hperm_ctx;
typedef struct hperm_jobs hperm_jobs;

/* Library version. */
hperm_status hperm_version(int32_t *major, int32_t *minor);

/* Fill *opts with the defaults listed above. */
hperm_status hperm_default_opts(hperm_opts *opts);

/* Create a context on the current HIP device. opts may be NULL (defaults). stream is a
 * hipStream_t to run on (e.g. torch.cuda.current_stream().cuda_stream), or NULL for a
 * library-owned stream. The context owns its device buffers (grown on demand) unless an
 * arena is set. Errors: HPERM_E_INVALID (option out of range), HPERM_E_DEVICE, NOMEM. */
hperm_status hperm_ctx_create(const hperm_opts *opts, void *stream, hperm_ctx **out);

/* A context without a device: only the host stages (hperm_expand_batch_csr,
 * hperm_jobs_from_dense, hperm_jobs_info/describe) work; GPU calls return HPERM_E_DEVICE. */
hperm_status hperm_ctx_create_host(const hperm_opts *opts, hperm_ctx **out);
void hperm_ctx_destroy(hperm_ctx *ctx);

/* Replace the context's options (same ranges as hperm_ctx_create). */
hperm_status hperm_ctx_set_opts(hperm_ctx *ctx, const hperm_opts *opts);

/* Copy the context's current options into *opts. */
hperm_status hperm_ctx_get_opts(const hperm_ctx *ctx, hperm_opts *opts);

/* Let the library sub-allocate every device buffer from [dev_ptr, dev_ptr + bytes) (device
 * memory owned by the caller, e.g. a torch tensor), valid until the context is destroyed
 * or the arena is replaced. dev_ptr = NULL returns to library-owned memory. A call whose
 * buffers do not fit returns HPERM_E_NOMEM and hperm_ctx_arena_required then gives the
 * bytes it needed. */
hperm_status hperm_ctx_set_arena(hperm_ctx *ctx, void *dev_ptr, size_t bytes);
size_t hperm_ctx_arena_required(const hperm_ctx *ctx);

/* per(A) of one n x n matrix given in CSR form: row_ptr[n+1] (row_ptr[0] = 0, non-decreasing),
 * col_idx[nnz] strictly increasing within a row, values val[nnz] (uint32, zeros allowed).
 * The problem statement of Algorithm H_per (Section 2.1) with non-negative integer entries.
 * n = 0 gives 1; a zero row or column gives 0 without GPU work.
 * Paths: the device expansion and continuation in exact rings (order above opts.device_expand,
 * proven bound below 2^102), else the host expansion with R-NW (bound below 2^180). When
 * either refuses a problem for its range (an expanded entry reaching 2^22, a row sum 2^24, or
 * the bound) and the problem's order exceeds opts.device_expand (in effect), it is evaluated
 * exactly by residues instead: the device path modulo K + 1 primes p with n (p - 1) < 2^24
 * (hperm_permanent_mod_batch_csr), K of them covering the bound min(prod row sums, prod column
 * sums), rebuilt by the Chinese remainder theorem and checked against the last (arith_mask
 * then names the residue ring).
 * Errors: HPERM_E_INVALID (n < 0 or n > 128, malformed CSR); HPERM_E_RANGE (an expanded
 * entry reaches 2^22 or a row sum 2^24, or the proven bound on per(A) exceeds 2^180, for a
 * problem the residue evaluation does not take; or a bound beyond 2^500);
 * HPERM_E_DEVICE; HPERM_E_NOMEM (device memory, or the job table outgrows max_table_mib);
 * HPERM_E_INTERNAL. */
hperm_status hperm_permanent_csr(hperm_ctx *ctx, int32_t n, const int32_t *row_ptr,
                                 const int32_t *col_idx, const uint32_t *val, hperm_result *out);

/* per(A) of a dense row-major n x n matrix a[n*n]; same rules as hperm_permanent_csr. */
hperm_status hperm_permanent_dense(hperm_ctx *ctx, int32_t n, const uint32_t *a,
                                   hperm_result *out);

/* For callers that cannot allocate memory during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): per(A) of one dense row-major
 * n x n matrix a[n*n] (host memory, borrowed for the call), 0 <= n <= 40, evaluated as a
 * single R-NW job (no expansion), with the same value as hperm_permanent_dense. The call makes
 * no hipMalloc/hipFree and no other allocation of device or pinned memory: every device buffer
 * of the run (job descriptor and data, queue, queue heads, job and problem accumulators) is a
 * slice of one fixed library array of 16 KiB per GPU (held until the process ends), and the
 * host side packs the job on the stack. Heads and accumulators are cleared at the start of
 * every call (the array keeps the previous call's contents). All calls on one GPU share that
 * array: calls that overlap on the same GPU (from different contexts or threads) race and
 * must be serialised by the caller; calls on one context are serialised by the library.
 * Runs on the context's stream and waits for it. Errors: HPERM_E_INVALID (n outside 0..40,
 * a NULL pointer, an entry >= 2^22, or the context is serving), HPERM_E_RANGE (a row sum
 * reaches 2^24, the bound exceeds 2^180, or a forced ring is too narrow), HPERM_E_DEVICE
 * (a HIP call failed, or the array's address could not be obtained), HPERM_E_INTERNAL. */
hperm_status hperm_permanent_dense_noalloc(hperm_ctx *ctx, int32_t n, const uint32_t *a,
                                           hperm_result *out);

/* A batch of problems in one device pass: all their jobs share one queue and one
 * persistent launch (Algorithm PH over several matrices). Problem k has order n[k] and
 * CSR arrays at row_ptr + rp_off[k], col_idx + nz_off[k], val + nz_off[k]. out[count]. */
hperm_status hperm_permanent_batch_csr(hperm_ctx *ctx, int32_t count, const int32_t *n,
                                       const int64_t *rp_off, const int64_t *nz_off,
                                       const int32_t *row_ptr, const int32_t *col_idx,
                                       const uint32_t *val, hperm_result *out);

/* per(A_k) modulo a prime for a batch of problems (layout as hperm_permanent_batch_csr), by the
 * device path in modular arithmetic: the expansion (2) of Algorithm H_per on the device with
 * every merged entry reduced modulo the prime, the device continuation of H_per, each leaf's
 * Nijenhuis-Wilf sum taken modulo the prime and normalised by the inverse of 2^(p-1), sums of
 * residues. Entries are reduced on entry, so no bound applies: the residues of values of any
 * size, for exact reconstruction by the Chinese remainder theorem over several primes (the
 * permanental polynomial beyond 2^180, per(A) beyond the exact paths' range). prime: an odd
 * prime below 2^18 with n[k] (prime - 1) < 2^24 (so every row sum of a node stays below 2^24).
 * Every n[k] must exceed the device expansion's order (opts.device_expand, 22 when off) and be
 * at most 128; opts.split_order (12 when off) is the continuation's target. residues[count]
 * (caller-owned) receives per(A_k) mod prime.
 * Errors: HPERM_E_INVALID (bad arrays, orders, a modulus that is not an odd prime below 2^18,
 * or the context is serving), HPERM_E_NOMEM, HPERM_E_DEVICE, HPERM_E_INTERNAL. */
hperm_status hperm_permanent_mod_batch_csr(hperm_ctx *ctx, int32_t count, const int32_t *n,
                                           const int64_t *rp_off, const int64_t *nz_off,
                                           const int32_t *row_ptr, const int32_t *col_idx,
                                           const uint32_t *val, uint32_t prime, uint64_t *residues);

/* One signed integer coefficient: |c| = sum_k limb[k] * 2^(64k), negative when c < 0. */
typedef struct hperm_coeff {
    uint64_t limb[8];
    int32_t nlimb;          /* limbs in use (0 means c = 0) */
    int32_t negative;
} hperm_coeff;

/* Permanental polynomial (the paper's application to chemical graphs): coeffs[k] = c_k with
 * per(xI - A) = sum_{k=0..n} c_k x^k, exactly, for a non-negative integer matrix A (CSR as for
 * hperm_permanent_csr). Computed from per(xI + A) at x = 0..n, n + 1 problems of one batched
 * pass (xI + A has non-negative entries; per(xI + A) = sum_k a_k x^k with a_k the sum of the
 * permanents of the principal sub-matrices of order n - k, and c_k = (-1)^(n-k) a_k), then
 * exact integer interpolation on the host. When the bound of per(nI + A) stays below 2^180 the
 * evaluations are exact integers, with m_cut raised to n for n <= 40 (each xI + A is one R-NW
 * job: no expansion, whose merges would multiply the large diagonal entries). Beyond that bound,
 * for device-expansion orders 23..64, the n + 1 evaluations are taken modulo each of K + 1
 * primes below 2^18 (hperm_permanent_mod_batch_csr) and interpolated modulo that prime; each
 * a_k is rebuilt by the Chinese remainder theorem over K primes whose product exceeds a bound
 * on the coefficients (a_k <= e_{n-k}(g), the elementary symmetric function of g_i = the row
 * sums, or Bregman's (r_i!)^(1/r_i) for a 0-1 matrix) and checked against the last prime
 * (C60: 6 primes, 366 evaluations of order 60, each a tree of about 2e9 leaves).
 * The context's options are restored afterwards. coeffs[n + 1] is caller-owned.
 * Must not be called while serving or concurrently with other calls on the context.
 * Errors: as for
 * hperm_permanent_batch_csr; HPERM_E_RANGE when a bound or an intermediate exceeds the
 * supported range; HPERM_E_INTERNAL when the interpolation fails its exactness checks. */
hperm_status hperm_permanental_polynomial(hperm_ctx *ctx, int32_t n, const int32_t *row_ptr,
                                          const int32_t *col_idx, const uint32_t *val,
                                          hperm_coeff *coeffs);

/* The host step of hperm_permanental_polynomial on its own: the coefficients of the integer
 * polynomial p of degree <= n with p(x) = values[x] for x = 0..n (values[(n + 1) * 8]: each a
 * non-negative little-endian 512-bit integer), by forward differences and the Newton
 * (falling-factorial) form, exactly; with alternate != 0 coefficient k is negated when n - k is
 * odd (p(x) = per(xI + A) then gives per(xI - A)). coeffs[n + 1]. Errors: HPERM_E_INVALID
 * (n out of 0..128, NULL arrays, or values that no integer-coefficient polynomial of degree n
 * takes), HPERM_E_RANGE (an intermediate beyond 500 bits). */
hperm_status hperm_polynomial_interpolate(int32_t n, const uint64_t *values, int32_t alternate,
                                          hperm_coeff *coeffs);

/* The residue form of that host step (the permanental polynomial beyond 2^180): a polynomial p
 * of degree <= n with coefficients a_k in [0, P), P the product of primes[0..nprimes-2], from
 * residues[j * (n + 1) + x] = p(x) mod primes[j], x = 0..n: p interpolated modulo each prime
 * (forward differences, Newton coefficients with the inverses of k!), each a_k rebuilt by the
 * Chinese remainder theorem over the first nprimes - 1 primes and checked against the last.
 * With alternate != 0, coefficient k is negated when n - k is odd. primes: distinct primes
 * above n, below 2^32, with P below 2^511; coeffs[n + 1]. Errors: HPERM_E_INVALID (n out of
 * 0..128, nprimes < 2, NULL arrays, a modulus that is not such a prime, or residues the check
 * prime contradicts: a coefficient outside [0, P) or a wrong residue), HPERM_E_RANGE (P
 * beyond 2^511). */
hperm_status hperm_polynomial_from_residues(int32_t n, int32_t nprimes, const uint32_t *primes,
                                            const uint64_t *residues, int32_t alternate, hperm_coeff *coeffs);

/* ---- stages (tests and benchmarks) ------------------------------------------------ */

/* Expand problems into jobs (steps 1-2 above) without running them. Same inputs as
 * hperm_permanent_batch_csr. The job table is owned by the library until hperm_jobs_free. */
hperm_status hperm_expand_batch_csr(hperm_ctx *ctx, int32_t count, const int32_t *n,
                                    const int64_t *rp_off, const int64_t *nz_off,
                                    const int32_t *row_ptr, const int32_t *col_idx,
                                    const uint32_t *val, hperm_jobs **out);

/* Jobs given directly: count dense row-major matrices, matrix k of order m[k] (1..40) at
 * a + off[k]; each job is evaluated by R-NW as it is (no expansion), as problem k. A matrix
 * with an empty line (per = 0) gives no job: its problem's total is 0 and the job indices skip
 * it (hperm_jobs_describe maps every job to its problem). */
hperm_status hperm_jobs_from_dense(hperm_ctx *ctx, int32_t count, const int32_t *m,
                                   const int64_t *off, const uint32_t *a, hperm_jobs **out);

/* Number of jobs; per job: order m, problem index, arithmetic mode, natural index. */
hperm_status hperm_jobs_info(const hperm_jobs *jobs, int32_t *n_jobs, int32_t *n_problems);
hperm_status hperm_jobs_describe(const hperm_jobs *jobs, int32_t *m, int32_t *problem,
                                 int32_t *arith, uint64_t *terms);

/* The sub-matrix of job `job` as the kernels hold it, row-major m x m into a[m*m] (m from
 * hperm_jobs_describe): rows in the job's order, Gray columns 0..m-2, then the fixed column.
 * It is a row and column permutation of the expansion's sub-matrix or of its transpose (the
 * same permanent). Host only; the caller owns a. HPERM_E_INVALID for a null pointer or a job
 * index out of range. */
hperm_status hperm_jobs_matrix(const hperm_jobs *jobs, int32_t job, uint32_t *a);

/* KKLLL estimates of every job's pattern (step 3): trials per job and seed as given.
 * keys[n_jobs] (may be NULL) receives log of the mean of the trials (natural log;
 * -INFINITY when every trial was singular). The keys are kept for ORDER_ESTIMATE. */
hperm_status hperm_estimate(hperm_ctx *ctx, hperm_jobs *jobs, int32_t trials, uint64_t seed,
                            float *keys);

/* Evaluate all jobs (steps 4-6) in the given order, persistent (1) or one launch per job
 * (0). per_job[n_jobs] (may be NULL) receives each job's exact permanent; totals[n_problems]
 * receives per(A) of every problem. ORDER_ESTIMATE requires hperm_estimate first. */
hperm_status hperm_run_jobs(hperm_ctx *ctx, hperm_jobs *jobs, int32_t order, int32_t persistent,
                            hperm_result *per_job, hperm_result *totals);

void hperm_jobs_free(hperm_jobs *jobs);

/* The device expansion as a stage (opts.device_expand = T and opts.split_order = t set; n > T):
 * per(A) of one CSR matrix (layout as hperm_permanent_csr) with the expansion tree built on the
 * GPU (expansion (2) with Algorithm H_per's line rule, Section 2.1, down to order T, then the
 * device continuation of H_per), keeping its first max_jobs jobs of order T in tree order (the
 * depth-first order of the expansion): mats[max_jobs * T * T] receives them as dense row-major
 * T x T matrices and values[max_jobs] their exact permanents; *n_sampled how many were kept.
 * stop_early != 0 ends the run once they are kept: *total then holds no value and has
 * max_m = 0; otherwise *total is per(A) (max_m = T) with n_jobs the jobs of order T and
 * subset_terms the leaves' subset-terms. Needs library-owned device memory (no arena).
 * Errors: HPERM_E_INVALID (options, malformed input, n <= T, an arena is set),
 * HPERM_E_RANGE (an entry or row sum beyond the kernels' limits, a bound beyond 2^102),
 * HPERM_E_DEVICE, HPERM_E_NOMEM, HPERM_E_INTERNAL. */
hperm_status hperm_device_expand_sample(hperm_ctx *ctx, int32_t n, const int32_t *row_ptr,
                                        const int32_t *col_idx, const uint32_t *val, int32_t max_jobs,
                                        int32_t stop_early, uint32_t *mats, hperm_result *values,
                                        int32_t *n_sampled, hperm_result *total);

/* Work estimate before a run (host only; Knuth's estimator of a search tree's size): `samples`
 * random descents from the root of per(A)'s expansion tree, each taking one child of a node
 * with equal probability, under the rule of the default path for the options given (opts may
 * be NULL for the defaults): every node above the device expansion's order T is split (the
 * host cut-off m_cut when the device expansion is off), then Algorithm H_per's rule (Section
 * 2.1: split while the sparsest line has 1..4 nonzeros) down to the target order t of the device
 * continuation (m_cut when it is off). Along a descent the product of the child counts above a
 * node estimates the number of nodes at its order without bias. nodes[n + 1] and leaves[n + 1]
 * receive the estimated nodes and leaves of each order 0..n (mean over the descents). The
 * tree's shape depends on the nonzero pattern only, so the descents walk the 0-1 pattern: any
 * entry values are accepted. seed drives SplitMix64. Errors: HPERM_E_INVALID (options,
 * malformed matrix, NULL arrays, samples < 1). */
hperm_status hperm_tree_estimate(const hperm_opts *opts, int32_t n, const int32_t *row_ptr,
                                 const int32_t *col_idx, const uint32_t *val, int32_t samples,
                                 uint64_t seed, double *nodes, double *leaves);

/* ---- autotuning of the persistent R-NW launches -------------------------------------- */

/* One tuned launch group: its ring (0: mod 2^64, 1: mod 2^128, 2: residues), order bucket
 * (0..4: orders <= 16, 20, 24, 32, 40) and walk variant (as in hperm_launch_stat); the lane
 * chunk as an offset from each job's own (2^chunk Gray indices per lane, so 2^(m-7-chunk) work
 * items of 64 lanes, i.e. waves, per job of order m) and the persistent grid as a percentage of
 * the resident one; the sample's R-NW milliseconds with the defaults and with the choice (both
 * 0 when the entry came from a cache). */
typedef struct hperm_tune_entry {
    int32_t ring, bucket, variant;
    int32_t chunk_delta;
    int32_t grid_pct;
    int32_t from_cache;
    double ms_default, ms_tuned;
} hperm_tune_entry;

/* Autotune the persistent R-NW launches (the work decomposition of Step 3, Section 3.3) for the
 * launch groups of a job table: per group, the kernel runs on a sample of the group's jobs
 * (natural order, about 2^33 subset-terms) with lane-chunk offsets -3..+1 and grids of 100, 75
 * and 50 % of the resident one, twice each; the fastest pair (kept only when 2 % faster than
 * the defaults) enters the context's tuning table, which every later persistent run on the
 * context applies (results never change: the chunk only regroups the same Gray indices). With
 * cache_path (may be NULL), entries for this GPU architecture are first read from that JSON
 * file (groups found there are not re-timed unless force != 0) and the table is written back
 * after tuning. jobs may be NULL: only the cache is read. out[max] receives the table (may be
 * NULL when max = 0) and *n its size. Errors: HPERM_E_INVALID (arguments, serving, an
 * unwritable cache), HPERM_E_DEVICE, HPERM_E_NOMEM. */
hperm_status hperm_autotune(hperm_ctx *ctx, hperm_jobs *jobs, const char *cache_path, int32_t force,
                            hperm_tune_entry *out, int32_t max, int32_t *n);

/* Forget the context's tuning (later runs use the expansion's chunks and resident grids). */
hperm_status hperm_tune_clear(hperm_ctx *ctx);

/* ---- scheduling study (the paper's load-balancing analysis) --------------------------- */

/* Work time of every job (natural index) in the last persistent hperm_run_jobs on these jobs
 * with opts.time_jobs = 1: the sum over the job's work items of the shader-clock cycles its
 * wave spent from taking the item to finishing it (waves sharing a SIMD stretch each other's
 * items, so the figures rank jobs and compare orders; they are not isolated times).
 * cycles[n_jobs]. HPERM_E_INVALID when no timed run has been made on the jobs. */
hperm_status hperm_jobs_cycles(const hperm_jobs *jobs, uint64_t *cycles);

/* List scheduling as in Step 3 of Algorithm PH: jobs are taken in the given order and each is
 * assigned to the machine with the smallest load so far (ties: the lowest machine index).
 * times[n] are the job times (any unit), order[n] a permutation of 0..n-1, machines >= 1.
 * *makespan receives the largest machine load; loads[machines] (may be NULL) every load.
 * Errors: HPERM_E_INVALID (n < 0, machines < 1, order not a permutation, NULL arrays). */
hperm_status hperm_list_schedule(int32_t n, const uint64_t *times, const int32_t *order,
                                 int32_t machines, uint64_t *makespan, uint64_t *loads);

/* Kendall's rank correlation of x[n] and y[n] with the tie correction of the paper's
 * equations for tied ranks: tau = S / sqrt((n(n-1)/2 - T)(n(n-1)/2 - U)), S the number of
 * concordant minus discordant pairs, T and U the pairs tied in x and in y (tau_b); O(n log n).
 * *z receives tau / sqrt(2(2n+5) / (9n(n-1))), the normal score under independence, and *p
 * the two-sided normal p-value. NaN inputs are rejected. Errors: HPERM_E_INVALID (n < 2, NULL
 * arrays, NaN, or every pair tied in x or in y). */
hperm_status hperm_kendall_tau(int32_t n, const double *x, const double *y, double *tau,
                               double *z, double *p);

/* The regression of Section 3.1 (eqs. 4-6): the time T of a sub-matrix against five of its
 * invariants, T = a0 + a1 P + a2 |D| + a3 S + a4 V1 + a5 V2.
 *
 * hperm_matrix_invariants: of the dense m x m matrix a (row-major, caller's host memory,
 * 1 <= m <= 128) out[0] = |det(a)| (partial-pivot elimination in long double: a float value),
 * out[1] = S, the number of nonzeros, out[2] = V1 and out[3] = V2, the population variances of
 * its row sums and of its column sums.
 *
 * hperm_ols: least squares of y[n] on the k columns of X (row-major n x k) with an intercept;
 * coef[k + 1] receives a0, a1..ak and *r2 the coefficient of determination as the paper
 * defines it, sum (yhat - ybar)^2 / sum (y - ybar)^2. HPERM_E_INVALID for NULL arrays,
 * non-finite values, n < k + 2, a constant or linearly dependent column.
 *
 * hperm_stepwise: Efroymson's stepwise selection on the same data: from the intercept alone,
 * the column with the largest partial F enters while that F exceeds f_enter; after each entry
 * the model column with the smallest partial F leaves while that F is below f_remove
 * (0 <= f_remove <= f_enter; 4.0 and 3.9 are the usual values). chosen[k] receives the chosen
 * columns in entry order, *n_chosen their number. */
hperm_status hperm_matrix_invariants(int32_t m, const uint32_t *a, double *out);
hperm_status hperm_ols(int32_t n, int32_t k, const double *X, const double *y, double *coef, double *r2);
hperm_status hperm_stepwise(int32_t n, int32_t k, const double *X, const double *y, double f_enter,
                            double f_remove, int32_t *chosen, int32_t *n_chosen);

/* ---- serving ------------------------------------------------------------------------ */

/* Start the serving loop of a context (continuous batching of requests):
 * - a request is admitted while fewer than max_requests (1..65536) are live, else
 *   hperm_submit returns HPERM_E_BUSY;
 * - worker threads expand admitted requests (steps 1-2) with the context's options;
 * - a dispatcher packs every expanded request, oldest first, into one batch while the
 *   batch's device buffers fit a free slice of the serving arena (arena_bytes of device
 *   memory allocated here; 0 means 2 GiB): admission by device memory. A request whose own
 *   buffers exceed the arena completes with HPERM_E_NOMEM;
 * - a batch is one device queue over all of its requests' jobs (steps 3-6), run on one of
 *   two streams at the default priority, so that the next batch starts while the previous
 *   one runs; at most two batches are in flight;
 * - a request the device expansion takes (opts.device_expand in effect, order above it, bound
 *   below 2^102) runs instead on a third stream by the device expansion, together with the
 *   other waiting requests of its order, overlapping the batches; so does, by residues (as in
 *   hperm_permanent_csr), a request above that order that the host expansion refuses for
 *   range, its work estimate counted once per prime, twice over;
 * - with opts.serve_limit_ms, a request whose estimated work exceeds the limit completes with
 *   HPERM_E_TOOBIG (admission by work);
 * - a request completes when its batch does; its result is bit-identical to the blocking
 *   call's.
 * While serving, the context refuses blocking GPU calls, hperm_ctx_set_opts and
 * hperm_ctx_set_arena (HPERM_E_INVALID). hperm_serve_stop (and hperm_ctx_destroy) finish
 * the batches in flight, drop requests not yet dispatched and free the arena; no other
 * call on the context may be in progress then. Errors: HPERM_E_INVALID (already serving,
 * max_requests out of range), HPERM_E_NOMEM (arena allocation), HPERM_E_DEVICE. */
hperm_status hperm_serve_start(hperm_ctx *ctx, int32_t max_requests, size_t arena_bytes);
hperm_status hperm_serve_stop(hperm_ctx *ctx);

/* Submit per(A) of a CSR matrix (n <= 128; same layout and limits as hperm_permanent_csr;
 * copied, so the arrays may be freed on return). *ticket identifies it. HPERM_E_BUSY when
 * every request slot is in use; HPERM_E_INVALID for a malformed matrix or when not serving. */
hperm_status hperm_submit(hperm_ctx *ctx, int32_t n, const int32_t *row_ptr,
                          const int32_t *col_idx, const uint32_t *val, uint64_t *ticket);

/* HPERM_NOT_READY while running; once done, returns the request's status (HPERM_OK and *out
 * filled, or its error, HPERM_E_CANCELLED for a cancelled one) exactly once and frees the
 * ticket; an unknown or already taken ticket gives HPERM_E_INVALID. The result's timing
 * fields hold the queue wait (t_expand_s: submit to dispatch in a batch), the batch's R-NW
 * time (t_rnw_s) and the latency (t_total_s: submit to completion). hperm_wait blocks until
 * done (timeout_s < 0: no limit) and returns HPERM_E_TIMEOUT when the limit passes first.
 * hperm_cancel drops a request that is not yet dispatched; one already running completes
 * but reports HPERM_E_CANCELLED. Submit/poll/wait/cancel may be called from any thread. */
hperm_status hperm_poll(hperm_ctx *ctx, uint64_t ticket, hperm_result *out);
hperm_status hperm_wait(hperm_ctx *ctx, uint64_t ticket, double timeout_s, hperm_result *out);
hperm_status hperm_cancel(hperm_ctx *ctx, uint64_t ticket);

/* ---- diagnostics -------------------------------------------------------------------- */

/* One R-NW kernel launch of the last hperm_run_jobs / hperm_permanent_* call. */
typedef struct hperm_launch_stat {
    int32_t ring;           /* 0: mod 2^64, 1: mod 2^128, 2: residues */
    int32_t bucket;         /* kernel instantiation: job orders <= 16, 20, 24, 32, 40 */
    int32_t n_jobs;         /* jobs in the launch (1 in one-launch-per-job mode) */
    int32_t persistent;
    int32_t variant;        /* walk variant: 0, or 1 / 2 for the paired walk of jobs whose
                               Gray column 0 reaches only the first 2 / 3 rows; 3 for the
                               device continuation of H_per (split_order); 4 for one group of
                               problems of one order run by the device expansion
                               (device_expand): then n_jobs = its jobs of order T, items = the
                               nodes it wrote, row_updates = its device H_per launches, ms =
                               the whole group on the device and alg_slots = the milliseconds
                               of its device H_per launches; 5 for such a group evaluated by
                               residues (ring 2; the figures of its one pass, which takes
                               every problem once per prime, and
                               row_updates = the number of primes); 6 / 7 for the four-step
                               walks (mod 2^64, lane chunks of 4 indices or more) of jobs whose
                               Gray column 0 reaches exactly the first a = 2 / 3 rows and Gray
                               column 1 (with rows disjoint from column 0's) only rows of
                               a..a+2, rows 0..a+2 having row sums below 2^7 */
    int32_t reserved;       /* variant 3: the launch's resident waves; variant 4 or 5: the
                               problems of the group */
    uint64_t items;         /* work items (64 lanes x 2^chunk Gray indices each) */
    uint64_t terms;         /* subset-terms: sum of 2^(m-1) over the jobs */
    uint64_t row_updates;   /* row-value updates of the Gray steps inside lane chunks */
    double alg_slots;       /* algorithmic 32-bit VALU issue slots of the launch for the
                               suffix-product Gray walk: per lane chunk of 2^c indices, m ring
                               multiplies to start, then for each flip of Gray column j < c
                               its nnz(j) row updates (1 slot each) and hi[j] ring multiplies
                               (hi[j] = 1 + the lowest row of Gray column j); plus one ring
                               addition per term. In the paired walk (variant v, b = v + 1)
                               each flip of column 0 is replaced by one pair sum (2(b-1) + 1
                               ring multiplies, one ring addition per two terms) and the other
                               flips multiply only hi[j] - b rows. In the four-step walks
                               (variant 6 / 7, b = 5 / 6) each block of four terms counts the
                               FP32 products and differences of its rows 0..b-1 (13 / 16
                               slots), two conversions and a 24-bit product (4), the 64 x
                               64-bit multiply by the suffix (1.4 ring multiplies) and one ring
                               addition; the flips of column j >= 2 multiply hi[j] - b rows. One ring multiply by a 32-bit factor costs mul = 5
                               (mod 2^64), 9 (mod 2^128) or 3 * 11 (residues) slots and one
                               ring addition add = 2, 4 or 3 * 3 slots; v_mad_u64_u32 and
                               v_mul_lo_u32 count 2 slots (half rate), other ops 1 */
    double ms;              /* duration from HIP events around the launch on its stream */
    /* device H_per launches (variant 3) only; items = jobs, terms = sum of 2^(m-1) over them: */
    uint64_t leaves;        /* leaves evaluated by R-NW */
    uint64_t leaf_terms;    /* subset-terms of those leaves: sum of 2^(p-1), p the leaf order */
    uint64_t splits;        /* nodes split by expansion (2) */
    uint64_t split_stops;   /* nodes evaluated whole because a child would break the entry
                               (2^22) or row-sum (2^24) bound */
    uint64_t deferred;      /* leaves replayed and evaluated modulo 2^128 by the second kernel
                               (orders above 16, or no bound admitting the 64-bit walk) */
    uint64_t deferred_bound;/* ... of which for want of a bound admitting the 64-bit walk */
} hperm_launch_stat;

/* Copy up to max launch records of the last call into out; *n receives the count. */
hperm_status hperm_last_launches(const hperm_ctx *ctx, hperm_launch_stat *out, int32_t max,
                                 int32_t *n);

const char *hperm_status_string(hperm_status s);
/* Message of the context's last error (empty string if none); valid until the next call. */
const char *hperm_last_error(const hperm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HPERM_H */
