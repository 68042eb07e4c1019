/*
 * npf.h -- C ABI of the MI355X (gfx950) library for high-order nonlinear participation
 * factors (NPFs) by batched tensor contraction (Sajjadi, Huang, Sun, arXiv 2509.08968).
 *
 * The library runs the hot path of the paper's vectorized method (Alg. 2) for one
 * diagonalizable system with n states, orders M = 2..N:
 *
 *   C_M[j,t] = (1/M!) sum_k Psi[j,k] sum_{a} A_M[k,a] Phi[a_1,t_1] .. Phi[a_M,t_M]
 *                                                  (Alg. 2 steps 1-4; eq. (4) numerator)
 *   D_M[j,t] = (lam[t_1] + .. + lam[t_M]) - lam[j],  |D| < eps -> D = eps (steps 5-9)
 *   h_M[j,t] = C_M[j,t] / D_M[j,t]                   (step 11; eq. (4))
 *   P_M[j,k] = - sum_{t in [n]^M} h_M[j,t] prod_i delta Psi[t_i,k]   (steps 12-19; eq. (7))
 *   NPF[k,i] = Phi[k,i] (delta Psi[i,k] + sum_{M=2..N} P_M[i,k])      (step 20; eq. (7))
 *
 * with Phi the right eigenvectors (columns), Psi = Phi^{-1} the left eigenvectors (rows),
 * lam the eigenvalues, A_M the M-th derivative tensor of the vector field at the
 * equilibrium (eq. (1)), symmetric in its M lower indices, and delta the excitation
 * magnitude of the kicked state (eq. (6)-(7)).
 *
 * Conventions
 *   - Sizes are int64_t.  Every array pointer passed to a compute call is a DEVICE pointer
 *     owned by the caller; the library never allocates or frees device memory.
 *   - Complex arrays are interleaved (re, im) double pairs (complex128), row-major:
 *       Phi[a*n + i] = Phi[state a, mode i];  Psi[i*n + k] = Psi[mode i, state k];
 *       lam[i];  P[j*n + k] (mode j, state k);  NPF[k*n + i] (state k, mode i).
 *   - Symmetric tensors are packed over sorted index tuples t_1 <= .. <= t_M (0-based) at
 *     the colex rank r(t) = sum_{i=1..M} binom(t_i + i - 1, i), so an order-M tensor over
 *     n states has U_M = binom(n + M - 1, M) entries per upper index.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Compute calls
 *     only enqueue work and return; they are ordered on `stream`.
 *   - Errors: calls return NPF_OK (0) or an NPF_E_* code.  Argument errors are found
 *     before anything is enqueued and nothing is written.  NPF_E_DEVICE reports a HIP
 *     launch error.  npf_last_error() gives a message for the calling thread.
 *   - A plan is an opaque host object holding only host metadata; it may be shared by
 *     calls on different streams, but calls that share a workspace must be serialised.
 */
#ifndef NPF_H
#define NPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NPF_OK 0
#define NPF_E_INVALID 1     /* bad argument, shape or size                        */
#define NPF_E_BUDGET 2      /* the memory budget is below the smallest block      */
#define NPF_E_DEVICE 3      /* a HIP call or kernel launch failed                 */
#define NPF_E_UNSUPPORTED 4 /* valid request the library does not serve           */

#define NPF_MAX_ORDER 6     /* largest N                                           */
#define NPF_ALL_BLOCKS (-1)

/* Arithmetic of the contractions (the divisor and the NPF accumulation are always FP64). */
#define NPF_FP64 0          /* FP64 operands, FP64 accumulation                    */
#define NPF_FP32 1          /* FP32 operands and intermediates, exact products
                               accumulated in FP64                               */
#define NPF_BF16X3 2        /* FP32 values split in three BF16 terms, six products
                               per multiply, FP32 accumulation per tile            */
/* NPF_FP32 and NPF_BF16X3 serve order_max <= 4 (npf_plan_create returns NPF_E_UNSUPPORTED
 * above): C is held in FP32 once per sorted tuple and shared by all of the tuple's
 * orderings, whose coherent error exceeds 1e-6 relative at orders 5 and 6. */

/* Storage of one derivative tensor A_M (device memory). */
#define NPF_SRC_DENSE 0     /* values[k*U_M + r]                                   */
#define NPF_SRC_SPARSE 1    /* compressed by sorted tuple: for c in [0, ncols):
                               rank col_rank[c], entries col_ptr[c]..col_ptr[c+1]-1
                               with state row_k[e] and value values[e]            */
#define NPF_SRC_HASH 2      /* generated on the device, never stored: entry (k, r) is
                               hash_value(seed, scale, M, k, r) as defined at
                               npf_hash_fill; needs n <= 512 and U_M < 2^40          */

typedef struct npf_tensor {
    int32_t kind;
    int32_t order;             /* M                                                  */
    const double *values;      /* dense [n*U_M] or sparse [nnz]                      */
    const int64_t *col_rank;   /* sparse: [ncols], strictly increasing               */
    const int64_t *col_ptr;    /* sparse: [ncols+1], col_ptr[0] = 0                  */
    const int32_t *row_k;      /* sparse: [nnz], 0 <= row_k < n                       */
    int64_t ncols;
    int64_t nnz;
    uint64_t seed;             /* hash: generator seed                               */
    double scale;              /* hash: scale of every entry                          */
} npf_tensor;

/* Problem description (host memory; copied by npf_plan_create). */
typedef struct npf_problem {
    int64_t n;                 /* states = modes, 1 <= n <= 512 (NPF_BF16X3: 256)     */
    int32_t order_max;         /* N, 2 <= N <= NPF_MAX_ORDER                          */
    int32_t precision;         /* NPF_FP64 / NPF_FP32 / NPF_BF16X3                    */
    double eps;                /* divisor clamp of Alg. 2 step 9, > 0                 */
    double tau;                /* mixed paths divide in FP64 when |D| < tau, >= 0     */
    double delta;              /* excitation magnitude of eq. (7)                     */
    int64_t hbm_budget_bytes;  /* workspace cap, the M_limit of Alg. 1; 0 = none      */
    int64_t block_modes;       /* output modes per block; 0 = chosen by the planner   */
    int32_t flags;             /* NPF_FLAG_* bits                                      */
    int32_t support_max;       /* 1..8: no row k of a sparse A_M involves more than this
                                  many distinct states; order 3 (for n > 64, or any n
                                  in FP64) and order 2 (for n > 96) then contract each
                                  row's lower indices over its own states first and apply
                                  Psi after (a row with more states makes the results
                                  NaN).  0: no bound, the upper index first everywhere.   */
    int32_t a_convention;      /* NPF_A_DERIVATIVE or NPF_A_TAYLOR (below)             */
    int32_t reserved;          /* 0                                                    */
    /* Output modes (the critical modes of Section III): the P_M rows and NPF columns of
     * these modes only are computed and written; the rest of P_out and npf_out is left
     * untouched.  n_modes = 0 (modes may be NULL) selects all n modes.  Otherwise
     * modes[0 .. n_modes-1] are distinct indices in [0, n) (host memory, copied). */
    int64_t n_modes;
    const int64_t *modes;
    /* Conjugate pairs of a real system (eq. (1) has real derivative tensors): conj_of[i]
     * is the mode whose eigenvalue, right and left eigenvectors are the complex conjugates
     * of mode i's (conj_of[i] = i for a real mode); host [n], an involution, or NULL.  For a
     * real A_M, C, h, P_M and the NPF of mode conj_of[i] are then the conjugates of mode i's
     * (with the tuple's modes conjugated too), so of each requested pair only the lower
     * index is computed and the other's P row and NPF column are filled by conjugation
     * (about half the work).  The caller vouches for the pairing; with host copies below
     * the planner checks it. */
    const int64_t *conj_of;
    /* Optional host copies (complex128, the layouts of the compute calls) for the
     * preconditions: |Psi Phi - I| <= check_tol entrywise (eigenvector normalisation of
     * Alg. 2), and for conj_of: lam, Phi columns and Psi rows of paired modes conjugate to
     * check_tol relative to their largest entry.  Any may be NULL (that check is skipped:
     * host_U and host_V are needed for the first and for the eigenvector part of the
     * second).  check_tol = 0 selects 1e-8. */
    const void *host_U, *host_V, *host_lambda;
    double check_tol;
} npf_problem;

/* Input convention of the derivative tensors (eq. (1) against Alg. 2 step 4). */
#define NPF_A_DERIVATIVE 0  /* A_M holds the M-th derivatives; C carries the 1/M! of
                               Alg. 2 step 4 (the Taylor coefficient is A_M / M!)   */
#define NPF_A_TAYLOR 1      /* A_M holds the Taylor coefficients of eq. (1) as printed
                               (x' = A1 x + A2 x x + ..): no 1/M! is applied        */

/* npf_run replays a HIP graph of its launch sequence when called again with the same
 * problem, pointers, descriptors and stream (the graph is captured on the first call; up to
 * 16 argument sets are kept for the life of the process, further ones run eagerly).
 * This flag disables that and always launches eagerly.  Graphs are never used on the
 * NULL stream, on a stream that is already capturing, or while profiling. */
#define NPF_FLAG_NO_GRAPH 1
/* When the plan has one block of modes and at least two orders, the orders' chains and last
 * stages run concurrently inside the replayed graph, each in workspace of its own (the
 * partial sums still run in order); this flag keeps them in sequence and the workspace
 * smaller.  Eager runs are always sequential. */
#define NPF_FLAG_SERIAL_ORDERS 2

typedef struct npf_plan_s *npf_plan_t;

typedef struct npf_plan_report {
    int64_t n;
    int32_t order_max;
    int32_t precision;
    int64_t workspace_bytes;           /* size of `ws` for every compute call          */
    int64_t block_modes;               /* J: output modes per block                    */
    int64_t n_blocks;                  /* ceil(n / J)  (the BC of Alg. 1 for mode j)   */
    int64_t unique_tuples[NPF_MAX_ORDER + 1];   /* U_M per order                       */
    int64_t modal_entries;             /* sum_M n * U_M, symmetric-unique entries      */
    int64_t output_modes;              /* modes whose P rows / NPF columns are written */
    int64_t computed_modes;            /* of which computed (the others by conjugation) */
} npf_plan_report;

/* Plan (host only, synchronous): validates the problem, fixes the output-mode block size
 * J under hbm_budget_bytes following the batch-size rule of Alg. 1 (steps 6-15) and the
 * workspace size.  Blocks run over the computed modes (all n, or the output modes less
 * the conjugates filled from their partners), in ascending order.  Returns NPF_E_BUDGET if
 * even the smallest block does not fit, NPF_E_INVALID for a bad mode list, pairing or a
 * failed precondition check (the message says which). */
int npf_plan_create(const npf_problem *problem, npf_plan_t *plan_out);
int npf_plan_info(npf_plan_t plan, npf_plan_report *report);
/* The computed modes in block order (computed[c], c < computed_modes: block b holds
 * c in [b*J, b*J + J)) and, per computed mode, the output mode filled by its conjugate
 * (filled[c], -1 for none).  Either pointer may be NULL. */
int npf_plan_modes(npf_plan_t plan, int64_t *computed, int64_t *filled);
/* Releases the plan (host metadata only: runs already enqueued are unaffected, and the
 * graphs npf_run instantiated stay cached for later plans of the same problem). */
void npf_plan_destroy(npf_plan_t plan);

/* Alg. 2 steps 1-4 for output-mode block `block` (computed modes c in [block*J,
 * min(computed_modes, block*J+J)), see npf_plan_modes; NPF_ALL_BLOCKS: all of them) of
 * order M: writes C_out[jj*U_M + r] (complex128, jj = c - first block's c) for the block's
 * modes and every sorted tuple r.  U, V: Psi, Phi as above.  ws: device workspace of at
 * least workspace_bytes.  The contraction runs in the plan's precision. */
int npf_modal_contract(npf_plan_t plan, int32_t order, int64_t block, const npf_tensor *A,
                       const void *U, const void *V, void *ws, int64_t ws_bytes,
                       void *C_out, void *stream);

/* Alg. 2 steps 5-11 in place on the block's C (as written by npf_modal_contract):
 * h = C / D with D = (lam[t_1] + .. + lam[t_M]) - lam[j] summed in FP64 over the sorted
 * tuple left to right; |D|^2 < eps^2 (FP64, no fused multiply-add) sets D = eps. */
int npf_normal_form(npf_plan_t plan, int32_t order, int64_t block, const void *lambda,
                    void *C_inout, void *stream);

/* Alg. 2 steps 12-19 for the block: P_acc[j*n + k] += -sum_{sorted t} m(t) h[j,t]
 * prod_i delta Psi[t_i,k], with m(t) the number of orderings of t; FP64.  j is the output
 * mode of each computed mode of the block; a mode filled by conjugation gets
 * P_acc[j'*n + k] += the conjugate of the same sum. */
int npf_assemble(npf_plan_t plan, int32_t order, int64_t block, const void *h,
                 const void *U, void *P_acc, void *stream);

/* ---------------------------------------------------------------- batched systems
 * Many operating points (systems of uneven n, each with its own orders 2..N) through the
 * whole hot path in one call: the per-step launches of all systems of the same padded
 * size run as single launches whose workgroups are shared out in proportion to each
 * system's work; systems run together in waves whose summed workspace fits the budget
 * (the batching of Alg. 1 applied across systems); the call replays one captured graph.
 * Split-BF16 precision only (problems[s].precision == NPF_BF16X3), N <= 4, n <= 256; every
 * system is one block of all its modes (no mode subset, conjugate pairing or Taylor
 * convention: NPF_E_UNSUPPORTED). */
typedef struct npf_batch_s *npf_batch_t;

typedef struct npf_batch_report {
    int64_t systems;
    int64_t waves;              /* groups of systems that run together                 */
    int64_t workspace_bytes;    /* device workspace npf_batch_run needs                 */
    int64_t modal_entries;      /* sum over systems and orders of n * U_M               */
    int64_t launches;           /* kernel launches per run                             */
    int64_t shared_launches;    /* of which launches over several systems              */
} npf_batch_report;

/* Host only, synchronous.  problems[count]: as for npf_plan_create (block_modes and
 * hbm_budget_bytes of each are ignored).  hbm_budget_bytes caps the workspace of a wave
 * (0 = all systems in one wave).  Errors: NPF_E_INVALID (bad problem, count < 1),
 * NPF_E_UNSUPPORTED (precision, order or size outside the batched kernels),
 * NPF_E_BUDGET (one system alone exceeds the budget). */
int npf_batch_create(const npf_problem *problems, int64_t count, int64_t hbm_budget_bytes,
                     npf_batch_t *batch_out);
int npf_batch_info(npf_batch_t batch, npf_batch_report *report);
void npf_batch_destroy(npf_batch_t batch);

/* Runs every system.  Host arrays of device pointers, one entry per system s:
 *   A[s*(NPF_MAX_ORDER-1) + M-2]   descriptor of A_M of system s (M = 2..N_s; host array)
 *   U[s], V[s], lambda[s]          Psi, Phi, eigenvalues as for npf_run
 *   P_out[s]                       [N_s-1][n][n] complex128 or NULL (P_out may be NULL)
 *   npf_out[s]                     [n][n] complex128
 * ws: device workspace of at least workspace_bytes, owned by the call until it completes.
 * Asynchronous on `stream`; on a non-NULL stream the launch sequence is captured once per
 * argument set and replayed.  Errors as npf_run. */
int npf_batch_run(npf_batch_t batch, const npf_tensor *A, const void *const *U,
                  const void *const *V, const void *const *lambda, void *ws, int64_t ws_bytes,
                  void *const *P_out, void *const *npf_out, void *stream);

/* Autotuner: times every shared launch for each candidate number of workgroups per
 * launch (eager runs with events on `stream`, synchronous), keeps the fastest per launch
 * and returns the chosen counts in chosen[launch] (nullable, shared_launches entries).
 * The same arguments as npf_batch_run; its outputs are written as by a run. */
int npf_batch_tune(npf_batch_t batch, const npf_tensor *A, const void *const *U,
                   const void *const *V, const void *const *lambda, void *ws, int64_t ws_bytes,
                   void *const *P_out, void *const *npf_out, void *stream, int64_t *chosen);

/* One shared launch of a batch (launches in run order), for measurement. */
typedef struct npf_batch_launch {
    int32_t wave;
    int32_t kind;               /* 0: chain stage `stage` of `order`; 1: fused last stage */
    int32_t npad;               /* padded size of the systems it runs                    */
    int32_t order, stage, systems;
    int64_t workgroups;
    double flops;               /* algorithmic flops (complex multiply-add = 8)          */
    double ms;                  /* duration in the last npf_batch_time run (0 before)    */
} npf_batch_launch;

/* Copies up to `cap` launch records into out (nullable) and their number into *count. */
int npf_batch_launches(npf_batch_t batch, npf_batch_launch *out, int64_t cap, int64_t *count);

/* One eager run with an event pair around every shared launch (synchronous); the
 * durations land in the launch records.  Arguments and outputs as npf_batch_run. */
int npf_batch_time(npf_batch_t batch, const npf_tensor *A, const void *const *U,
                   const void *const *V, const void *const *lambda, void *ws, int64_t ws_bytes,
                   void *const *P_out, void *const *npf_out, void *stream);

/* Materialises rows [k0, k1) of a hash-generated derivative tensor (the NPF_SRC_HASH
 * source; the paper's own tensors come from finite differences of the model, for which
 * this generator is the synthetic stand-in): out[(k - k0)*U_M + r] (device, FP64, caller
 * owned) for every colex rank r, U_M = binom(n + order - 1, order).  The entry is
 *   w = SplitMix64 output number (order << 49 | k << 40 | r) from seed (Steele, Lea and
 *       Flood 2014: z = seed + (idx + 1) * 0x9E3779B97F4A7C15, then the finaliser with
 *       shifts 30, 27, 31 and multipliers 0xBF58476D1CE4E5B9, 0x94D049BB133111EB),
 *   S = sum of the four 16-bit fields of w,
 *   value = ((S - 131070) * 2^-16 * sqrt(3)) * scale, rounded in that order,
 * an Irwin-Hall variate of mean 0 and variance scale^2.  Asynchronous on `stream`.
 * Errors: NPF_E_INVALID for n < 1 or n > 512, order outside [2, NPF_MAX_ORDER],
 * k0 < 0, k1 > n, k0 > k1, U_M >= 2^40 or a null out with k1 > k0. */
int npf_hash_fill(int64_t n, int32_t order, uint64_t seed, double scale, int64_t k0,
                  int64_t k1, double *out, void *stream);

/* A polynomial vector field x' = f(x), term by term (device memory, caller owned): term q
 * is coef[q] * prod_i x_{var[q*max_degree + i]} over the entries of var that are >= 0
 * (variables with repetition, padded with negative values); the terms of equation k are
 * eq_ptr[k] .. eq_ptr[k+1]-1 (eq_ptr has n + 1 entries, non-decreasing; values outside
 * [0, n_terms] are clamped).  x_eq is the expansion point x* [n], NULL for the origin. */
typedef struct npf_poly {
    int64_t n_terms;
    const int64_t *eq_ptr;
    const double *coef;
    const int32_t *var;
    int32_t max_degree;        /* 1..8 entries of var per term                        */
    int32_t reserved;
    const double *x_eq;
} npf_poly;

/* The numerical Taylor expansion of Alg. 1 (Section II-B) on the device: rows [k0, k1) of
 * the M-th derivative tensor of the field at x*, out[(k - k0)*U_M + r] (device, FP64,
 * caller owned) = d^M f_k / dx_{t_1} .. dx_{t_M} at x* for the sorted tuple t of colex
 * rank r, U_M = binom(n + order - 1, order): the convention NPF_A_DERIVATIVE, ready for
 * npf_run as an NPF_SRC_DENSE tensor (order 1 gives the Jacobian).  Each entry comes from
 * values of the field's terms at x* + s y_S, y_S the sums of the unit vectors of the
 * subsets S of t: the alternating sum over S (polarization) and Lagrange extraction of
 * the s^M coefficient are exact for polynomials, so only rounding separates the result
 * from the derivative.  A row with a variable >= n reads NaN.  Asynchronous on `stream`.
 * Errors: NPF_E_INVALID for a null poly, n < 1, order outside [1, NPF_MAX_ORDER],
 * max_degree outside [1, 8], n_terms < 0, a bad row range, U_M >= 2^40, or null arrays
 * where rows or terms are to be read or written. */
int npf_taylor_fill(int64_t n, int32_t order, const npf_poly *poly, int64_t k0, int64_t k1,
                    double *out, void *stream);

/* Alg. 2 step 20: NPF[k*n + i] = Phi[k,i] (delta Psi[i,k] + P_sum[i*n + k]).
 * P_sum may be NULL (the linear participation factors). */
int npf_finalize(npf_plan_t plan, const void *U, const void *V, const void *P_sum,
                 void *npf_out, void *stream);

/* The whole hot path, all orders 2..N and all blocks, with the last contraction, the
 * divisor, the division and the reduction fused: A[M-2] describes A_M.  Writes
 * P_out[(M-2)*n*n + j*n + k] (nullable) and NPF (nullable).  Deterministic: two calls on
 * the same inputs give bitwise equal results.  See NPF_FLAG_NO_GRAPH for graph replay;
 * a replayed graph reads the device buffers afresh, so new input values are honoured as
 * long as the pointers and descriptors are unchanged. */
int npf_run(npf_plan_t plan, const npf_tensor *A, const void *U, const void *V,
            const void *lambda, void *ws, int64_t ws_bytes, void *P_out, void *npf_out,
            void *stream);

/* Interaction participation factors of eqs. (8)-(9), after the NPFs of npf_run (whose
 * outputs P_out and npf_out it also writes, each nullable): with the corrected modal
 * initial condition of eq. (9),
 *   zeta*_k[a] = delta Psi[a,k] + sum_{M=2..N} P_M[a,k]      (= z(0) of eq. (7)),
 * the factor of order M is
 *   inpf_out[(M-2)*n*n + k*n + i] = Phi[k,i] sum_{t in [n]^M} h_M[i,t] prod_l zeta*_k[t_l]
 * (pNM of state k in mode i, eq. (8): h_M contracted with M factors zeta*), for M = 2..N
 * (inpf_out: [N-1][n][n] complex128, device).  The NPF of npf_run is the order-1 term of
 * the decomposition of eq. (6).  Runs a second pass of every order's chain, last
 * contraction and reduction with zeta* in place of zeta = delta Psi (about twice the time
 * of npf_run).  Needs every mode's P row: NPF_E_UNSUPPORTED for a plan with output modes
 * (conjugate pairs are fine).  Other errors as npf_run. */
int npf_run_interaction(npf_plan_t plan, const npf_tensor *A, const void *U, const void *V,
                        const void *lambda, void *ws, int64_t ws_bytes, void *P_out,
                        void *npf_out, void *inpf_out, void *stream);

/* npf_run for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same launch sequence, run eagerly with
 * the orders in sequence, on a workspace the library holds itself -- a static device array of
 * NPF_STATIC_WORKSPACE_BYTES per GPU, held until the process ends.  Allocates nothing.
 * Returns NPF_E_UNSUPPORTED when the plan's workspace_bytes exceed that size (plan with
 * NPF_FLAG_SERIAL_ORDERS or fewer modes per block to shrink it), NPF_E_INVALID for the
 * argument errors of npf_run or a plan that is profiling.  Every call on a GPU uses that
 * GPU's one array: calls that overlap on one GPU (on different streams or host threads)
 * race and must be serialised by the caller.  No part of the workspace needs clearing: each
 * call writes every part it reads before reading it. */
#define NPF_STATIC_WORKSPACE_BYTES (256ll << 20)
int npf_run_static(npf_plan_t plan, const npf_tensor *A, const void *U, const void *V,
                   const void *lambda, void *P_out, void *npf_out, void *stream);

/* Alg. 1 (batched derivative tensor) arithmetic, host only: for a tensor with n_dim
 * dimensions of extent n_s, bytes_per_entry bytes per entry and a limit of m_limit_gb
 * GiB per batch, writes the batch count per dimension BC[n_dim], the largest batch
 * extent per dimension max_batch[n_dim], the total size in GiB and the size of one batch
 * in GiB.  Returns the number of batches prod(BC), or -1 on bad arguments. */
int64_t npf_alg1_batches(int32_t n_dim, int64_t n_s, double m_limit_gb, int32_t bytes_per_entry,
                         int64_t *BC, int64_t *max_batch, double *total_gb, double *batch_gb);

/* Kernel timing (host, for measurement).  npf_plan_profile(plan, 1) clears earlier records
 * and makes later compute calls with this plan record a HIP event pair around every kernel
 * launch, on the launch stream; npf_plan_profile(plan, 0) stops recording.
 * npf_plan_kernel_times waits for the recorded events and writes, per kernel name, the
 * number of launches and their summed duration in milliseconds (at most `capacity`
 * entries; *count receives the number of names). */
typedef struct npf_kernel_time {
    char name[40];
    int64_t launches;
    double total_ms;
} npf_kernel_time;

int npf_plan_profile(npf_plan_t plan, int32_t enable);
int npf_plan_kernel_times(npf_plan_t plan, npf_kernel_time *out, int32_t capacity,
                          int32_t *count);

const char *npf_error_string(int code);
const char *npf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
