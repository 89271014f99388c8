/*
 * qnae: statevector simulation of depth-p QAOA on k-NAE-SAT for AMD MI355X
 * (gfx950). C ABI of libqnae.so.
 *
 * Method: Elkadi & Bondesan, "Quantum Approximate Optimisation for
 * Not-All-Equal SAT". The cost is the number of NAE-violated clauses
 * (Section 3.2), the QAOA state is prod_l U_B(beta_l) U_C(gamma_l) |+>
 * (Section 3.3), the phase is the diagonal unitary exp(-i gamma C(x))
 * (Appendix A.4) and the mixer is prod_j exp(-i beta X_j) applied as
 * butterflies on qubit pairs (Appendix A.4). The readouts are the success
 * probability <psi|{H_C = 0}|psi> (Definition of the success probability,
 * eq. psuccnae) and the expected cost <psi|H_C|psi> (Section 2.1).
 *
 * Conventions:
 *  - literals are DIMACS-style int32: +(v+1) is x_v, -(v+1) is NOT x_v, with
 *    0 <= v < n; a clause array is m rows of k literals, row-major;
 *  - basis index x = sum_v x_v 2^v (variable v is bit v of x);
 *  - the state is complex64 (interleaved float re, im), 2^n entries, in
 *    natural index order;
 *  - layer 0 is applied first; within a layer the phase comes before the mixer;
 *  - p_succ and E[C] are raw expectations on the evolved state, with no
 *    renormalisation; the norm is reported beside them.
 *
 * Every call returns an int status: QNAE_OK (0) or a negative error code. No
 * call throws. qnae_last_error() gives a message for the last failure of the
 * calling thread. Device pointers are plain HIP device addresses (for example
 * a torch tensor's data_ptr()); streams are hipStream_t passed as void*
 * (NULL is the default stream).
 */
#ifndef QNAE_H
#define QNAE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qnae_ctx qnae_ctx;

typedef struct {
    double p_success;     /* sum over C(x) = 0 of |psi(x)|^2 */
    double expected_cost; /* sum over x of C(x) |psi(x)|^2   */
    double norm;          /* sum over x of |psi(x)|^2        */
} qnae_result;

enum { QNAE_U8 = 1, QNAE_U16 = 2 };

enum {
    QNAE_OK = 0,
    QNAE_EINVAL = -1,   /* invalid argument; nothing was enqueued */
    QNAE_ENOMEM = -2,   /* device, pinned or host memory, or a host thread, could not be had */
    QNAE_EHIP = -3,     /* HIP runtime error (message has hipGetErrorString) */
    QNAE_EBUSY = -4,     /* server queue or pool full */
    QNAE_ETIMEDOUT = -5, /* server wait timed out */
    QNAE_ECANCELED = -6  /* server request cancelled */
};

/* Largest number of variables (qubits) accepted: 2^34 complex64 amplitudes
 * are 128 GiB, within one MI355X's 288 GB of HBM. */
#define QNAE_MAX_N 34

/* Create a context on HIP device `device` (make it current first if the
 * caller uses several). The context owns reusable device scratch (the state
 * when the caller passes none, block partial sums, phase tables), pinned
 * host staging and a small host thread pool. Every call on a context uses
 * that scratch, so calls on one context must not overlap: use one context per
 * calling thread. A server made from a context keeps its own pool, stream and
 * buffers and copies the context's tile shapes (tuned and default) when it is
 * made. *out is set to NULL on failure. */
int qnae_create(qnae_ctx **out, int device);

/* Release the context and everything it owns. Waits for its work. NULL is a
 * no-op. */
int qnae_destroy(qnae_ctx *ctx);

/* Message of the calling thread's last failed call (empty if none). The
 * pointer stays valid until the thread's next qnae call. ctx may be NULL. */
const char *qnae_last_error(const qnae_ctx *ctx);

/* Build the cost diagonal C(x) = number of clauses that are NAE-violated at
 * x, i.e. whose literals are all false or all true (Section 3.2,
 * eq. knaesatobj; Appendix A.2, eq. demorgannae), for every x in [0, 2^n).
 * Each literal is evaluated on its own, so a clause holding a variable with
 * both signs is never violated.
 *
 *   clauses      host, m * k int32 literals (read before the call returns;
 *                may be NULL when m = 0)
 *   m, n, k      0 <= m <= 65535, 1 <= n <= QNAE_MAX_N, 1 <= k <= 64
 *   cost_dev     caller-owned device buffer of 2^n elements of cost_dtype,
 *                16-byte aligned (written with 16-byte stores)
 *   cost_dtype   QNAE_U8 (requires m <= 255) or QNAE_U16
 *   num_solutions  optional host pointer; if not NULL the call waits for the
 *                stream and stores #{x : C(x) = 0}
 *   stream       hipStream_t the work is enqueued on
 *
 * Exact integer result (bit-exact). Without num_solutions the call is
 * asynchronous with respect to the host. Errors: QNAE_EINVAL for any bad
 * argument or literal (0, or |literal| > n), QNAE_EHIP, QNAE_ENOMEM. */
int qnae_build_cost_diagonal(qnae_ctx *ctx, const int32_t *clauses, int32_t m,
                             int32_t n, int32_t k, void *cost_dev,
                             int32_t cost_dtype, uint64_t *num_solutions,
                             void *stream);

/* Clause predicates: NAE (the paper's problem) and plain k-SAT, where an
 * OR-clause is violated exactly when every literal is false (Section 2.2). */
enum { QNAE_PRED_NAE = 0, QNAE_PRED_SAT = 1 };

/* qnae_build_cost_diagonal with the clause predicate chosen: C(x) = number of
 * clauses violated at x under `predicate`. Same arguments, results and
 * errors, plus QNAE_EINVAL for an unknown predicate. A k-SAT clause holding
 * a variable with both signs is never violated. */
int qnae_build_cost_diagonal_pred(qnae_ctx *ctx, const int32_t *clauses, int32_t m, int32_t n, int32_t k,
                                  int32_t predicate, void *cost_dev, int32_t cost_dtype,
                                  uint64_t *num_solutions, void *stream);

/* Run depth-p QAOA from |+> on the cost diagonal and read out p_succ, E[C]
 * and the norm (Section 3.3; Definition of the success probability).
 *
 *   cost_dev     device, 2^n elements of cost_dtype, values in [0, m],
 *                16-byte aligned
 *   n, m         1 <= n <= QNAE_MAX_N; m bounds the cost values (phase table
 *                length m + 1); m <= 255 for QNAE_U8, m <= 65535 for U16
 *   gammas, betas host FP64 arrays of length p (may be NULL when p = 0);
 *                layer l applies exp(-i gammas[l] C) then
 *                prod_j exp(-i betas[l] X_j)
 *   p            0 <= p <= 100000; p = 0 reads out |+>
 *   state_dev    optional caller-owned device complex64[2^n], 16-byte
 *                aligned; if not NULL it receives the final state, otherwise
 *                context scratch is used and the state is not kept
 *   out          host result
 *   stream       hipStream_t the work is enqueued on
 *
 * Synchronous: returns after *out is filled. Cost values above m give
 * undefined results. Errors: QNAE_EINVAL, QNAE_ENOMEM, QNAE_EHIP. */
int qnae_qaoa_run(qnae_ctx *ctx, const void *cost_dev, int32_t cost_dtype,
                  int32_t n, int32_t m, const double *gammas,
                  const double *betas, int32_t p, void *state_dev,
                  qnae_result *out, void *stream);

/* qnae_qaoa_run for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, kernels, sweep plan and results as qnae_qaoa_run (bit for bit,
 * under the same context's tile settings), but the call allocates nothing,
 * on the device or on the host: its device scratch (phase tables, mixer
 * forms, per-tile readout sums, the three result sums) is one static array
 * of 8.03 MiB that the library holds on each device it runs on until the
 * process ends, and its host staging is a fixed pinned buffer that
 * qnae_create reserved. Every call on a device shares that device's array
 * and keeps the last call's contents (nothing in it needs to start at zero),
 * so calls that overlap on one device race, also from different contexts.
 *
 *   state_dev    required for n > 14 (the sweeps update the state in place);
 *                optional, as in qnae_qaoa_run, for n <= 14
 *   limits       p <= 4096; p * (m + 1) <= 2^18 phase table entries;
 *                n - tile_bits <= 18 (n <= 31 with the default 13-bit tiles)
 *
 * Synchronous. Errors: QNAE_EINVAL (as qnae_qaoa_run, a size beyond the
 * limits, or a missing state_dev), QNAE_EHIP. */
int qnae_qaoa_run_noalloc(qnae_ctx *ctx, const void *cost_dev, int32_t cost_dtype, int32_t n, int32_t m,
                          const double *gammas, const double *betas, int32_t p, void *state_dev, qnae_result *out,
                          void *stream);

/* Gradient of F = w_psucc * p_succ + w_energy * E[C] with respect to every
 * gamma_l and beta_l, by the adjoint (reverse-mode) method written out by
 * hand: dF/dbeta_l = 2 Im <lam_l|sum_j X_j|psi_l> and
 * dF/dgamma_l = 2 Im <mu_l|C|phi_l>, with lam_p = W psi_p and
 * W = diag(w_psucc [C = 0] + w_energy C) (from d<psi|W|psi> = 2 Re <psi|W dpsi>
 * on the QAOA state of Section 3.3; the objective of Section 3.3's angle
 * training is the mean success probability).
 *
 * The forward pass runs in segments of `checkpoint_every` layers and keeps the
 * state at each segment end (checkpoint_every = 0 means 4). The reverse pass
 * applies the inverse layers to lam and psi together and restarts psi from
 * each checkpoint, so rounding in the uncomputed psi spans at most one segment.
 * Device memory: ceil(p / checkpoint_every) + 1 states of 2^n complex64 (n >
 * 13), held by the context.
 *
 *   dgammas, dbetas  host, p doubles each (may be NULL when p = 0)
 *   out              host readout of the forward state (as qnae_qaoa_run)
 * other arguments as qnae_qaoa_run. Synchronous. Errors: QNAE_EINVAL,
 * QNAE_ENOMEM, QNAE_EHIP. */
int qnae_qaoa_grad(qnae_ctx *ctx, const void *cost_dev, int32_t cost_dtype, int32_t n, int32_t m,
                   const double *gammas, const double *betas, int32_t p, double w_psucc, double w_energy,
                   int32_t checkpoint_every, double *dgammas, double *dbetas, qnae_result *out, void *stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent instances per launch (one GPU, ragged sizes).
 * ------------------------------------------------------------------------- */

/* One cost diagonal of a batch: the arguments of qnae_build_cost_diagonal_pred. */
typedef struct {
    const int32_t *clauses;   /* host, m * k literals (NULL when m = 0) */
    int32_t m, n, k;
    void *cost_dev;           /* caller-owned device buffer, 2^n of cost_dtype, 16-byte aligned */
    int32_t cost_dtype;       /* QNAE_U8 (m <= 255) or QNAE_U16 */
    uint64_t *num_solutions;  /* optional host pointer (the call then waits) */
    int32_t predicate;        /* QNAE_PRED_NAE (0) or QNAE_PRED_SAT */
    int32_t half;             /* 1: the lower half only, as qnae_build_cost_diagonal_z2
                                 (NAE; cost_dev holds 2^(n-1); counts are of the whole) */
} qnae_cost_job;

/* Builds `count` cost diagonals (same definition as qnae_build_cost_diagonal)
 * with one kernel launch per cost type. Clause arrays are read before the call
 * returns. Errors: QNAE_EINVAL (names the offending job), QNAE_ENOMEM,
 * QNAE_EHIP; nothing is enqueued when an argument is invalid. */
int qnae_build_cost_diagonal_batched(qnae_ctx *ctx, const qnae_cost_job *jobs, int32_t count, void *stream);

/* One QAOA solve of a batch: the arguments of qnae_qaoa_run. */
typedef struct {
    const void *cost_dev;  /* device, 2^n of cost_dtype, values in [0, m], 16-byte aligned */
    int32_t cost_dtype, n, m, p;
    const double *gammas;  /* host, p entries (layer 0 first) */
    const double *betas;   /* host, p entries */
    void *state_dev;       /* optional device complex64[2^n] for the final state, 16-byte aligned */
    int32_t half;          /* 1: half-state solve as qnae_qaoa_run_z2 (n > 14; cost_dev
                              and state_dev then hold 2^(n-1) entries) */
} qnae_instance;

/* Runs `count` independent depth-p QAOA solves (Section 3.3) together and
 * writes out[i] for inst[i]: instances with n <= 14 each run whole in one
 * workgroup, larger ones advance one sweep per launch side by side with the
 * others (tiles of all instances in one grid), each with the tile shape in use
 * for its n and cost type (qnae_autotune, qnae_autotune_batched,
 * qnae_set_tune). Results equal qnae_qaoa_run on each instance alone up to
 * FP32 rounding order. A batch of the same shape as one of the last 8 (the
 * same sizes, cost types, tile shapes and buffers) reuses its plan and
 * replays its captured launch sequence: only the angles' tables are rebuilt. States the caller does not
 * provide live in context scratch (sum of 2^n * 8 bytes). Synchronous.
 * Errors: QNAE_EINVAL (names the offending instance), QNAE_ENOMEM,
 * QNAE_EHIP. */
int qnae_qaoa_run_batched(qnae_ctx *ctx, const qnae_instance *inst, int32_t count, qnae_result *out,
                          void *stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of solve requests on one GPU.
 *
 * A server owns a device pool (one allocation, split by a buddy allocator)
 * and a scheduler thread. Requests wait in a FIFO queue and are admitted,
 * oldest first, while a slot is free and the pool can hold the request's
 * state (2^n * 8 bytes when n > 14), cost diagonal (2^n bytes, or 2^n * 2 when
 * m > 255) and tables. Every scheduler tick builds the cost diagonals of newly
 * admitted requests, runs small requests (n <= 14) to completion and advances
 * every other active request by one sweep, all requests sharing the same
 * launches; requests that finish are read out and their memory is freed, so
 * later arrivals join while earlier ones are still on the GPU. A request's
 * result equals qnae_qaoa_run on the same instance up to FP32 rounding order.
 * ------------------------------------------------------------------------- */

typedef struct qnae_server qnae_server;

/* pool_bytes: device memory for states, costs and tables (rounded down to a
 * power of two, at least 1 MiB); max_slots: requests on the GPU at once
 * (1 .. 65536). The server runs on the context's device and its own stream.
 * Errors: QNAE_EINVAL, QNAE_ENOMEM, QNAE_EHIP. */
int qnae_server_create(qnae_ctx *ctx, uint64_t pool_bytes, int32_t max_slots, qnae_server **out);

/* Queues one request (clauses, gammas and betas are copied before return;
 * literals as for qnae_build_cost_diagonal; 1 <= n <= QNAE_MAX_N). *ticket identifies
 * it for qnae_server_wait. Errors: QNAE_EINVAL (bad request, or one that can
 * never fit the pool), QNAE_EBUSY (queue of 1 << 20 requests full). */
int qnae_server_submit(qnae_server *server, const int32_t *clauses, int32_t m, int32_t n, int32_t k,
                       const double *gammas, const double *betas, int32_t p, uint64_t *ticket);

/* Waits for a request. timeout_ms < 0 waits without limit, 0 polls. On
 * success fills *out and, if latency_s is not NULL, the seconds from submit to
 * completion, and forgets the ticket. Errors: QNAE_ETIMEDOUT (not done yet;
 * the ticket stays valid), QNAE_EINVAL (unknown ticket), QNAE_EHIP (the
 * request failed on the device). */
int qnae_server_wait(qnae_server *server, uint64_t ticket, int32_t timeout_ms, qnae_result *out,
                     double *latency_s);

/* Cancels a request: a queued one leaves the queue, an active one is dropped
 * before the next scheduler tick (its pool blocks are freed). Returns QNAE_OK
 * when the request will not complete (qnae_server_wait then returns
 * QNAE_ECANCELED), 1 when it had already completed (its result can still be
 * collected). Errors: QNAE_EINVAL (unknown ticket). */
int qnae_server_cancel(qnae_server *server, uint64_t ticket);

/* Bytes of the pool held by requests now (0 once every request has ended,
 * completed, failed or cancelled). */
int qnae_server_pool_in_use(qnae_server *server, uint64_t *bytes);

/* Counters: completed requests, scheduler ticks, kernel launches, peak pool
 * bytes in use, requests waiting and active now. Any pointer may be NULL. */
int qnae_server_stats(qnae_server *server, uint64_t *completed, uint64_t *ticks, uint64_t *launches,
                      uint64_t *peak_pool_bytes, uint64_t *queued, uint64_t *active);

/* Finishes every request already submitted, stops the scheduler and frees the
 * pool. Results not yet collected are lost. NULL is a no-op. */
int qnae_server_destroy(qnae_server *server);

/* One gradient of a batch: the arguments of qnae_qaoa_grad for one instance. */
typedef struct {
    const void *cost_dev;  /* device, 2^n of cost_dtype, values in [0, m] */
    int32_t cost_dtype, n, m, p;
    const double *gammas;  /* host, p entries (layer 0 first) */
    const double *betas;   /* host, p entries */
    double *dgammas;       /* host output, p entries */
    double *dbetas;        /* host output, p entries */
} qnae_grad_job;

/* Gradients of w_psucc p_succ + w_energy E[C] for `count` instances (same
 * definition as qnae_qaoa_grad), e.g. the terms of the training objective
 * (1/t) sum_i p_succ(sigma_i) over t instances (Section 3.3, fixed-angle
 * pretraining). Instances with n <= 13 run together in one launch per cost
 * type, one workgroup each; larger ones run one after another. out[i]
 * receives instance i's readout. Synchronous. Errors: QNAE_EINVAL (names the
 * job), QNAE_ENOMEM, QNAE_EHIP. */
int qnae_qaoa_grad_batched(qnae_ctx *ctx, const qnae_grad_job *jobs, int32_t count, double w_psucc, double w_energy,
                           int32_t checkpoint_every, qnae_result *out, void *stream);

/* Half-state simulation for NAE instances. The NAE cost is symmetric under
 * flipping every variable (Section 2.2), and |+>, the phase and the mixer
 * commute with that flip, so psi(x) = psi(NOT x) at every layer: the state
 * and the cost diagonal are kept for x < 2^(n-1) only (the lower half), and
 * the mixer factor of variable n-1 pairs a stored index y with 2^(n-1)-1-y.
 * Half the memory and half the bytes per layer of qnae_qaoa_run.
 *
 * qnae_build_cost_diagonal_z2: as qnae_build_cost_diagonal (NAE predicate)
 * for x in [0, 2^(n-1)); cost_dev holds 2^(n-1) elements; *num_solutions,
 * if requested, counts the whole diagonal (twice the lower half). n >= 2.
 *
 * qnae_qaoa_run_z2: as qnae_qaoa_run on such a half diagonal; 15 <= n <=
 * QNAE_MAX_N (smaller n run whole in one workgroup: use qnae_qaoa_run).
 * state_dev, if not NULL, receives psi(x) for x < 2^(n-1) (2^(n-1)
 * complex64); the upper half is psi(x) = psi(2^n - 1 - x). Results equal
 * qnae_qaoa_run's within FP32 rounding. Errors as qnae_qaoa_run. */
int qnae_build_cost_diagonal_z2(qnae_ctx *ctx, const int32_t *clauses, int32_t m, int32_t n, int32_t k,
                                void *cost_dev, int32_t cost_dtype, uint64_t *num_solutions, void *stream);
int qnae_qaoa_run_z2(qnae_ctx *ctx, const void *cost_dev, int32_t cost_dtype, int32_t n, int32_t m,
                     const double *gammas, const double *betas, int32_t p, void *state_dev, qnae_result *out,
                     void *stream);

/* Draws `count` bitstrings from the outcome distribution |psi(x)|^2 / norm of
 * a state, as measuring the final QAOA state does (Section 4.2: the instance
 * running time is the number of draws until one satisfies the instance). The
 * draw for uniforms[q] is the smallest x whose cumulative mass, in index
 * order, exceeds uniforms[q] times the total: FP32 |psi|^2 summed in FP64
 * per tile of 4096 amplitudes, prefix sums over tiles; a uniform within about
 * 1e-7 of a cumulative boundary may therefore land on the neighbouring
 * outcome.
 *
 *   state_dev     device complex64[2^n], 16-byte aligned, e.g. the state
 *                 kept by qnae_qaoa_run
 *   cost_dev      optional device cost diagonal (cost_dtype QNAE_U8/U16);
 *                 with it, sample_costs[q] = C(samples[q])
 *   uniforms      host, count doubles in [0, 1) (the caller's random numbers)
 *   samples       host, count outcomes; sample_costs host or NULL
 *   count         0 <= count <= 2^24
 *
 * Synchronous. Errors: QNAE_EINVAL (bad n, count, pointer, cost_dtype, a
 * uniform outside [0, 1), or a state of zero norm), QNAE_ENOMEM, QNAE_EHIP. */
int qnae_sample(qnae_ctx *ctx, const void *state_dev, int32_t n, const void *cost_dev, int32_t cost_dtype,
                const double *uniforms, int32_t count, uint64_t *samples, int32_t *sample_costs, void *stream);

/* Tile shape of the sweep path (qnae_qaoa_run for n > 14). The mixer of one
 * layer is n butterfly passes over the state (appendix A.4); the library
 * fuses them into sweeps, each applying the passes of a group of index bits
 * to tiles of 2^tile_bits amplitudes held on chip. Every tile starts with a
 * contiguous run of 2^low_run_bits amplitudes; index bits from page_bit up
 * are spread over the groups so that a tile touches few memory pages
 * (page_bit 64: no spreading). With two groups besides the first, `split`
 * chooses which of the index bits below page_bit the third group mixes:
 * 0 the top run of them (the second group the run below), 1 the top run
 * less one and the second-lowest, 2 the top run less one and the lowest,
 * 3 the top three and every other one from the lowest up; other group counts
 * ignore it. The fastest shape depends on n and is found by timing, not by
 * formula. */
typedef struct {
    int32_t tile_bits;    /* 12, 13 or 14 */
    int32_t low_run_bits; /* 4 .. 6 */
    int32_t page_bit;     /* 4 .. 64 */
    int32_t split;        /* 0 .. 3 */
    double ms_per_layer;  /* measured by qnae_autotune; ignored by qnae_set_tune */
} qnae_tune;

/* Times every candidate shape (tile_bits 12..14 x low_run_bits 4..5 x
 * page_bit 18 or 64, split 0; then splits 1..3 of the fastest of those for
 * each tile size, when its groups have a third) on `reps` two-layer and
 * `reps` four-layer runs of
 * an n-qubit state in the context's scratch memory, on `stream`, ranks them
 * by the time per layer of a ten-layer run (extrapolated linearly in the
 * layer count from the two; written to ms_per_layer), keeps the fastest for
 * later qnae_qaoa_run calls at this n and cost type on this context, and
 * writes it to *out. Needs 2^n * (8 + cost bytes) of device memory. For n <= 14 the
 * whole circuit runs in one workgroup and there is nothing to tune: *out is
 * all zeros. Synchronous. Errors: QNAE_EINVAL (n outside [1, QNAE_MAX_N], bad
 * cost_dtype, reps outside [1, 1000], null out), QNAE_ENOMEM, QNAE_EHIP. */
int qnae_autotune(qnae_ctx *ctx, int32_t n, int32_t cost_dtype, int32_t reps, qnae_tune *out, void *stream);

/* The tile shape of the batched path, tuned on the batch itself: runs
 * qnae_qaoa_run_batched on `inst` under every candidate shape of
 * qnae_autotune, applied to all of its instances with n > 14 (one warm-up
 * run, then `reps` timed runs, wall clock, host preparation included), and
 * keeps the fastest for every (n, cost type) among those instances on this
 * context: later batched runs, single runs and servers made afterwards use
 * it. *out receives it, with ms_per_layer the time per instance-layer of the
 * whole batch (all zeros when no instance has n > 14). Cost diagonals are
 * only read; state buffers the instances name hold a final state of one of
 * the runs. Synchronous. Errors: those of qnae_qaoa_run_batched,
 * QNAE_EINVAL for reps outside [1, 100] or a null out. */
int qnae_autotune_batched(qnae_ctx *ctx, const qnae_instance *inst, int32_t count, int32_t reps, qnae_tune *out,
                          void *stream);

/* Sets (tune != NULL) or clears (NULL) the shape used at n and cost_dtype,
 * e.g. from a saved autotune result. qnae_get_tune writes the shape in use:
 * the tuned one if set, else the default (ms_per_layer 0). Errors:
 * QNAE_EINVAL (n outside [15, QNAE_MAX_N], bad cost_dtype or shape). */
int qnae_set_tune(qnae_ctx *ctx, int32_t n, int32_t cost_dtype, const qnae_tune *tune);
int qnae_get_tune(qnae_ctx *ctx, int32_t n, int32_t cost_dtype, qnae_tune *out);

/* Kernel timing with HIP events, for measurement. While enabled, the context
 * records an event pair around every kernel it launches, on the stream the
 * kernel runs on, and tallies per kernel kind the number of launches, the
 * summed event time and the algorithmic bytes (the state, cost and table
 * traffic the method needs, not what the hardware moved).
 * qnae_profile_read waits for the recorded events, writes up to `capacity`
 * entries, sets *count to the number of kinds seen and clears the tallies.
 * `name` points to static storage. */
typedef struct {
    const char *name;
    uint64_t launches;
    double total_ms;
    double bytes;
} qnae_kernel_stat;

int qnae_profile_enable(qnae_ctx *ctx, int on);
int qnae_profile_read(qnae_ctx *ctx, qnae_kernel_stat *out, int32_t capacity, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* QNAE_H */
