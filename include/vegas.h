/*
 * vegas.h -- C ABI of the MI355X (gfx950) Vegas iteration library (libvegas).
 *
 * The library runs the data-parallel hot path of Vegas adaptive Monte Carlo
 * integration, the method the paper integrates with (sec. 2.2: importance
 * sampling as implemented in Vegas -- a per-event stage that generates and
 * weights random points, then, once an integration pass is finished, a
 * refinement of how the random numbers are generated), on one GPU:
 *
 *   counter-based points -> per-dimension piecewise-linear grid map and
 *   Jacobian -> integrand -> sums of f*w and (f*w)^2 and per-dimension,
 *   per-bin histograms of (f*w)^2 -> iteration estimate and variance ->
 *   grid refinement -> inverse-variance combination ("value +- error",
 *   Table 1).
 *
 * Conventions for every entry point:
 *  - All calls return a vegas_status; they never throw or abort.  On a
 *    non-OK status vegas_last_error() returns a message (thread-local).
 *  - Argument validation happens before any HIP call.
 *  - Streams are hipStream_t values passed as void* (NULL = default stream).
 *    Every call only enqueues work on the given stream, except those marked
 *    "synchronises", which wait for the stream to finish.
 *  - Device memory is owned by the caller: the context lives in one
 *    caller-allocated device workspace (see vegas_workspace_size).  The
 *    library itself never allocates device memory; it owns only a small host
 *    context, a small pinned host staging buffer and, for batches, a HIP graph.
 *  - One context must not be used from two host threads at once.
 *
 * Limits: 1 <= dim <= 64, 2 <= n_bins <= 255, and the per-block LDS image of
 * the grid and histograms must fit the device (dim * n_bins * 24 bytes for
 * FP64, dim * n_bins * 16 bytes for FP32-mixed, at most 160 KiB).
 */
#ifndef VEGAS_H
#define VEGAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vegas_ctx vegas_ctx;
typedef struct vegas_batch vegas_batch;
typedef void* vegas_stream_t; /* a hipStream_t */

typedef enum {
    VEGAS_OK = 0,
    VEGAS_EINVAL = -1,      /* invalid argument */
    VEGAS_ESTATE = -2,      /* call not valid in the context's current state */
    VEGAS_EWORKSPACE = -3,  /* workspace too small or misaligned */
    VEGAS_EHIP = -4,        /* a HIP runtime call failed (message kept) */
    VEGAS_ENONFINITE = -5,  /* a recorded iteration had a non-finite estimate */
    VEGAS_EUNSUPPORTED = -6, /* valid request this build does not support */
    VEGAS_ECOMPILE = -7      /* a user integrand's source did not compile (log kept) */
} vegas_status;

/* Integrands (sec. 3.1).  params layout (FP64, host pointer at init):
 *  VEGAS_GAUSS     f = nu exp(-sum_i (x_i - mu_i)^2 / a^2),  nu = (a sqrt(pi))^-d
 *                  (Eq. lepage with centre mu; mu_i = 1/2 is the paper's case)
 *                  params = a, mu[0..d-1]                              (1 + d)
 *  VEGAS_BIMODAL   f = nu/2 [G(x; muA) + G(x; muB)], G as above
 *                  params = a, muA[0..d-1], muB[0..d-1]                (1 + 2d)
 *  VEGAS_GENZ_DISC f = 0 if any x_i <= a_i, else nu exp(sum c_i x_i)  (Eq. genzdisc)
 *                  params = c[0..d-1], a[0..d-1]                       (2d)
 *  VEGAS_GENZ_PEAK f = nu prod 1/(c_i^-2 + (x_i - a_i)^2)              (Eq. productpeak)
 *                  params = c[0..d-1], a[0..d-1]                       (2d)
 * For the Genz forms nu makes the integral over [0,1]^d one (sec. 3.1).
 *  VEGAS_USER      f given as device source code (see vegas_init_user); params
 *                  is the caller's array of 0..129 values, handed to f as is. */
enum { VEGAS_GAUSS = 0, VEGAS_BIMODAL = 1, VEGAS_GENZ_DISC = 2, VEGAS_GENZ_PEAK = 3, VEGAS_USER = 4 };

/* Precision of the map and integrand.  Sums, histograms, statistics and the
 * grid are FP64 in both. */
enum { VEGAS_FP64 = 0, VEGAS_FP32_MIXED = 1 };

/* Flags of vegas_iterate. */
#define VEGAS_CHUNK_BEGIN 1u /* first chunk of an iteration: accumulators restart */
#define VEGAS_CHUNK_END 2u   /* last chunk: statistics are computed, iteration recorded */
#define VEGAS_ITER_FULL 3u   /* a whole iteration in one call */
#define VEGAS_NO_COMBINE 4u  /* (with CHUNK_END) record it but keep it out of the combination */
#define VEGAS_REFINE 8u      /* (with CHUNK_END) refine the grid from this iteration's histograms */
#define VEGAS_NO_HIST 16u    /* no histograms this iteration (every chunk of it); not with REFINE */
#define VEGAS_NO_RECORD 32u  /* (with CHUNK_END) keep the estimate as the last iteration's only: no record
                                slot is used and the combination does not see it */

typedef struct {
    int32_t dim;          /* d */
    int32_t n_bins;       /* N, bins per dimension */
    int32_t integrand;    /* VEGAS_GAUSS ... */
    int32_t precision;    /* VEGAS_FP64 or VEGAS_FP32_MIXED */
    uint64_t seed;        /* Philox key */
    double alpha;         /* damping exponent of the refinement (>= 0) */
    const double* params; /* host pointer to n_params values, copied at init */
    int32_t n_params;
    int32_t problem;      /* problem index p in the Philox counter, 0 <= p < 2^24 */
} vegas_desc;

typedef struct {
    double integral;      /* inverse-variance combination of the combined iterations */
    double sigma;         /* its error */
    double chi2_dof;      /* chi^2 per degree of freedom (NaN with one iteration) */
    double last_integral; /* estimate of the last recorded iteration */
    double last_sigma;    /* its error */
    int64_t n_iter;       /* iterations recorded */
    int64_t n_combined;   /* iterations in the combination */
    int64_t n_events;     /* events over all recorded iterations */
    int64_t n_nonfinite;  /* recorded iterations whose estimate or variance was not finite */
} vegas_result_t;

/* Bytes of device workspace a context for *desc needs (no HIP call). */
vegas_status vegas_workspace_size(const vegas_desc* desc, size_t* bytes);

/* Create a context on the current HIP device in the caller's workspace
 * dev_ws (>= vegas_workspace_size bytes, 256-byte aligned; must stay valid
 * until vegas_destroy) and start from the uniform grid E_k = k/N in every
 * dimension.  The iteration index t starts at 0. */
vegas_status vegas_init_grid(vegas_ctx** out, const vegas_desc* desc, void* dev_ws,
                             size_t ws_bytes, vegas_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * vegas_init_grid, but the context's workspace is a static device array of
 * the library (4 MiB, enough for every admissible dim and n_bins; larger
 * needs give VEGAS_EUNSUPPORTED) and the host context is a static one, so the
 * call allocates no device, pinned or host memory.  Built-in integrands only
 * (VEGAS_USER: EUNSUPPORTED).  There is ONE such context per device (devices
 * 0..15): a new call on the device re-initialises it in place and returns the
 * same handle, so the previous handle's state is gone; calls that overlap on
 * one device, or work still running on the array from another stream, race.
 * Every other entry point works on the handle as on any context (copies to
 * the host go straight to the caller's memory, there being no pinned staging
 * buffer); vegas_destroy on it does nothing. */
vegas_status vegas_init_grid_noalloc(vegas_ctx** out, const vegas_desc* desc, vegas_stream_t stream);

/* User integrands: the paper's route for integrands written in C, C++ or GPU
 * code outside the framework (sec. 2.3), here as device source compiled at run
 * time for gfx950 with hipRTC.  `source` is HIP device code that defines
 *
 *   __device__ vegas_real vegas_integrand(const vegas_real* x, int dim, const double* params);
 *
 * returning f(x) at the point x[0..dim-1] in [0,1)^dim, where vegas_real is
 * double in a VEGAS_FP64 context and float in a VEGAS_FP32_MIXED one (the map
 * and f in FP32, the sums and histograms in FP64, as for the built-in
 * integrands); params points to the context's n_params FP64 values in device
 * memory (vegas_desc.params, or those of vegas_set_params_device).  The macro
 * VEGAS_DIM (= dim) is defined before the source, and VEGAS_FP32 in an
 * FP32-mixed context; the HIP device math library is available.  The
 * source may define other __device__ functions and constants; it must not
 * write memory it does not own, and the names vegas_user_* and namespace
 * vegas are reserved.  Everything else of an iteration (points, map,
 * Jacobian, sums, histograms, refinement, combination) is the library's path
 * in the context's precision, so a user integrand equal to a built-in one
 * gives its results up to rounding.  (In an FP32-mixed context the table has
 * no integrand centre to be offset from: x carries the FP32 map's absolute
 * error, at most about 2^-24 (3 W + 2 x) for a bin of width W, and f's
 * error follows from its slope.)
 *
 * vegas_init_user: as vegas_init_grid for desc->integrand == VEGAS_USER (else
 * EINVAL); 0 <= n_params <= 129 (params may be NULL when 0).  Compiles the
 * source for desc->dim and desc->precision (about a second; code objects are
 * kept per (dim, precision, source) for the process) and loads it on the
 * current device.  VEGAS_ECOMPILE if it does not compile,
 * with the compiler's messages in vegas_last_error() (lines of the source are
 * numbered from 1 in file "integrand").  Unsupported on a user context:
 * vegas_adjoint (EUNSUPPORTED) and batches.  vegas_init_grid refuses
 * VEGAS_USER (EINVAL). */
vegas_status vegas_init_user(vegas_ctx** out, const vegas_desc* desc, const char* source, void* dev_ws,
                             size_t ws_bytes, vegas_stream_t stream);

/* Compile `source` for dimension dim (1..64) and precision (VEGAS_FP64 or
 * VEGAS_FP32_MIXED) as vegas_init_user would, without a device: VEGAS_OK or
 * VEGAS_ECOMPILE.  When log is not NULL the compiler's messages (warnings too)
 * are copied there, NUL-terminated and cut to log_bytes. */
vegas_status vegas_user_compile(const char* source, int32_t dim, int32_t precision, char* log, size_t log_bytes);

/* The per-event stage of one integration pass (sec. 2.2: random points,
 * weighted by the grid's Jacobian, feed the integral's sums and the
 * accumulators the refinement later reads), as one call or in chunks.
 * Run n_events events (1 <= n_events <= 2^40) of the current iteration t.
 * Event e draws, for each group j of four dimensions,
 * Philox4x32-10(counter = (e mod 2^32, e div 2^32, t, p*256 + j),
 * key = (seed mod 2^32, seed div 2^32)); dimension i takes word i mod 4 of
 * group i div 4 as y = (k + 1/2)/2^32.  Within one iteration, successive
 * chunks continue the event index (the first chunk starts at e = 0).
 * flags: VEGAS_ITER_FULL for a one-call iteration, or CHUNK_BEGIN, none, ...,
 * CHUNK_END over several calls; REFINE and NO_COMBINE act at CHUNK_END.
 * VEGAS_NO_HIST skips the per-bin histograms (for an iteration on a frozen
 * grid: the estimate is unchanged); it must be given on every chunk of the
 * iteration or on none, never with REFINE, and the iteration's histogram row
 * (vegas_get_iteration) then reads zero and vegas_refine has nothing
 * to refine from.  EINVAL otherwise.
 * At CHUNK_END: I_t = S1/M, var_t = (S2/M - I_t^2)/(M-1) over the M events
 * of the iteration (M >= 2), the iteration is recorded and t advances.  A
 * context records at most 1024 iterations (then ESTATE until
 * vegas_reset_results); VEGAS_NO_RECORD iterations do not count.
 * The call only enqueues kernel launches (no copies, no memsets, no host
 * waits unless timing is enabled), so it can be recorded by stream capture
 * into a HIP graph.  Its host-side bookkeeping (t, the record index) advances
 * when the call is made, i.e. at capture time: a replayed graph re-runs the
 * recorded iterations with their recorded t and record slots. */
vegas_status vegas_iterate(vegas_ctx* ctx, int64_t n_events, uint32_t flags,
                           vegas_stream_t stream);

/* The forward pass of a differentiable estimate, with its gradient (Gaussian
 * integrand only; one whole iteration without histograms:
 * flags must hold VEGAS_ITER_FULL and VEGAS_NO_HIST, and may add
 * VEGAS_NO_COMBINE or VEGAS_NO_RECORD): as vegas_iterate -- the same events,
 * so the same estimate bit for bit -- and the same kernel also sums, as
 * vegas_adjoint does, each event's contribution to the gradient of the
 * estimate with respect to theta = (mu[0..d-1], a) (the derivative of
 * Eq. lepage's estimate with respect to its centre and width) at the
 * current grid and parameters:
 *   dev_G[j] = (1/M) sum_e w_e df/dtheta_j(x_e),  j = 0..d   (device FP64[d+1]).
 * A backward pass then needs no second sweep over the events:
 * vegas_grad_scale(dev_G, gout, grad) gives gout * dev_G. */
vegas_status vegas_iterate_grad(vegas_ctx* ctx, int64_t n_events, uint32_t flags, double* dev_G,
                                vegas_stream_t stream);

/* The whole forward pass of a differentiable estimate in one call (for
 * training loops, where every host call costs): vegas_set_params_device
 * (dev_params, n_params, is_fp32), then vegas_iterate_grad(n_events, flags,
 * dev_G), whose reduction also writes (I_t, sigma_t) of the iteration to
 * dev_out2[2] (device FP64).  dev_params_rest: NULL (all n_params values in
 * dev_params), or the values 1..n_params-1, with only value 0 in dev_params
 * (the Gaussian's a, with mu[0..d-1] in dev_params_rest: separate a and mu
 * arrays need no concatenation); both in the same type.  Gaussian
 * integrand; flags as for vegas_iterate_grad.  Arguments are checked before
 * anything is launched. */
vegas_status vegas_forward_grad(vegas_ctx* ctx, const void* dev_params, const void* dev_params_rest,
                                int32_t n_params, int32_t is_fp32,
                                int64_t n_events, uint32_t flags, double* dev_G, double* dev_out2,
                                vegas_stream_t stream);

/* dev_grad[j] = (*dev_gout) * dev_G[j], j < n (1 <= n <= 65), each rounded
 * once to FP64 or (grad_fp32) FP32; all pointers device memory. */
vegas_status vegas_grad_scale(const double* dev_G, const double* dev_gout, void* dev_grad, int32_t n,
                              int32_t grad_fp32, vegas_stream_t stream);

/* The refinement stage that follows a finished pass (sec. 2.2: once the
 * integration pass is done, the way points are generated is adapted): the
 * grid is refined from the histograms of the last completed iteration
 * (ESTATE if there is none, or if they were already used for a refinement). */
vegas_status vegas_refine(vegas_ctx* ctx, vegas_stream_t stream);

/* The result as the paper reports it, value +- error (Table 1): the
 * inverse-variance combination of the combined iterations.
 * Copy the combined result to *host_out.  Synchronises.  Returns
 * VEGAS_ENONFINITE (with *host_out filled) if any recorded iteration was not
 * finite. */
vegas_status vegas_result(vegas_ctx* ctx, vegas_result_t* host_out, vegas_stream_t stream);

/* Forget recorded iterations and the combination (the grid and t stay). */
vegas_status vegas_reset_results(vegas_ctx* ctx, vegas_stream_t stream);

/* Replace the integrand parameters from device memory (n_params values, FP64
 * if is_fp32 == 0, else FP32; same layout as vegas_desc.params).  One kernel
 * launch stores them, their derived constants and the grid tables. */
vegas_status vegas_set_params_device(vegas_ctx* ctx, const void* dev_params, int32_t n_params,
                                     int32_t is_fp32, vegas_stream_t stream);

/* Copy the context's current integrand parameters (FP64, n_params values) to
 * device memory dev_out. */
vegas_status vegas_get_params_device(vegas_ctx* ctx, double* dev_out, vegas_stream_t stream);

/* Change counters of the context: *grid_version advances whenever the edges
 * change (a refinement, vegas_set_edges, vegas_set_state), *params_version
 * whenever the integrand parameters do (vegas_set_params_device).  A caller
 * that keeps work for later (an adjoint after a forward pass) compares them
 * to know whether the context still holds what it used.  Either pointer may
 * be NULL. */
vegas_status vegas_get_versions(const vegas_ctx* ctx, int64_t* grid_version, int64_t* params_version);

/* Write (I_t, sigma_t) of the last finished iteration (recorded or
 * VEGAS_NO_RECORD) to dev_out[2] (device). */
vegas_status vegas_last_iteration_device(vegas_ctx* ctx, double* dev_out, vegas_stream_t stream);

/* Adjoint of the estimate of iteration `iteration` over events [0, n_events)
 * at fixed samples and the current (frozen) grid and parameters, Gaussian
 * integrand only (the derivative of Eq. lepage's estimate with respect to its
 * centre and width):
 * dev_grad[j] = gout * (1/M) sum_e w_e df/dtheta_j(x_e), theta = (mu[0..d-1], a),
 * with gout = *dev_gout (device FP64 scalar).  dev_grad is device memory of
 * d+1 values, FP64 (grad_fp32 == 0) or FP32 (each rounded once from the FP64
 * sum, for FP32 parameters).  The per-event terms are summed in FP64 in both
 * precisions of the context. */
vegas_status vegas_adjoint(vegas_ctx* ctx, int64_t iteration, int64_t n_events,
                           const double* dev_gout, void* dev_grad, int32_t grad_fp32,
                           vegas_stream_t stream);

/* Per-event record of events [first, first+count) of iteration `iteration`
 * on the current grid, into device FP64 dev_out[count][3d+2]:
 * b[0..d-1], delta[0..d-1], x[0..d-1], w, f  (values as the kernel computes
 * them in its precision, widened to FP64).  For parity checks. */
vegas_status vegas_dump_events(vegas_ctx* ctx, int64_t iteration, int64_t first, int64_t count,
                               double* dev_out, vegas_stream_t stream);

/* Copy grid edges (host FP64 [d][N+1]) out of / into the context.
 * vegas_get_edges synchronises; vegas_set_edges rebuilds the kernel tables. */
vegas_status vegas_get_edges(vegas_ctx* ctx, double* host_edges, vegas_stream_t stream);
vegas_status vegas_set_edges(vegas_ctx* ctx, const double* host_edges, vegas_stream_t stream);

/* Sums (S1, S2) and histograms H[d][N] of the last completed iteration
 * (host FP64; either pointer may be NULL).  Synchronises. */
vegas_status vegas_get_iteration(vegas_ctx* ctx, double* host_sums, double* host_hist,
                                 vegas_stream_t stream);

/* Checkpoint: the state is the grid, the iteration index, the recorded
 * iterations and the combination.  Because points are counter-based, a run
 * resumed from a state continues with the same points as an uninterrupted one.
 * vegas_get_state synchronises. */
vegas_status vegas_state_size(const vegas_ctx* ctx, size_t* bytes);
vegas_status vegas_get_state(vegas_ctx* ctx, void* host_buf, size_t bytes, vegas_stream_t stream);
vegas_status vegas_set_state(vegas_ctx* ctx, const void* host_buf, size_t bytes,
                             vegas_stream_t stream);

/* Current iteration index t (next iteration to run). */
vegas_status vegas_get_iteration_index(const vegas_ctx* ctx, int64_t* t);

/* Launch configuration of the event kernel: the number of blocks
 * (n_blocks = 0 restores the automatic choice).  Results do not depend on it
 * beyond FP64 rounding. */
vegas_status vegas_set_launch(vegas_ctx* ctx, int32_t n_blocks);
/* Histogram replicas per bin in the event kernel's LDS (1, 2, 4, 8 or 16;
 * lane l of a wave adds into replica l mod replicas, so with 16 every lane
 * has its own LDS bank pair); 0 restores the automatic choice (the most that
 * fit without losing a resident block).  Results do not depend on it beyond
 * FP64 rounding. */
vegas_status vegas_set_hist_replicas(vegas_ctx* ctx, int32_t replicas);
/* The automatic choice: blocks (compute units x resident blocks per unit),
 * resident blocks per compute unit, threads per block (1024, 768, 512 or
 * 256, whichever keeps the most waves resident) and histogram replicas in use.
 * Any pointer may be NULL. */
vegas_status vegas_get_launch(const vegas_ctx* ctx, int32_t* auto_blocks, int32_t* blocks_per_cu,
                              int32_t* threads, int32_t* replicas);

/* Kernel timing for benchmarks.  While enabled, each vegas_iterate records
 * HIP events on its stream before its event kernel, between the event kernel
 * and the reduction kernel, and after the reduction (at most 1024 calls are
 * kept).  vegas_timing_read synchronises on the last recorded event, returns
 * the summed event-kernel and reduction-kernel times in milliseconds and the
 * number of calls, and clears the record. */
vegas_status vegas_timing_enable(vegas_ctx* ctx, int32_t enable);
vegas_status vegas_timing_read(vegas_ctx* ctx, double* sample_ms, double* merge_ms, int64_t* count);

/* Time the event kernel alone, for measurement: launch it reps times
 * (1 <= reps <= 10000) back to back on the stream over n_events events of the
 * current iteration t (with histograms unless no_hist), between two HIP events
 * recorded on that stream, and set *ms to the elapsed time divided by reps.
 * The partial rows it writes are scratch: nothing is recorded and t does not
 * advance.  ESTATE while an iteration is open.  Synchronises. */
vegas_status vegas_time_event_kernel(vegas_ctx* ctx, int64_t n_events, int32_t reps, int32_t no_hist,
                                     double* ms, vegas_stream_t stream);

/* Issue-rate probe of the VALU instruction classes the event kernel's
 * throughput bound weighs (measurement only): four kernels, each thread
 * running `iters` steps of eight independent chains of
 *   0: v_mad_u64_u32 + v_bitop3_b32 (+ a register move), as in Philox,
 *   1: v_bitop3_b32,  2: v_fma_f32,  3: v_exp_f32 (a transcendental),
 * launched with 8 waves per SIMD on every compute unit (*host_blocks blocks
 * of 256 threads), each timed with HIP events after one warm-up launch:
 * host_ms[0..3] = milliseconds per launch.  dev_scratch receives one word
 * per thread (4 * 256 * *host_blocks bytes at least; EWORKSPACE otherwise).
 * Synchronises. */
vegas_status vegas_probe_issue_rates(void* dev_scratch, size_t bytes, int32_t iters, double* host_ms,
                                     int32_t* host_blocks, vegas_stream_t stream);

/* Free the host context (the workspace stays the caller's). */
vegas_status vegas_destroy(vegas_ctx* ctx);

/* Thread-local message for the last non-OK status of this thread. */
const char* vegas_last_error(void);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems, each with its own grid, run together.
 * Each problem p uses descs[p] (its problem field is the Philox p) and
 * n_events[p] events per iteration.  One run = n_iter iterations of every
 * problem; iterations 0..n_adapt-1 refine after themselves and are left out
 * of the combination, the remaining ones are combined on the frozen grid.
 * All iterations of all problems are recorded once as a HIP graph at plan
 * time and replayed by vegas_batch_run (one graph launch).  The plan's
 * tuning runs iterations of the batch; it leaves every problem at its start
 * (uniform grid, nothing recorded).  Synchronises.
 * ------------------------------------------------------------------------- */
vegas_status vegas_batch_workspace_size(const vegas_desc* descs, const int64_t* n_events,
                                        int32_t n, size_t* bytes);
vegas_status vegas_batch_plan(vegas_batch** out, const vegas_desc* descs, const int64_t* n_events,
                              int32_t n, void* dev_ws, size_t ws_bytes, int32_t n_iter,
                              int32_t n_adapt, vegas_stream_t stream);
/* Restart every problem from the uniform grid and t = 0, then run. */
vegas_status vegas_batch_run(vegas_batch* batch, vegas_stream_t stream);
/* Iteration k of every problem, eagerly, with the kernels the graph records
 * (for checks and step-by-step use): k = 0 first restarts every problem; the
 * steps run in order 0, 1, ..., n_iter-1 (ESTATE otherwise), and after the
 * last one the state is that of vegas_batch_run.  Iterations k < n_adapt
 * refine after themselves; later ones run without histograms. */
vegas_status vegas_batch_step(vegas_batch* batch, int32_t k, vegas_stream_t stream);
/* Sums (S1, S2) and histograms H[d_p][N_p] of problem p's last iteration
 * (host FP64; either pointer may be NULL; H is zero after an iteration
 * without histograms).  Synchronises. */
vegas_status vegas_batch_get_iteration(vegas_batch* batch, int32_t p, double* host_sums, double* host_hist,
                                       vegas_stream_t stream);
/* Results of every problem (host array of n).  Synchronises. */
vegas_status vegas_batch_results(vegas_batch* batch, vegas_result_t* host_out,
                                 vegas_stream_t stream);
/* Schedule chosen at plan time.  The plan groups problems by dimension
 * bucket (d <= 4, 8, 16, 32, 64), one launch of the persistent event kernel
 * per bucket, and tunes on the batch itself, timing with HIP events: first
 * the tile (events per work item, which also sets events per thread) over
 * 8192 ... 131072, then each bucket's launch shape, threads per block
 * {1024, 512, 256} x histogram replicas {1, 2, 4, 8, 16} (those whose LDS
 * fits), each bucket keeping its fastest.  A bucket's time is that of its
 * launches in one run: n_adapt with histograms and n_iter - n_adapt without.
 * Environment: VEGAS_BATCH_TILE, VEGAS_BATCH_THREADS, VEGAS_BATCH_REPLICAS
 * force a value (that dimension is not tuned); VEGAS_BATCH_TUNE_CACHE names
 * a file where unforced choices are kept per (device, batch) and read back
 * instead of tuning again.
 * vegas_batch_schedule: the tile, the largest bucket launch (blocks), the
 * work items per iteration and the chosen buckets' summed time (ms; 0 when
 * nothing was timed).  Any pointer may be NULL. */
vegas_status vegas_batch_schedule(const vegas_batch* batch, int64_t* tile_events, int32_t* blocks,
                                  int32_t* n_items, double* tuned_ms);
/* Bucket q of the schedule (q < 0: only *n_buckets and *from_cache): its
 * largest dimension, threads per block, histogram replicas, blocks of its
 * launch and timed ms per run (0 if not timed); *from_cache = 1 when the
 * schedule came from the tuning cache.  Any pointer may be NULL. */
vegas_status vegas_batch_bucket(const vegas_batch* batch, int32_t q, int32_t* n_buckets, int32_t* dmax,
                                int32_t* threads, int32_t* replicas, int32_t* blocks, double* tuned_ms,
                                int32_t* from_cache);
/* Edges of problem p (host FP64 [d_p][N_p+1]).  Synchronises. */
vegas_status vegas_batch_get_edges(vegas_batch* batch, int32_t p, double* host_edges,
                                   vegas_stream_t stream);
vegas_status vegas_batch_destroy(vegas_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* VEGAS_H */
