/*
 * vegas.h — C interface of the MI355X Vegas library (libvegas.so).
 *
 * One Vegas iteration (VegasFlow, arXiv:2010.09341, Sec. 1: Monte Carlo
 * importance sampling on adaptive grids after Lepage; Sec. 3.1: a user
 * integrand maps a batch of points of the unit hypercube to one value per
 * point, and a run is a number of iterations; Sec. 3.2: each iteration
 * informs the grid of the next) runs on one gfx950 GPU as hand-written HIP
 * kernels: counter-based Philox4x32-10 uniforms, the per-dimension grid map
 * and Jacobian, the integrand, the FP64 sums of w and w^2, and the
 * per-dimension, per-bin histogram of w^2; a second kernel refines the grid.
 *
 * Conventions for every call:
 *  - The return value is a status (VEGAS_OK or a negative VEGAS_E* code);
 *    results go through caller-owned pointers. vegas_strerror() names codes.
 *  - Arguments are validated before any device work. A call that fails
 *    validation changes nothing (the iteration counter does not advance).
 *  - Host pointers (double*, uint32_t*) are plain host memory owned by the
 *    caller. Device pointers are passed as void* and are named as such.
 *  - A handle is bound to the GPU that was current when it was created and
 *    owns its device memory unless a workspace is bound. A handle is not
 *    thread-safe; distinct handles are independent.
 *  - A device error (a failed launch or copy) poisons the handle: every later
 *    call except vegas_destroy returns VEGAS_EDEVICE.
 *
 * Layouts: grid edges are [dim][n_bins+1] doubles, row d holding the
 * increasing edges e_0 = 0 < e_1 < ... < e_nb = 1 of dimension d; the
 * histogram is [dim][n_bins] doubles, h[d][k] = sum of w^2 over the events of
 * the last iteration whose dimension d fell into bin k.
 *
 * Random stream: dimension d of event n (0 <= n < n_events) in iteration t
 * uses word d%4 of Philox4x32-10 with counter (n mod 2^32, n div 2^32, t, d/4)
 * and key (seed mod 2^32, seed div 2^32). The word r selects bin
 * k = floor(r * n_bins / 2^32) and the point at the centre of the remaining
 * 2^-32 cell of that bin (FP32-eval mode: at the centre of a 2^-23 cell).
 */
#ifndef VEGAS_H
#define VEGAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define VEGAS_OK 0
#define VEGAS_EINVAL (-1)     /* an argument is out of range                  */
#define VEGAS_ENOMEM (-2)     /* device or host allocation failed / too small */
#define VEGAS_EDEVICE (-3)    /* HIP error; the handle is poisoned            */
#define VEGAS_ESTATE (-4)     /* call not valid in the handle's state         */
#define VEGAS_ENONFINITE (-5) /* some weights were not finite (results valid) */
#define VEGAS_EBUSY (-6)      /* serving: no capacity now, try again          */
#define VEGAS_ECOMPILE (-7)   /* run-time integrand source did not compile    */

/* ---- precision modes --------------------------------------------------- */
/* FP64: map, Jacobian, integrand and all sums in binary64.
 * FP32_EVAL: map, integrand and log2 of the Jacobian in binary32; the weight
 * is formed in binary64 range from the binary32 log2-sum; sums, histogram and
 * refinement stay binary64. */
#define VEGAS_FP64 0
#define VEGAS_FP32_EVAL 1

/* ---- integrands (x in the unit hypercube, dimension D) ------------------
 * VEGAS_F_CONST    f = 1.                                         no params
 * VEGAS_F_SUM      f = sum_d x_d (the toy integrand of the Sec. 3.1 code
 *                  example).                                      no params
 * VEGAS_F_GAUSS    f = prod_d exp(-(x_d-c_d)^2/a^2)/(a sqrt(pi)).
 *                  params {a} (all c_d = 0.5) or {a, c_0..c_{D-1}};
 *                  default a = 0.1. 0 < a.
 * VEGAS_F_LO_TOY   D = 4; x = (x1, x2, u, v); s_hat = x1 x2 S, S = sqrt_s^2;
 *                  f = g(x1) g(x2) (1+c^2) BW(s_hat)/s_hat * 2 * 2 pi,
 *                  c = 2u-1, g(x) = x^-1/2 (1-x)^3,
 *                  BW = (m G/pi)/((s_hat-m^2)^2 + m^2 G^2), and f = 0 unless
 *                  sqrt(s_hat) > cut. params {sqrt_s, m, G, cut},
 *                  default {13000, 91.19, 2.5, 20}.
 * VEGAS_F_RAMBO24  D = 16; the 16 coordinates drive RAMBO (4 per particle:
 *                  cos theta = 2u-1, phi = 2 pi u', q0 = -ln(u'' u''')) for
 *                  four massless momenta at sqrt_s; W = (pi/2)^3 s^2 / 12.
 *                  mode 0: f = W prod_{i} 1/s_{i,i+1 mod 4}, f = 0 if any of
 *                  those four s_ij <= cut_frac * s; mode 1: f = W.
 *                  params {sqrt_s, cut_frac, mode}, default {1000, 0.01, 0}.
 * VEGAS_F_BW_FLAT  f = (G/(2 pi)) / ((x_0-m)^2 + G^2/4), flat in the other
 *                  dimensions. params {m, G}, default {0.5, 0.02}. 0 < G. */
#define VEGAS_F_CONST 0
#define VEGAS_F_SUM 1
#define VEGAS_F_GAUSS 2
#define VEGAS_F_LO_TOY 3
#define VEGAS_F_RAMBO24 4
#define VEGAS_F_BW_FLAT 5
#define VEGAS_N_INTEGRANDS 6

/* ---- integrands compiled at run time -------------------------------------
 * Sec. 3.1 has the user supply the integrand as a function of a batch of
 * points. vegas_integrand_compile() turns HIP C++ device source into an
 * integrand id in [VEGAS_F_USER, VEGAS_F_USER + VEGAS_MAX_USER), usable
 * wherever a built-in id is, except by the serving loop. The source defines
 *   __device__ double vegas_user_f64(const double *x, int dim, const double *p);
 *   __device__ float  vegas_user_f32(const float *x, int dim, const float *p);
 * each returning f at the point x (dim coordinates in the unit interval) for
 * the parameters p: those set with vegas_set_params for this id on the
 * handle (at most VEGAS_MAX_USER_PARAMS, the rest zero; rounded to binary32
 * for vegas_user_f32). The library multiplies by the Jacobian. FP64 mode
 * calls vegas_user_f64, FP32_EVAL mode vegas_user_f32. HIP's device math
 * functions (exp, log, sqrt, pow, sin, ..., their f-suffixed binary32 forms)
 * are available without an #include; the source may not #include anything
 * and may not define names that begin with vegas_ other than these two. */
#define VEGAS_F_USER 64
#define VEGAS_MAX_USER 64
#define VEGAS_MAX_USER_PARAMS 32

/* ---- limits ------------------------------------------------------------ */
#define VEGAS_MAX_DIM 32
#define VEGAS_MAX_BINS 512
/* dim * n_bins may not exceed this: each workgroup of the iteration kernel
 * keeps up to 16 interleaved copies of the w^2 histogram, 8 bytes per
 * (dimension, bin) each, in at most 64 KiB of LDS; larger grids get fewer
 * copies, down to one copy of 8192 cells (64 KiB). */
#define VEGAS_MAX_CELLS 8192
#define VEGAS_MAX_PARAMS (1 + VEGAS_MAX_DIM)
/* vegas_run may queue at most this many iterations per call. */
#define VEGAS_MAX_RUN_ITER 1024
/* A handle keeps at most this many per-iteration results (behind
 * vegas_result and in a checkpoint record); vegas_iterate / vegas_run return
 * VEGAS_ESTATE once it is full, until vegas_reset. */
#define VEGAS_MAX_HISTORY (1 << 24)
/* Largest refinement exponent: with 0 <= alpha <= 64 every compressed
 * weight of a non-empty smoothed bin stays a positive binary64 number
 * ((1-p)/(-ln p) >= 1/745 for every positive binary64 p < 1). */
#define VEGAS_MAX_ALPHA 64.0

typedef struct vegas_ctx *vegas_h;

/* Create a handle with the uniform grid e[d][i] = i/n_bins and iteration
 * counter t = 0, on the current GPU, in FP64 mode, with default integrand
 * parameters. The grid is Vegas's per-dimension adaptive grid of Sec. 1 (the
 * paper's VegasFlow(n_dim, n_events) constructor of the Sec. 3.1 listing
 * takes the dimension; the bin count is Vegas's). 1 <= dim <= VEGAS_MAX_DIM,
 * 2 <= n_bins <= VEGAS_MAX_BINS, dim * n_bins <= VEGAS_MAX_CELLS. *out
 * receives the handle (owned by the caller until vegas_destroy). Errors:
 * VEGAS_EINVAL (shape, NULL out), VEGAS_ENOMEM, VEGAS_EDEVICE; *out is then
 * NULL. */
int vegas_create(int dim, int n_bins, vegas_h *out);

/* Release the handle and the device memory it owns. NULL is accepted. */
int vegas_destroy(vegas_h h);

/* Back to the state of vegas_create (uniform grid, t = 0, no history),
 * keeping parameters, precision, stream and workspace. The grid is rewritten
 * by work queued on the handle's stream and not waited for; a device error
 * shows at the next call that synchronises. */
int vegas_reset(vegas_h h);

/* Set the parameters used when integrand_id is evaluated (see the integrand
 * list above). n_params = 0 restores the defaults. */
int vegas_set_params(vegas_h h, int integrand_id, const double *params, int n_params);

/* VEGAS_FP64 or VEGAS_FP32_EVAL; applies from the next iteration. */
int vegas_set_precision(vegas_h h, int prec);

/* Launch all work on this hipStream_t (e.g. torch.cuda.current_stream()).
 * NULL returns to the handle's own stream. The stream must outlive its use. */
int vegas_bind_stream(vegas_h h, void *hip_stream);

/* Device bytes a handle of this shape needs when a workspace is bound. */
int vegas_workspace_bytes(int dim, int n_bins, size_t *bytes);

/* Use caller-owned device memory (at least vegas_workspace_bytes bytes,
 * 256-byte aligned) instead of the handle's own. The grid, the iteration
 * counter and the history are preserved (copied into the new workspace).
 * The memory must stay valid until the handle is destroyed or another
 * workspace is bound. dev_ptr = NULL returns to handle-owned memory. */
int vegas_bind_workspace(vegas_h h, void *dev_ptr, size_t bytes);

/* One iteration (steps draw, map, evaluate, accumulate, histogram) of
 * n_events events (n_events >= 2) with Philox key `seed`, at the handle's
 * iteration counter t; then t += 1. This is one Vegas iteration of Sec. 1
 * (importance sampling through the adaptive grid) on the integrand of
 * Sec. 3.1 (a function of a batch of points of the unit hypercube); the
 * w^2 histogram it leaves is what informs the next grid (Sec. 3.2). Writes the iteration's estimate *I and
 * its standard deviation *sigma = sqrt((S2/N - I^2)/(N-1)). Non-finite
 * weights are counted, contribute zero, and make the call return
 * VEGAS_ENONFINITE with *I and *sigma still written. Synchronous. */
int vegas_iterate(vegas_h h, int integrand_id, int64_t n_events, uint64_t seed, double *I,
                  double *sigma);

/* Refine the grid from the histogram of the last iteration (Sec. 3.2: each
 * iteration informs the grid of the next; the steps are Vegas's, Sec. 1): smooth with the
 * (1,1,1)/3 kernel ((1,1)/2 at the ends), normalise to p_i, compress to
 * r_i = ((1-p_i)/(-ln p_i))^alpha, and place new edges so that every new bin
 * holds an equal share of r (linear inside old bins).
 * 0 <= alpha <= VEGAS_MAX_ALPHA.
 * VEGAS_ESTATE unless an iteration ran since the last refine. Synchronous. */
int vegas_refine(vegas_h h, double alpha);

/* A whole run (the paper's run_integration(n_iter) of the Sec. 3.1
 * listing): n_iter iterations from the
 * current state, refining with alpha after every iteration but the last,
 * queued back to back on the GPU with one synchronisation at the end.
 * I_t[i], sigma_t[i] (host, n_iter entries each, may be NULL) receive the
 * per-iteration results. 1 <= n_iter <= VEGAS_MAX_RUN_ITER. */
int vegas_run(vegas_h h, int integrand_id, int64_t n_events, uint64_t seed, int n_iter,
              double alpha, double *I_t, double *sigma_t);

/* Cumulative result over all iterations since create/reset: inverse-variance
 * mean, its sigma, and chi^2 per degree of freedom (0 for one iteration).
 * VEGAS_ESTATE before the first iteration. */
int vegas_result(vegas_h h, double *I, double *sigma, double *chi2_dof);

/* Copy the grid out / in (n = dim*(n_bins+1) doubles). vegas_set_grid checks
 * e_0 = 0, e_nb = 1 and strictly increasing rows. */
int vegas_get_grid(vegas_h h, double *edges, size_t n);
int vegas_set_grid(vegas_h h, const double *edges, size_t n);

/* Copy the histogram of the last iteration out / in (n = dim*n_bins). Setting
 * it (all entries finite and >= 0) makes a following vegas_refine valid. */
int vegas_get_hist(vegas_h h, double *hist, size_t n);
int vegas_set_hist(vegas_h h, const double *hist, size_t n);

/* Iteration counter t (the third Philox counter word of the next iteration). */
int vegas_get_iteration(vegas_h h, uint32_t *t);
int vegas_set_iteration(vegas_h h, uint32_t t);

/* Checkpoint and resume. The state of a handle — grid, last histogram,
 * iteration counter, the per-iteration results behind vegas_result,
 * parameters of the built-in integrands, precision and events limit — is a
 * flat host byte record of vegas_state_bytes bytes (run-time integrand ids
 * belong to the process; their parameters are not in it). vegas_save writes
 * it into buf (host, caller-owned); vegas_load restores it into a handle of
 * the same dim and n_bins (VEGAS_EINVAL for any other record, with the
 * handle unchanged).
 * Because every random number is a function of (seed, event, iteration,
 * dimension), a run resumed from a record continues exactly as the
 * uninterrupted run would have. */
int vegas_state_bytes(vegas_h h, size_t *bytes);
int vegas_save(vegas_h h, void *buf, size_t bytes);
int vegas_load(vegas_h h, const void *buf, size_t bytes);

/* Number of non-finite weights in the last iteration. */
int vegas_nonfinite(vegas_h h, int64_t *count);

/* Test hook: the weights w of events first .. first+count-1 at the current
 * grid and iteration counter, computed by the same device code as
 * vegas_iterate, into host memory w_out (count doubles). 0 <= count <= 2^26.
 * Does not change the state. */
int vegas_dump_weights(vegas_h h, int integrand_id, uint64_t seed, uint64_t first, int64_t count,
                       double *w_out);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * iteration like vegas_iterate, without a handle and without any
 * allocation. The grid is the caller's: edges_dev, [dim][n_bins+1] binary64
 * in device memory (read only). The outputs go to the caller's device
 * memory: result_dev receives 4 binary64 values (I, sigma, the count of
 * non-finite weights, t), hist_dev (may be NULL) the iteration's w^2
 * histogram, [dim][n_bins] binary64. t is the iteration counter of the
 * random stream; integrand_id is a built-in VEGAS_F_* with its parameters
 * (host, copied). The work is enqueued on `stream` (a hipStream_t; NULL is
 * the null stream) and not waited for. No refinement (vegas_refine's
 * arithmetic needs a handle). Every buffer between the kernels (grid
 * records, workgroup partials, histogram copies, the counter) lives in one
 * fixed device array of the library, VEGAS_NOALLOC_SCRATCH_BYTES per GPU,
 * held until the process ends; each call clears what must start at zero.
 * Calls that overlap on one GPU (other streams, other threads) race on that
 * array and must be serialised by the caller. VEGAS_EINVAL for a shape
 * beyond VEGAS_MAX_CELLS (the array's limit), an unknown precision, a
 * run-time integrand id, parameters the integrand does not take, n_events
 * < 2 or a NULL edges_dev/result_dev; VEGAS_EDEVICE on a HIP error. */
#define VEGAS_NOALLOC_SCRATCH_BYTES (1 << 20)
int vegas_iterate_noalloc(int dim, int n_bins, int prec, int integrand_id, const double *params,
                          int n_params, const double *edges_dev, int64_t n_events, uint64_t seed,
                          uint32_t t, double *hist_dev, double *result_dev, void *stream);

/* Launch shape of the iteration kernel: at most max_blocks workgroups of
 * `threads` threads (a multiple of 64 up to 1024). 0 selects the default: of
 * the powers of two from 64 up to the largest the kernel was built for
 * (1024, or 256 for the kernels that need more than 128 registers per
 * thread), the one that keeps the most waves resident (the largest among
 * equals), and enough workgroups to fill the GPU.
 * A thread count above what the integrand's kernel was built for makes the
 * next iteration return VEGAS_EINVAL. */
int vegas_set_launch(vegas_h h, int max_blocks, int threads);

/* The paper's events_limit (Sec. 3.1, and Fig. 2's batch-size experiment):
 * at most `limit` events per launch of the iteration kernel; an iteration of
 * n_events then runs as ceil(n_events/limit) launches on the handle's
 * stream, each adding to the partial sums of the ones before in a fixed
 * order. 0 (the default) runs every iteration as one launch. Random numbers
 * are drawn on the device, so no batch crosses PCIe. limit >= 0. */
int vegas_set_events_limit(vegas_h h, int64_t limit);

/* vegas_run captures its sequence of iterations in a hipGraph the first time
 * a configuration (integrand, parameters, precision, events, seed, iteration
 * count, alpha, launch shape, events limit, stream) is run and replays it
 * after that;
 * enable = 0 launches the kernels one by one instead. Default on. While
 * kernel timing (vegas_timing) is enabled, kernels are launched one by one so
 * that HIP events can bracket each iteration kernel. */
int vegas_set_graph(vegas_h h, int enable);

/* Kernel timing: enable != 0 records HIP events around every launch of the
 * iteration kernel on the handle's stream; *iterate_ms and *n_launches (may
 * be NULL) receive the summed duration and the launch count since the last
 * call with enable changed or since the counters were read with reset != 0. */
int vegas_timing(vegas_h h, int enable, int reset, double *iterate_ms, int64_t *n_launches);

/* Name of a status code. */
const char *vegas_strerror(int status);

/* Compile an integrand (see "integrands compiled at run time" above) for the
 * gfx950 GPU with hiprtc. source: NUL-terminated HIP C++.
 * dim = 0: kernels that take any dimension 1..VEGAS_MAX_DIM at run time;
 * 1 <= dim <= VEGAS_MAX_DIM: kernels for exactly that dimension (faster; the
 * id then serves only handles of that dimension).
 * *integrand_id receives the new id. On VEGAS_ECOMPILE the compiler's log
 * goes to log (at most log_bytes bytes including the NUL; log may be NULL).
 * VEGAS_ENOMEM when VEGAS_MAX_USER ids exist. Needs no GPU: the code object
 * is loaded onto a GPU the first time the id runs there. Ids live until the
 * process ends. Thread-safe. */
int vegas_integrand_compile(const char *source, int dim, int *integrand_id, char *log,
                            size_t log_bytes);

/* ---- serving: many integrals on one GPU -------------------------------- */
/* A server keeps every admitted integral's grid, histogram and partial sums
 * resident on the device, and runs their (integral, iteration, event-chunk)
 * work concurrently: a request that arrives while others run is admitted as
 * soon as a slot and device memory are free, and its chunks share the GPU
 * with the others'. Server calls are thread-safe. */
typedef struct vegas_srv *vegas_server;

typedef struct {
  int dim;            /* 1..VEGAS_MAX_DIM                                   */
  int n_bins;         /* 2..VEGAS_MAX_BINS, dim*n_bins <= VEGAS_MAX_CELLS   */
  int integrand_id;   /* VEGAS_F_*                                          */
  int n_params;       /* 0..VEGAS_MAX_PARAMS                                */
  const double *params; /* host; copied at submit                          */
  int64_t n_events;   /* events per iteration, >= 2                         */
  int n_iter;         /* iterations, 1..VEGAS_MAX_RUN_ITER                  */
  double alpha;       /* refinement exponent, >= 0                          */
  uint64_t seed;      /* Philox key                                         */
  int prec;           /* VEGAS_FP64 or VEGAS_FP32_EVAL                      */
} vegas_request;

/* Create a server on the current GPU. mem_budget_bytes bounds the device
 * memory of admitted integrals; max_slots bounds how many run at once
 * (1..4096); chunk_events is the work-item size in events (0 = default). */
int vegas_server_create(size_t mem_budget_bytes, int max_slots, int64_t chunk_events,
                        vegas_server *out);

/* Queue one integral (non-blocking); *ticket identifies it. Requests larger
 * than the whole budget are rejected with VEGAS_ENOMEM. */
int vegas_server_submit(vegas_server s, const vegas_request *r, uint64_t *ticket);

/* Wait for a ticket: cumulative *I, *sigma (inverse-variance over its
 * iterations), *chi2_dof, and *latency_s from submit to completion (any
 * pointer may be NULL). timeout_s < 0 waits forever; VEGAS_EBUSY on timeout. */
int vegas_server_wait(vegas_server s, uint64_t ticket, double timeout_s, double *I,
                      double *sigma, double *chi2_dof, double *latency_s);

/* Per-iteration results of a finished ticket (n_iter entries each). */
int vegas_server_iterations(vegas_server s, uint64_t ticket, double *I_t, double *sigma_t);

/* Forget a finished ticket: the server frees its record (results, per-
 * iteration estimates), after which wait and iterations on it return
 * VEGAS_EINVAL (a wait on it in another thread returns VEGAS_EINVAL too, if
 * the release comes first). A server keeps every ticket's record until it is released or
 * the server is destroyed, so a long-running server releases what it has
 * read. VEGAS_EBUSY while the ticket has not finished; VEGAS_EINVAL for an
 * unknown ticket. */
int vegas_server_release(vegas_server s, uint64_t ticket);

/* Counters: requests completed, events processed, device work items run,
 * peak concurrent integrals. Any pointer may be NULL. */
int vegas_server_stats(vegas_server s, int64_t *completed, int64_t *events, int64_t *work_items,
                       int64_t *peak_active);

/* The server advances every admitted integral by one iteration per tick.
 * A tick whose work equals the previous tick's (the same integrals, none
 * newly admitted, none at its last iteration) reuses the inputs already on
 * the device. With enable != 0, once 8 such ticks have followed each other
 * the tick's launches are captured in a hipGraph and replayed until the work
 * changes. Default 0: a tick is a few launches and the work changes every
 * few ticks, so capturing costs more than it saves. */
int vegas_server_set_graph(vegas_server s, int enable);

/* Ticks run so far and how many of them were hipGraph replays (either
 * pointer may be NULL). */
int vegas_server_ticks(vegas_server s, int64_t *ticks, int64_t *graph_ticks);

/* A lane (see vegas_server_set_lanes) runs the ticks up to the next
 * completion of one of its integrals as one chain: enqueued back to back and
 * collected once the lane's stream has drained, so that an integral's
 * iterations follow each other on the device without a host round trip
 * between them (each iteration still refines the grid the next one samples:
 * Sec. 3.2, every iteration informs the next). max_ticks bounds a chain
 * (1..32, default 32; 1 returns to the host after every tick); a chain also
 * carries at most about 3e8 events, and graph replay (above) runs one tick
 * per chain. VEGAS_EINVAL outside 1..32. Results do not depend on it. */
int vegas_server_set_chain(vegas_server s, int max_ticks);

/* Chains run so far (*chains; may be NULL). */
int vegas_server_chains(vegas_server s, int64_t *chains);

/* The server runs its chains on `lanes` HIP streams (1..8, default 4): an
 * admitted integral goes to an idle lane if there is one, where it starts at
 * once and its work overlaps the other lanes', else to the lane holding the
 * fewest integrals, joining that lane's next chain. With one lane, an
 * arriving request waits for the running chain. VEGAS_ESTATE while requests
 * are admitted or queued; VEGAS_EINVAL outside 1..8. Results do not depend
 * on it (an integral's estimate is the same in any lane and any mix). */
int vegas_server_set_lanes(vegas_server s, int lanes);

/* Drain all queued work, then release the server. No other call on the
 * server may be in progress (a wait in another thread included) or follow. */
int vegas_server_destroy(vegas_server s);

#ifdef __cplusplus
}
#endif

#endif /* VEGAS_H */
