/*
 * ai.h -- C ABI of libai.so: ensemble Dormand-Prince 5(4) integration of
 * atom + trapped-ion trajectories on an AMD Instinct MI355X (gfx950).
 *
 * Method (arXiv 2509.12381):
 *   - state y = (x_ion, v_ion, x_atom, v_atom), 12 components (Sec. 2.1,
 *     definition of y);
 *   - y' = f(t, y) with the atom-ion force of V(r) = -Cn/r^n + Cm/r^m and the
 *     Paul-trap term -(a_k + 2 q_k cos(omega_rf t)) omega_rf^2/4 x_k on the ion
 *     (Sec. 2.1, equation for f; general n, m in Sec. 4.1);
 *   - the ode45 algorithm (Fig. 2: Dormand-Prince 5(4) pair, initial step,
 *     weighted infinity-norm error test against RelTol/AbsTol, step-size
 *     control), one call integrating many independent trajectories, each from
 *     t0 to its own exit (Sec. 3.2 and 3.3: the arrayfun launch over arrays
 *     of initial conditions, outputs the end time, the final state and scalar
 *     observables);
 *   - the observables of Sec. 4.1 (angle, bounces, lifetime, position,
 *     transfer, dist, nsteps, KE) accumulated on the fly.
 *
 * Units are atomic units throughout.  All entry points are thread-safe; calls
 * on different streams are independent.
 */
#ifndef AI_H
#define AI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AI_NSTATE 12 /* state components per trajectory */
#define AI_NOBS 13   /* observable planes per trajectory */

/* Constants of the atom + trapped-ion system (Sec. 2.1 Hamiltonian; Sec. 4.1
 * inputs).  Exit rule: a trajectory ends once the atom-ion distance exceeds
 * r_exit after its first closest approach (a sign change of
 * (x_ion - x_atom) . (v_ion - v_atom) from negative to non-negative between
 * accepted steps, or a non-negative value at t0); r_exit = 0 disables it. */
typedef struct ai_params {
  double m_ion, m_atom;  /* masses (electron masses), > 0 */
  int32_t n, m;          /* exponents of V(r) = -Cn/r^n + Cm/r^m (Sec. 4.1), 1 <= n < m <= 16;
                            n=4, m=8 in every kernel, others in the plain double kernel */
  double Cn, Cm;         /* coefficients (C4 and C8 for n=4, m=8) */
  double a[3], q[3];     /* Paul-trap parameters per axis, paper form */
  double omega_rf;       /* trap radio frequency (inverse atomic time) */
  double r_exit;         /* exit radius after closest approach, >= 0; 0 = off */
  double r_bounce;       /* a closest approach inside this radius is a bounce */
  int64_t max_steps;     /* cap on accepted steps per trajectory, >= 1 (paper: 10^6) */
  double hmax;           /* step-size cap; 0 selects 0.1 (tmax - t0) */
} ai_params;

/* Observable planes of obs (index c of obs[c * ld + i]).  Counts are stored
 * as exact doubles. */
enum ai_obs {
  AI_OBS_TEND = 0,     /* end time of the trajectory */
  AI_OBS_STATUS = 1,   /* enum ai_status */
  AI_OBS_NSTEPS = 2,   /* accepted steps */
  AI_OBS_NFAILED = 3,  /* rejected attempts */
  AI_OBS_BOUNCES = 4,  /* closest approaches inside r_bounce */
  AI_OBS_LIFETIME = 5, /* time from first to last bounce if bounces >= 2, else 0 */
  AI_OBS_ANGLE = 6,    /* angle between the atom's initial and final velocity */
  AI_OBS_TRANSFER = 7, /* m_atom |v_atom(end) - v_atom(t0)| */
  AI_OBS_POSITION = 8, /* |x_ion| at the first bounce, 0 if none */
  AI_OBS_DIST = 9,     /* final atom-ion distance */
  AI_OBS_KE = 10,      /* final ion kinetic energy */
  AI_OBS_RMIN = 11,    /* smallest atom-ion distance seen at t0 and accepted steps */
  AI_OBS_HNEXT = 12    /* step size the controller proposes next */
};

/* Per-trajectory end status (never an error return). */
enum ai_status {
  AI_ST_ESCAPED = 1,   /* r > r_exit after closest approach */
  AI_ST_TMAX = 2,      /* reached tmax exactly */
  AI_ST_MAXSTEPS = 3,  /* max_steps accepted steps */
  AI_ST_HMIN = 4,      /* rejected at the smallest step 16 eps(t) */
  AI_ST_NONFINITE = 5  /* non-finite initial state, force or error estimate */
};

enum ai_kernel {
  AI_KERNEL_PLAIN = 0,     /* one trajectory per lane, grid covers n */
  AI_KERNEL_PERSISTENT = 1, /* resident waves refill exited lanes from a device queue */
  /* flag, OR-ed into either kernel: hand out trajectories by decreasing
   * predicted duration (the time at which the atom, on a straight line, is
   * r_exit away from the ion on its secular trap motion; capped at
   * tmax - t0; uniform when r_exit = 0), computed and sorted on the device.
   * Changes only which lane integrates which trajectory, never a result.
   * Takes 16 n bytes plus sort scratch from the stream-ordered allocator for
   * the call; ignored for n >= 2^32. */
  AI_SCHEDULE_LONGEST_FIRST = 16,
  /* flag, plain kernel only (AI_EUNSUPPORTED with the persistent kernel): the
   * precision variant.  Stage increments, forces and the error estimate's
   * sums run in single precision; the state accumulation, t, h, the trap
   * phase and the error norm stay double.  Stage positions are the double
   * state plus single-precision increments, and the ion-atom separation is
   * formed in double before narrowing.  Results differ from the double
   * kernels by the single-precision rounding of the stage arithmetic (each
   * observable's difference is stated with the tests). */
  AI_FP32_STAGES = 32,
  /* flag, any kernel and ai_integrate_batch[_async]: record HIP events on the
   * call's stream right before and after its integration kernel (schedule,
   * sort and observable kernels excluded); ai_kernel_time() returns that
   * duration once the stream has reached it.  The events belong to the calling
   * thread, which keeps its last 64 such calls. */
  AI_TIME_KERNEL = 64
};

/* Persistent kernel only, OR-ed into the kernel argument: a wave draws new
 * trajectories once at least k (1..64) of its lanes are idle, or all are;
 * k = 0 selects 1.  Groups of lanes started together tend to finish together.
 * With the longest-first schedule, waves also take a scheduling priority from
 * the predicted duration of the longest trajectory they hold. */
#define AI_REFILL_MIN(k) ((int32_t)(k) << 8)

/* With AI_SCHEDULE_LONGEST_FIRST (single calls with either kernel, and
 * batches), OR-ed into the kernel argument: how many of the leading positions
 * of the longest-first order (the trajectories predicted to take longest) run
 * four lanes each, one spatial axis per lane, so that they end sooner (the
 * launch ends with them): code 0 = 256 (the default), 1 = none, 2 = 1024,
 * 3 = 4096.  Changes which lanes integrate a trajectory, never a result.
 * Ignored with AI_FP32_STAGES. */
#define AI_WIDE(code) ((int32_t)(code) << 16)

enum ai_rc {
  AI_OK = 0,
  AI_WRTOL = 1,          /* warning: rtol below 100 eps was raised to 100 eps (as ode45 does) */
  AI_EINVAL = -1,        /* invalid argument; nothing was launched */
  AI_EHIP = -2,          /* HIP runtime error; text in ai_last_error() */
  AI_ENOMEM = -3,        /* device allocation failed */
  AI_EUNSUPPORTED = -4,  /* valid request this build does not run (see ai_params.n, m) */
  AI_EAGAIN = -5         /* ai_server_wait: the request has not finished within the timeout */
};

/* Integrate trajectories i = 0 .. n-1 and wait for the result.
 *
 * y0, final_state: device pointers to 12 planes, element (i, c) at ptr[c * ld + i];
 *   y0 is read only; final_state may equal y0 (in place) but must not overlap
 *   it otherwise.  final_state receives the state at the end time.
 * obs: device pointer to AI_NOBS planes with the same leading dimension ld;
 *   must not overlap y0 or final_state.
 * n >= 0 trajectories, ld >= n; n = 0 returns AI_OK without launching.
 * t0 < tmax, both finite: every trajectory starts at t0 and stops at tmax at
 *   the latest.  rtol > 0 and atol > 0 are ode45's RelTol and scalar AbsTol.
 * kernel: AI_KERNEL_PLAIN or AI_KERNEL_PERSISTENT, optionally OR
 *   AI_SCHEDULE_LONGEST_FIRST and (persistent) AI_REFILL_MIN(k); every
 *   combination gives bitwise-identical per-trajectory results.  Or
 *   AI_KERNEL_PLAIN | AI_FP32_STAGES (schedule optional): the precision
 *   variant, deterministic but not bitwise equal to the double kernels.
 * The caller owns every buffer.  Returns AI_OK, AI_WRTOL or a negative
 * ai_rc; a failing call leaves the outputs unspecified. */
int ai_integrate(const ai_params *p, const double *y0, int64_t n, int64_t ld, double t0,
                 double tmax, double rtol, double atol, double *final_state, double *obs,
                 int32_t kernel);

/* As ai_integrate, but enqueued on `stream` (a hipStream_t; NULL is the null
 * stream) and returning at once.  Buffers must stay allocated until the work
 * on the stream has completed; the library keeps no pointer after that.
 * The persistent kernel takes an 8-byte queue counter from the stream-ordered
 * allocator for the duration of the call.  The plain kernel without
 * AI_SCHEDULE_LONGEST_FIRST enqueues its one kernel and nothing else (no
 * allocation, no memset), so that call may be captured in a HIP graph and
 * replayed; the schedule and the persistent kernel allocate stream-ordered
 * memory here, so for capture use ai_integrate_static_async, whose scheduled
 * plain call enqueues kernels only. */
int ai_integrate_async(const ai_params *p, const double *y0, int64_t n, int64_t ld, double t0,
                       double tmax, double rtol, double atol, double *final_state, double *obs,
                       int32_t kernel, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): as
 * ai_integrate_async, but the schedule's workspace and the persistent kernel's
 * queue counter come from a scratch array of AI_STATIC_SCRATCH_BYTES that the
 * library holds in each device's memory until the process ends, so the call
 * allocates nothing.  A scheduled call takes at most AI_STATIC_MAX_SCHEDULED
 * trajectories (AI_EINVAL beyond; unscheduled calls take any n), and
 * AI_TIME_KERNEL is refused (AI_EINVAL).  Every call on a device shares that
 * device's scratch and it keeps the last call's contents (the queue counter
 * is cleared by a kernel at the start of each persistent call), so calls
 * whose work overlaps on one device, from any stream or thread, race: the
 * caller orders them.  Its plain kernel calls, scheduled or not, enqueue
 * kernels only (the schedule's counting sort writes every word it reads), so
 * they may be captured in a HIP graph and replayed. */
#define AI_STATIC_SCRATCH_BYTES (32ull << 20)
#define AI_STATIC_MAX_SCHEDULED (1 << 20)
int ai_integrate_static_async(const ai_params *p, const double *y0, int64_t n, int64_t ld,
                              double t0, double tmax, double rtol, double atol,
                              double *final_state, double *obs, int32_t kernel, void *stream);

/* Choose the fastest kernel configuration for an ensemble by running it: the
 * ensemble is integrated with each of AI_KERNEL_PLAIN,
 * AI_KERNEL_PLAIN | AI_SCHEDULE_LONGEST_FIRST | AI_WIDE(c) for c = 0, 1, 2
 * (256, none or 1024 four-lane trajectories) and AI_KERNEL_PERSISTENT |
 * AI_SCHEDULE_LONGEST_FIRST | AI_REFILL_MIN(k) for k = 1, 16, 64 (plain only
 * for exponents other than n=4, m=8) in two rounds; a round enqueues the
 * candidates back-to-back on the null stream, each as an untimed run followed
 * by a run between HIP events, so each is timed as in a sequence of its own
 * calls.  The best single time wins.  Every configuration gives bitwise the same results, so the outputs
 * hold the ensemble's results afterwards, as after ai_integrate.  Arguments as
 * for ai_integrate, except that final_state must not be y0 (the ensemble runs
 * several times).  *best_kernel (host) receives the fastest configuration, to
 * pass as `kernel` to later calls on similar ensembles, *best_ms (host) its
 * time.  Blocks until done; returns AI_OK, AI_WRTOL or a negative ai_rc. */
int ai_tune(const ai_params *p, const double *y0, int64_t n, int64_t ld, double t0,
            double tmax, double rtol, double atol, double *final_state, double *obs,
            int32_t *best_kernel, float *best_ms);

/* One ensemble of a batched call: its system, buffers, span and tolerances,
 * each with the meaning and constraints it has in ai_integrate. */
typedef struct ai_batch_item {
  ai_params params;
  const double *y0;           /* device, 12 planes of ld doubles */
  int64_t n, ld;
  double t0, tmax, rtol, atol;
  double *final_state;        /* device, 12 planes (may equal y0) */
  double *obs;                /* device, AI_NOBS planes */
} ai_batch_item;

/* Integrate `count` ensembles of possibly different systems, sizes, spans and
 * tolerances in one launch of the plain kernel: the trajectories of all items
 * form one index space (and, with AI_SCHEDULE_LONGEST_FIRST, are handed out by
 * decreasing predicted cost across items: the exit rule evaluated on samples
 * of the trap's exact linear motion with the atom in straight flight, times an
 * attempt rate for the item's trap frequency, q and rtol).  This is the batched form of
 * the paper's ode45gpu call (Sec. 3.3) for uneven ensembles (Sec. 4.2 sweeps
 * collision energy and trap parameters).
 *
 * items: host array of count >= 0 entries (read during the call only).
 * kernel: AI_KERNEL_PLAIN, optionally OR AI_SCHEDULE_LONGEST_FIRST; other
 *   flags give AI_EUNSUPPORTED.
 * Every item is validated as ai_integrate validates its arguments (and must
 * have n=4, m=8, else AI_EUNSUPPORTED); an invalid
 * item fails the whole call with AI_EINVAL before anything is launched (the
 * error text names the item).  Items with n = 0 are skipped.  Output buffers
 * of different items must not overlap.  Each trajectory's result is bitwise
 * the one ai_integrate gives for its item alone.  The call takes the items'
 * launch table (about 350 bytes per item) and, with the schedule, 16 bytes
 * per trajectory plus sort scratch from the stream-ordered allocator.
 * Returns AI_OK, AI_WRTOL if any item's rtol was raised, or a negative ai_rc. */
int ai_integrate_batch_async(const ai_batch_item *items, int32_t count, int32_t kernel,
                             void *stream);

/* As ai_integrate_batch_async on the null stream, waiting for the result. */
int ai_integrate_batch(const ai_batch_item *items, int32_t count, int32_t kernel);

/* Choose the fastest configuration for a batch by running it, as ai_tune does
 * for one ensemble: the batch is integrated with AI_KERNEL_PLAIN (index order)
 * and with AI_KERNEL_PLAIN | AI_SCHEDULE_LONGEST_FIRST | AI_WIDE(c) for c = 1,
 * 0, 2 (none, 256 or 1024 of the longest predicted trajectories four lanes
 * each), in two rounds, each candidate timed right after an untimed run of
 * itself.  Every configuration gives bitwise the same results, so the outputs
 * hold the batch's results afterwards.  Items as for ai_integrate_batch, but no
 * item may integrate in place.  *best_kernel and *best_ms (host) receive the
 * fastest configuration and its time.  Blocks until done; returns AI_OK,
 * AI_WRTOL or a negative ai_rc. */
int ai_tune_batch(const ai_batch_item *items, int32_t count, int32_t *best_kernel,
                  float *best_ms);

/* A batch prepared once and launched many times, for callers that capture
 * the launch in a HIP graph or repeat it on the same buffers (Sec. 4.2 sweeps
 * collision energy and trap parameters over the same ensembles).
 *
 * ai_batch_plan_create validates `items` as ai_integrate_batch does (kernel
 * AI_KERNEL_PLAIN, optionally | AI_SCHEDULE_LONGEST_FIRST), copies the
 * launch table to device memory it allocates and, with the schedule, orders
 * the trajectories by the cost predicted from the initial states present now.
 * Blocks until done.  The plan keeps the items' device pointers (y0,
 * final_state, obs), their sizes, spans, tolerances and systems; the caller
 * keeps those buffers allocated while the plan is used.  Returns AI_OK or
 * AI_WRTOL and *out, or a negative ai_rc and *out = NULL.
 *
 * ai_batch_plan_launch enqueues the batch's integration and observables
 * kernels on `stream` (hipStream_t; NULL = null stream) and nothing else: no
 * allocation, no copy, no memset, so it may be captured in a HIP graph and
 * replayed.  Each launch integrates the initial states that y0 holds when it
 * runs; the results are bitwise those of ai_integrate_batch on them (the
 * order computed at creation affects only the time, never the results).
 * Launches of one plan on different streams must not overlap (they write the
 * same outputs).  Returns the creation's AI_OK / AI_WRTOL or a negative
 * ai_rc.
 *
 * ai_batch_plan_destroy frees the plan's device memory; the caller makes sure
 * that no launch of the plan is still running or will be replayed. */
typedef struct ai_batch_plan ai_batch_plan;

int ai_batch_plan_create(const ai_batch_item *items, int32_t count, int32_t kernel,
                         ai_batch_plan **out);
int ai_batch_plan_launch(const ai_batch_plan *plan, void *stream);
int ai_batch_plan_destroy(ai_batch_plan *plan);

/* Replay one trajectory with its path: the integration ai_integrate performs
 * for it (same attempts, bitwise the same final state and observables), with
 * (t, y) recorded at t0 and at `refine` points per accepted step (Sec. 4.1
 * follows single trajectories, e.g. the longest-lived one of an ensemble).
 * Blocks until done.
 *
 * y0: device, the trajectory's 12 components (consecutive doubles).
 * refine: 1 .. 1024 points per accepted step, at fractions j/refine of the step,
 *   the last at its end.  Points inside a step come from the quintic Hermite
 *   interpolant of the positions through position, velocity and acceleration at
 *   both ends of the step (locally sixth order; ode45's own continuous extension
 *   is fourth order), velocities from its derivative.
 * capacity >= 0 points; t_out: device, capacity doubles; y_out: device, 12
 *   planes of capacity doubles (component c of point k at y_out[c*capacity+k]).
 *   Points beyond capacity are counted but not stored.
 * final_state: device, 12 doubles; obs: device, AI_NOBS doubles.
 * *points (host) receives the trajectory's number of points,
 *   1 + refine * accepted steps.
 * The potential may have any exponents ai_integrate accepts in its plain
 * kernel.  Returns AI_OK, AI_WRTOL or a negative ai_rc. */
int ai_trace(const ai_params *p, const double *y0, double t0, double tmax, double rtol,
             double atol, int32_t refine, int64_t capacity, double *t_out, double *y_out,
             double *final_state, double *obs, int64_t *points);

/* ---- Serving: a stream of integration requests ------------------------------
 *
 * The paper's ensemble call (Sec. 3.3) offered as a service: requests of
 * different systems, sizes, tolerances and precisions arrive over time and
 * each is answered as soon as its trajectories are done.  A server works on
 * the device that is current when it is created.  Requests are validated when
 * submitted and served in arrival order.  A request's results are bitwise
 * those of ai_integrate on it alone, whatever it shares the GPU with.  The
 * caller owns every buffer and keeps it allocated until ai_server_wait has
 * returned the request's completion.  A request's initial states must be in
 * its buffers when it is submitted (the server's streams and kernel do not
 * wait for work on other streams: synchronize whatever produced them first).
 * Two modes:
 *
 * AI_SERVE_RESIDENT (continuous batching): a resident kernel stays on the GPU
 * while requests flow.  The server owns a slab of device memory (slab_bytes)
 * and admits a request, in arrival order, once its footprint (its initial
 * states, final states and observables, 296 bytes per trajectory rounded up
 * to 256-byte planes) fits in the slab's free space and one of `ring` request
 * slots is free; it copies the initial states into the slab, publishes the
 * request to the kernel, and the kernel's waves take its trajectories as their
 * lanes free up, next to the earlier requests' trajectories (a lane of a wave
 * runs one trajectory of any request, with that request's constants and
 * precision).  When the kernel has counted all of a request's trajectories
 * done it signals the server, which copies the results out to the caller's
 * buffers and frees the slab space.  A request may give host memory (pinned
 * for asynchronous copies) or device memory of the server's device.  Requests
 * must have n = 4, m = 8 (else AI_EUNSUPPORTED at submission); a request
 * larger than the slab is refused (AI_EINVAL).  The kernel holds the GPU's
 * wave slots while it runs: each wave exits once it has found no work for
 * idle_ms, and the server relaunches the kernel when requests arrive again, so
 * other work on the device waits while requests are being served.
 *
 * AI_SERVE_LAUNCHES: one or more workers, each a thread with a stream of its
 * own; whenever its previous launch has finished, a worker takes every queued
 * request (in order, up to max_batch trajectories; at least one) into one
 * ai_integrate_batch_async launch, so requests that arrive while launches run
 * share the next one, and several workers keep launches overlapping.  A
 * request with AI_FP32_STAGES, or with exponents other than n=4, m=8, runs
 * alone (ai_integrate_async).  Buffers must be device memory of the server's
 * device. */
typedef struct ai_server ai_server;

enum ai_serve_mode { AI_SERVE_LAUNCHES = 0, AI_SERVE_RESIDENT = 1 };

typedef struct ai_server_config {
  int64_t max_batch;  /* launches: trajectories per launch, >= 0; 0 selects 2^22 */
  int32_t schedule;   /* launches: AI_SCHEDULE_LONGEST_FIRST or 0, for every launch */
  int32_t workers;    /* launches: launches in flight at once, 0 .. 16; 0 selects 3 */
  int32_t mode;       /* enum ai_serve_mode */
  int32_t ring;       /* resident: requests admitted at once, 0 .. 65536; 0 selects 1024 */
  int64_t slab_bytes; /* resident: device memory for admitted requests, >= 0; 0 selects 4 GiB */
  double idle_ms;     /* resident: a wave with no work exits after this long, >= 0; 0 selects 20 */
  int32_t refill_min; /* resident: free lanes a busy wave gathers before taking more, 0 .. 64;
                         0 selects 8 */
  int32_t reserved;   /* 0 */
} ai_server_config;

/* Completion record of a request.  Times are seconds of the host's monotonic
 * clock (CLOCK_MONOTONIC): submitted; taken into a launch (resident: published
 * to the kernel, its initial states in the slab); completed (resident: results
 * copied out). */
typedef struct ai_request_info {
  int32_t rc;          /* AI_OK, AI_WRTOL, or a negative ai_rc of its launch */
  int32_t batch_size;  /* requests in its launch (resident: requests on the GPU when it was
                          published, itself included) */
  int64_t batch_id;    /* launches are numbered 0, 1, ... per server (resident: the kernel
                          launch it was published to) */
  int64_t batch_trajectories; /* trajectories in its launch (resident: of those requests) */
  double submit_s, start_s, end_s;
  char error[128];     /* ai_last_error() text of a failed launch, else "" */
} ai_request_info;

/* Create a server (cfg may be NULL for the defaults).  Returns AI_OK,
 * AI_EINVAL, AI_EHIP or AI_ENOMEM; *out is NULL on failure. */
int ai_server_create(const ai_server_config *cfg, ai_server **out);

/* Queue one request: item as in ai_integrate_batch (buffers as the mode
 * allows), kernel AI_KERNEL_PLAIN or AI_KERNEL_PLAIN | AI_FP32_STAGES.
 * Validates it as ai_integrate does and returns its error without queueing
 * it, else AI_OK (or AI_WRTOL if its rtol will be raised) and a ticket,
 * unique per server.  Thread-safe. */
int ai_server_submit(ai_server *srv, const ai_batch_item *item, int32_t kernel,
                     uint64_t *ticket);

/* Wait up to timeout_s seconds (< 0: without limit) for the request of
 * `ticket` and fill *info.  Returns AI_OK once it has completed (its own
 * outcome is info->rc) and forgets the ticket; AI_EAGAIN if it has not
 * completed yet (wait again); AI_EINVAL for a ticket it does not hold. */
int ai_server_wait(ai_server *srv, uint64_t ticket, double timeout_s, ai_request_info *info);

/* Finish every queued request, stop the workers (resident: the kernel) and
 * release the server.
 * Requests not yet waited for are forgotten (their outputs are complete).  No
 * other call on the server may be in progress or follow. */
int ai_server_destroy(ai_server *srv);

/* The duration in milliseconds of the integration kernel of one of the calling
 * thread's calls made with AI_TIME_KERNEL: back = 0 for the last such call, 1
 * for the one before, ... up to 63 (the last 64 are kept), so calls can run
 * back to back and be read afterwards.  Returns AI_OK, AI_EAGAIN if the
 * stream has not reached that kernel's end yet, AI_EINVAL if there is no such
 * call (or ms is NULL), AI_EHIP. */
int ai_kernel_time(int32_t back, float *ms);

/* Launch facts of one kernel on the current device. */
typedef struct ai_kernel_info {
  int32_t block_threads;      /* threads per workgroup */
  int32_t vgprs;              /* vector registers per lane */
  int32_t spill_bytes;        /* private (scratch) bytes per lane; 0 = no spills */
  int32_t blocks_per_cu;      /* resident workgroups per CU at this register use */
  int32_t waves_per_simd;     /* resident waves per SIMD */
  int32_t compute_units;      /* CUs of the device */
  int64_t persistent_blocks;  /* grid of the persistent kernel */
} ai_kernel_info;

/* Fill *info for AI_KERNEL_PLAIN or AI_KERNEL_PERSISTENT, with AI_FP32_STAGES
 * for the single-precision-stage plain kernel (schedule and refill bits
 * ignored).  Returns AI_OK or a negative ai_rc. */
int ai_get_kernel_info(int32_t kernel, ai_kernel_info *info);

/* Text of the last error on the calling thread ("" if none). */
const char *ai_last_error(void);

int ai_nobs(void);    /* AI_NOBS */
int ai_version(void); /* library version, > 0 */

#ifdef __cplusplus
}
#endif

#endif /* AI_H */
