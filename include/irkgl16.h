/*
 * irkgl16.h -- C ABI of the MI355X (gfx950) IRKGL16 library.
 *
 * The library integrates many independent separable second-order Hamiltonian
 * systems  q'' = g(q),  p = m v,  H = sum |p|^2/(2m) + U(q)  (paper section 2.3,
 * eqs. sHam / Hamode2) with the fixed-step 8-stage Gauss-Legendre collocation
 * method of order 16 (section 2.2) in its floating-point-symplectic
 * second-order form (section 2.4, eqs. Gi, Qi2, qnvn2), solved by the
 * stage-wise fixed-point iteration with extrapolated initial guess
 * (section 2.5, eqs. IRK_init2, IRK_FP2) and the stopping rule of eq. stopping;
 * the state (q, v) is kept as a pair of binary64 numbers and updated with
 * compensated summation (section 5).  All arithmetic is IEEE binary64; every
 * step runs in HIP kernels on the GPU.
 *
 * Threading: a context is not thread-safe; use one per host thread.
 * Errors: every call returns a status code (below); no C++ exception crosses
 * this interface.
 */
#ifndef IRKGL16_H
#define IRKGL16_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define IRKGL16_OK 0
#define IRKGL16_EINVAL (-1)     /* bad argument: kind, n, d, mass, h, stride...  */
#define IRKGL16_ENOMEM (-2)     /* host or device allocation failed              */
#define IRKGL16_EDEVICE (-3)    /* no usable GPU, or a HIP runtime error         */
#define IRKGL16_ENONFINITE (-4) /* an instance produced NaN/Inf (others written) */
#define IRKGL16_ESCRATCH (-5)   /* irkgl16_integrate_static: the call needs more  */
                                /* than the fixed scratch (size limits below)     */
#define IRKGL16_ECANCELED (-6)  /* a served request was cancelled                */
#define IRKGL16_ENOCONV 1       /* warning: some steps stopped at max_iter       */

/* ---- force kinds -------------------------------------------------------- */
/* KEPLER : g(q) = -G q / |q|^3                      (n = 1, d = 2 or 3)
 * GRAVITY: g_a  = G sum_{b != a} m_b (q_b - q_a) / (|q_b - q_a|^2 + eps^2)^{3/2}
 *          (Plummer-softened Newtonian gravity; section 5.1.2, eq. Ham2)
 * CHAIN  : g_i  = [k_{i+1} V'(q_{i+1} - q_i) - k_i V'(q_i - q_{i-1})] / m_i,
 *          V'(s) = s + beta s^3, fixed ends q_0 = q_{n+1} = 0 (FPU-beta; d = 1) */
#define IRKGL16_KEPLER 0
#define IRKGL16_GRAVITY 1
#define IRKGL16_CHAIN 2

/* ---- option flags ------------------------------------------------------- */
/* q0/p0/q_out/p_out of irkgl16_integrate are device pointers and the work is
 * only enqueued on the context's stream (the caller synchronizes). */
#define IRKGL16_DEVICE_PTRS 1u
/* Plain form: one kernel launch per step per instance, instances in turn (the
 * comparison baseline for the batched persistent kernel). */
#define IRKGL16_PLAIN 2u
/* Reproducible arithmetic: every operation in the reference order of a plain
 * strict-IEEE evaluation of the formulas (separate multiply and add, sums from
 * zero in ascending index order, correctly rounded square root and division,
 * forces summed over ordered pairs), so results are bit-identical to such a
 * CPU implementation.  Slower; the default uses fused multiply-adds, a refined
 * reciprocal square root and pair symmetry (results then agree to rounding
 * level, and the fixed-point iteration counts, which are decided at rounding
 * level, may differ). */
#define IRKGL16_REPRODUCIBLE 4u
/* With IRKGL16_PLAIN: the launches of one step (one per instance) are
 * captured once into a HIP graph and the graph is replayed once per step
 * (instances that have finished do no work in later replays); launches of
 * whole-GPU (cooperative) instances stay outside the graph.  Results are
 * bit-identical to IRKGL16_PLAIN. */
#define IRKGL16_GRAPH 8u

typedef struct irkgl16_ctx irkgl16_ctx;

/* One instance.  n bodies (GRAVITY) or sites (CHAIN) of dimension d; Dq = n d
 * position components.  mass: GRAVITY n masses > 0 (required); CHAIN n site
 * masses > 0 or NULL (all 1); KEPLER ignored (1).  coupling: CHAIN n+1 bond
 * stiffnesses k_0..k_n or NULL (all 1).  G: KEPLER the gravitational parameter,
 * GRAVITY the constant.  eps >= 0 softening (GRAVITY).  beta: CHAIN.  The
 * arrays are host memory, read during irkgl16_create only. */
typedef struct {
  int32_t kind, n, d;
  const double *mass;
  const double *coupling;
  double G, eps, beta;
} irkgl16_problem;

/* max_iter: cap on fixed-point iterations per step (<= 0 means 100; the paper
 * sets none).  record_iters: keep the iteration count of every step.  flags:
 * IRKGL16_* option flags.  stages: s of the s-stage Gauss-Legendre member of
 * the family (order 2s; section 2.2): 0 or 8 for IRKGL16; 2, 4 or 6 (IRKGL4,
 * IRKGL8, IRKGL12, coefficients built as for s = 8, section 2.4) only for
 * contexts created by irkgl16_create_user / irkgl16_create_ode; anything else
 * is IRKGL16_EINVAL.  method: 0 for the implicit method; IRKGL16_STRANG or
 * IRKGL16_SUZ90 run an explicit symplectic baseline instead (section 4: the
 * Strang splitting of eq. Strang, or Suzuki's fourth-order composition of
 * five Strang steps, eq. comp_method, both in the ABA form of eq.
 * high_order_splitting with the exact flows of eq. flowAB: kicks
 * v += b_j h g(q, t_j) at t_j = t_{n-1} + (a_1 + ... + a_j) h between drifts
 * q += a_j h v, on the same two-double state); only for
 * irkgl16_create_user contexts (with stages 0 or 8), else IRKGL16_EINVAL.
 * Such a context costs 1 (Strang) or 5 (SUZ90) force evaluations per step and
 * reports no fixed-point iterations (zero counts). */
typedef struct {
  int32_t max_iter;
  int32_t record_iters;
  uint32_t flags;
  int32_t stages;
  int32_t method;
} irkgl16_options;

/* irkgl16_options.method */
#define IRKGL16_STRANG 1
#define IRKGL16_SUZ90 2

/* Results of the last irkgl16_integrate call.  The three pointers are
 * optional caller-owned host arrays filled when non-NULL:
 * inst_iterations[n_inst] (sum of k), inst_status[n_inst] (status code per
 * instance), step_iters[sum nsteps] (k of every step, instance-major; only with
 * record_iters). */
typedef struct {
  int64_t steps;              /* instance-steps done                        */
  int64_t iterations;         /* sum of k over all steps                    */
  int64_t nonconverged_steps; /* steps that stopped at max_iter             */
  int32_t max_k;              /* largest k of any step                      */
  int32_t n_nonfinite;        /* instances stopped by a NaN/Inf             */
  double device_ms;           /* GPU time of the call (HIP events, stream)  */
  int64_t *inst_iterations;
  int32_t *inst_status;
  uint8_t *step_iters;
} irkgl16_stats;

/* Create a context for n_inst instances (probs[n_inst], host memory, copied).
 * hip_stream: a hipStream_t to enqueue on, or NULL for a library-owned stream.
 * Returns IRKGL16_EDEVICE when no GPU is usable.  *out is NULL on failure. */
int irkgl16_create(irkgl16_ctx **out, const irkgl16_problem *probs, int32_t n_inst,
                   const irkgl16_options *opt, void *hip_stream);

/* Create a context whose instances share one force supplied as device source
 * (paper section 3.3: the user's right-hand side is a generic function that
 * the method evaluates at all 8 stages at once; eq. ivp2: q'' = g(q, t)).
 * force_src: NUL-terminated HIP device source, read during the call, that
 * defines
 *     __device__ void irkgl16_user_force(const double *q, double *g,
 *                                        const double *prm, double t);
 * which writes g(q, t) for the Dq = dq position components in q at time t;
 * prm points at the instance's n_params parameters (NULL when n_params == 0).
 * It is called at the stage times t = fl(fl((n-1) h) + fl(c_i h)) of step n
 * (eq. IRK_FP), time counted from 0 at the start of each integrate call.  It
 * must keep no state between calls; one stage's call runs on one lane, so
 * branches cost only divergence between the 8 stages of an instance.  The
 * macro IRKGL16_DQ holds dq.  Masses are 1 (p = v).
 * dq: 1..64.  params: n_inst x n_params doubles (host memory, copied),
 * instance-major.  The source is compiled once per process for each
 * (source, dq, arithmetic mode) with hiprtc for gfx950, with floating-point
 * contraction off (a*b+c is a multiply and an add unless the source calls fma),
 * into the small-system kernel: 8 instances per 64-lane wavefront.  The
 * context is then used with irkgl16_integrate like any other (flags as in
 * irkgl16_options; q0/p0 are n_inst x dq).  Returns IRKGL16_EINVAL for a bad
 * argument or a source that does not compile (irkgl16_user_compile_check
 * gives the compiler log), IRKGL16_EDEVICE when the code object cannot be
 * loaded or no GPU is usable.  The serving interface does not take user
 * forces. */
int irkgl16_create_user(irkgl16_ctx **out, const char *force_src, int32_t dq, int32_t n_params,
                        const double *params, int32_t n_inst, const irkgl16_options *opt,
                        void *hip_stream);

/* Compile force_src for dq components (as irkgl16_create_user does) without
 * a GPU; writes the compiler log (NUL-terminated, truncated to log_len bytes)
 * when log is non-NULL.  Returns IRKGL16_OK or IRKGL16_EINVAL. */
int irkgl16_user_compile_check(const char *force_src, int32_t dq, char *log, int64_t log_len);

/* Create a context for the FIRST-ORDER form (paper section 2.4, eqs. Yi2 and
 * yn2; section 2.5, eqs. IRK_init and IRK_FP): y' = f(t, y), y in R^D, for
 * problems that are not of the form q'' = g(q, t) (e.g. non-separable
 * Hamiltonians, eq. Ham_SBH).  Stages Y_i = y + sum_j mu_ij L_j with
 * L_i = h b_i f(t_i, Y_i), update y + sum_i L_i with the two-double state,
 * initial guess Y_i = y + sum_j nu_ij L_prev_j, stopping rule eq. stopping
 * over all D components.  rhs_src: NUL-terminated HIP device source that
 * defines
 *     __device__ void irkgl16_user_rhs(const double *y, double *f,
 *                                      const double *prm, double t);
 * writing f(t, y) for the D components (macro IRKGL16_DQ = D), with the same
 * rules, parameters, stage times and compilation as irkgl16_create_user.
 * D: 1..64.  With such a context irkgl16_integrate takes y0 in q0 (D values
 * per instance) and writes the y frames to q_out; p0 and p_out are not used
 * (may be NULL).  Errors as irkgl16_create_user
 * (irkgl16_ode_compile_check gives the compiler log). */
int irkgl16_create_ode(irkgl16_ctx **out, const char *rhs_src, int32_t D, int32_t n_params,
                       const double *params, int32_t n_inst, const irkgl16_options *opt,
                       void *hip_stream);

/* Compile rhs_src for D components (as irkgl16_create_ode does) without a
 * GPU; log as irkgl16_user_compile_check.  Returns IRKGL16_OK or
 * IRKGL16_EINVAL. */
int irkgl16_ode_compile_check(const char *rhs_src, int32_t D, char *log, int64_t log_len);

/* Integrate every instance from its initial state.
 * q0, p0: sum(Dq_i) doubles, instances concatenated in order (host memory, or
 *         device memory with IRKGL16_DEVICE_PTRS).  v = fl(p / m) on input.
 * h, nsteps, out_stride: n_inst values each (host memory, always).  h finite
 *         and nonzero (h < 0 integrates backwards); nsteps >= 0;
 *         out_stride >= 1 divides nsteps.
 * q_out, p_out: sum(Dq_i * (nsteps_i / out_stride_i + 1)) doubles, instance i
 *         as [frame][Dq_i]; frame f is the state after f * out_stride_i steps
 *         (frame 0 = initial state), q = q.hi and p = m * v.hi.  Frames after an
 *         instance became non-finite are NaN.
 * stats: nullable.  In host mode the call returns when outputs are complete;
 * with IRKGL16_DEVICE_PTRS it returns after enqueueing (stats, if given, force a
 * stream synchronization).  Returns the worst status over instances.
 * Scheduling (never changes results): the batched kernels run in chunks up to
 * step boundaries j ceil(max nsteps / c), c = min(C, max nsteps / 64) (at
 * least 1); between chunks a device kernel orders each class's work queue by
 * estimated remaining work (steps left times the iterations per step of the
 * last chunk) and moves gravitational instances of the few-body class that
 * needed at least P iterations per step to the stage-parallel kernel for the
 * next chunk (both kernels compute the same arithmetic).  Within a chunk, the
 * few-body kernel stops an instance at the end of a step once its recent
 * iterations per step (an exponential average over about 8 steps) reach E; it
 * catches up on the stage-parallel kernel in the next chunk.  Only classes
 * that can promote are chunked by default (and only while an auxiliary stream
 * is free for their promoted launches).  C = 8, P = 5 and E = 12 unless the
 * tuning table (tune_cache.json beside the library, or the file
 * IRKGL16_TUNE_CACHE names; written by the autotuner) sets sched/max_chunks =
 * C, sched/promote_k10 = 10 P or sched/evict_k10 = 10 E.  Environment, read by
 * irkgl16_create*, overriding the table: IRKGL16_CHUNKS = c (a positive
 * integer; fixed chunk count, every batched class chunked), IRKGL16_PROMOTE_K
 * = P, IRKGL16_EVICT_K = E (0: never, for either).  A promotable few-body
 * class with at least 128 instances per CU runs as two halves of alternate
 * instances, each chunked on its own stream without waiting for the other at
 * chunk boundaries, while the process's streams (the caller's and the default
 * one, the library's live contexts and servers, this context's) fit in HIP's
 * GPU_MAX_HW_QUEUES (4 unless set); IRKGL16_HALVES = 0 or 1, read by
 * irkgl16_create*, forces the choice. */
int irkgl16_integrate(irkgl16_ctx *ctx, const double *q0, const double *p0, const double *h,
                      const int64_t *nsteps, const int64_t *out_stride, double *q_out,
                      double *p_out, irkgl16_stats *stats);

/* Synchronize the context's stream and fill stats for the last integrate call.
 * Returns that call's worst status. */
int irkgl16_last_stats(irkgl16_ctx *ctx, irkgl16_stats *stats);

/* Release a context and its device memory.  NULL-safe. */
void irkgl16_destroy(irkgl16_ctx *ctx);

/* Static description of a status code. */
const char *irkgl16_strerror(int status);

/* ---- allocation-free integration ----------------------------------------
 * For callers that cannot allocate device memory while they integrate: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  One call does what irkgl16_create + irkgl16_integrate (with
 * IRKGL16_DEVICE_PTRS) + irkgl16_destroy do, with the same kernels and the
 * same results bit for bit, but calls no device or host allocator: the
 * per-call device data (coefficient table, instance descriptors, masses and
 * couplings, class work queues and their counters, per-instance statistics,
 * the resumable state records, iteration counts) lives in one fixed device
 * array of IRKGL16_STATIC_SCRATCH_BYTES per GPU, which exists from the
 * library's loading on that GPU until the process ends, and the host side
 * stages through fixed arrays.  The first call on a GPU looks up that array's
 * device address and creates three HIP events (kept until the process ends).
 *
 * probs, h, nsteps, out_stride: host memory, as irkgl16_create and
 *   irkgl16_integrate (read during the call).
 * q0, p0, q_out, p_out: DEVICE memory, layouts as irkgl16_integrate.
 * opt: nullable; flags may hold IRKGL16_REPRODUCIBLE (IRKGL16_DEVICE_PTRS is
 *   implied); stages 0 or 8, method 0; max_iter and record_iters as in
 *   irkgl16_options.
 * hip_stream: the hipStream_t the work is enqueued on (NULL: the null stream).
 * stats: nullable; when given, the call synchronizes the stream and fills it
 *   (step_iters only with record_iters); otherwise it returns after enqueueing
 *   and the caller synchronizes.
 * Scope: instances of the batched kernel classes -- Kepler, gravity up to 512
 *   bodies, FPU-beta chains up to 1024 sites; one launch per class, in turn on
 *   the one stream (no chunks, no promotion: those change only the schedule).
 *   A gravitational system of more than 512 bodies (whole-GPU kernel) is
 *   IRKGL16_EINVAL, as are the flags, stages or methods not listed above.
 * Limits: at most IRKGL16_STATIC_MAX_INST instances, and the call's scratch
 *   ((4 + 8) Dq doubles = 96 Dq bytes of state per instance, plus descriptors,
 *   statistics, masses, queues and, with record_iters, one byte per step)
 *   must fit IRKGL16_STATIC_SCRATCH_BYTES; otherwise IRKGL16_ESCRATCH, before
 *   any device work.
 * Concurrency: every call on a GPU reuses that GPU's array and keeps nothing
 *   from earlier calls (the setup kernel rewrites what must start at zero).
 *   Calls are serialized on the host; calls enqueued on different streams of
 *   one GPU without synchronization between them race on the array. */
#define IRKGL16_STATIC_SCRATCH_BYTES (32ll << 20)
#define IRKGL16_STATIC_MAX_INST 16384
int irkgl16_integrate_static(const irkgl16_problem *probs, int32_t n_inst,
                             const irkgl16_options *opt, void *hip_stream, const double *q0,
                             const double *p0, const double *h, const int64_t *nsteps,
                             const int64_t *out_stride, double *q_out, double *p_out,
                             irkgl16_stats *stats);

/* ---- serving ------------------------------------------------------------
 * A server integrates requests that arrive over time with continuous batching:
 * a serving thread admits pending requests (first come, first served) whenever
 * their device memory fits under cap_bytes, advances every resident request in
 * one batched launch per kernel class (classes concurrently; each class by the
 * number of steps that fits the target slice time, at most slice_steps), streams the
 * finished output frames of the slice to host memory, retires finished requests
 * and admits new ones before the next slice.  A request's resumable state
 * (two-double q and v, previous-step increments, counters) stays on the device
 * between slices, so its result is bit-identical to integrating it alone with
 * irkgl16_integrate under the same flags. */
typedef struct irkgl16_server irkgl16_server;

typedef struct {
  int64_t cap_bytes;   /* device memory for resident requests (> 0)            */
  int64_t slice_steps; /* steps per request per slice at most (<= 0: 1000)     */
  int32_t max_iter;    /* as in irkgl16_options                                */
  int32_t max_resident;/* resident requests at most (<= 0 means 65536)         */
  uint32_t flags;      /* IRKGL16_REPRODUCIBLE or 0                            */
  double slice_ms;     /* target slice duration in ms (<= 0 means 20): each    */
                       /* kernel class advances its requests by the steps that */
                       /* fit, from that class's measured time per step        */
} irkgl16_server_options;

typedef struct {
  int32_t status;      /* per-request status code                              */
  int64_t steps;       /* steps done                                           */
  int64_t iterations;  /* sum of k                                             */
  double submit_s;     /* seconds since server creation: submitted, admitted,  */
  double admit_s;      /* finished                                             */
  double done_s;
} irkgl16_request_info;

/* Start a server (creates the serving thread).  hip_stream as in
 * irkgl16_create.  Returns IRKGL16_EDEVICE without a usable GPU and
 * IRKGL16_ENOMEM if cap_bytes cannot be allocated. */
int irkgl16_server_create(irkgl16_server **out, const irkgl16_server_options *opt,
                          void *hip_stream);

/* Submit one request (problem as in irkgl16_create; q0, p0: Dq host doubles;
 * h, nsteps, out_stride as in irkgl16_integrate).  Everything is copied; the
 * call returns at once with a ticket.  EINVAL for invalid arguments or a request
 * larger than the whole cap. */
int irkgl16_submit(irkgl16_server *s, const irkgl16_problem *prob, const double *q0,
                   const double *p0, double h, int64_t nsteps, int64_t out_stride,
                   int64_t *ticket);

/* *done = 1 if the request has finished (0 otherwise).  EINVAL: unknown ticket. */
int irkgl16_poll(irkgl16_server *s, int64_t ticket, int32_t *done);

/* Block until the request finishes, copy its frames (layout as irkgl16_integrate
 * for one instance) into q_out/p_out (host, nullable), fill info (nullable), and
 * release the ticket.  Returns the request's status. */
int irkgl16_wait(irkgl16_server *s, int64_t ticket, double *q_out, double *p_out,
                 irkgl16_request_info *info);

/* Cancel a request.  A pending one is dropped (its frames after frame 0 are
 * NaN); a resident one stops when the current time slice ends, keeping the
 * frames of the steps it completed (later frames NaN).  irkgl16_wait then
 * returns IRKGL16_ECANCELED with the steps done in info.  A request that has
 * already finished is left as it is.  EINVAL: unknown ticket. */
int irkgl16_cancel(irkgl16_server *s, int64_t ticket);

/* Totals of a server since its creation. */
typedef struct {
  int64_t slices;             /* time slices run                                  */
  double slice_wall_s;        /* their summed wall time (set-up, uploads, kernels, */
                              /* copies of statistics and frames, harvest)        */
  double slice_device_s;      /* their summed device time, first upload to last   */
                              /* kernel (HIP events on the slice stream)          */
  int64_t requests_done;      /* finished requests, cancelled ones included       */
  int64_t requests_cancelled;
  int32_t max_resident;       /* most requests resident in one slice              */
  int32_t resident, pending;  /* now                                              */
} irkgl16_server_info;

int irkgl16_server_stats(irkgl16_server *s, irkgl16_server_info *out);

/* Stop the serving thread after the resident and pending requests finish, and
 * release everything.  NULL-safe. */
void irkgl16_server_destroy(irkgl16_server *s);

#ifdef __cplusplus
}
#endif
#endif /* IRKGL16_H */
