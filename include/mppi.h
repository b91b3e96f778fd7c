/*
 * mppi.h - C ABI of the MI355X MPPI + Gate-SDF library.
 *
 * One MPPI iteration (Section IV-A, update equation eq:mppi_update) for a
 * quadrotor whose cost uses a learned gate signed distance field
 * (Section III-B decoder g_phi; Section IV-B costs eqs. 5-9):
 *   1. sample K perturbed control sequences U^m = U* + dU^m, dU ~ N(0, Sigma);
 *   2. roll each out over T steps of the quadrotor model;
 *   3. query the Gate-SDF decoder at every predicted position, per gate;
 *   4. accumulate gate progress (eq. 5), perception alignment (eq. 6),
 *      SDF safety (eqs. 7-8) and control effort into J (eq. 9);
 *   5. form w_m = exp(-J_m/lambda) / sum_i exp(-J_i/lambda) and U* = sum w_m U^m;
 *      only U*_0 is applied and U* seeds the next cycle (Section IV-A).
 *
 * Conventions (readings of the paper where it is silent):
 *  - rollouts are K, horizon steps T, gates G (the paper writes M rollouts,
 *    K horizon steps);
 *  - state x = [p(3), q(4) as (w, x, y, z), v(3), omega(3)], world z up,
 *    Hamilton quaternions body -> world, thrust along body +z;
 *  - control u = [collective thrust (N), body rates wx, wy, wz (rad/s)]
 *    (MPPI_DYN_CTBR), or the paper's own input, the rates of the four rotor
 *    thrusts (N/s) with the thrusts and the body rate as state
 *    (MPPI_DYN_ROTOR_RATES, see mppi_dynamics);
 *  - noise: Philox4x64-10, counter (k, t, instance_id, tick), key (seed, 0),
 *    23-bit uniforms and Box-Muller, delta u = L n with L L^T = Sigma;
 *  - the SDF is queried at the T predicted positions p_1..p_T (flag
 *    MPPI_REQ_SDF_AT_P0 selects p_0..p_{T-1}); with several gates the field
 *    is the maximum over gates;
 *  - gate progress uses the telescoped form |p_T - wp|^2 - |p_0 - wp|^2.
 *
 * Ownership: the caller owns every request/result buffer; the engine copies
 * what it needs before a call returns (mppi_submit deep-copies the request).
 * The engine owns its device memory; an external device pool passed in the
 * config stays owned by the caller and must outlive the engine.
 *
 * Errors: every call returns an mppi_status.  A HIP runtime failure returns
 * MPPI_EDEVICE and is sticky: every later call on that engine returns it.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mppi_status {
  MPPI_OK = 0,
  MPPI_PENDING = 1,     /* mppi_poll: the solve has not finished yet */
  MPPI_EINVAL = -1,     /* invalid argument (see each call) */
  MPPI_ENOMEM = -2,     /* device memory exhausted, or a request that can never fit the budget */
  MPPI_EAGAIN = -3,     /* host queue full or every instance slot busy: retry later */
  MPPI_ENOTFOUND = -4,  /* unknown or already retired ticket */
  MPPI_ENUMERIC = -5,   /* every rollout cost was non-finite; U* left unchanged */
  MPPI_EDEVICE = -6     /* HIP runtime error (sticky) or no usable gfx950 device */
} mppi_status;

typedef enum mppi_precision {
  MPPI_PREC_FP32 = 0,   /* decoder hidden layers on FP32 matrix cores */
  MPPI_PREC_BF16 = 1,   /* BF16 weights and activations, FP32 accumulation */
  MPPI_PREC_BF16X2 = 2, /* BF16 weights, activations split hi + lo in BF16 (two products) */
  MPPI_PREC_FP8 = 3,    /* OCP FP8 E4M3 weights and activations, per-layer scales */
  MPPI_PREC_BF16X3 = 4, /* BF16 weights, activations split hi + mid + lo in BF16 (three products) */
  MPPI_PREC_F16X2 = 5   /* BF16-rounded weights held exactly in FP16 (per-layer power-of-two scale),
                           activations split hi + lo in FP16 (two products); activations are
                           capped at 65503 */
} mppi_precision;

typedef enum mppi_path {
  MPPI_PATH_PLAIN = 0,  /* one solve per launch sequence: rollout, SDF, cost, reduce kernels */
  MPPI_PATH_FUSED = 1   /* rollout + SDF + cost fused per tile, batched across solves;
                           BF16 / BF16X2 / BF16X3 / F16X2 / FP8 with H in {128, 256, 512} and 1-2 hidden H x H layers */
} mppi_path;

typedef enum mppi_sdf_kind {
  MPPI_SDF_MLP = 0,       /* learned decoder g_phi(z, p) (Section III-B) */
  MPPI_SDF_ANALYTIC = 1   /* guidance field s = c + |x| tan(alpha) - max(|y|,|z|) (eqs. 1-2) */
} mppi_sdf_kind;

/* Vehicle model (Section IV-A).  ROTOR_RATES: u = (dT_1 .. dT_4)/dt; rotor i
 * sits at body (x_i, y_i) = arm/sqrt(2) (s_x, s_y), (s_x, s_y) = (+,+), (-,-),
 * (+,-), (-,+) for i = 1..4, drag torque +/- yaw_coeff T_i about body z with
 * signs +, +, -, -; per step: T <- clip(T + u dt, 0, thrust_max),
 * omega <- clip(omega + dt J^-1 (tau(T) - omega x J omega), +-rate_max) with
 * J = diag(inertia), then the CTBR step with thrust sum T_i and body rate
 * omega.  The rotor thrusts at x0 come with each request (thrust0). */
typedef enum mppi_dynamics {
  MPPI_DYN_CTBR = 0,         /* collective thrust + body rates (rate follows the command) */
  MPPI_DYN_ROTOR_RATES = 1   /* rotor-thrust rates; state adds the 4 thrusts and the body rate */
} mppi_dynamics;

/* Config flags. */
#define MPPI_CFG_TIMING (1u << 0)  /* record per-kernel HIP event times (see mppi_get_stats) */
/* Served path on the fused decoder: one batched launch per admission pass
 * (up to three in flight on their own streams) instead of the work ring that
 * a persistent kernel serves (the default where it exists: H <= 256). */
#define MPPI_CFG_SERVE_BATCHES (1u << 1)

/* Create-time configuration (immutable for the engine's life). */
typedef struct mppi_config {
  int32_t precision;         /* mppi_precision */
  int32_t path;              /* mppi_path */
  int32_t sdf_kind;          /* mppi_sdf_kind */
  int32_t hidden;            /* decoder width H: 64, 128, 256 or 512 */
  int32_t n_hidden;          /* hidden layers L >= 2: widths 67 -> H (L times) -> 1 */
  int32_t latent_dim;        /* must be 64 */
  int32_t K_max, T_max, G_max;  /* per-solve limits: K <= 16384, T <= 128, G <= 8 */
  int32_t max_instances;     /* resident warm-start slots (instance table); an instance keeps its slot
                                for the engine's life, and a request for a new instance while the table is
                                full fails with EAGAIN (the served path fails that ticket alone) */
  int32_t max_inflight;      /* solves on the device at once (served path) */
  int32_t queue_depth;       /* host queue capacity of mppi_submit */
  int32_t device;            /* HIP device ordinal */
  uint32_t flags;            /* MPPI_CFG_* */
  uint64_t hbm_budget_bytes; /* admission budget for per-solve device memory */
  uint64_t seed;             /* Philox key word 0 */
  double mass;               /* kg */
  double gravity;            /* m/s^2 */
  double u_lo[4], u_hi[4];   /* control bounds; sampled controls are clipped to them */
  double sdf_c, sdf_tan_alpha;  /* analytic field parameters (eq. 2) */
  void* stream;              /* hipStream_t for the blocking path, or NULL: engine creates one */
  void* device_pool;         /* optional caller-owned device memory for per-solve buffers */
  uint64_t device_pool_bytes;
  int32_t dynamics;          /* mppi_dynamics */
  int32_t pe_freqs;          /* F in [0, 8]: the decoder reads PE(p) = [p, sin(2^k pi p), cos(2^k pi p), k < F]
                                (Section III-B PE; 0 = raw coordinates); plain path, or fused with H <= 256 */
  /* MPPI_DYN_ROTOR_RATES only (all > 0): principal inertia (kg m^2), arm
   * length (m), yaw drag torque per thrust (m), thrust and body-rate bounds */
  double inertia[3], arm_length, yaw_coeff, thrust_max, rate_max;
  /* Served path in batches (no work ring): the most work one batch launch
   * takes, in decoder query points (K T G summed over its solves); a batch
   * always takes at least the oldest admissible request.  Bounds how long a
   * request waits behind a burst.  0 = the default, 2^21 query points. */
  uint64_t wave_queries_max;
  /* Fused path, H = 512 (weights streamed through LDS): neuron blocks per
   * scheduling region of a K-step, i.e. how far ahead a wave reads its weight
   * fragments: 2, 4 or 8, or 0 = tuned: the first launch of each shape
   * (precision, H, max G, max T of the launch) times the three on that
   * launch's first tiles (two per compute unit, synchronously) and keeps the
   * fastest for the engine's life.  Every choice gives the same results bit
   * for bit (only the order of independent products changes).  Other values:
   * EINVAL.  mppi_step_noalloc never tunes: it takes a shape's tuned choice
   * if there is one, else 4. */
  int32_t wide_region;
} mppi_config;

/* Decoder weights, row-major float32 as a (n_out x n_in) matrix per layer
 * l = 0..n_hidden; layer 0 has n_in = 3 + 6 pe_freqs + latent_dim: the
 * gate-frame coordinates in columns 0..2, then for k = 0 .. pe_freqs-1 the
 * blocks sin(2^k pi p) (x, y, z) and cos(2^k pi p) (x, y, z), then the
 * latent code.
 * The library copies, quantises and packs them once in mppi_create. */
typedef struct mppi_sdf_weights {
  const float* const* W;     /* n_hidden + 1 pointers */
  const float* const* b;     /* n_hidden + 1 pointers */
  const float* act_scale;    /* FP8 only: n_hidden - 1 static scales of the inputs of hidden layers 2..L */
} mppi_sdf_weights;

/* One gate: latent code and the world pose of its frame (Section IV-B-3:
 * world points are mapped into that frame before querying the decoder).
 *
 * Object permanence (Section IV-B-3: while the gate is out of view the last
 * valid latent and its transform are kept and used): z == NULL marks gate g
 * of this request as not observed; the engine then uses the latent and frame
 * of gate g from the latest request of the same instance that observed it
 * (R and t of this entry are ignored).  The engine keeps that cache per
 * instance on the device as the folded first-layer term, so an unobserved
 * gate also skips the fold.  EINVAL when the instance has no observation of
 * gate g yet, or for the analytic field (which has no latent). */
typedef struct mppi_gate {
  const float* z;            /* latent_dim floats, or NULL: use the instance's cached gate g */
  double R[9];               /* row-major 3x3; columns are the gate axes in the world (x = normal) */
  double t[3];               /* gate origin in the world */
} mppi_gate;

#define MPPI_TICK_RESIDENT 0xFFFFFFFFu   /* use (and advance) the instance's resident tick */

/* Request flags. */
#define MPPI_REQ_NO_SHIFT   (1u << 0)  /* do not store the shifted U* as the next warm start */
#define MPPI_REQ_SDF_AT_P0  (1u << 1)  /* query p_0..p_{T-1} (the literal index range of eq. 8) */

/* One solve. */
typedef struct mppi_request {
  uint64_t instance_id;      /* drone/track instance owning the resident warm start */
  uint32_t tick;             /* Philox counter word 3, or MPPI_TICK_RESIDENT */
  uint32_t flags;            /* MPPI_REQ_* */
  int32_t K, T, G;           /* rollouts, horizon steps, gates */
  int32_t pad_;
  double dt;                 /* integration step (s) */
  double x0[13];             /* current state, |q| = 1 within 1e-6 */
  const double* U_nom;       /* T x 4 nominal, or NULL: the resident warm start (hover if new) */
  double Sigma[16];          /* 4x4 symmetric positive semi-definite noise covariance */
  double lambda;             /* temperature > 0 */
  double Q_gate, Q_vis, Q_sdf, d_safe, R_u;  /* cost weights (eq. 9) and clearance (eq. 7) */
  double wp[3];              /* target waypoint p_wp (eq. 5); also the gate centre for eq. 6 */
  const mppi_gate* gates;    /* G gates */
  double thrust0[4];         /* MPPI_DYN_ROTOR_RATES: rotor thrusts at x0, in [0, thrust_max]; x0[10..12] is the body rate */
} mppi_request;

/* Result of one solve (caller-owned buffers). */
typedef struct mppi_result {
  double* U_star;            /* T x 4, required: the updated sequence (eq. mppi_update) */
  double* weights;           /* optional K: normalised weights w_m */
  double* costs;             /* optional K: total cost J_m */
  float* samples;            /* optional K x T x 4: clipped sampled controls (plain path only) */
  float* positions;          /* optional K x (T+1) x 3: positions relative to p_0 (plain path only) */
  float* sdf;                /* optional K x T: max-over-gates field at the query points (plain and fused paths;
                                mppi_step only) */
  double u0[4];              /* U*_0, the action to apply */
  double J_min;              /* min_m J_m */
  double log_eta;            /* log sum_m exp(-J_m / lambda) */
  double ess;                /* effective sample size 1 / sum w_m^2 */
  uint32_t tick_used;        /* Philox tick this solve used */
  int32_t status;            /* mppi_status of the solve */
  uint64_t t_submit_ns, t_admit_ns, t_done_ns;  /* host monotonic clock */
} mppi_result;

typedef struct mppi_engine mppi_engine;

/* Create an engine on config->device.  Validates the config (EINVAL), copies
 * and packs the weights (W/b may be NULL for MPPI_SDF_ANALYTIC), allocates the
 * instance table and per-solve buffers.  Returns EDEVICE when no gfx950 device
 * is usable.  *out is set only on MPPI_OK. */
int mppi_create(const mppi_config* config, const mppi_sdf_weights* weights, mppi_engine** out);

/* Drain in-flight solves, stop the scheduler and free device memory.
 * Must not race other calls on the same engine. */
int mppi_destroy(mppi_engine* engine);

/* One blocking solve.  Its device memory counts against the admission
 * budget (EAGAIN while served solves hold the rest of it; ENOMEM if it can
 * never fit).  EINVAL: lambda <= 0 or non-finite, Sigma not PSD,
 * K/T/G outside [1, max], non-finite x0 or U_nom, |q| not within 1e-6 of 1,
 * NULL U_star/gates, rotor thrusts outside [0, thrust_max].  ENUMERIC: every cost non-finite (U_star = nominal,
 * the resident warm start is kept).  Uses the engine's own stream. */
int mppi_step(mppi_engine* engine, const mppi_request* request, mppi_result* result);

/* Queue a solve for the served path and return a ticket at once.  The request
 * is deep-copied.  EAGAIN: the host queue is full.  ENOMEM: the request's
 * device footprint exceeds the whole budget (it could never be admitted).
 * On the fused decoder with H <= 256 (and no MPPI_CFG_SERVE_BATCHES) the
 * scheduler publishes each admitted solve as work items (a prep item, then
 * one item per tile of 16 rollouts) into a ring in pinned host memory that a
 * persistent kernel consumes while it runs: a request starts on the compute
 * units that free up next, without a launch of its own, and its result comes
 * back in pinned memory without a copy.  Results are bit for bit those of
 * mppi_step.  While that kernel is resident (until about 2 ms after the last
 * served work) it holds every compute unit, so blocking solves and batches
 * on the same device wait for it.  Otherwise the served path launches one
 * batch per admission pass (see wave_queries_max). */
int mppi_submit(mppi_engine* engine, const mppi_request* request, uint64_t* ticket);

/* MPPI_PENDING while the ticket's solve runs; otherwise copies the outcome
 * into *result (U_star etc. must be sized for that request), retires the
 * ticket and returns the solve's status (EINVAL: an unobserved gate with no
 * cached observation; EAGAIN: a new instance while the instance table was
 * full).  ENOTFOUND: unknown/retired ticket. */
int mppi_poll(mppi_engine* engine, uint64_t ticket, mppi_result* result);

/* Block until every submitted solve has finished (results stay pollable). */
int mppi_drain(mppi_engine* engine);

/* Engine counters; kernel times are cumulative HIP event milliseconds, kept
 * only with MPPI_CFG_TIMING. */
typedef struct mppi_stats {
  uint64_t submitted, admitted, completed, failed;
  uint64_t waves;            /* served path: batched launches, or admission passes that published
                                work into the ring */
  uint64_t bytes_in_use, bytes_peak, budget;
  uint64_t sdf_launches;     /* launches of the dominant (SDF) kernel */
  double sdf_ms;             /* summed duration of those launches */
  uint64_t solve_launches;   /* timed solve sequences */
  double solve_ms;           /* summed duration of whole solve sequences */
  uint64_t tune_runs;        /* shapes tuned (mppi_config.wide_region = 0) */
  uint64_t wide_region;      /* region size of the last H = 512 launch (0: none yet) */
  uint64_t ring_launches;    /* launches of the served ring kernel (it stays resident while work
                                keeps arriving and ends after about 2 ms without any) */
} mppi_stats;

int mppi_get_stats(mppi_engine* engine, mppi_stats* out);
void mppi_reset_stats(mppi_engine* engine);

/* Static description of a status code. */
const char* mppi_status_str(int status);

/* Device bytes one solve of this shape takes from the admission budget on
 * this engine's path (its buffers plus, on the fused path, its share of a
 * batch launch's descriptor block). */
uint64_t mppi_solve_footprint(const mppi_engine* engine, int32_t K, int32_t T, int32_t G);

/* Staged batches: n requests validated, packed and copied into device memory
 * once, then launched any number of times with their inputs resident in HBM
 * (a fixed fleet ticking, or a benchmark).  Each launch is one MPPI iteration
 * (Section IV-A) of every request; requests with U_nom == NULL and
 * tick == MPPI_TICK_RESIDENT advance their resident warm start and tick on
 * the device at every launch.  Instance ids within a batch must be distinct
 * (EINVAL otherwise) and are held until mppi_batch_destroy (EAGAIN for other
 * calls on them meanwhile).  The staged solves hold their memory against the
 * admission budget until mppi_batch_destroy: ENOMEM if it can never fit,
 * EAGAIN while served solves hold too much of it.
 * Launches are asynchronous on the engine's stream; mppi_batch_wait blocks
 * until they finish; mppi_batch_results copies the latest outcome of request
 * i into results[i] (caller-owned, U_star sized T_i x 4).  Every mppi_batch_*
 * call that waits on or launches device work (like mppi_step and
 * mppi_step_noalloc) first ends a resident served-ring launch: the work
 * already published finishes, then the call proceeds, and the ring
 * relaunches for the next served request. */
typedef struct mppi_batch mppi_batch;
int mppi_batch_create(mppi_engine* engine, const mppi_request* requests, int32_t n, mppi_batch** out);
int mppi_batch_run(mppi_engine* engine, mppi_batch* batch);
int mppi_batch_wait(mppi_engine* engine, mppi_batch* batch);
int mppi_batch_results(mppi_engine* engine, mppi_batch* batch, mppi_result* results);
int mppi_batch_destroy(mppi_engine* engine, mppi_batch* batch);

/* For callers that cannot allocate device memory: code that sets up HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same blocking solve as mppi_step (same request, result, statuses and
 * kernels, on the engine's stream), but the solve's device buffers live in a
 * library-owned static device array of MPPI_NOALLOC_SCRATCH_BYTES per device
 * instead of the engine's pool: the call allocates no device or pinned host
 * memory (its host staging is pinned once in mppi_create) and does not count
 * against the admission budget.  ENOMEM when the solve needs more than the
 * array, i.e. when mppi_solve_footprint(engine, K, T, G) exceeds
 * MPPI_NOALLOC_SCRATCH_BYTES; EINVAL when the result asks for samples,
 * positions or field values (mppi_step exports them).  Every engine of the process on that
 * device shares the array and it keeps the last call's contents: the library
 * serialises these calls per device (overlapping calls wait; each process has
 * its own array). */
#define MPPI_NOALLOC_SCRATCH_BYTES (16u << 20)
int mppi_step_noalloc(mppi_engine* engine, const mppi_request* request, mppi_result* result);

#ifdef __cplusplus
}
#endif

#endif /* MPPI_H */
