/*
 * dbas_mppi.h -- C ABI of the MI355X (gfx950) DBaS-Log-MPPI library.
 *
 * One call of mppi_step runs one iteration of the sampling-based controller of
 * Wang, Jiang, Tao, Wan and Cheng, "DBaS-Log-MPPI: Efficient and Safe Trajectory Optimization via
 * Barrier States": draw K normal x log-normal perturbation sequences of
 * horizon T (Sec. IV-C), roll the barrier-state-augmented dynamics out for
 * every sample while accumulating the cost-to-go (Sec. IV-A, eq.
 * cost-to-go_bas; Algorithm 1), form the min-shifted exponential weights and
 * the weighted-average update of the control sequence (Sec. III-A, eq.
 * control_update), optionally smoothed along the horizon (Algorithm 1's
 * Savitzky-Golay filter), hand u0* out and shift the warm start (Algorithm 1,
 * closing loop).  The exploration rate S_e (Sec. IV-B) is either set by the
 * caller or, with adaptive_explore, recomputed after every iteration from the
 * barrier cost of U* (eq. scaling factor).
 *
 * Conventions for every call:
 *  - Plain C types only.  Pointers are host pointers unless the argument says
 *    "device" or a `mem` argument selects MPPI_MEM_DEVICE.
 *  - The library copies whatever it keeps; the caller owns its buffers and may
 *    free them when the call returns (for *_async calls: once the stream work
 *    has completed).
 *  - Every call returns an mppi_status (or void for destroy).  No exception or
 *    abort crosses the ABI.  After an error, mppi_last_error(handle) describes
 *    it.  A device error (MPPI_E_DEVICE) poisons the handle: every later call on
 *    it returns MPPI_E_DEVICE.
 *  - A handle is not thread-safe; distinct handles may be used from distinct
 *    threads.
 *
 * Layouts:  states are float[n] with n = 6 (QUAD6: x, z, theta, vx, vz,
 * omega), 5 (QUAD5: x, z, theta, vx, vz) or 4 (CAR: x, y, theta, v).  Every
 * model has m = 2 inputs: QUAD6 (thrust deviation of rotor 1, rotor 2) from
 * hover, QUAD5 (pitch rate, throttle), CAR (steering angle, acceleration).
 * Control sequences are float[T][2] row-major; references float[T+1][n].
 */
#ifndef DBAS_MPPI_H
#define DBAS_MPPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_ABI_VERSION 2u
#define MPPI_M 2          /* inputs per model */
#define MPPI_NMAX 6       /* largest state dimension */
#define MPPI_PMAX 16      /* most body shape points */
#define MPPI_JMAX 2048    /* most circular obstacles per controller */
#define MPPI_TMAX 1024    /* longest horizon */
#define MPPI_KMAX 262144  /* most samples */

typedef enum {
    MPPI_OK = 0,
    MPPI_E_INVALID = 1,   /* bad argument or configuration; nothing was launched */
    MPPI_E_NOMEM = 2,     /* a device or pinned-host allocation failed */
    MPPI_E_DEVICE = 3,    /* a HIP call failed; the handle is poisoned */
    MPPI_E_NUMERIC = 4,   /* no sample had a finite cost; U and the counter are unchanged */
    MPPI_E_BUSY = 5       /* (server) result not ready yet / no capacity */
} mppi_status;

typedef enum { MPPI_QUAD6 = 0, MPPI_QUAD5 = 1, MPPI_CAR = 2 } mppi_model;
typedef enum { MPPI_NORM_AUTO = 0, MPPI_NORM_ON = 1, MPPI_NORM_OFF = 2 } mppi_normaliser;
typedef enum { MPPI_INIT_REPEAT = 0, MPPI_INIT_ZERO = 1 } mppi_init_mode;
typedef enum { MPPI_MEM_HOST = 0, MPPI_MEM_DEVICE = 1 } mppi_mem;
/* Sampling law of the perturbations (Sec. IV-C; Sec. V's Vanilla baseline). */
typedef enum { MPPI_SAMPLE_NLN = 0, MPPI_SAMPLE_NORMAL = 1 } mppi_sampling;
/* Collision term of the running cost (Sec. IV-A). */
typedef enum { MPPI_COST_DBAS = 0, MPPI_COST_INDICATOR = 1 } mppi_cost_mode;

/*
 * Problem statement (Sec. III-A eq. mppi; Algorithm 1's Require list; Sec.
 * IV-B/IV-C sampling parameters; Sec. V-A/V-B models, limits, shape points).
 *  - sigma[c]: standard deviation of channel c, Sigma_u = diag(sigma^2); a
 *    channel with sigma = 0 is not sampled and carries no control cost.
 *  - Noise: du = sqrt(S_e) sigma_c n exp(mu_ln + sigma_ln z) with n, z
 *    independent standard normals (Sec. IV-C mixture, scaled per Alg. 1).
 *  - lambda > 0: temperature of exp(-(S - rho)/lambda).
 *  - gamma_u: control-cost weight of gamma_u U_t^T S_e^-1 Sigma_u^-1 v_t.
 *  - gamma_b in (0,1): barrier-state relaxation of eq. barrier_update.
 *  - r_b: R_B, weight of the barrier state in the running cost.
 *  - h_eps > 0: the barrier is B(h) = 1/max(h, h_eps).
 *  - Q, Qf: diagonal running and terminal weights on (x - x_ref).
 *  - shape[P][2]: body-frame shape points (along the heading, normal to it).
 *    The bodies of Sec. V run a faster form of the barrier: for the vehicle,
 *    8 points at the corners and side midpoints of a centred rectangle, in
 *    the order (a,b), (a,-b), (-a,b), (-a,-b), (a,0), (-a,0), (0,b), (0,-b);
 *    for the quadrotors, 7 points on the body axis (second coordinate 0),
 *    faster still when points 0, 1, 2 mirror points 6, 5, 4 about the
 *    centre.  Any other shape is accepted and computed in the general form.
 *  - u_min/u_max: actuator limits, applied inside the dynamics.
 *  - h_eps in [1e-9, 1e6].
 *  - tile_samples: samples per rollout workgroup (16, 32, 64, 128 or 256);
 *    0 chooses per shape (model, K, T, J, P, costmap, smoothing, cost
 *    mode): from the process cache, the MPPI_TUNE_CACHE file, the
 *    tile_table.txt shipped beside the library, else by timing the
 *    candidates (and appending the choice to the cache file).  The choice is
 *    made again when the obstacle count changes or a costmap is set or
 *    cleared.  The tile size fixes the order of the tile's reductions, so a
 *    shape found in a table gives the same results in every process.
 *  - export_noise: 0 (default) -- the noise lives only inside the rollout
 *    kernel and is never stored; 1 -- every iteration also writes it to
 *    device memory (K*T*8 bytes) so that mppi_get_noise can return it.
 *  - adaptive_explore: 0 (default) -- S_e stays as mppi_set_exploration set
 *    it (1 at creation); 1 -- after every iteration U* is rolled out once
 *    without noise from x0, its barrier cost C_B = sum_{t=1..T} R_B beta_t
 *    is formed, and the next iteration samples with
 *    S_e = explore_mu ln(e + max(C_B, 0)) (Sec. IV-B eq. scaling factor and
 *    the closing loop of Algorithm 1).  explore_mu in (0, 1), default 0.4.
 *  - sgf_half_window m, sgf_order p: Algorithm 1 smooths the weighted
 *    increment sum_k w_k du_k along the horizon with a Savitzky-Golay filter
 *    before adding it to U.  Every step t takes the value at t of the
 *    least-squares polynomial of degree p through the 2m+1 steps of its
 *    window; near the ends of the horizon the window is the first (last)
 *    2m+1 steps.  m = 0 (default) applies no smoothing; m > 0 needs
 *    T >= 2m+1, m <= 16 and 0 <= p <= min(2m, 8).
 *  - sampling, cost_mode, collision_weight: the paper's controller and its
 *    two baselines (Sec. IV-A, Sec. V and its mission table) are modes of the
 *    same iteration.  sampling = MPPI_SAMPLE_NLN (default) draws the normal x
 *    log-normal mixture; MPPI_SAMPLE_NORMAL draws its normal part alone,
 *    du = sqrt(S_e) sigma_c n (Vanilla MPPI).  cost_mode = MPPI_COST_DBAS
 *    (default) carries the barrier state and adds R_B beta_t; with
 *    MPPI_COST_INDICATOR there is no barrier state and every step adds
 *    collision_weight (finite, >= 0) when some shape point violates a
 *    constraint (h < 0 for a circle or the costmap), the weighted indicator
 *    of Vanilla MPPI and Log-MPPI.  Vanilla MPPI = (NORMAL, INDICATOR),
 *    Log-MPPI = (NLN, INDICATOR), DBaS-Log-MPPI = (NLN, DBAS) with
 *    adaptive_explore.  The indicator mode does not take adaptive_explore
 *    (its rate follows the barrier cost).
 */
typedef struct mppi_config {
    uint32_t abi_version;          /* must be MPPI_ABI_VERSION */
    int32_t model;                 /* mppi_model */
    int32_t K, T;                  /* samples (1..MPPI_KMAX), horizon (1..MPPI_TMAX) */
    float dt;
    float mass, gravity, arm, inertia, wheelbase;
    float u_min[MPPI_M], u_max[MPPI_M];
    float sigma[MPPI_M];
    float mu_ln, sigma_ln;
    float lambda, gamma_u, gamma_b, r_b, h_eps;
    float Q[MPPI_NMAX], Qf[MPPI_NMAX];
    int32_t P;
    float shape[MPPI_PMAX][2];
    uint64_t seed;                 /* Philox key */
    int32_t normaliser;            /* mppi_normaliser */
    int32_t init_mode;             /* mppi_init_mode */
    int32_t tile_samples;          /* 0 = autotune */
    int32_t export_noise;          /* 1: also store each iteration's noise (mppi_get_noise) */
    int32_t adaptive_explore;      /* 1: S_e follows the barrier cost of U* (Sec. IV-B) */
    float explore_mu;              /* coarseness factor mu in (0,1) of S_e = mu ln(e + C_B) */
    int32_t sgf_half_window;       /* Savitzky-Golay half window m (0: no smoothing) */
    int32_t sgf_order;             /* Savitzky-Golay polynomial order p, 0 <= p <= min(2m, 8) */
    int32_t sampling;              /* mppi_sampling */
    int32_t cost_mode;             /* mppi_cost_mode */
    float collision_weight;        /* weight of the collision indicator (MPPI_COST_INDICATOR) */
    int32_t reserved[2];           /* must be zero */
} mppi_config;

/* Where a handle runs.  stream: a hipStream_t owned by the caller (NULL: the
 * library creates its own, at default priority). */
typedef struct mppi_device {
    int32_t device;
    void* stream;
} mppi_device;

/* Checkpointable controller state: warm start U[T][2], Philox step counter,
 * exploration rate. */
typedef struct mppi_state {
    uint64_t counter;
    float S_e;
    int32_t T;
    float* U;                      /* host, T*2 floats, caller-allocated */
} mppi_state;

/* What the last completed iteration produced. */
typedef struct mppi_step_info {
    uint64_t counter;              /* counter the iteration's noise used */
    int32_t status;                /* mppi_status of the iteration */
    int32_t fp64_tiles;            /* sample tiles whose weights ran in FP64 */
    double rho;                    /* min_k S_k */
    double eta;                    /* sum_k exp(-(S_k - rho)/lambda) */
    float beta0;                   /* fused barrier at x0 */
    float beta_d;                  /* fused barrier at x_d = x_ref[T] */
    int32_t tile_samples;          /* samples per rollout workgroup used */
    int32_t tiles;                 /* sample tiles per iteration */
    float S_e;                     /* exploration rate the next iteration samples with */
    float cost_b;                  /* C_B of the last U* (adaptive_explore only, else 0) */
    int32_t barrier_form;          /* 0: the general form; 1: the layout form of Sec. V's bodies (see shape); 2: the quadrotor's mirrored-axis form */
    int32_t noise_kept;            /* 1: each rollout tile keeps its noise in LDS for the update sums; 0: it draws it again */
} mppi_step_info;

typedef struct mppi_ctrl mppi_t;

/* Fill *cfg with the defaults of `model` (the paper's limits, mass, frame,
 * inertia and shape points; sigma 0.5; lambda 1; gamma_u 2; gamma_b 0.5;
 * R_B 0.1; h_eps 1e-4; mu_ln 0, sigma_ln 0.3; Q as in the test workloads). */
int mppi_config_default(int32_t model, int32_t K, int32_t T, mppi_config* cfg);

/* Create a controller.  Allocates every device buffer it needs (sized by K, T)
 * and copies the configuration.  U starts at zero, counter at 0, S_e at 1, no
 * obstacles, no costmap, a zero reference.  Errors: INVALID (bad config),
 * NOMEM, DEVICE. */
int mppi_create(const mppi_config* cfg, const mppi_device* dev, mppi_t** out);

/* Free everything (NULL-safe).  Waits for the handle's pending work. */
void mppi_destroy(mppi_t* h);

/* Circular obstacles (Sec. V-A/V-B: h = |p - c|^2 - r^2): J rows of
 * (cx, cy, r), copied.  J = 0 clears them.  Errors: INVALID (J outside
 * 0..MPPI_JMAX, non-finite or negative r). */
int mppi_set_obstacles(mppi_t* h, int32_t J, const float* cxcyr, int32_t mem);

/* Optional signed-distance costmap, row-major sdf[H][W] in metres, cell
 * (col i, row j) centred at (x0 + (i+1/2) res, y0 + (j+1/2) res), sampled
 * bilinearly and clamped to the edge; each shape point adds B(sdf) to the
 * fused barrier.  sdf = NULL clears it.  Setting or clearing the costmap
 * chooses the tile size again (tile_samples = 0).  Errors: INVALID (W or H
 * < 2, res <= 0). */
int mppi_set_costmap(mppi_t* h, int32_t W, int32_t H, float x0, float y0, float res,
                     const float* sdf, int32_t mem);

/* Reference x_ref[T+1][n] for the running cost (step t uses x_ref[t+1]) and
 * the terminal cost (x_ref[T]); the desired equilibrium of eq.
 * barrier_update is x_d = x_ref[T]. */
int mppi_set_reference(mppi_t* h, const float* x_ref, int32_t mem);

/* Exploration rate S_e > 0 (Sec. IV-B); it scales the noise variance and
 * divides the control cost.  With adaptive_explore every iteration replaces
 * it for the next one; this call sets the rate the next iteration uses. */
int mppi_set_exploration(mppi_t* h, float S_e);

/* Overwrite the warm start U[T][2]. */
int mppi_set_controls(mppi_t* h, const float* U, int32_t mem);

/* One iteration from state x0 (host float[n]); writes u0* (host float[2]) and
 * blocks until it is available.  Errors: INVALID (non-finite x0), NUMERIC
 * (every cost non-finite: U and counter unchanged, u0 = current U[0]), DEVICE. */
int mppi_step(mppi_t* h, const float* x0, float* u0);

/* Stream-ordered iteration: x0 is a device float[n]; u0 (device float[2], may
 * be NULL) is written when the iteration completes.  Does not block.  The
 * iteration's status is read by mppi_synchronize or mppi_get_step_info. */
int mppi_step_async(mppi_t* h, const float* x0_device, float* u0_device);

/* Wait for the handle's stream; returns the status of the last iteration. */
int mppi_synchronize(mppi_t* h);

/* Inspection (host buffers, caller-allocated; each waits for the stream). */
int mppi_get_controls(mppi_t* h, float* U);              /* warm start, T*2 */
int mppi_get_last_optimal(mppi_t* h, float* Ustar);      /* U* before the shift, T*2 */
int mppi_get_costs(mppi_t* h, double* S);                /* S_k, K (compensated sum as FP64) */
int mppi_get_weights(mppi_t* h, double* w);              /* normalised weights, K */
int mppi_get_noise(mppi_t* h, float* du);                /* du[k][t][c], K*T*2; needs export_noise */
int mppi_get_step_info(mppi_t* h, mppi_step_info* info);
/* Raw Philox4x32-10 words of every (k, t) for the given counter:
 * words[(k*T + t)*4 + i], from the same device function the sampler uses. */
int mppi_get_philox_words(mppi_t* h, uint64_t counter, uint32_t* words);

/* Checkpoint / resume: a restored controller continues bit-identically. */
int mppi_get_state(mppi_t* h, mppi_state* st);
int mppi_set_state(mppi_t* h, const mppi_state* st);

const char* mppi_last_error(const mppi_t* h);
const char* mppi_status_string(int32_t status);

/* The stream (hipStream_t) a handle launches on. */
void* mppi_stream(const mppi_t* h);

/* Kernel timing.  mppi_profile_enable(h, every): with every = n > 0, every
 * n-th later iteration (the first one included) records HIP events on the
 * handle's stream around its rollout kernel and its update kernel (the
 * events themselves cost a few microseconds per recorded iteration, so a
 * period above 1 keeps timed loops close to their unprofiled speed);
 * every = 0 turns it off.
 * mppi_profile_read waits for the stream, returns the totals over the
 * iterations recorded since the last read, and clears them.  Turning it on
 * allocates events (up to 4096 iterations are kept; later ones are dropped
 * and counted in `dropped`). */
typedef struct mppi_profile {
    int64_t iterations;
    int64_t dropped;
    double rollout_ms;             /* summed rollout-kernel durations */
    double update_ms;              /* summed update-kernel durations */
} mppi_profile;

int mppi_profile_enable(mppi_t* h, int32_t every);
int mppi_profile_read(mppi_t* h, mppi_profile* out);

/* ------------------------------------------------------------------------ */
/* One iteration without a handle and without allocating: for callers that    */
/* cannot allocate device memory -- code under HIP graph capture, tight       */
/* serving loops, harnesses that forbid allocation.                           */
/* ------------------------------------------------------------------------ */

/* Bytes of the library's static per-GPU scratch array (held by each GPU the
 * library runs on until the process ends). */
#define MPPI_NOALLOC_SCRATCH_BYTES (8u << 20)

/* The world of one iteration, in caller-owned device memory (read only). */
typedef struct mppi_problem {
    int32_t J;                     /* circular obstacles, 0..MPPI_JMAX */
    const float* obs;              /* device [J][3] (cx, cy, r); NULL when J = 0 */
    int32_t map_w, map_h;          /* costmap size (>= 2 each) when sdf is not NULL */
    float map_x0, map_y0, map_res; /* costmap placement, as in mppi_set_costmap */
    const float* sdf;              /* device [map_h][map_w] signed distances, or NULL */
    const float* x_ref;            /* device [T+1][n] reference, as in mppi_set_reference */
} mppi_problem;

/* The iteration mppi_step runs for a controller of configuration `cfg`
 * whose warm start is U (device float[T][2]), Philox step counter `counter`
 * and exploration rate S_e, on the world `prob`, from state x0 (device
 * float[n]).  Writes (device buffers): U*[T][2] before the shift, the
 * shifted warm start Unext[T][2] (Algorithm 1's closing loop; equal to U
 * when the iteration fails NUMERIC), and, when not NULL, u0[2] and the
 * iteration's status (int32: MPPI_OK or MPPI_E_NUMERIC).  The next
 * iteration's counter is counter + 1 after MPPI_OK.
 * Stream-ordered on `stream` (hipStream_t, NULL: the null stream) of GPU
 * `device`; returns without waiting.  Allocates nothing: the per-iteration
 * scratch (costs, exponentials, tile partials, iteration state) is the
 * library's static array of MPPI_NOALLOC_SCRATCH_BYTES on that GPU, shared by
 * every call there, so calls on one GPU must not overlap (one stream, or a
 * wait in between); kernels only, no memset or copy, so a capture records it.
 * The tile size is cfg->tile_samples, or the heuristic one when it is 0 (no
 * timing).  Results equal mppi_step's for the same configuration and tile
 * size bit for bit.
 * Errors (nothing launched): INVALID for a bad configuration, a NULL required
 * pointer, adaptive_explore / sgf_half_window / export_noise set (they need a
 * handle), a world or horizon that does not fit the rollout's LDS, or a
 * scratch need (about 12 K + 16 T K / S + 28 K / S bytes) above
 * MPPI_NOALLOC_SCRATCH_BYTES; DEVICE for a HIP failure.  mppi_last_error(NULL)
 * describes it.  Obstacle and map values are not checked (device memory). */
int mppi_step_noalloc(const mppi_config* cfg, const mppi_problem* prob, int32_t device, void* stream,
                      const float* x0, const float* U, uint64_t counter, float S_e, float* Ustar, float* Unext,
                      float* u0, int32_t* status);

/* ------------------------------------------------------------------------ */
/* Batched iteration: many controllers (any mix of models, K, T, J) stepped  */
/* by persistent kernels (one per model and tile kind present), captured     */
/* once in a HIP graph.  Controllers stay owned by the caller and must       */
/* outlive the batch; each one's tile shape is its own (autotuned per model, */
/* K, T, J), so a controller's result is the same alone and in the batch.    */
/* ------------------------------------------------------------------------ */
typedef struct mppi_batch mppi_batch_t;

int mppi_batch_create(mppi_t* const* ctrls, int32_t n, const mppi_device* dev, mppi_batch_t** out);
void mppi_batch_destroy(mppi_batch_t* b);
/* x0s: host float[n][MPPI_NMAX] (row c holds controller c's state); u0s: host
 * float[n][2]; statuses (nullable): host int32[n].  Blocks.  Returns MPPI_OK
 * when every controller succeeded, else the first failing status. */
int mppi_batch_step(mppi_batch_t* b, const float* x0s, float* u0s, int32_t* statuses);
const char* mppi_batch_last_error(const mppi_batch_t* b);

/* ------------------------------------------------------------------------ */
/* Serving: robots submit control-step requests; a scheduler thread admits   */
/* them while launch slots and the device-memory budget allow, and batches   */
/* whatever is admitted into the next launch on one of several streams       */
/* (continuous batching).  Each robot keeps its warm start, Philox counter,  */
/* obstacles and reference resident on the device; requests of one robot run */
/* in submission order.                                                      */
/* ------------------------------------------------------------------------ */
typedef struct mppi_server mppi_server_t;

typedef struct mppi_server_config {
    uint32_t abi_version;
    int32_t device;
    int64_t budget_bytes;          /* device bytes for in-flight sample scratch */
    int32_t max_slots;             /* most requests in flight */
    int32_t streams;               /* launch streams (>= 1) */
    int32_t max_batch;             /* most requests per launch */
    int32_t reserved[7];
} mppi_server_config;

typedef struct mppi_server_stats {
    int64_t submitted, completed, launches, deferred_budget, deferred_slots;
    int64_t peak_bytes_in_flight;
    double mean_batch;
} mppi_server_stats;

int mppi_server_create(const mppi_server_config* cfg, mppi_server_t** out);
/* Stops the scheduler, waits for the launches in flight and frees everything.
 * Requests still queued are dropped; no other call on `s` may be running or
 * follow.  The server keeps each completed request until it is polled or
 * waited for. */
void mppi_server_destroy(mppi_server_t* s);
/* Register a robot.  The configuration, obstacles and costmap are copied into
 * server-owned device state.  id receives the robot index. */
int mppi_server_add_robot(mppi_server_t* s, const mppi_config* cfg, int32_t J, const float* cxcyr,
                          int32_t* id);
/* Queue one control step for robot id from state x0 (host float[n]) with
 * reference x_ref (host float[T+1][n], NULL keeps the last one).  t_arrival is
 * the caller's timestamp in seconds (monotonic clock).  ticket receives the
 * request handle. */
int mppi_server_submit(mppi_server_t* s, int32_t id, const float* x0, const float* x_ref,
                       double t_arrival, int64_t* ticket);
/* MPPI_OK and u0 (host float[2]) once the request completed, MPPI_E_BUSY while
 * it is pending.  latency (nullable) = completion time - t_arrival (s);
 * status (nullable) = the iteration's own status. */
int mppi_server_poll(mppi_server_t* s, int64_t ticket, float* u0, double* latency, int32_t* status);
/* Block until the request completed, then as poll. */
int mppi_server_wait(mppi_server_t* s, int64_t ticket, float* u0, double* latency, int32_t* status);
/* Monotonic clock of the server (s), for t_arrival. */
double mppi_server_now(const mppi_server_t* s);
int mppi_server_get_stats(mppi_server_t* s, mppi_server_stats* st);
/* Read back a robot's warm start U[T][2] and counter (for tests). */
int mppi_server_get_robot(mppi_server_t* s, int32_t id, float* U, uint64_t* counter);
const char* mppi_server_last_error(const mppi_server_t* s);

#ifdef __cplusplus
}
#endif
#endif
