/*
 * DBaS-Log-MPPI reference oracle: plain, slow, FP64 CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) includes, links or calls this code; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark do.  It shares no
 * header, helper, table or constant with the GPU implementation.
 *
 * Every function follows a named part of the paper (Wang, Jiang, Tao, Wan and Cheng, "DBaS-Log-MPPI:
 * Efficient and Safe Trajectory Optimization via Barrier States"):
 *   Sec. III-A  MPPI problem, cost-to-go, min-shifted exponential update
 *   Sec. III-B  discrete barrier states (eq. barrier_state, eq. barrier_update)
 *   Sec. IV-A   DBaS cost-to-go (eq. cost-to-go_bas)
 *   Sec. IV-B   adaptive exploration S_e (eq. scaling factor), taken as an input
 *   Sec. IV-C   normal x log-normal sampling (eq. nln mean and var)
 *   Algorithm 1 the loop order (sampling, rollout, cost, weighting, shift)
 *   Sec. V-A/B  planar quadrotor and Ackermann vehicle (eq. veh_dyn), shape
 *               points and the circular-obstacle function h
 *   Sec. IV-A, Sec. V and the mission table: the comparison controllers --
 *               Vanilla MPPI (normal sampling, weighted collision indicator)
 *               and Log-MPPI (normal x log-normal sampling, the same
 *               indicator) -- as modes of the same iteration
 * Where the paper is silent the reading used is stated at the function.
 *
 * Parity pins: every function here is pinned by the CPU tests against closed
 * forms, invariants, special cases or published known-answer vectors.  The
 * geometry and parameter choices the paper leaves open (the form of B, gamma_B,
 * the 6-state quadrotor, shape-point placement, wheelbase, the costmap lookup)
 * are "parity unpinned" by the paper itself: no printed value checks them.
 */
#ifndef DBAS_MPPI_ORACLE_H
#define DBAS_MPPI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_QUAD6 = 0, ORC_QUAD5 = 1, ORC_CAR = 2 };
enum { ORC_OK = 0, ORC_INVALID = 1, ORC_NUMERIC = 4 };
/* Sampling law of the perturbations: the normal x log-normal mixture of
 * Sec. IV-C, or the plain normal law of Vanilla MPPI. */
enum { ORC_SAMPLE_NLN = 0, ORC_SAMPLE_NORMAL = 1 };
/* Collision term of the running cost: the barrier state of Sec. IV-A, or the
 * weighted indicator of a constraint violation that Sec. IV-A describes for
 * Vanilla MPPI (and that the Log-MPPI baseline shares). */
enum { ORC_COST_DBAS = 0, ORC_COST_INDICATOR = 1 };

#define ORC_M 2          /* every model here has two inputs */
#define ORC_NMAX 6
#define ORC_PMAX 16

typedef struct {
    int model;                 /* ORC_QUAD6, ORC_QUAD5 or ORC_CAR */
    int K, T;                  /* samples, horizon */
    double dt;
    double mass, gravity, arm, inertia, wheelbase;
    double u_min[ORC_M], u_max[ORC_M];
    double sigma[ORC_M];       /* Sigma_u = diag(sigma^2) */
    double mu_ln, sigma_ln;    /* log-normal factor parameters */
    double lambda;             /* temperature in exp(-S/lambda) */
    double gamma_u;            /* control-cost weight */
    double gamma_b;            /* DBaS relaxation, in (0,1) */
    double r_b;                /* barrier-state cost weight R_B */
    double h_eps;              /* B(h) = 1/max(h, h_eps) */
    double Q[ORC_NMAX], Qf[ORC_NMAX];
    int P;                     /* number of body shape points */
    double shape[ORC_PMAX][2]; /* body-frame offsets (along heading, normal) */
    uint64_t seed;
    int init_zero;             /* 0: new last control repeats the old last, 1: zero */
    int sampling;              /* ORC_SAMPLE_NLN or ORC_SAMPLE_NORMAL */
    int cost_mode;             /* ORC_COST_DBAS or ORC_COST_INDICATOR */
    double collision_weight;   /* weight of the indicator term (ORC_COST_INDICATOR) */
    double sens_reach;         /* move per coordinate the barrier sensitivity covers (diagnostic; 0: first order) */
} orc_cfg;

typedef struct {
    int J;
    const double* obs;         /* J x 3: cx, cy, r */
    int map_w, map_h;          /* 0 = no costmap */
    double map_x0, map_y0, map_res;
    const double* sdf;         /* map_h x map_w, row-major, metres */
} orc_world;

int orc_state_dim(int model);

/* Worker threads of the per-sample loops (noise, rollouts, margins); 1 runs
 * them serially.  Every sample is computed by the same code whichever thread
 * runs it, and every cross-sample sum (weights, update) stays serial, so the
 * results do not depend on the count.  Returns the count in use. */
int orc_set_threads(int n);
int orc_threads(void);

/* Philox4x32-10 (Salmon et al., SC'11): counter ctr, key -> 4 words. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* 32-bit word -> uniform in (0,1): ((r >> 9) + 1/2) * 2^-23. */
double orc_uniform(uint32_t r);

/* Raw Philox words for every (k, t): words[(k*T + t)*4 + i]. */
void orc_noise_words(const orc_cfg* cfg, uint64_t counter, uint32_t* words);

/* Noise du[(k*T + t)*2 + c] for step counter `counter` and exploration S_e:
 * the NLN mixture, or (ORC_SAMPLE_NORMAL) its normal part alone. */
void orc_noise(const orc_cfg* cfg, double S_e, uint64_t counter, double* du);

/* One explicit-Euler step with the inputs saturated inside f. */
void orc_dynamics(const orc_cfg* cfg, const double* x, const double* v, double* xn);

/* World-frame shape points of state x: pts[2*i], pts[2*i+1]. */
void orc_shape_points(const orc_cfg* cfg, const double* x, double* pts);

/* Bilinear signed-distance lookup at world point (px, py). */
double orc_sdf_lookup(const orc_world* w, double px, double py);

/* Fused barrier sum_i sum_j B(h_ij(x)) (+ sum_i B(sdf(p_i))). */
double orc_fused_barrier(const orc_cfg* cfg, const orc_world* w, const double* x);

/* Smallest h over all shape points and constraints at state x (diagnostic). */
double orc_clearance(const orc_cfg* cfg, const orc_world* w, const double* x);

/* Bound on the change of the fused barrier at x, per metre, when every shape
 * point moves by at most r = sens_reach in each coordinate (diagnostic): the
 * sum over the terms of (|dh/dp_x| + |dh/dp_y|) times the steepest slope of
 * B = 1/max(h, h_eps) within the reach of h.  With r = 0 this is the largest
 * first-order change, sum over the unclamped terms of |dB/dp_x| + |dB/dp_y|. */
double orc_barrier_sensitivity(const orc_cfg* cfg, const orc_world* w, const double* x);

/* Collision indicator of state x: 1 when some shape point violates a
 * constraint (h < 0 for a circle or the costmap), else 0. */
int orc_collision(const orc_cfg* cfg, const orc_world* w, const double* x);

/* Rollout of one sample.  Returns its cost S.  Optional outputs:
 * X[(T+1)*n] states, beta[T+1] barrier states (beta[0] = beta_0; all zero
 * with the indicator cost), min_h the smallest clearance over steps 1..T,
 * sens the bound on |dS| per metre of shape-point displacement through the
 * barrier (0 with the indicator cost) (diagnostics for comparison
 * tolerances). */
double orc_rollout_one(const orc_cfg* cfg, const orc_world* w, const double* x0,
                       const double* U, const double* du_k, const double* x_ref,
                       double S_e, double beta_d, double* X, double* beta, double* min_h, double* sens);

/* Adaptive exploration (Sec. IV-B eq. scaling factor; closing loop of
 * Algorithm 1): the barrier cost C_B = sum_{t=1..T} R_B beta_t of the
 * noise-free rollout of U* from x0, and the next exploration rate
 * S_e = mu ln(e + C_B), returned.  C_B (optional output) is the raw sum; a
 * negative C_B (possible when beta_d is large) enters the logarithm as 0. */
double orc_exploration(const orc_cfg* cfg, const orc_world* w, const double* x0, const double* Ustar,
                       double beta_d, double mu, double* C_B);

/* Indicator margins of every sample's rollout (diagnostic for the indicator
 * cost): margin[k] = min over t = 1..T of |clearance(x_t)|, how far the
 * sample's closest decision of the indicator is from flipping. */
void orc_margins(const orc_cfg* cfg, const orc_world* w, const double* x0, const double* U, const double* du,
                 double* margin);

/* Min-shifted exponential weights.  Returns ORC_OK or ORC_NUMERIC. */
int orc_weights(const double* S, int K, double lambda, double* w, double* rho, double* eta);

/* U*[t][c] = U[t][c] + sum_k w_k du[k][t][c]. */
void orc_update(const double* U, const double* du, const double* w, int K, int T, double* Ustar);

/* Warm-start shift: Unext[t] = U*[t+1], Unext[T-1] = Initialize(U*[T-1]). */
void orc_shift(const orc_cfg* cfg, const double* Ustar, double* Unext);

/* One full iteration.  All outputs caller-allocated (any may be NULL except
 * Ustar/Unext/u0).  Returns ORC_OK or ORC_NUMERIC (then Ustar = Unext = U).
 * clear[K], sens[K] (optional): each sample's smallest clearance and barrier
 * sensitivity over its rollout (see orc_rollout_one). */
int orc_step(const orc_cfg* cfg, const orc_world* w, const double* x0, const double* U,
             const double* x_ref, double S_e, uint64_t counter,
             double* du, double* S, double* wts, double* Ustar, double* Unext, double* u0,
             double* rho, double* eta, double* beta0, double* beta_d, double* clear, double* sens);

#ifdef __cplusplus
}
#endif
#endif
