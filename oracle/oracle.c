/*
 * DBaS-Log-MPPI reference oracle (FP64, CPU).  TEST INFRASTRUCTURE ONLY:
 * see oracle.h for the scope rule and the list of paper passages followed.
 *
 * Plain loops, libm, no reordering beyond what the equations state.  The loop
 * order is Algorithm 1's: sample the noise, roll every sample out with the
 * barrier-state-augmented dynamics while accumulating its cost, form the
 * min-shifted exponential weights, take the weighted average of the noise,
 * then shift the warm start.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;

int orc_set_threads(int n)
{
#ifdef _OPENMP
    g_threads = n < 1 ? 1 : n;
#else
    (void)n;
    g_threads = 1;
#endif
    return g_threads;
}

int orc_threads(void) { return g_threads; }

int orc_state_dim(int model)
{
    switch (model) {
    case ORC_QUAD6: return 6;
    case ORC_QUAD5: return 5;
    case ORC_CAR: return 4;
    default: return 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two  */
/* 32x32->64 multiplies with the round keys bumped by the Weyl constants.     */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_uniform(uint32_t r)
{
    /* 23 high bits, centred in their cell: exact in binary32 and binary64. */
    return ((double)(r >> 9) + 0.5) * ldexp(1.0, -23);
}

/* Counter map: one Philox block per (sample k, step t) covers both inputs.
 * ctr = (k, t, counter_lo, counter_hi), key = (seed_lo, seed_hi). */
static void noise_block(const orc_cfg* cfg, uint64_t counter, int k, int t, uint32_t r[4])
{
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)t, (uint32_t)counter, (uint32_t)(counter >> 32)};
    uint32_t key[2] = {(uint32_t)cfg->seed, (uint32_t)(cfg->seed >> 32)};
    orc_philox4x32_10(ctr, key, r);
}

void orc_noise_words(const orc_cfg* cfg, uint64_t counter, uint32_t* words)
{
    for (int k = 0; k < cfg->K; ++k)
        for (int t = 0; t < cfg->T; ++t)
            noise_block(cfg, counter, k, t, words + ((size_t)k * cfg->T + t) * 4);
}

/* Sec. IV-C: Z = X1 * X2 with X1 normal and X2 log-normal.  Per Algorithm 1
 * the normal part is N(0, S_e Sigma_u), i.e. standard deviation
 * sqrt(S_e) sigma_c; the log-normal factor is exp(mu_ln + sigma_ln z) with an
 * independent standard normal z.  Standard normals come from the Box-Muller
 * transform of two uniforms each.  Vanilla MPPI's sampling (ORC_SAMPLE_NORMAL)
 * is the normal part alone. */
static void noise_sample(const orc_cfg* cfg, double S_e, uint64_t counter, int k, double* du_k)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int t = 0; t < cfg->T; ++t) {
        uint32_t r[4];
        noise_block(cfg, counter, k, t, r);
        double u0 = orc_uniform(r[0]), u1 = orc_uniform(r[1]);
        double u2 = orc_uniform(r[2]), u3 = orc_uniform(r[3]);
        double rad_n = sqrt(-2.0 * log(u0));
        double rad_z = sqrt(-2.0 * log(u2));
        double n[2] = {rad_n * cos(two_pi * u1), rad_n * sin(two_pi * u1)};
        double z[2] = {rad_z * cos(two_pi * u3), rad_z * sin(two_pi * u3)};
        for (int c = 0; c < ORC_M; ++c) {
            double normal_part = sqrt(S_e) * cfg->sigma[c] * n[c];
            if (cfg->sampling == ORC_SAMPLE_NORMAL) {
                du_k[t * ORC_M + c] = normal_part;
            } else {
                double lognormal_part = exp(cfg->mu_ln + cfg->sigma_ln * z[c]);
                du_k[t * ORC_M + c] = normal_part * lognormal_part;
            }
        }
    }
}

void orc_noise(const orc_cfg* cfg, double S_e, uint64_t counter, double* du)
{
    int k;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (k = 0; k < cfg->K; ++k) noise_sample(cfg, S_e, counter, k, du + (size_t)k * cfg->T * ORC_M);
}

/* ------------------------------------------------------------------------ */
/* Dynamics (eq. dynamics, Sec. V-A and V-B).  Explicit Euler: every new     */
/* component is computed from the old state.  The input limits the paper    */
/* gives are applied here, as actuator saturation inside f.                  */
/* ------------------------------------------------------------------------ */
static double clampd(double v, double lo, double hi)
{
    if (v < lo) return lo;
    if (v > hi) return hi;
    return v;
}

void orc_dynamics(const orc_cfg* cfg, const double* x, const double* v, double* xn)
{
    double u0 = clampd(v[0], cfg->u_min[0], cfg->u_max[0]);
    double u1 = clampd(v[1], cfg->u_min[1], cfg->u_max[1]);
    double dt = cfg->dt;
    if (cfg->model == ORC_QUAD6) {
        /* state (x, z, theta, vx, vz, omega); inputs: per-rotor thrust
         * deviations from hover, F_i = m g / 2 + u_i. */
        double m = cfg->mass, g = cfg->gravity;
        double F1 = 0.5 * m * g + u0;
        double F2 = 0.5 * m * g + u1;
        double th = x[2];
        xn[0] = x[0] + x[3] * dt;
        xn[1] = x[1] + x[4] * dt;
        xn[2] = x[2] + x[5] * dt;
        xn[3] = x[3] - (F1 + F2) / m * sin(th) * dt;
        xn[4] = x[4] + ((F1 + F2) / m * cos(th) - g) * dt;
        xn[5] = x[5] + (F2 - F1) * cfg->arm / cfg->inertia * dt;
    } else if (cfg->model == ORC_QUAD5) {
        /* Sec. V-A as printed: state (x, z, theta, vx, vz), inputs (pitch
         * rate omega, throttle u_t). */
        double m = cfg->mass, g = cfg->gravity;
        double th = x[2];
        double acc = (m * g + u1) / m;
        xn[0] = x[0] + x[3] * dt;
        xn[1] = x[1] + x[4] * dt;
        xn[2] = x[2] + u0 * dt;
        xn[3] = x[3] - acc * sin(th) * dt;
        xn[4] = x[4] + (acc * cos(th) - g) * dt;
    } else {
        /* Sec. V-B Ackermann model: state (x, y, theta, v), inputs
         * (steering phi, acceleration a). */
        double th = x[2], vel = x[3];
        xn[0] = x[0] + vel * cos(th) * dt;
        xn[1] = x[1] + vel * sin(th) * dt;
        xn[2] = x[2] + vel * tan(u0) / cfg->wheelbase * dt;
        xn[3] = x[3] + u1 * dt;
    }
}

/* Shape points: body-frame offset (s_along, s_normal) rotated by the heading
 * theta = x[2] and added to the position (x[0], x[1]). */
void orc_shape_points(const orc_cfg* cfg, const double* x, double* pts)
{
    double c = cos(x[2]), s = sin(x[2]);
    for (int i = 0; i < cfg->P; ++i) {
        double a = cfg->shape[i][0], b = cfg->shape[i][1];
        pts[2 * i] = x[0] + a * c - b * s;
        pts[2 * i + 1] = x[1] + a * s + b * c;
    }
}

/* Costmap reading: cell (col i, row j) holds the signed distance at its
 * centre (x0 + (i + 1/2) res, y0 + (j + 1/2) res); bilinear between centres,
 * clamped to the edge cells. */
double orc_sdf_lookup(const orc_world* w, double px, double py)
{
    double gx = (px - w->map_x0) / w->map_res - 0.5;
    double gy = (py - w->map_y0) / w->map_res - 0.5;
    gx = clampd(gx, 0.0, (double)(w->map_w - 1));
    gy = clampd(gy, 0.0, (double)(w->map_h - 1));
    int i0 = (int)floor(gx), j0 = (int)floor(gy);
    if (i0 > w->map_w - 2) i0 = w->map_w - 2;
    if (j0 > w->map_h - 2) j0 = w->map_h - 2;
    double fx = gx - i0, fy = gy - j0;
    const double* s = w->sdf;
    double s00 = s[(size_t)j0 * w->map_w + i0], s01 = s[(size_t)j0 * w->map_w + i0 + 1];
    double s10 = s[(size_t)(j0 + 1) * w->map_w + i0], s11 = s[(size_t)(j0 + 1) * w->map_w + i0 + 1];
    double top = (1.0 - fx) * s00 + fx * s01;
    double bot = (1.0 - fx) * s10 + fx * s11;
    return (1.0 - fy) * top + fy * bot;
}

/* Barrier function B (Sec. III-B): the inverse barrier 1/h, positive on the
 * safe set and unbounded at its boundary, evaluated at max(h, h_eps) so a
 * sampled collision gives a large finite value. */
static double barrier(const orc_cfg* cfg, double h)
{
    return 1.0 / (h > cfg->h_eps ? h : cfg->h_eps);
}

/* Fused barrier: the sum over all shape points and all constraints of B(h),
 * with h_ij = |p_i - c_j|^2 - r_j^2 for circular obstacles (Sec. V-A, V-B)
 * and h = sdf(p_i) for the costmap. */
double orc_fused_barrier(const orc_cfg* cfg, const orc_world* w, const double* x)
{
    double pts[2 * ORC_PMAX];
    orc_shape_points(cfg, x, pts);
    double sum = 0.0;
    for (int i = 0; i < cfg->P; ++i) {
        for (int j = 0; j < w->J; ++j) {
            double dx = pts[2 * i] - w->obs[3 * j];
            double dy = pts[2 * i + 1] - w->obs[3 * j + 1];
            double r = w->obs[3 * j + 2];
            double h = dx * dx + dy * dy - r * r;
            sum += barrier(cfg, h);
        }
        if (w->sdf != NULL && w->map_w > 0) sum += barrier(cfg, orc_sdf_lookup(w, pts[2 * i], pts[2 * i + 1]));
    }
    return sum;
}

/* Clearance of state x: the smallest h over all shape points and constraints
 * (INFINITY when there is none).  A diagnostic for the comparison tolerance,
 * not part of the controller. */
double orc_clearance(const orc_cfg* cfg, const orc_world* w, const double* x)
{
    double pts[2 * ORC_PMAX];
    orc_shape_points(cfg, x, pts);
    double m = INFINITY;
    for (int i = 0; i < cfg->P; ++i) {
        for (int j = 0; j < w->J; ++j) {
            double dx = pts[2 * i] - w->obs[3 * j];
            double dy = pts[2 * i + 1] - w->obs[3 * j + 1];
            double r = w->obs[3 * j + 2];
            double h = dx * dx + dy * dy - r * r;
            if (h < m) m = h;
        }
        if (w->sdf != NULL && w->map_w > 0) {
            double h = orc_sdf_lookup(w, pts[2 * i], pts[2 * i + 1]);
            if (h < m) m = h;
        }
    }
    return m;
}

/* Partial derivatives of the bilinear costmap reading at (px, py), from the
 * cell the lookup uses (zero along an axis where the point is clamped to the
 * edge). */
static void sdf_partials(const orc_world* w, double px, double py, double* dx_out, double* dy_out)
{
    double gx = (px - w->map_x0) / w->map_res - 0.5;
    double gy = (py - w->map_y0) / w->map_res - 0.5;
    int clamped_x = gx < 0.0 || gx > (double)(w->map_w - 1);
    int clamped_y = gy < 0.0 || gy > (double)(w->map_h - 1);
    gx = clampd(gx, 0.0, (double)(w->map_w - 1));
    gy = clampd(gy, 0.0, (double)(w->map_h - 1));
    int i0 = (int)floor(gx), j0 = (int)floor(gy);
    if (i0 > w->map_w - 2) i0 = w->map_w - 2;
    if (j0 > w->map_h - 2) j0 = w->map_h - 2;
    double fx = gx - i0, fy = gy - j0;
    const double* s = w->sdf;
    double s00 = s[(size_t)j0 * w->map_w + i0], s01 = s[(size_t)j0 * w->map_w + i0 + 1];
    double s10 = s[(size_t)(j0 + 1) * w->map_w + i0], s11 = s[(size_t)(j0 + 1) * w->map_w + i0 + 1];
    *dx_out = clamped_x ? 0.0 : ((1.0 - fy) * (s01 - s00) + fy * (s11 - s10)) / w->map_res;
    *dy_out = clamped_y ? 0.0 : ((1.0 - fx) * (s10 - s00) + fx * (s11 - s01)) / w->map_res;
}

/* Steepest slope of B(h) = 1/max(h, h_eps) over [h - d, h + d]: 1/(h - d)^2
 * at the near end when the interval stays above h_eps, 1/h_eps^2 when it
 * reaches the cap from above, 0 when it lies below the cap (B is flat there). */
static double barrier_slope(const orc_cfg* cfg, double h, double d)
{
    if (h + d <= cfg->h_eps) return 0.0;
    double lo = h - d > cfg->h_eps ? h - d : cfg->h_eps;
    return 1.0 / (lo * lo);
}

/* Sensitivity of the fused barrier at state x: a bound on its change per
 * metre when every shape point moves by at most r = sens_reach in each
 * coordinate.  A term's h then moves by at most d = r (|dh/dp_x| +
 * |dh/dp_y|), with dh/dp = 2 (p - c) for a circle and the bilinear reading's
 * partials for the costmap, and its B by at most d times the steepest slope
 * of B within [h - d, h + d].  With r = 0 the sum is the largest first-order
 * change, over the unclamped terms of |dB/dp_x| + |dB/dp_y|.  A diagnostic
 * for the comparison tolerance, not part of the controller. */
double orc_barrier_sensitivity(const orc_cfg* cfg, const orc_world* w, const double* x)
{
    double pts[2 * ORC_PMAX];
    orc_shape_points(cfg, x, pts);
    const double r = cfg->sens_reach;
    double s = 0.0;
    for (int i = 0; i < cfg->P; ++i) {
        for (int j = 0; j < w->J; ++j) {
            double dx = pts[2 * i] - w->obs[3 * j];
            double dy = pts[2 * i + 1] - w->obs[3 * j + 1];
            double rad = w->obs[3 * j + 2];
            double h = dx * dx + dy * dy - rad * rad;
            double g = 2.0 * (fabs(dx) + fabs(dy));
            s += g * barrier_slope(cfg, h, r * g);
        }
        if (w->sdf != NULL && w->map_w > 0) {
            double h = orc_sdf_lookup(w, pts[2 * i], pts[2 * i + 1]);
            double gx, gy;
            sdf_partials(w, pts[2 * i], pts[2 * i + 1], &gx, &gy);
            double g = fabs(gx) + fabs(gy);
            s += g * barrier_slope(cfg, h, r * g);
        }
    }
    return s;
}

/* Sec. IV-A: the constraint set is h >= 0 for every shape point and every
 * constraint; Vanilla MPPI's indicator marks a state that leaves it. */
int orc_collision(const orc_cfg* cfg, const orc_world* w, const double* x)
{
    return orc_clearance(cfg, w, x) < 0.0 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Rollout of one sample (Algorithm 1, the inner loop; eq. MPPI_BaS,         */
/* eq. barrier_update, eq. cost-to-go_bas).                                  */
/* With the indicator cost (the comparison controllers of Sec. V) there is   */
/* no barrier state: R_B beta is replaced by w_I 1[x_t violates a            */
/* constraint].                                                              */
/*   beta_0 = fused B(h(x0))                                                 */
/*   for t = 0..T-1:  v = U_t + du_t;  x <- f(x, v)                           */
/*       beta <- fused B(h(x)) - gamma_B (beta_d - beta)                     */
/*       S += q(x) + gamma_u U_t^T S_e^-1 Sigma_u^-1 v + R_B beta             */
/*   S += phi(x)                                                             */
/* q and phi are diagonal quadratics to the reference: q at step t uses      */
/* x_ref[t+1], phi uses x_ref[T].  A channel with sigma = 0 carries no noise */
/* and no control cost (Sigma_u^-1 restricted to the sampled channels).      */
/* ------------------------------------------------------------------------ */
double orc_rollout_one(const orc_cfg* cfg, const orc_world* w, const double* x0,
                       const double* U, const double* du_k, const double* x_ref,
                       double S_e, double beta_d, double* X, double* beta_out, double* min_h, double* sens)
{
    int n = orc_state_dim(cfg->model);
    if (min_h) *min_h = INFINITY;
    if (sens) *sens = 0.0;
    double x[ORC_NMAX], xn[ORC_NMAX];
    for (int a = 0; a < n; ++a) x[a] = x0[a];
    if (X) for (int a = 0; a < n; ++a) X[a] = x[a];
    const int dbas = cfg->cost_mode != ORC_COST_INDICATOR;
    double beta = dbas ? orc_fused_barrier(cfg, w, x) : 0.0;
    if (beta_out) beta_out[0] = beta;
    double S = 0.0;
    for (int t = 0; t < cfg->T; ++t) {
        double v[ORC_M];
        for (int c = 0; c < ORC_M; ++c) v[c] = U[t * ORC_M + c] + du_k[t * ORC_M + c];
        orc_dynamics(cfg, x, v, xn);
        for (int a = 0; a < n; ++a) x[a] = xn[a];
        double collision_term;
        if (dbas) {
            double b = orc_fused_barrier(cfg, w, x);
            beta = b - cfg->gamma_b * (beta_d - beta);
            collision_term = cfg->r_b * beta;
        } else {
            collision_term = cfg->collision_weight * (double)orc_collision(cfg, w, x);
        }
        const double* ref = x_ref + (size_t)(t + 1) * n;
        double q = 0.0;
        for (int a = 0; a < n; ++a) q += cfg->Q[a] * (x[a] - ref[a]) * (x[a] - ref[a]);
        double ctrl = 0.0;
        for (int c = 0; c < ORC_M; ++c)
            if (cfg->sigma[c] > 0.0)
                ctrl += U[t * ORC_M + c] * v[c] / (S_e * cfg->sigma[c] * cfg->sigma[c]);
        S += q + cfg->gamma_u * ctrl + collision_term;
        if (X) for (int a = 0; a < n; ++a) X[(size_t)(t + 1) * n + a] = x[a];
        if (beta_out) beta_out[t + 1] = beta;
        if (min_h) {
            double h = orc_clearance(cfg, w, x);
            if (h < *min_h) *min_h = h;
        }
        /* a change db_t of the fused barrier reaches the cost through
         * beta_t, beta_t+1, ... with weights summing to at most 1/(1-gamma_B) */
        if (sens && dbas) *sens += cfg->r_b / (1.0 - cfg->gamma_b) * orc_barrier_sensitivity(cfg, w, x);
    }
    const double* refT = x_ref + (size_t)cfg->T * n;
    double phi = 0.0;
    for (int a = 0; a < n; ++a) phi += cfg->Qf[a] * (x[a] - refT[a]) * (x[a] - refT[a]);
    return S + phi;
}

/* Sec. IV-B, eq. scaling factor, evaluated as the closing loop of
 * Algorithm 1 does: after the update, the augmented state is rolled out under
 * U* alone (no noise; inputs saturated inside f), its barrier state follows
 * eq. barrier_update from beta_0 = B(h(x0)), the barrier cost adds R_B beta_t
 * for t = 1..T, and the next exploration rate is mu ln(e + C_B), e = exp(1).
 * Reading: the paper takes the barrier state as positive; when beta_d makes
 * C_B negative, the logarithm sees 0, so S_e >= mu. */
double orc_exploration(const orc_cfg* cfg, const orc_world* w, const double* x0, const double* Ustar,
                       double beta_d, double mu, double* C_B_out)
{
    const int n = orc_state_dim(cfg->model);
    double x[ORC_NMAX], xn[ORC_NMAX];
    for (int a = 0; a < n; ++a) x[a] = x0[a];
    double beta = orc_fused_barrier(cfg, w, x);
    double C_B = 0.0;
    for (int t = 0; t < cfg->T; ++t) {
        orc_dynamics(cfg, x, Ustar + (size_t)t * ORC_M, xn);
        for (int a = 0; a < n; ++a) x[a] = xn[a];
        beta = orc_fused_barrier(cfg, w, x) - cfg->gamma_b * (beta_d - beta);
        C_B += cfg->r_b * beta;
    }
    if (C_B_out) *C_B_out = C_B;
    return mu * log(exp(1.0) + (C_B > 0.0 ? C_B : 0.0));
}

void orc_margins(const orc_cfg* cfg, const orc_world* w, const double* x0, const double* U, const double* du,
                 double* margin)
{
    const int n = orc_state_dim(cfg->model);
    int k;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (k = 0; k < cfg->K; ++k) {
        double x[ORC_NMAX], xn[ORC_NMAX];
        for (int a = 0; a < n; ++a) x[a] = x0[a];
        double m = INFINITY;
        for (int t = 0; t < cfg->T; ++t) {
            double v[ORC_M];
            for (int c = 0; c < ORC_M; ++c)
                v[c] = U[t * ORC_M + c] + du[((size_t)k * cfg->T + t) * ORC_M + c];
            orc_dynamics(cfg, x, v, xn);
            for (int a = 0; a < n; ++a) x[a] = xn[a];
            double h = fabs(orc_clearance(cfg, w, x));
            if (h < m) m = h;
        }
        margin[k] = m;
    }
}

/* eq. control_update: rho = min_k S_k; e_k = exp(-(S_k - rho)/lambda);
 * w_k = e_k / sum e.  A non-finite cost gets weight 0; if no cost is finite
 * the iteration is numerically failed. */
int orc_weights(const double* S, int K, double lambda, double* w, double* rho_out, double* eta_out)
{
    double rho = INFINITY;
    int any = 0;
    for (int k = 0; k < K; ++k)
        if (isfinite(S[k]) && S[k] < rho) { rho = S[k]; any = 1; }
    if (!any) {
        for (int k = 0; k < K; ++k) w[k] = 0.0;
        if (rho_out) *rho_out = NAN;
        if (eta_out) *eta_out = 0.0;
        return ORC_NUMERIC;
    }
    double eta = 0.0;
    for (int k = 0; k < K; ++k) {
        w[k] = isfinite(S[k]) ? exp(-(S[k] - rho) / lambda) : 0.0;
        eta += w[k];
    }
    for (int k = 0; k < K; ++k) w[k] /= eta;
    if (rho_out) *rho_out = rho;
    if (eta_out) *eta_out = eta;
    return ORC_OK;
}

void orc_update(const double* U, const double* du, const double* w, int K, int T, double* Ustar)
{
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < ORC_M; ++c) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc += w[k] * du[((size_t)k * T + t) * ORC_M + c];
            Ustar[t * ORC_M + c] = U[t * ORC_M + c] + acc;
        }
}

/* Algorithm 1, the closing loop: u_{t-1} <- u_t, then the last control is
 * (re)initialised once.  Reading: "Initialize" repeats the old last control
 * (or sets it to zero when configured). */
void orc_shift(const orc_cfg* cfg, const double* Ustar, double* Unext)
{
    int T = cfg->T;
    for (int t = 0; t + 1 < T; ++t)
        for (int c = 0; c < ORC_M; ++c) Unext[t * ORC_M + c] = Ustar[(t + 1) * ORC_M + c];
    for (int c = 0; c < ORC_M; ++c)
        Unext[(T - 1) * ORC_M + c] = cfg->init_zero ? 0.0 : Ustar[(T - 1) * ORC_M + c];
}

int orc_step(const orc_cfg* cfg, const orc_world* w, const double* x0, const double* U,
             const double* x_ref, double S_e, uint64_t counter,
             double* du_out, double* S_out, double* w_out, double* Ustar, double* Unext, double* u0,
             double* rho, double* eta, double* beta0_out, double* beta_d_out, double* clear, double* sens)
{
    int K = cfg->K, T = cfg->T, n = orc_state_dim(cfg->model);
    double* du = du_out ? du_out : (double*)malloc(sizeof(double) * (size_t)K * T * ORC_M);
    double* S = S_out ? S_out : (double*)malloc(sizeof(double) * (size_t)K);
    double* wt = w_out ? w_out : (double*)malloc(sizeof(double) * (size_t)K);

    /* Desired equilibrium x_d = the last reference state; beta_d = B(h(x_d)). */
    double beta_d = orc_fused_barrier(cfg, w, x_ref + (size_t)T * n);
    if (beta_d_out) *beta_d_out = beta_d;
    if (beta0_out) *beta0_out = orc_fused_barrier(cfg, w, x0);

    orc_noise(cfg, S_e, counter, du);
    int k;
#pragma omp parallel for schedule(dynamic, 16) num_threads(g_threads)
    for (k = 0; k < K; ++k)
        S[k] = orc_rollout_one(cfg, w, x0, U, du + (size_t)k * T * ORC_M, x_ref, S_e, beta_d, NULL, NULL,
                               clear ? clear + k : NULL, sens ? sens + k : NULL);
    int status = orc_weights(S, K, cfg->lambda, wt, rho, eta);
    if (status == ORC_OK) {
        orc_update(U, du, wt, K, T, Ustar);
        orc_shift(cfg, Ustar, Unext);
    } else {
        memcpy(Ustar, U, sizeof(double) * (size_t)T * ORC_M);
        memcpy(Unext, U, sizeof(double) * (size_t)T * ORC_M);
    }
    for (int c = 0; c < ORC_M; ++c) u0[c] = Ustar[c];

    if (!du_out) free(du);
    if (!S_out) free(S);
    if (!w_out) free(wt);
    return status;
}
