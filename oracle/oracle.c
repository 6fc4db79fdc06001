/*
 * FP64 CPU oracle for one Risk-Aware MPPI control step (RA-MPPI, Yin, Zhang
 * and Tsiotras, "Risk-Aware Model Predictive Path Integral Control Using
 * Conditional Value-at-Risk", arXiv 2209.12842).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP library: it has its own Philox4x32-10, its
 * own Box-Muller transform, its own dynamics and costs.
 *
 * Everything is computed in double precision, in the order the method states:
 *   Algorithm 1 (Risk-Aware MPPI):
 *     for every sampled control sequence: sample the control noise, apply the
 *     warm / zero-mean rule, roll the nominal model out and accumulate its
 *     cost S (Eq. 1, 3); for every disturbance draw roll the disturbed model
 *     out and accumulate the risk cost L (Eq. 6, 9); scale the risk costs
 *     (Eq. 18-19), keep the upper (1 - alpha) part and average it (Eq. 10-13);
 *     add the CVaR violation cost (Eq. 14-16); then form the weights (Eq. 17
 *     with Eq. 5) and the weighted average of the sampled controls (Eq. 4).
 *
 * Readings of the paper where it is silent or ambiguous (noise generator,
 * vehicle model, track geometry, tail size, B = 1, index ranges, shift) are
 * listed in the design notes next to this repository's sources; each one is
 * repeated at the point of use below.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -fPIC -shared oracle.c -lm (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Parameters.  Every floating value is a float32 value widened to double by  */
/* the caller, so that the oracle and the FP32 GPU path see the same inputs.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t K, T, M, n_obs;      /* samples, horizon, draws per sample, obstacles */
    double dt, wheelbase;        /* Euler step, kinematic-bicycle wheelbase */
    double u_lo[2], u_hi[2];     /* control box for (acceleration, steering) */
    double sigma_eps[2];         /* diag of the control-noise covariance (variances) */
    double sigma_w[4];           /* diag of the state-disturbance covariance (variances) */
    double alpha, lambda, gamma, eta, A, B, C_u;
    double c_bdry, c_obs, c_dev, c_v, v_ref, c4, c5;
    double track[5];             /* ellipse centre ox, oy, semi-axes a, b, half width */
    uint64_t seed;               /* Philox key = (low 32 bits, high 32 bits) */
    int32_t shift;               /* non-zero: shift the updated sequence by one step */
    int32_t noise_kind;          /* disturbance form: 0 Gaussian, 1 uniform, 2 impulse */
    double jump_prob, jump_size; /* impulse form: probability per step, jump length */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Noise.  The paper does not name a generator.  Reading: Philox4x32-10       */
/* (Salmon, Moraes, Dror, Shaw, SC'11), counter-based so that any (sample,    */
/* draw, time, call) noise can be regenerated independently.                  */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u   /* golden ratio fraction of 2^32 */
#define ORC_PHILOX_W1 0xBB67AE85u   /* (sqrt(3) - 1) fraction of 2^32 */

void orc_philox_constants(uint32_t out[4])
{
    out[0] = ORC_PHILOX_M0;
    out[1] = ORC_PHILOX_M1;
    out[2] = ORC_PHILOX_W0;
    out[3] = ORC_PHILOX_W1;
}

/* Philox4x32 with a given number of rounds.  One round multiplies words 0
 * and 2 by the two multipliers (full 64-bit products); the new words are
 * (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).  The key
 * is advanced by the two Weyl constants after every round. */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < rounds; ++r) {
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += ORC_PHILOX_W0;
        k1 += ORC_PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    orc_philox4x32(ctr, key, 10, out);
}

/* Batch form used by the statistics pins: n counters (n x 4) -> n x 4 words. */
void orc_philox_batch(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out)
{
    uint32_t key[2] = { (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32) };
    for (int64_t i = 0; i < n; ++i)
        orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* uint32 -> open interval (0, 1): the top 23 bits plus one half, times 2^-23.
 * The result has at most 24 significant bits, so it is exact in float32 too. */
double orc_uniform(uint32_t r)
{
    return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Box-Muller (Box & Muller 1958): two independent standard normals from two
 * uniforms in (0, 1). */
void orc_box_muller(double u0, double u1, double *z0, double *z1)
{
    const double two_pi = 6.283185307179586476925286766559;
    double rad = sqrt(-2.0 * log(u0));
    *z0 = rad * cos(two_pi * u1);
    *z1 = rad * sin(two_pi * u1);
}

/* Four standard normals from one Philox call: (z0, z1) from words 0 and 1,
 * (z2, z3) from words 2 and 3. */
void orc_normals4(const uint32_t ctr[4], uint64_t seed, double z[4])
{
    uint32_t key[2] = { (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32) };
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    orc_box_muller(orc_uniform(r[0]), orc_uniform(r[1]), &z[0], &z[1]);
    orc_box_muller(orc_uniform(r[2]), orc_uniform(r[3]), &z[2], &z[3]);
}

/* Batch form used by the distribution pins: n counters -> n x 4 normals. */
void orc_normals_batch(const uint32_t *ctr, int64_t n, uint64_t seed, double *z)
{
    for (int64_t i = 0; i < n; ++i) orc_normals4(ctr + 4 * i, seed, z + 4 * i);
}

/* Counter layout (reading): control noise of sample k at time t in call j is
 * (t, 0xFFFFFFFF, k, j); state disturbance of draw m of sample k is
 * (t, m, k, j). */
#define ORC_CTRL_WORD 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Dynamics F (Eq. 1).  The paper's vehicle model is not given; reading:     */
/* rear-axle kinematic bicycle, state (x, y, psi, v), control (a, delta),    */
/* forward Euler with step dt, no speed clamp and no angle wrap.             */
/* ------------------------------------------------------------------------ */
void orc_dynamics(const double x[4], const double u[2], double dt, double wheelbase, double out[4])
{
    double px = x[0], py = x[1], psi = x[2], v = x[3];
    out[0] = px + dt * v * cos(psi);
    out[1] = py + dt * v * sin(psi);
    out[2] = psi + dt * v * tan(u[1]) / wheelbase;
    out[3] = v + dt * u[0];
}

/* ------------------------------------------------------------------------ */
/* Running cost q (Eq. 20-22) on an elliptic track (reading: the centreline  */
/* is the ellipse ((X/a)^2 + (Y/b)^2 = 1); e is its Sampson signed distance, */
/* positive outside; d = half_width - |e| is the distance to the nearer      */
/* boundary, positive on the track).  Obstacle costs are summed over i.       */
/* ------------------------------------------------------------------------ */
void orc_track_terms(const orc_params *p, const double x[4], double *e_out, double *d_out)
{
    double X = x[0] - p->track[0], Y = x[1] - p->track[1];
    double a = p->track[2], b = p->track[3];
    double G = (X / a) * (X / a) + (Y / b) * (Y / b) - 1.0;
    double gx = 2.0 * X / (a * a), gy = 2.0 * Y / (b * b);
    double gn = sqrt(gx * gx + gy * gy);
    if (gn < 1e-12) gn = 1e-12;
    double e = G / gn;
    *e_out = e;
    *d_out = p->track[4] - fabs(e);
}

/* Smooth boundary cost, Eq. 21 (the outer max with 0 is kept as written). */
double orc_boundary_cost(double d)
{
    const double pi = 3.141592653589793238462643383279;
    double v = atan(-100.0 * d) / pi + 0.5;
    return v > 0.0 ? v : 0.0;
}

/* Number of obstacles whose disc strictly contains the point (Eq. 22 summed
 * over i).  The test d_i < r_i is evaluated as d_i^2 < r_i^2. */
int orc_obstacle_count(const double *obs, int n_obs, double px, double py)
{
    int cnt = 0;
    for (int i = 0; i < n_obs; ++i) {
        double dx = px - obs[3 * i + 0], dy = py - obs[3 * i + 1], r = obs[3 * i + 2];
        if (dx * dx + dy * dy < r * r) cnt += 1;
    }
    return cnt;
}

/* Distance from the point to the nearest obstacle boundary, min_i |d_i - r_i|.
 * Diagnostic only: rollouts that pass within FP32 error of a boundary may
 * legitimately flip an indicator between FP32 and FP64. */
double orc_obstacle_margin(const double *obs, int n_obs, double px, double py)
{
    double m = INFINITY;
    for (int i = 0; i < n_obs; ++i) {
        double dx = px - obs[3 * i + 0], dy = py - obs[3 * i + 1];
        double g = fabs(sqrt(dx * dx + dy * dy) - obs[3 * i + 2]);
        if (g < m) m = g;
    }
    return m;
}

/* q(x) = c_bdry*mu_bdry + c_obs*mu_obs + c_dev*e^2 + c_v*(v - v_ref)^2. */
double orc_running_cost(const orc_params *p, const double *obs, const double x[4])
{
    double e, d;
    orc_track_terms(p, x, &e, &d);
    double q = 0.0;
    q += p->c_bdry * orc_boundary_cost(d);
    q += p->c_obs * (double)orc_obstacle_count(obs, p->n_obs, x[0], x[1]);
    q += p->c_dev * e * e;
    q += p->c_v * (x[3] - p->v_ref) * (x[3] - p->v_ref);
    return q;
}

/* wrap to (-pi, pi] */
static double orc_wrap(double ang)
{
    const double pi = 3.141592653589793238462643383279;
    return ang - 2.0 * pi * ceil((ang - pi) / (2.0 * pi));
}

/* Progress along the centreline (reading for s(x)): the change of the
 * ellipse's parametric angle theta = atan2(Y/b, X/a) between the start
 * state and x, wrapped to (-pi, pi], times the mean semi-axis (a + b)/2. */
double orc_progress(const orc_params *p, const double x0[4], const double x[4])
{
    double a = p->track[2], b = p->track[3];
    double th0 = atan2((x0[1] - p->track[1]) / b, (x0[0] - p->track[0]) / a);
    double th = atan2((x[1] - p->track[1]) / b, (x[0] - p->track[0]) / a);
    return 0.5 * (a + b) * orc_wrap(th - th0);
}

/* Distance of the wrapped angle from the wrap point (diagnostic). */
double orc_progress_margin(const orc_params *p, const double x0[4], const double x[4])
{
    const double pi = 3.141592653589793238462643383279;
    double a = p->track[2], b = p->track[3];
    double th0 = atan2((x0[1] - p->track[1]) / b, (x0[0] - p->track[0]) / a);
    double th = atan2((x[1] - p->track[1]) / b, (x[0] - p->track[0]) / a);
    return pi - fabs(orc_wrap(th - th0));
}

/* Normalised radius sqrt((X/a)^2 + (Y/b)^2) of the point (1 on the
 * centreline, 0 at the ellipse centre).  Diagnostic: near the centre the
 * gradient of G vanishes and the Sampson distance e = G / |grad G| becomes
 * ill-conditioned (relative sensitivity about 1 / distance from the centre),
 * so rollouts that pass there amplify rounding of the state. */
double orc_track_radius(const orc_params *p, const double x[4])
{
    double X = (x[0] - p->track[0]) / p->track[2], Y = (x[1] - p->track[1]) / p->track[3];
    return sqrt(X * X + Y * Y);
}

/* Terminal cost, Eq. 23: phi = c4 - c5 * s(x). */
double orc_terminal_cost(const orc_params *p, const double x0[4], const double x[4])
{
    return p->c4 - p->c5 * orc_progress(p, x0, x);
}

/* ------------------------------------------------------------------------ */
/* Integers derived on the host (in double precision, by both sides).         */
/* ------------------------------------------------------------------------ */
/* Empirical VaR (Eq. 11): the smallest t with #(L <= t)/M >= alpha is the
 * k_alpha-th smallest value, k_alpha = ceil(alpha*M).  The tail (Eq. 12-13)
 * is every value >= VaR; without ties it holds the n_tail = M - k_alpha + 1
 * largest values. */
void orc_tail_size(double alpha, int M, int *k_alpha, int *n_tail)
{
    int k = (int)ceil(alpha * (double)M - 1e-9);
    if (k < 1) k = 1;
    if (k > M) k = M;
    *k_alpha = k;
    *n_tail = M - k + 1;
}

/* Warm / zero-mean rule of Algorithm 1: sample k keeps the mean sequence when
 * k < (1 - eta) K, otherwise it uses the noise alone. */
int orc_n_warm(double eta, int K)
{
    int n = (int)ceil((1.0 - eta) * (double)K - 1e-9);
    if (n < 0) n = 0;
    if (n > K) n = K;
    return n;
}

/* ------------------------------------------------------------------------ */
/* CVaR of one sample's M risk costs (Eq. 10-13 with the scaling of Eq. 18-19). */
/* ------------------------------------------------------------------------ */
static int orc_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* Scal (Eq. 18-19): L_a = B (L - Lbar) + Lbar with Lbar the mean over the
 * draws (the 1/N missing from Eq. 19 is restored).  B == 1 is the identity,
 * taken exactly. */
void orc_scale_risk(const double *L, int M, double B, double *La)
{
    if (B == 1.0) {
        for (int i = 0; i < M; ++i) La[i] = L[i];
        return;
    }
    double s = 0.0;
    for (int i = 0; i < M; ++i) s += L[i];
    double mean = s / (double)M;
    for (int i = 0; i < M; ++i) La[i] = B * (L[i] - mean) + mean;
}

/* Max + Average: the mean of the n_tail largest scaled risk costs, summed in
 * descending order.  `work` holds M doubles. */
double orc_cvar_with(const double *L, int M, double alpha, double B, double *work)
{
    int k_alpha, n_tail;
    orc_tail_size(alpha, M, &k_alpha, &n_tail);
    orc_scale_risk(L, M, B, work);
    qsort(work, (size_t)M, sizeof(double), orc_desc);
    double s = 0.0;
    for (int i = 0; i < n_tail; ++i) s += work[i];
    return s / (double)n_tail;
}

double orc_cvar(const double *L, int64_t M, double alpha, double B)
{
    double *work = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    double c = orc_cvar_with(L, (int)M, alpha, B, work);
    free(work);
    return c;
}

/* Batch: K samples of M costs each (row-major K x M). */
void orc_cvar_batch(const double *L, int K, int M, double alpha, double B, double *out)
{
    double *work = (double *)malloc(sizeof(double) * (size_t)M);
    for (int k = 0; k < K; ++k) out[k] = orc_cvar_with(L + (size_t)k * M, M, alpha, B, work);
    free(work);
}

/* CVaR violation cost (Eq. 14-15) and the modified cost (Eq. 16). */
double orc_filtered_cost(double S, double cvar, double A, double C_u)
{
    double jc = (cvar > C_u) ? A * cvar : 0.0;
    return S + jc;
}

/* ------------------------------------------------------------------------ */
/* Weights (Eq. 5 and 17) and the weighted average (Eq. 4).                   */
/* ------------------------------------------------------------------------ */
/* w[k] = exp(-(S~_k - beta)/lambda) with beta = min S~; w_hat = w / sum(w),
 * the sum taken in index order. */
void orc_weights(const double *St, int K, double lambda, double *w, double *w_hat)
{
    double beta = INFINITY;
    for (int k = 0; k < K; ++k) if (St[k] < beta) beta = St[k];
    double Z = 0.0;
    for (int k = 0; k < K; ++k) {
        w[k] = exp(-(St[k] - beta) / lambda);
        Z += w[k];
    }
    for (int k = 0; k < K; ++k) w_hat[k] = w[k] / Z;
}

/* V+_t = sum_k w_hat_k u_{k,t}; u is K x T x 2 row-major. */
void orc_update(const double *w_hat, const double *u, int K, int T, double *Vplus)
{
    for (int j = 0; j < 2 * T; ++j) Vplus[j] = 0.0;
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < 2 * T; ++j) Vplus[j] += w_hat[k] * u[(size_t)k * 2 * T + j];
}

/* Receding-horizon reuse (reading): after the first command is taken, the
 * sequence is moved left by one step and the last element is repeated. */
void orc_shift(const double *Vplus, int T, double *Vnext)
{
    for (int t = 0; t < T - 1; ++t) {
        Vnext[2 * t] = Vplus[2 * (t + 1)];
        Vnext[2 * t + 1] = Vplus[2 * (t + 1) + 1];
    }
    Vnext[2 * (T - 1)] = Vplus[2 * (T - 1)];
    Vnext[2 * (T - 1) + 1] = Vplus[2 * (T - 1) + 1];
}

/* ------------------------------------------------------------------------ */
/* Sampled controls: u_{k,t} = clamp(base + eps, u_lo, u_hi), base = v_t for  */
/* warm samples and 0 otherwise, eps = sqrt(diag Sigma_eps) * z (Eq. 2b-2c). */
/* ------------------------------------------------------------------------ */
void orc_sample_control(const orc_params *p, const double *V, uint32_t step_idx, int n_warm,
                        int k, int t, double out[2])
{
    uint32_t ctr[4] = { (uint32_t)t, ORC_CTRL_WORD, (uint32_t)k, step_idx };
    double z[4];
    orc_normals4(ctr, p->seed, z);
    double b0 = (k < n_warm) ? V[2 * t] : 0.0;
    double b1 = (k < n_warm) ? V[2 * t + 1] : 0.0;
    double a = b0 + sqrt(p->sigma_eps[0]) * z[0];
    double d = b1 + sqrt(p->sigma_eps[1]) * z[1];
    if (a < p->u_lo[0]) a = p->u_lo[0];
    if (a > p->u_hi[0]) a = p->u_hi[0];
    if (d < p->u_lo[1]) d = p->u_lo[1];
    if (d > p->u_hi[1]) d = p->u_hi[1];
    out[0] = a;
    out[1] = d;
}

/* All K x T sampled controls, row-major K x T x 2. */
void orc_controls(const orc_params *p, const double *V, uint32_t step_idx, double *u)
{
    int n_warm = orc_n_warm(p->eta, p->K);
    for (int k = 0; k < p->K; ++k)
        for (int t = 0; t < p->T; ++t)
            orc_sample_control(p, V, step_idx, n_warm, k, t, u + ((size_t)k * p->T + t) * 2);
}

/* Nominal rollout of one sample and its cost S (Eq. 3, 16 without J_C):
 * running cost at x_0..x_{T-1} (before each step) plus the control term
 * gamma * v_t^T Sigma_eps^-1 u_t (per step, on the applied control), plus the
 * terminal cost at x_T.  gamma == 0 drops the control term. */
double orc_nominal_cost(const orc_params *p, const double *obs, const double x0[4],
                        const double *V, const double *uk, double *margin, double *cond)
{
    double x[4] = { x0[0], x0[1], x0[2], x0[3] }, xn[4];
    double S = 0.0, mg = INFINITY, cd = INFINITY;
    for (int t = 0; t < p->T; ++t) {
        const double *ut = uk + 2 * t;
        S += orc_running_cost(p, obs, x);
        if (p->gamma != 0.0)
            S += p->gamma * (V[2 * t] * ut[0] / p->sigma_eps[0] + V[2 * t + 1] * ut[1] / p->sigma_eps[1]);
        if (margin) {
            double g = orc_obstacle_margin(obs, p->n_obs, x[0], x[1]);
            if (g < mg) mg = g;
        }
        if (cond) {
            double r = orc_track_radius(p, x);
            if (r < cd) cd = r;
        }
        orc_dynamics(x, ut, p->dt, p->wheelbase, xn);
        memcpy(x, xn, sizeof x);
    }
    if (p->c4 != 0.0 || p->c5 != 0.0) {
        S += orc_terminal_cost(p, x0, x);
        if (margin && p->c5 != 0.0) {
            /* the wrap in s(x) is a discontinuity of phi; express its margin in
             * metres of progress so it can share the obstacle-margin threshold */
            double g = orc_progress_margin(p, x0, x) * 0.5 * (p->track[2] + p->track[3]);
            if (g < mg) mg = g;
        }
    }
    if (margin) *margin = mg;
    if (cond) *cond = cd;
    return S;
}

/* Disturbance w_t of one (sample, draw, step) counter.  The method accepts
 * any zero-mean additive form (Eq. 6-7); the paper's experiments use three,
 * read here as:
 *   0 Gaussian: w = sqrt(diag Sigma_w) z, z standard normal (Box-Muller);
 *   1 uniform:  w_i ~ U[-h_i, h_i] with h_i = sqrt(3 Sigma_w,i), i.e. the same
 *               covariance as the Gaussian form (w_i = h_i (2 u_i - 1));
 *   2 impulse:  with probability jump_prob a jump of length jump_size in a
 *               uniformly random direction of the (x, y) plane, else zero
 *               (u_0 < jump_prob decides, angle 2 pi u_1). */
void orc_disturbance(const orc_params *p, const uint32_t ctr[4], double w[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    if (p->noise_kind == 0) {
        double z[4];
        orc_normals4(ctr, p->seed, z);
        for (int i = 0; i < 4; ++i) w[i] = sqrt(p->sigma_w[i]) * z[i];
        return;
    }
    uint32_t key[2] = { (uint32_t)(p->seed & 0xFFFFFFFFu), (uint32_t)(p->seed >> 32) };
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    if (p->noise_kind == 1) {
        for (int i = 0; i < 4; ++i) w[i] = sqrt(3.0 * p->sigma_w[i]) * (2.0 * orc_uniform(r[i]) - 1.0);
        return;
    }
    w[0] = w[1] = w[2] = w[3] = 0.0;
    if (orc_uniform(r[0]) < p->jump_prob) {
        double th = two_pi * orc_uniform(r[1]);
        w[0] = p->jump_size * cos(th);
        w[1] = p->jump_size * sin(th);
    }
}

/* Batch form for the distribution pins: n counters -> n x 4 disturbances. */
void orc_disturbance_batch(const orc_params *p, const uint32_t *ctr, int64_t n, double *w)
{
    for (int64_t i = 0; i < n; ++i) orc_disturbance(p, ctr + 4 * i, w + 4 * i);
}

/* Disturbed rollout of draw m of sample k and its risk cost L (Eq. 6, 9):
 * x~_{t+1} = F(x~_t, u_t) + w_t with w_t from orc_disturbance (additive
 * zero-mean noise, so that F = E[F~] as Eq. 7 requires); l = q. */
double orc_disturbed_cost(const orc_params *p, const double *obs, const double x0[4],
                          const double *uk, int k, int m, uint32_t step_idx, double *margin, double *cond)
{
    double x[4] = { x0[0], x0[1], x0[2], x0[3] }, xn[4];
    double L = 0.0, mg = INFINITY, cd = INFINITY;
    for (int t = 0; t < p->T; ++t) {
        L += orc_running_cost(p, obs, x);
        if (margin) {
            double g = orc_obstacle_margin(obs, p->n_obs, x[0], x[1]);
            if (g < mg) mg = g;
        }
        if (cond) {
            double r = orc_track_radius(p, x);
            if (r < cd) cd = r;
        }
        uint32_t ctr[4] = { (uint32_t)t, (uint32_t)m, (uint32_t)k, step_idx };
        double w[4];
        orc_disturbance(p, ctr, w);
        orc_dynamics(x, uk + 2 * t, p->dt, p->wheelbase, xn);
        for (int i = 0; i < 4; ++i) x[i] = xn[i] + w[i];
    }
    if (margin) *margin = mg;
    if (cond) *cond = cd;
    return L;
}

/* ------------------------------------------------------------------------ */
/* One full RA-MPPI iteration (Algorithm 1, one pass of the while loop).     */
/* Outputs (all caller-allocated, any may be NULL except Vplus):              */
/*   u [K*T*2], S [K], L [K*M], cvar [K], St [K], w_hat [K], Vplus [T*2],      */
/*   Vnext [T*2] (shifted when p->shift), obs_margin [K*M], nom_margin [K],    */
/*   obs_cond [K*M], nom_cond [K] (minimum normalised track radius).           */
/* Returns 0, or -1 on invalid sizes.                                         */
/* ------------------------------------------------------------------------ */
static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }

int orc_get_threads(void) { return g_threads; }

int orc_step(const orc_params *p, const double *obs, const double x0[4], const double *V,
             uint32_t step_idx, double *u_out, double *S_out, double *L_out, double *cvar_out,
             double *St_out, double *w_hat_out, double *Vplus, double *Vnext,
             double *obs_margin, double *nom_margin, double *obs_cond, double *nom_cond)
{
    int K = p->K, T = p->T, M = p->M;
    if (K <= 0 || T <= 0 || M <= 0 || p->n_obs < 0 || !Vplus) return -1;
    double *u = (double *)malloc(sizeof(double) * (size_t)K * T * 2);
    double *S = (double *)malloc(sizeof(double) * (size_t)K);
    double *L = (double *)malloc(sizeof(double) * (size_t)K * M);
    double *cv = (double *)malloc(sizeof(double) * (size_t)K);
    double *St = (double *)malloc(sizeof(double) * (size_t)K);
    double *w = (double *)malloc(sizeof(double) * (size_t)K);
    double *wh = (double *)malloc(sizeof(double) * (size_t)K);
    if (!u || !S || !L || !cv || !St || !w || !wh) {
        free(u); free(S); free(L); free(cv); free(St); free(w); free(wh);
        return -1;
    }

    orc_controls(p, V, step_idx, u);

    /* Per sample: nominal rollout and S; M disturbed rollouts and L; Scal,
     * Max, Average -> CVaR; filtering -> S~.  Samples are independent, so the
     * loop may run on several threads without changing any result. */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
#endif
    for (int k = 0; k < K; ++k) {
        const double *uk = u + (size_t)k * T * 2;
        double nm, nc;
        S[k] = orc_nominal_cost(p, obs, x0, V, uk, nom_margin ? &nm : NULL, nom_cond ? &nc : NULL);
        if (nom_margin) nom_margin[k] = nm;
        if (nom_cond) nom_cond[k] = nc;
        for (int m = 0; m < M; ++m) {
            double om, oc;
            L[(size_t)k * M + m] = orc_disturbed_cost(p, obs, x0, uk, k, m, step_idx, obs_margin ? &om : NULL,
                                                      obs_cond ? &oc : NULL);
            if (obs_margin) obs_margin[(size_t)k * M + m] = om;
            if (obs_cond) obs_cond[(size_t)k * M + m] = oc;
        }
        double *work = (double *)malloc(sizeof(double) * (size_t)M);
        cv[k] = orc_cvar_with(L + (size_t)k * M, M, p->alpha, p->B, work);
        free(work);
        St[k] = orc_filtered_cost(S[k], cv[k], p->A, p->C_u);
    }

    orc_weights(St, K, p->lambda, w, wh);
    orc_update(wh, u, K, T, Vplus);
    if (Vnext) {
        if (p->shift) orc_shift(Vplus, T, Vnext);
        else memcpy(Vnext, Vplus, sizeof(double) * (size_t)T * 2);
    }

    if (u_out) memcpy(u_out, u, sizeof(double) * (size_t)K * T * 2);
    if (S_out) memcpy(S_out, S, sizeof(double) * (size_t)K);
    if (L_out) memcpy(L_out, L, sizeof(double) * (size_t)K * M);
    if (cvar_out) memcpy(cvar_out, cv, sizeof(double) * (size_t)K);
    if (St_out) memcpy(St_out, St, sizeof(double) * (size_t)K);
    if (w_hat_out) memcpy(w_hat_out, wh, sizeof(double) * (size_t)K);
    free(u); free(S); free(L); free(cv); free(St); free(w); free(wh);
    return 0;
}

/* Risk costs of a subset of samples only (used to time the oracle on a
 * bounded sample of a large workload).  Computes the controls of samples
 * k0..k0+nk-1, their nominal costs and all their disturbed rollouts. */
int orc_rollout_subset(const orc_params *p, const double *obs, const double x0[4], const double *V,
                       uint32_t step_idx, int k0, int nk, double *S_out, double *L_out)
{
    int T = p->T, M = p->M;
    int n_warm = orc_n_warm(p->eta, p->K);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
#endif
    for (int j = 0; j < nk; ++j) {
        int k = k0 + j;
        double *uk = (double *)malloc(sizeof(double) * (size_t)T * 2);
        for (int t = 0; t < T; ++t) orc_sample_control(p, V, step_idx, n_warm, k, t, uk + 2 * t);
        S_out[j] = orc_nominal_cost(p, obs, x0, V, uk, NULL, NULL);
        for (int m = 0; m < M; ++m)
            L_out[(size_t)j * M + m] = orc_disturbed_cost(p, obs, x0, uk, k, m, step_idx, NULL, NULL);
        free(uk);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gradient of the free energy with respect to the mean sequence V.          */
/*                                                                            */
/* J(V) = -lambda log((1/K) sum_k exp(-S~_k(V)/lambda)) with the noise held    */
/* fixed; dJ/dV = sum_k w_hat_k dS~_k/dV (the weights of Eq. 17).  With       */
/* Eq. 14-16 and 18-19: dS~_k = dS_k + A 1[CVaR_k > C_u] dCVaR_k, and         */
/* dCVaR_k = (1/n_tail) sum over the tail of dL_a = B dL_m + (1 - B) dLbar.   */
/* Indicators (collisions, the C_u test, tail membership) have zero gradient  */
/* almost everywhere.  u = clamp(v + eps) has du/dv = 1 strictly inside the   */
/* box for warm samples and 0 otherwise.  Rollouts are differentiated by the  */
/* backward (adjoint) recursion of the Euler steps.                           */
/* ------------------------------------------------------------------------ */

/* Gradient of the running cost q with respect to the state (Eq. 20-21; the
 * obstacle indicator of Eq. 22 contributes nothing). */
void orc_running_cost_grad(const orc_params *p, const double x[4], double g[4])
{
    const double pi = 3.141592653589793238462643383279;
    double a = p->track[2], b = p->track[3];
    double X = x[0] - p->track[0], Y = x[1] - p->track[1];
    double G = (X / a) * (X / a) + (Y / b) * (Y / b) - 1.0;
    double gx = 2.0 * X / (a * a), gy = 2.0 * Y / (b * b);
    double gn = sqrt(gx * gx + gy * gy);
    double deX = 0.0, deY = 0.0, e;
    if (gn < 1e-12) {
        e = G / 1e-12;
        deX = gx / 1e-12;
        deY = gy / 1e-12;
    } else {
        e = G / gn;
        deX = gx / gn - G * gx * (2.0 / (a * a)) / (gn * gn * gn);
        deY = gy / gn - G * gy * (2.0 / (b * b)) / (gn * gn * gn);
    }
    g[0] = 2.0 * p->c_dev * e * deX;
    g[1] = 2.0 * p->c_dev * e * deY;
    g[2] = 0.0;
    g[3] = 2.0 * p->c_v * (x[3] - p->v_ref);
    if (p->c_bdry != 0.0) {
        double d = p->track[4] - fabs(e);
        double dmu_dd = -100.0 / (pi * (1.0 + 1e4 * d * d));
        double sgn = (e > 0.0) - (e < 0.0);
        g[0] += p->c_bdry * dmu_dd * (-sgn) * deX;
        g[1] += p->c_bdry * dmu_dd * (-sgn) * deY;
    }
}

/* Gradient of the terminal cost (Eq. 23) with respect to x_T. */
void orc_terminal_cost_grad(const orc_params *p, const double x[4], double g[4])
{
    double a = p->track[2], b = p->track[3];
    double xi = (x[0] - p->track[0]) / a, et = (x[1] - p->track[1]) / b;
    double r2 = xi * xi + et * et;
    double k = -p->c5 * 0.5 * (a + b);
    g[0] = (r2 > 0.0) ? k * (-et / (a * r2)) : 0.0;
    g[1] = (r2 > 0.0) ? k * (xi / (b * r2)) : 0.0;
    g[2] = 0.0;
    g[3] = 0.0;
}

/* Backward recursion through one rollout given its states xs[0..T] and
 * controls uk: gu[t] = dCost/du_t, where Cost = sum_{t<T} q(x_t) [+ phi(x_T)]. */
static void orc_rollout_adjoint(const orc_params *p, const double *xs, const double *uk, int terminal,
                                double *gu)
{
    int T = p->T;
    double lam[4] = { 0.0, 0.0, 0.0, 0.0 };
    if (terminal && (p->c4 != 0.0 || p->c5 != 0.0)) orc_terminal_cost_grad(p, xs + 4 * T, lam);
    for (int t = T - 1; t >= 0; --t) {
        const double *x = xs + 4 * t;
        double psi = x[2], v = x[3], delta = uk[2 * t + 1];
        double c = cos(psi), s = sin(psi), tn = tan(delta), sec2 = 1.0 + tn * tn;
        double dt = p->dt, L = p->wheelbase;
        /* controls: d(psi')/d(delta) = dt v sec^2(delta)/L, d(v')/d(a) = dt */
        gu[2 * t + 0] = dt * lam[3];
        gu[2 * t + 1] = dt * v * sec2 / L * lam[2];
        double gq[4];
        orc_running_cost_grad(p, x, gq);
        double nl[4];
        nl[0] = gq[0] + lam[0];
        nl[1] = gq[1] + lam[1];
        nl[2] = gq[2] + lam[0] * (-dt * v * s) + lam[1] * (dt * v * c) + lam[2];
        nl[3] = gq[3] + lam[0] * (dt * c) + lam[1] * (dt * s) + lam[2] * (dt * tn / L) + lam[3];
        lam[0] = nl[0]; lam[1] = nl[1]; lam[2] = nl[2]; lam[3] = nl[3];
    }
}

/* States of the nominal (m < 0) or disturbed (draw m) rollout of sample k. */
static void orc_rollout_states(const orc_params *p, const double x0[4], const double *uk, int k, int m,
                               uint32_t step_idx, double *xs)
{
    for (int i = 0; i < 4; ++i) xs[i] = x0[i];
    for (int t = 0; t < p->T; ++t) {
        double xn[4];
        orc_dynamics(xs + 4 * t, uk + 2 * t, p->dt, p->wheelbase, xn);
        if (m >= 0) {
            uint32_t ctr[4] = { (uint32_t)t, (uint32_t)m, (uint32_t)k, step_idx };
            double w[4];
            orc_disturbance(p, ctr, w);
            for (int i = 0; i < 4; ++i) xn[i] += w[i];
        }
        for (int i = 0; i < 4; ++i) xs[4 * (t + 1) + i] = xn[i];
    }
}

/* du/dv of sample k at step t (per component). */
static void orc_control_jacobian(const orc_params *p, const double *V, uint32_t step_idx, int n_warm, int k, int t,
                                 double dudv[2])
{
    if (k >= n_warm) { dudv[0] = dudv[1] = 0.0; return; }
    uint32_t ctr[4] = { (uint32_t)t, ORC_CTRL_WORD, (uint32_t)k, step_idx };
    double z[4];
    orc_normals4(ctr, p->seed, z);
    double raw0 = V[2 * t] + sqrt(p->sigma_eps[0]) * z[0];
    double raw1 = V[2 * t + 1] + sqrt(p->sigma_eps[1]) * z[1];
    dudv[0] = (raw0 > p->u_lo[0] && raw0 < p->u_hi[0]) ? 1.0 : 0.0;
    dudv[1] = (raw1 > p->u_lo[1] && raw1 < p->u_hi[1]) ? 1.0 : 0.0;
}

/* dS~_k/dV (T x 2) of one sample; also returns S~_k. */
static double orc_sample_grad(const orc_params *p, const double *obs, const double x0[4], const double *V,
                              uint32_t step_idx, int n_warm, int k, double *gS, double *xs, double *gu,
                              double *L, double *La, int *idx)
{
    int T = p->T, M = p->M;
    double *uk = (double *)malloc(sizeof(double) * 2 * (size_t)T);
    double *dudv = (double *)malloc(sizeof(double) * 2 * (size_t)T);
    for (int t = 0; t < T; ++t) {
        orc_sample_control(p, V, step_idx, n_warm, k, t, uk + 2 * t);
        orc_control_jacobian(p, V, step_idx, n_warm, k, t, dudv + 2 * t);
    }
    /* nominal: running + control + terminal cost */
    double S = orc_nominal_cost(p, obs, x0, V, uk, NULL, NULL);
    orc_rollout_states(p, x0, uk, k, -1, step_idx, xs);
    orc_rollout_adjoint(p, xs, uk, 1, gu);
    for (int t = 0; t < T; ++t) {
        for (int c = 0; c < 2; ++c) {
            double g = gu[2 * t + c] * dudv[2 * t + c];
            if (p->gamma != 0.0)
                g += p->gamma / p->sigma_eps[c] * (uk[2 * t + c] + V[2 * t + c] * dudv[2 * t + c]);
            gS[2 * t + c] = g;
        }
    }
    /* risk: CVaR of the scaled draws */
    for (int m = 0; m < M; ++m) L[m] = orc_disturbed_cost(p, obs, x0, uk, k, m, step_idx, NULL, NULL);
    orc_scale_risk(L, M, p->B, La);
    int k_alpha, n_tail;
    orc_tail_size(p->alpha, M, &k_alpha, &n_tail);
    /* tail = the n_tail largest scaled costs (indices sorted by value, descending) */
    for (int m = 0; m < M; ++m) idx[m] = m;
    for (int i = 1; i < M; ++i) {          /* insertion sort, stable, descending */
        int v = idx[i], j = i - 1;
        while (j >= 0 && La[idx[j]] < La[v]) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
    double cv = 0.0;
    for (int i = 0; i < n_tail; ++i) cv += La[idx[i]];
    cv /= (double)n_tail;
    double St = orc_filtered_cost(S, cv, p->A, p->C_u);
    if (cv > p->C_u && p->A != 0.0) {
        /* dCVaR = (1/n_tail) sum_tail [B dL_m + (1 - B) dLbar] */
        double *dsum = (double *)calloc(2 * (size_t)T, sizeof(double));
        double *dmean = (double *)calloc(2 * (size_t)T, sizeof(double));
        char *in_tail = (char *)calloc((size_t)M, 1);
        for (int i = 0; i < n_tail; ++i) in_tail[idx[i]] = 1;
        for (int m = 0; m < M; ++m) {
            if (!in_tail[m] && p->B == 1.0) continue;
            orc_rollout_states(p, x0, uk, k, m, step_idx, xs);
            orc_rollout_adjoint(p, xs, uk, 0, gu);
            for (int j = 0; j < 2 * T; ++j) {
                double g = gu[j] * dudv[j];
                if (in_tail[m]) dsum[j] += g;
                dmean[j] += g / (double)M;
            }
        }
        for (int j = 0; j < 2 * T; ++j) {
            double d = (p->B == 1.0) ? dsum[j] / n_tail
                                     : (p->B * dsum[j] + (1.0 - p->B) * n_tail * dmean[j]) / n_tail;
            gS[j] += p->A * d;
        }
        free(dsum); free(dmean); free(in_tail);
    }
    free(uk); free(dudv);
    return St;
}

/* Free energy J and its gradient dJ/dV (T x 2; may be NULL). */
double orc_free_energy(const orc_params *p, const double *obs, const double x0[4], const double *V,
                       uint32_t step_idx, double *grad)
{
    int K = p->K, T = p->T, M = p->M;
    int n_warm = orc_n_warm(p->eta, K);
    double *St = (double *)malloc(sizeof(double) * (size_t)K);
    double *G = grad ? (double *)malloc(sizeof(double) * (size_t)K * 2 * T) : NULL;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
#endif
    for (int k = 0; k < K; ++k) {
        double *xs = (double *)malloc(sizeof(double) * 4 * (size_t)(T + 1));
        double *gu = (double *)malloc(sizeof(double) * 2 * (size_t)T);
        double *L = (double *)malloc(sizeof(double) * (size_t)M);
        double *La = (double *)malloc(sizeof(double) * (size_t)M);
        int *idx = (int *)malloc(sizeof(int) * (size_t)M);
        double *gS = G ? G + (size_t)k * 2 * T : (double *)malloc(sizeof(double) * 2 * (size_t)T);
        St[k] = orc_sample_grad(p, obs, x0, V, step_idx, n_warm, k, gS, xs, gu, L, La, idx);
        if (!G) free(gS);
        free(xs); free(gu); free(L); free(La); free(idx);
    }
    double beta = INFINITY;
    for (int k = 0; k < K; ++k) if (St[k] < beta) beta = St[k];
    double Z = 0.0;
    for (int k = 0; k < K; ++k) Z += exp(-(St[k] - beta) / p->lambda);
    double J = beta - p->lambda * log(Z / (double)K);
    if (grad) {
        for (int j = 0; j < 2 * T; ++j) grad[j] = 0.0;
        for (int k = 0; k < K; ++k) {
            double wh = exp(-(St[k] - beta) / p->lambda) / Z;
            for (int j = 0; j < 2 * T; ++j) grad[j] += wh * G[(size_t)k * 2 * T + j];
        }
        free(G);
    }
    free(St);
    return J;
}
