/*
 * ramppi.h - C ABI of the MI355X (gfx950) Risk-Aware MPPI control step.
 *
 * The library computes one iteration of Risk-Aware Model Predictive Path
 * Integral control (Yin, Zhang, Tsiotras, arXiv 2209.12842, Algorithm 1):
 * K control sequences are sampled around the mean sequence V (Eq. 2b-2c), each
 * is rolled through the nominal model (Eq. 1) for its cost S (Eq. 3) and
 * through M disturbed models (Eq. 6) for the risk costs L (Eq. 9); the
 * per-sample CVaR of the scaled risk costs (Eq. 10-13, 18-19) adds the
 * violation cost (Eq. 14-16), and the path-integral weights (Eq. 17) give the
 * new sequence V+ as the weighted average of the sampled sequences (Eq. 4).
 *
 * Notation: K samples (the paper's M), T horizon steps (the paper's K), M
 * disturbance draws per sample (the paper's N).  Vehicle model: kinematic
 * bicycle with state (x, y, psi, v) and control (acceleration, steering).
 *
 * Memory: the caller owns every device buffer (the workspace, V, the stage
 * buffers) and every stream; the library owns only the host-side handle and a
 * small pinned host buffer for the first command.  Pointers named *_dev are
 * device pointers, *_host host pointers.  `stream` is a hipStream_t (NULL is
 * the default stream).  All calls only enqueue work on `stream` unless stated.
 *
 * Errors: every call returns an mppi_status; arguments are validated on the
 * host before any device call.  MPPI_EINVAL: bad sizes, parameters or NULL
 * pointers.  MPPI_EUNSUPPORTED: a valid request beyond this library's limits.
 * MPPI_EDEVICE: no usable HIP device or a HIP runtime failure.  The message of
 * the last failure on the calling thread is returned by mppi_last_error().
 */
#ifndef RAMPPI_H
#define RAMPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mppi_handle mppi_handle;

typedef enum {
    MPPI_OK = 0,
    MPPI_EINVAL = -1,
    MPPI_ENOMEM = -2,
    MPPI_EDEVICE = -3,
    MPPI_EUNSUPPORTED = -4
} mppi_status;

/* Disturbance forms of the disturbed model x~' = F(x~, u) + w (Eq. 6-7). */
enum {
    MPPI_NOISE_GAUSSIAN = 0,      /* w = sqrt(diag sigma_w) z, z standard normal */
    MPPI_NOISE_UNIFORM = 1,       /* w_i ~ U[-h_i, h_i], h_i = sqrt(3 sigma_w_i) (same covariance) */
    MPPI_NOISE_IMPULSE = 2        /* with probability jump_prob, a jump of length jump_size in a
                                     uniformly random (x, y) direction; otherwise zero */
};

enum {
    MPPI_F_DEBUG = 1u,            /* also write L (K x M) and normalised weights */
    MPPI_F_SHIFT = 2u,            /* V <- V+ shifted left by one step, last repeated */
    MPPI_F_ALLOW_ZERO_NOISE = 4u, /* accept zero variances (then gamma must be 0) */
    MPPI_F_GRAD = 8u,             /* workspace also holds the buffers of mppi_grad */
    MPPI_F_SPLIT_UPDATE = 16u     /* always run the update as a launch of its own (see mppi_step) */
};

/* Library limits (MPPI_EUNSUPPORTED beyond them). */
#define MPPI_MAX_M 1024
#define MPPI_MAX_OBS 1024
#define MPPI_MAX_T 4096

/*
 * Controller parameters.  Every field is read by mppi_create and copied.
 *   K, T, M      samples, horizon, disturbance draws per sample (K, T, M >= 1).
 *   n_obs        number of circular obstacles (>= 0).
 *   dt           Euler step [s] (> 0); wheelbase [m] (> 0) of the bicycle.
 *   u_lo, u_hi   control box, (acceleration, steering); u_lo < u_hi.
 *   sigma_eps    control-noise variances (Eq. 2c), > 0.
 *   sigma_w      state-disturbance variances for (x, y, psi, v), >= 0.
 *   alpha        CVaR level in (0, 1) (Eq. 10-11).
 *   lambda       temperature of the weights (Eq. 5, 17), > 0.
 *   gamma        control-cost weight in [0, lambda] (Eq. 3).
 *   eta          share of zero-mean samples in [0, 1] (Algorithm 1).
 *   A, B, C_u    CVaR penalty gain, risk-scaling factor, CVaR bound (Eq. 14-19).
 *   c_bdry, c_obs, c_dev, c_v, v_ref   running-cost weights (Eq. 20-22):
 *                q = c_bdry mu_bdry + c_obs mu_obs + c_dev e^2 + c_v (v - v_ref)^2;
 *                all finite, c_v >= 0 (the speed term is formed as the square
 *                of sqrt(c_v) (v - v_ref)).
 *   c4, c5       terminal cost phi = c4 - c5 s(x_T) (Eq. 23).
 *   track        elliptic centreline: centre (ox, oy), semi-axes (a, b) > 0,
 *                half width; e is the signed Sampson distance to it.
 *   seed         Philox4x32-10 key (low word, high word).
 *   flags        MPPI_F_* bits.
 *   noise_kind   MPPI_NOISE_*; jump_prob in [0, 1] and jump_size >= 0 are read
 *                by the impulse form only.
 */
typedef struct {
    int32_t K, T, M, n_obs;
    float dt, wheelbase;
    float u_lo[2], u_hi[2];
    float sigma_eps[2];
    float sigma_w[4];
    float alpha, lambda, gamma, eta, A, B, C_u;
    float c_bdry, c_obs, c_dev, c_v, v_ref, c4, c5;
    float track[5];
    uint64_t seed;
    uint32_t flags;
    uint32_t noise_kind;
    float jump_prob, jump_size;
} mppi_params;

/* Device pointers into the workspace, valid while the handle lives.
 *   u        T x K x 2 sampled controls, time-major: u[(t*K + k)*2 + c];
 *            written with MPPI_F_DEBUG and by mppi_grad (otherwise the update
 *            draws the controls it needs again and none are stored).
 *   S        K nominal costs (Eq. 3).
 *   L        K x M risk costs (Eq. 9), row-major; written with MPPI_F_DEBUG.
 *   cvar     K CVaR values (Eq. 12, on the scaled costs of Eq. 18).
 *   S_tilde  K modified costs (Eq. 16).
 *   w_hat    K normalised weights (Eq. 17); written with MPPI_F_DEBUG.
 *   u0       2 floats: the first command of V+ before any shift. */
typedef struct {
    const float *u, *S, *L, *cvar, *S_tilde, *w_hat, *u0;
} mppi_debug_ptrs;

/* Checks a parameter set without touching any device (Algorithm 1 inputs).
 * Returns MPPI_OK, MPPI_EINVAL or MPPI_EUNSUPPORTED. */
mppi_status mppi_validate(const mppi_params *p);

/* Bytes of device workspace a handle with these parameters needs; 0 when
 * mppi_validate rejects them.  No device call. */
size_t mppi_workspace_bytes(const mppi_params *p);

/* Creates a controller.  obstacles_host: n_obs x 3 floats (cx, cy, r), r > 0,
 * copied into the workspace on `stream` (may be NULL when n_obs == 0); the
 * copy is ordered by angle around the obstacles' centroid, which speeds up
 * the obstacle test and changes no result (the cost counts every hit).
 * workspace_dev: caller-owned device memory of at least
 * mppi_workspace_bytes(p) bytes, 256-byte aligned, which must outlive the
 * handle.  On success *out receives the handle.  Synchronises `stream` once. */
mppi_status mppi_create(const mppi_params *p, const float *obstacles_host,
                        void *workspace_dev, size_t workspace_bytes,
                        void *stream, mppi_handle **out);

/* One RA-MPPI iteration (Algorithm 1, one pass of its loop).
 *   x0        host, 4 floats: the measured state (finite).  A heading of
 *             magnitude above 100 rad is reduced modulo 2 pi (in FP64) before
 *             the rollouts start from it.
 *   V_dev     device, T x 2 floats row-major: in, the mean sequence V; out, V+
 *             (Eq. 4), shifted when MPPI_F_SHIFT is set.
 *   step_idx  call counter; it is the fourth Philox counter word, so the same
 *             (seed, step_idx, x0, V) reproduces the same result bit for bit.
 *   u0_host   NULL, or host memory for 2 floats: the first command of V+
 *             before any shift.  When set, the call returns as soon as the
 *             update kernel has stored the command into mapped host memory
 *             (it polls a completion word, so the kernel may still be
 *             finishing its other writes; later work on `stream` is ordered
 *             after it as usual).
 * Enqueues one kernel on `stream` when every workgroup of the step can be
 * resident on the device at once (the workgroups that finish a chunk of
 * samples then also run its update, and the last one the merge), else two
 * (rollouts, then the update; for M > 256 three: rollouts over consecutive
 * (sample, draw) pairs, the per-sample CVaR, the update);
 * MPPI_F_SPLIT_UPDATE forces the latter.  All give the same bits. */
mppi_status mppi_step(mppi_handle *h, const float x0[4], float *V_dev,
                      uint32_t step_idx, float *u0_host, void *stream);

/* mppi_step for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * RA-MPPI iteration without a handle or a workspace.  The step's workspace is
 * a static device array of the library (32 MiB per device, held from the
 * first call on a device until the process ends; its address is looked up
 * once per device); the call allocates nothing, neither device nor host
 * memory.
 *   p             parameters as for mppi_create; MPPI_F_DEBUG and MPPI_F_GRAD
 *                 are rejected (MPPI_EINVAL: they need a handle),
 *                 MPPI_F_SPLIT_UPDATE is implied, MPPI_F_SHIFT is honoured.
 *                 MPPI_EUNSUPPORTED when the step's workspace
 *                 (mppi_workspace_bytes) exceeds 32 MiB.
 *   obstacles_dev device, n_obs x 3 floats (cx, cy, r), r > 0 (not checked:
 *                 the values stay on the device); may be NULL when n_obs = 0.
 *   x0, step_idx  as for mppi_step.
 *   V_dev         device, T x 2 floats: in V, out V+ (as for mppi_step).
 *   u0_dev        device, 2 floats receiving the first command before any
 *                 shift, or NULL.
 * Enqueues three kernels on `stream` (obstacle staging and counter reset,
 * rollouts, update) and returns; the results equal those of mppi_step with
 * the same inputs, bit for bit.  Every call on a device shares that device's
 * scratch, which keeps the last call's contents: calls that overlap on one
 * device (on different streams, or from several threads) race and must be
 * ordered by the caller. */
mppi_status mppi_step_noalloc(const mppi_params *p, const float *obstacles_dev, const float x0[4], float *V_dev,
                              uint32_t step_idx, float *u0_dev, void *stream);

/* Free energy of the sampled costs and its gradient with respect to V, for
 * differentiating through one controller step (Eq. 2, with the modified
 * costs of Eq. 14-16 and the weights of Eq. 17; noise held fixed):
 *   J(V) = -lambda log((1/K) sum_k exp(-S~_k(V) / lambda)),
 *   dJ/dV = sum_k w_hat_k dS~_k/dV,
 *   dS~_k = dS_k + A 1[CVaR_k > C_u] (1/n_tail) sum_{m in tail_k}
 *           (B dL_{k,m} + (1 - B) dLbar_k),
 * where n_tail = M - ceil(alpha M) + 1 and the derivative of every indicator
 * (collisions, the C_u test, tail membership, the box clamp) is taken as zero:
 * du/dv is 1 strictly inside the control box for the (1 - eta) K samples
 * that follow V, else 0.  The handle must have been created with
 * MPPI_F_GRAD in its flags (MPPI_EINVAL otherwise).
 *   x0, step_idx  as for mppi_step (the same samples and draws).
 *   V_dev     device, T x 2 floats: the mean sequence; read, not changed.
 *   grad_dev  device, T x 2 floats: receives dJ/dV.
 *   J_dev     device, 1 float: receives J; may be NULL.
 * Recomputes the step's rollouts (forward) and one adjoint recursion per
 * sample of non-zero weight and per rollout that reaches its gradient: the
 * nominal one and the tail draws (every draw when B != 1).  Enqueues the
 * kernels on `stream` and returns; it overwrites the buffers mppi_debug_view
 * points to. */
mppi_status mppi_grad(mppi_handle *h, const float x0[4], const float *V_dev, uint32_t step_idx,
                      float *grad_dev, float *J_dev, void *stream);

/* ---- Persistent serving of the receding-horizon loop ----
 *
 * The step of Algorithm 1 repeated at each control instant (Sec. IV: the
 * controller replans from every measured state), without one kernel launch
 * per step: mppi_serve_start launches one kernel that stays resident on
 * `stream` and runs one step per request.  Each served step computes
 * exactly what mppi_step computes from the same x0, step_idx and V (same
 * kernels' device code; bit-identical V+ and first command) and leaves V+
 * (shifted when MPPI_F_SHIFT) in V_dev, which the session keeps.
 *
 * mppi_serve_start(h, V_dev, idle_ms, stream)
 *   Only for handles whose step runs as one launch (every workgroup
 *   resident at once; MPPI_EUNSUPPORTED otherwise, or when the serving
 *   kernel itself cannot be resident).  The kernel occupies the GPU until
 *   mppi_serve_stop, or until no request arrives for idle_ms milliseconds
 *   (1 <= idle_ms <= 60000), when it leaves by itself.  While a session
 *   runs, other work that needs the GPU's compute units waits behind it,
 *   and mppi_step / mppi_grad on the handle return MPPI_EINVAL.
 * mppi_serve_step(h, x0, step_idx, u0_host)
 *   Posts the measured state (host, 4 floats, finite) and the step's call
 *   index, waits for the step and writes the first command v+_0 (before
 *   the shift) to u0_host (host, 2 floats).  MPPI_EDEVICE when the session
 *   has ended by its idle limit (the handle is then no longer serving).
 * mppi_serve_stop(h)
 *   Ends the session and waits for the kernel to leave; MPPI_OK when no
 *   session runs.
 * Requests travel through mapped pinned host memory owned by the handle;
 * one thread at a time may drive a session.  One session per GPU at a time:
 * a second one cannot become resident until the first ends (its steps then
 * wait, at most until the first session's idle limit).  A session is not
 * meant for HIP graph capture. */
mppi_status mppi_serve_start(mppi_handle *h, float *V_dev, uint32_t idle_ms, void *stream);
mppi_status mppi_serve_step(mppi_handle *h, const float x0[4], uint32_t step_idx, float *u0_host);
mppi_status mppi_serve_stop(mppi_handle *h);

/* Destroys the host handle (NULL is accepted); the workspace stays the
 * caller's.  Ends a serving session first.  Waits for nothing else: the
 * caller must not free the workspace while a step is still running on the
 * device. */
mppi_status mppi_destroy(mppi_handle *h);

/* Message of the last non-OK status returned on this thread ("" if none). */
const char *mppi_last_error(void);

/* Device pointers of the intermediate results of the last step. */
mppi_status mppi_debug_view(const mppi_handle *h, mppi_debug_ptrs *out);

/* Kernel timing with HIP events recorded on the step's stream around the
 * rollout kernel and around the update kernel.  enable = 1 starts recording
 * (and clears earlier records), enable = 2 resumes recording and keeps
 * them, enable = 0 pauses (records kept), so that a caller can time a
 * sample of its steps; mppi_timing_read waits for the recorded steps,
 * returns the summed milliseconds and the step count, and clears the
 * records.  At most 4096 steps are kept. */
mppi_status mppi_timing_enable(mppi_handle *h, int enable);
mppi_status mppi_timing_read(mppi_handle *h, double *rollout_ms, double *update_ms, int32_t *n_steps);

/* Work counter of the rollout kernel's obstacle test: the number of
 * (wave, state step, obstacle) candidates that passed the broad phase and
 * were tested exactly, summed over the steps enqueued while timing was
 * enabled, since the last call.  Waits for `stream`, then clears the
 * counters (this one and the group-test counter of mppi_timing_work). */
mppi_status mppi_timing_candidates(mppi_handle *h, void *stream, uint64_t *n_candidates);

/* Both work counters of the obstacle test: the candidates as above, and the
 * broad-phase group tests (a wave box against 64 table entries) that ran,
 * per wave, after the group skip.  Waits for `stream`, then clears both. */
mppi_status mppi_timing_work(mppi_handle *h, void *stream, uint64_t *n_candidates, uint64_t *n_group_tests);

/* ---- Stage entry points (same device code as the fused step) ---- */

/* Philox4x32-10 (Salmon et al. 2011) of n counters: ctr_dev n x 4 uint32,
 * out_dev n x 4 uint32, key = (seed low word, seed high word). */
mppi_status mppi_philox(uint64_t seed, const uint32_t *ctr_dev, uint32_t *out_dev,
                        int64_t n, void *stream);

/* Box-Muller normals from the Philox words of n counters: out_dev n x 4 floats,
 * (z0, z1) from words (0, 1) and (z2, z3) from words (2, 3); each word r maps
 * to the uniform ((r >> 9) + 1/2) 2^-23. */
mppi_status mppi_normals(uint64_t seed, const uint32_t *ctr_dev, float *out_dev,
                         int64_t n, void *stream);

/* Per-row CVaR (Eq. 10-13 on the scaled costs of Eq. 18-19): L_dev K x M
 * floats row-major, cvar_dev K floats: the mean of the M - ceil(alpha M) + 1
 * largest values of B (L - mean) + mean.  1 <= M <= MPPI_MAX_M. */
mppi_status mppi_cvar(const float *L_dev, int32_t K, int32_t M, float alpha, float B,
                      float *cvar_dev, void *stream);

/* ---- Batched serving: many independent controllers per launch ---- */

typedef struct mppi_batch mppi_batch;

/* Workspace bytes for a batch of n controllers with parameters p[0..n-1]
 * (each valid for mppi_create, with M <= 256); 0 when any is rejected.  No
 * device call. */
size_t mppi_batch_workspace_bytes(int32_t n, const mppi_params *p);

/* Creates a batch of n independent controllers (Algorithm 1 for each), served
 * by one step call.  p[i] and obstacles_host[i] (n_obs_i x 3, copied) are as
 * for mppi_create; V_dev[i] is controller i's caller-owned T_i x 2 mean
 * sequence, updated in place by every step and fixed for the batch's life;
 * workspace_dev holds mppi_batch_workspace_bytes(n, p) bytes, 256-byte
 * aligned.  The library owns the handle, a private capture stream and two
 * small mapped pinned host buffers (inputs and first commands).
 * Synchronises `stream`. */
mppi_status mppi_batch_create(int32_t n, const mppi_params *p, const float *const *obstacles_host,
                              float *const *V_dev, void *workspace_dev, size_t workspace_bytes,
                              void *stream, mppi_batch **out);

/* One step of every controller: x0_host n x 4 measured states (finite),
 * step_idx_host n call indices, u0_host NULL or n x 2 (first commands before
 * any shift; the call then waits for the step).  The step is three kernels:
 * per-controller set-up, one persistent rollout launch whose workgroups take
 * (controller, workgroup) items from a queue, and one update launch over every
 * controller's chunks; with the graph on (the default) they are replayed from
 * a HIP graph captured on the first step.  Controller i's results equal those
 * of mppi_step with the same parameters and inputs.  Before writing the inputs
 * the call waits for the previous step of this batch. */
mppi_status mppi_batch_step(mppi_batch *b, const float *x0_host, const uint32_t *step_idx_host,
                            float *u0_host, void *stream);

/* Picks the persistent grid (workgroups per compute unit, powers of two up to
 * the occupancy limit) and the queue order (0: controller order, 1: longest
 * workgroups first) by timing `trials` steps of each candidate with the last
 * inputs; the mean sequences are restored afterwards.  Writes the choice to
 * the non-NULL outputs. */
mppi_status mppi_batch_autotune(mppi_batch *b, int32_t trials, void *stream, int32_t *wg_per_cu,
                                int32_t *order);

/* enable != 0: replay the step from a HIP graph (the default); 0: launch. */
mppi_status mppi_batch_set_graph(mppi_batch *b, int enable);

/* Kernel timing of batched steps: while enabled, steps launch their three
 * kernels directly (not from the graph; the kernels are the same) with HIP
 * events on the step's stream around the persistent rollout kernel and
 * around the update kernel.  mppi_batch_timing_read waits for the recorded
 * steps, returns the summed milliseconds and the step count, and clears the
 * records.  At most 4096 steps are kept. */
mppi_status mppi_batch_timing_enable(mppi_batch *b, int enable);
mppi_status mppi_batch_timing_read(mppi_batch *b, double *rollout_ms, double *update_ms, int32_t *n_steps);
/* As mppi_timing_candidates and mppi_timing_work, over the batch's timed steps. */
mppi_status mppi_batch_timing_candidates(mppi_batch *b, void *stream, uint64_t *n_candidates);
mppi_status mppi_batch_timing_work(mppi_batch *b, void *stream, uint64_t *n_candidates, uint64_t *n_group_tests);

/* Device pointers of controller i's intermediate results (see mppi_debug_ptrs). */
mppi_status mppi_batch_debug_view(const mppi_batch *b, int32_t i, mppi_debug_ptrs *out);

/* Waits for the batch's last step and destroys the handle (NULL is accepted). */
mppi_status mppi_batch_destroy(mppi_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* RAMPPI_H */
