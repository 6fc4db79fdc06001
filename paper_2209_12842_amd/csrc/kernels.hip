// Kernels of the RA-MPPI control step for gfx950.
//
// One step is three launches on the caller's stream:
//   k_obstacle_frame  the obstacle table in the frame of the start position;
//   k_rollout   nominal workgroups (one lane per sample k: sampled controls,
//               nominal rollout, cost S; Eq. 1-3) and disturbed workgroups
//               (one lane per pair (k, m): disturbed rollout and risk cost L,
//               Eq. 6, 9; then scaling and the CVaR tail mean per sample,
//               Eq. 10-13, 18-19), with the sample's controls staged in LDS
//               and the obstacle table read through scalar loads;
//   k_update    per 256-sample chunk: S~ = S + J_C (Eq. 14-16), the chunk's
//               minimum, weight sum and weighted control sums (Eq. 17); the
//               last workgroup merges the chunks (log-sum-exp), forms V+
//               (Eq. 4), the optional shift and the first command (also
//               stored straight into mapped host memory when it is wanted).
// Every reduction runs in a fixed order, so a step is bit-reproducible.
#include "device.h"
#include "launch.h"

namespace ramppi {

// Obstacle table of one step in the local frame centred on the start
// position: tab[i] = (-2 cx, -2 cy, r^2 - cx^2 - cy^2, 0) for i < n_obs, and
// entries up to the next multiple of 8 that no point can hit (tab.z = -inf).
__global__ void __launch_bounds__(256) k_obstacle_frame(const float4* __restrict__ obs, int n_obs, float fx,
                                                        float fy, float4* __restrict__ tab) {
    const int n_pad = (n_obs + 7) & ~7;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += gridDim.x * blockDim.x) {
        if (i < n_obs) {
            const float4 o = obs[i];  // cx, cy, r, unused
            const float cx = o.x - fx;
            const float cy = o.y - fy;
            tab[i] = make_float4(-2.0f * cx, -2.0f * cy, __fmaf_rn(o.z, o.z, -__fmaf_rn(cx, cx, cy * cy)), 0.0f);
        } else {
            tab[i] = make_float4(0.0f, 0.0f, -__builtin_inff(), 0.0f);
        }
    }
}

// LDS layout of k_rollout (dynamic shared memory, in this order):
//   float2 ctl[spb * T]   (dt a, tan(delta) / wheelbase) of the WG's samples
//   float  vals[spb * M]  risk costs of the WG's samples
//   float  tail[spb * M]  tail slots (descending)
//   float  means[spb]     mean risk cost per sample (risk scaling)
// Scal, Max and Average of Algorithm 1 for the spb samples of a workgroup.
// vals holds the raw risk costs (thread tid owns slot tid for tid < spb * M);
// returns the CVaR in the m == 0 lane of each sample.
__device__ __forceinline__ float cvar_epilogue(float* vals, float* tail, float* means, int spb, int M,
                                               int n_tail, int scale_risk, float B) {
    const int tid = threadIdx.x;
    const int sl = tid / M;
    const int m = tid - sl * M;
    const bool own = sl < spb;
    __syncthreads();  // vals and tail initialisation visible
    if (scale_risk) {
        if (own && m == 0) {
            float s = 0.0f;
            for (int j = 0; j < M; ++j) s += vals[sl * M + j];
            means[sl] = s / (float)M;
        }
        __syncthreads();
        if (own) {
            const float mu = means[sl];
            vals[tid] = __fmaf_rn(B, vals[tid] - mu, mu);
        }
        __syncthreads();
    }
    if (own) tail_rank_scatter(vals + sl * M, tail + sl * M, M, m, n_tail);
    __syncthreads();
    float cv = 0.0f;
    if (own && m == 0) cv = tail_sum(tail + sl * M, n_tail);
    return cv;
}

template <int kNoise>
__global__ void __launch_bounds__(1024) k_rollout(StepConst c, const ObstacleOct* __restrict__ tab,
                                                  const float* __restrict__ V, float2* __restrict__ u_out,
                                                  float* __restrict__ S_out, float* __restrict__ cvar_out,
                                                  float* __restrict__ L_out) {
    extern __shared__ float2 smem[];
    float2* ctl = smem;
    float* vals = reinterpret_cast<float*>(ctl + (size_t)c.spb * c.T);
    float* tail = vals + c.spb * c.M;
    float* means = tail + c.spb * c.M;
    const int tid = threadIdx.x;
    const int n_oct = (c.n_obs + 7) >> 3;

    if ((int)blockIdx.x < c.n_nom_wg) {
        // ---- nominal rollouts: one lane per sample ----
        const int k = blockIdx.x * blockDim.x + tid;
        if (k >= c.K) return;
        State s{0.0f, 0.0f, c.psi0, c.v0};
        float acc = 0.0f, ctrl = 0.0f;
        int cnt = 0;
        for (int t = 0; t < c.T; ++t) {
            const float2 u = sample_control(c, V, k, t);
            u_out[(size_t)t * c.K + k] = u;
            acc += smooth_cost(c, s);
            cnt += obstacle_hits(tab, n_oct, s.x, s.y);
            if (c.use_ctrl) {
                const float term = __fmaf_rn(V[2 * t] * c.inv_var0, u.x, V[2 * t + 1] * c.inv_var1 * u.y);
                ctrl = __fmaf_rn(c.gamma, term, ctrl);
            }
            bicycle_step(s, c.dt * u.x, tanf(u.y) * c.inv_wheelbase, c.dt);
        }
        float S = __fmaf_rn(c.c_obs, (float)cnt, acc);
        if (c.use_ctrl) S += ctrl;
        if (c.use_term) S += terminal_cost(c, s);
        S_out[k] = S;
        return;
    }

    // ---- disturbed rollouts: one lane per (sample, draw) ----
    const int wg = blockIdx.x - c.n_nom_wg;
    const int spb = c.spb, M = c.M, T = c.T;
    for (int idx = tid; idx < spb * T; idx += blockDim.x) {
        const int sl = idx / T;
        const int t = idx - sl * T;
        const int kk = wg * spb + sl;
        float2 cu = make_float2(0.0f, 0.0f);
        if (kk < c.K) {
            const float2 u = sample_control(c, V, kk, t);
            cu = make_float2(c.dt * u.x, tanf(u.y) * c.inv_wheelbase);
        }
        ctl[idx] = cu;
    }
    __syncthreads();

    const int sl = tid / M;
    const int m = tid - sl * M;
    const int k = wg * spb + sl;
    const bool active = (sl < spb) && (k < c.K);
    float L = 0.0f;
    if (active) {
        const float2* ck = ctl + sl * T;
        State s{0.0f, 0.0f, c.psi0, c.v0};
        float acc = 0.0f;
        int cnt = 0;
        for (int t = 0; t < T; ++t) {
            acc += smooth_cost(c, s);
            cnt += obstacle_hits(tab, n_oct, s.x, s.y);
            if (t + 1 < T) {  // the last draw cannot reach the risk cost
                const uint4 r = philox4x32_10((uint32_t)t, (uint32_t)m, (uint32_t)k, c.step_idx, c.key0, c.key1);
                const float4 w = disturbance<kNoise>(c, r);
                const float2 cc = ck[t];
                bicycle_step(s, cc.x, cc.y, c.dt);
                s.x += w.x;
                s.y += w.y;
                s.psi += w.z;
                s.v += w.w;
            }
        }
        L = __fmaf_rn(c.c_obs, (float)cnt, acc);
        if (c.debug) L_out[(size_t)k * M + m] = L;
    }
    if (sl < spb) {
        vals[tid] = L;
        tail[tid] = __builtin_nanf("");
    }
    const float cv = cvar_epilogue(vals, tail, means, spb, M, c.n_tail, c.scale_risk, c.B);
    if (active && m == 0) cvar_out[k] = cv;
}

// Block-wide reductions over 256 threads (4 waves), fixed order.
__device__ __forceinline__ float block_min_256(float v, float* red) {
    v = wave_min(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    return fminf(fminf(red[0], red[1]), fminf(red[2], red[3]));
}

__device__ __forceinline__ float block_sum_256(float v, float* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Weights and update (Eq. 14-17 and Eq. 4), one launch of G workgroups of
// 256 threads, each owning a chunk of up to 256 samples:
//  1. S~ = S + J_C per sample; the chunk's minimum beta_b, its weights
//     exp(-(S~ - beta_b)/lambda) and their sum Z_b;
//  2. the chunk's weighted control sums N_b[t] = sum_k w_k u_{k,t}, thread
//     (t, part) summing a contiguous slice of the chunk, the slices then added
//     in order;
//  3. the partials (beta_b, Z_b, N_b) go to the workspace; the workgroup that
//     finishes last (an acquire-release counter, which it resets for the next
//     launch) merges them: beta = min beta_b, scale_b = exp(-(beta_b -
//     beta)/lambda), V+ = sum_b scale_b N_b / sum_b scale_b Z_b, then writes V
//     (shifted when asked), the first command and, in debug mode, w_hat.
// No workgroup waits for another, and every sum runs in a fixed order.
// LDS (dynamic): w[256] | slice sums [parts][2T] | scale[G] | vp[2T].
__global__ void __launch_bounds__(256) k_update(StepConst c, int G, int parts, const float* __restrict__ S,
                                                const float* __restrict__ cvar, const float2* __restrict__ u,
                                                float* __restrict__ S_tilde, float* part, unsigned* counter,
                                                float* __restrict__ V, float* __restrict__ u0,
                                                float* __restrict__ u0_host, float* __restrict__ w_hat) {
    extern __shared__ float ush[];
    __shared__ float red[4];
    __shared__ int is_last;
    const int T = c.T, K = c.K;
    float* wsh = ush;
    float* psh = wsh + 256;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int k0 = b * 256;
    const int n = min(256, K - k0);
    const int stride = 2 + 2 * T;

    // 1. modified costs and chunk weights
    float st = __builtin_inff();
    if (tid < n) {
        const float cv = cvar[k0 + tid];
        const float jc = (cv > c.C_u) ? c.A * cv : 0.0f;  // Eq. 14-15
        st = S[k0 + tid] + jc;                             // Eq. 16
        S_tilde[k0 + tid] = st;
    }
    const float beta_b = block_min_256(st, red);
    const float w = (tid < n) ? expf(-(st - beta_b) / c.lambda) : 0.0f;
    wsh[tid] = w;
    const float Z_b = block_sum_256(w, red);  // also publishes wsh

    // 2. weighted control sums over slices of the chunk
    const int slice = (n + parts - 1) / parts;
    for (int idx = tid; idx < T * parts; idx += 256) {
        const int t = idx % T;
        const int pr = idx / T;
        const int ka = pr * slice, kb = min(n, ka + slice);
        const float2* ut = u + (size_t)t * K + k0;
        float ax = 0.0f, ay = 0.0f;
        for (int k = ka; k < kb; ++k) {
            const float2 uu = ut[k];
            ax = __fmaf_rn(wsh[k], uu.x, ax);
            ay = __fmaf_rn(wsh[k], uu.y, ay);
        }
        psh[(size_t)pr * 2 * T + 2 * t] = ax;
        psh[(size_t)pr * 2 * T + 2 * t + 1] = ay;
    }
    __syncthreads();
    float* pb = part + (size_t)b * stride;
    for (int j = tid; j < 2 * T; j += 256) {
        float acc = 0.0f;
        for (int pr = 0; pr < parts; ++pr) acc += psh[(size_t)pr * 2 * T + j];
        pb[2 + j] = acc;
    }
    if (tid == 0) {
        pb[0] = beta_b;
        pb[1] = Z_b;
    }

    // 3. the last workgroup to finish merges every chunk
    __syncthreads();
    if (tid == 0) {
        const unsigned done = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        is_last = (done == (unsigned)(G - 1));
        if (is_last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!is_last) return;
    __atomic_thread_fence(__ATOMIC_ACQUIRE);

    float* scale = psh;               // reuses the slice sums
    float* vp = scale + G;
    float bmin = __builtin_inff();
    for (int bb = tid; bb < G; bb += 256) bmin = fminf(bmin, part[(size_t)bb * stride]);
    const float beta = block_min_256(bmin, red);
    float z = 0.0f;
    for (int bb = tid; bb < G; bb += 256) {
        const float sc = expf(-(part[(size_t)bb * stride] - beta) / c.lambda);
        scale[bb] = sc;
        z = __fmaf_rn(part[(size_t)bb * stride + 1], sc, z);
    }
    const float Z = block_sum_256(z, red);  // also publishes scale
    const float invZ = 1.0f / Z;
    for (int j = tid; j < 2 * T; j += 256) {
        float acc = 0.0f;
        for (int bb = 0; bb < G; ++bb) acc = __fmaf_rn(part[(size_t)bb * stride + 2 + j], scale[bb], acc);
        vp[j] = acc * invZ;
    }
    __syncthreads();
    const int shift = (c.flags & 2u) != 0;
    for (int j = tid; j < 2 * T; j += 256) {
        int src = j;
        if (shift) src = min(j + 2, 2 * T - 2 + (j & 1));
        V[j] = vp[src];
    }
    if (tid < 2) {
        u0[tid] = vp[tid];
        if (u0_host) u0_host[tid] = vp[tid];  // mapped pinned host memory
    }
    if (c.debug) {
        for (int k = tid; k < K; k += 256) w_hat[k] = expf(-(S_tilde[k] - beta) / c.lambda) * invZ;
    }
}

// ---- stage kernels (same device functions as the fused step) ----

__global__ void k_philox(uint32_t key0, uint32_t key1, const uint4* __restrict__ ctr, uint4* __restrict__ out,
                         int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 cc = ctr[i];
    out[i] = philox4x32_10(cc.x, cc.y, cc.z, cc.w, key0, key1);
}

__global__ void k_normals(uint32_t key0, uint32_t key1, const uint4* __restrict__ ctr, float4* __restrict__ out,
                          int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 cc = ctr[i];
    out[i] = normals4(philox4x32_10(cc.x, cc.y, cc.z, cc.w, key0, key1));
}

__global__ void __launch_bounds__(1024) k_cvar(const float* __restrict__ L, int K, int M, int spb, int n_tail,
                                               int scale_risk, float B, float* __restrict__ cvar_out) {
    extern __shared__ float csh[];
    float* vals = csh;
    float* tail = vals + spb * M;
    float* means = tail + spb * M;
    const int tid = threadIdx.x;
    const int sl = tid / M;
    const int m = tid - sl * M;
    const int k = blockIdx.x * spb + sl;
    const bool active = (sl < spb) && (k < K);
    if (sl < spb) {
        vals[tid] = active ? L[(size_t)k * M + m] : 0.0f;
        tail[tid] = __builtin_nanf("");
    }
    const float cv = cvar_epilogue(vals, tail, means, spb, M, n_tail, scale_risk, B);
    if (active && m == 0) cvar_out[k] = cv;
}

// ---- launchers ----

int update_parts(int T) { return T >= 256 ? 1 : 256 / T; }

size_t update_lds_bytes(int T, int G) {
    const size_t slices = (size_t)update_parts(T) * 2 * T;
    const size_t merge = (size_t)G + 2 * (size_t)T;
    return 4 * (256 + (slices > merge ? slices : merge));
}

hipError_t launch_step(const StepConst& c, const StepBuffers& b, int block, size_t lds_rollout, int G,
                       size_t lds_update, hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_mid) {
    const int n_dist_wg = (c.K + c.spb - 1) / c.spb;
    if (c.n_obs > 0)
        hipLaunchKernelGGL(k_obstacle_frame, dim3((c.n_obs + 255) / 256), dim3(256), 0, stream, b.obs, c.n_obs,
                           c.fx, c.fy, b.tab);
    if (ev_start) (void)hipEventRecord(ev_start, stream);
    const ObstacleOct* tab = reinterpret_cast<const ObstacleOct*>(b.tab);
    const dim3 grid(c.n_nom_wg + n_dist_wg);
    if (c.noise_kind == 1)
        hipLaunchKernelGGL(k_rollout<1>, grid, dim3(block), lds_rollout, stream, c, tab, b.V, b.u, b.S, b.cvar, b.L);
    else if (c.noise_kind == 2)
        hipLaunchKernelGGL(k_rollout<2>, grid, dim3(block), lds_rollout, stream, c, tab, b.V, b.u, b.S, b.cvar, b.L);
    else
        hipLaunchKernelGGL(k_rollout<0>, grid, dim3(block), lds_rollout, stream, c, tab, b.V, b.u, b.S, b.cvar, b.L);
    if (ev_mid) (void)hipEventRecord(ev_mid, stream);
    hipLaunchKernelGGL(k_update, dim3(G), dim3(256), lds_update, stream, c, G, update_parts(c.T), b.S, b.cvar, b.u,
                       b.S_tilde, b.part, b.counter, b.Vout, b.u0, b.u0_host, b.w_hat);
    return hipGetLastError();
}

hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n, hipStream_t stream) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)blocks), dim3(256), 0, stream, (uint32_t)(seed & 0xFFFFFFFFu),
                       (uint32_t)(seed >> 32), reinterpret_cast<const uint4*>(ctr), reinterpret_cast<uint4*>(out), n);
    return hipGetLastError();
}

hipError_t launch_normals(uint64_t seed, const uint32_t* ctr, float* out, int64_t n, hipStream_t stream) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_normals, dim3((unsigned)blocks), dim3(256), 0, stream, (uint32_t)(seed & 0xFFFFFFFFu),
                       (uint32_t)(seed >> 32), reinterpret_cast<const uint4*>(ctr), reinterpret_cast<float4*>(out),
                       n);
    return hipGetLastError();
}

hipError_t launch_cvar(const float* L, int K, int M, int spb, int block, int n_tail, int scale_risk, float B,
                       float* out, hipStream_t stream) {
    const int blocks = (K + spb - 1) / spb;
    const size_t lds = sizeof(float) * (size_t)(2 * spb * M + spb);
    hipLaunchKernelGGL(k_cvar, dim3(blocks), dim3(block), lds, stream, L, K, M, spb, n_tail, scale_risk, B, out);
    return hipGetLastError();
}

}  // namespace ramppi
