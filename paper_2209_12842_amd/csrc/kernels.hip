// Kernels of the RA-MPPI control step for gfx950.
//
// One step is four launches on the caller's stream:
//   k_obstacle_frame  the obstacle table in the frame of the start position;
//   k_rollout   nominal workgroups (one lane per sample k: sampled controls,
//               nominal rollout, cost S; Eq. 1-3) and disturbed workgroups
//               (one lane per pair (k, m): disturbed rollout and risk cost L,
//               Eq. 6, 9; then scaling and the CVaR tail mean per sample,
//               Eq. 10-13, 18-19), with the sample's controls staged in LDS
//               and the obstacle table read through scalar loads;
//   k_partials  per 256-sample chunk: S~ = S + J_C (Eq. 14-16), the chunk's
//               minimum, its weight sum and its weighted control sums (Eq. 17);
//   k_merge     one workgroup: log-sum-exp merge of the chunks, V+ (Eq. 4),
//               the optional shift and the first command.
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
                const float4 z = normals4(r);
                const float2 cc = ck[t];
                bicycle_step(s, cc.x, cc.y, c.dt);
                s.x = __fmaf_rn(c.sw0, z.x, s.x);
                s.y = __fmaf_rn(c.sw1, z.y, s.y);
                s.psi = __fmaf_rn(c.sw2, z.z, s.psi);
                s.v = __fmaf_rn(c.sw3, z.w, s.v);
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

// Chunk partials: part[b] = (beta_b, Z_b, N_b[0..2T-1]) with
// beta_b = min S~ over the chunk, Z_b = sum exp(-(S~ - beta_b)/lambda),
// N_b[t] = sum exp(-(S~ - beta_b)/lambda) u_t.
__global__ void __launch_bounds__(256) k_partials(StepConst c, const float* __restrict__ S,
                                                  const float* __restrict__ cvar, const float2* __restrict__ u,
                                                  float* __restrict__ S_tilde, float* __restrict__ part) {
    __shared__ float wsh[256];
    __shared__ float red[4];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int k = b * 256 + tid;
    const int stride = 2 + 2 * c.T;
    float st = __builtin_inff();
    if (k < c.K) {
        const float cv = cvar[k];
        const float jc = (cv > c.C_u) ? c.A * cv : 0.0f;  // Eq. 14-15
        st = S[k] + jc;                                    // Eq. 16
        S_tilde[k] = st;
    }
    const float beta = block_min_256(st, red);
    const float w = (k < c.K) ? expf(-(st - beta) / c.lambda) : 0.0f;
    wsh[tid] = w;
    const float Z = block_sum_256(w, red);  // also publishes wsh
    const int lane = tid & 63, wv = tid >> 6;
    for (int t = wv; t < c.T; t += 4) {
        float ax = 0.0f, ay = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int kk = b * 256 + lane + 64 * j;
            if (kk < c.K) {
                const float2 uu = u[(size_t)t * c.K + kk];
                const float ww = wsh[lane + 64 * j];
                ax = __fmaf_rn(ww, uu.x, ax);
                ay = __fmaf_rn(ww, uu.y, ay);
            }
        }
        ax = wave_sum(ax);
        ay = wave_sum(ay);
        if (lane == 0) {
            part[(size_t)b * stride + 2 + 2 * t] = ax;
            part[(size_t)b * stride + 3 + 2 * t] = ay;
        }
    }
    if (tid == 0) {
        part[(size_t)b * stride] = beta;
        part[(size_t)b * stride + 1] = Z;
    }
}

// Merge of the G chunk partials (one workgroup of 256 threads):
// beta = min beta_b, scale_b = exp(-(beta_b - beta)/lambda),
// V+ = sum_b scale_b N_b / sum_b scale_b Z_b.  LDS: scale[G], vp[2T].
__global__ void __launch_bounds__(256) k_merge(StepConst c, int G, const float* __restrict__ part,
                                               const float* __restrict__ S_tilde, float* __restrict__ V,
                                               float* __restrict__ u0, float* __restrict__ w_hat) {
    extern __shared__ float msh[];
    float* scale = msh;
    float* vp = msh + G;
    __shared__ float red[4];
    const int tid = threadIdx.x;
    const int stride = 2 + 2 * c.T;
    float bmin = __builtin_inff();
    for (int b = tid; b < G; b += 256) bmin = fminf(bmin, part[(size_t)b * stride]);
    const float beta = block_min_256(bmin, red);
    float z = 0.0f;
    for (int b = tid; b < G; b += 256) {
        const float sc = expf(-(part[(size_t)b * stride] - beta) / c.lambda);
        scale[b] = sc;
        z = __fmaf_rn(part[(size_t)b * stride + 1], sc, z);
    }
    const float Z = block_sum_256(z, red);  // also publishes scale
    const float invZ = 1.0f / Z;
    for (int j = tid; j < 2 * c.T; j += 256) {
        float acc = 0.0f;
        for (int b = 0; b < G; ++b) acc = __fmaf_rn(part[(size_t)b * stride + 2 + j], scale[b], acc);
        vp[j] = acc * invZ;
    }
    __syncthreads();
    const int shift = (c.flags & 2u) != 0;
    for (int j = tid; j < 2 * c.T; j += 256) {
        int src = j;
        if (shift) src = min(j + 2, 2 * c.T - 2 + (j & 1));
        V[j] = vp[src];
    }
    if (tid < 2) u0[tid] = vp[tid];
    if (c.debug) {
        for (int k = tid; k < c.K; k += 256) w_hat[k] = expf(-(S_tilde[k] - beta) / c.lambda) * invZ;
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

hipError_t launch_step(const StepConst& c, const StepBuffers& b, int block, size_t lds_rollout, int G,
                       size_t lds_merge, hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_mid) {
    const int n_dist_wg = (c.K + c.spb - 1) / c.spb;
    if (c.n_obs > 0)
        hipLaunchKernelGGL(k_obstacle_frame, dim3((c.n_obs + 255) / 256), dim3(256), 0, stream, b.obs, c.n_obs,
                           c.fx, c.fy, b.tab);
    if (ev_start) (void)hipEventRecord(ev_start, stream);
    hipLaunchKernelGGL(k_rollout, dim3(c.n_nom_wg + n_dist_wg), dim3(block), lds_rollout, stream, c,
                       reinterpret_cast<const ObstacleOct*>(b.tab), b.V, b.u, b.S, b.cvar, b.L);
    if (ev_mid) (void)hipEventRecord(ev_mid, stream);
    hipLaunchKernelGGL(k_partials, dim3(G), dim3(256), 0, stream, c, b.S, b.cvar, b.u, b.S_tilde, b.part);
    hipLaunchKernelGGL(k_merge, dim3(1), dim3(256), lds_merge, stream, c, G, b.part, b.S_tilde, b.Vout, b.u0,
                       b.w_hat);
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
