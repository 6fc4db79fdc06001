// Kernels of the RA-MPPI control step for gfx950.
//
// One step is one launch of k_rollout when every workgroup of the step can
// be resident at once (the update then runs in the workgroups that finish
// each chunk: fused_update), else two launches on the caller's stream; a
// serving session (k_serve) runs the one-launch step once per request:
//   k_rollout   nominal workgroups (one lane per sample k: sampled controls,
//               nominal rollout, cost S; Eq. 1-3) and disturbed workgroups
//               (one lane per pair (k, m): disturbed rollout and risk cost L,
//               Eq. 6, 9; then scaling and the CVaR tail mean per sample,
//               Eq. 10-13, 18-19); every workgroup stages the obstacle table
//               in the frame of the start position into LDS, and the
//               disturbed ones also their samples' controls;
//   k_update    per 256-sample chunk: S~ = S + J_C (Eq. 14-16), the chunk's
//               minimum, weight sum and weighted control sums (Eq. 17); the
//               last workgroup merges the chunks (log-sum-exp), forms V+
//               (Eq. 4), the optional shift and the first command (also
//               stored straight into mapped host memory when it is wanted).
// Every reduction runs in a fixed order, so a step is bit-reproducible.
#include "launch.h"
#include "step_device.h"

namespace ramppi {

// Workgroup order of the two-launch rollout kernel: the disturbed workgroups
// first, the nominal ones last, so that where a grid is a little larger than
// what the device holds at once the workgroups that wait for a place are the
// nominal ones, which take a fraction of a disturbed workgroup's time (the
// paper's K = 1024, M = 300 step in its per-sample layout, of whose 1028
// five-wave workgroups 768 start at once: launch 72 -> 67 us; the large step
// is unchanged).  The one-launch kernel keeps the nominal workgroups first:
// they then start on compute units of their own choosing rather than as the
// third workgroup of a unit (c2 about 1 us shorter that way).
__device__ __forceinline__ int rollout_item(const StepConst& c) {
    const int n_dist = (int)gridDim.x - c.n_nom_wg;
    const int b = (int)blockIdx.x;
    return b < n_dist ? c.n_nom_wg + b : b - n_dist;
}

template <int kNoise, bool kFuse>
__device__ __forceinline__ void rollout_launch_body(const StepConst& c, const float4* __restrict__ obs,
                                                    const float* __restrict__ V, float2* __restrict__ u_out,
                                                    float* __restrict__ S_out, float* __restrict__ cvar_out,
                                                    float* __restrict__ L_out, int* __restrict__ ranks,
                                                    int* __restrict__ tail_idx, unsigned long long* __restrict__ work,
                                                    const FuseArgs* __restrict__ fa) {
    extern __shared__ float2 smem[];
    const int item = kFuse ? (int)blockIdx.x : rollout_item(c);
    rollout_body<kNoise>(c, obs, V, u_out, S_out, cvar_out, L_out, item, smem, ranks, tail_idx, work);
    if constexpr (kFuse) {
        __shared__ float red[16];
        __shared__ int flag_sh;
        __shared__ int fin_sh[8];
        const FuseArgs f = global_view(*fa);
        // V is read by the rollouts and rewritten by the merge, which runs
        // only after every rollout of the step has finished
        fused_update(c, f, blockIdx.x, S_out, cvar_out, u_out, const_cast<float*>(V),
                     reinterpret_cast<float*>(smem), red, &flag_sh, fin_sh);
    }
}

// The rollouts of the two-launch step (the large grids, which hold many
// waves per SIMD).  Compiled for five waves per SIMD: the register budget
// then holds the per-step constants and keys in vector registers with room
// for a fifth wave (measured on the large step: 0.71 -> 0.68 ms; the
// one-launch kernel, whose grid holds two or three waves per SIMD, runs
// faster with the registers it needs).
template <int kNoise>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5)))
    k_rollout(StepConst c, const float4* __restrict__ obs, const float* __restrict__ V, float2* __restrict__ u_out,
              float* __restrict__ S_out, float* __restrict__ cvar_out, float* __restrict__ L_out,
              int* __restrict__ ranks, int* __restrict__ tail_idx, unsigned long long* __restrict__ work,
              const FuseArgs* __restrict__ fa) {
    rollout_launch_body<kNoise, false>(c, obs, V, u_out, S_out, cvar_out, L_out, ranks, tail_idx, work, fa);
}

// The one-launch step: rollouts, then the update in the workgroups that
// finish each chunk.
template <int kNoise>
__global__ void __launch_bounds__(1024)
    k_rollout_fused(StepConst c, const float4* __restrict__ obs, const float* __restrict__ V,
                    float2* __restrict__ u_out, float* __restrict__ S_out, float* __restrict__ cvar_out,
                    float* __restrict__ L_out, int* __restrict__ ranks, int* __restrict__ tail_idx,
                    unsigned long long* __restrict__ work, const FuseArgs* __restrict__ fa) {
    rollout_launch_body<kNoise, true>(c, obs, V, u_out, S_out, cvar_out, L_out, ranks, tail_idx, work, fa);
}

// Persistent serving: the one-launch step in a loop, one iteration per
// request (steps 1, 2, ... of the session).  Thread 0 of workgroup 0 takes
// the requests from host memory; the others wait on its device-memory word.
// Every wait is bounded, so every wave leaves even if no request comes.
template <int kNoise>
__global__ void __launch_bounds__(1024) k_serve(StepConst c0, const float4* __restrict__ obs, float* V,
                                                float2* __restrict__ u_out, float* __restrict__ S_out,
                                                float* __restrict__ cvar_out, float* __restrict__ L_out,
                                                const FuseArgs* __restrict__ fa, ServeArgs sa_arg) {
    extern __shared__ float2 smem[];
    const ServeArgs sa = global_view(sa_arg);
    __shared__ float red[16];
    __shared__ int flag_sh;
    __shared__ int fin_sh[8];
    __shared__ int leave_sh;
    for (unsigned seq = 1;; ++seq) {
        if (threadIdx.x == 0) leave_sh = blockIdx.x == 0 ? serve_wait_leader(sa, seq) : serve_wait_member(sa, seq);
        __syncthreads();
        if (leave_sh) break;
        // Every word of the step constants passes through an empty asm per
        // request: the compiler then derives what the step needs (the
        // Philox round keys, ...) inside the loop instead of keeping it live
        // across requests, which spilled it into VGPR lanes of the hot loop.
        StepConst c = c0;
        {
            uint32_t* wc = reinterpret_cast<uint32_t*>(&c);
#pragma unroll
            for (int i = 0; i < (int)(sizeof(StepConst) / 4); ++i) asm volatile("" : "+s"(wc[i]));
        }
        const ServeReq* r = sa.req_dev;
        c.fx = r->fx;
        c.fy = r->fy;
        c.tox = r->tox;
        c.toy = r->toy;
        c.theta0 = r->theta0;
        c.psi0 = r->psi0;
        c.v0 = r->v0;
        c.step_idx = r->step_idx;
        c.u0_seq = seq;
        rollout_body<kNoise>(c, obs, V, u_out, S_out, cvar_out, L_out, blockIdx.x, smem);
        const FuseArgs f = global_view(*fa);
        fused_update(c, f, blockIdx.x, S_out, cvar_out, u_out, V, reinterpret_cast<float*>(smem), red, &flag_sh,
                     fin_sh);
        __syncthreads();  // LDS and leave_sh are reused by the next request
    }
}

__global__ void __launch_bounds__(256) k_update(StepConst c, int G, int parts, const float* __restrict__ S,
                                                const float* __restrict__ cvar, const float2* __restrict__ u,
                                                float* __restrict__ S_tilde, float* part, unsigned* counter,
                                                float* __restrict__ V, float* __restrict__ u0,
                                                float* __restrict__ u0_host, float* __restrict__ w_hat) {
    extern __shared__ float ush[];
    __shared__ float red[16];
    __shared__ int is_last;
    update_body(c, blockIdx.x, G, parts, S, cvar, u, S_tilde, part, counter, V, u0, u0_host, w_hat, ush, red,
                &is_last);
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

// The CVaR pass of the flattened two-launch step (M > 256): one sample per
// workgroup of P threads, P the power of two at or above M (at most 1024).
// The M stored risk costs are scaled as cvar_epilogue scales them (the mean
// summed by one thread in draw order), padded to P with -inf, sorted by the
// same bitonic stages (larger first, equal costs by smaller draw index), and
// the n_tail largest are summed in that order: the bits of cvar_epilogue,
// whose ranks by counting would cost M comparisons per lane here.
__global__ void __launch_bounds__(1024) k_cvar_sorted(const float* __restrict__ L, int M, int n_tail,
                                                      int scale_risk, float B, float* __restrict__ cvar_out) {
    extern __shared__ float srt[];
    __shared__ float mean_sh;
    const int P = (int)blockDim.x, tid = (int)threadIdx.x;
    float* vals = srt;                              // P
    int* ids = reinterpret_cast<int*>(srt + P);     // P
    const float* Lk = L + (size_t)blockIdx.x * M;
    float v = tid < M ? Lk[tid] : -__builtin_inff();
    if (scale_risk) {
        vals[tid] = v;
        __syncthreads();
        if (tid == 0) {
            float s = 0.0f;
            for (int j = 0; j < M; ++j) s += vals[j];
            mean_sh = s / (float)M;
        }
        __syncthreads();
        const float mu = mean_sh;
        if (tid < M) v = __fmaf_rn(B, v - mu, mu);
    }
    int id = tid;
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j >= 64; j >>= 1) {  // partner in another wave
            __syncthreads();
            vals[tid] = v;
            ids[tid] = id;
            __syncthreads();
            bitonic_cx(v, id, vals[tid ^ j], ids[tid ^ j], tid, j, k);
        }
        bitonic_wave_stages(v, id, tid, k);
    }
    __syncthreads();
    vals[tid] = v;
    __syncthreads();
    if (tid == 0) cvar_out[blockIdx.x] = tail_sum(vals, n_tail);
}

// ---- launchers ----

template <bool kFuse>
static void launch_rollout_t(const StepConst& c, const StepBuffers& b, dim3 grid, int block, size_t lds,
                             hipStream_t stream, int* ranks, int* tail_idx, const FuseArgs* fa) {
    if constexpr (kFuse) {
        if (c.noise_kind == 1)
            hipLaunchKernelGGL(k_rollout_fused<1>, grid, dim3(block), lds, stream, c, b.obs, b.V, b.u, b.S, b.cvar,
                               b.L, ranks, tail_idx, b.work, fa);
        else if (c.noise_kind == 2)
            hipLaunchKernelGGL(k_rollout_fused<2>, grid, dim3(block), lds, stream, c, b.obs, b.V, b.u, b.S, b.cvar,
                               b.L, ranks, tail_idx, b.work, fa);
        else
            hipLaunchKernelGGL(k_rollout_fused<0>, grid, dim3(block), lds, stream, c, b.obs, b.V, b.u, b.S, b.cvar,
                               b.L, ranks, tail_idx, b.work, fa);
    } else {
        if (c.noise_kind == 1)
            hipLaunchKernelGGL(k_rollout<1>, grid, dim3(block), lds, stream, c, b.obs, b.V, b.u, b.S, b.cvar, b.L,
                               ranks, tail_idx, b.work, fa);
        else if (c.noise_kind == 2)
            hipLaunchKernelGGL(k_rollout<2>, grid, dim3(block), lds, stream, c, b.obs, b.V, b.u, b.S, b.cvar, b.L,
                               ranks, tail_idx, b.work, fa);
        else
            hipLaunchKernelGGL(k_rollout<0>, grid, dim3(block), lds, stream, c, b.obs, b.V, b.u, b.S, b.cvar, b.L,
                               ranks, tail_idx, b.work, fa);
    }
}

hipError_t launch_rollout(const StepConst& c, const StepBuffers& b, int block, size_t lds_rollout, int n_dist_wg,
                          hipStream_t stream, int* ranks, int* tail_idx) {
    launch_rollout_t<false>(c, b, dim3(c.n_nom_wg + n_dist_wg), block, lds_rollout, stream, ranks, tail_idx,
                            nullptr);
    return hipGetLastError();
}

hipError_t fused_rollout_capacity(int noise_kind, int block, size_t lds, int* blocks_per_cu) {
    if (noise_kind == 1)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_rollout_fused<1>, block, lds);
    if (noise_kind == 2)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_rollout_fused<2>, block, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_rollout_fused<0>, block, lds);
}

hipError_t serve_capacity(int noise_kind, int block, size_t lds, int* blocks_per_cu) {
    if (noise_kind == 1) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_serve<1>, block, lds);
    if (noise_kind == 2) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_serve<2>, block, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_serve<0>, block, lds);
}

hipError_t launch_serve(const StepConst& c, const StepBuffers& b, int block, size_t lds, const FuseArgs* fa,
                        const ServeArgs& sa, hipStream_t stream) {
    const dim3 grid(c.n_nom_wg + (c.K + c.spb - 1) / c.spb);
    if (c.noise_kind == 1)
        hipLaunchKernelGGL(k_serve<1>, grid, dim3(block), lds, stream, c, b.obs, b.Vout, b.u, b.S, b.cvar, b.L, fa,
                           sa);
    else if (c.noise_kind == 2)
        hipLaunchKernelGGL(k_serve<2>, grid, dim3(block), lds, stream, c, b.obs, b.Vout, b.u, b.S, b.cvar, b.L, fa,
                           sa);
    else
        hipLaunchKernelGGL(k_serve<0>, grid, dim3(block), lds, stream, c, b.obs, b.Vout, b.u, b.S, b.cvar, b.L, fa,
                           sa);
    return hipGetLastError();
}

int update_parts(int T) { return T >= 256 ? 1 : 256 / T; }

size_t update_lds_bytes(int T, int G) {
    // slice sums, the list of non-zero weights, the mean sequence
    const size_t slices = (size_t)update_parts(T) * 2 * T + 257 + 256 + 2 * (size_t)T;
    const size_t merge = 2 * (size_t)G + 2 * (size_t)T;
    return 4 * (256 + (slices > merge ? slices : merge));
}

hipError_t launch_step(const StepConst& c, const StepBuffers& b, int block, size_t lds_rollout, int G,
                       size_t lds_update, hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_mid,
                       const FuseArgs* fa) {
    const int64_t n_dist = c.flat ? ((int64_t)c.K * c.M + block - 1) / block : (c.K + c.spb - 1) / c.spb;
    const dim3 grid((unsigned)(c.n_nom_wg + n_dist));
    if (ev_start) (void)hipEventRecord(ev_start, stream);
    if (fa) {  // one launch: the update runs in the workgroups that finish each chunk
        launch_rollout_t<true>(c, b, grid, block, lds_rollout > lds_update ? lds_rollout : lds_update, stream,
                               nullptr, nullptr, fa);
        if (ev_mid) (void)hipEventRecord(ev_mid, stream);
    } else {
        launch_rollout_t<false>(c, b, grid, block, lds_rollout, stream, nullptr, nullptr, nullptr);
        if (c.flat) {  // each sample's CVaR from the stored risk costs (one sample per workgroup)
            int P = 64;
            while (P < c.M) P <<= 1;
            hipLaunchKernelGGL(k_cvar_sorted, dim3(c.K), dim3(P), 2 * sizeof(float) * (size_t)P, stream, b.L, c.M,
                               c.n_tail, c.scale_risk, c.B, b.cvar);
        }
        if (ev_mid) (void)hipEventRecord(ev_mid, stream);
        hipLaunchKernelGGL(k_update, dim3(G), dim3(256), lds_update, stream, c, G, update_parts(c.T), b.S, b.cvar,
                           b.u, b.S_tilde, b.part, b.counter, b.Vout, b.u0, b.u0_host, b.w_hat);
    }
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
