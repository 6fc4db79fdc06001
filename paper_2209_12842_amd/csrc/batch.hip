// Batched serving: one step of many independent controllers (uneven K, T, M
// and obstacle counts) in three launches that a HIP graph can hold:
//   k_batch_prep     one thread per controller: reads the controller's
//                    measured state and call index from mapped host memory
//                    and completes its per-step constants;
//   k_batch_rollout  persistent: a fixed grid of workgroups takes
//                    (controller, workgroup) items from a queue (an atomic
//                    counter over an item list ordered by the host, by
//                    default longest first) and runs the same rollout body as
//                    the single-controller kernel; every workgroup leaves
//                    when the queue is empty, and the last one to leave
//                    resets the queue for the next launch;
//   k_batch_update   one workgroup per (controller, chunk) item, the same
//                    update body as the single-controller kernel, merged per
//                    controller by its last chunk.
// Nothing waits for another workgroup, so every wave reaches its exit.
#include "launch.h"
#include "step_device.h"

namespace ramppi {

// Per-step constants that depend on the measured state (the same arithmetic
// as the host-side fill for a single controller).
__device__ __forceinline__ void set_dynamic(StepConst& c, const BatchCtl& b, const BatchInput& in) {
    c.fx = in.x0[0];
    c.fy = in.x0[1];
    c.tox = in.x0[0] - b.track[0];
    c.toy = in.x0[1] - b.track[1];
    c.theta0 = (float)atan2(((double)in.x0[1] - (double)b.track[1]) / (double)b.track[3],
                            ((double)in.x0[0] - (double)b.track[0]) / (double)b.track[2]);
    c.psi0 = start_heading(in.x0[2]);
    c.v0 = in.x0[3];
    c.step_idx = in.step_idx;
}

__global__ void __launch_bounds__(64) k_batch_prep(BatchCtl* __restrict__ ctls, const BatchInput* __restrict__ inputs,
                                                   int n_ctl) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i < n_ctl) set_dynamic(ctls[i].c, ctls[i], inputs[i]);
}

// The loop of the persistent rollout kernel: kNoise >= 0 is the one
// disturbance form of every controller of the batch; -1 picks it per item.
template <int kNoise>
__device__ __forceinline__ void batch_rollout_loop(const BatchCtl* __restrict__ ctls, const int2* __restrict__ items,
                                                   int n_items, unsigned* queue, unsigned long long* __restrict__ work) {
    extern __shared__ float2 bsmem[];
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = (int)atomicAdd(&queue[0], 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(item_sh);
        __syncthreads();  // every lane has read item_sh before it is overwritten
        if (it >= n_items) break;
        const int2 cw = items[it];
        const BatchCtl& b = ctls[__builtin_amdgcn_readfirstlane(cw.x)];
        const int w = __builtin_amdgcn_readfirstlane(cw.y);
        const StepConst c = b.c;
        // the controller's buffers, read from device memory: in the global
        // address space (as_global)
        const float4* obs = as_global(b.obs);
        const float* V = as_global(b.V);
        float2* u = as_global(b.u);
        float* S = as_global(b.S);
        float* cvar = as_global(b.cvar);
        float* L = as_global(b.L);
        if constexpr (kNoise >= 0) {
            rollout_body<kNoise>(c, obs, V, u, S, cvar, L, w, bsmem, nullptr, nullptr, work);
        } else {
            if (c.noise_kind == 1)
                rollout_body<1>(c, obs, V, u, S, cvar, L, w, bsmem, nullptr, nullptr, work);
            else if (c.noise_kind == 2)
                rollout_body<2>(c, obs, V, u, S, cvar, L, w, bsmem, nullptr, nullptr, work);
            else
                rollout_body<0>(c, obs, V, u, S, cvar, L, w, bsmem, nullptr, nullptr, work);
        }
        __syncthreads();  // LDS is reused by the next item
    }
    if (threadIdx.x == 0) {
        const unsigned done = __hip_atomic_fetch_add(&queue[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {  // every other workgroup has left: reset for the next launch
            __hip_atomic_store(&queue[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&queue[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Controllers of several disturbance forms.
__global__ void __launch_bounds__(256) k_batch_rollout(const BatchCtl* __restrict__ ctls,
                                                       const int2* __restrict__ items, int n_items,
                                                       unsigned* queue, unsigned long long* __restrict__ work) {
    batch_rollout_loop<-1>(ctls, items, n_items, queue, work);
}

// One disturbance form for the whole batch: compiled, like the two-launch
// rollout kernel, for five waves per SIMD (the kernel for several forms
// needs the registers of the largest and holds four; on the 64-controller
// batch the rollout launch 3.62 -> 3.57 ms).
template <int kNoise>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
    k_batch_rollout_one(const BatchCtl* __restrict__ ctls, const int2* __restrict__ items, int n_items,
                        unsigned* queue, unsigned long long* __restrict__ work) {
    batch_rollout_loop<kNoise>(ctls, items, n_items, queue, work);
}

__global__ void __launch_bounds__(256) k_batch_update(const BatchCtl* __restrict__ ctls,
                                                      const int2* __restrict__ uitems) {
    extern __shared__ float bush[];
    __shared__ float red[16];
    __shared__ int is_last;
    const int2 cb = uitems[blockIdx.x];
    const BatchCtl& b = ctls[cb.x];
    const StepConst c = b.c;
    update_body(c, cb.y, b.G, b.parts, as_global(b.S), as_global(b.cvar), as_global(b.u), as_global(b.S_tilde),
                as_global(b.part), as_global(b.counter), as_global(b.V), as_global(b.u0), as_global(b.u0_host),
                as_global(b.w_hat), bush, red, &is_last);
}

hipError_t launch_batch(const BatchLaunch& L, hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_mid) {
    hipLaunchKernelGGL(k_batch_prep, dim3((L.n_ctl + 63) / 64), dim3(64), 0, stream, L.ctls, L.inputs, L.n_ctl);
    if (ev_start) (void)hipEventRecord(ev_start, stream);
    const dim3 grid(L.grid_rollout);
    if (L.noise_kind == 0)
        hipLaunchKernelGGL(k_batch_rollout_one<0>, grid, dim3(256), L.lds_rollout, stream, L.ctls, L.items, L.n_items,
                           L.queue, L.work);
    else if (L.noise_kind == 1)
        hipLaunchKernelGGL(k_batch_rollout_one<1>, grid, dim3(256), L.lds_rollout, stream, L.ctls, L.items, L.n_items,
                           L.queue, L.work);
    else if (L.noise_kind == 2)
        hipLaunchKernelGGL(k_batch_rollout_one<2>, grid, dim3(256), L.lds_rollout, stream, L.ctls, L.items, L.n_items,
                           L.queue, L.work);
    else
        hipLaunchKernelGGL(k_batch_rollout, grid, dim3(256), L.lds_rollout, stream, L.ctls, L.items, L.n_items,
                           L.queue, L.work);
    if (ev_mid) (void)hipEventRecord(ev_mid, stream);
    hipLaunchKernelGGL(k_batch_update, dim3(L.n_uitems), dim3(256), L.lds_update, stream, L.ctls, L.uitems);
    return hipGetLastError();
}

hipError_t batch_rollout_occupancy(int* wg_per_cu, size_t lds_rollout, int noise_kind) {
    if (noise_kind == 0)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, k_batch_rollout_one<0>, 256, lds_rollout);
    if (noise_kind == 1)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, k_batch_rollout_one<1>, 256, lds_rollout);
    if (noise_kind == 2)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, k_batch_rollout_one<2>, 256, lds_rollout);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, k_batch_rollout, 256, lds_rollout);
}

}  // namespace ramppi
