// Host-side launchers of the RA-MPPI kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device.h"
#include "step_device.h"

namespace ramppi {

// Device buffers of one step (all inside the caller's workspace except V).
struct StepBuffers {
    const float4* obs;  // n_obs x (cx, cy, r, 0)
    const float* V;     // T x 2, the mean sequence (read by k_rollout)
    float* Vout;        // T x 2, V+ (written by k_merge; the same memory as V)
    float2* u;          // T x K sampled controls, time-major
    float* S;           // K
    float* cvar;        // K
    float* S_tilde;     // K
    float* w_hat;       // K
    float* L;           // K x M
    float* part;        // G x (2 + 2T)
    unsigned* counter;  // chunks finished in the current update (0 between launches)
    float* u0;          // 2
    float* u0_host;     // 2 floats of mapped pinned host memory, or null
    unsigned long long* work;  // kWorkSlots broad-phase candidate counters, or null
    unsigned* chunk_ctr;       // G per-chunk contributor counters (zero between launches)
};

// One controller of a batch, in device memory: its step constants (the static
// part written at creation, the per-step part by k_batch_prep) and buffers.
struct BatchCtl {
    StepConst c;
    const float4* obs;
    float* V;
    float2* u;
    float* S;
    float* cvar;
    float* S_tilde;
    float* w_hat;
    float* L;
    float* part;
    unsigned* counter;
    float* u0;
    float* u0_host;  // mapped pinned output, 2 floats
    int32_t G, parts;
    float track[4];  // ellipse centre and semi-axes, for the per-step constants
};

// Per-step inputs of one controller, in mapped pinned host memory.
struct BatchInput {
    float x0[4];
    uint32_t step_idx;
    uint32_t pad[3];
};

struct BatchLaunch {
    BatchCtl* ctls;
    const BatchInput* inputs;  // device address of the mapped inputs
    const int2* items;         // rollout items (controller, workgroup), in queue order
    const int2* uitems;        // update items (controller, chunk)
    unsigned* queue;           // 2 counters, zero between launches
    unsigned long long* work;  // kWorkSlots broad-phase candidate counters, or null
    int n_ctl, n_items, n_uitems, grid_rollout;
    int noise_kind;            // the disturbance form of every controller, or -1 when they differ
    size_t lds_rollout, lds_update;
};

hipError_t launch_batch(const BatchLaunch& L, hipStream_t stream, hipEvent_t ev_start = nullptr,
                        hipEvent_t ev_mid = nullptr);
hipError_t batch_rollout_occupancy(int* wg_per_cu, size_t lds_rollout, int noise_kind);

// Buffers of the gradient of the free energy (see grad.hip).
struct GradArgs {
    const float* V;
    const float2* u;
    const float* cvar;
    const float* w_hat;
    const int* act_list;
    const int* n_act;
    const int* tail_idx;
    const int* ranks;
    int* ranks_w;       // written by the forward rollout
    int* tail_w;
    float4* states;     // T x stride recomputed states
    float* rows;        // 2T x stride gradient rows
    float* rpart;       // blocks x 2T
    unsigned* counter;
    float* grad_out;    // T x 2
    int R;              // lanes per weighted sample: nominal + tail (or + all draws)
    int stride;         // lane capacity K R
};

int update_parts(int T);
size_t update_lds_bytes(int T, int G);
// One step on `stream`: with fa (the update's buffers in device memory) a
// single launch whose workgroups also run the update, else the rollout launch
// and then the update launch.
hipError_t launch_step(const StepConst& c, const StepBuffers& b, int block, size_t lds_rollout, int G,
                       size_t lds_update, hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_mid,
                       const FuseArgs* fa);
hipError_t launch_rollout(const StepConst& c, const StepBuffers& b, int block, size_t lds_rollout, int n_dist_wg,
                          hipStream_t stream, int* ranks, int* tail_idx);
// Workgroups of the one-launch step (rollouts and update) resident per CU.
hipError_t fused_rollout_capacity(int noise_kind, int block, size_t lds, int* blocks_per_cu);
// Persistent serving (k_serve): resident workgroups per CU, and the launch.
hipError_t serve_capacity(int noise_kind, int block, size_t lds, int* blocks_per_cu);
hipError_t launch_serve(const StepConst& c, const StepBuffers& b, int block, size_t lds, const FuseArgs* fa,
                        const ServeArgs& sa, hipStream_t stream);
hipError_t launch_grad(const StepConst& c, const StepBuffers& b, const GradArgs& a, const GradOut& go, int block,
                       size_t lds_rollout, int G, size_t lds_update, int n_lane_blocks, hipStream_t stream);
hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n, hipStream_t stream);
hipError_t launch_normals(uint64_t seed, const uint32_t* ctr, float* out, int64_t n, hipStream_t stream);
hipError_t launch_cvar(const float* L, int K, int M, int spb, int block, int n_tail, int scale_risk, float B,
                       float* out, hipStream_t stream);

}  // namespace ramppi
