// Gradient of the free energy with respect to the mean sequence, on the
// device.  J(V) = -lambda log((1/K) sum_k exp(-S~_k/lambda)) with the noise
// fixed, and dJ/dV = sum_k w_hat_k dS~_k/dV, where (Eq. 14-19)
//   dS~_k = dS_k + A 1[CVaR_k > C_u] (1/n_tail) sum_tail (B dL_m + (1 - B) dLbar).
// After the forward rollout (which records each draw's rank in its sample)
// and the update in gradient mode (which writes J, w_hat and the list of
// samples of non-zero weight), k_grad_rollouts gives one lane to every
// (weighted sample, rollout that reaches its gradient): the nominal rollout
// and the tail draws (every draw when B != 1).  The lane recomputes its
// rollout from the same Philox counters, keeping the states of this rollout
// only, runs the adjoint (backward) recursion of the Euler steps, and writes
// its coefficient times dCost/dV as one row.  k_grad_reduce adds the rows in
// a fixed order.  Indicators (collisions, the C_u test, tail membership) have
// zero gradient almost everywhere; du/dv is 1 strictly inside the box for
// warm samples and 0 otherwise.
#include "launch.h"
#include "step_device.h"

namespace ramppi {

// du/dv of sample k at step t, per component (1 strictly inside the box for
// warm samples, else 0), from the same control draw as sample_control; v is
// (v_t0, v_t1).
// Computed in every lane and selected (no branch).
__device__ __forceinline__ float2 control_jacobian(const StepConst& c, float2 v, int k, int t) {
    const uint4 r = philox4x32_10((uint32_t)t, kCtrlWord, (uint32_t)k, c.step_idx, c.key0, c.key1);
    float z0, z1;
    box_muller(uniform01(r.x), uniform01(r.y), z0, z1);
    const float a = __fmaf_rn(c.se0, z0, v.x);
    const float d = __fmaf_rn(c.se1, z1, v.y);
    const bool warm = k < c.n_warm;
    return make_float2((warm && a > c.u_lo0 && a < c.u_hi0) ? 1.0f : 0.0f,
                       (warm && d > c.u_lo1 && d < c.u_hi1) ? 1.0f : 0.0f);
}

// Steps by which the gradient rollouts load ahead of their use.
constexpr int kGradAhead = 4;

template <int kNoise>
__global__ void __launch_bounds__(256) k_grad_rollouts(StepConst c, GradArgs a) {
    const int l = blockIdx.x * 256 + threadIdx.x;
    const int n_rows = *a.n_act * a.R;
    if (l >= n_rows) return;  // no barrier in this kernel
    const int T = c.T, K = c.K, M = c.M;
    const int slot = l / a.R;
    const int j = l - slot * a.R;
    const int k = a.act_list[slot];
    const float wk = a.w_hat[k];
    float coef;
    int m = -1;
    if (j == 0) {
        coef = wk;
    } else {
        const bool risk = (a.cvar[k] > c.C_u) && (c.A != 0.0f);
        if (!c.scale_risk) {
            m = a.tail_idx[(size_t)k * c.n_tail + (j - 1)];
            coef = risk ? wk * c.A / (float)c.n_tail : 0.0f;
        } else {
            m = j - 1;
            const bool in_tail = a.ranks[(size_t)k * M + m] < c.n_tail;
            coef = risk ? wk * c.A * ((in_tail ? c.B / (float)c.n_tail : 0.0f) + (1.0f - c.B) / (float)M) : 0.0f;
        }
    }
    if (coef == 0.0f) {
        for (int q = 0; q < 2 * T; ++q) a.rows[(size_t)q * a.stride + l] = 0.0f;
        return;
    }
    // forward: the rollout again, keeping its states.  Each step's loads are
    // issued kGradAhead steps ahead (a lane's chain of steps would otherwise
    // wait a memory round trip per step; the index is clamped, the extra
    // loads at the end unused); the ring of loaded values is indexed by the
    // unrolled position, so it stays in registers.  The disturbance is drawn
    // in every lane and added where it belongs (a select, not a branch), so
    // a whole run of kGradAhead steps is one block the compiler can
    // interleave.
    State s{0.0f, 0.0f, c.psi0, c.v0};
    const bool disturbed = m >= 0;
    float2 ur[kGradAhead];
#pragma unroll
    for (int i = 0; i < kGradAhead; ++i) ur[i] = a.u[(size_t)min(i, T - 1) * K + k];
    auto fstep = [&](int t, float2& slot) {
        a.states[(size_t)t * a.stride + l] = make_float4(s.x, s.y, s.psi, s.v);
        const float2 uu = slot;
        slot = a.u[(size_t)min(t + kGradAhead, T - 1) * K + k];
        bicycle_step(s, c.dt * uu.x, tan_steer(uu.y) * c.inv_wheelbase, c.dt);
        const uint4 r = philox4x32_10((uint32_t)t, (uint32_t)m, (uint32_t)k, c.step_idx, c.key0, c.key1);
        const State n = disturbed_successor<kNoise>(c, r, s);
        const bool add = disturbed && t + 1 < T;
        s.x = add ? n.x : s.x;
        s.y = add ? n.y : s.y;
        s.psi = add ? n.psi : s.psi;
        s.v = add ? n.v : s.v;
    };
    for (int tb = 0; tb < T; tb += kGradAhead) {
        if (tb + kGradAhead <= T) {
#pragma unroll
            for (int i = 0; i < kGradAhead; ++i) fstep(tb + i, ur[i]);
        } else {
#pragma unroll
            for (int i = 0; i < kGradAhead; ++i)
                if (tb + i < T) fstep(tb + i, ur[i]);
        }
    }
    // backward: lam = dCost/dx_{t}, seeded with the terminal cost (nominal
    // only); states, controls and v_t loaded kGradAhead steps ahead likewise
    float4 lam = (m < 0 && c.use_term) ? terminal_cost_grad(c, s) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 xr[kGradAhead];
    float2 uq[kGradAhead], vr[kGradAhead];
#pragma unroll
    for (int i = 0; i < kGradAhead; ++i) {
        const int t = max(T - 1 - i, 0);
        xr[i] = a.states[(size_t)t * a.stride + l];
        uq[i] = a.u[(size_t)t * K + k];
        vr[i] = make_float2(a.V[2 * t], a.V[2 * t + 1]);
    }
    const bool ctrl_term = m < 0 && c.use_ctrl;  // d/dv of gamma v^T Sigma^-1 u(v), nominal rollout only
    auto bstep = [&](int t, float4& xs, float2& us, float2& vs) {
        const float4 xv = xs;
        const State x{xv.x, xv.y, xv.z, xv.w};
        const float2 uu = us;
        const float2 vt = vs;
        const int tn = max(t - kGradAhead, 0);
        xs = a.states[(size_t)tn * a.stride + l];
        us = a.u[(size_t)tn * K + k];
        vs = make_float2(a.V[2 * tn], a.V[2 * tn + 1]);
        const float tnd = tan_steer(uu.y);
        const float r = x.psi * 0.159154943091895335769f;  // as in bicycle_step
        const float sn = __builtin_amdgcn_sinf(r), cs = __builtin_amdgcn_cosf(r);
        const float dt = c.dt, dv = dt * x.v;
        const float gua = dt * lam.w;                                                 // d v' / d a
        const float gud = dv * __fmaf_rn(tnd, tnd, 1.0f) * c.inv_wheelbase * lam.z;   // d psi' / d delta
        const float4 gq = smooth_cost_grad(c, x);
        float4 nl;
        nl.x = gq.x + lam.x;
        nl.y = gq.y + lam.y;
        nl.z = gq.z + __fmaf_rn(-dv * sn, lam.x, __fmaf_rn(dv * cs, lam.y, lam.z));
        nl.w = gq.w + __fmaf_rn(dt * cs, lam.x, __fmaf_rn(dt * sn, lam.y, __fmaf_rn(dt * tnd * c.inv_wheelbase,
                                                                                   lam.z, lam.w)));
        lam = nl;
        const float2 dudv = control_jacobian(c, vt, k, t);
        float g0 = gua * dudv.x, g1 = gud * dudv.y;
        const float h0 = __fmaf_rn(c.gamma * c.inv_var0, __fmaf_rn(vt.x, dudv.x, uu.x), g0);
        const float h1 = __fmaf_rn(c.gamma * c.inv_var1, __fmaf_rn(vt.y, dudv.y, uu.y), g1);
        g0 = ctrl_term ? h0 : g0;
        g1 = ctrl_term ? h1 : g1;
        a.rows[(size_t)(2 * t) * a.stride + l] = coef * g0;
        a.rows[(size_t)(2 * t + 1) * a.stride + l] = coef * g1;
    };
    for (int tb = T - 1; tb >= 0; tb -= kGradAhead) {
        if (tb - (kGradAhead - 1) >= 0) {
#pragma unroll
            for (int i = 0; i < kGradAhead; ++i) bstep(tb - i, xr[i], uq[i], vr[i]);
        } else {
#pragma unroll
            for (int i = 0; i < kGradAhead; ++i)
                if (tb - i >= 0) bstep(tb - i, xr[i], uq[i], vr[i]);
        }
    }
}

// Sum of the gradient rows: block b adds rows [256 b, 256 b + 256), wave w
// taking outputs q = w, w + 4, ... (lane i adds rows i, i + 64, i + 128,
// i + 192, then the wave adds its lanes).  Only the nb blocks that hold rows
// work (the others would add zeros): with one, its sums are dJ/dV; else the
// last of them to finish adds the block sums in block order, writes dJ/dV
// and resets its counter.  Either way the bits are those of adding every
// block's sum in order.
__global__ void __launch_bounds__(256) k_grad_reduce(int T, int G3, GradArgs a) {
    __shared__ int is_last;
    const int n_rows = *a.n_act * a.R;
    const int nb = max(1, min(G3, (n_rows + 255) / 256));
    const int b = blockIdx.x, tid = threadIdx.x;
    if (b >= nb) return;  // uniform per block
    const int lane = tid & 63, wv = tid >> 6;
    const int l0 = b * 256;
    float* out = nb == 1 ? a.grad_out : a.rpart + (size_t)b * 2 * T;
    for (int q = wv; q < 2 * T; q += 4) {
        const float* rq = a.rows + (size_t)q * a.stride + l0;
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l = lane + 64 * i;
            if (l0 + l < n_rows) acc += rq[l];
        }
        acc = wave_sum(acc);
        if (lane == 0) out[q] = acc;
    }
    if (nb == 1) return;
    __syncthreads();
    if (tid == 0) {
        const unsigned done = __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        is_last = (done == (unsigned)(nb - 1));
        if (is_last) __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!is_last) return;
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    for (int q = tid; q < 2 * T; q += 256) {
        float acc = 0.0f;
        int bb = 0;
        for (; bb + 16 <= nb; bb += 16) {  // 16 loads in flight, then the sums in order
            float pv[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) pv[i] = a.rpart[(size_t)(bb + i) * 2 * T + q];
#pragma unroll
            for (int i = 0; i < 16; ++i) acc += pv[i];
        }
        for (; bb < nb; ++bb) acc += a.rpart[(size_t)bb * 2 * T + q];
        a.grad_out[q] = acc;
    }
}

__global__ void __launch_bounds__(256) k_update_grad(StepConst c, int G, int parts, const float* __restrict__ S,
                                                     const float* __restrict__ cvar, const float2* __restrict__ u,
                                                     float* __restrict__ S_tilde, float* part, unsigned* counter,
                                                     float* __restrict__ w_hat, GradOut go) {
    extern __shared__ float ush[];
    __shared__ float red[16];
    __shared__ int is_last;
    update_body(c, blockIdx.x, G, parts, S, cvar, u, S_tilde, part, counter, nullptr, nullptr, nullptr, w_hat, ush,
                red, &is_last, &go);
}

hipError_t launch_grad(const StepConst& c, const StepBuffers& b, const GradArgs& a, const GradOut& go, int block,
                       size_t lds_rollout, int G, size_t lds_update, int n_lane_blocks, hipStream_t stream) {
    const int n_dist_wg = (c.K + c.spb - 1) / c.spb;
    (void)launch_rollout(c, b, block, lds_rollout, n_dist_wg, stream, a.ranks_w, a.tail_w);
    hipLaunchKernelGGL(k_update_grad, dim3(G), dim3(256), lds_update, stream, c, G, update_parts(c.T), b.S, b.cvar,
                       b.u, b.S_tilde, b.part, b.counter, b.w_hat, go);
    const dim3 grid(n_lane_blocks);
    if (c.noise_kind == 1)
        hipLaunchKernelGGL(k_grad_rollouts<1>, grid, dim3(256), 0, stream, c, a);
    else if (c.noise_kind == 2)
        hipLaunchKernelGGL(k_grad_rollouts<2>, grid, dim3(256), 0, stream, c, a);
    else
        hipLaunchKernelGGL(k_grad_rollouts<0>, grid, dim3(256), 0, stream, c, a);
    hipLaunchKernelGGL(k_grad_reduce, dim3(n_lane_blocks), dim3(256), 0, stream, c.T, n_lane_blocks, a);
    return hipGetLastError();
}

}  // namespace ramppi
