// Device bodies of one RA-MPPI step, shared by the single-controller
// kernels and the batched (many-controller) kernels.
#pragma once

#include "device.h"

namespace ramppi {

// Outputs of the update in gradient mode (the free energy, the list of
// samples of non-zero weight and its length).
struct GradOut {
    float* J;
    int* act_list;
    int* n_act;
};

// Entry i of the obstacle table of a step, in the local frame centred on the
// start position (fx, fy), with cx, cy relative to it:
// (-2 cx, -2 cy, r^2 - cx^2 - cy^2, q), q = (1 + 2^-16) r^2 + 2^-15 (cx^2 + cy^2)
// the squared reach of the broad-phase test (obstacle_hits_culled); entries
// i >= n_obs are padding that no point can hit, (0, 0, -inf, -inf).
__device__ __forceinline__ float4 obstacle_entry(const float4* __restrict__ obs, int n_obs, int i, float fx,
                                                 float fy) {
    if (i < n_obs) {
        const float4 o = obs[i];  // cx, cy, r, unused
        const float cx = o.x - fx;
        const float cy = o.y - fy;
        const float c2 = __fmaf_rn(cx, cx, cy * cy);
        const float q = __fmaf_rn(1.0000152587890625f * o.z, o.z, 3.0517578125e-05f * c2);
        return make_float4(-2.0f * cx, -2.0f * cy, __fmaf_rn(o.z, o.z, -c2), q);
    }
    return make_float4(0.0f, 0.0f, -__builtin_inff(), -__builtin_inff());
}

// The group boxes of the broad phase's group skip (kGroupPad): for each group
// g of 64 table entries, the union of its discs' squares |x - cx|, |y - cy|
// <= sqrt(q) widened by kGroupPad, as (x0, x1, y0, y1) in gbox[g]; entries
// n_grp..63 get a box that meets nothing.  One whole wave computes them
// (lane j takes entry 64 g + j, computed as obstacle_entry computes it),
// before the barrier that precedes the rollouts.
__device__ __forceinline__ void group_bounds(const float4* __restrict__ obs, int n_obs, int n_grp, float fx,
                                             float fy, float4* gbox) {
    const int lane = threadIdx.x & 63;
    const float inf = __builtin_inff();
    if (lane >= n_grp) gbox[lane] = make_float4(inf, -inf, inf, -inf);
    for (int g = 0; g < n_grp; ++g) {
        const int i = 64 * g + lane;
        const bool valid = i < n_obs;
        const float4 e = obstacle_entry(obs, n_obs, i, fx, fy);
        const float cx = -0.5f * e.x, cy = -0.5f * e.y;  // exact: e.x = -2 cx
        const float R = valid ? __builtin_amdgcn_sqrtf(e.w) : 0.0f;
        const float x0 = wave_min(valid ? cx - R : inf), x1 = wave_maxf(valid ? cx + R : -inf);
        const float y0 = wave_min(valid ? cy - R : inf), y1 = wave_maxf(valid ? cy + R : -inf);
        if (lane == 0) gbox[g] = make_float4(x0 - kGroupPad, x1 + kGroupPad, y0 - kGroupPad, y1 + kGroupPad);
    }
}

// LDS layout of k_rollout (dynamic shared memory, in this order):
//   float2 ctl[spb * T]   (dt a, tan(delta) / wheelbase) of the WG's samples
//   float  vals[spb * M]  risk costs of the WG's samples
//   float  tail[spb * M]  tail slots (descending)
//   float  means[spb]     mean risk cost per sample (risk scaling)
//   float4 otab[64 n_grp] the obstacle table, padded to groups of 64 entries
//                         (16-byte aligned; n_grp = ceil(n_obs / 64))
//   float4 gbox[64]       the groups' boxes for the group skip (group_bounds)
// rollout_otab_offset gives the offset of otab in floats.  Every workgroup
// writes otab and gbox from the raw obstacles before its rollouts.
__host__ __device__ __forceinline__ int rollout_otab_offset(int spb, int T, int M) {
    return (2 * spb * T + 2 * spb * M + spb + 3) & ~3;
}

__host__ __device__ __forceinline__ int rollout_n_grp(int n_obs) { return (n_obs + 63) >> 6; }

// Compile-time switches for the per-step lambdas of the rollouts.
struct BoolTrue {
    static constexpr bool value = true;
};
struct BoolFalse {
    static constexpr bool value = false;
};
constexpr BoolTrue kTrue{};
constexpr BoolFalse kFalse{};

// Slots of the broad-phase work counters (wave w of item i adds to slot
// (16 i + w) mod kWorkSlots, spreading the atomics): exact tests in
// work[0..kWorkSlots), group tests in work[kWorkSlots..2 kWorkSlots).
constexpr int kWorkSlots = 256;
// Time steps whose points share one broad-phase box (obstacle_hits_culled):
// a longer run divides the box and group tests over more steps but widens
// the box by the distance travelled; 6 gave the shortest steps on the 50- and
// 200-obstacle tracks (horizons 50 and 100).
constexpr int kCullSteps = 6;
// Scal, Max and Average of Algorithm 1 for the spb samples of a workgroup.
// vals holds the raw risk costs (thread tid owns slot tid for tid < spb * M);
// returns the CVaR in the m == 0 lane of each sample.  The descending order
// of a sample's M costs (equal costs by smaller draw index) comes from a
// bitonic sort in registers when M is a power of two and the workgroup is
// exactly spb * M lanes (stages within a wave through lane exchanges, wider
// ones through LDS), otherwise from counting each cost's rank in LDS.  Either
// way the n_tail largest land in tail[0..n_tail-1] in that order and are
// summed in it, so both give the same bits.  pos_out / id_out receive one
// (position, draw index) pair of the sorted order per lane; together the
// lanes of a sample cover every draw once.  tid is the thread's index in the
// workgroup (a caller may pass a copy the compiler cannot tie to values it
// derived from the index earlier).
__device__ __forceinline__ float cvar_epilogue(float* vals, float* tail, float* means, int spb, int M,
                                               int n_tail, int scale_risk, float B, int* pos_out = nullptr,
                                               int* id_out = nullptr, int tid = (int)threadIdx.x) {
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
    if ((M & (M - 1)) == 0 && (int)blockDim.x == spb * M) {
        float v = vals[tid];  // every lane owns a slot
        int id = m;
        for (int k = 2; k <= M; k <<= 1) {
            for (int j = k >> 1; j >= 64; j >>= 1) {  // partner in another wave
                int* ids = reinterpret_cast<int*>(tail);
                __syncthreads();
                vals[tid] = v;
                ids[tid] = id;
                __syncthreads();
                bitonic_cx(v, id, vals[tid ^ j], ids[tid ^ j], m, j, k);
            }
            bitonic_wave_stages(v, id, m, k);
        }
        __syncthreads();  // tail free again
        if (m < n_tail) tail[tid] = v;
        if (pos_out) *pos_out = m;
        if (id_out) *id_out = id;
    } else if (own) {
        const int rank = tail_rank_scatter(vals + sl * M, tail + sl * M, M, m, n_tail);
        if (pos_out) *pos_out = rank;
        if (id_out) *id_out = m;
    }
    __syncthreads();
    float cv = 0.0f;
    if (own && m == 0) cv = tail_sum(tail + sl * M, n_tail);
    return cv;
}

// One workgroup's share of the rollouts of a step: item < n_nom_wg is a
// nominal workgroup (one lane per sample), otherwise a disturbed workgroup
// (spb samples of M lanes).  Ends with every lane past its last LDS access
// (the caller may reuse the LDS after a barrier).
template <int kNoise>
__device__ __forceinline__ void rollout_body(const StepConst& c, const float4* __restrict__ obs,
                                             const float* __restrict__ V, float2* __restrict__ u_out,
                                             float* __restrict__ S_out, float* __restrict__ cvar_out,
                                             float* __restrict__ L_out, int item, float2* smem,
                                             int* __restrict__ ranks = nullptr, int* __restrict__ tail_idx = nullptr,
                                             unsigned long long* __restrict__ work = nullptr) {
    float2* ctl = smem;
    float* vals = reinterpret_cast<float*>(ctl + (size_t)c.spb * c.T);
    float* tail = vals + c.spb * c.M;
    float* means = tail + c.spb * c.M;
    const int tid = threadIdx.x;
    const int spb = c.spb, M = c.M, T = c.T;
    const int n_grp = rollout_n_grp(c.n_obs);
    float4* otab = reinterpret_cast<float4*>(reinterpret_cast<float*>(smem) + rollout_otab_offset(spb, T, M));
    float4* gbox = otab + 64 * n_grp;
    for (int i = tid; i < n_grp * 64; i += blockDim.x) otab[i] = obstacle_entry(obs, c.n_obs, i, c.fx, c.fy);
    if (n_grp > 1 && tid < 64) group_bounds(obs, c.n_obs, n_grp, c.fx, c.fy, gbox);
    int n_cand = 0;   // exact obstacle tests (state step, obstacle) of this wave (wave-uniform)
    int n_gtest = 0;  // broad-phase group tests of this wave (wave-uniform)

    if (item < c.n_nom_wg) {
        // ---- nominal rollouts: one lane per sample; lanes past K repeat
        // the last sample (the obstacle test works on whole waves) and write
        // nothing.  V is staged into LDS (the controls' region, unused here),
        // so that no step waits for a global load ----
        __builtin_amdgcn_s_setprio(0);
        float* vsh = reinterpret_cast<float*>(ctl);  // 2T floats <= 2 spb T
        for (int i = tid; i < 2 * T; i += blockDim.x) vsh[i] = V[i];
        __syncthreads();  // otab and V staged
        const int k = item * blockDim.x + tid;
        const bool act = k < c.K;
        const bool store = act && c.store_u;
        const int kc = act ? k : c.K - 1;
        const float4 e0 = n_grp > 0 ? otab[tid & 63] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        State s{0.0f, 0.0f, c.psi0, c.v0};
        float acc = 0.0f, ctrl = 0.0f;
        int cnt = 0;
        const StepConst cn = with_vector_constants_nominal(c);
        const PhiloxVKeys vk = philox_vkeys(c.key0, c.key1);
        const uint32_t exp_word = in_vgpr_u(0x7Fu);
        // one nominal state step: the sampled control, running and control
        // costs at x_t (the control cost is summed in every case and used
        // when asked, so that the step holds no branch), then x_{t+1}
        auto step = [&](auto bdry, int t, float& px, float& py) {
            const float2 u = sample_control(cn, vsh, kc, t, vk, exp_word);
            if (store) u_out[(size_t)t * c.K + k] = u;
            acc = smooth_cost_acc<decltype(bdry)::value>(cn, s, acc);
            px = s.x;
            py = s.y;
            const float term = __fmaf_rn(vsh[2 * t] * cn.inv_var0, u.x, vsh[2 * t + 1] * cn.inv_var1 * u.y);
            ctrl = __fmaf_rn(cn.gamma, term, ctrl);
            bicycle_step(s, cn.dt * u.x, tan_steer(u.y) * cn.inv_wheelbase, cn.dt);
        };
        for (int t0 = 0; t0 < T; t0 += kCullSteps) {  // the obstacle test runs once per kCullSteps points
            float px[kCullSteps], py[kCullSteps];
            int n = kCullSteps;
            if (t0 + kCullSteps <= T) {  // a whole run of steps with no branch between them
                if (c.use_bdry) {
#pragma unroll
                    for (int i = 0; i < kCullSteps; ++i) step(kTrue, t0 + i, px[i], py[i]);
                } else {
#pragma unroll
                    for (int i = 0; i < kCullSteps; ++i) step(kFalse, t0 + i, px[i], py[i]);
                }
            } else {
                n = 0;
#pragma unroll
                for (int i = 0; i < kCullSteps; ++i) {
                    const int t = t0 + i;
                    if (t < T) {
                        if (c.use_bdry)
                            step(kTrue, t, px[i], py[i]);
                        else
                            step(kFalse, t, px[i], py[i]);
                        n = i + 1;
                    } else {
                        px[i] = px[i > 0 ? i - 1 : 0];
                        py[i] = py[i > 0 ? i - 1 : 0];
                    }
                }
            }
            if (n_grp > 0) cnt += obstacle_hits_culled<kCullSteps>(otab, gbox, n_grp, e0, px, py, n, n_cand, n_gtest);
        }
        float S = __fmaf_rn(c.c_obs, (float)cnt, acc);
        if (c.use_ctrl) S += ctrl;
        if (c.use_term) S += terminal_cost(c, s);
        if (act) S_out[k] = S;
        if (work && (tid & 63) == 0) {
            const int slot = (item * 16 + (tid >> 6)) & (kWorkSlots - 1);
            atomicAdd(&work[slot], (unsigned long long)n_cand);
            atomicAdd(&work[kWorkSlots + slot], (unsigned long long)n_gtest);
        }
        return;
    }

    // ---- disturbed rollouts: one lane per (sample, draw) ----
    // Where nominal and disturbed waves share a SIMD, the disturbed ones take
    // the issue slots first: there are M of them per sample against one
    // nominal lane per sample.  On the receding-horizon workload (K = 2048,
    // M = 64) this order gave the shortest one-launch step of the three
    // (equal priorities and nominal first were 2.7 us slower), although its
    // nominal waves then finish a few microseconds after the disturbed ones.
    __builtin_amdgcn_s_setprio(2);
    const int wg = item - c.n_nom_wg;
    // The workgroup's samples: spb of them, or with c.flat the (at most spb)
    // samples of its blockDim consecutive (sample, draw) pairs, k_first the
    // first of them.
    // (K M < 2^31 is checked on the host, so the pair indices fit 32 bits)
    const uint32_t KM = (uint32_t)c.K * (uint32_t)M;
    const uint32_t g0 = (uint32_t)wg * blockDim.x;  // flat: the first pair
    const int k_first = c.flat ? (int)(g0 / (uint32_t)M) : wg * spb;
    const int n_smp = c.flat ? (int)((min(g0 + blockDim.x, KM) - 1u) / (uint32_t)M) - k_first + 1 : spb;
    for (int idx = tid; idx < n_smp * T; idx += blockDim.x) {
        const int sl = idx / T;
        const int t = idx - sl * T;
        const int kk = k_first + sl;
        float2 cu = make_float2(0.0f, 0.0f);
        if (kk < c.K) {
            const float2 u = sample_control(c, V, kk, t);
            cu = make_float2(c.dt * u.x, tan_steer(u.y) * c.inv_wheelbase);
        }
        ctl[idx] = cu;
    }
    __syncthreads();

    int sl, m, k;
    if (c.flat) {  // lanes past the last pair repeat it, their results dropped
        const uint32_t g = min(g0 + (uint32_t)tid, KM - 1u);
        k = (int)(g / (uint32_t)M);
        m = (int)(g - (uint32_t)k * (uint32_t)M);
        sl = k - k_first;
    } else {
        sl = tid / M;
        m = tid - sl * M;
        k = wg * spb + sl;
    }
    float L = 0.0f;
    {
        const StepConst cv = with_vector_constants(c);
        const PhiloxVKeys vk = philox_vkeys(c.key0, c.key1);
        const uint32_t exp_word = in_vgpr_u(0x7Fu);
        // every lane runs a rollout (the obstacle test works on whole waves);
        // lanes past the workgroup's last sample repeat its controls, and the
        // results of inactive lanes are dropped
        const float2* ck = ctl + min(sl, n_smp - 1) * T;
        const float4 e0 = n_grp > 0 ? otab[tid & 63] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        State s{0.0f, 0.0f, c.psi0, c.v0};
        float acc = 0.0f;
        int cnt = 0;
        // one disturbed state step: running cost at x_t, then (t < T - 1; the
        // last draw cannot reach the risk cost) x_{t+1}
        auto step = [&](auto bdry, int t, bool advance, float& px, float& py) {
            acc = smooth_cost_acc<decltype(bdry)::value>(cv, s, acc);
            px = s.x;
            py = s.y;
            if (advance) {
                const uint4 r = philox4x32_10((uint32_t)t, (uint32_t)m, (uint32_t)k, c.step_idx, c.key0, c.key1, vk);
                const float2 cc = ck[t];
                bicycle_step(s, cc.x, cc.y, cv.dt);
                s = disturbed_successor<kNoise>(cv, r, s, exp_word);
            }
        };
        for (int t0 = 0; t0 < T; t0 += kCullSteps) {  // the obstacle test runs once per kCullSteps points
            float px[kCullSteps], py[kCullSteps];
            int n = kCullSteps;
            if (t0 + kCullSteps < T) {
                // a whole run of steps with no branch between them, so that
                // the noise of later steps can be computed beside the
                // dynamics of earlier ones
                if (c.use_bdry) {
#pragma unroll
                    for (int i = 0; i < kCullSteps; ++i) step(kTrue, t0 + i, true, px[i], py[i]);
                } else {
#pragma unroll
                    for (int i = 0; i < kCullSteps; ++i) step(kFalse, t0 + i, true, px[i], py[i]);
                }
            } else {
                n = 0;
#pragma unroll
                for (int i = 0; i < kCullSteps; ++i) {
                    const int t = t0 + i;
                    if (t < T) {
                        if (c.use_bdry)
                            step(kTrue, t, t + 1 < T, px[i], py[i]);
                        else
                            step(kFalse, t, t + 1 < T, px[i], py[i]);
                        n = i + 1;
                    } else {
                        px[i] = px[i > 0 ? i - 1 : 0];
                        py[i] = py[i > 0 ? i - 1 : 0];
                    }
                }
            }
            if (n_grp > 0) cnt += obstacle_hits_culled<kCullSteps>(otab, gbox, n_grp, e0, px, py, n, n_cand, n_gtest);
        }
        L = __fmaf_rn(c.c_obs, (float)cnt, acc);
    }
    if (c.flat) {
        // the risk costs go to memory; a separate pass forms each sample's
        // CVaR from them (k_cvar_sorted, the same order); the pair index again
        // from a copy of the thread index (see below)
        int tid_f = tid;
        asm volatile("" : "+v"(tid_f));
        const uint32_t g = (uint32_t)wg * blockDim.x + (uint32_t)tid_f;
        if (g < KM) L_out[g] = L;
        if (work && (tid & 63) == 0) {
            const int slot = (item * 16 + (tid >> 6)) & (kWorkSlots - 1);
            atomicAdd(&work[slot], (unsigned long long)n_cand);
            atomicAdd(&work[kWorkSlots + slot], (unsigned long long)n_gtest);
        }
        return;
    }
    // The lane's sample and draw again, from copies of the thread index and
    // of M that the compiler cannot tie to the ones above: the values derived
    // before the rollout (the quotient, the divisor's reciprocal) then need
    // no register through it (the rollout kernel runs at its register limit,
    // and keeping them cost scratch-memory spills).
    int tid_e = tid, M_e = M;
    asm volatile("" : "+v"(tid_e), "+s"(M_e));
    const int sl_e = tid_e / M_e;
    const int m_e = tid_e - sl_e * M_e;
    const int k_e = wg * spb + sl_e;
    const bool active_e = (sl_e < spb) && (k_e < c.K);
    if (active_e && c.debug) L_out[(size_t)k_e * M + m_e] = L;
    if (sl_e < spb) {
        vals[tid_e] = active_e ? L : 0.0f;
        tail[tid_e] = __builtin_nanf("");
    }
    int pos = M, id = m_e;
    const float cv = cvar_epilogue(vals, tail, means, spb, M_e, c.n_tail, c.scale_risk, c.B, &pos, &id, tid_e);
    if (active_e && m_e == 0) cvar_out[k_e] = cv;
    if (c.grad && active_e) {  // tail membership for the gradient
        ranks[(size_t)k_e * M + id] = pos;
        if (pos < c.n_tail) tail_idx[(size_t)k_e * c.n_tail + pos] = id;
    }
    if (work && (tid & 63) == 0) {
        const int slot = (item * 16 + (tid >> 6)) & (kWorkSlots - 1);
        atomicAdd(&work[slot], (unsigned long long)n_cand);
        atomicAdd(&work[kWorkSlots + slot], (unsigned long long)n_gtest);
    }
}

// Sum and minimum of 256 values held in LDS (v[0..255]) in a fixed order that
// does not depend on the workgroup size: wave-sized segments of 64 values are
// reduced by the butterflies of wave_sum / wave_min, the four segment results
// combined as (s0 + s1) + (s2 + s3).  Every thread of the workgroup (a
// multiple of 64 threads) must call them; the result is returned to all.
// red holds at least 16 floats of LDS.
__device__ __forceinline__ float seg_sum_256(const float* v, float* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();  // v written
    for (int sg = wv; sg < 4; sg += nw) {
        const float x = wave_sum(v[64 * sg + lane]);
        if (lane == 0) red[sg] = x;
    }
    __syncthreads();
    const float r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();  // red and v free again
    return r;
}

__device__ __forceinline__ float seg_min_256(const float* v, float* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    for (int sg = wv; sg < 4; sg += nw) {
        const float x = wave_min(v[64 * sg + lane]);
        if (lane == 0) red[sg] = x;
    }
    __syncthreads();
    const float r = fminf(fminf(red[0], red[1]), fminf(red[2], red[3]));
    __syncthreads();
    return r;
}

// Weights and update (Eq. 14-17 and Eq. 4), in chunks of 256 samples; any
// workgroup size that is a multiple of 64 gives the same bits.
//  1. (update_chunk) S~ = S + J_C per sample of chunk b; the chunk's minimum
//     beta_b, its weights exp(-(S~ - beta_b)/lambda) and their sum Z_b;
//  2. (update_chunk) the chunk's weighted control sums N_b[t] = sum_k w_k
//     u_{k,t}, item (t, part) summing a contiguous slice of the chunk, the
//     slices then added in order; (beta_b, Z_b, N_b) go to part[b];
//  3. (update_merge, run by whoever finishes the last chunk) beta = min
//     beta_b, scale_b = exp(-(beta_b - beta)/lambda), V+ = sum_b scale_b N_b /
//     sum_b scale_b Z_b; then V (shifted when asked), the first command and,
//     in debug mode, w_hat; in gradient mode J, every w_hat and the list of
//     samples of non-zero weight instead, V unchanged.
// LDS (dynamic, ush): w[256] | slice sums [parts][2T] | nzpos[257] |
// nzlist[256] | mean sequence [2T], then for the merge v[256] | scale[G] |
// zb[G] | vp[2T] (update_lds_bytes).
//
// With kRegen the chunk draws the controls of its samples of non-zero
// weight again from the same Philox counters and the same V (which the merge
// rewrites only after every chunk is in) instead of reading stored ones:
// sample_control is the function that drew them, so the values are the same
// bits.  Stored controls would have been written by workgroups on other
// XCDs, and each round of loads waits about 1.4 us for memory, while a
// redrawn control costs a few tens of instructions; so a step stores no
// controls unless the debug view or the gradient asks for them, and even a
// chunk whose every weight is non-zero is summed sooner than by loading.
// Where the controls are stored, the two-launch update reads them (the
// one-launch update still draws them), so the bit-exact comparison of the
// two forms in debug mode also checks that the drawn controls are the stored
// ones.
template <int kB, bool kRegen = false>
__device__ __forceinline__ void update_chunk(const StepConst& c, int b, int parts, const float* __restrict__ S,
                                             const float* __restrict__ cvar, const float2* __restrict__ u,
                                             float* __restrict__ S_tilde, float* __restrict__ part, float* ush,
                                             float* red, const float* __restrict__ V = nullptr) {
    const int T = c.T, K = c.K;
    const int tid = threadIdx.x, nt = blockDim.x;
    float* wsh = ush;
    float* psh = wsh + 256;
    int* nzpos = reinterpret_cast<int*>(psh + (size_t)parts * 2 * T);  // 257
    int* nzlist = nzpos + 257;                                          // 256
    float* vsh = reinterpret_cast<float*>(nzlist + 256);                // 2T
    const int k0 = b * 256;
    const int n = min(256, K - k0);
    const int stride = 2 + 2 * T;
    const int slice = (n + parts - 1) / parts;
    // V (for the redrawn controls) is staged into LDS after the first step
    // below, but the thread's first value is loaded now, so that its load and
    // the first wave's loads of S and CVaR wait on memory together
    const bool has_v = kRegen && tid < 2 * T;
    const float v_first = has_v ? V[tid] : 0.0f;

    // 1. modified costs, the chunk's minimum beta_b, its weights and their
    // sum Z_b, and the samples of non-zero weight, all by the first wave:
    // lane l holds samples l, l + 64, l + 128 and l + 192 (the four 64-value
    // segments of seg_min_256 / seg_sum_256, reduced by the same butterflies
    // and combined in the same order, so the bits are theirs), and no
    // barrier separates the steps.  The samples of non-zero weight go to
    // nzlist in index order (exp underflows to an exact zero once a cost
    // exceeds the chunk's minimum by about 104 lambda), nzpos[k] counting
    // how many come before sample k.  A zero weight adds 0 * u, which leaves
    // a sum exactly as it is, so the sums below skip those samples and still
    // give the bits of the full sums.
    float beta_b = 0.0f, Z_b = 0.0f;
    if (tid < 64) {
        // the eight loads first (a lane past the chunk's end reads its last
        // sample and drops it), so that they wait on memory once, not once
        // per segment
        float cvl[4], sl[4];
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
            const int i = min(64 * sg + tid, n - 1);
            cvl[sg] = cvar[k0 + i];
            sl[sg] = S[k0 + i];
        }
        float w[4];
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
            const int i = 64 * sg + tid;
            float st = __builtin_inff();
            if (i < n) {
                const float cv = cvl[sg];
                const float jc = (cv > c.C_u) ? c.A * cv : 0.0f;  // Eq. 14-15
                st = sl[sg] + jc;                                  // Eq. 16
                S_tilde[k0 + i] = st;
            }
            w[sg] = st;
        }
        beta_b = wave_min(fminf(fminf(w[0], w[1]), fminf(w[2], w[3])));  // a minimum: exact in any order
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) w[sg] = (64 * sg + tid < n) ? expf(-(w[sg] - beta_b) / c.lambda) : 0.0f;
        Z_b = (wave_sum(w[0]) + wave_sum(w[1])) + (wave_sum(w[2]) + wave_sum(w[3]));
        int off = 0;
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
            const int k = 64 * sg + tid;
            const uint64_t bal = __builtin_amdgcn_ballot_w64(w[sg] != 0.0f);
            const int q = off + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            nzpos[k] = q;
            if (w[sg] != 0.0f) nzlist[q] = k;
            wsh[k] = w[sg];
            off += __builtin_popcountll(bal);
        }
        if (tid == 0) nzpos[256] = off;
    }
    if (kRegen) {
        if (has_v) vsh[tid] = v_first;
        for (int i = tid + nt; i < 2 * T; i += nt) vsh[i] = V[i];
    }
    __syncthreads();  // wsh, nzpos, nzlist and V published

    // 2. weighted control sums over slices of the chunk, in index order
    for (int idx = tid; idx < T * parts; idx += nt) {
        const int t = idx / parts;  // neighbouring lanes read the slices of one row
        const int pr = idx % parts;
        const int ka = pr * slice, kb = min(n, ka + slice);
        float ax = 0.0f, ay = 0.0f;
        int q = ka < kb ? nzpos[ka] : 0;
        const int qb = ka < kb ? nzpos[kb] : 0;
        if constexpr (kRegen) {
            for (; q < qb; ++q) {
                const int k = nzlist[q];
                const float ww = wsh[k];
                const float2 uu = sample_control(c, vsh, k0 + k, t);
                ax = __fmaf_rn(ww, uu.x, ax);
                ay = __fmaf_rn(ww, uu.y, ay);
            }
        } else {
            const float2* ut = u + (size_t)t * K + k0;
            for (; q + kB <= qb; q += kB) {  // kB loads in flight, then the sums in order
                float2 uu[kB];
                float ww[kB];
#pragma unroll
                for (int i = 0; i < kB; ++i) {
                    const int k = nzlist[q + i];
                    ww[i] = wsh[k];
                    uu[i] = ut[k];
                }
#pragma unroll
                for (int i = 0; i < kB; ++i) {
                    ax = __fmaf_rn(ww[i], uu[i].x, ax);
                    ay = __fmaf_rn(ww[i], uu[i].y, ay);
                }
            }
            if (q < qb) {  // the rest in one more round
                float2 uu[kB];
                float ww[kB];
#pragma unroll
                for (int i = 0; i < kB; ++i) {
                    const bool in = q + i < qb;
                    const int k = in ? nzlist[q + i] : 0;
                    ww[i] = in ? wsh[k] : 0.0f;
                    uu[i] = in ? ut[k] : make_float2(0.0f, 0.0f);
                }
#pragma unroll
                for (int i = 0; i < kB; ++i) {
                    if (q + i < qb) {
                        ax = __fmaf_rn(ww[i], uu[i].x, ax);
                        ay = __fmaf_rn(ww[i], uu[i].y, ay);
                    }
                }
            }
        }
        psh[(size_t)pr * 2 * T + 2 * t] = ax;
        psh[(size_t)pr * 2 * T + 2 * t + 1] = ay;
    }
    __syncthreads();
    float* pb = part + (size_t)b * stride;
    for (int j = tid; j < 2 * T; j += nt) {
        float acc = 0.0f;
        for (int pr = 0; pr < parts; ++pr) acc += psh[(size_t)pr * 2 * T + j];
        pb[2 + j] = acc;
    }
    if (tid == 0) {
        pb[0] = beta_b;
        pb[1] = Z_b;
    }
    __syncthreads();  // LDS free for the caller
}

// The merge's last part, once vp (2T) holds V+ in LDS and beta, Z (and
// invZ = 1 / Z) are known: V (shifted when asked), the first command and the
// completion word, w_hat in debug mode; in gradient mode J, every w_hat and
// the samples of non-zero weight instead, V unchanged.
__device__ __forceinline__ void merge_finish(const StepConst& c, float beta, float Z, float invZ, const float* vp,
                                             const float* __restrict__ S_tilde, float* __restrict__ V,
                                             float* __restrict__ u0, float* __restrict__ u0_host,
                                             float* __restrict__ w_hat, float* red, const GradOut* go) {
    const int T = c.T, K = c.K;
    const int tid = threadIdx.x, nt = blockDim.x;
    __syncthreads();
    if (go) {
        // gradient mode: V stays as it is; write J = beta - lambda log(Z/K),
        // every w_hat, and the samples of non-zero weight in increasing order
        if (tid == 0) *go->J = beta - c.lambda * logf(Z / (float)K);
        // thread i takes the contiguous samples [i q, (i + 1) q): its count of
        // non-zero weights, an exclusive prefix of the counts in thread order
        // (lane scan, then the wave totals), and its samples go to the list
        // from there, so the list is in increasing order
        const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
        const int q = (K + nt - 1) / nt;
        const int ka = min(K, tid * q), kb = min(K, ka + q);
        int cnt = 0;
        for (int k = ka; k < kb; ++k) {
            const float wk = expf(-(S_tilde[k] - beta) / c.lambda) * invZ;
            w_hat[k] = wk;
            cnt += wk > 0.0f;
        }
        int incl = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(incl, d);
            if (lane >= d) incl += o;
        }
        if (lane == 63) red[wv] = __int_as_float(incl);
        __syncthreads();
        int pos = incl - cnt, total = 0;
        for (int w = 0; w < nw; ++w) {
            const int cw = __float_as_int(red[w]);
            pos += (w < wv) ? cw : 0;
            total += cw;
        }
        for (int k = ka; k < kb; ++k)
            if (w_hat[k] > 0.0f) go->act_list[pos++] = k;  // this thread's own stores
        if (tid == 0) *go->n_act = total;
        return;
    }
    const int shift = (c.flags & 2u) != 0;
    for (int j = tid; j < 2 * T; j += nt) {
        int src = j;
        if (shift) src = min(j + 2, 2 * T - 2 + (j & 1));
        V[j] = vp[src];
    }
    if (tid < 2) u0[tid] = vp[tid];
    // The completion word may release the next served step, whose workgroups
    // read V: every wave's stores of V must precede thread 0's release, so
    // the workgroup meets at a barrier first (with T > 32 the stores come
    // from more than one wave).
    if (u0_host) __syncthreads();
    if (tid == 0 && u0_host) {  // mapped pinned host memory
        u0_host[0] = vp[0];
        u0_host[1] = vp[1];
        if (c.u0_seq)  // completion word, ordered after the command at system scope
            __hip_atomic_store(reinterpret_cast<unsigned*>(u0_host + 2), c.u0_seq, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (c.debug) {
        for (int k = tid; k < K; k += nt) w_hat[k] = expf(-(S_tilde[k] - beta) / c.lambda) * invZ;
    }
}

template <int kB>
__device__ __forceinline__ void update_merge(const StepConst& c, int G, const float* __restrict__ part,
                                             const float* __restrict__ S_tilde, float* __restrict__ V,
                                             float* __restrict__ u0, float* __restrict__ u0_host,
                                             float* __restrict__ w_hat, float* ush, float* red,
                                             const GradOut* go = nullptr) {
    const int T = c.T;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int stride = 2 + 2 * T;
    float* vsh = ush;  // 256 per-virtual-thread values
    float* scale = vsh + 256;
    float* zb = scale + G;
    float* vp = zb + G;
    // rows of the weighted sums loaded before beta and Z are known
    constexpr int kP = kB > 8 ? kB : 8;

    // The first kP rows of the weighted sums (thread j < 2T) do not depend
    // on beta or Z: their loads are issued first.
    float pre[kP];
    const int n_pre = G < kP ? G : kP;
    const bool has_pre = tid < 2 * T;
    if (has_pre) {
#pragma unroll
        for (int i = 0; i < kP; ++i) pre[i] = i < n_pre ? part[(size_t)i * stride + 2 + tid] : 0.0f;
    }
    float beta, Z;
    if (G <= 64) {
        // one wave, chunk b in lane b: the minimum (exact in any order), the
        // scales, and Z by the butterfly of seg_sum_256's first segment (its
        // other three segments hold zeros, whose sums add nothing to a
        // positive Z, so the bits are the same); one barrier publishes them
        if (tid < 64) {
            const bool in = tid < G;
            const float be = in ? part[(size_t)tid * stride] : __builtin_inff();
            const float z0 = in ? part[(size_t)tid * stride + 1] : 0.0f;
            const float bmin = wave_min(be);
            const float sc = in ? expf(-(be - bmin) / c.lambda) : 0.0f;
            const float zs = wave_sum(__fmaf_rn(z0, sc, 0.0f));
            if (in) scale[tid] = sc;
            if (tid == 0) {
                red[0] = bmin;
                red[1] = zs;
            }
        }
        __syncthreads();
        beta = red[0];
        Z = red[1];
    } else {
        // virtual thread i (of 256) takes chunks i, i + 256, ...; beta_b and
        // Z_b are read once and kept in LDS
        for (int i = tid; i < 256; i += nt) {
            float m = __builtin_inff();
            for (int bb = i; bb < G; bb += 256) {
                const float be = part[(size_t)bb * stride];
                scale[bb] = be;
                zb[bb] = part[(size_t)bb * stride + 1];
                m = fminf(m, be);
            }
            vsh[i] = m;
        }
        beta = seg_min_256(vsh, red);  // also publishes scale (beta_b) and zb
        for (int i = tid; i < 256; i += nt) {
            float z = 0.0f;
            for (int bb = i; bb < G; bb += 256) {
                const float sc = expf(-(scale[bb] - beta) / c.lambda);
                scale[bb] = sc;
                z = __fmaf_rn(zb[bb], sc, z);
            }
            vsh[i] = z;
        }
        Z = seg_sum_256(vsh, red);  // also publishes scale
    }
    const float invZ = 1.0f / Z;
    for (int j = tid; j < 2 * T; j += nt) {
        float acc = 0.0f;
        int bb = 0;
        if (j == tid && has_pre) {  // the prefetched rows, summed in the same order
#pragma unroll
            for (int i = 0; i < kP; ++i)
                if (i < n_pre) acc = __fmaf_rn(pre[i], scale[i], acc);
            bb = n_pre;
        }
        for (; bb + kB <= G; bb += kB) {  // kB loads in flight, then the sums in order
            float pv[kB];
#pragma unroll
            for (int i = 0; i < kB; ++i) pv[i] = part[(size_t)(bb + i) * stride + 2 + j];
#pragma unroll
            for (int i = 0; i < kB; ++i) acc = __fmaf_rn(pv[i], scale[bb + i], acc);
        }
        if (bb < G) {  // the rest in one more round (padding terms 0 * 0)
            float pv[kB], sv[kB];
#pragma unroll
            for (int i = 0; i < kB; ++i) {
                const bool in = bb + i < G;
                pv[i] = in ? part[(size_t)(bb + i) * stride + 2 + j] : 0.0f;
                sv[i] = in ? scale[bb + i] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < kB; ++i) acc = __fmaf_rn(pv[i], sv[i], acc);
        }
        vp[j] = acc * invZ;
    }
    merge_finish(c, beta, Z, invZ, vp, S_tilde, V, u0, u0_host, w_hat, red, go);
}

// The merge when there is one chunk (K <= 256), run by the workgroup that
// has just written its partial record: beta = beta_0, every scale is
// exp(0) = 1 and Z = Z_0, so V+ = N_0 / Z_0 -- the bits of update_merge
// with G = 1, without the counter, the reductions or a device-scope wait.
__device__ __forceinline__ void update_merge_single(const StepConst& c, const float* part,
                                                    const float* __restrict__ S_tilde, float* __restrict__ V,
                                                    float* __restrict__ u0, float* __restrict__ u0_host,
                                                    float* __restrict__ w_hat, float* ush, float* red,
                                                    const GradOut* go = nullptr) {
    const float beta = part[0];
    const float Z = part[1];
    const float invZ = 1.0f / Z;
    float* vp = ush + 256 + 2;  // the place update_merge gives it for G = 1
    for (int j = threadIdx.x; j < 2 * c.T; j += blockDim.x) vp[j] = part[2 + j] * invZ;
    merge_finish(c, beta, Z, invZ, vp, S_tilde, V, u0, u0_host, w_hat, red, go);
}

// Thread 0 adds one to a device-scope counter with acquire-release order
// (after the barrier that orders the workgroup's earlier stores before it);
// returns to every thread whether this made it reach `target`, in which case
// the counter is reset to zero and every thread has acquired what the other
// increments published.
__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned target, int* flag_sh) {
    __syncthreads();
    if (threadIdx.x == 0) {
        // a release increment; only the last arrival acquires (the others
        // leave their caches as they are)
        const unsigned done = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        *flag_sh = (done == target - 1u);
        if (*flag_sh) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    const bool last = *flag_sh != 0;
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return last;
}

// Loads in flight per thread in the update run inside the rollout launch,
// whose register budget is the rollout's (the separate update launch uses 16).
constexpr int kFuseBatch = 4;

// Buffers of the update run inside the rollout launch (one step in one
// kernel), held in device memory so that they occupy no registers during the
// rollouts.
struct FuseArgs {
    unsigned* chunk_ctr;  // G counters of finished contributors (zero between launches)
    unsigned* counter;    // chunks finished (zero between launches)
    float* S_tilde;
    float* part;
    float* u0;
    float* u0_host;       // mapped host buffer, written when the step asks for the first command
    float* w_hat;
    int G, parts;
};

// FuseArgs as read from device memory, its pointers in the global address
// space (as_global).
__device__ __forceinline__ FuseArgs global_view(const FuseArgs& f) {
    FuseArgs g = f;
    g.chunk_ctr = as_global(f.chunk_ctr);
    g.counter = as_global(f.counter);
    g.S_tilde = as_global(f.S_tilde);
    g.part = as_global(f.part);
    g.u0 = as_global(f.u0);
    g.u0_host = as_global(f.u0_host);
    g.w_hat = as_global(f.w_hat);
    return g;
}

// ---- persistent serving: one resident launch runs step after step ----

// One served step's request: the per-step constants the host derives from
// the measured state (the same arithmetic as for a launched step), written
// into mapped host memory with seq last; the leader workgroup copies it to
// device memory for the others.
struct ServeReq {
    uint32_t seq;   // request number, 1, 2, ... within a session
    uint32_t stop;  // non-zero: leave the loop
    uint32_t step_idx;
    uint32_t pad0;
    float fx, fy, tox, toy, theta0, psi0, v0, pad1;
};
static_assert(sizeof(ServeReq) == 48, "ServeReq is read as three 16-byte words");

struct ServeArgs {
    const ServeReq* req_host;  // mapped host memory (device address)
    ServeReq* req_dev;         // device copy read by every workgroup
    unsigned* go;              // request number being served, or kServeExit
    uint64_t idle_ticks;       // longest wait for a request (s_memrealtime ticks, 100 MHz)
};

__device__ __forceinline__ ServeArgs global_view(const ServeArgs& a) {
    ServeArgs g = a;
    g.req_host = as_global(a.req_host);
    g.req_dev = as_global(a.req_dev);
    g.go = as_global(a.go);
    return g;
}

constexpr unsigned kServeExit = 0xFFFFFFFFu;

// Workgroup 0's thread 0: waits for request seq in host memory, copies it to
// device memory and publishes seq in `go`; on a stop request or after
// idle_ticks without one it publishes kServeExit.  Returns whether to leave.
__device__ __forceinline__ bool serve_wait_leader(const ServeArgs& sa, unsigned seq) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        // relaxed polls (no cache invalidation while other workgroups may
        // still be finishing the last step), one acquire once it has come
        if (__hip_atomic_load(&sa.req_host->seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == seq) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            const ServeReq* r = sa.req_host;
            if (__hip_atomic_load(&r->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) break;
            // three 16-byte reads across PCIe instead of one per field
            // (after the acquire above, so they see the posted request)
            ServeReq* d = sa.req_dev;
            const uint4 a = *reinterpret_cast<const uint4*>(r);
            const float4 b = *reinterpret_cast<const float4*>(&r->fx);
            const float4 e = *reinterpret_cast<const float4*>(&r->theta0);
            d->step_idx = a.z;
            d->fx = b.x;
            d->fy = b.y;
            d->tox = b.z;
            d->toy = b.w;
            d->theta0 = e.x;
            d->psi0 = e.y;
            d->v0 = e.z;
            __hip_atomic_store(sa.go, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if (__builtin_amdgcn_s_memrealtime() - t0 > sa.idle_ticks) break;
        __builtin_amdgcn_s_sleep(1);
    }
    __hip_atomic_store(sa.go, kServeExit, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Thread 0 of every other workgroup: waits until `go` names request seq
// (serve) or kServeExit (leave); leaves too after twice the leader's limit.
__device__ __forceinline__ bool serve_wait_member(const ServeArgs& sa, unsigned seq) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        const unsigned g = __hip_atomic_load(sa.go, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (g == seq) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return false;
        }
        if (g == kServeExit || __builtin_amdgcn_s_memrealtime() - t0 > 2 * sa.idle_ticks) return true;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Workgroups of a rollout launch whose samples fall in chunk b: the nominal
// workgroups (block samples each) and the disturbed ones (spb samples each).
__device__ __forceinline__ unsigned chunk_contributors(const StepConst& c, int b, int block) {
    const int klo = 256 * b, khi = min(c.K, klo + 256) - 1;
    return (unsigned)((khi / block - klo / block + 1) + (khi / c.spb - klo / c.spb + 1));
}

// After a rollout workgroup has stored its results: it counts itself in the
// chunks its samples fall in, and for every chunk it completes runs that
// chunk's update (its inputs S, CVaR and u are then all stored, published by
// the other workgroups' releases); the workgroup that completes the last
// chunk merges them.  No workgroup waits for another.
__device__ __forceinline__ void fused_update(const StepConst& c, const FuseArgs& f, int item, const float* S,
                                             const float* cvar, const float2* u, float* V, float* ush, float* red,
                                             int* flag_sh, int* fin_sh) {
    int lo, hi;
    if (item < c.n_nom_wg) {
        lo = item * (int)blockDim.x;
        hi = min(c.K, lo + (int)blockDim.x);
    } else {
        lo = (item - c.n_nom_wg) * c.spb;
        hi = min(c.K, lo + c.spb);
    }
    __syncthreads();  // the workgroup's stores precede thread 0's release; LDS free
    if (threadIdx.x == 0) {
        int nf = 0;
        for (int b = lo >> 8; b <= (hi - 1) >> 8; ++b) {
            const unsigned target = chunk_contributors(c, b, (int)blockDim.x);
            // a release increment; only the workgroup that completes the
            // chunk acquires, so the others keep their caches
            const unsigned done =
                __hip_atomic_fetch_add(&f.chunk_ctr[b], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (done == target - 1u) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(&f.chunk_ctr[b], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                fin_sh[nf++] = b;
            }
        }
        fin_sh[7] = nf;
    }
    __syncthreads();
    const int nf = fin_sh[7];
    if (nf == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int i = 0; i < nf; ++i) {
        update_chunk<kFuseBatch, true>(c, fin_sh[i], f.parts, S, cvar, u, f.S_tilde, f.part, ush, red, V);
        if (f.G == 1)  // its own record, visible to the workgroup after update_chunk's barrier
            update_merge_single(c, f.part, f.S_tilde, V, f.u0, c.u0_seq ? f.u0_host : nullptr, f.w_hat, ush, red);
        else if (arrive_last(f.counter, (unsigned)f.G, flag_sh))
            update_merge<kFuseBatch>(c, f.G, f.part, f.S_tilde, V, f.u0, c.u0_seq ? f.u0_host : nullptr, f.w_hat,
                                     ush, red);
    }
}

// One chunk of the update, and the merge when it is the last chunk to finish
// (a separate launch of G workgroups, one chunk each).  No workgroup waits
// for another, and every sum runs in a fixed order.
__device__ __forceinline__ void update_body(const StepConst& c, int b, int G, int parts, const float* __restrict__ S,
                                            const float* __restrict__ cvar, const float2* __restrict__ u,
                                            float* __restrict__ S_tilde, float* part, unsigned* counter,
                                            float* __restrict__ V, float* __restrict__ u0,
                                            float* __restrict__ u0_host, float* __restrict__ w_hat, float* ush,
                                            float* red, int* flag_sh, const GradOut* go = nullptr) {
    // the stored controls when the rollouts stored them (debug and
    // gradient modes), else the same controls drawn again
    if (c.store_u)
        update_chunk<16>(c, b, parts, S, cvar, u, S_tilde, part, ush, red);
    else
        update_chunk<16, true>(c, b, parts, S, cvar, u, S_tilde, part, ush, red, V);
    if (G == 1) {
        update_merge_single(c, part, S_tilde, V, u0, u0_host, w_hat, ush, red, go);
        return;
    }
    if (!arrive_last(counter, (unsigned)G, flag_sh)) return;
    update_merge<16>(c, G, part, S_tilde, V, u0, u0_host, w_hat, ush, red, go);
}

}  // namespace ramppi
