// Device building blocks of the RA-MPPI step for gfx950 (MI355X).
//
// Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the Box-Muller
// transform (Box & Muller 1958).  Model: rear-axle kinematic bicycle with a
// forward-Euler step (Eq. 1).  Costs: the running cost of Eq. 20-22 on an
// elliptic centreline with the signed Sampson distance, the terminal cost of
// Eq. 23.  Risk: the tail mean of Eq. 10-13 on the scaled costs of Eq. 18-19.
//
// All arithmetic is FP32 (round to nearest even, no fast-math), except the
// integer Philox rounds and the integer collision counts.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <stdint.h>

namespace ramppi {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;
// Second counter word of the control-noise stream (disturbance draws use m).
constexpr uint32_t kCtrlWord = 0xFFFFFFFFu;

// Philox4x32 with 10 rounds.  Round: words 0 and 2 are multiplied by the two
// multipliers (full 64-bit products); the new counter is
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key
// then advances by the two Weyl constants.
// a ^ b ^ k in one instruction (gfx950's three-input bitwise operation with
// the truth table of XOR3); k is the key word, the same in every lane, read
// from a scalar register (xor3_key) or from a vector register that holds it
// in every lane (xor3_vkey).
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "s"(k));
    return d;
}

__device__ __forceinline__ uint32_t xor3_vkey(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "v"(k));
    return d;
}

// A lane-uniform value copied into a vector register.  A VALU instruction of
// gfx950 that reads a scalar register does not pair with a VALU instruction
// of another wave in the same cycle (measured: an FMA with a scalar operand
// takes about 4.7 SIMD clocks per wave, one with vector operands about 3),
// so the constants that the rollout steps read at every step are kept in
// vector registers.
__device__ __forceinline__ float in_vgpr(float s) {
    float v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

__device__ __forceinline__ uint32_t in_vgpr_u(uint32_t s) {
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// A pointer read from device memory (not a kernel argument) into device or
// mapped host memory, in the global address space.  The compiler cannot tell
// where such a pointer points and accesses it with flat instructions, which
// also count against the LDS counter: every later wait for an LDS access
// then waits for them too (after a device-scope acquire, a memory round
// trip).  The integer round trip keeps the compiler from folding the
// address-space cast away, so the accesses through the result compile to
// global instructions.
template <class T>
__device__ __forceinline__ T* as_global(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

// The keys of the fourth to the tenth round in vector registers (the rounds
// before them XOR words that are still the same in every lane, on the
// scalar unit).
struct PhiloxVKeys {
    uint32_t k0[7], k1[7];
};

__device__ __forceinline__ PhiloxVKeys philox_vkeys(uint32_t k0, uint32_t k1) {
    PhiloxVKeys v;
#pragma unroll
    for (int r = 0; r < 7; ++r) {
        v.k0[r] = in_vgpr_u(k0 + (uint32_t)(r + 3) * kPhiloxW0);
        v.k1[r] = in_vgpr_u(k1 + (uint32_t)(r + 3) * kPhiloxW1);
    }
    return v;
}

// kVecKeys: the keys of rounds 4 to 10 come from vk (vector registers),
// otherwise from the scalar key schedule.  Both give the same words.
template <bool kVecKeys>
__device__ __forceinline__ uint4 philox4x32_10_rounds(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                      uint32_t k0, uint32_t k1, const PhiloxVKeys* vk) {
    {
        // first round in plain C: counter words that are the same in every
        // lane (the time step, the call index) then stay on the scalar unit
        const uint64_t p0 = (uint64_t)c0 * kPhiloxM0;
        const uint64_t p1 = (uint64_t)c2 * kPhiloxM1;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)c0 * kPhiloxM0;  // one v_mad_u64_u32 each
        const uint64_t p1 = (uint64_t)c2 * kPhiloxM1;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        // the second and third rounds still see words that are the same in
        // every lane (from the first round's scalar words): plain XORs let
        // the compiler fold the key into them on the scalar unit; from the
        // fourth round on every word differs per lane
        uint32_t n0, n2;
        if (r < 3) {
            n0 = hi1 ^ c1 ^ k0;
            n2 = hi0 ^ c3 ^ k1;
        } else if (kVecKeys) {
            n0 = xor3_vkey(hi1, c1, vk->k0[r - 3]);
            n2 = xor3_vkey(hi0, c3, vk->k1[r - 3]);
        } else {
            n0 = xor3_key(hi1, c1, k0);
            n2 = xor3_key(hi0, c3, k1);
        }
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
    return philox4x32_10_rounds<false>(c0, c1, c2, c3, k0, k1, nullptr);
}

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1, const PhiloxVKeys& vk) {
    return philox4x32_10_rounds<true>(c0, c1, c2, c3, k0, k1, &vk);
}

// uint32 -> (0, 1): ((r >> 9) + 1/2) 2^-23, exact in FP32.  Built as the
// float 1 + (r >> 9) 2^-23 (exponent bits 0x7F over the top 23 bits of r, one
// funnel shift) minus (1 - 2^-24), a subtraction that is exact (both lie in
// [1/2, 2] of each other and the result needs 24 significant bits).
__device__ __forceinline__ float uniform01(uint32_t r) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, r, 9u)) - 0x1.fffffep-1f;
}

// The same map with the exponent word 0x7F passed in (a vector register
// holding it keeps the shift from reading a scalar register).
__device__ __forceinline__ float uniform01(uint32_t r, uint32_t exp_word) {
    return __uint_as_float(__builtin_amdgcn_alignbit(exp_word, r, 9u)) - 0x1.fffffep-1f;
}

// Two standard normals from two uniforms (Box-Muller).  The hardware
// logarithm is base 2 and the hardware sine / cosine take revolutions, so
// -2 ln u0 = -2 ln(2) log2(u0) and cos(2 pi u1) is v_cos_f32(u1).  u0 lies in
// [2^-24, 1), a normal number, and u1 in (0, 1), inside the hardware range.
__device__ __forceinline__ void box_muller(float u0, float u1, float& z0, float& z1) {
    const float rad = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u0));
    z0 = rad * __builtin_amdgcn_cosf(u1);
    z1 = rad * __builtin_amdgcn_sinf(u1);
}

// Disturbance of one (sample, draw, step) from its Philox words, in the form
// selected at compile time: Gaussian sqrt(Sigma_w) z; uniform h (2u - 1) with
// h = sqrt(3 Sigma_w); impulse: a jump of length jump_size at angle 2 pi u1 in
// the (x, y) plane when u0 < jump_prob, otherwise zero.
template <int kNoise>
__device__ __forceinline__ float4 disturbance(const struct StepConst& c, uint4 r);

__device__ __forceinline__ float4 normals4(uint4 r) {
    float4 z;
    box_muller(uniform01(r.x), uniform01(r.y), z.x, z.y);
    box_muller(uniform01(r.z), uniform01(r.w), z.z, z.w);
    return z;
}

// Per-launch constants of one step, passed by value as a kernel argument.
struct StepConst {
    int32_t K, T, M, n_obs;
    int32_t spb;         // samples per disturbed workgroup
    int32_t n_nom_wg;    // nominal workgroups: items 0 .. n_nom_wg - 1 (rollout_item orders the grid)
    int32_t n_warm;      // samples k < n_warm keep the mean sequence
    int32_t n_tail;      // M - ceil(alpha M) + 1
    float dt, inv_wheelbase;
    float u_lo0, u_lo1, u_hi0, u_hi1;
    float se0, se1;      // control-noise standard deviations
    float sw0, sw1, sw2, sw3;  // disturbance scales: standard deviations (Gaussian) or half widths (uniform)
    int32_t noise_kind;        // 0 Gaussian, 1 uniform, 2 impulse
    float jump_prob, jump_size;
    float gamma, inv_var0, inv_var1;
    float A, B, C_u, lambda;
    float c_bdry, c_obs, c_dev, c_v, v_ref, c4, c5;
    float rc_v, rc_v_ref;  // sqrt(c_v) and sqrt(c_v) v_ref: the speed term as (rc_v v - rc_v_ref)^2
    // track: offsets of the local frame from the ellipse centre, and shape
    float tox, toy, inv_a, inv_b, g_a, g_b, hw, half_ab;
    float theta0;        // ellipse angle of the start point
    float psi0, v0;      // start heading and speed (position is the frame origin)
    float fx, fy;        // frame origin (the start position)
    uint32_t key0, key1, step_idx, flags;
    int32_t use_bdry, use_term, use_ctrl, scale_risk, debug;
    int32_t grad;        // record tail ranks for the gradient of the free energy
    int32_t store_u;     // store the sampled controls (debug view, gradient); without them
                         // the update draws the controls it needs again
    int32_t flat;        // disturbed workgroups take blockDim consecutive (sample, draw)
                         // pairs (at most spb samples) and store L; the CVaR is a separate pass
    uint32_t u0_seq;     // nonzero: after the first command, store this value to
                         // the word after it in mapped host memory (the host waits on it)
};

struct State {
    float x, y, psi, v;  // position in the local frame
};

// The step constants with the fields that the disturbed rollout steps read
// (dynamics, running cost, disturbance scales) in vector registers.
__device__ __forceinline__ StepConst with_vector_constants(const StepConst& c) {
    StepConst v = c;
    v.dt = in_vgpr(c.dt);
    v.tox = in_vgpr(c.tox);
    v.toy = in_vgpr(c.toy);
    v.inv_a = in_vgpr(c.inv_a);
    v.inv_b = in_vgpr(c.inv_b);
    v.g_a = in_vgpr(c.g_a);
    v.g_b = in_vgpr(c.g_b);
    v.c_dev = in_vgpr(c.c_dev);
    v.rc_v = in_vgpr(c.rc_v);
    v.rc_v_ref = in_vgpr(c.rc_v_ref);
    v.sw0 = in_vgpr(c.sw0);
    v.sw1 = in_vgpr(c.sw1);
    v.sw2 = in_vgpr(c.sw2);
    v.sw3 = in_vgpr(c.sw3);
    return v;
}

// with_vector_constants plus the fields of the nominal rollouts' steps
// (control sampling, clamp and control cost).
__device__ __forceinline__ StepConst with_vector_constants_nominal(const StepConst& c) {
    StepConst v = with_vector_constants(c);
    v.se0 = in_vgpr(c.se0);
    v.se1 = in_vgpr(c.se1);
    v.u_lo0 = in_vgpr(c.u_lo0);
    v.u_lo1 = in_vgpr(c.u_lo1);
    v.u_hi0 = in_vgpr(c.u_hi0);
    v.u_hi1 = in_vgpr(c.u_hi1);
    v.inv_var0 = in_vgpr(c.inv_var0);
    v.inv_var1 = in_vgpr(c.inv_var1);
    v.gamma = in_vgpr(c.gamma);
    v.inv_wheelbase = in_vgpr(c.inv_wheelbase);
    return v;
}


template <int kNoise>
__device__ __forceinline__ float4 disturbance(const StepConst& c, uint4 r) {
    if (kNoise == 0) {
        const float4 z = normals4(r);
        return make_float4(c.sw0 * z.x, c.sw1 * z.y, c.sw2 * z.z, c.sw3 * z.w);
    } else if (kNoise == 1) {
        return make_float4(c.sw0 * __fmaf_rn(2.0f, uniform01(r.x), -1.0f),
                           c.sw1 * __fmaf_rn(2.0f, uniform01(r.y), -1.0f),
                           c.sw2 * __fmaf_rn(2.0f, uniform01(r.z), -1.0f),
                           c.sw3 * __fmaf_rn(2.0f, uniform01(r.w), -1.0f));
    } else {
        const float u1 = uniform01(r.y);
        const float j = uniform01(r.x) < c.jump_prob ? c.jump_size : 0.0f;
        return make_float4(j * __builtin_amdgcn_cosf(u1), j * __builtin_amdgcn_sinf(u1), 0.0f, 0.0f);
    }
}

// The state-independent part of one disturbance: in the Gaussian form the
// two Box-Muller radii and the uniforms of the two angles (ra, rb, u1, u3);
// in the uniform form the four values 2u - 1; in the impulse form the jump
// length (0 without a jump) and its angle's uniform.
template <int kNoise>
__device__ __forceinline__ float4 disturbance_draw(const StepConst& c, uint4 r, uint32_t exp_word) {
    if (kNoise == 0) {
        const float ra =
            __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(uniform01(r.x, exp_word)));
        const float rb =
            __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(uniform01(r.z, exp_word)));
        return make_float4(ra, rb, uniform01(r.y, exp_word), uniform01(r.w, exp_word));
    } else if (kNoise == 1) {
        return make_float4(__fmaf_rn(2.0f, uniform01(r.x, exp_word), -1.0f),
                           __fmaf_rn(2.0f, uniform01(r.y, exp_word), -1.0f),
                           __fmaf_rn(2.0f, uniform01(r.z, exp_word), -1.0f),
                           __fmaf_rn(2.0f, uniform01(r.w, exp_word), -1.0f));
    } else {
        const float j = uniform01(r.x, exp_word) < c.jump_prob ? c.jump_size : 0.0f;
        return make_float4(j, uniform01(r.y, exp_word), 0.0f, 0.0f);
    }
}

// The disturbed successor F(x, u) + w from a disturbance_draw, each
// component's disturbance folded into its addition by one fused
// multiply-add: sqrt(Sigma_w) rad cos(2 pi u) (Gaussian), h (2u - 1)
// (uniform), jump cos(2 pi u) and jump sin(2 pi u) on x, y (impulse;
// heading and speed unchanged).
template <int kNoise>
__device__ __forceinline__ State disturbed_successor_drawn(const StepConst& c, float4 d, const State& s) {
    if (kNoise == 0)
        return State{__fmaf_rn(c.sw0 * d.x, __builtin_amdgcn_cosf(d.z), s.x),
                     __fmaf_rn(c.sw1 * d.x, __builtin_amdgcn_sinf(d.z), s.y),
                     __fmaf_rn(c.sw2 * d.y, __builtin_amdgcn_cosf(d.w), s.psi),
                     __fmaf_rn(c.sw3 * d.y, __builtin_amdgcn_sinf(d.w), s.v)};
    if (kNoise == 1)
        return State{__fmaf_rn(c.sw0, d.x, s.x), __fmaf_rn(c.sw1, d.y, s.y), __fmaf_rn(c.sw2, d.z, s.psi),
                     __fmaf_rn(c.sw3, d.w, s.v)};
    return State{__fmaf_rn(d.x, __builtin_amdgcn_cosf(d.y), s.x), __fmaf_rn(d.x, __builtin_amdgcn_sinf(d.y), s.y),
                 s.psi, s.v};
}

// The disturbed successor F(x, u) + w (Eq. 6) of a state s that already
// holds F(x, u), for the disturbance of Philox words r: disturbance_draw,
// then disturbed_successor_drawn (each component's scale and disturbance
// folded into its addition by one fused multiply-add).  Every rollout that
// needs the disturbed dynamics (the risk costs and the gradient's
// recomputation) goes through these two, so all of them see the same
// states.  The fused multiply-adds are written out, so the bits do not
// depend on which multiply-add pairs the compiler would contract.
// exp_word: 0x7F, the exponent word of uniform01 (in a vector register in
// the hot loop).
template <int kNoise>
__device__ __forceinline__ State disturbed_successor(const StepConst& c, uint4 r, const State& s,
                                                     uint32_t exp_word = 0x7Fu) {
    return disturbed_successor_drawn<kNoise>(c, disturbance_draw<kNoise>(c, r, exp_word), s);
}

// Headings beyond this magnitude (radians) are reduced modulo 2 pi before a
// rollout starts (start_heading), so that every heading a rollout reaches
// stays well inside the input range of the hardware sine and cosine.
constexpr double kMaxStartHeading = 100.0;

// The start heading of a rollout: x0's heading, reduced modulo 2 pi (in FP64,
// exactly) when its magnitude exceeds kMaxStartHeading.  The host and the
// batched path's prep kernel both call this, so they agree bit for bit.
__host__ __device__ __forceinline__ float start_heading(float psi) {
    if (fabs((double)psi) <= kMaxStartHeading) return psi;
    return (float)remainder((double)psi, 6.283185307179586476925);
}

// Forward-Euler bicycle step: da = dt a, kappa = tan(delta) / wheelbase.
// The hardware sine and cosine take the heading in revolutions as it is:
// they reduce it themselves, with the same largest error (1.25e-7 against
// FP64 over every float of 1/4 <= |r| < 64 revolutions) as after an explicit
// reduction to [-1/2, 1/2], which would cost two more instructions per step.
// A rollout's heading stays within about 15 rad of its start heading, so
// |r| < 64 whenever |psi0| <= kMaxStartHeading.
__device__ __forceinline__ void bicycle_step(State& s, float da, float kappa, float dt) {
    const float r = s.psi * 0.159154943091895335769f;
    const float sn = __builtin_amdgcn_sinf(r);
    const float cs = __builtin_amdgcn_cosf(r);
    const float dv = dt * s.v;
    s.x = __fmaf_rn(dv, cs, s.x);
    s.y = __fmaf_rn(dv, sn, s.y);
    s.psi = __fmaf_rn(dv, kappa, s.psi);
    {
        // da is the rounded product dt a in every rollout (nominal, disturbed
        // and the gradient's recomputation): never fused with the multiply
        // that produced it, so all of them see the same dynamics
#pragma clang fp contract(off)
        s.v = s.v + da;
    }
}

// tan of a steering angle (|d| < pi/2; the control box keeps it well inside):
// the hardware sine and cosine of d in revolutions and one reciprocal.  Used
// by every rollout (nominal, disturbed, and the gradient's recomputation), so
// all of them see the same dynamics.
__device__ __forceinline__ float tan_steer(float d) {
    const float r = d * 0.159154943091895335769f;
    return __builtin_amdgcn_sinf(r) * __builtin_amdgcn_rcpf(__builtin_amdgcn_cosf(r));
}

// Track and speed terms of q added to the running sum acc: acc + c_dev e^2 +
// c_v (v - v_ref)^2 [+ c_bdry mu_bdry when kBdry; the rollouts pick the
// instantiation once, so that a run of steps holds no branch].  Each term
// is folded into the sum by its own fused multiply-add.
template <bool kBdry>
__device__ __forceinline__ float smooth_cost_acc(const StepConst& c, const State& s, float acc) {
    const float X = s.x + c.tox;
    const float Y = s.y + c.toy;
    const float xa = X * c.inv_a;
    const float yb = Y * c.inv_b;
    const float G = __fmaf_rn(xa, xa, __fmaf_rn(yb, yb, -1.0f));
    const float gx = X * c.g_a;   // 2 X / a^2
    const float gy = Y * c.g_b;   // 2 Y / b^2
    const float gn2 = fmaxf(__fmaf_rn(gx, gx, gy * gy), 1e-24f);
    const float dv = __fmaf_rn(c.rc_v, s.v, -c.rc_v_ref);  // sqrt(c_v) (v - v_ref)
    acc = __fmaf_rn(c.c_dev * G, G * __builtin_amdgcn_rcpf(gn2), acc);
    acc = __fmaf_rn(dv, dv, acc);
    if (kBdry) {
        const float e = G * rsqrtf(gn2);
        const float d = c.hw - fabsf(e);
        const float mu = fmaxf(0.0f, atanf(-100.0f * d) * 0.318309886183790671538f + 0.5f);
        acc = __fmaf_rn(c.c_bdry, mu, acc);
    }
    return acc;
}

// Obstacle test (Eq. 22) on the table of a step (obstacle_entry): the point
// p is inside disc i iff |p|^2 + tab.x px + tab.y py < tab.z, evaluated as
// two FMAs on rho = |p|^2 and one compare.

// Wave-wide maximum of a 32-bit unsigned value over all 64 lanes (every lane
// active): rows of 16 lanes reduce with DPP lane permutations; then rows 1
// and 3 take in the last lane of the row before (row_bcast:15) and rows 2
// and 3 the last lane of row 1 (row_bcast:31), each one DPP maximum whose
// row mask leaves the other rows as they are, and lane 63, which then holds
// the wave's maximum, is read into a scalar register.  The result is
// wave-uniform.  Non-negative floats order like their bit patterns, so it
// also serves for the maximum of |x|.
template <int kCtrl>
__device__ __forceinline__ uint32_t dpp_max_u32(uint32_t v) {
    const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xF, 0xF, false);
    return v > o ? v : o;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = dpp_max_u32<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_max_u32<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_max_u32<0x141>(v);  // row_half_mirror
    v = dpp_max_u32<0x140>(v);  // row_mirror: every lane holds its row's maximum
    // written out because the compiler builds each broadcast step from a
    // move, a DPP move and a maximum; the s_nop gives the two wait states a
    // DPP read of a VGPR that a VALU instruction has just written needs
    asm volatile(
        "s_nop 1\n\t"
        "v_max_u32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_u32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ float lane_f32(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Number of hits of S consecutive points of a rollout (S time steps; only
// the first n count) on the obstacle discs (a point is inside a disc iff
// strictly closer to its centre than r), for a wave whose points lie close
// together (the M draws of one sample).  Broad phase: a box around the
// wave's points of all S steps, [xc - Rx, xc + Rx] x [yc - Ry, yc + Ry] with
// (xc, yc) the first lane's first point and Rx, Ry the largest distances of
// the lanes' points from it along x and y, against every disc, lane j
// testing entry 64 g + j of the table staged in LDS (otab, n_grp groups of
// 64): d2 = squared distance from the disc centre to the box, candidate iff
// d2 - 2^-15 P^2 < q (evaluated as dx^2 + (dy^2 - 2^-15 P^2), two fused
// multiply-adds), where P^2 = (|xc| + Rx)^2 + (|yc| + Ry)^2 bounds |p|^2
// over the box.  The margin exceeds the rounding error of both this test and
// the exact test (each a few units in the last place of r^2 + |c|^2 + |p|^2,
// the box edges a few units in the last place of P) by more than twenty
// times, so a disc that is not a candidate fails the exact test at every
// point of every lane.  Narrow phase: the exact test of each candidate at
// the S points, its entry broadcast from lane j.  One box serves S steps,
// which divides the cost of the box and the group tests by S; the count is
// an integer, so the grouping leaves it exact.  Every lane of the wave must
// be active.  n_cand counts the exact tests per lane (candidates times
// points, wave-uniform).  The caller holds
// lane j's entry of the first group in registers (e0, read once per
// rollout: the table does not change within a step); later groups are read
// from LDS at every call.
template <int S>
__device__ __forceinline__ void cull_group(const float4 e, const float4* grp, float bx0, float bx1, float by0,
                                           float by1, float p2, const float (&px)[S], const float (&py)[S],
                                           const float (&rho)[S], int n, int& cnt, int& n_cand) {
    const float cx = -0.5f * e.x, cy = -0.5f * e.y;
    const float dx = fmaxf(fmaxf(bx0 - cx, cx - bx1), 0.0f);
    const float dy = fmaxf(fmaxf(by0 - cy, cy - by1), 0.0f);
    uint64_t cand = __builtin_amdgcn_ballot_w64(__fmaf_rn(dx, dx, __fmaf_rn(dy, dy, -p2)) < e.w);
    while (cand) {
        const int j = __builtin_ctzll(cand);
        cand &= cand - 1;
        n_cand += n;
        // the candidate's entry read from LDS at one address for the whole
        // wave: it arrives in vector registers, so that the tests below
        // read no scalar register (see in_vgpr)
        const float4 ej = grp[j];
        const float a = ej.x, b = ej.y, z = ej.z;
        // one compare of the smallest of the S test values tells whether the
        // lane is inside the disc at any point (points past n repeat a valid
        // point, so they add no false alarm); only then are the points
        // compared one by one and counted, and the wave skips that when no
        // lane is inside (most candidates of the box test are near misses)
        float d[S];
#pragma unroll
        for (int u = 0; u < S; ++u) d[u] = __fmaf_rn(a, px[u], __fmaf_rn(b, py[u], rho[u]));
        float dmin = d[0];
#pragma unroll
        for (int u = 1; u < S; ++u) dmin = fminf(dmin, d[u]);
        if (dmin < z) {
#pragma unroll
            for (int u = 0; u < S; ++u) cnt += (u < n && d[u] < z) ? 1 : 0;
        }
    }
}

// Group skip of the broad phase (tables of more than one group).  Each group
// of 64 table entries has a bounding box: the union of its discs' squares
// |x - cx|, |y - cy| <= sqrt(q), widened by kGroupPad on every side
// (group_bounds).  A wave box that does not meet it is farther than
// sqrt(q) + kGroupPad from every centre of the group in x or in y, so each
// disc's squared distance exceeds (sqrt(q) + kGroupPad)^2 > q + 2^-15 P^2
// as long as 2^-7.5 P <= kGroupPad - 0.086 (P <= 256 m; beyond that every
// group is tested): the broad phase would reject the whole group, and the
// wave skips its test.  With the table sorted by angle around the
// obstacles' centroid (the host does that), a box along a track meets one or
// two groups.  The boxes are tested four compares per box for all groups at
// once: lane g holds group g's box (gb), lanes past the last group an empty
// one.
constexpr float kGroupPad = 1.5f;
constexpr float kGroupPadP2 = 65536.0f;  // P^2 up to which kGroupPad covers the broad-phase margin

// px, py: the S points (entries past n repeat a valid point).  gbox: the 64
// group boxes in LDS (see kGroupPad; boxes past n_grp meet nothing), read at
// every call rather than held in registers through the rollout; n_grp == 1
// tests the one group directly.  n_gtest counts the group tests run
// (wave-uniform).
template <int S>
__device__ __forceinline__ int obstacle_hits_culled(const float4* __restrict__ otab, const float4* gbox, int n_grp,
                                                    float4 e0, const float (&px)[S], const float (&py)[S], int n,
                                                    int& n_cand, int& n_gtest) {
    const float xc = in_vgpr(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(px[0]))));
    const float yc = in_vgpr(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(py[0]))));
    float mx = fabsf(px[0] - xc), my = fabsf(py[0] - yc);
    float rho[S];
#pragma unroll
    for (int u = 0; u < S; ++u) {
        if (u > 0) {
            mx = fmaxf(mx, fabsf(px[u] - xc));
            my = fmaxf(my, fabsf(py[u] - yc));
        }
        rho[u] = __fmaf_rn(px[u], px[u], py[u] * py[u]);
    }
    const float rx = __uint_as_float(wave_max_u32(__float_as_uint(mx)));
    const float ry = __uint_as_float(wave_max_u32(__float_as_uint(my)));
    const float bx0 = xc - rx, bx1 = xc + rx, by0 = yc - ry, by1 = yc + ry;
    const float ax = fabsf(xc) + rx, ay = fabsf(yc) + ry;
    const float P2 = __fmaf_rn(ax, ax, ay * ay);
    const float p2 = 3.0517578125e-05f * P2;  // 2^-15 P^2
    const int lane = threadIdx.x & 63;
    int cnt = 0;
    if (n_grp == 1) {
        cull_group<S>(e0, otab, bx0, bx1, by0, by1, p2, px, py, rho, n, cnt, n_cand);
        ++n_gtest;
        return cnt;
    }
    const float4 gb = gbox[lane];  // 64 entries, empty past n_grp
    // four compare masks combined on the scalar unit
    uint64_t gm = __builtin_amdgcn_ballot_w64(gb.x <= bx1) & __builtin_amdgcn_ballot_w64(gb.y >= bx0) &
                  __builtin_amdgcn_ballot_w64(gb.z <= by1) & __builtin_amdgcn_ballot_w64(gb.w >= by0);
    // (P2 is the same in every lane: the ballot makes that known, so that
    // the mask stays in scalar registers)
    if (__builtin_amdgcn_ballot_w64(P2 > kGroupPadP2) != 0ull) gm = (n_grp >= 64) ? ~0ull : ((1ull << n_grp) - 1ull);
    if (gm & 1ull) {
        cull_group<S>(e0, otab, bx0, bx1, by0, by1, p2, px, py, rho, n, cnt, n_cand);
        ++n_gtest;
    }
    gm &= ~1ull;
    while (gm) {
        const int g = __builtin_ctzll(gm);
        gm &= gm - 1ull;
        cull_group<S>(otab[g * 64 + lane], otab + g * 64, bx0, bx1, by0, by1, p2, px, py, rho, n, cnt, n_cand);
        ++n_gtest;
    }
    return cnt;
}

// Sampled control (Eq. 2b-2c with the warm / zero-mean rule of Algorithm 1):
// u = clamp(base + sqrt(Sigma_eps) z, u_lo, u_hi), base = v_t for k < n_warm.
__device__ __forceinline__ float2 sample_control_from(const StepConst& c, const float* __restrict__ V, int k, int t,
                                                     uint4 r, uint32_t exp_word) {
    float z0, z1;
    box_muller(uniform01(r.x, exp_word), uniform01(r.y, exp_word), z0, z1);
    // every lane reads v_t (t < T, in bounds) and warm samples keep it: a
    // select, not a branch
    const bool warm = k < c.n_warm;
    const float v0 = V[2 * t], v1 = V[2 * t + 1];
    const float b0 = warm ? v0 : 0.0f;
    const float b1 = warm ? v1 : 0.0f;
    float a = __fmaf_rn(c.se0, z0, b0);
    float d = __fmaf_rn(c.se1, z1, b1);
    a = fminf(fmaxf(a, c.u_lo0), c.u_hi0);
    d = fminf(fmaxf(d, c.u_lo1), c.u_hi1);
    return make_float2(a, d);
}

__device__ __forceinline__ float2 sample_control(const StepConst& c, const float* __restrict__ V, int k, int t) {
    const uint4 r = philox4x32_10((uint32_t)t, kCtrlWord, (uint32_t)k, c.step_idx, c.key0, c.key1);
    return sample_control_from(c, V, k, t, r, 0x7Fu);
}

// The same draw with the Philox keys and the exponent word in vector
// registers (the nominal rollouts' steps).
__device__ __forceinline__ float2 sample_control(const StepConst& c, const float* __restrict__ V, int k, int t,
                                                 const PhiloxVKeys& vk, uint32_t exp_word) {
    const uint4 r = philox4x32_10((uint32_t)t, kCtrlWord, (uint32_t)k, c.step_idx, c.key0, c.key1, vk);
    return sample_control_from(c, V, k, t, r, exp_word);
}

// Angle wrap to (-pi, pi].
__device__ __forceinline__ float wrap_pi(float ang) {
    const float two_pi = 6.28318530717958647692f;
    const float pi = 3.14159265358979323846f;
    return ang - two_pi * ceilf((ang - pi) * (1.0f / two_pi));
}

// Terminal cost, Eq. 23, with s(x) the mean-radius arc of the ellipse angle.
__device__ __forceinline__ float terminal_cost(const StepConst& c, const State& s) {
    const float X = s.x + c.tox;
    const float Y = s.y + c.toy;
    const float th = atan2f(Y * c.inv_b, X * c.inv_a);
    const float prog = c.half_ab * wrap_pi(th - c.theta0);
    return c.c4 - c.c5 * prog;
}

// Tail mean over the M (scaled) risk costs of one sample, held in LDS
// (vals[0..M-1]); each of the M lanes calls it with its own index m.  The
// lane's rank counts the strictly larger values plus the equal values with a
// smaller index, so ranks are a permutation of 0..M-1 and the n_tail largest
// values land, in descending order, in tail[0..n_tail-1].  The caller
// synchronises the workgroup between this and tail_sum.
__device__ __forceinline__ int tail_rank_scatter(const float* vals, float* tail, int M, int m, int n_tail) {
    const float v = vals[m];
    int rank = 0;
    for (int j = 0; j < M; ++j) {
        const float o = vals[j];
        rank += (o > v) | ((o == v) & (j < m));
    }
    if (rank < n_tail) tail[rank] = v;
    return rank;
}

// Value of lane (lane ^ j) of the wave, j a power of two below 64, every
// lane active: DPP quad permutations for 1 and 2, a rotation of the 16-lane
// row by 8 for 8, the swizzle unit's xor mode (within 32 lanes) for 4 and 16,
// and a backward permute through the LDS crossbar for 32.
template <int kJ>
__device__ __forceinline__ int lane_xor(int v) {
    if constexpr (kJ == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    else if constexpr (kJ == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    else if constexpr (kJ == 8) return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
    else if constexpr (kJ == 4 || kJ == 16) return __builtin_amdgcn_ds_swizzle(v, (kJ << 10) | 0x1F);
    else return __builtin_amdgcn_ds_bpermute((int)(((threadIdx.x & 63) ^ 32u) << 2), v);
}

// One compare-exchange of a bitonic network whose order puts larger values
// first and equal values by smaller index: lane i (position i in its
// segment) pairs with i ^ j; in merge blocks of size k it keeps the earlier
// of the two when it is the lower lane of an ascending block or the upper
// lane of a descending one, else the later.
__device__ __forceinline__ void bitonic_cx(float& v, int& id, float pv, int pid, int i, int j, int k) {
    const bool mine_first = (v > pv) || (v == pv && id < pid);
    const bool take_first = ((i & j) == 0) == ((i & k) == 0);
    if (take_first != mine_first) {
        v = pv;
        id = pid;
    }
}

template <int kJ>
__device__ __forceinline__ void bitonic_cx_lanes(float& v, int& id, int i, int k) {
    const float pv = __int_as_float(lane_xor<kJ>(__float_as_int(v)));
    const int pid = lane_xor<kJ>(id);
    bitonic_cx(v, id, pv, pid, i, kJ, k);
}

// In-wave stages (j < 64) of merge block k of the bitonic sort.
__device__ __forceinline__ void bitonic_wave_stages(float& v, int& id, int i, int k) {
    if (k > 32) bitonic_cx_lanes<32>(v, id, i, k);
    if (k > 16) bitonic_cx_lanes<16>(v, id, i, k);
    if (k > 8) bitonic_cx_lanes<8>(v, id, i, k);
    if (k > 4) bitonic_cx_lanes<4>(v, id, i, k);
    if (k > 2) bitonic_cx_lanes<2>(v, id, i, k);
    bitonic_cx_lanes<1>(v, id, i, k);
}

__device__ __forceinline__ float tail_sum(const float* tail, int n_tail) {
    float s = 0.0f;
    for (int r = 0; r < n_tail; ++r) s += tail[r];
    return s / (float)n_tail;
}

// Wave64 reductions with a fixed butterfly order (results are identical on
// every run and in every lane).
__device__ __forceinline__ float xor_f32_32(float v) { return __int_as_float(lane_xor<32>(__float_as_int(v))); }
__device__ __forceinline__ float xor_f32_16(float v) { return __int_as_float(lane_xor<16>(__float_as_int(v))); }
__device__ __forceinline__ float xor_f32_8(float v) { return __int_as_float(lane_xor<8>(__float_as_int(v))); }
__device__ __forceinline__ float xor_f32_4(float v) { return __int_as_float(lane_xor<4>(__float_as_int(v))); }
__device__ __forceinline__ float xor_f32_2(float v) { return __int_as_float(lane_xor<2>(__float_as_int(v))); }
__device__ __forceinline__ float xor_f32_1(float v) { return __int_as_float(lane_xor<1>(__float_as_int(v))); }

// Butterfly over distances 32, 16, ..., 1 (lane exchanges of lane_xor); every
// lane of the wave must be active.
__device__ __forceinline__ float wave_sum(float v) {
    v += xor_f32_32(v);
    v += xor_f32_16(v);
    v += xor_f32_8(v);
    v += xor_f32_4(v);
    v += xor_f32_2(v);
    v += xor_f32_1(v);
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
    v = fminf(v, xor_f32_32(v));
    v = fminf(v, xor_f32_16(v));
    v = fminf(v, xor_f32_8(v));
    v = fminf(v, xor_f32_4(v));
    v = fminf(v, xor_f32_2(v));
    v = fminf(v, xor_f32_1(v));
    return v;
}

__device__ __forceinline__ float wave_maxf(float v) { return -wave_min(-v); }

// ---- gradients (adjoint of one rollout) ----

// Gradient of the smooth running-cost terms with respect to the state
// (the obstacle indicator contributes nothing): c_dev e^2, c_v (v - v_ref)^2
// and c_bdry mu_bdry(d), with e = G / |grad G| and d = hw - |e|.
__device__ __forceinline__ float4 smooth_cost_grad(const StepConst& c, const State& s) {
    const float X = s.x + c.tox;
    const float Y = s.y + c.toy;
    const float xa = X * c.inv_a;
    const float yb = Y * c.inv_b;
    const float G = __fmaf_rn(xa, xa, __fmaf_rn(yb, yb, -1.0f));
    const float gx = X * c.g_a;
    const float gy = Y * c.g_b;
    const float gn2 = fmaxf(__fmaf_rn(gx, gx, gy * gy), 1e-24f);
    const float rgn = rsqrtf(gn2);
    const float e = G * rgn;
    const float k3 = G * rgn * rgn * rgn;          // G / |grad G|^3
    const float deX = gx * rgn - k3 * gx * c.g_a;  // de/dX (g_a = 2/a^2)
    const float deY = gy * rgn - k3 * gy * c.g_b;
    float fx = 2.0f * c.c_dev * e * deX;
    float fy = 2.0f * c.c_dev * e * deY;
    if (c.use_bdry) {
        const float d = c.hw - fabsf(e);
        const float dmu = -100.0f * 0.318309886183790671538f / __fmaf_rn(1e4f * d, d, 1.0f);
        const float sg = (e > 0.0f) ? -1.0f : ((e < 0.0f) ? 1.0f : 0.0f);  // d(d)/de = -sign(e)
        fx = __fmaf_rn(c.c_bdry * dmu * sg, deX, fx);
        fy = __fmaf_rn(c.c_bdry * dmu * sg, deY, fy);
    }
    return make_float4(fx, fy, 0.0f, 2.0f * c.c_v * (s.v - c.v_ref));
}

// Gradient of the terminal cost (Eq. 23) with respect to x_T.
__device__ __forceinline__ float4 terminal_cost_grad(const StepConst& c, const State& s) {
    const float xi = (s.x + c.tox) * c.inv_a;
    const float et = (s.y + c.toy) * c.inv_b;
    const float r2 = __fmaf_rn(xi, xi, et * et);
    if (!(r2 > 0.0f)) return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float k = -c.c5 * c.half_ab / r2;
    return make_float4(k * (-et * c.inv_a), k * (xi * c.inv_b), 0.0f, 0.0f);
}

}  // namespace ramppi
