// C ABI of the RA-MPPI library: parameter validation, workspace layout,
// handle management and launches.  Declarations and contracts: ramppi.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "launch.h"
#include "ramppi.h"

namespace {

thread_local std::string g_err;

mppi_status fail(mppi_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
mppi_status fail(mppi_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

mppi_status hip_fail(hipError_t e, const char* what) {
    return fail(MPPI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int kPartBlock = 256;           // samples per weight chunk
constexpr size_t kMaxLdsBytes = 64 * 1024;  // per workgroup
constexpr int kMaxK = 1 << 20;
constexpr int kMaxTimedSteps = 4096;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite(float v) { return std::isfinite(v); }

// Dynamic LDS of the rollout kernel: controls, risk costs, tail slots and
// means of the workgroup's samples, then the obstacle table in groups of 64.
size_t rollout_lds_bytes(int spb, const mppi_params* p) {
    if ((int64_t)spb * p->T > (1 << 24)) return SIZE_MAX;  // far beyond any LDS
    // the table (64 entries per group), then 64 group boxes
    const size_t n_grp = (size_t)ramppi::rollout_n_grp(p->n_obs);
    return 4 * (size_t)ramppi::rollout_otab_offset(spb, p->T, p->M) + 16 * 64 * n_grp + (n_grp > 1 ? 16 * 64 : 0);
}

// The order in which the obstacles are staged: by angle around their
// centroid, so that each group of 64 consecutive table entries covers one
// stretch of a track-like layout and a wave's box meets few groups (the
// group skip of the broad phase).  The hit count is a sum over all
// obstacles, so the order changes no result.
std::vector<int> obstacle_order(const float* o, int n) {
    std::vector<int> idx(n > 0 ? n : 0);
    if (n <= 64) {  // one group: the order does not matter
        for (int i = 0; i < n; ++i) idx[i] = i;
        return idx;
    }
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < n; ++i) {
        mx += o[3 * i];
        my += o[3 * i + 1];
    }
    mx /= n;
    my /= n;
    std::vector<double> ang(n);
    for (int i = 0; i < n; ++i) {
        idx[i] = i;
        ang[i] = std::atan2((double)o[3 * i + 1] - my, (double)o[3 * i] - mx);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return ang[a] < ang[b]; });
    return idx;
}

// Mapped pinned bytes per handle: the first command (2 floats), its
// completion word, one spare word, then the serving request.
constexpr size_t kPinnedBytes = 16 + sizeof(ramppi::ServeReq);
// Longest idle limit of a serving launch.
constexpr uint32_t kMaxServeIdleMs = 60000;

// Launch geometry derived from the sizes.
struct Geometry {
    int spb, block, n_nom_wg, G;
    size_t lds_rollout, lds_update;
};

Geometry geometry(const mppi_params* p) {
    Geometry g;
    g.spb = p->M >= 256 ? 1 : 256 / p->M;
    g.block = (g.spb * p->M + 63) / 64 * 64;
    g.n_nom_wg = (p->K + g.block - 1) / g.block;
    g.G = (p->K + kPartBlock - 1) / kPartBlock;
    g.lds_rollout = rollout_lds_bytes(g.spb, p);
    g.lds_update = ramppi::update_lds_bytes(p->T, g.G);
    return g;
}

// Integer tail size and warm count, computed in double precision.
void derived_counts(const mppi_params* p, int* n_tail, int* n_warm) {
    int ka = (int)std::ceil((double)p->alpha * (double)p->M - 1e-9);
    if (ka < 1) ka = 1;
    if (ka > p->M) ka = p->M;
    *n_tail = p->M - ka + 1;
    int nw = (int)std::ceil((1.0 - (double)p->eta) * (double)p->K - 1e-9);
    if (nw < 0) nw = 0;
    if (nw > p->K) nw = p->K;
    *n_warm = nw;
}

// Workspace layout (byte offsets), each buffer 256-byte aligned.
struct Layout {
    size_t obs, u, S, cvar, S_tilde, w_hat, L, part, u0, counter, work, chunk, fuse, serve;
    // gradient buffers (MPPI_F_GRAD)
    size_t ranks, tail_idx, act_list, n_act, J, states, rows, rpart, gcounter;
    int R, stride, n_lane_blocks;
    size_t total;
};

Layout layout(const mppi_params* p) {
    const Geometry g = geometry(p);
    Layout l;
    size_t o = 0;
    l.obs = o;     o += align_up(16 * (size_t)(p->n_obs > 0 ? p->n_obs : 1));
    l.u = o;       o += align_up(8 * (size_t)p->K * p->T);
    l.S = o;       o += align_up(4 * (size_t)p->K);
    l.cvar = o;    o += align_up(4 * (size_t)p->K);
    l.S_tilde = o; o += align_up(4 * (size_t)p->K);
    l.w_hat = o;   o += align_up(4 * (size_t)p->K);
    l.L = o;       o += align_up(4 * (size_t)p->K * p->M);
    l.part = o;    o += align_up(4 * (size_t)g.G * (2 + 2 * (size_t)p->T));
    l.u0 = o;      o += align_up(8);
    l.counter = o; o += align_up(4);
    l.work = o;    o += align_up(16 * (size_t)ramppi::kWorkSlots);
    l.chunk = o;   o += align_up(4 * (size_t)g.G);
    l.fuse = o;    o += align_up(sizeof(ramppi::FuseArgs));
    l.serve = o;   o += align_up(sizeof(ramppi::ServeReq) + sizeof(unsigned));  // request copy, go word
    l.ranks = l.tail_idx = l.act_list = l.n_act = l.J = l.states = l.rows = l.rpart = l.gcounter = 0;
    l.R = l.stride = l.n_lane_blocks = 0;
    if (p->flags & MPPI_F_GRAD) {
        int n_tail = 0, n_warm = 0;
        derived_counts(p, &n_tail, &n_warm);
        l.R = 1 + (p->B != 1.0f ? p->M : n_tail);
        l.n_lane_blocks = (int)(((int64_t)p->K * l.R + 255) / 256);
        l.stride = 256 * l.n_lane_blocks;
        l.ranks = o;    o += align_up(4 * (size_t)p->K * p->M);
        l.tail_idx = o; o += align_up(4 * (size_t)p->K * n_tail);
        l.act_list = o; o += align_up(4 * (size_t)p->K);
        l.n_act = o;    o += align_up(4);
        l.J = o;        o += align_up(4);
        l.states = o;   o += align_up(16 * (size_t)p->T * l.stride);
        l.rows = o;     o += align_up(4 * 2 * (size_t)p->T * l.stride);
        l.rpart = o;    o += align_up(4 * 2 * (size_t)p->T * l.n_lane_blocks);
        l.gcounter = o; o += align_up(4);
    }
    l.total = o;
    return l;
}

mppi_status check_device(int* dev) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(MPPI_EDEVICE, "no HIP device available");
    e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return MPPI_OK;
}

// Per-launch constants that depend only on the parameters and the geometry.
void fill_static(ramppi::StepConst* cp, const mppi_params& p, const Geometry& g, int n_tail, int n_warm) {
    ramppi::StepConst& c = *cp;
    std::memset(&c, 0, sizeof c);
    c.K = p.K;
    c.T = p.T;
    c.M = p.M;
    c.n_obs = p.n_obs;
    c.spb = g.spb;
    c.n_nom_wg = g.n_nom_wg;
    c.n_warm = n_warm;
    c.n_tail = n_tail;
    c.dt = p.dt;
    c.inv_wheelbase = (float)(1.0 / (double)p.wheelbase);
    c.u_lo0 = p.u_lo[0];
    c.u_lo1 = p.u_lo[1];
    c.u_hi0 = p.u_hi[0];
    c.u_hi1 = p.u_hi[1];
    c.se0 = (float)std::sqrt((double)p.sigma_eps[0]);
    c.se1 = (float)std::sqrt((double)p.sigma_eps[1]);
    c.sw0 = (float)std::sqrt((double)p.sigma_w[0]);
    c.sw1 = (float)std::sqrt((double)p.sigma_w[1]);
    c.sw2 = (float)std::sqrt((double)p.sigma_w[2]);
    c.sw3 = (float)std::sqrt((double)p.sigma_w[3]);
    c.noise_kind = (int32_t)p.noise_kind;
    if (p.noise_kind == MPPI_NOISE_UNIFORM) {  // half widths sqrt(3 sigma_w) in the sw slots
        c.sw0 = (float)std::sqrt(3.0 * p.sigma_w[0]);
        c.sw1 = (float)std::sqrt(3.0 * p.sigma_w[1]);
        c.sw2 = (float)std::sqrt(3.0 * p.sigma_w[2]);
        c.sw3 = (float)std::sqrt(3.0 * p.sigma_w[3]);
    }
    c.jump_prob = p.jump_prob;
    c.jump_size = p.jump_size;
    c.gamma = p.gamma;
    c.use_ctrl = p.gamma != 0.0f;
    c.inv_var0 = c.use_ctrl ? (float)(1.0 / (double)p.sigma_eps[0]) : 0.0f;
    c.inv_var1 = c.use_ctrl ? (float)(1.0 / (double)p.sigma_eps[1]) : 0.0f;
    c.A = p.A;
    c.B = p.B;
    c.C_u = p.C_u;
    c.lambda = p.lambda;
    c.scale_risk = p.B != 1.0f;
    c.c_bdry = p.c_bdry;
    c.c_obs = p.c_obs;
    c.c_dev = p.c_dev;
    c.c_v = p.c_v;
    c.v_ref = p.v_ref;
    c.rc_v = (float)std::sqrt((double)p.c_v);
    c.rc_v_ref = (float)(std::sqrt((double)p.c_v) * (double)p.v_ref);
    c.c4 = p.c4;
    c.c5 = p.c5;
    c.use_bdry = p.c_bdry != 0.0f;
    c.use_term = (p.c4 != 0.0f) || (p.c5 != 0.0f);
    const double a = p.track[2], b = p.track[3];
    c.inv_a = (float)(1.0 / a);
    c.inv_b = (float)(1.0 / b);
    c.g_a = (float)(2.0 / (a * a));
    c.g_b = (float)(2.0 / (b * b));
    c.hw = p.track[4];
    c.half_ab = (float)(0.5 * (a + b));
    c.key0 = (uint32_t)(p.seed & 0xFFFFFFFFu);
    c.key1 = (uint32_t)(p.seed >> 32);
    c.flags = p.flags;
    c.debug = (p.flags & MPPI_F_DEBUG) != 0;
    c.store_u = c.debug;  // the update draws the controls it needs again
    c.flat = 0;
}

// Per-launch constants that depend on the measured state and the call index
// (the batched path computes the same fields on the device, ramppi::set_dynamic).
void fill_dynamic(ramppi::StepConst* cp, const mppi_params& p, const float x0[4], uint32_t step_idx) {
    ramppi::StepConst& c = *cp;
    c.fx = x0[0];
    c.fy = x0[1];
    c.tox = x0[0] - p.track[0];
    c.toy = x0[1] - p.track[1];
    c.theta0 = (float)std::atan2(((double)x0[1] - p.track[1]) / (double)p.track[3],
                                 ((double)x0[0] - p.track[0]) / (double)p.track[2]);
    c.psi0 = ramppi::start_heading(x0[2]);
    c.v0 = x0[3];
    c.step_idx = step_idx;
}

}  // namespace

struct mppi_handle {
    mppi_params p;
    Geometry g;
    Layout l;
    int n_tail, n_warm, device;
    char* ws;
    float* u0_pinned;      // mapped, coherent pinned host memory: 2 floats + completion word
    float* u0_pinned_dev;  // its device address
    uint32_t u0_seq;       // last completion value requested
    bool fuse;             // one launch per step (the whole grid is resident at once)
    bool flat;             // two launches with the flattened disturbed layout (M > 256)
    bool serving;          // a persistent serving launch is resident (mppi_serve_start)
    uint32_t serve_seq;    // last request posted in the session
    hipStream_t serve_stream;
    ramppi::ServeReq* req;  // mapped pinned host memory after the command words
    bool timing;
    std::vector<hipEvent_t> ev;  // 3 per timed step: start, after rollout, end
    int n_timed;
};

namespace {

ramppi::StepBuffers step_buffers(const mppi_handle* h, float* V_dev) {
    ramppi::StepBuffers bufs;
    bufs.obs = reinterpret_cast<const float4*>(h->ws + h->l.obs);
    bufs.V = V_dev;
    bufs.Vout = V_dev;
    bufs.u = reinterpret_cast<float2*>(h->ws + h->l.u);
    bufs.S = reinterpret_cast<float*>(h->ws + h->l.S);
    bufs.cvar = reinterpret_cast<float*>(h->ws + h->l.cvar);
    bufs.S_tilde = reinterpret_cast<float*>(h->ws + h->l.S_tilde);
    bufs.w_hat = reinterpret_cast<float*>(h->ws + h->l.w_hat);
    bufs.L = reinterpret_cast<float*>(h->ws + h->l.L);
    bufs.part = reinterpret_cast<float*>(h->ws + h->l.part);
    bufs.u0 = reinterpret_cast<float*>(h->ws + h->l.u0);
    bufs.counter = reinterpret_cast<unsigned*>(h->ws + h->l.counter);
    bufs.u0_host = nullptr;
    bufs.work = nullptr;
    bufs.chunk_ctr = reinterpret_cast<unsigned*>(h->ws + h->l.chunk);
    return bufs;
}

// Sums and clears the broad-phase work counters (kWorkSlots exact-test
// slots, then kWorkSlots group-test slots; waits for `s`).  group_tests may
// be NULL.
hipError_t read_work(unsigned long long* dev, hipStream_t s, uint64_t* candidates, uint64_t* group_tests) {
    unsigned long long host[2 * ramppi::kWorkSlots];
    hipError_t e = hipMemcpyAsync(host, dev, sizeof host, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemsetAsync(dev, 0, sizeof host, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    uint64_t c = 0, g = 0;
    for (int i = 0; i < ramppi::kWorkSlots; ++i) {
        c += host[i];
        g += host[ramppi::kWorkSlots + i];
    }
    *candidates = c;
    if (group_tests) *group_tests = g;
    return e;
}

}  // namespace

extern "C" {

mppi_status mppi_validate(const mppi_params* p) {
    if (!p) return fail(MPPI_EINVAL, "params is NULL");
    if (p->K < 1 || p->T < 1 || p->M < 1 || p->n_obs < 0)
        return fail(MPPI_EINVAL, "sizes must satisfy K, T, M >= 1 and n_obs >= 0 (got K=%d T=%d M=%d n_obs=%d)",
                    p->K, p->T, p->M, p->n_obs);
    if (p->flags &
        ~(uint32_t)(MPPI_F_DEBUG | MPPI_F_SHIFT | MPPI_F_ALLOW_ZERO_NOISE | MPPI_F_GRAD | MPPI_F_SPLIT_UPDATE))
        return fail(MPPI_EINVAL, "unknown flag bits 0x%x", p->flags);
    if (!(finite(p->dt) && p->dt > 0)) return fail(MPPI_EINVAL, "dt must be finite and > 0");
    if (!(finite(p->wheelbase) && p->wheelbase > 0)) return fail(MPPI_EINVAL, "wheelbase must be finite and > 0");
    for (int i = 0; i < 2; ++i)
        if (!(finite(p->u_lo[i]) && finite(p->u_hi[i]) && p->u_lo[i] < p->u_hi[i]))
            return fail(MPPI_EINVAL, "control box %d must be finite with u_lo < u_hi", i);
    const bool zero_ok = (p->flags & MPPI_F_ALLOW_ZERO_NOISE) != 0;
    bool eps_zero = false;
    for (int i = 0; i < 2; ++i) {
        const float s = p->sigma_eps[i];
        if (!finite(s) || s < 0 || (s == 0 && !zero_ok))
            return fail(MPPI_EINVAL, "sigma_eps[%d] must be a finite variance > 0", i);
        eps_zero |= (s == 0);
    }
    for (int i = 0; i < 4; ++i)
        if (!finite(p->sigma_w[i]) || p->sigma_w[i] < 0)
            return fail(MPPI_EINVAL, "sigma_w[%d] must be a finite variance >= 0", i);
    if (!(p->alpha > 0 && p->alpha < 1)) return fail(MPPI_EINVAL, "alpha must lie in (0, 1)");
    if (!(finite(p->lambda) && p->lambda > 0)) return fail(MPPI_EINVAL, "lambda must be finite and > 0");
    if (!(finite(p->gamma) && p->gamma >= 0 && p->gamma <= p->lambda))
        return fail(MPPI_EINVAL, "gamma must lie in [0, lambda]");
    if (eps_zero && p->gamma != 0) return fail(MPPI_EINVAL, "a zero control variance needs gamma = 0");
    if (!(p->eta >= 0 && p->eta <= 1)) return fail(MPPI_EINVAL, "eta must lie in [0, 1]");
    if (!(finite(p->A) && p->A >= 0)) return fail(MPPI_EINVAL, "A must be finite and >= 0");
    if (!(finite(p->B) && p->B >= 0)) return fail(MPPI_EINVAL, "B must be finite and >= 0");
    if (std::isnan(p->C_u)) return fail(MPPI_EINVAL, "C_u must not be NaN");
    const float w[7] = {p->c_bdry, p->c_obs, p->c_dev, p->c_v, p->v_ref, p->c4, p->c5};
    for (int i = 0; i < 7; ++i)
        if (!finite(w[i])) return fail(MPPI_EINVAL, "cost weights must be finite");
    if (!(p->c_v >= 0)) return fail(MPPI_EINVAL, "c_v must be >= 0");
    if (!(finite(p->track[0]) && finite(p->track[1]))) return fail(MPPI_EINVAL, "track centre must be finite");
    if (!(finite(p->track[2]) && p->track[2] > 0 && finite(p->track[3]) && p->track[3] > 0))
        return fail(MPPI_EINVAL, "track semi-axes must be finite and > 0");
    if (!(finite(p->track[4]) && p->track[4] >= 0)) return fail(MPPI_EINVAL, "track half width must be >= 0");
    if (p->noise_kind > MPPI_NOISE_IMPULSE) return fail(MPPI_EINVAL, "unknown noise_kind %u", p->noise_kind);
    if (!(p->jump_prob >= 0 && p->jump_prob <= 1)) return fail(MPPI_EINVAL, "jump_prob must lie in [0, 1]");
    if (!(finite(p->jump_size) && p->jump_size >= 0)) return fail(MPPI_EINVAL, "jump_size must be finite and >= 0");
    if (p->M > MPPI_MAX_M) return fail(MPPI_EUNSUPPORTED, "M = %d exceeds %d", p->M, MPPI_MAX_M);
    if (p->n_obs > MPPI_MAX_OBS) return fail(MPPI_EUNSUPPORTED, "n_obs = %d exceeds %d", p->n_obs, MPPI_MAX_OBS);
    if (p->T > MPPI_MAX_T) return fail(MPPI_EUNSUPPORTED, "T = %d exceeds %d", p->T, MPPI_MAX_T);
    if (p->K > kMaxK) return fail(MPPI_EUNSUPPORTED, "K = %d exceeds %d", p->K, kMaxK);
    if ((int64_t)p->K * p->M > (int64_t)INT32_MAX) return fail(MPPI_EUNSUPPORTED, "K * M exceeds 2^31 - 1");
    if ((p->flags & MPPI_F_GRAD) && (int64_t)p->K * (1 + p->M) > (int64_t)INT32_MAX / 4)
        return fail(MPPI_EUNSUPPORTED, "K (1 + M) too large for the gradient buffers");
    const Geometry g = geometry(p);
    if (g.lds_rollout > kMaxLdsBytes)
        return fail(MPPI_EUNSUPPORTED, "rollout LDS need %zu B exceeds %zu B (reduce T or M)", g.lds_rollout,
                    kMaxLdsBytes);
    if (g.lds_update > kMaxLdsBytes)
        return fail(MPPI_EUNSUPPORTED, "update LDS need %zu B exceeds %zu B (reduce K or T)", g.lds_update,
                    kMaxLdsBytes);
    return MPPI_OK;
}

size_t mppi_workspace_bytes(const mppi_params* p) {
    if (mppi_validate(p) != MPPI_OK) return 0;
    return layout(p).total;
}

mppi_status mppi_create(const mppi_params* p, const float* obstacles_host, void* workspace_dev,
                        size_t workspace_bytes, void* stream, mppi_handle** out) {
    if (!out) return fail(MPPI_EINVAL, "out is NULL");
    *out = nullptr;
    mppi_status st = mppi_validate(p);
    if (st != MPPI_OK) return st;
    if (p->n_obs > 0 && !obstacles_host) return fail(MPPI_EINVAL, "obstacles_host is NULL with n_obs > 0");
    for (int i = 0; i < p->n_obs; ++i) {
        const float* o = obstacles_host + 3 * i;
        if (!(finite(o[0]) && finite(o[1]) && finite(o[2]) && o[2] > 0))
            return fail(MPPI_EINVAL, "obstacle %d must have a finite centre and a radius > 0", i);
    }
    const Layout l = layout(p);
    if (!workspace_dev) return fail(MPPI_EINVAL, "workspace_dev is NULL");
    if (((uintptr_t)workspace_dev) % kAlign) return fail(MPPI_EINVAL, "workspace_dev must be 256-byte aligned");
    if (workspace_bytes < l.total)
        return fail(MPPI_EINVAL, "workspace has %zu B, needs %zu B", workspace_bytes, l.total);
    int dev = 0;
    st = check_device(&dev);
    if (st != MPPI_OK) return st;

    mppi_handle* h = new (std::nothrow) mppi_handle();
    if (!h) return fail(MPPI_ENOMEM, "host allocation failed");
    h->p = *p;
    h->g = geometry(p);
    h->l = l;
    derived_counts(p, &h->n_tail, &h->n_warm);
    h->device = dev;
    h->ws = static_cast<char*>(workspace_dev);
    h->timing = false;
    h->n_timed = 0;
    h->u0_seq = 0;
    h->serving = false;
    h->serve_seq = 0;
    h->serve_stream = nullptr;
    // command (2 floats), completion word, then the serving request
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->u0_pinned), kPinnedBytes,
                                 hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) std::memset(h->u0_pinned, 0, kPinnedBytes);
    h->req = e == hipSuccess ? reinterpret_cast<ramppi::ServeReq*>(h->u0_pinned + 4) : nullptr;
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipHostMalloc");
    }
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&h->u0_pinned_dev), h->u0_pinned, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(h->u0_pinned);
        delete h;
        return hip_fail(e, "hipHostGetDevicePointer");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<float> staged(4 * (size_t)(p->n_obs > 0 ? p->n_obs : 1), 0.0f);
    const std::vector<int> order = obstacle_order(obstacles_host, p->n_obs);
    for (int i = 0; i < p->n_obs; ++i) {
        staged[4 * i + 0] = obstacles_host[3 * order[i] + 0];
        staged[4 * i + 1] = obstacles_host[3 * order[i] + 1];
        staged[4 * i + 2] = obstacles_host[3 * order[i] + 2];
    }
    e = hipMemcpyAsync(h->ws + l.obs, staged.data(), 16 * (size_t)p->n_obs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + l.counter, 0, 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + l.work, 0, 16 * (size_t)ramppi::kWorkSlots, s);
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + l.chunk, 0, 4 * (size_t)h->g.G, s);
    if (e == hipSuccess && (p->flags & MPPI_F_GRAD)) e = hipMemsetAsync(h->ws + l.gcounter, 0, 4, s);
    // one launch per step when every workgroup of the step can be resident at
    // once (the update then runs in the workgroups that finish each chunk)
    h->fuse = false;
    ramppi::FuseArgs fa;
    std::memset(&fa, 0, sizeof fa);
    if (e == hipSuccess && !(p->flags & MPPI_F_SPLIT_UPDATE)) {
        int per_cu = 0, n_cu = 0;
        e = ramppi::fused_rollout_capacity((int)p->noise_kind, h->g.block,
                                           std::max(h->g.lds_rollout, h->g.lds_update), &per_cu);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        const int64_t grid = h->g.n_nom_wg + ((int64_t)p->K + h->g.spb - 1) / h->g.spb;
        h->fuse = e == hipSuccess && (int64_t)per_cu * n_cu >= grid;
        fa.chunk_ctr = reinterpret_cast<unsigned*>(h->ws + l.chunk);
        fa.counter = reinterpret_cast<unsigned*>(h->ws + l.counter);
        fa.S_tilde = reinterpret_cast<float*>(h->ws + l.S_tilde);
        fa.part = reinterpret_cast<float*>(h->ws + l.part);
        fa.u0 = reinterpret_cast<float*>(h->ws + l.u0);
        fa.u0_host = h->u0_pinned_dev;
        fa.w_hat = reinterpret_cast<float*>(h->ws + l.w_hat);
        fa.G = h->g.G;
        fa.parts = ramppi::update_parts(p->T);
        if (e == hipSuccess) e = hipMemcpyAsync(h->ws + l.fuse, &fa, sizeof fa, hipMemcpyHostToDevice, s);
    }
    // Two-launch steps whose samples need more than four waves (M > 256):
    // the disturbed workgroups of five or more waves start only three to a
    // compute unit at once, so their lanes are laid out instead as 256
    // consecutive (sample, draw) pairs per workgroup (at most two samples,
    // four waves) and each sample's CVaR is formed by a separate pass from
    // the stored risk costs.  The gradient keeps the per-sample layout (its
    // tail ranks come from the rollout's own CVaR pass).
    h->flat = !h->fuse && p->M > 256 && !(p->flags & MPPI_F_GRAD);
    if (h->flat) {
        h->g.spb = 2;
        h->g.block = 256;
        h->g.n_nom_wg = (p->K + 255) / 256;
        h->g.lds_rollout = rollout_lds_bytes(2, p);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipHostFree(h->u0_pinned);
        delete h;
        return hip_fail(e, "obstacle upload");
    }
    *out = h;
    return MPPI_OK;
}

mppi_status mppi_destroy(mppi_handle* h) {
    if (!h) return MPPI_OK;
    if (h->serving) (void)mppi_serve_stop(h);
    for (hipEvent_t ev : h->ev) (void)hipEventDestroy(ev);
    if (h->u0_pinned) (void)hipHostFree(h->u0_pinned);
    delete h;
    return MPPI_OK;
}

const char* mppi_last_error(void) { return g_err.c_str(); }

mppi_status mppi_step(mppi_handle* h, const float x0[4], float* V_dev, uint32_t step_idx, float* u0_host,
                      void* stream) {
    if (!h) return fail(MPPI_EINVAL, "handle is NULL");
    if (!x0) return fail(MPPI_EINVAL, "x0 is NULL");
    if (!V_dev) return fail(MPPI_EINVAL, "V_dev is NULL");
    if (h->serving) return fail(MPPI_EINVAL, "the handle is serving (mppi_serve_stop first)");
    for (int i = 0; i < 4; ++i)
        if (!finite(x0[i])) return fail(MPPI_EINVAL, "x0[%d] is not finite", i);
    const mppi_params& p = h->p;
    const Geometry& g = h->g;
    hipStream_t s = static_cast<hipStream_t>(stream);

    ramppi::StepConst c;
    fill_static(&c, p, g, h->n_tail, h->n_warm);
    fill_dynamic(&c, p, x0, step_idx);
    c.flat = h->flat;

    ramppi::StepBuffers bufs = step_buffers(h, V_dev);
    bufs.u0_host = u0_host ? h->u0_pinned_dev : nullptr;
    if (u0_host) {
        h->u0_seq = h->u0_seq + 1 ? h->u0_seq + 1 : 1;  // never 0
        c.u0_seq = h->u0_seq;
    }

    hipEvent_t ev_start = nullptr, ev_mid = nullptr, ev_end = nullptr;
    if (h->timing && h->n_timed < kMaxTimedSteps) {
        hipEvent_t* e3 = &h->ev[3 * (size_t)h->n_timed];
        ev_start = e3[0];
        ev_mid = e3[1];
        ev_end = e3[2];
    }
    if (h->timing) bufs.work = reinterpret_cast<unsigned long long*>(h->ws + h->l.work);
    const ramppi::FuseArgs* fa = h->fuse ? reinterpret_cast<const ramppi::FuseArgs*>(h->ws + h->l.fuse) : nullptr;
    hipError_t e =
        ramppi::launch_step(c, bufs, g.block, g.lds_rollout, g.G, g.lds_update, s, ev_start, ev_mid, fa);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    if (ev_end) {
        e = hipEventRecord(ev_end, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        h->n_timed++;
    }
    if (u0_host) {
        // the update kernel stores the command and then the completion word
        // into the mapped pinned buffer: poll the word (asking the stream now
        // and then, so that a failed step still returns) rather than waiting
        // for the whole stream
        const uint32_t* word = reinterpret_cast<const uint32_t*>(h->u0_pinned + 2);
        for (uint64_t spin = 1;; ++spin) {
            if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == h->u0_seq) break;
            if ((spin & 1023) == 0) {
                const hipError_t q = hipStreamQuery(s);
                if (q == hipSuccess) {  // the step is complete, so is its word
                    if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == h->u0_seq) break;
                    return fail(MPPI_EDEVICE, "the step completed without its first command");
                }
                if (q != hipErrorNotReady) return hip_fail(q, "first-command readback");
            }
            __builtin_ia32_pause();
        }
        u0_host[0] = h->u0_pinned[0];
        u0_host[1] = h->u0_pinned[1];
    }
    return MPPI_OK;
}

}  // extern "C"

namespace {

// Scratch memory of mppi_step_noalloc: the step's workspace (obstacle table,
// sampled controls, per-sample costs, chunk partials, counters) in a static
// device array, so that the call allocates nothing.  Each device that runs
// the call holds its own copy until the process ends.  Host code uses only
// the device address that hipGetSymbolAddress returns for the current device
// (g_scratch_dev), never the array's name.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxScratchDevices];

// The scratch's device address on device `dev` (looked up once per device,
// with that device current).
mppi_status scratch_address(int dev, char** out) {
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(MPPI_EUNSUPPORTED, "device %d is beyond the %d devices the scratch table covers", dev,
                    kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch_dev[dev] = static_cast<char*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return MPPI_OK;
}

// Stages the caller's obstacles (n_obs x 3 floats) as the table's float4
// entries and zeroes the update's counters, which must start at zero (a fill
// kernel rather than a memset, so that the call can be captured in a graph).
__global__ void k_noalloc_prep(const float* __restrict__ obs3, int n_obs, float4* __restrict__ obs4,
                               unsigned* __restrict__ counter, unsigned* __restrict__ chunk_ctr, int G) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_obs) obs4[i] = make_float4(obs3[3 * i], obs3[3 * i + 1], obs3[3 * i + 2], 0.0f);
    if (i < G) chunk_ctr[i] = 0u;
    if (i == 0) *counter = 0u;
}

}  // namespace

extern "C" {

mppi_status mppi_step_noalloc(const mppi_params* p, const float* obstacles_dev, const float x0[4], float* V_dev,
                              uint32_t step_idx, float* u0_dev, void* stream) {
    if (!p) return fail(MPPI_EINVAL, "params is NULL");
    mppi_status st = mppi_validate(p);
    if (st != MPPI_OK) return st;
    if (p->flags & (MPPI_F_DEBUG | MPPI_F_GRAD))
        return fail(MPPI_EINVAL, "MPPI_F_DEBUG and MPPI_F_GRAD need a handle (mppi_create)");
    if (p->n_obs > 0 && !obstacles_dev) return fail(MPPI_EINVAL, "obstacles_dev is NULL with n_obs > 0");
    if (!x0) return fail(MPPI_EINVAL, "x0 is NULL");
    if (!V_dev) return fail(MPPI_EINVAL, "V_dev is NULL");
    for (int i = 0; i < 4; ++i)
        if (!finite(x0[i])) return fail(MPPI_EINVAL, "x0[%d] is not finite", i);
    const Layout l = layout(p);
    if (l.total > kScratchBytes)
        return fail(MPPI_EUNSUPPORTED, "the step needs %zu B of scratch, more than the %zu B of mppi_step_noalloc",
                    l.total, kScratchBytes);
    int dev = 0;
    st = check_device(&dev);
    if (st != MPPI_OK) return st;
    char* ws = nullptr;
    st = scratch_address(dev, &ws);
    if (st != MPPI_OK) return st;

    const Geometry g = geometry(p);
    int n_tail = 0, n_warm = 0;
    derived_counts(p, &n_tail, &n_warm);
    ramppi::StepConst c;
    fill_static(&c, *p, g, n_tail, n_warm);
    fill_dynamic(&c, *p, x0, step_idx);
    c.u0_seq = 0;

    ramppi::StepBuffers bufs;
    bufs.obs = reinterpret_cast<const float4*>(ws + l.obs);
    bufs.V = V_dev;
    bufs.Vout = V_dev;
    bufs.u = reinterpret_cast<float2*>(ws + l.u);
    bufs.S = reinterpret_cast<float*>(ws + l.S);
    bufs.cvar = reinterpret_cast<float*>(ws + l.cvar);
    bufs.S_tilde = reinterpret_cast<float*>(ws + l.S_tilde);
    bufs.w_hat = reinterpret_cast<float*>(ws + l.w_hat);
    bufs.L = reinterpret_cast<float*>(ws + l.L);
    bufs.part = reinterpret_cast<float*>(ws + l.part);
    bufs.u0 = u0_dev ? u0_dev : reinterpret_cast<float*>(ws + l.u0);
    bufs.counter = reinterpret_cast<unsigned*>(ws + l.counter);
    bufs.u0_host = nullptr;
    bufs.work = nullptr;
    bufs.chunk_ctr = reinterpret_cast<unsigned*>(ws + l.chunk);

    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n_prep = std::max(std::max(p->n_obs, g.G), 1);
    hipLaunchKernelGGL(k_noalloc_prep, dim3((n_prep + 255) / 256), dim3(256), 0, s, obstacles_dev, p->n_obs,
                       reinterpret_cast<float4*>(ws + l.obs), bufs.counter, bufs.chunk_ctr, g.G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "obstacle staging launch");
    // always the two-launch form (rollouts, then the update): it needs no
    // occupancy query and gives the same bits as the one-launch step
    e = ramppi::launch_step(c, bufs, g.block, g.lds_rollout, g.G, g.lds_update, s, nullptr, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    return MPPI_OK;
}

mppi_status mppi_serve_start(mppi_handle* h, float* V_dev, uint32_t idle_ms, void* stream) {
    if (!h) return fail(MPPI_EINVAL, "handle is NULL");
    if (!V_dev) return fail(MPPI_EINVAL, "V_dev is NULL");
    if (h->serving) return fail(MPPI_EINVAL, "the handle is already serving");
    if (idle_ms < 1 || idle_ms > kMaxServeIdleMs)
        return fail(MPPI_EINVAL, "idle_ms = %u outside [1, %u]", idle_ms, kMaxServeIdleMs);
    if (!h->fuse) return fail(MPPI_EUNSUPPORTED, "the step does not run as one launch, so it cannot be served");
    const mppi_params& p = h->p;
    const Geometry& g = h->g;
    const size_t lds = std::max(g.lds_rollout, g.lds_update);
    int per_cu = 0, n_cu = 0;
    hipError_t e = ramppi::serve_capacity((int)p.noise_kind, g.block, lds, &per_cu);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
    if (e != hipSuccess) return hip_fail(e, "serving occupancy");
    const int64_t grid = g.n_nom_wg + ((int64_t)p.K + g.spb - 1) / g.spb;
    if ((int64_t)per_cu * n_cu < grid)
        return fail(MPPI_EUNSUPPORTED, "the serving grid (%lld workgroups) cannot be resident at once",
                    (long long)grid);
    hipStream_t s = static_cast<hipStream_t>(stream);

    ramppi::StepConst c;
    const float x0[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // the per-step fields come with each request
    fill_static(&c, p, g, h->n_tail, h->n_warm);
    fill_dynamic(&c, p, x0, 0);
    ramppi::StepBuffers bufs = step_buffers(h, V_dev);
    // workspace: request copy | go word
    char* sv = h->ws + h->l.serve;
    ramppi::ServeArgs sa;
    sa.req_host = reinterpret_cast<const ramppi::ServeReq*>(h->u0_pinned_dev + 4);
    sa.req_dev = reinterpret_cast<ramppi::ServeReq*>(sv);
    sa.go = reinterpret_cast<unsigned*>(sv + sizeof(ramppi::ServeReq));
    sa.idle_ticks = 100000ull * idle_ms;  // s_memrealtime runs at 100 MHz

    // a new session: requests and completions count from 1 again
    std::memset(h->req, 0, sizeof(ramppi::ServeReq));
    __atomic_store_n(reinterpret_cast<uint32_t*>(h->u0_pinned + 2), 0u, __ATOMIC_RELEASE);
    e = hipMemsetAsync(sa.go, 0, sizeof(unsigned), s);
    if (e == hipSuccess)
        e = ramppi::launch_serve(c, bufs, g.block, lds,
                                 reinterpret_cast<const ramppi::FuseArgs*>(h->ws + h->l.fuse), sa, s);
    if (e != hipSuccess) return hip_fail(e, "serving launch");
    h->serving = true;
    h->serve_seq = 0;
    h->serve_stream = s;
    return MPPI_OK;
}

namespace {

// Posts the next request: the per-step fields first, its number last.
void post_request(mppi_handle* h, const ramppi::StepConst* c, uint32_t stop) {
    ramppi::ServeReq* r = h->req;
    if (c) {
        r->step_idx = c->step_idx;
        r->fx = c->fx;
        r->fy = c->fy;
        r->tox = c->tox;
        r->toy = c->toy;
        r->theta0 = c->theta0;
        r->psi0 = c->psi0;
        r->v0 = c->v0;
    }
    r->stop = stop;
    __atomic_store_n(&r->seq, ++h->serve_seq, __ATOMIC_RELEASE);
}

}  // namespace

mppi_status mppi_serve_step(mppi_handle* h, const float x0[4], uint32_t step_idx, float* u0_host) {
    if (!h) return fail(MPPI_EINVAL, "handle is NULL");
    if (!x0 || !u0_host) return fail(MPPI_EINVAL, "x0 or u0_host is NULL");
    if (!h->serving) return fail(MPPI_EINVAL, "the handle is not serving (mppi_serve_start first)");
    for (int i = 0; i < 4; ++i)
        if (!finite(x0[i])) return fail(MPPI_EINVAL, "x0[%d] is not finite", i);
    ramppi::StepConst c;
    fill_dynamic(&c, h->p, x0, step_idx);
    post_request(h, &c, 0u);
    const uint32_t* word = reinterpret_cast<const uint32_t*>(h->u0_pinned + 2);
    for (uint64_t spin = 1;; ++spin) {
        if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == h->serve_seq) break;
        if ((spin & 1023) == 0) {
            const hipError_t q = hipStreamQuery(h->serve_stream);
            if (q == hipSuccess) {  // the serving launch has left (its idle limit passed)
                if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == h->serve_seq) break;
                h->serving = false;
                h->u0_seq = std::max(h->u0_seq, h->serve_seq);
                return fail(MPPI_EDEVICE, "the serving launch has stopped (no request within its idle limit)");
            }
            if (q != hipErrorNotReady) return hip_fail(q, "serving readback");
        }
        __builtin_ia32_pause();
    }
    u0_host[0] = h->u0_pinned[0];
    u0_host[1] = h->u0_pinned[1];
    return MPPI_OK;
}

mppi_status mppi_serve_stop(mppi_handle* h) {
    if (!h) return fail(MPPI_EINVAL, "handle is NULL");
    if (!h->serving) return MPPI_OK;
    post_request(h, nullptr, 1u);
    const hipError_t e = hipStreamSynchronize(h->serve_stream);
    h->serving = false;
    // launched steps after the session use completion values above every served one
    h->u0_seq = std::max(h->u0_seq, h->serve_seq);
    if (e != hipSuccess) return hip_fail(e, "serving stop");
    return MPPI_OK;
}

mppi_status mppi_grad(mppi_handle* h, const float x0[4], const float* V_dev, uint32_t step_idx, float* grad_dev,
                      float* J_dev, void* stream) {
    if (!h) return fail(MPPI_EINVAL, "handle is NULL");
    if (!(h->p.flags & MPPI_F_GRAD)) return fail(MPPI_EINVAL, "the handle was created without MPPI_F_GRAD");
    if (!x0 || !V_dev || !grad_dev) return fail(MPPI_EINVAL, "x0, V_dev or grad_dev is NULL");
    if (h->serving) return fail(MPPI_EINVAL, "the handle is serving (mppi_serve_stop first)");
    for (int i = 0; i < 4; ++i)
        if (!finite(x0[i])) return fail(MPPI_EINVAL, "x0[%d] is not finite", i);
    const mppi_params& p = h->p;
    const Geometry& g = h->g;
    const Layout& l = h->l;
    hipStream_t s = static_cast<hipStream_t>(stream);

    ramppi::StepConst c;
    fill_static(&c, p, g, h->n_tail, h->n_warm);
    fill_dynamic(&c, p, x0, step_idx);
    c.grad = 1;
    c.debug = 0;
    c.store_u = 1;  // the gradient's recomputed rollouts read the controls

    ramppi::StepBuffers bufs = step_buffers(h, const_cast<float*>(V_dev));
    bufs.Vout = nullptr;
    ramppi::GradArgs a;
    a.V = V_dev;
    a.u = bufs.u;
    a.cvar = bufs.cvar;
    a.w_hat = bufs.w_hat;
    a.act_list = reinterpret_cast<const int*>(h->ws + l.act_list);
    a.n_act = reinterpret_cast<const int*>(h->ws + l.n_act);
    a.tail_idx = reinterpret_cast<const int*>(h->ws + l.tail_idx);
    a.ranks = reinterpret_cast<const int*>(h->ws + l.ranks);
    a.ranks_w = reinterpret_cast<int*>(h->ws + l.ranks);
    a.tail_w = reinterpret_cast<int*>(h->ws + l.tail_idx);
    a.states = reinterpret_cast<float4*>(h->ws + l.states);
    a.rows = reinterpret_cast<float*>(h->ws + l.rows);
    a.rpart = reinterpret_cast<float*>(h->ws + l.rpart);
    a.counter = reinterpret_cast<unsigned*>(h->ws + l.gcounter);
    a.grad_out = grad_dev;
    a.R = l.R;
    a.stride = l.stride;
    ramppi::GradOut go;
    go.J = J_dev ? J_dev : reinterpret_cast<float*>(h->ws + l.J);
    go.act_list = reinterpret_cast<int*>(h->ws + l.act_list);
    go.n_act = reinterpret_cast<int*>(h->ws + l.n_act);
    const hipError_t e =
        ramppi::launch_grad(c, bufs, a, go, g.block, g.lds_rollout, g.G, g.lds_update, l.n_lane_blocks, s);
    if (e != hipSuccess) return hip_fail(e, "gradient launch");
    return MPPI_OK;
}

mppi_status mppi_debug_view(const mppi_handle* h, mppi_debug_ptrs* out) {
    if (!h || !out) return fail(MPPI_EINVAL, "handle or out is NULL");
    out->u = reinterpret_cast<const float*>(h->ws + h->l.u);
    out->S = reinterpret_cast<const float*>(h->ws + h->l.S);
    out->L = reinterpret_cast<const float*>(h->ws + h->l.L);
    out->cvar = reinterpret_cast<const float*>(h->ws + h->l.cvar);
    out->S_tilde = reinterpret_cast<const float*>(h->ws + h->l.S_tilde);
    out->w_hat = reinterpret_cast<const float*>(h->ws + h->l.w_hat);
    out->u0 = reinterpret_cast<const float*>(h->ws + h->l.u0);
    return MPPI_OK;
}

mppi_status mppi_timing_enable(mppi_handle* h, int enable) {
    if (!h) return fail(MPPI_EINVAL, "handle is NULL");
    if (enable && h->ev.empty()) {
        h->ev.resize(3 * (size_t)kMaxTimedSteps, nullptr);
        for (auto& ev : h->ev) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
    }
    h->timing = enable != 0;
    if (enable == 1) h->n_timed = 0;  // 2 resumes, 0 pauses: the records stay
    return MPPI_OK;
}

mppi_status mppi_timing_read(mppi_handle* h, double* rollout_ms, double* update_ms, int32_t* n_steps) {
    if (!h || !rollout_ms || !update_ms || !n_steps) return fail(MPPI_EINVAL, "NULL argument");
    double r = 0.0, u = 0.0;
    for (int i = 0; i < h->n_timed; ++i) {
        hipEvent_t* e3 = &h->ev[3 * (size_t)i];
        hipError_t e = hipEventSynchronize(e3[2]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float a = 0.0f, b = 0.0f;
        e = hipEventElapsedTime(&a, e3[0], e3[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, e3[1], e3[2]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        r += a;
        u += b;
    }
    *rollout_ms = r;
    *update_ms = u;
    *n_steps = h->n_timed;
    h->n_timed = 0;
    return MPPI_OK;
}

mppi_status mppi_timing_work(mppi_handle* h, void* stream, uint64_t* n_candidates, uint64_t* n_group_tests) {
    if (!h || !n_candidates || !n_group_tests) return fail(MPPI_EINVAL, "NULL argument");
    const hipError_t e = read_work(reinterpret_cast<unsigned long long*>(h->ws + h->l.work),
                                   static_cast<hipStream_t>(stream), n_candidates, n_group_tests);
    if (e != hipSuccess) return hip_fail(e, "broad-phase counters");
    return MPPI_OK;
}

mppi_status mppi_timing_candidates(mppi_handle* h, void* stream, uint64_t* n_candidates) {
    if (!h || !n_candidates) return fail(MPPI_EINVAL, "NULL argument");
    const hipError_t e = read_work(reinterpret_cast<unsigned long long*>(h->ws + h->l.work),
                                   static_cast<hipStream_t>(stream), n_candidates, nullptr);
    if (e != hipSuccess) return hip_fail(e, "candidate counters");
    return MPPI_OK;
}

mppi_status mppi_philox(uint64_t seed, const uint32_t* ctr_dev, uint32_t* out_dev, int64_t n, void* stream) {
    if (n < 0) return fail(MPPI_EINVAL, "n < 0");
    if (n == 0) return MPPI_OK;
    if (!ctr_dev || !out_dev) return fail(MPPI_EINVAL, "NULL buffer");
    if (n > ((int64_t)1 << 31) * 256 - 1) return fail(MPPI_EUNSUPPORTED, "n too large");
    int dev;
    mppi_status st = check_device(&dev);
    if (st != MPPI_OK) return st;
    hipError_t e = ramppi::launch_philox(seed, ctr_dev, out_dev, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? MPPI_OK : hip_fail(e, "philox launch");
}

mppi_status mppi_normals(uint64_t seed, const uint32_t* ctr_dev, float* out_dev, int64_t n, void* stream) {
    if (n < 0) return fail(MPPI_EINVAL, "n < 0");
    if (n == 0) return MPPI_OK;
    if (!ctr_dev || !out_dev) return fail(MPPI_EINVAL, "NULL buffer");
    if (n > ((int64_t)1 << 31) * 256 - 1) return fail(MPPI_EUNSUPPORTED, "n too large");
    int dev;
    mppi_status st = check_device(&dev);
    if (st != MPPI_OK) return st;
    hipError_t e = ramppi::launch_normals(seed, ctr_dev, out_dev, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? MPPI_OK : hip_fail(e, "normals launch");
}

mppi_status mppi_cvar(const float* L_dev, int32_t K, int32_t M, float alpha, float B, float* cvar_dev,
                      void* stream) {
    if (K < 0 || M < 1) return fail(MPPI_EINVAL, "need K >= 0 and M >= 1");
    if (M > MPPI_MAX_M) return fail(MPPI_EUNSUPPORTED, "M = %d exceeds %d", M, MPPI_MAX_M);
    if (!(alpha > 0 && alpha < 1)) return fail(MPPI_EINVAL, "alpha must lie in (0, 1)");
    if (!(finite(B) && B >= 0)) return fail(MPPI_EINVAL, "B must be finite and >= 0");
    if (K == 0) return MPPI_OK;
    if (!L_dev || !cvar_dev) return fail(MPPI_EINVAL, "NULL buffer");
    if ((int64_t)K * M > (int64_t)INT32_MAX) return fail(MPPI_EUNSUPPORTED, "K * M exceeds 2^31 - 1");
    int dev;
    mppi_status st = check_device(&dev);
    if (st != MPPI_OK) return st;
    mppi_params q;
    std::memset(&q, 0, sizeof q);
    q.K = K;
    q.M = M;
    q.alpha = alpha;
    int n_tail, n_warm;
    derived_counts(&q, &n_tail, &n_warm);
    const int spb = M >= 256 ? 1 : 256 / M;
    const int block = (spb * M + 63) / 64 * 64;
    hipError_t e = ramppi::launch_cvar(L_dev, K, M, spb, block, n_tail, B != 1.0f, B, cvar_dev,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? MPPI_OK : hip_fail(e, "cvar launch");
}


// ======================================================================
// Batched serving (many independent controllers per launch)
// ======================================================================
}  // extern "C"

namespace {

constexpr int kBatchBlock = 256;
constexpr int kMaxBatch = 65535;

// Rollout geometry of a controller inside a batch: workgroups of 256 lanes.
Geometry batch_geometry(const mppi_params* p) {
    Geometry g = geometry(p);
    g.spb = p->M >= kBatchBlock ? 1 : kBatchBlock / p->M;
    g.block = kBatchBlock;
    g.n_nom_wg = (p->K + kBatchBlock - 1) / kBatchBlock;
    g.lds_rollout = rollout_lds_bytes(g.spb, p);
    return g;
}

int n_dist_wg(const mppi_params* p, const Geometry& g) { return (p->K + g.spb - 1) / g.spb; }

struct BatchLayout {
    size_t ctls, items, uitems, queue, vbackup, work;
    std::vector<size_t> ctl_base;
    size_t total;
    int n_items, n_uitems;
    int noise_kind;  // the disturbance form of every controller, or -1 when they differ
    size_t lds_rollout, lds_update;
};

mppi_status batch_check(int32_t n, const mppi_params* p) {
    if (n < 1 || n > kMaxBatch) return fail(MPPI_EINVAL, "batch size must lie in [1, %d]", kMaxBatch);
    if (!p) return fail(MPPI_EINVAL, "params is NULL");
    for (int i = 0; i < n; ++i) {
        mppi_status st = mppi_validate(&p[i]);
        if (st != MPPI_OK) {
            std::string m = g_err;
            return fail(st, "controller %d: %s", i, m.c_str());
        }
        if (p[i].M > kBatchBlock)
            return fail(MPPI_EUNSUPPORTED, "controller %d: M = %d exceeds %d in a batch", i, p[i].M, kBatchBlock);
        const Geometry g = batch_geometry(&p[i]);
        if (g.lds_rollout > kMaxLdsBytes)
            return fail(MPPI_EUNSUPPORTED, "controller %d: rollout LDS need %zu B exceeds %zu B", i, g.lds_rollout,
                        kMaxLdsBytes);
    }
    return MPPI_OK;
}

BatchLayout batch_layout(int32_t n, const mppi_params* p) {
    BatchLayout bl;
    bl.n_items = 0;
    bl.n_uitems = 0;
    bl.lds_rollout = 0;
    bl.lds_update = 0;
    bl.noise_kind = (int)p[0].noise_kind;
    size_t vback = 0;
    for (int i = 0; i < n; ++i) {
        if ((int)p[i].noise_kind != bl.noise_kind) bl.noise_kind = -1;
        const Geometry g = batch_geometry(&p[i]);
        bl.n_items += g.n_nom_wg + n_dist_wg(&p[i], g);
        bl.n_uitems += g.G;
        bl.lds_rollout = std::max(bl.lds_rollout, g.lds_rollout);
        bl.lds_update = std::max(bl.lds_update, g.lds_update);
        vback += align_up(8 * (size_t)p[i].T);
    }
    size_t o = 0;
    bl.ctls = o;    o += align_up(sizeof(ramppi::BatchCtl) * (size_t)n);
    bl.items = o;   o += align_up(8 * (size_t)bl.n_items);
    bl.uitems = o;  o += align_up(8 * (size_t)bl.n_uitems);
    bl.queue = o;   o += align_up(8);
    bl.work = o;    o += align_up(16 * (size_t)ramppi::kWorkSlots);
    bl.vbackup = o; o += vback;
    bl.ctl_base.resize(n);
    for (int i = 0; i < n; ++i) {
        bl.ctl_base[i] = o;
        o += layout(&p[i]).total;
    }
    bl.total = o;
    return bl;
}

}  // namespace

struct mppi_batch {
    int n, device, num_cu, wg_per_cu, wg_max, order;
    std::vector<mppi_params> p;
    std::vector<ramppi::BatchCtl> ctl;  // host copy (device pointers inside)
    std::vector<float*> V;
    BatchLayout bl;
    char* ws;
    ramppi::BatchInput* in_host;
    ramppi::BatchInput* in_dev;
    float* out_host;
    float* out_dev;
    std::vector<int2> items[2];  // 0: controller order, 1: longest first
    bool use_graph, captured, pending;
    hipStream_t cap;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipEvent_t done;
    bool timing;
    std::vector<hipEvent_t> ev;  // 3 per timed step: start, after rollout, end
    int n_timed;
};

namespace {

ramppi::BatchLaunch batch_launch_args(const mppi_batch* b) {
    ramppi::BatchLaunch L;
    L.ctls = reinterpret_cast<ramppi::BatchCtl*>(b->ws + b->bl.ctls);
    L.inputs = b->in_dev;
    L.items = reinterpret_cast<const int2*>(b->ws + b->bl.items);
    L.uitems = reinterpret_cast<const int2*>(b->ws + b->bl.uitems);
    L.queue = reinterpret_cast<unsigned*>(b->ws + b->bl.queue);
    L.work = nullptr;
    L.n_ctl = b->n;
    L.n_items = b->bl.n_items;
    L.n_uitems = b->bl.n_uitems;
    L.grid_rollout = b->wg_per_cu * b->num_cu;
    L.noise_kind = b->bl.noise_kind;
    L.lds_rollout = b->bl.lds_rollout;
    L.lds_update = b->bl.lds_update;
    return L;
}

void batch_release(mppi_batch* b) {
    for (hipEvent_t ev : b->ev) (void)hipEventDestroy(ev);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->in_host) (void)hipHostFree(b->in_host);
    if (b->out_host) (void)hipHostFree(b->out_host);
    delete b;
}

void drop_graph(mppi_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->captured = false;
}

hipError_t upload_items(mppi_batch* b, int order, hipStream_t s) {
    const std::vector<int2>& it = b->items[order];
    return hipMemcpyAsync(b->ws + b->bl.items, it.data(), 8 * it.size(), hipMemcpyHostToDevice, s);
}

hipError_t batch_launch(mppi_batch* b, hipStream_t s, bool graph) {
    const ramppi::BatchLaunch L = batch_launch_args(b);
    if (!graph) return ramppi::launch_batch(L, s);
    if (!b->captured) {
        hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return e;
        e = ramppi::launch_batch(L, b->cap);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap, &g);
        if (e == hipSuccess) e = e2;
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return e;
        }
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return e;
        }
        b->graph = g;
        b->captured = true;
    }
    return hipGraphLaunch(b->exec, s);
}

}  // namespace

extern "C" {

size_t mppi_batch_workspace_bytes(int32_t n, const mppi_params* p) {
    if (batch_check(n, p) != MPPI_OK) return 0;
    return batch_layout(n, p).total;
}

mppi_status mppi_batch_create(int32_t n, const mppi_params* p, const float* const* obstacles_host,
                              float* const* V_dev, void* workspace_dev, size_t workspace_bytes, void* stream,
                              mppi_batch** out) {
    if (!out) return fail(MPPI_EINVAL, "out is NULL");
    *out = nullptr;
    mppi_status st = batch_check(n, p);
    if (st != MPPI_OK) return st;
    if (!obstacles_host || !V_dev) return fail(MPPI_EINVAL, "obstacles_host or V_dev is NULL");
    for (int i = 0; i < n; ++i) {
        if (!V_dev[i]) return fail(MPPI_EINVAL, "V_dev[%d] is NULL", i);
        if (p[i].n_obs > 0 && !obstacles_host[i]) return fail(MPPI_EINVAL, "obstacles_host[%d] is NULL", i);
        for (int j = 0; j < p[i].n_obs; ++j) {
            const float* o = obstacles_host[i] + 3 * j;
            if (!(finite(o[0]) && finite(o[1]) && finite(o[2]) && o[2] > 0))
                return fail(MPPI_EINVAL, "controller %d obstacle %d must have a finite centre and a radius > 0", i,
                            j);
        }
    }
    const BatchLayout bl = batch_layout(n, p);
    if (!workspace_dev) return fail(MPPI_EINVAL, "workspace_dev is NULL");
    if (((uintptr_t)workspace_dev) % kAlign) return fail(MPPI_EINVAL, "workspace_dev must be 256-byte aligned");
    if (workspace_bytes < bl.total) return fail(MPPI_EINVAL, "workspace has %zu B, needs %zu B", workspace_bytes, bl.total);
    int dev = 0;
    st = check_device(&dev);
    if (st != MPPI_OK) return st;

    mppi_batch* b = new (std::nothrow) mppi_batch();
    if (!b) return fail(MPPI_ENOMEM, "host allocation failed");
    b->n = n;
    b->device = dev;
    b->p.assign(p, p + n);
    b->V.assign(V_dev, V_dev + n);
    b->bl = bl;
    b->ws = static_cast<char*>(workspace_dev);
    b->in_host = nullptr;
    b->out_host = nullptr;
    b->use_graph = true;
    b->captured = false;
    b->pending = false;
    b->cap = nullptr;
    b->graph = nullptr;
    b->exec = nullptr;
    b->done = nullptr;
    b->timing = false;
    b->n_timed = 0;
    hipError_t e = hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = ramppi::batch_rollout_occupancy(&b->wg_max, bl.lds_rollout, bl.noise_kind);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->in_host), sizeof(ramppi::BatchInput) * (size_t)n,
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&b->in_dev), b->in_host, 0);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->out_host), 2 * sizeof(float) * (size_t)n,
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&b->out_dev), b->out_host, 0);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_release(b);
        return hip_fail(e, "batch set-up");
    }
    if (b->wg_max < 1) b->wg_max = 1;
    b->wg_per_cu = b->wg_max;
    b->order = 1;
    std::memset(b->in_host, 0, sizeof(ramppi::BatchInput) * (size_t)n);

    // controllers: static constants and buffer addresses; item lists
    b->ctl.resize(n);
    std::vector<std::pair<double, int2>> cost_items;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int2> uitems;
    for (int i = 0; i < n; ++i) {
        const Geometry g = batch_geometry(&p[i]);
        const Layout l = layout(&p[i]);
        int n_tail, n_warm;
        derived_counts(&p[i], &n_tail, &n_warm);
        ramppi::BatchCtl& c = b->ctl[i];
        std::memset(&c, 0, sizeof c);
        fill_static(&c.c, p[i], g, n_tail, n_warm);
        char* base = b->ws + bl.ctl_base[i];
        c.obs = reinterpret_cast<const float4*>(base + l.obs);
        c.V = V_dev[i];
        c.u = reinterpret_cast<float2*>(base + l.u);
        c.S = reinterpret_cast<float*>(base + l.S);
        c.cvar = reinterpret_cast<float*>(base + l.cvar);
        c.S_tilde = reinterpret_cast<float*>(base + l.S_tilde);
        c.w_hat = reinterpret_cast<float*>(base + l.w_hat);
        c.L = reinterpret_cast<float*>(base + l.L);
        c.part = reinterpret_cast<float*>(base + l.part);
        c.counter = reinterpret_cast<unsigned*>(base + l.counter);
        c.u0 = reinterpret_cast<float*>(base + l.u0);
        c.u0_host = b->out_dev + 2 * (size_t)i;
        c.G = g.G;
        c.parts = ramppi::update_parts(p[i].T);
        for (int j = 0; j < 4; ++j) c.track[j] = p[i].track[j];
        // the cost of any workgroup of this controller: T steps of the
        // per-step work plus three instructions per obstacle
        const double cost = (double)p[i].T * (40.0 + 3.0 * (double)((p[i].n_obs + 7) / 8 * 8));
        const int nw = g.n_nom_wg + n_dist_wg(&p[i], g);
        for (int w = 0; w < nw; ++w) {
            b->items[0].push_back(make_int2(i, w));
            cost_items.push_back({cost, make_int2(i, w)});
        }
        for (int ch = 0; ch < g.G; ++ch) uitems.push_back(make_int2(i, ch));
        std::vector<float> staged(4 * (size_t)(p[i].n_obs > 0 ? p[i].n_obs : 1), 0.0f);
        const std::vector<int> order = obstacle_order(obstacles_host[i], p[i].n_obs);
        for (int j = 0; j < p[i].n_obs; ++j)
            for (int q = 0; q < 3; ++q) staged[4 * j + q] = obstacles_host[i][3 * order[j] + q];
        if (e == hipSuccess && p[i].n_obs > 0)
            e = hipMemcpyAsync(base + l.obs, staged.data(), 16 * (size_t)p[i].n_obs, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(base + l.counter, 0, 4, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // staged is a local buffer
    }
    std::stable_sort(cost_items.begin(), cost_items.end(),
                     [](const std::pair<double, int2>& a, const std::pair<double, int2>& c) { return a.first > c.first; });
    for (auto& ci : cost_items) b->items[1].push_back(ci.second);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + bl.ctls, b->ctl.data(), sizeof(ramppi::BatchCtl) * (size_t)n,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = upload_items(b, b->order, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + bl.uitems, uitems.data(), 8 * uitems.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(b->ws + bl.queue, 0, 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(b->ws + bl.work, 0, 16 * (size_t)ramppi::kWorkSlots, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        batch_release(b);
        return hip_fail(e, "batch upload");
    }
    *out = b;
    return MPPI_OK;
}

mppi_status mppi_batch_step(mppi_batch* b, const float* x0_host, const uint32_t* step_idx_host, float* u0_host,
                            void* stream) {
    if (!b) return fail(MPPI_EINVAL, "batch is NULL");
    if (!x0_host || !step_idx_host) return fail(MPPI_EINVAL, "x0_host or step_idx_host is NULL");
    for (int i = 0; i < 4 * b->n; ++i)
        if (!finite(x0_host[i])) return fail(MPPI_EINVAL, "x0 of controller %d is not finite", i / 4);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (b->pending) {  // the previous step may still read the inputs
        e = hipEventSynchronize(b->done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    for (int i = 0; i < b->n; ++i) {
        for (int j = 0; j < 4; ++j) b->in_host[i].x0[j] = x0_host[4 * i + j];
        b->in_host[i].step_idx = step_idx_host[i];
    }
    if (b->timing && b->n_timed < kMaxTimedSteps) {
        hipEvent_t* e3 = &b->ev[3 * (size_t)b->n_timed];
        ramppi::BatchLaunch L = batch_launch_args(b);
        L.work = reinterpret_cast<unsigned long long*>(b->ws + b->bl.work);
        e = ramppi::launch_batch(L, s, e3[0], e3[1]);
        if (e == hipSuccess) e = hipEventRecord(e3[2], s);
        if (e == hipSuccess) b->n_timed++;
    } else {
        e = batch_launch(b, s, b->use_graph);
    }
    if (e == hipSuccess) e = hipEventRecord(b->done, s);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    b->pending = true;
    if (u0_host) {
        e = hipEventSynchronize(b->done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        std::memcpy(u0_host, b->out_host, 2 * sizeof(float) * (size_t)b->n);
    }
    return MPPI_OK;
}

mppi_status mppi_batch_set_graph(mppi_batch* b, int enable) {
    if (!b) return fail(MPPI_EINVAL, "batch is NULL");
    b->use_graph = enable != 0;
    return MPPI_OK;
}

mppi_status mppi_batch_timing_enable(mppi_batch* b, int enable) {
    if (!b) return fail(MPPI_EINVAL, "batch is NULL");
    if (enable && b->ev.empty()) {
        b->ev.resize(3 * (size_t)kMaxTimedSteps, nullptr);
        for (auto& ev : b->ev) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
    }
    b->timing = enable != 0;
    b->n_timed = 0;
    return MPPI_OK;
}

mppi_status mppi_batch_timing_read(mppi_batch* b, double* rollout_ms, double* update_ms, int32_t* n_steps) {
    if (!b || !rollout_ms || !update_ms || !n_steps) return fail(MPPI_EINVAL, "NULL argument");
    double r = 0.0, u = 0.0;
    for (int i = 0; i < b->n_timed; ++i) {
        hipEvent_t* e3 = &b->ev[3 * (size_t)i];
        hipError_t e = hipEventSynchronize(e3[2]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float x = 0.0f, y = 0.0f;
        e = hipEventElapsedTime(&x, e3[0], e3[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&y, e3[1], e3[2]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        r += x;
        u += y;
    }
    *rollout_ms = r;
    *update_ms = u;
    *n_steps = b->n_timed;
    b->n_timed = 0;
    return MPPI_OK;
}

mppi_status mppi_batch_timing_work(mppi_batch* b, void* stream, uint64_t* n_candidates, uint64_t* n_group_tests) {
    if (!b || !n_candidates || !n_group_tests) return fail(MPPI_EINVAL, "NULL argument");
    const hipError_t e = read_work(reinterpret_cast<unsigned long long*>(b->ws + b->bl.work),
                                   static_cast<hipStream_t>(stream), n_candidates, n_group_tests);
    if (e != hipSuccess) return hip_fail(e, "broad-phase counters");
    return MPPI_OK;
}

mppi_status mppi_batch_timing_candidates(mppi_batch* b, void* stream, uint64_t* n_candidates) {
    if (!b || !n_candidates) return fail(MPPI_EINVAL, "NULL argument");
    const hipError_t e = read_work(reinterpret_cast<unsigned long long*>(b->ws + b->bl.work),
                                   static_cast<hipStream_t>(stream), n_candidates, nullptr);
    if (e != hipSuccess) return hip_fail(e, "candidate counters");
    return MPPI_OK;
}

mppi_status mppi_batch_autotune(mppi_batch* b, int32_t trials, void* stream, int32_t* wg_per_cu, int32_t* order) {
    if (!b) return fail(MPPI_EINVAL, "batch is NULL");
    if (trials < 1) return fail(MPPI_EINVAL, "trials must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess && b->pending) e = hipEventSynchronize(b->done);
    // keep the mean sequences: tuning runs real steps, which update them
    size_t off = b->bl.vbackup;
    for (int i = 0; e == hipSuccess && i < b->n; ++i) {
        e = hipMemcpyAsync(b->ws + off, b->V[i], 8 * (size_t)b->p[i].T, hipMemcpyDeviceToDevice, s);
        off += align_up(8 * (size_t)b->p[i].T);
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    const int saved_wg = b->wg_per_cu, saved_order = b->order;
    float best = -1.0f;
    int best_wg = saved_wg, best_order = saved_order;
    for (int ord = 0; e == hipSuccess && ord < 2; ++ord) {
        e = upload_items(b, ord, s);
        for (int wg = 1; e == hipSuccess && wg <= b->wg_max; wg *= 2) {
            b->wg_per_cu = wg;
            e = batch_launch(b, s, false);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(t0, s);
            for (int r = 0; e == hipSuccess && r < trials; ++r) e = batch_launch(b, s, false);
            if (e == hipSuccess) e = hipEventRecord(t1, s);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e == hipSuccess && (best < 0.0f || ms < best)) {
                best = ms;
                best_wg = wg;
                best_order = ord;
            }
        }
    }
    b->wg_per_cu = best_wg;
    b->order = best_order;
    if (e == hipSuccess) e = upload_items(b, best_order, s);
    off = b->bl.vbackup;
    for (int i = 0; e == hipSuccess && i < b->n; ++i) {
        e = hipMemcpyAsync(b->V[i], b->ws + off, 8 * (size_t)b->p[i].T, hipMemcpyDeviceToDevice, s);
        off += align_up(8 * (size_t)b->p[i].T);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    drop_graph(b);  // the grid changed: capture again on the next step
    b->pending = false;
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (wg_per_cu) *wg_per_cu = best_wg;
    if (order) *order = best_order;
    return MPPI_OK;
}

mppi_status mppi_batch_debug_view(const mppi_batch* b, int32_t i, mppi_debug_ptrs* out) {
    if (!b || !out) return fail(MPPI_EINVAL, "batch or out is NULL");
    if (i < 0 || i >= b->n) return fail(MPPI_EINVAL, "controller index %d out of range", i);
    const ramppi::BatchCtl& c = b->ctl[i];
    out->u = reinterpret_cast<const float*>(c.u);
    out->S = c.S;
    out->L = c.L;
    out->cvar = c.cvar;
    out->S_tilde = c.S_tilde;
    out->w_hat = c.w_hat;
    out->u0 = c.u0;
    return MPPI_OK;
}

mppi_status mppi_batch_destroy(mppi_batch* b) {
    if (!b) return MPPI_OK;
    if (b->pending) (void)hipEventSynchronize(b->done);
    batch_release(b);
    return MPPI_OK;
}

}  // extern "C"

