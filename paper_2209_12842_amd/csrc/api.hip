// C ABI of the RA-MPPI library: parameter validation, workspace layout,
// handle management and launches.  Declarations and contracts: ramppi.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
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
    g.lds_rollout = 8 * (size_t)g.spb * p->T + 4 * (2 * (size_t)g.spb * p->M + g.spb);
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
    size_t obs, tab, u, S, cvar, S_tilde, w_hat, L, part, u0, counter, total;
};

Layout layout(const mppi_params* p) {
    const Geometry g = geometry(p);
    Layout l;
    size_t o = 0;
    l.obs = o;     o += align_up(16 * (size_t)(p->n_obs > 0 ? p->n_obs : 1));
    l.tab = o;     o += align_up(16 * (size_t)(p->n_obs > 0 ? (p->n_obs + 7) / 8 * 8 : 8));
    l.u = o;       o += align_up(8 * (size_t)p->K * p->T);
    l.S = o;       o += align_up(4 * (size_t)p->K);
    l.cvar = o;    o += align_up(4 * (size_t)p->K);
    l.S_tilde = o; o += align_up(4 * (size_t)p->K);
    l.w_hat = o;   o += align_up(4 * (size_t)p->K);
    l.L = o;       o += align_up(4 * (size_t)p->K * p->M);
    l.part = o;    o += align_up(4 * (size_t)g.G * (2 + 2 * (size_t)p->T));
    l.u0 = o;      o += align_up(8);
    l.counter = o; o += align_up(4);
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

}  // namespace

struct mppi_handle {
    mppi_params p;
    Geometry g;
    Layout l;
    int n_tail, n_warm, device;
    char* ws;
    float* u0_pinned;      // mapped, coherent pinned host memory (2 floats)
    float* u0_pinned_dev;  // its device address
    bool timing;
    std::vector<hipEvent_t> ev;  // 3 per timed step: start, after rollout, end
    int n_timed;
};

extern "C" {

mppi_status mppi_validate(const mppi_params* p) {
    if (!p) return fail(MPPI_EINVAL, "params is NULL");
    if (p->K < 1 || p->T < 1 || p->M < 1 || p->n_obs < 0)
        return fail(MPPI_EINVAL, "sizes must satisfy K, T, M >= 1 and n_obs >= 0 (got K=%d T=%d M=%d n_obs=%d)",
                    p->K, p->T, p->M, p->n_obs);
    if (p->flags & ~(uint32_t)(MPPI_F_DEBUG | MPPI_F_SHIFT | MPPI_F_ALLOW_ZERO_NOISE))
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
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->u0_pinned), 2 * sizeof(float),
                                 hipHostMallocMapped | hipHostMallocCoherent);
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
    for (int i = 0; i < p->n_obs; ++i) {
        staged[4 * i + 0] = obstacles_host[3 * i + 0];
        staged[4 * i + 1] = obstacles_host[3 * i + 1];
        staged[4 * i + 2] = obstacles_host[3 * i + 2];
    }
    e = hipMemcpyAsync(h->ws + l.obs, staged.data(), 16 * (size_t)p->n_obs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + l.counter, 0, 4, s);
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
    for (int i = 0; i < 4; ++i)
        if (!finite(x0[i])) return fail(MPPI_EINVAL, "x0[%d] is not finite", i);
    const mppi_params& p = h->p;
    const Geometry& g = h->g;
    hipStream_t s = static_cast<hipStream_t>(stream);

    ramppi::StepConst c;
    std::memset(&c, 0, sizeof c);
    c.K = p.K;
    c.T = p.T;
    c.M = p.M;
    c.n_obs = p.n_obs;
    c.spb = g.spb;
    c.n_nom_wg = g.n_nom_wg;
    c.n_warm = h->n_warm;
    c.n_tail = h->n_tail;
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
    c.c4 = p.c4;
    c.c5 = p.c5;
    c.use_bdry = p.c_bdry != 0.0f;
    c.use_term = (p.c4 != 0.0f) || (p.c5 != 0.0f);
    c.fx = x0[0];
    c.fy = x0[1];
    c.tox = x0[0] - p.track[0];
    c.toy = x0[1] - p.track[1];
    const double a = p.track[2], b = p.track[3];
    c.inv_a = (float)(1.0 / a);
    c.inv_b = (float)(1.0 / b);
    c.g_a = (float)(2.0 / (a * a));
    c.g_b = (float)(2.0 / (b * b));
    c.hw = p.track[4];
    c.half_ab = (float)(0.5 * (a + b));
    c.theta0 = (float)std::atan2(((double)x0[1] - p.track[1]) / b, ((double)x0[0] - p.track[0]) / a);
    c.psi0 = x0[2];
    c.v0 = x0[3];
    c.key0 = (uint32_t)(p.seed & 0xFFFFFFFFu);
    c.key1 = (uint32_t)(p.seed >> 32);
    c.step_idx = step_idx;
    c.flags = p.flags;
    c.debug = (p.flags & MPPI_F_DEBUG) != 0;

    ramppi::StepBuffers bufs;
    bufs.obs = reinterpret_cast<const float4*>(h->ws + h->l.obs);
    bufs.tab = reinterpret_cast<float4*>(h->ws + h->l.tab);
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
    bufs.u0_host = u0_host ? h->u0_pinned_dev : nullptr;

    hipEvent_t ev_start = nullptr, ev_mid = nullptr, ev_end = nullptr;
    if (h->timing && h->n_timed < kMaxTimedSteps) {
        hipEvent_t* e3 = &h->ev[3 * (size_t)h->n_timed];
        ev_start = e3[0];
        ev_mid = e3[1];
        ev_end = e3[2];
    }
    hipError_t e = ramppi::launch_step(c, bufs, g.block, g.lds_rollout, g.G, g.lds_update, s, ev_start, ev_mid);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    if (ev_end) {
        e = hipEventRecord(ev_end, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        h->n_timed++;
    }
    if (u0_host) {
        // the update kernel stored the command into the mapped pinned buffer
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "first-command readback");
        u0_host[0] = h->u0_pinned[0];
        u0_host[1] = h->u0_pinned[1];
    }
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
    h->n_timed = 0;
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

}  // extern "C"
