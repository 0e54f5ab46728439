// C ABI of librfvr: argument validation, workspace layout and launches.
// Every check runs before the first enqueue, so a failing call enqueues nothing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "rfvr_impl.hpp"

namespace rfvr {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return RFVR_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return RFVR_E_HIP;
}

static constexpr int kMaxFreq = 8192;

static int check_aperture(const rfvr_aperture* ap) {
    if (!ap) { set_error("aperture descriptor is NULL"); return RFVR_E_INVALID; }
    if (ap->n_meas < 1 || ap->n_meas > RFVR_MAX_MEAS) {
        set_error("n_meas must be in [1, RFVR_MAX_MEAS] (got %d)", ap->n_meas);
        return RFVR_E_INVALID;
    }
    if (ap->n_freq < 1 || ap->n_freq > kMaxFreq) {
        set_error("n_freq must be in [1, %d] (got %d)", kMaxFreq, ap->n_freq);
        return RFVR_E_INVALID;
    }
    if (!ap->tx) { set_error("aperture tx is NULL"); return RFVR_E_INVALID; }
    if (!std::isfinite(ap->f0_hz) || !std::isfinite(ap->df_hz) || ap->f0_hz <= 0.0 || ap->df_hz < 0.0) {
        set_error("f0_hz must be finite and > 0, df_hz finite and >= 0");
        return RFVR_E_INVALID;
    }
    return RFVR_OK;
}

static int check_samples(const rfvr_samples* sm) {
    if (!sm) { set_error("samples descriptor is NULL"); return RFVR_E_INVALID; }
    if (sm->n_ray < 1 || sm->n_z < 1) {
        set_error("n_ray and n_z must be >= 1 (got %d, %d)", sm->n_ray, sm->n_z);
        return RFVR_E_INVALID;
    }
    if (sm->n_ray > RFVR_MAX_RAYS || (int64_t)sm->n_ray * sm->n_z > RFVR_MAX_POINTS) {
        set_error("n_ray <= RFVR_MAX_RAYS and n_ray * n_z <= RFVR_MAX_POINTS are required");
        return RFVR_E_INVALID;
    }
    if (!sm->xyz) { set_error("samples xyz is NULL"); return RFVR_E_INVALID; }
    return RFVR_OK;
}

// the shift of the transmittance needs Phi at the ray origins and at every
// antenna: with a bistatic aperture phi_rx comes with phi_ray and phi_tx
static int check_fields(const rfvr_fields* fl, const rfvr_aperture* ap) {
    if (!fl) { set_error("fields descriptor is NULL"); return RFVR_E_INVALID; }
    if (!fl->sdf || !fl->grad || !fl->refl) { set_error("fields sdf/grad/refl must not be NULL"); return RFVR_E_INVALID; }
    if (!std::isfinite(fl->s) || fl->s <= 0.0f) { set_error("fields s must be finite and > 0"); return RFVR_E_INVALID; }
    if (!std::isfinite(fl->amp_tx)) { set_error("fields amp_tx must be finite"); return RFVR_E_INVALID; }
    if (!ap->rx && fl->phi_rx) { set_error("phi_rx is for bistatic apertures only (rx is NULL)"); return RFVR_E_INVALID; }
    if (ap->rx && (fl->phi_ray && fl->phi_tx) != (fl->phi_rx != nullptr)) {
        set_error("a bistatic aperture takes phi_ray, phi_tx and phi_rx together, or none of them");
        return RFVR_E_INVALID;
    }
    return RFVR_OK;
}

static int check_flags(uint32_t flags) {
    if ((flags & ~(RFVR_SPEC_MASK | RFVR_PHASE_NAIVE32 | RFVR_ACCUMULATE | RFVR_TERMS_DIRECT |
                   RFVR_WEIGHT_SEGMENT)) != 0 ||
        (flags & RFVR_SPEC_MASK) == 3u) {
        set_error("unknown flag bits 0x%x", flags);
        return RFVR_E_INVALID;
    }
    return RFVR_OK;
}

static RenderGeom make_geom(const rfvr_aperture* ap, int n_ray, int n_z) {
    RenderGeom g;
    g.n_meas = ap->n_meas;
    g.n_freq = ap->n_freq;
    g.n_ray = n_ray;
    g.n_z = n_z;
    g.n_pts = (long)n_ray * n_z;
    g.K0 = 2.0 * ap->f0_hz / kSpeedOfLight;
    g.Kd = 2.0 * ap->df_hz / kSpeedOfLight;
    g.seg = 0;
    g.bi = ap->rx ? 1 : 0;
    g.rxa = nullptr;
    return g;
}

static int padded_freq(int n_freq) { return (n_freq + 31) / 32 * 32; }

// the segment weight integrates T'^2 rho of one antenna's shift over a segment;
// the bistatic round trip (T_tx T_rx) has the sample weight only
static int check_bistatic_weight(const RenderGeom& g) {
    if (g.bi && g.seg) {
        set_error("RFVR_WEIGHT_SEGMENT is not defined for bistatic apertures (rx != NULL)");
        return RFVR_E_UNSUPPORTED;
    }
    return RFVR_OK;
}

// transmitter records, and receiver records of a bistatic aperture (g.rxa set
// to them); fl: the fields whose phi_tx / phi_rx shift the transmittance, or
// NULL when the shift is off
static int build_ant_records(const rfvr_aperture* ap, const rfvr_fields* fl, AntRec* ant, AntRec* rxa,
                             RenderGeom& g, hipStream_t st) {
    int rc;
    if ((rc = hip_status(launch_ant_records(ap->tx, fl ? fl->phi_tx : nullptr, ap->n_meas, ant, st),
                         "transmitter records")))
        return rc;
    if (rxa && (rc = hip_status(launch_ant_records(ap->rx, fl ? fl->phi_rx : nullptr, ap->n_meas, rxa, st),
                                "receiver records")))
        return rc;
    g.rxa = rxa;
    return RFVR_OK;
}

static int render_splits(const RenderGeom& g) {
    const int F = freq_chunk(g.n_freq);
    const int n_chunks = (g.n_freq + F - 1) / F;
    return choose_point_splits(g.n_pts, g.n_meas * n_chunks);
}

static int check_ws(void* ws, size_t have, size_t need) {
    if (need > 0 && (!ws || have < need)) {
        set_error("workspace too small: need %zu bytes, got %zu", need, ws ? have : (size_t)0);
        return RFVR_E_WORKSPACE;
    }
    if (ws && (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("workspace must be 256-byte aligned");
        return RFVR_E_WORKSPACE;
    }
    return RFVR_OK;
}

// The term sums go through the Chebyshev-moment kernels unless the caller asks
// for the per-frequency kernels or the FP32-radian phase study; the plan
// (decided on the device per launch) can still fall back to the latter.
static bool use_cheb(uint32_t flags) { return (flags & (RFVR_PHASE_NAIVE32 | RFVR_TERMS_DIRECT)) == 0; }

static size_t ws_cheb(long n_pts, int n_meas) {
    return align256(sizeof(float) * 6 * cheb_bbox_blocks(n_pts)) + align256(sizeof(ChebPlan)) +
           align256(sizeof(MeasCheb) * n_meas);
}

struct ChebWs {
    float* bbox;
    ChebPlan* plan;
    MeasCheb* meas;
};

static ChebWs take_cheb(WsCursor& cur, long n_pts, int n_meas) {
    ChebWs c;
    c.bbox = cur.take<float>((size_t)6 * cheb_bbox_blocks(n_pts));
    c.plan = cur.take<ChebPlan>(1);
    c.meas = cur.take<MeasCheb>(n_meas);
    return c;
}

// split partials of a reduction over points: per-frequency [ns][meas][freq]
// or moments [ns][meas][kChebMaxOrder] (only one of the two runs)
static size_t partial_count(long n_pts, int n_meas, int n_freq, int ns_direct) {
    const size_t d = (size_t)ns_direct * n_meas * n_freq;
    const size_t c = (size_t)cheb_point_splits(n_pts, n_meas) * n_meas * kChebMaxOrder;
    return d > c ? d : c;
}

// ---------------------------------------------------------------- workspace layouts
// antenna records: transmitters, and receivers of a bistatic aperture
static size_t ant_bytes(int n_meas, bool bi) { return (bi ? 2 : 1) * align256(sizeof(AntRec) * n_meas); }

static size_t ws_render_forward(const RenderGeom& g) {
    const int ns = render_splits(g);
    return ant_bytes(g.n_meas, g.bi) + align256(sizeof(PtRec) * g.n_pts) +
           align256(sizeof(float2) * partial_count(g.n_pts, g.n_meas, g.n_freq, ns)) +
           align256(sizeof(float2) * (size_t)g.n_meas * kChebMaxOrder) + ws_cheb(g.n_pts, g.n_meas);
}

static size_t ws_render_backward(const RenderGeom& g) {
    const size_t np = padded_freq(g.n_freq);
    return ant_bytes(g.n_meas, g.bi) + align256(sizeof(PtRec) * g.n_pts) +
           4 * align256(sizeof(float) * g.n_pts) +               // alpha, trans, g_b, g_T
           align256(sizeof(float) * 3 * g.n_pts) +               // g_n
           align256(sizeof(float) * g.n_pts) +                   // g_alpha
           align256(sizeof(float2) * g.n_meas * np) +            // padded g_signal
           2 * align256(sizeof(float) * g.n_ray) +               // per-ray partials
           align256(sizeof(float2) * (size_t)g.n_meas * kChebMaxOrder) + ws_cheb(g.n_pts, g.n_meas);
}

static size_t ws_mf_forward(const rfvr_aperture* ap, long n_q, int two) {
    const size_t np = padded_freq(ap->n_freq);
    return ant_bytes(ap->n_meas, ap->rx != nullptr) +
           (two ? 2 : 1) * (align256(sizeof(float2) * ap->n_meas * np) +
                            align256(sizeof(float2) * (size_t)ap->n_meas * kChebMaxOrder)) +
           ws_cheb(n_q, ap->n_meas);
}

static int mf_splits(const rfvr_aperture* ap, long n_q) {
    const int F = freq_chunk(ap->n_freq);
    return choose_point_splits(n_q, ap->n_meas * ((ap->n_freq + F - 1) / F));
}

static size_t ws_mf_backward(const rfvr_aperture* ap, long n_q) {
    const int ns = mf_splits(ap, n_q);
    return ant_bytes(ap->n_meas, ap->rx != nullptr) + align256(sizeof(QRec) * n_q) +
           align256(sizeof(float2) * partial_count(n_q, ap->n_meas, ap->n_freq, ns)) +
           align256(sizeof(float2) * (size_t)ap->n_meas * kChebMaxOrder) + ws_cheb(n_q, ap->n_meas);
}

static int loss_blocks(long n) {
    long b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

// Scratch of rfvr_mf_forward_static: one library-owned device array per GPU,
// held until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host that name is only a stand-in): its device address is
// looked up once per device and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[RFVR_MF_STATIC_SCRATCH_BYTES];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int static_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index %d beyond the %d devices the static scratch serves", dev, kMaxDevices);
        return RFVR_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u)) {
            set_error("static scratch address %p is not 256-byte aligned", p);
            return RFVR_E_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RFVR_OK;
}

}  // namespace rfvr

using namespace rfvr;

extern "C" {

const char* rfvr_last_error(void) { return g_err; }
int rfvr_version(void) { return 100; }

// ---------------------------------------------------------------- render
size_t rfvr_render_forward_ws_bytes(const rfvr_aperture* ap, const rfvr_samples* sm) {
    if (check_aperture(ap) || check_samples(sm)) return 0;
    return ws_render_forward(make_geom(ap, sm->n_ray, sm->n_z));
}

// element counts of the per-point calls
static bool count_ok(int64_t n) { return n >= 1 && n <= RFVR_MAX_POINTS; }

static int check_count(const char* what, int64_t n) {
    if (!count_ok(n)) {
        set_error("%s must be in [1, RFVR_MAX_POINTS] (got %lld)", what, (long long)n);
        return RFVR_E_INVALID;
    }
    return RFVR_OK;
}

int rfvr_render_forward(const rfvr_aperture* ap, const rfvr_samples* sm, const rfvr_fields* fl,
                        uint32_t flags, float* signal, float* alpha_out, float* trans_out,
                        void* ws, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_aperture(ap)) || (rc = check_samples(sm)) || (rc = check_fields(fl, ap)) ||
        (rc = check_flags(flags)))
        return rc;
    if (!signal) { set_error("signal output is NULL"); return RFVR_E_INVALID; }
    RenderGeom g = make_geom(ap, sm->n_ray, sm->n_z);
    g.seg = (flags & RFVR_WEIGHT_SEGMENT) ? 1 : 0;
    if ((rc = check_bistatic_weight(g))) return rc;
    if ((rc = check_ws(ws, ws_bytes, ws_render_forward(g)))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    WsCursor cur{reinterpret_cast<char*>(ws), 0};
    AntRec* ant = cur.take<AntRec>(g.n_meas);
    AntRec* rxa = g.bi ? cur.take<AntRec>(g.n_meas) : nullptr;
    PtRec* rec = cur.take<PtRec>(g.n_pts);
    const int ns = render_splits(g);
    float2* partial = cur.take<float2>(partial_count(g.n_pts, g.n_meas, g.n_freq, ns));
    float2* M = cur.take<float2>((size_t)g.n_meas * kChebMaxOrder);
    const ChebWs cw = take_cheb(cur, g.n_pts, g.n_meas);
    const int use_phi = (fl->phi_ray && fl->phi_tx) ? 1 : 0;
    if ((rc = build_ant_records(ap, use_phi ? fl : nullptr, ant, rxa, g, st))) return rc;
    if ((rc = hip_status(launch_render_prep(g, sm->xyz, sm->ray_weight, sm->point_weight, fl->sdf, fl->grad, fl->refl,
                                            fl->phi_ray, use_phi, fl->s, fl->log_s_ptr, fl->amp_tx, fl->amp_ptr, rec,
                                            alpha_out, trans_out, st),
                         "render prep")))
        return rc;
    const ChebPlan* sel = nullptr;
    if (use_cheb(flags)) {
        if ((rc = hip_status(launch_cheb_plan(sm->xyz, g.n_pts, ant, g.rxa, g.n_meas, g.Kd, g.n_freq, cw.bbox, cw.meas,
                                              cw.plan, st), "term plan")))
            return rc;
        sel = cw.plan;
        if ((rc = hip_status(launch_cheb_points(g, 0, flags, ant, cw.meas, cw.plan, rec,
                                                cheb_point_splits(g.n_pts, g.n_meas), partial, M,
                                                reinterpret_cast<float2*>(signal), 0, st),
                             "render moment kernels")))
            return rc;
    }
    if ((rc = hip_status(launch_reduce_points_render(g, ant, rec, flags, ns, partial, sel, st),
                         "render term kernel")))
        return rc;
    return hip_status(launch_split_sum(partial, ns, (long)g.n_meas * g.n_freq, 0,
                                       reinterpret_cast<float2*>(signal), sel, st),
                      "render split sum");
}

size_t rfvr_render_backward_ws_bytes(const rfvr_aperture* ap, const rfvr_samples* sm) {
    if (check_aperture(ap) || check_samples(sm)) return 0;
    return ws_render_backward(make_geom(ap, sm->n_ray, sm->n_z));
}

int rfvr_render_backward(const rfvr_aperture* ap, const rfvr_samples* sm, const rfvr_fields* fl,
                         uint32_t flags, const float* g_signal, float* g_sdf, float* g_grad,
                         float* g_refl, float* g_amp, float* g_s, void* ws, size_t ws_bytes,
                         void* stream) {
    int rc;
    if ((rc = check_aperture(ap)) || (rc = check_samples(sm)) || (rc = check_fields(fl, ap)) ||
        (rc = check_flags(flags)))
        return rc;
    if (!g_signal) { set_error("g_signal is NULL"); return RFVR_E_INVALID; }
    if (sm->point_weight) { set_error("point weights are supported by rfvr_render_forward only"); return RFVR_E_UNSUPPORTED; }
    RenderGeom g = make_geom(ap, sm->n_ray, sm->n_z);
    g.seg = (flags & RFVR_WEIGHT_SEGMENT) ? 1 : 0;
    if ((rc = check_bistatic_weight(g))) return rc;
    if ((rc = check_ws(ws, ws_bytes, ws_render_backward(g)))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int acc = (flags & RFVR_ACCUMULATE) ? 1 : 0;
    const int np = padded_freq(g.n_freq);
    WsCursor cur{reinterpret_cast<char*>(ws), 0};
    AntRec* ant = cur.take<AntRec>(g.n_meas);
    AntRec* rxa = g.bi ? cur.take<AntRec>(g.n_meas) : nullptr;
    PtRec* rec = cur.take<PtRec>(g.n_pts);
    float* alpha = cur.take<float>(g.n_pts);
    float* trans = cur.take<float>(g.n_pts);
    float* gb = cur.take<float>(g.n_pts);
    float* gT = cur.take<float>(g.n_pts);
    float* gn = cur.take<float>(3 * (size_t)g.n_pts);
    float* galpha = cur.take<float>(g.n_pts);
    float2* gpad = cur.take<float2>((size_t)g.n_meas * np);
    float* pamp = cur.take<float>(g.n_ray);
    float* ps = cur.take<float>(g.n_ray);
    float2* B = cur.take<float2>((size_t)g.n_meas * kChebMaxOrder);
    const ChebWs cw = take_cheb(cur, g.n_pts, g.n_meas);
    const int use_phi = (fl->phi_ray && fl->phi_tx) ? 1 : 0;
    if ((rc = build_ant_records(ap, use_phi ? fl : nullptr, ant, rxa, g, st))) return rc;
    if ((rc = hip_status(launch_render_prep(g, sm->xyz, sm->ray_weight, nullptr, fl->sdf, fl->grad, fl->refl,
                                            fl->phi_ray, use_phi, fl->s, fl->log_s_ptr, fl->amp_tx, fl->amp_ptr, rec,
                                            alpha, trans, st),
                         "render prep")))
        return rc;
    if ((rc = hip_status(launch_pad_signal(reinterpret_cast<const float2*>(g_signal), g.n_meas,
                                           g.n_freq, np, gpad, st),
                         "pad g_signal")))
        return rc;
    const ChebPlan* sel = nullptr;
    if (use_cheb(flags)) {
        if ((rc = hip_status(launch_cheb_plan(sm->xyz, g.n_pts, ant, g.rxa, g.n_meas, g.Kd, g.n_freq, cw.bbox, cw.meas,
                                              cw.plan, st), "term plan")))
            return rc;
        sel = cw.plan;
        if ((rc = hip_status(launch_cheb_coef(g, cw.plan, cw.meas, reinterpret_cast<const float2*>(g_signal), B,
                                              st), "render adjoint coefficients")))
            return rc;
        if ((rc = hip_status(launch_cheb_render_bwd(g, flags, cw.plan, ant, cw.meas, rec, B, gb, gT, gn, st),
                             "render adjoint series kernels")))
            return rc;
    }
    if ((rc = hip_status(launch_render_bwd_points(g, ant, rec, gpad, np, flags, gb, gT, gn, sel, st),
                         "render adjoint term kernel")))
        return rc;
    if ((rc = hip_status(launch_scan_adjoint(g, sm->ray_weight, fl->sdf, fl->grad, fl->refl, fl->s,
                                             fl->log_s_ptr, fl->amp_tx, fl->amp_ptr, alpha, trans, gb, gT, gn, galpha,
                                             pamp, ps,
                                             g_sdf, g_grad, g_refl, acc, st),
                         "scan adjoint")))
        return rc;
    if (g_amp && (rc = hip_status(launch_sum_scalars(pamp, g.n_ray, g_amp, acc, st), "sum g_amp")))
        return rc;
    if (g_s && (rc = hip_status(launch_sum_scalars(ps, g.n_ray, g_s, acc, st), "sum g_s")))
        return rc;
    return RFVR_OK;
}

// ---------------------------------------------------------------- matched filter
size_t rfvr_mf_forward_ws_bytes(const rfvr_aperture* ap, int64_t n_q, int two_signals) {
    if (check_aperture(ap) || !count_ok(n_q)) return 0;
    return ws_mf_forward(ap, (long)n_q, two_signals);
}

int rfvr_mf_forward(const rfvr_aperture* ap, const float* xyz_q, int64_t n_q, uint32_t flags,
                    const float* signal, float* z, float* power, const float* signal2, float* z2,
                    float* power2, void* ws, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_aperture(ap))) return rc;
    if (flags & ~(uint32_t)(RFVR_PHASE_NAIVE32 | RFVR_TERMS_DIRECT)) {
        set_error("only RFVR_PHASE_NAIVE32 and RFVR_TERMS_DIRECT are meaningful here");
        return RFVR_E_INVALID;
    }
    if (!xyz_q || !signal) { set_error("xyz_q and signal are required"); return RFVR_E_INVALID; }
    if ((rc = check_count("n_q", n_q))) return rc;
    const int two = signal2 ? 1 : 0;
    if ((rc = check_ws(ws, ws_bytes, ws_mf_forward(ap, (long)n_q, two)))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    RenderGeom g = make_geom(ap, 1, 1);
    const int np = padded_freq(ap->n_freq);
    WsCursor cur{reinterpret_cast<char*>(ws), 0};
    AntRec* ant = cur.take<AntRec>(ap->n_meas);
    AntRec* rxa = g.bi ? cur.take<AntRec>(ap->n_meas) : nullptr;
    float2* sp = cur.take<float2>((size_t)ap->n_meas * np);
    float2* sp2 = two ? cur.take<float2>((size_t)ap->n_meas * np) : nullptr;
    float2* B = cur.take<float2>((size_t)ap->n_meas * kChebMaxOrder);
    float2* B2 = two ? cur.take<float2>((size_t)ap->n_meas * kChebMaxOrder) : nullptr;
    const ChebWs cw = take_cheb(cur, (long)n_q, ap->n_meas);
    if ((rc = build_ant_records(ap, nullptr, ant, rxa, g, st))) return rc;
    if ((rc = hip_status(launch_pad_signal(reinterpret_cast<const float2*>(signal), ap->n_meas,
                                           ap->n_freq, np, sp, st), "pad signal")))
        return rc;
    if (two && (rc = hip_status(launch_pad_signal(reinterpret_cast<const float2*>(signal2),
                                                  ap->n_meas, ap->n_freq, np, sp2, st), "pad signal2")))
        return rc;
    const ChebPlan* sel = nullptr;
    if (use_cheb(flags)) {
        if ((rc = hip_status(launch_cheb_plan(xyz_q, (long)n_q, ant, g.rxa, ap->n_meas, g.Kd, ap->n_freq, cw.bbox,
                                              cw.meas, cw.plan, st), "term plan")))
            return rc;
        sel = cw.plan;
        if ((rc = hip_status(launch_cheb_coef(g, cw.plan, cw.meas, reinterpret_cast<const float2*>(signal), B, st),
                             "mf coefficients")))
            return rc;
        if (two && (rc = hip_status(launch_cheb_coef(g, cw.plan, cw.meas, reinterpret_cast<const float2*>(signal2),
                                                     B2, st), "mf coefficients")))
            return rc;
        if ((rc = hip_status(launch_cheb_mf(g, cw.plan, (long)n_q, xyz_q, ant, cw.meas, B, B2,
                                            reinterpret_cast<float2*>(z), power, reinterpret_cast<float2*>(z2),
                                            power2, st), "mf series kernels")))
            return rc;
    }
    return hip_status(launch_mf_forward(g, ant, xyz_q, (long)n_q, sp, sp2, np, flags,
                                        reinterpret_cast<float2*>(z), power,
                                        reinterpret_cast<float2*>(z2), power2, sel, st),
                      "mf forward");
}

int rfvr_mf_forward_static(const rfvr_aperture* ap, const float* xyz_q, int64_t n_q, uint32_t flags,
                           const float* signal, float* z, float* power, const float* signal2, float* z2,
                           float* power2, void* stream) {
    int rc;
    if ((rc = check_aperture(ap))) return rc;
    if ((rc = check_count("n_q", n_q))) return rc;
    const size_t need = ws_mf_forward(ap, (long)n_q, signal2 ? 1 : 0);
    if (need > (size_t)RFVR_MF_STATIC_SCRATCH_BYTES) {
        set_error("rfvr_mf_forward_static: this call needs %zu bytes of scratch, above the static "
                  "RFVR_MF_STATIC_SCRATCH_BYTES = %zu (use rfvr_mf_forward with a workspace)",
                  need, (size_t)RFVR_MF_STATIC_SCRATCH_BYTES);
        return RFVR_E_INVALID;
    }
    void* ws = nullptr;
    if ((rc = static_scratch(&ws))) return rc;
    return rfvr_mf_forward(ap, xyz_q, n_q, flags, signal, z, power, signal2, z2, power2, ws,
                           (size_t)RFVR_MF_STATIC_SCRATCH_BYTES, stream);
}

size_t rfvr_mf_backward_ws_bytes(const rfvr_aperture* ap, int64_t n_q) {
    if (check_aperture(ap) || !count_ok(n_q)) return 0;
    return ws_mf_backward(ap, (long)n_q);
}

int rfvr_mf_backward(const rfvr_aperture* ap, const float* xyz_q, int64_t n_q, const float* z,
                     const float* power, const float* g_power, uint32_t flags, float* g_signal,
                     void* ws, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_aperture(ap)) || (rc = check_flags(flags))) return rc;
    if (!xyz_q || !z || !power || !g_power || !g_signal) {
        set_error("xyz_q, z, power, g_power and g_signal are required");
        return RFVR_E_INVALID;
    }
    if ((rc = check_count("n_q", n_q))) return rc;
    if ((rc = check_ws(ws, ws_bytes, ws_mf_backward(ap, (long)n_q)))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    RenderGeom g = make_geom(ap, 1, 1);
    g.n_pts = (long)n_q;
    const int ns = mf_splits(ap, (long)n_q);
    WsCursor cur{reinterpret_cast<char*>(ws), 0};
    AntRec* ant = cur.take<AntRec>(ap->n_meas);
    AntRec* rxa = g.bi ? cur.take<AntRec>(ap->n_meas) : nullptr;
    QRec* rec = cur.take<QRec>((size_t)n_q);
    float2* partial = cur.take<float2>(partial_count((long)n_q, ap->n_meas, ap->n_freq, ns));
    float2* M = cur.take<float2>((size_t)ap->n_meas * kChebMaxOrder);
    const ChebWs cw = take_cheb(cur, (long)n_q, ap->n_meas);
    const int acc = (flags & RFVR_ACCUMULATE) ? 1 : 0;
    if ((rc = build_ant_records(ap, nullptr, ant, rxa, g, st))) return rc;
    if ((rc = hip_status(launch_mf_bwd_records(xyz_q, (long)n_q, reinterpret_cast<const float2*>(z),
                                               power, g_power, rec, st), "mf adjoint records")))
        return rc;
    const ChebPlan* sel = nullptr;
    if (use_cheb(flags)) {
        if ((rc = hip_status(launch_cheb_plan(xyz_q, (long)n_q, ant, g.rxa, ap->n_meas, g.Kd, ap->n_freq, cw.bbox,
                                              cw.meas, cw.plan, st), "term plan")))
            return rc;
        sel = cw.plan;
        if ((rc = hip_status(launch_cheb_points(g, 1, flags, ant, cw.meas, cw.plan, rec,
                                                cheb_point_splits((long)n_q, ap->n_meas), partial, M,
                                                reinterpret_cast<float2*>(g_signal), acc, st),
                             "mf adjoint moment kernels")))
            return rc;
    }
    if ((rc = hip_status(launch_reduce_points_mf(g, ant, rec, flags, ns, partial, sel, st),
                         "mf adjoint term kernel")))
        return rc;
    return hip_status(launch_split_sum(partial, ns, (long)ap->n_meas * ap->n_freq, acc,
                                       reinterpret_cast<float2*>(g_signal), sel, st),
                      "mf adjoint split sum");
}

// ---------------------------------------------------------------- term evaluation order
size_t rfvr_term_order_ws_bytes(const rfvr_aperture* ap, int64_t n_pts) {
    if (check_aperture(ap) || !count_ok(n_pts)) return 0;
    return ant_bytes(ap->n_meas, ap->rx != nullptr) + ws_cheb((long)n_pts, ap->n_meas);
}

int rfvr_term_order(const rfvr_aperture* ap, const float* xyz, int64_t n_pts, int32_t* order, void* ws,
                    size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_aperture(ap))) return rc;
    if (!xyz || !order) { set_error("xyz and order are required"); return RFVR_E_INVALID; }
    if ((rc = check_count("n_pts", n_pts))) return rc;
    if ((rc = check_ws(ws, ws_bytes, rfvr_term_order_ws_bytes(ap, n_pts)))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    RenderGeom g = make_geom(ap, 1, 1);
    WsCursor cur{reinterpret_cast<char*>(ws), 0};
    AntRec* ant = cur.take<AntRec>(ap->n_meas);
    AntRec* rxa = g.bi ? cur.take<AntRec>(ap->n_meas) : nullptr;
    const ChebWs cw = take_cheb(cur, (long)n_pts, ap->n_meas);
    if ((rc = build_ant_records(ap, nullptr, ant, rxa, g, st))) return rc;
    if ((rc = hip_status(launch_cheb_plan(xyz, (long)n_pts, ant, g.rxa, ap->n_meas, g.Kd, ap->n_freq, cw.bbox, cw.meas,
                                          cw.plan, st), "term plan")))
        return rc;
    return hip_status(launch_cheb_order(cw.plan, order, st), "term order");
}

// ---------------------------------------------------------------- loss
size_t rfvr_loss_ws_bytes(int64_t n) {
    if (!count_ok(n)) return 0;
    return align256(sizeof(double) * loss_blocks((long)n));
}

int rfvr_loss_l2(int64_t n, const float* p, const float* p_star, const float* mask, float* loss,
                 float* g_p, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !p_star || !loss) { set_error("p, p_star and loss are required"); return RFVR_E_INVALID; }
    int rc;
    if ((rc = check_count("n", n))) return rc;
    if ((rc = check_ws(ws, ws_bytes, rfvr_loss_ws_bytes(n)))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nb = loss_blocks((long)n);
    double* part = reinterpret_cast<double*>(ws);
    if ((rc = hip_status(launch_loss_partial((long)n, p, p_star, mask, g_p, part, nb, st), "loss partial")))
        return rc;
    return hip_status(launch_loss_final(part, nb, (long)n, loss, st), "loss final");
}

// ---------------------------------------------------------------- sampling
static int sample_basis(const rfvr_sample_desc* d, double basis[9]) {
    if (d->n_ray_x < 1 || d->n_ray_y < 1 || (int64_t)d->n_ray_x * d->n_ray_y > RFVR_MAX_RAYS) {
        set_error("ray counts must be >= 1 with n_ray_x * n_ray_y <= RFVR_MAX_RAYS");
        return RFVR_E_INVALID;
    }
    if (!(d->half_extent > 0.0f) || !std::isfinite(d->half_extent)) { set_error("half_extent must be finite and > 0"); return RFVR_E_INVALID; }
    if (!std::isfinite(d->plane_offset)) { set_error("plane_offset must be finite"); return RFVR_E_INVALID; }
    double w[3] = {d->primary_dir[0], d->primary_dir[1], d->primary_dir[2]};
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(w[c]) || !std::isfinite((double)d->centre[c])) { set_error("non-finite direction or centre"); return RFVR_E_INVALID; }
    double nw = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (!(nw > 0.0)) { set_error("primary_dir must be non-zero"); return RFVR_E_INVALID; }
    for (int c = 0; c < 3; ++c) w[c] /= nw;
    double ref[3] = {0.0, 1.0, 0.0};
    if (std::fabs(w[1]) >= 0.9) { ref[0] = 1.0; ref[1] = 0.0; }
    double e1[3] = {ref[1] * w[2] - ref[2] * w[1], ref[2] * w[0] - ref[0] * w[2], ref[0] * w[1] - ref[1] * w[0]};
    double n1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int c = 0; c < 3; ++c) e1[c] /= n1;
    double e2[3] = {w[1] * e1[2] - w[2] * e1[1], w[2] * e1[0] - w[0] * e1[2], w[0] * e1[1] - w[1] * e1[0]};
    const double b[9] = {e1[0], e1[1], e1[2], e2[0], e2[1], e2[2], w[0], w[1], w[2]};
    for (int k = 0; k < 9; ++k) basis[k] = b[k];
    return RFVR_OK;
}

int rfvr_sample_points(const rfvr_sample_desc* d, float* xyz, float* u, float* ray_origin,
                       void* stream) {
    if (!d || !xyz) { set_error("descriptor and xyz are required"); return RFVR_E_INVALID; }
    if (d->n_z < 1 || (int64_t)d->n_ray_x * d->n_ray_y * d->n_z > RFVR_MAX_POINTS) {
        set_error("n_z must be >= 1 and rays * n_z <= RFVR_MAX_POINTS");
        return RFVR_E_INVALID;
    }
    if (d->mode != RFVR_SAMPLE_GRID && d->mode != RFVR_SAMPLE_STRATIFIED) { set_error("unknown sampling mode %d", d->mode); return RFVR_E_INVALID; }
    double basis[9];
    int rc;
    if ((rc = sample_basis(d, basis))) return rc;
    return hip_status(launch_sample_points(*d, basis, xyz, u, ray_origin,
                                           reinterpret_cast<hipStream_t>(stream)),
                      "sample points");
}

int rfvr_sample_naive(const rfvr_sample_desc* d, const float* tx, int32_t n_ant, float* xyz, float* jac,
                      void* stream) {
    if (!d || !tx || !xyz || n_ant < 1 || n_ant > RFVR_MAX_MEAS) {
        set_error("descriptor, tx, xyz and n_ant in [1, RFVR_MAX_MEAS] are required");
        return RFVR_E_INVALID;
    }
    if (d->n_z < 1) { set_error("n_z must be >= 1"); return RFVR_E_INVALID; }
    double basis[9];
    int rc;
    if ((rc = sample_basis(d, basis))) return rc;
    if ((int64_t)n_ant * d->n_ray_x * d->n_ray_y * d->n_z > RFVR_MAX_POINTS) {
        set_error("n_ant * rays * n_z must not exceed RFVR_MAX_POINTS");
        return RFVR_E_INVALID;
    }
    return hip_status(launch_sample_naive(*d, basis, tx, n_ant, xyz, jac, reinterpret_cast<hipStream_t>(stream)),
                      "naive sampling");
}

int rfvr_sample_importance(const rfvr_sample_desc* d, const float* logits, int32_t n_bins,
                           int32_t n_imp, int32_t n_uni, float* xyz, float* u, float* ray_origin,
                           void* stream) {
    if (!d || !xyz || !logits) { set_error("descriptor, logits and xyz are required"); return RFVR_E_INVALID; }
    if (n_bins < 1 || n_bins > 64 || n_imp < 0 || n_uni < 0 || n_imp > RFVR_MAX_RAY_SAMPLES ||
        n_uni > RFVR_MAX_RAY_SAMPLES || n_imp + n_uni < 1 || n_imp + n_uni > RFVR_MAX_RAY_SAMPLES) {
        set_error("need 1 <= n_bins <= 64 and 1 <= n_imp + n_uni <= RFVR_MAX_RAY_SAMPLES (1024)");
        return RFVR_E_INVALID;
    }
    if (d->mode != RFVR_SAMPLE_GRID && d->mode != RFVR_SAMPLE_STRATIFIED) {
        set_error("mode must be RFVR_SAMPLE_GRID (levels at the middle of their strata) or RFVR_SAMPLE_STRATIFIED");
        return RFVR_E_INVALID;
    }
    double basis[9];
    int rc;
    if ((rc = sample_basis(d, basis))) return rc;
    if ((int64_t)d->n_ray_x * d->n_ray_y * (n_imp + n_uni) > RFVR_MAX_POINTS) {
        set_error("rays * (n_imp + n_uni) must not exceed RFVR_MAX_POINTS");
        return RFVR_E_INVALID;
    }
    return hip_status(launch_sample_importance(*d, basis, logits, n_bins, n_imp, n_uni, xyz, u, ray_origin,
                                               reinterpret_cast<hipStream_t>(stream)),
                      "importance sampling");
}

int rfvr_proposal_targets(int32_t n_ray, int32_t n_k, const float* u, const float* alpha,
                          const float* trans, float lo, float hi, int32_t n_bins, int32_t n_dilate,
                          float* targets, void* stream) {
    if (n_ray < 1 || n_ray > RFVR_MAX_RAYS || n_k < 1 || n_k > RFVR_MAX_RAY_SAMPLES || n_bins < 1 || n_bins > 64 ||
        n_dilate < 0 || n_dilate >= n_bins || !u || !alpha || !trans || !targets) {
        set_error("need 1 <= n_ray <= RFVR_MAX_RAYS, 1 <= n_k <= RFVR_MAX_RAY_SAMPLES (1024), 1 <= n_bins <= 64, "
                  "0 <= n_dilate < n_bins and all arrays");
        return RFVR_E_INVALID;
    }
    if (!(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi)) { set_error("need finite lo < hi"); return RFVR_E_INVALID; }
    return hip_status(launch_proposal_targets(n_ray, n_k, u, alpha, trans, lo, hi, n_bins, n_dilate, targets,
                                              reinterpret_cast<hipStream_t>(stream)),
                      "proposal targets");
}

size_t rfvr_bce_ws_bytes(int64_t n) { return rfvr_loss_ws_bytes(n); }

size_t rfvr_mask_ws_bytes(int64_t n) {
    if (!count_ok(n)) return 0;
    return align256(sizeof(float) * (loss_blocks((long)n) + 1));
}

int rfvr_mask_update(int64_t n, const float* power, const float* power_ref, float* history, float tau_hi,
                     float tau_lo, float* mask, void* ws, size_t ws_bytes, void* stream) {
    if (!power || !power_ref || !history || !mask) {
        set_error("power, power_ref, history and mask are required");
        return RFVR_E_INVALID;
    }
    if (!count_ok(n)) { set_error("n must be in [1, RFVR_MAX_POINTS]"); return RFVR_E_INVALID; }
    if (!std::isfinite(tau_hi) || !std::isfinite(tau_lo) || tau_hi < 0.0f || tau_lo < 0.0f) {
        set_error("tau_hi and tau_lo must be finite and >= 0");
        return RFVR_E_INVALID;
    }
    int rc;
    if ((rc = check_ws(ws, ws_bytes, rfvr_mask_ws_bytes(n)))) return rc;
    const int nb = loss_blocks((long)n);
    return hip_status(launch_mask_update((long)n, power, power_ref, history, tau_hi, tau_lo, mask,
                                         reinterpret_cast<float*>(ws), nb, reinterpret_cast<hipStream_t>(stream)),
                      "mask update");
}

int rfvr_bce(int64_t n, const float* logits, const float* t, float* loss, float* g_logits,
             void* ws, size_t ws_bytes, void* stream) {
    if (!logits || !t || !loss) { set_error("logits, t and loss are required"); return RFVR_E_INVALID; }
    int rc;
    if ((rc = check_count("n", n))) return rc;
    if ((rc = check_ws(ws, ws_bytes, rfvr_bce_ws_bytes(n)))) return rc;
    const int nb = loss_blocks((long)n);
    return hip_status(launch_bce((long)n, logits, t, loss, g_logits, reinterpret_cast<double*>(ws), nb,
                                 reinterpret_cast<hipStream_t>(stream)),
                      "bce");
}

// ---------------------------------------------------------------- occupancy
int rfvr_occupancy(int64_t n, float s, const float* sdf, float* phi, void* stream) {
    if (!sdf || !phi) { set_error("sdf and phi are required"); return RFVR_E_INVALID; }
    if (!count_ok(n)) { set_error("n must be in [1, RFVR_MAX_POINTS]"); return RFVR_E_INVALID; }
    if (!std::isfinite(s) || s <= 0.0f) { set_error("s must be finite and > 0"); return RFVR_E_INVALID; }
    return hip_status(launch_occupancy((long)n, s, nullptr, sdf, phi, reinterpret_cast<hipStream_t>(stream)),
                      "occupancy");
}

int rfvr_occupancy_logs(int64_t n, const float* log_s, const float* sdf, float* phi, void* stream) {
    if (!sdf || !phi || !log_s) { set_error("log_s, sdf and phi are required"); return RFVR_E_INVALID; }
    if (!count_ok(n)) { set_error("n must be in [1, RFVR_MAX_POINTS]"); return RFVR_E_INVALID; }
    return hip_status(launch_occupancy((long)n, 1.0f, log_s, sdf, phi, reinterpret_cast<hipStream_t>(stream)),
                      "occupancy");
}

// ---------------------------------------------------------------- AdamW
int rfvr_adamw(int64_t n, float* p, const float* g, float* m, float* v, int64_t t, float lr,
               float b1, float b2, float eps, float wd, void* stream) {
    if (!count_ok(n) || !p || !g || !m || !v || t < 1) {
        set_error("n in [1, RFVR_MAX_POINTS], t >= 1 and all arrays are required");
        return RFVR_E_INVALID;
    }
    if (!std::isfinite(lr) || !std::isfinite(b1) || !std::isfinite(b2) || !std::isfinite(eps) || !std::isfinite(wd) ||
        b1 < 0.0f || b1 >= 1.0f || b2 < 0.0f || b2 >= 1.0f) {
        set_error("invalid AdamW hyper-parameters");
        return RFVR_E_INVALID;
    }
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)t));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)t));
    return hip_status(launch_adamw((long)n, p, g, m, v, lr, b1, b2, eps, wd, bc1, bc2,
                                   reinterpret_cast<hipStream_t>(stream)),
                      "adamw");
}

// ---------------------------------------------------------------- several scenes per call
// Each scene runs through the single-scene entry point, in scene order on the
// stream, with the packed arrays offset per scene.  Every scene's descriptors
// are checked first as the single-scene call checks them, and the arguments
// shared by all scenes fail on the first scene, so an invalid call enqueues
// nothing; only a HIP runtime error can stop the loop after earlier scenes.
static int scene_error(int s, int rc) {
    char msg[480];
    snprintf(msg, sizeof msg, "%s", rfvr_last_error());
    set_error("scene %d: %s", s, msg);
    return rc;
}

// what each single-scene call checks of its descriptors, for every scene
enum SceneCall { SC_RENDER_FWD, SC_RENDER_BWD, SC_FILTER };
static int check_scenes(int32_t n, const rfvr_scene* sc, SceneCall call) {
    if (n < 1 || !sc) { set_error("n_scenes must be >= 1 and scenes non-NULL"); return RFVR_E_INVALID; }
    for (int s = 0; s < n; ++s) {
        int rc;
        if ((rc = check_aperture(&sc[s].ap)) || (rc = check_samples(&sc[s].sm)) ||
            (call != SC_FILTER && (rc = check_fields(&sc[s].fl, &sc[s].ap))))
            return scene_error(s, rc);
        if (call == SC_RENDER_BWD && sc[s].sm.point_weight) {
            set_error("scene %d: point weights are supported by rfvr_render_forward only", s);
            return RFVR_E_UNSUPPORTED;
        }
    }
    return RFVR_OK;
}

static size_t scene_signal(const rfvr_scene& s) { return 2 * (size_t)s.ap.n_meas * s.ap.n_freq; }
static size_t scene_points(const rfvr_scene& s) { return (size_t)s.sm.n_ray * s.sm.n_z; }
extern "C++" {
template <class T> static T* at(T* p, size_t off) { return p ? p + off : nullptr; }
}

size_t rfvr_render_forward_batched_ws_bytes(int32_t n, const rfvr_scene* sc) {
    size_t m = 0;
    for (int s = 0; sc && s < n; ++s) m = std::max(m, rfvr_render_forward_ws_bytes(&sc[s].ap, &sc[s].sm));
    return m;
}

int rfvr_render_forward_batched(int32_t n, const rfvr_scene* sc, uint32_t flags, float* signal,
                                float* alpha_out, float* trans_out, void* ws, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_scenes(n, sc, SC_RENDER_FWD)) || (rc = check_flags(flags))) return rc;
    if (!signal) { set_error("signal output is NULL"); return RFVR_E_INVALID; }
    if ((rc = check_ws(ws, ws_bytes, rfvr_render_forward_batched_ws_bytes(n, sc)))) return rc;
    size_t so = 0, po = 0;
    for (int s = 0; s < n; ++s) {
        if ((rc = rfvr_render_forward(&sc[s].ap, &sc[s].sm, &sc[s].fl, flags, signal + so, at(alpha_out, po),
                                      at(trans_out, po), ws, ws_bytes, stream)))
            return scene_error(s, rc);
        so += scene_signal(sc[s]);
        po += scene_points(sc[s]);
    }
    return RFVR_OK;
}

size_t rfvr_render_backward_batched_ws_bytes(int32_t n, const rfvr_scene* sc) {
    size_t m = 0;
    for (int s = 0; sc && s < n; ++s) m = std::max(m, rfvr_render_backward_ws_bytes(&sc[s].ap, &sc[s].sm));
    return m;
}

int rfvr_render_backward_batched(int32_t n, const rfvr_scene* sc, uint32_t flags, const float* g_signal,
                                 float* g_sdf, float* g_grad, float* g_refl, float* g_amp, float* g_s,
                                 void* ws, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_scenes(n, sc, SC_RENDER_BWD)) || (rc = check_flags(flags))) return rc;
    if (!g_signal) { set_error("g_signal is NULL"); return RFVR_E_INVALID; }
    if ((rc = check_ws(ws, ws_bytes, rfvr_render_backward_batched_ws_bytes(n, sc)))) return rc;
    size_t so = 0, po = 0;
    for (int s = 0; s < n; ++s) {
        if ((rc = rfvr_render_backward(&sc[s].ap, &sc[s].sm, &sc[s].fl, flags, g_signal + so, at(g_sdf, po),
                                       at(g_grad, 3 * po), at(g_refl, po), at(g_amp, (size_t)s), at(g_s, (size_t)s),
                                       ws, ws_bytes, stream)))
            return scene_error(s, rc);
        so += scene_signal(sc[s]);
        po += scene_points(sc[s]);
    }
    return RFVR_OK;
}

size_t rfvr_mf_forward_batched_ws_bytes(int32_t n, const rfvr_scene* sc, int two_signals) {
    size_t m = 0;
    for (int s = 0; sc && s < n; ++s)
        m = std::max(m, rfvr_mf_forward_ws_bytes(&sc[s].ap, (int64_t)scene_points(sc[s]), two_signals));
    return m;
}

int rfvr_mf_forward_batched(int32_t n, const rfvr_scene* sc, uint32_t flags, const float* signal, float* z,
                            float* power, const float* signal2, float* z2, float* power2, void* ws,
                            size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_scenes(n, sc, SC_FILTER))) return rc;
    if (!signal) { set_error("signal is NULL"); return RFVR_E_INVALID; }
    if ((rc = check_ws(ws, ws_bytes, rfvr_mf_forward_batched_ws_bytes(n, sc, signal2 ? 1 : 0)))) return rc;
    size_t so = 0, po = 0;
    for (int s = 0; s < n; ++s) {
        if ((rc = rfvr_mf_forward(&sc[s].ap, sc[s].sm.xyz, (int64_t)scene_points(sc[s]), flags, signal + so,
                                  at(z, 2 * po), at(power, po), at(signal2, so), at(z2, 2 * po), at(power2, po),
                                  ws, ws_bytes, stream)))
            return scene_error(s, rc);
        so += scene_signal(sc[s]);
        po += scene_points(sc[s]);
    }
    return RFVR_OK;
}

size_t rfvr_mf_backward_batched_ws_bytes(int32_t n, const rfvr_scene* sc) {
    size_t m = 0;
    for (int s = 0; sc && s < n; ++s)
        m = std::max(m, rfvr_mf_backward_ws_bytes(&sc[s].ap, (int64_t)scene_points(sc[s])));
    return m;
}

int rfvr_mf_backward_batched(int32_t n, const rfvr_scene* sc, const float* z, const float* power,
                             const float* g_power, uint32_t flags, float* g_signal, void* ws, size_t ws_bytes,
                             void* stream) {
    int rc;
    if ((rc = check_scenes(n, sc, SC_FILTER))) return rc;
    if (!z || !power || !g_power || !g_signal) {
        set_error("z, power, g_power and g_signal are required");
        return RFVR_E_INVALID;
    }
    if ((rc = check_ws(ws, ws_bytes, rfvr_mf_backward_batched_ws_bytes(n, sc)))) return rc;
    size_t so = 0, po = 0;
    for (int s = 0; s < n; ++s) {
        if ((rc = rfvr_mf_backward(&sc[s].ap, sc[s].sm.xyz, (int64_t)scene_points(sc[s]), z + 2 * po, power + po,
                                   g_power + po, flags, g_signal + so, ws, ws_bytes, stream)))
            return scene_error(s, rc);
        so += scene_signal(sc[s]);
        po += scene_points(sc[s]);
    }
    return RFVR_OK;
}

// ---------------------------------------------------------------- several networks per call
static int check_nets(int32_t n, const rfvr_mlp* nets, const int64_t* cnt) {
    if (n < 1 || !nets || !cnt) { set_error("n_nets must be >= 1, nets and n non-NULL"); return RFVR_E_INVALID; }
    for (int s = 0; s < n; ++s) {
        if (rfvr_mlp_param_count(&nets[s]) < 0) return scene_error(s, RFVR_E_INVALID);
        if (!count_ok(cnt[s]) || !nets[s].params) {
            set_error("net %d: n in [1, RFVR_MAX_POINTS] and params are required", s);
            return RFVR_E_INVALID;
        }
    }
    return RFVR_OK;
}

size_t rfvr_mlp_forward_grouped_ws_bytes(int32_t n, const rfvr_mlp* nets, const int64_t* cnt) {
    size_t m = 0;
    for (int s = 0; nets && cnt && s < n; ++s) m = std::max(m, rfvr_mlp_forward_ws_bytes(&nets[s], cnt[s]));
    return m;
}

int rfvr_mlp_forward_grouped(int32_t n, const rfvr_mlp* nets, const float* xyz, const int64_t* cnt, float* sdf,
                             float* grad, float* refl, void* ws, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_nets(n, nets, cnt))) return rc;
    if (!xyz) { set_error("xyz is NULL"); return RFVR_E_INVALID; }
    if ((rc = check_ws(ws, ws_bytes, rfvr_mlp_forward_grouped_ws_bytes(n, nets, cnt)))) return rc;
    size_t po = 0;
    for (int s = 0; s < n; ++s) {
        if ((rc = rfvr_mlp_forward(&nets[s], xyz + 3 * po, cnt[s], at(sdf, po), at(grad, 3 * po), at(refl, po), ws,
                                   ws_bytes, stream)))
            return scene_error(s, rc);
        po += (size_t)cnt[s];
    }
    return RFVR_OK;
}

size_t rfvr_mlp_backward_grouped_ws_bytes(int32_t n, const rfvr_mlp* nets, const int64_t* cnt) {
    size_t m = 0;
    for (int s = 0; nets && cnt && s < n; ++s) m = std::max(m, rfvr_mlp_backward_ws_bytes(&nets[s], cnt[s]));
    return m;
}

int rfvr_mlp_backward_grouped(int32_t n, const rfvr_mlp* nets, const float* xyz, const int64_t* cnt,
                              const float* g_sdf, const float* g_grad, const float* g_refl, uint32_t flags,
                              float* g_params, void* ws, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_nets(n, nets, cnt))) return rc;
    if (!xyz || !g_params) { set_error("xyz and g_params are required"); return RFVR_E_INVALID; }
    if (flags & ~(uint32_t)RFVR_ACCUMULATE) { set_error("only RFVR_ACCUMULATE is meaningful here"); return RFVR_E_INVALID; }
    if ((rc = check_ws(ws, ws_bytes, rfvr_mlp_backward_grouped_ws_bytes(n, nets, cnt)))) return rc;
    size_t po = 0, go = 0;
    for (int s = 0; s < n; ++s) {
        if ((rc = rfvr_mlp_backward(&nets[s], xyz + 3 * po, cnt[s], at(g_sdf, po), at(g_grad, 3 * po),
                                    at(g_refl, po), flags, g_params + go, ws, ws_bytes, stream)))
            return scene_error(s, rc);
        po += (size_t)cnt[s];
        go += (size_t)rfvr_mlp_param_count(&nets[s]);
    }
    return RFVR_OK;
}

}  // extern "C"
