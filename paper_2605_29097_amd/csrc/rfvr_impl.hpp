// Internal declarations of librfvr (not part of the C ABI).
//
// Device-side conventions shared by the term kernels:
//  * complex values are float2 {re, im};
//  * phases are handled in revolutions: the term for (pair, frequency n) is
//    exp(-+ j 2 pi (theta0 + n * delta)) with theta0 = f0 * d / c and
//    delta = df * d / c, d the round-trip path length;
//  * the default phase mode forms d and the fractional part of theta0 in
//    FP64 (the only step whose conditioning needs it) and runs everything else
//    in FP32, with the hardware sin/cos that take revolutions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/rfvr.h"

namespace rfvr {

constexpr double kSpeedOfLight = 299792458.0;
constexpr float kAlphaEps = 1e-5f;

// Per-point record consumed by the render kernels (48 bytes).  With the
// sample weight (default):
//   x    = the sample point
//   b    = A' * w_r * a * alpha      (amplitude without the per-pair factors)
//   tp   = T - Phi(primary-ray origin)  (lensless transmittance before the per-
//          antenna shift; equals T when the correction is off)
//   sq   = 1: the pair's factor is the square of the shifted value T'
// With the segment weight (RFVR_WEIGHT_SEGMENT):
//   x    = the midpoint of the sample and the next one on its ray
//   b    = A' * w_r * a * alpha * T,  tp = T (1 - alpha/2) - Phi(origin)
//   sq   = 0: the pair's factor is the shifted value itself
struct alignas(16) PtRec {
    double x, y, z;
    float b, tp, nx, ny, nz, sq;
};
static_assert(sizeof(PtRec) == 48, "PtRec layout");

// Per-query record of the matched-filter adjoint: h = g_P * z / P.
struct alignas(16) QRec {
    double x, y, z;
    float hr, hi;
};
static_assert(sizeof(QRec) == 32, "QRec layout");

// Per-measurement record (positions in FP64 so the path length is exact in the
// inputs; phi = Phi_s at the antenna, 0 when the correction is off).  A
// bistatic launch holds one array for the transmitters and one for the
// receivers.
struct alignas(16) AntRec {
    double x, y, z;
    float phi, pad;
};
static_assert(sizeof(AntRec) == 32, "AntRec layout");

// ----------------------------------------------------------------------------
// device helpers
// ----------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__)
#define RFVR_DEV __device__ __forceinline__
#else
#define RFVR_DEV __host__ __device__ inline
#endif

// |d| in FP64 from an FP32 reciprocal square root and one Newton step
// (relative error ~1e-14); also returns y ~ 1/|d| in FP32.
__device__ __forceinline__ double range_f64(double dx, double dy, double dz, float& y) {
    double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    y = __builtin_amdgcn_rsqf((float)r2);
    double yd = (double)y;
    double r0 = r2 * yd;
    double e = __builtin_fma(-r0, r0, r2);
    return __builtin_fma(e, 0.5 * yd, r0);
}

// fractional part in [0, 1) of an FP64 value, returned in FP32
__device__ __forceinline__ float frac_rev(double t) {
    return (float)__builtin_amdgcn_fract(t);
}

// cos / sin of 2*pi*x for x in revolutions (|x| < 256)
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

// Opacity between consecutive samples with logits a = s f_k, b = s f_{k+1}:
// clamp((Phi(a) - Phi(b)) / (Phi(a) + eps), 0, 1).  The difference is formed
// as Phi(b) (1 - Phi(a)) expm1(a - b), an exact identity of the logistic CDF
// that avoids cancellation when both samples are far outside the surface.
__device__ __forceinline__ float alpha_pair(float a, float b) {
    if (!(a >= b)) return 0.0f;
    float diff = sigmoidf_(b) * sigmoidf_(-a) * expm1f(a - b);
    float al = diff / (sigmoidf_(a) + kAlphaEps);
    return fminf(al, 1.0f);
}

// the specular factor from its raw value w_o . w_r: clamped at 0 (CLAMP), raw
// (RAW) or 1 (OFF); live = 1 where it is not clamped
template <int SPEC>
__device__ __forceinline__ void spec_clamp(float sr, float& spec, float& live) {
    if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
        spec = 1.0f;
        live = 0.0f;
    } else if constexpr (SPEC == (int)RFVR_SPEC_RAW) {
        spec = sr;
        live = 1.0f;
    } else {
        spec = fmaxf(sr, 0.0f);
        live = sr >= 0.0f ? 1.0f : 0.0f;
    }
}

// monostatic pair (w_r = -w_i), from nd = n_hat . w_i: w_o . w_r = 2 nd^2 - 1
template <int SPEC>
__device__ __forceinline__ void spec_factor(float nd, float& spec, float& live) {
    if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
        spec_clamp<SPEC>(0.0f, spec, live);
    } else {
        spec_clamp<SPEC>(__builtin_fmaf(2.0f * nd, nd, -1.0f), spec, live);
    }
}

// bistatic pair, from ni = n_hat . w_i, nr = n_hat . w_r and ir = w_i . w_r
// (w_i from the transmitter to the point, w_r from the point to the receiver):
// w_o = w_i - 2 ni n_hat, so w_o . w_r = ir - 2 ni nr (App. A, Radar
// Reflections); its gradient in n_hat is -2 (nr w_i + ni w_r)
template <int SPEC>
__device__ __forceinline__ void spec_factor_bi(float ni, float nr, float ir, float& spec, float& live) {
    spec_clamp<SPEC>(__builtin_fmaf(-2.0f * ni, nr, ir), spec, live);
}

// ---------------------------------------------------------------------------
// pair phase set-up
// ---------------------------------------------------------------------------
// A pair's frequencies are visited by a recurrence in the step phasor
// w = exp(-+ j 2 pi delta).  Rounding of w grows linearly along a walk and the
// rendered signal is a heavily cancelling sum (Fresnel zones), so:
//  * w comes from a correctly rounded sin/cos (cos_sin_rev_cr32);
//  * walks are short: every S frequencies the phasor is re-seeded from an
//    FP64-reduced phase at the centre of the sub-chunk and walked S/2 steps
//    up and S/2 steps down.
// Re-seed phasors use the hardware sin/cos (errors do not accumulate).
struct PairGeom {
    double r;   // |x - tx| (FP64)
    float y;    // ~1/r
    float rf;   // r in FP32 (NAIVE mode)
};

template <bool NAIVE>
__device__ __forceinline__ PairGeom pair_geom(double dx, double dy, double dz);

// Bistatic pair: d_t = x - tx, d_r = x - rx.  The phase and the range band run
// on the mean range r = (r_t + r_r) / 2, whose doubled value is the path
// length, as 2 |x - tx| is for a monostatic pair; the amplitude takes
// y_t y_r ~ 1 / (r_t r_r).
struct BiGeom {
    PairGeom g;   // g.r (g.rf in NAIVE mode) = (r_t + r_r) / 2; g.y unused
    float yt, yr; // ~1/r_t, ~1/r_r
};

template <bool NAIVE>
__device__ __forceinline__ BiGeom bi_geom(double tx_, double ty_, double tz_, double rx_, double ry_, double rz_) {
    const PairGeom a = pair_geom<NAIVE>(tx_, ty_, tz_), b = pair_geom<NAIVE>(rx_, ry_, rz_);
    BiGeom o;
    o.g.r = 0.5 * (a.r + b.r);
    o.g.rf = 0.5f * (a.rf + b.rf);
    o.g.y = 0.0f;
    o.yt = a.y;
    o.yr = b.y;
    return o;
}

template <bool NAIVE>
__device__ __forceinline__ PairGeom pair_geom(double dx, double dy, double dz) {
    PairGeom g;
    if constexpr (!NAIVE) {
        g.r = range_f64(dx, dy, dz, g.y);
        g.rf = 0.0f;
    } else {
        const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
        g.rf = sqrtf(fx * fx + fy * fy + fz * fz);
        g.y = 1.0f / g.rf;
        g.r = 0.0;
    }
    return g;
}

// cos/sin of 2 pi * (K * r): FP64 product and reduction, hardware sin/cos;
// NAIVE: FP32 radians (2 pi K) * r and library sin/cos.
template <bool NAIVE>
__device__ __forceinline__ void seed_phasor(const PairGeom& g, double K, float& c, float& s) {
    if constexpr (!NAIVE) {
        const float t = frac_rev(g.r * K);
        c = cos_rev(t);
        s = sin_rev(t);
    } else {
        sincosf((float)(6.283185307179586 * K) * g.rf, &s, &c);
    }
}

// ---------------------------------------------------------------------------
// correctly rounded cos / sin of 2 pi d for an FP64 phase d (revolutions):
// d mod 1 = k / 1024 + e with |e| <= 1/2048; cos/sin(2 pi k / 1024) from a
// table and cos/sin(2 pi e) from their Taylor series (|2 pi e| <= pi / 1024),
// combined by the angle-sum identities.  The table is built at compile time in
// FP64 from the Taylor series of cos and sin on the first octant and the
// 45-degree rotation.
// ---------------------------------------------------------------------------
namespace phase_table {
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double taylor_sin(double x) {
    double t = x, s = x;
    for (int n = 1; n < 14; ++n) { t *= -x * x / ((2 * n) * (2 * n + 1)); s += t; }
    return s;
}
constexpr double taylor_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int n = 1; n < 14; ++n) { t *= -x * x / ((2 * n - 1) * (2 * n)); s += t; }
    return s;
}
struct Table {
    double v[2 * 1024];
    constexpr Table() : v() {
        const double h = 0.70710678118654752440084436210484903928;   // cos 45 deg
        for (int k = 0; k < 1024; ++k) {
            const int q = (k * 8) / 1024;                                // octant
            const double a = 2.0 * kPi * ((double)k / 1024.0 - q / 8.0);  // [0, pi/4)
            double c = taylor_cos(a), s = taylor_sin(a);
            for (int i = 0; i < q; ++i) {
                const double nc = h * (c - s), ns = h * (c + s);
                c = nc;
                s = ns;
            }
            v[2 * k] = c;
            v[2 * k + 1] = s;
        }
    }
};
}  // namespace phase_table
// The same table split into FP32 hi/lo parts (c_hi, c_lo, s_hi, s_lo): with
// x = 2 pi e, cos(a + x) = cos a + [cos a (cos x - 1) - sin a sin x] (and the
// sine alike).  The bracket is below 3.2e-3 in magnitude, so FP32 evaluates it
// to ~4e-10 and the final addition rounds once: cos/sin within 3.1e-8
// absolute (half an ulp of values near 1), with five FP64 operations (the
// reduction of d).
struct TableHiLo {
    float v[4 * 1024];
    constexpr TableHiLo() : v() {
        const phase_table::Table t{};
        for (int k = 0; k < 1024; ++k) {
            const double c = t.v[2 * k], s = t.v[2 * k + 1];
            const float ch = (float)c, sh = (float)s;
            v[4 * k] = ch;
            v[4 * k + 1] = (float)(c - (double)ch);
            v[4 * k + 2] = sh;
            v[4 * k + 3] = (float)(s - (double)sh);
        }
    }
};
__device__ constexpr TableHiLo kPhaseTableHiLo{};

__device__ __forceinline__ void cos_sin_rev_cr32(double d, float& c, float& s) {
    const double dr = __builtin_amdgcn_fract(d) * 1024.0;
    const double kf = __builtin_rint(dr);
    const int k = (int)kf & 1023;
    const float x = (float)((dr - kf) * (6.283185307179586476925 / 1024.0));   // |x| <= pi/1024
    const float x2 = x * x;
    const float cm = x2 * __builtin_fmaf(x2, 1.0f / 24.0f, -0.5f);             // cos x - 1
    const float sx = __builtin_fmaf(x * x2, __builtin_fmaf(x2, 1.0f / 120.0f, -1.0f / 6.0f), x);
    const float4 t = *reinterpret_cast<const float4*>(&kPhaseTableHiLo.v[4 * k]);
    c = t.x + __builtin_fmaf(t.x, cm, __builtin_fmaf(-t.z, sx, t.y));
    s = t.z + __builtin_fmaf(t.z, cm, __builtin_fmaf(t.x, sx, t.w));
}

// correctly rounded step phasor cos/sin of 2 pi * (Kd * r); the point
// reductions' three-term recurrence amplifies the rounding of cos by
// 1 / sin(2 pi delta), so it needs that accuracy
template <bool NAIVE>
__device__ __forceinline__ void step_phasor(const PairGeom& g, double Kd, float& c, float& s) {
    if constexpr (!NAIVE) {
        cos_sin_rev_cr32(g.r * Kd, c, s);
    } else {
        sincosf((float)(6.283185307179586 * Kd) * g.rf, &s, &c);
    }
}

// ----------------------------------------------------------------------------
// host-side internals shared between translation units
// ----------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int hip_status(hipError_t e, const char* what);

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bump allocator over the caller's workspace.
struct WsCursor {
    char* base;
    size_t used;
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + used);
        used += align256(count * sizeof(T));
        return p;
    }
};

// Chebyshev-moment evaluation of the term sums (cheb.hip): per-measurement
// range interval [rc - h, rc + h] of a launch and the chosen order K (0: the
// per-frequency kernels run instead).
struct alignas(16) MeasCheb {
    double rc, h, inv_h, pad;
};
struct alignas(16) ChebPlan {
    int K, pad;
    double zmax;
};

// Launchers (render.hip)
struct RenderGeom {
    int n_meas, n_freq, n_ray, n_z;
    long n_pts;
    double K0, Kd;        // 2 f0 / c and 2 df / c (revolutions per metre of range)
    int seg;              // 1: segment weight (RFVR_WEIGHT_SEGMENT), 0: sample weight
    int bi;               // 1: bistatic aperture (separate receivers)
    const AntRec* rxa;    // its receiver records (set once built), or NULL
};
int choose_point_splits(long n_pts, int lanes_total);
int freq_chunk(int n_freq);

hipError_t launch_ant_records(const float* tx, const float* phi_tx, int n_meas, AntRec* out,
                              hipStream_t st);
hipError_t launch_render_prep(const RenderGeom& g, const float* xyz, const float* ray_w, const float* pt_w,
                              const float* sdf, const float* grad, const float* refl,
                              const float* phi_ray, int use_phi, float s, const float* log_s, float amp,
                              const float* amp_ptr, PtRec* rec, float* alpha_out, float* trans_out,
                              hipStream_t st);
// sel: NULL, or the plan of the Chebyshev path (these kernels then return at
// once unless it chose the per-frequency kernels, K == 0)
hipError_t launch_reduce_points_render(const RenderGeom& g, const AntRec* ant, const PtRec* rec,
                                       uint32_t flags, int n_split, float2* partial, const ChebPlan* sel,
                                       hipStream_t st);
hipError_t launch_reduce_points_mf(const RenderGeom& g, const AntRec* ant, const QRec* rec,
                                   uint32_t flags, int n_split, float2* partial, const ChebPlan* sel,
                                   hipStream_t st);
hipError_t launch_split_sum(const float2* partial, int n_split, long n_out, int accumulate,
                            float2* out, const ChebPlan* sel, hipStream_t st);
hipError_t launch_pad_signal(const float2* sig, int n_meas, int n_freq, int np, float2* out,
                             hipStream_t st);
hipError_t launch_render_bwd_points(const RenderGeom& g, const AntRec* ant, const PtRec* rec,
                                    const float2* gsig_pad, int np, uint32_t flags, float* g_b,
                                    float* g_T, float* g_n, const ChebPlan* sel, hipStream_t st);
hipError_t launch_scan_adjoint(const RenderGeom& g, const float* ray_w, const float* sdf,
                               const float* grad, const float* refl, float s, const float* log_s, float amp,
                               const float* amp_ptr, const float* alpha, const float* trans,
                               const float* g_b, const float* g_T, const float* g_n,
                               float* g_alpha_tmp, float* part_amp, float* part_s, float* g_sdf,
                               float* g_grad, float* g_refl, int accumulate, hipStream_t st);
hipError_t launch_sum_scalars(const float* part, int n, float* out, int accumulate,
                              hipStream_t st);

// Launchers (mf.hip)
hipError_t launch_mf_forward(const RenderGeom& g, const AntRec* ant, const float* xyz_q, long n_q,
                             const float2* sig_pad, const float2* sig2_pad, int np, uint32_t flags,
                             float2* z, float* power, float2* z2, float* power2, const ChebPlan* sel,
                             hipStream_t st);
hipError_t launch_mf_bwd_records(const float* xyz_q, long n_q, const float2* z, const float* power,
                                 const float* g_power, QRec* rec, hipStream_t st);

// Launchers (misc.hip)
hipError_t launch_loss_partial(long n, const float* p, const float* ps, const float* mask,
                               float* g_p, double* part, int n_blocks, hipStream_t st);
hipError_t launch_loss_final(const double* part, int n_blocks, long n, float* loss, hipStream_t st);
hipError_t launch_sample_points(const rfvr_sample_desc& d, const double basis[9], float* xyz,
                                float* u, float* origin, hipStream_t st);
hipError_t launch_occupancy(long n, float s, const float* log_s, const float* f, float* phi, hipStream_t st);
hipError_t launch_mask_update(long n, const float* p, const float* p_ref, float* hist, float tau_hi,
                              float tau_lo, float* mask, float* part, int nb, hipStream_t st);
hipError_t launch_sample_importance(const rfvr_sample_desc& d, const double basis[9], const float* logits,
                                    int n_bins, int n_imp, int n_uni, float* xyz, float* u, float* origin,
                                    hipStream_t st);
hipError_t launch_sample_naive(const rfvr_sample_desc& d, const double basis[9], const float* tx, int n_ant,
                               float* xyz, float* jac, hipStream_t st);
hipError_t launch_proposal_targets(int n_ray, int n_k, const float* u, const float* alpha, const float* trans,
                                   float lo, float hi, int n_bins, int n_dilate, float* targets, hipStream_t st);
hipError_t launch_bce(long n, const float* z, const float* t, float* loss, float* g, double* part, int nb,
                      hipStream_t st);
hipError_t launch_adamw(long n, float* p, const float* g, float* m, float* v, float lr, float b1,
                        float b2, float eps, float wd, float bc1, float bc2, hipStream_t st);

// Launchers (cheb.hip)
constexpr int kChebMaxOrder = 64;
int cheb_bbox_blocks(long n);
int cheb_point_splits(long n_pts, int n_meas);
hipError_t launch_cheb_order(const ChebPlan* plan, int32_t* order, hipStream_t st);
hipError_t launch_cheb_plan(const float* xyz, long n, const AntRec* ant, const AntRec* rxa, int n_meas,
                            double Kd, int n_freq, float* bbox_part, MeasCheb* meas, ChebPlan* plan,
                            hipStream_t st);
hipError_t launch_cheb_points(const RenderGeom& g, int kind, uint32_t flags, const AntRec* ant,
                              const MeasCheb* meas, const ChebPlan* plan, const void* rec, int n_split,
                              float2* partial, float2* M, float2* out, int accumulate, hipStream_t st);
hipError_t launch_cheb_coef(const RenderGeom& g, const ChebPlan* plan, const MeasCheb* meas, const float2* sig,
                            float2* B, hipStream_t st);
hipError_t launch_cheb_mf(const RenderGeom& g, const ChebPlan* plan, long n_q, const float* xq,
                          const AntRec* ant, const MeasCheb* meas, const float2* B, const float2* B2,
                          float2* z, float* power, float2* z2, float* power2, hipStream_t st);
hipError_t launch_cheb_render_bwd(const RenderGeom& g, uint32_t flags, const ChebPlan* plan, const AntRec* ant,
                                  const MeasCheb* meas, const PtRec* rec, const float2* B, float* g_b,
                                  float* g_T, float* g_n, hipStream_t st);

}  // namespace rfvr
