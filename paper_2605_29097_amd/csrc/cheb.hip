// Term sums of signal tracing and the matched filter (Eq. ref_sim, Eq. mf-sm
// and their adjoints) evaluated through Chebyshev moments of the residual
// range.  Same sums as the per-frequency kernels (render.hip, mf.hip), fewer
// operations per (measurement, point) pair.
//
// A pair's phasor at frequency n is exp(s j 2 pi (K0 + n Kd) r), s = -1 for
// the reductions over points (render forward, filter adjoint) and +1 for the
// reductions over frequencies (filter forward, render adjoint).  It is split at
// the centre of the band, Kc = K0 + nc Kd with nc = (n_freq - 1) / 2, and
// dn = n - nc in [-nc, nc].  Every point of a launch lies in an axis-aligned
// box, so for measurement i its range r lies in [rc_i - h_i, rc_i + h_i]
// (distances from the transmitter to the box; for a bistatic pair r is the
// mean of the distances from the transmitter and to the receiver, and the band
// the mean of their two bands).  With x = (r - rc) / h in
// [-1, 1] and z_n = 2 pi dn Kd h (of either sign),
//   exp(s j 2 pi dn Kd r) = exp(s j 2 pi dn Kd rc) exp(s j z_n x)
// and the Jacobi-Anger expansion
//   exp(s j z x) = sum_k eps_k (s j)^k J_k(z) T_k(x),  eps_0 = 1, eps_k = 2,
// (T_k Chebyshev polynomials, J_k Bessel functions of the first kind, with
// J_k(-z) = (-1)^k J_k(z)) turns
//   * a reduction over points into K moments per measurement,
//       M_ik = sum_j a_ij exp(-j 2 pi Kc r_ij) T_k(x_ij),
//       out[i][n] = exp(-j 2 pi dn Kd rc_i) sum_k eps_k (-j)^k J_k(z_in) M_ik;
//   * a reduction over frequencies into a Chebyshev series per measurement,
//       B_ik = eps_k j^k sum_n g[i][n] exp(+j 2 pi dn Kd rc_i) J_k(z_in),
//       sum_n g[i][n] exp(+j 2 pi (K0 + n Kd) r) = exp(+j 2 pi Kc r) sum_k B_ik T_k(x),
//     evaluated per pair with T_k from their three-term recurrence.
// Centring the band halves the largest |z| (against splitting at f0), and with
// it the number of orders the series needs.  Since |T_k| <= 1 on [-1, 1] and
// |J_k(z)| <= (|z|/2)^k / k!, cutting the series at K changes each output by at
// most 2 (z/2)^K / K! / (1 - z / (2K + 2)) (z = max |z_n|) times the sum of the
// magnitudes of its terms' weights.  A one-block plan kernel takes the largest
// z of the launch and picks the smallest K of kChebKs whose
// bound is below kChebTol, or 0 (the per-frequency kernels) when none is (a
// wide range spread) or K is not below the number of frequencies.  The choice
// stays on the device: every candidate kernel is launched and all but the
// chosen one return at once, so no host synchronisation is needed.
//
// Per pair both cost 3 FP32 operations per order (recurrence of T_k and a
// complex multiply-add by a real), against 4 per frequency in the
// per-frequency kernels; the FP64 range and the one phasor exp(-+j 2 pi Kc r)
// (hardware sin / cos of the FP64-reduced phase, at Kc) are set up once per pair.  Bessel values come from Miller's backward
// recurrence in FP64 (first pass: normalisation J_0 + 2 sum J_2m = 1 and the
// number of rescalings; second pass: the values, consumed as produced).
#include <cmath>
#include <type_traits>

#include "rfvr_impl.hpp"

namespace rfvr {

constexpr int kChebKs[] = {24, 28, 32, 40, 48, 64};
constexpr int kChebKMax = kChebMaxOrder;
// truncation bound, relative to the sum of the term magnitudes: of the order of
// the FP32 rounding of the sums themselves (a lane's moments accumulate a
// point split of ~2k points in FP32)
constexpr double kChebTol = 1e-6;

// ---------------------------------------------------------------------------
// bounding box of a launch's points: per-block min / max, then the plan
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bbox_partial(const float* __restrict__ xyz, long n, long per,
                                                      float* __restrict__ part) {
    __shared__ float s[6][256];
    const int t = threadIdx.x;
    const long b0 = (long)blockIdx.x * per;
    long b1 = b0 + per;
    if (b1 > n) b1 = n;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long j = b0 + t; j < b1; j += 256) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float v = xyz[3 * j + c];
            lo[c] = fminf(lo[c], v);
            hi[c] = fmaxf(hi[c], v);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        s[c][t] = lo[c];
        s[3 + c][t] = hi[c];
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                s[c][t] = fminf(s[c][t], s[c][t + w]);
                s[3 + c][t] = fmaxf(s[3 + c][t], s[3 + c][t + w]);
            }
        }
        __syncthreads();
    }
    if (t < 6) part[(long)blockIdx.x * 6 + t] = s[t][0];
}

// log of 2 (z/2)^K / K! / (1 - z/(2K+2)), the truncation bound; +inf when the
// geometric tail does not converge
__device__ double cheb_log_bound(int K, double z) {
    const double q = 0.5 * z;
    if (q <= 0.0) return -INFINITY;
    if (q >= (double)(K + 1)) return INFINITY;
    double lf = 0.0;
    for (int m = 2; m <= K; ++m) lf += log((double)m);
    return (double)K * log(q) - lf + log(2.0) - log1p(-q / (double)(K + 1));
}

__global__ __launch_bounds__(256) void k_cheb_plan(const float* __restrict__ part, int nb,
                                                   const AntRec* __restrict__ ant,
                                                   const AntRec* __restrict__ rxa, int n_meas, double Kd,
                                                   int n_freq, MeasCheb* __restrict__ meas,
                                                   ChebPlan* __restrict__ plan) {
    __shared__ float sb[6][256];
    __shared__ double sz[256];
    const int t = threadIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = t; b < nb; b += 256) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], part[6 * b + c]);
            hi[c] = fmaxf(hi[c], part[6 * b + 3 + c]);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sb[c][t] = lo[c];
        sb[3 + c][t] = hi[c];
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sb[c][t] = fminf(sb[c][t], sb[c][t + w]);
                sb[3 + c][t] = fmaxf(sb[3 + c][t], sb[3 + c][t + w]);
            }
        }
        __syncthreads();
    }
    const double bl[3] = {(double)sb[0][0], (double)sb[1][0], (double)sb[2][0]};
    const double bh[3] = {(double)sb[3][0], (double)sb[4][0], (double)sb[5][0]};
    const bool finite = isfinite(bl[0]) && isfinite(bl[1]) && isfinite(bl[2]) && isfinite(bh[0]) &&
                        isfinite(bh[1]) && isfinite(bh[2]);
    // distances from an antenna to the box: nearest face, farthest corner
    auto band = [&](const AntRec& a, double& lo_, double& hi_) {
        const double p[3] = {a.x, a.y, a.z};
        double n2 = 0.0, f2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double qn = fmax(fmax(bl[c] - p[c], p[c] - bh[c]), 0.0);
            const double qf = fmax(fabs(p[c] - bl[c]), fabs(p[c] - bh[c]));
            n2 += qn * qn;
            f2 += qf * qf;
        }
        lo_ = sqrt(n2);
        hi_ = sqrt(f2);
    };
    double zl = 0.0;
    for (int i = t; i < n_meas; i += 256) {
        double rlo, rhi;
        band(ant[i], rlo, rhi);
        if (rxa) {
            double lo2, hi2;
            band(rxa[i], lo2, hi2);
            rlo = 0.5 * (rlo + lo2);
            rhi = 0.5 * (rhi + hi2);
        }
        MeasCheb m;
        m.rc = 0.5 * (rlo + rhi);
        // margin for the rounding of the per-pair FP64 range (relative ~1e-14)
        m.h = 0.5 * (rhi - rlo) * (1.0 + 1e-12) + 1e-12 * (rhi + 1.0);
        m.inv_h = 1.0 / m.h;
        m.pad = 0.0;
        meas[i] = m;
        zl = fmax(zl, 6.283185307179586 * (0.5 * (double)(n_freq - 1)) * Kd * m.h);
    }
    sz[t] = zl;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) sz[t] = fmax(sz[t], sz[t + w]);
        __syncthreads();
    }
    if (t == 0) {
        const double zmax = sz[0];
        int K = 0;
        if (finite) {
            for (int c = 0; c < (int)(sizeof(kChebKs) / sizeof(kChebKs[0])); ++c) {
                const int k = kChebKs[c];
                if (k >= n_freq) break;
                if (cheb_log_bound(k, zmax) <= log(kChebTol)) { K = k; break; }
            }
        }
        ChebPlan p;
        p.K = K;
        p.pad = 0;
        p.zmax = zmax;
        *plan = p;
    }
}

// ---------------------------------------------------------------------------
// Bessel values J_k(z), k < nk, by Miller's backward recurrence (FP64).
// visit(k, J_k) is called for k = nk-1 down to 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int miller_start(int nk, double z) {
    const int a = nk > (int)z + 1 ? nk : (int)z + 1;
    return 2 * ((a + 20 + (int)(3.0 * cbrt(z + 1.0)) + (int)sqrt(40.0 * a)) / 2);
}

template <class Visit>
__device__ __forceinline__ void bessel_j_desc_pos(double z, int nk, Visit visit) {
    if (!(z > 1e-300)) {
        for (int k = nk - 1; k >= 1; --k) visit(k, 0.0);
        visit(0, 1.0);
        return;
    }
    const int m0 = miller_start(nk, z);
    const double iz2 = 2.0 / z;
    double jp = 0.0, jc = 1e-200, norm = 0.0;
    int stot = 0;
    for (int m = m0; m >= 1; --m) {
        const double jm = (double)m * iz2 * jc - jp;
        jp = jc;
        jc = jm;
        const int k = m - 1;
        if (k > 0 && (k & 1) == 0) norm += 2.0 * jc;
        if (fabs(jc) > 1e200) { jp *= 1e-200; jc *= 1e-200; norm *= 1e-200; ++stot; }
    }
    norm += jc;
    const double inv = 1.0 / norm;
    jp = 0.0;
    jc = 1e-200;
    int s = 0;
    for (int m = m0; m >= 1; --m) {
        const double jm = (double)m * iz2 * jc - jp;
        jp = jc;
        jc = jm;
        const int k = m - 1;
        if (k < nk) {
            const int d = stot - s;
            visit(k, d == 0 ? jc * inv : (d == 1 ? jc * 1e-200 * inv : 0.0));
        }
        if (fabs(jc) > 1e200) { jp *= 1e-200; jc *= 1e-200; ++s; }
    }
}

// J_k(z) for z of either sign: J_k(-z) = (-1)^k J_k(z)
template <class Visit>
__device__ __forceinline__ void bessel_j_desc(double z, int nk, Visit visit) {
    if (z >= 0.0) {
        bessel_j_desc_pos(z, nk, visit);
    } else {
        bessel_j_desc_pos(-z, nk, [&](int k, double J) { visit(k, (k & 1) ? -J : J); });
    }
}

// ---------------------------------------------------------------------------
// moments over points: signal tracing forward (KIND 0) and filter adjoint
// (KIND 1).  Lane = measurement; the lanes of a work-group walk the same point
// records in step, read as wave-uniform scalar loads; point splits dealt over
// the XCDs as in the per-frequency kernel.
// partial[split][meas][kChebKMax] (k < K written).
// ---------------------------------------------------------------------------
template <int K, int KIND, int SPEC, bool BI>
__global__ __launch_bounds__(256) void k_cheb_points(
    int n_meas, const AntRec* __restrict__ ant, const AntRec* __restrict__ rxa, const MeasCheb* __restrict__ meas,
    const ChebPlan* __restrict__ plan, double Kc, const void* __restrict__ recs_v, long n_pts,
    long pts_per_split, int n_split, int gx, float2* __restrict__ partial) {
    if (plan->K != K) return;
    using Rec = typename std::conditional<KIND == 0, PtRec, QRec>::type;
    const long bid = blockIdx.x;
    const int lb = (int)((bid / 8) % gx);
    const long split = (bid / (8L * gx)) * 8 + (bid % 8);
    if (split >= n_split) return;
    const int i = lb * blockDim.x + threadIdx.x;
    const bool live_lane = i < n_meas;
    const int ic = live_lane ? i : n_meas - 1;
    const AntRec A = ant[ic];
    AntRec Rx = A;
    if constexpr (BI) Rx = rxa[ic];
    const MeasCheb mc = meas[ic];
    float mr[K], mi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) mr[k] = mi[k] = 0.0f;
    const long j0 = split * pts_per_split;
    long j1 = j0 + pts_per_split;
    if (j1 > n_pts) j1 = n_pts;
    // every lane of the work-group takes the same point at the same time: its
    // record is a wave-uniform (scalar) load.  The next record is requested
    // once the current one has been read (scalar loads complete out of order,
    // so any wait is for all of them) and lands during the moment updates.
    const Rec* recs = reinterpret_cast<const Rec*>(recs_v);
    Rec cur = recs[j0 < j1 ? j0 : 0];
    for (long j = j0; j < j1; ++j) {
        double r;
        float cr, ci;
        if constexpr (KIND == 0 && !BI) {
            const PtRec& P = cur;
            const double dx = P.x - A.x, dy = P.y - A.y, dz = P.z - A.z;
            float y;
            r = range_f64(dx, dy, dz, y);
            float spec, live;
            if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
                spec = 1.0f;
            } else {
                const float nd = (P.nx * (float)dx + P.ny * (float)dy + P.nz * (float)dz) * y;
                spec_factor<SPEC>(nd, spec, live);
            }
            const float T = fminf(fmaxf(P.tp + A.phi, 0.0f), 1.0f);
            cr = P.b * spec * (T * (P.sq != 0.0f ? T : 1.0f)) * (y * y);
            ci = 0.0f;
        } else if constexpr (KIND == 0) {
            // bistatic (sample weight only): b spec T_tx T_rx / (r_t r_r)
            const PtRec& P = cur;
            const double dx = P.x - A.x, dy = P.y - A.y, dz = P.z - A.z;
            const double ex = P.x - Rx.x, ey = P.y - Rx.y, ez = P.z - Rx.z;
            float yt, yr;
            r = 0.5 * (range_f64(dx, dy, dz, yt) + range_f64(ex, ey, ez, yr));
            float spec, live;
            if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
                spec = 1.0f;
            } else {
                const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
                const float fex = (float)ex, fey = (float)ey, fez = (float)ez;
                const float ni = (P.nx * fdx + P.ny * fdy + P.nz * fdz) * yt;
                const float nr = -(P.nx * fex + P.ny * fey + P.nz * fez) * yr;
                const float ir = -(fdx * fex + fdy * fey + fdz * fez) * (yt * yr);
                spec_factor_bi<SPEC>(ni, nr, ir, spec, live);
            }
            const float Tt = fminf(fmaxf(P.tp + A.phi, 0.0f), 1.0f);
            const float Tr = fminf(fmaxf(P.tp + Rx.phi, 0.0f), 1.0f);
            cr = P.b * spec * (Tt * Tr) * (yt * yr);
            ci = 0.0f;
        } else {
            const QRec& Q = cur;
            float y;
            r = range_f64(Q.x - A.x, Q.y - A.y, Q.z - A.z, y);
            if constexpr (BI) {
                float yr;
                r = 0.5 * (r + range_f64(Q.x - Rx.x, Q.y - Rx.y, Q.z - Rx.z, yr));
            }
            cr = Q.hr;
            ci = Q.hi;
        }
        // weight times exp(-j 2 pi Kc r)
        const float t0 = frac_rev(r * Kc);
        const float c0 = cos_rev(t0), s0 = sin_rev(t0);
        const float br = __builtin_fmaf(cr, c0, ci * s0);
        const float bi = __builtin_fmaf(ci, c0, -cr * s0);
        const float x = (float)((r - mc.rc) * mc.inv_h);
        const Rec nxt = recs[j + 1 < j1 ? j + 1 : j];
        __builtin_amdgcn_sched_barrier(0);
        const float x2 = x + x;
        mr[0] += br;
        mi[0] += bi;
        float tm = 1.0f, tk = x;
        mr[1] = __builtin_fmaf(br, x, mr[1]);
        mi[1] = __builtin_fmaf(bi, x, mi[1]);
#pragma unroll
        for (int k = 2; k < K; ++k) {
            const float tn = __builtin_fmaf(x2, tk, -tm);
            tm = tk;
            tk = tn;
            mr[k] = __builtin_fmaf(br, tn, mr[k]);
            mi[k] = __builtin_fmaf(bi, tn, mi[k]);
        }
        cur = nxt;
    }
    if (live_lane) {
        float2* out = partial + ((size_t)split * n_meas + i) * kChebKMax;
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = make_float2(mr[k], mi[k]);
    }
}

// fixed-order sum over the splits of the moments: M[i][k] for k < K.  A
// work-group takes 32 outputs; its 8 thread groups sum every 8th split in FP64,
// then the 8 group sums are added in order.
constexpr int kMsOut = 32, kMsGroups = 8;
__global__ __launch_bounds__(256) void k_cheb_moment_sum(const float2* __restrict__ partial, int n_split,
                                                         int n_meas, const ChebPlan* __restrict__ plan,
                                                         float2* __restrict__ M) {
    __shared__ double sr[kMsGroups][kMsOut], si[kMsGroups][kMsOut];
    const int K = plan->K;
    if (K == 0) return;
    const int ol = threadIdx.x % kMsOut, gi = threadIdx.x / kMsOut;
    const long o = (long)blockIdx.x * kMsOut + ol;
    const bool live = o < (long)n_meas * kChebKMax && (int)(o % kChebKMax) < K;
    double ar = 0.0, ai = 0.0;
    if (live) {
        for (int s = gi; s < n_split; s += kMsGroups) {
            const float2 v = partial[(size_t)s * n_meas * kChebKMax + o];
            ar += v.x;
            ai += v.y;
        }
    }
    sr[gi][ol] = ar;
    si[gi][ol] = ai;
    __syncthreads();
    if (gi != 0 || !live) return;
    double tr = 0.0, ti = 0.0;
    for (int g = 0; g < kMsGroups; ++g) {
        tr += sr[g][ol];
        ti += si[g][ol];
    }
    M[o] = make_float2((float)tr, (float)ti);
}

// out[i][n] (+)= exp(-j 2 pi dn Kd rc_i) sum_k eps_k (-j)^k J_k(z_in) M_ik
__global__ __launch_bounds__(256) void k_cheb_out(const ChebPlan* __restrict__ plan,
                                                  const MeasCheb* __restrict__ meas,
                                                  const float2* __restrict__ M, int n_meas, int n_freq,
                                                  double Kd, int accumulate, float2* __restrict__ out) {
    const int K = plan->K;
    if (K == 0) return;
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)n_meas * n_freq) return;
    const int i = (int)(o / n_freq), n = (int)(o % n_freq);
    const MeasCheb mc = meas[i];
    const double dn = (double)n - 0.5 * (double)(n_freq - 1);
    const double z = 6.283185307179586 * dn * Kd * mc.h;
    const float2* Mi = M + (size_t)i * kChebKMax;
    double ar = 0.0, ai = 0.0;
    bessel_j_desc(z, K, [&](int k, double J) {
        const double e = k == 0 ? J : 2.0 * J;
        const float2 m = Mi[k];
        // (-j)^k: 1, -j, -1, j
        double vr, vi;
        switch (k & 3) {
            case 0: vr = m.x; vi = m.y; break;
            case 1: vr = m.y; vi = -m.x; break;
            case 2: vr = -m.x; vi = -m.y; break;
            default: vr = -m.y; vi = m.x; break;
        }
        ar += e * vr;
        ai += e * vi;
    });
    double s, c;
    const double ph = dn * Kd * mc.rc;
    sincos(6.283185307179586 * (ph - floor(ph)), &s, &c);
    // times exp(-j phase)
    const float re = (float)(ar * c + ai * s), im = (float)(ai * c - ar * s);
    if (accumulate) {
        float2 v = out[o];
        v.x += re;
        v.y += im;
        out[o] = v;
    } else {
        out[o] = make_float2(re, im);
    }
}

// B[i][k] = eps_k j^k sum_n g[i][n] exp(+j 2 pi dn Kd rc_i) J_k(z_in), k < K;
// one wave per measurement, lane-private sums in LDS, then a fixed-order sum
// over lanes per k
__global__ __launch_bounds__(64) void k_cheb_coef(const ChebPlan* __restrict__ plan,
                                                  const MeasCheb* __restrict__ meas,
                                                  const float2* __restrict__ g, int n_meas, int n_freq,
                                                  double Kd, float2* __restrict__ B) {
    __shared__ double2 acc[kChebKMax][64];
    const int K = plan->K;
    if (K == 0) return;
    const int i = blockIdx.x, lane = threadIdx.x;
    const MeasCheb mc = meas[i];
    for (int k = 0; k < K; ++k) acc[k][lane] = make_double2(0.0, 0.0);
    for (int n = lane; n < n_freq; n += 64) {
        const float2 gv = g[(size_t)i * n_freq + n];
        const double dn = (double)n - 0.5 * (double)(n_freq - 1);
        const double ph = dn * Kd * mc.rc;
        double s, c;
        sincos(6.283185307179586 * (ph - floor(ph)), &s, &c);
        const double wr = gv.x * c - gv.y * s, wi = gv.x * s + gv.y * c;   // g exp(+j phase)
        const double z = 6.283185307179586 * dn * Kd * mc.h;
        bessel_j_desc(z, K, [&](int k, double J) {
            double2 a = acc[k][lane];
            a.x += wr * J;
            a.y += wi * J;
            acc[k][lane] = a;
        });
    }
    __syncthreads();
    for (int k = lane; k < K; k += 64) {
        double sr = 0.0, si = 0.0;
        for (int l = 0; l < 64; ++l) {
            sr += acc[k][l].x;
            si += acc[k][l].y;
        }
        const double e = k == 0 ? 1.0 : 2.0;
        // j^k: 1, j, -1, -j
        double vr, vi;
        switch (k & 3) {
            case 0: vr = sr; vi = si; break;
            case 1: vr = -si; vi = sr; break;
            case 2: vr = -sr; vi = -si; break;
            default: vr = si; vi = -sr; break;
        }
        B[(size_t)i * kChebKMax + k] = make_float2((float)(e * vr), (float)(e * vi));
    }
}

// sum_k B_k T_k(x) (complex coefficients, real x) with T_k from their
// three-term recurrence: 3 operations per order (Clenshaw's backward form
// takes 4), the coefficients being wave-uniform scalar operands
template <int K>
__device__ __forceinline__ void cheb_series(const float2* __restrict__ Bi, float x, float& sr, float& si) {
    const float x2 = x + x;
    float2 c = Bi[0];
    sr = c.x;
    si = c.y;
    c = Bi[1];
    sr = __builtin_fmaf(c.x, x, sr);
    si = __builtin_fmaf(c.y, x, si);
    float tm = 1.0f, tk = x;
#pragma unroll
    for (int k = 2; k < K; ++k) {
        const float tn = __builtin_fmaf(x2, tk, -tm);
        tm = tk;
        tk = tn;
        c = Bi[k];
        sr = __builtin_fmaf(c.x, tn, sr);
        si = __builtin_fmaf(c.y, tn, si);
    }
}

// two series with the same argument, sharing the recurrence
template <int K>
__device__ __forceinline__ void cheb_series2(const float2* __restrict__ Bi, const float2* __restrict__ Ci, float x,
                                             float& sr, float& si, float& s2r, float& s2i) {
    const float x2 = x + x;
    float2 c = Bi[0], d = Ci[0];
    sr = c.x;
    si = c.y;
    s2r = d.x;
    s2i = d.y;
    c = Bi[1];
    d = Ci[1];
    sr = __builtin_fmaf(c.x, x, sr);
    si = __builtin_fmaf(c.y, x, si);
    s2r = __builtin_fmaf(d.x, x, s2r);
    s2i = __builtin_fmaf(d.y, x, s2i);
    float tm = 1.0f, tk = x;
#pragma unroll
    for (int k = 2; k < K; ++k) {
        const float tn = __builtin_fmaf(x2, tk, -tm);
        tm = tk;
        tk = tn;
        c = Bi[k];
        d = Ci[k];
        sr = __builtin_fmaf(c.x, tn, sr);
        si = __builtin_fmaf(c.y, tn, si);
        s2r = __builtin_fmaf(d.x, tn, s2r);
        s2i = __builtin_fmaf(d.y, tn, s2i);
    }
}

// ---------------------------------------------------------------------------
// matched filter forward: lane = query point, loop over measurements
// (records, plan and coefficients are wave-uniform loads)
// ---------------------------------------------------------------------------
template <int K, bool TWO, bool BI>
__global__ __launch_bounds__(256) void k_cheb_mf(const ChebPlan* __restrict__ plan, long n_q,
                                                 const float* __restrict__ xq, int n_meas,
                                                 const AntRec* __restrict__ ant,
                                                 const AntRec* __restrict__ rxa,
                                                 const MeasCheb* __restrict__ meas,
                                                 const float2* __restrict__ B, const float2* __restrict__ B2,
                                                 double Kc, float2* __restrict__ z, float* __restrict__ power,
                                                 float2* __restrict__ z2, float* __restrict__ power2) {
    if (plan->K != K) return;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long qc = q < n_q ? q : n_q - 1;
    const double px = (double)xq[3 * qc], py = (double)xq[3 * qc + 1], pz = (double)xq[3 * qc + 2];
    float zr = 0.0f, zi = 0.0f, z2r = 0.0f, z2i = 0.0f;
    for (int i = 0; i < n_meas; ++i) {
        const AntRec A = ant[i];
        const MeasCheb mc = meas[i];
        float y;
        double r = range_f64(px - A.x, py - A.y, pz - A.z, y);
        if constexpr (BI) {
            const AntRec Rx = rxa[i];
            float yr;
            r = 0.5 * (r + range_f64(px - Rx.x, py - Rx.y, pz - Rx.z, yr));
        }
        const float x = (float)((r - mc.rc) * mc.inv_h);
        const float t0 = frac_rev(r * Kc);
        const float c0 = cos_rev(t0), s0 = sin_rev(t0);       // exp(+j 2 pi Kc r)
        float sr, si;
        if constexpr (TWO) {
            float s2r, s2i;
            cheb_series2<K>(B + (size_t)i * kChebKMax, B2 + (size_t)i * kChebKMax, x, sr, si, s2r, s2i);
            z2r = __builtin_fmaf(c0, s2r, __builtin_fmaf(-s0, s2i, z2r));
            z2i = __builtin_fmaf(c0, s2i, __builtin_fmaf(s0, s2r, z2i));
        } else {
            cheb_series<K>(B + (size_t)i * kChebKMax, x, sr, si);
        }
        zr = __builtin_fmaf(c0, sr, __builtin_fmaf(-s0, si, zr));
        zi = __builtin_fmaf(c0, si, __builtin_fmaf(s0, sr, zi));
    }
    if (q >= n_q) return;
    if (z) z[q] = make_float2(zr, zi);
    if (power) power[q] = sqrtf(zr * zr + zi * zi);
    if constexpr (TWO) {
        if (z2) z2[q] = make_float2(z2r, z2i);
        if (power2) power2[q] = sqrtf(z2r * z2r + z2i * z2i);
    }
}

// ---------------------------------------------------------------------------
// signal tracing adjoint: lane = point, loop over measurements; the pair's
// G = Re(sum_n g[i][n] exp(+j 2 pi (K0 + n Kd) r)) then the chain rule of the
// per-frequency kernel
// ---------------------------------------------------------------------------
template <int K, int SPEC, bool BI>
__global__ __launch_bounds__(256) void k_cheb_render_bwd(const ChebPlan* __restrict__ plan, long n_pts,
                                                         const PtRec* __restrict__ rec, int n_meas,
                                                         const AntRec* __restrict__ ant,
                                                         const AntRec* __restrict__ rxa,
                                                         const MeasCheb* __restrict__ meas,
                                                         const float2* __restrict__ B, double Kc,
                                                         float* __restrict__ g_b, float* __restrict__ g_T,
                                                         float* __restrict__ g_n) {
    if (plan->K != K) return;
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const PtRec P = rec[j < n_pts ? j : n_pts - 1];
    float gb = 0.0f, gt = 0.0f, gn0 = 0.0f, gn1 = 0.0f, gn2 = 0.0f;
    for (int i = 0; i < n_meas; ++i) {
        const AntRec A = ant[i];
        const MeasCheb mc = meas[i];
        const double dx = P.x - A.x, dy = P.y - A.y, dz = P.z - A.z;
        float y;
        double r = range_f64(dx, dy, dz, y);
        AntRec Rx = A;
        double ex = 0.0, ey = 0.0, ez = 0.0;
        float yr = 0.0f;
        if constexpr (BI) {
            Rx = rxa[i];
            ex = P.x - Rx.x; ey = P.y - Rx.y; ez = P.z - Rx.z;
            r = 0.5 * (r + range_f64(ex, ey, ez, yr));
        }
        const float x = (float)((r - mc.rc) * mc.inv_h);
        float sr, si;
        cheb_series<K>(B + (size_t)i * kChebKMax, x, sr, si);
        const float t0 = frac_rev(r * Kc);
        const float c0 = cos_rev(t0), s0 = sin_rev(t0);
        const float G = c0 * sr - s0 * si;                     // Re(exp(+j 2 pi Kc r) S)
        if constexpr (BI) {
            // c = b spec T_tx T_rx y_t y_r (sample weight): dc/db, dc/dT
            // (times b after the loop) and dc/dn_hat (times -2 b after the loop)
            const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
            const float fex = (float)ex, fey = (float)ey, fez = (float)ez;
            float spec, live = 0.0f, ni = 0.0f, nr = 0.0f;
            if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
                spec = 1.0f;
            } else {
                ni = (P.nx * fdx + P.ny * fdy + P.nz * fdz) * y;
                nr = -(P.nx * fex + P.ny * fey + P.nz * fez) * yr;
                const float ir = -(fdx * fex + fdy * fey + fdz * fez) * (y * yr);
                spec_factor_bi<SPEC>(ni, nr, ir, spec, live);
            }
            const float Ut = P.tp + A.phi, Ur = P.tp + Rx.phi;
            const float Tt = fminf(fmaxf(Ut, 0.0f), 1.0f), Tr = fminf(fmaxf(Ur, 0.0f), 1.0f);
            const float dT = (Tt == Ut ? Tr : 0.0f) + (Tr == Ur ? Tt : 0.0f);
            const float gy = G * (y * yr);
            const float gs = gy * spec, T2 = Tt * Tr;
            gb = __builtin_fmaf(gs, T2, gb);
            gt = __builtin_fmaf(gs, dT, gt);
            if constexpr (SPEC != (int)RFVR_SPEC_OFF) {
                // nr w_i + ni w_r with w_i = d_t y_t, w_r = -d_r y_r
                const float ct = gy * T2 * live * (nr * y), cq = -gy * T2 * live * (ni * yr);
                gn0 = __builtin_fmaf(ct, fdx, __builtin_fmaf(cq, fex, gn0));
                gn1 = __builtin_fmaf(ct, fdy, __builtin_fmaf(cq, fey, gn1));
                gn2 = __builtin_fmaf(ct, fdz, __builtin_fmaf(cq, fez, gn2));
            }
            continue;
        }
        const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
        float spec, live = 0.0f, nd = 0.0f;
        if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
            spec = 1.0f;
        } else {
            nd = (P.nx * fdx + P.ny * fdy + P.nz * fdz) * y;
            spec_factor<SPEC>(nd, spec, live);
        }
        const float Tr = P.tp + A.phi;
        const float T = fminf(fmaxf(Tr, 0.0f), 1.0f);
        // transmittance factor T^2 (sample weight) or T (segment weight) and
        // its derivative where the clamp is inactive
        const float dT = T == Tr ? (P.sq != 0.0f ? T + T : 1.0f) : 0.0f;
        const float gy = G * (y * y);
        const float gs = gy * spec, T2 = T * (P.sq != 0.0f ? T : 1.0f);
        gb = __builtin_fmaf(gs, T2, gb);
        gt = __builtin_fmaf(gs, dT, gt);                       // times b after the loop
        if constexpr (SPEC != (int)RFVR_SPEC_OFF) {
            const float cn = gy * T2 * (nd * y) * live;        // times 4 b after the loop
            gn0 = __builtin_fmaf(cn, fdx, gn0);
            gn1 = __builtin_fmaf(cn, fdy, gn1);
            gn2 = __builtin_fmaf(cn, fdz, gn2);
        }
    }
    if (j >= n_pts) return;
    g_b[j] = gb;
    g_T[j] = P.b * gt;
    const float b4 = (BI ? -2.0f : 4.0f) * P.b;
    g_n[3 * j] = b4 * gn0;
    g_n[3 * j + 1] = b4 * gn1;
    g_n[3 * j + 2] = b4 * gn2;
}

__global__ void k_cheb_order(const ChebPlan* __restrict__ plan, int32_t* __restrict__ order) {
    if (threadIdx.x == 0) *order = plan->K;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int cheb_bbox_blocks(long n) {
    long b = (n + 4095) / 4096;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_cheb_order(const ChebPlan* plan, int32_t* order, hipStream_t st) {
    hipLaunchKernelGGL(k_cheb_order, dim3(1), dim3(64), 0, st, plan, order);
    return hipGetLastError();
}

hipError_t launch_cheb_plan(const float* xyz, long n, const AntRec* ant, const AntRec* rxa, int n_meas,
                            double Kd, int n_freq, float* bbox_part, MeasCheb* meas, ChebPlan* plan,
                            hipStream_t st) {
    const int nb = cheb_bbox_blocks(n);
    const long per = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(256), 0, st, xyz, n, per, bbox_part);
    hipLaunchKernelGGL(k_cheb_plan, dim3(1), dim3(256), 0, st, bbox_part, nb, ant, rxa, n_meas, Kd, n_freq, meas,
                       plan);
    return hipGetLastError();
}

// wavenumber at the centre of the band (revolutions per metre of range)
static double band_centre(const RenderGeom& g) { return g.K0 + 0.5 * (double)(g.n_freq - 1) * g.Kd; }

template <int KIND, int SPEC, bool BI>
static void launch_cp_all(const RenderGeom& g, const AntRec* ant, const MeasCheb* meas, const ChebPlan* plan,
                          const void* rec, int n_split, float2* partial, hipStream_t st) {
    const int gx = (g.n_meas + 255) / 256;
    const long groups = (n_split + 7) / 8;
    dim3 grid((unsigned)(groups * 8 * gx));
    const long per = (g.n_pts + n_split - 1) / n_split;
    const double Kc = band_centre(g);
#define RFVR_CP(KK)                                                                                           \
    hipLaunchKernelGGL((k_cheb_points<KK, KIND, SPEC, BI>), grid, dim3(256), 0, st, g.n_meas, ant, g.rxa, meas, \
                       plan, Kc, rec, g.n_pts, per, n_split, gx, partial)
    RFVR_CP(24);
    RFVR_CP(28);
    RFVR_CP(32);
    RFVR_CP(40);
    RFVR_CP(48);
    RFVR_CP(64);
#undef RFVR_CP
}

// Point splits of the moment kernels: twice the waves of the per-frequency
// kernels' rule (8192, eight per SIMD).  A lane's work per point is short at
// the lower orders, where five waves per SIMD fit, and more resident waves
// hide the per-tile barriers and LDS reads; >= 128 points per split.
int cheb_point_splits(long n_pts, int n_meas) {
    const long waves_per_split = (n_meas + 63) / 64;
    long ns = (8192 + waves_per_split - 1) / waves_per_split;
    const long max_by_pts = (n_pts + 127) / 128;
    if (ns > max_by_pts) ns = max_by_pts;
    if (ns < 1) ns = 1;
    if (ns > 65535) ns = 65535;
    return (int)ns;
}

hipError_t launch_cheb_points(const RenderGeom& g, int kind, uint32_t flags, const AntRec* ant,
                              const MeasCheb* meas, const ChebPlan* plan, const void* rec, int n_split,
                              float2* partial, float2* M, float2* out, int accumulate, hipStream_t st) {
    const auto all = [&](auto kind_c, auto spec_c) {
        constexpr int KI = decltype(kind_c)::value, SP = decltype(spec_c)::value;
        if (g.rxa) launch_cp_all<KI, SP, true>(g, ant, meas, plan, rec, n_split, partial, st);
        else launch_cp_all<KI, SP, false>(g, ant, meas, plan, rec, n_split, partial, st);
    };
    using I1 = std::integral_constant<int, 1>;
    using I0 = std::integral_constant<int, 0>;
    if (kind == 1) {
        all(I1{}, std::integral_constant<int, RFVR_SPEC_OFF>{});
    } else {
        switch (flags & RFVR_SPEC_MASK) {
            case RFVR_SPEC_RAW: all(I0{}, std::integral_constant<int, RFVR_SPEC_RAW>{}); break;
            case RFVR_SPEC_OFF: all(I0{}, std::integral_constant<int, RFVR_SPEC_OFF>{}); break;
            default: all(I0{}, std::integral_constant<int, RFVR_SPEC_CLAMP>{}); break;
        }
    }
    const long nm = (long)g.n_meas * kChebKMax;
    hipLaunchKernelGGL(k_cheb_moment_sum, dim3((unsigned)((nm + kMsOut - 1) / kMsOut)), dim3(kMsOut * kMsGroups), 0,
                       st, partial, n_split, g.n_meas, plan, M);
    const long no = (long)g.n_meas * g.n_freq;
    hipLaunchKernelGGL(k_cheb_out, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, st, plan, meas, M, g.n_meas,
                       g.n_freq, g.Kd, accumulate, out);
    return hipGetLastError();
}

hipError_t launch_cheb_coef(const RenderGeom& g, const ChebPlan* plan, const MeasCheb* meas, const float2* sig,
                            float2* B, hipStream_t st) {
    hipLaunchKernelGGL(k_cheb_coef, dim3(g.n_meas), dim3(64), 0, st, plan, meas, sig, g.n_meas, g.n_freq, g.Kd,
                       B);
    return hipGetLastError();
}

template <bool TWO, bool BI>
static void launch_cmf_all(const RenderGeom& g, const ChebPlan* plan, long n_q, const float* xq,
                           const AntRec* ant, const MeasCheb* meas, const float2* B, const float2* B2,
                           float2* z, float* power, float2* z2, float* power2, hipStream_t st) {
    dim3 grid((unsigned)((n_q + 255) / 256));
    const double Kc = band_centre(g);
#define RFVR_CMF(KK)                                                                                     \
    hipLaunchKernelGGL((k_cheb_mf<KK, TWO, BI>), grid, dim3(256), 0, st, plan, n_q, xq, g.n_meas, ant, g.rxa, \
                       meas, B, B2, Kc, z, power, z2, power2)
    RFVR_CMF(24);
    RFVR_CMF(28);
    RFVR_CMF(32);
    RFVR_CMF(40);
    RFVR_CMF(48);
    RFVR_CMF(64);
#undef RFVR_CMF
}

hipError_t launch_cheb_mf(const RenderGeom& g, const ChebPlan* plan, long n_q, const float* xq,
                          const AntRec* ant, const MeasCheb* meas, const float2* B, const float2* B2,
                          float2* z, float* power, float2* z2, float* power2, hipStream_t st) {
    if (B2) {
        if (g.rxa) launch_cmf_all<true, true>(g, plan, n_q, xq, ant, meas, B, B2, z, power, z2, power2, st);
        else launch_cmf_all<true, false>(g, plan, n_q, xq, ant, meas, B, B2, z, power, z2, power2, st);
    } else {
        if (g.rxa) launch_cmf_all<false, true>(g, plan, n_q, xq, ant, meas, B, B2, z, power, z2, power2, st);
        else launch_cmf_all<false, false>(g, plan, n_q, xq, ant, meas, B, B2, z, power, z2, power2, st);
    }
    return hipGetLastError();
}

template <int SPEC, bool BI>
static void launch_crb_all(const RenderGeom& g, const ChebPlan* plan, const AntRec* ant, const MeasCheb* meas,
                           const PtRec* rec, const float2* B, float* g_b, float* g_T, float* g_n,
                           hipStream_t st) {
    dim3 grid((unsigned)((g.n_pts + 255) / 256));
    const double Kc = band_centre(g);
#define RFVR_CRB(KK)                                                                                        \
    hipLaunchKernelGGL((k_cheb_render_bwd<KK, SPEC, BI>), grid, dim3(256), 0, st, plan, g.n_pts, rec, g.n_meas,  \
                       ant, g.rxa, meas, B, Kc, g_b, g_T, g_n)
    RFVR_CRB(24);
    RFVR_CRB(28);
    RFVR_CRB(32);
    RFVR_CRB(40);
    RFVR_CRB(48);
    RFVR_CRB(64);
#undef RFVR_CRB
}

hipError_t launch_cheb_render_bwd(const RenderGeom& g, uint32_t flags, const ChebPlan* plan, const AntRec* ant,
                                  const MeasCheb* meas, const PtRec* rec, const float2* B, float* g_b,
                                  float* g_T, float* g_n, hipStream_t st) {
    const auto all = [&](auto spec_c) {
        constexpr int SP = decltype(spec_c)::value;
        if (g.rxa) launch_crb_all<SP, true>(g, plan, ant, meas, rec, B, g_b, g_T, g_n, st);
        else launch_crb_all<SP, false>(g, plan, ant, meas, rec, B, g_b, g_T, g_n, st);
    };
    switch (flags & RFVR_SPEC_MASK) {
        case RFVR_SPEC_RAW: all(std::integral_constant<int, RFVR_SPEC_RAW>{}); break;
        case RFVR_SPEC_OFF: all(std::integral_constant<int, RFVR_SPEC_OFF>{}); break;
        default: all(std::integral_constant<int, RFVR_SPEC_CLAMP>{}); break;
    }
    return hipGetLastError();
}

}  // namespace rfvr
