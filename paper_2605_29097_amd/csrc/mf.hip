// Matched filter (Eq. mf-sm; App. A.4 Alg. 1) and the records of its adjoint.
//
// Forward: one lane per query point; all lanes of a wave walk the same
// measurements, so the measurement record and the signal row are scalar loads.
// For a measurement, sum_n s[n] exp(+j 2 pi (theta0 + n delta)) =
// exp(+j 2 pi theta_mid) * sum_n s[n] w^(n - mid), a Laurent polynomial of the
// signal row in w = exp(+j 2 pi delta) around the middle frequency, evaluated
// by Horner's rule in w (upper half) and conj(w) (lower half): 4 FMA per term
// once the pair's range (FP64), centre phase (FP64 reduction) and accurately
// rounded step phasor are set up.  A second
// signal (e.g. the measured one) can be filtered at the same points sharing the
// set-up.  The adjoint reduces over points (render.hip, KIND 1).
#include "rfvr_impl.hpp"

namespace rfvr {

template <bool TWO, bool NAIVE>
__global__ __launch_bounds__(256) void k_mf_forward(
    long n_q, const float* __restrict__ xq, int n_meas, const AntRec* __restrict__ ant,
    const float2* __restrict__ sig, const float2* __restrict__ sig2, int np, double K0,
    double Kd, float2* __restrict__ z, float* __restrict__ power, float2* __restrict__ z2,
    float* __restrict__ power2) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = q < n_q;
    const long qq = ok ? q : n_q - 1;
    const double px = (double)xq[3 * qq], py = (double)xq[3 * qq + 1], pz = (double)xq[3 * qq + 2];
    const int mid = np / 2;                        // multiple of 16
    const double Km = K0 + (double)mid * Kd;
    float zr = 0.0f, zi = 0.0f, z2r = 0.0f, z2i = 0.0f;
    for (int i = 0; i < n_meas; ++i) {
        const AntRec A = ant[i];
        const PairGeom geo = pair_geom<NAIVE>(px - A.x, py - A.y, pz - A.z);
        float cw, sw;
        step_phasor<NAIVE>(geo, Kd, cw, sw);       // w = exp(+j 2 pi delta)
        const float2* row = sig + (size_t)i * np;
        const float2* row2 = TWO ? sig2 + (size_t)i * np : nullptr;
        // H = sum_n s[n] w^(n - mid): upper half by Horner in w from the top,
        // lower half by Horner in conj(w) from the bottom
        float hr = 0.0f, hi = 0.0f, lr = 0.0f, li = 0.0f;
        float h2r = 0.0f, h2i = 0.0f, l2r = 0.0f, l2i = 0.0f;
        for (int n0 = np - 16; n0 >= mid; n0 -= 16) {
#pragma unroll
            for (int u = 15; u >= 0; --u) {
                const float2 sv = row[n0 + u];
                const float tr = __builtin_fmaf(-hi, sw, __builtin_fmaf(hr, cw, sv.x));
                hi = __builtin_fmaf(hi, cw, __builtin_fmaf(hr, sw, sv.y));
                hr = tr;
                if constexpr (TWO) {
                    const float2 sv2 = row2[n0 + u];
                    const float t2 = __builtin_fmaf(-h2i, sw, __builtin_fmaf(h2r, cw, sv2.x));
                    h2i = __builtin_fmaf(h2i, cw, __builtin_fmaf(h2r, sw, sv2.y));
                    h2r = t2;
                }
            }
        }
        for (int n0 = 0; n0 < mid; n0 += 16) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const float2 sv = row[n0 + u];
                const float tr = __builtin_fmaf(li, sw, __builtin_fmaf(lr, cw, sv.x));
                li = __builtin_fmaf(li, cw, __builtin_fmaf(-lr, sw, sv.y));
                lr = tr;
                if constexpr (TWO) {
                    const float2 sv2 = row2[n0 + u];
                    const float t2 = __builtin_fmaf(l2i, sw, __builtin_fmaf(l2r, cw, sv2.x));
                    l2i = __builtin_fmaf(l2i, cw, __builtin_fmaf(-l2r, sw, sv2.y));
                    l2r = t2;
                }
            }
        }
        hr = __builtin_fmaf(lr, cw, __builtin_fmaf(li, sw, hr));
        hi = __builtin_fmaf(li, cw, __builtin_fmaf(-lr, sw, hi));
        float c0, s0;
        seed_phasor<NAIVE>(geo, Km, c0, s0);      // exp(+j 2 pi theta_mid)
        zr = __builtin_fmaf(c0, hr, __builtin_fmaf(-s0, hi, zr));
        zi = __builtin_fmaf(c0, hi, __builtin_fmaf(s0, hr, zi));
        if constexpr (TWO) {
            h2r = __builtin_fmaf(l2r, cw, __builtin_fmaf(l2i, sw, h2r));
            h2i = __builtin_fmaf(l2i, cw, __builtin_fmaf(-l2r, sw, h2i));
            z2r = __builtin_fmaf(c0, h2r, __builtin_fmaf(-s0, h2i, z2r));
            z2i = __builtin_fmaf(c0, h2i, __builtin_fmaf(s0, h2r, z2i));
        }
    }
    if (ok) {
        if (z) z[q] = make_float2(zr, zi);
        if (power) power[q] = sqrtf(zr * zr + zi * zi);
        if constexpr (TWO) {
            if (z2) z2[q] = make_float2(z2r, z2i);
            if (power2) power2[q] = sqrtf(z2r * z2r + z2i * z2i);
        }
    }
}

hipError_t launch_mf_forward(const RenderGeom& g, const AntRec* ant, const float* xyz_q, long n_q,
                             const float2* sig_pad, const float2* sig2_pad, int np, uint32_t flags,
                             float2* z, float* power, float2* z2, float* power2, hipStream_t st) {
    dim3 grid((unsigned)((n_q + 255) / 256));
    const bool naive = (flags & RFVR_PHASE_NAIVE32) != 0;
    if (sig2_pad) {
        if (naive)
            hipLaunchKernelGGL((k_mf_forward<true, true>), grid, dim3(256), 0, st, n_q, xyz_q,
                               g.n_meas, ant, sig_pad, sig2_pad, np, g.K0, g.Kd, z, power, z2,
                               power2);
        else
            hipLaunchKernelGGL((k_mf_forward<true, false>), grid, dim3(256), 0, st, n_q, xyz_q,
                               g.n_meas, ant, sig_pad, sig2_pad, np, g.K0, g.Kd, z, power, z2,
                               power2);
    } else {
        if (naive)
            hipLaunchKernelGGL((k_mf_forward<false, true>), grid, dim3(256), 0, st, n_q, xyz_q,
                               g.n_meas, ant, sig_pad, sig2_pad, np, g.K0, g.Kd, z, power, z2,
                               power2);
        else
            hipLaunchKernelGGL((k_mf_forward<false, false>), grid, dim3(256), 0, st, n_q, xyz_q,
                               g.n_meas, ant, sig_pad, sig2_pad, np, g.K0, g.Kd, z, power, z2,
                               power2);
    }
    return hipGetLastError();
}

// h_q = g_P,q * z_q / P_q (0 where P_q == 0), with the point in FP64
__global__ void k_mf_bwd_records(const float* __restrict__ xq, long n_q,
                                 const float2* __restrict__ z, const float* __restrict__ power,
                                 const float* __restrict__ g_power, QRec* __restrict__ rec) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_q) return;
    const float P = power[q];
    const float sc = P > 0.0f ? g_power[q] / P : 0.0f;
    const float2 zz = z[q];
    QRec r;
    r.x = (double)xq[3 * q];
    r.y = (double)xq[3 * q + 1];
    r.z = (double)xq[3 * q + 2];
    r.hr = sc * zz.x;
    r.hi = sc * zz.y;
    rec[q] = r;
}

hipError_t launch_mf_bwd_records(const float* xyz_q, long n_q, const float2* z, const float* power,
                                 const float* g_power, QRec* rec, hipStream_t st) {
    hipLaunchKernelGGL(k_mf_bwd_records, dim3((unsigned)((n_q + 255) / 256)), dim3(256), 0, st,
                       xyz_q, n_q, z, power, g_power, rec);
    return hipGetLastError();
}

}  // namespace rfvr
