// Matched filter (Eq. mf-sm; App. A (Code Implementation) Alg. 1) and the records of its adjoint.
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

#ifndef RFVR_HORNER_PPL
#define RFVR_HORNER_PPL 1
#endif
constexpr int kHornerPPL = RFVR_HORNER_PPL;   // query points per lane

template <bool TWO, bool NAIVE, bool BI>
__global__ __launch_bounds__(256) void k_mf_forward(
    long n_q, const float* __restrict__ xq, int n_meas, const AntRec* __restrict__ ant,
    const AntRec* __restrict__ rxa,
    const float2* __restrict__ sig, const float2* __restrict__ sig2, int np, double K0,
    double Kd, float2* __restrict__ z, float* __restrict__ power, float2* __restrict__ z2,
    float* __restrict__ power2, const ChebPlan* __restrict__ sel) {
    if (sel && sel->K != 0) return;              // the Chebyshev path took this launch
    constexpr int PPL = kHornerPPL;
    const long q0 = (long)blockIdx.x * blockDim.x * PPL + threadIdx.x;
    double px[PPL], py[PPL], pz[PPL];
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        long q = q0 + (long)u * blockDim.x;
        if (q >= n_q) q = n_q - 1;
        px[u] = (double)xq[3 * q];
        py[u] = (double)xq[3 * q + 1];
        pz[u] = (double)xq[3 * q + 2];
    }
    const int mid = np / 2;                        // multiple of 16
    const double Km = K0 + (double)mid * Kd;
    float zr[PPL], zi[PPL], z2r[PPL], z2i[PPL];
#pragma unroll
    for (int u = 0; u < PPL; ++u) { zr[u] = zi[u] = z2r[u] = z2i[u] = 0.0f; }
    for (int i = 0; i < n_meas; ++i) {
        const AntRec A = ant[i];
        PairGeom geo[PPL];
        float cw[PPL], sw[PPL];
#pragma unroll
        for (int u = 0; u < PPL; ++u) {
            if constexpr (BI) {
                const AntRec Rx = rxa[i];
                geo[u] = bi_geom<NAIVE>(px[u] - A.x, py[u] - A.y, pz[u] - A.z, px[u] - Rx.x, py[u] - Rx.y,
                                        pz[u] - Rx.z).g;
            } else {
                geo[u] = pair_geom<NAIVE>(px[u] - A.x, py[u] - A.y, pz[u] - A.z);
            }
            step_phasor<NAIVE>(geo[u], Kd, cw[u], sw[u]);       // w = exp(+j 2 pi delta)
        }
        const float2* row = sig + (size_t)i * np;
        const float2* row2 = TWO ? sig2 + (size_t)i * np : nullptr;
        // H = sum_n s[n] w^(n - mid): upper half by Horner in w from the top,
        // lower half by Horner in conj(w) from the bottom
        float hr[PPL], hi[PPL], lr[PPL], li[PPL], h2r[PPL], h2i[PPL], l2r[PPL], l2i[PPL];
#pragma unroll
        for (int u = 0; u < PPL; ++u) hr[u] = hi[u] = lr[u] = li[u] = h2r[u] = h2i[u] = l2r[u] = l2i[u] = 0.0f;
        for (int n0 = np - 16; n0 >= mid; n0 -= 16) {
#pragma unroll
            for (int k = 15; k >= 0; --k) {
                const float2 sv = row[n0 + k];
                float2 sv2;
                if constexpr (TWO) sv2 = row2[n0 + k];
#pragma unroll
                for (int u = 0; u < PPL; ++u) {
                    const float tr = __builtin_fmaf(-hi[u], sw[u], __builtin_fmaf(hr[u], cw[u], sv.x));
                    hi[u] = __builtin_fmaf(hi[u], cw[u], __builtin_fmaf(hr[u], sw[u], sv.y));
                    hr[u] = tr;
                    if constexpr (TWO) {
                        const float t2 = __builtin_fmaf(-h2i[u], sw[u], __builtin_fmaf(h2r[u], cw[u], sv2.x));
                        h2i[u] = __builtin_fmaf(h2i[u], cw[u], __builtin_fmaf(h2r[u], sw[u], sv2.y));
                        h2r[u] = t2;
                    }
                }
            }
        }
        for (int n0 = 0; n0 < mid; n0 += 16) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const float2 sv = row[n0 + k];
                float2 sv2;
                if constexpr (TWO) sv2 = row2[n0 + k];
#pragma unroll
                for (int u = 0; u < PPL; ++u) {
                    const float tr = __builtin_fmaf(li[u], sw[u], __builtin_fmaf(lr[u], cw[u], sv.x));
                    li[u] = __builtin_fmaf(li[u], cw[u], __builtin_fmaf(-lr[u], sw[u], sv.y));
                    lr[u] = tr;
                    if constexpr (TWO) {
                        const float t2 = __builtin_fmaf(l2i[u], sw[u], __builtin_fmaf(l2r[u], cw[u], sv2.x));
                        l2i[u] = __builtin_fmaf(l2i[u], cw[u], __builtin_fmaf(-l2r[u], sw[u], sv2.y));
                        l2r[u] = t2;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < PPL; ++u) {
            const float Hr = __builtin_fmaf(lr[u], cw[u], __builtin_fmaf(li[u], sw[u], hr[u]));
            const float Hi = __builtin_fmaf(li[u], cw[u], __builtin_fmaf(-lr[u], sw[u], hi[u]));
            float c0, s0;
            seed_phasor<NAIVE>(geo[u], Km, c0, s0);      // exp(+j 2 pi theta_mid)
            zr[u] = __builtin_fmaf(c0, Hr, __builtin_fmaf(-s0, Hi, zr[u]));
            zi[u] = __builtin_fmaf(c0, Hi, __builtin_fmaf(s0, Hr, zi[u]));
            if constexpr (TWO) {
                const float H2r = __builtin_fmaf(l2r[u], cw[u], __builtin_fmaf(l2i[u], sw[u], h2r[u]));
                const float H2i = __builtin_fmaf(l2i[u], cw[u], __builtin_fmaf(-l2r[u], sw[u], h2i[u]));
                z2r[u] = __builtin_fmaf(c0, H2r, __builtin_fmaf(-s0, H2i, z2r[u]));
                z2i[u] = __builtin_fmaf(c0, H2i, __builtin_fmaf(s0, H2r, z2i[u]));
            }
        }
    }
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        const long q = q0 + (long)u * blockDim.x;
        if (q >= n_q) continue;
        if (z) z[q] = make_float2(zr[u], zi[u]);
        if (power) power[q] = sqrtf(zr[u] * zr[u] + zi[u] * zi[u]);
        if constexpr (TWO) {
            if (z2) z2[q] = make_float2(z2r[u], z2i[u]);
            if (power2) power2[q] = sqrtf(z2r[u] * z2r[u] + z2i[u] * z2i[u]);
        }
    }
}

hipError_t launch_mf_forward(const RenderGeom& g, const AntRec* ant, const float* xyz_q, long n_q,
                             const float2* sig_pad, const float2* sig2_pad, int np, uint32_t flags,
                             float2* z, float* power, float2* z2, float* power2, const ChebPlan* sel,
                             hipStream_t st) {
    dim3 grid((unsigned)((n_q + 256L * kHornerPPL - 1) / (256L * kHornerPPL)));
    const bool naive = (flags & RFVR_PHASE_NAIVE32) != 0;
#define RFVR_MFF(TV, NV, BV)                                                                                 \
    hipLaunchKernelGGL((k_mf_forward<TV, NV, BV>), grid, dim3(256), 0, st, n_q, xyz_q, g.n_meas, ant, g.rxa, \
                       sig_pad, sig2_pad, np, g.K0, g.Kd, z, power, z2, power2, sel)
#define RFVR_MFF_B(TV, NV)            \
    if (g.rxa) RFVR_MFF(TV, NV, true); \
    else RFVR_MFF(TV, NV, false)
    if (sig2_pad) {
        if (naive) { RFVR_MFF_B(true, true); }
        else { RFVR_MFF_B(true, false); }
    } else {
        if (naive) { RFVR_MFF_B(false, true); }
        else { RFVR_MFF_B(false, false); }
    }
#undef RFVR_MFF_B
#undef RFVR_MFF
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
