// Render kernels: lensless alpha blending (per-ray scan), signal tracing
// (reduction over points) and its adjoint (reduction over frequencies and
// measurements), and the adjoint of the transmittance scan.
//
// Signal tracing, Eq. ref_sim / App. A (Code Implementation) Alg. 2, rebuilt for gfx950:
//  * forward: a lane owns one (measurement, frequency chunk) pair and keeps the
//    chunk's complex accumulators in VGPRs; all lanes of a work-group walk the
//    same points, whose records are staged through LDS in double-buffered
//    tiles of 64 (one wide load per record, broadcast reads, the next tile's
//    global loads in flight).  Per (measurement, point) the path length (FP64)
//    and the correctly rounded step phasor are set up once; every 32
//    frequencies a phasor is re-seeded from an FP64-reduced phase at the
//    sub-chunk centre and the sub-chunk is walked both ways (f_n is linear in
//    n) by the three-term recurrence p_{n+1} = 2 cos(2 pi delta) p_n - p_{n-1}
//    (one FMA per term and part, plus the accumulate).  Points are split across
//    work-groups (XCD-aware) and the partial sums reduced in a fixed order (no
//    atomics).
//  * backward: a lane owns one point; all lanes walk the same measurements, so
//    measurement records and the incoming signal gradient row are scalar loads.
//    sum_n g[n] exp(+j 2 pi (theta0 + n delta)) is, around the middle
//    frequency, a Laurent polynomial in w = exp(j 2 pi delta), evaluated by
//    Horner's rule in w and conj(w) (4 FMA per term).
#include "rfvr_impl.hpp"

namespace rfvr {

int freq_chunk(int n_freq) { return n_freq <= 16 ? 16 : (n_freq <= 32 ? 32 : 64); }

int choose_point_splits(long n_pts, int lanes_total) {
    long waves_per_split = (lanes_total + 63) / 64;
    const long target_waves = 4096;           // 16 waves per SIMD on 256 CUs
    long ns = (target_waves + waves_per_split - 1) / waves_per_split;
    long max_by_pts = (n_pts + 127) / 128;    // keep >= 128 points per split
    if (ns > max_by_pts) ns = max_by_pts;
    if (ns < 1) ns = 1;
    if (ns > 65535) ns = 65535;
    return (int)ns;
}

// ---------------------------------------------------------------------------
// measurement records
// ---------------------------------------------------------------------------
__global__ void k_ant_records(const float* __restrict__ tx, const float* __restrict__ phi_tx,
                              int n_meas, AntRec* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_meas) return;
    AntRec a;
    a.x = (double)tx[3 * i];
    a.y = (double)tx[3 * i + 1];
    a.z = (double)tx[3 * i + 2];
    a.phi = phi_tx ? phi_tx[i] : 0.0f;
    a.pad = 0.0f;
    out[i] = a;
}

hipError_t launch_ant_records(const float* tx, const float* phi_tx, int n_meas, AntRec* out,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_ant_records, dim3((n_meas + 255) / 256), dim3(256), 0, st, tx, phi_tx,
                       n_meas, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-ray prep: opacity, transmittance (product scan across the wave) and the
// per-point records.  One wave per ray, 64 samples per step.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_render_prep(
    int n_ray, int n_z, const float* __restrict__ xyz, const float* __restrict__ ray_w,
    const float* __restrict__ pt_w, const float* __restrict__ sdf, const float* __restrict__ grad, const float* __restrict__ refl,
    const float* __restrict__ phi_ray, int use_phi, float s_h, const float* __restrict__ log_s, float amp_h,
    const float* __restrict__ amp_ptr, int seg, PtRec* __restrict__ rec, float* __restrict__ alpha_out,
    float* __restrict__ trans_out) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= n_ray) return;                       // uniform per wave
    const int r = wave;
    const float amp = amp_ptr ? amp_ptr[0] : amp_h;
    const float s = log_s ? expf(log_s[0]) : s_h;
    const float w = ray_w ? ray_w[r] : 1.0f;
    const float pr = use_phi ? phi_ray[r] : 0.0f;
    const size_t base = (size_t)r * n_z;
    float carry = 1.0f;
    for (int k0 = 0; k0 < n_z; k0 += 64) {
        const int k = k0 + lane;
        const bool valid = k < n_z;
        float alpha = 0.0f;
        if (k + 1 < n_z) alpha = alpha_pair(s * sdf[base + k], s * sdf[base + k + 1]);
        float incl = 1.0f - alpha;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            float t = __shfl_up(incl, d, 64);
            if (lane >= d) incl *= t;
        }
        float excl = __shfl_up(incl, 1, 64);
        if (lane == 0) excl = 1.0f;
        const float T = carry * excl;
        carry *= __shfl(incl, 63, 64);
        if (valid) {
            const size_t j = base + k;
            PtRec p;
            p.x = (double)xyz[3 * j];
            p.y = (double)xyz[3 * j + 1];
            p.z = (double)xyz[3 * j + 2];
            p.b = amp * w * refl[j] * alpha * (pt_w ? pt_w[j] : 1.0f);
            p.tp = T - pr;
            p.sq = 1.0f;
            if (seg) {
                // the segment to the next sample: its midpoint (exact in FP64
                // from the FP32 inputs), the exact integral of T^2 rho over it
                // alpha T (T (1 - alpha/2) + dPhi) split as b and tp
                if (k + 1 < n_z) {
                    p.x = 0.5 * (p.x + (double)xyz[3 * j + 3]);
                    p.y = 0.5 * (p.y + (double)xyz[3 * j + 4]);
                    p.z = 0.5 * (p.z + (double)xyz[3 * j + 5]);
                }
                p.b *= T;
                p.tp = T * (1.0f - 0.5f * alpha) - pr;
                p.sq = 0.0f;
            }
            float gx = grad[3 * j], gy = grad[3 * j + 1], gz = grad[3 * j + 2];
            float inv = 1.0f / fmaxf(sqrtf(gx * gx + gy * gy + gz * gz), 1e-12f);
            p.nx = gx * inv;
            p.ny = gy * inv;
            p.nz = gz * inv;
            rec[j] = p;
            if (alpha_out) alpha_out[j] = alpha;
            if (trans_out) trans_out[j] = T;
        }
    }
}

hipError_t launch_render_prep(const RenderGeom& g, const float* xyz, const float* ray_w,
                              const float* pt_w, const float* sdf, const float* grad, const float* refl,
                              const float* phi_ray, int use_phi, float s, const float* log_s, float amp,
                              const float* amp_ptr, PtRec* rec, float* alpha_out, float* trans_out,
                              hipStream_t st) {
    const int waves_per_block = 4;
    dim3 grid((g.n_ray + waves_per_block - 1) / waves_per_block);
    hipLaunchKernelGGL(k_render_prep, grid, dim3(256), 0, st, g.n_ray, g.n_z, xyz, ray_w, pt_w, sdf,
                       grad, refl, phi_ray, use_phi, s, log_s, amp, amp_ptr, g.seg, rec, alpha_out, trans_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reduction over points: signal tracing forward (KIND 0) and matched-filter
// adjoint (KIND 1).  Lane t -> measurement i = t % n_meas, chunk c = t / n_meas;
// grid.y = point split.
// ---------------------------------------------------------------------------
// Seeds every kSeed frequencies: the walks run kSeed/2 steps each way; longer
// walks trade fewer seeds for rounding growth (16: 4.1e-5, 32: 5.7e-5, 64: 9.9e-5
// relative error of the 2^20-point signal against the FP64 reference).
constexpr int kSeed = 32;

template <int F, int KIND, int SPEC, bool NAIVE, bool BI>
__global__ __launch_bounds__(256) void k_reduce_points(
    int n_meas, int n_freq, int n_chunks, const AntRec* __restrict__ ant, const AntRec* __restrict__ rxa,
    double K0, double Kd,
    const void* __restrict__ recs_v, long n_pts, long pts_per_split, int n_split, int gx,
    float2* __restrict__ partial, const ChebPlan* __restrict__ sel) {
    if (sel && sel->K != 0) return;              // the Chebyshev path took this launch
    constexpr int S = F < kSeed ? F : kSeed;     // re-seed interval
    constexpr int NS = F / S;
    // point records of the block's split are staged through LDS in tiles of
    // TILE, shared by the 4 waves; the next tile is fetched into registers
    // while the current one is consumed
    constexpr int TILE = 64;
    constexpr int RB = KIND == 0 ? (int)sizeof(PtRec) : (int)sizeof(QRec);
    constexpr int V4 = TILE * RB / 16;           // float4 per tile (192 or 128)
    __shared__ float4 sRec[2][V4];
    // 1-D grid, XCD-aware: work-groups are dealt round-robin over the 8 XCDs
    // (id % 8), so the gx lane blocks of one point split get ids of one residue
    // mod 8 and read the split's records through one L2
    const long bid = blockIdx.x;
    const int lb = (int)((bid / 8) % gx);
    const long split = (bid / (8L * gx)) * 8 + (bid % 8);
    if (split >= n_split) return;                 // padding work-groups (whole block)
    const int t = lb * blockDim.x + threadIdx.x;
    int i = t % n_meas;
    int c = t / n_meas;
    const bool live_lane = c < n_chunks;
    if (!live_lane) c = n_chunks - 1;
    const AntRec A = ant[i];
    AntRec Rx = A;
    if constexpr (BI) Rx = rxa[i];
    double Kc[NS];                                // phase rate at each sub-chunk centre
#pragma unroll
    for (int m = 0; m < NS; ++m) Kc[m] = K0 + (double)(c * F + m * S + S / 2) * Kd;

    float ar[F], ai[F];
#pragma unroll
    for (int n = 0; n < F; ++n) {
        ar[n] = 0.0f;
        ai[n] = 0.0f;
    }
    const long j0 = split * pts_per_split;
    long j1 = j0 + pts_per_split;
    if (j1 > n_pts) j1 = n_pts;
    const float4* src = reinterpret_cast<const float4*>(recs_v);
    const int tid = threadIdx.x;
    // tile loader: element v of tile starting at jt (zero beyond j1)
    auto fetch = [&](long jt) {
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const long e = jt * (RB / 16) + tid;
        if (tid < V4 && e < j1 * (RB / 16)) v = src[e];
        return v;
    };
    float4 pre = fetch(j0);
    int buf = 0;
    for (long jt = j0; jt < j1; jt += TILE) {
        if (tid < V4) sRec[buf][tid] = pre;
        __syncthreads();
        if (jt + TILE < j1) pre = fetch(jt + TILE);
        const int cnt = (j1 - jt) < TILE ? (int)(j1 - jt) : TILE;
        for (int k = 0; k < cnt; ++k) {
            float wr, wi, cr, ci;          // step phasor, complex weight of the pair
            PairGeom g;
            if constexpr (KIND == 0 && !BI) {
                const PtRec P = reinterpret_cast<const PtRec*>(sRec[buf])[k];
                const double dx = P.x - A.x, dy = P.y - A.y, dz = P.z - A.z;
                g = pair_geom<NAIVE>(dx, dy, dz);
                float spec, live;
                if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
                    spec = 1.0f;
                } else {
                    float nd = (P.nx * (float)dx + P.ny * (float)dy + P.nz * (float)dz) * g.y;
                    spec_factor<SPEC>(nd, spec, live);
                }
                const float T = fminf(fmaxf(P.tp + A.phi, 0.0f), 1.0f);
                cr = P.b * spec * (T * (P.sq != 0.0f ? T : 1.0f)) * (g.y * g.y);
                ci = 0.0f;
            } else if constexpr (KIND == 0) {
                // bistatic (sample weight only): b spec T_tx T_rx / (r_t r_r)
                const PtRec P = reinterpret_cast<const PtRec*>(sRec[buf])[k];
                const double dx = P.x - A.x, dy = P.y - A.y, dz = P.z - A.z;
                const double ex = P.x - Rx.x, ey = P.y - Rx.y, ez = P.z - Rx.z;
                const BiGeom b = bi_geom<NAIVE>(dx, dy, dz, ex, ey, ez);
                g = b.g;
                float spec, live;
                if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
                    spec = 1.0f;
                } else {
                    const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
                    const float fex = (float)ex, fey = (float)ey, fez = (float)ez;
                    const float ni = (P.nx * fdx + P.ny * fdy + P.nz * fdz) * b.yt;
                    const float nr = -(P.nx * fex + P.ny * fey + P.nz * fez) * b.yr;
                    const float ir = -(fdx * fex + fdy * fey + fdz * fez) * (b.yt * b.yr);
                    spec_factor_bi<SPEC>(ni, nr, ir, spec, live);
                }
                const float Tt = fminf(fmaxf(P.tp + A.phi, 0.0f), 1.0f);
                const float Tr = fminf(fmaxf(P.tp + Rx.phi, 0.0f), 1.0f);
                cr = P.b * spec * (Tt * Tr) * (b.yt * b.yr);
                ci = 0.0f;
            } else {
                const QRec Q = reinterpret_cast<const QRec*>(sRec[buf])[k];
                const double dx = Q.x - A.x, dy = Q.y - A.y, dz = Q.z - A.z;
                if constexpr (BI) {
                    g = bi_geom<NAIVE>(dx, dy, dz, Q.x - Rx.x, Q.y - Rx.y, Q.z - Rx.z).g;
                } else {
                    g = pair_geom<NAIVE>(dx, dy, dz);
                }
                cr = Q.hr;
                ci = Q.hi;
            }
            {
                float cw, sw;
                step_phasor<NAIVE>(g, Kd, cw, sw);
                wr = cw;
                wi = -sw;                  // exp(-j 2 pi delta)
            }
#pragma unroll
            for (int m = 0; m < NS; ++m) {
                float c0, s0;
                seed_phasor<NAIVE>(g, Kc[m], c0, s0);
                // (cr + j ci) * exp(-j 2 pi theta_centre)
                const float pr0 = __builtin_fmaf(cr, c0, ci * s0);
                const float pi0 = __builtin_fmaf(ci, c0, -cr * s0);
                // three-term recurrence p_{n+1} = 2 cos(2 pi delta) p_n - p_{n-1}
                // (both parts), seeded with p_0 and p_{+-1} = p_0 w^{+-1}
                const float k2 = 2.0f * wr;
                {
                    float ar0 = pr0, ai0 = pi0;
                    float ar1 = __builtin_fmaf(pr0, wr, -pi0 * wi), ai1 = __builtin_fmaf(pr0, wi, pi0 * wr);
                    ar[m * S + S / 2] += ar0;
                    ai[m * S + S / 2] += ai0;
#pragma unroll
                    for (int u = S / 2 + 1; u < S; ++u) {
                        ar[m * S + u] += ar1;
                        ai[m * S + u] += ai1;
                        const float tr = __builtin_fmaf(k2, ar1, -ar0), ti = __builtin_fmaf(k2, ai1, -ai0);
                        ar0 = ar1; ai0 = ai1; ar1 = tr; ai1 = ti;
                    }
                    ar0 = pr0; ai0 = pi0;
                    ar1 = __builtin_fmaf(pr0, wr, pi0 * wi);
                    ai1 = __builtin_fmaf(pi0, wr, -pr0 * wi);
#pragma unroll
                    for (int u = S / 2 - 1; u >= 0; --u) {
                        ar[m * S + u] += ar1;
                        ai[m * S + u] += ai1;
                        const float tr = __builtin_fmaf(k2, ar1, -ar0), ti = __builtin_fmaf(k2, ai1, -ai0);
                        ar0 = ar1; ai0 = ai1; ar1 = tr; ai1 = ti;
                    }
                }
            }
        }
        __syncthreads();
        buf ^= 1;
    }
    if (live_lane) {
        float2* out = partial + ((size_t)split * n_meas + i) * n_freq + (size_t)c * F;
        const int nv = n_freq - c * F;
#pragma unroll
        for (int n = 0; n < F; ++n)
            if (n < nv) out[n] = make_float2(ar[n], ai[n]);
    }
}

template <int F, int KIND, int SPEC, bool NAIVE, bool BI>
static hipError_t launch_rp_bi(const RenderGeom& g, const AntRec* ant, const void* rec, int n_split,
                               float2* partial, const ChebPlan* sel, hipStream_t st) {
    const int n_chunks = (g.n_freq + F - 1) / F;
    const long lanes = (long)g.n_meas * n_chunks;
    const int gx = (int)((lanes + 255) / 256);
    const long groups = (n_split + 7) / 8;                // 8 splits per group, one per XCD
    dim3 grid((unsigned)(groups * 8 * gx));
    const long per = (g.n_pts + n_split - 1) / n_split;
    hipLaunchKernelGGL((k_reduce_points<F, KIND, SPEC, NAIVE, BI>), grid, dim3(256), 0, st, g.n_meas,
                       g.n_freq, n_chunks, ant, g.rxa, g.K0, g.Kd, rec, g.n_pts, per, n_split, gx, partial, sel);
    return hipGetLastError();
}

template <int F, int KIND, int SPEC, bool NAIVE>
static hipError_t launch_rp(const RenderGeom& g, const AntRec* ant, const void* rec, int n_split,
                            float2* partial, const ChebPlan* sel, hipStream_t st) {
    if (g.rxa) return launch_rp_bi<F, KIND, SPEC, NAIVE, true>(g, ant, rec, n_split, partial, sel, st);
    return launch_rp_bi<F, KIND, SPEC, NAIVE, false>(g, ant, rec, n_split, partial, sel, st);
}

template <int KIND, int SPEC, bool NAIVE>
static hipError_t launch_rp_f(const RenderGeom& g, const AntRec* ant, const void* rec, int n_split,
                              float2* partial, const ChebPlan* sel, hipStream_t st) {
    switch (freq_chunk(g.n_freq)) {
        case 16: return launch_rp<16, KIND, SPEC, NAIVE>(g, ant, rec, n_split, partial, sel, st);
        case 32: return launch_rp<32, KIND, SPEC, NAIVE>(g, ant, rec, n_split, partial, sel, st);
        default: return launch_rp<64, KIND, SPEC, NAIVE>(g, ant, rec, n_split, partial, sel, st);
    }
}

hipError_t launch_reduce_points_render(const RenderGeom& g, const AntRec* ant, const PtRec* rec,
                                       uint32_t flags, int n_split, float2* partial, const ChebPlan* sel,
                                       hipStream_t st) {
    const bool naive = (flags & RFVR_PHASE_NAIVE32) != 0;
    switch (flags & RFVR_SPEC_MASK) {
        case RFVR_SPEC_RAW:
            return naive ? launch_rp_f<0, RFVR_SPEC_RAW, true>(g, ant, rec, n_split, partial, sel, st)
                         : launch_rp_f<0, RFVR_SPEC_RAW, false>(g, ant, rec, n_split, partial, sel, st);
        case RFVR_SPEC_OFF:
            return naive ? launch_rp_f<0, RFVR_SPEC_OFF, true>(g, ant, rec, n_split, partial, sel, st)
                         : launch_rp_f<0, RFVR_SPEC_OFF, false>(g, ant, rec, n_split, partial, sel, st);
        default:
            return naive ? launch_rp_f<0, RFVR_SPEC_CLAMP, true>(g, ant, rec, n_split, partial, sel, st)
                         : launch_rp_f<0, RFVR_SPEC_CLAMP, false>(g, ant, rec, n_split, partial, sel, st);
    }
}

hipError_t launch_reduce_points_mf(const RenderGeom& g, const AntRec* ant, const QRec* rec,
                                   uint32_t flags, int n_split, float2* partial, const ChebPlan* sel,
                                   hipStream_t st) {
    const bool naive = (flags & RFVR_PHASE_NAIVE32) != 0;
    return naive ? launch_rp_f<1, RFVR_SPEC_OFF, true>(g, ant, rec, n_split, partial, sel, st)
                 : launch_rp_f<1, RFVR_SPEC_OFF, false>(g, ant, rec, n_split, partial, sel, st);
}

// fixed-order sum of split partials: out[o] (+)= sum_s partial[s][o]
__global__ void k_split_sum(const float2* __restrict__ partial, int n_split, long n_out,
                            int accumulate, float2* __restrict__ out, const ChebPlan* __restrict__ sel) {
    if (sel && sel->K != 0) return;
    long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_out) return;
    float sr = 0.0f, si = 0.0f;
    for (int s = 0; s < n_split; ++s) {
        float2 v = partial[(size_t)s * n_out + o];
        sr += v.x;
        si += v.y;
    }
    if (accumulate) {
        float2 p = out[o];
        sr += p.x;
        si += p.y;
    }
    out[o] = make_float2(sr, si);
}

hipError_t launch_split_sum(const float2* partial, int n_split, long n_out, int accumulate,
                            float2* out, const ChebPlan* sel, hipStream_t st) {
    hipLaunchKernelGGL(k_split_sum, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st,
                       partial, n_split, n_out, accumulate, out, sel);
    return hipGetLastError();
}

// zero-padded copy of a [n_meas][n_freq] complex array to [n_meas][np]
__global__ void k_pad_signal(const float2* __restrict__ sig, int n_meas, int n_freq, int np,
                             float2* __restrict__ out) {
    long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)n_meas * np) return;
    int i = (int)(o / np), n = (int)(o % np);
    out[o] = n < n_freq ? sig[(size_t)i * n_freq + n] : make_float2(0.0f, 0.0f);
}

hipError_t launch_pad_signal(const float2* sig, int n_meas, int n_freq, int np, float2* out,
                             hipStream_t st) {
    long n = (long)n_meas * np;
    hipLaunchKernelGGL(k_pad_signal, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sig,
                       n_meas, n_freq, np, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// signal tracing adjoint: one lane per point, Horner over the frequencies of
// each measurement's gradient row (scalar loads), chain rule per pair.
// ---------------------------------------------------------------------------
#ifndef RFVR_HORNER_PPL
#define RFVR_HORNER_PPL 1
#endif
constexpr int kBwdPPL = RFVR_HORNER_PPL;      // points per lane

template <int SPEC, bool NAIVE, bool BI>
__global__ __launch_bounds__(256) void k_render_bwd_points(
    long n_pts, const PtRec* __restrict__ rec, int n_meas, const AntRec* __restrict__ ant,
    const AntRec* __restrict__ rxa,
    const float2* __restrict__ gsig, int np, double K0, double Kd, float* __restrict__ g_b,
    float* __restrict__ g_T, float* __restrict__ g_n, const ChebPlan* __restrict__ sel) {
    if (sel && sel->K != 0) return;              // the Chebyshev path took this launch
    constexpr int PPL = kBwdPPL;
    const long j0 = (long)blockIdx.x * blockDim.x * PPL + threadIdx.x;
    PtRec P[PPL];
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        long j = j0 + (long)u * blockDim.x;
        P[u] = rec[j < n_pts ? j : n_pts - 1];
    }
    const int mid = np / 2;                        // multiple of 16
    const double Km = K0 + (double)mid * Kd;
    float gb[PPL], gt[PPL], gn0[PPL], gn1[PPL], gn2[PPL];
#pragma unroll
    for (int u = 0; u < PPL; ++u) gb[u] = gt[u] = gn0[u] = gn1[u] = gn2[u] = 0.0f;
    for (int i = 0; i < n_meas; ++i) {
        const AntRec A = ant[i];
        AntRec Rx = A;
        if constexpr (BI) Rx = rxa[i];
        PairGeom geo[PPL];
        float cw[PPL], sw[PPL], yr[PPL];
        double dx[PPL], dy[PPL], dz[PPL], ex[PPL], ey[PPL], ez[PPL];
#pragma unroll
        for (int u = 0; u < PPL; ++u) {
            dx[u] = P[u].x - A.x; dy[u] = P[u].y - A.y; dz[u] = P[u].z - A.z;
            if constexpr (BI) {
                ex[u] = P[u].x - Rx.x; ey[u] = P[u].y - Rx.y; ez[u] = P[u].z - Rx.z;
                const BiGeom b = bi_geom<NAIVE>(dx[u], dy[u], dz[u], ex[u], ey[u], ez[u]);
                geo[u] = b.g;
                geo[u].y = b.yt;                            // y holds 1/r_t here
                yr[u] = b.yr;
            } else {
                geo[u] = pair_geom<NAIVE>(dx[u], dy[u], dz[u]);
            }
            step_phasor<NAIVE>(geo[u], Kd, cw[u], sw[u]);       // w = exp(+j 2 pi delta)
        }
        const float2* g = gsig + (size_t)i * np;
        // H = sum_n g[n] w^(n - mid): upper half by Horner in w from the top,
        // lower half by Horner in conj(w) from the bottom
        float hr[PPL], hi[PPL], lr[PPL], li[PPL];
#pragma unroll
        for (int u = 0; u < PPL; ++u) hr[u] = hi[u] = lr[u] = li[u] = 0.0f;
        for (int n0 = np - 16; n0 >= mid; n0 -= 16) {
#pragma unroll
            for (int k = 15; k >= 0; --k) {
                const float2 gv = g[n0 + k];
#pragma unroll
                for (int u = 0; u < PPL; ++u) {
                    const float tr = __builtin_fmaf(-hi[u], sw[u], __builtin_fmaf(hr[u], cw[u], gv.x));
                    hi[u] = __builtin_fmaf(hi[u], cw[u], __builtin_fmaf(hr[u], sw[u], gv.y));
                    hr[u] = tr;
                }
            }
        }
        for (int n0 = 0; n0 < mid; n0 += 16) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const float2 gv = g[n0 + k];
#pragma unroll
                for (int u = 0; u < PPL; ++u) {
                    const float tr = __builtin_fmaf(li[u], sw[u], __builtin_fmaf(lr[u], cw[u], gv.x));
                    li[u] = __builtin_fmaf(li[u], cw[u], __builtin_fmaf(-lr[u], sw[u], gv.y));
                    lr[u] = tr;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < PPL; ++u) {
            // H = Hup + conj(w) * Hlow
            const float Hr = __builtin_fmaf(lr[u], cw[u], __builtin_fmaf(li[u], sw[u], hr[u]));
            const float Hi = __builtin_fmaf(li[u], cw[u], __builtin_fmaf(-lr[u], sw[u], hi[u]));
            float c0, s0;
            seed_phasor<NAIVE>(geo[u], Km, c0, s0);
            const float G = c0 * Hr - s0 * Hi;       // Re(exp(+j 2 pi theta_mid) H)
            const float y = geo[u].y;
            const float fdx = (float)dx[u], fdy = (float)dy[u], fdz = (float)dz[u];
            if constexpr (BI) {
                // c = b spec T_tx T_rx y_t y_r (sample weight)
                const float fex = (float)ex[u], fey = (float)ey[u], fez = (float)ez[u];
                float spec, live = 0.0f, ni = 0.0f, nr = 0.0f;
                if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
                    spec = 1.0f;
                } else {
                    ni = (P[u].nx * fdx + P[u].ny * fdy + P[u].nz * fdz) * y;
                    nr = -(P[u].nx * fex + P[u].ny * fey + P[u].nz * fez) * yr[u];
                    const float ir = -(fdx * fex + fdy * fey + fdz * fez) * (y * yr[u]);
                    spec_factor_bi<SPEC>(ni, nr, ir, spec, live);
                }
                const float Ut = P[u].tp + A.phi, Ur = P[u].tp + Rx.phi;
                const float Tt = fminf(fmaxf(Ut, 0.0f), 1.0f), Tr = fminf(fmaxf(Ur, 0.0f), 1.0f);
                const float mt = (Ut >= 0.0f && Ut <= 1.0f) ? 1.0f : 0.0f;
                const float mr = (Ur >= 0.0f && Ur <= 1.0f) ? 1.0f : 0.0f;
                const float T2 = Tt * Tr;
                const float gy = G * (y * yr[u]);
                gb[u] = __builtin_fmaf(gy * spec, T2, gb[u]);
                gt[u] = __builtin_fmaf(gy * P[u].b * spec, __builtin_fmaf(mt, Tr, Tt * mr), gt[u]);
                if constexpr (SPEC != (int)RFVR_SPEC_OFF) {
                    // d spec / d n_hat = -2 (nr w_i + ni w_r), w_i = d_t y_t, w_r = -d_r y_r
                    const float cb = -2.0f * gy * P[u].b * T2 * live;
                    const float ct = cb * (nr * y), cq = -cb * (ni * yr[u]);
                    gn0[u] = __builtin_fmaf(ct, fdx, __builtin_fmaf(cq, fex, gn0[u]));
                    gn1[u] = __builtin_fmaf(ct, fdy, __builtin_fmaf(cq, fey, gn1[u]));
                    gn2[u] = __builtin_fmaf(ct, fdz, __builtin_fmaf(cq, fez, gn2[u]));
                }
                continue;
            }
            float spec, live = 0.0f;
            float nd = 0.0f;
            if constexpr (SPEC == (int)RFVR_SPEC_OFF) {
                spec = 1.0f;
            } else {
                nd = (P[u].nx * fdx + P[u].ny * fdy + P[u].nz * fdz) * y;
                spec_factor<SPEC>(nd, spec, live);
            }
            const float Tr = P[u].tp + A.phi;
            const float T = fminf(fmaxf(Tr, 0.0f), 1.0f);
            const float mT = (Tr >= 0.0f && Tr <= 1.0f) ? 1.0f : 0.0f;
            // transmittance factor T^2 (sample weight) or T (segment weight)
            const bool sq = P[u].sq != 0.0f;
            const float Tf = T * (sq ? T : 1.0f);
            const float gy = G * (y * y);
            gb[u] = __builtin_fmaf(gy * spec, Tf, gb[u]);
            gt[u] = __builtin_fmaf(gy * P[u].b * spec, (sq ? 2.0f * T : 1.0f) * mT, gt[u]);
            if constexpr (SPEC != (int)RFVR_SPEC_OFF) {
                // d spec / d n_hat = 4 (n.w_i) w_i, w_i = d * y
                const float cn = gy * P[u].b * Tf * (4.0f * nd * y) * live;
                gn0[u] = __builtin_fmaf(cn, fdx, gn0[u]);
                gn1[u] = __builtin_fmaf(cn, fdy, gn1[u]);
                gn2[u] = __builtin_fmaf(cn, fdz, gn2[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        const long j = j0 + (long)u * blockDim.x;
        if (j >= n_pts) continue;
        g_b[j] = gb[u];
        g_T[j] = gt[u];
        g_n[3 * j] = gn0[u];
        g_n[3 * j + 1] = gn1[u];
        g_n[3 * j + 2] = gn2[u];
    }
}

template <int SPEC>
static hipError_t launch_rbp(const RenderGeom& g, const AntRec* ant, const PtRec* rec,
                             const float2* gsig, int np, bool naive, float* g_b, float* g_T,
                             float* g_n, const ChebPlan* sel, hipStream_t st) {
    dim3 grid((unsigned)((g.n_pts + 256L * kBwdPPL - 1) / (256L * kBwdPPL)));
#define RFVR_RBP(NV, BV)                                                                                    \
    hipLaunchKernelGGL((k_render_bwd_points<SPEC, NV, BV>), grid, dim3(256), 0, st, g.n_pts, rec, g.n_meas, \
                       ant, g.rxa, gsig, np, g.K0, g.Kd, g_b, g_T, g_n, sel)
    if (naive) {
        if (g.rxa) RFVR_RBP(true, true);
        else RFVR_RBP(true, false);
    } else {
        if (g.rxa) RFVR_RBP(false, true);
        else RFVR_RBP(false, false);
    }
#undef RFVR_RBP
    return hipGetLastError();
}

hipError_t launch_render_bwd_points(const RenderGeom& g, const AntRec* ant, const PtRec* rec,
                                    const float2* gsig_pad, int np, uint32_t flags, float* g_b,
                                    float* g_T, float* g_n, const ChebPlan* sel, hipStream_t st) {
    const bool naive = (flags & RFVR_PHASE_NAIVE32) != 0;
    switch (flags & RFVR_SPEC_MASK) {
        case RFVR_SPEC_RAW:
            return launch_rbp<RFVR_SPEC_RAW>(g, ant, rec, gsig_pad, np, naive, g_b, g_T, g_n, sel, st);
        case RFVR_SPEC_OFF:
            return launch_rbp<RFVR_SPEC_OFF>(g, ant, rec, gsig_pad, np, naive, g_b, g_T, g_n, sel, st);
        default:
            return launch_rbp<RFVR_SPEC_CLAMP>(g, ant, rec, gsig_pad, np, naive, g_b, g_T, g_n,
                                               sel, st);
    }
}

// ---------------------------------------------------------------------------
// adjoint of the per-ray scan: one wave per ray.
//   R_k = g_T[k+1] + (1 - alpha_{k+1}) R_{k+1}, R_{n_z-1} = 0  (suffix scan of
//   affine maps across the wave, chunks from the far end), g_alpha = direct -
//   T R; then alpha(Phi_k, Phi_{k+1}), Phi = sigmoid(s f), n_hat = g/|g|.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_adjoint(
    int n_ray, int n_z, const float* __restrict__ ray_w, const float* __restrict__ sdf,
    const float* __restrict__ grad, const float* __restrict__ refl, float s_h, const float* __restrict__ log_s,
    float amp_h, const float* __restrict__ amp_ptr, const float* __restrict__ alpha,
    const float* __restrict__ trans,
    const float* __restrict__ g_b, const float* __restrict__ g_T, const float* __restrict__ g_n,
    float* g_alpha_tmp, float* __restrict__ part_amp, float* __restrict__ part_s,
    float* __restrict__ g_sdf, float* __restrict__ g_grad, float* __restrict__ g_refl,
    int accumulate, int seg) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= n_ray) return;
    const int r = wave;
    const float amp = amp_ptr ? amp_ptr[0] : amp_h;
    const float s = log_s ? expf(log_s[0]) : s_h;
    const size_t base = (size_t)r * n_z;
    const float w = ray_w ? ray_w[r] : 1.0f;
    const int nch = (n_z + 63) / 64;
    float r_in = 0.0f, pamp = 0.0f, ps = 0.0f;
    for (int cc = nch - 1; cc >= 0; --cc) {
        const int k = cc * 64 + lane;
        float A = 0.0f, B = 0.0f;
        if (k + 1 < n_z) {
            const size_t jn = base + k + 1;
            A = 1.0f - alpha[jn];
            B = g_T[jn];
            // segment weight: g_T holds dL/dTbar, Tbar = T (1 - alpha/2), and b
            // carries T: dL/dT = dL/dTbar (1 - alpha/2) + dL/db A' w a alpha
            if (seg) B = __builtin_fmaf(g_b[jn] * amp * w * refl[jn], alpha[jn], B * (1.0f - 0.5f * alpha[jn]));
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const float A2 = __shfl_down(A, d, 64), B2 = __shfl_down(B, d, 64);
            if (lane + d < 64) {
                B = __builtin_fmaf(A, B2, B);
                A = A * A2;
            }
        }
        const float R = __builtin_fmaf(A, r_in, B);
        const float R0 = __shfl(R, 0, 64);
        if (k < n_z) {
            const size_t j = base + k;
            const float gb = g_b[j], al = alpha[j], a = refl[j], Tj = trans[j];
            // b = A' w a alpha (sample weight) or A' w a alpha T (segment
            // weight, whose Tbar = T (1 - alpha/2) adds -T/2 dL/dTbar)
            const float ta = seg ? al * Tj : al;
            const float direct = seg ? __builtin_fmaf(gb * amp * w * a, Tj, -0.5f * Tj * g_T[j]) : gb * amp * w * a;
            g_alpha_tmp[j] = direct - Tj * R;
            pamp = __builtin_fmaf(gb * w * a, ta, pamp);
            if (g_refl) {
                float v = gb * amp * w * ta;
                g_refl[j] = accumulate ? g_refl[j] + v : v;
            }
        }
        r_in = R0;
    }
    __threadfence();
    for (int cc = 0; cc < nch; ++cc) {
        const int k = cc * 64 + lane;
        if (k >= n_z) continue;
        const size_t j = base + k;
        const float fk = sdf[j];
        const float xk = s * fk;
        const float phik = sigmoidf_(xk);
        float gphi = 0.0f;
        if (k + 1 < n_z) {
            const float fnx = sdf[j + 1];
            if (xk >= s * fnx) {
                const float phin = sigmoidf_(s * fnx);
                const float D = phik + kAlphaEps;
                gphi += g_alpha_tmp[j] * (phin + kAlphaEps) / (D * D);
            }
        }
        if (k >= 1) {
            const float fp = sdf[j - 1];
            if (s * fp >= xk) gphi -= g_alpha_tmp[j - 1] / (sigmoidf_(s * fp) + kAlphaEps);
        }
        const float dens = phik * sigmoidf_(-xk);
        if (g_sdf) {
            float v = gphi * s * dens;
            g_sdf[j] = accumulate ? g_sdf[j] + v : v;
        }
        ps = __builtin_fmaf(gphi * fk, dens, ps);
        if (g_grad) {
            const float gx = grad[3 * j], gy = grad[3 * j + 1], gz = grad[3 * j + 2];
            const float nrm = sqrtf(gx * gx + gy * gy + gz * gz);
            const float n0 = g_n[3 * j], n1 = g_n[3 * j + 1], n2 = g_n[3 * j + 2];
            float o0, o1, o2;
            if (nrm >= 1e-12f) {
                const float inv = 1.0f / nrm;
                const float hx = gx * inv, hy = gy * inv, hz = gz * inv;
                const float dd = hx * n0 + hy * n1 + hz * n2;
                o0 = (n0 - hx * dd) * inv;
                o1 = (n1 - hy * dd) * inv;
                o2 = (n2 - hz * dd) * inv;
            } else {
                o0 = n0 * 1e12f;
                o1 = n1 * 1e12f;
                o2 = n2 * 1e12f;
            }
            if (accumulate) {
                o0 += g_grad[3 * j];
                o1 += g_grad[3 * j + 1];
                o2 += g_grad[3 * j + 2];
            }
            g_grad[3 * j] = o0;
            g_grad[3 * j + 1] = o1;
            g_grad[3 * j + 2] = o2;
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        pamp += __shfl_xor(pamp, d, 64);
        ps += __shfl_xor(ps, d, 64);
    }
    if (lane == 0) {
        part_amp[r] = pamp;
        part_s[r] = log_s ? ps * s : ps;            // dL/d(log s) = s dL/ds
    }
}

hipError_t launch_scan_adjoint(const RenderGeom& g, const float* ray_w, const float* sdf,
                               const float* grad, const float* refl, float s, const float* log_s, float amp,
                               const float* amp_ptr, const float* alpha, const float* trans,
                               const float* g_b, const float* g_T, const float* g_n,
                               float* g_alpha_tmp, float* part_amp, float* part_s, float* g_sdf,
                               float* g_grad, float* g_refl, int accumulate, hipStream_t st) {
    dim3 grid((g.n_ray + 3) / 4);
    hipLaunchKernelGGL(k_scan_adjoint, grid, dim3(256), 0, st, g.n_ray, g.n_z, ray_w, sdf, grad,
                       refl, s, log_s, amp, amp_ptr, alpha, trans, g_b, g_T, g_n, g_alpha_tmp, part_amp, part_s,
                       g_sdf, g_grad, g_refl, accumulate, g.seg);
    return hipGetLastError();
}

// deterministic sum of n floats into out[0] (one work-group, fixed order)
__global__ __launch_bounds__(256) void k_sum_scalars(const float* __restrict__ part, int n,
                                                     float* __restrict__ out, int accumulate) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) acc += (double)part[k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float v = (float)sh[0];
        out[0] = accumulate ? out[0] + v : v;
    }
}

hipError_t launch_sum_scalars(const float* part, int n, float* out, int accumulate,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_sum_scalars, dim3(1), dim3(256), 0, st, part, n, out, accumulate);
    return hipGetLastError();
}

}  // namespace rfvr
