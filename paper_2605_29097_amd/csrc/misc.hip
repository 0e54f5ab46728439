// Small bandwidth-bound kernels: L2 heatmap loss, lensless primary-ray
// sampling and the AdamW update.
#include "rfvr_impl.hpp"

namespace rfvr {

// ---------------------------------------------------------------------------
// loss (Sec. Overview step 5): per-block FP64 partial sums, fixed-order final
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss_partial(long n, const float* __restrict__ p,
                                                      const float* __restrict__ ps,
                                                      const float* __restrict__ mask,
                                                      float* __restrict__ g_p,
                                                      double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    const float inv_n2 = (float)(2.0 / (double)n);
    for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < n; q += (long)gridDim.x * 256) {
        const float m = mask ? mask[q] : 1.0f;
        const float d = p[q] - ps[q];
        acc += (double)(m * d) * (double)d;
        if (g_p) g_p[q] = inv_n2 * m * d;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, int nb,
                                                    long n, float* __restrict__ loss) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nb; k += 256) acc += part[k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(sh[0] / (double)n);
}

hipError_t launch_loss_partial(long n, const float* p, const float* ps, const float* mask,
                               float* g_p, double* part, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_loss_partial, dim3(n_blocks), dim3(256), 0, st, n, p, ps, mask, g_p, part);
    return hipGetLastError();
}

hipError_t launch_loss_final(const double* part, int n_blocks, long n, float* loss,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, part, n_blocks, n, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// lensless primary-ray sampling (Sec. Lensless Sampling, Primary Ray)
// counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): k-th output from
// state x is mix(x + (k+1) * 0x9E3779B97F4A7C15).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sm64_output(uint64_t state, uint64_t k) {
    return sm64_mix(state + (k + 1ull) * 0x9E3779B97F4A7C15ull);
}

struct SampleArgs {
    double e1[3], e2[3], w[3];
    double base[3];      // centre projected onto the aperture plane
    double lo;           // c.w - h
    double h;
    double off;          // aperture plane offset along w (ray origins)
    int n_rx, n_ry, n_z, mode;
    uint64_t key;        // per-step stream key
};

__global__ void k_sample_points(SampleArgs a, float* __restrict__ xyz, float* __restrict__ u_out,
                                float* __restrict__ origin) {
    const long n_ray = (long)a.n_rx * a.n_ry;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ray * a.n_z) return;
    const long r = t / a.n_z;
    const int k = (int)(t % a.n_z);
    const int ix = (int)(r % a.n_rx), iy = (int)(r / a.n_rx);
    const double lx = -a.h + (ix + 0.5) * 2.0 * a.h / a.n_rx;
    const double ly = -a.h + (iy + 0.5) * 2.0 * a.h / a.n_ry;
    double o[3];
    for (int c = 0; c < 3; ++c) o[c] = a.base[c] + lx * a.e1[c] + ly * a.e2[c];
    double frac = 0.5;
    if (a.mode == RFVR_SAMPLE_STRATIFIED) {
        const uint64_t v = sm64_output(a.key, (uint64_t)t);
        frac = (double)(v >> 40) * (1.0 / 16777216.0);
    }
    const double u = a.lo + ((double)k + frac) * (2.0 * a.h / a.n_z);
    for (int c = 0; c < 3; ++c) xyz[3 * t + c] = (float)(o[c] + u * a.w[c]);
    if (u_out) u_out[t] = (float)u;
    if (origin && k == 0)
        for (int c = 0; c < 3; ++c) origin[3 * r + c] = (float)(o[c] + a.off * a.w[c]);
}

hipError_t launch_sample_points(const rfvr_sample_desc& d, const double basis[9], float* xyz,
                                float* u, float* origin, hipStream_t st) {
    SampleArgs a;
    for (int c = 0; c < 3; ++c) {
        a.e1[c] = basis[c];
        a.e2[c] = basis[3 + c];
        a.w[c] = basis[6 + c];
    }
    const double cx = d.centre[0], cy = d.centre[1], cz = d.centre[2];
    const double cw = cx * a.w[0] + cy * a.w[1] + cz * a.w[2];
    a.base[0] = cx - cw * a.w[0];
    a.base[1] = cy - cw * a.w[1];
    a.base[2] = cz - cw * a.w[2];
    a.h = d.half_extent;
    a.off = d.plane_offset;
    a.lo = cw - a.h;
    a.n_rx = d.n_ray_x;
    a.n_ry = d.n_ray_y;
    a.n_z = d.n_z;
    a.mode = d.mode;
    // host copy of the same generator for the per-step key
    auto mix = [](uint64_t z) {
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    a.key = mix(d.seed + (d.step + 1ull) * 0x9E3779B97F4A7C15ull);
    const long n = (long)d.n_ray_x * d.n_ray_y * d.n_z;
    hipLaunchKernelGGL(k_sample_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a,
                       xyz, u, origin);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// AdamW (Loshchilov & Hutter): bc1 = 1 - b1^t, bc2 = 1 - b2^t
// ---------------------------------------------------------------------------
__global__ void k_adamw(long n, float* __restrict__ p, const float* __restrict__ g,
                        float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                        float eps, float wd, float bc1, float bc2) {
    long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float upd = (mk / bc1) / (sqrtf(vk / bc2) + eps) + wd * p[k];
    p[k] = p[k] - lr * upd;
}

hipError_t launch_adamw(long n, float* p, const float* g, float* m, float* v, float lr, float b1,
                        float b2, float eps, float wd, float bc1, float bc2, hipStream_t st) {
    hipLaunchKernelGGL(k_adamw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, m, v,
                       lr, b1, b2, eps, wd, bc1, bc2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// importance sampling from the proposal's bin logits: one wave per ray, lane b
// holds bin b (CDF by a wave scan); slot j = s*64 + lane sits in register s of
// its lane (S registers cover up to 64*S slots), and ranks sort in place
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(256) void k_sample_importance(SampleArgs a, const float* __restrict__ logits,
                                                           int n_bins, int n_imp, int n_uni,
                                                           float* __restrict__ xyz, float* __restrict__ u_out,
                                                           float* __restrict__ origin) {
    const long n_ray = (long)a.n_rx * a.n_ry;
    const long r = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= n_ray) return;                                    // uniform per wave
    const int ix = (int)(r % a.n_rx), iy = (int)(r / a.n_rx);
    const double lx = -a.h + (ix + 0.5) * 2.0 * a.h / a.n_rx;
    const double ly = -a.h + (iy + 0.5) * 2.0 * a.h / a.n_ry;
    double o[3];
    for (int c = 0; c < 3; ++c) o[c] = a.base[c] + lx * a.e1[c] + ly * a.e2[c];
    const double lo = a.lo, hi = a.lo + 2.0 * a.h;
    // pdf and inclusive CDF over the bins, in FP64 so that the bin each level
    // falls in is decided as a double-precision evaluation decides it
    double p = 0.0;
    if (lane < n_bins) p = 1.0 / (1.0 + exp(-(double)logits[r * n_bins + lane])) + 1e-3;
    double cdf = p;
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(cdf, d, 64);
        if (lane >= d) cdf += t;
    }
    const double total = __shfl(cdf, n_bins - 1, 64);
    p /= total;
    cdf /= total;
    const int K = n_uni + n_imp;
    double u[S], v[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = s * 64 + lane;
        u[s] = hi + 1.0;                                       // slots >= K sort last
        v[s] = 0.0;
        if (j < K) {
            // mode 0: every slot at the middle of its stratum; else drawn
            const uint64_t v64 = sm64_output(a.key, (uint64_t)(r * K + j));
            const double xi = a.mode == 0 ? 0.5 : (double)(v64 >> 40) * (1.0 / 16777216.0);
            if (j < n_uni) u[s] = lo + ((double)j + xi) * (hi - lo) / n_uni;
            else v[s] = ((double)(j - n_uni) + xi) / n_imp;
        }
    }
    // inverse CDF for importance slots: bin = number of CDF values <= v
    int b[S];
#pragma unroll
    for (int s = 0; s < S; ++s) b[s] = 0;
    for (int q = 0; q < n_bins; ++q) {
        const double c = __shfl(cdf, q, 64);
#pragma unroll
        for (int s = 0; s < S; ++s) b[s] += (c <= v[s]) ? 1 : 0;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = s * 64 + lane;
        const int bs = b[s] > n_bins - 1 ? n_bins - 1 : b[s];
        const double below = __shfl(cdf, bs > 0 ? bs - 1 : 0, 64);   // all lanes shuffle
        const double prev = bs > 0 ? below : 0.0;
        const double pb = __shfl(p, bs, 64);
        const double frac = fmin(fmax((v[s] - prev) / pb, 0.0), 1.0);
        if (j >= n_uni && j < K) u[s] = lo + ((double)bs + frac) * ((hi - lo) / n_bins);
    }
    // rank = number of slots before this one in (u, slot) order
    int rank[S];
#pragma unroll
    for (int s = 0; s < S; ++s) rank[s] = 0;
#pragma unroll
    for (int s2 = 0; s2 < S; ++s2) {
        for (int l = 0; l < 64; ++l) {
            const int t = s2 * 64 + l;
            if (t >= K) break;                                 // uniform
            const double ut = __shfl(u[s2], l, 64);
#pragma unroll
            for (int s = 0; s < S; ++s)
                rank[s] += (ut < u[s] || (ut == u[s] && t < s * 64 + lane)) ? 1 : 0;
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = s * 64 + lane;
        if (j < K) {
            const long o_j = r * K + rank[s];
            for (int c = 0; c < 3; ++c) xyz[3 * o_j + c] = (float)(o[c] + u[s] * a.w[c]);
            if (u_out) u_out[o_j] = (float)u[s];
        }
    }
    if (origin && lane < 3) origin[3 * r + lane] = (float)(o[lane] + a.off * a.w[lane]);
}

hipError_t launch_sample_importance(const rfvr_sample_desc& d, const double basis[9], const float* logits,
                                    int n_bins, int n_imp, int n_uni, float* xyz, float* u, float* origin,
                                    hipStream_t st) {
    SampleArgs a;
    for (int c = 0; c < 3; ++c) {
        a.e1[c] = basis[c];
        a.e2[c] = basis[3 + c];
        a.w[c] = basis[6 + c];
    }
    const double cx = d.centre[0], cy = d.centre[1], cz = d.centre[2];
    const double cw = cx * a.w[0] + cy * a.w[1] + cz * a.w[2];
    a.base[0] = cx - cw * a.w[0];
    a.base[1] = cy - cw * a.w[1];
    a.base[2] = cz - cw * a.w[2];
    a.h = d.half_extent;
    a.off = d.plane_offset;
    a.lo = cw - a.h;
    a.n_rx = d.n_ray_x;
    a.n_ry = d.n_ray_y;
    a.n_z = n_imp + n_uni;
    a.mode = d.mode == RFVR_SAMPLE_GRID ? 0 : 2;      // 0: fixed mid-stratum levels, 2: drawn
    auto mix = [](uint64_t z) {
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    a.key = mix(d.seed + (d.step + 1ull) * 0x9E3779B97F4A7C15ull);
    const long n_ray = (long)d.n_ray_x * d.n_ray_y;
    const dim3 grid((unsigned)((n_ray + 3) / 4));
    const int K = n_imp + n_uni;
    if (K <= 64)
        hipLaunchKernelGGL(k_sample_importance<1>, grid, dim3(256), 0, st, a, logits, n_bins, n_imp, n_uni, xyz, u, origin);
    else if (K <= 128)
        hipLaunchKernelGGL(k_sample_importance<2>, grid, dim3(256), 0, st, a, logits, n_bins, n_imp, n_uni, xyz, u, origin);
    else if (K <= 256)
        hipLaunchKernelGGL(k_sample_importance<4>, grid, dim3(256), 0, st, a, logits, n_bins, n_imp, n_uni, xyz, u, origin);
    else if (K <= 512)
        hipLaunchKernelGGL(k_sample_importance<8>, grid, dim3(256), 0, st, a, logits, n_bins, n_imp, n_uni, xyz, u, origin);
    else                                                       // K <= RFVR_MAX_RAY_SAMPLES = 1024
        hipLaunchKernelGGL(k_sample_importance<16>, grid, dim3(256), 0, st, a, logits, n_bins, n_imp, n_uni, xyz, u, origin);
    return hipGetLastError();
}

// per-antenna sampling: rays from each antenna through the lateral grid on the
// plane through the cube centre, samples at the cell centres of the ray's
// segment between the cube's two planes normal to w; volume Jacobian
// (dist / dist to the grid point)^2 relative to a lensless cell
__global__ void k_sample_naive(SampleArgs a, const float* __restrict__ tx, int n_ant,
                               float* __restrict__ xyz, float* __restrict__ jac) {
    const long n_ray = (long)a.n_rx * a.n_ry;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)n_ant * n_ray * a.n_z) return;
    const int k = (int)(t % a.n_z);
    const long r = (t / a.n_z) % n_ray;
    const int i = (int)(t / ((long)a.n_z * n_ray));
    const int ix = (int)(r % a.n_rx), iy = (int)(r / a.n_rx);
    const double lx = -a.h + (ix + 0.5) * 2.0 * a.h / a.n_rx;
    const double ly = -a.h + (iy + 0.5) * 2.0 * a.h / a.n_ry;
    double p[3], d[3];
    for (int q = 0; q < 3; ++q) {
        p[q] = (double)tx[3 * i + q];
        d[q] = a.base[q] + lx * a.e1[q] + ly * a.e2[q] - p[q];      // base: the cube centre
    }
    const double rc = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int q = 0; q < 3; ++q) d[q] /= rc;
    const double cw = d[0] * a.w[0] + d[1] * a.w[1] + d[2] * a.w[2];        // cos of the ray to w
    const double pw = p[0] * a.w[0] + p[1] * a.w[1] + p[2] * a.w[2];
    const double s_in = (a.lo - pw) / cw, s_out = (a.lo + 2.0 * a.h - pw) / cw;
    const double dist = s_in + ((double)k + 0.5) * (s_out - s_in) / a.n_z;
    for (int q = 0; q < 3; ++q) xyz[3 * t + q] = (float)(p[q] + dist * d[q]);
    if (jac) jac[t] = (float)((dist / rc) * (dist / rc));
}

hipError_t launch_sample_naive(const rfvr_sample_desc& d, const double basis[9], const float* tx, int n_ant,
                               float* xyz, float* jac, hipStream_t st) {
    SampleArgs a;
    for (int c = 0; c < 3; ++c) {
        a.e1[c] = basis[c];
        a.e2[c] = basis[3 + c];
        a.w[c] = basis[6 + c];
    }
    const double cx = d.centre[0], cy = d.centre[1], cz = d.centre[2];
    const double cw = cx * a.w[0] + cy * a.w[1] + cz * a.w[2];
    a.h = d.half_extent;
    a.lo = cw - a.h;
    a.n_rx = d.n_ray_x;
    a.n_ry = d.n_ray_y;
    a.n_z = d.n_z;
    a.mode = 0;
    a.off = 0.0;
    a.key = 0;
    // the lateral grid is centred on the cube centre (held in base)
    a.base[0] = cx;
    a.base[1] = cy;
    a.base[2] = cz;
    const long n = (long)n_ant * d.n_ray_x * d.n_ray_y * d.n_z;
    hipLaunchKernelGGL(k_sample_naive, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, tx, n_ant,
                       xyz, jac);
    return hipGetLastError();
}

// proposal targets: the blend weight T alpha of sample k is the opacity of the
// segment [u_k, u_{k+1}] it covers, spread over the bins the segment overlaps
// in proportion to the overlap (the last sample and zero-length segments: the
// bin of u_k); then normalised by the ray's largest bin.  One wave per ray,
// lane b owns bin b and walks the ray's segments in order, in FP64 (the
// operations and their order are those of a double-precision reference).
__global__ __launch_bounds__(256) void k_proposal_targets(int n_ray, int n_k, const float* __restrict__ u,
                                                          const float* __restrict__ alpha,
                                                          const float* __restrict__ trans, float lo, float hi,
                                                          int n_bins, int n_dilate, float* __restrict__ targets) {
    const long r = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= n_ray) return;
    const double dlo = lo, span = (double)hi - (double)lo;
    const double e0 = dlo + span * (double)lane / (double)n_bins;
    const double e1 = dlo + span * (double)(lane + 1) / (double)n_bins;
    const float* ur = u + r * n_k;
    const float* tr = trans + r * n_k;
    const float* ar = alpha + r * n_k;
    double W = 0.0;
    for (int k = 0; k < n_k; ++k) {                            // uniform trip count
        const double a = (double)ur[k];
        const double e = k + 1 < n_k ? (double)ur[k + 1] : a;
        const double w = (double)(tr[k] * ar[k]);
        if (e > a) {
            const double ov = fmin(e, e1) - fmax(a, e0);
            if (ov > 0.0) W += w * ov / (e - a);
        } else {
            int b = (int)floor((a - dlo) / span * (double)n_bins);
            b = b < 0 ? 0 : (b > n_bins - 1 ? n_bins - 1 : b);
            if (b == lane) W += w;
        }
    }
    const float Wf = (float)W;
    float mx = lane < n_bins ? Wf : 0.0f;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d, 64));
    const float t = fminf(1.0f, Wf / fmaxf(mx, 1e-3f));
    // depth dilation: the largest t of the bin and the n_dilate bins in front
    float td = t;
    for (int d = 1; d <= n_dilate; ++d) {                     // uniform trip count
        const float v = __shfl_up(t, d, 64);
        if (lane >= d) td = fmaxf(td, v);
    }
    if (lane < n_bins) targets[r * n_bins + lane] = td;
}

hipError_t launch_proposal_targets(int n_ray, int n_k, const float* u, const float* alpha, const float* trans,
                                   float lo, float hi, int n_bins, int n_dilate, float* targets, hipStream_t st) {
    const dim3 grid((unsigned)((n_ray + 3) / 4));
    hipLaunchKernelGGL(k_proposal_targets, grid, dim3(256), 0, st, n_ray, n_k, u, alpha, trans, lo, hi, n_bins,
                       n_dilate, targets);
    return hipGetLastError();
}

// BCE: per-block FP64 partials, fixed-order final
__global__ __launch_bounds__(256) void k_bce_partial(long n, const float* __restrict__ z, const float* __restrict__ t,
                                                     float* __restrict__ g, double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    const float inv_n = (float)(1.0 / (double)n);
    for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < n; q += (long)gridDim.x * 256) {
        const float zq = z[q], tq = t[q];
        const float spn = fmaxf(-zq, 0.0f) + log1pf(expf(-fabsf(zq)));   // softplus(-z)
        const float spp = spn + zq;                                       // softplus(z)
        acc += (double)(tq * spn + (1.0f - tq) * spp);
        if (g) g[q] = (sigmoidf_(zq) - tq) * inv_n;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

hipError_t launch_bce(long n, const float* z, const float* t, float* loss, float* g, double* part, int nb,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_bce_partial, dim3(nb), dim3(256), 0, st, n, z, t, g, part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, part, nb, n, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dynamic loss masking: peak of the reference heatmap, then mask and history
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_max_partial(long n, const float* __restrict__ x,
                                                     float* __restrict__ part) {
    __shared__ float sh[256];
    float m = 0.0f;
    for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < n; q += (long)gridDim.x * 256) m = fmaxf(m, x[q]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + d]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_max_final(const float* __restrict__ part, int nb,
                                                   float* __restrict__ out) {
    __shared__ float sh[256];
    float m = 0.0f;
    for (int k = threadIdx.x; k < nb; k += 256) m = fmaxf(m, part[k]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + d]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ __launch_bounds__(256) void k_mask_update(long n, const float* __restrict__ p,
                                                     float* __restrict__ hist, const float* __restrict__ peak,
                                                     float tau_hi, float tau_lo, float* __restrict__ mask) {
    const long q = (long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const float hi = __fmul_rn(tau_hi, peak[0]);
    const float h = hist[q], pq = p[q];
    const bool drop = (h >= hi) && (pq < __fmul_rn(tau_lo, h));
    mask[q] = drop ? 0.0f : 1.0f;
    hist[q] = fmaxf(h, pq);
}

hipError_t launch_mask_update(long n, const float* p, const float* p_ref, float* hist, float tau_hi,
                              float tau_lo, float* mask, float* part, int nb, hipStream_t st) {
    hipLaunchKernelGGL(k_max_partial, dim3(nb), dim3(256), 0, st, n, p_ref, part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, st, part, nb, part + nb);
    hipLaunchKernelGGL(k_mask_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, hist,
                       part + nb, tau_hi, tau_lo, mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// occupancy Phi = sigmoid(s f)
// ---------------------------------------------------------------------------
__global__ void k_occupancy(long n, float s_h, const float* __restrict__ log_s, const float* __restrict__ f,
                            float* __restrict__ phi) {
    const float s = log_s ? expf(log_s[0]) : s_h;
    long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) phi[k] = sigmoidf_(s * f[k]);
}

hipError_t launch_occupancy(long n, float s, const float* log_s, const float* f, float* phi, hipStream_t st) {
    hipLaunchKernelGGL(k_occupancy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, s, log_s, f, phi);
    return hipGetLastError();
}

}  // namespace rfvr
