/*
 * rfvr.h -- C ABI of librfvr, an MI355X (gfx950) implementation of lensless RF
 * volumetric rendering: GeRaF, "Neural Geometry Reconstruction from Radio
 * Frequency Signals" (arXiv 2605.29097).
 *
 * Conventions (all entry points)
 * ------------------------------
 * - Array pointers are DEVICE pointers into caller-owned, C-contiguous memory,
 *   unless marked "host".  Descriptors are host structs read during the call
 *   and not retained.  Complex arrays are interleaved {re, im} float pairs.
 * - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *   stream).  Every call only enqueues work on that stream; no call blocks the
 *   host.  Kernel-time faults surface at the caller's next synchronisation.
 * - `ws` / `ws_bytes`: device workspace owned by the caller, at least the size
 *   returned by the matching rfvr_*_ws_bytes() query, 256-byte aligned.  Its
 *   contents are scratch on entry and on exit.
 * - Return value: RFVR_OK, or a negative code.  All argument checks happen
 *   before anything is enqueued, so a failed call has enqueued nothing.
 *   rfvr_last_error() returns a thread-local message for the last failure.
 * - Outputs are overwritten, except gradient outputs when `flags` contains
 *   RFVR_ACCUMULATE, which then add into the existing contents.
 * - Reductions use a fixed split and a fixed summation order and no floating
 *   point atomics: results are bitwise reproducible for fixed shapes.
 * - NaN/Inf inside arrays propagate; only descriptor scalars are checked.
 *
 * Notation: i = measurement (a transmitter and its receiver: the same antenna
 * for a monostatic aperture, rx = NULL), n = frequency with
 * f_n = f0 + n*df, j = sample point laid out [n_ray][n_z] along primary rays
 * (depth u ascending), c = 299792458 m/s.
 */
#ifndef RFVR_H
#define RFVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RFVR_OK             0
#define RFVR_E_INVALID     -1   /* bad size, NULL required pointer, non-finite scalar */
#define RFVR_E_WORKSPACE   -2   /* ws NULL or ws_bytes below the query              */
#define RFVR_E_UNSUPPORTED -3   /* valid arguments, combination not provided        */
#define RFVR_E_HIP         -4   /* HIP launch / runtime error                       */

/* Size limits of one call: at most RFVR_MAX_POINTS points (samples, query
 * points, network inputs, elements of the per-point calls; for the per-antenna
 * sampler antennas x rays x depths), RFVR_MAX_RAYS primary rays and
 * RFVR_MAX_MEAS measurements, so that every launch stays well inside the 2^32
 * work-items of a one-dimensional grid (one wave per ray in the per-ray
 * kernels).  Larger inputs are split by the caller; a call beyond a limit
 * returns RFVR_E_INVALID and a workspace query returns 0. */
#define RFVR_MAX_POINTS 2147483647LL  /* 2^31 - 1 */
#define RFVR_MAX_RAYS   33554432      /* 2^25     */
#define RFVR_MAX_MEAS   1048576       /* 2^20     */

/* flags */
#define RFVR_SPEC_CLAMP     0x0u  /* specular factor max(0, w_o . w_r)   (default)  */
#define RFVR_SPEC_RAW       0x1u  /* w_o . w_r                                       */
#define RFVR_SPEC_OFF       0x2u  /* factor 1 (the paper's "without radar physics") */
#define RFVR_SPEC_MASK      0x3u
#define RFVR_PHASE_FP64RR   0x0u  /* path length and phase reduction in FP64 (default) */
#define RFVR_PHASE_NAIVE32  0x4u  /* radians 2 pi f d / c formed in FP32 (precision study) */
#define RFVR_ACCUMULATE     0x8u  /* gradient outputs add into existing contents   */
#define RFVR_TERMS_DIRECT   0x10u /* per-frequency evaluation of the term sums (see below) */
#define RFVR_WEIGHT_SEGMENT 0x20u /* render: each sample's segment weighted by the exact
                                     integral of T^2 rho over it, placed at its midpoint
                                     (see the render section) */

/* Evaluation of the term sums (Eq. ref_sim, Eq. mf-sm and their adjoints).
 * By default the four term entry points (render forward / backward, matched
 * filter forward / backward) evaluate the sums through Chebyshev moments of
 * each measurement's range interval over the launch's bounding box: the
 * phasor exp(-+j 2 pi (f0 + n df) 2r/c) is split at the centre of the band
 * and its offset from there, exp(-+j 2 pi (n - (n_freq-1)/2) df 2r/c), is
 * expanded in Chebyshev polynomials of the normalised range (Jacobi-Anger
 * expansion), cut at the smallest order K in {24, 28, 32, 40, 48, 64} whose
 * truncation bound 2 (z/2)^K / K! / (1 - z/(2K+2)) (z = 2 pi
 * ((n_freq - 1)/2) df 2h/c, h the half-width of the widest interval) is below
 * 1e-6 of the sum of the term magnitudes.  The choice is made on the device
 * for every call; when no K qualifies (a range spread too wide for the band)
 * or K is not below n_freq, the per-frequency kernels run, which
 * RFVR_TERMS_DIRECT (and RFVR_PHASE_NAIVE32) also select.  Both evaluate the
 * same sums; they differ by rounding. */


/* Measurement geometry and FMCW sweep (Sec. "Radar Basics", Eq. fmcw; App. C). */
typedef struct rfvr_aperture {
    int32_t      n_meas;   /* number of (tx, rx) measurements, >= 1             */
    const float* tx;       /* [n_meas][3] transmitter positions, metres         */
    const float* rx;       /* [n_meas][3] receiver positions (bistatic), or NULL
                              (monostatic, rx = tx); see the render below       */
    double       f0_hz;    /* first sweep frequency                              */
    double       df_hz;    /* frequency step                                     */
    int32_t      n_freq;   /* >= 1                                               */
} rfvr_aperture;

/* Lensless sample set (Sec. "Lensless Sampling", Primary Ray). */
typedef struct rfvr_samples {
    int32_t      n_ray, n_z;   /* >= 1 each                                          */
    const float* xyz;          /* [n_ray][n_z][3] points, depth ascending per ray    */
    const float* ray_weight;   /* [n_ray] Monte-Carlo weight w_r, or NULL (= 1)      */
    const float* point_weight; /* [n_ray*n_z] volume weight per sample multiplying its
                                  amplitude, or NULL (= 1); rfvr_render_forward only
                                  (the per-antenna renderer's Jacobian)            */
} rfvr_samples;

/* Per-point fields of the current scene estimate (Sec. "Opaque density
 * representation", "Signal representation"). */
typedef struct rfvr_fields {
    const float* sdf;      /* [n_ray*n_z] signed distance f, metres                  */
    const float* grad;     /* [n_ray*n_z][3] grad_x f (normal before normalising)    */
    const float* refl;     /* [n_ray*n_z] reflectiveness a                           */
    const float* phi_ray;  /* [n_ray] Phi_s(f) at primary-ray origins, detached; or NULL */
    const float* phi_tx;   /* [n_meas] Phi_s(f) at transmitters, detached; or NULL   */
    const float* phi_rx;   /* [n_meas] Phi_s(f) at receivers, detached: with a bistatic
                              aperture, given exactly when phi_ray and phi_tx are;
                              NULL for a monostatic one (else RFVR_E_INVALID)     */
    float        s;        /* logistic sharpness (1/m), finite, > 0                  */
    float        amp_tx;   /* learnt global amplitude A'_tx, finite                  */
    const float* amp_ptr;  /* device [1] or NULL; when set, A'_tx is read from device
                              memory at kernel time (no host round trip per step)   */
    const float* log_s_ptr;/* device [1] or NULL; when set, s = exp(log_s_ptr[0]) is read
                              at kernel time (the field s is then unused but must still
                              be finite and > 0) and rfvr_render_backward's g_s output
                              is dL/d(log s) = s dL/ds: a log-parameterised learnable s
                              updated on the device (rfvr_adamw) with no host round trip */
} rfvr_fields;

/* ------------------------------------------------------------------------
 * Render (signal tracing with lensless alpha blending)
 *
 * Computes, for every measurement i and frequency n (Eq. ref_sim with the
 * amplitude of Eq. signal_amp_tracing and Eq. reflection_angle):
 *   Phi_k  = 1 / (1 + exp(-s f_k))                         per ray
 *   alpha_k = clamp((Phi_k - Phi_{k+1}) / (Phi_k + 1e-5), 0, 1), alpha_{n_z-1} = 0
 *                                            (NeuS discretisation, Sec. Discretization)
 *   T_k    = prod_{m<k} (1 - alpha_m)
 *   T'_ik  = clamp(T_k + phi_tx[i] - phi_ray[r], 0, 1)     (Eq. lens-less-transmittance;
 *            T'_ik = T_k when phi_tx or phi_ray is NULL)
 *   c_ij   = A' w_r a_j alpha_j T'^2 spec_ij / r_ij^2,  r_ij = |x_j - tx_i|,
 *            spec = 2 (n_hat . w_i)^2 - 1 (monostatic w_o . w_r), see RFVR_SPEC_*
 *   s[i,n] = sum_j c_ij exp(-j 2 pi f_n 2 r_ij / c)
 * A bistatic aperture (rx != NULL; Eq. signal_amp_tracing with separate
 * antennas, App. A, Radar Reflections) takes the path tx_i -> x_j -> rx_i:
 *   c_ij   = A' w_r a_j alpha_j T'tx_ij T'rx_ij spec_ij / (rt_ij rr_ij),
 *   rt = |x_j - tx_i|, rr = |rx_i - x_j|, w_i = (x_j - tx_i)/rt, w_r = (rx_i - x_j)/rr,
 *   spec = w_o . w_r = w_i . w_r - 2 (n_hat . w_i)(n_hat . w_r),
 *   T'tx as T' above, T'rx = clamp(T_k + phi_rx[i] - phi_ray[r], 0, 1),
 *   s[i,n] = sum_j c_ij exp(-j 2 pi f_n (rt_ij + rr_ij) / c);
 * with rx = tx it equals the monostatic render.  RFVR_WEIGHT_SEGMENT is defined
 * for monostatic apertures only (RFVR_E_UNSUPPORTED otherwise).
 * With RFVR_WEIGHT_SEGMENT, sample j instead stands for the segment from it to
 * the next sample of its ray: the weight alpha_j T'^2 becomes the exact
 * integral of the round-trip weight T(u)^2 rho(u) over that segment (Eq.
 * signal_amp_tracing, discretised as NeuS's T alpha is the integral of T rho),
 *   alpha_j T_j clamp(Tbar_j + phi_tx[i] - phi_ray[r], 0, 1),  Tbar_j = T_j (1 - alpha_j/2)
 * ((T_j^2 - T_{j+1}^2)/2 without the shift; on a real ray T' rho' du' = T rho du,
 * so the shift enters once), and the contribution sits at the segment's
 * midpoint m_j = (x_j + x_{j+1})/2 (the last sample, alpha = 0, at itself):
 * r_ij, the phase and spec are taken at m_j, n_hat and a at x_j.  The sum
 * then does not depend on how the samples split a ray, so sparse (importance)
 * samples estimate the same signal as dense ones.
 * signal: [n_meas][n_freq] complex (output).  alpha_out/trans_out: optional
 * [n_ray*n_z] outputs (NULL to skip).
 * ------------------------------------------------------------------------ */
size_t rfvr_render_forward_ws_bytes(const rfvr_aperture* ap, const rfvr_samples* sm);
int rfvr_render_forward(const rfvr_aperture* ap, const rfvr_samples* sm, const rfvr_fields* fl,
                        uint32_t flags, float* signal, float* alpha_out, float* trans_out,
                        void* ws, size_t ws_bytes, void* stream);

/* Adjoint of rfvr_render_forward (App. A, Differentiable Matched Filter & Signal
 * Tracing, and Code Implementation, Alg. 2 backward), with the
 * per-term phases and amplitudes recomputed rather than stored:
 *   G_ij = sum_n Re(g_signal[i,n] exp(+j 2 pi f_n 2 r_ij / c))
 *          (bistatic: path rt_ij + rr_ij instead of 2 r_ij),
 * chained through the amplitude, the transmittance product scan, alpha(Phi),
 * Phi(s f) and n_hat = grad / max(|grad|, 1e-12).  phi_* are detached.
 * Clamps pass gradient on their closed interval.
 * g_signal: [n_meas][n_freq] complex (input, PyTorch convention dL/dRe + j dL/dIm).
 * Outputs (any may be NULL to skip): g_sdf [n_ray*n_z], g_grad [n_ray*n_z][3],
 * g_refl [n_ray*n_z], g_amp [1] (dL/dA'), g_s [1] (dL/ds). */
size_t rfvr_render_backward_ws_bytes(const rfvr_aperture* ap, const rfvr_samples* sm);
int rfvr_render_backward(const rfvr_aperture* ap, const rfvr_samples* sm, const rfvr_fields* fl,
                         uint32_t flags, const float* g_signal, float* g_sdf, float* g_grad,
                         float* g_refl, float* g_amp, float* g_s,
                         void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Matched filter (filter-based rendering, Eq. mf-sm; App. A, Code Implementation, Alg. 1)
 *   z_q = sum_{i,n} signal[i,n] exp(+j 2 pi f_n d_iq / c),  power_q = |z_q|
 * with the round trip d_iq = 2 |x_q - tx_i| (monostatic) or
 * |x_q - tx_i| + |rx_i - x_q| (bistatic).
 * xyz_q: [n_q][3] query points.  signal2: optional second signal filtered at
 * the same points (e.g. the measured one), with outputs z2/power2.
 * Any of z, power, z2, power2 may be NULL.  flags: 0 or RFVR_PHASE_NAIVE32.
 * ------------------------------------------------------------------------ */
size_t rfvr_mf_forward_ws_bytes(const rfvr_aperture* ap, int64_t n_q, int two_signals);
int rfvr_mf_forward(const rfvr_aperture* ap, const float* xyz_q, int64_t n_q, uint32_t flags,
                    const float* signal, float* z, float* power,
                    const float* signal2, float* z2, float* power2,
                    void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid allocation): the matched
 * filter forward with no workspace argument.  Arguments, outputs, flags and
 * errors are those of rfvr_mf_forward, whose kernels it runs; its scratch is a
 * library-owned device array of RFVR_MF_STATIC_SCRATCH_BYTES on each GPU it
 * runs on, looked up on the first call on that device and held until the
 * process ends.  It allocates nothing.  A call whose rfvr_mf_forward_ws_bytes()
 * exceeds RFVR_MF_STATIC_SCRATCH_BYTES returns RFVR_E_INVALID and enqueues
 * nothing (1024 measurements x 128 frequencies need 1.6 MB with one
 * signal, 3.1 MB with two).  Every call on one GPU uses that GPU's one array,
 * which keeps the last call's contents (nothing in it needs clearing between
 * calls): calls that overlap in time on one GPU, on different streams or
 * from several host threads, race and give wrong results, so the caller
 * orders them (one stream, or events).  The work runs on the device that is
 * current when the call is made; `stream` must belong to it. */
#define RFVR_MF_STATIC_SCRATCH_BYTES (32u << 20)
int rfvr_mf_forward_static(const rfvr_aperture* ap, const float* xyz_q, int64_t n_q, uint32_t flags,
                           const float* signal, float* z, float* power, const float* signal2, float* z2,
                           float* power2, void* stream);

/* Adjoint of rfvr_mf_forward through power = |z| (App. A, Code Implementation,
 * Alg. 1 backward):
 *   g_signal[i,n] = sum_q g_power_q (z_q / power_q) exp(-j 2 pi f_n d_iq / c),
 * a point with power_q == 0 contributes nothing.  z: [n_q] complex, power: [n_q],
 * g_power: [n_q] inputs; g_signal: [n_meas][n_freq] complex output. */
size_t rfvr_mf_backward_ws_bytes(const rfvr_aperture* ap, int64_t n_q);
int rfvr_mf_backward(const rfvr_aperture* ap, const float* xyz_q, int64_t n_q,
                     const float* z, const float* power, const float* g_power,
                     uint32_t flags, float* g_signal, void* ws, size_t ws_bytes, void* stream);

/* The order K that the term entry points choose for measurements ap and
 * points xyz [n_pts][3] (device), written to *order (device int32; 0 = the
 * per-frequency kernels), as described with RFVR_TERMS_DIRECT.  Asynchronous
 * on stream like every other call; RFVR_E_WORKSPACE below the query. */
size_t rfvr_term_order_ws_bytes(const rfvr_aperture* ap, int64_t n_pts);
int rfvr_term_order(const rfvr_aperture* ap, const float* xyz, int64_t n_pts, int32_t* order,
                    void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Several scenes or scan planes in one call (Sec. 3 problem statement: an
 * object is scanned from several radar planes, each with its own aperture
 * and primary rays; Sec. "Number of Radar Scanning Planes").  scenes: host
 * array of n_scenes >= 1 descriptors, each holding what the single-scene
 * call takes (fields: render calls only; the matched filter runs at each
 * scene's sample points, n_q = n_ray * n_z).  Arrays are packed in scene
 * order: signals [sum_s n_meas_s * n_freq_s] complex, per-point arrays
 * [sum_s n_ray_s * n_z_s] (times 3 for positions and gradients, times 2 for
 * complex z), per-scene scalars (g_amp, g_s) [n_scenes].  Every scene is
 * checked before anything is enqueued (an error names the scene); the scenes
 * then run one after another on stream, reusing the workspace, whose size is
 * the largest single-scene requirement.  Same errors as the single calls; a
 * HIP runtime error (RFVR_E_HIP) in a later scene leaves the earlier scenes'
 * work enqueued.
 * ------------------------------------------------------------------------ */
typedef struct rfvr_scene {
    rfvr_aperture ap;
    rfvr_samples  sm;
    rfvr_fields   fl;
} rfvr_scene;
size_t rfvr_render_forward_batched_ws_bytes(int32_t n_scenes, const rfvr_scene* scenes);
int rfvr_render_forward_batched(int32_t n_scenes, const rfvr_scene* scenes, uint32_t flags, float* signal,
                                float* alpha_out, float* trans_out, void* ws, size_t ws_bytes,
                                void* stream);
size_t rfvr_render_backward_batched_ws_bytes(int32_t n_scenes, const rfvr_scene* scenes);
int rfvr_render_backward_batched(int32_t n_scenes, const rfvr_scene* scenes, uint32_t flags,
                                 const float* g_signal, float* g_sdf, float* g_grad, float* g_refl,
                                 float* g_amp, float* g_s, void* ws, size_t ws_bytes, void* stream);
size_t rfvr_mf_forward_batched_ws_bytes(int32_t n_scenes, const rfvr_scene* scenes, int two_signals);
int rfvr_mf_forward_batched(int32_t n_scenes, const rfvr_scene* scenes, uint32_t flags, const float* signal,
                            float* z, float* power, const float* signal2, float* z2, float* power2,
                            void* ws, size_t ws_bytes, void* stream);
size_t rfvr_mf_backward_batched_ws_bytes(int32_t n_scenes, const rfvr_scene* scenes);
int rfvr_mf_backward_batched(int32_t n_scenes, const rfvr_scene* scenes, const float* z, const float* power,
                             const float* g_power, uint32_t flags, float* g_signal, void* ws,
                             size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * L2 heatmap loss (Sec. Overview, step 5):
 *   loss = (1/n) sum_q m_q (p_q - p*_q)^2 ,  g_p = 2 m (p - p*) / n
 * mask may be NULL (m = 1).  loss: [1] float output; g_p: [n] output or NULL.
 * ------------------------------------------------------------------------ */
size_t rfvr_loss_ws_bytes(int64_t n);
int rfvr_loss_l2(int64_t n, const float* p, const float* p_star, const float* mask,
                 float* loss, float* g_p, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Lensless primary-ray sampling (Sec. "Lensless Sampling", Primary Ray)
 * Rays run parallel to primary_dir from the aperture plane (normal to
 * primary_dir at signed distance plane_offset from the world origin along the
 * unit primary direction w_p) through a cube of centre `centre` and half side
 * `half_extent`; lateral grid of cell centres, ray r = iy*n_ray_x + ix,
 * lateral axes e1 = unit(y x w_p) (x x w_p if w_p is within ~26 deg of y),
 * e2 = w_p x e1.  Depth u over [c.w_p - h, c.w_p + h] in n_z strata:
 *   GRID:       u_k = lo + (k + 1/2) 2h/n_z
 *   STRATIFIED: u_k = lo + (k + xi) 2h/n_z, xi = (SplitMix64(key, r*n_z+k) >> 40) 2^-24,
 *               key = SplitMix64(seed, step) (k-th output of SplitMix64 from a
 *               state = mix(state + (k+1) * 0x9E3779B97F4A7C15))
 * Outputs: xyz [n_ray][n_z][3], u [n_ray][n_z] (NULL to skip), ray_origin
 * [n_ray][3] (NULL to skip): the ray's foot on the aperture plane, where the
 * occupancy of Eq. lens-less-transmittance is evaluated.  u is measured along
 * w_p from the parallel plane through the world origin.
 * ------------------------------------------------------------------------ */
#define RFVR_SAMPLE_GRID        0
#define RFVR_SAMPLE_STRATIFIED  1
typedef struct rfvr_sample_desc {
    float    centre[3];
    float    half_extent;
    float    primary_dir[3];     /* need not be normalised; non-zero */
    int32_t  n_ray_x, n_ray_y, n_z;
    int32_t  mode;               /* RFVR_SAMPLE_* */
    uint64_t seed, step;
    float    plane_offset;       /* aperture plane: {x : x . w_p = plane_offset} */
} rfvr_sample_desc;
int rfvr_sample_points(const rfvr_sample_desc* d, float* xyz, float* u, float* ray_origin,
                       void* stream);

/* ------------------------------------------------------------------------
 * SDF network with reflectiveness head (Sec. "Opaque density representation",
 * "Signal representation"; App. C).  x_hat = (x - centre)/half_size,
 * gamma = [x_hat, sin(2^k pi x_hat), cos(2^k pi x_hat) for k < pe_octaves]
 * (3 + 6*pe_octaves values), h_l = softplus_beta(W h_{l-1} + b) for n_layers
 * layers of `width`, f = half_size (w_out . h + b_out) metres,
 * head g_k = relu(Wh g_{k-1} + bh) for head_layers layers of head_width on
 * the last trunk activation, a = sigmoid(wh_out . g + bh_out).
 * params: flat float32 vector, row-major [out][in] matrices in the order
 *   W_0,b_0,...,W_{L-1},b_{L-1}, w_out,b_out, Wh_0,bh_0,...,wh_out,bh_out.
 * ------------------------------------------------------------------------ */
#define RFVR_PREC_FP32 0
#define RFVR_PREC_BF16 1         /* BF16 matrix operands, FP32 accumulation */
#define RFVR_PREC_BF16X3 2       /* BF16 MFMA on split operands, x = big + small with
                                    big = bf16(x), small = bf16(x - big); products
                                    big*big + big*small + small*big, FP32 accumulation */
#define RFVR_PREC_F16 3          /* FP32 accumulation.  Forward products (trunk layers,
                                    head, the grad_x f sweep; also where the plain backward
                                    recomputes them): FP16 MFMA, the weights rounded once,
                                    the per-point operand split as big + small in FP16,
                                    products big*w + small*w.  Backward products (tangent,
                                    adjoints, weight gradients), whose values scale with
                                    the upstream gradients and exceed FP16's range: BF16
                                    operands, one product */
/* In every 16-bit form the layer that reads the positional encoding keeps FP32
 * operands. */
typedef struct rfvr_mlp {
    int32_t      n_layers;       /* 1..16 */
    int32_t      width;          /* multiple of 64, <= 512 */
    int32_t      pe_octaves;     /* 0..12 */
    int32_t      head_width;     /* multiple of 64, <= 256 */
    int32_t      head_layers;    /* 1..4 */
    float        softplus_beta;  /* > 0 */
    float        centre[3];
    float        half_size;      /* > 0 */
    int32_t      precision;      /* RFVR_PREC_* */
    const float* params;         /* device, rfvr_mlp_param_count() floats */
} rfvr_mlp;
int64_t rfvr_mlp_param_count(const rfvr_mlp* net);

/* f [n], grad = grad_x f [n][3], refl = a [n]; any output may be NULL. */
size_t rfvr_mlp_forward_ws_bytes(const rfvr_mlp* net, int64_t n);
int rfvr_mlp_forward(const rfvr_mlp* net, const float* xyz, int64_t n, float* sdf, float* grad,
                     float* refl, void* ws, size_t ws_bytes, void* stream);

/* Parameter gradient of J = sum_q g_sdf f + g_grad . grad_x f + g_refl a,
 * including the second-order path through grad_x f; activations recomputed.
 * Inputs g_sdf/g_grad/g_refl may be NULL (= 0).  g_params: rfvr_mlp_param_count()
 * floats, overwritten unless flags has RFVR_ACCUMULATE. */
size_t rfvr_mlp_backward_ws_bytes(const rfvr_mlp* net, int64_t n);
int rfvr_mlp_backward(const rfvr_mlp* net, const float* xyz, int64_t n, const float* g_sdf,
                      const float* g_grad, const float* g_refl, uint32_t flags, float* g_params,
                      void* ws, size_t ws_bytes, void* stream);

/* Several networks in one call (one per scene, e.g. scenes trained side by
 * side): nets host [n_nets], n host [n_nets] point counts (>= 1 each), points
 * xyz packed [sum n][3]; outputs and upstream gradients packed per point as
 * for the single calls; g_params packed by rfvr_mlp_param_count of each net.
 * Every net is checked before anything is enqueued; the nets then run one
 * after another on stream, reusing the workspace (the largest single-net
 * requirement); as for the batched scenes, only a HIP runtime error can stop
 * the loop after earlier nets.  flags: as rfvr_mlp_backward, applied to every
 * net. */
size_t rfvr_mlp_forward_grouped_ws_bytes(int32_t n_nets, const rfvr_mlp* nets, const int64_t* n);
int rfvr_mlp_forward_grouped(int32_t n_nets, const rfvr_mlp* nets, const float* xyz, const int64_t* n,
                             float* sdf, float* grad, float* refl, void* ws, size_t ws_bytes, void* stream);
size_t rfvr_mlp_backward_grouped_ws_bytes(int32_t n_nets, const rfvr_mlp* nets, const int64_t* n);
int rfvr_mlp_backward_grouped(int32_t n_nets, const rfvr_mlp* nets, const float* xyz, const int64_t* n,
                              const float* g_sdf, const float* g_grad, const float* g_refl, uint32_t flags,
                              float* g_params, void* ws, size_t ws_bytes, void* stream);

/* Training pair: the same two operations, sharing a caller-owned reserve
 * (device, 256-byte aligned, rfvr_mlp_reserve_bytes() bytes: for every trunk
 * layer its activation H = softplus(Z) and the gradient sweep's adjoint of f
 * to the pre-activation Z, float32 [n][width] each; softplus'(Z) and
 * exp(-beta Z) are recovered from H; then for every head layer its output
 * before the relu, float32 [n][head_width]).  rfvr_mlp_forward_train computes
 * what rfvr_mlp_forward does (running the gradient sweep and the head even
 * when grad or refl is NULL) and fills the reserve; rfvr_mlp_backward_train
 * reads it instead of recomputing the primal and head layers and the adjoint
 * of the tangent pass (the sweep's adjoint scaled by half_size), so per trunk
 * layer it runs two matrix products fewer than rfvr_mlp_backward.  The caller keeps
 * net (params unchanged), xyz and n the same between the two calls and does
 * not write the reserve in between; nothing checks this, and a mismatch gives
 * wrong gradients without an error.  Outputs agree with the plain calls to
 * float32 rounding.  A NULL or zero-sized reserve is RFVR_E_INVALID, a short
 * or misaligned one RFVR_E_WORKSPACE. */
size_t rfvr_mlp_reserve_bytes(const rfvr_mlp* net, int64_t n);
size_t rfvr_mlp_forward_train_ws_bytes(const rfvr_mlp* net, int64_t n);
int rfvr_mlp_forward_train(const rfvr_mlp* net, const float* xyz, int64_t n, float* sdf, float* grad,
                           float* refl, void* reserve, size_t reserve_bytes, void* ws, size_t ws_bytes,
                           void* stream);
size_t rfvr_mlp_backward_train_ws_bytes(const rfvr_mlp* net, int64_t n);
int rfvr_mlp_backward_train(const rfvr_mlp* net, const float* xyz, int64_t n, const float* g_sdf,
                            const float* g_grad, const float* g_refl, uint32_t flags, float* g_params,
                            const void* reserve, size_t reserve_bytes, void* ws, size_t ws_bytes,
                            void* stream);

/* ------------------------------------------------------------------------
 * AdamW update (App. C: AdamW with cosine annealing), step t >= 1:
 *   m = b1 m + (1-b1) g ; v = b2 v + (1-b2) g^2
 *   p -= lr * ( m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps) + wd * p )
 * ------------------------------------------------------------------------ */
int rfvr_adamw(int64_t n, float* p, const float* g, float* m, float* v, int64_t t, float lr,
               float b1, float b2, float eps, float wd, void* stream);

/* ------------------------------------------------------------------------
 * Learned proposal sampler (not in the paper: it concentrates the samples of
 * Sec. Lensless Sampling where the render's own blend weights are, keeping
 * stratified uniform samples as the fallback).
 *
 * Network: gamma_L(x_hat) -> [Linear(width) -> relu] x layers -> Linear(1),
 * x_hat = (x - centre)/half_size; flat float32 params
 *   W_0 [width][3+6L], b_0, ..., W_{layers-1} [width][width], b, w_out [width], b_out [1].
 * ------------------------------------------------------------------------ */
typedef struct rfvr_proposal {
    int32_t      pe_octaves;     /* 0..5 (3 + 6 L <= 64)         */
    int32_t      width;          /* 64                           */
    int32_t      layers;         /* 1..4                         */
    float        centre[3];
    float        half_size;      /* > 0                          */
    const float* params;         /* device                       */
} rfvr_proposal;
int64_t rfvr_proposal_param_count(const rfvr_proposal* net);
size_t rfvr_proposal_ws_bytes(const rfvr_proposal* net, int64_t n);
/* logits [n] at points xyz [n][3].  The proposal calls evaluate all n points
 * in one pass (two threads per point in its matrix products), so they take at
 * most RFVR_MAX_POINTS / 2 + 1 = 2^30 points. */
int rfvr_proposal_forward(const rfvr_proposal* net, const float* xyz, int64_t n, float* logits,
                          void* ws, size_t ws_bytes, void* stream);
/* g_params (+)= d/dparams sum_q g_logits[q] z_q (activations recomputed). */
int rfvr_proposal_backward(const rfvr_proposal* net, const float* xyz, int64_t n,
                           const float* g_logits, uint32_t flags, float* g_params,
                           void* ws, size_t ws_bytes, void* stream);

/* Largest number of samples per ray of the proposal calls below. */
#define RFVR_MAX_RAY_SAMPLES 1024

/* Importance samples along the primary rays of `d` (its n_z is ignored).
 * logits: [n_ray][n_bins] at the centres of n_bins equal depth bins over
 * [c.w_p - h, c.w_p + h].  pdf_b = (sigmoid(z_b) + 1e-3) / sum.  With d->mode
 * RFVR_SAMPLE_STRATIFIED slot s of ray r draws xi = (SplitMix64(key,
 * r*(n_uni+n_imp) + s) >> 40) 2^-24 from the step's stream key (as
 * rfvr_sample_points does); with RFVR_SAMPLE_GRID xi = 1/2 for every slot (the
 * depths then move only with the logits).  Slots s < n_uni are stratified
 * uniform over the whole range, u = lo + (s + xi)(hi - lo)/n_uni; the others
 * invert the CDF at v = (s - n_uni + xi)/n_imp, linearly inside the bin.
 * Depths are sorted per ray (ties keep slot order).  n_bins <= 64,
 * n_imp + n_uni <= RFVR_MAX_RAY_SAMPLES.  Outputs xyz [n_ray][n_uni+n_imp][3], u (or NULL),
 * ray_origin [n_ray][3] (or NULL). */
int rfvr_sample_importance(const rfvr_sample_desc* d, const float* logits, int32_t n_bins,
                           int32_t n_imp, int32_t n_uni, float* xyz, float* u, float* ray_origin,
                           void* stream);

/* Proposal targets: per ray, the blend weights w_k = trans_k * alpha_k of the
 * render at depths u [n_ray][n_k] (ascending): w_k is the opacity of the
 * segment [u_k, u_{k+1}], spread over the n_bins equal bins of [lo, hi] that
 * the segment overlaps in proportion to the overlap (the last sample, and a
 * segment of zero length, add w_k to the bin of u_k), giving W_b;
 * t_b = min(1, W_b / max(max_b W_b, 1e-3)).  Overlaps and sums in FP64.
 * n_dilate >= 1 dilates the targets in depth: bin b takes the largest t over
 * bins b - n_dilate .. b (so samples continue past a front surface into the
 * object behind it).  targets: [n_ray][n_bins].  n_k <= RFVR_MAX_RAY_SAMPLES,
 * n_bins <= 64, 0 <= n_dilate < n_bins. */
int rfvr_proposal_targets(int32_t n_ray, int32_t n_k, const float* u, const float* alpha,
                          const float* trans, float lo, float hi, int32_t n_bins, int32_t n_dilate,
                          float* targets, void* stream);

/* Mean binary cross-entropy of sigmoid(z) against t and its gradient
 * g = (sigmoid(z) - t) / n.  loss: [1] output. */
size_t rfvr_bce_ws_bytes(int64_t n);
int rfvr_bce(int64_t n, const float* logits, const float* t, float* loss, float* g_logits,
             void* ws, size_t ws_bytes, void* stream);

/* Per-antenna ("naive") sampling, the brute-force Monte Carlo of Sec.
 * Integration that the lensless sampling replaces: for antenna i, ray r runs
 * from tx_i through the r-th point of the lateral grid of cell centres on the
 * plane through the cube centre normal to w_p (grid as rfvr_sample_points);
 * its n_z samples sit at the cell centres of the ray's segment between the
 * planes x . w_p = c . w_p -+ h (the antenna must lie before the first plane).
 * jac = (|x - tx_i| / |g_r - tx_i|)^2 is the sample's volume relative to a
 * lensless cell (spherical volume element of a ray through a grid cell), to be
 * passed as point_weight.  Outputs xyz [n_ant][n_ray][n_z][3], jac
 * [n_ant][n_ray][n_z] (NULL to skip).  d's n_z is used; mode, seed, step and
 * plane_offset are ignored. */
int rfvr_sample_naive(const rfvr_sample_desc* d, const float* tx, int32_t n_ant, float* xyz,
                      float* jac, void* stream);

/* Dynamic loss masking (Sec. Optimization): a point whose rendered filter
 * output was high in an earlier iteration but is low now is left out of the
 * loss.  With S = max_q power_ref[q] (the measured heatmap's peak):
 *   mask[q] = 0 if history[q] >= tau_hi * S and power[q] < tau_lo * history[q],
 *             else 1;
 *   then history[q] = max(history[q], power[q]).
 * All comparisons in FP32 (products rounded to FP32 first).  history [n] is
 * caller-owned state, zero before the first iteration; mask [n] output, usable
 * as the mask of rfvr_loss_l2.  tau_hi, tau_lo finite and >= 0. */
size_t rfvr_mask_ws_bytes(int64_t n);
int rfvr_mask_update(int64_t n, const float* power, const float* power_ref, float* history,
                     float tau_hi, float tau_lo, float* mask, void* ws, size_t ws_bytes,
                     void* stream);

/* Occupancy at the detached ray / antenna origins (Eq. lens-less-transmittance):
 *   phi[k] = 1 / (1 + exp(-s * sdf[k])),  k < n.  s finite and > 0. */
int rfvr_occupancy(int64_t n, float s, const float* sdf, float* phi, void* stream);
/* The same with s = exp(log_s[0]) read from device memory at kernel time
 * (log_s: device [1], as rfvr_fields.log_s_ptr). */
int rfvr_occupancy_logs(int64_t n, const float* log_s, const float* sdf, float* phi, void* stream);

/* Library information. */
const char* rfvr_last_error(void);
int rfvr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RFVR_H */
