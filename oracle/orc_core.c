/*
 * FP64 CPU oracle for lensless RF volumetric rendering (GeRaF, arXiv 2605.29097).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition of the
 * direct sums the method computes; it is compiled by oracle/build.py and is
 * called only from tests, the smoke check and the CPU-baseline leg of the
 * benchmark.  It shares no code, header or constant with the HIP library.
 *
 * Every sum is taken in double precision in the natural index order, with one
 * sin/cos pair per term (no recurrences, no blocking).  Complex values are
 * split into separate real/imaginary arrays.  Index conventions:
 *   i = measurement (antenna), n = frequency (f_n = f0 + n*df),
 *   j = point, flat over [n_ray][n_z] (ray index r = j / n_z).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

static const double SPEED_OF_LIGHT = 299792458.0; /* m/s */
static const double TWO_PI = 6.283185307179586476925286766559;

enum { SPEC_CLAMP = 0, SPEC_RAW = 1, SPEC_OFF = 2 };

/* Phase of term (i, j, n) in revolutions: f_n * d / c with d the round-trip
 * path length (FMCW model, Sec. "Radar Basics", Eq. fmcw).  Only the
 * fractional part matters for sin/cos; taking it first is exact in FP64 up to
 * the rounding of the product. */
static double phase_rev(double f0, double df, int n, double d)
{
    double theta = (f0 + (double)n * df) * d / SPEED_OF_LIGHT;
    return theta - floor(theta);
}

/* Geometry, amplitude and amplitude partials of one (measurement, point) pair.
 * Sec. "Signal Amplitude Tracing" (Eq. signal_amp_tracing), the specular factor
 * of Sec. "Reflections"/App. A.3, free-space decay of Eq. reflection_angle with
 * the 4*pi absorbed into the learnt amplitude, and the lensless transmittance
 * shift of Eq. lens-less-transmittance. */
typedef struct {
    double d;          /* round-trip path length r_t + r_r                      */
    double c;          /* amplitude c_ij                                        */
    double dc_dbase;   /* dc / d(amp * w * refl * alpha)                         */
    double dc_dT;      /* dc / d T_j (primary-ray transmittance)                 */
    double dc_dn[3];   /* dc / d n_hat                                           */
} pair_t;

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* seg = 0: the round trip weighs the sample by T_tx T_rx (T'^2 monostatic).
 * seg = 1 (monostatic only): the caller passes base = amp w refl alpha T and
 * T = the segment's mean transmittance; the pair's factor is then the single
 * shifted value clamp(T + dtx, 0, 1) (see orc_render). */
static void pair_eval(const double* tx, const double* rx, const double* x,
                      const double* nh, double base, double T, double dtx, double drx,
                      int spec_mode, int seg, pair_t* p)
{
    double dt[3] = {x[0] - tx[0], x[1] - tx[1], x[2] - tx[2]};
    double rt = sqrt(dt[0] * dt[0] + dt[1] * dt[1] + dt[2] * dt[2]);
    double wi[3] = {dt[0] / rt, dt[1] / rt, dt[2] / rt};      /* incident dir  */
    double rr, wr[3];                                         /* to receiver   */
    if (rx) {
        double e[3] = {rx[0] - x[0], rx[1] - x[1], rx[2] - x[2]};
        rr = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        wr[0] = e[0] / rr; wr[1] = e[1] / rr; wr[2] = e[2] / rr;
    } else {
        rr = rt;
        wr[0] = -wi[0]; wr[1] = -wi[1]; wr[2] = -wi[2];
    }
    /* ideal specular direction w_o = w_i - 2 (n.w_i) n ; factor w_o . w_r */
    double ni = nh[0] * wi[0] + nh[1] * wi[1] + nh[2] * wi[2];
    double nr = nh[0] * wr[0] + nh[1] * wr[1] + nh[2] * wr[2];
    double wo[3] = {wi[0] - 2.0 * ni * nh[0], wi[1] - 2.0 * ni * nh[1], wi[2] - 2.0 * ni * nh[2]};
    double spec_raw = wo[0] * wr[0] + wo[1] * wr[1] + wo[2] * wr[2];
    double spec;
    int spec_live;
    if (spec_mode == SPEC_OFF) {
        spec = 1.0; spec_live = 0;
    } else if (spec_mode == SPEC_RAW) {
        spec = spec_raw; spec_live = 1;
    } else {
        spec = spec_raw > 0.0 ? spec_raw : 0.0;
        spec_live = spec_raw >= 0.0;
    }
    double ttx_raw = T + dtx, trx_raw = T + drx;
    double ttx = clamp01(ttx_raw), trx = clamp01(trx_raw);
    double mtx = (ttx_raw >= 0.0 && ttx_raw <= 1.0) ? 1.0 : 0.0;
    double mrx = (trx_raw >= 0.0 && trx_raw <= 1.0) ? 1.0 : 0.0;
    double geo = 1.0 / (rt * rr);
    double tt = seg ? ttx : ttx * trx;                      /* transmittance factor   */
    double dtt = seg ? mtx : (mtx * trx + ttx * mrx);       /* its derivative in T    */

    p->d = rt + rr;
    p->c = base * spec * tt * geo;
    p->dc_dbase = spec * tt * geo;
    p->dc_dT = base * spec * geo * dtt;
    for (int k = 0; k < 3; ++k) {
        double ds = spec_live ? -2.0 * (nr * wi[k] + ni * wr[k]) : 0.0;
        p->dc_dn[k] = base * tt * geo * ds;
    }
}

/* Per-pair inputs common to render and its adjoint. */
typedef struct {
    int n_meas; const double* tx; const double* rx;
    int n_freq; double f0, df;
    int n_ray, n_z; const double* xyz; const double* ray_w;
    const double* nhat; const double* refl; const double* alpha; const double* trans;
    const double* phi_ray; const double* phi_tx; const double* phi_rx;
    double amp; int spec_mode; int seg;
} scene_t;

static void scene_pair(const scene_t* S, int i, long j, pair_t* p)
{
    long r = j / S->n_z;
    double w = S->ray_w ? S->ray_w[r] : 1.0;
    double base = S->amp * w * S->refl[j] * S->alpha[j];
    double dtx = 0.0, drx = 0.0;
    if (S->phi_ray && S->phi_tx) dtx = S->phi_tx[i] - S->phi_ray[r];
    if (S->rx) {
        if (S->phi_ray && S->phi_rx) drx = S->phi_rx[i] - S->phi_ray[r];
    } else {
        drx = dtx;
    }
    pair_eval(S->tx + 3 * (long)i, S->rx ? S->rx + 3 * (long)i : NULL, S->xyz + 3 * j,
              S->nhat + 3 * j, base, S->trans[j], dtx, drx, S->spec_mode, S->seg, p);
}

/* Signal tracing, Eq. ref_sim: s[i,n] = sum_j c_ij exp(-j 2 pi f_n d_ij / c).
 * The per-point arrays are what the weight needs (render.py prepares them):
 * seg = 0: alpha_j and T_j at the sample points; seg = 1: alpha_j T_j, the
 * segment's mean transmittance and the segment midpoints as positions. */
void orc_render(int n_meas, const double* tx, const double* rx,
                int n_freq, double f0, double df,
                int n_ray, int n_z, const double* xyz, const double* ray_w,
                const double* nhat, const double* refl, const double* alpha,
                const double* trans, const double* phi_ray, const double* phi_tx,
                const double* phi_rx, double amp, int spec_mode, int seg,
                double* s_re, double* s_im)
{
    scene_t S = {n_meas, tx, rx, n_freq, f0, df, n_ray, n_z, xyz, ray_w, nhat, refl,
                 alpha, trans, phi_ray, phi_tx, phi_rx, amp, spec_mode, seg};
    long n_pts = (long)n_ray * n_z;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_meas; ++i) {
        for (int n = 0; n < n_freq; ++n) { s_re[(long)i * n_freq + n] = 0.0; s_im[(long)i * n_freq + n] = 0.0; }
        for (long j = 0; j < n_pts; ++j) {
            pair_t p;
            scene_pair(&S, i, j, &p);
            if (p.c == 0.0) continue;       /* its terms are exact zeros */
            for (int n = 0; n < n_freq; ++n) {
                double ph = TWO_PI * phase_rev(f0, df, n, p.d);
                s_re[(long)i * n_freq + n] += p.c * cos(ph);
                s_im[(long)i * n_freq + n] -= p.c * sin(ph);
            }
        }
    }
}

/* Adjoint of signal tracing (App. A, Differentiable Matched Filter & Signal Tracing): G_ij = sum_n Re(g_s[i,n] exp(+j phase)),
 * then the chain rule into the per-point quantities the amplitude depends on.
 * Outputs (per point j, summed over measurements):
 *   g_base  = dL/d(amp*w*refl*alpha),  g_trans = dL/dT_j,  g_nhat = dL/dn_hat_j. */
void orc_render_adjoint(int n_meas, const double* tx, const double* rx,
                        int n_freq, double f0, double df,
                        int n_ray, int n_z, const double* xyz, const double* ray_w,
                        const double* nhat, const double* refl, const double* alpha,
                        const double* trans, const double* phi_ray, const double* phi_tx,
                        const double* phi_rx, double amp, int spec_mode, int seg,
                        const double* gs_re, const double* gs_im,
                        double* g_base, double* g_trans, double* g_nhat)
{
    scene_t S = {n_meas, tx, rx, n_freq, f0, df, n_ray, n_z, xyz, ray_w, nhat, refl,
                 alpha, trans, phi_ray, phi_tx, phi_rx, amp, spec_mode, seg};
    long n_pts = (long)n_ray * n_z;
#pragma omp parallel for schedule(dynamic, 64)
    for (long j = 0; j < n_pts; ++j) {
        double gb = 0.0, gt = 0.0, gn0 = 0.0, gn1 = 0.0, gn2 = 0.0;
        for (int i = 0; i < n_meas; ++i) {
            pair_t p;
            scene_pair(&S, i, j, &p);
            double G = 0.0;
            for (int n = 0; n < n_freq; ++n) {
                double ph = TWO_PI * phase_rev(f0, df, n, p.d);
                G += gs_re[(long)i * n_freq + n] * cos(ph) - gs_im[(long)i * n_freq + n] * sin(ph);
            }
            gb += G * p.dc_dbase;
            gt += G * p.dc_dT;
            gn0 += G * p.dc_dn[0]; gn1 += G * p.dc_dn[1]; gn2 += G * p.dc_dn[2];
        }
        g_base[j] = gb; g_trans[j] = gt;
        g_nhat[3 * j] = gn0; g_nhat[3 * j + 1] = gn1; g_nhat[3 * j + 2] = gn2;
    }
}

/* Round-trip path length from measurement i to query point x. */
static double path_len(const double* tx, const double* rx, const double* x)
{
    double a = x[0] - tx[0], b = x[1] - tx[1], c = x[2] - tx[2];
    double rt = sqrt(a * a + b * b + c * c);
    if (!rx) return 2.0 * rt;
    double e = rx[0] - x[0], f = rx[1] - x[1], g = rx[2] - x[2];
    return rt + sqrt(e * e + f * f + g * g);
}

/* Matched filter, Eq. mf-sm: z_q = sum_{i,n} s[i,n] exp(+j 2 pi f_n d_iq / c). */
void orc_mf(int n_meas, const double* tx, const double* rx,
            int n_freq, double f0, double df,
            long n_q, const double* xq, const double* s_re, const double* s_im,
            double* z_re, double* z_im)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (long q = 0; q < n_q; ++q) {
        double zr = 0.0, zi = 0.0;
        for (int i = 0; i < n_meas; ++i) {
            double d = path_len(tx + 3 * (long)i, rx ? rx + 3 * (long)i : NULL, xq + 3 * q);
            for (int n = 0; n < n_freq; ++n) {
                double ph = TWO_PI * phase_rev(f0, df, n, d);
                double c = cos(ph), s = sin(ph);
                double a = s_re[(long)i * n_freq + n], b = s_im[(long)i * n_freq + n];
                zr += a * c - b * s;
                zi += a * s + b * c;
            }
        }
        z_re[q] = zr; z_im[q] = zi;
    }
}

/* Adjoint of the (linear) matched filter: g_s[i,n] = sum_q g_z,q exp(-j phase). */
void orc_mf_adjoint(int n_meas, const double* tx, const double* rx,
                    int n_freq, double f0, double df,
                    long n_q, const double* xq, const double* gz_re, const double* gz_im,
                    double* gs_re, double* gs_im)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_meas; ++i) {
        for (int n = 0; n < n_freq; ++n) { gs_re[(long)i * n_freq + n] = 0.0; gs_im[(long)i * n_freq + n] = 0.0; }
        for (long q = 0; q < n_q; ++q) {
            double d = path_len(tx + 3 * (long)i, rx ? rx + 3 * (long)i : NULL, xq + 3 * q);
            double a = gz_re[q], b = gz_im[q];
            for (int n = 0; n < n_freq; ++n) {
                double ph = TWO_PI * phase_rev(f0, df, n, d);
                double c = cos(ph), s = sin(ph);
                gs_re[(long)i * n_freq + n] += a * c + b * s;
                gs_im[(long)i * n_freq + n] += b * c - a * s;
            }
        }
    }
}

int orc_version(void) { return 1; }
