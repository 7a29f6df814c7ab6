/*
 * Seeded-input generator: frequency-domain TaylorF2 (3.5PN, non-spinning,
 * stationary-phase approximation) template spectra, band-packed.
 *
 * This file produces INPUTS only (the signal model the search correlates
 * against); it holds none of the search's arithmetic (no PSD weighting, no
 * normalisation, no filtering).  The phasing is the standard 3.5PN
 * stationary-phase expansion from the post-Newtonian literature (Buonanno,
 * Iyer, Ochsner, Pan & Sathyaprakash 2009, Phys. Rev. D 80, 084043,
 * Eq. (3.18) with the coefficients of their Eq. (3.3)), written here from the
 * formula:
 *
 *   h(f)   = f^(-7/6) exp(-i Psi(f))
 *   Psi(f) = 2 pi f t_c - phi_c - pi/4 + 3/(128 eta v^5) sum_k alpha_k v^k
 *   v      = (pi M f)^(1/3),  M = total mass in seconds,  eta = m1 m2 / M^2
 *
 * Amplitude normalisation is arbitrary (the search normalises every template).
 * The spectrum is cut at the Schwarzschild ISCO frequency 1/(6^(3/2) pi M).
 *
 * Layout: template t occupies out[2*(offset[t] + (k - k0[t])) + {0,1}] for
 * bins k in [k0[t], k1[t]]; bins below kstart[t] are written as zero (they
 * only pad the start to an aligned bin).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define MSUN_SEC 4.925490947641267e-06 /* G M_sun / c^3 in seconds */
#define EULER_GAMMA 0.57721566490153286061

void synth_taylorf2(int32_t n_tmpl, const double *m1, const double *m2,
                    const double *tc, const double *phic, double df,
                    const int32_t *k0, const int32_t *kstart, const int32_t *k1,
                    const int64_t *offset, float *out)
{
    const double pi = M_PI;
    /* Per-bin powers of f shared by every template: f^(1/3), ln f, f^(-7/6). */
    int32_t kmax = 0;
    for (int32_t t = 0; t < n_tmpl; ++t) if (k1[t] > kmax) kmax = k1[t];
    double *f13 = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    double *lnf = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    double *amp = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
#pragma omp parallel for schedule(static)
    for (int32_t k = 1; k <= kmax; ++k) {
        const double f = k * df;
        f13[k] = cbrt(f);
        lnf[k] = log(f);
        amp[k] = pow(f, -7.0 / 6.0);
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t t = 0; t < n_tmpl; ++t) {
        const double M = (m1[t] + m2[t]) * MSUN_SEC;
        const double eta = m1[t] * m2[t] / ((m1[t] + m2[t]) * (m1[t] + m2[t]));
        const double eta2 = eta * eta, eta3 = eta2 * eta;
        const double a2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
        const double a3 = -16.0 * pi;
        const double a4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta2;
        const double a5 = pi * (38645.0 / 756.0 - 65.0 / 9.0 * eta);
        const double a6c = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi * pi
                         - 6848.0 / 21.0 * EULER_GAMMA
                         + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi * pi) * eta
                         + 76055.0 / 1728.0 * eta2 - 127825.0 / 1296.0 * eta3;
        const double a6l = -6848.0 / 21.0;
        const double a7 = pi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta2);
        const double log_vlso = -0.5 * log(6.0);
        const double pref = 3.0 / (128.0 * eta);
        /* v = (pi M f)^(1/3) = c13 f^(1/3),  ln v = ln c13 + ln(f) / 3 */
        const double c13 = cbrt(pi * M);
        const double lnc13 = log(c13);
        float *o = out + 2 * offset[t];
        for (int32_t k = k0[t]; k <= k1[t]; ++k) {
            float *p = o + 2 * (int64_t)(k - k0[t]);
            if (k < kstart[t] || k <= 0) { p[0] = 0.f; p[1] = 0.f; continue; }
            const double f = k * df;
            const double v = c13 * f13[k];
            const double v2 = v * v, v3 = v2 * v, v4 = v3 * v, v5 = v4 * v;
            const double v6 = v5 * v, v7 = v6 * v;
            const double lv = lnc13 + lnf[k] / 3.0;
            const double series = 1.0 + a2 * v2 + a3 * v3 + a4 * v4
                                + a5 * (1.0 + 3.0 * (lv - log_vlso)) * v5
                                + (a6c + a6l * (log(4.0) + lv)) * v6 + a7 * v7;
            const double psi = 2.0 * pi * f * tc[t] - phic[t] - 0.25 * pi + pref / v5 * series;
            double s, c;
            sincos(psi, &s, &c);
            p[0] = (float)(amp[k] * c);
            p[1] = (float)(-amp[k] * s);
        }
    }
    free(f13);
    free(lnf);
    free(amp);
}
