/*
 * Oracle O1: direct evaluation of the discretised measurement equation.
 *
 * TEST INFRASTRUCTURE ONLY.  Built by oracle/build.py into
 * oracle/_build/libwgoracle.so and called from oracle/o1.py; the product
 * library never links or loads it, and it shares no code with the HIP path.
 *
 * Forward, eq. (3) of Sect. 2:
 *     d_k = sum_{l in L} sum_{m in M} I_lm / n_lm * exp(-2 pi i [u_k l + v_k m - w_k (n_lm - 1)])
 * Adjoint, the direct adjoint used for validation in Sect. 5 with the real
 * part taken (the dirty image is real):
 *     I_lm = Re( 1/n_lm * sum_k d_k exp(+2 pi i [u_k l + v_k m - w_k (n_lm - 1)]) )
 * with u_k = uvw[r,0] * f_c / c (effective coordinates, Sect. 2),
 * l = (p - npix_x/2) * pixsize_x, m = (q - npix_y/2) * pixsize_y, and
 * n - 1 = -(l^2 + m^2) / (1 + n) to avoid cancellation.
 *
 * Everything is FP64.  Each phase (in turns) has its nearest integer removed
 * before the sine and cosine are taken; sums are Kahan-compensated.
 * Parallelised with OpenMP over the independent outputs.
 */
#include <math.h>
#include <stdint.h>

static const double C_LIGHT = 299792458.0;
static const double TWO_PI = 6.283185307179586476925286766559;

typedef struct { double s, c; } kahan_t;

static inline void kahan_add(kahan_t *k, double x) {
    double y = x - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

static inline void pixel_lmn(int p, int q, int npix_x, int npix_y, double dx, double dy,
                             double *l, double *m, double *n, double *nm1) {
    *l = (double)(p - npix_x / 2) * dx;
    *m = (double)(q - npix_y / 2) * dy;
    double rho = (*l) * (*l) + (*m) * (*m);
    *n = sqrt(1.0 - rho);
    *nm1 = -rho / (1.0 + *n);
}

/* Forward for a list of visibilities (linear indices r*nchan + c) and a list of
 * pixels (p, q, value).  out_re/out_im have nvis entries. */
int o1_forward(int64_t nrow, int64_t nchan, const double *uvw, const double *freq,
               int npix_x, int npix_y, double pixsize_x, double pixsize_y, int do_w,
               int64_t nvis, const int64_t *vis_idx,
               int64_t npts, const int32_t *pix_p, const int32_t *pix_q, const double *pix_val,
               double *out_re, double *out_im) {
    (void)nrow;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nvis; ++t) {
        int64_t k = vis_idx[t];
        int64_t r = k / nchan, c = k % nchan;
        double s = freq[c] / C_LIGHT;
        double u = uvw[3 * r + 0] * s, v = uvw[3 * r + 1] * s;
        double w = do_w ? uvw[3 * r + 2] * s : 0.0;
        kahan_t ar = {0.0, 0.0}, ai = {0.0, 0.0};
        for (int64_t j = 0; j < npts; ++j) {
            double l, m, n, nm1;
            pixel_lmn(pix_p[j], pix_q[j], npix_x, npix_y, pixsize_x, pixsize_y, &l, &m, &n, &nm1);
            double ph = u * l + v * m - w * nm1;
            ph -= nearbyint(ph);
            double amp = pix_val[j] / n;
            double sn = sin(TWO_PI * ph), cs = cos(TWO_PI * ph);
            /* exp(-2 pi i ph) = cos - i sin */
            kahan_add(&ar, amp * cs);
            kahan_add(&ai, -amp * sn);
        }
        out_re[t] = ar.s;
        out_im[t] = ai.s;
    }
    return 0;
}

/* Adjoint at a list of pixels, summing over all nrow*nchan visibilities whose
 * select flag is non-zero (select may be NULL = all). */
int o1_adjoint(int64_t nrow, int64_t nchan, const double *uvw, const double *freq,
               int npix_x, int npix_y, double pixsize_x, double pixsize_y, int do_w,
               const double *vis_re, const double *vis_im, const uint8_t *select,
               int64_t npts, const int32_t *pix_p, const int32_t *pix_q, double *out) {
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < npts; ++j) {
        double l, m, n, nm1;
        pixel_lmn(pix_p[j], pix_q[j], npix_x, npix_y, pixsize_x, pixsize_y, &l, &m, &n, &nm1);
        kahan_t acc = {0.0, 0.0};
        for (int64_t r = 0; r < nrow; ++r) {
            for (int64_t c = 0; c < nchan; ++c) {
                int64_t k = r * nchan + c;
                if (select && !select[k]) continue;
                double s = freq[c] / C_LIGHT;
                double u = uvw[3 * r + 0] * s, v = uvw[3 * r + 1] * s;
                double w = do_w ? uvw[3 * r + 2] * s : 0.0;
                double ph = u * l + v * m - w * nm1;
                ph -= nearbyint(ph);
                double sn = sin(TWO_PI * ph), cs = cos(TWO_PI * ph);
                /* Re(d * exp(+2 pi i ph)) = re*cos - im*sin */
                kahan_add(&acc, vis_re[k] * cs - vis_im[k] * sn);
            }
        }
        out[j] = acc.s / n;
    }
    return 0;
}
