/*
 * FP64 CPU oracle for LiDAR depth densification (test infrastructure only).
 *
 * This file is test infrastructure, not the product. Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it. It shares no source,
 * header, table or helper with the GPU library.
 *
 * What it computes, each function citing the passage it follows:
 *
 *   oracle_project       Sec. 2 (the sweeps of one viewpoint, combined, are
 *                        mapped into its camera as a single sparse depth
 *                        image) with a nearest-depth z-buffer; the collision
 *                        rule is the reading stated below.
 *   oracle_densify       Eq. 1-4 (joint bilateral filter, gather form) over
 *                        the square window of Algorithm 1, in double.
 *   oracle_densify_plain Eq. 1-4 evaluated literally (product of the two
 *                        Gaussians, no common factor removed); used to pin
 *                        oracle_densify on inputs where nothing underflows.
 *   oracle_densify_alg1  Algorithm 1 steps 1-5 (materialised weight volume,
 *                        transpose-convolution scatter, normalisation).
 *   oracle_densify_grad  derivative of the Eq. 1 output with respect to the
 *                        input depths and the two Gaussian widths (Sec. 4:
 *                        the filter parameters are trainable by
 *                        backpropagation).
 *
 * Readings where the paper is silent (each one is listed in the design
 * notes): depth is camera-frame Z; pixel (col,row) covers u in [col,col+1),
 * v in [row,row+1) (floor, not round); points with Z <= 0, non-finite
 * values, (float)Z == 0 or (float)Z == inf, or u,v outside the image are
 * culled; the nearest (smallest float Z) point wins a pixel and an exact
 * float tie goes to the smaller merged index; the window is the full
 * (2r+1)^2 square including the centre, clipped at the image border
 * (equivalent to zero-padding D and B); colour distance is the squared L2
 * norm of raw 0..255 RGB; an output pixel is valid iff its window holds at
 * least one valid sample, and invalid pixels carry depth 0.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 * No FMA contraction, so every product and sum below rounds on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define EMPTY_KEY UINT64_MAX

static uint32_t float_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return u;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Projection of merged points into the camera and nearest-depth z-buffer.
 *
 * pts      n x 3 float32 world xyz, merged sweep order (index i = position)
 * pose     camera-from-world [R|t], row-major 3x4 doubles
 * intr     fx, fy, cx, cy
 * keys     W*H uint64 out: (bits(float Z) << 32) | i of the winner, or
 *          UINT64_MAX where no point landed
 * depth    W*H float out: float Z of the winner, 0 elsewhere (may be NULL)
 * valid    W*H uint8 out: 1 where a point landed (may be NULL)
 *
 * Returns the number of points that landed in the image.
 */
/* Projection core. With sweep != NULL a point of an older sweep
 * (sweep[i] != latest) whose pixel lies in the motion mask is dropped
 * before it competes for the pixel (afterimage removal, below). */
static int64_t project_core(const float *pts, int64_t n, const double *pose,
                            const double *intr, int32_t width, int32_t height,
                            uint64_t *keys, float *depth, uint8_t *valid,
                            const int8_t *sweep, int8_t latest,
                            const uint8_t *motion) {
    const double fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    const int64_t npix = (int64_t)width * height;
    int64_t landed = 0;
    for (int64_t p = 0; p < npix; ++p) keys[p] = EMPTY_KEY;
    for (int64_t i = 0; i < n; ++i) {
        const double x = (double)pts[3 * i + 0];
        const double y = (double)pts[3 * i + 1];
        const double z = (double)pts[3 * i + 2];
        /* rigid transform, each row summed left to right */
        double X = pose[0] * x;
        X = X + pose[1] * y;
        X = X + pose[2] * z;
        X = X + pose[3];
        double Y = pose[4] * x;
        Y = Y + pose[5] * y;
        Y = Y + pose[6] * z;
        Y = Y + pose[7];
        double Z = pose[8] * x;
        Z = Z + pose[9] * y;
        Z = Z + pose[10] * z;
        Z = Z + pose[11];
        if (!(Z > 0.0) || !isfinite(Z)) continue;
        /* pinhole model: pixel coordinate = focal * (X/Z) + principal point */
        const double u = fx * (X / Z) + cx;
        const double v = fy * (Y / Z) + cy;
        if (!(u >= 0.0 && u < (double)width)) continue;
        if (!(v >= 0.0 && v < (double)height)) continue;
        const int64_t col = (int64_t)floor(u);
        const int64_t row = (int64_t)floor(v);
        const float zf = (float)Z;
        if (zf == 0.0f || isinf(zf)) continue;
        const uint64_t key = ((uint64_t)float_bits(zf) << 32) | (uint64_t)(uint32_t)i;
        const int64_t pix = row * width + col;
        if (sweep && sweep[i] != latest && motion[pix]) continue;
        if (key < keys[pix]) keys[pix] = key;
        ++landed;
    }
    for (int64_t p = 0; p < npix; ++p) {
        const int hit = keys[p] != EMPTY_KEY;
        if (valid) valid[p] = (uint8_t)hit;
        if (depth) {
            if (hit) {
                uint32_t b = (uint32_t)(keys[p] >> 32);
                float f;
                memcpy(&f, &b, sizeof f);
                depth[p] = f;
            } else {
                depth[p] = 0.0f;
            }
        }
    }
    return landed;
}

int64_t oracle_project(const float *pts, int64_t n, const double *pose,
                       const double *intr, int32_t width, int32_t height,
                       uint64_t *keys, float *depth, uint8_t *valid) {
    return project_core(pts, n, pose, intr, width, height, keys, depth, valid,
                        NULL, 0, NULL);
}

/* 1/(2 sigma^2); an infinite sigma makes its Gaussian identically 1. */
static double half_inv_var(double sigma) {
    if (isinf(sigma)) return 0.0;
    return 1.0 / (2.0 * sigma * sigma);
}

/* squared L2 distance of two RGB triplets in raw 0..255 units (exact) */
static int64_t color_dist2(const uint8_t *rgb, int64_t p, int64_t q) {
    int64_t c = 0;
    for (int ch = 0; ch < 3; ++ch) {
        const int64_t d = (int64_t)rgb[3 * p + ch] - (int64_t)rgb[3 * q + ch];
        c += d * d;
    }
    return c;
}

/*
 * Joint bilateral filter, Eq. 1-4, gather form.
 *
 * For each pixel x, over the valid samples n in the (2r+1)^2 window around x
 * (clipped to the image):
 *     w(x,n) = exp(-|I(x)-I(n)|^2 / (2 sr^2)) * exp(-|x-n|^2 / (2 ss^2))
 *     out(x) = sum w D(n) / sum w
 * The two Gaussians are combined into exp(E) with
 *     E = -c/(2 sr^2) - s/(2 ss^2),
 * and every weight of one output pixel is divided by the same positive
 * constant exp(Emax(x)) before summing (Emax = largest E in the window).
 * That constant cancels between numerator and denominator, so the ratio is
 * Eq. 1 unchanged; it only keeps the weights away from underflow.
 *
 * depth   H*W float32 sparse depth (read only where valid == 1)
 * valid   H*W uint8 sample mask B
 * rgb     H*W*3 uint8 guide image, interleaved
 * out     H*W double dense depth (0 where mask == 0)
 * mask    H*W uint8 output validity: 1 iff the window holds a valid sample
 * count   H*W int32 number of valid samples in the window (may be NULL)
 * wsum    H*W double sum of the rescaled weights (may be NULL)
 * emax    H*W double the per-pixel Emax used above (may be NULL)
 *
 * Returns the number of (output pixel, valid sample) pairs.
 */
int64_t oracle_densify(const float *depth, const uint8_t *valid,
                       const uint8_t *rgb, int32_t height, int32_t width,
                       int32_t r, double sigma_s, double sigma_r, double *out,
                       uint8_t *mask, int32_t *count, double *wsum,
                       double *emax) {
    const double kr = half_inv_var(sigma_r);
    const double ks = half_inv_var(sigma_s);
    int64_t pairs = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : pairs)
    for (int32_t y = 0; y < height; ++y) {
        for (int32_t x = 0; x < width; ++x) {
            const int64_t p = (int64_t)y * width + x;
            /* pass 1: count and largest exponent */
            int32_t cnt = 0;
            double em = -INFINITY;
            for (int32_t b = -r; b <= r; ++b) {
                const int32_t yy = y + b;
                if (yy < 0 || yy >= height) continue;
                for (int32_t a = -r; a <= r; ++a) {
                    const int32_t xx = x + a;
                    if (xx < 0 || xx >= width) continue;
                    const int64_t q = (int64_t)yy * width + xx;
                    if (!valid[q]) continue;
                    const double c = (double)color_dist2(rgb, p, q);
                    const double s = (double)(a * a + b * b);
                    const double e = -(c * kr) - (s * ks);
                    if (e > em) em = e;
                    ++cnt;
                }
            }
            /* pass 2: weighted sums */
            double num = 0.0, den = 0.0;
            if (cnt > 0) {
                for (int32_t b = -r; b <= r; ++b) {
                    const int32_t yy = y + b;
                    if (yy < 0 || yy >= height) continue;
                    for (int32_t a = -r; a <= r; ++a) {
                        const int32_t xx = x + a;
                        if (xx < 0 || xx >= width) continue;
                        const int64_t q = (int64_t)yy * width + xx;
                        if (!valid[q]) continue;
                        const double c = (double)color_dist2(rgb, p, q);
                        const double s = (double)(a * a + b * b);
                        const double e = -(c * kr) - (s * ks);
                        const double w = exp(e - em);
                        num += w * (double)depth[q];
                        den += w;
                    }
                }
            }
            out[p] = cnt > 0 ? num / den : 0.0;
            mask[p] = (uint8_t)(cnt > 0);
            if (count) count[p] = cnt;
            if (wsum) wsum[p] = den;
            if (emax) emax[p] = em;
            pairs += cnt;
        }
    }
    return pairs;
}

/*
 * Sensitivity of Eq. 1-4 to errors in the weights: for each pixel with a
 * valid sample, S(x) = sum_i w_i |D_i - out(x)| / sum_i w_i over the same
 * window and weights as oracle_densify, with out = its output (passed in).
 * Since out is a weighted mean, multiplying each weight by (1 + e_i) with
 * |e_i| <= e moves it by at most e S(x) / (1 - e): the per-pixel bound of
 * reduced-precision weights. S = 0 where the window holds no sample.
 */
void oracle_densify_spread(const float *depth, const uint8_t *valid,
                           const uint8_t *rgb, int32_t height, int32_t width,
                           int32_t r, double sigma_s, double sigma_r,
                           const double *out, double *spread) {
    const double kr = half_inv_var(sigma_r);
    const double ks = half_inv_var(sigma_s);
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t y = 0; y < height; ++y) {
        for (int32_t x = 0; x < width; ++x) {
            const int64_t p = (int64_t)y * width + x;
            double em = -INFINITY;
            for (int32_t b = -r; b <= r; ++b) {
                const int32_t yy = y + b;
                if (yy < 0 || yy >= height) continue;
                for (int32_t a = -r; a <= r; ++a) {
                    const int32_t xx = x + a;
                    if (xx < 0 || xx >= width) continue;
                    const int64_t q = (int64_t)yy * width + xx;
                    if (!valid[q]) continue;
                    const double e = -((double)color_dist2(rgb, p, q) * kr) -
                                     ((double)(a * a + b * b) * ks);
                    if (e > em) em = e;
                }
            }
            double dev = 0.0, den = 0.0;
            if (em > -INFINITY) {
                for (int32_t b = -r; b <= r; ++b) {
                    const int32_t yy = y + b;
                    if (yy < 0 || yy >= height) continue;
                    for (int32_t a = -r; a <= r; ++a) {
                        const int32_t xx = x + a;
                        if (xx < 0 || xx >= width) continue;
                        const int64_t q = (int64_t)yy * width + xx;
                        if (!valid[q]) continue;
                        const double e = -((double)color_dist2(rgb, p, q) * kr) -
                                         ((double)(a * a + b * b) * ks);
                        const double w = exp(e - em);
                        dev += w * fabs((double)depth[q] - out[p]);
                        den += w;
                    }
                }
            }
            spread[p] = den > 0.0 ? dev / den : 0.0;
        }
    }
}

/*
 * Eq. 1-4 taken literally: w = w_c * w_p with each Gaussian evaluated on its
 * own and no rescaling. Where every weight of a window underflows the ratio
 * is 0/0; callers use it only on inputs where that cannot happen.
 */
void oracle_densify_plain(const float *depth, const uint8_t *valid,
                          const uint8_t *rgb, int32_t height, int32_t width,
                          int32_t r, double sigma_s, double sigma_r,
                          double *out, uint8_t *mask) {
    const double kr = half_inv_var(sigma_r);
    const double ks = half_inv_var(sigma_s);
    for (int32_t y = 0; y < height; ++y) {
        for (int32_t x = 0; x < width; ++x) {
            const int64_t p = (int64_t)y * width + x;
            double num = 0.0, den = 0.0;
            int32_t cnt = 0;
            for (int32_t b = -r; b <= r; ++b) {
                for (int32_t a = -r; a <= r; ++a) {
                    const int32_t xx = x + a, yy = y + b;
                    if (xx < 0 || xx >= width || yy < 0 || yy >= height) continue;
                    const int64_t q = (int64_t)yy * width + xx;
                    if (!valid[q]) continue;
                    const double wc = exp(-(double)color_dist2(rgb, p, q) * kr);
                    const double wp = exp(-(double)(a * a + b * b) * ks);
                    num += (double)depth[q] * wc * wp;
                    den += wc * wp;
                    ++cnt;
                }
            }
            out[p] = cnt > 0 ? num / den : 0.0;
            mask[p] = (uint8_t)(cnt > 0);
        }
    }
}

/*
 * Algorithm 1, steps 1-5, with the weight volume materialised.
 *
 * Step 1-3 build w(x,y,k), k = (2r+1)(r+a) + (r+b), from the colour
 * difference between the source (x,y) and its neighbour (x+a,y+b) and the
 * offset's spatial Gaussian; step 4 scatters D(x,y) w and B(x,y) w to
 * (x+a,y+b) (targets outside the image are dropped; D is read as 0 where
 * B = 0); step 5 divides. A separate count volume scattered the same way
 * gives the validity mask. Memory is H*W*(2r+1)^2 doubles: tiny inputs only.
 * Returns 0, or -1 if the volume cannot be allocated.
 */
int oracle_densify_alg1(const float *depth, const uint8_t *valid,
                        const uint8_t *rgb, int32_t height, int32_t width,
                        int32_t r, double sigma_s, double sigma_r, double *out,
                        uint8_t *mask) {
    const int32_t side = 2 * r + 1;
    const int64_t taps = (int64_t)side * side;
    const int64_t npix = (int64_t)height * width;
    double *w = (double *)malloc(sizeof(double) * (size_t)(npix * taps));
    double *dacc = (double *)calloc((size_t)npix, sizeof(double));
    double *wacc = (double *)calloc((size_t)npix, sizeof(double));
    int32_t *cacc = (int32_t *)calloc((size_t)npix, sizeof(int32_t));
    if (!w || !dacc || !wacc || !cacc) {
        free(w); free(dacc); free(wacc); free(cacc);
        return -1;
    }
    const double kr = half_inv_var(sigma_r);
    const double ks = half_inv_var(sigma_s);
    /* steps 1 and 2: colour difference per channel, then colour Gaussian */
    for (int32_t y = 0; y < height; ++y)
        for (int32_t x = 0; x < width; ++x)
            for (int32_t a = -r; a <= r; ++a)
                for (int32_t b = -r; b <= r; ++b) {
                    const int64_t k = (int64_t)side * (r + a) + (r + b);
                    const int64_t idx = ((int64_t)y * width + x) * taps + k;
                    const int32_t xx = x + a, yy = y + b;
                    if (xx < 0 || xx >= width || yy < 0 || yy >= height) {
                        w[idx] = 0.0; /* never scattered: target is outside */
                        continue;
                    }
                    double sq = 0.0;
                    for (int ch = 0; ch < 3; ++ch) {
                        const double d = (double)rgb[3 * ((int64_t)y * width + x) + ch] -
                                         (double)rgb[3 * ((int64_t)yy * width + xx) + ch];
                        sq += d * d;
                    }
                    w[idx] = exp(-sq * kr);
                }
    /* step 3: Hadamard product with the spatial Gaussian of each offset */
    for (int64_t pix = 0; pix < npix; ++pix)
        for (int32_t a = -r; a <= r; ++a)
            for (int32_t b = -r; b <= r; ++b) {
                const int64_t k = (int64_t)side * (r + a) + (r + b);
                w[pix * taps + k] *= exp(-(double)(a * a + b * b) * ks);
            }
    /* step 4: transpose convolution, scattering depth and mask */
    for (int32_t y = 0; y < height; ++y)
        for (int32_t x = 0; x < width; ++x) {
            const int64_t src = (int64_t)y * width + x;
            const double dsrc = valid[src] ? (double)depth[src] : 0.0;
            const double bsrc = valid[src] ? 1.0 : 0.0;
            for (int32_t a = -r; a <= r; ++a)
                for (int32_t b = -r; b <= r; ++b) {
                    const int32_t xx = x + a, yy = y + b;
                    if (xx < 0 || xx >= width || yy < 0 || yy >= height) continue;
                    const int64_t k = (int64_t)side * (r + a) + (r + b);
                    const int64_t dst = (int64_t)yy * width + xx;
                    dacc[dst] += dsrc * w[src * taps + k];
                    wacc[dst] += bsrc * w[src * taps + k];
                    cacc[dst] += valid[src] ? 1 : 0;
                }
        }
    /* step 5: normalisation */
    for (int64_t pix = 0; pix < npix; ++pix) {
        mask[pix] = (uint8_t)(cacc[pix] > 0);
        out[pix] = cacc[pix] > 0 ? dacc[pix] / wacc[pix] : 0.0;
    }
    free(w); free(dacc); free(wacc); free(cacc);
    return 0;
}

/*
 * Gradient of a scalar loss L through the filter, given g = dL/d out.
 *
 * With E_i = -c_i/(2 sr^2) - s_i/(2 ss^2), w_i = exp(E_i), W = sum w_i and
 * out = sum w_i D_i / W over the valid samples i of the window of x:
 *     d out / d D_i  = w_i / W
 *     d out / d sr   = sum_i w_i (c_i / sr^3) (D_i - out) / W
 *     d out / d ss   = sum_i w_i (s_i / ss^3) (D_i - out) / W
 * (d E_i / d sr = c_i / sr^3, and the quotient rule gives the D_i - out
 * factor). Pixels with mask 0 contribute nothing. An infinite sigma has a
 * zero derivative.
 *
 * g         H*W double upstream gradient (read where the output is valid)
 * grad_d    H*W double out: dL/dD at every pixel (0 where valid == 0)
 * grad_ss   out: dL/d sigma_s
 * grad_sr   out: dL/d sigma_r
 */
void oracle_densify_grad(const float *depth, const uint8_t *valid,
                         const uint8_t *rgb, int32_t height, int32_t width,
                         int32_t r, double sigma_s, double sigma_r,
                         const double *g, double *grad_d, double *grad_ss,
                         double *grad_sr) {
    const double kr = half_inv_var(sigma_r);
    const double ks = half_inv_var(sigma_s);
    const double dsr = isinf(sigma_r) ? 0.0 : 1.0 / (sigma_r * sigma_r * sigma_r);
    const double dss = isinf(sigma_s) ? 0.0 : 1.0 / (sigma_s * sigma_s * sigma_s);
    const int64_t npix = (int64_t)height * width;
    for (int64_t p = 0; p < npix; ++p) grad_d[p] = 0.0;
    double gs = 0.0, gr = 0.0;
    for (int32_t y = 0; y < height; ++y) {
        for (int32_t x = 0; x < width; ++x) {
            const int64_t p = (int64_t)y * width + x;
            const double gp = g[p];
            /* forward for this pixel: Emax, W, out */
            int32_t cnt = 0;
            double em = -INFINITY;
            for (int32_t b = -r; b <= r; ++b)
                for (int32_t a = -r; a <= r; ++a) {
                    const int32_t xx = x + a, yy = y + b;
                    if (xx < 0 || xx >= width || yy < 0 || yy >= height) continue;
                    const int64_t q = (int64_t)yy * width + xx;
                    if (!valid[q]) continue;
                    const double e = -((double)color_dist2(rgb, p, q) * kr) -
                                     ((double)(a * a + b * b) * ks);
                    if (e > em) em = e;
                    ++cnt;
                }
            if (cnt == 0 || gp == 0.0) continue;
            double num = 0.0, den = 0.0;
            for (int32_t b = -r; b <= r; ++b)
                for (int32_t a = -r; a <= r; ++a) {
                    const int32_t xx = x + a, yy = y + b;
                    if (xx < 0 || xx >= width || yy < 0 || yy >= height) continue;
                    const int64_t q = (int64_t)yy * width + xx;
                    if (!valid[q]) continue;
                    const double e = -((double)color_dist2(rgb, p, q) * kr) -
                                     ((double)(a * a + b * b) * ks);
                    const double w = exp(e - em);
                    num += w * (double)depth[q];
                    den += w;
                }
            const double o = num / den;
            /* backward */
            double ar = 0.0, as = 0.0;
            for (int32_t b = -r; b <= r; ++b)
                for (int32_t a = -r; a <= r; ++a) {
                    const int32_t xx = x + a, yy = y + b;
                    if (xx < 0 || xx >= width || yy < 0 || yy >= height) continue;
                    const int64_t q = (int64_t)yy * width + xx;
                    if (!valid[q]) continue;
                    const double c = (double)color_dist2(rgb, p, q);
                    const double s = (double)(a * a + b * b);
                    const double w = exp(-(c * kr) - (s * ks) - em) / den;
                    grad_d[q] += gp * w;
                    ar += w * c * ((double)depth[q] - o);
                    as += w * s * ((double)depth[q] - o);
                }
            gr += gp * ar * dsr;
            gs += gp * as * dss;
        }
    }
    *grad_ss = gs;
    *grad_sr = gr;
}

/* ------------------------------------------------------------------------
 * Two-stage filtering (Sec. 5: a first pass at one third of the resolution
 * in each dimension, reached by pooling, then a pass at full resolution on
 * the restored map). The paper names pooling and restoring without saying
 * how; the readings here:
 *   pooling   3x3 cells (the last row and column of cells may be partial:
 *             they pool only the pixels inside the image); the pooled depth
 *             is the mean of the cell's valid depths, summed in double in
 *             row-major order and rounded once to float; the pooled mask
 *             says whether the cell holds a valid depth; the pooled colour
 *             is the rounded mean of every pixel of the cell per channel,
 *             floor((sum + n/2) / n) in integers;
 *   restoring nearest neighbour: full-resolution pixel (x, y) takes cell
 *             (x / 3, y / 3) (integer division); the second pass sees the
 *             original depth where B = 1, else the restored first-pass depth
 *             where the first pass is valid, else nothing.
 * ---------------------------------------------------------------------- */

void oracle_pool3(const float *depth, const uint8_t *valid, const uint8_t *rgb,
                  int32_t h, int32_t w, float *depth1, uint8_t *valid1,
                  uint8_t *rgb1) {
    const int32_t h1 = (h + 2) / 3, w1 = (w + 2) / 3;
    for (int32_t cy = 0; cy < h1; ++cy) {
        for (int32_t cx = 0; cx < w1; ++cx) {
            double sum = 0.0;
            int n_valid = 0, n_pix = 0;
            int csum[3] = {0, 0, 0};
            for (int32_t y = 3 * cy; y < 3 * cy + 3 && y < h; ++y) {
                for (int32_t x = 3 * cx; x < 3 * cx + 3 && x < w; ++x) {
                    const int64_t p = (int64_t)y * w + x;
                    ++n_pix;
                    for (int c = 0; c < 3; ++c) csum[c] += rgb[3 * p + c];
                    if (valid[p]) {
                        sum = sum + (double)depth[p];
                        ++n_valid;
                    }
                }
            }
            const int64_t q = (int64_t)cy * w1 + cx;
            depth1[q] = n_valid ? (float)(sum / (double)n_valid) : 0.0f;
            valid1[q] = (uint8_t)(n_valid > 0);
            for (int c = 0; c < 3; ++c)
                rgb1[3 * q + c] = (uint8_t)((csum[c] + n_pix / 2) / n_pix);
        }
    }
}

void oracle_restore_merge(const float *depth, const uint8_t *valid,
                          const float *out1, const uint8_t *mask1, int32_t h,
                          int32_t w, float *depth2, uint8_t *valid2) {
    const int32_t w1 = (w + 2) / 3;
    for (int32_t y = 0; y < h; ++y) {
        for (int32_t x = 0; x < w; ++x) {
            const int64_t p = (int64_t)y * w + x;
            const int64_t q = (int64_t)(y / 3) * w1 + x / 3;
            if (valid[p]) {
                depth2[p] = depth[p];
                valid2[p] = 1;
            } else if (mask1[q]) {
                depth2[p] = out1[q];
                valid2[p] = 1;
            } else {
                depth2[p] = 0.0f;
                valid2[p] = 0;
            }
        }
    }
}

/* ------------------------------------------------------------------------
 * Occluded-point removal (Sec. 4.1: the merged depth map is averaged and
 * points lying well behind the average are dropped as hidden from the
 * camera). Readings: the average at a valid pixel is the mean of the valid
 * depths in its (2k+1)^2 window (centre included, clipped at the border),
 * summed in double in row-major order; the pixel's sample is dropped when
 * D - mean > tau * mean, evaluated in double. One pass over the original
 * map.
 * ---------------------------------------------------------------------- */

void oracle_remove_occluded(const float *depth, const uint8_t *valid, int32_t h,
                            int32_t w, int32_t k, double tau, uint8_t *valid_out) {
    for (int32_t y = 0; y < h; ++y) {
        for (int32_t x = 0; x < w; ++x) {
            const int64_t p = (int64_t)y * w + x;
            if (!valid[p]) {
                valid_out[p] = 0;
                continue;
            }
            double sum = 0.0;
            int n = 0;
            for (int32_t yy = y - k; yy <= y + k; ++yy) {
                if (yy < 0 || yy >= h) continue;
                for (int32_t xx = x - k; xx <= x + k; ++xx) {
                    if (xx < 0 || xx >= w) continue;
                    const int64_t q = (int64_t)yy * w + xx;
                    if (valid[q]) {
                        sum = sum + (double)depth[q];
                        ++n;
                    }
                }
            }
            const double mean = sum / (double)n;
            valid_out[p] = (uint8_t)!((double)depth[p] - mean > tau * mean);
        }
    }
}

/* ------------------------------------------------------------------------
 * Contour removal and back-projection to a coloured point cloud (Sec. 5:
 * unreliable depths along object contours are removed by thresholding the
 * depth gradient; Sec. 2: each viewpoint's coloured points are placed in
 * the common world frame). Readings: the gradient at a valid output pixel
 * is the largest |D(n) - D(x)| over its valid 4-neighbours (0 if it has
 * none), in double; the pixel is removed when that exceeds tau * D(x). A
 * kept pixel (col, row) becomes the camera point ((col + 0.5 - cx) Z / fx,
 * (row + 0.5 - cy) Z / fy, Z), Z = D(x), then the world point
 * R^T (p_c - t) for the camera-from-world pose [R|t], each coordinate a
 * left-to-right sum in double without FMA, rounded once to float. Points
 * are written in row-major pixel order with the pixel's colour.
 * ---------------------------------------------------------------------- */

static int contour_keep(const float *d, const uint8_t *m, int32_t h, int32_t w,
                        int32_t x, int32_t y, double tau) {
    const int64_t p = (int64_t)y * w + x;
    const double z = (double)d[p];
    double g = 0.0;
    const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    for (int i = 0; i < 4; ++i) {
        const int32_t xx = x + dx[i], yy = y + dy[i];
        if (xx < 0 || xx >= w || yy < 0 || yy >= h) continue;
        const int64_t q = (int64_t)yy * w + xx;
        if (!m[q]) continue;
        const double diff = fabs((double)d[q] - z);
        if (diff > g) g = diff;
    }
    return !(g > tau * z);
}

int64_t oracle_backproject(const float *dense, const uint8_t *mask,
                           const uint8_t *rgb, int32_t h, int32_t w,
                           const double *pose, const double *K, double tau,
                           float *xyz, uint8_t *rgb_out) {
    const double fx = K[0], fy = K[1], cx = K[2], cy = K[3];
    int64_t n = 0;
    for (int32_t y = 0; y < h; ++y) {
        for (int32_t x = 0; x < w; ++x) {
            const int64_t p = (int64_t)y * w + x;
            if (!mask[p] || !contour_keep(dense, mask, h, w, x, y, tau)) continue;
            const double Z = (double)dense[p];
            const double Xc = ((double)x + 0.5 - cx) * Z / fx;
            const double Yc = ((double)y + 0.5 - cy) * Z / fy;
            const double a = Xc - pose[3], b = Yc - pose[7], c = Z - pose[11];
            for (int i = 0; i < 3; ++i) {
                double s = pose[0 + i] * a;
                s = s + pose[4 + i] * b;
                s = s + pose[8 + i] * c;
                xyz[3 * n + i] = (float)s;
            }
            for (int i = 0; i < 3; ++i) rgb_out[3 * n + i] = rgb[3 * p + i];
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------------
 * Afterimage removal (Sec. 4.1: moving regions are found from the colour
 * change between consecutive RGB frames, thresholded at tau_m and closed
 * morphologically; there, points not from the most recent LiDAR frame are
 * discarded). Readings: motion where the squared RGB distance exceeds
 * tau_m^2 (in double); closing with a (2k+1)^2 square, the dilation
 * treating pixels outside the image as still, the erosion treating them as
 * moving (so the closing never removes motion at the border); the most
 * recent frame is the sweep with id `latest`.
 * ---------------------------------------------------------------------- */

void oracle_motion_mask(const uint8_t *rgb, const uint8_t *rgb_prev, int32_t h,
                        int32_t w, double tau, int32_t k, uint8_t *mask) {
    const int64_t n = (int64_t)h * w;
    uint8_t *raw = (uint8_t *)malloc((size_t)n);
    uint8_t *dil = (uint8_t *)malloc((size_t)n);
    for (int64_t p = 0; p < n; ++p) {
        int c = 0;
        for (int ch = 0; ch < 3; ++ch) {
            const int d = (int)rgb[3 * p + ch] - (int)rgb_prev[3 * p + ch];
            c += d * d;
        }
        raw[p] = (uint8_t)((double)c > tau * tau);
    }
    for (int32_t y = 0; y < h; ++y)
        for (int32_t x = 0; x < w; ++x) {
            uint8_t any = 0;
            for (int32_t yy = y - k; yy <= y + k; ++yy)
                for (int32_t xx = x - k; xx <= x + k; ++xx)
                    if (yy >= 0 && yy < h && xx >= 0 && xx < w &&
                        raw[(int64_t)yy * w + xx])
                        any = 1;
            dil[(int64_t)y * w + x] = any;
        }
    for (int32_t y = 0; y < h; ++y)
        for (int32_t x = 0; x < w; ++x) {
            uint8_t all = 1;
            for (int32_t yy = y - k; yy <= y + k; ++yy)
                for (int32_t xx = x - k; xx <= x + k; ++xx)
                    if (yy >= 0 && yy < h && xx >= 0 && xx < w &&
                        !dil[(int64_t)yy * w + xx])
                        all = 0;
            mask[(int64_t)y * w + x] = all;
        }
    free(raw);
    free(dil);
}

int64_t oracle_project_motion(const float *pts, int64_t n, const int8_t *sweep,
                              int8_t latest, const uint8_t *motion,
                              const double *pose, const double *intr,
                              int32_t width, int32_t height, uint64_t *keys,
                              float *depth, uint8_t *valid) {
    return project_core(pts, n, pose, intr, width, height, keys, depth, valid,
                        sweep, latest, motion);
}
