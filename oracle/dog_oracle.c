/*
 * Difference-of-Gaussians blob detector: FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes (arXiv:2010.08486, "Towards Online Steering of Flame Spray
 * Pyrolysis Nanoparticle Synthesis"):
 *   - scale space L(x,y,sigma) = g(sigma) * I                 (Sec. 3)
 *   - a ladder of Gaussian standard deviations sigma_i          (Sec. 4, Eq. 1;
 *     geometric form, see the readings below)
 *   - Gaussian kernels sampled out to truncate*sigma            (Sec. 4.1)
 *   - adjacent differences scaled by sigma_i (the DoG)          (Sec. 4, Eq. 2-3)
 *   - 3x3x3 maximum filter over (x, y, scale), kept where the
 *     value equals the neighbourhood maximum and exceeds the
 *     threshold                                                 (Sec. 4 and the
 *                                                                Thresh mask, Sec. 4.1)
 *   - blob radius sqrt(2)*sigma and overlap pruning             (Sec. 3, Sec. 4.1)
 *
 * Readings of points where the paper is silent or differs from the target
 * configuration:
 *   R1 ladder: geometric, k = floor(ln(smax/smin)/ln(ratio)) + 1 DoG planes,
 *      sigma_i = smin * ratio^i for i = 0..k (k+1 Gaussian planes).  The
 *      paper's Eq. 1 is arithmetic; the arithmetic form is also provided.
 *   R2 sign: D_i = sigma_i * (L_i - L_{i+1}), so bright blobs on a dark
 *      background give positive maxima (Eq. 2 with the opposite sign).
 *   R3 radius r = floor(truncate*sigma + 0.5); weights normalised over the
 *      truncated support so they sum to 1.
 *   R4 boundary: half-sample symmetric reflection, period 2n, for any offset.
 *   R5 the max filter ignores neighbours outside the cube (equivalent to
 *      -inf padding); equality is exact in FP64; every tied voxel is kept.
 *   R6 threshold: strict D > thr on the scaled response.
 *   R7 pruning: normalised overlap = lens area / area of the smaller disk;
 *      pairs visited in (y, x, scale) order; when the overlap exceeds the
 *      limit the blob with the smaller sigma is removed (the later one on a
 *      tie).  overlap >= 1 disables pruning.
 *   R7b coalescing: the same visits; the survivor takes the mean sigma of
 *      the pair, which later pairs see.
 *   R11 preprocessing (the optional first step of Sec. 4.1): Gaussian
 *      smoothing (sigma given, truncate 4, reflection), then a contrast
 *      stretch that saturates the given fraction of pixels, half at each
 *      end: with N pixels and m = floor(fraction * N / 2), lo and hi are the
 *      m-th smallest and m-th largest smoothed values (0-based order
 *      statistics m and N-1-m), and out = clamp((s - lo)/(hi - lo), 0, 1)
 *      (0 everywhere when hi == lo).
 *   R12 radius histogram: bin centres sqrt(2)*sigma_i for the k DoG scales;
 *      a blob goes to the nearest centre, the lower one on a tie.
 *
 * Everything is FP64 with round-to-nearest-even.  The only parallelism is an
 * OpenMP loop over independent output rows; every output value is computed by
 * the same sequence of operations whatever the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_PLANES 64

/* Thread count of the row loops (1 when built without OpenMP). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of DoG planes k of the geometric ladder (reading R1). */
int orc_num_dog_planes(double smin, double smax, double ratio)
{
    double x = log(smax / smin) / log(ratio);
    return (int)floor(x) + 1;
}

/* sigma_i = smin * ratio^i, i = 0..k (k+1 Gaussian planes). */
void orc_sigmas_geometric(double smin, double ratio, int k, double *out)
{
    for (int i = 0; i <= k; ++i)
        out[i] = smin * pow(ratio, (double)i);
}

/* Sec. 4, Eq. 1: arithmetic ladder with n_bin+1 values,
 * sigma_i = smin + i * (smax - smin) / n_bin for i = 0..n_bin. */
void orc_sigmas_arithmetic(double smin, double smax, int n_bin, double *out)
{
    double ds = (smax - smin) / (double)n_bin;
    for (int i = 0; i <= n_bin; ++i)
        out[i] = smin + (double)i * ds;
}

/* Kernel radius: sampling out to truncate*sigma, rounded to the nearest
 * integer (reading R3). */
int orc_radius(double sigma, double truncate)
{
    return (int)floor(truncate * sigma + 0.5);
}

/* Truncated, normalised Gaussian: w[j + r] for j = -r..r (Sec. 4.1). */
void orc_weights(double sigma, int r, double *w)
{
    double sum = 0.0;
    for (int j = -r; j <= r; ++j) {
        double v = exp(-(double)j * (double)j / (2.0 * sigma * sigma));
        w[j + r] = v;
        sum += v;
    }
    for (int j = -r; j <= r; ++j)
        w[j + r] /= sum;
}

/* Half-sample symmetric reflection of index t into [0, n) (reading R4):
 * the sequence is extended as x[0..n-1], x[n-1..0], x[0..n-1], ... */
int64_t orc_reflect(int64_t t, int64_t n)
{
    if (t >= 0 && t < n)
        return t;
    int64_t p = 2 * n;
    int64_t u = t % p;
    if (u < 0)
        u += p;
    return (u < n) ? u : (p - 1 - u);
}

/* One Gaussian blur, row pass (along x) then column pass (along y), both in
 * FP64 with reflection at the borders.  in, tmp and out are H x W, dense. */
void orc_blur(const double *in, int64_t H, int64_t W, double sigma,
              double truncate, double *tmp, double *out)
{
    int r = orc_radius(sigma, truncate);
    double *w = (double *)malloc(sizeof(double) * (size_t)(2 * r + 1));
    orc_weights(sigma, r, w);

#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int j = -r; j <= r; ++j)
                acc += w[j + r] * in[y * W + orc_reflect(x + j, W)];
            tmp[y * W + x] = acc;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int j = -r; j <= r; ++j)
                acc += w[j + r] * tmp[orc_reflect(y + j, H) * W + x];
            out[y * W + x] = acc;
        }
    }
    free(w);
}

/* Scale space and DoG for an explicit list of n_g = k+1 sigmas.
 * image: H x W fp32 with row stride `stride` (elements).
 * L: n_g planes H x W; D: k planes H x W with D_i = sigma_i*(L_i - L_{i+1})
 * (Sec. 4, Eq. 2-3, sign per reading R2).  Either output may be NULL only
 * if not wanted; L is then allocated internally. */
int orc_planes_sigmas(const float *image, int64_t H, int64_t W, int64_t stride,
                      int n_g, const double *sigmas, double truncate,
                      double *L, double *D)
{
    if (n_g < 2 || n_g > ORC_MAX_PLANES + 1 || H < 1 || W < 1 || stride < W)
        return -1;
    size_t px = (size_t)H * (size_t)W;
    double *img = (double *)malloc(sizeof(double) * px);
    double *tmp = (double *)malloc(sizeof(double) * px);
    double *Lb = L ? L : (double *)malloc(sizeof(double) * px * (size_t)n_g);
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x)
            img[y * W + x] = (double)image[y * stride + x];
    for (int i = 0; i < n_g; ++i)
        orc_blur(img, H, W, sigmas[i], truncate, tmp, Lb + (size_t)i * px);
    if (D) {
        for (int i = 0; i + 1 < n_g; ++i) {
            const double *a = Lb + (size_t)i * px;
            const double *b = Lb + (size_t)(i + 1) * px;
            double *d = D + (size_t)i * px;
            for (size_t p = 0; p < px; ++p)
                d[p] = sigmas[i] * (a[p] - b[p]);
        }
    }
    if (!L)
        free(Lb);
    free(tmp);
    free(img);
    return 0;
}

/* Geometric-ladder convenience wrapper.  Returns k, or -1 on bad input. */
int orc_planes(const float *image, int64_t H, int64_t W, int64_t stride,
               double smin, double smax, double ratio, double truncate,
               double *L, double *D)
{
    int k = orc_num_dog_planes(smin, smax, ratio);
    if (k < 1 || k > ORC_MAX_PLANES)
        return -1;
    double s[ORC_MAX_PLANES + 1];
    orc_sigmas_geometric(smin, ratio, k, s);
    if (orc_planes_sigmas(image, H, W, stride, k + 1, s, truncate, L, D) != 0)
        return -1;
    return k;
}

/* Maximum of D over the 3x3x3 neighbourhood of (i, y, x), neighbours outside
 * the k x H x W cube ignored (reading R5).  The centre is included. */
double orc_neigh_max(const double *D, int k, int64_t H, int64_t W, int i,
                     int64_t y, int64_t x)
{
    size_t px = (size_t)H * (size_t)W;
    double m = -INFINITY;
    for (int di = -1; di <= 1; ++di) {
        int ii = i + di;
        if (ii < 0 || ii >= k)
            continue;
        for (int64_t dy = -1; dy <= 1; ++dy) {
            int64_t yy = y + dy;
            if (yy < 0 || yy >= H)
                continue;
            for (int64_t dx = -1; dx <= 1; ++dx) {
                int64_t xx = x + dx;
                if (xx < 0 || xx >= W)
                    continue;
                double v = D[(size_t)ii * px + (size_t)(yy * W + xx)];
                if (v > m)
                    m = v;
            }
        }
    }
    return m;
}

/* Local-maximum search with threshold (Sec. 4: a value equal to the maximum
 * of its 3x3x3 neighbourhood is a local maximum; Sec. 4.1 Thresh: and it
 * must exceed the threshold).  Writes up to `cap` blobs as (y, x, i) triples
 * and responses, in (y, x, i) order.  Returns the total number found (which
 * may exceed cap). */
int64_t orc_nms(const double *D, int k, int64_t H, int64_t W, double thr,
                int32_t *yxi, double *resp, int64_t cap)
{
    size_t px = (size_t)H * (size_t)W;
    int64_t n = 0;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            for (int i = 0; i < k; ++i) {
                double v = D[(size_t)i * px + (size_t)(y * W + x)];
                if (!(v > thr))
                    continue;
                if (v != orc_neigh_max(D, k, H, W, i, y, x))
                    continue;
                if (n < cap) {
                    yxi[3 * n + 0] = (int32_t)y;
                    yxi[3 * n + 1] = (int32_t)x;
                    yxi[3 * n + 2] = (int32_t)i;
                    if (resp)
                        resp[n] = v;
                }
                ++n;
            }
        }
    }
    return n;
}

/* Area of intersection of two disks of radii r1, r2 whose centres are d
 * apart (circle-circle lens). */
double orc_lens_area(double d, double r1, double r2)
{
    if (d >= r1 + r2)
        return 0.0;
    double rmin = r1 < r2 ? r1 : r2;
    if (d <= fabs(r1 - r2))
        return M_PI * rmin * rmin;
    double c1 = (d * d + r1 * r1 - r2 * r2) / (2.0 * d * r1);
    double c2 = (d * d + r2 * r2 - r1 * r1) / (2.0 * d * r2);
    if (c1 > 1.0) c1 = 1.0;
    if (c1 < -1.0) c1 = -1.0;
    if (c2 > 1.0) c2 = 1.0;
    if (c2 < -1.0) c2 = -1.0;
    double k = (-d + r1 + r2) * (d + r1 - r2) * (d - r1 + r2) * (d + r1 + r2);
    if (k < 0.0)
        k = 0.0;
    return r1 * r1 * acos(c1) + r2 * r2 * acos(c2) - 0.5 * sqrt(k);
}

/* Normalised overlap of two blobs of scale sigma (radius sqrt(2)*sigma,
 * Sec. 3): intersection over the area of the smaller disk. */
double orc_overlap_fraction(double y1, double x1, double s1,
                            double y2, double x2, double s2)
{
    double r1 = M_SQRT2 * s1, r2 = M_SQRT2 * s2;
    double d = sqrt((y1 - y2) * (y1 - y2) + (x1 - x2) * (x1 - x2));
    double rmin = r1 < r2 ? r1 : r2;
    return orc_lens_area(d, r1, r2) / (M_PI * rmin * rmin);
}

/* Overlap pruning (Sec. 4.1; reading R7).  Blobs must be given in (y, x,
 * scale) order.  keep[n] is set to 1 for survivors, 0 for removed blobs.
 * Returns the number kept. */
int64_t orc_prune(int64_t n, const int32_t *y, const int32_t *x,
                  const double *sigma, double overlap, uint8_t *keep)
{
    for (int64_t a = 0; a < n; ++a)
        keep[a] = 1;
    if (overlap < 1.0) {
        for (int64_t a = 0; a < n; ++a) {
            if (!keep[a])
                continue;
            for (int64_t b = a + 1; b < n; ++b) {
                if (!keep[b])
                    continue;
                double f = orc_overlap_fraction(y[a], x[a], sigma[a],
                                                y[b], x[b], sigma[b]);
                if (f > overlap) {
                    if (sigma[a] < sigma[b]) {
                        keep[a] = 0;
                        break;
                    }
                    keep[b] = 0;
                }
            }
        }
    }
    int64_t m = 0;
    for (int64_t a = 0; a < n; ++a)
        m += keep[a];
    return m;
}

/* Coalescing form of the overlap step (Sec. 4.1: overlapping blobs are
 * coalesced by averaging the radius; reading R7b).  Same visiting order and
 * overlap test as orc_prune, on the blobs' current sigmas: of an overlapping
 * pair the blob with the smaller sigma is removed (b on a tie) and the other
 * takes the mean of the two sigmas, which later pairs then see.  sigma_out[n]
 * receives every blob's final sigma (meaningful for survivors).  Returns the
 * number kept. */
int64_t orc_prune_coalesce(int64_t n, const int32_t *y, const int32_t *x,
                           const double *sigma, double overlap, uint8_t *keep,
                           double *sigma_out)
{
    for (int64_t a = 0; a < n; ++a) {
        keep[a] = 1;
        sigma_out[a] = sigma[a];
    }
    if (overlap < 1.0) {
        for (int64_t a = 0; a < n; ++a) {
            if (!keep[a])
                continue;
            for (int64_t b = a + 1; b < n; ++b) {
                if (!keep[b])
                    continue;
                double f = orc_overlap_fraction(y[a], x[a], sigma_out[a],
                                                y[b], x[b], sigma_out[b]);
                if (f > overlap) {
                    double mean = 0.5 * (sigma_out[a] + sigma_out[b]);
                    if (sigma_out[a] < sigma_out[b]) {
                        keep[a] = 0;
                        sigma_out[b] = mean;
                        break;
                    }
                    keep[b] = 0;
                    sigma_out[a] = mean;
                }
            }
        }
    }
    int64_t m = 0;
    for (int64_t a = 0; a < n; ++a)
        m += keep[a];
    return m;
}

static int orc_cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Preprocessing (Sec. 4.1, optional first step; reading R11).  image: H x W
 * fp32 with row stride `stride`; sigma 0 skips the smoothing.  smoothed and
 * out are H x W (smoothed may be NULL); lo_hi[0..1] receive the stretch
 * limits.  Returns 0, or -1 on bad input. */
int orc_preprocess(const float *image, int64_t H, int64_t W, int64_t stride,
                   double sigma, double saturated, double *smoothed, double *out,
                   double *lo_hi)
{
    if (H < 1 || W < 1 || stride < W || !(sigma >= 0.0) || !(saturated >= 0.0) ||
        !(saturated < 1.0))
        return -1;
    int64_t N = H * W;
    double *in = (double *)malloc(sizeof(double) * (size_t)N);
    double *s = (double *)malloc(sizeof(double) * (size_t)N);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)N);
    double *sorted = (double *)malloc(sizeof(double) * (size_t)N);
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x)
            in[y * W + x] = (double)image[y * stride + x];
    if (sigma > 0.0)
        orc_blur(in, H, W, sigma, 4.0, tmp, s);
    else
        memcpy(s, in, sizeof(double) * (size_t)N);
    memcpy(sorted, s, sizeof(double) * (size_t)N);
    qsort(sorted, (size_t)N, sizeof(double), orc_cmp_double);
    int64_t m = (int64_t)floor(saturated * (double)N / 2.0);
    if (m > (N - 1) / 2)
        m = (N - 1) / 2;
    double lo = sorted[m], hi = sorted[N - 1 - m];
    for (int64_t i = 0; i < N; ++i) {
        double v = 0.0;
        if (hi > lo) {
            v = (s[i] - lo) / (hi - lo);
            if (v < 0.0)
                v = 0.0;
            if (v > 1.0)
                v = 1.0;
        }
        out[i] = v;
    }
    if (smoothed)
        memcpy(smoothed, s, sizeof(double) * (size_t)N);
    lo_hi[0] = lo;
    lo_hi[1] = hi;
    free(in);
    free(s);
    free(tmp);
    free(sorted);
    return 0;
}

/* Radius histogram (Sec. 4.1: blobs are histogrammed with bin centres at
 * the detectable radii sqrt(2)*sigma_i, i = 0..k-1; reading R12): each blob's
 * radius sqrt(2)*s goes to the nearest centre, the lower one on a tie.  The
 * common factor sqrt(2) is left out: the nearest radius is the nearest
 * sigma.  counts[k] receives the bin counts. */
void orc_radius_histogram(int k, const double *ladder, int64_t n, const double *blob_sigma,
                          int64_t *counts)
{
    for (int i = 0; i < k; ++i)
        counts[i] = 0;
    for (int64_t b = 0; b < n; ++b) {
        double s = blob_sigma[b];
        int best = 0;
        double bd = fabs(s - ladder[0]);
        for (int i = 1; i < k; ++i) {
            double d = fabs(s - ladder[i]);
            if (d < bd) {
                bd = d;
                best = i;
            }
        }
        counts[best] += 1;
    }
}

/* Whole detector on one fp32 image: ladder, planes, DoG, local maxima,
 * threshold, then pruning.  Writes up to cap blobs (y, x, i) with sigma and
 * response, sorted by (y, x, i).  *n_raw receives the count before pruning.
 * Returns the count after pruning, or -1 on bad input or when memory for the
 * DoG cube or the candidate lists cannot be allocated. */
int64_t orc_detect(const float *image, int64_t H, int64_t W, int64_t stride,
                   double smin, double smax, double ratio, double threshold,
                   double overlap, double truncate, int32_t *yxi,
                   double *sig, double *resp, int64_t cap, int64_t *n_raw)
{
    if (!(smin > 0.0) || !(smax >= smin) || !(ratio > 1.0) || !(truncate > 0.0))
        return -1;
    int k = orc_num_dog_planes(smin, smax, ratio);
    if (k < 1 || k > ORC_MAX_PLANES)
        return -1;
    double s[ORC_MAX_PLANES + 1];
    orc_sigmas_geometric(smin, ratio, k, s);
    size_t px = (size_t)H * (size_t)W;
    double *D = (double *)malloc(sizeof(double) * px * (size_t)k);
    if (!D)
        return -1;
    if (orc_planes_sigmas(image, H, W, stride, k + 1, s, truncate, NULL, D) != 0) {
        free(D);
        return -1;
    }
    int64_t n = orc_nms(D, k, H, W, threshold, NULL, NULL, 0);
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *c = (int32_t *)malloc(sizeof(int32_t) * 3 * nn);
    double *v = (double *)malloc(sizeof(double) * nn);
    int32_t *ys = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *xs = (int32_t *)malloc(sizeof(int32_t) * nn);
    double *ss = (double *)malloc(sizeof(double) * nn);
    uint8_t *keep = (uint8_t *)malloc(nn);
    if (!c || !v || !ys || !xs || !ss || !keep) {
        free(D);
        free(c);
        free(v);
        free(ys);
        free(xs);
        free(ss);
        free(keep);
        return -1;
    }
    orc_nms(D, k, H, W, threshold, c, v, n);
    free(D);

    for (int64_t a = 0; a < n; ++a) {
        ys[a] = c[3 * a];
        xs[a] = c[3 * a + 1];
        ss[a] = s[c[3 * a + 2]];
    }
    int64_t m = orc_prune(n, ys, xs, ss, overlap, keep);
    int64_t o = 0;
    for (int64_t a = 0; a < n; ++a) {
        if (!keep[a])
            continue;
        if (o < cap) {
            yxi[3 * o + 0] = c[3 * a + 0];
            yxi[3 * o + 1] = c[3 * a + 1];
            yxi[3 * o + 2] = c[3 * a + 2];
            if (sig)
                sig[o] = ss[a];
            if (resp)
                resp[o] = v[a];
        }
        ++o;
    }
    if (n_raw)
        *n_raw = n;
    free(keep);
    free(ss);
    free(xs);
    free(ys);
    free(v);
    free(c);
    return m;
}
