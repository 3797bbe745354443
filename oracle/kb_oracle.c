/*
 * kb_oracle.c - plain FP64 C oracle of the maximum-likelihood shift-and-stack
 * search (Whidden et al. 2019, "Fast algorithms for slow moving asteroids").
 *
 * TEST INFRASTRUCTURE ONLY.  The tests and the benchmark's CPU-baseline leg
 * call it (through oracle/cref.py); the HIP library never includes, links or
 * calls it, and it shares no code with that library.
 *
 * It computes, with plain loops in IEEE double and no contraction of a
 * multiply and an add (built with -ffp-contract=off), exactly what the numpy
 * oracle in oracle/core.py computes, in the same order of operations, so the
 * two agree bit for bit:
 *   validity and weights      Sec. 2.1.5, the masking paragraph
 *   psi, phi                  Sec. 2.1.5, the Psi and Phi equations (a
 *                             cross-correlation with zero outside the frame)
 *   displacements             Sec. 2.2, linear trajectories from the earliest
 *                             image: floor(v * tau + 0.5)
 *   Psi, Phi, n_obs           Sec. 2.1.5, the coadd equations, summed in
 *                             increasing image order over in-frame pixels
 *   nu, alpha                 Sec. 2.1.5, alpha = Psi / Phi, nu = Psi / sqrt(Phi)
 *   best k per start pixel    Sec. 2.2 (every start pixel and velocity is
 *                             evaluated), ranked by nu descending, ties by
 *                             ascending velocity index
 * It is a reference, not a fast program: one start row, one trajectory and
 * one image at a time.  The ORC_MUTATION_* switches plant known mistakes for
 * the tests that show the pins catch them; the oracle is built without them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* A pixel carries information when it is not masked and its image value and
 * variance are finite with a positive variance (Sec. 2.1.5, masking). */
static int pixel_valid(float img, float var, const uint8_t *mask, int64_t at) {
    if (mask && mask[at] != 0) return 0;
    return isfinite(img) && isfinite(var) && var > 0.0f;
}

/*
 * Likelihood planes of images [i0, i1) for output rows [r0, r1):
 *   psi[y][x] = sum_{u,v} a(y + u - cy, x + v - cx) * T[u][v]
 *   phi[y][x] = sum_{u,v} w(y + u - cy, x + v - cx) * T[u][v]^2
 * with a = img / var and w = 1 / var at valid pixels and 0 elsewhere,
 * out-of-frame taps skipped, taps summed in row-major (u, v) order, and
 * psi = phi = 0 at invalid pixels.  Outputs are [i1 - i0][r1 - r0][w];
 * ok (nullable) receives the validity of the output pixels.
 */
void orc_planes(const float *img, const float *var, const uint8_t *mask, int64_t n, int64_t h,
                int64_t w, const float *psf, int64_t ph, int64_t pw, int64_t i0, int64_t i1,
                int64_t r0, int64_t r1, double *psi, double *phi, uint8_t *ok) {
    const int64_t cy = ph / 2, cx = pw / 2;
    (void)n;
    for (int64_t i = i0; i < i1; ++i) {
        const int64_t img_off = i * h * w;
        for (int64_t y = r0; y < r1; ++y) {
            for (int64_t x = 0; x < w; ++x) {
                const int64_t out = ((i - i0) * (r1 - r0) + (y - r0)) * w + x;
                const int64_t here = img_off + y * w + x;
                const int ok_here = pixel_valid(img[here], var[here], mask, here);
                double s_psi = 0.0, s_phi = 0.0;
                for (int64_t u = 0; u < ph; ++u) {
                    const int64_t yy = y + u - cy;
                    if (yy < 0 || yy >= h) continue;
                    for (int64_t v = 0; v < pw; ++v) {
#ifdef ORC_MUTATION_CONVOLVE   /* planted mistake: convolution, not correlation */
                        const int64_t xx = x - v + cx;
#else
                        const int64_t xx = x + v - cx;
#endif
                        if (xx < 0 || xx >= w) continue;
                        const int64_t at = img_off + yy * w + xx;
                        const double tv = (double)psf[u * pw + v];
                        double a = 0.0, wt = 0.0;
                        if (pixel_valid(img[at], var[at], mask, at)) {
                            wt = 1.0 / (double)var[at];
                            a = (double)img[at] / (double)var[at];
                        }
                        const double t_psi = tv * a;
                        const double t_phi = (tv * tv) * wt;
                        s_psi += t_psi;
                        s_phi += t_phi;
                    }
                }
                psi[out] = ok_here ? s_psi : 0.0;
                phi[out] = ok_here ? s_phi : 0.0;
                if (ok) ok[out] = (uint8_t)ok_here;
            }
        }
    }
}

/* floor(v * tau + 0.5): the product, the sum and the floor as separate IEEE
 * double operations (halves round toward +infinity). */
static int64_t offset_of(double v, double tau) {
    const double prod = v * tau;
#ifdef ORC_MUTATION_RINT   /* planted mistake: halves to even */
    return (int64_t)nearbyint(prod);
#else
    const double shifted = prod + 0.5;
    return (int64_t)floor(shifted);
#endif
}

/* Is candidate (nu_a, j_a) ranked before (nu_b, j_b)? */
static int ranks_before(double nu_a, int64_t j_a, double nu_b, int64_t j_b) {
    return nu_a > nu_b || (nu_a == nu_b && j_a < j_b);
}

/* Visiting order of the velocities: by vy, then vx, then index.  Every
 * trajectory is evaluated independently and the ranking is a total order, so
 * the order of evaluation does not change the result; visiting velocities of
 * equal or close vy one after another reads the same plane rows again while
 * they are still in the CPU's caches. */
static const double *g_sort_vel;
static int by_vy_vx(const void *a, const void *b) {
    const int64_t ja = *(const int64_t *)a, jb = *(const int64_t *)b;
    const double ya = g_sort_vel[2 * ja + 1], yb = g_sort_vel[2 * jb + 1];
    if (ya != yb) return ya < yb ? -1 : 1;
    const double xa = g_sort_vel[2 * ja], xb = g_sort_vel[2 * jb];
    if (xa != xb) return xa < xb ? -1 : 1;
    return ja < jb ? -1 : (ja > jb ? 1 : 0);
}

/*
 * The best k_out trajectories of every start pixel of rows [row_lo, row_hi):
 *   planes    psi, phi (double) and ok (uint8) [n][plane_rows][w], holding
 *             frame rows [plane_row0, plane_row0 + plane_rows); every in-frame
 *             row a trajectory of these start rows visits must be inside.
 *   t, vel    times [n] and velocities [n_vel][2] (vx, vy).
 *   outputs   [row_hi - row_lo][w][k_out], ranked: nu, alpha, Phi, n_obs, j.
 * For each start row and each velocity j (in the visiting order above), the
 * sums of every start pixel of the row are formed image by image, then each
 * pixel's trajectory is scored and offered to that pixel's ranked list.
 * Not thread-safe (the visiting order's comparator reads a static).
 * Returns 0, -1 when a trajectory visits a row outside the planes, -2 when
 * out of memory.
 */
int orc_search_rows(const double *psi, const double *phi, const uint8_t *ok, int64_t n,
                    int64_t h, int64_t w, int64_t plane_row0, int64_t plane_rows,
                    const double *t, const double *vel, int64_t n_vel, int64_t k_out,
                    int64_t row_lo, int64_t row_hi, double *out_nu, double *out_alpha,
                    double *out_phi, int32_t *out_nobs, int32_t *out_vel) {
    int64_t *disp = malloc(sizeof(int64_t) * 2 * (size_t)(n_vel * n));
    double *Psi = malloc(sizeof(double) * (size_t)w);
    double *Phi = malloc(sizeof(double) * (size_t)w);
    double *Fsave = malloc(sizeof(double) * (size_t)w);
    int64_t *cnt = malloc(sizeof(int64_t) * (size_t)w);
    int64_t *len = malloc(sizeof(int64_t) * (size_t)w);
    int64_t *visit = malloc(sizeof(int64_t) * (size_t)n_vel);
    int rc = 0;
    if (!disp || !Psi || !Phi || !Fsave || !cnt || !len || !visit) {
        rc = -2;
        goto done;
    }
    for (int64_t j = 0; j < n_vel; ++j)
        for (int64_t i = 0; i < n; ++i) {
            const double tau = t[i] - t[0];
            disp[(j * n + i) * 2] = offset_of(vel[2 * j], tau);
            disp[(j * n + i) * 2 + 1] = offset_of(vel[2 * j + 1], tau);
        }
    for (int64_t j = 0; j < n_vel; ++j) visit[j] = j;
    g_sort_vel = vel;
    qsort(visit, (size_t)n_vel, sizeof(int64_t), by_vy_vx);
    for (int64_t y0 = row_lo; y0 < row_hi && rc == 0; ++y0) {
        for (int64_t x0 = 0; x0 < w; ++x0) len[x0] = 0;
        for (int64_t jj = 0; jj < n_vel; ++jj) {
            const int64_t j = visit[jj];
            for (int64_t x0 = 0; x0 < w; ++x0) {
                Psi[x0] = 0.0;
                Phi[x0] = 0.0;
                cnt[x0] = 0;
            }
            /* Psi, Phi, n_obs of trajectory j from every start pixel of row y0:
             * image by image in increasing order, in-frame pixels only. */
            for (int64_t i = 0; i < n; ++i) {
                const int64_t dx = disp[(j * n + i) * 2], dy = disp[(j * n + i) * 2 + 1];
                const int64_t y = y0 + dy;
                if (y < 0 || y >= h) continue;
                const int64_t r = y - plane_row0;
                if (r < 0 || r >= plane_rows) {
                    rc = -1;
                    goto done;
                }
                const int64_t row = (i * plane_rows + r) * w + dx;
                /* start columns whose column x0 + dx is inside the frame */
                const int64_t lo = dx < 0 ? -dx : 0, hi = dx > 0 ? w - dx : w;
                for (int64_t x0 = lo; x0 < hi; ++x0) {
                    Psi[x0] += psi[row + x0];
                    Phi[x0] += phi[row + x0];
                    cnt[x0] += ok[row + x0];
                }
            }
            /* scores (Psi, Phi are overwritten by nu, alpha), then the ranked
             * list of each start pixel */
            for (int64_t x0 = 0; x0 < w; ++x0) {
                const double P = Psi[x0], F = Phi[x0];
#ifdef ORC_MUTATION_NO_SQRT   /* planted mistake: nu = Psi / Phi */
                Psi[x0] = F > 0.0 ? P / F : -INFINITY;
#else
                Psi[x0] = F > 0.0 ? P / sqrt(F) : -INFINITY;
#endif
                Phi[x0] = F > 0.0 ? P / F : 0.0;
                Fsave[x0] = F;
            }
            for (int64_t x0 = 0; x0 < w; ++x0) {
                const double nu = Psi[x0], alpha = Phi[x0];
                const int64_t px = ((y0 - row_lo) * w + x0) * k_out;
                double *nu_l = out_nu + px, *al_l = out_alpha + px, *ph_l = out_phi + px;
                int32_t *no_l = out_nobs + px, *j_l = out_vel + px;
                const int64_t m = len[x0];
                if (m == k_out && !ranks_before(nu, j, nu_l[m - 1], j_l[m - 1])) continue;
                int64_t p = m < k_out ? m : k_out - 1;
                while (p > 0 && ranks_before(nu, j, nu_l[p - 1], j_l[p - 1])) {
                    nu_l[p] = nu_l[p - 1];
                    al_l[p] = al_l[p - 1];
                    ph_l[p] = ph_l[p - 1];
                    no_l[p] = no_l[p - 1];
                    j_l[p] = j_l[p - 1];
                    --p;
                }
                nu_l[p] = nu;
                al_l[p] = alpha;
                ph_l[p] = Fsave[x0];
                no_l[p] = (int32_t)cnt[x0];
                j_l[p] = (int32_t)j;
                if (m < k_out) len[x0] = m + 1;
            }
        }
    }
done:
    free(disp);
    free(Psi);
    free(Phi);
    free(Fsave);
    free(cnt);
    free(len);
    free(visit);
    return rc;
}
