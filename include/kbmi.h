/*
 * kbmi.h - C ABI of the maximum-likelihood shift-and-stack trajectory search
 * (Whidden et al. 2019, "Fast algorithms for slow moving asteroids") on
 * AMD Instinct MI355X (gfx950).
 *
 * The search has three device stages and one host helper:
 *   kb_make_psi_phi   likelihood images psi, phi of every image    (Sec. 2.1.5)
 *   kb_search         coadd psi, phi along every linear trajectory  (Sec. 2.1.5
 *                     coadd, Sec. 2.2) and keep the k_cand best per start pixel
 *   kb_topk           order each start pixel's candidates and keep k
 *   kb_displacements  the integer pixel offsets every kernel uses   (Sec. 2.2)
 * one optional stage before it:
 *   kb_mask_bright    mask pixels above a count level           (Sec. 5.2)
 * a threshold mode of the search and its duplicate clustering:
 *   kb_search_threshold   every trajectory with nu >= nu_min     (Sec. 2.2)
 *   kb_cluster_hits   group near-identical hits, keep the best  (Sec. 3.3)
 * and two stages after the search:
 *   kb_lightcurve_filter  drop outlying observations from each candidate's
 *                     light curve and refit nu, alpha           (Sec. 3.3)
 *   kb_stamps         coadded postage stamps and moment filter  (Sec. 3.3)
 *
 * Conventions shared by every call
 *   - Pixel (x, y) is column x, row y of a row-major [h][w] frame; integer
 *     coordinates are pixel centres.  Image stacks are [n_img][h][w].
 *   - Times t[n_img] are in days and must be non-decreasing; trajectories
 *     start at every pixel of image 0 (the earliest observation, Sec. 3.2).
 *   - vel[n_vel][2] holds (vx, vy) in pixels per day.  The trajectory of start
 *     pixel (x0, y0) and velocity j visits, in image i,
 *         x0 + floor(vx_j * (t_i - t_0) + 0.5),  y0 + floor(vy_j * (t_i - t_0) + 0.5)
 *     with the product, the sum and the floor evaluated in IEEE double as
 *     separate operations (halves round toward +infinity).
 *   - Device pointers are HIP device memory owned by the caller.  Host
 *     pointers (marked "host") are read before the call returns.  The library
 *     allocates no device memory and keeps no pointer after a call returns.
 *     Tables that a call sends to its workspace go through pinned host
 *     buffers the library keeps per device (at most 32, reused once the copy
 *     out of them has completed), so calls do not wait for their stream.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     enqueued asynchronously on it; the caller keeps every device buffer
 *     alive until the stream has passed the work.  Calls on different streams
 *     may run concurrently.
 *   - Every argument is checked before anything is enqueued; a failed check
 *     returns KB_EINVAL or KB_EUNSUPPORTED, writes nothing, and leaves a
 *     message for kb_last_error().  A failed launch returns KB_EDEVICE.
 *     Faults inside kernels surface at the caller's next synchronisation.
 *     No C++ exception crosses this interface.
 */
#ifndef KBMI_H
#define KBMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KB_ABI_VERSION 1

/* Largest per-pixel candidate count kb_search keeps (k_cand). */
#define KB_MAX_KCAND 64
/* Largest PSF side length kb_make_psi_phi accepts (odd sizes only). */
#define KB_MAX_PSF 25
/* Largest image count kb_lightcurve_filter accepts (one bit per image in its
 * rejection mask). */
#define KB_MAX_LC_IMAGES 64
/* Largest stamp radius kb_stamps accepts (stamps of (2R+1)^2 pixels). */
#define KB_MAX_STAMP_RADIUS 15

typedef enum kb_status {
    KB_OK = 0,
    KB_EINVAL = -1,        /* invalid argument; nothing was enqueued */
    KB_ENOMEM = -2,        /* caller-provided workspace too small */
    KB_EDEVICE = -3,       /* HIP runtime error while enqueueing */
    KB_EUNSUPPORTED = -4   /* valid request outside what this build implements */
} kb_status;

/* Storage type of the likelihood planes read by kb_search. */
typedef enum kb_dtype {
    KB_F32 = 0,            /* float32 (psi, phi) pairs */
    KB_F16 = 1,            /* scaled IEEE half (psi, phi) pairs */
    KB_BF16 = 2            /* scaled bfloat16 (psi, phi) pairs */
} kb_dtype;

/* KB_ABI_VERSION of the loaded library. */
int kb_abi_version(void);

/* Message describing the last non-OK status returned on this thread
 * ("" if none).  The pointer stays valid until the next call on this thread. */
const char *kb_last_error(void);

/*
 * kb_displacements - integer pixel offsets of every trajectory (Sec. 2.2:
 * linear trajectories y_i = y_0 + v t_i from the earliest image).
 *   t     host, float64 [n_img], non-decreasing, finite.
 *   vel   host, float64 [n_vel][2] (vx, vy) px/day, finite.
 *   disp  host, int32 [n_vel][n_img][2] out: (dx, dy) per velocity and image,
 *         exactly as defined in the header comment.
 * Errors: KB_EINVAL for null pointers, n_img < 1, n_vel < 1, non-finite or
 * decreasing times, non-finite velocities, or |v * (t_i - t_0)| >= 2^30.
 * Pure host code; usable without a GPU.
 */
kb_status kb_displacements(const double *t, int64_t n_img, const double *vel,
                           int64_t n_vel, int32_t *disp);

/*
 * kb_make_psi_phi - per-image likelihood images for a diagonal pixel
 * covariance (Sec. 2.1.5, the Psi and Phi equations and the masking rule;
 * Sec. 2.3 computes them on the GPU with one single-pass 2-D kernel):
 *     valid(p) = mask(p) == 0 and img(p), var(p) finite and var(p) > 0
 *     psi(y) = sum_u,v valid * img/var (y + (u - cy, v - cx)) * T[u][v]
 *     phi(y) = sum_u,v valid / var     (y + (u - cy, v - cx)) * T[u][v]^2
 * a cross-correlation with zero outside the frame, centre (cy, cx) =
 * (psf_h / 2, psf_w / 2); psi = phi = 0 where valid(y) is false.
 *   img, var  device, float32 [n_img][h][w].
 *   mask      device, uint8 [n_img][h][w], nonzero = bad pixel; may be NULL.
 *   psf       host, float32 [psf_h][psf_w], odd sizes <= KB_MAX_PSF, used as
 *             given (the caller normalises it).
 *   psi_phi   device out, float32 [n_img][h][w][2]: (psi, phi) interleaved.
 *             A valid pixel whose phi is +0 is stored with phi = -0.0 so that
 *             the stored bit pattern of phi is nonzero exactly at valid pixels.
 *   lp_dtype  KB_F32 = no 16-bit copy.  KB_F16 / KB_BF16 also write
 *             psi_phi_lp (device, 16-bit [n_img][h][w][2] pairs) holding
 *             round-to-nearest-even(value * s) with one power-of-two scale s
 *             per image and plane, chosen so that max|value| * s lies in
 *             [2^13, 2^14), written to lp_scale (device, float32 [n_img][2]:
 *             s_psi, s_phi).  A valid pixel whose scaled phi rounds to +0
 *             stores -0, so the phi half is nonzero exactly at valid pixels.
 *             The 16-bit copy only ranks; kb_topk re-scores from float32.
 * Errors: KB_EINVAL for null required pointers (psi_phi_lp and lp_scale with
 * a 16-bit lp_dtype), n_img < 1, h < 1, w < 1, even PSF sizes or an unknown
 * lp_dtype; KB_EUNSUPPORTED for a PSF side > KB_MAX_PSF.
 */
kb_status kb_make_psi_phi(const float *img, const float *var, const uint8_t *mask,
                          int64_t n_img, int64_t h, int64_t w,
                          const float *psf, int64_t psf_h, int64_t psf_w,
                          float *psi_phi, int32_t lp_dtype, void *psi_phi_lp,
                          float *lp_scale, void *stream);

/*
 * kb_mask_bright - the bright-pixel mask applied before the planes are built
 * (Sec. 5.2, the additional mask of pixels above a fixed count level): every
 * pixel of every image whose value exceeds `threshold` is masked in that
 * image, mask[i][y][x] |= (img[i][y][x] > threshold).  A pixel equal to the
 * threshold, or NaN, is left as it was.  Masked pixels then carry no weight
 * in kb_make_psi_phi.
 *   img   device, float32 [n_img][h][w].
 *   mask  device, uint8 [n_img][h][w], updated in place (bit 0 is set).
 * Errors: KB_EINVAL for null pointers, bad sizes or a NaN threshold.
 */
kb_status kb_mask_bright(const float *img, uint8_t *mask, int64_t n_img, int64_t h, int64_t w,
                         float threshold, void *stream);

/* Bytes of device workspace kb_search and kb_topk need for a stack of n_img
 * frames of h x w and n_vel velocities (displacement table, visiting order,
 * 16-bit scales); 0 for invalid sizes. */
size_t kb_search_workspace_bytes(int64_t n_img, int64_t h, int64_t w, int64_t n_vel);

/*
 * kb_search - exhaustive evaluation of every (start pixel, velocity) pair
 * (Sec. 2.2) by coadding the likelihood images along the trajectory
 * (Sec. 2.1.5 coadd equations) and scoring it (Sec. 2.1.5: alpha_ML = Psi/Phi,
 * nu = Psi/sqrt(Phi)):
 *     Psi = sum_i psi_i(p_i), Phi = sum_i phi_i(p_i), n_obs = #terms
 * over the images i in increasing order whose trajectory pixel p_i is inside
 * the frame and valid; float32 arithmetic.  If Phi > 0: nu = Psi/sqrt(Phi),
 * alpha = Psi/Phi; otherwise nu = -inf, alpha = 0.  For every start pixel the
 * k_cand best trajectories in the order (nu descending, velocity index
 * ascending) are kept.
 *   planes     device, [n_img][h][w][2] pairs as written by kb_make_psi_phi:
 *              float32 (dtype KB_F32) or its scaled 16-bit copy (KB_F16,
 *              KB_BF16; each value is decoded and multiplied by 1/s, exactly,
 *              before it is summed in float32).
 *   lp_scale   device float32 [n_img][2] for 16-bit planes; NULL for KB_F32.
 *   t, vel     host, as for kb_displacements.
 *   k_cand     1 <= k_cand <= min(n_vel, KB_MAX_KCAND).
 *   cand_nu, cand_alpha  device out, float32 [h][w][k_cand].
 *   cand_vel   device out, int32 [h][w][k_cand]: velocity index j.
 *   cand_nobs  device out, int16 [h][w][k_cand]: n_obs.
 *              Each pixel's k_cand entries are the best set, written in rank
 *              order (kb_topk accepts them in any order).
 *   workspace  device, >= kb_search_workspace_bytes(n_img, h, w, n_vel)
 *              bytes, 256-byte aligned; overwritten.
 * Limits: n_img <= 32767, n_vel <= 65535, w <= 2^27, h <= 2^30.
 * The displacement table is copied host-to-device on `stream`
 * (asynchronously, through the library's pinned staging buffers).
 * Errors: KB_EINVAL for bad sizes, pointers or times; KB_ENOMEM for a short
 * workspace; KB_EUNSUPPORTED for k_cand > KB_MAX_KCAND.
 */
kb_status kb_search(const void *planes, int32_t dtype, const float *lp_scale,
                    int64_t n_img, int64_t h, int64_t w,
                    const double *t, const double *vel, int64_t n_vel, int64_t k_cand,
                    float *cand_nu, float *cand_alpha, int32_t *cand_vel,
                    int16_t *cand_nobs, void *workspace, size_t workspace_bytes,
                    void *stream);

/*
 * kb_topk - final per-pixel selection: order each start pixel's k_cand
 * candidates by (nu descending, velocity index ascending; entries equal in
 * both keep their list order) and keep the first k (Sec. 2.2 asks for the
 * trajectories maximising nu).
 *   psi_phi_f32  device float32 planes [n_img][h][w][2] to re-score every
 *                candidate from before ordering (used after a 16-bit search),
 *                or NULL to keep the candidates' scores.  A re-scored entry
 *                is computed with exactly the float32 search's arithmetic
 *                (image order, same score expressions), so it equals the
 *                plain path's value for that trajectory bit for bit.
 *   t, vel, n_vel, workspace  as for kb_search (used only when re-scoring).
 *   cand_*       device, as written by kb_search (any order within a pixel;
 *                with re-scoring only cand_vel is read).
 *   nu, alpha, vel_idx, nobs  device out, [h][w][k] in rank order.  Either
 *                separate from the candidate arrays, or (k == k_cand, no
 *                re-scoring) the four candidate arrays themselves: each
 *                pixel's list is then put in rank order in place, and a block
 *                of lists already in rank order (as kb_search writes them) is
 *                checked and not rewritten.
 * Errors: KB_EINVAL for bad sizes or pointers, k > k_cand, outputs that are
 * some but not all of the candidate arrays, ordering in place with k < k_cand
 * or with re-scoring, or (re-scoring) bad times/velocities or workspace;
 * KB_ENOMEM for a short workspace; KB_EUNSUPPORTED for k_cand > KB_MAX_KCAND.
 */
kb_status kb_topk(const float *psi_phi_f32, int64_t n_img, int64_t h, int64_t w,
                  const double *t, const double *vel, int64_t n_vel,
                  const float *cand_nu, const float *cand_alpha,
                  const int32_t *cand_vel, const int16_t *cand_nobs,
                  int64_t k_cand, int64_t k,
                  float *nu, float *alpha, int32_t *vel_idx, int16_t *nobs,
                  void *workspace, size_t workspace_bytes, void *stream);

/*
 * kb_lightcurve_filter - outlier filter on each candidate's light curve and
 * refit of its likelihood (Sec. 3.3, filtering of candidate trajectories; the
 * paper names the filter only as a Kalman-filter variant, this is the variant
 * implemented).
 * Candidate (x0, y0, j) observes image i when its trajectory pixel (the
 * displacements of kb_displacements) is inside the frame and valid; the
 * observation's flux estimate is psi_i/phi_i with variance 1/phi_i.  The flux
 * is modelled as a random walk with variance q per day (q = 0: constant).  An
 * information-form Kalman filter runs forward and backward over the
 * observations; the estimate at observation k from all the others has
 * information J_k = Jf_k + Jb_k and H_k = Hf_k + Hb_k (estimate H_k/J_k), and
 *     r_k = (psi_k J_k - phi_k H_k)^2 / ((phi_k J_k)(J_k + phi_k))
 * is its squared standardised residual (0 if the divisor is not positive).
 * While the largest r_k (lowest image index among equal values) exceeds
 * sigma_cut^2, that observation is dropped and the filter is rerun on the
 * rest.  Then Psi', Phi' are summed over the kept observations in image order,
 * nu' = Psi'/sqrt(Phi'), alpha' = Psi'/Phi' (nu' = -inf, alpha' = 0 if
 * Phi' <= 0), n_obs' = number kept.  All filter arithmetic is IEEE double with
 * every operation separately rounded (prediction: d = 1 + (q dtau) J,
 * J <- J/d, H <- H/d, dtau from tau_i = t_i - t_0; update: J += phi_i,
 * H += psi_i), so each decision is reproducible from the float32 planes.
 *   psi_phi    device, float32 [n_img][h][w][2] planes from kb_make_psi_phi
 *              (invalid pixels hold (+0, +0)).
 *   t, vel     host, as for kb_displacements; n_img <= KB_MAX_LC_IMAGES.
 *   cand_vel   device, int32 [h][w][k] velocity indices, e.g. kb_topk's output;
 *              an index outside [0, n_vel) yields nu' = -inf, alpha' = 0,
 *              n_obs' = 0.
 *   sigma_cut  the cut in standard deviations (5 in the paper), > 0.
 *   q          process-noise variance of the flux per day, >= 0.
 *   nu, alpha  device out, float32 [h][w][k], same order as cand_vel (not
 *              re-ranked); they may alias kb_topk's nu and alpha outputs.
 *   nobs       device out, int16 [h][w][k].
 *   rejected   device out or NULL, uint64 [h][w][k]: bit i set when image i
 *              was an observation and was dropped.
 *   workspace  device, 256-byte aligned, >= kb_search_workspace_bytes(n_img,
 *              h, w, n_vel) bytes; tau and the velocities are copied into it
 *              asynchronously on `stream`.
 * Errors: KB_EINVAL for null pointers, bad sizes, times or velocities,
 * sigma_cut not finite and positive, q not finite and >= 0; KB_ENOMEM for a
 * short workspace; KB_EUNSUPPORTED for n_img > KB_MAX_LC_IMAGES.
 */
kb_status kb_lightcurve_filter(const float *psi_phi, int64_t n_img, int64_t h, int64_t w,
                               const double *t, const double *vel, int64_t n_vel,
                               const int32_t *cand_vel, int64_t k, double sigma_cut, double q,
                               float *nu, float *alpha, int16_t *nobs, uint64_t *rejected,
                               void *workspace, size_t workspace_bytes, void *stream);

/* One trajectory kept by kb_search_threshold (24 bytes). */
typedef struct kb_hit {
    int32_t x, y;       /* start pixel in image 0 */
    int32_t vel;        /* velocity index */
    float nu, alpha;    /* scores, bitwise the values kb_search gives it */
    int16_t nobs;       /* n_obs */
    int16_t reserved;   /* 0 */
} kb_hit;

/*
 * kb_search_threshold - threshold mode of the search (Sec. 2.2; Sec. 3.2
 * keeps every trajectory with nu >= 10): every (start pixel, velocity) whose
 * nu >= nu_min is appended to `hits`, with the coadd and scores of kb_search
 * (same sums in image order, same float32 score arithmetic).
 *   psi_phi    device, float32 [n_img][h][w][2] planes; h, w < 2^24.
 *   t, vel     host, as for kb_displacements.
 *   nu_min     finite threshold.
 *   hits       device out, kb_hit [max_hits]; the order of the hits is
 *              unspecified (slots are reserved by atomics).
 *   n_hits     device out, uint64: the number of trajectories with
 *              nu >= nu_min, also when it exceeds max_hits; then only
 *              max_hits of them, an unspecified subset, are stored, and the
 *              call can be repeated with a larger list.
 *   workspace  device, 256-byte aligned, >= kb_search_workspace_bytes(...).
 * Errors: KB_EINVAL for null pointers, bad sizes, times or velocities, a
 * non-finite threshold or a negative max_hits; KB_ENOMEM for a short
 * workspace; KB_EUNSUPPORTED for frames of 2^24 or more on a side.
 */
kb_status kb_search_threshold(const float *psi_phi, int64_t n_img, int64_t h, int64_t w,
                              const double *t, const double *vel, int64_t n_vel, float nu_min,
                              kb_hit *hits, int64_t max_hits, uint64_t *n_hits, void *workspace,
                              size_t workspace_bytes, void *stream);

/* Device workspace bytes kb_cluster_hits needs (0 for invalid sizes). */
size_t kb_cluster_workspace_bytes(int64_t n_hits, int64_t n_vel);

/*
 * kb_cluster_hits - duplicate clustering of kept trajectories (Sec. 3.3, last
 * paragraph: similar (x, y, vx, vy) are grouped with DBSCAN and the most
 * likely of each group is kept).  Reading: DBSCAN with min_samples = 1, so
 * the groups are the connected components of the graph joining hits a, b with
 *     ((dx*dx + dy*dy) + du*du) + dv*dv <= eps*eps     (IEEE double, in order)
 *     dx = x_a - x_b, dy = y_a - y_b, du = s*vx_a - s*vx_b, dv = s*vy_a - s*vy_b,
 * i.e. Euclidean distance over (x, y, s*vx, s*vy) with the velocity scaled by
 * a time s (days).  Each group's representative is its hit with the largest
 * nu, ties to the smallest (y, x, vel); the result does not depend on the
 * order of `hits`.
 *   hits    device, kb_hit [n_hits] (e.g. kb_search_threshold's list), at
 *           most 2^30 hits, distinct trajectories; a hit whose vel is
 *           outside [0, n_vel) forms a group of its own.
 *   vel     host, float64 [n_vel][2], the grid the hits index.
 *   rep     device out, int32 [n_hits]: index in `hits` of each hit's group
 *           representative (rep[i] == i for representatives).
 *   workspace  device, 256-byte aligned, >= kb_cluster_workspace_bytes.
 * Pairs are found through a grid of cells slightly wider than eps over
 * (x, y, s*vx, s*vy), kept in a hash table in the workspace: each hit is
 * tested against the hits of its own and its 80 neighbouring cells, so the
 * work grows with the hits and their neighbours within eps, not with n^2.
 * Errors: KB_EINVAL for null pointers, bad sizes or velocities, s or eps not
 * finite and >= 0; KB_ENOMEM for a short workspace; KB_EUNSUPPORTED for more
 * hits than one launch covers.
 */
kb_status kb_cluster_hits(const kb_hit *hits, int64_t n_hits, const double *vel, int64_t n_vel,
                          double s, double eps, int32_t *rep, void *workspace,
                          size_t workspace_bytes, void *stream);

/*
 * kb_stamps - coadded postage stamps of candidate trajectories and the
 * central-moment filter (Sec. 3.3, second paragraph; the paper names neither
 * the coadd nor the comparison, this is the variant implemented).
 * For candidate (x, y, vel) and offsets u, v in [-R, R]:
 *     S(u, v) = (sum over kept images i of img_i(x_i + u, y_i + v)) / n(u, v)
 * over the pixels inside the frame and valid (mask 0, finite image, finite
 * positive variance), summed in image order in double; S = 0 where n = 0.
 * (x_i, y_i) is the trajectory pixel floor(v * tau_i + 0.5) from (x, y), as
 * in kb_displacements.  Moments in one row-major pass (v outer, u inner):
 *     M00 = sum S, M10 = sum u S, M01 = sum v S, M20 = sum (u u) S,
 *     M02 = sum (v v) S, M11 = sum (u v) S;
 *     ub = M10/M00, vb = M01/M00, m20 = M20/M00 - ub ub,
 *     m02 = M02/M00 - vb vb, m11 = M11/M00 - ub vb
 * (separately rounded double operations).  pass = M00 > 0 and |ub|, |vb| <=
 * max_offset and |m11| <= max_m11 and m2_min <= m20, m02 <= m2_max: the
 * stamp resembles a Gaussian centred on it, whose centroid is 0, m11 is 0 and
 * m20 = m02 its variance.
 *   img, var, mask  device, [n_img][h][w] float32, float32, uint8 (mask may
 *              be NULL: nothing masked); n_img <= KB_MAX_LC_IMAGES.
 *   t, vel     host, as for kb_displacements.
 *   cand       device, kb_hit [n_cand] (x, y, vel are used); a vel outside
 *              [0, n_vel) gives an all-zero stamp, NaN moments, pass 0.
 *   drop       device or NULL, uint64 [n_cand]: bit i set excludes image i
 *              (e.g. the light-curve filter's rejection mask).
 *   radius     R in [0, KB_MAX_STAMP_RADIUS].
 *   stamps     device out or NULL, float32 [n_cand][2R+1][2R+1].
 *   moments    device out or NULL, float64 [n_cand][6]: M00, ub, vb, m20,
 *              m02, m11 (NaN where M00 = 0).
 *   pass       device out, uint8 [n_cand].
 *   workspace  device, 256-byte aligned, >= kb_search_workspace_bytes(n_img,
 *              h, w, n_vel); tau and the velocities are copied into it.
 * Errors: KB_EINVAL for null pointers, bad sizes, times or velocities, a bad
 * radius or NaN bounds; KB_ENOMEM for a short workspace; KB_EUNSUPPORTED for
 * n_img > KB_MAX_LC_IMAGES.
 */
kb_status kb_stamps(const float *img, const float *var, const uint8_t *mask, int64_t n_img,
                    int64_t h, int64_t w, const double *t, const double *vel, int64_t n_vel,
                    const kb_hit *cand, const uint64_t *drop, int64_t n_cand, int32_t radius,
                    double max_offset, double max_m11, double m2_min, double m2_max,
                    float *stamps, double *moments, uint8_t *pass, void *workspace,
                    size_t workspace_bytes, void *stream);

/*
 * Batched search (serving).  One stack of a batch: the kb_search arguments of
 * that stack.  Every field has kb_search's meaning and rules.
 */
typedef struct kb_job {
    const void *planes;        /* device [n_img][h][w][2] pairs of the batch dtype */
    const float *lp_scale;     /* device float32 [n_img][2] for 16-bit planes, else NULL */
    int64_t n_img, h, w;
    const double *t;           /* host [n_img] */
    const double *vel;         /* host [n_vel][2] */
    int64_t n_vel;
    float *cand_nu;            /* device out [h][w][k_cand] ... */
    float *cand_alpha;
    int32_t *cand_vel;
    int16_t *cand_nobs;
} kb_job;

/* Device workspace bytes kb_search_batch needs for these jobs (0 if any job
 * has invalid sizes). */
size_t kb_search_batch_workspace_bytes(const kb_job *jobs, int64_t n_jobs);

/*
 * kb_search_batch - kb_search for several stacks in one persistent launch
 * per image-count class (at most three: n_img <= 8, <= 16, > 16; the serving
 * path: small stacks share the GPU instead of each under-filling it).  The
 * launch's grid is what the GPU holds at once; its work items are the jobs'
 * start-pixel tiles, packed tile after tile, except that a job of float32
 * planes large enough for kb_search's paced block order starts at a
 * generation boundary and keeps that order.  All jobs share `dtype` and
 * `k_cand`.  Each job's candidates are exactly what kb_search would write
 * for it alone (same arithmetic, same order), whatever else is in the batch.
 *   jobs       host array of n_jobs (1 <= n_jobs <= 4096) descriptors; read
 *              before return.
 *   workspace  device, >= kb_search_batch_workspace_bytes(jobs, n_jobs),
 *              256-byte aligned; overwritten.
 * The displacement tables and job descriptors are copied host-to-device on
 * `stream` (asynchronously, through the library's pinned staging buffers).
 * Errors: as kb_search for any job (the message names the job index), plus
 * KB_EINVAL for n_jobs out of range or more workgroups than one launch holds.
 */
kb_status kb_search_batch(const kb_job *jobs, int64_t n_jobs, int32_t dtype, int64_t k_cand,
                          void *workspace, size_t workspace_bytes, void *stream);

/* Size of the fixed device array behind kb_search_noalloc (per device). */
#define KB_NOALLOC_SCRATCH_BYTES (8u << 20)

/*
 * kb_search_noalloc - kb_search for callers that cannot allocate memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, rules and results as kb_search (bit for bit:
 * the same table, the same kernels), without the workspace: the gather
 * table, visiting order, 16-bit scales and pacing counters live in a fixed
 * device array of KB_NOALLOC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends.  The call allocates nothing
 * (no device, pinned or managed memory); times and velocities reach the
 * device through kernel arguments, and the table is built there.
 *   Limit: the stack must fit the array:
 *     kb_search_workspace_bytes(n_img, h, w, n_vel) + 8 n_img + 20 n_vel
 *     (+ up to 1 KB of alignment) <= KB_NOALLOC_SCRATCH_BYTES,
 *   e.g. n_img <= 16 with n_vel <= 29954, n_img <= 32 with n_vel <= 15648;
 *   beyond that it returns KB_EUNSUPPORTED and enqueues nothing.
 *   Sharing: every call on a device uses that device's one array and leaves
 *   its contents behind.  Calls on one stream are ordered by the stream;
 *   calls that overlap on one device (other streams, other host threads,
 *   kb_search_noalloc beside itself) race on the array and must not be made.
 *   The first call on a device looks up the array's address (not inside a
 *   graph capture); later calls only enqueue kernels.
 * Errors: as kb_search, plus KB_EUNSUPPORTED when the stack exceeds the array.
 */
kb_status kb_search_noalloc(const void *planes, int32_t dtype, const float *lp_scale,
                            int64_t n_img, int64_t h, int64_t w,
                            const double *t, const double *vel, int64_t n_vel, int64_t k_cand,
                            float *cand_nu, float *cand_alpha, int32_t *cand_vel,
                            int16_t *cand_nobs, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KBMI_H */
