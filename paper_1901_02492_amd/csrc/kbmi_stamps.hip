// Coadded postage stamps and the central-moment filter of libkbmi (Sec. 3.3,
// second paragraph: the remaining candidates' coadded stamps are kept when
// their central moments resemble those of a Gaussian centred on the stamp).
//
// One wave per candidate.  Its displacements are computed once
// (floor(v * tau + 0.5) in double, as everywhere else); each stamp pixel (one
// lane) averages the science-image pixels of the kept images in image order
// in double, and the raw moments about the stamp centre are then accumulated
// over the stamp in row-major order.  Every product, sum and
// quotient is a separately rounded IEEE double operation in a fixed order, so
// the outputs are a reproducible function of the inputs:
//   S(u, v) = (sum_i img_i) / n(u, v)  over valid in-frame pixels (0 if none)
//   M00 += S, M10 += u S, M01 += v S, M20 += (u u) S, M02 += (v v) S,
//   M11 += (u v) S
//   ub = M10/M00, vb = M01/M00, m20 = M20/M00 - ub ub, m02 = M02/M00 - vb vb,
//   m11 = M11/M00 - ub vb
// and the stamp passes when M00 > 0, |ub|, |vb| <= max_offset,
// |m11| <= max_m11 and m2_min <= m20, m02 <= m2_max.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kbmi_common.h"

namespace kbmi {
namespace {

constexpr int ST_WAVES = 4;                  // candidates (one wave each) per workgroup
constexpr int ST_THREADS = 64 * ST_WAVES;

// floor(v * tau + 0.5) without the clamp of the search's table: a stamp
// reaches R pixels past its centre, so an offset beyond the frame must stay
// exact (|v * tau| < 2^30 is checked on the host).
__device__ inline int stamp_offset(double v, double tau) {
#pragma clang fp contract(off)
    return (int)floor(v * tau + 0.5);
}

struct StampLimits {
    double max_offset, max_m11, m2_min, m2_max;
};

// One wave per candidate.  The lanes cover the stamp's pixels (row-major,
// 64 at a time), so the lanes of one load read runs of adjacent pixels of one
// image row; each lane sums its pixel over the kept images in image order.
// The stamp goes to LDS, and lanes 0-5 take one raw moment each in row-major
// order, with the pixel weights from a table in LDS: every value is the same
// sequence of double operations as one thread per candidate walking the
// stamp.
template <int NB>
__global__ __launch_bounds__(ST_THREADS) void stamp_kernel(
    const float *__restrict__ img, const float *__restrict__ var,
    const uint8_t *__restrict__ mask, int n_img, int h, int w, const double *__restrict__ tau,
    const double2 *__restrict__ vels, int n_vel, const kb_hit *__restrict__ cand,
    const uint64_t *__restrict__ drop, int64_t n_cand, int R, StampLimits lim,
    float *__restrict__ stamps, double *__restrict__ moments, uint8_t *__restrict__ pass) {
#pragma clang fp contract(off)
    // [ST_WAVES][side * side] stamps, then the six moment weights of every
    // stamp pixel [6][side * side]: 1, u, v, u u, v v, u v (exact in double).
    extern __shared__ double s_stamp[];
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * ST_WAVES + wave;
    const bool live = c < n_cand;
    const int side = 2 * R + 1;
    const int npix = side * side;
    double *S_l = s_stamp + (size_t)wave * npix;
    double *W_l = s_stamp + (size_t)ST_WAVES * npix;
    for (int e = (int)threadIdx.x; e < npix; e += ST_THREADS) {
        const int a = e / side, b = e - a * side;
        const double u = (double)(b - R), v = (double)(a - R);
        W_l[e] = 1.0;
        W_l[npix + e] = u;
        W_l[2 * npix + e] = v;
        W_l[3 * npix + e] = u * u;
        W_l[4 * npix + e] = v * v;
        W_l[5 * npix + e] = u * v;
    }
    kb_hit hit{};
    bool ok_vel = false;
    if (live) {
        hit = cand[c];
        ok_vel = hit.vel >= 0 && hit.vel < n_vel;
    }
    int dx[NB], dy[NB];
    uint64_t use = 0;   // images this candidate may use
    {
        const double2 vj = ok_vel ? vels[hit.vel] : make_double2(0.0, 0.0);
        const uint64_t dropped = (live && drop) ? drop[c] : 0;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            dx[i] = 0;
            dy[i] = 0;
            if (ok_vel && i < n_img) {
                dx[i] = stamp_offset(vj.x, tau[i]);
                dy[i] = stamp_offset(vj.y, tau[i]);
                if (!((dropped >> i) & 1u)) use |= uint64_t(1) << i;
            }
        }
    }
    for (int e = lane; e < npix; e += 64) {
        const int a = e / side, b = e - a * side;
        double acc = 0.0;
        int cnt = 0;
        // Images in groups of 16: a group's loads are all issued before the
        // first is used (a term that is not read loads element 0 and is then
        // skipped), then its terms are added in image order.
#pragma unroll
        for (int i0 = 0; i0 < NB; i0 += 16) {
            float im[16], va[16];
            uint8_t mk[16];
            bool in[16];
#pragma unroll
            for (int b16 = 0; b16 < 16; ++b16) {
                const int i = i0 + b16;
                const int64_t yy = (int64_t)hit.y + dy[i] + (a - R);
                const int64_t xx = (int64_t)hit.x + dx[i] + (b - R);
                in[b16] = ((use >> i) & 1u) && yy >= 0 && yy < h && xx >= 0 && xx < w;
                const size_t p = in[b16] ? ((size_t)i * h + yy) * (size_t)w + xx : 0;
                im[b16] = img[p];
                va[b16] = var[p];
                mk[b16] = mask ? mask[p] : 0;
            }
#pragma unroll
            for (int b16 = 0; b16 < 16; ++b16) {
                const bool valid = in[b16] && mk[b16] == 0 && isfinite(im[b16]) &&
                                   isfinite(va[b16]) && va[b16] > 0.f;
                if (valid) {
                    acc = acc + (double)im[b16];
                    ++cnt;
                }
            }
            if (i0 + 16 < NB) __builtin_amdgcn_sched_barrier(0);
        }
        const double S = cnt > 0 ? acc / (double)cnt : 0.0;   // exact int -> double
        S_l[e] = S;
        if (live && stamps) stamps[c * npix + e] = (float)S;
    }
    __syncthreads();
    if (!live) return;
    // Lane m < 6 accumulates raw moment m in row-major order, M += w_m * S
    // with its weight from LDS (1 * S is S): the operations of the six sums
    // of one pass over the stamp, six lanes at a time.
    double M = 0.0;
    if (lane < 6) {
        const double *w_m = W_l + (size_t)lane * npix;
        for (int e = 0; e < npix; ++e) M = M + w_m[e] * S_l[e];
    }
    const double M00 = __shfl(M, 0), M10 = __shfl(M, 1), M01 = __shfl(M, 2);
    const double M20 = __shfl(M, 3), M02 = __shfl(M, 4), M11 = __shfl(M, 5);
    if (lane != 0) return;
    const double ub = M10 / M00, vb = M01 / M00;
    const double m20 = M20 / M00 - ub * ub;
    const double m02 = M02 / M00 - vb * vb;
    const double m11 = M11 / M00 - ub * vb;
    const bool ok = ok_vel && M00 > 0.0 && fabs(ub) <= lim.max_offset &&
                    fabs(vb) <= lim.max_offset && fabs(m11) <= lim.max_m11 &&
                    m20 >= lim.m2_min && m20 <= lim.m2_max && m02 >= lim.m2_min &&
                    m02 <= lim.m2_max;
    pass[c] = ok ? 1 : 0;
    if (moments) {
        double *o = moments + c * 6;
        o[0] = M00;
        o[1] = ub;
        o[2] = vb;
        o[3] = m20;
        o[4] = m02;
        o[5] = m11;
    }
}

template <int NB>
kb_status launch_stamps(const float *img, const float *var, const uint8_t *mask, int n_img,
                        int h, int w, const double *tau, const double2 *vels, int n_vel,
                        const kb_hit *cand, const uint64_t *drop, int64_t n_cand, int R,
                        StampLimits lim, float *stamps, double *moments, uint8_t *pass,
                        hipStream_t s) {
    const int64_t blocks = (n_cand + ST_WAVES - 1) / ST_WAVES;
    const size_t lds = (size_t)(ST_WAVES + 6) * (2 * R + 1) * (2 * R + 1) * sizeof(double);
    hipLaunchKernelGGL(stamp_kernel<NB>, dim3((unsigned)blocks), dim3(ST_THREADS), lds, s, img, var,
                       mask, n_img, h, w, tau, vels, n_vel, cand, drop, n_cand, R, lim, stamps,
                       moments, pass);
    return launch_status("stamp_kernel");
}

}  // namespace
}  // namespace kbmi

using namespace kbmi;

extern "C" {

kb_status kb_stamps(const float *img, const float *var, const uint8_t *mask, int64_t n_img,
                    int64_t h, int64_t w, const double *t, const double *vel, int64_t n_vel,
                    const kb_hit *cand, const uint64_t *drop, int64_t n_cand, int32_t radius,
                    double max_offset, double max_m11, double m2_min, double m2_max,
                    float *stamps, double *moments, uint8_t *pass, void *workspace,
                    size_t workspace_bytes, void *stream) {
    clear_error();
    if (n_cand < 0) return fail(KB_EINVAL, "n_cand must be >= 0");
    if (!img || !var || !t || !vel || !pass || (n_cand > 0 && !cand))
        return fail(KB_EINVAL, "img, var, times, velocities, candidates and pass must be non-null");
    kb_status st = check_frame(n_img, h, w);
    if (st != KB_OK) return st;
    if (n_img > KB_MAX_LC_IMAGES)
        return fail(KB_EUNSUPPORTED, "stamps take at most %d images (got %lld)",
                    KB_MAX_LC_IMAGES, (long long)n_img);
    if (n_vel < 1 || n_vel > 65535)
        return fail(KB_EINVAL, "n_vel must be in [1, 65535] (got %lld)", (long long)n_vel);
    if (radius < 0 || radius > KB_MAX_STAMP_RADIUS)
        return fail(KB_EINVAL, "radius must be in [0, %d] (got %d)", KB_MAX_STAMP_RADIUS,
                    (int)radius);
    if (std::isnan(max_offset) || std::isnan(max_m11) || std::isnan(m2_min) || std::isnan(m2_max))
        return fail(KB_EINVAL, "filter bounds must not be NaN");
    if (n_cand > (int64_t)ST_WAVES * 2147483647LL)
        return fail(KB_EINVAL, "too many candidates for one launch");
    st = check_times_velocities(t, n_img, vel, n_vel);
    if (st != KB_OK) return st;
    if (!workspace) return fail(KB_EINVAL, "stamps need a workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KB_EINVAL, "workspace must be 256-byte aligned");
    const size_t ws_need = workspace_layout(n_img, h, w, n_vel).total;
    if (workspace_bytes < ws_need)
        return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", ws_need, workspace_bytes);
    if (n_cand == 0) return KB_OK;
    hipStream_t s = (hipStream_t)stream;
    size_t vel_off = 0;
    st = upload_tau_vel(t, n_img, vel, n_vel, workspace, s, &vel_off);
    if (st != KB_OK) return st;
    const char *ws = static_cast<const char *>(workspace);
    const double *tau = reinterpret_cast<const double *>(ws);
    const double2 *vels = reinterpret_cast<const double2 *>(ws + vel_off);
    const StampLimits lim{max_offset, max_m11, m2_min, m2_max};
    if (n_img <= 16)
        return launch_stamps<16>(img, var, mask, (int)n_img, (int)h, (int)w, tau, vels,
                                 (int)n_vel, cand, drop, n_cand, radius, lim, stamps, moments,
                                 pass, s);
    if (n_img <= 32)
        return launch_stamps<32>(img, var, mask, (int)n_img, (int)h, (int)w, tau, vels,
                                 (int)n_vel, cand, drop, n_cand, radius, lim, stamps, moments,
                                 pass, s);
    return launch_stamps<64>(img, var, mask, (int)n_img, (int)h, (int)w, tau, vels, (int)n_vel,
                             cand, drop, n_cand, radius, lim, stamps, moments, pass, s);
}

}  // extern "C"
