// Light-curve outlier filter of libkbmi (Sec. 3.3, filtering of candidate
// trajectories): for every candidate trajectory, the per-image likelihood
// values along it are run through a Kalman filter on the flux; observations
// more than sigma_cut standard deviations from the estimate made without them
// are dropped one at a time (largest first), and nu, alpha and n_obs are
// recomputed from what remains.
//
// One thread per candidate; a workgroup takes the candidates of a tile of
// start pixels of one row, grouped by velocity before they are gathered (so
// the lanes of one load mostly share a velocity and read adjacent pixels).
// A candidate's light curve (at most KB_MAX_LC_IMAGES pairs) is gathered once
// into registers; the filter then runs in IEEE double with
// every product, sum and quotient rounded separately, so that each keep or
// drop decision is a reproducible function of the float32 planes:
//   prediction over dtau (random-walk flux, variance q per day):
//       d = 1 + (q * dtau) * J,  J <- J / d,  H <- H / d
//   update with observation i:  J <- J + phi_i,  H <- H + psi_i
//   leave-one-out information at k:  J_k = Jf_k + Jb_k,  H_k = Hf_k + Hb_k
//       (forward prediction into k plus backward prediction into k)
//   squared standardised residual:
//       r_k = (a * a) / ((phi_k * J_k) * (J_k + phi_k)),  a = psi_k J_k - phi_k H_k
//       (0 when the divisor is not positive)
// The observation with the largest r_k (lowest image among equal values) is
// dropped while r_k > sigma_cut^2; each drop reruns the filter on the rest.
// The refit sums the kept pairs in image order in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "kbmi_common.h"
#include "kbmi_group.h"

namespace kbmi {
namespace {

constexpr int LC_THREADS = 256;
constexpr int LC_PAIRS = 4096;                       // pairs of a grouped workgroup, at most
constexpr int LC_MAXQ = LC_PAIRS / GR_THREADS;       // pairs per thread, at most
constexpr int LC_PX = 64;                            // start pixels per grouped tile, at most
static_assert(LC_THREADS == GR_THREADS, "the grouped filter uses the shared grouping");

// The filter of one candidate c (start pixel p, velocity index j; an index
// outside [0, n_vel) has no observation).
template <int NB>
__device__ __forceinline__ void filter_candidate(int64_t c, int64_t p, int j, int h, int w, int n_img,
                                        const float2 *__restrict__ planes,
                                        const double *__restrict__ tau,
                                        const double2 *__restrict__ vels, int n_vel, double c2,
                                        double q, float *__restrict__ nu,
                                        float *__restrict__ alpha, int16_t *__restrict__ nobs,
                                        uint64_t *__restrict__ rejected) {
#pragma clang fp contract(off)
    float2 v[NB];
    uint64_t obs = 0;   // bit i: image i observes the trajectory
#pragma unroll
    for (int i = 0; i < NB; ++i) v[i] = make_float2(0.f, 0.f);
    if (j >= 0 && j < n_vel) {
        const int y0 = (int)(p / w), x0 = (int)(p - (int64_t)y0 * w);
        const double2 vj = vels[j];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (i < n_img) {
                const double ti = tau[i];
                const int y = y0 + displacement(vj.y, ti, h);
                const int x = x0 + displacement(vj.x, ti, w);
                if ((unsigned)y < (unsigned)h && (unsigned)x < (unsigned)w) {
                    v[i] = planes[((size_t)i * h + y) * (size_t)w + x];
                    // Validity is carried by phi's bits: invalid pixels hold +0.
                    if (__float_as_uint(v[i].y) != 0u) obs |= uint64_t(1) << i;
                }
            }
        }
    }

    uint64_t keep = obs;
    const bool walk = q > 0.0;
    for (;;) {
        double Jf[NB], Hf[NB];
        double J = 0.0, H = 0.0, tp = 0.0;
        bool seen = false;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if ((keep >> i) & 1u) {
                const double ti = tau[i];
                if (seen && walk) {
                    const double s = q * (ti - tp);
                    const double d = 1.0 + s * J;
                    J = J / d;
                    H = H / d;
                }
                Jf[i] = J;
                Hf[i] = H;
                J = J + (double)v[i].y;
                H = H + (double)v[i].x;
                tp = ti;
                seen = true;
            }
        }
        J = 0.0;
        H = 0.0;
        tp = 0.0;
        seen = false;
        double rmax = -1.0;
        int worst = 0;
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
            if ((keep >> i) & 1u) {
                const double ti = tau[i];
                if (seen && walk) {
                    const double s = q * (tp - ti);
                    const double d = 1.0 + s * J;
                    J = J / d;
                    H = H / d;
                }
                const double ps = (double)v[i].x, ph = (double)v[i].y;
                const double Jk = Jf[i] + J, Hk = Hf[i] + H;
                const double a = ps * Jk - ph * Hk;
                const double dv = (ph * Jk) * (Jk + ph);
                const double r = dv > 0.0 ? (a * a) / dv : 0.0;
                if (r >= rmax) {    // descending i: the lowest index wins a tie
                    rmax = r;
                    worst = i;
                }
                J = J + ph;
                H = H + ps;
                tp = ti;
                seen = true;
            }
        }
        if (!(rmax > c2)) break;
        keep &= ~(uint64_t(1) << worst);   // at most popcount(obs) iterations
    }

    double P = 0.0, F = 0.0;
    int n = 0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if ((keep >> i) & 1u) {
            P = P + (double)v[i].x;
            F = F + (double)v[i].y;
            ++n;
        }
    }
    float out_nu = -INFINITY, out_al = 0.f;
    if (F > 0.0) {
        out_nu = (float)(P / sqrt(F));
        out_al = (float)(P / F);
    }
    nu[c] = out_nu;
    alpha[c] = out_al;
    nobs[c] = (int16_t)n;
    if (rejected) rejected[c] = obs & ~keep;
}

// One thread per candidate, in list order (lists longer than LC_PAIRS).
template <int NB>
__global__ __launch_bounds__(LC_THREADS) void lightcurve_kernel(
    int64_t ncand, int k, int h, int w, int n_img, const float2 *__restrict__ planes,
    const double *__restrict__ tau, const double2 *__restrict__ vels, int n_vel, double c2,
    double q, const int32_t *__restrict__ cand_vel, float *__restrict__ nu,
    float *__restrict__ alpha, int16_t *__restrict__ nobs, uint64_t *__restrict__ rejected) {
    const int64_t c = (int64_t)blockIdx.x * LC_THREADS + threadIdx.x;
    if (c >= ncand) return;
    filter_candidate<NB>(c, c / k, cand_vel[c], h, w, n_img, planes, tau, vels, n_vel, c2, q,
                         nu, alpha, nobs, rejected);
}

// A workgroup per tile of pt start pixels of one row and their pt * k
// candidates, grouped by velocity before they are gathered (the re-score's
// grouping); XCD x walks down tile columns x, x + 8, ... as the re-score
// does, so the eight XCDs sweep adjacent columns at about the same rows.
template <int NB>
__global__ __launch_bounds__(LC_THREADS, NB == 16 ? 3 : 1) void lightcurve_grouped_kernel(
    int k, int pt, int h, int w, int row0, int n_rows, int n_img,
    const float2 *__restrict__ planes, const double *__restrict__ tau,
    const double2 *__restrict__ vels, int n_vel, double c2, double q,
    const int32_t *__restrict__ cand_vel, float *__restrict__ nu, float *__restrict__ alpha,
    int16_t *__restrict__ nobs, uint64_t *__restrict__ rejected) {
    __shared__ int32_t s_vj[LC_PAIRS];
    __shared__ uint16_t s_ord[LC_PAIRS];
    __shared__ uint32_t s_bin[GR_BINS + 8];
    const int n_ct = (w + pt - 1) / pt;
    const int64_t kb = (int64_t)(blockIdx.x >> 3);
    const int64_t ct64 = 8 * (kb / n_rows) + (int64_t)(blockIdx.x & 7u);
    if (ct64 >= n_ct) return;
    const int64_t row = row0 + kb % n_rows;
    const int ct = (int)ct64;
    const int64_t p0 = row * w + (int64_t)ct * pt;
    const int npx = min(pt, w - ct * pt);
    const int np = npx * k;
    const int t = (int)threadIdx.x;
    const int64_t c0 = p0 * (int64_t)k;
    const int n_sorted = group_pairs_by_velocity<LC_MAXQ>(cand_vel + c0, np, n_vel, s_vj, s_ord,
                                                          s_bin, s_bin + GR_BINS);
    for (int pos = t; pos < n_sorted; pos += LC_THREADS) {
        const int qq = s_ord[pos];
        filter_candidate<NB>(c0 + qq, p0 + qq / k, s_vj[qq], h, w, n_img, planes, tau, vels,
                             n_vel, c2, q, nu, alpha, nobs, rejected);
    }
    // Candidates whose index is outside the grid have no observation: what
    // filter_candidate gives them (nu = -inf, alpha = 0, nothing kept).
    for (int qq = t; qq < np; qq += LC_THREADS)
        if (s_vj[qq] < 0) {
            nu[c0 + qq] = -INFINITY;
            alpha[c0 + qq] = 0.f;
            nobs[c0 + qq] = 0;
            if (rejected) rejected[c0 + qq] = 0;
        }
}

template <int NB>
kb_status launch_lightcurve(int64_t ncand, int k, int h, int w, int n_img, const float2 *planes,
                            const double *tau, const double2 *vels, int n_vel, double c2,
                            double q, const int32_t *cv, float *nu, float *al, int16_t *no,
                            uint64_t *rej, hipStream_t s) {
    if (k > LC_PAIRS) {
        const int64_t blocks = (ncand + LC_THREADS - 1) / LC_THREADS;
        hipLaunchKernelGGL(lightcurve_kernel<NB>, dim3((unsigned)blocks), dim3(LC_THREADS), 0, s,
                           ncand, k, h, w, n_img, planes, tau, vels, n_vel, c2, q, cv, nu, al,
                           no, rej);
        return launch_status("lightcurve_kernel");
    }
    // Eight workgroups per row for each group of eight tile columns; rows in
    // launches of at most 2^31 - 1 workgroups.
    const int pt = std::min(LC_PX, LC_PAIRS / k);
    const int64_t n_ct = ((int64_t)w + pt - 1) / pt;
    const int64_t per_row = 8 * ((n_ct + 7) / 8);
    const int64_t max_rows = 2147483647LL / per_row;
    for (int64_t r0 = 0; r0 < h; r0 += max_rows) {
        const int n_rows = (int)std::min<int64_t>(max_rows, h - r0);
        hipLaunchKernelGGL(lightcurve_grouped_kernel<NB>, dim3((unsigned)(per_row * n_rows)),
                           dim3(LC_THREADS), 0, s, k, pt, h, w, (int)r0, n_rows, n_img, planes,
                           tau, vels, n_vel, c2, q, cv, nu, al, no, rej);
        const kb_status st = launch_status("lightcurve_grouped_kernel");
        if (st != KB_OK) return st;
    }
    return KB_OK;
}

}  // namespace
}  // namespace kbmi

using namespace kbmi;

extern "C" {

kb_status kb_lightcurve_filter(const float *psi_phi, int64_t n_img, int64_t h, int64_t w,
                               const double *t, const double *vel, int64_t n_vel,
                               const int32_t *cand_vel, int64_t k, double sigma_cut, double q,
                               float *nu, float *alpha, int16_t *nobs, uint64_t *rejected,
                               void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!psi_phi || !t || !vel || !cand_vel || !nu || !alpha || !nobs)
        return fail(KB_EINVAL, "planes, times, velocities, candidates and outputs must be non-null");
    kb_status st = check_frame(n_img, h, w);
    if (st != KB_OK) return st;
    if (n_img > KB_MAX_LC_IMAGES)
        return fail(KB_EUNSUPPORTED, "the light-curve filter takes at most %d images (got %lld)",
                    KB_MAX_LC_IMAGES, (long long)n_img);
    if (n_vel < 1 || n_vel > 65535)
        return fail(KB_EINVAL, "n_vel must be in [1, 65535] (got %lld)", (long long)n_vel);
    if (k < 1 || k > 65535) return fail(KB_EINVAL, "k must be in [1, 65535] (got %lld)", (long long)k);
    if (!(std::isfinite(sigma_cut) && sigma_cut > 0.0))
        return fail(KB_EINVAL, "sigma_cut must be finite and positive");
    if (!(std::isfinite(q) && q >= 0.0)) return fail(KB_EINVAL, "q must be finite and >= 0");
    const double c2 = sigma_cut * sigma_cut;
    if (!std::isfinite(c2)) return fail(KB_EINVAL, "sigma_cut squared overflows");
    const int64_t ncand = h * w * k;
    if ((ncand + LC_THREADS - 1) / LC_THREADS > 2147483647LL)
        return fail(KB_EINVAL, "too many candidates for one launch");
    st = check_times_velocities(t, n_img, vel, n_vel);
    if (st != KB_OK) return st;
    if (!workspace) return fail(KB_EINVAL, "the filter needs a workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KB_EINVAL, "workspace must be 256-byte aligned");
    const size_t ws_need = workspace_layout(n_img, h, w, n_vel).total;
    if (workspace_bytes < ws_need)
        return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", ws_need, workspace_bytes);

    hipStream_t s = (hipStream_t)stream;
    size_t vel_off = 0;
    st = upload_tau_vel(t, n_img, vel, n_vel, workspace, s, &vel_off);
    if (st != KB_OK) return st;
    const char *ws = static_cast<const char *>(workspace);
    const double *tau = reinterpret_cast<const double *>(ws);
    const double2 *vels = reinterpret_cast<const double2 *>(ws + vel_off);
    const float2 *planes = reinterpret_cast<const float2 *>(psi_phi);
    if (n_img <= 16)
        return launch_lightcurve<16>(ncand, (int)k, (int)h, (int)w, (int)n_img, planes, tau,
                                     vels, (int)n_vel, c2, q, cand_vel, nu, alpha, nobs,
                                     rejected, s);
    if (n_img <= 32)
        return launch_lightcurve<32>(ncand, (int)k, (int)h, (int)w, (int)n_img, planes, tau,
                                     vels, (int)n_vel, c2, q, cand_vel, nu, alpha, nobs,
                                     rejected, s);
    return launch_lightcurve<64>(ncand, (int)k, (int)h, (int)w, (int)n_img, planes, tau, vels,
                                 (int)n_vel, c2, q, cand_vel, nu, alpha, nobs, rejected, s);
}

}  // extern "C"
