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
constexpr int LC_PAIRS = 4032;                       // pairs of a grouped workgroup, at most
constexpr int LC_MAXQ = (LC_PAIRS + GR_THREADS - 1) / GR_THREADS;   // pairs per thread, at most
constexpr int LC_PX = 64;                            // start pixels per grouped tile, at most
static_assert(LC_THREADS == GR_THREADS, "the grouped filter uses the shared grouping");

// The light curve of candidate (start pixel p, velocity index j; an index
// outside [0, n_vel) has no observation) into v; returns the observed images'
// bits.  Every image's load is issued before any is used (an out-of-frame or
// missing term reads pixel 0 and is then replaced by +0), so the loads of a
// light curve are in flight together.
template <int NB>
__device__ __forceinline__ uint64_t gather_light_curve(int64_t p, int j, int h, int w, int n_img,
                                                       const float2 *__restrict__ planes,
                                                       const double *__restrict__ tau,
                                                       const double2 *__restrict__ vels,
                                                       int n_vel, float2 (&v)[NB]) {
    const bool has = j >= 0 && j < n_vel;
    const double2 vj = vels[has ? j : 0];
    const int y0 = (int)(p / w), x0 = (int)(p - (int64_t)y0 * w);
    bool ok[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const double ti = tau[i < n_img ? i : 0];
        const int y = y0 + displacement(vj.y, ti, h);
        const int x = x0 + displacement(vj.x, ti, w);
        ok[i] = has && i < n_img && (unsigned)y < (unsigned)h && (unsigned)x < (unsigned)w;
        const size_t at = ok[i] ? ((size_t)i * h + y) * (size_t)w + x : 0;
        v[i] = planes[at];
    }
    uint64_t obs = 0;   // bit i: image i observes the trajectory
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if (!ok[i]) v[i] = make_float2(0.f, 0.f);
        // Validity is carried by phi's bits: invalid pixels hold +0.
        if (__float_as_uint(v[i].y) != 0u) obs |= uint64_t(1) << i;
    }
    return obs;
}

// J / d and H / d, each correctly rounded (IEEE double), by the hardware's
// division sequence: scale the divisor and the numerator against each other,
// refine the reciprocal of the scaled divisor (two Newton steps), form the
// quotient, correct it with a fused residual and fix up the special cases.
// The refined reciprocal depends only on the scaled divisor, so H's quotient
// reuses J's wherever both numerators leave the divisor scaled alike (always,
// short of exponents 2^1000 apart); elsewhere H's is refined on its own.  Each
// quotient takes exactly the steps of a division of its own.
__device__ __forceinline__ double refined_rcp(double ds) {
    const double r = __builtin_amdgcn_rcp(ds);
    const double e0 = __builtin_fma(-ds, r, 1.0);
    const double r1 = __builtin_fma(r, e0, r);
    const double e1 = __builtin_fma(-ds, r1, 1.0);
    return __builtin_fma(r1, e1, r1);
}
__device__ __forceinline__ double quotient(double a, double d, double ds, double r) {
    bool flag;
    const double ns = __builtin_amdgcn_div_scale(a, d, true, &flag);
    const double m = ns * r;
    const double rem = __builtin_fma(-ds, m, ns);
    return __builtin_amdgcn_div_fixup(__builtin_amdgcn_div_fmas(rem, r, m, flag), d, a);
}
__device__ __forceinline__ void divide_pair(double &J, double &H, double d) {
    bool unused;
    const double dsj = __builtin_amdgcn_div_scale(J, d, false, &unused);
    const double dsh = __builtin_amdgcn_div_scale(H, d, false, &unused);
    const double rj = refined_rcp(dsj);
    double rh = rj;
    const bool alike = __double_as_longlong(dsj) == __double_as_longlong(dsh);
    if (__builtin_expect(__any(!alike), 0)) {
        if (!alike) rh = refined_rcp(dsh);
    }
    J = quotient(J, d, dsj, rj);
    H = quotient(H, d, dsh, rh);
}

// One round of the filter over the kept observations: the largest squared
// standardised residual (-1 if none is kept) and, in `worst`, its image (the
// lowest among equal values).
template <int NB>
__device__ __forceinline__ double filter_round(const float2 (&v)[NB], uint64_t keep,
                                               const double *__restrict__ tau, double q,
                                               int &worst) {
#pragma clang fp contract(off)
    const bool walk = q > 0.0;
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
                divide_pair(J, H, d);
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
    worst = 0;
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
        if ((keep >> i) & 1u) {
            const double ti = tau[i];
            if (seen && walk) {
                const double s = q * (tp - ti);
                const double d = 1.0 + s * J;
                divide_pair(J, H, d);
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
    return rmax;
}

// The refit from the kept observations, summed in image order in double.
template <int NB>
__device__ __forceinline__ void refit(const float2 (&v)[NB], uint64_t keep, float &out_nu,
                                      float &out_al, int &n) {
#pragma clang fp contract(off)
    double P = 0.0, F = 0.0;
    n = 0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if ((keep >> i) & 1u) {
            P = P + (double)v[i].x;
            F = F + (double)v[i].y;
            ++n;
        }
    }
    out_nu = -INFINITY;
    out_al = 0.f;
    if (F > 0.0) {
        out_nu = (float)(P / sqrt(F));
        out_al = (float)(P / F);
    }
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
    float2 v[NB];
    const uint64_t obs =
        gather_light_curve<NB>(c / k, cand_vel[c], h, w, n_img, planes, tau, vels, n_vel, v);
    uint64_t keep = obs;
    for (;;) {   // at most popcount(obs) + 1 rounds
        int worst;
        if (!(filter_round<NB>(v, keep, tau, q, worst) > c2)) break;
        keep &= ~(uint64_t(1) << worst);
    }
    float o_nu, o_al;
    int n;
    refit<NB>(v, keep, o_nu, o_al, n);
    nu[c] = o_nu;
    alpha[c] = o_al;
    nobs[c] = (int16_t)n;
    if (rejected) rejected[c] = obs & ~keep;
}

// LDS of a grouped workgroup for np_max pairs: per pair its velocity index
// (then its nu), alpha, grouped order, two queue slots and n_obs, then the
// grouping state.
size_t lightcurve_lds_bytes(int np_max) {
    return (((size_t)np_max * (4 + 4 + 2 + 2 + 2 + 1) + 15) & ~(size_t)15) + 16 +
           group_lds_bytes();
}

// A workgroup per tile of pt start pixels of one row and their pt * k
// candidates, grouped by velocity before they are gathered (the re-score's
// grouping); XCD x walks down tile columns x, x + 8, ... as the re-score
// does, so the eight XCDs sweep adjacent columns at about the same rows.
//
// The lanes of a wave filter different candidates in step, so a lane that
// drops an observation holds its whole wave for another round, and on
// workloads where most candidates drop one observation nearly every wave runs
// two or three rounds.  With NB = 16 the rounds are therefore taken in
// passes: pass 0 runs the first round of every candidate; a candidate that
// drops an observation is queued, and pass p runs round p + 1 of the queued
// candidates (regathering their light curves) until the queue is empty.  Each
// candidate still runs the same rounds in the same order, so its results do
// not change.  A pass-0 queue entry holds the pair and the image it dropped;
// later entries hold the pair, with its dropped images in the grouped-order
// slot it no longer needs.  Results are staged in LDS and written as
// contiguous runs of the tile's candidates.
template <int NB>
__global__ __launch_bounds__(LC_THREADS, NB == 16 ? 3 : 1) void lightcurve_grouped_kernel(
    int k, int pt, int h, int w, int row0, int n_rows, int n_img,
    const float2 *__restrict__ planes, const double *__restrict__ tau,
    const double2 *__restrict__ vels, int n_vel, double c2, double q,
    const int32_t *__restrict__ cand_vel, float *__restrict__ nu, float *__restrict__ alpha,
    int16_t *__restrict__ nobs, uint64_t *__restrict__ rejected) {
    extern __shared__ __align__(16) unsigned char lc_lds[];
    const int np_max = pt * k;
    int32_t *s_vj = reinterpret_cast<int32_t *>(lc_lds);   // velocity index, then nu (bits)
    float *s_al = reinterpret_cast<float *>(lc_lds + (size_t)np_max * 4);
    uint16_t *s_ord = reinterpret_cast<uint16_t *>(lc_lds + (size_t)np_max * 8);
    uint16_t *s_q0 = s_ord + np_max;
    uint16_t *s_q1 = s_q0 + np_max;
    uint8_t *s_no = reinterpret_cast<uint8_t *>(s_q1 + np_max);
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(lc_lds + (((size_t)np_max * 15 + 15) & ~15ull));
    uint32_t *s_bin = s_cnt + 4;
    static_assert(LC_PAIRS <= 4096, "a queue entry holds a 12-bit pair index");
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
    if (t < 2) s_cnt[t] = 0u;   // queue lengths (the grouping's barriers publish them)
    const int n_sorted = group_pairs_by_velocity<LC_MAXQ>(cand_vel + c0, np, n_vel, s_vj, s_ord,
                                                          s_bin, s_bin + GR_BINS);
    // Candidates whose index is outside the grid have no observation:
    // nu = -inf, alpha = 0, nothing kept.
    for (int qq = t; qq < np; qq += LC_THREADS)
        if (s_vj[qq] < 0) {
            s_vj[qq] = (int32_t)__float_as_uint(-INFINITY);
            s_al[qq] = 0.f;
            s_no[qq] = 0;
            if (rejected) rejected[c0 + qq] = 0;
        }
    int n_items = n_sorted;
#pragma unroll 1
    for (int pass = 0; n_items > 0; ++pass) {
        uint16_t *q_in = (pass & 1) ? s_q0 : s_q1;    // read by passes >= 1
        uint16_t *q_out = (pass & 1) ? s_q1 : s_q0;
        uint32_t *n_out = s_cnt + (pass & 1);
        for (int it = t; it < n_items; it += LC_THREADS) {
            int qq;
            uint64_t dropped = 0;
            if (pass == 0) {
                qq = s_ord[it];
            } else if (pass == 1) {
                const uint32_t e = q_in[it];
                qq = (int)(e & 0xFFFu);
                dropped = uint64_t(1) << (e >> 12);
            } else {
                qq = q_in[it];
                dropped = s_ord[qq];
            }
            float2 v[NB];
            const uint64_t obs = gather_light_curve<NB>(p0 + qq / k, s_vj[qq], h, w, n_img,
                                                        planes, tau, vels, n_vel, v);
            uint64_t keep = obs & ~dropped;
            bool queued = false;
            for (;;) {   // at most popcount(obs) + 1 rounds
                int worst;
                if (!(filter_round<NB>(v, keep, tau, q, worst) > c2)) break;
                keep &= ~(uint64_t(1) << worst);
                if constexpr (NB == 16) {
                    // The next round in the next pass.
                    const uint32_t slot = atomicAdd(n_out, 1u);
                    if (pass == 0) {
                        q_out[slot] = (uint16_t)(qq | (worst << 12));
                    } else {
                        s_ord[qq] = (uint16_t)(obs & ~keep);
                        q_out[slot] = (uint16_t)qq;
                    }
                    queued = true;
                    break;
                }
            }
            if (!queued) {
                float o_nu, o_al;
                int n;
                refit<NB>(v, keep, o_nu, o_al, n);
                s_vj[qq] = (int32_t)__float_as_uint(o_nu);
                s_al[qq] = o_al;
                s_no[qq] = (uint8_t)n;
                if (rejected) rejected[c0 + qq] = obs & ~keep;
            }
        }
        __syncthreads();
        if constexpr (NB == 16) {
            n_items = (int)*n_out;
            __syncthreads();              // every thread has read the count
            if (t == 0) *n_out = 0u;      // this counter serves pass + 2
        } else {
            n_items = 0;
        }
    }
    for (int qq = t; qq < np; qq += LC_THREADS) {
        nu[c0 + qq] = __uint_as_float((uint32_t)s_vj[qq]);
        alpha[c0 + qq] = s_al[qq];
        nobs[c0 + qq] = (int16_t)s_no[qq];
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
                           dim3(LC_THREADS), lightcurve_lds_bytes(pt * k), s, k, pt, h, w,
                           (int)r0, n_rows, n_img, planes, tau, vels, n_vel, c2, q, cv, nu, al,
                           no, rej);
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
