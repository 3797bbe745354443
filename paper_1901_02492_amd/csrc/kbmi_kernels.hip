// HIP kernels and device entry points of libkbmi (gfx950 / CDNA4, wave64).
//
//   psi_phi_kernel   likelihood images psi, phi (Sec. 2.1.5 Psi/Phi equations,
//                    masking paragraph; Sec. 2.3 single-pass 2-D kernel)
//   search_kernel    coadd along every linear trajectory and keep the best
//                    k_cand per start pixel (Sec. 2.1.5 coadd equations and
//                    nu; Sec. 2.2 exhaustive search over (y0, v))
//   topk_kernel      order each pixel's candidates and keep k
//
// The search is a gather-sum, not a contraction, so nothing here uses MFMA.
// Each lane owns one start pixel; a wave covers 64 adjacent pixels of one row,
// so for a fixed (velocity, image) the wave's 64 reads are one contiguous
// 512-byte run of interleaved (psi, phi) pairs.  Reads go through raw buffer
// loads whose hardware range check returns zero for columns outside the frame
// and for rows outside the frame (a zero-length buffer), so out-of-frame
// positions add exactly +0 and count nothing, without per-lane branches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "kbmi_internal.h"

// Launch-shape defaults (compile-time tunables).
#ifndef KBMI_STRIP_TILES
#define KBMI_STRIP_TILES 4      // start-pixel tiles per strip of the tile order
#endif
#ifndef KBMI_QUEUE
#define KBMI_QUEUE 16           // queued candidates per lane before a merge
#endif

namespace kbmi {
namespace {

// ---------------------------------------------------------------------------
// Raw buffer access (stride 0: an access is out of range when its byte offset
// is >= the buffer's record count, and then a load returns 0).
// ---------------------------------------------------------------------------
constexpr int kBufferFlags = 0x00020000;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kBufferFlags);
}

// ---------------------------------------------------------------------------
// Likelihood images.
// ---------------------------------------------------------------------------
struct PsfTaps {
    float t[KB_MAX_PSF * KB_MAX_PSF];
};

constexpr int PP_TW = 64;       // output tile width (one wave's lanes)
constexpr int PP_TH = 16;       // output tile height
constexpr int PP_THREADS = 256; // 4 waves; each thread produces 4 rows of one column
constexpr int PP_LW = PP_TW + KB_MAX_PSF - 1;
constexpr int PP_LH = PP_TH + KB_MAX_PSF - 1;

__global__ __launch_bounds__(PP_THREADS) void psi_phi_kernel(
    const float *__restrict__ img, const float *__restrict__ var,
    const uint8_t *__restrict__ mask, int h, int w, int ph, int pw, PsfTaps psf,
    float2 *__restrict__ out) {
    __shared__ float s_a[PP_LH * PP_LW];
    __shared__ float s_w[PP_LH * PP_LW];
    __shared__ uint8_t s_ok[PP_LH * PP_LW];

    const int i = blockIdx.z;
    const int tx0 = blockIdx.x * PP_TW;
    const int ty0 = blockIdx.y * PP_TH;
    const int cy = ph / 2, cx = pw / 2;
    const int lh = PP_TH + ph - 1, lw = PP_TW + pw - 1;
    const size_t plane = (size_t)i * (size_t)h * (size_t)w;

    // Stage a = valid * img / var and w = valid / var for the tile plus halo.
    for (int idx = threadIdx.x; idx < lh * lw; idx += PP_THREADS) {
        const int ly = idx / lw, lx = idx - ly * lw;
        const int gy = ty0 + ly - cy, gx = tx0 + lx - cx;
        float a = 0.f, wt = 0.f;
        uint8_t ok = 0;
        if (gy >= 0 && gy < h && gx >= 0 && gx < w) {
            const size_t p = plane + (size_t)gy * w + gx;
            const float im = img[p], vr = var[p];
            const bool good = (mask == nullptr || mask[p] == 0) && isfinite(im) &&
                              isfinite(vr) && vr > 0.f;
            if (good) {
                wt = 1.0f / vr;
                a = im / vr;
                ok = 1;
            }
        }
        s_a[ly * PP_LW + lx] = a;
        s_w[ly * PP_LW + lx] = wt;
        s_ok[ly * PP_LW + lx] = ok;
    }
    __syncthreads();

    const int lx = threadIdx.x & (PP_TW - 1);
    const int ly0 = threadIdx.x / PP_TW;   // rows ly0, ly0 + 4, ly0 + 8, ly0 + 12
    float ps[4] = {0.f, 0.f, 0.f, 0.f}, pf[4] = {0.f, 0.f, 0.f, 0.f};
    for (int u = 0; u < ph; ++u) {
        for (int v = 0; v < pw; ++v) {
            const float tv = psf.t[u * pw + v];
            const float t2 = tv * tv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = (ly0 + 4 * r + u) * PP_LW + lx + v;
                ps[r] = fmaf(s_a[o], tv, ps[r]);
                pf[r] = fmaf(s_w[o], t2, pf[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gy = ty0 + ly0 + 4 * r, gx = tx0 + lx;
        if (gy < h && gx < w) {
            float2 res = make_float2(0.f, 0.f);
            if (s_ok[(ly0 + 4 * r + cy) * PP_LW + lx + cx]) {
                // phi >= 0 always; a valid pixel keeps a nonzero bit pattern.
                res = make_float2(ps[r], pf[r] > 0.f ? pf[r] : -0.0f);
            }
            out[plane + (size_t)gy * w + gx] = res;
        }
    }
}

// ---------------------------------------------------------------------------
// Candidate keys.  A candidate is ordered by (nu descending, j ascending); the
// 64-bit key (order-preserving bits of nu) << 32 | (0xFFFF - j) << 16 | n_obs
// compares the same way as unsigned integers.  n_obs never decides an order
// because j is unique within a pixel.  Key 0 is below every real candidate
// (nu = -inf maps to 0x007FFFFF) and marks an empty slot.
// ---------------------------------------------------------------------------
__device__ inline uint32_t nu_order_bits(float nu) {
    uint32_t u = __float_as_uint(nu);
    if (u == 0x80000000u) u = 0u;   // -0 ranks equal to +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline float nu_from_order_bits(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ inline uint64_t make_key(float nu, int j, uint32_t nobs) {
    return ((uint64_t)nu_order_bits(nu) << 32) |
           (uint64_t)(((uint32_t)(0xFFFF - j) << 16) | (nobs & 0xFFFFu));
}

// Start-pixel tiles: one wave = 64 adjacent pixels of one row.  Tiles are
// enumerated in strips `strip` tiles wide (all rows of a strip, then the next
// strip) so that consecutive workgroups cover a compact 2-D patch, and the
// workgroup index is remapped so that each of the 8 XCDs (which receive
// workgroups round-robin) walks one contiguous range of that order and its
// L2 sees neighbouring patches.
struct TileMap {
    int nseg;     // tiles per row
    int h;        // rows
    int strip;    // tiles per strip
    int nblocks;  // nseg * h

    __device__ inline void map(int b, int &row, int &seg) const {
        const int xcd = b & 7, k = b >> 3;
        const int q = nblocks >> 3, r = nblocks & 7;
        const int t = xcd * q + (xcd < r ? xcd : r) + k;
        const int fs = nseg / strip;
        const int full = fs * h * strip;
        if (t < full) {
            const int s = t / (h * strip);
            const int rem = t - s * h * strip;
            row = rem / strip;
            seg = s * strip + (rem - (rem / strip) * strip);
        } else {
            const int rw = nseg - fs * strip;
            const int rem = t - full;
            row = rem / rw;
            seg = fs * strip + (rem - (rem / rw) * rw);
        }
    }
};

// ---------------------------------------------------------------------------
// Trajectory search.
//
// One wave (one workgroup) owns 64 adjacent start pixels of one row and walks
// every velocity in the host-chosen visiting order.  Per velocity each lane
// gathers its trajectory's N (psi, phi) pairs (one coalesced 512-byte run per
// image across the wave), sums them in image order and scores nu.
//
// Per-pixel selection keeps a descending list of KM >= k_cand keys in
// registers.  Inserting into it costs a compare-and-swap per slot, and the wave
// pays for it whenever any lane inserts, so candidates are first filtered
// against a per-lane threshold (the list's last key at the last merge) and
// parked in a per-lane LDS queue of PB entries; the queue is merged into the
// list only when some lane's queue is full (and at the end).  A candidate that
// fails the threshold can never enter the final list: the threshold only rises.
//
// The loads of up to NB images are issued together before they are summed in
// image order; larger stacks are summed in batches of NB images.  The kernel
// is bounded to two waves per SIMD: memory-level parallelism comes from the
// waves, each holding one velocity's NB loads in flight.
// ---------------------------------------------------------------------------
template <int KM, int NB, int PB>
__global__ __launch_bounds__(64, 2) void search_kernel(
    const float2 *__restrict__ planes, int n_img, int h, int w,
    const int2 *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
    int n_vel, int k_cand, TileMap tiles, float *__restrict__ cand_nu,
    float *__restrict__ cand_alpha, int32_t *__restrict__ cand_vel,
    int16_t *__restrict__ cand_nobs) {
    constexpr int kLdsWords = (3 * PB > KM ? 3 * PB : KM) * 64;
    __shared__ uint32_t lds[kLdsWords];
    uint32_t *q_hi = lds;
    uint32_t *q_lo = lds + PB * 64;
    float *q_al = reinterpret_cast<float *>(lds + 2 * PB * 64);

    const int lane = (int)threadIdx.x;
    int row, seg;
    tiles.map(blockIdx.x, row, seg);
    const int x0 = seg * 64 + lane;
    const uint32_t row_bytes = (uint32_t)w * 8u;
    const size_t img_stride = (size_t)h * (size_t)w;

    uint64_t key[KM];
    float al[KM];
#pragma unroll
    for (int s = 0; s < KM; ++s) {
        key[s] = 0;
        al[s] = 0.f;
    }
    uint64_t thr = 0;   // admission threshold (list tail at the last merge)
    int nq = 0;         // queued candidates of this lane

    // Issue the loads of images [i0, i0 + NB) of visited velocity jj.  The
    // table row is fetched whole first (its padding entries lie outside the
    // frame); rows outside the frame get a zero-length buffer, so their loads
    // return 0 and add nothing, with no branch.
    const size_t img_bytes = img_stride * sizeof(float2);
    auto issue = [&](int jj, int i0, u32x2(&v)[NB]) {
        const int4 *t4 = reinterpret_cast<const int4 *>(disp + (size_t)jj * disp_stride + i0);
        int4 dd[NB / 2];
#pragma unroll
        for (int q = 0; q < NB / 2; ++q) dd[q] = t4[q];
        // Recomputed per velocity (not hoisted): keeps NB image bases out of
        // the scalar register file.
        const char *pbase = reinterpret_cast<const char *>(planes) + (size_t)i0 * img_bytes;
        asm volatile("" : "+s"(pbase));
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int dx = (b & 1) ? dd[b / 2].z : dd[b / 2].x;
            const int dy = (b & 1) ? dd[b / 2].w : dd[b / 2].y;
            const int yy = row + dy;
            const bool in_rows = (unsigned)yy < (unsigned)h;
            const char *rb = pbase + (size_t)b * img_bytes +
                             (size_t)(in_rows ? yy : 0) * (size_t)row_bytes;
            const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(in_rows ? rb : pbase,
                                                          in_rows ? row_bytes : 0u);
            v[b] = __builtin_amdgcn_raw_buffer_load_b64(rs, (x0 + dx) * 8, 0, 0);
        }
    };
    // Sum in image order.  Empty slots hold +0, which leaves every sum unchanged.
    auto accumulate = [&](const u32x2(&v)[NB], float &P, float &F) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            P += __uint_as_float(v[b].x);
            F += __uint_as_float(v[b].y);
        }
    };
    // n_obs: stored phi is nonzero exactly at valid pixels; empty slots are 0.
    auto count = [&](const u32x2(&v)[NB]) {
        uint32_t c = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) c += v[b].y != 0u;
        return c;
    };
    auto insert = [&](uint64_t nk, float a) {
#pragma unroll
        for (int s = 0; s < KM; ++s) {
            const bool c = nk > key[s];
            const uint64_t tk = c ? key[s] : nk;
            key[s] = c ? nk : key[s];
            nk = tk;
            const float ta = c ? al[s] : a;
            al[s] = c ? a : al[s];
            a = ta;
        }
    };
    auto merge_queue = [&]() {
        for (int b = 0; b < PB; ++b) {
            if (!__any(b < nq)) break;
            if (b < nq) {
                const uint64_t nk = ((uint64_t)q_hi[b * 64 + lane] << 32) | q_lo[b * 64 + lane];
                if (nk > key[KM - 1]) insert(nk, q_al[b * 64 + lane]);
            }
        }
        nq = 0;
        thr = key[KM - 1];
    };
    // Score one trajectory (Sec. 2.1.5: nu = Psi / sqrt(Phi), alpha = Psi / Phi)
    // and queue it if it beats the admission threshold.  n_obs only sits in
    // the low bits of the key and never decides an order, so it is counted
    // only for queued candidates.
    auto finish = [&](int j, float P, float F, uint32_t c) {
        const float nu = F > 0.f ? P / sqrtf(F) : -INFINITY;
        const uint64_t nk = make_key(nu, j, 0u);
        if (nk > thr) {
            q_hi[nq * 64 + lane] = (uint32_t)(nk >> 32);
            q_lo[nq * 64 + lane] = (uint32_t)nk | c;
            q_al[nq * 64 + lane] = F > 0.f ? P / F : 0.f;
            ++nq;
        }
        if (__any(nq == PB)) merge_queue();
    };

    if (n_img <= NB) {
        for (int jj = 0; jj < n_vel; ++jj) {
            const int j = vel_index[jj];   // fetched before the gathers are issued
            u32x2 v[NB];
            issue(jj, 0, v);
            float P = 0.f, F = 0.f;
            accumulate(v, P, F);
            finish(j, P, F, count(v));
        }
    } else {
        for (int jj = 0; jj < n_vel; ++jj) {
            const int j = vel_index[jj];
            float P = 0.f, F = 0.f;
            uint32_t c = 0;
            for (int i0 = 0; i0 < n_img; i0 += NB) {
                u32x2 v[NB];
                issue(jj, i0, v);
                accumulate(v, P, F);
                c += count(v);
            }
            finish(j, P, F, c);
        }
    }
    merge_queue();

    // Write the rank-ordered list: stage each field through LDS so that the
    // wave's stores cover the contiguous [pixels][k_cand] run of its pixels
    // (one pixel's k_cand <= 64 entries per store instruction).
    const int npx = (w - seg * 64) < 64 ? (w - seg * 64) : 64;
    const size_t base = ((size_t)row * (size_t)w + (size_t)seg * 64) * (size_t)k_cand;
    __syncthreads();
#pragma unroll
    for (int field = 0; field < 4; ++field) {
#pragma unroll
        for (int s = 0; s < KM; ++s) {
            const uint32_t hi = (uint32_t)(key[s] >> 32), lo = (uint32_t)key[s];
            uint32_t v;
            if (field == 0) v = __float_as_uint(nu_from_order_bits(hi));
            else if (field == 1) v = __float_as_uint(al[s]);
            else if (field == 2) v = (uint32_t)(0xFFFF - (int)(lo >> 16));
            else v = lo & 0xFFFFu;
            lds[lane * KM + s] = v;
        }
        __syncthreads();
        if (lane < k_cand) {
            for (int p = 0; p < npx; ++p) {
                const uint32_t v = lds[p * KM + lane];
                const size_t o = base + (size_t)p * (size_t)k_cand + (size_t)lane;
                if (field == 0) cand_nu[o] = __uint_as_float(v);
                else if (field == 1) cand_alpha[o] = __uint_as_float(v);
                else if (field == 2) cand_vel[o] = (int32_t)v;
                else cand_nobs[o] = (int16_t)v;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Final selection.  One wave handles 64 consecutive pixels: their candidate
// runs are loaded with coalesced reads into LDS, each lane checks that its
// pixel's candidates are in rank order (kb_search leaves them so), and the
// first k of every pixel are written back with coalesced stores.  A pixel
// whose candidates are not in order is ranked by counting, for each
// candidate, the candidates that precede it.
// ---------------------------------------------------------------------------
template <int KM>
__global__ __launch_bounds__(64) void topk_kernel(
    int64_t npix, int k_cand, int k, const float *__restrict__ cand_nu,
    const float *__restrict__ cand_alpha, const int32_t *__restrict__ cand_vel,
    const int16_t *__restrict__ cand_nobs, float *__restrict__ nu, float *__restrict__ alpha,
    int32_t *__restrict__ vel, int16_t *__restrict__ nobs) {
    __shared__ uint32_t s_nu[64 * KM], s_al[64 * KM], s_vel[64 * KM];
    __shared__ uint16_t s_no[64 * KM];
    __shared__ uint8_t s_rank[64 * KM];
    const int lane = (int)threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int npx = (npix - p0) < 64 ? (int)(npix - p0) : 64;
    const int total = npx * k_cand;
    const size_t ib = (size_t)p0 * (size_t)k_cand;
    for (int idx = lane; idx < total; idx += 64) {
        s_nu[idx] = __float_as_uint(cand_nu[ib + idx]);
        s_al[idx] = __float_as_uint(cand_alpha[ib + idx]);
        s_vel[idx] = (uint32_t)cand_vel[ib + idx];
        s_no[idx] = (uint16_t)cand_nobs[ib + idx];
    }
    __syncthreads();
    auto key_at = [&](int idx) {
        return make_key(__uint_as_float(s_nu[idx]), (int)s_vel[idx], s_no[idx]);
    };
    bool ordered = true;
    if (lane < npx) {
        const int o = lane * k_cand;
        uint64_t prev = key_at(o);
        for (int s = 1; s < k_cand; ++s) {
            const uint64_t cur = key_at(o + s);
            ordered = ordered && prev > cur;
            prev = cur;
        }
    }
    if (__all(ordered)) {
        for (int idx = lane; idx < total; idx += 64) s_rank[idx] = (uint8_t)(idx % k_cand);
    } else if (lane < npx) {
        const int o = lane * k_cand;
        for (int s = 0; s < k_cand; ++s) {
            const uint64_t ks = key_at(o + s);
            int r = 0;
            for (int t = 0; t < k_cand; ++t) r += key_at(o + t) > ks;
            s_rank[o + s] = (uint8_t)r;
        }
    }
    __syncthreads();
    // Scatter into the output by rank; entries ranked >= k are dropped.  The
    // writes of a wave cover the contiguous [npx][k] run.
    const size_t ob = (size_t)p0 * (size_t)k;
    for (int idx = lane; idx < total; idx += 64) {
        const int r = s_rank[idx];
        if (r < k) {
            const size_t o = ob + (size_t)(idx / k_cand) * (size_t)k + (size_t)r;
            nu[o] = __uint_as_float(s_nu[idx]);
            alpha[o] = __uint_as_float(s_al[idx]);
            vel[o] = (int32_t)s_vel[idx];
            nobs[o] = (int16_t)s_no[idx];
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers.
// ---------------------------------------------------------------------------
kb_status launch_status(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(KB_EDEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
    return KB_OK;
}

template <int KM, int NB>
kb_status launch_search_nb(const float2 *planes, int n_img, int h, int w, const int2 *disp,
                           const int32_t *vel_index, int n_vel, int k_cand, float *cn, float *ca,
                           int32_t *cv, int16_t *co, hipStream_t stream) {
    static_assert(NB == 8 || NB == 16, "table rows are padded for batches of 8 or 16");
    const int stride = (int)table_stride(n_img);
    constexpr int PB = KBMI_QUEUE;
    TileMap tm;
    tm.nseg = (w + 63) / 64;
    tm.h = h;
    tm.strip = tm.nseg < KBMI_STRIP_TILES ? tm.nseg : KBMI_STRIP_TILES;
    tm.nblocks = tm.nseg * h;
    hipLaunchKernelGGL((search_kernel<KM, NB, PB>), dim3(tm.nblocks), dim3(64), 0, stream,
                       planes, n_img, h, w, disp, stride, vel_index, n_vel, k_cand, tm, cn, ca,
                       cv, co);
    return launch_status("search_kernel");
}

template <int KM>
kb_status launch_search_km(const float2 *planes, int n_img, int h, int w, const int2 *disp,
                           const int32_t *vel_index, int n_vel, int k_cand, float *cn, float *ca,
                           int32_t *cv, int16_t *co, hipStream_t stream) {
    if (n_img <= 8)
        return launch_search_nb<KM, 8>(planes, n_img, h, w, disp, vel_index, n_vel, k_cand, cn,
                                       ca, cv, co, stream);
    return launch_search_nb<KM, 16>(planes, n_img, h, w, disp, vel_index, n_vel, k_cand, cn, ca,
                                    cv, co, stream);
}

template <int KM>
kb_status launch_topk_km(int64_t npix, int k_cand, int k, const float *cn, const float *ca,
                         const int32_t *cv, const int16_t *co, float *nu, float *al,
                         int32_t *vi, int16_t *no, hipStream_t stream) {
    const int64_t blocks = (npix + 63) / 64;
    hipLaunchKernelGGL((topk_kernel<KM>), dim3((unsigned)blocks), dim3(64), 0, stream, npix,
                       k_cand, k, cn, ca, cv, co, nu, al, vi, no);
    return launch_status("topk_kernel");
}

// List lengths compiled for the search: every even length up to KB_MAX_KCAND
// (each slot costs registers and compare-and-swap work on every insertion).
#define KB_SEARCH_KM_LIST(X)                                                              \
    X(2) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26) X(28) X(30) \
    X(32) X(34) X(36) X(38) X(40) X(42) X(44) X(46) X(48) X(50) X(52) X(54) X(56) X(58)  \
    X(60) X(62) X(64)

#define KB_DISPATCH_KM(kc, FN, ...)                  \
    ((kc) <= 8    ? FN<8>(__VA_ARGS__)               \
     : (kc) <= 16 ? FN<16>(__VA_ARGS__)              \
     : (kc) <= 24 ? FN<24>(__VA_ARGS__)              \
     : (kc) <= 32 ? FN<32>(__VA_ARGS__)              \
     : (kc) <= 40 ? FN<40>(__VA_ARGS__)              \
     : (kc) <= 48 ? FN<48>(__VA_ARGS__)              \
     : (kc) <= 56 ? FN<56>(__VA_ARGS__)              \
                  : FN<64>(__VA_ARGS__))

kb_status check_frame(int64_t n_img, int64_t h, int64_t w) {
    if (n_img < 1 || n_img > 32767)
        return fail(KB_EINVAL, "n_img must be in [1, 32767] (got %lld)", (long long)n_img);
    if (h < 1 || w < 1) return fail(KB_EINVAL, "h and w must be >= 1");
    if (w > (int64_t(1) << 27)) return fail(KB_EINVAL, "w must be <= 2^27");
    if (h > (int64_t(1) << 30)) return fail(KB_EINVAL, "h must be <= 2^30");
    const int64_t nseg = (w + 63) / 64;
    if (nseg * h > 2147483647LL) return fail(KB_EINVAL, "frame too large for one launch");
    return KB_OK;
}

// Copy the clamped displacement table into the workspace.  The host copy is
// pageable and temporary, so the call waits until it has reached the device.
kb_status upload_table(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
                       int64_t h, int64_t w, void *workspace, hipStream_t stream) {
    // Velocities in visiting order, then the table of the reordered grid.
    std::vector<int32_t> order(static_cast<size_t>(n_vel));
    velocity_order(vel, n_vel, order.data());
    std::vector<double> vel_visit(static_cast<size_t>(n_vel) * 2);
    for (int64_t j = 0; j < n_vel; ++j) {
        vel_visit[2 * j] = vel[2 * order[j]];
        vel_visit[2 * j + 1] = vel[2 * order[j] + 1];
    }
    std::vector<int32_t> dense(static_cast<size_t>(n_img) * n_vel * 2);
    displacement_table(t, n_img, vel_visit.data(), n_vel, dense.data(), w, h);
    // Pad each row to the stride with (0, h): row + h is outside the frame.
    const int64_t stride = table_stride(n_img);
    std::vector<int32_t> table(static_cast<size_t>(stride) * n_vel * 2);
    for (int64_t j = 0; j < n_vel; ++j)
        for (int64_t i = 0; i < stride; ++i) {
            const bool real = i < n_img;
            table[(j * stride + i) * 2] = real ? dense[(j * n_img + i) * 2] : 0;
            table[(j * stride + i) * 2 + 1] = real ? dense[(j * n_img + i) * 2 + 1] : (int32_t)h;
        }
    char *ws = static_cast<char *>(workspace);
    hipError_t e = hipMemcpyAsync(ws, table.data(), table.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + table_bytes(n_img, n_vel), order.data(),
                           order.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return fail(KB_EDEVICE, "displacement table upload failed: %s", hipGetErrorString(e));
    return KB_OK;
}

}  // namespace
}  // namespace kbmi

using namespace kbmi;

extern "C" {

kb_status kb_make_psi_phi(const float *img, const float *var, const uint8_t *mask,
                          int64_t n_img, int64_t h, int64_t w, const float *psf,
                          int64_t psf_h, int64_t psf_w, float *psi_phi, int32_t lp_dtype,
                          void *psi_phi_lp, float *lp_scale, void *stream) {
    clear_error();
    if (!img || !var || !psf || !psi_phi)
        return fail(KB_EINVAL, "img, var, psf and psi_phi must be non-null");
    kb_status st = check_frame(n_img, h, w);
    if (st != KB_OK) return st;
    if (psf_h < 1 || psf_w < 1 || psf_h % 2 == 0 || psf_w % 2 == 0)
        return fail(KB_EINVAL, "PSF sizes must be odd and >= 1 (got %lld x %lld)",
                    (long long)psf_h, (long long)psf_w);
    if (psf_h > KB_MAX_PSF || psf_w > KB_MAX_PSF)
        return fail(KB_EUNSUPPORTED, "PSF sides above %d are not supported", KB_MAX_PSF);
    if (n_img > 65535 || (h + PP_TH - 1) / PP_TH > 65535)
        return fail(KB_EUNSUPPORTED, "frame or stack too large for one plane launch");
    if (lp_dtype != KB_F32) {
        if (lp_dtype != KB_F16 && lp_dtype != KB_BF16)
            return fail(KB_EINVAL, "lp_dtype must be KB_F32, KB_F16 or KB_BF16");
        return fail(KB_EUNSUPPORTED, "16-bit plane copies are not implemented in this build");
    }
    (void)psi_phi_lp;
    (void)lp_scale;
    PsfTaps taps{};
    for (int64_t u = 0; u < psf_h * psf_w; ++u) taps.t[u] = psf[u];
    const dim3 grid((unsigned)((w + PP_TW - 1) / PP_TW), (unsigned)((h + PP_TH - 1) / PP_TH),
                    (unsigned)n_img);
    hipLaunchKernelGGL(psi_phi_kernel, grid, dim3(PP_THREADS), 0, (hipStream_t)stream, img, var,
                       mask, (int)h, (int)w, (int)psf_h, (int)psf_w, taps,
                       reinterpret_cast<float2 *>(psi_phi));
    return launch_status("psi_phi_kernel");
}

kb_status kb_search(const void *planes, int32_t dtype, const float *lp_scale, int64_t n_img,
                    int64_t h, int64_t w, const double *t, const double *vel, int64_t n_vel,
                    int64_t k_cand, float *cand_nu, float *cand_alpha, int32_t *cand_vel,
                    int16_t *cand_nobs, void *workspace, size_t workspace_bytes,
                    void *stream) {
    clear_error();
    if (!planes || !cand_nu || !cand_alpha || !cand_vel || !cand_nobs)
        return fail(KB_EINVAL, "planes and candidate outputs must be non-null");
    kb_status st = check_frame(n_img, h, w);
    if (st != KB_OK) return st;
    if (n_vel < 1 || n_vel > 65535)
        return fail(KB_EINVAL, "n_vel must be in [1, 65535] (got %lld)", (long long)n_vel);
    if (k_cand < 1 || k_cand > n_vel)
        return fail(KB_EINVAL, "k_cand must be in [1, n_vel] (got %lld)", (long long)k_cand);
    if (k_cand > KB_MAX_KCAND)
        return fail(KB_EUNSUPPORTED, "k_cand above %d is not supported", KB_MAX_KCAND);
    st = check_times_velocities(t, n_img, vel, n_vel);
    if (st != KB_OK) return st;
    if (dtype != KB_F32) {
        if (dtype != KB_F16 && dtype != KB_BF16)
            return fail(KB_EINVAL, "dtype must be KB_F32, KB_F16 or KB_BF16");
        return fail(KB_EUNSUPPORTED, "16-bit planes are not implemented in this build");
    }
    (void)lp_scale;
    if (!workspace) return fail(KB_EINVAL, "workspace must be non-null");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KB_EINVAL, "workspace must be 256-byte aligned");
    const size_t ws_need = table_bytes(n_img, n_vel) + order_bytes(n_vel);
    if (workspace_bytes < ws_need)
        return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", ws_need, workspace_bytes);
    hipStream_t s = (hipStream_t)stream;
    st = upload_table(t, n_img, vel, n_vel, h, w, workspace, s);
    if (st != KB_OK) return st;
    const int kc = (int)k_cand;
    const int32_t *vel_index = reinterpret_cast<const int32_t *>(
        static_cast<const char *>(workspace) + table_bytes(n_img, n_vel));
    const int km = (kc + 1) & ~1;
    switch (km) {
#define KB_SEARCH_CASE(K)                                                                      \
    case K:                                                                                    \
        return launch_search_km<K>(reinterpret_cast<const float2 *>(planes), (int)n_img, (int)h, \
                                   (int)w, reinterpret_cast<const int2 *>(workspace), vel_index, \
                                   (int)n_vel, kc, cand_nu, cand_alpha, cand_vel, cand_nobs, s);
        KB_SEARCH_KM_LIST(KB_SEARCH_CASE)
#undef KB_SEARCH_CASE
    }
    return fail(KB_EUNSUPPORTED, "k_cand above %d is not supported", KB_MAX_KCAND);
}

kb_status kb_topk(const float *psi_phi_f32, int64_t n_img, int64_t h, int64_t w,
                  const double *t, const double *vel, int64_t n_vel, const float *cand_nu,
                  const float *cand_alpha, const int32_t *cand_vel, const int16_t *cand_nobs,
                  int64_t k_cand, int64_t k, float *nu, float *alpha, int32_t *vel_idx,
                  int16_t *nobs, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!cand_nu || !cand_alpha || !cand_vel || !cand_nobs || !nu || !alpha || !vel_idx || !nobs)
        return fail(KB_EINVAL, "candidate inputs and outputs must be non-null");
    kb_status st = check_frame(n_img, h, w);
    if (st != KB_OK) return st;
    if (k_cand < 1 || k < 1 || k > k_cand)
        return fail(KB_EINVAL, "need 1 <= k <= k_cand (got k=%lld, k_cand=%lld)", (long long)k,
                    (long long)k_cand);
    if (k_cand > KB_MAX_KCAND)
        return fail(KB_EUNSUPPORTED, "k_cand above %d is not supported", KB_MAX_KCAND);
    if (psi_phi_f32 != nullptr)
        return fail(KB_EUNSUPPORTED, "re-scoring is not implemented in this build");
    (void)t;
    (void)vel;
    (void)n_vel;
    (void)workspace;
    (void)workspace_bytes;
    const int64_t npix = h * w;
    if ((npix + 63) / 64 > 2147483647LL) return fail(KB_EINVAL, "frame too large");
    const int kc = (int)k_cand;
    return KB_DISPATCH_KM(kc, launch_topk_km, npix, kc, (int)k, cand_nu, cand_alpha, cand_vel,
                          cand_nobs, nu, alpha, vel_idx, nobs, (hipStream_t)stream);
}

}  // extern "C"
