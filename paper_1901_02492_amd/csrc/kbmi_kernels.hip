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

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "kbmi_common.h"
#include "kbmi_device.h"
#include "kbmi_group.h"


namespace kbmi {

kb_status launch_status(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(KB_EDEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
    return KB_OK;
}

namespace {

// ---------------------------------------------------------------------------
// Likelihood images.
// ---------------------------------------------------------------------------
struct PsfTaps {
    float t[KB_MAX_PSF * KB_MAX_PSF];
};

constexpr int PP_TW = 64;       // output tile width
constexpr int PP_TH = 16;       // output tile height
constexpr int PP_THREADS = 256; // 4 waves; each thread produces 4 columns of one row
// LDS of one tile with its halo for a PSF of ph rows and PW columns: the
// (a, w) pairs, then the validity bytes (sized at launch, so a small PSF
// leaves room for more resident workgroups).
template <int PW>
constexpr size_t psi_phi_lds_bytes(int ph) {
    return (size_t)(PP_TH + ph - 1) * (size_t)(PP_TW + PW - 1) * (sizeof(float2) + 1);
}

// psi = a (x) T and phi = w (x) T^2 (cross-correlations with zero padding) for
// one 64 x 16 output tile of one image, with a = valid * img / var and
// w = valid / var staged in LDS for the tile plus its halo as interleaved
// pairs.  The PSF width PW is a compile-time constant: each thread computes 4
// adjacent columns of one output row and, per PSF row, reads the
// (4 + PW - 1)-pixel segment it needs once (16-byte LDS reads), so one LDS
// read serves about three FMAs.  Per output the taps are summed row by row,
// left to right.
template <int PW>
__global__ __launch_bounds__(PP_THREADS) void psi_phi_kernel(
    const float *__restrict__ img, const float *__restrict__ var,
    const uint8_t *__restrict__ mask, int h, int w, int ph, PsfTaps psf,
    float2 *__restrict__ out, uint32_t *__restrict__ maxabs) {
    constexpr int LW = PP_TW + PW - 1;        // staged columns (even: PW is odd)
    constexpr int SEG = 4 + PW - 1;           // pixels one thread reads per PSF row
    static_assert(PW % 2 == 1 && LW % 2 == 0 && SEG % 2 == 0, "odd PSF widths only");
    extern __shared__ __align__(16) unsigned char pp_lds[];
    float2 *s_aw = reinterpret_cast<float2 *>(pp_lds);
    uint8_t *s_ok = pp_lds + (size_t)(PP_TH + ph - 1) * LW * sizeof(float2);

    const int i = blockIdx.z;
    const int tx0 = blockIdx.x * PP_TW;
    const int ty0 = blockIdx.y * PP_TH;
    const int cy = ph / 2, cx = PW / 2;
    const int lh = PP_TH + ph - 1;
    const size_t plane = (size_t)i * (size_t)h * (size_t)w;

    for (int idx = threadIdx.x; idx < lh * LW; idx += PP_THREADS) {
        const int ly = idx / LW, lx = idx - ly * LW;
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
        s_aw[idx] = make_float2(a, wt);
        s_ok[idx] = ok;
    }
    __syncthreads();

    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    float ps[4] = {0.f, 0.f, 0.f, 0.f}, pf[4] = {0.f, 0.f, 0.f, 0.f};
    for (int u = 0; u < ph; ++u) {
        const float4 *row = reinterpret_cast<const float4 *>(s_aw + (ty + u) * LW + 4 * tx);
        float2 seg[SEG];
#pragma unroll
        for (int q = 0; q < SEG / 2; ++q) {
            const float4 x = row[q];
            seg[2 * q] = make_float2(x.x, x.y);
            seg[2 * q + 1] = make_float2(x.z, x.w);
        }
#pragma unroll
        for (int v = 0; v < PW; ++v) {
            const float tv = psf.t[u * PW + v];
            const float t2 = tv * tv;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ps[c] = fmaf(seg[c + v].x, tv, ps[c]);
                pf[c] = fmaf(seg[c + v].y, t2, pf[c]);
            }
        }
    }
    const int gy = ty0 + ty;
    float mp = 0.f, mf = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int gx = tx0 + 4 * tx + c;
        if (gy < h && gx < w) {
            float2 res = make_float2(0.f, 0.f);
            if (s_ok[(ty + cy) * LW + 4 * tx + c + cx]) {
                // phi >= 0 always; a valid pixel keeps a nonzero bit pattern.
                res = make_float2(ps[c], pf[c] > 0.f ? pf[c] : -0.0f);
                mp = fmaxf(mp, fabsf(ps[c]));
                mf = fmaxf(mf, pf[c]);
            }
            out[plane + (size_t)gy * w + gx] = res;
        }
    }
    if (maxabs != nullptr) {
        __shared__ float s_red[2][PP_THREADS / 64];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            mp = fmaxf(mp, __shfl_xor(mp, off));
            mf = fmaxf(mf, __shfl_xor(mf, off));
        }
        if ((threadIdx.x & 63) == 0) {
            s_red[0][threadIdx.x / 64] = mp;
            s_red[1][threadIdx.x / 64] = mf;
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            float m = 0.f;
#pragma unroll
            for (int q = 0; q < PP_THREADS / 64; ++q) m = fmaxf(m, s_red[threadIdx.x][q]);
            atomicMax(&maxabs[2 * i + threadIdx.x], __float_as_uint(m));
        }
    }
}

// ---------------------------------------------------------------------------
// 16-bit plane copies.  Per image and plane the scale is the power of two s
// with max|value| * s in [2^13, 2^14): the scaled values keep FP16's full
// precision and stay far below its overflow.  Stored value = RNE(value * s);
// a valid pixel whose scaled phi rounds to +0 stores -0 so that the phi bits
// stay nonzero exactly at valid pixels.  The search multiplies by 1/s, which
// is exact.
// ---------------------------------------------------------------------------
__global__ void lp_zero_kernel(uint32_t *__restrict__ maxabs, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) maxabs[t] = 0u;
}

__global__ void lp_scale_kernel(float *__restrict__ scale, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const float m = scale[t];   // max |value| (stored through its bit pattern)
        float sc = 1.f;
        if (m > 0.f && isfinite(m)) {
            int e;
            frexpf(m, &e);                       // m = f * 2^e, f in [0.5, 1)
            int x = 14 - e;
            x = x < -126 ? -126 : (x > 127 ? 127 : x);
            sc = ldexpf(1.f, x);
        }
        scale[t] = sc;
    }
}

__device__ inline uint16_t to_lp(float v, int fmt) {
    if (fmt == KB_F16) {
        const _Float16 hv = (_Float16)v;            // round to nearest even
        return __builtin_bit_cast(uint16_t, hv);
    }
    // bfloat16, round to nearest even (inputs are finite)
    const uint32_t u = __float_as_uint(v);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ __launch_bounds__(256) void lp_convert_kernel(
    const float2 *__restrict__ planes, size_t npix_img, const float *__restrict__ scale, int fmt,
    uint32_t *__restrict__ out) {
    const int i = blockIdx.y;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < npix_img;
         q += (size_t)gridDim.x * blockDim.x) {
        const size_t e = (size_t)i * npix_img + q;
        const float2 v = planes[e];
        const uint32_t fbits = __float_as_uint(v.y);
        uint32_t packed = 0u;
        if (fbits != 0u) {                            // valid pixel
            const uint16_t hp = to_lp(v.x * scale[2 * i], fmt);
            uint16_t hf = to_lp(v.y * scale[2 * i + 1], fmt);
            if ((hf & 0x7FFFu) == 0u) hf = 0x8000u;   // keep the validity bit pattern
            packed = (uint32_t)hp | ((uint32_t)hf << 16);
        }
        out[e] = packed;
    }
}

// ---------------------------------------------------------------------------
// Final selection.  One thread per candidate: a 256-thread block holds whole
// pixels (256 / k_cand of them), reads their candidates' nu and velocity
// index with coalesced loads, and each thread checks that its candidate
// precedes the next one of the same pixel.  The order is (nu descending,
// velocity index ascending); n_obs and alpha never decide it, so they are
// read only by blocks that write.  When every pixel of the block is in rank
// order (kb_search leaves them so) the first k of each are copied out;
// otherwise each candidate's rank is the number of candidates of its pixel
// that precede it (equal keys, which only a repeated velocity gives, in list
// order).  In place (outputs are the candidate arrays, k == k_cand) an
// ordered block reads nothing more and writes nothing; an unordered one
// loads all its entries before the barrier that precedes its writes.  A
// workgroup takes TK_G groups of pixels with all their loads in flight at
// once (one group per workgroup is bound by workgroup dispatch).
// ---------------------------------------------------------------------------
constexpr int TK_THREADS = 256;
constexpr int TK_G = 4;

__global__ __launch_bounds__(TK_THREADS) void topk_kernel(
    int64_t npix, int k_cand, int k, bool in_place, const float *cand_nu,
    const float *cand_alpha, const int32_t *cand_vel, const int16_t *cand_nobs, float *nu,
    float *alpha, int32_t *vel, int16_t *nobs) {
    __shared__ uint64_t s_key[TK_G][TK_THREADS];
    const int ppb = TK_THREADS / k_cand;
    const int t = (int)threadIdx.x;
    const int lp = t / k_cand, s = t - lp * k_cand;
    int64_t p[TK_G];
    bool active[TK_G];
    size_t e[TK_G];
    float v_nu[TK_G];
    int32_t v_vel[TK_G];
    uint64_t key[TK_G];
#pragma unroll
    for (int g = 0; g < TK_G; ++g) {
        p[g] = ((int64_t)blockIdx.x * TK_G + g) * ppb + lp;
        active[g] = lp < ppb && p[g] < npix;
        e[g] = (size_t)p[g] * (size_t)k_cand + (size_t)s;
        v_nu[g] = active[g] ? cand_nu[e[g]] : 0.f;
        v_vel[g] = active[g] ? cand_vel[e[g]] : 0;
    }
#pragma unroll
    for (int g = 0; g < TK_G; ++g) {
        key[g] = active[g] ? make_key(v_nu[g], v_vel[g], 0u) : 0ull;
        s_key[g][t] = key[g];
    }
    __syncthreads();
    bool out_of_order = false;
#pragma unroll
    for (int g = 0; g < TK_G; ++g)
        out_of_order |= active[g] && s + 1 < k_cand && !(key[g] > s_key[g][t + 1]);
    const bool reorder = __syncthreads_or(out_of_order);
    if (!reorder && in_place) return;
    float v_al[TK_G];
    int16_t v_no[TK_G];
#pragma unroll
    for (int g = 0; g < TK_G; ++g) {
        v_al[g] = active[g] ? cand_alpha[e[g]] : 0.f;
        v_no[g] = active[g] ? cand_nobs[e[g]] : (int16_t)0;
    }
    int rank[TK_G];
#pragma unroll
    for (int g = 0; g < TK_G; ++g) {
        rank[g] = s;
        if (reorder) {
            rank[g] = 0;
            const uint64_t *pk = s_key[g] + lp * k_cand;
            for (int r = 0; r < k_cand; ++r)
                rank[g] += (pk[r] > key[g]) | ((pk[r] == key[g]) & (r < s));
        }
    }
    if (reorder && in_place) __syncthreads();   // every entry of the block is read
#pragma unroll
    for (int g = 0; g < TK_G; ++g)
        if (active[g] && rank[g] < k) {
            const size_t o = (size_t)p[g] * (size_t)k + (size_t)rank[g];
            nu[o] = v_nu[g];
            alpha[o] = v_al[g];
            vel[o] = v_vel[g];
            nobs[o] = v_no[g];
        }
}

// ---------------------------------------------------------------------------
// Re-scoring selection (after a 16-bit search): every candidate's Psi, Phi and
// n_obs are recomputed from the float32 planes with exactly the arithmetic of
// the float32 search (image order, out-of-frame terms adding +0, the same
// score expressions), so a re-scored entry is bitwise the plain path's value
// for that trajectory.  Then every pixel's candidates are ranked by counting.
//
// A workgroup owns RS_PX consecutive start pixels and their RS_PX * k_cand
// (pixel, velocity) pairs.  Gathering the pairs in list order would give each
// lane of a load its own cache line (the lanes of a wave hold different
// velocities of one or two pixels).  Instead the pairs are first grouped by
// velocity with a counting sort in LDS (velocity ranges of n_vel / 1024 when
// there are more than 1024 velocities), so adjacent lanes mostly share a
// velocity and read adjacent pixels of one row: a few cache lines per load
// instead of 64.  The order only changes which lane computes a pair, not its
// arithmetic.  Results go to LDS by pair, and the ranking reads them in list
// order.
// ---------------------------------------------------------------------------
// Start pixels per re-score workgroup (32: half the LDS, more workgroups per
// CU, each XCD's concurrent tiles over twice the rows; measured 36.3 ms
// against 35.5 ms at 64 for the survey stack's FP16 candidates).
#ifndef KBMI_RS_PX
#define KBMI_RS_PX 64
#endif
constexpr int RS_PX = KBMI_RS_PX;                           // start pixels per workgroup
constexpr int RS_MAXQ = RS_PX * KB_MAX_KCAND / TK_THREADS;  // pairs per thread, at most
static_assert(TK_THREADS == GR_THREADS, "the re-score groups its pairs by velocity");

size_t rescore_lds_bytes(int k_cand) {
    const size_t np = (size_t)RS_PX * (size_t)k_cand;
    return np * 8 + np * 4 + ((np * 2 + 7) & ~(size_t)7) + group_lds_bytes();
}

__global__ __launch_bounds__(TK_THREADS) void topk_rescore_kernel(
    int h, int w, int row0, int n_rows, int n_img, const float2 *__restrict__ planes,
    const double *__restrict__ tau, const double2 *__restrict__ vels, int n_vel, int k_cand,
    int k, const int32_t *__restrict__ cand_vel, float *__restrict__ nu,
    float *__restrict__ alpha, int32_t *__restrict__ vel, int16_t *__restrict__ nobs) {
    extern __shared__ __align__(16) unsigned char rs_lds[];
    const int np_max = RS_PX * k_cand;
    uint64_t *s_key = reinterpret_cast<uint64_t *>(rs_lds);
    // s_al holds each pair's velocity index until the pair is scored (by the
    // one thread that then writes its alpha there).
    float *s_al = reinterpret_cast<float *>(rs_lds + (size_t)np_max * 8);
    int32_t *s_vj = reinterpret_cast<int32_t *>(s_al);
    uint16_t *s_ord = reinterpret_cast<uint16_t *>(rs_lds + (size_t)np_max * 12);
    uint32_t *s_bin = reinterpret_cast<uint32_t *>(
        rs_lds + (size_t)np_max * 12 + (((size_t)np_max * 2 + 7) & ~(size_t)7));
    uint32_t *s_tot = s_bin + GR_BINS;

    // Tiles are RS_PX pixels of one row (the last of a row may be shorter).
    // Workgroups reach the 8 XCDs round-robin, and XCD x walks down tile
    // columns x, x + 8, ...: at any time the eight XCDs sweep eight adjacent
    // columns at about the same rows, and the concurrent tiles of one XCD
    // (about a hundred rows of one column) read overlapping pieces of the
    // same plane rows through its L2.
    const int n_ct = (w + RS_PX - 1) / RS_PX;
    const int64_t kb = (int64_t)(blockIdx.x >> 3);
    const int64_t ct64 = 8 * (kb / n_rows) + (int64_t)(blockIdx.x & 7u);
    if (ct64 >= n_ct) return;
    const int64_t row = row0 + kb % n_rows;
    const int ct = (int)ct64;
    const int64_t p0 = row * w + (int64_t)ct * RS_PX;
    const int npx = min(RS_PX, w - ct * RS_PX);
    const int np = npx * k_cand;
    const int t = (int)threadIdx.x;
    const int32_t *cv = cand_vel + p0 * (int64_t)k_cand;

    // Group the pairs by velocity.  A candidate index outside the grid (not
    // written by kb_search) is dropped: key 0 ranks below every scored one.
    const int n_sorted =
        group_pairs_by_velocity<RS_MAXQ>(cv, np, n_vel, s_vj, s_ord, s_bin, s_tot);
    for (int q = t; q < np; q += TK_THREADS)
        if (s_vj[q] < 0) s_key[q] = 0ull;

    // Score the pairs in velocity-grouped order.
    for (int pos = t; pos < n_sorted; pos += TK_THREADS) {
        const int q = s_ord[pos];
        const int j = s_vj[q];
        const int lp = q / k_cand;
        const int64_t p = p0 + lp;
        const int y0 = (int)(p / w), x0 = (int)(p - (int64_t)y0 * w);
        const double2 vj = vels[j];
        float P = 0.f, F = 0.f;
        uint32_t c = 0;
        for (int i0 = 0; i0 < n_img; i0 += 8) {
            float2 v[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int i = i0 + b;
                const double ti = tau[i < n_img ? i : 0];
                const int y = y0 + displacement(vj.y, ti, h), x = x0 + displacement(vj.x, ti, w);
                const bool ok = i < n_img && (unsigned)y < (unsigned)h && (unsigned)x < (unsigned)w;
                const size_t idx = ok ? ((size_t)i * h + y) * (size_t)w + x : 0;
                const float2 raw = planes[idx];
                v[b] = ok ? raw : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                P += v[b].x;
                F += v[b].y;
                c += __float_as_uint(v[b].y) != 0u;
            }
        }
        const float r = inv_sqrt_phi(F);
        const float v_nu = score_nu(P, F, r);
        s_key[q] = make_key(v_nu, j, c);
        s_al[q] = score_alpha(P, v_nu, F, r);
    }
    __syncthreads();

    // Rank every pair among its pixel's candidates: keys above it, then equal
    // keys (only unscored ones can be equal) earlier in the list.
#pragma unroll
    for (int r = 0; r < RS_MAXQ; ++r) {
        const int q = t + r * TK_THREADS;
        if (q < np) {
            const int lp = q / k_cand, s = q - lp * k_cand;
            const uint64_t key = s_key[q];
            const uint64_t *pk = s_key + lp * k_cand;
            int rank = 0;
            for (int u = 0; u < k_cand; ++u) {
                const uint64_t o = pk[u];
                rank += (o > key) | ((o == key) & (u < s));
            }
            if (rank < k) {
                const int64_t o = (p0 + lp) * (int64_t)k + rank;
                const bool scored = key != 0ull;
                nu[o] = scored ? key_nu(key) : -INFINITY;
                alpha[o] = scored ? s_al[q] : 0.f;
                vel[o] = scored ? key_vel(key) : cv[q];
                nobs[o] = (int16_t)(scored ? key_nobs(key) : 0);
            }
        }
    }
}

// Bright-pixel mask (Sec. 5.2): mask[p] |= img[p] > threshold, per image.
// Sixteen pixels per thread with 16-byte loads and stores where both arrays
// are 16-byte aligned; the rest one by one.
__global__ void mask_bright_kernel(const float *__restrict__ img, uint8_t *__restrict__ mask,
                                   int64_t n16, float thr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n16; g += stride) {
        const float4 *src = reinterpret_cast<const float4 *>(img) + 4 * g;
        const auto bits = [thr](const float4 v) {
            return (v.x > thr ? 1u : 0u) | (v.y > thr ? 1u << 8 : 0u) |
                   (v.z > thr ? 1u << 16 : 0u) | (v.w > thr ? 1u << 24 : 0u);
        };
        uint4 m = reinterpret_cast<const uint4 *>(mask)[g];
        m.x |= bits(src[0]);
        m.y |= bits(src[1]);
        m.z |= bits(src[2]);
        m.w |= bits(src[3]);
        reinterpret_cast<uint4 *>(mask)[g] = m;
    }
}

__global__ void mask_bright_tail_kernel(const float *__restrict__ img,
                                        uint8_t *__restrict__ mask, int64_t begin, int64_t end,
                                        float thr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < end; p += stride)
        if (img[p] > thr) mask[p] = (uint8_t)(mask[p] | 1u);
}

// ---------------------------------------------------------------------------
// Host-side launch helpers.
// ---------------------------------------------------------------------------

// 1/s per image and plane for the 16-bit search, padded with 0 to the table
// stride (padding images then contribute exactly 0).
__global__ void inv_scale_kernel(const float *__restrict__ scale, int n_img, int stride,
                                 float2 *__restrict__ inv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < stride)
        inv[i] = i < n_img ? make_float2(1.0f / scale[2 * i], 1.0f / scale[2 * i + 1])
                           : make_float2(0.f, 0.f);
}

kb_status launch_topk_rescore(int h, int w, int n_img, const float2 *planes, const double *tau,
                              const double2 *vels, int n_vel, int k_cand, int k,
                              const int32_t *cv, float *nu, float *al, int32_t *vi, int16_t *no,
                              hipStream_t stream) {
    // Eight workgroups per row for each group of eight tile columns; rows in
    // launches of at most 2^31 - 1 workgroups.
    const int64_t n_ct = ((int64_t)w + RS_PX - 1) / RS_PX;
    const int64_t per_row = 8 * ((n_ct + 7) / 8);
    const int64_t max_rows = 2147483647LL / per_row;
    for (int64_t r0 = 0; r0 < h; r0 += max_rows) {
        const int n_rows = (int)std::min<int64_t>(max_rows, h - r0);
        hipLaunchKernelGGL(topk_rescore_kernel, dim3((unsigned)(per_row * n_rows)),
                           dim3(TK_THREADS), rescore_lds_bytes(k_cand), stream, h, w, (int)r0,
                           n_rows, n_img, planes, tau, vels, n_vel, k_cand, k, cv, nu, al, vi,
                           no);
        const kb_status st = launch_status("topk_rescore_kernel");
        if (st != KB_OK) return st;
    }
    return KB_OK;
}

kb_status launch_topk(int64_t npix, int k_cand, int k, bool in_place, const float *cn,
                      const float *ca, const int32_t *cv, const int16_t *co, float *nu,
                      float *al, int32_t *vi, int16_t *no, hipStream_t stream) {
    const int64_t ppb = TK_THREADS / k_cand;
    const int64_t groups = (npix + ppb - 1) / ppb;
    const int64_t blocks = (groups + TK_G - 1) / TK_G;
    hipLaunchKernelGGL(topk_kernel, dim3((unsigned)blocks), dim3(TK_THREADS), 0, stream, npix,
                       k_cand, k, in_place, cn, ca, cv, co, nu, al, vi, no);
    return launch_status("topk_kernel");
}

}  // namespace

kb_status check_search_args(const void *planes, int32_t dtype, const float *lp_scale,
                            int64_t n_img, int64_t h, int64_t w, const double *t,
                            const double *vel, int64_t n_vel, int64_t k_cand,
                            const void *cand_nu, const void *cand_alpha, const void *cand_vel,
                            const void *cand_nobs) {
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
    if (dtype != KB_F32 && dtype != KB_F16 && dtype != KB_BF16)
        return fail(KB_EINVAL, "dtype must be KB_F32, KB_F16 or KB_BF16");
    if (dtype != KB_F32 && !lp_scale) return fail(KB_EINVAL, "16-bit planes need lp_scale");
    return KB_OK;
}

kb_status launch_search_in(const void *planes, int32_t dtype, const float *lp_scale,
                           int64_t n_img, int64_t h, int64_t w, int64_t n_vel, int64_t k_cand,
                           float *cand_nu, float *cand_alpha, int32_t *cand_vel,
                           int16_t *cand_nobs, void *workspace, const int32_t dy_range[2],
                           hipStream_t s) {
    char *wsb = static_cast<char *>(workspace);
    const WorkspaceLayout lay = workspace_layout(n_img, h, w, n_vel);
    StackView sv;
    sv.planes = planes;
    sv.inv_scale = reinterpret_cast<const float2 *>(wsb + lay.inv_scale);
    sv.n_img = (int)n_img;
    sv.h = (int)h;
    sv.w = (int)w;
    sv.disp = reinterpret_cast<const GatherEntry *>(wsb + lay.table);
    sv.disp_stride = (int)table_stride(n_img);
    sv.vel_index = reinterpret_cast<const int32_t *>(wsb + lay.order);
    sv.n_vel = (int)n_vel;
    sv.k_cand = (int)k_cand;
    sv.cand_nu = cand_nu;
    sv.cand_alpha = cand_alpha;
    sv.cand_vel = cand_vel;
    sv.cand_nobs = cand_nobs;
    sv.sync = reinterpret_cast<uint32_t *>(wsb + lay.sync);
    // Start rows whose displaced rows are inside the frame for every image and
    // velocity: their gathers need no row check.
    sv.row_lo = (int)std::min<int64_t>(h, -(int64_t)dy_range[0]);
    sv.row_hi = (int)std::max<int64_t>(0, h - (int64_t)dy_range[1]);
    if (dtype != KB_F32) {
        const int stride = (int)table_stride(n_img);
        hipLaunchKernelGGL(inv_scale_kernel, dim3((stride + 63) / 64), dim3(64), 0, s, lp_scale,
                           (int)n_img, stride, const_cast<float2 *>(sv.inv_scale));
        const kb_status st = launch_status("inv_scale_kernel");
        if (st != KB_OK) return st;
    }
    return launch_search(dtype, km_for((int)k_cand), sv, s);
}

// Dispatch to the translation unit of (plane format, list-length group).
kb_status launch_search(int fmt, int km, const StackView &v, hipStream_t s) {
    if (km_index(km) < 0)
        return fail(KB_EUNSUPPORTED, "no search compiled for list length %d", km);
    switch (fmt * kKmGroups + km_group(km)) {
#define KB_GROUP(F, G)                                \
    case F * kKmGroups + G:                           \
        return launch_search_group<F, G>(km, v, s);
#define KB_FMT(F)                                                                    \
    KB_GROUP(F, 0) KB_GROUP(F, 1) KB_GROUP(F, 2) KB_GROUP(F, 3) KB_GROUP(F, 4)       \
    KB_GROUP(F, 5) KB_GROUP(F, 6) KB_GROUP(F, 7)
        KB_FMT(0) KB_FMT(1) KB_FMT(2)
#undef KB_FMT
#undef KB_GROUP
    }
    return fail(KB_EUNSUPPORTED, "no search compiled for format %d, list length %d", fmt, km);
}

kb_status launch_search_batch(int fmt, int km, const BatchJob *jobs, int n_jobs,
                              int n_img_class, int k_cand, int generations, uint32_t *sync,
                              int *grid, hipStream_t s) {
    if (km_index(km) < 0)
        return fail(KB_EUNSUPPORTED, "no batched search compiled for list length %d", km);
    switch (fmt * kKmGroups + km_group(km)) {
#define KB_GROUP(F, G)                                                                      \
    case F * kKmGroups + G:                                                                 \
        return launch_search_batch_group<F, G>(km, jobs, n_jobs, n_img_class, k_cand,      \
                                               generations, sync, grid, s);
#define KB_FMT(F)                                                                    \
    KB_GROUP(F, 0) KB_GROUP(F, 1) KB_GROUP(F, 2) KB_GROUP(F, 3) KB_GROUP(F, 4)       \
    KB_GROUP(F, 5) KB_GROUP(F, 6) KB_GROUP(F, 7)
        KB_FMT(0) KB_FMT(1) KB_FMT(2)
#undef KB_FMT
#undef KB_GROUP
    }
    return fail(KB_EUNSUPPORTED, "no batched search compiled for format %d, list length %d",
                fmt, km);
}

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

// ---------------------------------------------------------------------------
// Host staging of table uploads.  Each upload is copied into a pinned host
// buffer, sent with an asynchronous copy on the caller's stream, and followed
// by an event; a buffer is reused once its event has completed.  Calls thus
// return without waiting for their stream.  Buffers are kept per device (at
// most kStagingPerDevice; beyond that a call waits for one of them) until the
// process ends.
// ---------------------------------------------------------------------------
namespace {
struct StagingBuffer {
    void *host;
    size_t cap;
    hipEvent_t done;
    int device;
};
constexpr int kStagingPerDevice = 32;
std::mutex g_staging_mu;
std::vector<StagingBuffer *> g_staging;
}  // namespace

kb_status staged_copy(void *dst, const void *src, size_t bytes, hipStream_t stream) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(KB_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_staging_mu);
    StagingBuffer *b = nullptr;
    int owned = 0;
    for (StagingBuffer *x : g_staging) {
        if (x->device != dev) continue;
        ++owned;
        if (!b && x->cap >= bytes && hipEventQuery(x->done) == hipSuccess) b = x;
    }
    if (!b && owned >= kStagingPerDevice) {
        // Wait for this device's first buffer and resize it if needed.
        for (StagingBuffer *x : g_staging)
            if (x->device == dev) {
                b = x;
                break;
            }
        e = hipEventSynchronize(b->done);
        if (e == hipSuccess && b->cap < bytes) {
            e = hipHostFree(b->host);
            b->host = nullptr;
            b->cap = 0;
            if (e == hipSuccess) e = hipHostMalloc(&b->host, bytes, hipHostMallocDefault);
            if (e == hipSuccess) b->cap = bytes;
        }
        if (e != hipSuccess)
            return fail(KB_EDEVICE, "staging buffer: %s", hipGetErrorString(e));
    }
    if (!b) {
        b = new StagingBuffer{nullptr, 0, nullptr, dev};
        const size_t cap = std::max(bytes, static_cast<size_t>(1) << 16);
        e = hipHostMalloc(&b->host, cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (b->host) (void)hipHostFree(b->host);
            delete b;
            return fail(KB_ENOMEM, "pinned staging buffer of %zu bytes: %s", cap,
                        hipGetErrorString(e));
        }
        b->cap = cap;
        g_staging.push_back(b);
    }
    std::memcpy(b->host, src, bytes);
    e = hipMemcpyAsync(dst, b->host, bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(b->done, stream);
    if (e != hipSuccess) return fail(KB_EDEVICE, "table upload failed: %s", hipGetErrorString(e));
    return KB_OK;
}

kb_status upload_tau_vel(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
                         void *workspace, hipStream_t stream, size_t *vel_off) {
    // tau_i = t_i - t_0, as the host table computes it, then the velocities.
    const size_t off = (static_cast<size_t>(n_img) * sizeof(double) + 15) / 16 * 16;
    std::vector<char> staged(off + static_cast<size_t>(2 * n_vel) * sizeof(double));
    double *tau = reinterpret_cast<double *>(staged.data());
    for (int64_t i = 0; i < n_img; ++i) tau[i] = t[i] - t[0];
    std::memcpy(staged.data() + off, vel, static_cast<size_t>(2 * n_vel) * sizeof(double));
    *vel_off = off;
    return staged_copy(workspace, staged.data(), staged.size(), stream);
}

// Copy the gather table (for planes of `pix_bytes` bytes per pair) and the
// visiting order into the workspace, asynchronously on `stream`.
kb_status upload_table(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
                       int64_t h, int64_t w, int64_t pix_bytes, void *workspace,
                       hipStream_t stream, bool visiting_order, int32_t *dy_range) {
    const size_t tb = table_bytes(n_img, n_vel);
    std::vector<char> host(tb + static_cast<size_t>(n_vel) * sizeof(int32_t));
    const GatherEntry *tab = reinterpret_cast<const GatherEntry *>(host.data());
    gather_table(t, n_img, vel, n_vel, h, w, pix_bytes, visiting_order,
                 reinterpret_cast<GatherEntry *>(host.data()),
                 reinterpret_cast<int32_t *>(host.data() + tb));
    if (dy_range) {
        const int64_t stride = table_stride(n_img);
        int32_t lo = 0, hi = 0;
        for (int64_t j = 0; j < n_vel; ++j)
            for (int64_t i = 0; i < n_img; ++i) {
                lo = std::min(lo, tab[j * stride + i].dy);
                hi = std::max(hi, tab[j * stride + i].dy);
            }
        dy_range[0] = lo;
        dy_range[1] = hi;
    }
    // The order follows the (256-byte rounded) table directly in the workspace.
    return staged_copy(workspace, host.data(), host.size(), stream);
}

}  // namespace kbmi

using namespace kbmi;

extern "C" {

kb_status kb_mask_bright(const float *img, uint8_t *mask, int64_t n_img, int64_t h, int64_t w,
                         float threshold, void *stream) {
    clear_error();
    if (!img || !mask) return fail(KB_EINVAL, "img and mask must be non-null");
    kb_status st = check_frame(n_img, h, w);
    if (st != KB_OK) return st;
    if (std::isnan(threshold)) return fail(KB_EINVAL, "threshold must not be NaN");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = n_img * h * w;
    const bool aligned = reinterpret_cast<uintptr_t>(img) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(mask) % 16 == 0;
    const int64_t n16 = aligned ? n / 16 : 0;
    if (n16 > 0) {
        const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 8192);
        hipLaunchKernelGGL(mask_bright_kernel, dim3((unsigned)blocks), dim3(256), 0, s, img, mask,
                           n16, threshold);
        st = launch_status("mask_bright_kernel");
        if (st != KB_OK) return st;
    }
    if (16 * n16 < n) {
        const int64_t rest = n - 16 * n16;
        const int64_t blocks = std::min<int64_t>((rest + 255) / 256, 8192);
        hipLaunchKernelGGL(mask_bright_tail_kernel, dim3((unsigned)blocks), dim3(256), 0, s, img,
                           mask, 16 * n16, n, threshold);
        st = launch_status("mask_bright_tail_kernel");
    }
    return st;
}

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
        if (!psi_phi_lp || !lp_scale)
            return fail(KB_EINVAL, "a 16-bit copy needs psi_phi_lp and lp_scale");
    }
    PsfTaps taps{};
    for (int64_t u = 0; u < psf_h * psf_w; ++u) taps.t[u] = psf[u];
    const dim3 grid((unsigned)((w + PP_TW - 1) / PP_TW), (unsigned)((h + PP_TH - 1) / PP_TH),
                    (unsigned)n_img);
    hipStream_t s = (hipStream_t)stream;
    const bool lp = lp_dtype != KB_F32;
    uint32_t *maxabs = lp ? reinterpret_cast<uint32_t *>(lp_scale) : nullptr;
    const int nsc = (int)(2 * n_img);
    if (lp) {
        hipLaunchKernelGGL(lp_zero_kernel, dim3((nsc + 255) / 256), dim3(256), 0, s, maxabs, nsc);
        kb_status ls = launch_status("lp_zero_kernel");
        if (ls != KB_OK) return ls;
    }
    float2 *pp = reinterpret_cast<float2 *>(psi_phi);
    switch (psf_w) {
#define KB_PSF_W(PW)                                                                         \
    case PW:                                                                                 \
        hipLaunchKernelGGL(psi_phi_kernel<PW>, grid, dim3(PP_THREADS),                       \
                           psi_phi_lds_bytes<PW>((int)psf_h), s, img, var, mask, (int)h,      \
                           (int)w, (int)psf_h, taps, pp, maxabs);                           \
        break;
        KB_PSF_W(1) KB_PSF_W(3) KB_PSF_W(5) KB_PSF_W(7) KB_PSF_W(9) KB_PSF_W(11) KB_PSF_W(13)
        KB_PSF_W(15) KB_PSF_W(17) KB_PSF_W(19) KB_PSF_W(21) KB_PSF_W(23) KB_PSF_W(25)
#undef KB_PSF_W
    default:
        return fail(KB_EUNSUPPORTED, "PSF width %lld is not an odd size <= %d", (long long)psf_w,
                    KB_MAX_PSF);
    }
    kb_status ls = launch_status("psi_phi_kernel");
    if (ls != KB_OK || !lp) return ls;
    hipLaunchKernelGGL(lp_scale_kernel, dim3((nsc + 255) / 256), dim3(256), 0, s, lp_scale, nsc);
    ls = launch_status("lp_scale_kernel");
    if (ls != KB_OK) return ls;
    const size_t npix_img = (size_t)h * (size_t)w;
    const size_t bx = std::min<size_t>((npix_img + 255) / 256, 2048);
    hipLaunchKernelGGL(lp_convert_kernel, dim3((unsigned)bx, (unsigned)n_img), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(psi_phi), npix_img, lp_scale,
                       (int)lp_dtype, static_cast<uint32_t *>(psi_phi_lp));
    return launch_status("lp_convert_kernel");
}

kb_status kb_search(const void *planes, int32_t dtype, const float *lp_scale, int64_t n_img,
                    int64_t h, int64_t w, const double *t, const double *vel, int64_t n_vel,
                    int64_t k_cand, float *cand_nu, float *cand_alpha, int32_t *cand_vel,
                    int16_t *cand_nobs, void *workspace, size_t workspace_bytes,
                    void *stream) {
    clear_error();
    kb_status st = check_search_args(planes, dtype, lp_scale, n_img, h, w, t, vel, n_vel,
                                     k_cand, cand_nu, cand_alpha, cand_vel, cand_nobs);
    if (st != KB_OK) return st;
    if (!workspace) return fail(KB_EINVAL, "workspace must be non-null");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KB_EINVAL, "workspace must be 256-byte aligned");
    const size_t ws_need = workspace_layout(n_img, h, w, n_vel).total;
    if (workspace_bytes < ws_need)
        return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", ws_need, workspace_bytes);
    hipStream_t s = (hipStream_t)stream;
    int32_t dy_range[2] = {0, 0};
    st = upload_table(t, n_img, vel, n_vel, h, w, dtype == KB_F32 ? 8 : 4, workspace, s, true,
                      dy_range);
    if (st != KB_OK) return st;
    return launch_search_in(planes, dtype, lp_scale, n_img, h, w, n_vel, k_cand, cand_nu,
                            cand_alpha, cand_vel, cand_nobs, workspace, dy_range, s);
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
    const int64_t npix = h * w;
    if ((npix + 3) / 4 > 2147483647LL) return fail(KB_EINVAL, "frame too large");
    const bool in_place = (const void *)nu == (const void *)cand_nu &&
                          (const void *)alpha == (const void *)cand_alpha &&
                          (const void *)vel_idx == (const void *)cand_vel &&
                          (const void *)nobs == (const void *)cand_nobs;
    const void *outs[4] = {nu, alpha, vel_idx, nobs};
    const void *cands[4] = {cand_nu, cand_alpha, cand_vel, cand_nobs};
    for (const void *o : outs)
        for (const void *c : cands)
            if (o == c && !in_place)
                return fail(KB_EINVAL, "outputs must be the candidate arrays (all four) or "
                                       "separate from them");
    if (in_place && (k != k_cand || psi_phi_f32 != nullptr))
        return fail(KB_EINVAL, "ordering in place needs k == k_cand and no re-scoring");
    if (psi_phi_f32 != nullptr) {
        if (n_vel < 1 || n_vel > 65535)
            return fail(KB_EINVAL, "n_vel must be in [1, 65535] (got %lld)", (long long)n_vel);
        st = check_times_velocities(t, n_img, vel, n_vel);
        if (st != KB_OK) return st;
        if (!workspace) return fail(KB_EINVAL, "re-scoring needs a workspace");
        if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
            return fail(KB_EINVAL, "workspace must be 256-byte aligned");
        const size_t ws_need = workspace_layout(n_img, h, w, n_vel).total;
        if (workspace_bytes < ws_need)
            return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", ws_need,
                        workspace_bytes);
        hipStream_t s = (hipStream_t)stream;
        size_t vel_off = 0;
        st = upload_tau_vel(t, n_img, vel, n_vel, workspace, s, &vel_off);
        if (st != KB_OK) return st;
        char *ws = static_cast<char *>(workspace);
        return launch_topk_rescore((int)h, (int)w, (int)n_img,
                                   reinterpret_cast<const float2 *>(psi_phi_f32),
                                   reinterpret_cast<const double *>(ws),
                                   reinterpret_cast<const double2 *>(ws + vel_off), (int)n_vel,
                                   (int)k_cand, (int)k, cand_vel, nu, alpha, vel_idx, nobs, s);
    }
    (void)workspace_bytes;
    return launch_topk(npix, (int)k_cand, (int)k, in_place, cand_nu, cand_alpha, cand_vel,
                       cand_nobs, nu, alpha, vel_idx, nobs, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Batch workspace: the device job descriptors (in launch order: the jobs of
// image-count class 0, then 1, then 2), the per-XCD counters of the three
// launches (3 x 8 words), then per job its table, visiting order and 16-bit
// inverse scales (each 256-byte aligned; job order as given).
struct BatchLayout {
    std::vector<size_t> table, order, inv_scale;
    size_t sync, total;
};

size_t round256(size_t n) { return (n + 255) & ~static_cast<size_t>(255); }

bool batch_layout(const kb_job *jobs, int64_t n_jobs, BatchLayout &l) {
    if (!jobs || n_jobs < 1 || n_jobs > 4096) return false;
    size_t off = round256(sizeof(BatchJob) * static_cast<size_t>(n_jobs));
    l.sync = off;
    off += 256;
    l.table.resize(n_jobs);
    l.order.resize(n_jobs);
    l.inv_scale.resize(n_jobs);
    for (int64_t q = 0; q < n_jobs; ++q) {
        const kb_job &j = jobs[q];
        if (j.n_img < 1 || j.n_vel < 1 || j.h < 1 || j.w < 1) return false;
        l.table[q] = off;
        off += table_bytes(j.n_img, j.n_vel);
        l.order[q] = off;
        off += order_bytes(j.n_vel);
        l.inv_scale[q] = off;
        off += round256(static_cast<size_t>(table_stride(j.n_img)) * 8);
    }
    l.total = off;
    return true;
}

// Image-count class of a job: the batch launches one kernel per class (one
// load batch of 8 or 16 per velocity, or batches of 16), like kb_search.
int image_class(int64_t n_img) { return n_img <= 8 ? 0 : (n_img <= 16 ? 1 : 2); }

}  // namespace

extern "C" {

size_t kb_search_batch_workspace_bytes(const kb_job *jobs, int64_t n_jobs) {
    BatchLayout l;
    return batch_layout(jobs, n_jobs, l) ? l.total : 0;
}

kb_status kb_search_batch(const kb_job *jobs, int64_t n_jobs, int32_t dtype, int64_t k_cand,
                          void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!jobs || n_jobs < 1 || n_jobs > 4096)
        return fail(KB_EINVAL, "n_jobs must be in [1, 4096] (got %lld)", (long long)n_jobs);
    if (dtype != KB_F32 && dtype != KB_F16 && dtype != KB_BF16)
        return fail(KB_EINVAL, "dtype must be KB_F32, KB_F16 or KB_BF16");
    if (k_cand < 1) return fail(KB_EINVAL, "k_cand must be >= 1");
    if (k_cand > KB_MAX_KCAND)
        return fail(KB_EUNSUPPORTED, "k_cand above %d is not supported", KB_MAX_KCAND);
    for (int64_t q = 0; q < n_jobs; ++q) {
        const kb_job &j = jobs[q];
        if (!j.planes || !j.cand_nu || !j.cand_alpha || !j.cand_vel || !j.cand_nobs)
            return fail(KB_EINVAL, "job %lld: planes and candidate outputs must be non-null",
                        (long long)q);
        kb_status st = check_frame(j.n_img, j.h, j.w);
        if (st != KB_OK) return fail(st, "job %lld: %s", (long long)q, kb_last_error());
        if (j.n_vel < 1 || j.n_vel > 65535)
            return fail(KB_EINVAL, "job %lld: n_vel must be in [1, 65535]", (long long)q);
        if (k_cand > j.n_vel)
            return fail(KB_EINVAL, "job %lld: k_cand exceeds n_vel", (long long)q);
        st = check_times_velocities(j.t, j.n_img, j.vel, j.n_vel);
        if (st != KB_OK) return fail(st, "job %lld: %s", (long long)q, kb_last_error());
        if (dtype != KB_F32 && !j.lp_scale)
            return fail(KB_EINVAL, "job %lld: 16-bit planes need lp_scale", (long long)q);
    }
    BatchLayout lay;
    batch_layout(jobs, n_jobs, lay);
    if (!workspace) return fail(KB_EINVAL, "workspace must be non-null");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KB_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < lay.total)
        return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", lay.total, workspace_bytes);

    // Work items of each class's persistent launch.  A job of float32 planes
    // large enough for the paced block order (as kb_search chooses it) starts
    // at a generation boundary and takes its whole block sequence; the others
    // are packed densely, tile after tile.
    const int kc = (int)k_cand;
    const int km = km_for(kc);
    hipStream_t s = (hipStream_t)stream;
    int grid[3] = {0, 0, 0}, count[3] = {0, 0, 0}, first[3] = {0, 0, 0};
    int64_t gens[3] = {0, 0, 0};
    std::vector<int> launch_order;
    for (int c = 0; c < 3; ++c) {
        first[c] = (int)launch_order.size();
        for (int64_t q = 0; q < n_jobs; ++q)
            if (image_class(jobs[q].n_img) == c) launch_order.push_back((int)q);
        count[c] = (int)launch_order.size() - first[c];
        if (count[c] > 0) {
            kb_status st = launch_search_batch(dtype, km, nullptr, 0, c, kc, 0, nullptr,
                                               &grid[c], s);
            if (st != KB_OK) return st;
        }
    }
    char *ws = static_cast<char *>(workspace);
    std::vector<char> host(lay.total, 0);
    BatchJob *desc = reinterpret_cast<BatchJob *>(host.data());
    for (int c = 0; c < 3; ++c) {
        int64_t cursor = 0;
        const int g = grid[c];
        for (int pos = first[c]; pos < first[c] + count[c]; ++pos) {
            const int q = launch_order[pos];
            const kb_job &j = jobs[q];
            gather_table(j.t, j.n_img, j.vel, j.n_vel, j.h, j.w, dtype == KB_F32 ? 8 : 4, true,
                         reinterpret_cast<GatherEntry *>(host.data() + lay.table[q]),
                         reinterpret_cast<int32_t *>(host.data() + lay.order[q]));
            BatchJob &d = desc[pos];
            d.planes = j.planes;
            d.inv_scale = reinterpret_cast<const float2 *>(ws + lay.inv_scale[q]);
            d.disp = reinterpret_cast<const GatherEntry *>(ws + lay.table[q]);
            d.vel_index = reinterpret_cast<const int32_t *>(ws + lay.order[q]);
            d.cand_nu = j.cand_nu;
            d.cand_alpha = j.cand_alpha;
            d.cand_vel = j.cand_vel;
            d.cand_nobs = j.cand_nobs;
            d.n_img = (int)j.n_img;
            d.h = (int)j.h;
            d.w = (int)j.w;
            d.disp_stride = (int)table_stride(j.n_img);
            d.n_vel = (int)j.n_vel;
            d.nseg = (int)((j.w + 63) / 64);
            d.strip = d.nseg < KBMI_STRIP_TILES ? d.nseg : KBMI_STRIP_TILES;
            const int64_t tiles = (int64_t)d.nseg * j.h;
            const bool block = KBMI_PERSIST_BS > 0 && dtype == KB_F32 &&
                               (g / 8) % KBMI_PERSIST_BS == 0 && tiles >= 4 * (int64_t)g;
            d.dense = block ? 0 : 1;
            d.bs = KBMI_PERSIST_BS > 0 ? KBMI_PERSIST_BS : 1;
            d.brows = (g / 8) / d.bs;
            d.nbc = (d.nseg + d.bs - 1) / d.bs;
            d.nbr = (d.h + d.brows - 1) / d.brows;
            if (block) {
                cursor = (cursor + g - 1) / g * g;
                d.item_begin = (int)std::min<int64_t>(cursor, 2147483647LL);
                cursor += (int64_t)((d.nbc + 7) / 8) * d.nbr * g;
            } else {
                d.item_begin = (int)std::min<int64_t>(cursor, 2147483647LL);
                cursor += tiles;
            }
            if (cursor + g > 2147483647LL)
                return fail(KB_EINVAL, "batch holds more work items than one launch");
        }
        gens[c] = g > 0 ? (cursor + g - 1) / g : 0;
    }
    kb_status up = staged_copy(ws, host.data(), host.size(), s);
    if (up != KB_OK) return up;
    if (dtype != KB_F32) {
        for (int64_t q = 0; q < n_jobs; ++q) {
            const int stride = (int)table_stride(jobs[q].n_img);
            hipLaunchKernelGGL(inv_scale_kernel, dim3((stride + 63) / 64), dim3(64), 0, s,
                               jobs[q].lp_scale, (int)jobs[q].n_img, stride,
                               reinterpret_cast<float2 *>(ws + lay.inv_scale[q]));
            kb_status st = launch_status("inv_scale_kernel");
            if (st != KB_OK) return st;
        }
    }
    for (int c = 0; c < 3; ++c) {
        if (count[c] == 0) continue;
        const BatchJob *dj = reinterpret_cast<const BatchJob *>(ws) + first[c];
        uint32_t *sync = reinterpret_cast<uint32_t *>(ws + lay.sync) + 8 * c;
        kb_status st = launch_search_batch(dtype, km, dj, count[c], c, kc, (int)gens[c], sync,
                                           &grid[c], s);
        if (st != KB_OK) return st;
    }
    return KB_OK;
}

}  // extern "C"
