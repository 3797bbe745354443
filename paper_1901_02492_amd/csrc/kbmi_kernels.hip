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
    float2 *__restrict__ out, uint32_t *__restrict__ maxabs) {
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
    if (maxabs != nullptr) {
        // Per-image max |psi| and max phi for the 16-bit copy's scale: a block
        // reduction, then one atomic max per block and plane (non-negative
        // floats order like their bit patterns).
        __shared__ float s_red[2][PP_THREADS / 64];
        float mp = 0.f, mf = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gy = ty0 + ly0 + 4 * r, gx = tx0 + lx;
            if (gy < h && gx < w && s_ok[(ly0 + 4 * r + cy) * PP_LW + lx + cx]) {
                mp = fmaxf(mp, fabsf(ps[r]));
                mf = fmaxf(mf, pf[r]);
            }
        }
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
template <int FMT>
struct PlaneLoad {                       // one (psi, phi) pair as loaded
    typedef u32x2 type;                  // float32: two words
};
template <>
struct PlaneLoad<KB_F16> {
    typedef uint32_t type;               // 16-bit: psi low half, phi high half
};
template <>
struct PlaneLoad<KB_BF16> {
    typedef uint32_t type;
};

__device__ inline float lp_value(uint32_t bits16, int fmt) {
    if (fmt == KB_F16) return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
    return __uint_as_float(bits16 << 16);
}

// One search problem as the host launchers see it.
struct StackView {
    const void *planes;        // [n_img][h][w] (psi, phi) pairs of format FMT
    const float2 *inv_scale;   // 16-bit planes: (1/s_psi, 1/s_phi) per image, padded with 0
    int n_img, h, w;
    const int2 *disp;          // displacement rows in visiting order, `disp_stride` pairs each
    int disp_stride;
    const int32_t *vel_index;  // original index of each visited velocity
    int n_vel, k_cand;
    float *cand_nu, *cand_alpha;
    int32_t *cand_vel;
    int16_t *cand_nobs;
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
template <int KM, int NB, int PB, int FMT>
__global__ __launch_bounds__(64, 2) void search_kernel(
    const void *__restrict__ planes, const float2 *__restrict__ inv_scale, int n_img, int h,
    int w, const int2 *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
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
    typedef typename PlaneLoad<FMT>::type LoadT;
    constexpr uint32_t kPix = FMT == KB_F32 ? 8u : 4u;   // bytes per (psi, phi) pair
    const uint32_t row_bytes = (uint32_t)w * kPix;
    const size_t img_bytes = (size_t)h * (size_t)w * kPix;

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
    auto issue = [&](int jj, int i0, LoadT(&v)[NB]) {
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
            if constexpr (FMT == KB_F32)
                v[b] = __builtin_amdgcn_raw_buffer_load_b64(rs, (x0 + dx) * (int)kPix, 0, 0);
            else
                v[b] = __builtin_amdgcn_raw_buffer_load_b32(rs, (x0 + dx) * (int)kPix, 0, 0);
        }
    };
    // Sum in image order.  Empty slots hold +0, which leaves every sum
    // unchanged.  16-bit values are decoded and unscaled by an exact power of
    // two inside the FMA (the product is exact, so the sum rounds once).
    auto accumulate = [&](int i0, const LoadT(&v)[NB], float &P, float &F) {
        if constexpr (FMT == KB_F32) {
            (void)i0;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                P += __uint_as_float(v[b].x);
                F += __uint_as_float(v[b].y);
            }
        } else {
            const float4 *sc4 = reinterpret_cast<const float4 *>(inv_scale + i0);
            float4 ss[NB / 2];
#pragma unroll
            for (int q = 0; q < NB / 2; ++q) ss[q] = sc4[q];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float isp = (b & 1) ? ss[b / 2].z : ss[b / 2].x;
                const float isf = (b & 1) ? ss[b / 2].w : ss[b / 2].y;
                P = fmaf(lp_value(v[b] & 0xFFFFu, FMT), isp, P);
                F = fmaf(lp_value(v[b] >> 16, FMT), isf, F);
            }
        }
    };
    // n_obs: the stored phi is nonzero exactly at valid pixels; empty slots are 0.
    auto count = [&](const LoadT(&v)[NB]) {
        uint32_t c = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if constexpr (FMT == KB_F32) c += v[b].y != 0u;
            else c += (v[b] >> 16) != 0u;
        }
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
    // and queue it if it beats the admission threshold.  n_obs sits in the
    // low bits of the key and never decides an order.
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
            LoadT v[NB];
            issue(jj, 0, v);
            float P = 0.f, F = 0.f;
            accumulate(0, v, P, F);
            finish(j, P, F, count(v));
        }
    } else {
        for (int jj = 0; jj < n_vel; ++jj) {
            const int j = vel_index[jj];
            float P = 0.f, F = 0.f;
            uint32_t c = 0;
            for (int i0 = 0; i0 < n_img; i0 += NB) {
                LoadT v[NB];
                issue(jj, i0, v);
                accumulate(i0, v, P, F);
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
// Final selection.  One thread per candidate: a 256-thread block holds whole
// pixels (256 / k_cand of them), reads their candidate runs with coalesced
// loads, and each thread checks that its candidate precedes the next one of
// the same pixel.  When every pixel of the block is in rank order (kb_search
// leaves them so) the first k of each are copied out; otherwise each
// candidate's rank is the number of candidates of its pixel that precede it.
// ---------------------------------------------------------------------------
constexpr int TK_THREADS = 256;

__global__ __launch_bounds__(TK_THREADS) void topk_kernel(
    int64_t npix, int k_cand, int k, const float *__restrict__ cand_nu,
    const float *__restrict__ cand_alpha, const int32_t *__restrict__ cand_vel,
    const int16_t *__restrict__ cand_nobs, float *__restrict__ nu, float *__restrict__ alpha,
    int32_t *__restrict__ vel, int16_t *__restrict__ nobs) {
    __shared__ uint64_t s_key[TK_THREADS];
    const int ppb = TK_THREADS / k_cand;
    const int t = (int)threadIdx.x;
    const int lp = t / k_cand, s = t - lp * k_cand;
    const int64_t p = (int64_t)blockIdx.x * ppb + lp;
    const bool active = lp < ppb && p < npix;
    uint64_t key = 0;
    float v_nu = 0.f, v_al = 0.f;
    int32_t v_vel = 0;
    int16_t v_no = 0;
    if (active) {
        const size_t e = (size_t)p * (size_t)k_cand + (size_t)s;
        v_nu = cand_nu[e];
        v_al = cand_alpha[e];
        v_vel = cand_vel[e];
        v_no = cand_nobs[e];
        key = make_key(v_nu, v_vel, (uint16_t)v_no);
    }
    s_key[t] = key;
    __syncthreads();
    const bool out_of_order = active && s + 1 < k_cand && !(key > s_key[t + 1]);
    int rank = s;
    if (__syncthreads_or(out_of_order)) {
        rank = 0;
        for (int r = 0; r < k_cand; ++r) rank += s_key[lp * k_cand + r] > key;
    }
    if (active && rank < k) {
        const size_t o = (size_t)p * (size_t)k + (size_t)rank;
        nu[o] = v_nu;
        alpha[o] = v_al;
        vel[o] = v_vel;
        nobs[o] = v_no;
    }
}

// ---------------------------------------------------------------------------
// Re-scoring selection (after a 16-bit search): every candidate's Psi, Phi and
// n_obs are recomputed from the float32 planes with exactly the arithmetic of
// the float32 search (image order, out-of-frame terms adding +0, the same
// score expressions), so a re-scored entry is bitwise the plain path's value
// for that trajectory.  Then every pixel's candidates are ranked by counting.
// table: displacements in the original velocity order, rows of `stride`.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TK_THREADS) void topk_rescore_kernel(
    int64_t npix, int h, int w, int n_img, const float2 *__restrict__ planes,
    const int2 *__restrict__ table, int stride, int n_vel, int k_cand, int k,
    const int32_t *__restrict__ cand_vel, float *__restrict__ nu, float *__restrict__ alpha,
    int32_t *__restrict__ vel, int16_t *__restrict__ nobs) {
    __shared__ uint64_t s_key[TK_THREADS];
    const int ppb = TK_THREADS / k_cand;
    const int t = (int)threadIdx.x;
    const int lp = t / k_cand;
    const int64_t p = (int64_t)blockIdx.x * ppb + lp;
    const bool active = lp < ppb && p < npix;
    uint64_t key = 0;
    float v_nu = 0.f, v_al = 0.f;
    int32_t j = 0;
    uint32_t c = 0;
    if (active) j = cand_vel[(size_t)p * (size_t)k_cand + (size_t)(t - lp * k_cand)];
    // A candidate index outside the grid (not written by kb_search) is dropped.
    const bool scored = active && j >= 0 && j < n_vel;
    if (scored) {
        const int y0 = (int)(p / w), x0 = (int)(p - (int64_t)y0 * w);
        const int2 *tj = table + (size_t)j * (size_t)stride;
        float P = 0.f, F = 0.f;
        for (int i0 = 0; i0 < n_img; i0 += 8) {
            float2 v[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int i = i0 + b;
                const int2 d = tj[i < n_img ? i : 0];
                const int y = y0 + d.y, x = x0 + d.x;
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
        v_nu = F > 0.f ? P / sqrtf(F) : -INFINITY;
        v_al = F > 0.f ? P / F : 0.f;
        key = make_key(v_nu, j, c);
    }
    s_key[t] = key;
    __syncthreads();
    int rank = 0;
    for (int r = 0; r < k_cand; ++r) rank += s_key[lp * k_cand + r] > key;
    if (active && rank < k) {
        const size_t o = (size_t)p * (size_t)k + (size_t)rank;
        nu[o] = scored ? v_nu : -INFINITY;
        alpha[o] = v_al;
        vel[o] = j;
        nobs[o] = (int16_t)c;
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

struct SearchLaunch {
    StackView sv;
    int fmt;
    hipStream_t stream;
};

TileMap tile_map(int w, int h) {
    TileMap tm;
    tm.nseg = (w + 63) / 64;
    tm.h = h;
    tm.strip = tm.nseg < KBMI_STRIP_TILES ? tm.nseg : KBMI_STRIP_TILES;
    tm.nblocks = tm.nseg * h;
    return tm;
}

template <int KM, int NB, int FMT>
kb_status launch_search_fmt(const SearchLaunch &a) {
    constexpr int PB = KBMI_QUEUE;
    const StackView &v = a.sv;
    const TileMap tm = tile_map(v.w, v.h);
    hipLaunchKernelGGL((search_kernel<KM, NB, PB, FMT>), dim3(tm.nblocks), dim3(64), 0, a.stream,
                       v.planes, v.inv_scale, v.n_img, v.h, v.w, v.disp, v.disp_stride,
                       v.vel_index, v.n_vel, v.k_cand, tm, v.cand_nu, v.cand_alpha, v.cand_vel,
                       v.cand_nobs);
    return launch_status("search_kernel");
}

template <int KM, int NB>
kb_status launch_search_nb(const SearchLaunch &a) {
    static_assert(NB == 8 || NB == 16, "table rows are padded for batches of 8 or 16");
    if (a.fmt == KB_F16) return launch_search_fmt<KM, NB, KB_F16>(a);
    if (a.fmt == KB_BF16) return launch_search_fmt<KM, NB, KB_BF16>(a);
    return launch_search_fmt<KM, NB, KB_F32>(a);
}

template <int KM>
kb_status launch_search_km(const SearchLaunch &a) {
    if (a.sv.n_img <= 8) return launch_search_nb<KM, 8>(a);
    return launch_search_nb<KM, 16>(a);
}

// 1/s per image and plane for the 16-bit search, padded with 0 to the table
// stride (padding images then contribute exactly 0).
__global__ void inv_scale_kernel(const float *__restrict__ scale, int n_img, int stride,
                                 float2 *__restrict__ inv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < stride)
        inv[i] = i < n_img ? make_float2(1.0f / scale[2 * i], 1.0f / scale[2 * i + 1])
                           : make_float2(0.f, 0.f);
}

kb_status launch_topk_rescore(int64_t npix, int h, int w, int n_img, const float2 *planes,
                              const int2 *table, int stride, int n_vel, int k_cand, int k,
                              const int32_t *cv,
                              float *nu, float *al, int32_t *vi, int16_t *no, hipStream_t stream) {
    const int64_t ppb = TK_THREADS / k_cand;
    const int64_t blocks = (npix + ppb - 1) / ppb;
    hipLaunchKernelGGL(topk_rescore_kernel, dim3((unsigned)blocks), dim3(TK_THREADS), 0, stream,
                       npix, h, w, n_img, planes, table, stride, n_vel, k_cand, k, cv, nu, al, vi,
                       no);
    return launch_status("topk_rescore_kernel");
}

kb_status launch_topk(int64_t npix, int k_cand, int k, const float *cn, const float *ca,
                      const int32_t *cv, const int16_t *co, float *nu, float *al, int32_t *vi,
                      int16_t *no, hipStream_t stream) {
    const int64_t ppb = TK_THREADS / k_cand;
    const int64_t blocks = (npix + ppb - 1) / ppb;
    hipLaunchKernelGGL(topk_kernel, dim3((unsigned)blocks), dim3(TK_THREADS), 0, stream, npix,
                       k_cand, k, cn, ca, cv, co, nu, al, vi, no);
    return launch_status("topk_kernel");
}

// List lengths compiled for the search: every even length up to KB_MAX_KCAND
// (each slot costs registers and compare-and-swap work on every insertion).
#define KB_SEARCH_KM_LIST(X)                                                              \
    X(2) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26) X(28) X(30) \
    X(32) X(34) X(36) X(38) X(40) X(42) X(44) X(46) X(48) X(50) X(52) X(54) X(56) X(58)  \
    X(60) X(62) X(64)

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
                       int64_t h, int64_t w, void *workspace, hipStream_t stream,
                       bool visiting_order = true) {
    // Velocities in visiting order, then the table of the reordered grid.
    std::vector<int32_t> order(static_cast<size_t>(n_vel));
    if (visiting_order)
        velocity_order(vel, n_vel, order.data());
    else
        for (int64_t j = 0; j < n_vel; ++j) order[j] = static_cast<int32_t>(j);
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
    hipLaunchKernelGGL(psi_phi_kernel, grid, dim3(PP_THREADS), 0, s, img, var, mask, (int)h,
                       (int)w, (int)psf_h, (int)psf_w, taps, reinterpret_cast<float2 *>(psi_phi),
                       maxabs);
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
    if (dtype != KB_F32 && !lp_scale)
        return fail(KB_EINVAL, "16-bit planes need lp_scale");
    if (!workspace) return fail(KB_EINVAL, "workspace must be non-null");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KB_EINVAL, "workspace must be 256-byte aligned");
    const size_t ws_need = workspace_layout(n_img, h, w, n_vel).total;
    if (workspace_bytes < ws_need)
        return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", ws_need, workspace_bytes);
    hipStream_t s = (hipStream_t)stream;
    st = upload_table(t, n_img, vel, n_vel, h, w, workspace, s);
    if (st != KB_OK) return st;
    const int kc = (int)k_cand;
    char *wsb = static_cast<char *>(workspace);
    const WorkspaceLayout lay = workspace_layout(n_img, h, w, n_vel);
    SearchLaunch a;
    StackView &sv = a.sv;
    sv.planes = planes;
    sv.inv_scale = reinterpret_cast<const float2 *>(wsb + lay.inv_scale);
    sv.n_img = (int)n_img;
    sv.h = (int)h;
    sv.w = (int)w;
    sv.disp = reinterpret_cast<const int2 *>(wsb + lay.table);
    sv.disp_stride = (int)table_stride(n_img);
    sv.vel_index = reinterpret_cast<const int32_t *>(wsb + lay.order);
    sv.n_vel = (int)n_vel;
    sv.k_cand = kc;
    sv.cand_nu = cand_nu;
    sv.cand_alpha = cand_alpha;
    sv.cand_vel = cand_vel;
    sv.cand_nobs = cand_nobs;
    a.fmt = dtype;
    a.stream = s;
    if (dtype != KB_F32) {
        const int stride = (int)table_stride(n_img);
        hipLaunchKernelGGL(inv_scale_kernel, dim3((stride + 63) / 64), dim3(64), 0, s, lp_scale,
                           (int)n_img, stride, const_cast<float2 *>(sv.inv_scale));
        st = launch_status("inv_scale_kernel");
        if (st != KB_OK) return st;
    }
    const int km = (kc + 1) & ~1;
    switch (km) {
#define KB_SEARCH_CASE(K) \
    case K:               \
        return launch_search_km<K>(a);
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
    const int64_t npix = h * w;
    if ((npix + 3) / 4 > 2147483647LL) return fail(KB_EINVAL, "frame too large");
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
        st = upload_table(t, n_img, vel, n_vel, h, w, workspace, s, false);
        if (st != KB_OK) return st;
        return launch_topk_rescore(npix, (int)h, (int)w, (int)n_img,
                                   reinterpret_cast<const float2 *>(psi_phi_f32),
                                   reinterpret_cast<const int2 *>(workspace),
                                   (int)table_stride(n_img), (int)n_vel, (int)k_cand, (int)k,
                                   cand_vel, nu, alpha, vel_idx, nobs, s);
    }
    (void)workspace_bytes;
    return launch_topk(npix, (int)k_cand, (int)k, cand_nu, cand_alpha, cand_vel, cand_nobs, nu,
                       alpha, vel_idx, nobs, (hipStream_t)stream);
}

}  // extern "C"
