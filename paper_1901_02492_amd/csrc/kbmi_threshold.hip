// Threshold mode and duplicate clustering of libkbmi.
//
//   search_threshold_kernel  every trajectory whose nu reaches a threshold
//                            (Sec. 2.2; Sec. 3.2 keeps nu >= 10), appended
//                            to a device list by wave-wide compaction
//   cluster kernels          groups of hits within eps in (x, y, s*vx, s*vy)
//                            (DBSCAN with min_samples = 1, Sec. 3.3) by
//                            lock-free union-find, and each group's best hit
//
// The threshold search gathers and scores exactly as the top-k search does
// (same table, loads, image order and score functions), so a hit's nu, alpha
// and n_obs are bitwise the values the top-k path gives that trajectory.  It
// keeps no list, so it needs few registers; it runs in the top-k search's
// paced persistent order with two velocities' gathers in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "kbmi_common.h"
#include "kbmi_device.h"

namespace kbmi {
namespace {

constexpr int TH_NB = 16;          // table entries per batch (the table stride unit)
constexpr int TH_STRIP = 4;        // tiles per strip of the tile order

#ifndef KBMI_TH_PERSIST
#define KBMI_TH_PERSIST 1   // threshold search: paced persistent order (float32 search's)
#endif

// One tile: 64 adjacent start pixels of one row, every velocity.
__device__ __forceinline__ void threshold_tile(
    const float2 *__restrict__ planes, int n_img, int h, int w,
    const GatherEntry *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
    int n_vel, int row, int seg, float nu_min, kb_hit *__restrict__ hits, uint64_t cap,
    unsigned long long *__restrict__ n_hits) {
    const int lane = (int)threadIdx.x;
    const int x0 = seg * 64 + lane;
    const uint32_t row_bytes = (uint32_t)w * 8u;
    const uint64_t row0 = reinterpret_cast<uint64_t>(planes) + (uint64_t)row * row_bytes;
    const const_i32 *visit = (const const_i32 *)(const void *)vel_index;
    const uint64_t below = (uint64_t(1) << lane) - 1;

    auto fetch = [&](int jj, int i0, i32x4(&e)[TH_NB]) {
        const const_i32x4 *t4 =
            (const const_i32x4 *)(const void *)(disp + (size_t)jj * disp_stride + i0);
#pragma unroll
        for (int b = 0; b < TH_NB; ++b) e[b] = t4[b];
    };
    // Rows outside the frame (padding entries included) get a zero-length
    // buffer: the load returns 0 without an access.
    auto issue = [&](const i32x4(&e)[TH_NB], u32x2(&v)[TH_NB]) {
#pragma unroll
        for (int b = 0; b < TH_NB; ++b) {
            const int yy = row + e[b].y;
            const bool in_rows = (unsigned)yy < (unsigned)h;
            const uint64_t off = ((uint64_t)(uint32_t)e[b].w << 32) | (uint32_t)e[b].z;
            const i32x4 rs = buffer_words(row0 + off, in_rows ? row_bytes : 0u);
            v[b] = raw_load_b64(rs, (x0 + e[b].x) * 8, 0, 0);
        }
    };
    auto accumulate = [&](const u32x2(&v)[TH_NB], float &P, float &F, uint32_t &c) {
#pragma unroll
        for (int b = 0; b < TH_NB; ++b) {
            P += __uint_as_float(v[b].x);
            F += __uint_as_float(v[b].y);
            c += min(v[b].y, 1u);
        }
    };
    // Score one trajectory and append it if nu >= nu_min: one atomic per
    // wave reserves the wave's slots in the list.
    auto finish = [&](int j, float P, float F, uint32_t c) {
        const float r = inv_sqrt_phi(F);
        const float nu = score_nu(P, F, r);
        const bool pass = x0 < w && nu >= nu_min;
        const uint64_t bal = __ballot(pass);
        if (bal != 0) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(n_hits, (unsigned long long)__popcll(bal));
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
            const uint64_t idx = (((uint64_t)hi << 32) | lo) + (uint64_t)__popcll(bal & below);
            if (pass && idx < cap) {
                kb_hit hit;
                hit.x = x0;
                hit.y = row;
                hit.vel = j;
                hit.nu = nu;
                hit.alpha = score_alpha(nu, F, r);
                hit.nobs = (int16_t)c;
                hit.reserved = 0;
                hits[idx] = hit;
            }
        }
    };

    if (n_img <= TH_NB) {
        // Two velocities in flight: the gathers of visit jj+1 are issued
        // before visit jj is summed and scored; a visit past the end repeats
        // the last row and is never scored.
        i32x4 e[TH_NB];
        u32x2 va[TH_NB], vb[TH_NB];
        const int last = n_vel - 1;
        fetch(0, 0, e);
        issue(e, va);
        int j_cur = visit[0];
        int nxt = last < 1 ? last : 1;
        fetch(nxt, 0, e);
        int j_nxt = visit[nxt];
        auto step = [&](int jj, u32x2(&cur)[TH_NB], u32x2(&ahead)[TH_NB]) {
            issue(e, ahead);
            __builtin_amdgcn_sched_barrier(0);
            const int n2 = jj + 2 < last ? jj + 2 : last;
            fetch(n2, 0, e);
            const int j2 = visit[n2];
            __builtin_amdgcn_sched_barrier(0);
            float P = 0.f, F = 0.f;
            uint32_t c = 0;
            accumulate(cur, P, F, c);
            finish(j_cur, P, F, c);
            j_cur = j_nxt;
            j_nxt = j2;
        };
        int jj = 0;
        for (; jj + 1 < n_vel; jj += 2) {
            step(jj, va, vb);
            step(jj + 1, vb, va);
        }
        if (jj < n_vel) step(jj, va, vb);
    } else {
        for (int jj = 0; jj < n_vel; ++jj) {
            float P = 0.f, F = 0.f;
            uint32_t c = 0;
            for (int i0 = 0; i0 < n_img; i0 += TH_NB) {
                i32x4 e[TH_NB];
                fetch(jj, i0, e);
                u32x2 v[TH_NB];
                issue(e, v);
                accumulate(v, P, F, c);
            }
            finish(visit[jj], P, F, c);
        }
    }
}

// Strip tile order, one wave per tile.
__global__ __launch_bounds__(64) void search_threshold_kernel(
    const float2 *__restrict__ planes, int n_img, int h, int w,
    const GatherEntry *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
    int n_vel, int nseg, int ntiles, float nu_min, kb_hit *__restrict__ hits, uint64_t cap,
    unsigned long long *__restrict__ n_hits) {
    int row, seg;
    strip_tile(xcd_remap((int)blockIdx.x, ntiles), nseg, h, TH_STRIP, row, seg);
    threshold_tile(planes, n_img, h, w, disp, disp_stride, vel_index, n_vel, row, seg, nu_min,
                   hits, cap, n_hits);
}

// The paced persistent order of the float32 top-k search: per generation each
// XCD covers one block of start pixels and its waves wait (a bounded time) for
// each other at the end of the generation, so that their gathers share the
// XCD's L2.  The wait only shapes timing.
__global__ __launch_bounds__(64) void search_threshold_persistent_kernel(
    const float2 *__restrict__ planes, int n_img, int h, int w,
    const GatherEntry *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
    int n_vel, PersistMap pm, float nu_min, kb_hit *__restrict__ hits, uint64_t cap,
    unsigned long long *__restrict__ n_hits, uint32_t *sync) {
    uint32_t *xcd_count = sync + (blockIdx.x & 7);
    const uint32_t per_xcd = gridDim.x >> 3;
    int spin = pm.spin;
    for (int gen = 0; gen < pm.generations; ++gen) {
        int row, seg;
        if (pm.map(gen, (int)blockIdx.x, row, seg))
            threshold_tile(planes, n_img, h, w, disp, disp_stride, vel_index, n_vel, row, seg,
                           nu_min, hits, cap, n_hits);
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(xcd_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = (uint32_t)(gen + 1) * per_xcd;
        int i = 0;
        for (; i < spin; ++i) {
            if (__hip_atomic_load(xcd_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                target)
                break;
            __builtin_amdgcn_s_sleep(8);
        }
        if (i == spin) spin = 0;
    }
}

int threshold_grid() {
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, search_threshold_persistent_kernel, 64, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = std::min(per_cu, KBMI_PERSIST_PER_CU) * cus;
    }
    return cached[dev];
}

__global__ void zero_u64_kernel(unsigned long long *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

// ---------------------------------------------------------------------------
// Clustering.  parent[] forms a forest in which every edge points to a
// smaller index: uniting two roots hooks the larger under the smaller with a
// compare-and-swap, and a failed swap means the root was hooked meanwhile, to
// a smaller index, so the loop makes progress and ends.  The root of each tree
// is therefore the smallest index of its component.
// ---------------------------------------------------------------------------
constexpr int CL_TILE = 256;

__device__ inline int cl_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int cl_find(int32_t *parent, int a) {
    int p = cl_load(parent + a);
    while (p != a) {
        a = p;
        p = cl_load(parent + a);
    }
    return a;
}

__device__ inline void cl_unite(int32_t *parent, int a, int b) {
    for (;;) {
        a = cl_find(parent, a);
        b = cl_find(parent, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicCAS(parent + b, b, a);
        if (old == b) return;
        b = old;
    }
}

__global__ void cl_init_kernel(int32_t *parent, uint32_t *best_nu, uint64_t *best_key,
                               int32_t *rep_of_root, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) {
        parent[i] = i;
        best_nu[i] = 0u;
        best_key[i] = ~0ull;
        rep_of_root[i] = -1;
    }
}

// Block (bx, by) compares the hits of tile by with those of tile bx >= by;
// pair (i, j), i < j, is joined when d2 <= eps2 with
// d2 = ((dx*dx + dy*dy) + du*du) + dv*dv in double, u = s * vx, v = s * vy.
// A hit whose velocity index is outside the grid gets NaN coordinates, which
// compare false with everything: it stays a group of its own.
__device__ inline double2 cl_vel(const double2 *vel, int n_vel, int j) {
    return (unsigned)j < (unsigned)n_vel ? vel[j] : make_double2(NAN, NAN);
}

__global__ __launch_bounds__(CL_TILE) void cl_pairs_kernel(const kb_hit *__restrict__ hits, int n,
                                                         const double2 *__restrict__ vel,
                                                         int n_vel, double s, double eps2,
                                                         int32_t *parent) {
#pragma clang fp contract(off)
    const int ti = (int)blockIdx.y, tj = (int)blockIdx.x;
    if (tj < ti) return;
    __shared__ double sx[CL_TILE], sy[CL_TILE], su[CL_TILE], sv[CL_TILE];
    const int jl = tj * CL_TILE + (int)threadIdx.x;
    if (jl < n) {
        const kb_hit hj = hits[jl];
        const double2 vj = cl_vel(vel, n_vel, hj.vel);
        sx[threadIdx.x] = (double)hj.x;
        sy[threadIdx.x] = (double)hj.y;
        su[threadIdx.x] = s * vj.x;
        sv[threadIdx.x] = s * vj.y;
    }
    __syncthreads();
    const int i = ti * CL_TILE + (int)threadIdx.x;
    if (i >= n) return;
    const kb_hit hi = hits[i];
    const double2 vi = cl_vel(vel, n_vel, hi.vel);
    const double xi = (double)hi.x, yi = (double)hi.y, ui = s * vi.x, vv = s * vi.y;
    const int jn = min(CL_TILE, n - tj * CL_TILE);
    for (int q = 0; q < jn; ++q) {
        const int j = tj * CL_TILE + q;
        if (j <= i) continue;
        const double dx = xi - sx[q], dy = yi - sy[q], du = ui - su[q], dv = vv - sv[q];
        const double d2 = ((dx * dx + dy * dy) + du * du) + dv * dv;
        if (d2 <= eps2) cl_unite(parent, i, j);
    }
}

__global__ void cl_flatten_kernel(int32_t *parent, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) parent[i] = cl_find(parent, i);
}

__device__ inline uint64_t cl_key(const kb_hit &h) {
    return ((uint64_t)(uint32_t)h.y << 40) | ((uint64_t)(uint32_t)h.x << 16) |
           (uint64_t)(uint32_t)h.vel;
}

__global__ void cl_best_nu_kernel(const kb_hit *__restrict__ hits, const int32_t *root,
                                  uint32_t *best_nu, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) atomicMax(best_nu + root[i], nu_order_bits(hits[i].nu));
}

__global__ void cl_best_key_kernel(const kb_hit *__restrict__ hits, const int32_t *root,
                                   const uint32_t *best_nu, uint64_t *best_key, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) {
        const kb_hit h = hits[i];
        const int r = root[i];
        if (nu_order_bits(h.nu) == best_nu[r])
            atomicMin(reinterpret_cast<unsigned long long *>(best_key + r),
                      (unsigned long long)cl_key(h));
    }
}

__global__ void cl_rep_kernel(const kb_hit *__restrict__ hits, const int32_t *root,
                              const uint32_t *best_nu, const uint64_t *best_key,
                              int32_t *rep_of_root, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) {
        const kb_hit h = hits[i];
        const int r = root[i];
        if (nu_order_bits(h.nu) == best_nu[r] && cl_key(h) == best_key[r]) rep_of_root[r] = i;
    }
}

__global__ void cl_out_kernel(const int32_t *root, const int32_t *rep_of_root, int32_t *rep,
                              int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) rep[i] = rep_of_root[root[i]];
}

size_t r256(size_t n) { return (n + 255) & ~static_cast<size_t>(255); }

struct ClusterLayout {
    size_t parent, best_nu, best_key, rep_of_root, vel, total;
};

ClusterLayout cluster_layout(int64_t n_hits, int64_t n_vel) {
    ClusterLayout l{};
    const size_t n = static_cast<size_t>(n_hits);
    l.parent = 0;
    l.best_nu = l.parent + r256(n * sizeof(int32_t));
    l.best_key = l.best_nu + r256(n * sizeof(uint32_t));
    l.rep_of_root = l.best_key + r256(n * sizeof(uint64_t));
    l.vel = l.rep_of_root + r256(n * sizeof(int32_t));
    l.total = l.vel + r256(static_cast<size_t>(n_vel) * 2 * sizeof(double));
    return l;
}

}  // namespace
}  // namespace kbmi

using namespace kbmi;

extern "C" {

kb_status kb_search_threshold(const float *psi_phi, int64_t n_img, int64_t h, int64_t w,
                              const double *t, const double *vel, int64_t n_vel, float nu_min,
                              kb_hit *hits, int64_t max_hits, uint64_t *n_hits, void *workspace,
                              size_t workspace_bytes, void *stream) {
    clear_error();
    if (!psi_phi || !t || !vel || !n_hits || (!hits && max_hits > 0))
        return fail(KB_EINVAL, "planes, times, velocities, the hit list and its counter must "
                               "be non-null");
    kb_status st = check_frame(n_img, h, w);
    if (st != KB_OK) return st;
    if (n_vel < 1 || n_vel > 65535)
        return fail(KB_EINVAL, "n_vel must be in [1, 65535] (got %lld)", (long long)n_vel);
    if (max_hits < 0) return fail(KB_EINVAL, "max_hits must be >= 0");
    if (!std::isfinite(nu_min)) return fail(KB_EINVAL, "nu_min must be finite");
    if (w >= (int64_t(1) << 24) || h >= (int64_t(1) << 24))
        return fail(KB_EUNSUPPORTED, "threshold mode takes frames below 2^24 on each side");
    st = check_times_velocities(t, n_img, vel, n_vel);
    if (st != KB_OK) return st;
    if (!workspace) return fail(KB_EINVAL, "the threshold search needs a workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KB_EINVAL, "workspace must be 256-byte aligned");
    const WorkspaceLayout lay = workspace_layout(n_img, h, w, n_vel);
    if (workspace_bytes < lay.total)
        return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", lay.total, workspace_bytes);
    hipStream_t s = (hipStream_t)stream;
    st = upload_table(t, n_img, vel, n_vel, h, w, 8, workspace, s);
    if (st != KB_OK) return st;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<unsigned long long *>(n_hits));
    st = launch_status("zero_u64_kernel");
    if (st != KB_OK) return st;
    char *ws = static_cast<char *>(workspace);
    const int nseg = (int)((w + 63) / 64);
    const int64_t ntiles = (int64_t)nseg * h;
    const int grid = KBMI_TH_PERSIST ? threshold_grid() : 0;
    const int per_xcd = grid / 8;
    if (grid >= 8 && grid % 8 == 0 && per_xcd % KBMI_PERSIST_BS == 0 && ntiles >= 4 * (int64_t)grid) {
        PersistMap pm;
        pm.nseg = nseg;
        pm.h = (int)h;
        pm.bs = KBMI_PERSIST_BS;
        pm.brows = per_xcd / KBMI_PERSIST_BS;
        pm.nbc = (nseg + pm.bs - 1) / pm.bs;
        pm.nbr = ((int)h + pm.brows - 1) / pm.brows;
        pm.generations = (pm.nbc + 7) / 8 * pm.nbr;
        pm.spin = KBMI_PERSIST_SPIN;
        uint32_t *sync = reinterpret_cast<uint32_t *>(ws + lay.sync);
        hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, sync, 8);
        st = launch_status("zero_words_kernel");
        if (st != KB_OK) return st;
        hipLaunchKernelGGL(search_threshold_persistent_kernel, dim3((unsigned)grid), dim3(64), 0,
                           s, reinterpret_cast<const float2 *>(psi_phi), (int)n_img, (int)h,
                           (int)w, reinterpret_cast<const GatherEntry *>(ws + lay.table),
                           (int)table_stride(n_img),
                           reinterpret_cast<const int32_t *>(ws + lay.order), (int)n_vel, pm,
                           nu_min, hits, (uint64_t)max_hits,
                           reinterpret_cast<unsigned long long *>(n_hits), sync);
        return launch_status("search_threshold_persistent_kernel");
    }
    hipLaunchKernelGGL(search_threshold_kernel, dim3((unsigned)ntiles), dim3(64), 0, s,
                       reinterpret_cast<const float2 *>(psi_phi), (int)n_img, (int)h, (int)w,
                       reinterpret_cast<const GatherEntry *>(ws + lay.table),
                       (int)table_stride(n_img), reinterpret_cast<const int32_t *>(ws + lay.order),
                       (int)n_vel, nseg, (int)ntiles, nu_min, hits, (uint64_t)max_hits,
                       reinterpret_cast<unsigned long long *>(n_hits));
    return launch_status("search_threshold_kernel");
}

size_t kb_cluster_workspace_bytes(int64_t n_hits, int64_t n_vel) {
    if (n_hits < 0 || n_vel < 1) return 0;
    return cluster_layout(n_hits, n_vel).total;
}

kb_status kb_cluster_hits(const kb_hit *hits, int64_t n_hits, const double *vel, int64_t n_vel,
                          double s, double eps, int32_t *rep, void *workspace,
                          size_t workspace_bytes, void *stream) {
    clear_error();
    if (n_hits < 0) return fail(KB_EINVAL, "n_hits must be >= 0");
    if (n_hits == 0) return KB_OK;
    if (!hits || !vel || !rep || !workspace)
        return fail(KB_EINVAL, "hits, velocities, rep and workspace must be non-null");
    if (n_vel < 1 || n_vel > 65535)
        return fail(KB_EINVAL, "n_vel must be in [1, 65535] (got %lld)", (long long)n_vel);
    if (n_hits > (int64_t)CL_TILE * 65535)
        return fail(KB_EUNSUPPORTED, "at most %d hits per call", CL_TILE * 65535);
    if (!(std::isfinite(s) && s >= 0.0)) return fail(KB_EINVAL, "s must be finite and >= 0");
    if (!(std::isfinite(eps) && eps >= 0.0)) return fail(KB_EINVAL, "eps must be finite and >= 0");
    for (int64_t j = 0; j < 2 * n_vel; ++j)
        if (!std::isfinite(vel[j])) return fail(KB_EINVAL, "velocities must be finite");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KB_EINVAL, "workspace must be 256-byte aligned");
    const ClusterLayout lay = cluster_layout(n_hits, n_vel);
    if (workspace_bytes < lay.total)
        return fail(KB_ENOMEM, "workspace needs %zu bytes (got %zu)", lay.total, workspace_bytes);
    hipStream_t st_ = (hipStream_t)stream;
    char *ws = static_cast<char *>(workspace);
    kb_status st = staged_copy(ws + lay.vel, vel, static_cast<size_t>(2 * n_vel) * sizeof(double),
                               st_);
    if (st != KB_OK) return st;
    int32_t *parent = reinterpret_cast<int32_t *>(ws + lay.parent);
    uint32_t *best_nu = reinterpret_cast<uint32_t *>(ws + lay.best_nu);
    uint64_t *best_key = reinterpret_cast<uint64_t *>(ws + lay.best_key);
    int32_t *rep_of_root = reinterpret_cast<int32_t *>(ws + lay.rep_of_root);
    const double2 *dvel = reinterpret_cast<const double2 *>(ws + lay.vel);
    const int n = (int)n_hits;
    const dim3 b1((unsigned)((n + 255) / 256)), t1(256);
    hipLaunchKernelGGL(cl_init_kernel, b1, t1, 0, st_, parent, best_nu, best_key, rep_of_root, n);
    if ((st = launch_status("cl_init_kernel")) != KB_OK) return st;
    const unsigned tiles = (unsigned)((n + CL_TILE - 1) / CL_TILE);
    hipLaunchKernelGGL(cl_pairs_kernel, dim3(tiles, tiles), dim3(CL_TILE), 0, st_, hits, n, dvel,
                       (int)n_vel, s, eps * eps, parent);
    if ((st = launch_status("cl_pairs_kernel")) != KB_OK) return st;
    hipLaunchKernelGGL(cl_flatten_kernel, b1, t1, 0, st_, parent, n);
    if ((st = launch_status("cl_flatten_kernel")) != KB_OK) return st;
    hipLaunchKernelGGL(cl_best_nu_kernel, b1, t1, 0, st_, hits, parent, best_nu, n);
    if ((st = launch_status("cl_best_nu_kernel")) != KB_OK) return st;
    hipLaunchKernelGGL(cl_best_key_kernel, b1, t1, 0, st_, hits, parent, best_nu, best_key, n);
    if ((st = launch_status("cl_best_key_kernel")) != KB_OK) return st;
    hipLaunchKernelGGL(cl_rep_kernel, b1, t1, 0, st_, hits, parent, best_nu, best_key,
                       rep_of_root, n);
    if ((st = launch_status("cl_rep_kernel")) != KB_OK) return st;
    hipLaunchKernelGGL(cl_out_kernel, b1, t1, 0, st_, parent, rep_of_root, rep, n);
    return launch_status("cl_out_kernel");
}

}  // extern "C"
