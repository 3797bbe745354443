// Threshold mode and duplicate clustering of libkbmi.
//
//   search_threshold_kernel  every trajectory whose nu reaches a threshold
//                            (Sec. 2.2; Sec. 3.2 keeps nu >= 10), appended
//                            to a device list by wave-wide compaction
//   cluster kernels          groups of hits within eps in (x, y, s*vx, s*vy)
//                            (DBSCAN with min_samples = 1, Sec. 3.3) by
//                            lock-free union-find, and each group's best hit
//
// The threshold search runs the top-k search's own gathers (visit_velocities:
// same table, loads, image order) and score functions, so a hit's nu, alpha
// and n_obs are bitwise the values the top-k path gives that trajectory.  It
// keeps no list, so it needs few registers; it runs in the top-k search's
// paced persistent order with two batches' gathers in flight.
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

// One tile: 64 adjacent start pixels of one row, every velocity, with the
// top-k search's gathers (visit_velocities); each trajectory is scored and
// appended if nu >= nu_min: one atomic per wave reserves the wave's slots.
template <bool MB, bool INTERIOR>
__device__ __forceinline__ void threshold_tile(
    const float2 *__restrict__ planes, int n_img, int h, int w,
    const GatherEntry *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
    int n_vel, int row, int seg, float nu_min, kb_hit *__restrict__ hits, uint64_t cap,
    unsigned long long *__restrict__ n_hits) {
    const int lane = (int)threadIdx.x;
    const int x0 = seg * 64 + lane;
    const uint64_t below = (uint64_t(1) << lane) - 1;
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
                hit.alpha = score_alpha(P, nu, F, r);
                hit.nobs = (int16_t)c;
                hit.reserved = 0;
                hits[idx] = hit;
            }
        }
    };
    visit_velocities<TH_NB, KB_F32, true, true, MB, INTERIOR, false>(
        nullptr, planes, nullptr, n_img, h, w, disp, disp_stride, vel_index, n_vel, row, seg,
        finish);
}

// Strip tile order, one wave per tile.
template <bool MB>
__global__ __launch_bounds__(64) void search_threshold_kernel(
    const float2 *__restrict__ planes, int n_img, int h, int w,
    const GatherEntry *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
    int n_vel, int nseg, int ntiles, float nu_min, kb_hit *__restrict__ hits, uint64_t cap,
    unsigned long long *__restrict__ n_hits, int row_lo, int row_hi) {
    int row, seg;
    strip_tile(xcd_remap((int)blockIdx.x, ntiles), nseg, h, TH_STRIP, row, seg);
    if (KBMI_INTERIOR && row >= row_lo && row < row_hi)
        threshold_tile<MB, true>(planes, n_img, h, w, disp, disp_stride, vel_index, n_vel, row,
                                 seg, nu_min, hits, cap, n_hits);
    else
        threshold_tile<MB, false>(planes, n_img, h, w, disp, disp_stride, vel_index, n_vel, row,
                                  seg, nu_min, hits, cap, n_hits);
}

// The paced persistent order of the float32 top-k search: per generation each
// XCD covers one block of start pixels and its waves wait (a bounded time) for
// each other at the end of the generation, so that their gathers share the
// XCD's L2.  The wait only shapes timing.
template <bool MB>
__global__ __launch_bounds__(64) void search_threshold_persistent_kernel(
    const float2 *__restrict__ planes, int n_img, int h, int w,
    const GatherEntry *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
    int n_vel, PersistMap pm, float nu_min, kb_hit *__restrict__ hits, uint64_t cap,
    unsigned long long *__restrict__ n_hits, uint32_t *sync, int row_lo, int row_hi) {
    uint32_t *xcd_count = sync + (blockIdx.x & 7);
    const uint32_t per_xcd = gridDim.x >> 3;
    int spin = pm.spin;
    for (int gen = 0; gen < pm.generations; ++gen) {
        int row, seg;
        if (pm.map(gen, (int)blockIdx.x, row, seg)) {
            if (KBMI_INTERIOR && row >= row_lo && row < row_hi)
                threshold_tile<MB, true>(planes, n_img, h, w, disp, disp_stride, vel_index,
                                         n_vel, row, seg, nu_min, hits, cap, n_hits);
            else
                threshold_tile<MB, false>(planes, n_img, h, w, disp, disp_stride, vel_index,
                                          n_vel, row, seg, nu_min, hits, cap, n_hits);
        }
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

template <bool MB>
int threshold_grid() {
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, search_threshold_persistent_kernel<MB>, 64, 0) != hipSuccess ||
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
constexpr int CL_THREADS = 256;

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

// Pairs are found through a grid of cells of side c = eps (1 + 2^-20) over
// the four coordinates (x, y, u, v), u = s * vx, v = s * vy: two hits within
// distance eps differ by at most eps in every coordinate, so their cells
// differ by at most one in every coordinate, and each hit only meets the hits
// of its own and the 80 neighbouring cells.  The cells sit in an
// open-addressing hash table (cell key -> list of the cell's hits).  Pair
// (i, j), i < j, is joined when d2 <= eps2 with
// d2 = ((dx*dx + dy*dy) + du*du) + dv*dv in double.  A hit whose velocity
// index is outside the grid gets no cell: it stays a group of its own.
__device__ inline double2 cl_vel(const double2 *vel, int n_vel, int j) {
    return (unsigned)j < (unsigned)n_vel ? vel[j] : make_double2(NAN, NAN);
}

constexpr uint64_t kEmptyCell = ~0ull;

__device__ inline int64_t cl_cell(double coord, double inv_c) {
#pragma clang fp contract(off)
    const double q = floor(coord * inv_c);
    return (int64_t)fmin(fmax(q, -4.0e18), 4.0e18);
}

// 64-bit key of cell (a, b, c, d) (a finalising mix of a packed sum; distinct
// cells may share a key, which only adds hits whose distance is then tested).
__device__ inline uint64_t cl_cell_key(int64_t a, int64_t b, int64_t c, int64_t d) {
    uint64_t z = (uint64_t)a * 0x9E3779B97F4A7C15ull + (uint64_t)b * 0xC2B2AE3D27D4EB4Full +
                 (uint64_t)c * 0x165667B19E3779F9ull + (uint64_t)d * 0xD6E8FEB86659FD93ull;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z == kEmptyCell ? kEmptyCell - 1 : z;
}

struct ClHit {
    double x, y, u, v;
    bool ok;
};

__device__ inline ClHit cl_hit(const kb_hit *hits, const double2 *vel, int n_vel, double s,
                               int i) {
#pragma clang fp contract(off)
    const kb_hit h = hits[i];
    const double2 vj = cl_vel(vel, n_vel, h.vel);
    ClHit r;
    r.x = (double)h.x;
    r.y = (double)h.y;
    r.u = s * vj.x;
    r.v = s * vj.y;
    r.ok = (unsigned)h.vel < (unsigned)n_vel;
    return r;
}

__global__ void cl_table_init_kernel(uint64_t *table_key, int32_t *table_head, int64_t slots) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < slots;
         i += (int64_t)gridDim.x * blockDim.x) {
        table_key[i] = kEmptyCell;
        table_head[i] = -1;
    }
}

// Hit i joins the list of its cell (pushed at the head; the lists are read by
// the next kernel only).
__global__ __launch_bounds__(CL_THREADS) void cl_insert_kernel(
    const kb_hit *__restrict__ hits, int n, const double2 *__restrict__ vel, int n_vel, double s,
    double inv_c, uint64_t *table_key, int32_t *table_head, uint64_t mask,
    int32_t *__restrict__ next) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const ClHit h = cl_hit(hits, vel, n_vel, s, i);
    next[i] = -1;
    if (!h.ok) return;
    const uint64_t key = cl_cell_key(cl_cell(h.x, inv_c), cl_cell(h.y, inv_c),
                                     cl_cell(h.u, inv_c), cl_cell(h.v, inv_c));
    uint64_t slot = key & mask;
    for (;;) {
        const uint64_t prev = atomicCAS(reinterpret_cast<unsigned long long *>(table_key + slot),
                                        (unsigned long long)kEmptyCell,
                                        (unsigned long long)key);
        if (prev == kEmptyCell || prev == key) {
            next[i] = atomicExch(table_head + slot, i);
            return;
        }
        slot = (slot + 1) & mask;   // the table has at least twice as many slots as hits
    }
}

__global__ __launch_bounds__(CL_THREADS) void cl_grid_pairs_kernel(
    const kb_hit *__restrict__ hits, int n, const double2 *__restrict__ vel, int n_vel, double s,
    double inv_c, double eps2, const uint64_t *__restrict__ table_key,
    const int32_t *__restrict__ table_head, uint64_t mask, const int32_t *__restrict__ next,
    int32_t *parent) {
#pragma clang fp contract(off)
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const ClHit hi = cl_hit(hits, vel, n_vel, s, i);
    if (!hi.ok) return;
    const int64_t c0 = cl_cell(hi.x, inv_c), c1 = cl_cell(hi.y, inv_c);
    const int64_t c2 = cl_cell(hi.u, inv_c), c3 = cl_cell(hi.v, inv_c);
    for (int o = 0; o < 81; ++o) {
        const int d0 = o % 3 - 1, d1 = (o / 3) % 3 - 1, d2c = (o / 9) % 3 - 1, d3 = o / 27 - 1;
        const uint64_t key = cl_cell_key(c0 + d0, c1 + d1, c2 + d2c, c3 + d3);
        uint64_t slot = key & mask;
        for (;;) {
            const uint64_t k = table_key[slot];
            if (k == kEmptyCell) break;
            if (k == key) {
                for (int j = table_head[slot]; j >= 0; j = next[j]) {
                    if (j <= i) continue;
                    const ClHit hj = cl_hit(hits, vel, n_vel, s, j);
                    const double dx = hi.x - hj.x, dy = hi.y - hj.y, du = hi.u - hj.u,
                                 dv = hi.v - hj.v;
                    const double dd = ((dx * dx + dy * dy) + du * du) + dv * dv;
                    if (dd <= eps2) cl_unite(parent, i, j);
                }
                break;
            }
            slot = (slot + 1) & mask;
        }
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
    size_t parent, best_nu, best_key, rep_of_root, vel, next, table_key, table_head, total;
    uint64_t slots;   // hash-table slots: a power of two >= 2 * n_hits
};

ClusterLayout cluster_layout(int64_t n_hits, int64_t n_vel) {
    ClusterLayout l{};
    const size_t n = static_cast<size_t>(n_hits);
    l.slots = 64;
    while (l.slots < 2 * static_cast<uint64_t>(n)) l.slots <<= 1;
    l.parent = 0;
    l.best_nu = l.parent + r256(n * sizeof(int32_t));
    l.best_key = l.best_nu + r256(n * sizeof(uint32_t));
    l.rep_of_root = l.best_key + r256(n * sizeof(uint64_t));
    l.vel = l.rep_of_root + r256(n * sizeof(int32_t));
    l.next = l.vel + r256(static_cast<size_t>(n_vel) * 2 * sizeof(double));
    l.table_key = l.next + r256(n * sizeof(int32_t));
    l.table_head = l.table_key + r256(l.slots * sizeof(uint64_t));
    l.total = l.table_head + r256(l.slots * sizeof(int32_t));
    return l;
}

template <bool MB>
kb_status launch_threshold(const float *psi_phi, int64_t n_img, int64_t h, int64_t w,
                           int64_t n_vel, float nu_min, kb_hit *hits, int64_t max_hits,
                           uint64_t *n_hits, void *workspace, int row_lo, int row_hi,
                           hipStream_t s) {
    char *ws = static_cast<char *>(workspace);
    const WorkspaceLayout lay = workspace_layout(n_img, h, w, n_vel);
    const int nseg = (int)((w + 63) / 64);
    const int64_t ntiles = (int64_t)nseg * h;
    const int grid = KBMI_TH_PERSIST ? threshold_grid<MB>() : 0;
    const int per_xcd = grid / 8;
    const GatherEntry *disp = reinterpret_cast<const GatherEntry *>(ws + lay.table);
    const int32_t *order = reinterpret_cast<const int32_t *>(ws + lay.order);
    if (grid >= 8 && grid % 8 == 0 && per_xcd % KBMI_PERSIST_BS == 0 &&
        ntiles >= 4 * (int64_t)grid) {
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
        kb_status st = launch_status("zero_words_kernel");
        if (st != KB_OK) return st;
        hipLaunchKernelGGL(search_threshold_persistent_kernel<MB>, dim3((unsigned)grid), dim3(64),
                           0, s, reinterpret_cast<const float2 *>(psi_phi), (int)n_img, (int)h,
                           (int)w, disp, (int)table_stride(n_img), order, (int)n_vel, pm, nu_min,
                           hits, (uint64_t)max_hits,
                           reinterpret_cast<unsigned long long *>(n_hits), sync, row_lo, row_hi);
        return launch_status("search_threshold_persistent_kernel");
    }
    hipLaunchKernelGGL(search_threshold_kernel<MB>, dim3((unsigned)ntiles), dim3(64), 0, s,
                       reinterpret_cast<const float2 *>(psi_phi), (int)n_img, (int)h, (int)w,
                       disp, (int)table_stride(n_img), order, (int)n_vel, nseg, (int)ntiles,
                       nu_min, hits, (uint64_t)max_hits,
                       reinterpret_cast<unsigned long long *>(n_hits), row_lo, row_hi);
    return launch_status("search_threshold_kernel");
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
    int32_t dy_range[2] = {0, 0};
    st = upload_table(t, n_img, vel, n_vel, h, w, 8, workspace, s, true, dy_range);
    if (st != KB_OK) return st;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<unsigned long long *>(n_hits));
    st = launch_status("zero_u64_kernel");
    if (st != KB_OK) return st;
    // Start rows whose displaced rows are all inside the frame.
    const int row_lo = (int)std::min<int64_t>(h, -(int64_t)dy_range[0]);
    const int row_hi = (int)std::max<int64_t>(0, h - (int64_t)dy_range[1]);
    return n_img > TH_NB
               ? launch_threshold<true>(psi_phi, n_img, h, w, n_vel, nu_min, hits, max_hits,
                                        n_hits, workspace, row_lo, row_hi, s)
               : launch_threshold<false>(psi_phi, n_img, h, w, n_vel, nu_min, hits, max_hits,
                                         n_hits, workspace, row_lo, row_hi, s);
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
    if (n_hits > (int64_t(1) << 30))
        return fail(KB_EUNSUPPORTED, "at most 2^30 hits per call");
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
    uint64_t *table_key = reinterpret_cast<uint64_t *>(ws + lay.table_key);
    int32_t *table_head = reinterpret_cast<int32_t *>(ws + lay.table_head);
    int32_t *next = reinterpret_cast<int32_t *>(ws + lay.next);
    const uint64_t mask = lay.slots - 1;
    // Cells slightly wider than eps, so that rounding in coordinate / side
    // never separates two hits at distance eps by two cells (eps = 0: cells
    // of side 1; only identical hits join).
    const double side = eps > 0.0 ? eps * (1.0 + 0x1p-20) : 1.0;
    const double inv_c = 1.0 / side;
    hipLaunchKernelGGL(cl_table_init_kernel, dim3(2048), dim3(256), 0, st_, table_key, table_head,
                       (int64_t)lay.slots);
    if ((st = launch_status("cl_table_init_kernel")) != KB_OK) return st;
    hipLaunchKernelGGL(cl_insert_kernel, b1, dim3(CL_THREADS), 0, st_, hits, n, dvel, (int)n_vel,
                       s, inv_c, table_key, table_head, mask, next);
    if ((st = launch_status("cl_insert_kernel")) != KB_OK) return st;
    hipLaunchKernelGGL(cl_grid_pairs_kernel, b1, dim3(CL_THREADS), 0, st_, hits, n, dvel,
                       (int)n_vel, s, inv_c, eps * eps, table_key, table_head, mask, next, parent);
    if ((st = launch_status("cl_grid_pairs_kernel")) != KB_OK) return st;
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
