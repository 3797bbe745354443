// Trajectory-search launchers for one plane format (KBMI_FMT: 0 = float32,
// 1 = IEEE half, 2 = bfloat16) and one group of list lengths (KBMI_GROUP);
// the build compiles this file once per (format, group).
#include <algorithm>

#include "kbmi_device.h"

#ifndef KBMI_FMT
#error "compile with -DKBMI_FMT=0|1|2"
#endif
#ifndef KBMI_GROUP
#error "compile with -DKBMI_GROUP=0..7"
#endif

namespace kbmi {
namespace {

TileMap tile_map(int w, int h) {
    TileMap tm;
    tm.nseg = (w + 63) / 64;
    tm.h = h;
    tm.strip = tm.nseg < KBMI_STRIP_TILES ? tm.nseg : KBMI_STRIP_TILES;
    tm.nblocks = tm.nseg * h;
    tm.sw = (KBMI_SUPER_W > 0 && tm.nseg % (8 * KBMI_SUPER_W) == 0) ? KBMI_SUPER_W : 0;
    return tm;
}

// Workgroups of the persistent grid for `Kernel` (0 if unknown): the number
// the device holds at once, at most KBMI_PERSIST_PER_CU per CU, cached per
// device and per kernel instance.  The cap keeps each XCD's block of start
// pixels small enough for its L2 when a short candidate list lets more waves
// fit.
template <auto Kernel>
int resident_workgroups() {
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, Kernel, 64, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess)
            return 0;
        cached[dev] = std::min(per_cu, KBMI_PERSIST_PER_CU) * cus;
    }
    return cached[dev];
}

template <int KM, int NB, bool MB>
kb_status launch_one(const StackView &v, hipStream_t s) {
    constexpr int PB = KBMI_QUEUE;
    static_assert(NB == 8 || NB == 16, "table rows are padded for batches of 8 or 16");
    // The persistent order pays where gathers dominate (float32 planes); the
    // 16-bit search keeps the super-strip order, which measured faster (60 ms
    // against 76 ms on a 15 x 4096^2 stack at 600 velocities, K = 50).
    if (KBMI_PERSIST_BS > 0 && (KBMI_FMT == KB_F32 || KBMI_PERSIST_LP)) {
        auto kernel = search_persistent_kernel<KM, NB, PB, KBMI_FMT, MB>;
        const int grid =
            resident_workgroups<search_persistent_kernel<KM, NB, PB, KBMI_FMT, MB>>();
        const int nseg = (v.w + 63) / 64;
        const int per_xcd = grid / 8;
        // Worth it only when the frame holds several generations of blocks.
        if (grid >= 8 && grid % 8 == 0 && per_xcd % KBMI_PERSIST_BS == 0 &&
            (int64_t)nseg * v.h >= 4 * (int64_t)grid) {
            PersistMap pm;
            pm.nseg = nseg;
            pm.h = v.h;
            pm.bs = KBMI_PERSIST_BS;
            pm.brows = per_xcd / KBMI_PERSIST_BS;
            pm.nbc = (nseg + pm.bs - 1) / pm.bs;
            pm.nbr = (v.h + pm.brows - 1) / pm.brows;
            pm.generations = (pm.nbc + 7) / 8 * pm.nbr;
            pm.spin = KBMI_PERSIST_SPIN;
            hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, v.sync, 8);
            kb_status st = launch_status("zero_words_kernel");
            if (st != KB_OK) return st;
            hipLaunchKernelGGL(kernel, dim3(grid), dim3(64), 0, s, v.planes, v.inv_scale,
                               v.n_img, v.h, v.w, v.disp, v.disp_stride, v.vel_index, v.n_vel,
                               v.k_cand, pm, v.cand_nu, v.cand_alpha, v.cand_vel, v.cand_nobs,
                               v.sync, v.row_lo, v.row_hi);
            return launch_status("search_persistent_kernel");
        }
    }
    const TileMap tm = tile_map(v.w, v.h);
    hipLaunchKernelGGL((search_kernel<KM, NB, PB, KBMI_FMT, MB>), dim3(tm.nblocks), dim3(64), 0, s,
                       v.planes, v.inv_scale, v.n_img, v.h, v.w, v.disp, v.disp_stride,
                       v.vel_index, v.n_vel, v.k_cand, tm, v.cand_nu, v.cand_alpha, v.cand_vel,
                       v.cand_nobs, v.row_lo, v.row_hi);
    return launch_status("search_kernel");
}

template <int KM>
kb_status launch_km(const StackView &v, hipStream_t s) {
    // One batch of 8 or 16 loads per velocity, or batches of 16 (MB).
    if (v.n_img <= 8) return launch_one<KM, 8, false>(v, s);
    if (v.n_img <= 16) return launch_one<KM, 16, false>(v, s);
    return launch_one<KM, 16, true>(v, s);
}

template <int KM, int NB, bool MB>
kb_status launch_batch_one(const BatchJob *jobs, int n_jobs, int k_cand, int generations,
                           uint32_t *sync, int *grid, hipStream_t s) {
    constexpr int PB = KBMI_QUEUE;
    auto kernel = search_batch_kernel<KM, NB, PB, KBMI_FMT, MB>;
    const int g = resident_workgroups<search_batch_kernel<KM, NB, PB, KBMI_FMT, MB>>();
    if (g < 8 || g % 8 != 0)
        return fail(KB_EDEVICE, "batched search: no persistent grid for this device (%d)", g);
    if (!jobs) {
        *grid = g;
        return KB_OK;
    }
    if (*grid != g) return fail(KB_EDEVICE, "batched search: grid changed (%d, %d)", *grid, g);
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, sync, 8);
    kb_status st = launch_status("zero_words_kernel");
    if (st != KB_OK) return st;
    hipLaunchKernelGGL(kernel, dim3(g), dim3(64), 0, s, jobs, n_jobs, generations,
                       KBMI_PERSIST_SPIN, k_cand, sync);
    return launch_status("search_batch_kernel");
}

template <int KM>
kb_status launch_batch_km(const BatchJob *jobs, int n_jobs, int n_img_class, int k_cand,
                          int generations, uint32_t *sync, int *grid, hipStream_t s) {
    if (n_img_class == 0)
        return launch_batch_one<KM, 8, false>(jobs, n_jobs, k_cand, generations, sync, grid, s);
    if (n_img_class == 1)
        return launch_batch_one<KM, 16, false>(jobs, n_jobs, k_cand, generations, sync, grid, s);
    return launch_batch_one<KM, 16, true>(jobs, n_jobs, k_cand, generations, sync, grid, s);
}

// List lengths of this translation unit's group are compiled; the others are
// left to their own units (the dispatcher never sends them here).
template <int K>
kb_status launch_in_group(const StackView &v, hipStream_t s) {
    if constexpr (km_group(K) == KBMI_GROUP) return launch_km<K>(v, s);
    else return fail(KB_EUNSUPPORTED, "list length %d is not compiled in this group", K);
}

template <int K>
kb_status launch_batch_in_group(const BatchJob *jobs, int n_jobs, int n_img_class, int k_cand,
                                int generations, uint32_t *sync, int *grid, hipStream_t s) {
    if constexpr (km_group(K) == KBMI_GROUP)
        return launch_batch_km<K>(jobs, n_jobs, n_img_class, k_cand, generations, sync, grid, s);
    else return fail(KB_EUNSUPPORTED, "list length %d is not compiled in this group", K);
}

}  // namespace

template <>
kb_status launch_search_group<KBMI_FMT, KBMI_GROUP>(int km, const StackView &v, hipStream_t s) {
    switch (km) {
#define KB_CASE(K) \
    case K:        \
        return launch_in_group<K>(v, s);
        KB_SEARCH_KM_LIST(KB_CASE)
#undef KB_CASE
    }
    return fail(KB_EUNSUPPORTED, "k_cand above %d is not supported", KB_MAX_KCAND);
}

template <>
kb_status launch_search_batch_group<KBMI_FMT, KBMI_GROUP>(int km, const BatchJob *jobs,
                                                           int n_jobs, int n_img_class,
                                                           int k_cand, int generations,
                                                           uint32_t *sync, int *grid,
                                                           hipStream_t s) {
    switch (km) {
#define KB_CASE(K)                                                                     \
    case K:                                                                            \
        return launch_batch_in_group<K>(jobs, n_jobs, n_img_class, k_cand, generations, \
                                        sync, grid, s);
        KB_SEARCH_KM_LIST(KB_CASE)
#undef KB_CASE
    }
    return fail(KB_EUNSUPPORTED, "k_cand above %d is not supported", KB_MAX_KCAND);
}

}  // namespace kbmi
