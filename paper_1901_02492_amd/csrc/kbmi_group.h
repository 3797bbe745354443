// Grouping of a workgroup's (start pixel, velocity) pairs by velocity, shared
// by the kernels that gather along many candidates' trajectories (the FP32
// re-score of kb_topk and the light-curve filter).  A tile's candidates come
// in pixel order with unrelated velocities, so gathering them in list order
// gives every lane of a load its own cache line.  Sorted by velocity (a
// counting sort in LDS), the lanes of one load mostly share a velocity and
// read adjacent pixels of one plane row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kbmi {

constexpr int GR_THREADS = 256;   // threads of a grouping workgroup
constexpr int GR_BINS = 1024;     // counting-sort bins: one per velocity up to 1024
static_assert(GR_BINS == 4 * GR_THREADS, "the scan takes 4 bins per thread");

// LDS bytes of the grouping state for up to np_max pairs: the bin counts
// (uint32 [GR_BINS]) and 8 scan words; the caller's vj (int32 [np_max]) and
// ord (uint16 [np_max]) arrays come on top.
constexpr size_t group_lds_bytes() { return (size_t)GR_BINS * 4 + 32; }

// Pairs q in [0, np) of this workgroup have velocity index cv[q] (global
// memory); np <= MAXQ * GR_THREADS.  Every thread of the workgroup calls this.
// On return (after a barrier): vj[q] = cv[q] when 0 <= cv[q] < n_vel, else -1;
// ord[0 .. n) lists the valid q grouped by bin j * nb / n_vel
// (nb = min(n_vel, GR_BINS)), bins in increasing order; returns n.
template <int MAXQ>
__device__ inline int group_pairs_by_velocity(const int32_t *__restrict__ cv, int np, int n_vel,
                                              int32_t *vj, uint16_t *ord, uint32_t *bin,
                                              uint32_t *tot) {
    const int t = (int)threadIdx.x;
    const int nb = n_vel < GR_BINS ? n_vel : GR_BINS;
    for (int b = t; b < GR_BINS; b += GR_THREADS) bin[b] = 0u;
    __syncthreads();

    // Count pairs per bin; remember each pair's bin and place within it.
    // The thread's indices are all loaded before the first is used.
    int32_t jv[MAXQ];
#pragma unroll
    for (int r = 0; r < MAXQ; ++r) {
        const int q = t + r * GR_THREADS;
        jv[r] = q < np ? cv[q] : -1;
    }
    uint32_t slot[MAXQ];
#pragma unroll
    for (int r = 0; r < MAXQ; ++r) {
        const int q = t + r * GR_THREADS;
        slot[r] = 0xFFFFFFFFu;
        if (q < np) {
            const int32_t j = jv[r];
            const bool ok = j >= 0 && j < n_vel;
            vj[q] = ok ? j : -1;
            if (ok) {
                const uint32_t b = (uint32_t)(((int64_t)j * nb) / n_vel);
                slot[r] = (b << 16) | atomicAdd(&bin[b], 1u);
            }
        }
    }
    __syncthreads();

    // Exclusive scan of the bin counts: 4 bins per thread, then across lanes
    // and waves.
    {
        uint32_t c4[4], run = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            c4[e] = run;
            run += bin[4 * t + e];
        }
        const int lane = t & 63, wv = t >> 6;
        uint32_t inc = run;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d, 64);
            if (lane >= d) inc += o;
        }
        if (lane == 63) tot[wv] = inc;
        __syncthreads();
        uint32_t base = inc - run;
        for (int v2 = 0; v2 < wv; ++v2) base += tot[v2];
#pragma unroll
        for (int e = 0; e < 4; ++e) bin[4 * t + e] = base + c4[e];
        if (t == GR_THREADS - 1) tot[4] = base + run;   // pairs to process
    }
    __syncthreads();
    const int n_sorted = (int)tot[4];
#pragma unroll
    for (int r = 0; r < MAXQ; ++r)
        if (slot[r] != 0xFFFFFFFFu)
            ord[bin[slot[r] >> 16] + (slot[r] & 0xFFFFu)] = (uint16_t)(t + r * GR_THREADS);
    __syncthreads();
    return n_sorted;
}

}  // namespace kbmi
