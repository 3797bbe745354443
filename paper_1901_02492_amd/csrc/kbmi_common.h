// Host helpers of the entry points and device helpers shared by the plane,
// top-k and filter translation units (not the search kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "kbmi_internal.h"

namespace kbmi {

kb_status launch_status(const char *what);

// Host helpers defined in kbmi_kernels.hip.
// Frame limits common to every kernel: 1 <= n_img <= 32767, h <= 2^30, w <= 2^27.
kb_status check_frame(int64_t n_img, int64_t h, int64_t w);
// Asynchronous host-to-device copy through a pinned staging buffer (the call
// does not wait for its stream).
kb_status staged_copy(void *dst, const void *src, size_t bytes, hipStream_t stream);
// Send tau_i = t_i - t_0 (double [n_img], at the workspace start) and the
// velocities (double2 [n_vel], at byte offset *vel_off, 16-byte aligned) to
// the workspace, for kernels that compute displacements on the device.
kb_status upload_tau_vel(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
                         void *workspace, hipStream_t stream, size_t *vel_off);
// Send the gather table (planes of `pix_bytes` bytes per pair; velocities in
// visiting order unless visiting_order is false) and the visiting order to
// the workspace (workspace_layout offsets).
// If dy_range is given it receives the smallest and largest row displacement
// of the table's real entries.
kb_status upload_table(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
                       int64_t h, int64_t w, int64_t pix_bytes, void *workspace,
                       hipStream_t stream, bool visiting_order = true,
                       int32_t *dy_range = nullptr);

// Argument checks of kb_search (and its allocation-free variant).
kb_status check_search_args(const void *planes, int32_t dtype, const float *lp_scale,
                            int64_t n_img, int64_t h, int64_t w, const double *t,
                            const double *vel, int64_t n_vel, int64_t k_cand,
                            const void *cand_nu, const void *cand_alpha, const void *cand_vel,
                            const void *cand_nobs);
// Enqueue the search on checked arguments whose tables are already in
// `workspace` (workspace_layout offsets; the inverse scales of 16-bit planes
// are written here): dy_range is the smallest and largest row displacement of
// the table's real entries.
kb_status launch_search_in(const void *planes, int32_t dtype, const float *lp_scale,
                           int64_t n_img, int64_t h, int64_t w, int64_t n_vel, int64_t k_cand,
                           float *cand_nu, float *cand_alpha, int32_t *cand_vel,
                           int16_t *cand_nobs, void *workspace, const int32_t dy_range[2],
                           hipStream_t s);

// One displacement on the device: floor(v * tau + 0.5) as a separate IEEE
// double multiply, add and floor (no contraction), clamped to [-lim, lim],
// which rounds exactly as the host table does.
__device__ inline int displacement(double v, double tau, int lim) {
#pragma clang fp contract(off)
    const double f = floor(v * tau + 0.5);
    return (int)fmin(fmax(f, -(double)lim), (double)lim);
}

}  // namespace kbmi
