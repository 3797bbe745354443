// Declarations shared by the host-side helpers and the HIP launchers of libkbmi.
#pragma once

#include <cstddef>
#include <cstdint>

#include "kbmi.h"

namespace kbmi {

// Record the message kb_last_error() returns on this thread; returns `st`.
kb_status fail(kb_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// Checks shared by kb_displacements, kb_search and kb_topk: times finite and
// non-decreasing, velocities finite, every |v * (t_i - t_0)| < 2^30.
kb_status check_times_velocities(const double *t, int64_t n_img, const double *vel,
                                 int64_t n_vel);

// Displacement table d[j][i] = (floor(vx_j tau_i + 0.5), floor(vy_j tau_i + 0.5)),
// tau_i = t_i - t_0, as separate IEEE double operations.  With clamp_w > 0 and
// clamp_h > 0 each offset is clamped to [-clamp, clamp]: an offset at least a
// frame extent long puts every start pixel outside the frame either way, and the
// clamp keeps byte offsets inside 32 bits.  Arguments must already be checked.
void displacement_table(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
                        int32_t *disp, int64_t clamp_w, int64_t clamp_h);

// Order in which the search visits the velocities: along a Hilbert curve over
// the (vx, vy) bounding box, so consecutive velocities shift every image's
// gather window by little and neighbouring workgroups reuse cached rows.  Any
// order gives the same result (ranking uses the original index).
void velocity_order(const double *vel, int64_t n_vel, int32_t *order);

// Device workspace layout: the clamped displacement table in visiting order at
// offset 0, one row of table_stride(n_img) (dx, dy) pairs per velocity (a
// multiple of 16; the rows are padded with entries that lie outside the frame
// so that the search can fetch whole batches of 8 or 16 with wide scalar
// loads), then the original index of each visited velocity (int32 [n_vel]).
int64_t table_stride(int64_t n_img);
size_t table_bytes(int64_t n_img, int64_t n_vel);
size_t order_bytes(int64_t n_vel);
// Whole workspace of kb_search / kb_topk (byte offsets, 256-byte aligned): the
// table, the visiting order and the 16-bit search's per-image inverse scales
// (float2 [table_stride]).
struct WorkspaceLayout {
    size_t table, order, inv_scale, total;
};
WorkspaceLayout workspace_layout(int64_t n_img, int64_t h, int64_t w, int64_t n_vel);

}  // namespace kbmi
