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

// Smallest and largest row offset floor(vy * tau_i + 0.5) (clamped to
// [-clamp_h, clamp_h]) over every velocity and image, with image 0's 0 included.
void dy_extent(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
               int64_t clamp_h, int32_t out[2]);

#if defined(__HIPCC__)
#define KBMI_HD __host__ __device__
#else
#define KBMI_HD
#endif

// Key of a velocity in the visiting order: its index along a Hilbert curve of
// order 16 (rotate-and-flip construction) over the velocities' bounding box
// [lo, hi], each axis quantised to 16 bits.  Host and device compute it with
// the same IEEE operations.
KBMI_HD inline uint32_t hilbert_index(uint32_t x, uint32_t y) {
    uint32_t d = 0;
    for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u;
        const uint32_t ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = (s - 1) - (x & (s - 1)) + (x & ~(s - 1));
                y = (s - 1) - (y & (s - 1)) + (y & ~(s - 1));
            }
            const uint32_t tmp = x;
            x = y;
            y = tmp;
        }
    }
    return d;
}
KBMI_HD inline uint32_t hilbert_key(double vx, double vy, const double lo[2],
                                    const double hi[2]) {
    uint32_t q[2];
    const double v[2] = {vx, vy};
    for (int a = 0; a < 2; ++a) {
        const double span = hi[a] - lo[a];
        const double u = span > 0 ? (v[a] - lo[a]) / span : 0.0;
        const double c = u * 65535.0;
        q[a] = (uint32_t)(c < 0.0 ? 0.0 : (c > 65535.0 ? 65535.0 : c));
    }
    return hilbert_index(q[0], q[1]);
}

// One entry of the search's gather table (16 bytes): the displacement (dx, dy)
// of one image for one velocity, and the byte offset of the displaced row from
// the start row in the planes, image * image_bytes + dy * row_bytes, so that
// the search forms a row address with one 64-bit add.
struct alignas(16) GatherEntry {
    int32_t dx, dy;
    int64_t offset;
};
static_assert(sizeof(GatherEntry) == 16, "gather entries are fetched as 16-byte words");

// Device workspace layout: the gather table at offset 0, one row of
// table_stride(n_img) entries per velocity in visiting order (a multiple of
// 16; rows are padded with entries whose row lies outside the frame, so that
// the search fetches whole batches of 8 or 16 with wide scalar loads, and
// whose column is outside the frame too), then the
// original index of each visited velocity (int32 [n_vel]).
int64_t table_stride(int64_t n_img);
size_t table_bytes(int64_t n_img, int64_t n_vel);
size_t order_bytes(int64_t n_vel);

// Fill `table` (table_bytes(n_img, n_vel) bytes) and `order` (int32 [n_vel])
// for planes of `pix_bytes` bytes per (psi, phi) pair: velocities in visiting
// order (or the given order), offsets clamped to the frame extent.  Arguments
// must already be checked.
void gather_table(const double *t, int64_t n_img, const double *vel, int64_t n_vel, int64_t h,
                  int64_t w, int64_t pix_bytes, bool visiting_order, GatherEntry *table,
                  int32_t *order);
// Whole workspace of kb_search / kb_topk (byte offsets, 256-byte aligned): the
// table, the visiting order, the 16-bit search's per-image inverse scales
// (float2 [table_stride]) and the persistent search's per-XCD generation
// counters (uint32 [8], zeroed by each launch).
struct WorkspaceLayout {
    size_t table, order, inv_scale, sync, total;
};
WorkspaceLayout workspace_layout(int64_t n_img, int64_t h, int64_t w, int64_t n_vel);

}  // namespace kbmi
