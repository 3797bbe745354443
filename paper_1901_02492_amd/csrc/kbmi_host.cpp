// Host-side part of libkbmi: error reporting, argument checks and the
// displacement table (Sec. 2.2 linear trajectories started at the earliest
// image).  Built with -ffp-contract=off: the product v * tau, the sum with 0.5
// and the floor must stay three separately rounded IEEE double operations so
// that every offset equals the documented definition bit for bit.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "kbmi_internal.h"

namespace kbmi {

static thread_local std::string g_last_error;

kb_status fail(kb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_error() { g_last_error.clear(); }

static constexpr double kMaxOffset = 1073741824.0;  // 2^30

kb_status check_times_velocities(const double *t, int64_t n_img, const double *vel,
                                 int64_t n_vel) {
    if (!t || !vel) return fail(KB_EINVAL, "t and vel must be non-null host arrays");
    if (n_img < 1) return fail(KB_EINVAL, "n_img must be >= 1 (got %lld)", (long long)n_img);
    if (n_vel < 1) return fail(KB_EINVAL, "n_vel must be >= 1 (got %lld)", (long long)n_vel);
    for (int64_t i = 0; i < n_img; ++i) {
        if (!std::isfinite(t[i])) return fail(KB_EINVAL, "t[%lld] is not finite", (long long)i);
        if (i > 0 && t[i] < t[i - 1])
            return fail(KB_EINVAL, "times must be non-decreasing (t[%lld] < t[%lld])",
                        (long long)i, (long long)(i - 1));
    }
    const double tau_max = t[n_img - 1] - t[0];
    if (!std::isfinite(tau_max)) return fail(KB_EINVAL, "time span is not finite");
    for (int64_t j = 0; j < n_vel; ++j) {
        for (int a = 0; a < 2; ++a) {
            const double v = vel[2 * j + a];
            if (!std::isfinite(v))
                return fail(KB_EINVAL, "vel[%lld][%d] is not finite", (long long)j, a);
            if (std::fabs(v) * tau_max >= kMaxOffset)
                return fail(KB_EINVAL, "|vel[%lld][%d] * time span| must be < 2^30",
                            (long long)j, a);
        }
    }
    return KB_OK;
}

// floor(v * tau + 0.5) as a separately rounded product, sum and floor,
// clamped to [-clamp, clamp] when clamp > 0.
static int32_t offset_of(double v, double tau, int64_t clamp) {
    volatile double prod = v * tau;        // rounded product
    volatile double shifted = prod + 0.5;  // rounded sum
    int64_t d = static_cast<int64_t>(std::floor(shifted));
    if (clamp > 0) d = d < -clamp ? -clamp : (d > clamp ? clamp : d);
    return static_cast<int32_t>(d);
}

void displacement_table(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
                        int32_t *disp, int64_t clamp_w, int64_t clamp_h) {
    const double t0 = t[0];
    for (int64_t j = 0; j < n_vel; ++j) {
        for (int64_t i = 0; i < n_img; ++i) {
            const double tau = t[i] - t0;
            disp[(j * n_img + i) * 2] = offset_of(vel[2 * j], tau, clamp_w);
            disp[(j * n_img + i) * 2 + 1] = offset_of(vel[2 * j + 1], tau, clamp_h);
        }
    }
}

void dy_extent(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
               int64_t clamp_h, int32_t out[2]) {
    int32_t lo = 0, hi = 0;
    for (int64_t j = 0; j < n_vel; ++j)
        for (int64_t i = 0; i < n_img; ++i) {
            const int32_t d = offset_of(vel[2 * j + 1], t[i] - t[0], clamp_h);
            lo = std::min(lo, d);
            hi = std::max(hi, d);
        }
    out[0] = lo;
    out[1] = hi;
}

#ifndef KBMI_HILBERT_ORDER
#define KBMI_HILBERT_ORDER 1
#endif

void velocity_order(const double *vel, int64_t n_vel, int32_t *order) {
    if (!KBMI_HILBERT_ORDER) {
        for (int64_t j = 0; j < n_vel; ++j) order[j] = static_cast<int32_t>(j);
        return;
    }
    double lo[2] = {vel[0], vel[1]}, hi[2] = {vel[0], vel[1]};
    for (int64_t j = 1; j < n_vel; ++j)
        for (int a = 0; a < 2; ++a) {
            lo[a] = std::min(lo[a], vel[2 * j + a]);
            hi[a] = std::max(hi[a], vel[2 * j + a]);
        }
    std::vector<std::pair<uint32_t, int32_t>> keyed(static_cast<size_t>(n_vel));
    for (int64_t j = 0; j < n_vel; ++j) {
        keyed[static_cast<size_t>(j)] = {hilbert_key(vel[2 * j], vel[2 * j + 1], lo, hi),
                                         static_cast<int32_t>(j)};
    }
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const auto &a, const auto &b) { return a.first < b.first; });
    for (int64_t j = 0; j < n_vel; ++j) order[j] = keyed[static_cast<size_t>(j)].second;
}

size_t order_bytes(int64_t n_vel) {
    const size_t raw = static_cast<size_t>(n_vel) * sizeof(int32_t);
    return (raw + 255) & ~static_cast<size_t>(255);
}

int64_t table_stride(int64_t n_img) { return (n_img + 15) / 16 * 16; }

static size_t align256(size_t n) { return (n + 255) & ~static_cast<size_t>(255); }

WorkspaceLayout workspace_layout(int64_t n_img, int64_t h, int64_t w, int64_t n_vel) {
    WorkspaceLayout l;
    l.table = 0;
    l.order = l.table + table_bytes(n_img, n_vel);
    l.inv_scale = l.order + order_bytes(n_vel);
    l.sync = l.inv_scale + align256(static_cast<size_t>(table_stride(n_img)) * 8);
    l.total = l.sync + 256;
    (void)h;
    (void)w;
    return l;
}

size_t table_bytes(int64_t n_img, int64_t n_vel) {
    const size_t raw = static_cast<size_t>(table_stride(n_img)) * static_cast<size_t>(n_vel) *
                       sizeof(GatherEntry);
    return (raw + 255) & ~static_cast<size_t>(255);
}

void gather_table(const double *t, int64_t n_img, const double *vel, int64_t n_vel, int64_t h,
                  int64_t w, int64_t pix_bytes, bool visiting_order, GatherEntry *table,
                  int32_t *order) {
    if (visiting_order)
        velocity_order(vel, n_vel, order);
    else
        for (int64_t j = 0; j < n_vel; ++j) order[j] = static_cast<int32_t>(j);
    std::vector<double> vel_visit(static_cast<size_t>(n_vel) * 2);
    for (int64_t j = 0; j < n_vel; ++j) {
        vel_visit[2 * j] = vel[2 * order[j]];
        vel_visit[2 * j + 1] = vel[2 * order[j] + 1];
    }
    std::vector<int32_t> dense(static_cast<size_t>(n_img) * n_vel * 2);
    displacement_table(t, n_img, vel_visit.data(), n_vel, dense.data(), w, h);
    // Padding entries (w, h): row + h is outside the frame for every start row,
    // and column x0 + w is outside it for every start column, so a padding
    // entry reads nothing whether a load's buffer covers its row or not.
    const int64_t stride = table_stride(n_img);
    const int64_t row_bytes = w * pix_bytes, image_bytes = h * row_bytes;
    for (int64_t j = 0; j < n_vel; ++j)
        for (int64_t i = 0; i < stride; ++i) {
            GatherEntry &e = table[j * stride + i];
            if (i < n_img) {
                e.dx = dense[(j * n_img + i) * 2];
                e.dy = dense[(j * n_img + i) * 2 + 1];
                e.offset = i * image_bytes + static_cast<int64_t>(e.dy) * row_bytes;
            } else {
                e.dx = static_cast<int32_t>(w);
                e.dy = static_cast<int32_t>(h);
                e.offset = 0;
            }
        }
}

}  // namespace kbmi

extern "C" {

int kb_abi_version(void) { return KB_ABI_VERSION; }

const char *kb_last_error(void) { return kbmi::g_last_error.c_str(); }

kb_status kb_displacements(const double *t, int64_t n_img, const double *vel, int64_t n_vel,
                           int32_t *disp) {
    kbmi::clear_error();
    kb_status st = kbmi::check_times_velocities(t, n_img, vel, n_vel);
    if (st != KB_OK) return st;
    if (!disp) return kbmi::fail(KB_EINVAL, "disp must be a non-null host array");
    kbmi::displacement_table(t, n_img, vel, n_vel, disp, 0, 0);
    return KB_OK;
}

size_t kb_search_workspace_bytes(int64_t n_img, int64_t h, int64_t w, int64_t n_vel) {
    if (n_img < 1 || n_vel < 1 || h < 1 || w < 1) return 0;
    return kbmi::workspace_layout(n_img, h, w, n_vel).total;
}

}  // extern "C"
