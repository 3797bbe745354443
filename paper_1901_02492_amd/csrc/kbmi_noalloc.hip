// kb_search_noalloc: kb_search for callers that cannot allocate memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// allocation).  The workspace kb_search takes from its caller (gather table,
// visiting order, 16-bit inverse scales, pacing counters) lives here in one
// fixed device array, `scratch`, of KB_NOALLOC_SCRATCH_BYTES; nothing is
// allocated, on the device or in pinned host memory.
//
// The host sends the times and velocities to the device through kernel
// arguments (at most 3584 bytes per launch), and the device builds
// the visiting order and the gather table from them: each displacement is
// floor(v * tau + 0.5) as a separate IEEE double multiply, add and floor,
// clamped like the host table, so the table is bit for bit the one kb_search
// sends, and the search kernels are kb_search's own.
//
// Every call on a device shares that device's array and leaves its contents
// behind; calls that overlap on one device (two streams, two host threads)
// race on it.  Calls on one stream are ordered by the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "kbmi_common.h"
#include "kbmi_device.h"

// The fixed device array behind kb_search_noalloc (one copy per device).
static __device__ __align__(256) unsigned char scratch[KB_NOALLOC_SCRATCH_BYTES];

namespace kbmi {
namespace {

// Device address of `scratch` on each device, looked up once per device with
// that device current (each device holds its own copy of the array).  The
// array's name is a host-side stand-in and is never passed to a kernel.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

kb_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(KB_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(KB_EUNSUPPORTED, "device index %d above %d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(KB_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return KB_OK;
}

// ---------------------------------------------------------------------------
// Host-to-device transfer through kernel arguments.
// ---------------------------------------------------------------------------
constexpr int kArgWords = 448;   // 3584 bytes of payload per launch
struct ArgChunk {
    uint64_t w[kArgWords];
};
// Explicit arguments plus the runtime's hidden ones stay within 4 KB.
static_assert(sizeof(ArgChunk) + 16 + 256 <= 4096, "kernel arguments are limited to 4 KB");

__global__ void store_words_kernel(uint64_t *__restrict__ dst, ArgChunk c, int n) {
    const int i = (int)threadIdx.x;
    for (int k = i; k < n; k += (int)blockDim.x) dst[k] = c.w[k];
}

// Copy `n` doubles produced by `value(k)` to dst (device) on `s`.
template <class F>
kb_status send_doubles(double *dst, int64_t n, F value, hipStream_t s) {
    for (int64_t k0 = 0; k0 < n; k0 += kArgWords) {
        const int m = (int)std::min<int64_t>(kArgWords, n - k0);
        ArgChunk c;
        for (int k = 0; k < m; ++k) {
            const double v = value(k0 + k);
            std::memcpy(&c.w[k], &v, 8);
        }
        hipLaunchKernelGGL(store_words_kernel, dim3(1), dim3(256), 0, s,
                           reinterpret_cast<uint64_t *>(dst + k0), c, m);
        const kb_status st = launch_status("store_words_kernel");
        if (st != KB_OK) return st;
    }
    return KB_OK;
}

// ---------------------------------------------------------------------------
// Visiting order and gather table on the device.
// ---------------------------------------------------------------------------
struct Box {
    double lo[2], hi[2];
};

__global__ void hilbert_keys_kernel(const double2 *__restrict__ vel, int n_vel, Box box,
                                    uint32_t *__restrict__ key) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_vel) key[j] = hilbert_key(vel[j].x, vel[j].y, box.lo, box.hi);
}

// order[rank(j)] = j, rank by (key, j): the stable sort of the host order.
__global__ void __launch_bounds__(256) order_kernel(const uint32_t *__restrict__ key, int n_vel,
                                                    int32_t *__restrict__ order) {
    __shared__ uint32_t tile[256];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t kj = j < n_vel ? key[j] : 0u;
    int rank = 0;
    for (int t0 = 0; t0 < n_vel; t0 += 256) {
        __syncthreads();
        const int i = t0 + (int)threadIdx.x;
        tile[threadIdx.x] = i < n_vel ? key[i] : 0u;
        __syncthreads();
        const int m = min(256, n_vel - t0);
        for (int q = 0; q < m; ++q) {
            const uint32_t ki = tile[q];
            rank += (ki < kj || (ki == kj && t0 + q < j)) ? 1 : 0;
        }
    }
    if (j < n_vel) order[rank] = j;
}

// Entry (jj, i) of the gather table: the displacement of image i for the
// jj-th visited velocity and its byte offset; padding entries (i >= n_img)
// are (w, h, 0), outside the frame in both axes.
__global__ void table_kernel(const double *__restrict__ tau, const double2 *__restrict__ vel,
                             const int32_t *__restrict__ order, int n_img, int stride,
                             int n_vel, int h, int w, int64_t row_bytes, int64_t image_bytes,
                             GatherEntry *__restrict__ table) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n_vel * stride) return;
    const int jj = (int)(e / stride), i = (int)(e - (int64_t)jj * stride);
    GatherEntry g;
    if (i < n_img) {
        const double2 v = vel[order[jj]];
        g.dx = displacement(v.x, tau[i], w);
        g.dy = displacement(v.y, tau[i], h);
        g.offset = (int64_t)i * image_bytes + (int64_t)g.dy * row_bytes;
    } else {
        g.dx = w;
        g.dy = h;
        g.offset = 0;
    }
    table[e] = g;
}

size_t align256(size_t n) { return (n + 255) & ~static_cast<size_t>(255); }

}  // namespace
}  // namespace kbmi

using namespace kbmi;

extern "C" {

kb_status kb_search_noalloc(const void *planes, int32_t dtype, const float *lp_scale,
                            int64_t n_img, int64_t h, int64_t w, const double *t,
                            const double *vel, int64_t n_vel, int64_t k_cand, float *cand_nu,
                            float *cand_alpha, int32_t *cand_vel, int16_t *cand_nobs,
                            void *stream) {
    clear_error();
    kb_status st = check_search_args(planes, dtype, lp_scale, n_img, h, w, t, vel, n_vel,
                                     k_cand, cand_nu, cand_alpha, cand_vel, cand_nobs);
    if (st != KB_OK) return st;
    // The search's workspace, then tau [n_img], the velocities [n_vel][2] and
    // their order keys [n_vel].
    const WorkspaceLayout lay = workspace_layout(n_img, h, w, n_vel);
    const size_t tau_off = align256(lay.total);
    const size_t vel_off = align256(tau_off + static_cast<size_t>(n_img) * 8);
    const size_t key_off = align256(vel_off + static_cast<size_t>(n_vel) * 16);
    const size_t need = align256(key_off + static_cast<size_t>(n_vel) * 4);
    if (need > static_cast<size_t>(KB_NOALLOC_SCRATCH_BYTES))
        return fail(KB_EUNSUPPORTED,
                    "this stack needs %zu bytes of scratch; kb_search_noalloc holds %zu "
                    "(use kb_search with a workspace)",
                    need, static_cast<size_t>(KB_NOALLOC_SCRATCH_BYTES));
    void *base = nullptr;
    st = scratch_address(&base);
    if (st != KB_OK) return st;
    char *ws = static_cast<char *>(base);
    hipStream_t s = (hipStream_t)stream;
    double *tau = reinterpret_cast<double *>(ws + tau_off);
    double *velv = reinterpret_cast<double *>(ws + vel_off);
    uint32_t *key = reinterpret_cast<uint32_t *>(ws + key_off);
    int32_t *order = reinterpret_cast<int32_t *>(ws + lay.order);
    st = send_doubles(tau, n_img, [&](int64_t i) { return t[i] - t[0]; }, s);
    if (st != KB_OK) return st;
    st = send_doubles(velv, 2 * n_vel, [&](int64_t k) { return vel[k]; }, s);
    if (st != KB_OK) return st;
    Box box;
    for (int a = 0; a < 2; ++a) box.lo[a] = box.hi[a] = vel[a];
    for (int64_t j = 1; j < n_vel; ++j)
        for (int a = 0; a < 2; ++a) {
            box.lo[a] = std::min(box.lo[a], vel[2 * j + a]);
            box.hi[a] = std::max(box.hi[a], vel[2 * j + a]);
        }
    const unsigned vblocks = (unsigned)((n_vel + 255) / 256);
    hipLaunchKernelGGL(hilbert_keys_kernel, dim3(vblocks), dim3(256), 0, s,
                       reinterpret_cast<const double2 *>(velv), (int)n_vel, box, key);
    st = launch_status("hilbert_keys_kernel");
    if (st != KB_OK) return st;
    hipLaunchKernelGGL(order_kernel, dim3(vblocks), dim3(256), 0, s, key, (int)n_vel, order);
    st = launch_status("order_kernel");
    if (st != KB_OK) return st;
    const int stride = (int)table_stride(n_img);
    const int64_t pix_bytes = dtype == KB_F32 ? 8 : 4;
    const int64_t entries = n_vel * stride;
    hipLaunchKernelGGL(table_kernel, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, s,
                       tau, reinterpret_cast<const double2 *>(velv), order, (int)n_img, stride,
                       (int)n_vel, (int)h, (int)w, w * pix_bytes, h * w * pix_bytes,
                       reinterpret_cast<GatherEntry *>(ws + lay.table));
    st = launch_status("table_kernel");
    if (st != KB_OK) return st;
    int32_t dy_range[2];
    dy_extent(t, n_img, vel, n_vel, h, dy_range);
    return launch_search_in(planes, dtype, lp_scale, n_img, h, w, n_vel, k_cand, cand_nu,
                            cand_alpha, cand_vel, cand_nobs, ws, dy_range, s);
}

}  // extern "C"
