// Measurement helper (not part of the search library): the throughput of the
// search's gather pattern on this GPU, the roof that bounds the search kernel.
//
// The search's memory work is, per wave, batches of raw buffer loads of 8
// bytes per lane: one contiguous (usually unaligned) 512-byte run per load,
// at a row and column offset that change from load to load, each batch
// summed once it has arrived.  This kernel issues exactly that pattern with
// no selection work: every wave issues `iters` batches of NB loads at
// pseudo-random rows of a region and pseudo-random (8-byte granular) column
// offsets, then adds what arrived.  With a region of a few MB (inside each
// XCD's 4 MB L2) it measures the cache-served gather peak; with a region of
// many GB it measures gathers served by HBM.
//
//   kbp_gather_peak  one timed launch; returns the kernel time in ms
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ u32x2 raw_load_b64(i32x4 rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2i32");
__device__ uint32_t raw_load_b32(i32x4 rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.i32");

__device__ inline i32x4 buffer_words(uint64_t base, uint32_t bytes) {
    i32x4 r;
    r.x = (int)(uint32_t)base;
    r.y = (int)(uint32_t)(base >> 32);
    r.z = (int)bytes;
    r.w = 0x00020000;
    return r;
}

// rows x row_bytes region; a load reads 64 lanes x W bytes (W = 8 or 4) from
// row r at byte offset (col + lane) * W, col < cols (the run stays in its row).
template <int NB, int W>
__global__ __launch_bounds__(64) void gather_peak_kernel(const unsigned char *__restrict__ region,
                                                         uint32_t rows, uint32_t row_bytes,
                                                         uint32_t cols, int iters, uint32_t seed,
                                                         float *__restrict__ sink) {
    const int lane = (int)threadIdx.x;
    uint32_t st = seed ^ (blockIdx.x * 0x9E3779B9u);
    const uint64_t base = reinterpret_cast<uint64_t>(region);
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
        u32x2 v[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            st = st * 1664525u + 1013904223u;            // wave-uniform generator
            const uint32_t r = __umulhi(st, rows);
            const uint32_t c = __umulhi(st * 2654435761u, cols);
            const i32x4 rs = buffer_words(base + (uint64_t)r * row_bytes, row_bytes);
            const int off = (int)((c + (uint32_t)lane) * (uint32_t)W);
            if constexpr (W == 8) {
                v[b] = raw_load_b64(rs, off, 0, 0);
            } else {
                v[b].x = raw_load_b32(rs, off, 0, 0);
                v[b].y = 0u;
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
            acc += __uint_as_float(v[b].x) + __uint_as_float(v[b].y);
    }
    if (acc == 1.2345f) sink[blockIdx.x * 64 + lane] = acc;   // keeps the loads alive
}

}  // namespace

extern "C" {

// One launch of `waves` one-wave workgroups, each issuing iters batches of
// nb (16 or 32) loads of `width` (8 or 4) bytes per lane over region
// [rows][row_bytes] (device memory, at least rows * row_bytes bytes;
// row_bytes a multiple of 8 and >= 512).  sink: device float32 of at least
// waves * 64 entries (written only to keep the loads alive).  Returns the
// kernel's time in ms from HIP events on `stream`, or a negative value on a
// bad argument or HIP error.  Bytes requested: waves * iters * nb * 64 * width.
double kbp_gather_peak(const void *region, uint32_t rows, uint32_t row_bytes, int waves,
                       int iters, int nb, int width, uint32_t seed, float *sink, void *stream) {
    if (!region || !sink || rows < 1 || row_bytes < 512 || row_bytes % 8 != 0 || waves < 1 ||
        iters < 1 || (nb != 16 && nb != 32) || (width != 4 && width != 8))
        return -1.0;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -2.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -2.0;
    }
    const uint32_t cols = row_bytes / (uint32_t)width - 64 + 1;
    const unsigned char *reg = static_cast<const unsigned char *>(region);
    double ms = -3.0;
    if (hipEventRecord(e0, s) == hipSuccess) {
        if (nb == 16 && width == 8)
            hipLaunchKernelGGL((gather_peak_kernel<16, 8>), dim3(waves), dim3(64), 0, s, reg,
                               rows, row_bytes, cols, iters, seed, sink);
        else if (nb == 32 && width == 8)
            hipLaunchKernelGGL((gather_peak_kernel<32, 8>), dim3(waves), dim3(64), 0, s, reg,
                               rows, row_bytes, cols, iters, seed, sink);
        else if (nb == 16)
            hipLaunchKernelGGL((gather_peak_kernel<16, 4>), dim3(waves), dim3(64), 0, s, reg,
                               rows, row_bytes, cols, iters, seed, sink);
        else
            hipLaunchKernelGGL((gather_peak_kernel<32, 4>), dim3(waves), dim3(64), 0, s, reg,
                               rows, row_bytes, cols, iters, seed, sink);
        float f = 0.f;
        if (hipGetLastError() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
            hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&f, e0, e1) == hipSuccess)
            ms = f;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // extern "C"
