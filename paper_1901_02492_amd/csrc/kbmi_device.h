// Device-side building blocks of libkbmi shared by its translation units:
// raw buffer access, candidate keys, the start-pixel tile order, and the
// trajectory-search kernels (instantiated per plane format by kbmi_search.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <utility>

#include "kbmi_internal.h"
#include "kbmi_merge_network.h"

// Launch-shape defaults (compile-time tunables).
#ifndef KBMI_STRIP_TILES
#define KBMI_STRIP_TILES 4      // start-pixel tiles per strip of the tile order
#endif
#ifndef KBMI_QUEUE
#define KBMI_QUEUE 16           // queued candidates per lane before a merge
#endif
#ifndef KBMI_PREFETCH
#define KBMI_PREFETCH 1         // single-stack search: fetch the next table row early
#endif
#ifndef KBMI_PIPELINE
#define KBMI_PIPELINE 1         // single-stack search: keep two velocities' gathers in flight
#endif
#ifndef KBMI_SUPER_W
#define KBMI_SUPER_W 2          // tiles per XCD strip in the super-strip order (0: off)
#endif
#ifndef KBMI_PERSIST_BS
#define KBMI_PERSIST_BS 2       // float32 planes: tiles per block row in the persistent order (0: off)
#endif
#ifndef KBMI_PIPE_MAX_LP
#define KBMI_PIPE_MAX_LP 56     // 16-bit planes: longest list with two velocities' gathers in flight
#endif
#ifndef KBMI_PERSIST_LP
#define KBMI_PERSIST_LP 0       // 16-bit planes also take the persistent order
#endif
#ifndef KBMI_PERSIST_SPIN
#define KBMI_PERSIST_SPIN 4000  // bound of a wave's wait at a generation boundary
#endif

#ifndef KBMI_PERSIST_PER_CU
#define KBMI_PERSIST_PER_CU 8   // persistent grid: at most this many one-wave workgroups per CU
#endif
#ifndef KBMI_NET_MAX_F32
#define KBMI_NET_MAX_F32 64     // longest list merged by the comparator network (float32)
#endif
#ifndef KBMI_NET_MAX_LP
#define KBMI_NET_MAX_LP 64      // 16-bit planes
#endif
#ifndef KBMI_LP_SC_MIN_KM
#define KBMI_LP_SC_MIN_KM 0     // 16-bit planes: lists of at least this length read their scales from LDS
#endif
// Float32, one batch of images: how many trailing padding slots may be
// skipped by uniform branches.  1: the survey's 15 images skip their one
// padding slot (83.5 -> 80.5 ms).  3 also serves 13 and 14 images (13 x
// 4096^2 at 32000 velocities: 3549 -> 3254 ms) but the two extra branches
// cost the 15-image search 80.4 -> 81.3 ms.
#ifndef KBMI_SKIP_TAIL
#define KBMI_SKIP_TAIL 1
#endif
#ifndef KBMI_INTERIOR
#define KBMI_INTERIOR 1         // start rows with every displaced row in frame skip the row check
#endif
// List lengths compiled for the search (each slot costs registers and
// compare-and-swap work on every insertion); a search keeps k_cand
// candidates in the shortest compiled list of at least k_cand slots, which
// gives the same best k_cand.  Every length in this list must be in
// kKmList below, in the same order.
#define KB_SEARCH_KM_LIST(X)                                                                \
    X(2) X(4) X(6) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(36) X(40) X(44) X(48) X(50) \
    X(52) X(56) X(60) X(64)

namespace kbmi {

// One search problem as the host launchers see it.
struct StackView {
    const void *planes;        // [n_img][h][w] (psi, phi) pairs of the plane format
    const float2 *inv_scale;   // 16-bit planes: (1/s_psi, 1/s_phi) per image, padded with 0
    int n_img, h, w;
    const GatherEntry *disp;   // gather-table rows in visiting order, `disp_stride` entries each
    int disp_stride;
    const int32_t *vel_index;  // original index of each visited velocity
    int n_vel, k_cand;
    float *cand_nu, *cand_alpha;
    int32_t *cand_vel;
    int16_t *cand_nobs;
    uint32_t *sync;            // per-XCD generation counters of the persistent search
    int row_lo, row_hi;        // start rows whose displaced rows are all in the frame
};

// One stack of a batched search, as the batch kernel reads it from device
// memory.  The launch's work items are its jobs' tiles: job j owns items
// [item_begin_j, item_begin_{j+1}).  A dense job's items are its tiles in
// strip order; a block job starts at a generation boundary and its items are
// the paced persistent order of a single-stack search (generation
// (item - item_begin) / grid, workgroup (item - item_begin) % grid), slots
// past its frame's edge included and skipped.
struct BatchJob {
    const void *planes;
    const float2 *inv_scale;
    const GatherEntry *disp;
    const int32_t *vel_index;
    float *cand_nu, *cand_alpha;
    int32_t *cand_vel;
    int16_t *cand_nobs;
    int n_img, h, w, disp_stride, n_vel;
    int item_begin;
    int nseg;                  // tiles per row
    int dense;                 // 1: strip order (strip tiles wide); 0: block order
    int strip;
    int bs, brows, nbc, nbr;   // block order (PersistMap's fields)
};

kb_status launch_status(const char *what);

// Search launchers.  km is the (even) compiled list length >= k_cand.  The
// list lengths are split into kKmGroups groups, km in group (km / 2 - 1) %
// kKmGroups, and the build compiles kbmi_search.hip once per plane format and
// group (the translation units compile in parallel); launch_search and
// launch_search_batch dispatch to them.
constexpr int kKmGroups = 8;
constexpr int kKmList[] = {2, 4, 6, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 50, 52, 56, 60, 64};
constexpr int kKmCount = (int)(sizeof(kKmList) / sizeof(kKmList[0]));
static_assert(kKmList[kKmCount - 1] == KB_MAX_KCAND, "the longest list is KB_MAX_KCAND");
constexpr int km_index(int km) {
    for (int i = 0; i < kKmCount; ++i)
        if (kKmList[i] == km) return i;
    return -1;
}
constexpr int km_group(int km) { return km_index(km) % kKmGroups; }
// The compiled list length for k_cand (1 <= k_cand <= KB_MAX_KCAND).
constexpr int km_for(int k_cand) {
    for (int i = 0; i < kKmCount; ++i)
        if (kKmList[i] >= k_cand) return kKmList[i];
    return -1;
}
template <int FMT, int G>
kb_status launch_search_group(int km, const StackView &v, hipStream_t s);
template <int FMT, int G>
kb_status launch_search_batch_group(int km, const BatchJob *jobs, int n_jobs, int n_img_class,
                                    int k_cand, int generations, uint32_t *sync, int *grid,
                                    hipStream_t s);
#define KBMI_DECLARE_GROUP(F, G)                                                          \
    template <>                                                                           \
    kb_status launch_search_group<F, G>(int, const StackView &, hipStream_t);             \
    template <>                                                                           \
    kb_status launch_search_batch_group<F, G>(int, const BatchJob *, int, int, int, int,    \
                                              uint32_t *, int *, hipStream_t);
#define KBMI_DECLARE_FMT(F)                                                                 \
    KBMI_DECLARE_GROUP(F, 0) KBMI_DECLARE_GROUP(F, 1) KBMI_DECLARE_GROUP(F, 2)             \
    KBMI_DECLARE_GROUP(F, 3) KBMI_DECLARE_GROUP(F, 4) KBMI_DECLARE_GROUP(F, 5)             \
    KBMI_DECLARE_GROUP(F, 6) KBMI_DECLARE_GROUP(F, 7)
KBMI_DECLARE_FMT(0)
KBMI_DECLARE_FMT(1)
KBMI_DECLARE_FMT(2)
#undef KBMI_DECLARE_FMT
#undef KBMI_DECLARE_GROUP
kb_status launch_search(int fmt, int km, const StackView &v, hipStream_t s);
// One persistent launch of `generations` generations over the jobs of one
// image-count class (0: n_img <= 8, 1: <= 16, 2: > 16), whose descriptors
// (device) already hold their item ranges for a grid of *grid workgroups;
// sync: 8 per-XCD counters (zeroed here).  With jobs == nullptr nothing is
// launched and *grid receives that class's grid.
kb_status launch_search_batch(int fmt, int km, const BatchJob *jobs, int n_jobs,
                              int n_img_class, int k_cand, int generations, uint32_t *sync,
                              int *grid, hipStream_t s);

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// The gather table, the visiting order and the inverse scales do not change
// during a launch: they are read through the constant address space, so
// their wave-uniform loads stay scalar whatever else the kernel writes.
typedef __attribute__((address_space(4))) const i32x4 const_i32x4;
typedef __attribute__((address_space(4))) const f32x4 const_f32x4;
typedef __attribute__((address_space(4))) const int32_t const_i32;

// Raw buffer loads with the descriptor as four plain words.
__device__ u32x2 raw_load_b64(i32x4 rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2i32");
__device__ uint32_t raw_load_b32(i32x4 rsrc, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.i32");

namespace {

// ---------------------------------------------------------------------------
// Raw buffer access.  A descriptor is four scalar words: the 48-bit base
// address, the record count in bytes (stride 0: an access is out of range when
// its byte offset is >= the record count, and then a load returns 0 without
// touching memory), and the format word.  The loads take the descriptor as a
// plain vector so that building one costs no masking.
// ---------------------------------------------------------------------------
constexpr int kBufferFlags = 0x00020000;


__device__ inline i32x4 buffer_words(uint64_t base, uint32_t bytes) {
    i32x4 r;
    r.x = (int)(uint32_t)base;
    r.y = (int)(uint32_t)(base >> 32);
    r.z = (int)bytes;
    r.w = kBufferFlags;
    return r;
}

// ---------------------------------------------------------------------------
// Candidate keys.  A candidate is ordered by (nu descending, j ascending); the
// 63-bit key (order-preserving bits of nu) << 31 | (0xFFFF - j) << 15 | n_obs
// compares the same way as unsigned integers.  n_obs never decides an order
// because j is unique within a pixel.  Key 0 is below every real candidate
// (nu = -inf maps to 0x007FFFFF) and marks an empty slot.
//
// Read as an IEEE double, such a key is non-negative (bit 63 is clear) and
// finite (the order bits are clamped to those of +inf, so the exponent field
// never reaches all ones), and doubles of that kind order exactly like their
// bit patterns: the FP64 max/min instructions move a key in one instruction.
// ---------------------------------------------------------------------------
__device__ inline uint32_t nu_order_bits(float nu) {
    uint32_t u = __float_as_uint(nu);
    if (u == 0x80000000u) u = 0u;   // -0 ranks equal to +0
    const uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return min(o, 0xFF800000u);     // nothing ranks above +inf
}

__device__ inline float nu_from_order_bits(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ inline uint64_t make_key(float nu, int j, uint32_t nobs) {
    return ((uint64_t)nu_order_bits(nu) << 31) |
           (uint64_t)(((uint32_t)(0xFFFF - j) << 15) | (nobs & 0x7FFFu));
}
__device__ inline float key_nu(uint64_t k) { return nu_from_order_bits((uint32_t)(k >> 31)); }
__device__ inline int32_t key_vel(uint64_t k) {
    return 0xFFFF - (int32_t)((uint32_t)(k >> 15) & 0xFFFFu);
}
__device__ inline int32_t key_nobs(uint64_t k) { return (int32_t)((uint32_t)k & 0x7FFFu); }

// k, n <- max(k, n), min(k, n) as keys, in place.
__device__ inline void key_exchange(uint64_t &k, uint64_t &n) {
    double kd = __builtin_bit_cast(double, k), t;
    asm("v_min_f64 %0, %1, %2\n\tv_max_f64 %1, %1, %2"
        : "=&v"(t), "+v"(kd)
        : "v"(__builtin_bit_cast(double, n)));
    k = __builtin_bit_cast(uint64_t, kd);
    n = __builtin_bit_cast(uint64_t, t);
}

// k <- max(k, n) as keys.
__device__ inline uint64_t key_max(uint64_t k, uint64_t n) {
    double kd = __builtin_bit_cast(double, k);
    asm("v_max_f64 %0, %0, %1" : "+v"(kd) : "v"(__builtin_bit_cast(double, n)));
    return __builtin_bit_cast(uint64_t, kd);
}

// Merging a batch of 16 queued candidates into the descending list of KM
// (registers 0..KM-1 of r/ra; the batch in KM..KM+15) with the generated
// comparator network, keeping the best KM.  Alpha follows its key.
template <int KIND, int A, int B, int N>
__device__ __forceinline__ void net_op(uint64_t (&r)[N], float (&ra)[N]) {
    const bool c = r[B] > r[A];
    if constexpr (KIND == 0) {
        key_exchange(r[A], r[B]);
        const float t = c ? ra[B] : ra[A];
        ra[B] = c ? ra[A] : ra[B];
        ra[A] = t;
        // Materialise both outputs here (no code): otherwise the alpha
        // selects sink to their uses and every compare result stays live.
        asm volatile("" : "+v"(r[A]), "+v"(r[B]), "+v"(ra[A]), "+v"(ra[B]));
    } else {
        r[A] = key_max(r[A], r[B]);
        ra[A] = c ? ra[B] : ra[A];
        asm volatile("" : "+v"(r[A]), "+v"(ra[A]));
    }
}
template <int KM, int N, size_t... I>
__device__ __forceinline__ void net_run(uint64_t (&r)[N], float (&ra)[N],
                                        std::index_sequence<I...>) {
    // Applied in program order: interleaving the network's independent
    // exchanges would only lengthen live ranges past the register file.
    ((net_op<MergeNetwork<KM>::ops[I].kind, MergeNetwork<KM>::ops[I].a,
             MergeNetwork<KM>::ops[I].b>(r, ra),
      __builtin_amdgcn_sched_barrier(0)),
     ...);
}
template <int KM, int N, size_t... S>
__device__ __forceinline__ void net_place(uint64_t (&r)[N], float (&ra)[N],
                                          std::index_sequence<S...>) {
    // List slot s takes register perm[s] (fixed swaps of the network).
    const uint64_t k[KM] = {r[MergeNetwork<KM>::perm[S]]...};
    const float a[KM] = {ra[MergeNetwork<KM>::perm[S]]...};
    ((r[S] = k[S], ra[S] = a[S]), ...);
}
template <int KM, int N>
__device__ __forceinline__ void net_merge(uint64_t (&r)[N], float (&ra)[N]) {
    net_run<KM>(r, ra, std::make_index_sequence<MergeNetwork<KM>::n_ops>());
    net_place<KM>(r, ra, std::make_index_sequence<KM>());
}

// Scores of one trajectory (Sec. 2.1.5): nu = Psi / sqrt(Phi) and
// alpha = Psi / Phi; Phi = 0 (no valid observation) gives nu = -inf and
// alpha = 0.  Every kernel scores with these functions, so equal sums give
// bitwise equal scores.
// KBMI_IEEE_SCORE 0: both from the hardware reciprocal square root r of Phi
// (within 1 ulp for normal inputs; Phi below 2^-100 is scaled by 2^64 first,
// so no denormal reaches it): nu = Psi * r, alpha = nu * r.
// KBMI_IEEE_SCORE 1: a correctly rounded square root and divisions.
#ifndef KBMI_IEEE_SCORE
#define KBMI_IEEE_SCORE 0
#endif
__device__ inline float inv_sqrt_phi(float F) {
    if (KBMI_IEEE_SCORE) return 0.f;
    const bool tiny = F < 0x1p-100f;
    const float r = __builtin_amdgcn_rsqf(tiny ? F * 0x1p64f : F);
    return tiny ? r * 0x1p32f : r;
}
__device__ inline float score_nu(float P, float F, float r) {
    if (KBMI_IEEE_SCORE) return F > 0.f ? P / sqrtf(F) : -INFINITY;
    return F > 0.f ? P * r : -INFINITY;
}
__device__ inline float score_alpha(float P, float nu, float F, float r) {
    if (KBMI_IEEE_SCORE) return F > 0.f ? P / F : 0.f;
    (void)P;
    return F > 0.f ? nu * r : 0.f;
}

// Start-pixel tiles: one wave = 64 adjacent pixels of one row.  Tiles are
// enumerated in strips `strip` tiles wide (all rows of a strip, then the next
// strip) so that consecutive workgroups cover a compact 2-D patch, and the
// workgroup index is remapped so that each of the 8 XCDs (which receive
// workgroups round-robin) walks one contiguous range of that order and its
// L2 sees neighbouring patches.
__device__ inline int xcd_remap(int b, int nblocks) {
    const int xcd = b & 7, k = b >> 3;
    const int q = nblocks >> 3, r = nblocks & 7;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

__device__ inline void strip_tile(int t, int nseg, int h, int strip, int &row, int &seg) {
    const int fs = nseg / strip;
    const int full = fs * h * strip;
    if (t < full) {
        const int s = t / (h * strip);
        const int rem = t - s * h * strip;
        row = rem / strip;
        seg = s * strip + (rem - (rem / strip) * strip);
    } else {
        const int rw = nseg - fs * strip;
        const int rem = t - full;
        row = rem / rw;
        seg = fs * strip + (rem - (rem / rw) * rw);
    }
}

// Super-strip order (used when nseg is a multiple of 8 * sw): the frame is
// cut into vertical super-strips 8 * sw tiles wide; within one, XCD x owns
// the sw-tile strip x and walks it top to bottom.  The eight XCDs then sweep
// down the same super-strip together, so the rows that later start rows
// gather again (every velocity reaches up to the longest displacement) stay
// within a window the memory-side cache can hold.
__device__ inline void superstrip_tile(int b, int h, int sw, int &row, int &seg) {
    const int xcd = b & 7, m = b >> 3;
    const int per = sw * h;
    const int ss = m / per;
    const int rem = m - ss * per;
    row = rem / sw;
    seg = (ss * 8 + xcd) * sw + (rem - row * sw);
}

struct TileMap {
    int nseg;     // tiles per row
    int h;        // rows
    int strip;    // tiles per strip
    int nblocks;  // nseg * h
    int sw;       // > 0: super-strip order with sw-tile strips per XCD

    __device__ inline void map(int b, int &row, int &seg) const {
        if (sw > 0) superstrip_tile(b, h, sw, row, seg);
        else strip_tile(xcd_remap(b, nblocks), nseg, h, strip, row, seg);
    }
};

// Persistent order: the grid is exactly the number of workgroups the GPU
// holds at once, and workgroup w processes one tile per generation.  In a
// generation, XCD x (workgroups w = 8k + x, dispatched round-robin over the
// XCDs) covers one block of bs x brows tiles (k -> row k / bs, seg k % bs),
// the eight XCDs take eight side-by-side blocks, and generations move down
// the frame, then to the next eight block columns.  Waves that start a
// generation together walk the velocities roughly in step, so one velocity's
// gathers find the rows the block read for the previous ones still in L2.
// Every in-frame tile belongs to exactly one (generation, workgroup); slots
// past the frame's edge are skipped.
struct PersistMap {
    int nseg, h;
    int bs, brows;     // block: bs tiles wide, brows rows tall (bs * brows = grid / 8)
    int nbc, nbr;      // blocks per row of blocks, rows of blocks
    int generations;   // ceil(nbc / 8) * nbr
    int spin;          // bound of a wave's wait at a generation boundary (0: no wait)
    __device__ inline bool map(int gen, int w, int &row, int &seg) const {
        const int xcd = w & 7, k = w >> 3;
        const int sc = gen / nbr;
        const int br = gen - sc * nbr;
        const int bc = sc * 8 + xcd;
        const int q = k / bs;
        row = br * brows + q;
        seg = bc * bs + (k - q * bs);
        return bc < nbc && row < h && seg < nseg;
    }
};

template <int FMT>
struct PlaneLoad {                       // one (psi, phi) pair as loaded
    typedef u32x2 type;                  // float32: two words
};
template <>
struct PlaneLoad<KB_F16> {
    typedef uint32_t type;               // 16-bit: psi low half, phi high half
};
template <>
struct PlaneLoad<KB_BF16> {
    typedef uint32_t type;
};

__device__ inline float lp_value(uint32_t bits16, int fmt) {
    if (fmt == KB_F16) return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
    return __uint_as_float(bits16 << 16);
}

// ---------------------------------------------------------------------------
// Trajectory search.
//
// One wave (one workgroup) owns 64 adjacent start pixels of one row and walks
// every velocity in the host-chosen visiting order.  Per velocity each lane
// gathers its trajectory's N (psi, phi) pairs (one coalesced 512-byte run per
// image across the wave), sums them in image order and scores nu.
//
// Per-pixel selection keeps a descending list of KM >= k_cand keys in
// registers.  Inserting into it costs a compare-and-swap per slot, and the wave
// pays for it whenever any lane inserts, so candidates are first filtered
// against a per-lane threshold (the list's last key at the last merge) and
// parked in a per-lane LDS queue of PB entries; the queue is merged into the
// list only when some lane's queue is full (and at the end).  A candidate that
// fails the threshold can never enter the final list: the threshold only rises.
//
// The loads of up to NB images are issued together before they are summed in
// image order; larger stacks are summed in batches of NB images.  The kernel
// is bounded to two waves per SIMD: memory-level parallelism comes from the
// waves, each holding one velocity's NB loads in flight.
// ---------------------------------------------------------------------------
// LDS of a search workgroup: the candidate queue (3 words per entry and
// lane), also used to stage the output (KM words per lane), then the inverse
// scales of 16-bit planes of up to kSearchScaleWords / 2 images.
constexpr int kSearchScaleWords = 128;
template <int KM, int PB>
constexpr int search_queue_words() {
    return (3 * PB > KM ? 3 * PB : KM) * 64;
}
template <int KM, int PB>
constexpr int search_lds_words() {
    return search_queue_words<KM, PB>() + kSearchScaleWords;
}

// The gathers of one tile (start row `row`, start columns seg*64 .. seg*64+63)
// for every velocity in the host-chosen visiting order: per velocity each lane
// sums its trajectory's N (psi, phi) pairs in image order (one coalesced
// 64 * pair-size run per image across the wave) and counts n_obs, then calls
// finish(j, Psi, Phi, n_obs) with the velocity's original index j.  All
// scalar arguments are wave-uniform.
//   NB        loads per batch (8 or 16; the table stride is a multiple of 16)
//   PF        fetch the next table row while the gathers are in flight
//   PIPE      two batches' gathers in flight (PF only; costs a second buffer)
//   MB        more images than one batch (launched for n_img > NB only)
//   INTERIOR  every displaced row of this start row is inside the frame
//   LDS_SC    16-bit planes in one batch: the inverse scales are read from LDS
//             per velocity instead of held in 2 NB vector registers (for
//             long lists, whose slots need those registers)
//   sc_lds    16-bit planes with MB or LDS_SC: LDS for kSearchScaleWords
//             inverse scales
template <int NB, int FMT, bool PF, bool PIPE, bool MB, bool INTERIOR, bool LDS_SC,
          class Finish>
__device__ __forceinline__ void visit_velocities(
    float *sc_lds, const void *__restrict__ planes, const float2 *__restrict__ inv_scale,
    int n_img, int h, int w, const GatherEntry *__restrict__ disp, int disp_stride,
    const int32_t *__restrict__ vel_index, int n_vel, int row, int seg, Finish &&finish) {
    const int lane = (int)threadIdx.x;
    const int x0 = seg * 64 + lane;
    typedef typename PlaneLoad<FMT>::type LoadT;
    constexpr uint32_t kPix = FMT == KB_F32 ? 8u : 4u;   // bytes per (psi, phi) pair
    const uint32_t row_bytes = (uint32_t)w * kPix;
    const const_i32 *visit = (const const_i32 *)(const void *)vel_index;
    // Byte address of the start row in image 0; a table entry's offset moves
    // it to the displaced row of its image.
    const uint64_t row0 = reinterpret_cast<uint64_t>(planes) + (uint64_t)row * row_bytes;
    // Fetch entries [i0, i0 + NB) of table row jj (wide scalar loads).
    auto fetch = [&](int jj, int i0, i32x4(&e)[NB]) {
        const const_i32x4 *t4 =
            (const const_i32x4 *)(const void *)(disp + (size_t)jj * disp_stride + i0);
#pragma unroll
        for (int b = 0; b < NB; ++b) e[b] = t4[b];
    };
    // Issue the gathers of one batch of table entries, from entry `from` on
    // (a compile-time 0 or 1).  A row outside the frame (padding entries
    // included) gets a zero-length buffer, so its loads return 0 and add
    // nothing, with no branch.  With a record count of 0 every lane fails the
    // range check before an address is formed, so the base of such a buffer
    // (which may point outside the planes) is never dereferenced.  no_entry0:
    // entry 0 (image 0, whose pair is loaded once per tile) gets a zero-length
    // buffer too, so its load touches no memory.
    // nl: entries of this batch that hold images (later ones are padding).
    // Float32 planes skip the padding slots' loads (their registers hold 0).
    // 16-bit planes issue them like the others: a padding entry's column
    // x0 + w fails the range check (and its row, outside the frame, gets a
    // zero-length buffer off interior tiles), so the load returns 0 and
    // touches no memory; with no branch, the wait before a batch's sums counts
    // exactly the loads of the batch behind it (25 images at 4000 velocities:
    // 16-bit 974 -> 889 ms; float32 902 -> 1655 ms, so float32 keeps the skip).
    // skip_last (float32 planes): one batch holding every image but the last
    // slot (n_img = NB - 1, the survey's 15 images): that slot's load is
    // skipped by one uniform branch, which leaves the wait before the
    // previous batch's sums at most one load short: 83.5 -> 80.5 ms on the
    // survey stack.  16-bit planes issue it (the branch measured 57.8 ->
    // 61.2 ms there).
    auto issue = [&](const i32x4(&e)[NB], auto &v, int from, bool no_entry0, int nl,
                     bool skip_last = false) {
        constexpr int NV = (int)(sizeof(v) / sizeof(v[0]));   // NB, or NB / 2
#pragma unroll
        for (int b = 0; b < NV; ++b) {
            if (b < from) continue;
            const bool tail = KBMI_SKIP_TAIL == 1
                                  ? (b == NV - 1 && skip_last)
                                  : (skip_last && b >= NV - KBMI_SKIP_TAIL && b >= n_img);
            if ((FMT == KB_F32 && b >= nl) || tail) {
                v[b] = LoadT{};
                continue;
            }
            const uint64_t off = ((uint64_t)(uint32_t)e[b].w << 32) | (uint32_t)e[b].z;
            // Interior tiles: every real entry's row is in the frame; a padding
            // entry's column (x0 + w) fails the buffer's range check instead.
            // 16-bit planes over several batches issue up to 15 padding slots
            // per velocity; there an entry with dy >= h (padding, or a
            // trajectory that has left the frame, out of it for any start row)
            // gets a zero-length buffer, because lanes that fail the range check
            // of a non-empty buffer cost far more than a buffer that holds
            // nothing (25 images: 1110 -> 882 ms).  Elsewhere the extra scalar
            // compare costs more than it saves.
            constexpr bool kPadCheck = MB && FMT != KB_F32;
            bool in_rows = INTERIOR ? (!kPadCheck || e[b].y < h)
                                    : (unsigned)(row + e[b].y) < (unsigned)h;
            if (b == 0) in_rows = in_rows && !no_entry0;
            const i32x4 rs = buffer_words(row0 + off, in_rows ? row_bytes : 0u);
            if constexpr (FMT == KB_F32)
                v[b] = raw_load_b64(rs, (x0 + e[b].x) * (int)kPix, 0, 0);
            else
                v[b] = raw_load_b32(rs, (x0 + e[b].x) * (int)kPix, 0, 0);
        }
    };
    // Sum in image order.  Empty slots hold +0, which leaves every sum
    // unchanged.  16-bit values are decoded and unscaled by an exact power of
    // two inside the FMA (the product is exact, so the sum rounds once).
    // 16-bit planes: the inverse scales (1/s_psi, 1/s_phi) of images
    // [i0, i0 + NB), uniform values.
    typedef f32x4 Scales[NB / 2];
    auto load_scales = [&](int i0, Scales &ss) {
        const const_f32x4 *sc4 = (const const_f32x4 *)(const void *)(inv_scale + i0);
#pragma unroll
        for (int q = 0; q < NB / 2; ++q) ss[q] = sc4[q];
    };
    // v: a batch of NB loads, or NB / 2 (with as many scale pairs in ss).
    auto accumulate = [&](const auto &ss, const auto &v, float &P, float &F, int from) {
        constexpr int NV = (int)(sizeof(v) / sizeof(v[0]));
        if constexpr (FMT == KB_F32) {
            (void)ss;
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                if (b < from) continue;
                P += __uint_as_float(v[b].x);
                F += __uint_as_float(v[b].y);
            }
        } else {
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                if (b < from) continue;
                const float isp = (b & 1) ? ss[b / 2].z : ss[b / 2].x;
                const float isf = (b & 1) ? ss[b / 2].w : ss[b / 2].y;
                P = fmaf(lp_value(v[b] & 0xFFFFu, FMT), isp, P);
                F = fmaf(lp_value(v[b] >> 16, FMT), isf, F);
            }
        }
    };
    // n_obs: the stored phi is nonzero exactly at valid pixels; empty slots are 0.
    auto count = [&](const auto &v, int from) {
        constexpr int NV = (int)(sizeof(v) / sizeof(v[0]));
        uint32_t c = 0;
#pragma unroll
        for (int b = 0; b < NV; ++b) {
            if (b < from) continue;
            if constexpr (FMT == KB_F32) {
                // min(bits, 1) as one vector instruction: the compiler's
                // compare-and-carry form routes each term through a scalar
                // mask and needs wait states before its use.
                uint32_t m;
                asm("v_min_u32 %0, %1, 1" : "=v"(m) : "v"(v[b].y));
                c += m;
            } else {
                // Both halves at once: min(psi16, 1) | min(phi16, 1) << 16;
                // at most 16 terms, so the low half never carries.
                uint32_t m;
                asm("v_pk_min_u16 %0, %1, %2" : "=v"(m) : "v"(v[b]), "v"(0x00010001u));
                c += m;
            }
        }
        if constexpr (FMT != KB_F32) c >>= 16;
        return c;
    };
    // With all images in one batch the scales are loop-invariant: they are
    // kept in vector registers (the scalar file holds the table row), or in
    // LDS (LDS_SC).
    Scales ss0 = {};
    if constexpr (FMT != KB_F32 && !MB) {
        if (n_img <= NB) {
            if constexpr (LDS_SC) {
                const float *isc = reinterpret_cast<const float *>(inv_scale);
                for (int q = lane; q < 2 * NB; q += 64) sc_lds[q] = isc[q];
                __syncthreads();
            } else {
                load_scales(0, ss0);
#pragma unroll
                for (int q = 0; q < NB / 2; ++q) asm volatile("" : "+v"(ss0[q]));
            }
        }
    }
    // Inverse scales of batch `part` from LDS.
    auto lds_scales = [&](int part, Scales &ss) {
        const f32x4 *s4 = reinterpret_cast<const f32x4 *>(sc_lds + 2 * NB * part);
#pragma unroll
        for (int q = 0; q < NB / 2; ++q) ss[q] = s4[q];
    };
    // Image 0 is the start image: its displacement is (0, 0) for every
    // velocity (tau_0 = 0), so the pipelined paths load its pair once per tile
    // and start every trajectory's sums from it, 0 + value first, exactly the
    // additions the per-velocity loads would make.
    float P0 = 0.f, F0 = 0.f;
    uint32_t c0 = 0;
    auto hoist_image0 = [&](float isp0, float isf0) {
        const i32x4 rs = buffer_words(row0, row_bytes);
        if constexpr (FMT == KB_F32) {
            const u32x2 v0 = raw_load_b64(rs, x0 * (int)kPix, 0, 0);
            P0 = 0.f + __uint_as_float(v0.x);
            F0 = 0.f + __uint_as_float(v0.y);
            asm("v_min_u32 %0, %1, 1" : "=v"(c0) : "v"(v0.y));
        } else {
            const uint32_t v0 = raw_load_b32(rs, x0 * (int)kPix, 0, 0);
            P0 = fmaf(lp_value(v0 & 0xFFFFu, FMT), isp0, 0.f);
            F0 = fmaf(lp_value(v0 >> 16, FMT), isf0, 0.f);
            c0 = (v0 >> 16) != 0u ? 1u : 0u;
        }
    };
    constexpr bool kPipe = PF && PIPE;
    const bool skip_last = FMT == KB_F32 && !MB &&
                           (KBMI_SKIP_TAIL == 1 ? n_img == NB - 1 : n_img >= NB - KBMI_SKIP_TAIL);
    // 16-bit planes of more than one batch keep every image's scales in LDS
    // (read per batch), up to kMaxLdsScaleImages images.
    constexpr int kMaxLdsScaleImages = kSearchScaleWords / 2;
    // The whole visit of one batch after another, for more images than the
    // pipelined paths take (and lists too long for two batches in flight).
    auto serial_path = [&]() {
        for (int jj = 0; jj < n_vel; ++jj) {
            const int j = visit[jj];
            float P = 0.f, F = 0.f;
            uint32_t c = 0;
            for (int i0 = 0; i0 < n_img; i0 += NB) {
                i32x4 e[NB];
                fetch(jj, i0, e);
                LoadT v[NB];
                issue(e, v, 0, false, NB);
                Scales ss = {};
                if constexpr (FMT != KB_F32) load_scales(i0, ss);
                accumulate(ss, v, P, F, 0);
                c += count(v, 0);
            }
            finish(j, P, F, c);
        }
    };
    // NB + 1 <= n_img <= NB + NB / 2 + 1 (17 to 25 images): image 0 hoisted,
    // the other images fill one batch of NB (images 1..NB) and one of NB / 2
    // (images NB + 1 .. NB + NB / 2), with two batches in flight: at most
    // NB / 2 padding slots per velocity, none at 25 images, where the
    // general sequence below issues 2 NB - 1 slots for 24 images.  The 16-bit
    // search is bound by issued load instructions (padding slots cost as much
    // as real ones).  Same sums in the same image order.  16-bit planes only:
    // float32 planes skip their padding slots' loads already, and the second
    // path spills the float32 kernels' registers.
    auto split_path = [&]() {
        constexpr int NH = NB / 2;
        if constexpr (FMT != KB_F32) {
            // Inverse scales of images 1 .. NB + NH into LDS, image 1 first, so
            // that each batch reads whole f32x4 words (the table of scales
            // holds 2 * table_stride(n_img) >= 2 (NB + NH + 1) floats).
            const float *isc = reinterpret_cast<const float *>(inv_scale);
            for (int q = lane; q < 2 * (NB + NH); q += 64) sc_lds[q] = isc[q + 2];
            __syncthreads();
            hoist_image0(isc[0], isc[1]);
        } else {
            hoist_image0(1.f, 1.f);
        }
        const int nl_b = n_img - 1 - NB;          // images in batch B (0 .. NH)
        const int last = n_vel - 1;
        auto fetch_b = [&](int jj, i32x4(&e)[NB]) {
            const const_i32x4 *t4 = (const const_i32x4 *)(const void *)(
                disp + (size_t)jj * disp_stride + 1 + NB);
#pragma unroll
            for (int b = 0; b < NH; ++b) e[b] = t4[b];
        };
        i32x4 e[NB];
        LoadT va[NB], vb[NH];
        fetch(0, 1, e);
        issue(e, va, 0, false, NB);               // A(0): images 1 .. NB
        fetch_b(0, e);
        int jn = last < 1 ? last : 1;
        for (int jj = 0; jj < n_vel; ++jj) {
            const int j = visit[jj];
            issue(e, vb, 0, false, nl_b);         // B(jj) behind A(jj)
            __builtin_amdgcn_sched_barrier(0);
            fetch(jn, 1, e);
            __builtin_amdgcn_sched_barrier(0);
            float P = P0, F = F0;
            uint32_t c = c0;
            {
                Scales ss = {};
                if constexpr (FMT != KB_F32) lds_scales(0, ss);
                accumulate(ss, va, P, F, 0);
                c += count(va, 0);
            }
            issue(e, va, 0, false, NB);           // A(jj + 1) (the last repeats)
            __builtin_amdgcn_sched_barrier(0);
            fetch_b(jn, e);
            __builtin_amdgcn_sched_barrier(0);
            {
                f32x4 ssb[NH / 2] = {};
                if constexpr (FMT != KB_F32) {
                    const f32x4 *s4 = reinterpret_cast<const f32x4 *>(sc_lds + 2 * NB);
#pragma unroll
                    for (int q = 0; q < NH / 2; ++q) ssb[q] = s4[q];
                }
                accumulate(ssb, vb, P, F, 0);
                c += count(vb, 0);
            }
            finish(j, P, F, c);
            jn = jj + 2 < last ? jj + 2 : last;
        }
    };
    if constexpr (MB) {
        // More images than one batch (MB): launched for n_img > NB only.
        if (FMT != KB_F32 && kPipe && NB == 16 && n_img <= NB + NB / 2 + 1) {
            if constexpr (FMT != KB_F32) split_path();
        } else if (kPipe && (FMT == KB_F32 || n_img <= kMaxLdsScaleImages)) {
            // Each velocity's table row is read as nbat batches of NB entries,
            // and the batches of all velocities form one sequence with two
            // batches in flight (the gathers of batch q+1 are issued before
            // batch q is summed, the entries of q+2 fetched behind them).  A
            // velocity's sums run over its batches in image order and it is
            // scored after its last batch.  Batch 0 of each velocity skips
            // image 0's memory access (hoisted, as above).
            const int nbat = (n_img + NB - 1) / NB;
            if constexpr (FMT != KB_F32) {
                // (1/s_psi, 1/s_phi) of every image (padding 0) into LDS.
                const float *isc = reinterpret_cast<const float *>(inv_scale);
                for (int q = lane; q < 2 * nbat * NB; q += 64) sc_lds[q] = isc[q];
                __syncthreads();
                hoist_image0(sc_lds[0], sc_lds[1]);
            } else {
                hoist_image0(1.f, 1.f);
            }
            const int nq = n_vel * nbat;
            const int lastq = nq - 1;
            // Positions (velocity, part) of the batch being summed and of the
            // batch whose entries sit in e; they advance one batch per step (the
            // latter stops at the last batch, which the end then repeats).
            int jj_c = 0, p_c = 0;       // (jj_c is kept for symmetry with the fetch side)
            int jj_f = 0, p_f = 0;
            auto advance = [&](int &jj_, int &p_) {
                if (++p_ == nbat) {
                    p_ = 0;
                    ++jj_;
                }
            };
            // Image entries of the last batch of a velocity (the rest pad).
            const int nl_last = n_img - (nbat - 1) * NB;
            i32x4 e[NB];
            LoadT va[NB], vb[NB];
            fetch(jj_f, p_f * NB, e);
            issue(e, va, 0, true, NB);
            int jc = visit[0];           // velocity index of the batch being summed
            int q_f = 1;                 // flat index of the batch whose entries are in e
            advance(jj_f, p_f);
            fetch(jj_f, p_f * NB, e);
            int je = visit[jj_f];
            float P = P0, F = F0;
            uint32_t c = c0;
            auto step = [&](LoadT(&cur)[NB], LoadT(&ahead)[NB]) {
                // batch q + 1 (repeats the last at the end)
                issue(e, ahead, 0, p_f == 0, p_f == nbat - 1 ? nl_last : NB);
                const int ja = je;
                __builtin_amdgcn_sched_barrier(0);
                if (q_f < lastq) {
                    ++q_f;
                    advance(jj_f, p_f);
                }
                fetch(jj_f, p_f * NB, e);
                je = visit[jj_f];
                __builtin_amdgcn_sched_barrier(0);
                Scales ss = {};
                if constexpr (FMT != KB_F32) lds_scales(p_c, ss);
                accumulate(ss, cur, P, F, 0);
                c += count(cur, 0);
                if (p_c == nbat - 1) {
                    finish(jc, P, F, c);
                    P = P0;
                    F = F0;
                    c = c0;
                }
                advance(jj_c, p_c);
                jc = ja;
            };
            int q = 0;
            for (; q + 1 < nq; q += 2) {
                step(va, vb);
                step(vb, va);
            }
            if (q < nq) step(va, vb);
        } else {
            serial_path();
        }
    } else if (n_img <= NB && kPipe) {
        // Two velocities in flight: the gathers of visit jj+1 are issued
        // before visit jj is summed and scored, and the table row of jj+2 is
        // fetched behind them (into the registers the row of jj+1 just left).
        // The load buffers alternate, so the loop runs in pairs of visits; a
        // visit past the end repeats the last row and is never scored.
        if constexpr (LDS_SC) hoist_image0(sc_lds[0], sc_lds[1]);
        else hoist_image0(ss0[0].x, ss0[0].y);
        i32x4 e[NB];
        LoadT va[NB], vb[NB];
        fetch(0, 0, e);
        issue(e, va, 1, false, NB, skip_last);
        const int last = n_vel - 1;
        int j_cur = visit[0];
        int nxt = last < 1 ? last : 1;
        fetch(nxt, 0, e);
        int j_nxt = visit[nxt];
        auto step = [&](int jj, LoadT(&cur)[NB], LoadT(&ahead)[NB]) {
            issue(e, ahead, 1, false, NB, skip_last);  // visit jj + 1
            __builtin_amdgcn_sched_barrier(0);
            const int n2 = jj + 2 < last ? jj + 2 : last;
            fetch(n2, 0, e);
            const int j2 = visit[n2];
            __builtin_amdgcn_sched_barrier(0);
            float P = P0, F = F0;
            if constexpr (LDS_SC) {
                Scales ss = {};
                lds_scales(0, ss);
                accumulate(ss, cur, P, F, 1);
            } else {
                accumulate(ss0, cur, P, F, 1);
            }
            finish(j_cur, P, F, c0 + count(cur, 1));
            j_cur = j_nxt;
            j_nxt = j2;
        };
        int jj = 0;
        for (; jj + 1 < n_vel; jj += 2) {
            step(jj, va, vb);
            step(jj + 1, vb, va);
        }
        if (jj < n_vel) step(jj, va, vb);
    } else if (n_img <= NB && PF) {
        // The next velocity's table row is fetched while this velocity's
        // gathers are in flight (image 0 hoisted as above).
        if constexpr (LDS_SC) hoist_image0(sc_lds[0], sc_lds[1]);
        else hoist_image0(ss0[0].x, ss0[0].y);
        i32x4 e[NB];
        fetch(0, 0, e);
        int j_next = visit[0];
        for (int jj = 0; jj < n_vel; ++jj) {
            const int j = j_next;
            LoadT v[NB];
            issue(e, v, 1, false, NB, skip_last);
            // Keep the next row's fetch right behind the gathers (the scheduler
            // would otherwise sink it below the sums).
            __builtin_amdgcn_sched_barrier(0);
            const int jn = jj + 1 < n_vel ? jj + 1 : jj;
            fetch(jn, 0, e);
            j_next = visit[jn];
            __builtin_amdgcn_sched_barrier(0);
            float P = P0, F = F0;
            if constexpr (LDS_SC) {
                Scales ss = {};
                lds_scales(0, ss);
                accumulate(ss, v, P, F, 1);
            } else {
                accumulate(ss0, v, P, F, 1);
            }
            finish(j, P, F, c0 + count(v, 1));
        }
    } else if (n_img <= NB) {
        for (int jj = 0; jj < n_vel; ++jj) {
            const int j = visit[jj];
            i32x4 e[NB];
            fetch(jj, 0, e);
            LoadT v[NB];
            issue(e, v, 0, false, NB);
            float P = 0.f, F = 0.f;
            if constexpr (LDS_SC) {
                Scales ss = {};
                lds_scales(0, ss);
                accumulate(ss, v, P, F, 0);
            } else {
                accumulate(ss0, v, P, F, 0);
            }
            finish(j, P, F, count(v, 0));
        }
    } else {
        serial_path();
    }
}

// The search of one tile (start row `row`, start columns seg*64 .. seg*64+63).
// All scalar arguments are wave-uniform.  INTERIOR: every displaced row of
// this start row is inside the frame, so the gathers skip the row check.
template <int KM, int NB, int PB, int FMT, bool PF, bool MB, bool INTERIOR = false>
__device__ __forceinline__ void search_tile(
    uint32_t *lds, const void *__restrict__ planes, const float2 *__restrict__ inv_scale,
    int n_img, int h, int w, const GatherEntry *__restrict__ disp, int disp_stride,
    const int32_t *__restrict__ vel_index, int n_vel, int k_cand, int row, int seg,
    float *__restrict__ cand_nu, float *__restrict__ cand_alpha, int32_t *__restrict__ cand_vel,
    int16_t *__restrict__ cand_nobs) {
    uint32_t *q_hi = lds;
    uint32_t *q_lo = lds + PB * 64;
    float *q_al = reinterpret_cast<float *>(lds + 2 * PB * 64);

    const int lane = (int)threadIdx.x;

    // The list (slots 0..KM-1, descending); with the network merge, slots
    // KM..KM+15 receive the queued batch during a merge.
    // Longer lists merge one queued entry at a time where the 16 batch slots
    // would not fit beside the list (16-bit planes also hold their scales).
    constexpr bool kNet = KM >= 16 && PB == 16 &&
                          KM <= (FMT == KB_F32 ? KBMI_NET_MAX_F32 : KBMI_NET_MAX_LP);
    constexpr int KR = kNet ? KM + 16 : KM;
    uint64_t key[KR];
    float al[KR];
#pragma unroll
    for (int s = 0; s < KR; ++s) {
        key[s] = 0;
        al[s] = 0.f;
    }
    uint64_t thr = 0;   // admission threshold (list tail at the last merge)
    int nq = 0;         // queued candidates of this lane

    // One pass of the insertion network: slot s keeps the larger key, the
    // smaller moves on (keys within a pixel are distinct, so one compare
    // decides where alpha goes).
    auto insert = [&](uint64_t nk, float a) {
#pragma unroll
        for (int s = 0; s < KM; ++s) {
            const bool c = nk > key[s];
            key_exchange(key[s], nk);
            const float ta = c ? al[s] : a;
            al[s] = c ? a : al[s];
            a = ta;
        }
    };
    auto merge_queue = [&]() {
        if constexpr (kNet) {
            // The lane's queue (entries past nq read as empty) into the batch
            // slots, then one network merge.
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                const uint64_t nk = ((uint64_t)q_hi[b * 64 + lane] << 32) | q_lo[b * 64 + lane];
                const float na = q_al[b * 64 + lane];
                key[KM + b] = b < nq ? nk : 0;
                al[KM + b] = b < nq ? na : 0.f;
            }
            net_merge<KM>(key, al);
        } else {
            for (int b = 0; b < PB; ++b) {
                if (!__any(b < nq)) break;
                if (b < nq) {
                    const uint64_t nk =
                        ((uint64_t)q_hi[b * 64 + lane] << 32) | q_lo[b * 64 + lane];
                    if (nk > key[KM - 1]) insert(nk, q_al[b * 64 + lane]);
                }
            }
        }
        nq = 0;
        thr = key[KM - 1];
    };
    // Score one trajectory (Sec. 2.1.5: nu = Psi / sqrt(Phi), alpha = Psi / Phi)
    // and queue it if it beats the admission threshold.  n_obs sits in the
    // low bits of the key and never decides an order.
    auto finish = [&](int j, float P, float F, uint32_t c) {
        const float r = inv_sqrt_phi(F);
        const float nu = score_nu(P, F, r);
        const uint64_t nk = make_key(nu, j, 0u);
        if (nk > thr) {
            q_hi[nq * 64 + lane] = (uint32_t)(nk >> 32);
            q_lo[nq * 64 + lane] = (uint32_t)nk | c;
            q_al[nq * 64 + lane] = score_alpha(P, nu, F, r);
            ++nq;
        }
        if (__any(nq == PB)) merge_queue();
    };

    // Two velocities' gathers fit beside the list up to KM = 50 with float32
    // loads and up to KM = 56 with 16-bit loads, whose scales then sit in LDS
    // (longer lists spill registers with the second load buffer).
    visit_velocities<NB, FMT, PF,
                     (KBMI_PIPELINE != 0 && KM <= (FMT == KB_F32 ? 50 : KBMI_PIPE_MAX_LP)), MB,
                     INTERIOR,
                     (FMT != KB_F32 && KM >= KBMI_LP_SC_MIN_KM)>(
        reinterpret_cast<float *>(lds + search_queue_words<KM, PB>()), planes, inv_scale, n_img,
        h, w, disp, disp_stride, vel_index, n_vel, row, seg, finish);
    merge_queue();

    // Write the rank-ordered list: stage each field through LDS so that the
    // wave's stores cover the contiguous [pixels][k_cand] run of its pixels
    // (one pixel's k_cand <= 64 entries per store instruction).
    const int npx = (w - seg * 64) < 64 ? (w - seg * 64) : 64;
    const size_t base = ((size_t)row * (size_t)w + (size_t)seg * 64) * (size_t)k_cand;
    __syncthreads();
#pragma unroll
    for (int field = 0; field < 4; ++field) {
#pragma unroll
        for (int s = 0; s < KM; ++s) {
            uint32_t v;
            if (field == 0) v = __float_as_uint(key_nu(key[s]));
            else if (field == 1) v = __float_as_uint(al[s]);
            else if (field == 2) v = (uint32_t)key_vel(key[s]);
            else v = (uint32_t)key_nobs(key[s]);
            lds[lane * KM + s] = v;
        }
        __syncthreads();
        if (lane < k_cand) {
            for (int p = 0; p < npx; ++p) {
                const uint32_t v = lds[p * KM + lane];
                const size_t o = base + (size_t)p * (size_t)k_cand + (size_t)lane;
                if (field == 0) cand_nu[o] = __uint_as_float(v);
                else if (field == 1) cand_alpha[o] = __uint_as_float(v);
                else if (field == 2) cand_vel[o] = (int32_t)v;
                else cand_nobs[o] = (int16_t)v;
            }
        }
        __syncthreads();
    }
}

template <int KM, int NB, int PB, int FMT, bool MB>
__global__ __launch_bounds__(64, 2) void search_kernel(
    const void *__restrict__ planes, const float2 *__restrict__ inv_scale, int n_img, int h,
    int w, const GatherEntry *__restrict__ disp, int disp_stride, const int32_t *__restrict__ vel_index,
    int n_vel, int k_cand, TileMap tiles, float *__restrict__ cand_nu,
    float *__restrict__ cand_alpha, int32_t *__restrict__ cand_vel,
    int16_t *__restrict__ cand_nobs, int row_lo, int row_hi) {
    __shared__ uint32_t lds[search_lds_words<KM, PB>()];
    int row, seg;
    tiles.map(blockIdx.x, row, seg);
    if (KBMI_INTERIOR && row >= row_lo && row < row_hi)
        search_tile<KM, NB, PB, FMT, KBMI_PREFETCH != 0, MB, true>(
            lds, planes, inv_scale, n_img, h, w, disp, disp_stride, vel_index, n_vel, k_cand,
            row, seg, cand_nu, cand_alpha, cand_vel, cand_nobs);
    else
        search_tile<KM, NB, PB, FMT, KBMI_PREFETCH != 0, MB>(
            lds, planes, inv_scale, n_img, h, w, disp, disp_stride, vel_index, n_vel, k_cand,
            row, seg, cand_nu, cand_alpha, cand_vel, cand_nobs);
}

// The single-stack search in the persistent order (large frames).
template <int KM, int NB, int PB, int FMT, bool MB>
__global__ __launch_bounds__(64, 2) void search_persistent_kernel(
    const void *__restrict__ planes, const float2 *__restrict__ inv_scale, int n_img, int h,
    int w, const GatherEntry *__restrict__ disp, int disp_stride,
    const int32_t *__restrict__ vel_index, int n_vel, int k_cand, PersistMap pm,
    float *__restrict__ cand_nu, float *__restrict__ cand_alpha, int32_t *__restrict__ cand_vel,
    int16_t *__restrict__ cand_nobs, uint32_t *sync, int row_lo, int row_hi) {
    __shared__ uint32_t lds[search_lds_words<KM, PB>()];
    uint32_t *xcd_count = sync + (blockIdx.x & 7);
    const uint32_t per_xcd = gridDim.x >> 3;
    int spin = pm.spin;   // 0 once a wait has timed out (the XCD's workgroups are
                          // not all resident, e.g. beside another launch)
    for (int gen = 0; gen < pm.generations; ++gen) {
        int row, seg;
        if (pm.map(gen, (int)blockIdx.x, row, seg)) {
            if (KBMI_INTERIOR && row >= row_lo && row < row_hi)
                search_tile<KM, NB, PB, FMT, KBMI_PREFETCH != 0, MB, true>(
                    lds, planes, inv_scale, n_img, h, w, disp, disp_stride, vel_index, n_vel,
                    k_cand, row, seg, cand_nu, cand_alpha, cand_vel, cand_nobs);
            else
                search_tile<KM, NB, PB, FMT, KBMI_PREFETCH != 0, MB>(
                    lds, planes, inv_scale, n_img, h, w, disp, disp_stride, vel_index, n_vel,
                    k_cand, row, seg, cand_nu, cand_alpha, cand_vel, cand_nobs);
        }
        // Generation boundary: wait (a bounded time) until every workgroup of
        // this XCD has finished the generation, so its waves start the next
        // block together.  The wait only shapes timing; no result depends on it.
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

__global__ void zero_words_kernel(uint32_t *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Batched search: one persistent launch covers the tiles of several stacks
// (the serving path).  The grid is the number of workgroups the GPU holds at
// once; in generation g, workgroup w processes work item g * grid + w (see
// BatchJob), then waits with the others of its XCD as in the single-stack
// persistent search.  Each tile runs exactly the single-stack search, so a
// stack's results do not depend on what it is batched with.
// ---------------------------------------------------------------------------
template <int KM, int NB, int PB, int FMT, bool MB>
__global__ __launch_bounds__(64, 2) void search_batch_kernel(const BatchJob *__restrict__ jobs_,
                                                             int n_jobs, int generations,
                                                             int spin, int k_cand,
                                                             uint32_t *sync) {
    __shared__ uint32_t lds[search_lds_words<KM, PB>()];
    // The descriptors do not change during the launch: read through the
    // constant address space, their fields stay in scalar registers.
    typedef __attribute__((address_space(4))) const BatchJob CJob;
    const CJob *jobs = (const CJob *)(const void *)jobs_;
    uint32_t *xcd_count = sync + (blockIdx.x & 7);
    const int grid = (int)gridDim.x;
    const uint32_t per_xcd = gridDim.x >> 3;
    int j = 0;
    for (int gen = 0; gen < generations; ++gen) {
        const int item = gen * grid + (int)blockIdx.x;
        while (j + 1 < n_jobs && item >= jobs[j + 1].item_begin) ++j;
        const CJob &jb = jobs[j];
        const int li = item - jb.item_begin;
        int row = 0, seg = 0;
        bool ok;
        if (jb.dense) {
            ok = li < jb.nseg * jb.h;
            if (ok) strip_tile(li, jb.nseg, jb.h, jb.strip, row, seg);
        } else {
            PersistMap pm;
            pm.nseg = jb.nseg;
            pm.h = jb.h;
            pm.bs = jb.bs;
            pm.brows = jb.brows;
            pm.nbc = jb.nbc;
            pm.nbr = jb.nbr;
            const int gl = li / grid;
            ok = gl < ((jb.nbc + 7) / 8) * jb.nbr && pm.map(gl, li - gl * grid, row, seg);
        }
        if (ok)
            search_tile<KM, NB, PB, FMT, KBMI_PREFETCH != 0, MB>(
                lds, jb.planes, jb.inv_scale, jb.n_img, jb.h, jb.w, jb.disp, jb.disp_stride,
                jb.vel_index, jb.n_vel, k_cand, row, seg, jb.cand_nu, jb.cand_alpha,
                jb.cand_vel, jb.cand_nobs);
        // Generation boundary (as in the single-stack persistent search).
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

}  // namespace
}  // namespace kbmi
