// Device building blocks: precision types, sliced-ELL matrix view, block
// reductions, XCD-aware work distribution.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "amp_controller.hpp"

namespace amp {

typedef _Float16 half_t;

#ifndef AMP_NT
#define AMP_NT 256
#endif
constexpr int NT = AMP_NT;   // threads per work-group of the streaming kernels (a multiple of 64)
#ifndef AMP_NTS
#define AMP_NTS 256
#endif
constexpr int NTS = AMP_NTS; // threads per work-group of the sliced-ELL kernels (a multiple of 64)
// Threads per work-group of the iteration's product kernel, and the minimum
// waves per SIMD its FP16/FP32 variants are compiled for.  Measured on the
// 256^3 Q1 solve (product launch average): 16 slots per pass at 4 waves
// 626 us, at 5 or 6 waves 637-658 us; 8 slots per pass 649 us at 4-6
// waves and 773 us at 8 (64 VGPRs); 24 or 32 slots per pass 880-1256 us.
#ifndef AMP_NTP
#define AMP_NTP 512
#endif
constexpr int NTP = AMP_NTP;
#ifndef AMP_SPMV_WAVES
#define AMP_SPMV_WAVES 4
#endif
constexpr int WAVE = 64;     // CDNA wavefront width
constexpr int SLICE = 64;    // sliced-ELL slice height (one row per lane)
constexpr int VEC = 4;       // consecutive elements per thread in streaming kernels
#ifndef AMP_GMAX
#define AMP_GMAX 1024
#endif
constexpr int GMAX = AMP_GMAX;   // upper bound on work-groups of a reducing kernel
constexpr int GSTREAM = 1024;    // upper bound on work-groups of a streaming kernel
constexpr int PAD = NT * VEC;  // internal vectors are padded to a multiple of this
// Largest n: padded vectors hold at most 2^29 entries, so the byte offset of
// any gathered FP64 entry fits 32 bits (at32).
constexpr int64_t kMaxRows = ((int64_t)1 << 29) - PAD;
constexpr int NXCD = 8;      // accelerator complex dies; work-groups are dealt to them round-robin

// Round x to the storage type T once, to nearest even.  FP64 -> FP16 is not
// a plain cast (that rounds to FP32 first and then to FP16: two roundings):
// x is rounded to FP32 with round-to-odd (the RNE result, moved to its odd
// neighbour towards x when inexact and even), and that value rounded to
// FP16; with 24 >= 11 + 2 significand bits the result is the correctly
// rounded FP16 value of x (Boldo and Melquiond, "When double rounding is
// odd", 2005).
template <typename T>
__device__ __forceinline__ T narrow(double x) {
    return (T)x;
}
template <>
__device__ __forceinline__ _Float16 narrow<_Float16>(double x) {
    float f = (float)x;
    if ((double)f != x && !__builtin_isinf(f) && !__builtin_isnan(f) && !(__float_as_uint(f) & 1u))
        f = nextafterf(f, (double)f < x ? __builtin_inff() : -__builtin_inff());
    return (_Float16)f;
}
template <typename T>
__device__ __forceinline__ T narrow(float x) {
    return (T)x;
}

template <int U> struct Prec;
template <> struct Prec<64> { typedef double T; typedef double C; };
template <> struct Prec<32> { typedef float T; typedef float C; };
template <> struct Prec<16> { typedef half_t T; typedef float C; };  // FP16 storage, FP32 arithmetic

// Sliced ELL: slice s holds rows [64 s, 64 s + 64), its entries column-major
// (slot sptr[s] + 64 j + lane is entry j of row 64 s + lane).  A slice is
// stored in one of two modes:
//  * index mode (soff[s] < 0): slot j of a row holds the row's j-th entry and
//    its column in col[]; padding slots have col = row and value 0;
//  * offset mode (soff[s] >= 0): slot j of every row of the slice holds the
//    entry at column row + offs[soff[s] + j] (one shared, sorted list of
//    column offsets per slice, value 0 where the row has no such entry), so
//    no per-entry column index is read.  Stencil matrices in natural order
//    store every slice this way.
// Per-slice descriptor of the product kernels (16 bytes).
struct alignas(16) SliceRec {
    int64_t ptr;    // first slot of the slice
    int32_t soff;   // start of the slice's offset list (offset mode) or -1 (index mode)
    int32_t width;  // slots per row
};

// Column-offset lists as constant-address-space memory (they do not change
// during a launch): wave-uniform reads of them compile to scalar loads.
typedef const __attribute__((address_space(4))) int32_t *KOffs;

struct Sell {
    int64_t n, np, nslices;
    const SliceRec *srec;
    const int64_t *sptr;
    const int32_t *col;
    const int32_t *soff;  // per slice: start of its offsets in offs, or -1
    const int32_t *offs;
    KOffs koffs;          // offs, for scalar reads
    int64_t guard;        // zero margin (elements) around the gathered z and p vectors
    int lgL;              // log2 of the lanes per row (0: one row per lane; > 0 only with index-mode slices)
    const double *v64;   // FP64 values
    const float *v32;    // FP32 values, diagonal slot = fl32(row sum) (difference form)
    const float *v32p;   // FP32 values, plain
};

constexpr int kOffMax = 32;  // longest per-slice offset list
// Capacity of the memory-side cache.  A matrix plane larger than this is
// streamed from HBM every application anyway, and the product and Chebyshev
// step load it with a non-temporal hint so it does not displace the
// gathered vectors; a smaller one stays cached between applications, which
// the hint would prevent.
constexpr int64_t kMallBytes = (int64_t)256 << 20;

// Issue priority from a wave's progress through its work-group's range.
// The work-groups sharing a CU start together, but the hardware favours the
// oldest waves: left alone, the first work-group finishes microseconds
// before the last, and the CU runs that tail with few loads in flight.  A
// wave that is ahead lowers its priority so the others catch up.  Timing
// only: no result depends on it.
__device__ __forceinline__ void progress_prio(int64_t done, int64_t span) {
    if (done * 4 >= span * 3) __builtin_amdgcn_s_setprio(0);
    else if (done * 2 >= span) __builtin_amdgcn_s_setprio(1);
    else if (done * 4 >= span) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(3);
}

// a[i] through a 32-bit byte offset from a base pointer the whole wave
// shares: the load takes its base from scalar registers and one offset
// register per lane, with no 64-bit address arithmetic per slot.  For
// gathers by row index: i < np <= 2^29 keeps i * sizeof(T) below 2^32.
template <typename T>
__device__ __forceinline__ T at32(const T *a, uint32_t i) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(a) + i * (uint32_t)sizeof(T));
}

// at32 with a non-temporal hint: for data streamed once per launch (matrix
// values, a row's own vector entries), so it does not displace the gathered
// vectors from the caches.
template <typename T>
__device__ __forceinline__ T at32nt(const T *a, uint32_t i) {
    return __builtin_nontemporal_load(reinterpret_cast<const T *>(reinterpret_cast<const char *>(a) + i * (uint32_t)sizeof(T)));
}

// at32nt when NT, else at32 (chosen at compile time: a run-time choice
// between two loads of one address may be merged into one plain load).
template <bool NT, typename T>
__device__ __forceinline__ T at32t(const T *a, uint32_t i) {
    if constexpr (NT) return at32nt(a, i);
    else return at32(a, i);
}

// a[i] = v through a 32-bit byte offset (as at32).
template <typename T>
__device__ __forceinline__ void st32(T *a, uint32_t i, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(a) + i * (uint32_t)sizeof(T)) = v;
}

// Columns of slots j0 .. j0 + kChunk - 1 of one row of a slice, one functor
// per storage mode.  Slots at or past the row width w give a valid column
// (the caller adds nothing for them).
#ifndef AMP_CHUNK
#define AMP_CHUNK 8
#endif
constexpr int kChunk = AMP_CHUNK;   // 4 or 8

struct alignas(4 * kChunk) OffChunk {
    int32_t o[kChunk];
};

struct OffCols {
    const int32_t *offs;  // the slice's offset list: aligned to and padded with 0 to a multiple of kChunk
    int64_t row, np;
    __device__ __forceinline__ void chunk(int j0, int /*w*/, int32_t *c, bool *dg) const {
        const OffChunk o = *reinterpret_cast<const OffChunk *>(offs + j0);   // one scalar load
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            // row + o in [0, np) as one unsigned 32-bit test: row < np < 2^31
            // and |o| < 2^31, so a negative sum wraps to at least 2^31
            const uint32_t cc = (uint32_t)row + (uint32_t)o.o[u];
            c[u] = (int32_t)(cc < (uint32_t)np ? cc : (uint32_t)row);
            dg[u] = o.o[u] == 0;
        }
    }
};

struct IdxCols {
    const int32_t *col;   // &col[sptr[s] + lane]
    int64_t row;
    __device__ __forceinline__ void chunk(int j0, int w, int32_t *c, bool *dg) const {
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int j = j0 + u < w ? j0 + u : w - 1;
            c[u] = col[(int64_t)j * SLICE];
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) dg[u] = c[u] == row;
    }
};

// A slice's descriptor is fetched one slice ahead with a vector load (four
// lanes read its four words; loads complete in order, so waiting for it
// does not wait for the scalar loads of the current slice), then broadcast.
__device__ __forceinline__ uint32_t rec_word(const SliceRec *srec, int64_t s, int64_t hi) {
    return (s < hi) ? reinterpret_cast<const uint32_t *>(srec + s)[threadIdx.x & 3] : 0u;
}

__device__ __forceinline__ SliceRec rec_from(uint32_t v) {
    SliceRec r;
    const uint32_t lo = __builtin_amdgcn_readlane(v, 0), hi = __builtin_amdgcn_readlane(v, 1);
    r.ptr = (int64_t)(((uint64_t)hi << 32) | lo);
    r.soff = (int32_t)__builtin_amdgcn_readlane(v, 2);
    r.width = (int32_t)__builtin_amdgcn_readlane(v, 3);
    return r;
}

template <typename F>
__device__ __forceinline__ void with_rec_cols(const SliceRec &r, const int32_t *col, const int32_t *offs, int64_t np,
                                              int64_t sl, int lane, F &&f) {
    const int64_t row = sl * SLICE + lane;
    if (r.soff >= 0) f(OffCols{offs + r.soff, row, np});
    else f(IdxCols{col + r.ptr + lane, row});
}

// f(cols) with the column functor of slice sl's mode.  The mode is uniform
// over the wave (one slice per wave), so each mode's loop is compiled
// without per-slot branches.
template <typename F>
__device__ __forceinline__ void with_cols(const int64_t *sptr, const int32_t *col, const int32_t *soff,
                                          const int32_t *offs, int64_t np, int64_t sl, int lane, F &&f) {
    const int32_t so = __builtin_amdgcn_readfirstlane(soff[sl]);   // multiple of kChunk, or -1
    const int64_t row = sl * SLICE + lane;
    if (so >= 0) f(OffCols{offs + so, row, np});
    else f(IdxCols{col + sptr[sl] + lane, row});
}

// Work-group index with consecutive indices on one XCD: dispatch deals
// work-groups to the 8 XCDs round-robin, so hardware group b runs on XCD
// b % 8; renumbering gives XCD x the contiguous block range
// [x G/8, (x+1) G/8) and thus a contiguous row range (its L2 then holds the
// rows' neighbours).  G must be a multiple of 8 for an exact split.
__device__ __forceinline__ int xcd_index(int b, int G) {
    if (G % NXCD) return b;
    return (b % NXCD) * (G / NXCD) + b / NXCD;
}
__device__ __forceinline__ int xcd_block() { return xcd_index(blockIdx.x, gridDim.x); }

// Read one dword of every 64-byte line of the first `bytes` bytes of the
// kernel's argument segment (the explicit arguments).  Issued at entry,
// these scalar loads bring the lines into the scalar cache while the first
// global loads are in flight; without them a field first used inside a
// later branch (the controller's configuration) costs a miss there.  The
// caller passes the result to pin() after its first barrier.
template <int BYTES>
__device__ __forceinline__ uint32_t touch_args() {
    const uint32_t *ka = (const uint32_t *)__builtin_amdgcn_kernarg_segment_ptr();
    uint32_t acc = 0;
#pragma unroll
    for (int o = 0; o + 4 <= BYTES; o += 64) acc ^= ka[o / 4];
    return acc;
}
__device__ __forceinline__ void pin(uint32_t v) { asm volatile("" ::"s"(v)); }

// A work-group's share of one system's work: logical index lb of G groups.
// A single-system launch uses the whole grid (grid_wg); a batched launch
// reads (system, lb) from its task table and G from the system's config.
struct Wg {
    int lb, G;
};

__device__ __forceinline__ Wg grid_wg() { return Wg{xcd_block(), (int)gridDim.x}; }

// The same for a launch whose grid size G the caller passes as an argument
// (the iteration kernels: their first loads then wait for nothing but the
// preloaded arguments).  G must be the launch's grid size.
__device__ __forceinline__ Wg launch_wg(int G) { return Wg{xcd_index(blockIdx.x, G), G}; }

// [lo, hi) share of `total` units for work-group lb of G, in multiples of `quantum`.
__device__ __forceinline__ void block_range(int64_t total, int64_t quantum, int lb, int G,
                                            int64_t &lo, int64_t &hi) {
    const int64_t units = (total + quantum - 1) / quantum;
    const int64_t per = units / G, rem = units % G;
    const int64_t u0 = lb * per + (lb < rem ? lb : rem);
    const int64_t u1 = u0 + per + (lb < rem ? 1 : 0);
    lo = u0 * quantum;
    hi = u1 * quantum < total ? u1 * quantum : total;
}

// Slices of one wave when the work is dealt per XCD: XCD x (logical
// work-groups [x G/8, (x+1) G/8), see xcd_index) owns the x-th eighth of the
// slices, and that share is dealt round-robin to the XCD's waves, so the
// slices in flight on an XCD at any moment are one compact window (compact
// DRAM pages; the window's neighbours are in the XCD's L2).  The wave's
// slices are first, first + stride, ... below hi.
__device__ __forceinline__ void xcd_wave_slices(int64_t nslices, Wg wg, int nw, int wave, int64_t &first,
                                                int64_t &stride, int64_t &hi) {
    if (wg.G >= NXCD && wg.G % NXCD == 0) {
        const int per = wg.G / NXCD, x = wg.lb / per, lbx = wg.lb % per;
        int64_t lo;
        block_range(nslices, 1, x, NXCD, lo, hi);
        first = lo + (int64_t)lbx * nw + wave;
        stride = (int64_t)per * nw;
    } else {
        first = (int64_t)wg.lb * nw + wave;
        stride = (int64_t)wg.G * nw;
        hi = nslices;
    }
}

// Lane l's value of v (l uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// A double moved across lanes by a DPP pattern; lanes of rows outside
// ROW_MASK receive `ident`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v, double ident) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v), o = __builtin_bit_cast(uint64_t, ident);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u, CTRL, ROW_MASK,
                                                              0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32),
                                                              CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Wave-wide sum / maximum (all 64 lanes active), in a fixed tree of DPP
// steps: pairs, quads, half-rows, rows of 16, then rows 0+1 into row 1,
// rows 2+3 into row 3, and row 1 into rows 2-3; lane 63 holds the total,
// which every lane receives.  Every lane's result is the same value.
static_assert(WAVE == 64, "wave64 reduction");
__device__ __forceinline__ double wave_sum(double v) {
    v = v + dpp_f64<0xB1, 0xF>(v, 0.0);    // quad_perm [1,0,3,2]
    v = v + dpp_f64<0x4E, 0xF>(v, 0.0);    // quad_perm [2,3,0,1]
    v = v + dpp_f64<0x141, 0xF>(v, 0.0);   // row_half_mirror
    v = v + dpp_f64<0x140, 0xF>(v, 0.0);   // row_mirror
    v = v + dpp_f64<0x142, 0xA>(v, 0.0);   // row_bcast:15 into rows 1, 3
    v = v + dpp_f64<0x143, 0xC>(v, 0.0);   // row_bcast:31 into rows 2, 3
    return readlane_f64(v, WAVE - 1);
}

// (maxima of absolute values: 0 is the identity)
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f64<0xB1, 0xF>(v, 0.0));
    v = fmax(v, dpp_f64<0x4E, 0xF>(v, 0.0));
    v = fmax(v, dpp_f64<0x141, 0xF>(v, 0.0));
    v = fmax(v, dpp_f64<0x140, 0xF>(v, 0.0));
    v = fmax(v, dpp_f64<0x142, 0xA>(v, 0.0));
    v = fmax(v, dpp_f64<0x143, 0xC>(v, 0.0));
    return readlane_f64(v, WAVE - 1);
}

// Sum / max over the work-group (BS threads) in a fixed order; result in every thread.
template <int BS = NT>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[BS / WAVE];
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < BS / WAVE; ++i) t += sh[i];
    return t;
}

template <int BS = NT>
__device__ __forceinline__ double block_max(double v) {
    __shared__ double sh[BS / WAVE];
    v = wave_max(v);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < BS / WAVE; ++i) t = fmax(t, sh[i]);
    return t;
}

// NS sums followed by NM maxima over the work-group in one exchange; each
// result equals that of block_sum / block_max on its value (same order).
template <int NS, int NM, int BS = NT>
__device__ __forceinline__ void block_reduce(double *v) {
    constexpr int K = NS + NM, NW = BS / WAVE;
    __shared__ double sh[K][NW];
#pragma unroll
    for (int t = 0; t < K; ++t) v[t] = (t < NS) ? wave_sum(v[t]) : wave_max(v[t]);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int t = 0; t < K; ++t) sh[t][w] = v[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < K; ++t) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) r = (t < NS) ? r + sh[t][i] : fmax(r, sh[t][i]);
        v[t] = r;
    }
}

// Totals of a producer kernel's per-work-group partials (G of each), summed
// (or maxed) in the same fixed order by every work-group that calls it.
template <int BS = NT>
__device__ __forceinline__ double reduce_sum(const double *part, int G) {
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += BS) s += part[i];
    return block_sum<BS>(s);
}

template <int BS = NT>
__device__ __forceinline__ double reduce_max(const double *part, int G) {
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += BS) s = fmax(s, part[i]);
    return block_max<BS>(s);
}

// Partials of a producer kernel held in registers: thread t holds entries
// t, t + BS, ... of each of K arrays.  Loading them is split from reducing
// them so that a kernel can issue these loads together with its other
// prologue loads (state, body data) and wait for all of them once.
template <int K, int BS = NT>
struct PartRegs {
    static constexpr int J = GMAX / BS;
    double v[K][J];
};

// Entries i < G of the arrays part[t * GMAX + i], t < K (1 <= G <= GMAX).
// Slots past G load entry G - 1 (ignored by the reduction): every load is
// unconditional, so all of them are in flight at once.
template <int K, int BS = NT>
__device__ __forceinline__ void load_parts(const double *part, int G, PartRegs<K, BS> &pr) {
#pragma unroll
    for (int j = 0; j < PartRegs<K, BS>::J; ++j) {
        const int i = threadIdx.x + j * BS;
        const int ic = i < G ? i : G - 1;
#pragma unroll
        for (int t = 0; t < K; ++t) pr.v[t][j] = part[t * GMAX + ic];
    }
}

// NS sums followed by NM maxima of the first G entries of loaded partials;
// each result equals that of reduce_sum / reduce_max on its array (same
// per-thread order, same tree).
template <int NS, int NM, int BS = NT>
__device__ __forceinline__ void reduce_loaded(const PartRegs<NS + NM, BS> &pr, int G, double *out) {
    constexpr int K = NS + NM, NW = BS / WAVE;
    __shared__ double sh[K][NW];
    double v[K];
#pragma unroll
    for (int t = 0; t < K; ++t) v[t] = 0.0;
#pragma unroll
    for (int j = 0; j < PartRegs<K, BS>::J; ++j) {
        if (threadIdx.x + j * BS < G) {
#pragma unroll
            for (int t = 0; t < K; ++t) v[t] = (t < NS) ? v[t] + pr.v[t][j] : fmax(v[t], pr.v[t][j]);
        }
    }
#pragma unroll
    for (int t = 0; t < K; ++t) v[t] = (t < NS) ? wave_sum(v[t]) : wave_max(v[t]);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int t = 0; t < K; ++t) sh[t][w] = v[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < K; ++t) {
        double r = 0.0;
        for (int i = 0; i < NW; ++i) r = (t < NS) ? r + sh[t][i] : fmax(r, sh[t][i]);
        out[t] = r;
    }
}

}  // namespace amp
