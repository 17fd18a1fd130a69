// Device building blocks: precision types, sliced-ELL matrix view, block
// reductions with a deterministic last-work-group finish.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "amp_controller.hpp"

namespace amp {

typedef _Float16 half_t;

constexpr int NT = 256;      // threads per work-group of every kernel
constexpr int WAVE = 64;     // CDNA wavefront width
constexpr int SLICE = 64;    // sliced-ELL slice height (one row per lane)
constexpr int VEC = 4;       // consecutive elements per thread in streaming kernels
constexpr int GMAX = 2048;   // upper bound on work-groups of a reducing kernel
constexpr int PAD = NT * VEC;  // internal vectors are padded to a multiple of this

template <int U> struct Prec;
template <> struct Prec<64> { typedef double T; typedef double C; };
template <> struct Prec<32> { typedef float T; typedef float C; };
template <> struct Prec<16> { typedef half_t T; typedef float C; };  // FP16 storage, FP32 arithmetic

// Sliced ELL: slice s holds rows [64 s, 64 s + 64), its entries column-major
// (slot sptr[s] + 64 j + lane is entry j of row 64 s + lane).  Padding slots
// have col = row and value 0.
struct Sell {
    int64_t n, np, nslices;
    const int64_t *sptr;
    const int32_t *col;
    const double *v64;   // FP64 values
    const float *v32;    // FP32 values, diagonal slot = fl32(row sum) (difference form)
    const float *v32p;   // FP32 values, plain
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Sum over the work-group, identical order on every call; result in all threads.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[NT / WAVE];
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i) t += sh[i];
    return t;
}

// Atomic max of a non-negative double through its bit pattern (order
// independent, so deterministic).  NaN compares above +inf.
__device__ __forceinline__ void atomic_max_abs(unsigned long long *dst, double v_nonneg) {
    unsigned long long bits = (unsigned long long)__double_as_longlong(v_nonneg);
    atomicMax(dst, bits);
}

__device__ __forceinline__ double bits_to_double(unsigned long long b) {
    return __longlong_as_double((long long)b);
}

// Block-level max then one atomic per work-group.
__device__ __forceinline__ void block_max_to(unsigned long long *dst, double v) {
    v = wave_max(v);
    if ((threadIdx.x % WAVE) == 0) atomic_max_abs(dst, v);
}

// Publish this work-group's partial sums and report whether it is the last
// work-group to finish.  In the last work-group every thread may read all
// partials afterwards.
__device__ __forceinline__ bool arrive_last(Ctrl *c, double *part, const double *vals, int nv) {
    __shared__ int last;
    if (threadIdx.x == 0) {
        for (int j = 0; j < nv; ++j) part[j * gridDim.x + blockIdx.x] = vals[j];
        __threadfence();
        unsigned int t = __hip_atomic_fetch_add(&c->counter, 1u, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// Fixed-order total of one partial array (called by the whole last work-group).
__device__ __forceinline__ double finish_sum(const double *part) {
    double s = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += NT) s += part[i];
    return block_sum(s);
}

}  // namespace amp
