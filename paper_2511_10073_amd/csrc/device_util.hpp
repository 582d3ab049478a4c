// Wave64 / workgroup reduction and scan helpers (gfx950: 64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ahr {

constexpr int kWave = 64;

// A pointer into device global memory (address space 1).  Loads through it
// are global loads even where the address was formed as an integer, which
// would otherwise give flat loads that also count against the LDS counter.
template <class T>
using GlobalPtr = const __attribute__((address_space(1))) T*;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}

// Inclusive scan over the wave.
__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t v) {
    int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int64_t u = __shfl_up(v, o);
        if (l >= o) v += u;
    }
    return v;
}

// Block-wide sum; every thread gets the result. red: BT/64 slots.
template <int BT>
__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t* red) {
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int w = 0; w < BT / kWave; ++w) t += red[w];
    return t;
}

// Fixed-order block sum of doubles (deterministic for a given block size).
template <int BT>
__device__ __forceinline__ double block_sum_f64(double v, double* red) {
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double t = 0;
#pragma unroll
    for (int w = 0; w < BT / kWave; ++w) t += red[w];
    return t;
}

// Block exclusive scan of int64; *total gets the block sum. red: BT/64 slots.
template <int BT>
__device__ __forceinline__ int64_t block_exclusive_scan_i64(int64_t v, int64_t* red, int64_t* total) {
    int64_t inc = wave_incl_scan_i64(v);
    __syncthreads();
    if (lane_id() == kWave - 1) red[wave_id()] = inc;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BT / kWave; ++w) {
        int64_t r = red[w];
        if (w < wave_id()) before += r;
        tot += r;
    }
    *total = tot;
    return before + inc - v;
}

// Ordered compaction inside a block: returns the slot of a set flag among
// the set flags of this pass (in thread order) and the pass total.
template <int BT>
__device__ __forceinline__ int block_rank(bool flag, int* red, int* total) {
    uint64_t m = __ballot(flag);
    int l = lane_id();
    uint64_t lt = l ? (~0ull >> (kWave - l)) : 0ull;
    int in_wave = __popcll(m & lt);
    __syncthreads();
    if (l == 0) red[wave_id()] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BT / kWave; ++w) {
        int r = red[w];
        if (w < wave_id()) before += r;
        tot += r;
    }
    *total = tot;
    return before + in_wave;
}

__device__ __forceinline__ float bits_f(int v) { return __int_as_float(v); }
__device__ __forceinline__ int f_bits(float v) { return __float_as_int(v); }

}  // namespace ahr
