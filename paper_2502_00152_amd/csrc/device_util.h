// Device helpers: complex arithmetic on double2, fixed-order block reductions
// and the XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>

namespace hisq {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, 32 CUs each

// ------------------------------------------------------------ complex math
__device__ __forceinline__ void cmac(double2 &acc, double2 a, double2 b) {
    // acc += a * b
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

__device__ __forceinline__ void cmac_conj(double2 &acc, double2 a, double2 b) {
    // acc += conj(a) * b
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}

__device__ __forceinline__ double redot(double2 a, double2 b) {
    // Re(conj(a) * b)
    return fma(a.x, b.x, a.y * b.y);
}

// ------------------------------------------------------------- block order
// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8).  Renumber them so that each XCD receives one contiguous range of
// logical blocks: neighbouring sites then share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
    const int q = nblocks / kNumXcd, r = nblocks % kNumXcd;
    const int x = b % kNumXcd, j = b / kNumXcd;
    return x * q + (x < r ? x : r) + j;
}

// Chunks of n logical blocks dealt round-robin to the XCDs: XCD x takes the
// chunks x, x + 8, x + 16, ...  All XCDs then work on the same stretch of 8 n
// blocks at the same time, so the data around it is shared in the
// last-level cache, while the n consecutive blocks of a chunk share the
// XCD's L2.  The tail that does not fill a whole round keeps dispatch order.
__device__ __forceinline__ int xcd_block_chunked(int b, int nblocks, int n) {
    const int x = b % kNumXcd, j = b / kNumXcd;
    const int rounds = nblocks / (kNumXcd * n);
    if (j >= rounds * n) return b;
    return ((j / n) * kNumXcd + x) * n + j % n;
}

// Logical block of workgroup b for a remap mode: 0 dispatch order, 1 one
// contiguous range per XCD, n >= 2 chunks of n blocks round-robin.
__device__ __forceinline__ int remap_block(int mode, int b, int nblocks) {
    return mode == 1 ? xcd_block(b, nblocks) : mode > 1 ? xcd_block_chunked(b, nblocks, mode) : b;
}

// ---------------------------------------------------------- reductions
// Sum over the 64 lanes of a wave, in a fixed order; result in every lane.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Block-wide sum of NV values per thread.  The result is returned in thread 0
// (other threads get unspecified values).  `lds` holds NV * (BS/64) doubles.
template <int NV, int BS>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    constexpr int NW = BS / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) lds[j * NW + w] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double s = 0.0;
            for (int k = 0; k < NW; ++k) s += lds[j * NW + k];
            v[j] = s;
        }
    }
    __syncthreads();
}

}  // namespace hisq
