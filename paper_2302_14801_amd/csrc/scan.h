// scan.h -- wave64 / workgroup prefix sums used by several kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lod {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations and meets the other waves, but, unlike
// __syncthreads(), does not wait for outstanding global loads and stores, so
// prefetched loads and stores stay in flight across it.  Use __syncthreads()
// where waves exchange data through global memory.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Inclusive scan across the 64 lanes of a wavefront.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T t = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += t;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Exclusive scan over a workgroup of WG threads (WG a multiple of 64, at most
// 1024).  `sh` must hold WG/64 + 1 values.  Returns the exclusive prefix of the
// calling thread and writes the workgroup total to *total.  Contains barriers:
// every thread of the workgroup must call it.
template <int WG, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* sh, T* total) {
  constexpr int NW = WG / 64;
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x / 64;
  T inc = wave_incl_scan(v);
  if (lane == 63) sh[w] = inc;
  lds_barrier();
  if (threadIdx.x == 0) {
    T s = 0;
    for (int i = 0; i < NW; ++i) {
      T t = sh[i];
      sh[i] = s;
      s += t;
    }
    sh[NW] = s;
  }
  lds_barrier();
  T r = sh[w] + inc - v;
  *total = sh[NW];
  lds_barrier();
  return r;
}

}  // namespace lod
