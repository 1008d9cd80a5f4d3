// Wave64 / workgroup prefix-sum helpers (device only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pp {

constexpr int kWave = 64;

__device__ inline int lane_id() { return __lane_id(); }

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ inline int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int t = __shfl_up(v, off, kWave);
    if (lane >= off) v += t;
  }
  return v;
}

__device__ inline int wave_sum(int v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Exclusive prefix sum over a workgroup of BLOCK threads; returns the
// exclusive value for this thread and writes the block total to *total.
// `lds` must hold BLOCK/64 + 1 ints.  Contains __syncthreads().
template <int BLOCK>
__device__ inline int block_excl_scan(int v, int* lds, int* total) {
  constexpr int NW = BLOCK / kWave;
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  const int incl = wave_incl_scan(v);
  if (lane == kWave - 1) lds[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int i = 0; i < NW; ++i) {
      int t = lds[i];
      lds[i] = acc;
      acc += t;
    }
    lds[NW] = acc;
  }
  __syncthreads();
  const int res = lds[w] + incl - v;
  *total = lds[NW];
  __syncthreads();
  return res;
}

}  // namespace pp
