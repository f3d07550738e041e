// Device helpers: deterministic reductions and the last-block pattern.
#pragma once

#include <hip/hip_runtime.h>

namespace tosimp {

// Sum over a 64-lane wavefront with a fixed butterfly order (deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block sum for NT threads; result valid in thread 0.  sbuf holds NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sbuf) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sbuf[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += sbuf[i];
  }
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* sbuf) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sbuf[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r = fmax(r, sbuf[i]);
  }
  __syncthreads();
  return r;
}

// Called by every thread of a block after thread 0 stored the block's partial.
// Returns true in exactly one block: the last of `expected` arriving blocks.  The
// release fence before the counter increment and the acquire fence after it make
// every other block's partial visible to the last block (agent scope, across XCDs).
__device__ __forceinline__ bool last_block_arrive(unsigned* cnt, unsigned expected) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned t = atomicAdd(cnt, 1u);
    s_last = (t == expected - 1u);
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

// Sum n partials (stride `stride` doubles apart) in a fixed order; valid in thread 0.
template <int NT>
__device__ __forceinline__ double sum_partials(const double* part, int n, int stride,
                                               double* sbuf) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += part[(size_t)i * stride];
  return block_sum<NT>(s, sbuf);
}

template <int NT>
__device__ __forceinline__ double max_partials(const double* part, int n, int stride,
                                               double* sbuf) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s = fmax(s, part[(size_t)i * stride]);
  return block_max<NT>(s, sbuf);
}

template <typename T>
__device__ __forceinline__ bool finite_val(T v) {
  return v == v && v - v == T(0);
}

}  // namespace tosimp
