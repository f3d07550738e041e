// Device helpers: deterministic block reductions and two-kernel grid reductions.
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

// Grid reductions take two launches: the reduction kernel stores NV block sums per block
// (store_block_sums) and a one-block finalize kernel adds them in block order and hands
// the totals to a functor (thread 0), which updates the solver state.  The kernel
// boundary orders the two.  A single-kernel "last block finishes" scheme needs a
// device-scope release fence in every block, which on a multi-XCD GPU writes back that
// XCD's L2 cache: thousands of such fences cost far more than the second launch.
template <int NV, int NT = 256>
__device__ __forceinline__ void store_block_sums(const double (&v)[NV], double* partials,
                                                 double* sbuf) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = block_sum<NT>(v[k], sbuf);
    if (threadIdx.x == 0) partials[(size_t)NV * blockIdx.x + k] = s;
  }
}

// Each thread adds the partials i = t, t + 256, t + 512, ... of every sum in increasing i
// (the order fixes the result bit for bit); the loads of U consecutive strides are
// issued before their additions, so a thread waits for about n / (256 U) load latencies
// instead of n / 256.
template <int NV, typename F>
__global__ __launch_bounds__(256) void finalize_sum_kernel(const double* partials, int nb, F f) {
  constexpr int NT = 256;
  constexpr int U = NV <= 2 ? 8 : (NV <= 4 ? 4 : 2);
  __shared__ double sbuf[4];
  double s[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) s[k] = 0.0;
  int i = threadIdx.x;
  for (; i + (U - 1) * NT < nb; i += U * NT) {
    double v[U][NV];
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int k = 0; k < NV; ++k) v[j][k] = partials[(size_t)NV * (i + j * NT) + k];
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += v[j][k];
  }
  for (; i < nb; i += NT)
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] += partials[(size_t)NV * i + k];
  double tot[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = block_sum<NT>(s[k], sbuf);
  if (threadIdx.x == 0) f(tot);
}

template <typename F>
__global__ __launch_bounds__(256) void finalize_max_kernel(const double* partials, int nb, F f) {
  __shared__ double sbuf[4];
  double tot[1];
  tot[0] = max_partials<256>(partials, nb, 1, sbuf);
  if (threadIdx.x == 0) f(tot);
}

template <int NV, typename F>
inline hipError_t launch_finalize_sum(hipStream_t s, const double* partials, int nb, F f) {
  finalize_sum_kernel<NV, F><<<1, 256, 0, s>>>(partials, nb, f);
  return hipGetLastError();
}

template <typename F>
inline hipError_t launch_finalize_max(hipStream_t s, const double* partials, int nb, F f) {
  finalize_max_kernel<F><<<1, 256, 0, s>>>(partials, nb, f);
  return hipGetLastError();
}

// XCD-major item layout for kernels whose items read neighbours one plane of the mesh
// away: the hardware deals blocks to the 8 XCDs round-robin (block b runs on XCD b % 8),
// so block b takes slot (b % 8) per_xcd + b / 8 and each XCD sweeps one contiguous range
// of items; a neighbouring plane is then read by the XCD that already holds it in its L2.
// Launch 8 per_xcd blocks with per_xcd = ceil(ceil(n / blockDim) / 8); items >= n return.
__device__ __forceinline__ int64_t xcd_item(int per_xcd) {
  const int b = blockIdx.x;
  const int64_t slot = (int64_t)(b & 7) * per_xcd + (b >> 3);
  return slot * blockDim.x + threadIdx.x;
}

inline int xcd_per(int64_t n, int threads) {
  return (int)(((n + threads - 1) / threads + 7) / 8);
}

template <typename T>
__device__ __forceinline__ bool finite_val(T v) {
  return v == v && v - v == T(0);
}

}  // namespace tosimp
