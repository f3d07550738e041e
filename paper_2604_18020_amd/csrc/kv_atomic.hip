// Atomic-scatter forms of the operator y = K_c(x) v, kept beside the deterministic
// owner-computes kernel (kv.hip) as measured alternatives.
//
// Paper: Alg. "Fused Gather-GEMM-Scatter" gathers the 24 DOFs of an element, multiplies
// by E_e K_E and adds the 24 results into y with atomic additions, after y has been
// cleared.  Two forms are built here:
//  * element: that algorithm as stated, one thread per element, 24 global atomic
//    additions per element (K_E applied in the same exact Hadamard factorisation as the
//    main kernel, so the comparison isolates the scatter).
//  * brick: the additions reduced in LDS first.  A block takes an 8 x 8 x 4 brick of
//    elements, stages its 9 x 9 x 5 node window of v in LDS, adds every element's 24
//    results into LDS accumulators (LDS atomics), then writes each window node once:
//    nodes whose every element lies in the brick with a plain store, nodes on the brick's
//    faces (shared with neighbouring bricks) with a global atomic addition.
// Both clear y first (one pass that writes 0 on free DOFs and v on fixed DOFs); fixed
// DOFs then receive no additions.  The order of the atomic additions is not fixed, so
// results agree with the main kernel to rounding, not bit for bit.
#include "common.h"
#include "hex.h"

namespace tosimp {

namespace {

template <typename T, typename XT>
struct AtomicArgs {
  const T* v;
  T* y;
  const XT* x;
  const uint8_t* mask;
  int nx, ny, nz;
  int bricks_x, bricks_y, nbricks, per_xcd;
  T E0mEmin, Emin, penal;
  bool cube;
  HexK<T> k;
};

template <typename T, typename XT>
__device__ __forceinline__ T atomic_modulus(const AtomicArgs<T, XT>& A, XT xv) {
  const T x = (T)xv;
  const T xp = A.cube ? x * x * x : (x > T(0) ? pow(x, A.penal) : T(0));
  return A.Emin + xp * A.E0mEmin;
}

// y = v on fixed DOFs, 0 elsewhere (the cleared output the additions go into).
template <typename T>
__global__ __launch_bounds__(256) void atomic_clear_kernel(const T* __restrict__ v,
                                                           const uint8_t* __restrict__ mask,
                                                           T* __restrict__ y, int64_t n_node) {
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < n_node;
       n += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t m = mask[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) y[3 * n + c] = ((m >> c) & 1) ? v[3 * n + c] : T(0);
  }
}

// The algorithm as stated: one thread per element, 24 global atomic additions.
template <typename T, typename XT>
__global__ __launch_bounds__(256) void kv_atomic_element(AtomicArgs<T, XT> A) {
  const int64_t n_elem = (int64_t)A.nx * A.ny * A.nz;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  const int ex = (int)(e % A.nx);
  const int64_t r = e / A.nx;
  const int ey = (int)(r % A.ny), ez = (int)(r / A.ny);
  const int64_t NX1 = A.nx + 1, plane = NX1 * (A.ny + 1);
  const int64_t n0 = ex + NX1 * (ey + (int64_t)(A.ny + 1) * ez);
  int64_t node[8];
  T v[8][3];
  uint8_t m[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    node[q] = n0 + (q & 1) + ((q >> 1) & 1) * NX1 + ((q >> 2) & 1) * plane;
    m[q] = A.mask[node[q]];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[q][c] = ((m[q] >> c) & 1) ? T(0) : A.v[3 * node[q] + c];
  }
  T y[8][3];
  hex_apply(atomic_modulus(A, A.x[e]), A.k, v, y);
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (!((m[q] >> c) & 1)) unsafeAtomicAdd(&A.y[3 * node[q] + c], y[q][c]);
}

constexpr int kBX = 8, kBY = 8, kBZ = 4;  // elements per brick (256, one per thread)
constexpr int kWX = kBX + 1, kWY = kBY + 1, kWZ = kBZ + 1;
constexpr int kWin = kWX * kWY * kWZ;    // 405 window nodes
static_assert(kBX * kBY * kBZ == 256, "one element per thread");

// Additions reduced in LDS per brick; only nodes on brick faces use global atomics.
template <typename T, typename XT>
__global__ __launch_bounds__(256) void kv_atomic_brick(AtomicArgs<T, XT> A) {
  __shared__ T sv[kWin][3];
  __shared__ T sacc[kWin][3];
  __shared__ uint8_t sm[kWin];
  const int bid = blockIdx.x;
  const int b = (bid & 7) * A.per_xcd + (bid >> 3);  // contiguous brick range per XCD
  if (b >= A.nbricks) return;
  const int bx = b % A.bricks_x, rest = b / A.bricks_x;
  const int by = rest % A.bricks_y, bz = rest / A.bricks_y;
  const int i0 = bx * kBX, j0 = by * kBY, k0 = bz * kBZ;
  const int64_t NX1 = A.nx + 1, NY1 = A.ny + 1;
  const int tid = threadIdx.x;

  for (int q = tid; q < kWin; q += 256) {
    const int il = q % kWX, jl = (q / kWX) % kWY, kl = q / (kWX * kWY);
    const int i = i0 + il, j = j0 + jl, k = k0 + kl;
    const bool in = i <= A.nx && j <= A.ny && k <= A.nz;
    uint8_t m = 7;
    T vv[3] = {T(0), T(0), T(0)};
    if (in) {
      const int64_t n = i + NX1 * (j + NY1 * k);
      m = A.mask[n];
#pragma unroll
      for (int c = 0; c < 3; ++c) vv[c] = ((m >> c) & 1) ? T(0) : A.v[3 * n + c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sv[q][c] = vv[c];
      sacc[q][c] = T(0);
    }
    sm[q] = in ? m : (uint8_t)0xff;
  }
  __syncthreads();

  {
    const int exl = tid % kBX, eyl = (tid / kBX) % kBY, ezl = tid / (kBX * kBY);
    const int ex = i0 + exl, ey = j0 + eyl, ez = k0 + ezl;
    if (ex < A.nx && ey < A.ny && ez < A.nz) {
      const int q0 = exl + kWX * (eyl + kWY * ezl);
      int qs[8];
      T v[8][3];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        qs[q] = q0 + (q & 1) + ((q >> 1) & 1) * kWX + ((q >> 2) & 1) * kWX * kWY;
#pragma unroll
        for (int c = 0; c < 3; ++c) v[q][c] = sv[qs[q]][c];
      }
      const XT xv = A.x[ex + (int64_t)A.nx * (ey + (int64_t)A.ny * ez)];
      T y[8][3];
      hex_apply(atomic_modulus(A, xv), A.k, v, y);
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(&sacc[qs[q]][c], y[q][c]);
    }
  }
  __syncthreads();

  for (int q = tid; q < kWin; q += 256) {
    const uint8_t m = sm[q];
    if (m == 0xff) continue;  // outside the mesh
    const int il = q % kWX, jl = (q / kWX) % kWY, kl = q / (kWX * kWY);
    const int i = i0 + il, j = j0 + jl, k = k0 + kl;
    // Every element around the node lies in this brick (or outside the mesh).
    const bool own = (i == 0 || il > 0) && (i == A.nx || il < kBX) &&
                     (j == 0 || jl > 0) && (j == A.ny || jl < kBY) &&
                     (k == 0 || kl > 0) && (k == A.nz || kl < kBZ);
    T* yn = A.y + 3 * (i + NX1 * (j + NY1 * k));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if ((m >> c) & 1) continue;  // fixed: y = v from the clearing pass
      if (own)
        yn[c] = sacc[q][c];
      else
        unsafeAtomicAdd(&yn[c], sacc[q][c]);
    }
  }
}

template <typename T, typename XT>
hipError_t atomic_launch_t(const tosimp_ctx* c, const XT* x, const T* v, T* y, int variant) {
  AtomicArgs<T, XT> A{};
  A.v = v; A.y = y; A.x = x; A.mask = c->ws.mask;
  A.nx = c->nx; A.ny = c->ny; A.nz = c->nz;
  A.E0mEmin = (T)(c->E0 - c->Emin); A.Emin = (T)c->Emin; A.penal = (T)c->penal;
  A.cube = c->penal == 3.0;
  A.k = HexK<T>{(T)c->hc.ad, (T)c->hc.ao, (T)c->hc.cs, (T)c->hc.bd,
                (T)c->hc.bo, (T)c->hc.cd, (T)c->hc.co, (T)c->hc.hg};
  atomic_clear_kernel<T><<<dim3(2048), dim3(256), 0, c->stream>>>(v, c->ws.mask, y, c->n_node);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (variant == TOSIMP_SCATTER_ATOMIC_ELEMENT) {
    const int64_t blocks = (c->n_elem + 255) / 256;
    kv_atomic_element<T, XT><<<dim3((unsigned)blocks), dim3(256), 0, c->stream>>>(A);
  } else {
    A.bricks_x = (c->nx + kBX - 1) / kBX;
    A.bricks_y = (c->ny + kBY - 1) / kBY;
    const int bricks_z = (c->nz + kBZ - 1) / kBZ;
    A.nbricks = A.bricks_x * A.bricks_y * bricks_z;
    A.per_xcd = (A.nbricks + 7) / 8;
    kv_atomic_brick<T, XT><<<dim3(8 * A.per_xcd), dim3(256), 0, c->stream>>>(A);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t kv_atomic_launch(const tosimp_ctx* c, int prec, int xdtype, const void* x,
                            const void* v, void* y, int variant) {
  if (prec == TOSIMP_PREC_FP64) {
    if (xdtype == TOSIMP_F64)
      return atomic_launch_t<double, double>(c, (const double*)x, (const double*)v,
                                             (double*)y, variant);
    return atomic_launch_t<double, float>(c, (const float*)x, (const double*)v, (double*)y,
                                          variant);
  }
  if (xdtype == TOSIMP_F64)
    return atomic_launch_t<float, double>(c, (const double*)x, (const float*)v, (float*)y,
                                          variant);
  return atomic_launch_t<float, float>(c, (const float*)x, (const float*)v, (float*)y, variant);
}

}  // namespace tosimp
