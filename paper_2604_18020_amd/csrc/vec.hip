// Vector kernels of the CG solvers, refinement loop and Lanczos (FP64 / FP32 storage,
// FP64 reductions).
//
// Paper: Sec. "Preconditioned Conjugate Gradient and Warm-Start Strategy" (Jacobi-PCG,
// stop on the unpreconditioned ||r_k|| / ||f||) and Sec. "BF16 Arithmetic in the
// Conjugate Gradient Solver" (refinement r = f - K u, e ~ K^-1 r, u += e).
//
// Every kernel uses a fixed grid and a grid-stride loop, so each block's share of a
// reduction is fixed; block partials are summed in block order by a one-block finalize
// kernel.  Reductions are therefore bit-reproducible.  All dot products, norms, alpha
// and beta are FP64 whatever the vector type.  Solver control lives in a device
// SolverState: once `done` is set every later kernel of the batch returns at once, so
// the host enqueues batches of iterations and polls only between batches.
#include "common.h"
#include "dev.h"

namespace tosimp {

// Streaming solver kernels use a fixed grid per mesh (eight blocks per CU at most, a
// few 16-byte vectors per thread), hence a fixed reduction order.
static int vec_blocks(const tosimp_ctx* c) {
  const int64_t want = (c->n_dof + 8 * kRedThreads - 1) / (8 * kRedThreads);
  return (int)(want < 1 ? 1 : (want > 2048 ? 2048 : want));
}

// r = b - K u (masked), z = r * dinv, p = z; accumulates ||r||^2, <r,z>, ||b||^2.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void pcg_init_kernel(
    const T* __restrict__ b, const T* __restrict__ Ku, T* __restrict__ r,
    T* __restrict__ p, const T* __restrict__ dinv, const uint8_t* __restrict__ mask,
    int64_t n_dof, SolverState* st, double* partials, int use_Ku) {
  __shared__ double sred[kRedThreads / 64];
  double rr = 0.0, rz = 0.0, bb = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n_dof;
       i += (int64_t)gridDim.x * kRedThreads) {
    const int64_t n = i / 3;
    const int c = (int)(i - 3 * n);
    const bool fixed = (mask[n] >> c) & 1;
    const T bv = fixed ? T(0) : b[i];
    const T rv = use_Ku ? (fixed ? T(0) : bv - Ku[i]) : bv;
    const T zv = rv * dinv[n];
    r[i] = rv;
    p[i] = zv;
    rr += (double)rv * (double)rv;
    rz += (double)rv * (double)zv;
    bb += (double)bv * (double)bv;
  }
  const double v[3] = {rr, rz, bb};
  store_block_sums<3>(v, partials, sred);
}

struct PcgInitFin {
  SolverState* st;
  __device__ void operator()(const double* t) const {
    const double RR = t[0], RZ = t[1], BB = t[2];
    st->rr = RR;
    st->rz = RZ;
    st->bb = BB;
    st->tol2 = st->aux * BB;  // aux holds tol^2 on entry
    st->iter = 0;
    st->done = (BB == 0.0 || RR <= st->tol2) ? 1 : 0;
    if (!finite_val(RR) || !finite_val(RZ)) st->done = 3;
  }
};

// Vector width of the streaming kernels: 16 bytes per lane per array.
template <typename T>
struct Vec;
template <>
struct Vec<double> {
  typedef double2 type;
  static constexpr int W = 2;
};
template <>
struct Vec<float> {
  typedef float4 type;
  static constexpr int W = 4;
};

template <typename T>
__device__ __forceinline__ T vget(const typename Vec<T>::type& v, int k) {
  return reinterpret_cast<const T*>(&v)[k];
}
template <typename T>
__device__ __forceinline__ void vset(typename Vec<T>::type& v, int k, T x) {
  reinterpret_cast<T*>(&v)[k] = x;
}

// r -= alpha q and (WU) u += alpha p; block sums of ||r||^2 and <r, r dinv>
// (PcgUpdateFin then counts the iteration, tests convergence and forms beta).  Flat over
// DOFs, 16 bytes per lane per array (the node of DOF i is i / 3; n_dof < 2^31, so 32-bit
// arithmetic).  Jacobi-PCG leaves u to the direction kernel, which reads p anyway.
template <typename T, bool WU>
__global__ __launch_bounds__(kRedThreads) void pcg_update_kernel(
    T* __restrict__ u, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
    const T* __restrict__ dinv, int n_dof, SolverState* st, double* partials) {
  typedef typename Vec<T>::type VT;
  constexpr int W = Vec<T>::W;
  __shared__ double sred[kRedThreads / 64];
  if (st->done) return;
  const T alpha = (T)st->alpha;
  double rr = 0.0, rz = 0.0;
  const int nvec = n_dof / W;
  for (int v = blockIdx.x * kRedThreads + threadIdx.x; v < nvec; v += gridDim.x * kRedThreads) {
    VT rv = reinterpret_cast<const VT*>(r)[v];
    const VT qv = reinterpret_cast<const VT*>(q)[v];
    if constexpr (WU) {
      VT uv = reinterpret_cast<const VT*>(u)[v];
      const VT pv = reinterpret_cast<const VT*>(p)[v];
#pragma unroll
      for (int k = 0; k < W; ++k) vset<T>(uv, k, vget<T>(uv, k) + alpha * vget<T>(pv, k));
      reinterpret_cast<VT*>(u)[v] = uv;
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const unsigned i = (unsigned)(v * W + k);
      const T d = dinv[i / 3u];
      const T rn = vget<T>(rv, k) - alpha * vget<T>(qv, k);
      vset<T>(rv, k, rn);
      rr += (double)rn * (double)rn;
      rz += (double)rn * (double)(rn * d);
    }
    reinterpret_cast<VT*>(r)[v] = rv;
  }
  // tail (n_dof not a multiple of W), handled by block 0
  if (blockIdx.x == 0) {
    for (int i = nvec * W + threadIdx.x; i < n_dof; i += kRedThreads) {
      const T d = dinv[(unsigned)i / 3u];
      if constexpr (WU) u[i] += alpha * p[i];
      const T rn = r[i] - alpha * q[i];
      r[i] = rn;
      rr += (double)rn * (double)rn;
      rz += (double)rn * (double)(rn * d);
    }
  }
  const double v[2] = {rr, rz};
  store_block_sums<2>(v, partials, sred);
}

// Counts the iteration, tests convergence and forms beta.  When the iteration ends the
// solve and u is left to the direction kernel (which then does not run), the step
// u += alpha p is marked pending for pcg_finish_kernel.
struct PcgUpdateFin {
  SolverState* st;
  int u_deferred;
  __device__ void operator()(const double* t) const {
    if (st->done) return;
    const double RR = t[0], RZ = t[1];
    st->iter += 1;
    st->rr = RR;
    const double beta = RZ / st->rz;
    st->beta = beta;
    st->rz = RZ;
    if (!finite_val(RR) || !finite_val(beta)) st->done = 3;
    else if (RR <= st->tol2) st->done = 1;
    else if (st->iter >= st->maxit) st->done = 2;
    if (st->done && u_deferred) st->upend = 1;
  }
};

// u += alpha p (when u is given) and p = r dinv + beta p, flat over DOFs, 16 bytes per
// lane: the old p is read once for both.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void pcg_direction_kernel(
    const T* __restrict__ r, T* __restrict__ p, T* __restrict__ u, const T* __restrict__ dinv,
    int n_dof, const SolverState* st) {
  typedef typename Vec<T>::type VT;
  constexpr int W = Vec<T>::W;
  if (st->done) return;
  const T alpha = (T)st->alpha;
  const T beta = (T)st->beta;
  const int nvec = n_dof / W;
  for (int v = blockIdx.x * kRedThreads + threadIdx.x; v < nvec; v += gridDim.x * kRedThreads) {
    const VT rv = reinterpret_cast<const VT*>(r)[v];
    VT pv = reinterpret_cast<const VT*>(p)[v];
    if (u) {
      VT uv = reinterpret_cast<const VT*>(u)[v];
#pragma unroll
      for (int k = 0; k < W; ++k) vset<T>(uv, k, vget<T>(uv, k) + alpha * vget<T>(pv, k));
      reinterpret_cast<VT*>(u)[v] = uv;
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const unsigned i = (unsigned)(v * W + k);
      vset<T>(pv, k, vget<T>(rv, k) * dinv[i / 3u] + beta * vget<T>(pv, k));
    }
    reinterpret_cast<VT*>(p)[v] = pv;
  }
  if (blockIdx.x == 0)
    for (int i = nvec * W + threadIdx.x; i < n_dof; i += kRedThreads) {
      if (u) u[i] += alpha * p[i];
      p[i] = r[i] * dinv[(unsigned)i / 3u] + beta * p[i];
    }
}

// The step u += alpha p of the iteration that ended the solve (see PcgUpdateFin).
template <typename T>
__global__ __launch_bounds__(kRedThreads) void pcg_finish_kernel(T* __restrict__ u,
                                                                 const T* __restrict__ p,
                                                                 int n_dof, const SolverState* st) {
  typedef typename Vec<T>::type VT;
  constexpr int W = Vec<T>::W;
  if (!st->upend) return;
  const T alpha = (T)st->alpha;
  const int nvec = n_dof / W;
  for (int v = blockIdx.x * kRedThreads + threadIdx.x; v < nvec; v += gridDim.x * kRedThreads) {
    VT uv = reinterpret_cast<const VT*>(u)[v];
    const VT pv = reinterpret_cast<const VT*>(p)[v];
#pragma unroll
    for (int k = 0; k < W; ++k) vset<T>(uv, k, vget<T>(uv, k) + alpha * vget<T>(pv, k));
    reinterpret_cast<VT*>(u)[v] = uv;
  }
  if (blockIdx.x == 0)
    for (int i = nvec * W + threadIdx.x; i < n_dof; i += kRedThreads) u[i] += alpha * p[i];
}

template <typename T>
hipError_t launch_pcg_init(const tosimp_ctx* c, const T* b, const T* Ku, T* r, T* p,
                           const void* dinv, SolverState* st, double* partials, int use_Ku) {
  pcg_init_kernel<T><<<kRedBlocks, kRedThreads, 0, c->stream>>>(
      b, Ku, r, p, (const T*)dinv, c->ws.mask, c->n_dof, st, partials, use_Ku);
  return launch_finalize_sum<3>(c->stream, partials, kRedBlocks, PcgInitFin{st});
}

template <typename T>
hipError_t launch_pcg_update(const tosimp_ctx* c, T* u, T* r, const T* p, const T* q,
                             const void* dinv, SolverState* st, double* partials) {
  const int nb = vec_blocks(c);
  if (u)
    pcg_update_kernel<T, true><<<nb, kRedThreads, 0, c->stream>>>(
        u, r, p, q, (const T*)dinv, (int)c->n_dof, st, partials);
  else
    pcg_update_kernel<T, false><<<nb, kRedThreads, 0, c->stream>>>(
        nullptr, r, nullptr, q, (const T*)dinv, (int)c->n_dof, st, partials);
  return launch_finalize_sum<2>(c->stream, partials, nb, PcgUpdateFin{st, u ? 0 : 1});
}

template <typename T>
hipError_t launch_pcg_direction(const tosimp_ctx* c, const T* r, T* p, T* u, const void* dinv,
                                SolverState* st) {
  pcg_direction_kernel<T><<<vec_blocks(c), kRedThreads, 0, c->stream>>>(
      r, p, u, (const T*)dinv, (int)c->n_dof, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_finish(const tosimp_ctx* c, T* u, const T* p, SolverState* st) {
  pcg_finish_kernel<T><<<vec_blocks(c), kRedThreads, 0, c->stream>>>(u, p, (int)c->n_dof, st);
  return hipGetLastError();
}

template hipError_t launch_pcg_init<double>(const tosimp_ctx*, const double*, const double*,
                                            double*, double*, const void*, SolverState*,
                                            double*, int);
template hipError_t launch_pcg_init<float>(const tosimp_ctx*, const float*, const float*,
                                           float*, float*, const void*, SolverState*,
                                           double*, int);
template hipError_t launch_pcg_update<double>(const tosimp_ctx*, double*, double*,
                                              const double*, const double*, const void*,
                                              SolverState*, double*);
template hipError_t launch_pcg_update<float>(const tosimp_ctx*, float*, float*, const float*,
                                             const float*, const void*, SolverState*,
                                             double*);
template hipError_t launch_pcg_direction<double>(const tosimp_ctx*, const double*, double*,
                                                 double*, const void*, SolverState*);
template hipError_t launch_pcg_direction<float>(const tosimp_ctx*, const float*, float*, float*,
                                                const void*, SolverState*);
template hipError_t launch_pcg_finish<double>(const tosimp_ctx*, double*, const double*,
                                              SolverState*);
template hipError_t launch_pcg_finish<float>(const tosimp_ctx*, float*, const float*,
                                             SolverState*);

// ------------------------------------------------------------------ misc vectors
__global__ void mask_vec_kernel(double* v, const uint8_t* mask, int64_t n_dof) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_dof;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = i / 3;
    if ((mask[n] >> (int)(i - 3 * n)) & 1) v[i] = 0.0;
  }
}

hipError_t launch_mask_vec(const tosimp_ctx* c, double* v) {
  mask_vec_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(v, c->ws.mask, c->n_dof);
  return hipGetLastError();
}

// r = b - Ku (masked) and ||r||^2 into st->rr (FP64 true residual of refinement).
__global__ __launch_bounds__(kRedThreads) void residual64_kernel(
    const double* __restrict__ b, const double* __restrict__ Ku, double* __restrict__ r,
    const uint8_t* __restrict__ mask, int64_t n_dof, double* partials, SolverState* st) {
  __shared__ double sred[kRedThreads / 64];
  double rr = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n_dof;
       i += (int64_t)gridDim.x * kRedThreads) {
    const int64_t n = i / 3;
    const bool fixed = (mask[n] >> (int)(i - 3 * n)) & 1;
    const double rv = fixed ? 0.0 : b[i] - Ku[i];
    r[i] = rv;
    rr += rv * rv;
  }
  const double v[1] = {rr};
  store_block_sums<1>(v, partials, sred);
}

struct SetRr {
  SolverState* st;
  __device__ void operator()(const double* t) const { st->rr = t[0]; }
};

hipError_t launch_residual64(const tosimp_ctx* c, const double* b, const double* Ku,
                             double* r, double* partials, SolverState* st) {
  residual64_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(b, Ku, r, c->ws.mask,
                                                               c->n_dof, partials, st);
  return launch_finalize_sum<1>(c->stream, partials, kRedBlocks, SetRr{st});
}

__global__ void scale_to32_kernel(const double* r, double inv_s, float* r32, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r32[i] = (float)(r[i] * inv_s);
}

hipError_t launch_scale_to32(const tosimp_ctx* c, const double* r, double inv_s, float* r32) {
  scale_to32_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(r, inv_s, r32, c->n_dof);
  return hipGetLastError();
}

__global__ void axpy_from32_kernel(double* u, double s, const float* e, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    u[i] += s * (double)e[i];
}

hipError_t launch_axpy_from32(const tosimp_ctx* c, double* u, double s, const float* e) {
  axpy_from32_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(u, s, e, c->n_dof);
  return hipGetLastError();
}

__global__ void cast_kernel(const double* x, float* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// y = (float)(a - b): the error of an iterate against a reference, formed in FP64 before
// the cast (harvested training targets).
__global__ void diff_cast_kernel(const double* a, const double* b, float* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)(a[i] - b[i]);
}

hipError_t launch_diff_cast32(const tosimp_ctx* c, const double* a, const double* b, float* y,
                              int64_t n) {
  diff_cast_kernel<<<2048, 256, 0, c->stream>>>(a, b, y, n);
  return hipGetLastError();
}

hipError_t launch_cast32(const tosimp_ctx* c, const double* x, float* y, int64_t n) {
  cast_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(x, y, n);
  return hipGetLastError();
}

hipError_t launch_copy_cast_x(const tosimp_ctx* c, const double* x, float* x32) {
  cast_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(x, x32, c->n_elem);
  return hipGetLastError();
}

__global__ void zero_kernel(uint32_t* p, int64_t nwords) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_fill_zero(const tosimp_ctx* c, void* p, int64_t bytes) {
  zero_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>((uint32_t*)p, bytes / 4);
  return hipGetLastError();
}

__global__ __launch_bounds__(kRedThreads) void fill64_kernel(double* __restrict__ p, int64_t n,
                                                             double v) {
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    p[i] = v;
}

hipError_t launch_fill64(const tosimp_ctx* c, double* p, int64_t n, double v) {
  fill64_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(p, n, v);
  return hipGetLastError();
}

// <a, b> over n values into st->aux (what = 0) or st->rr (what = 1).
__global__ __launch_bounds__(kRedThreads) void dot64_kernel(const double* __restrict__ a,
                                                            const double* __restrict__ b,
                                                            int64_t n, double* partials,
                                                            SolverState* st, int what) {
  __shared__ double sred[kRedThreads / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    s += a[i] * b[i];
  const double v[1] = {s};
  store_block_sums<1>(v, partials, sred);
  (void)st;
  (void)what;
}

struct SetDot {
  SolverState* st;
  int what;
  __device__ void operator()(const double* t) const {
    if (what == 0) st->aux = t[0];
    else st->rr = t[0];
  }
};

hipError_t launch_dot64(const tosimp_ctx* c, const double* a, const double* b, int64_t n,
                        double* partials, SolverState* st, int what) {
  dot64_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(a, b, n, partials, st, what);
  return launch_finalize_sum<1>(c->stream, partials, kRedBlocks, SetDot{st, what});
}

// ------------------------------------------------------------------ Lanczos
// w = (s o w) - alpha_j q - beta_{j-1} q_prev, ||w|| -> beta_j (s: optional per-node
// scaling for the Jacobi-scaled operator; q_prev and beta_{j-1} may be null at j = 0).
__global__ __launch_bounds__(kRedThreads) void lanczos_update_kernel(
    double* __restrict__ w, const double* __restrict__ q, const double* __restrict__ qprev,
    const double* alpha_j, const double* beta_jm1, const double* __restrict__ s_node,
    int64_t n_dof, double* partials) {
  __shared__ double sred[kRedThreads / 64];
  const double a = *alpha_j;
  const double bprev = beta_jm1 ? *beta_jm1 : 0.0;
  double ss = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n_dof;
       i += (int64_t)gridDim.x * kRedThreads) {
    double wv = w[i];
    if (s_node) wv *= s_node[i / 3];
    wv -= a * q[i];
    if (qprev) wv -= bprev * qprev[i];
    w[i] = wv;
    ss += wv * wv;
  }
  const double v[1] = {ss};
  store_block_sums<1>(v, partials, sred);
}

struct SetSqrt {
  double* out;
  __device__ void operator()(const double* t) const { *out = sqrt(t[0]); }
};

hipError_t launch_lanczos_update(const tosimp_ctx* c, double* w, const double* q,
                                 const double* qprev, const double* alpha_j,
                                 const double* beta_jm1, const double* scale_node,
                                 double* partials, double* beta_j) {
  lanczos_update_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(
      w, q, qprev, alpha_j, beta_jm1, scale_node, c->n_dof, partials);
  return launch_finalize_sum<1>(c->stream, partials, kRedBlocks, SetSqrt{beta_j});
}

__global__ void lanczos_normalize_kernel(const double* w, const double* beta_j, double* qn,
                                         int64_t n) {
  const double b = *beta_j;
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    qn[i] = w[i] * inv;
}

hipError_t launch_lanczos_normalize(const tosimp_ctx* c, const double* w, const double* beta_j,
                                    double* qnext) {
  lanczos_normalize_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(w, beta_j, qnext,
                                                                      c->n_dof);
  return hipGetLastError();
}

__global__ void node_scale_kernel(const double* s, const double* v, double* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = v[i] * s[i / 3];
}

hipError_t launch_node_scale(const tosimp_ctx* c, const double* s_node, const double* v,
                             double* out) {
  node_scale_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(s_node, v, out, c->n_dof);
  return hipGetLastError();
}

__global__ void sqrt_node_kernel(const double* d, double* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = sqrt(d[i]);
}

hipError_t launch_sqrt_node(const tosimp_ctx* c, const double* dinv, double* out) {
  sqrt_node_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(dinv, out, c->n_node);
  return hipGetLastError();
}

// alpha = <r,z> / <p, q> for operators that do not fuse the dot (MFMA variant).
__global__ __launch_bounds__(kRedThreads) void alpha_dot32_kernel(const float* __restrict__ p,
                                                                  const float* __restrict__ q,
                                                                  int64_t n, double* partials,
                                                                  SolverState* st) {
  __shared__ double sred[kRedThreads / 64];
  if (st->done) return;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    s += (double)p[i] * (double)q[i];
  const double v[1] = {s};
  store_block_sums<1>(v, partials, sred);
}

// alpha = <r, z> / <p, K p> (breakdown when <p, K p> is not positive and finite).
struct AlphaFin {
  SolverState* st;
  __device__ void operator()(const double* t) const {
    if (st->done) return;
    const double tot = t[0];
    st->pq = tot;
    if (!(tot > 0.0) || !finite_val(tot)) {
      st->done = 3;
      st->alpha = 0.0;
    } else {
      st->alpha = st->rz / tot;
    }
  }
};

hipError_t launch_alpha_from_dot32(const tosimp_ctx* c, const float* p, const float* q,
                                   double* partials, SolverState* st) {
  alpha_dot32_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(p, q, c->n_dof, partials, st);
  return launch_finalize_sum<1>(c->stream, partials, kRedBlocks, AlphaFin{st});
}

__global__ void sqrt_scalar_kernel(const SolverState* st, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = sqrt(st->rr);
}

hipError_t launch_sqrt_scalar(const tosimp_ctx* c, const SolverState* st, double* out) {
  sqrt_scalar_kernel<<<1, 64, 0, c->stream>>>(st, out);
  return hipGetLastError();
}

}  // namespace tosimp
