// Geometric multigrid: a V-cycle preconditioner built on the fused operator, and CG
// preconditioned by it.
//
// Paper: Sec. "Path to Geometric Multigrid Integration" (the fused kernel as the
// fine-grid smoother, a restriction R and prolongation P = R^T between grids, a direct
// solve on the coarsest grid).  Design on gfx950:
//  * Hierarchy: level l + 1 has ceil(n / 2) elements per axis of twice the edge;
//    coarsening stops once an axis has one element.  Coarse operators are
//    re-discretised: the element stiffness scales with the edge (kscale = 2^l) and a
//    coarse element's modulus is the sum of its existing children's moduli over eight.
//    Every level's operator is the same fused kernel (kv_level_launch, moduli given).
//  * Boundary conditions: a coarse DOF is fixed when a fine DOF in its interpolation
//    support is; fixed rows are identity and every V-cycle vector is zero on them.
//  * Smoother: Chebyshev iteration of degree k on D^-1 K over [lam / alpha, lam] with
//    lam = lambda_max(K_E) / K_E[0][0], an upper bound of lambda_max(D^-1 K) for any
//    density field; the same polynomial before and after the coarse correction, so the
//    V-cycle is symmetric.  The first pre-smoothing step starts from zero and needs no
//    operator application.
//  * Transfer: trilinear interpolation P and R = P^T as gathers (each coarse node sums
//    its <= 27 fine nodes, each fine node its <= 8 coarse nodes): no atomics, fixed
//    order, deterministic.
//  * Coarsest level: dense inverse of the assembled constrained operator, computed in
//    FP64 on the host (Cholesky) once per set-up, applied as a matrix-vector product.
//  * CG: FP64 reductions and scalars on the device (SolverState), host polls every
//    check_every iterations; vectors in FP64 (plain mode) or FP32 (refinement inner solve).
//    Batches of check_every iterations are captured once as a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "dev.h"
#include "hex.h"

namespace tosimp {

namespace {

constexpr int kMgMaxLevels = 12;
constexpr int kMgCoarseMax = 1536;  // DOFs of the dense coarsest level

struct MgLevel {
  int nx = 0, ny = 0, nz = 0;
  int64_t n_node = 0, n_elem = 0, n_dof = 0;
  double kscale = 1;
  double* E64 = nullptr;
  float* E32 = nullptr;
  uint8_t* mask = nullptr;  // level 0: the context's mask (not owned)
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  void* b = nullptr;   // right-hand side (coarse levels; level 0: the caller's vector)
  void* x = nullptr;   // iterate (coarse levels; level 0: the caller's vector)
  void* t = nullptr;   // operator output
  void* dd = nullptr;  // Chebyshev direction
  void* xa = nullptr;  // second iterate buffer (fused smoothing steps alternate x / xa)
};

// An instantiated MG-CG batch, reused by later solves whose launches would be the same:
// the graph bakes in the vector pointers, the solver-state slot, the batch size, the
// Chebyshev coefficients and the SIMP exponent (the hierarchy's own buffers live as long
// as the hierarchy, which owns the cache).
struct MgGraph {
  int tsize = 0, k = 0, degree = 0, slot = 0;
  double alpha = 0, penal = 0;
  const void* ptr[7] = {};
  hipGraphExec_t exec = nullptr;
};
constexpr size_t kMgGraphCache = 16;

struct MgState {
  std::vector<MgGraph> graphs;
  // <r, z> of the current V-cycle, fused into its last finest-level smoothing pass when
  // requested (partials per operator tile; dot_tiles stays 0 when not fused)
  double* dot_part = nullptr;
  int dot_tiles = 0;
  int tail = -1;  // first level of the single-workgroup tail (-1: none)
  int tail_off[kMgMaxLevels][5] = {};  // LDS offsets of b, x, dd, dinv, E per tail level
  int tail_oer = 0;     // LDS offset of the element results
  int tail_values = 0;  // LDS values in all (bytes: times the vector type's size)
  int nlev = 0;
  MgLevel L[kMgMaxLevels];
  int nc = 0;  // coarsest DOFs
  double* Ainv64 = nullptr;
  float* Ainv32 = nullptr;
  double lam = 0;  // lambda_max(K_E) / K_E[0][0]
};

MgState* mg_of(tosimp_ctx* c) { return (MgState*)c->mg; }

// ------------------------------------------------------------------------ kernels
template <typename T>
__global__ __launch_bounds__(256) void simp_modulus_kernel(const double* __restrict__ x,
                                                           int64_t n, double Emin,
                                                           double E0mEmin, double penal,
                                                           double* __restrict__ E64,
                                                           float* __restrict__ E32) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double xv = x[e];
    const double xp = penal == 3.0 ? xv * xv * xv : (xv > 0.0 ? pow(xv, penal) : 0.0);
    const double E = Emin + xp * E0mEmin;
    E64[e] = E;
    E32[e] = (float)E;
  }
}

// Coarse modulus: (sum of the existing children) / 8.
__global__ __launch_bounds__(256) void restrict_modulus_kernel(
    const double* __restrict__ Ef, int fx, int fy, int fz, double* __restrict__ Ec,
    float* __restrict__ Ec32, int cx, int cy, int cz) {
  const int64_t n = (int64_t)cx * cy * cz;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int I = (int)(e % cx);
    const int64_t r = e / cx;
    const int J = (int)(r % cy), K = (int)(r / cy);
    double s = 0.0;
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c;
          if (i < fx && j < fy && k < fz) s += Ef[i + (int64_t)fx * (j + (int64_t)fy * k)];
        }
    const double v = s / 8.0;
    Ec[e] = v;
    Ec32[e] = (float)v;
  }
}

// Coarse BC byte: OR of the fine BC bytes over the node's interpolation support.
__global__ __launch_bounds__(256) void coarse_mask_kernel(const uint8_t* __restrict__ mf, int fx,
                                                          int fy, int fz,
                                                          uint8_t* __restrict__ mc, int cx,
                                                          int cy, int cz) {
  const int CX = cx + 1, CY = cy + 1;
  const int64_t n = (int64_t)CX * CY * (cz + 1);
  for (int64_t N = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; N < n;
       N += (int64_t)gridDim.x * blockDim.x) {
    const int I = (int)(N % CX);
    const int64_t r = N / CX;
    const int J = (int)(r % CY), K = (int)(r / CY);
    unsigned m = 0;
    for (int k = max(2 * K - 1, 0); k <= min(2 * K + 1, fz); ++k)
      for (int j = max(2 * J - 1, 0); j <= min(2 * J + 1, fy); ++j)
        for (int i = max(2 * I - 1, 0); i <= min(2 * I + 1, fx); ++i)
          m |= mf[i + (int64_t)(fx + 1) * (j + (int64_t)(fy + 1) * k)];
    mc[N] = (uint8_t)m;
  }
}

// Chebyshev step.  FIRST_ZERO: first step from a zero iterate (r = b): x = dd = c2 b dinv.
// FIRST: first step from x (r = b - t): dd = c2 r dinv; x += dd.  Otherwise
// dd = c1 dd + c2 r dinv; x += dd.  Fixed DOFs stay zero (b and t vanish there).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void cheb_kernel(const T* __restrict__ b,
                                                   const T* __restrict__ t, T* __restrict__ x,
                                                   T* __restrict__ dd,
                                                   const T* __restrict__ dinv, T c1, T c2,
                                                   int64_t n_dof, const SolverState* st) {
  if (st && st->done) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_dof;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T di = dinv[i / 3];
    if (MODE == 0) {
      const T d = c2 * (b[i] * di);
      dd[i] = d;
      x[i] = d;
    } else {
      const T r = b[i] - t[i];
      const T d = MODE == 1 ? c2 * (r * di) : c1 * dd[i] + c2 * (r * di);
      dd[i] = d;
      x[i] += d;
    }
  }
}

// bc = P^T (b - t) on the coarse grid, zero on fixed coarse DOFs.  Fine nodes of the
// support in index order (k, j, i), weights 1 (even offset) / 1/2 (odd) per axis.  One
// coarse node per thread, blocks laid out XCD-major (the fine planes a node gathers stay
// in its XCD's L2).
template <typename T>
__global__ __launch_bounds__(256) void restrict_residual_kernel(
    const T* __restrict__ bf, const T* __restrict__ tf, int fx, int fy, int fz,
    T* __restrict__ bc, const uint8_t* __restrict__ mc, int cx, int cy, int cz,
    const SolverState* st, int per_xcd) {
  if (st && st->done) return;
  const int CX = cx + 1, CY = cy + 1;
  const int64_t n = (int64_t)CX * CY * (cz + 1);
  {
    const int64_t N = xcd_item(per_xcd);
    if (N >= n) return;
    const int I = (int)(N % CX);
    const int64_t r = N / CX;
    const int J = (int)(r % CY), K = (int)(r / CY);
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int k = max(2 * K - 1, 0); k <= min(2 * K + 1, fz); ++k) {
      const T wk = k == 2 * K ? T(1) : T(0.5);
      for (int j = max(2 * J - 1, 0); j <= min(2 * J + 1, fy); ++j) {
        const T wj = j == 2 * J ? T(1) : T(0.5);
        for (int i = max(2 * I - 1, 0); i <= min(2 * I + 1, fx); ++i) {
          const T w = (i == 2 * I ? T(1) : T(0.5)) * wj * wk;
          const int64_t f = 3 * (i + (int64_t)(fx + 1) * (j + (int64_t)(fy + 1) * k));
          s0 += w * (bf[f] - tf[f]);
          s1 += w * (bf[f + 1] - tf[f + 1]);
          s2 += w * (bf[f + 2] - tf[f + 2]);
        }
      }
    }
    const unsigned m = mc[N];
    bc[3 * N] = (m & 1) ? T(0) : s0;
    bc[3 * N + 1] = (m & 2) ? T(0) : s1;
    bc[3 * N + 2] = (m & 4) ? T(0) : s2;
  }
}

// xf += P xc on free fine DOFs.  One fine node per thread, blocks laid out XCD-major.
template <typename T>
__global__ __launch_bounds__(256) void prolong_add_kernel(
    T* __restrict__ xf, const uint8_t* __restrict__ mf, int fx, int fy, int fz,
    const T* __restrict__ xc, int cx, int cy, int cz, const SolverState* st, int per_xcd) {
  if (st && st->done) return;
  const int FX = fx + 1, FY = fy + 1, CX = cx + 1, CY = cy + 1;
  const int64_t n = (int64_t)FX * FY * (fz + 1);
  {
    const int64_t nf = xcd_item(per_xcd);
    if (nf >= n) return;
    const int i = (int)(nf % FX);
    const int64_t r = nf / FX;
    const int j = (int)(r % FY), k = (int)(r / FY);
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1;
    const int k0 = k >> 1, k1 = (k + 1) >> 1;
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int K = k0; K <= k1; ++K) {
      const T wk = k0 == k1 ? T(1) : T(0.5);
      for (int J = j0; J <= j1; ++J) {
        const T wj = j0 == j1 ? T(1) : T(0.5);
        for (int I = i0; I <= i1; ++I) {
          const T w = (i0 == i1 ? T(1) : T(0.5)) * wj * wk;
          const int64_t c = 3 * (I + (int64_t)CX * (J + (int64_t)CY * K));
          s0 += w * xc[c];
          s1 += w * xc[c + 1];
          s2 += w * xc[c + 2];
        }
      }
    }
    const unsigned m = mf[nf];
    if (!(m & 1)) xf[3 * nf] += s0;
    if (!(m & 2)) xf[3 * nf + 1] += s1;
    if (!(m & 4)) xf[3 * nf + 2] += s2;
  }
}

// x = Ainv b on the coarsest level: one wave per row, FP64 accumulation, fixed order.
template <typename T>
__global__ __launch_bounds__(256) void dense_solve_kernel(const T* __restrict__ Ainv,
                                                          const T* __restrict__ b,
                                                          T* __restrict__ x, int n,
                                                          const SolverState* st) {
  if (st && st->done) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += (double)Ainv[(int64_t)row * n + j] * (double)b[j];
  s = wave_sum(s);
  if (lane == 0) x[row] = (T)s;
}

// -------------------------------------------------------- single-workgroup tail
// The smallest levels (at most kTailNodes nodes each, down to the dense coarsest) run
// as one workgroup that walks its part of the V-cycle with barriers between the steps:
// there a launch costs more than the work.  Every vector of these levels, their moduli
// and inverse diagonals, and one level's element results live in LDS (the top level's
// right-hand side is read from and its iterate written to device memory).  The
// operator goes element by element (each thread one element's 24 results), then each
// node sums its up to eight elements' results in a fixed order and applies the
// Chebyshev update at once; a visit's first two steps form the first iterate c0 D^-1 b
// while gathering.  The steps are those of the per-level kernels.
constexpr int kTailNodes = 512;  // largest level a single workgroup takes
constexpr int kTailMaxLevels = 6;
constexpr int kTailThreads = 512;
constexpr int kChebMax = 16;

template <typename T>
struct TailLevel {
  int nx, ny, nz;
  const T* E;           // device memory (copied in)
  const T* dinv;        // device memory (copied in)
  const uint8_t* mask;  // device memory
  const T* b_in;        // top level: the right-hand side
  T* x_out;             // top level: the iterate
  HexK<T> k;            // element constants of the level's edge
  int ob, ox, odd, odi, oE;  // LDS offsets (in values of T) of b, x, dd, dinv, E
};

template <typename T>
struct TailArgs {
  TailLevel<T> L[kTailMaxLevels];
  int nlev;  // levels from the tail's first; the last one is solved densely
  const T* Ainv;
  int nc;
  int oer;   // LDS offset of the element results
  T c1[kChebMax], c2[kChebMax];
  int degree;
  const SolverState* st;
};

enum TailStep { kTailFirst2 = 3, kTailCheb1 = 1, kTailCheb2 = 2, kTailResidual = 4 };

// Element phase: er[24 e + 3 q + c] = E_e (K_E v_e) with v the level's x, or (FIRST2)
// the first iterate c0 b D^-1 formed on the fly.
template <typename T, bool FIRST2>
__device__ void tail_elem(const TailLevel<T>& L, T* S, T* er, T c0) {
  const int NX1 = L.nx + 1, NY1 = L.ny + 1;
  const int ne = L.nx * L.ny * L.nz;
  const T* x = S + L.ox;
  const T* b = S + L.ob;
  const T* di = S + L.odi;
  const T* E = S + L.oE;
  for (int e = threadIdx.x; e < ne; e += kTailThreads) {
    const int ex = e % L.nx, r = e / L.nx;
    const int ey = r % L.ny, ez = r / L.ny;
    T v[8][3];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int n = (ex + (q & 1)) + NX1 * ((ey + ((q >> 1) & 1)) + NY1 * (ez + (q >> 2)));
#pragma unroll
      for (int c = 0; c < 3; ++c) v[q][c] = FIRST2 ? c0 * (b[3 * n + c] * di[n]) : x[3 * n + c];
    }
    T y[8][3];
    hex_apply(E[e], L.k, v, y);
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) er[24 * e + 3 * q + c] = y[q][c];
  }
  __syncthreads();
}

// Node phase: t = K_c v at each node (fixed rows t = v), then the step's update.
template <typename T, int STEP>
__device__ void tail_node(const TailLevel<T>& L, T* S, const T* er, T c0, T c1, T c2) {
  const int NX1 = L.nx + 1, NY1 = L.ny + 1;
  const int nn = NX1 * NY1 * (L.nz + 1);
  T* x = S + L.ox;
  T* dd = S + L.odd;
  const T* b = S + L.ob;
  const T* di = S + L.odi;
  for (int n = threadIdx.x; n < nn; n += kTailThreads) {
    const int i = n % NX1, r = n / NX1;
    const int j = r % NY1, k = r / NY1;
    T s[3] = {T(0), T(0), T(0)};
    for (int ez = k - 1; ez <= k; ++ez) {
      if (ez < 0 || ez >= L.nz) continue;
      for (int ey = j - 1; ey <= j; ++ey) {
        if (ey < 0 || ey >= L.ny) continue;
        for (int ex = i - 1; ex <= i; ++ex) {
          if (ex < 0 || ex >= L.nx) continue;
          const int q = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
          const T* yr = er + 24 * (ex + L.nx * (ey + L.ny * ez)) + 3 * q;
          s[0] += yr[0];
          s[1] += yr[1];
          s[2] += yr[2];
        }
      }
    }
    const unsigned m = L.mask[n];
    const T dn = di[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int I = 3 * n + c;
      const T v = STEP == kTailFirst2 ? c0 * (b[I] * dn) : x[I];
      const T t = ((m >> c) & 1) ? v : s[c];
      const T rr = b[I] - t;
      if (STEP == kTailResidual) {
        dd[I] = rr;  // dd is dead until the next visit's first step overwrites it
      } else {
        const T dprev = STEP == kTailFirst2 ? v : dd[I];
        const T d = STEP == kTailCheb1 ? c2 * (rr * dn) : c1 * dprev + c2 * (rr * dn);
        dd[I] = d;
        x[I] = v + d;
      }
    }
  }
  __syncthreads();
}

// x = dd = c2 b D^-1 (the first step from zero when the degree is 1).
template <typename T>
__device__ void tail_first(const TailLevel<T>& L, T* S, T c2) {
  const int nd = 3 * (L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  T* x = S + L.ox;
  T* dd = S + L.odd;
  const T* b = S + L.ob;
  const T* di = S + L.odi;
  for (int i = threadIdx.x; i < nd; i += kTailThreads) {
    const T d = c2 * (b[i] * di[i / 3]);
    dd[i] = d;
    x[i] = d;
  }
  __syncthreads();
}

// C.b = P^T r_F (r_F in F's dd), zero on fixed coarse DOFs.
template <typename T>
__device__ void tail_restrict(const TailLevel<T>& F, const TailLevel<T>& C, T* S) {
  const T* rf = S + F.odd;
  T* bc = S + C.ob;
  const int CX = C.nx + 1, CY = C.ny + 1;
  const int n = CX * CY * (C.nz + 1);
  for (int N = threadIdx.x; N < n; N += kTailThreads) {
    const int I = N % CX, r = N / CX;
    const int J = r % CY, K = r / CY;
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int k = max(2 * K - 1, 0); k <= min(2 * K + 1, F.nz); ++k) {
      const T wk = k == 2 * K ? T(1) : T(0.5);
      for (int j = max(2 * J - 1, 0); j <= min(2 * J + 1, F.ny); ++j) {
        const T wj = j == 2 * J ? T(1) : T(0.5);
        for (int i = max(2 * I - 1, 0); i <= min(2 * I + 1, F.nx); ++i) {
          const T w = (i == 2 * I ? T(1) : T(0.5)) * wj * wk;
          const int f = 3 * (i + (F.nx + 1) * (j + (F.ny + 1) * k));
          s0 += w * rf[f];
          s1 += w * rf[f + 1];
          s2 += w * rf[f + 2];
        }
      }
    }
    const unsigned m = C.mask[N];
    bc[3 * N] = (m & 1) ? T(0) : s0;
    bc[3 * N + 1] = (m & 2) ? T(0) : s1;
    bc[3 * N + 2] = (m & 4) ? T(0) : s2;
  }
  __syncthreads();
}

// F.x += P C.x on free fine DOFs.
template <typename T>
__device__ void tail_prolong(const TailLevel<T>& F, const TailLevel<T>& C, T* S) {
  T* xf = S + F.ox;
  const T* xc = S + C.ox;
  const int FX = F.nx + 1, FY = F.ny + 1, CX = C.nx + 1, CY = C.ny + 1;
  const int n = FX * FY * (F.nz + 1);
  for (int nf = threadIdx.x; nf < n; nf += kTailThreads) {
    const int i = nf % FX, r = nf / FX;
    const int j = r % FY, k = r / FY;
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1;
    const int k0 = k >> 1, k1 = (k + 1) >> 1;
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int K = k0; K <= k1; ++K) {
      const T wk = k0 == k1 ? T(1) : T(0.5);
      for (int J = j0; J <= j1; ++J) {
        const T wj = j0 == j1 ? T(1) : T(0.5);
        for (int I = i0; I <= i1; ++I) {
          const T w = (i0 == i1 ? T(1) : T(0.5)) * wj * wk;
          const int c = 3 * (I + CX * (J + CY * K));
          s0 += w * xc[c];
          s1 += w * xc[c + 1];
          s2 += w * xc[c + 2];
        }
      }
    }
    const unsigned m = F.mask[nf];
    if (!(m & 1)) xf[3 * nf] += s0;
    if (!(m & 2)) xf[3 * nf + 1] += s1;
    if (!(m & 4)) xf[3 * nf + 2] += s2;
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void mg_tail_kernel(TailArgs<T> A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char tail_lds[];
  if (A.st && A.st->done) return;
  T* S = reinterpret_cast<T*>(tail_lds);
  T* er = S + A.oer;
  const int last = A.nlev - 1;
  // copy in: moduli and inverse diagonals of the smoothed levels, the top right-hand side
  for (int l = 0; l < last; ++l) {
    const TailLevel<T>& L = A.L[l];
    const int ne = L.nx * L.ny * L.nz, nn = (L.nx + 1) * (L.ny + 1) * (L.nz + 1);
    for (int i = threadIdx.x; i < ne; i += kTailThreads) S[L.oE + i] = L.E[i];
    for (int i = threadIdx.x; i < nn; i += kTailThreads) S[L.odi + i] = L.dinv[i];
  }
  {
    const TailLevel<T>& L = A.L[0];
    const int nd = 3 * (L.nx + 1) * (L.ny + 1) * (L.nz + 1);
    for (int i = threadIdx.x; i < nd; i += kTailThreads) S[L.ob + i] = L.b_in[i];
  }
  __syncthreads();
  for (int l = 0; l < last; ++l) {
    const TailLevel<T>& L = A.L[l];
    if (A.degree >= 2) {
      tail_elem<T, true>(L, S, er, A.c2[0]);
      tail_node<T, kTailFirst2>(L, S, er, A.c2[0], A.c1[1], A.c2[1]);
    } else {
      tail_first(L, S, A.c2[0]);
    }
    for (int s = 2; s < A.degree; ++s) {
      tail_elem<T, false>(L, S, er, T(0));
      tail_node<T, kTailCheb2>(L, S, er, T(0), A.c1[s], A.c2[s]);
    }
    tail_elem<T, false>(L, S, er, T(0));
    tail_node<T, kTailResidual>(L, S, er, T(0), T(0), T(0));
    tail_restrict(L, A.L[l + 1], S);
  }
  {
    // x = Ainv b, one row per thread, FP64 sums in column order
    const TailLevel<T>& C = A.L[last];
    const T* bc = S + C.ob;
    T* xc = S + C.ox;
    for (int row = threadIdx.x; row < A.nc; row += kTailThreads) {
      double s = 0.0;
      for (int j = 0; j < A.nc; ++j) s += (double)A.Ainv[row * A.nc + j] * (double)bc[j];
      xc[row] = (T)s;
    }
    __syncthreads();
  }
  for (int l = last - 1; l >= 0; --l) {
    const TailLevel<T>& L = A.L[l];
    tail_prolong(L, A.L[l + 1], S);
    tail_elem<T, false>(L, S, er, T(0));
    tail_node<T, kTailCheb1>(L, S, er, T(0), T(0), A.c2[0]);
    for (int s = 1; s < A.degree; ++s) {
      tail_elem<T, false>(L, S, er, T(0));
      tail_node<T, kTailCheb2>(L, S, er, T(0), A.c1[s], A.c2[s]);
    }
  }
  {
    const TailLevel<T>& L = A.L[0];
    const int nd = 3 * (L.nx + 1) * (L.ny + 1) * (L.nz + 1);
    for (int i = threadIdx.x; i < nd; i += kTailThreads) L.x_out[i] = S[L.ox + i];
  }
}

// ------------------------------------------------------------- CG kernels (device state)
// r = b - Ku (Ku may be null: zero initial iterate), zero on fixed DOFs; sums of
// ||r||^2 and ||b||^2.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void mgcg_init_kernel(
    const T* __restrict__ b, const T* __restrict__ Ku, T* __restrict__ r,
    const uint8_t* __restrict__ mask, int64_t n_dof, double* partials) {
  __shared__ double sred[kRedThreads / 64];
  double rr = 0.0, bb = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n_dof;
       i += (int64_t)gridDim.x * kRedThreads) {
    const bool fixed = (mask[i / 3] >> (int)(i % 3)) & 1;
    const T bv = fixed ? T(0) : b[i];
    const T rv = fixed ? T(0) : (Ku ? bv - Ku[i] : bv);
    r[i] = rv;
    rr += (double)rv * (double)rv;
    bb += (double)bv * (double)bv;
  }
  const double v[2] = {rr, bb};
  store_block_sums<2>(v, partials, sred);
}

struct MgInitFin {
  SolverState* st;
  __device__ void operator()(const double* t) const {
    const double RR = t[0], BB = t[1];
    st->rr = RR;
    st->bb = BB;
    st->tol2 = st->aux * BB;  // aux holds tol^2 on entry
    st->iter = 0;
    st->rz = 0.0;
    st->done = (BB == 0.0 || RR <= st->tol2) ? 1 : 0;
    if (!finite_val(RR)) st->done = 3;
  }
};

template <typename T>
__global__ __launch_bounds__(kRedThreads) void dot_rz_kernel(const T* __restrict__ r,
                                                             const T* __restrict__ z,
                                                             int64_t n, const SolverState* st,
                                                             double* partials) {
  __shared__ double sred[kRedThreads / 64];
  if (st->done) return;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    s += (double)r[i] * (double)z[i];
  const double v[1] = {s};
  store_block_sums<1>(v, partials, sred);
}

struct MgRzFin {
  SolverState* st;
  __device__ void operator()(const double* t) const {
    if (st->done) return;
    const double RZ = t[0];
    st->beta = st->iter == 0 ? 0.0 : RZ / st->rz;
    st->rz = RZ;
    if (!finite_val(RZ) || !(RZ > 0.0)) st->done = 3;  // the V-cycle is SPD: <r, z> > 0
  }
};

// p = z (first iteration) or z + beta p.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void mg_direction_kernel(const T* __restrict__ z,
                                                                   T* __restrict__ p, int64_t n,
                                                                   const SolverState* st) {
  if (st->done) return;
  const bool first = st->iter == 0;
  const T beta = (T)st->beta;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    p[i] = first ? z[i] : z[i] + beta * p[i];
}

// u += alpha p, r -= alpha q; sums of ||r||^2.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void mg_update_kernel(
    T* __restrict__ u, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
    int64_t n, const SolverState* st, double* partials) {
  __shared__ double sred[kRedThreads / 64];
  if (st->done) return;
  const T alpha = (T)st->alpha;
  double rr = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    u[i] += alpha * p[i];
    const T rn = r[i] - alpha * q[i];
    r[i] = rn;
    rr += (double)rn * (double)rn;
  }
  const double v[1] = {rr};
  store_block_sums<1>(v, partials, sred);
}

struct MgUpdateFin {
  SolverState* st;
  __device__ void operator()(const double* t) const {
    if (st->done) return;
    const double RR = t[0];
    st->iter += 1;
    st->rr = RR;
    if (!finite_val(RR)) st->done = 3;
    else if (RR <= st->tol2) st->done = 1;
    else if (st->iter >= st->maxit) st->done = 2;
  }
};

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(2048, (n + 255) / 256)); }

// ------------------------------------------------------------------------ host side
// Largest eigenvalue of a symmetric n x n matrix (cyclic Jacobi rotations).
double sym_lambda_max(std::vector<double> a, int n) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = 0.5 * (a[q * n + q] - a[p * n + p]) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  double m = a[0];
  for (int i = 1; i < n; ++i) m = std::max(m, a[i * n + i]);
  return m;
}

// Dense constrained stiffness of a small level (host, FP64), element stiffness K_E
// scaled by kscale, fixed rows and columns replaced by identity.
void assemble_dense(const tosimp_ctx* c, int nx, int ny, int nz, double kscale,
                    const std::vector<double>& E, const std::vector<uint8_t>& mask,
                    std::vector<double>& A) {
  const int NX = nx + 1, NY = ny + 1;
  const int nd = 3 * NX * NY * (nz + 1);
  A.assign((size_t)nd * nd, 0.0);
  for (int ez = 0; ez < nz; ++ez)
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex) {
        const double Ee = E[ex + nx * (ey + ny * ez)] * kscale;
        int dof[24];
        for (int a = 0; a < 8; ++a) {
          const int node = (ex + (a & 1)) + NX * ((ey + ((a >> 1) & 1)) + NY * (ez + ((a >> 2) & 1)));
          for (int cc = 0; cc < 3; ++cc) dof[3 * a + cc] = 3 * node + cc;
        }
        for (int i = 0; i < 24; ++i)
          for (int j = 0; j < 24; ++j) A[(size_t)dof[i] * nd + dof[j]] += Ee * c->KE[i * 24 + j];
      }
  for (int d = 0; d < nd; ++d)
    if ((mask[d / 3] >> (d % 3)) & 1) {
      for (int j = 0; j < nd; ++j) {
        A[(size_t)d * nd + j] = 0.0;
        A[(size_t)j * nd + d] = 0.0;
      }
      A[(size_t)d * nd + d] = 1.0;
    }
}

// Inverse of an SPD matrix by Cholesky (host, FP64); false if not positive definite.
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / d;
    }
  }
  // columns of A^-1: solve L L^T x = e_j
  std::vector<double> y(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) {
      double t = i == j ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * y[k];
      y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * y[k];
      y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) A[(size_t)i * n + j] = y[i];
  }
  return true;
}

hipError_t mg_alloc(void** p, size_t bytes) { return hipMalloc(p, bytes < 256 ? 256 : bytes); }

// Builds the level geometry and allocates every buffer (once per mesh).
int mg_create_impl(tosimp_ctx* ctx);
int mg_create(tosimp_ctx* ctx) {
  if (ctx->mg) return TOSIMP_OK;
  const int rc = mg_create_impl(ctx);
  if (rc) mg_release(ctx);  // no half-built hierarchy survives a failure
  return rc;
}
int mg_create_impl(tosimp_ctx* ctx) {
  MgState* M = new (std::nothrow) MgState();
  if (!M) return tosimp_fail(ctx, TOSIMP_ENOMEM, "multigrid state");
  ctx->mg = M;
  int nx = ctx->nx, ny = ctx->ny, nz = ctx->nz;
  double ks = ctx->h;
  for (;;) {
    MgLevel& L = M->L[M->nlev];
    L.nx = nx; L.ny = ny; L.nz = nz;
    L.n_node = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    L.n_elem = (int64_t)nx * ny * nz;
    L.n_dof = 3 * L.n_node;
    L.kscale = ks / ctx->h;  // relative to the fine element (the constants hold h)
    ++M->nlev;
    if (std::min(nx, std::min(ny, nz)) < 2 || M->nlev == kMgMaxLevels) break;
    nx = (nx + 1) / 2; ny = (ny + 1) / 2; nz = (nz + 1) / 2;
    ks *= 2.0;
  }
  MgLevel& C = M->L[M->nlev - 1];
  if (M->nlev < 2 || C.n_dof > kMgCoarseMax)
    return tosimp_fail(ctx, TOSIMP_EINVAL,
                       "multigrid: the coarsest grid of this mesh has " +
                           std::to_string(C.n_dof) + " DOFs (at most " +
                           std::to_string(kMgCoarseMax) + " and two levels are needed)");
  M->nc = (int)C.n_dof;
  for (int l = 0; l < M->nlev; ++l) {
    MgLevel& L = M->L[l];
    const size_t nd = (size_t)L.n_dof, ne = (size_t)L.n_elem, nn = (size_t)L.n_node;
    TOSIMP_HIP(ctx, mg_alloc((void**)&L.E64, ne * 8));
    TOSIMP_HIP(ctx, mg_alloc((void**)&L.E32, ne * 4));
    TOSIMP_HIP(ctx, mg_alloc((void**)&L.dinv64, nn * 8));
    TOSIMP_HIP(ctx, mg_alloc((void**)&L.dinv32, nn * 4));
    if (l > 0) {
      TOSIMP_HIP(ctx, mg_alloc((void**)&L.mask, nn));
      TOSIMP_HIP(ctx, mg_alloc(&L.b, nd * 8));
      TOSIMP_HIP(ctx, mg_alloc(&L.x, nd * 8));
    } else {
      L.mask = ctx->ws.mask;
    }
    TOSIMP_HIP(ctx, mg_alloc(&L.t, nd * 8));
    TOSIMP_HIP(ctx, mg_alloc(&L.dd, nd * 8));
    TOSIMP_HIP(ctx, mg_alloc(&L.xa, nd * 8));
  }
  TOSIMP_HIP(ctx, mg_alloc((void**)&M->Ainv64, (size_t)M->nc * M->nc * 8));
  TOSIMP_HIP(ctx, mg_alloc((void**)&M->Ainv32, (size_t)M->nc * M->nc * 4));
  // The tail: the longest run of coarsest levels (at least one smoothed level above the
  // dense one, at most kTailMaxLevels, none with more than kTailNodes nodes) whose LDS
  // arena, sized for FP64, fits a workgroup; none if even the last two do not fit.
  M->tail = -1;
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) !=
          hipSuccess ||
      hipFuncSetAttribute((const void*)mg_tail_kernel<double>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) != hipSuccess ||
      hipFuncSetAttribute((const void*)mg_tail_kernel<float>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) != hipSuccess) {
    (void)hipGetLastError();
    lds_max = 0;  // no tail
  }
  // Arena layout from level `first` down: b, x, dd, dinv, E per smoothed level (b, x on the
  // dense one), then one level's element results; returns its size in values.
  auto layout = [&](int first, bool store) -> int {
    int off = 0;
    for (int i = 0; first + i < M->nlev; ++i) {
      const MgLevel& L = M->L[first + i];
      const bool dense = first + i == M->nlev - 1;
      const int o[5] = {off, off + (int)L.n_dof, off + 2 * (int)L.n_dof,
                        off + (dense ? 2 : 3) * (int)L.n_dof,
                        off + (dense ? 2 * (int)L.n_dof : 3 * (int)L.n_dof + (int)L.n_node)};
      off = dense ? o[3] : o[4] + (int)L.n_elem;
      off = (off + 1) & ~1;  // 16-byte alignment for FP64 pairs
      if (store)
        for (int k = 0; k < 5; ++k) M->tail_off[i][k] = o[k];
    }
    if (store) M->tail_oer = off;
    off += 24 * (int)M->L[first].n_elem;
    if (store) M->tail_values = off;
    return off;
  };
  for (int l = M->nlev - 2; l >= 0 && lds_max > 0; --l) {
    if (M->nlev - l > kTailMaxLevels || M->L[l].n_node > kTailNodes) break;
    if ((size_t)layout(l, false) * 8 > (size_t)lds_max) break;
    M->tail = l;
  }
  if (M->tail >= 0) layout(M->tail, true);
  std::vector<double> ke(ctx->KE, ctx->KE + 576);
  M->lam = sym_lambda_max(ke, 24) / ctx->KE[0];
  return TOSIMP_OK;
}

// Moduli, masks and diagonals of every level and the coarsest inverse for density x.
int mg_setup(tosimp_ctx* ctx, const double* x) {
  int rc = mg_create(ctx);
  if (rc) return rc;
  MgState* M = mg_of(ctx);
  MgLevel& F = M->L[0];
  simp_modulus_kernel<double><<<grid_for(F.n_elem), 256, 0, ctx->stream>>>(
      x, F.n_elem, ctx->Emin, ctx->E0 - ctx->Emin, ctx->penal, F.E64, F.E32);
  TOSIMP_HIP(ctx, hipGetLastError());
  for (int l = 1; l < M->nlev; ++l) {
    MgLevel &P = M->L[l - 1], &L = M->L[l];
    restrict_modulus_kernel<<<grid_for(L.n_elem), 256, 0, ctx->stream>>>(
        P.E64, P.nx, P.ny, P.nz, L.E64, L.E32, L.nx, L.ny, L.nz);
    coarse_mask_kernel<<<grid_for(L.n_node), 256, 0, ctx->stream>>>(P.mask, P.nx, P.ny, P.nz,
                                                                    L.mask, L.nx, L.ny, L.nz);
    TOSIMP_HIP(ctx, hipGetLastError());
  }
  for (int l = 0; l < M->nlev; ++l) {
    MgLevel& L = M->L[l];
    TOSIMP_HIP(ctx, launch_diag_level(ctx, L.E64, L.nx, L.ny, L.nz, L.kscale, L.dinv64, L.dinv32));
  }
  // coarsest: dense constrained operator, inverted on the host
  MgLevel& C = M->L[M->nlev - 1];
  std::vector<double> E((size_t)C.n_elem);
  std::vector<uint8_t> mask((size_t)C.n_node);
  TOSIMP_HIP(ctx, hipMemcpyAsync(E.data(), C.E64, E.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipMemcpyAsync(mask.data(), C.mask, mask.size(), hipMemcpyDeviceToHost,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<double> A;
  assemble_dense(ctx, C.nx, C.ny, C.nz, C.kscale, E, mask, A);
  if (!spd_inverse(A, M->nc))
    return tosimp_fail(ctx, TOSIMP_EBREAKDOWN, "multigrid: coarsest operator not positive definite");
  std::vector<float> A32(A.size());
  for (size_t i = 0; i < A.size(); ++i) A32[i] = (float)A[i];
  TOSIMP_HIP(ctx, hipMemcpyAsync(M->Ainv64, A.data(), A.size() * 8, hipMemcpyHostToDevice,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipMemcpyAsync(M->Ainv32, A32.data(), A32.size() * 4, hipMemcpyHostToDevice,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));  // host vectors leave scope
  return TOSIMP_OK;
}

// Chebyshev coefficients: step 1 uses c2 = 1 / theta; step k >= 2 c1 = rho' rho,
// c2 = 2 rho' / delta with rho' = 1 / (2 sigma - rho).
struct ChebCoef {
  double c1[16], c2[16];
};
ChebCoef cheb_coef(double lam, double alpha, int degree) {
  ChebCoef k{};
  const double lo = lam / alpha, hi = lam;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  k.c1[0] = 0.0;
  k.c2[0] = 1.0 / theta;
  for (int s = 1; s < degree; ++s) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    k.c1[s] = rn * rho;
    k.c2[s] = 2.0 * rn / delta;
    rho = rn;
  }
  return k;
}

template <typename T>
const T* lev_E(const MgLevel& L) {
  if constexpr (sizeof(T) == 8) return (const T*)L.E64; else return (const T*)L.E32;
}
template <typename T>
const T* lev_dinv(const MgLevel& L) {
  if constexpr (sizeof(T) == 8) return (const T*)L.dinv64; else return (const T*)L.dinv32;
}

// The V-cycle from the tail's first level down, in one single-workgroup launch.
template <typename T>
int tail_vcycle(tosimp_ctx* ctx, MgState* M, const ChebCoef& K, int degree,
                const SolverState* st) {
  TailArgs<T> A{};
  A.nlev = M->nlev - M->tail;
  for (int i = 0; i < A.nlev; ++i) {
    const MgLevel& L = M->L[M->tail + i];
    TailLevel<T>& D = A.L[i];
    D.nx = L.nx;
    D.ny = L.ny;
    D.nz = L.nz;
    D.E = lev_E<T>(L);
    D.dinv = lev_dinv<T>(L);
    D.mask = L.mask;
    D.b_in = (const T*)L.b;
    D.x_out = (T*)L.x;
    const double ks = L.kscale;
    D.k = HexK<T>{(T)(ks * ctx->hc.ad), (T)(ks * ctx->hc.ao), (T)(ks * ctx->hc.cs),
                  (T)(ks * ctx->hc.bd), (T)(ks * ctx->hc.bo), (T)(ks * ctx->hc.cd),
                  (T)(ks * ctx->hc.co), (T)(ks * ctx->hc.hg)};
    D.ob = M->tail_off[i][0];
    D.ox = M->tail_off[i][1];
    D.odd = M->tail_off[i][2];
    D.odi = M->tail_off[i][3];
    D.oE = M->tail_off[i][4];
  }
  if constexpr (sizeof(T) == 8) A.Ainv = (const T*)M->Ainv64; else A.Ainv = (const T*)M->Ainv32;
  A.nc = M->nc;
  A.oer = M->tail_oer;
  for (int s = 0; s < degree && s < kChebMax; ++s) {
    A.c1[s] = (T)K.c1[s];
    A.c2[s] = (T)K.c2[s];
  }
  A.degree = degree;
  A.st = st;
  mg_tail_kernel<T><<<1, kTailThreads, (size_t)M->tail_values * sizeof(T), ctx->stream>>>(A);
  TOSIMP_HIP(ctx, hipGetLastError());
  return TOSIMP_OK;
}

// One V-cycle from level l: x_l ~ K_l^-1 b_l (x_l overwritten).
template <typename T>
int vcycle(tosimp_ctx* ctx, MgState* M, int l, const ChebCoef& K, int degree,
           const SolverState* st) {
  constexpr int prec = sizeof(T) == 8 ? TOSIMP_PREC_FP64 : TOSIMP_PREC_FP32;
  if (l == M->tail) return tail_vcycle<T>(ctx, M, K, degree, st);
  MgLevel& L = M->L[l];
  T *b = (T*)L.b, *x = (T*)L.x, *t = (T*)L.t, *dd = (T*)L.dd;
  const int nd = (int)L.n_dof;
  const int g = grid_for(L.n_dof);
  if (l == M->nlev - 1) {
    const T* Ainv;
    if constexpr (sizeof(T) == 8) Ainv = (const T*)M->Ainv64; else Ainv = (const T*)M->Ainv32;
    dense_solve_kernel<T><<<(M->nc + 3) / 4, 256, 0, ctx->stream>>>(Ainv, b, x, M->nc, st);
    TOSIMP_HIP(ctx, hipGetLastError());
    return TOSIMP_OK;
  }
  const T* E = lev_E<T>(L);
  const T* dinv = lev_dinv<T>(L);
  // Every smoothing step after a visit's first applies the operator and the Chebyshev
  // update in one pass (t = K x stays in registers) and writes the new iterate to the
  // other buffer; 2 degree - 1 such passes per visit (the first one also forms the first
  // step's iterate), so starting in xa ends in x.
  T* xs[2] = {x, (T*)L.xa};
  int cur = 1;
  auto fused = [&](int mode, double c1, double c2, bool with_dot = false) -> hipError_t {
    KvCheb ch;
    ch.mode = mode;
    ch.b = b;
    ch.dd = dd;
    ch.dinv = dinv;
    ch.c1 = c1;
    ch.c2 = c2;
    if (with_dot) {
      ch.dot = M->dot_part;
      ch.dot_tiles = &M->dot_tiles;
    }
    const hipError_t e = kv_level_launch(ctx, prec, E, xs[cur], xs[cur ^ 1], L.nx, L.ny, L.nz,
                                         L.mask, L.kscale, st, &ch);
    cur ^= 1;
    return e;
  };
  // pre-smoothing from zero: the first two steps in one pass (the first step's iterate
  // c2 D^-1 b is formed while the operator stages its planes)
  if (degree >= 2) {
    KvCheb ch;
    ch.mode = 3;
    ch.b = b;
    ch.dd = dd;
    ch.dinv = dinv;
    ch.c0 = K.c2[0];
    ch.c1 = K.c1[1];
    ch.c2 = K.c2[1];
    TOSIMP_HIP(ctx, kv_level_launch(ctx, prec, E, b, xs[cur ^ 1], L.nx, L.ny, L.nz, L.mask,
                                    L.kscale, st, &ch));
    cur ^= 1;
  } else {
    cheb_kernel<T, 0><<<g, 256, 0, ctx->stream>>>(b, nullptr, xs[cur], dd, dinv, T(0),
                                                  (T)K.c2[0], nd, st);
    TOSIMP_HIP(ctx, hipGetLastError());
  }
  for (int s = 2; s < degree; ++s) TOSIMP_HIP(ctx, fused(2, K.c1[s], K.c2[s]));
  // coarse-grid correction
  TOSIMP_HIP(ctx, kv_level_launch(ctx, prec, E, xs[cur], t, L.nx, L.ny, L.nz, L.mask,
                                  L.kscale, st));
  MgLevel& Cn = M->L[l + 1];
  {
    const int per = xcd_per(Cn.n_node, 256);
    restrict_residual_kernel<T><<<8 * per, 256, 0, ctx->stream>>>(
        b, t, L.nx, L.ny, L.nz, (T*)Cn.b, Cn.mask, Cn.nx, Cn.ny, Cn.nz, st, per);
  }
  TOSIMP_HIP(ctx, hipGetLastError());
  int rc = vcycle<T>(ctx, M, l + 1, K, degree, st);
  if (rc) return rc;
  {
    const int per = xcd_per(L.n_node, 256);
    prolong_add_kernel<T><<<8 * per, 256, 0, ctx->stream>>>(
        xs[cur], L.mask, L.nx, L.ny, L.nz, (const T*)Cn.x, Cn.nx, Cn.ny, Cn.nz, st, per);
  }
  TOSIMP_HIP(ctx, hipGetLastError());
  // post-smoothing from x (same polynomial); on the finest level the last pass also
  // forms <b, x> when the caller asked for it
  const bool dot_here = l == 0 && M->dot_part != nullptr;
  TOSIMP_HIP(ctx, fused(1, 0.0, K.c2[0], dot_here && degree == 1));
  for (int s = 1; s < degree; ++s)
    TOSIMP_HIP(ctx, fused(2, K.c1[s], K.c2[s], dot_here && s == degree - 1));
  if (cur != 0) return tosimp_fail(ctx, TOSIMP_ESTATE, "multigrid: smoothing parity");
  return TOSIMP_OK;
}

int check_degree_alpha(tosimp_ctx* ctx, int* degree, double* alpha) {
  if (*degree == 0) *degree = 2;
  if (*alpha == 0) *alpha = 20.0;
  if (*degree < 1 || *degree > 16 || !(*alpha > 1.0) || !std::isfinite(*alpha))
    return tosimp_fail(ctx, TOSIMP_EINVAL, "multigrid: degree 1..16 and alpha > 1 needed");
  return TOSIMP_OK;
}

}  // namespace

// z = V(r) on the fine level (set-up must be current).
template <typename T>
int mg_apply(tosimp_ctx* ctx, const T* r, T* z, int degree, double alpha, const SolverState* st,
             double* dot_part, int* dot_tiles) {
  MgState* M = mg_of(ctx);
  M->L[0].b = const_cast<T*>(r);
  M->L[0].x = z;
  M->dot_part = dot_part;
  M->dot_tiles = 0;
  const ChebCoef K = cheb_coef(M->lam, alpha, degree);
  const int rc = vcycle<T>(ctx, M, 0, K, degree, st);
  if (dot_tiles) *dot_tiles = M->dot_tiles;
  M->L[0].b = M->L[0].x = nullptr;
  M->dot_part = nullptr;
  return rc;
}

// CG on K_c(x) u = b preconditioned by one V-cycle per iteration (set-up done by the
// caller).  r, z, p, q: n_dof work vectors of T.  x: element values of the operator's
// type (FP64 densities for T = double, the FP32 copy for T = float).
template <typename T>
int mg_pcg(tosimp_ctx* ctx, const void* x, const T* b, T* u, T* r, T* z, T* p, T* q,
           int slot, double tol, int maxit, int check_every, bool zero_guess, int degree,
           double alpha, bool graphs, MgPcgResult* res) {
  constexpr int prec = sizeof(T) == 8 ? TOSIMP_PREC_FP64 : TOSIMP_PREC_FP32;
  constexpr int xdt = sizeof(T) == 8 ? TOSIMP_F64 : TOSIMP_F32;
  Workspace& w = ctx->ws;
  SolverState* st = w.st + slot;
  SolverState* sh = w.st_host + slot;
  *sh = SolverState{};
  sh->aux = tol * tol;
  sh->maxit = maxit < 1 ? 1 : maxit;
  TOSIMP_HIP(ctx, hipMemcpyAsync(st, sh, sizeof(SolverState), hipMemcpyHostToDevice, ctx->stream));
  double* part = w.partials;
  double* kvpart = w.partials + 2 * kMaxPartials;
  const int64_t n = ctx->n_dof;
  if (zero_guess) {
    TOSIMP_HIP(ctx, launch_fill_zero(ctx, u, n * (int64_t)sizeof(T)));
    mgcg_init_kernel<T><<<kRedBlocks, kRedThreads, 0, ctx->stream>>>(b, nullptr, r, w.mask, n, part);
  } else {
    TOSIMP_HIP(ctx, kv_launch(ctx, prec, xdt, x, u, q, nullptr, st, nullptr, 0, false, true));
    mgcg_init_kernel<T><<<kRedBlocks, kRedThreads, 0, ctx->stream>>>(b, q, r, w.mask, n, part);
  }
  TOSIMP_HIP(ctx, launch_finalize_sum<2>(ctx->stream, part, kRedBlocks, MgInitFin{st}));
  if (check_every < 1) check_every = 1;
  const int g = grid_for(n);
  // One batch of k iterations (every kernel returns at once after convergence).
  auto batch = [&](int k) -> int {
    for (int i = 0; i < k; ++i) {
      // <r, z> comes out of the V-cycle's last finest-level pass (per-tile partials),
      // else (the whole V-cycle in the single-workgroup tail) from its own kernel
      int tiles = 0;
      int rc = mg_apply<T>(ctx, r, z, degree, alpha, st, kvpart, &tiles);
      if (rc) return rc;
      if (tiles > 0) {
        TOSIMP_HIP(ctx, launch_finalize_sum<1>(ctx->stream, kvpart, tiles, MgRzFin{st}));
      } else {
        dot_rz_kernel<T><<<g, kRedThreads, 0, ctx->stream>>>(r, z, n, st, part);
        TOSIMP_HIP(ctx, launch_finalize_sum<1>(ctx->stream, part, g, MgRzFin{st}));
      }
      mg_direction_kernel<T><<<g, kRedThreads, 0, ctx->stream>>>(z, p, n, st);
      TOSIMP_HIP(ctx, kv_launch(ctx, prec, xdt, x, p, q, kvpart, st, nullptr, 1, true, true));
      mg_update_kernel<T><<<g, kRedThreads, 0, ctx->stream>>>(u, r, p, q, n, st, part);
      TOSIMP_HIP(ctx, launch_finalize_sum<1>(ctx->stream, part, g, MgUpdateFin{st}));
    }
    return TOSIMP_OK;
  };
  // Batch sizes: check_every and its halvings down to 1.  The first batch has the full
  // size; after it, each batch is the smallest size that covers the iterations the
  // observed contraction of ||r||^2 per iteration still needs, so that few iterations are
  // enqueued past convergence (they return at once, but each of their launches still
  // costs a few microseconds).  Batches run as HIP graphs (a V-cycle is a few dozen
  // launches, which bound the iteration on small meshes): each size is captured on first
  // use, after one eager batch, and kept in the hierarchy's cache for later solves with
  // the same launches (refinement steps, SIMP iterations).  The graphs hold only this
  // library's kernels (no memset or copy nodes).
  MgState* M = mg_of(ctx);
  std::vector<int> sizes;
  for (int k = check_every; k >= 1; k /= 2) sizes.push_back(k);
  const void* ptrs[7] = {x, b, u, r, z, p, q};
  auto cached = [&](int k) -> MgGraph* {
    for (MgGraph& gph : M->graphs) {
      if (gph.tsize != (int)sizeof(T) || gph.k != k || gph.degree != degree ||
          gph.slot != slot || gph.alpha != alpha || gph.penal != ctx->penal)
        continue;
      if (std::equal(ptrs, ptrs + 7, gph.ptr)) return &gph;
    }
    return nullptr;
  };
  int batches = 0, it_prev = 0;
  double rr_prev = 0.0;
  for (;;) {
    TOSIMP_HIP(ctx, hipMemcpyAsync(sh, st, sizeof(SolverState), hipMemcpyDeviceToHost, ctx->stream));
    TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (sh->done) break;
    int want = check_every;
    if (batches > 0 && sh->iter > it_prev && rr_prev > 0.0 && sh->rr > 0.0 &&
        sh->rr < rr_prev && sh->tol2 > 0.0) {
      const double per_it = std::log(sh->rr / rr_prev) / (double)(sh->iter - it_prev);
      const double need = std::log(sh->tol2 / sh->rr) / per_it;  // both logs negative
      if (std::isfinite(need)) want = (int)std::min<double>(check_every, std::ceil(need));
    }
    // the smallest size that covers the estimate (at most check_every)
    size_t si = 0;
    while (si + 1 < sizes.size() && sizes[si + 1] >= want) ++si;
    const int k = sizes[si];
    it_prev = sh->iter;
    rr_prev = sh->rr;
    MgGraph* gph = graphs ? cached(k) : nullptr;
    if (graphs && !gph && batches >= 1) {
      hipGraph_t gr = nullptr;
      TOSIMP_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
      const int rc = batch(k);
      const hipError_t ee = hipStreamEndCapture(ctx->stream, &gr);
      if (rc) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
      }
      TOSIMP_HIP(ctx, ee);
      MgGraph fresh;
      fresh.tsize = (int)sizeof(T);
      fresh.k = k;
      fresh.degree = degree;
      fresh.slot = slot;
      fresh.alpha = alpha;
      fresh.penal = ctx->penal;
      std::copy(ptrs, ptrs + 7, fresh.ptr);
      const hipError_t ie = hipGraphInstantiate(&fresh.exec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      TOSIMP_HIP(ctx, ie);
      if (M->graphs.size() >= kMgGraphCache) {  // drop the oldest
        (void)hipGraphExecDestroy(M->graphs.front().exec);
        M->graphs.erase(M->graphs.begin());
      }
      M->graphs.push_back(fresh);
      gph = &M->graphs.back();
    }
    if (gph) {
      TOSIMP_HIP(ctx, hipGraphLaunch(gph->exec, ctx->stream));
    } else {
      const int rc = batch(k);
      if (rc) return rc;
    }
    ++batches;
  }
  res->iters = sh->iter;
  res->done = sh->done;
  res->rr = sh->rr;
  res->bb = sh->bb;
  return TOSIMP_OK;
}

template int mg_apply<double>(tosimp_ctx*, const double*, double*, int, double, const SolverState*,
                              double*, int*);
template int mg_apply<float>(tosimp_ctx*, const float*, float*, int, double, const SolverState*,
                             double*, int*);
template int mg_pcg<double>(tosimp_ctx*, const void*, const double*, double*, double*, double*,
                            double*, double*, int, double, int, int, bool, int, double, bool,
                            MgPcgResult*);
template int mg_pcg<float>(tosimp_ctx*, const void*, const float*, float*, float*, float*,
                           float*, float*, int, double, int, int, bool, int, double, bool,
                           MgPcgResult*);

int mg_prepare(tosimp_ctx* ctx, const double* x, int* degree, double* alpha) {
  int rc = check_degree_alpha(ctx, degree, alpha);
  if (rc) return rc;
  return mg_setup(ctx, x);
}

int mg_levels(tosimp_ctx* ctx, int* dims, int cap) {
  int rc = mg_create(ctx);
  if (rc) return rc;
  MgState* M = mg_of(ctx);
  for (int l = 0; l < M->nlev && l < cap; ++l) {
    dims[3 * l] = M->L[l].nx;
    dims[3 * l + 1] = M->L[l].ny;
    dims[3 * l + 2] = M->L[l].nz;
  }
  return M->nlev;
}

void mg_release(tosimp_ctx* ctx) {
  MgState* M = ctx ? mg_of(ctx) : nullptr;
  if (!M) return;
  for (int l = 0; l < M->nlev; ++l) {
    MgLevel& L = M->L[l];
    void* ps[] = {L.E64, L.E32, L.dinv64, L.dinv32, L.t, L.dd, L.xa};
    for (void* p : ps)
      if (p) (void)hipFree(p);
    if (l > 0) {
      if (L.mask) (void)hipFree(L.mask);
      if (L.b) (void)hipFree(L.b);
      if (L.x) (void)hipFree(L.x);
    }
  }
  if (M->Ainv64) (void)hipFree(M->Ainv64);
  if (M->Ainv32) (void)hipFree(M->Ainv32);
  for (MgGraph& g : M->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  delete M;
  ctx->mg = nullptr;
}

}  // namespace tosimp
