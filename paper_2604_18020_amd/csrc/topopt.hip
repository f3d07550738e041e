// SIMP kernels: element sensitivities, cone density filter, OC bisection (FP64).
//
// Paper: Sec. "Three-Dimensional SIMP Topology Optimization" (analytic sensitivities,
// cone filter of radius rmin, optimality-criteria update with bisection on the volume
// multiplier).  The update rule, the filter chain rule and the bisection constants are
// the standard density-filter SIMP ones (bracket [0, 1e9], relative width 1e-3).
#include "common.h"
#include "dev.h"

namespace tosimp {

// ------------------------------------------------------------ sensitivities
// ce_e = u_e^T K_E u_e evaluated in the Hadamard basis as hat^T S hat (hat = H u_e);
// dc_e = -p x^(p-1) (E0 - Emin) ce_e.  dc may be x itself (each thread reads x_e before
// writing dc_e), so neither carries __restrict__.
__global__ __launch_bounds__(256) void sensitivity_kernel(
    const double* x, const double* __restrict__ u, double* dc,
    int nx, int ny, int nz, HadConsts k, double penal, double E0mEmin, int per_xcd) {
  const int64_t n_elem = (int64_t)nx * ny * nz;
  const int64_t NX1 = nx + 1, plane = NX1 * (ny + 1);
  {
    const int64_t e = xcd_item(per_xcd);
    if (e >= n_elem) return;
    const int ex = (int)(e % nx);
    const int64_t r = e / nx;
    const int ey = (int)(r % ny);
    const int ez = (int)(r / ny);
    const int64_t n0 = ex + NX1 * ey + plane * ez;
    double h[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int64_t n = n0 + (a & 1) + NX1 * ((a >> 1) & 1) + plane * ((a >> 2) & 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) h[a][c] = u[3 * n + c];
    }
    // Butterflies along x, y, z: afterwards h[m][c] is mode m (bit set = difference).
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (!(a & bit))
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double s = h[a][c] + h[a | bit][c], d = h[a | bit][c] - h[a][c];
            h[a][c] = s;
            h[a | bit][c] = d;
          }
    const double sA = k.ao * (h[1][0] + h[2][1] + h[4][2]);
    const double sC = k.co * (h[3][2] + h[5][1] + h[6][0]);
    const double s1 = k.cs * (h[1][1] + h[2][0]);
    const double s2 = k.cs * (h[1][2] + h[4][0]);
    const double s3 = k.cs * (h[2][2] + h[4][1]);
    double ce = 0.0;
    ce += h[1][0] * (k.ad * h[1][0] + sA) + h[2][1] * (k.ad * h[2][1] + sA) +
          h[4][2] * (k.ad * h[4][2] + sA);
    ce += s1 * (h[1][1] + h[2][0]) + s2 * (h[1][2] + h[4][0]) + s3 * (h[2][2] + h[4][1]);
    ce += h[3][0] * (k.bd * h[3][0] + k.bo * h[6][2]) + h[6][2] * (k.bo * h[3][0] + k.bd * h[6][2]);
    ce += h[3][1] * (k.bd * h[3][1] + k.bo * h[5][2]) + h[5][2] * (k.bo * h[3][1] + k.bd * h[5][2]);
    ce += h[5][0] * (k.bd * h[5][0] + k.bo * h[6][1]) + h[6][1] * (k.bo * h[5][0] + k.bd * h[6][1]);
    ce += h[3][2] * (k.cd * h[3][2] + sC) + h[5][1] * (k.cd * h[5][1] + sC) +
          h[6][0] * (k.cd * h[6][0] + sC);
    ce += k.hg * (h[7][0] * h[7][0] + h[7][1] * h[7][1] + h[7][2] * h[7][2]);
    const double xv = x[e];
    const double dxp = penal == 3.0 ? 3.0 * xv * xv
                                    : (xv > 0.0 ? penal * pow(xv, penal - 1.0) : 0.0);
    dc[e] = -dxp * E0mEmin * ce;
  }
}

hipError_t launch_sensitivity(const tosimp_ctx* c, const double* xphys, const double* u,
                              double* dc) {
  const int per = xcd_per(c->n_elem, 256);
  sensitivity_kernel<<<8 * per, 256, 0, c->stream>>>(xphys, u, dc, c->nx, c->ny, c->nz, c->hc,
                                                     c->penal, c->E0 - c->Emin, per);
  return hipGetLastError();
}

// ------------------------------------------------------------------ filter
// Cone filter over the offset cube [-R, R]^3 with weights w (zero outside the cone).
// mode 0: out = sum w in_j / Hs_e; mode 1: out = sum w in_j / Hs_j; mode 2: Hs = sum w.
__global__ __launch_bounds__(256) void filter_kernel(const double* __restrict__ in,
                                                     double* __restrict__ out,
                                                     const double* __restrict__ Hs,
                                                     const double* __restrict__ w, int R,
                                                     int nx, int ny, int nz, int mode,
                                                     int per_xcd) {
  const int64_t n_elem = (int64_t)nx * ny * nz;
  const int W = 2 * R + 1;
  {
    const int64_t e = xcd_item(per_xcd);
    if (e >= n_elem) return;
    const int ex = (int)(e % nx);
    const int64_t r = e / nx;
    const int ey = (int)(r % ny);
    const int ez = (int)(r / ny);
    double s = 0.0;
    for (int dk = -R; dk <= R; ++dk) {
      const int jz = ez + dk;
      if (jz < 0 || jz >= nz) continue;
      for (int dj = -R; dj <= R; ++dj) {
        const int jy = ey + dj;
        if (jy < 0 || jy >= ny) continue;
        for (int di = -R; di <= R; ++di) {
          const int jx = ex + di;
          if (jx < 0 || jx >= nx) continue;
          const double wt = w[(di + R) + W * ((dj + R) + W * (dk + R))];
          if (wt <= 0.0) continue;
          const int64_t j = jx + (int64_t)nx * (jy + (int64_t)ny * jz);
          if (mode == 2) s += wt;
          else if (mode == 1) s += wt * (in[j] / Hs[j]);
          else s += wt * in[j];
        }
      }
    }
    out[e] = mode == 0 ? s / Hs[e] : s;
  }
}

// Radius-one filter (rmin in (1, 2]: the 27-point offset cube), the common case.  The cone
// weight depends only on the distance, so with w0..w3 the weights at distance 0, 1, sqrt 2
// and sqrt 3, and per plane z the centre value c, the sum F of its four in-plane face
// neighbours and the sum G of its four in-plane diagonal neighbours,
//   A(z) = w0 c + w1 F + w2 G   (the plane's own contribution),
//   B(z) = w1 c + w2 F + w3 G   (its contribution to the planes above and below),
// and the filtered value is B(z-1) + A(z) + B(z+1).  A block sweeps a 64 x 4 element tile
// up a chunk of z planes, staging each plane with a one-element halo in LDS (values
// outside the mesh staged as 0); the adjoint stages in / Hs, the forward multiplies the
// sum by 1 / Hs.
constexpr int kFtX = 64, kFtY = 4, kFtKz = 8;
constexpr int kFwX = kFtX + 2, kFwY = kFtY + 2, kFwin = kFwX * kFwY;  // 396 staged values

template <int MODE>
__global__ __launch_bounds__(256) void filter_sweep_kernel(const double* __restrict__ in,
                                                           double* __restrict__ out,
                                                           const double* __restrict__ hinv,
                                                           double w0, double w1, double w2,
                                                           double w3, int nx, int ny, int nz,
                                                           int tiles_x, int tiles_y,
                                                           int ntiles, int per_xcd) {
  __shared__ double sp[2][kFwin];
  const int bid = blockIdx.x;
  const int t = (bid & 7) * per_xcd + (bid >> 3);  // contiguous tile range per XCD
  if (t >= ntiles) return;
  const int tx = t % tiles_x, rest = t / tiles_x;
  const int ty = rest % tiles_y, cz = rest / tiles_y;
  const int x0 = tx * kFtX - 1, y0 = ty * kFtY - 1;
  const int k0 = cz * kFtKz, k1 = min(k0 + kFtKz, nz);  // output planes [k0, k1)
  const int tid = threadIdx.x;
  const int lx = tid % kFtX, ly = tid / kFtX;
  const int ex = x0 + 1 + lx, ey = y0 + 1 + ly;
  const bool own = ex < nx && ey < ny;
  const int layer = nx * ny;
  // staged slots of this thread (two per plane at most: 396 values over 256 threads)
  int soff[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int q = tid + 256 * s;
    const int i = x0 + q % kFwX, j = y0 + q / kFwX;
    soff[s] = (q < kFwin && i >= 0 && i < nx && j >= 0 && j < ny) ? i + nx * j : -1;
  }
  double Bm2 = 0.0, Am1 = 0.0, Bm1 = 0.0;  // B(z-2), A(z-1), B(z-1)
  for (int z = k0 - 1; z <= k1; ++z) {
    double* P = sp[(z - k0 + 1) & 1];
    const bool zin = z >= 0 && z < nz;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int q = tid + 256 * s;
      if (q < kFwin) {
        double v = 0.0;
        if (zin && soff[s] >= 0) {
          const int j = soff[s] + layer * z;
          v = MODE == TOSIMP_FILTER_ADJOINT ? in[j] * hinv[j] : in[j];
        }
        P[q] = v;
      }
    }
    __syncthreads();
    const int q = (ly + 1) * kFwX + lx + 1;
    const double c = P[q];
    const double F = (P[q - 1] + P[q + 1]) + (P[q - kFwX] + P[q + kFwX]);
    const double G = (P[q - kFwX - 1] + P[q - kFwX + 1]) + (P[q + kFwX - 1] + P[q + kFwX + 1]);
    const double A = w0 * c + w1 * F + w2 * G;
    const double B = w1 * c + w2 * F + w3 * G;
    // plane z - 1 is complete: B(z-2) + A(z-1) + B(z)
    if (z - 1 >= k0 && own) {
      const int e = ex + nx * ey + layer * (z - 1);
      const double sum = Bm2 + Am1 + B;
      out[e] = MODE == TOSIMP_FILTER_FORWARD ? sum * hinv[e] : sum;
    }
    Bm2 = Bm1;
    Am1 = A;
    Bm1 = B;
    // the other buffer is rewritten next step; this one two steps on, after the next
    // barrier, so one barrier per plane suffices
  }
}

hipError_t launch_filter(const tosimp_ctx* c, const double* in, double* out, int mode) {
  if (c->fR == 1) {
    // weights at distance 0, 1, sqrt 2, sqrt 3 (offset-cube layout di + 3 (dj + 3 dk))
    const double w0 = c->fw_host[13], w1 = c->fw_host[14], w2 = c->fw_host[17],
                 w3 = c->fw_host[26];
    const int tiles_x = (c->nx + kFtX - 1) / kFtX, tiles_y = (c->ny + kFtY - 1) / kFtY;
    const int ntiles = tiles_x * tiles_y * ((c->nz + kFtKz - 1) / kFtKz);
    const int per = (ntiles + 7) / 8;
    if (mode == TOSIMP_FILTER_ADJOINT)
      filter_sweep_kernel<TOSIMP_FILTER_ADJOINT><<<8 * per, 256, 0, c->stream>>>(
          in, out, c->ws.Hsinv, w0, w1, w2, w3, c->nx, c->ny, c->nz, tiles_x, tiles_y, ntiles, per);
    else
      filter_sweep_kernel<TOSIMP_FILTER_FORWARD><<<8 * per, 256, 0, c->stream>>>(
          in, out, c->ws.Hsinv, w0, w1, w2, w3, c->nx, c->ny, c->nz, tiles_x, tiles_y, ntiles, per);
    return hipGetLastError();
  }
  const int per = xcd_per(c->n_elem, 256);
  filter_kernel<<<8 * per, 256, 0, c->stream>>>(in, out, c->ws.Hs, c->ws.fw, c->fR, c->nx,
                                                c->ny, c->nz, mode, per);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void reciprocal_kernel(const double* __restrict__ in,
                                                         double* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = 1.0 / in[i];
}

hipError_t launch_reciprocal(const tosimp_ctx* c, const double* in, double* out, int64_t n) {
  reciprocal_kernel<<<2048, 256, 0, c->stream>>>(in, out, n);
  return hipGetLastError();
}

hipError_t launch_filter_rowsum(const tosimp_ctx* c, double* Hs) {
  const int per = xcd_per(c->n_elem, 256);
  filter_kernel<<<8 * per, 256, 0, c->stream>>>(nullptr, Hs, nullptr, c->ws.fw, c->fR, c->nx,
                                                c->ny, c->nz, 2, per);
  return hipGetLastError();
}

// -------------------------------------------------------------- projection
// Smoothed Heaviside projection of the filtered density (the projection equation of the
// three-field scheme): out = (tanh(beta eta) + tanh(beta (in - eta))) / den with
// den = tanh(beta eta) + tanh(beta (1 - eta)); with g, the chain-rule product
// out = g beta (1 - tanh^2(beta (in - eta))) / den.  Elementwise, 16 bytes (24 with g)
// per element; out may be in or g itself.  With y = beta (in - eta), each form takes one
// exponential: tanh|y| = -m / (2 + m) with m = expm1(-2|y|) (no cancellation near y = 0),
// and 1 - tanh^2 y = 4 s / (1 + s)^2 with s = exp(-2|y|) (no cancellation where tanh is
// near 1); the constant divisions are folded into factors on the host.
__global__ __launch_bounds__(256) void project_kernel(const double* in, const double* g,
                                                      double* out, int64_t n, double beta,
                                                      double eta, double tbe_den, double inv_den,
                                                      double four_beta_den) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double y = beta * (in[e] - eta);
    if (g) {
      const double s = exp(-2.0 * fabs(y));
      const double q = 1.0 / (1.0 + s);
      out[e] = g[e] * (four_beta_den * s * q * q);
    } else {
      const double m = expm1(-2.0 * fabs(y));
      const double t = -m / (2.0 + m);
      out[e] = tbe_den + copysign(t, y) * inv_den;
    }
  }
}

hipError_t launch_project(const tosimp_ctx* c, const double* in, const double* g, double* out,
                          double beta, double eta) {
  const double tbe = tanh(beta * eta), den = tbe + tanh(beta * (1.0 - eta));
  const int64_t n = c->n_elem;
  const int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
  project_kernel<<<blocks, 256, 0, c->stream>>>(in, g, out, n, beta, eta, tbe / den, 1.0 / den,
                                                4.0 * beta / den);
  return hipGetLastError();
}

// --------------------------------------------------------------------- OC
__device__ __forceinline__ double oc_x(double xv, double dcv, double dvv, double lmid,
                                       double move) {
  double xn = sqrt(-dcv / (dvv * lmid)) * xv;
  xn = fmin(fmin(xn, xv + move), 1.0);
  xn = fmax(fmax(xn, xv - move), 0.0);
  return xn;
}

// One bisection step: volume dv^T x_new(lmid) against the target moves l1 or l2.
__global__ __launch_bounds__(kRedThreads) void oc_step_kernel(
    const double* __restrict__ x, const double* __restrict__ dc, const double* __restrict__ dv,
    double move, int64_t n, OcState* oc, double* partials) {
  __shared__ double sred[kRedThreads / 64];
  if (oc->done) return;
  const double lmid = 0.5 * (oc->l2 + oc->l1);
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    s += dv[i] * oc_x(x[i], dc[i], dv[i], lmid, move);
  const double v[1] = {s};
  store_block_sums<1>(v, partials, sred);
}

// The volume at lmid moves l1 or l2; stop once the bracket is 1e-3 relative.
struct OcStepFin {
  OcState* oc;
  __device__ void operator()(const double* t) const {
    if (oc->done) return;
    const double lmid = 0.5 * (oc->l2 + oc->l1);
    const double vol = t[0];
    oc->vol = vol;
    oc->lmid = lmid;
    if (vol > oc->target) oc->l1 = lmid;
    else oc->l2 = lmid;
    oc->steps += 1;
    if (!((oc->l2 - oc->l1) / (oc->l1 + oc->l2) > 1e-3)) oc->done = 1;
  }
};

// x_new at the last evaluated multiplier and change = max |x_new - x|.
__global__ __launch_bounds__(kRedThreads) void oc_final_kernel(
    const double* __restrict__ x, const double* __restrict__ dc, const double* __restrict__ dv,
    double move, int64_t n, OcState* oc, double* __restrict__ xnew, double* partials) {
  __shared__ double sred[kRedThreads / 64];
  const double lmid = oc->lmid;
  double mx = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    const double xv = x[i];
    const double xn = oc_x(xv, dc[i], dv[i], lmid, move);
    xnew[i] = xn;
    mx = fmax(mx, fabs(xn - xv));
  }
  const double bm = block_max<kRedThreads>(mx, sred);
  if (threadIdx.x == 0) partials[blockIdx.x] = bm;
}

struct OcChangeFin {
  OcState* oc;
  __device__ void operator()(const double* t) const { oc->change = t[0]; }
};

hipError_t launch_oc_step(const tosimp_ctx* c, const double* x, const double* dc,
                          const double* dv, double move, OcState* oc, double* partials) {
  oc_step_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(x, dc, dv, move, c->n_elem, oc,
                                                            partials);
  return launch_finalize_sum<1>(c->stream, partials, kRedBlocks, OcStepFin{oc});
}

hipError_t launch_oc_final(const tosimp_ctx* c, const double* x, const double* dc,
                           const double* dv, double move, OcState* oc, double* xnew,
                           double* partials) {
  oc_final_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(x, dc, dv, move, c->n_elem, oc,
                                                             xnew, partials);
  return launch_finalize_max(c->stream, partials, kRedBlocks, OcChangeFin{oc});
}

hipError_t launch_oc_init(const tosimp_ctx*, OcState*, double) { return hipSuccess; }

// ------------------------------------------------- OC with the projected volume
// Three-field scheme: the bisection's volume is that of the projected density,
// sum_e project(filter(x_new))_e, which is not linear in x_new: each step writes x_new at
// the midpoint multiplier, then filters, projects and sums it (same block order every
// step).  The projection is evaluated as in project_kernel.
__device__ __forceinline__ double project_value(double xbar, double beta, double eta,
                                                double tbe_den, double inv_den) {
  const double y = beta * (xbar - eta);
  const double m = expm1(-2.0 * fabs(y));
  return tbe_den + copysign(-m / (2.0 + m), y) * inv_den;
}

__global__ __launch_bounds__(kRedThreads) void oc_xnew_kernel(
    const double* __restrict__ x, const double* __restrict__ dc, const double* __restrict__ dv,
    double move, int64_t n, const OcState* oc, double* __restrict__ xn) {
  if (oc->done) return;
  const double lmid = 0.5 * (oc->l2 + oc->l1);
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    xn[i] = oc_x(x[i], dc[i], dv[i], lmid, move);
}

__global__ __launch_bounds__(kRedThreads) void filter_project_sum_kernel(
    const double* __restrict__ in, const double* __restrict__ Hs, const double* __restrict__ w,
    int R, int nx, int ny, int nz, double beta, double eta, double tbe_den, double inv_den,
    const OcState* oc, double* partials) {
  __shared__ double sred[kRedThreads / 64];
  if (oc && oc->done) return;
  const int64_t n_elem = (int64_t)nx * ny * nz;
  const int W = 2 * R + 1;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; e < n_elem;
       e += (int64_t)gridDim.x * kRedThreads) {
    const int ex = (int)(e % nx);
    const int64_t r = e / nx;
    const int ey = (int)(r % ny);
    const int ez = (int)(r / ny);
    double s = 0.0;
    for (int dk = -R; dk <= R; ++dk) {
      const int jz = ez + dk;
      if (jz < 0 || jz >= nz) continue;
      for (int dj = -R; dj <= R; ++dj) {
        const int jy = ey + dj;
        if (jy < 0 || jy >= ny) continue;
        for (int di = -R; di <= R; ++di) {
          const int jx = ex + di;
          if (jx < 0 || jx >= nx) continue;
          const double wt = w[(di + R) + W * ((dj + R) + W * (dk + R))];
          if (wt <= 0.0) continue;
          s += wt * in[jx + (int64_t)nx * (jy + (int64_t)ny * jz)];
        }
      }
    }
    acc += project_value(s / Hs[e], beta, eta, tbe_den, inv_den);
  }
  const double v[1] = {acc};
  store_block_sums<1>(v, partials, sred);
}

static void projection_factors(double beta, double eta, double* tbe_den, double* inv_den) {
  const double tbe = tanh(beta * eta), den = tbe + tanh(beta * (1.0 - eta));
  *tbe_den = tbe / den;
  *inv_den = 1.0 / den;
}

hipError_t launch_oc_step_projected(const tosimp_ctx* c, const double* x, const double* dc,
                                    const double* dv, double move, double beta, double eta,
                                    double* xn, OcState* oc, double* partials) {
  double tbe_den, inv_den;
  projection_factors(beta, eta, &tbe_den, &inv_den);
  oc_xnew_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(x, dc, dv, move, c->n_elem, oc, xn);
  filter_project_sum_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(
      xn, c->ws.Hs, c->ws.fw, c->fR, c->nx, c->ny, c->nz, beta, eta, tbe_den, inv_den, oc,
      partials);
  return launch_finalize_sum<1>(c->stream, partials, kRedBlocks, OcStepFin{oc});
}

// ------------------------------------------------------------------ grayness
// g = 4/n sum_e rho_e (1 - rho_e): block sums of rho (1 - rho), finished into *out.
__global__ __launch_bounds__(kRedThreads) void gray_kernel(const double* __restrict__ rho,
                                                           int64_t n, double* partials) {
  __shared__ double sred[kRedThreads / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    s += rho[i] * (1.0 - rho[i]);
  const double v[1] = {s};
  store_block_sums<1>(v, partials, sred);
}

struct GrayFin {
  double* out;
  double scale;
  __device__ void operator()(const double* t) const { *out = scale * t[0]; }
};

hipError_t launch_grayness(const tosimp_ctx* c, const double* rho, double* partials,
                           double* out) {
  gray_kernel<<<kRedBlocks, kRedThreads, 0, c->stream>>>(rho, c->n_elem, partials);
  return launch_finalize_sum<1>(c->stream, partials, kRedBlocks,
                                GrayFin{out, 4.0 / (double)c->n_elem});
}

}  // namespace tosimp
