// C ABI entry points: context, set-up, operator, solvers, SIMP pieces, Lanczos.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "common.h"

using namespace tosimp;

int tosimp_fail(tosimp_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define REQUIRE(cond, code, msg)                          \
  do {                                                    \
    if (!(cond)) return tosimp_fail(ctx, code, msg);      \
  } while (0)

namespace {

// True when the byte ranges [a, a + an) and [b, b + bn) overlap.
bool overlaps(const void* a, int64_t an, const void* b, int64_t bn) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + (uintptr_t)bn && pb < pa + (uintptr_t)an;
}

// ------------------------------------------------ Lanczos scratch without allocation
// Device storage of tosimp_lanczos_noalloc: alpha[0..k) followed by beta[-1..k) of a
// run of at most kLanczosScratchSteps steps (256 KiB).  Each device holds its own copy
// until the process ends; every call on a device reuses it, so overlapping calls on one
// device race.  Host code never passes `scratch` itself (a host-side stand-in): it uses
// the device address that hipGetSymbolAddress returns, resolved once per device with
// that device current (tosimp_create).
constexpr int kLanczosScratchSteps = 16383;
__device__ __align__(256) double scratch[2 * (kLanczosScratchSteps + 1)];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device `device` (resolved on first use).
hipError_t scratch_address(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[device] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

// ------------------------------------------------------------- element stiffness
// K_E of a cube of edge h, unit Young's modulus, Poisson ratio nu: sum over the
// 2x2x2 Gauss points of B^T D B |J| w (exact for trilinear shape functions).
void element_stiffness(double nu, double h, double* KE) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  double D[6][6] = {};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D[i][j] = lam;
  for (int i = 0; i < 3; ++i) D[i][i] += 2.0 * mu;
  for (int i = 3; i < 6; ++i) D[i][i] = mu;
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  std::memset(KE, 0, sizeof(double) * 576);
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double xi[3] = {g[qx], g[qy], g[qz]};
        double dN[8][3];
        for (int a = 0; a < 8; ++a) {
          double f[3], df[3];
          for (int d = 0; d < 3; ++d) {
            const int bit = (a >> d) & 1;
            f[d] = bit ? xi[d] : 1.0 - xi[d];
            df[d] = bit ? 1.0 : -1.0;
          }
          // physical gradient on a cube of edge h: d/dX = (1/h) d/dxi
          dN[a][0] = df[0] * f[1] * f[2] / h;
          dN[a][1] = f[0] * df[1] * f[2] / h;
          dN[a][2] = f[0] * f[1] * df[2] / h;
        }
        double B[6][24] = {};
        for (int a = 0; a < 8; ++a) {
          B[0][3 * a] = dN[a][0];
          B[1][3 * a + 1] = dN[a][1];
          B[2][3 * a + 2] = dN[a][2];
          B[3][3 * a] = dN[a][1];
          B[3][3 * a + 1] = dN[a][0];
          B[4][3 * a + 1] = dN[a][2];
          B[4][3 * a + 2] = dN[a][1];
          B[5][3 * a] = dN[a][2];
          B[5][3 * a + 2] = dN[a][0];
        }
        const double wJ = 0.125 * h * h * h;
        double DB[6][24];
        for (int i = 0; i < 6; ++i)
          for (int j = 0; j < 24; ++j) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += D[i][k] * B[k][j];
            DB[i][j] = s;
          }
        for (int i = 0; i < 24; ++i)
          for (int j = 0; j < 24; ++j) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += B[k][i] * DB[k][j];
            KE[i * 24 + j] += s * wJ;
          }
      }
}

// S = H K_E H^T in the tensor Hadamard basis; returns false if S does not have the
// cube's 45-entry pattern (then the factored kernels cannot be used).
bool hadamard_consts(const double* KE, HadConsts* hc, double* max_dev) {
  double H[24][24] = {};
  for (int m = 0; m < 8; ++m)
    for (int a = 0; a < 8; ++a) {
      double s = 1.0;
      for (int d = 0; d < 3; ++d)
        if ((m >> d) & 1) s *= ((a >> d) & 1) ? 1.0 : -1.0;
      for (int c = 0; c < 3; ++c) H[3 * m + c][3 * a + c] = s;
    }
  double S[24][24];
  double T[24][24];
  for (int i = 0; i < 24; ++i)
    for (int j = 0; j < 24; ++j) {
      double s = 0;
      for (int k = 0; k < 24; ++k) s += H[i][k] * KE[k * 24 + j];
      T[i][j] = s;
    }
  double smax = 0;
  for (int i = 0; i < 24; ++i)
    for (int j = 0; j < 24; ++j) {
      double s = 0;
      for (int k = 0; k < 24; ++k) s += T[i][k] * H[j][k];
      S[i][j] = s;
      smax = std::max(smax, std::fabs(s));
    }
  auto at = [&](int m, int c, int m2, int c2) { return S[3 * m + c][3 * m2 + c2]; };
  const double Ad = at(1, 0, 1, 0), Ao = at(1, 0, 2, 1), Cs = at(1, 1, 1, 1);
  const double Bd = at(3, 0, 3, 0), Bo = at(3, 0, 6, 2), Cd = at(3, 2, 3, 2);
  const double Co = at(3, 2, 5, 1), Hg = at(7, 0, 7, 0);
  double M[24][24] = {};
  auto put = [&](int m, int c, int m2, int c2, double v) { M[3 * m + c][3 * m2 + c2] = v; };
  const int nb[3][2] = {{1, 0}, {2, 1}, {4, 2}};
  for (auto& p : nb)
    for (auto& q : nb) put(p[0], p[1], q[0], q[1], (p[0] == q[0]) ? Ad : Ao);
  const int sh[3][4] = {{1, 1, 2, 0}, {1, 2, 4, 0}, {2, 2, 4, 1}};
  for (auto& s : sh) {
    put(s[0], s[1], s[0], s[1], Cs);
    put(s[0], s[1], s[2], s[3], Cs);
    put(s[2], s[3], s[0], s[1], Cs);
    put(s[2], s[3], s[2], s[3], Cs);
  }
  const int bp[3][4] = {{3, 0, 6, 2}, {3, 1, 5, 2}, {5, 0, 6, 1}};
  for (auto& s : bp) {
    put(s[0], s[1], s[0], s[1], Bd);
    put(s[0], s[1], s[2], s[3], Bo);
    put(s[2], s[3], s[0], s[1], Bo);
    put(s[2], s[3], s[2], s[3], Bd);
  }
  const int tw[3][2] = {{3, 2}, {5, 1}, {6, 0}};
  for (auto& p : tw)
    for (auto& q : tw) put(p[0], p[1], q[0], q[1], (p[0] == q[0]) ? Cd : Co);
  for (int c = 0; c < 3; ++c) put(7, c, 7, c, Hg);
  double dev = 0;
  for (int i = 0; i < 24; ++i)
    for (int j = 0; j < 24; ++j) dev = std::max(dev, std::fabs(S[i][j] - M[i][j]));
  *max_dev = dev / smax;
  const double s = 1.0 / 64.0;
  hc->ad = (Ad - Ao) * s;
  hc->ao = Ao * s;
  hc->cs = Cs * s;
  hc->bd = Bd * s;
  hc->bo = Bo * s;
  hc->cd = (Cd - Co) * s;
  hc->co = Co * s;
  hc->hg = Hg * s;
  return *max_dev <= 1e-12;
}

void free_ws(tosimp_ctx* c) {
  nn_release(c);  // the network's tensors are sized for the mesh
  mg_release(c);  // so is the multigrid hierarchy
  Workspace& w = c->ws;
  void* dev[] = {w.mask, w.f,   w.Hs,  w.Hsinv, w.dv,  w.fw,  w.dinv, w.dinv32,  w.r,
                 w.p,    w.q,   w.w,   w.r32, w.p32, w.q32,  w.e32,     w.z32,
                 w.x32,  w.etmp, w.partials, w.lanczos, w.st, w.oc, w.ke_mfma};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (w.st_host) (void)hipHostFree(w.st_host);
  if (w.oc_host) (void)hipHostFree(w.oc_host);
  w = Workspace{};
}

template <typename P>
hipError_t dmalloc(P** p, size_t bytes) {
  return hipMalloc((void**)p, bytes < 256 ? 256 : bytes);
}

int check_ready(tosimp_ctx* ctx, bool need_bcs = true) {
  if (!ctx) return TOSIMP_EINVAL;
  if (!ctx->has_mesh) return tosimp_fail(ctx, TOSIMP_ESTATE, "no mesh: call tosimp_set_mesh first");
  (void)need_bcs;
  return TOSIMP_OK;
}

int set_device(tosimp_ctx* ctx) {
  TOSIMP_HIP(ctx, hipSetDevice(ctx->device));
  return TOSIMP_OK;
}

// Cone filter of radius ctx->rmin: weights max(0, rmin - |offset|) on the offset cube,
// the row sums Hs = H 1, their reciprocals, and dv = H (1 / Hs) (the adjoint filter of
// ones).  Uses etmp.
int load_filter(tosimp_ctx* ctx) {
  Workspace& w = ctx->ws;
  ctx->fR = (int)std::ceil(ctx->rmin) - 1;
  const int W = 2 * ctx->fR + 1;
  for (int i = 0; i < kMaxFilterTaps; ++i) ctx->fw_host[i] = 0.0;
  for (int dk = 0; dk < W; ++dk)
    for (int dj = 0; dj < W; ++dj)
      for (int di = 0; di < W; ++di) {
        const double d = std::sqrt((double)((di - ctx->fR) * (di - ctx->fR) +
                                            (dj - ctx->fR) * (dj - ctx->fR) +
                                            (dk - ctx->fR) * (dk - ctx->fR)));
        ctx->fw_host[di + W * (dj + W * dk)] = std::max(0.0, ctx->rmin - d);
      }
  TOSIMP_HIP(ctx, hipMemcpyAsync(w.fw, ctx->fw_host, sizeof(double) * kMaxFilterTaps,
                                 hipMemcpyHostToDevice, ctx->stream));
  TOSIMP_HIP(ctx, launch_filter_rowsum(ctx, w.Hs));
  TOSIMP_HIP(ctx, launch_reciprocal(ctx, w.Hs, w.Hsinv, ctx->n_elem));
  TOSIMP_HIP(ctx, launch_fill64(ctx, w.etmp, ctx->n_elem, 1.0));
  TOSIMP_HIP(ctx, launch_filter(ctx, w.etmp, w.dv, TOSIMP_FILTER_ADJOINT));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TOSIMP_OK;
}

}  // namespace

// ===================================================================== lifecycle
extern "C" {

const char* tosimp_version(void) { return "tosimp 0.1 (gfx950)"; }

int tosimp_create(int device, void* stream, tosimp_ctx** out) {
  if (!out) return TOSIMP_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TOSIMP_EINVAL;
  tosimp_ctx* c = new (std::nothrow) tosimp_ctx();
  if (!c) return TOSIMP_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return TOSIMP_EHIP;
  }
  // The allocation-free Lanczos entry point's device storage, once per device.
  if (scratch_address(device, &c->scratch) != hipSuccess) {
    delete c;
    return TOSIMP_EHIP;
  }
  *out = c;
  return TOSIMP_OK;
}

int tosimp_destroy(tosimp_ctx* ctx) {
  if (!ctx) return TOSIMP_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->own_stream) {
    (void)hipStreamSynchronize(ctx->own_stream);
    (void)hipStreamDestroy(ctx->own_stream);
    (void)hipEventDestroy(ctx->ev_in);
    (void)hipEventDestroy(ctx->ev_out);
  }
  free_ws(ctx);
  nn_release(ctx);
  mg_release(ctx);
  delete ctx;
  return TOSIMP_OK;
}

int tosimp_set_stream(tosimp_ctx* ctx, void* stream) {
  if (!ctx) return TOSIMP_EINVAL;
  ctx->stream = (hipStream_t)stream;
  return TOSIMP_OK;
}

const char* tosimp_last_error(const tosimp_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

int tosimp_counts(const tosimp_ctx* ctx, int64_t* n_elem, int64_t* n_node, int64_t* n_dof) {
  if (!ctx || !ctx->has_mesh) return ctx ? TOSIMP_ESTATE : TOSIMP_EINVAL;
  if (n_elem) *n_elem = ctx->n_elem;
  if (n_node) *n_node = ctx->n_node;
  if (n_dof) *n_dof = ctx->n_dof;
  return TOSIMP_OK;
}

// ===================================================================== set-up
int tosimp_set_mesh(tosimp_ctx* ctx, int nx, int ny, int nz, double h, double E0,
                    double Emin, double nu, double penal, double rmin) {
  if (!ctx) return TOSIMP_EINVAL;
  REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, TOSIMP_EINVAL, "mesh sizes must be >= 1");
  REQUIRE(h > 0 && std::isfinite(h), TOSIMP_EINVAL, "h must be positive");
  REQUIRE(E0 > 0 && Emin >= 0 && Emin < E0, TOSIMP_EINVAL, "need 0 <= Emin < E0");
  REQUIRE(nu > -1.0 && nu < 0.5, TOSIMP_EINVAL, "nu must be in (-1, 0.5)");
  REQUIRE(penal >= 1.0 && penal <= 16.0, TOSIMP_EINVAL, "penal must be in [1, 16]");
  REQUIRE(rmin > 0 && rmin <= kMaxFilterR + 1, TOSIMP_EINVAL, "rmin must be in (0, 4]");
  const int64_t n_elem = (int64_t)nx * ny * nz;
  const int64_t n_node = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  // The fused operator addresses an FP64 DOF vector through a buffer resource with
  // 32-bit byte offsets and gives lanes outside the mesh the offset 0x7FFFFFF0, which
  // must lie past the end of every array: 24 bytes per node <= 0x7FFFFFF0.
  REQUIRE(24 * n_node <= (int64_t)0x7FFFFFF0, TOSIMP_EINVAL,
          "mesh too large (more than 89,478,484 nodes)");
  int rc = set_device(ctx);
  if (rc) return rc;
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  free_ws(ctx);
  ctx->has_mesh = ctx->has_bcs = ctx->has_loads = false;
  ctx->kappa_uniform = 0;
  ctx->nx = nx; ctx->ny = ny; ctx->nz = nz;
  ctx->n_elem = n_elem; ctx->n_node = n_node; ctx->n_dof = 3 * n_node;
  ctx->h = h; ctx->E0 = E0; ctx->Emin = Emin; ctx->nu = nu; ctx->penal = penal;
  ctx->rmin = rmin;
  element_stiffness(nu, h, ctx->KE);
  double dev = 0;
  if (!hadamard_consts(ctx->KE, &ctx->hc, &dev))
    return tosimp_fail(ctx, TOSIMP_EINVAL, "element stiffness lacks the cube pattern");
  ctx->kd = ctx->KE[0];
  for (int i = 1; i < 24; ++i)
    REQUIRE(std::fabs(ctx->KE[i * 25] - ctx->kd) <= 1e-14 * ctx->kd, TOSIMP_EINVAL,
            "unequal diagonal of K_E");
  Workspace& w = ctx->ws;
  const size_t nd = (size_t)ctx->n_dof, nn = (size_t)n_node, ne = (size_t)n_elem;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  A(dmalloc(&w.mask, nn));
  A(dmalloc(&w.f, nd * 8));
  A(dmalloc(&w.Hs, ne * 8));
  A(dmalloc(&w.Hsinv, ne * 8));
  A(dmalloc(&w.dv, ne * 8));
  A(dmalloc(&w.fw, sizeof(double) * kMaxFilterTaps));
  A(dmalloc(&w.dinv, nn * 8));
  A(dmalloc(&w.dinv32, nn * 4));
  A(dmalloc(&w.r, nd * 8));
  A(dmalloc(&w.p, nd * 8));
  A(dmalloc(&w.q, nd * 8));
  A(dmalloc(&w.w, nd * 8));
  A(dmalloc(&w.r32, nd * 4));
  A(dmalloc(&w.p32, nd * 4));
  A(dmalloc(&w.q32, nd * 4));
  A(dmalloc(&w.e32, nd * 4));
  A(dmalloc(&w.z32, nd * 4));
  A(dmalloc(&w.x32, ne * 4));
  A(dmalloc(&w.etmp, ne * 8 * 6));
  // partial sums: 2 kMaxPartials for the vector kernels, then one slot per operator tile
  w.kv_part_cap = std::max<int64_t>(2 * kMaxPartials, kv_num_blocks(ctx));
  A(dmalloc(&w.partials, sizeof(double) * (2 * kMaxPartials + w.kv_part_cap)));
  A(dmalloc(&w.st, sizeof(SolverState) * 3));
  A(dmalloc(&w.oc, sizeof(OcState)));
  A(dmalloc(&w.ke_mfma, sizeof(uint16_t) * 2 * 2 * 64 * 8));
  if (e == hipSuccess) e = hipHostMalloc((void**)&w.st_host, sizeof(SolverState) * 3);
  if (e == hipSuccess) e = hipHostMalloc((void**)&w.oc_host, sizeof(OcState));
  if (e != hipSuccess) {
    free_ws(ctx);
    return tosimp_fail(ctx, TOSIMP_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
  }
  TOSIMP_HIP(ctx, hipMemsetAsync(w.mask, 0, nn, ctx->stream));
  TOSIMP_HIP(ctx, hipMemsetAsync(w.f, 0, nd * 8, ctx->stream));
  TOSIMP_HIP(ctx, hipMemsetAsync(w.st, 0, sizeof(SolverState) * 3, ctx->stream));
  TOSIMP_HIP(ctx, hipMemsetAsync(w.oc, 0, sizeof(OcState), ctx->stream));
  {
    // K_E (24x24, zero-padded to 32x32) in the A-operand lane layout of
    // v_mfma_f32_16x16x32_{bf16,f16}: lane l holds row 16 t + l % 16, columns
    // 8 (l / 16) .. + 7 of row tile t; rounding to nearest even.
    std::vector<uint16_t> tab(2 * 2 * 64 * 8);
    for (int pr = 0; pr < 2; ++pr)
      for (int t = 0; t < 2; ++t)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 8; ++j) {
            const int m = 16 * t + l % 16, k = 8 * (l / 16) + j;
            const float v = (m < 24 && k < 24) ? (float)ctx->KE[m * 24 + k] : 0.0f;
            uint16_t bits;
            if (pr == 0) {
              uint32_t u;
              std::memcpy(&u, &v, 4);
              bits = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
            } else {
              const _Float16 hv = (_Float16)v;
              std::memcpy(&bits, &hv, 2);
            }
            tab[((pr * 2 + t) * 64 + l) * 8 + j] = bits;
          }
    TOSIMP_HIP(ctx, hipMemcpyAsync(w.ke_mfma, tab.data(), tab.size() * 2, hipMemcpyHostToDevice,
                                   ctx->stream));
    TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  if ((rc = load_filter(ctx))) return rc;
  ctx->has_mesh = true;
  return TOSIMP_OK;
}

int tosimp_set_params(tosimp_ctx* ctx, double penal, double rmin) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(penal >= 1.0 && penal <= 16.0, TOSIMP_EINVAL, "penal must be in [1, 16]");
  REQUIRE(rmin > 0 && rmin <= kMaxFilterR + 1, TOSIMP_EINVAL, "rmin must be in (0, 4]");
  if ((rc = set_device(ctx))) return rc;
  ctx->penal = penal;
  if (rmin != ctx->rmin) {
    ctx->rmin = rmin;
    if ((rc = load_filter(ctx))) return rc;
  }
  return TOSIMP_OK;
}

int tosimp_set_bcs(tosimp_ctx* ctx, const int64_t* fixed, int64_t n) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(n >= 0 && (n == 0 || fixed), TOSIMP_EINVAL, "bad fixed-DOF list");
  std::vector<uint8_t> m((size_t)ctx->n_node, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t d = fixed[i];
    REQUIRE(d >= 0 && d < ctx->n_dof, TOSIMP_EINVAL, "fixed DOF id out of range");
    m[(size_t)(d / 3)] |= (uint8_t)(1u << (d % 3));
  }
  if ((rc = set_device(ctx))) return rc;
  TOSIMP_HIP(ctx, hipMemcpyAsync(ctx->ws.mask, m.data(), m.size(), hipMemcpyHostToDevice,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->has_bcs = true;
  ctx->kappa_uniform = 0;
  return TOSIMP_OK;
}

int tosimp_set_loads(tosimp_ctx* ctx, const double* f_dev) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(f_dev, TOSIMP_EINVAL, "null load vector");
  if ((rc = set_device(ctx))) return rc;
  const size_t nd = (size_t)ctx->n_dof;
  std::vector<double> f(nd);
  std::vector<uint8_t> m((size_t)ctx->n_node);
  TOSIMP_HIP(ctx, hipMemcpyAsync(f.data(), f_dev, nd * 8, hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipMemcpyAsync(m.data(), ctx->ws.mask, m.size(), hipMemcpyDeviceToHost,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (size_t i = 0; i < nd; ++i) {
    REQUIRE(std::isfinite(f[i]), TOSIMP_EINVAL, "non-finite load");
    if ((m[i / 3] >> (i % 3)) & 1)
      REQUIRE(f[i] == 0.0, TOSIMP_EINVAL, "load on a fixed DOF");
  }
  TOSIMP_HIP(ctx, hipMemcpyAsync(ctx->ws.f, f_dev, nd * 8, hipMemcpyDeviceToDevice, ctx->stream));
  ctx->has_loads = true;
  return TOSIMP_OK;
}

// ===================================================================== operator
int tosimp_apply_K(tosimp_ctx* ctx, const void* x, int xdtype, const void* v, void* y,
                   int prec) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && v && y, TOSIMP_EINVAL, "null pointer");
  REQUIRE(xdtype == TOSIMP_F64 || xdtype == TOSIMP_F32, TOSIMP_EINVAL, "bad xdtype");
  const bool vzero = (prec & TOSIMP_V_ZERO_ON_FIXED) != 0;
  const int scatter = prec & (TOSIMP_SCATTER_ATOMIC_ELEMENT | TOSIMP_SCATTER_ATOMIC_BRICK);
  prec &= ~(TOSIMP_V_ZERO_ON_FIXED | TOSIMP_SCATTER_ATOMIC_ELEMENT | TOSIMP_SCATTER_ATOMIC_BRICK);
  REQUIRE(prec >= TOSIMP_PREC_FP64 && prec <= TOSIMP_PREC_FP16_MFMA, TOSIMP_EINVAL,
          "bad precision");
  REQUIRE(scatter != (TOSIMP_SCATTER_ATOMIC_ELEMENT | TOSIMP_SCATTER_ATOMIC_BRICK) &&
              (!scatter || prec == TOSIMP_PREC_FP64 || prec == TOSIMP_PREC_FP32),
          TOSIMP_EINVAL, "one scatter form, FP64 or FP32 only");
  {
    const int64_t vb = ctx->n_dof * (prec == TOSIMP_PREC_FP64 ? 8 : 4);
    const int64_t xb = ctx->n_elem * (xdtype == TOSIMP_F64 ? 8 : 4);
    REQUIRE(!overlaps(v, vb, y, vb) && !overlaps(x, xb, y, vb), TOSIMP_EINVAL,
            "y must not overlap v or xphys");
  }
  if ((rc = set_device(ctx))) return rc;
  if (scatter) {
    TOSIMP_HIP(ctx, kv_atomic_launch(ctx, prec, xdtype, x, v, y, scatter));
  } else if (prec == TOSIMP_PREC_BF16_MFMA || prec == TOSIMP_PREC_FP16_MFMA) {
    TOSIMP_HIP(ctx, kv_mfma_launch(ctx, prec, xdtype, x, (const float*)v, (float*)y,
                                   ctx->ws.st, false));
  } else {
    TOSIMP_HIP(ctx, kv_launch(ctx, prec, xdtype, x, v, y, nullptr, ctx->ws.st, nullptr, 0,
                              false, vzero));
  }
  return TOSIMP_OK;
}

int tosimp_diag_K(tosimp_ctx* ctx, const void* x, int xdtype, void* d, int dtype) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && d, TOSIMP_EINVAL, "null pointer");
  REQUIRE((xdtype == TOSIMP_F64 || xdtype == TOSIMP_F32) &&
              (dtype == TOSIMP_F64 || dtype == TOSIMP_F32),
          TOSIMP_EINVAL, "bad dtype");
  if ((rc = set_device(ctx))) return rc;
  TOSIMP_HIP(ctx, launch_diag_full(ctx, xdtype, x, dtype, d));
  return TOSIMP_OK;
}

}  // extern "C"

// ===================================================================== solvers
namespace {

int kappa_run(tosimp_ctx* ctx, const double* x, const double* v0, int kmax, int jacobi,
              double rtol, int window, double* lmin, double* lmax, int* steps, int* converged);
int oc_run(tosimp_ctx* ctx, const double* x, const double* dc, const double* dv,
           double volfrac, double move, double beta, double eta, double* x_new,
           double* xphys_new, double* tmp, double* change, int* steps, double* volume);

struct PcgResult {
  int iters = 0;
  int done = 0;
  int harvested = 0;
  double rr = 0, bb = 0;
};

// Optional copies of (r_k, u_k) taken at the host polls of an FP64 solve.
struct Harvest {
  float* r = nullptr;
  float* u = nullptr;
  const double* ustar = nullptr;  // if set, u receives ustar - u_k (formed in FP64)
  int cap = 0;
};

// Jacobi-PCG on K_c(x) with vectors of type T; b, u, dinv of type T.  When zero_guess
// the initial iterate is 0 (u is cleared) and no initial operator application is made.
template <typename T>
int run_pcg(tosimp_ctx* ctx, int prec, const void* x, int xdtype, const T* b, T* u,
            const T* dinv, int slot, double tol, int maxit, int check_every, bool zero_guess,
            PcgResult* res, const Harvest* hv = nullptr, bool graphs = false) {
  Workspace& w = ctx->ws;
  T *r, *p, *q;
  if constexpr (sizeof(T) == 8) {
    r = (T*)w.r; p = (T*)w.p; q = (T*)w.q;
  } else {
    r = (T*)w.r32; p = (T*)w.p32; q = (T*)w.q32;
  }
  SolverState* st = w.st + slot;
  SolverState* sh = w.st_host + slot;
  // Stage the initial state through the pinned mirror (no pageable async copy).
  *sh = SolverState{};
  sh->aux = tol * tol;
  sh->maxit = maxit < 1 ? 1 : maxit;
  TOSIMP_HIP(ctx, hipMemcpyAsync(st, sh, sizeof(SolverState), hipMemcpyHostToDevice,
                                 ctx->stream));
  double* part = w.partials;
  double* kvpart = w.partials + 2 * kMaxPartials;
  if (zero_guess) {
    TOSIMP_HIP(ctx, launch_fill_zero(ctx, u, ctx->n_dof * (int64_t)sizeof(T)));
    TOSIMP_HIP(ctx, launch_pcg_init<T>(ctx, b, nullptr, r, p, dinv, st, part, 0));
  } else {
    // u was masked on entry to the solve; every CG vector stays zero on fixed DOFs
    TOSIMP_HIP(ctx, kv_launch(ctx, prec, xdtype, x, u, q, nullptr, st, nullptr, 0, false, true));
    TOSIMP_HIP(ctx, launch_pcg_init<T>(ctx, b, q, r, p, dinv, st, part, 1));
  }
  const bool mfma = prec == TOSIMP_PREC_BF16_MFMA || prec == TOSIMP_PREC_FP16_MFMA;
  if (check_every < 1) check_every = 1;
  // One batch of check_every iterations (every kernel returns at once after convergence).
  auto batch = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    for (int i = 0; i < check_every && e == hipSuccess; ++i) {
      if (mfma) {
        // MFMA operator computes q only; the step length comes from a separate dot.
        e = kv_mfma_launch(ctx, prec, xdtype, x, (const float*)p, (float*)q, st, true);
        if (e == hipSuccess)
          e = launch_alpha_from_dot32(ctx, (const float*)p, (const float*)q, kvpart, st);
      } else {
        e = kv_launch(ctx, prec, xdtype, x, p, q, kvpart, st, nullptr, 1, true, true);
      }
      // r and the step length first; u moves with the direction update (one read of p)
      if (e == hipSuccess) e = launch_pcg_update<T>(ctx, nullptr, r, nullptr, q, dinv, st, part);
      if (e == hipSuccess) e = launch_pcg_direction<T>(ctx, r, p, u, dinv, st);
    }
    return e;
  };
  // After one eager batch, the batch is captured once into a HIP graph and replayed: on
  // small meshes the iteration is bound by kernel launches.  The graph holds only this
  // library's kernels (no memset or copy nodes).
  hipGraphExec_t exec = nullptr;
  int batches = 0;
  struct ExecGuard {
    hipGraphExec_t* e;
    ~ExecGuard() {
      if (*e) (void)hipGraphExecDestroy(*e);
    }
  } guard{&exec};
  for (;;) {
    TOSIMP_HIP(ctx, hipMemcpyAsync(sh, st, sizeof(SolverState), hipMemcpyDeviceToHost,
                                   ctx->stream));
    TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (sh->done) break;
    if constexpr (sizeof(T) == 8) {
      if (hv && res->harvested < hv->cap) {
        const size_t off = (size_t)res->harvested * ctx->n_dof;
        TOSIMP_HIP(ctx, launch_cast32(ctx, (const double*)r, hv->r + off, ctx->n_dof));
        if (hv->ustar)
          TOSIMP_HIP(ctx, launch_diff_cast32(ctx, hv->ustar, (const double*)u, hv->u + off,
                                             ctx->n_dof));
        else
          TOSIMP_HIP(ctx, launch_cast32(ctx, (const double*)u, hv->u + off, ctx->n_dof));
        res->harvested += 1;
      }
    }
    if (graphs && batches == 1 && !exec) {
      hipGraph_t g = nullptr;
      TOSIMP_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
      const hipError_t ce = batch();
      const hipError_t ee = hipStreamEndCapture(ctx->stream, &g);
      TOSIMP_HIP(ctx, ce);
      TOSIMP_HIP(ctx, ee);
      const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      TOSIMP_HIP(ctx, ie);
    }
    if (exec) {
      TOSIMP_HIP(ctx, hipGraphLaunch(exec, ctx->stream));
    } else {
      TOSIMP_HIP(ctx, batch());
    }
    ++batches;
  }
  // the step of the iteration that ended the solve, if its direction update did not run
  TOSIMP_HIP(ctx, launch_pcg_finish<T>(ctx, u, p, st));
  res->iters = sh->iter;
  res->done = sh->done;
  res->rr = sh->rr;
  res->bb = sh->bb;
  return TOSIMP_OK;
}

// The conditioning estimate of the precision rule (enforce_rule = 2): Lanczos with the
// stopping rule (rtol 1e-3 over windows of 50 steps, at most 5,000 steps) on the
// Jacobi-scaled operator at uniform density (kappa does not depend on the uniform
// value or on the penalty), from a seeded normal start vector zeroed on fixed DOFs.
// Computed once per mesh and set of boundary conditions.  Uses the last etmp slot, w.r,
// w.p, w.q, w.w and w.dinv.
int kappa_uniform(tosimp_ctx* ctx, double* kappa) {
  if (ctx->kappa_uniform <= 0) {
    Workspace& w = ctx->ws;
    int rc = 0;
    double* xu = w.etmp + 5 * ctx->n_elem;  // the last slot: free during any solve
    TOSIMP_HIP(ctx, launch_fill64(ctx, xu, ctx->n_elem, 1.0));
    std::vector<double> h((size_t)ctx->n_dof);
    std::mt19937_64 gen(42);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (double& v : h) v = nd(gen);
    TOSIMP_HIP(ctx, hipMemcpyAsync(w.r, h.data(), h.size() * 8, hipMemcpyHostToDevice,
                                   ctx->stream));
    TOSIMP_HIP(ctx, launch_mask_vec(ctx, w.r));
    double lo = 0, hi = 0;
    int steps = 0, conv = 0;
    if ((rc = kappa_run(ctx, xu, w.r, 5000, 1, 1e-3, 50, &lo, &hi, &steps, &conv)))
      return rc;
    if (!(lo > 0) || !(hi > 0) || !std::isfinite(hi / lo))
      return tosimp_fail(ctx, TOSIMP_EBREAKDOWN, "conditioning estimate failed");
    ctx->kappa_uniform = hi / lo;
    ctx->kappa_converged = conv;
    ctx->kappa_steps = steps;
  }
  *kappa = ctx->kappa_uniform;
  return TOSIMP_OK;
}

double unit_roundoff(int prec) {
  switch (prec) {
    case TOSIMP_PREC_FP64: return std::ldexp(1.0, -53);
    case TOSIMP_PREC_FP32: return std::ldexp(1.0, -24);
    case TOSIMP_PREC_FP16_MFMA: return std::ldexp(1.0, -11);
    case TOSIMP_PREC_BF16_MFMA: return std::ldexp(1.0, -8);
  }
  return 1.0;
}

// ||b - K_c u|| in FP64 into *rr (uses w.q as scratch and w.r as the residual).
int true_residual(tosimp_ctx* ctx, const double* x, const double* b, const double* u,
                  double* rr) {
  Workspace& w = ctx->ws;
  SolverState* st = w.st + 2;
  TOSIMP_HIP(ctx, kv_launch(ctx, TOSIMP_PREC_FP64, TOSIMP_F64, x, u, w.q, nullptr, st, nullptr,
                            0, false, true));
  TOSIMP_HIP(ctx, launch_residual64(ctx, b, w.q, w.r, w.partials, st));
  TOSIMP_HIP(ctx, hipMemcpyAsync(w.st_host + 2, st, sizeof(SolverState), hipMemcpyDeviceToHost,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *rr = w.st_host[2].rr;
  return TOSIMP_OK;
}

int dot_host(tosimp_ctx* ctx, const double* a, const double* b, int64_t n, double* out) {
  Workspace& w = ctx->ws;
  SolverState* st = w.st + 2;
  TOSIMP_HIP(ctx, launch_dot64(ctx, a, b, n, w.partials, st, 0));
  TOSIMP_HIP(ctx, hipMemcpyAsync(w.st_host + 2, st, sizeof(SolverState), hipMemcpyDeviceToHost,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *out = w.st_host[2].aux;
  return TOSIMP_OK;
}

}  // namespace

namespace {
int pcg_solve_impl(tosimp_ctx* ctx, const double* x, const double* b, double* u,
                   const tosimp_solve_opts* o, tosimp_solve_stats* stats) {
  int rc = 0;
  REQUIRE(x && b && u && o, TOSIMP_EINVAL, "null pointer");
  REQUIRE(o->tol > 0 && o->maxit >= 0, TOSIMP_EINVAL, "bad tol/maxit");
  REQUIRE(o->mode == TOSIMP_SOLVE_PLAIN_FP64 || o->mode == TOSIMP_SOLVE_IR, TOSIMP_EINVAL,
          "bad solve mode");
  REQUIRE(!overlaps(u, 8 * ctx->n_dof, b, 8 * ctx->n_dof) &&
              !overlaps(u, 8 * ctx->n_dof, x, 8 * ctx->n_elem),
          TOSIMP_EINVAL, "u must not overlap b or xphys");
  REQUIRE(((uintptr_t)u & 15) == 0 && ((uintptr_t)b & 15) == 0, TOSIMP_EINVAL,
          "u and b must be 16-byte aligned");
  if ((rc = set_device(ctx))) return rc;
  tosimp_solve_stats s{};
  Workspace& w = ctx->ws;
  TOSIMP_HIP(ctx, launch_mask_vec(ctx, u));
  REQUIRE(o->precond == TOSIMP_PRECOND_JACOBI || o->precond == TOSIMP_PRECOND_NN ||
              o->precond == TOSIMP_PRECOND_MG,
          TOSIMP_EINVAL, "bad preconditioner");
  int mg_deg = o->mg_degree;
  double mg_alpha = o->mg_alpha;
  if (o->precond == TOSIMP_PRECOND_MG) {
    if ((rc = mg_prepare(ctx, x, &mg_deg, &mg_alpha))) return rc;
  }
  if (o->mode == TOSIMP_SOLVE_PLAIN_FP64 && o->precond == TOSIMP_PRECOND_MG) {
    // CG in FP64 preconditioned by an FP64 V-cycle (warm start from u)
    MgPcgResult pr;
    rc = mg_pcg<double>(ctx, x, b, u, w.r, w.w, w.p, w.q, 0, o->tol, o->maxit, o->check_every,
                        false, mg_deg, mg_alpha, !o->eager, &pr);
    if (rc) return rc;
    s.iterations = pr.iters;
    s.rel_residual = pr.bb > 0 ? std::sqrt(pr.rr / pr.bb) : 0.0;
    s.status = pr.done == 3 ? TOSIMP_EBREAKDOWN
                            : (pr.done == 2 ? TOSIMP_NOT_CONVERGED : TOSIMP_OK);
    double rr = 0;
    if ((rc = true_residual(ctx, x, b, u, &rr))) return rc;
    s.true_rel_residual = pr.bb > 0 ? std::sqrt(rr / pr.bb) : 0.0;
  } else if (o->mode == TOSIMP_SOLVE_PLAIN_FP64) {
    REQUIRE(o->precond == TOSIMP_PRECOND_JACOBI, TOSIMP_EINVAL,
            "plain FP64 mode uses the Jacobi or multigrid preconditioner");
    TOSIMP_HIP(ctx, launch_diag_inv(ctx, x, w.dinv, nullptr));
    PcgResult pr;
    Harvest hv;
    int every = o->check_every;
    if (o->harvest_r || o->harvest_u) {
      REQUIRE(o->harvest_r && o->harvest_u && o->harvest_cap >= 1 && o->harvest_every >= 1,
              TOSIMP_EINVAL, "harvest needs both arrays, harvest_cap >= 1, harvest_every >= 1");
      hv.r = o->harvest_r;
      hv.u = o->harvest_u;
      hv.ustar = o->harvest_ustar;
      hv.cap = o->harvest_cap;
      every = o->harvest_every;
    }
    rc = run_pcg<double>(ctx, TOSIMP_PREC_FP64, x, TOSIMP_F64, b, u, w.dinv, 0, o->tol,
                         o->maxit, every, false, &pr, hv.cap ? &hv : nullptr, !o->eager);
    if (rc) return rc;
    s.harvested = pr.harvested;
    s.iterations = pr.iters;
    s.rel_residual = pr.bb > 0 ? std::sqrt(pr.rr / pr.bb) : 0.0;
    s.status = pr.done == 3 ? TOSIMP_EBREAKDOWN
                            : (pr.done == 2 ? TOSIMP_NOT_CONVERGED : TOSIMP_OK);
    double rr = 0;
    if ((rc = true_residual(ctx, x, b, u, &rr))) return rc;
    s.true_rel_residual = pr.bb > 0 ? std::sqrt(rr / pr.bb) : 0.0;
  } else {
    int ip = o->inner_prec;
    REQUIRE(ip == TOSIMP_PREC_FP32 || ip == TOSIMP_PREC_BF16_MFMA || ip == TOSIMP_PREC_FP16_MFMA,
            TOSIMP_EINVAL, "IR inner precision must be FP32 or an MFMA precision");
    REQUIRE(o->inner_tol > 0 && o->inner_tol < 1 && o->max_outer >= 1, TOSIMP_EINVAL,
            "bad inner_tol/max_outer");
    REQUIRE(o->enforce_rule >= 0 && o->enforce_rule <= 2, TOSIMP_EINVAL, "bad enforce_rule");
    if (o->enforce_rule) {
      double kappa = o->kappa;
      if (o->enforce_rule == 2) {
        if ((rc = kappa_uniform(ctx, &kappa))) return rc;
      }
      REQUIRE(kappa > 0, TOSIMP_EINVAL, "enforce_rule 1 needs kappa > 0");
      s.kappa = kappa;
      if (unit_roundoff(ip) * kappa >= 1.0) {
        if (stats) *stats = s;
        return tosimp_fail(ctx, TOSIMP_EPRECISION,
                           "inner precision refused: unit roundoff * kappa >= 1");
      }
    }
    TOSIMP_HIP(ctx, launch_diag_inv(ctx, x, w.dinv, w.dinv32));
    TOSIMP_HIP(ctx, launch_copy_cast_x(ctx, x, w.x32));
    double bb = 0;
    if ((rc = dot_host(ctx, b, b, ctx->n_dof, &bb))) return rc;
    const double bn = std::sqrt(bb);
    int total = 0, outer = 0, fallbacks = 0, restarts = 0, escalations = 0, slow = 0;
    double prev = -1, rel = 0;
    int status = TOSIMP_OK;
    for (;;) {
      double rr = 0;
      if ((rc = true_residual(ctx, x, b, u, &rr))) return rc;  // residual left in w.r
      rel = bn > 0 ? std::sqrt(rr) / bn : 0.0;
      if (!std::isfinite(rel)) { status = TOSIMP_EBREAKDOWN; break; }
      if (rel <= o->tol || bn == 0) break;
      if (outer >= o->max_outer || total >= o->maxit) { status = TOSIMP_NOT_CONVERGED; break; }
      if (prev > 0 && rel > 0.5 * prev) {
        // two outer steps in a row that did not halve the residual: a matrix-core inner
        // precision is raised to FP32; at FP32 the solve stops (stagnation)
        if (++slow >= 2) {
          if (ip == TOSIMP_PREC_FP32) { status = TOSIMP_NOT_CONVERGED; break; }
          ip = TOSIMP_PREC_FP32;
          ++escalations;
          slow = 0;
        }
      } else {
        slow = 0;
      }
      prev = rel;
      const double sc = std::sqrt(rr);
      TOSIMP_HIP(ctx, launch_scale_to32(ctx, w.r, 1.0 / sc, w.e32));  // rhs in e32
      // Inner target: inner_tol, but no tighter than the reduction still needed to
      // reach tol (with a safety factor for the inner solve's own rounding).
      const double need = 0.3 * o->tol * bn / sc;
      const double itol = std::min(0.5, std::max(o->inner_tol, need));
      int it = 0, done = 0;
      if (o->precond == TOSIMP_PRECOND_MG) {
        REQUIRE(ip == TOSIMP_PREC_FP32, TOSIMP_EINVAL,
                "the multigrid inner solve runs in FP32");
        MgPcgResult pr;
        rc = mg_pcg<float>(ctx, w.x32, w.e32, w.z32, w.r32, (float*)w.w, w.p32, w.q32, 1, itol,
                           o->maxit - total, o->check_every, true, mg_deg, mg_alpha, !o->eager,
                           &pr);
        if (rc) return rc;
        it = pr.iters;
        done = pr.done;
      } else if (o->precond == TOSIMP_PRECOND_NN) {
        int fb = 0;
        const int stall = o->nn_stall == 0 ? 50 : o->nn_stall;
        rc = nn_fcg_solve(ctx, ip, w.x32, w.e32, w.z32, itol, o->maxit - total,
                          o->check_every, o->fcg_window, stall, &it, &fb, &done);
        if (rc < 0) return rc;
        fallbacks += fb;
        if (done == 4) {
          // The learned solve stagnated: plain Jacobi-PCG continues from its iterate on
          // the same right-hand side and tolerance, with the iterations left.
          PcgResult pr;
          rc = run_pcg<float>(ctx, ip, w.x32, TOSIMP_F32, w.e32, w.z32, w.dinv32, 1, itol,
                              o->maxit - total - it, o->check_every, false, &pr, nullptr,
                              !o->eager);
          if (rc) return rc;
          it += pr.iters;
          done = pr.done;
          ++restarts;
        }
      } else {
        PcgResult pr;
        rc = run_pcg<float>(ctx, ip, w.x32, TOSIMP_F32, w.e32, w.z32, w.dinv32, 1,
                            itol, o->maxit - total, o->check_every, true, &pr, nullptr,
                            !o->eager);
        if (rc) return rc;
        it = pr.iters;
        done = pr.done;
      }
      total += it;
      ++outer;
      TOSIMP_HIP(ctx, launch_axpy_from32(ctx, u, sc, w.z32));
      if (done == 3 && it == 0) { status = TOSIMP_EBREAKDOWN; break; }
    }
    s.iterations = total;
    s.outer_iterations = outer;
    s.fallbacks = fallbacks;
    s.restarts = restarts;
    s.escalations = escalations;
    s.rel_residual = rel;
    s.true_rel_residual = rel;
    s.status = status;
    if (status == TOSIMP_OK && (fallbacks > 0 || restarts > 0)) s.status = TOSIMP_FALLBACK_USED;
  }
  // b^T u and its second-order form b^T u + u^T r (r = b - K u, left in w.r by the final
  // true-residual evaluation of either mode).
  if (s.status >= 0) {
    double bu = 0, ur = 0;
    if ((rc = dot_host(ctx, b, u, ctx->n_dof, &bu))) return rc;
    if ((rc = dot_host(ctx, u, w.r, ctx->n_dof, &ur))) return rc;
    s.b_dot_u = bu;
    s.b_dot_u_corrected = bu + ur;
  }
  if (stats) *stats = s;
  if (s.status < 0) return tosimp_fail(ctx, s.status, "solve failed (breakdown)");
  return s.status;
}
}  // namespace

extern "C" {

// The solve runs on the context's own stream (non-blocking, default priority), ordered
// after the caller's stream by an event and before any later work on it by another, so
// that its iteration batches can be captured as HIP graphs whatever stream the caller
// uses (the legacy default stream cannot be captured).
int tosimp_pcg_solve(tosimp_ctx* ctx, const double* x, const double* b, double* u,
                     const tosimp_solve_opts* o, tosimp_solve_stats* stats) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(o, TOSIMP_EINVAL, "null pointer");
  if ((rc = set_device(ctx))) return rc;
  if (!ctx->own_stream) {
    TOSIMP_HIP(ctx, hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
    TOSIMP_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    TOSIMP_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
  }
  hipStream_t user = ctx->stream;
  TOSIMP_HIP(ctx, hipEventRecord(ctx->ev_in, user));
  TOSIMP_HIP(ctx, hipStreamWaitEvent(ctx->own_stream, ctx->ev_in, 0));
  ctx->stream = ctx->own_stream;
  rc = pcg_solve_impl(ctx, x, b, u, o, stats);
  ctx->stream = user;
  TOSIMP_HIP(ctx, hipEventRecord(ctx->ev_out, ctx->own_stream));
  TOSIMP_HIP(ctx, hipStreamWaitEvent(user, ctx->ev_out, 0));
  return rc;
}

// ===================================================================== SIMP pieces
int tosimp_sensitivity(tosimp_ctx* ctx, const double* x, const double* u, double* dc,
                       double* c_host) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && u && dc, TOSIMP_EINVAL, "null pointer");
  REQUIRE(!overlaps(dc, 8 * ctx->n_elem, u, 8 * ctx->n_dof), TOSIMP_EINVAL,
          "dc must not overlap u");
  REQUIRE(dc == x || !overlaps(dc, 8 * ctx->n_elem, x, 8 * ctx->n_elem), TOSIMP_EINVAL,
          "dc must be xphys itself or not overlap it");
  if ((rc = set_device(ctx))) return rc;
  TOSIMP_HIP(ctx, launch_sensitivity(ctx, x, u, dc));
  if (c_host) {
    Workspace& w = ctx->ws;
    SolverState* st = w.st + 2;
    TOSIMP_HIP(ctx, launch_dot64(ctx, w.f, u, ctx->n_dof, w.partials, st, 0));
    TOSIMP_HIP(ctx, hipMemcpyAsync(w.st_host + 2, st, sizeof(SolverState),
                                   hipMemcpyDeviceToHost, ctx->stream));
    TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *c_host = w.st_host[2].aux;
  }
  return TOSIMP_OK;
}

int tosimp_filter(tosimp_ctx* ctx, const double* in, double* out, int mode) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(in && out, TOSIMP_EINVAL, "null pointer");
  REQUIRE(!overlaps(in, 8 * ctx->n_elem, out, 8 * ctx->n_elem), TOSIMP_EINVAL,
          "in and out must not overlap");
  REQUIRE(mode == TOSIMP_FILTER_FORWARD || mode == TOSIMP_FILTER_ADJOINT, TOSIMP_EINVAL,
          "bad filter mode");
  if ((rc = set_device(ctx))) return rc;
  TOSIMP_HIP(ctx, launch_filter(ctx, in, out, mode));
  return TOSIMP_OK;
}

int tosimp_project(tosimp_ctx* ctx, const double* in, const double* g, double* out,
                   double beta, double eta) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(in && out, TOSIMP_EINVAL, "null pointer");
  REQUIRE(beta > 0 && std::isfinite(beta) && eta >= 0 && eta <= 1, TOSIMP_EINVAL,
          "need beta > 0 (finite) and 0 <= eta <= 1");
  const int64_t nb = 8 * ctx->n_elem;
  REQUIRE((out == in || !overlaps(out, nb, in, nb)) &&
              (!g || out == g || !overlaps(out, nb, g, nb)),
          TOSIMP_EINVAL, "out must be in, g, or not overlap them");
  if ((rc = set_device(ctx))) return rc;
  TOSIMP_HIP(ctx, launch_project(ctx, in, g, out, beta, eta));
  return TOSIMP_OK;
}

int tosimp_oc_update(tosimp_ctx* ctx, const double* x, const double* dc, double volfrac,
                     double move, double* x_new, double* xphys_new, double* change_host,
                     int* steps_host) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && dc && x_new && xphys_new, TOSIMP_EINVAL, "null pointer");
  {
    const int64_t nb = 8 * ctx->n_elem;
    REQUIRE(!overlaps(x_new, nb, x, nb) && !overlaps(x_new, nb, dc, nb) &&
                !overlaps(xphys_new, nb, x_new, nb),
            TOSIMP_EINVAL, "x_new must not overlap x, dc or xphys_new");
  }
  REQUIRE(volfrac > 0 && volfrac <= 1 && move > 0, TOSIMP_EINVAL, "bad volfrac/move");
  if ((rc = set_device(ctx))) return rc;
  return oc_run(ctx, x, dc, ctx->ws.dv, volfrac, move, 0.0, 0.0, x_new, xphys_new, nullptr,
                change_host, steps_host, nullptr);
}

}  // extern "C"

namespace {

// OC bisection on the host-polled device state: the density-filter volume dv^T x_new
// (beta <= 0) or the projected volume sum project(filter(x_new)) (beta > 0); writes
// x_new and its physical density (filtered, then projected when beta > 0), and returns
// the change, the step count and the volume at the final multiplier.  tmp: n_elem.
int oc_run(tosimp_ctx* ctx, const double* x, const double* dc, const double* dv,
           double volfrac, double move, double beta, double eta, double* x_new,
           double* xphys_new, double* tmp, double* change, int* steps, double* volume) {
  Workspace& w = ctx->ws;
  *w.oc_host = OcState{};
  w.oc_host->l1 = 0.0;
  w.oc_host->l2 = 1e9;
  w.oc_host->target = volfrac * (double)ctx->n_elem;
  TOSIMP_HIP(ctx, hipMemcpyAsync(w.oc, w.oc_host, sizeof(OcState), hipMemcpyHostToDevice,
                                 ctx->stream));
  for (int batch = 0; batch < 16; ++batch) {
    for (int i = 0; i < 16; ++i) {
      if (beta > 0)
        TOSIMP_HIP(ctx, launch_oc_step_projected(ctx, x, dc, dv, move, beta, eta, x_new, w.oc,
                                                 w.partials));
      else
        TOSIMP_HIP(ctx, launch_oc_step(ctx, x, dc, dv, move, w.oc, w.partials));
    }
    TOSIMP_HIP(ctx, hipMemcpyAsync(w.oc_host, w.oc, sizeof(OcState), hipMemcpyDeviceToHost,
                                   ctx->stream));
    TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (w.oc_host->done) break;
  }
  REQUIRE(w.oc_host->done, TOSIMP_EINVAL, "OC bisection did not terminate");
  TOSIMP_HIP(ctx, launch_oc_final(ctx, x, dc, dv, move, w.oc, x_new, w.partials));
  if (beta > 0) {
    TOSIMP_HIP(ctx, launch_filter(ctx, x_new, tmp, TOSIMP_FILTER_FORWARD));
    TOSIMP_HIP(ctx, launch_project(ctx, tmp, nullptr, xphys_new, beta, eta));
  } else {
    TOSIMP_HIP(ctx, launch_filter(ctx, x_new, xphys_new, TOSIMP_FILTER_FORWARD));
  }
  TOSIMP_HIP(ctx, hipMemcpyAsync(w.oc_host, w.oc, sizeof(OcState), hipMemcpyDeviceToHost,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (change) *change = w.oc_host->change;
  if (steps) *steps = w.oc_host->steps;
  if (volume) *volume = w.oc_host->vol;
  return TOSIMP_OK;
}

// After the solve of K(xphys) u = f: sensitivities chained to the design x (through the
// projection when beta > 0, then the adjoint filter), the volume gradient, and the OC
// update.  x_new / xphys_new receive the new design and its physical density.  Uses
// etmp slots 0..3 (slot 0 must hold filter(x) when beta > 0).
int design_update(tosimp_ctx* ctx, const double* x, const double* xphys, const double* u,
                  double volfrac, double move, double beta, double eta, double* x_new,
                  double* xphys_new, double* compliance, double* change, int* steps,
                  double* volume) {
  Workspace& w = ctx->ws;
  const size_t ne = (size_t)ctx->n_elem;
  double* xbar = w.etmp;
  double* b1 = w.etmp + ne;
  double* dcx = w.etmp + 2 * ne;
  double* dvx = w.etmp + 3 * ne;
  int rc = tosimp_sensitivity(ctx, xphys, u, b1, compliance);
  if (rc) return rc;
  const double* dv = w.dv;
  if (beta > 0) {
    TOSIMP_HIP(ctx, launch_project(ctx, xbar, b1, b1, beta, eta));  // dc / dxbar
    TOSIMP_HIP(ctx, launch_filter(ctx, b1, dcx, TOSIMP_FILTER_ADJOINT));
    TOSIMP_HIP(ctx, launch_fill64(ctx, b1, ctx->n_elem, 1.0));
    TOSIMP_HIP(ctx, launch_project(ctx, xbar, b1, b1, beta, eta));  // dxphys / dxbar
    TOSIMP_HIP(ctx, launch_filter(ctx, b1, dvx, TOSIMP_FILTER_ADJOINT));
    dv = dvx;
  } else {
    TOSIMP_HIP(ctx, launch_filter(ctx, b1, dcx, TOSIMP_FILTER_ADJOINT));
  }
  return oc_run(ctx, x, dcx, dv, volfrac, move, beta, eta, x_new, xphys_new, b1, change,
                steps, volume);
}

int check_beta_eta(tosimp_ctx* ctx, double beta, double eta) {
  REQUIRE(std::isfinite(beta) && (beta <= 0 || (eta >= 0 && eta <= 1)), TOSIMP_EINVAL,
          "projection needs a finite beta and 0 <= eta <= 1");
  return TOSIMP_OK;
}

// One continuation step of the SIMP-120 protocol: (penal, beta, move, rmin) of
// iteration `it` (1-based) from phases (5 values each: last iteration, penal, beta,
// move, rmin at the phase end or <= 0 to keep it).  Within a phase with a radius target
// the radius moves linearly from the previous phase's end value, reaching the target on
// the phase's last iteration; past the last phase its values hold.
void continuation(const double* ph, int nph, double rmin0, int it, double* penal,
                  double* beta, double* move, double* rmin) {
  int start = 1;
  double r_prev = rmin0;
  for (int k = 0; k < nph; ++k) {
    const int last = (int)ph[5 * k];
    const double r_end = ph[5 * k + 4] > 0 ? ph[5 * k + 4] : r_prev;
    if (it <= last || k == nph - 1) {
      *penal = ph[5 * k + 1];
      *beta = ph[5 * k + 2];
      *move = ph[5 * k + 3];
      if (it <= last) {
        const double frac = (double)(it - start + 1) / (double)(last - start + 1);
        *rmin = r_prev + (r_end - r_prev) * frac;
      } else {
        *rmin = r_end;
      }
      return;
    }
    start = last + 1;
    r_prev = r_end;
  }
}

// The paper's four phases (Sec. "Experimental Setup").
const double kPaperPhases[20] = {15, 1.5, 1.0, 0.20, 0.0,  40, 3.5, 4.0, 0.15, 1.35,
                                 65, 4.5, 16.0, 0.08, 1.25, 120, 4.5, 32.0, 0.05, 1.20};

}  // namespace

extern "C" {

int tosimp_simp_step(tosimp_ctx* ctx, double* x, double* xphys, double* u,
                     const tosimp_step_opts* o, tosimp_step_stats* stats) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && xphys && u && o, TOSIMP_EINVAL, "null pointer");
  REQUIRE(ctx->has_loads, TOSIMP_ESTATE, "no loads: call tosimp_set_loads first");
  if ((rc = check_beta_eta(ctx, o->beta, o->eta))) return rc;
  {
    const int64_t nb = 8 * ctx->n_elem;
    REQUIRE(!overlaps(x, nb, xphys, nb) && !overlaps(u, 8 * ctx->n_dof, x, nb) &&
                !overlaps(u, 8 * ctx->n_dof, xphys, nb),
            TOSIMP_EINVAL, "x, xphys and u must not overlap");
  }
  if ((rc = set_device(ctx))) return rc;
  Workspace& w = ctx->ws;
  const size_t ne = (size_t)ctx->n_elem;
  double* xn = w.etmp + 4 * ne;
  double* xpn = w.etmp + 5 * ne;
  tosimp_step_stats s{};
  if (o->beta > 0) TOSIMP_HIP(ctx, launch_filter(ctx, x, w.etmp, TOSIMP_FILTER_FORWARD));
  rc = tosimp_pcg_solve(ctx, xphys, w.f, u, &o->solve, &s.solve);
  if (rc < 0) return rc;
  TOSIMP_HIP(ctx, launch_grayness(ctx, xphys, w.partials, &w.st[2].aux));
  TOSIMP_HIP(ctx, hipMemcpyAsync(w.st_host + 2, w.st + 2, sizeof(SolverState),
                                 hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  s.grayness = w.st_host[2].aux;
  double vol = 0;
  int rc2 = design_update(ctx, x, xphys, u, o->volfrac, o->move, o->beta, o->eta, xn, xpn,
                          &s.compliance, &s.change, &s.bisection_steps, &vol);
  if (rc2) return rc2;
  s.volume = vol / (double)ne;
  TOSIMP_HIP(ctx, hipMemcpyAsync(x, xn, ne * 8, hipMemcpyDeviceToDevice, ctx->stream));
  TOSIMP_HIP(ctx, hipMemcpyAsync(xphys, xpn, ne * 8, hipMemcpyDeviceToDevice, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (stats) *stats = s;
  return rc;
}

int tosimp_grayness(tosimp_ctx* ctx, const double* rho, double* g_host) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(rho && g_host, TOSIMP_EINVAL, "null pointer");
  if ((rc = set_device(ctx))) return rc;
  Workspace& w = ctx->ws;
  TOSIMP_HIP(ctx, launch_grayness(ctx, rho, w.partials, &w.st[2].aux));
  TOSIMP_HIP(ctx, hipMemcpyAsync(w.st_host + 2, w.st + 2, sizeof(SolverState),
                                 hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *g_host = w.st_host[2].aux;
  return TOSIMP_OK;
}

int tosimp_simp_protocol(tosimp_ctx* ctx, double* x, double* x_sel, double* xphys, double* u,
                         const tosimp_protocol_opts* o, tosimp_protocol_record* rec,
                         int* it_selected, double* c_selected) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && x_sel && xphys && u && o && rec, TOSIMP_EINVAL, "null pointer");
  REQUIRE(ctx->has_loads, TOSIMP_ESTATE, "no loads: call tosimp_set_loads first");
  REQUIRE(o->iters >= 1 && o->volfrac > 0 && o->volfrac <= 1 && o->restart_factor > 0,
          TOSIMP_EINVAL, "bad iters, volfrac or restart_factor");
  REQUIRE(o->nphases >= 0 && (o->nphases == 0 || o->phases), TOSIMP_EINVAL, "bad phases");
  if ((rc = check_beta_eta(ctx, 1.0, o->eta))) return rc;
  {
    const int64_t nb = 8 * ctx->n_elem, nu = 8 * ctx->n_dof;
    REQUIRE(!overlaps(x, nb, x_sel, nb) && !overlaps(x, nb, xphys, nb) &&
                !overlaps(x_sel, nb, xphys, nb) && !overlaps(u, nu, x, nb) &&
                !overlaps(u, nu, x_sel, nb) && !overlaps(u, nu, xphys, nb),
            TOSIMP_EINVAL, "x, x_sel, xphys and u must not overlap");
  }
  const double* ph = o->nphases ? o->phases : kPaperPhases;
  const int nph = o->nphases ? o->nphases : 4;
  for (int k = 0; k < nph; ++k)
    REQUIRE(ph[5 * k] >= 1 && (k == 0 || ph[5 * k] > ph[5 * (k - 1)]) && ph[5 * k + 1] >= 1 &&
                ph[5 * k + 2] > 0 && ph[5 * k + 3] > 0 && ph[5 * k + 4] <= kMaxFilterR + 1,
            TOSIMP_EINVAL, "bad continuation phase");
  if ((rc = set_device(ctx))) return rc;
  Workspace& w = ctx->ws;
  const size_t ne = (size_t)ctx->n_elem;
  double* xn = w.etmp + 4 * ne;
  double* xpn = w.etmp + 5 * ne;
  const double rmin0 = ctx->rmin, penal0 = ctx->penal;
  bool have_sel = false;
  double csel = 0;
  int itsel = 0;
  for (int it = 1; it <= o->iters; ++it) {
    tosimp_protocol_record r{};
    r.it = it;
    continuation(ph, nph, rmin0, it, &r.penal, &r.beta, &r.move, &r.rmin);
    if ((rc = tosimp_set_params(ctx, r.penal, r.rmin))) return rc;
    TOSIMP_HIP(ctx, launch_filter(ctx, x, w.etmp, TOSIMP_FILTER_FORWARD));
    TOSIMP_HIP(ctx, launch_project(ctx, w.etmp, nullptr, xphys, r.beta, o->eta));
    tosimp_solve_stats ss{};
    rc = tosimp_pcg_solve(ctx, xphys, w.f, u, &o->solve, &ss);
    if (rc < 0) return rc;
    r.cg_iterations = ss.iterations;
    r.compliance = ss.b_dot_u;
    if ((rc = tosimp_grayness(ctx, xphys, &r.grayness))) return rc;
    if (have_sel && r.compliance > o->restart_factor * csel) {
      // restart from the selected design field
      r.restart = 1;
      TOSIMP_HIP(ctx, hipMemcpyAsync(x, x_sel, ne * 8, hipMemcpyDeviceToDevice, ctx->stream));
      rec[it - 1] = r;
      continue;
    }
    if (r.penal >= o->eligible_penal && r.grayness < o->eligible_gray) {
      r.eligible = 1;
      if (!have_sel || r.compliance < csel) {
        have_sel = true;
        csel = r.compliance;
        itsel = it;
        r.selected = 1;
        TOSIMP_HIP(ctx, hipMemcpyAsync(x_sel, x, ne * 8, hipMemcpyDeviceToDevice, ctx->stream));
      }
    }
    double c = 0, vol = 0;
    if ((rc = design_update(ctx, x, xphys, u, o->volfrac, r.move, r.beta, o->eta, xn, xpn, &c,
                            &r.change, &r.bisection_steps, &vol)))
      return rc;
    TOSIMP_HIP(ctx, hipMemcpyAsync(x, xn, ne * 8, hipMemcpyDeviceToDevice, ctx->stream));
    rec[it - 1] = r;
  }
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if ((rc = tosimp_set_params(ctx, penal0, rmin0))) return rc;
  if (it_selected) *it_selected = have_sel ? itsel : 0;
  if (c_selected) *c_selected = have_sel ? csel : 0.0;
  return TOSIMP_OK;
}

// ===================================================================== Lanczos
}  // extern "C"

namespace {

// Device state of a Lanczos run: the current and previous basis vectors (swapped every
// step), the optional Jacobi scaling, and the device arrays of alpha and beta.
struct LanczosRun {
  const double* x = nullptr;
  double* q = nullptr;
  double* qprev = nullptr;
  double* s_node = nullptr;
  double* dal = nullptr;  // alpha[0..k)
  double* dbe = nullptr;  // beta[-1..k): dbe[0] = ||v0||, dbe[j + 1] = beta_j
};

// Sets up a run of at most k steps from v0 (workspace vectors w.p, w.q as the basis,
// w.w for K q, w.r for the scaled input; v0 is read before the first step).
// coeffs: caller-provided device storage of 2 (k + 1) doubles for alpha and beta, or
// nullptr to use (and grow) the workspace's.
int lanczos_begin(tosimp_ctx* ctx, const double* x, const double* v0, int k, int jacobi,
                  LanczosRun* L, double* coeffs = nullptr) {
  Workspace& w = ctx->ws;
  if (coeffs) {
    L->dal = coeffs;
    L->dbe = coeffs + (k + 1);
  } else {
    if (w.lanczos_cap < k + 1) {
      if (w.lanczos) TOSIMP_HIP(ctx, hipFree(w.lanczos));
      w.lanczos = nullptr;
      w.lanczos_cap = 0;
      TOSIMP_HIP(ctx, hipMalloc((void**)&w.lanczos, sizeof(double) * 2 * (size_t)(k + 1)));
      w.lanczos_cap = k + 1;
    }
    L->dal = w.lanczos;
    L->dbe = w.lanczos + w.lanczos_cap;
  }
  L->x = x;
  L->s_node = nullptr;
  SolverState* st = w.st + 2;
  if (jacobi) {
    // sqrt(dinv) per node, in place (every solve recomputes w.dinv at its start)
    TOSIMP_HIP(ctx, launch_diag_inv(ctx, x, w.dinv, nullptr));
    L->s_node = w.dinv;
    TOSIMP_HIP(ctx, launch_sqrt_node(ctx, w.dinv, L->s_node));
  }
  L->q = w.p;
  L->qprev = w.q;
  // q0 = v0 / ||v0||
  TOSIMP_HIP(ctx, launch_dot64(ctx, v0, v0, ctx->n_dof, w.partials, st, 1));
  TOSIMP_HIP(ctx, launch_sqrt_scalar(ctx, st, L->dbe));
  TOSIMP_HIP(ctx, launch_lanczos_normalize(ctx, v0, L->dbe, L->q));
  return TOSIMP_OK;
}

// Steps j0 .. j1-1 (asynchronous).
int lanczos_steps(tosimp_ctx* ctx, LanczosRun* L, int j0, int j1) {
  Workspace& w = ctx->ws;
  SolverState* st = w.st + 2;
  double *wv = w.w, *tmp = w.r;
  for (int j = j0; j < j1; ++j) {
    const double* in = L->q;
    if (L->s_node) {
      TOSIMP_HIP(ctx, launch_node_scale(ctx, L->s_node, L->q, tmp));
      in = tmp;
    }
    TOSIMP_HIP(ctx, kv_launch(ctx, TOSIMP_PREC_FP64, TOSIMP_F64, L->x, in, wv, w.partials, st,
                              L->dal + j, 2, false));
    TOSIMP_HIP(ctx, launch_lanczos_update(ctx, wv, L->q, j > 0 ? L->qprev : nullptr,
                                          L->dal + j, j > 0 ? L->dbe + j : nullptr, L->s_node,
                                          w.partials + kMaxPartials, L->dbe + j + 1));
    TOSIMP_HIP(ctx, launch_lanczos_normalize(ctx, wv, L->dbe + j + 1, L->qprev));
    std::swap(L->q, L->qprev);
  }
  return TOSIMP_OK;
}

// Copies the coefficients of the first k steps to the host and returns in *m the order
// of the tridiagonal (m < k only on an invariant subspace: the first beta <= 0).
int lanczos_fetch(tosimp_ctx* ctx, const LanczosRun& L, int k, std::vector<double>& a,
                  std::vector<double>& b, int* m) {
  std::vector<double> hb(k + 1);
  a.resize(k);
  TOSIMP_HIP(ctx, hipMemcpyAsync(a.data(), L.dal, sizeof(double) * k, hipMemcpyDeviceToHost,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipMemcpyAsync(hb.data(), L.dbe, sizeof(double) * (k + 1),
                                 hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int mm = k;
  for (int j = 0; j < k - 1; ++j)
    if (!(hb[j + 1] > 0.0)) {
      mm = j + 1;
      break;
    }
  b.assign(hb.begin() + 1, hb.begin() + 1 + std::max(mm - 1, 0));
  a.resize(mm);
  *m = mm;
  return TOSIMP_OK;
}

// Lanczos with the stopping rule (see tosimp_kappa).
int kappa_run(tosimp_ctx* ctx, const double* x, const double* v0, int kmax, int jacobi,
              double rtol, int window, double* lmin, double* lmax, int* steps, int* converged) {
  LanczosRun L;
  int rc = lanczos_begin(ctx, x, v0, kmax, jacobi, &L);
  if (rc) return rc;
  std::vector<double> a, b;
  double prev = 0.0;
  bool have_prev = false;
  int j = 0;
  for (;;) {
    const int j1 = std::min(kmax, j + window);
    if ((rc = lanczos_steps(ctx, &L, j, j1))) return rc;
    j = j1;
    int m = 0;
    if ((rc = lanczos_fetch(ctx, L, j, a, b, &m))) return rc;
    double lo = 0, hi = 0;
    tosimp_tridiag_extremes(a.data(), b.empty() ? nullptr : b.data(), m, &lo, &hi);
    if (m < j) {  // invariant subspace: the extremes of T_m are exact
      *lmin = lo; *lmax = hi; *steps = m; *converged = 1;
      return TOSIMP_OK;
    }
    if (j % window == 0 && have_prev && std::fabs(lo - prev) <= rtol * std::fabs(lo)) {
      *lmin = lo; *lmax = hi; *steps = j; *converged = 1;
      return TOSIMP_OK;
    }
    if (j >= kmax) {
      *lmin = lo; *lmax = hi; *steps = j; *converged = 0;
      return TOSIMP_OK;
    }
    prev = lo;
    have_prev = true;
  }
}

}  // namespace

extern "C" {

int tosimp_lanczos(tosimp_ctx* ctx, const double* x, const double* v0, int k, int jacobi,
                   double* alpha_host, double* beta_host, int* steps_host) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && v0 && alpha_host && beta_host && k >= 1, TOSIMP_EINVAL, "bad arguments");
  if ((rc = set_device(ctx))) return rc;
  LanczosRun L;
  if ((rc = lanczos_begin(ctx, x, v0, k, jacobi, &L))) return rc;
  if ((rc = lanczos_steps(ctx, &L, 0, k))) return rc;
  std::vector<double> a, b;
  int m = 0;
  if ((rc = lanczos_fetch(ctx, L, k, a, b, &m))) return rc;
  for (int j = 0; j < m; ++j) alpha_host[j] = a[j];
  for (int j = 0; j + 1 < m; ++j) beta_host[j] = b[j];
  if (steps_host) *steps_host = m;
  return TOSIMP_OK;
}

int tosimp_lanczos_noalloc(tosimp_ctx* ctx, const double* x, const double* v0, int k,
                           int jacobi, double* alpha_host, double* beta_host,
                           int* steps_host) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && v0 && alpha_host && beta_host && k >= 1, TOSIMP_EINVAL, "bad arguments");
  REQUIRE(k <= kLanczosScratchSteps, TOSIMP_EINVAL,
          "tosimp_lanczos_noalloc: k = " + std::to_string(k) + " exceeds the " +
              std::to_string(kLanczosScratchSteps) + " steps of its fixed device storage");
  REQUIRE(ctx->scratch, TOSIMP_ESTATE, "no device address for the Lanczos storage");
  if ((rc = set_device(ctx))) return rc;
  LanczosRun L;
  if ((rc = lanczos_begin(ctx, x, v0, k, jacobi, &L, ctx->scratch))) return rc;
  if ((rc = lanczos_steps(ctx, &L, 0, k))) return rc;
  // beta_0 .. beta_{k-2} straight into the caller's array, then the order m (the first
  // beta <= 0 ends an invariant subspace) and alpha_0 .. alpha_{m-1}.
  if (k > 1)
    TOSIMP_HIP(ctx, hipMemcpyAsync(beta_host, L.dbe + 1, sizeof(double) * (k - 1),
                                   hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int m = k;
  for (int j = 0; j < k - 1; ++j)
    if (!(beta_host[j] > 0.0)) {
      m = j + 1;
      break;
    }
  TOSIMP_HIP(ctx, hipMemcpyAsync(alpha_host, L.dal, sizeof(double) * m, hipMemcpyDeviceToHost,
                                 ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (steps_host) *steps_host = m;
  return TOSIMP_OK;
}

int tosimp_kappa(tosimp_ctx* ctx, const double* x, const double* v0, int kmax, int jacobi,
                 double rtol, int window, double* lmin, double* lmax, int* steps,
                 int* converged) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && v0 && lmin && lmax && steps && converged, TOSIMP_EINVAL, "null pointer");
  REQUIRE(kmax >= 1 && window >= 1 && rtol > 0, TOSIMP_EINVAL, "need kmax, window >= 1, rtol > 0");
  if ((rc = set_device(ctx))) return rc;
  return kappa_run(ctx, x, v0, kmax, jacobi, rtol, window, lmin, lmax, steps, converged);
}

int tosimp_mg_apply(tosimp_ctx* ctx, const double* x, const void* r, void* z, int prec,
                    int degree, double alpha) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(x && r && z, TOSIMP_EINVAL, "null pointer");
  REQUIRE(prec == TOSIMP_PREC_FP64 || prec == TOSIMP_PREC_FP32, TOSIMP_EINVAL,
          "multigrid precision must be FP64 or FP32");
  const int64_t vb = ctx->n_dof * (prec == TOSIMP_PREC_FP64 ? 8 : 4);
  REQUIRE(!overlaps(z, vb, r, vb) && !overlaps(z, vb, x, 8 * ctx->n_elem), TOSIMP_EINVAL,
          "z must not overlap r or xphys");
  if ((rc = set_device(ctx))) return rc;
  if ((rc = mg_prepare(ctx, x, &degree, &alpha))) return rc;
  if (prec == TOSIMP_PREC_FP64)
    return mg_apply<double>(ctx, (const double*)r, (double*)z, degree, alpha, nullptr);
  return mg_apply<float>(ctx, (const float*)r, (float*)z, degree, alpha, nullptr);
}

int tosimp_mg_levels(tosimp_ctx* ctx, int* dims_host, int cap) {
  int rc = check_ready(ctx);
  if (rc) return rc;
  REQUIRE(dims_host && cap >= 1, TOSIMP_EINVAL, "bad arguments");
  if ((rc = set_device(ctx))) return rc;
  return mg_levels(ctx, dims_host, cap);
}

// Number of eigenvalues of the tridiagonal (a, b) smaller than s (Sturm count).
static int sturm_count(const double* a, const double* b, int m, double s) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < m; ++i) {
    const double b2 = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - s) - (i > 0 ? b2 / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0) ++cnt;
  }
  return cnt;
}

int tosimp_tridiag_extremes(const double* a, const double* b, int m, double* lmin,
                            double* lmax) {
  if (!a || m < 1 || (m > 1 && !b) || !lmin || !lmax) return TOSIMP_EINVAL;
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto kth = [&](int kk) {  // kk-th smallest eigenvalue (0-based)
    double l = lo, h = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (l + h);
      if (mid <= l || mid >= h) break;
      if (sturm_count(a, b, m, mid) > kk) h = mid;
      else l = mid;
    }
    return 0.5 * (l + h);
  };
  *lmin = kth(0);
  *lmax = kth(m - 1);
  return TOSIMP_OK;
}

}  // extern "C"
