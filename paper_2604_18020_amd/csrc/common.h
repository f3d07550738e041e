// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "tosimp.h"

namespace tosimp {

// ---------------------------------------------------------------------------------
// Element stiffness in the tensor Hadamard basis.
//
// Per axis the basis is {v0 + v1, v1 - v0}; the 8 modes of an element are the tensor
// products, mode m = mx + 2 my + 4 mz (bit set = difference along that axis).  With H
// the resulting 24x24 transform (acting on each displacement component), H^T H = 8 I
// per component pair, so K_E = H^T S H / 64 with S = H K_E H^T.  On a cube S has 45
// non-zeros in eight distinct values, grouped by the strain states they represent:
//   normal block   {(1,x),(2,y),(4,z)}: diagonal ad + ao, off-diagonal ao
//   shear pairs    {(1,y),(2,x)}, {(1,z),(4,x)}, {(2,z),(4,y)}: all four entries cs
//   bending pairs  {(3,x),(6,z)}, {(3,y),(5,z)}, {(5,x),(6,y)}: diagonal bd, off bo
//   twist block    {(3,z),(5,y),(6,x)}: diagonal cd + co, off-diagonal co
//   hourglass      (7,c): diagonal hg
// Constants stored here already include the 1/64 normalisation and the edge length.
// ---------------------------------------------------------------------------------
struct HadConsts {
  double ad, ao, cs, bd, bo, cd, co, hg;
};

// Filter stencil (cone weights on the integer offset cube [-R, R]^3).
constexpr int kMaxFilterR = 3;
constexpr int kMaxFilterTaps = (2 * kMaxFilterR + 1) * (2 * kMaxFilterR + 1) * (2 * kMaxFilterR + 1);

// Device-side scalar state of an iterative solve; one instance per solver level.
struct SolverState {
  double rz;      // <r, z> of the current iterate
  double alpha;   // step length
  double beta;    // direction update coefficient
  double rr;      // ||r||^2
  double bb;      // ||b||^2
  double tol2;    // tol^2 * ||b||^2
  double pq;      // <p, K p>
  double aux;     // scratch scalar (tol^2 on entry; FCG: fallback flag)
  double s_rn;    // two-stage preconditioner: <r, n> and <n, K n>
  double s_nkn;
  int iter;       // completed iterations
  int maxit;      // iteration cap
  int done;       // 0 running, 1 converged, 2 cap, 3 breakdown
  int nfallback;  // flexible CG: preconditioner fallbacks taken
  int upend;      // Jacobi-PCG: the last iteration's u += alpha p is still to be applied
  double rmin;    // flexible CG stagnation guard: smallest ||r||^2 so far,
  int kmin;       //   the iteration that reached it,
  int stall;      //   and the iterations without a new minimum that stop the solve (0: off)
};

// Device-side state of the OC bisection.
struct OcState {
  double l1, l2, lmid, target, vol, change;
  int steps, done;
};

constexpr int kRedBlocks = 1024;   // fixed grid of the vector kernels (deterministic)
constexpr int kRedThreads = 256;
constexpr int kMaxPartials = 65536;

// Workspace owned by a context (device pointers unless noted).
struct Workspace {
  uint8_t* mask = nullptr;     // n_node: bit c set = DOF 3n+c fixed
  double* f = nullptr;         // n_dof load vector
  double* Hs = nullptr;        // n_elem filter row sums
  double* Hsinv = nullptr;     // n_elem 1 / Hs
  double* dv = nullptr;        // n_elem H(1/Hs)
  double* fw = nullptr;        // filter weights, (2R+1)^3
  double* dinv = nullptr;      // n_node inverse Jacobi diagonal (FP64)
  float* dinv32 = nullptr;     // n_node inverse Jacobi diagonal (FP32)
  double* r = nullptr;         // FP64 vectors, n_dof each
  double* p = nullptr;
  double* q = nullptr;
  double* w = nullptr;
  float* r32 = nullptr;        // FP32 vectors, n_dof each
  float* p32 = nullptr;
  float* q32 = nullptr;
  float* e32 = nullptr;
  float* z32 = nullptr;
  float* x32 = nullptr;        // n_elem FP32 density copy
  double* etmp = nullptr;      // n_elem scratch (x 6)
  double* partials = nullptr;  // 2 kMaxPartials + kv_part_cap
  int64_t kv_part_cap = 0;     // operator tiles a fused dot may use
  uint16_t* ke_mfma = nullptr; // K_E in the MFMA A-operand layout: [bf16|f16][2][64][8]
  double* lanczos = nullptr;   // 2 x (kmax) alpha/beta on device
  int lanczos_cap = 0;
  SolverState* st = nullptr;   // 2 solver states (outer / inner)
  OcState* oc = nullptr;
  SolverState* st_host = nullptr;  // pinned host mirror
  OcState* oc_host = nullptr;
};

}  // namespace tosimp

struct tosimp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;     // the caller's stream
  hipStream_t own_stream = nullptr; // the solver's stream (created on first use)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::string err;
  bool has_mesh = false, has_bcs = false, has_loads = false;
  int nx = 0, ny = 0, nz = 0;
  int64_t n_elem = 0, n_node = 0, n_dof = 0;
  double h = 1, E0 = 1, Emin = 1e-9, nu = 0.3, penal = 3, rmin = 1.5;
  double KE[576];              // host FP64 element stiffness (edge h)
  double kd = 0;               // common diagonal entry of K_E
  tosimp::HadConsts hc{};
  int fR = 0;                  // filter half-width
  double fw_host[tosimp::kMaxFilterTaps];
  tosimp::Workspace ws;
  void* nn = nullptr;          // learned preconditioner state (nn.hip)
  double* scratch = nullptr;   // device address of the allocation-free Lanczos storage
  void* mg = nullptr;          // multigrid hierarchy (mg.hip), sized for the mesh
  // conditioning estimate of the Jacobi-scaled operator at uniform density (0: not yet
  // computed for the current mesh and boundary conditions)
  double kappa_uniform = 0;
  int kappa_converged = 0, kappa_steps = 0;
};

// ------------------------------------------------------------------ error plumbing
int tosimp_fail(tosimp_ctx* ctx, int code, const std::string& msg);
#define TOSIMP_HIP(ctx, call)                                                          \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return tosimp_fail(ctx, TOSIMP_EHIP,                                             \
                         std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

// ----------------------------------------------------------- kernel launch wrappers
namespace tosimp {

// Operator kernels (kv.hip, kv_mfma.hip).  kv_launch: y = K_c(x) v with an optional
// fused <v, y> finished into st (FIN_ALPHA) or *out (FIN_SCALAR); guarded launches
// return at once when st->done is set; premasked: the caller guarantees v = 0 on fixed
// DOFs (then the plane BC bytes are not read).
hipError_t kv_launch(const tosimp_ctx* c, int prec, int xdtype, const void* x,
                     const void* v, void* y, double* partials, SolverState* st,
                     double* out, int fin, bool guarded, bool premasked = false);
// Atomic-scatter alternatives (kv_atomic.hip); variant is a TOSIMP_SCATTER_* flag.
hipError_t kv_atomic_launch(const tosimp_ctx* c, int prec, int xdtype, const void* x,
                            const void* v, void* y, int variant);
hipError_t kv_mfma_launch(const tosimp_ctx* c, int prec, int xdtype, const void* x,
                          const float* v, float* y, SolverState* st, bool guarded);
hipError_t launch_apply_K(const tosimp_ctx* c, int prec, int xdtype, const void* x,
                          const void* v, void* y, double* dot_partials, int* nblocks);
int kv_num_blocks(const tosimp_ctx* c);
hipError_t launch_diag_inv(const tosimp_ctx* c, const double* xphys, double* dinv64,
                           float* dinv32);
hipError_t launch_diag_inv32(const tosimp_ctx* c, const float* x32, float* dinv32);
hipError_t launch_diag_full(const tosimp_ctx* c, int xdtype, const void* x, int dtype,
                            void* d);
// Multigrid levels: operator with element moduli given and K_E scaled by kscale (v zero
// on fixed DOFs), and the per-node inverse Jacobi diagonal of such a level.  With ch
// (mode 1 / 2) the launch is a whole Chebyshev smoothing step: t = K v stays in
// registers, dd <- c2 (b - t) dinv (mode 1) or c1 dd + c2 (b - t) dinv (mode 2), and y
// receives the new iterate v + dd (y, v and dd distinct).  Mode 3 is the first two steps
// from a zero iterate in one pass: v must be b, the operator acts on x1 = c0 b dinv
// (formed while staging), and the update is mode 2's with dd = x1.
struct KvCheb {
  int mode = 0;
  const void* b = nullptr;
  void* dd = nullptr;
  const void* dinv = nullptr;  // per node, of the operator's type
  double c0 = 0, c1 = 0, c2 = 0;
  // Modes 1 and 2: with dot set the pass also stores, per operator tile, the FP64 sum of
  // b . y over the tile's owned nodes into dot[0..tiles) and the tile count into
  // *dot_tiles (no finalize is launched).
  double* dot = nullptr;
  int* dot_tiles = nullptr;
};
hipError_t kv_level_launch(const tosimp_ctx* c, int prec, const void* E, const void* v,
                           void* y, int nx, int ny, int nz, const uint8_t* mask,
                           double kscale, const SolverState* st = nullptr,
                           const KvCheb* ch = nullptr);

// Geometric multigrid (mg.hip).  mg_prepare: hierarchy for density x (FP64) with the
// Chebyshev degree and alpha (0 = defaults 2 and 20, validated); mg_apply: z = V(r) on the
// fine level (with dot_part, <r, z> as per-tile partials of the last finest-level pass,
// *dot_tiles of them, 0 if the V-cycle had no such pass); mg_pcg: CG preconditioned by V(.) (slot: solver-state slot); mg_levels:
// level dims into dims[3 l + {0,1,2}], returns the level count (or a negative status);
// mg_release: frees the hierarchy (mesh change, destroy).
struct MgPcgResult {
  int iters = 0, done = 0;
  double rr = 0, bb = 0;
};
int mg_prepare(tosimp_ctx* ctx, const double* x, int* degree, double* alpha);
template <typename T>
int mg_apply(tosimp_ctx* ctx, const T* r, T* z, int degree, double alpha, const SolverState* st,
             double* dot_part = nullptr, int* dot_tiles = nullptr);
template <typename T>
int mg_pcg(tosimp_ctx* ctx, const void* x, const T* b, T* u, T* r, T* z, T* p, T* q,
           int slot, double tol, int maxit, int check_every, bool zero_guess, int degree,
           double alpha, bool graphs, MgPcgResult* res);
int mg_levels(tosimp_ctx* ctx, int* dims, int cap);
void mg_release(tosimp_ctx* ctx);
hipError_t launch_diag_level(const tosimp_ctx* c, const double* E, int nx, int ny, int nz,
                             double kscale, double* dinv64, float* dinv32);

// Solver kernels (vec.hip).
hipError_t launch_finalize_dot(const tosimp_ctx* c, const double* partials, int n,
                               SolverState* st, int what);
template <typename T>
hipError_t launch_pcg_init(const tosimp_ctx* c, const T* b, const T* Ku, T* r, T* p,
                           const void* dinv, SolverState* st, double* partials, int use_Ku);
// u == nullptr: u is left to launch_pcg_direction (and launch_pcg_finish).
template <typename T>
hipError_t launch_pcg_update(const tosimp_ctx* c, T* u, T* r, const T* p, const T* q,
                             const void* dinv, SolverState* st, double* partials);
template <typename T>
hipError_t launch_pcg_direction(const tosimp_ctx* c, const T* r, T* p, T* u, const void* dinv,
                                SolverState* st);
template <typename T>
hipError_t launch_pcg_finish(const tosimp_ctx* c, T* u, const T* p, SolverState* st);
hipError_t launch_mask_vec(const tosimp_ctx* c, double* v);
hipError_t launch_residual64(const tosimp_ctx* c, const double* b, const double* Ku,
                             double* r, double* partials, SolverState* st);
hipError_t launch_scale_to32(const tosimp_ctx* c, const double* r, double inv_s, float* r32);
hipError_t launch_axpy_from32(const tosimp_ctx* c, double* u, double s, const float* e);
hipError_t launch_copy_cast_x(const tosimp_ctx* c, const double* x, float* x32);
hipError_t launch_cast32(const tosimp_ctx* c, const double* x, float* y, int64_t n);
hipError_t launch_diff_cast32(const tosimp_ctx* c, const double* a, const double* b, float* y,
                              int64_t n);
hipError_t launch_fill_zero(const tosimp_ctx* c, void* p, int64_t bytes);
hipError_t launch_fill64(const tosimp_ctx* c, double* p, int64_t n, double v);
hipError_t launch_dot64(const tosimp_ctx* c, const double* a, const double* b, int64_t n,
                        double* partials, SolverState* st, int what);
hipError_t launch_lanczos_update(const tosimp_ctx* c, double* w, const double* q,
                                 const double* qprev, const double* alpha_j,
                                 const double* beta_jm1, const double* scale_node,
                                 double* partials, double* beta_j);
hipError_t launch_lanczos_normalize(const tosimp_ctx* c, const double* w, const double* beta_j,
                                    double* qnext);
hipError_t launch_node_scale(const tosimp_ctx* c, const double* s_node, const double* v,
                             double* out);
hipError_t launch_sqrt_node(const tosimp_ctx* c, const double* dinv, double* out);
hipError_t launch_alpha_from_dot32(const tosimp_ctx* c, const float* p, const float* q,
                                   double* partials, SolverState* st);
hipError_t launch_sqrt_scalar(const tosimp_ctx* c, const SolverState* st, double* out);

// Learned preconditioner (nn.hip).  nn_fcg_solve: flexible CG on K_c(x32) e = b32 with
// the network as preconditioner (Jacobi fallback), FP32 vectors, zero initial guess.
void nn_release(tosimp_ctx* ctx);
// stall > 0: stop with *done = 4 once ||r|| has made no new minimum for stall iterations.
int nn_fcg_solve(tosimp_ctx* ctx, int prec, const float* x32, const float* b32, float* e32,
                 double tol, int maxit, int check_every, int window, int stall, int* iters,
                 int* fallbacks, int* done);

// SIMP kernels (topopt.hip).
hipError_t launch_sensitivity(const tosimp_ctx* c, const double* xphys, const double* u,
                              double* dc);
// mode: TOSIMP_FILTER_FORWARD / _ADJOINT with the context's row sums.
hipError_t launch_filter(const tosimp_ctx* c, const double* in, double* out, int mode);
hipError_t launch_reciprocal(const tosimp_ctx* c, const double* in, double* out, int64_t n);
hipError_t launch_filter_rowsum(const tosimp_ctx* c, double* Hs);
hipError_t launch_project(const tosimp_ctx* c, const double* in, const double* g, double* out,
                          double beta, double eta);
hipError_t launch_oc_init(const tosimp_ctx* c, OcState* oc, double target);
hipError_t launch_oc_step(const tosimp_ctx* c, const double* x, const double* dc,
                          const double* dv, double move, OcState* oc, double* partials);
hipError_t launch_oc_final(const tosimp_ctx* c, const double* x, const double* dc,
                           const double* dv, double move, OcState* oc, double* xnew,
                           double* partials);
hipError_t launch_oc_step_projected(const tosimp_ctx* c, const double* x, const double* dc,
                                    const double* dv, double move, double beta, double eta,
                                    double* xn, OcState* oc, double* partials);
hipError_t launch_grayness(const tosimp_ctx* c, const double* rho, double* partials,
                           double* out);

}  // namespace tosimp
