/*
 * tosimp.h -- C ABI of the MI355X (gfx950) matrix-free 3D SIMP library.
 *
 * Problem (paper Sec. "Three-Dimensional SIMP Topology Optimization", Eq. tomin):
 * minimise the compliance f^T u subject to K(x) u = f and a volume fraction, on a
 * structured grid of nx*ny*nz cubic trilinear (Q1) hexahedra of edge h.
 *
 * Conventions shared by every entry point
 *   Numbering   node (i,j,k) has id n = i + (nx+1)*(j + (ny+1)*k); DOF 3*n + c
 *               (c = 0,1,2 for x,y,z, interleaved); element (ex,ey,ez) has id
 *               ex + nx*(ey + ny*ez); local node a = ax + 2*ay + 4*az.
 *   Operator    K_c = P K P + (I - P), P the diagonal free-DOF mask: fixed rows and
 *               columns are identity, so CG on K_c solves the free block exactly.
 *   Memory      every array argument named *_dev is caller-owned device memory on
 *               the context's device (contiguous, no strides); *_host is host memory.
 *               The library never frees caller memory.  It owns only a workspace it
 *               allocates in tosimp_set_mesh (and tosimp_nn_create) and frees on
 *               re-mesh or destroy.
 *   Streams     work is enqueued on the context's stream (tosimp_set_stream).  Entry
 *               points that return host scalars synchronise that stream; the others
 *               are asynchronous.
 *   Errors      every entry point returns an int status: 0 = OK, > 0 = informational
 *               with a valid result, < 0 = error with outputs unspecified; the text of
 *               the last error is tosimp_last_error(ctx).  Nothing aborts and no C++
 *               exception crosses the ABI.  A context is not thread-safe.
 */
#ifndef TOSIMP_H
#define TOSIMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------ */
#define TOSIMP_OK 0
#define TOSIMP_NOT_CONVERGED 1   /* iteration cap hit; the iterate is valid          */
#define TOSIMP_FALLBACK_USED 2   /* a preconditioner fallback was taken              */
#define TOSIMP_EINVAL (-1)       /* bad argument (null pointer, size, enum, layout)  */
#define TOSIMP_ESTATE (-2)       /* call order violated (e.g. no mesh set)           */
#define TOSIMP_EHIP (-3)         /* HIP runtime error                                 */
#define TOSIMP_EBREAKDOWN (-4)   /* CG breakdown: p^T K p <= 0 or non-finite         */
#define TOSIMP_EPRECISION (-5)   /* precision refused by the conditioning rule       */
#define TOSIMP_ENOMEM (-6)       /* workspace allocation failed                       */

/* ---- element types and operator precisions ------------------------------------ */
#define TOSIMP_F64 0
#define TOSIMP_F32 1

#define TOSIMP_PREC_FP64 0       /* FP64 storage and arithmetic                       */
#define TOSIMP_PREC_FP32 1       /* FP32 storage and arithmetic                       */
#define TOSIMP_PREC_BF16_MFMA 2  /* FP32 storage, BF16 MFMA contraction, FP32 acc.    */
#define TOSIMP_PREC_FP16_MFMA 3  /* FP32 storage, FP16 MFMA contraction, FP32 acc.    */
/* Flag OR-ed into the precision of tosimp_apply_K: the caller guarantees v = 0 on every
 * fixed DOF (as for every CG vector); the per-node BC bytes of v's planes are then not
 * read.  The result is bit-identical to the call without the flag for such v.        */
#define TOSIMP_V_ZERO_ON_FIXED 0x100
/* Scatter forms of tosimp_apply_K, OR-ed into the precision (FP64 / FP32 only), kept as
 * measured alternatives to the default owner-computes pass (paper Alg. "Fused
 * Gather-GEMM-Scatter" scatters with atomic additions).  Both clear y first, then add
 * element results with atomics; the order of the additions is not fixed, so results
 * agree with the default to rounding, not bit for bit, and vary from call to call.
 *   ATOMIC_ELEMENT: one thread per element, 24 global atomic additions per element.
 *   ATOMIC_BRICK:   8x8x4-element bricks reduced in LDS; only nodes on brick faces use
 *                   global atomic additions.                                         */
#define TOSIMP_SCATTER_ATOMIC_ELEMENT 0x200
#define TOSIMP_SCATTER_ATOMIC_BRICK 0x400

/* ---- filter modes -------------------------------------------------------------- */
#define TOSIMP_FILTER_FORWARD 0  /* out = H in / Hs                                   */
#define TOSIMP_FILTER_ADJOINT 1  /* out = H (in / Hs)                                 */

/* ---- solver modes -------------------------------------------------------------- */
#define TOSIMP_SOLVE_PLAIN_FP64 0 /* Jacobi-PCG, FP64 vectors and reductions           */
#define TOSIMP_SOLVE_IR 1         /* FP64 refinement around a low-precision inner CG  */

#define TOSIMP_PRECOND_JACOBI 0
#define TOSIMP_PRECOND_NN 1       /* learned U-Net correction in flexible CG          */
#define TOSIMP_PRECOND_MG 2       /* geometric-multigrid V-cycle (see tosimp_mg_apply) */

typedef struct tosimp_ctx tosimp_ctx;

typedef struct tosimp_solve_opts {
  double tol;        /* stop when ||r|| <= tol * ||b|| (see tosimp_pcg_solve)         */
  int maxit;         /* cap on CG iterations (plain) or on inner iterations in total  */
  int mode;          /* TOSIMP_SOLVE_*                                                */
  int inner_prec;    /* TOSIMP_PREC_* of the inner solve in IR mode                   */
  double inner_tol;  /* IR: relative tolerance of each inner solve, loosened to       */
                     /*   min(0.5, 0.3 tol ||b|| / ||r||) when that reaches tol       */
  int max_outer;     /* cap on refinement steps in IR mode                            */
  int precond;       /* TOSIMP_PRECOND_*                                              */
  int check_every;   /* host convergence polls every this many iterations (>= 1)      */
  int enforce_rule;  /* refuse inner precisions failing u * kappa < 1 (EPRECISION):    */
                     /*   0 off; 1 with the caller's kappa; 2 with the library's own   */
                     /*   estimate (see tosimp_pcg_solve)                               */
  double kappa;      /* condition estimate used by enforce_rule 1                      */
  float* harvest_r;  /* PLAIN_FP64 only, optional (NULL = off): device FP32 array of    */
  float* harvest_u;  /*   harvest_cap x n_dof each, receiving r_k and u_k every          */
  int harvest_cap;   /*   harvest_every iterations (k = 0, he, 2 he, ...) until full;    */
  int harvest_every; /*   tosimp_nn_make_targets turns u_k into e_k = u* - u_k           */
  int fcg_window;    /* PRECOND_NN: flexible CG keeps this many directions (1..16; 0 = 1) */
  int eager;         /* 1: launch every kernel directly; 0: Jacobi-PCG replays batches of */
                     /*    check_every iterations as a HIP graph (same kernels, same order) */
  int nn_stall;      /* PRECOND_NN: once ||r|| has made no new minimum for this many       */
                     /*   iterations of an inner solve, plain Jacobi-PCG continues it from  */
                     /*   the current iterate (0 = 50, < 0 = never)                          */
  int mg_degree;     /* PRECOND_MG: Chebyshev smoothing degree (1..16; 0 = 2)               */
  double mg_alpha;   /* PRECOND_MG: smoothing interval [lam / alpha, lam] (> 1; 0 = 20)     */
  const double* harvest_ustar; /* optional with harvesting (NULL = off): device FP64 n_dof  */
                     /*   reference solution; harvest_u then receives ustar - u_k formed in  */
                     /*   FP64 before the cast (the error, not the iterate)                  */
} tosimp_solve_opts;

typedef struct tosimp_solve_stats {
  int iterations;          /* total CG iterations (inner iterations in IR mode)      */
  int outer_iterations;    /* refinement steps (0 in plain mode)                     */
  int fallbacks;           /* NN -> Jacobi fallbacks taken                           */
  int status;              /* same value the call returned                           */
  double rel_residual;     /* final ||r|| / ||b|| the solver judged convergence on   */
  double true_rel_residual;/* ||b - K u|| / ||b|| recomputed in FP64 at exit         */
  int harvested;           /* (r_k, u_k) pairs written to the harvest arrays         */
  int restarts;            /* NN inner solves continued by Jacobi-PCG (nn_stall)     */
  double b_dot_u;          /* b^T u (the compliance when b = f)                      */
  double b_dot_u_corrected;/* b^T u + u^T (b - K u) = 2 b^T u - u^T K u: differs from */
                           /* b^T u* by -||u - u*||_K^2 only (second order in u - u*) */
  int escalations;         /* IR: inner precision raised to FP32 after stagnation    */
  double kappa;            /* the kappa enforce_rule used (0 when off)               */
} tosimp_solve_stats;

typedef struct tosimp_step_opts {
  double volfrac;    /* target volume fraction                                       */
  double move;       /* OC move limit                                                 */
  tosimp_solve_opts solve;
  double beta;       /* > 0: three-field scheme with projection sharpness beta;       */
                     /*   <= 0: density-filter scheme (no projection)                 */
  double eta;        /* projection threshold (three-field scheme)                     */
} tosimp_step_opts;

typedef struct tosimp_step_stats {
  double compliance; /* f^T u after the solve                                         */
  double change;     /* max |x_new - x|                                               */
  double volume;     /* mean of the new physical density                              */
  int bisection_steps;
  tosimp_solve_stats solve;
  double grayness;   /* 4/n sum xphys (1 - xphys) of the density the solve used       */
} tosimp_step_stats;

/* The SIMP-120 protocol (paper Sec. "Experimental Setup"): see tosimp_simp_protocol. */
typedef struct tosimp_protocol_opts {
  int iters;              /* outer iterations (the paper: 120)                        */
  double volfrac;         /* volume fraction of the projected density                 */
  double eta;             /* projection threshold (the paper: 0.5)                    */
  double restart_factor;  /* restart when c > restart_factor * c_selected (1.12)      */
  double eligible_penal;  /* selection needs penal >= this (3.0) ...                  */
  double eligible_gray;   /* ... and grayness < this (0.25)                           */
  int nphases;            /* 0: the paper's four phases; else phases[5 * nphases]:     */
  const double* phases;   /*   last iteration, penal, beta, move, rmin at the phase   */
                          /*   end (<= 0: unchanged), host memory                      */
  tosimp_solve_opts solve;
} tosimp_protocol_opts;

typedef struct tosimp_protocol_record {
  int it;                 /* 1-based iteration                                        */
  int cg_iterations;
  int bisection_steps;    /* 0 on a restart                                           */
  int restart;            /* 1: the next design is the selected one (no update)       */
  int eligible;           /* penal and grayness admit the iterate to selection        */
  int selected;           /* 1: the iterate became the selected one                   */
  double penal, beta, move, rmin;
  double compliance;      /* f^T u                                                     */
  double grayness;        /* of the projected density                                  */
  double change;          /* max |x_new - x| of the update (0 on a restart)            */
} tosimp_protocol_record;

/* ---- lifecycle ------------------------------------------------------------------
 * tosimp_create: make a context on HIP device `device` using `stream` (a hipStream_t,
 * NULL for the default stream).  *out receives the handle.  tosimp_destroy frees the
 * workspace (synchronising the stream first); NULL is accepted.                      */
int tosimp_create(int device, void* stream, tosimp_ctx** out);
int tosimp_destroy(tosimp_ctx* ctx);
int tosimp_set_stream(tosimp_ctx* ctx, void* stream);
const char* tosimp_last_error(const tosimp_ctx* ctx);
/* Library version string and a NUL-separated list of compiled GPU targets. */
const char* tosimp_version(void);

/* ---- problem set-up ---------------------------------------------------------------
 * tosimp_set_mesh (paper Sec. "Three-Dimensional SIMP Topology Optimization",
 * Eq. simp): nx, ny, nz >= 1 elements of edge h > 0; SIMP modulus
 * E_e = Emin + x_e^penal (E0 - Emin); Poisson ratio nu in (-1, 0.5); density-filter
 * radius rmin > 0 (in element edges).  Builds the 24x24 element stiffness by 2x2x2
 * Gauss quadrature and its exact factorisation in the tensor Hadamard basis, the filter
 * weights, and allocates the workspace (EINVAL on bad sizes, among them meshes of more
 * than 89,478,484 nodes, the limit of the operator's 32-bit byte offsets into an FP64
 * DOF vector; ENOMEM on failure).  Clears any previous boundary conditions and loads. */
int tosimp_set_mesh(tosimp_ctx* ctx, int nx, int ny, int nz, double h, double E0,
                    double Emin, double nu, double penal, double rmin);
/* Dirichlet set: `n` DOF ids (host, any order, duplicates allowed) held at zero.
 * EINVAL if an id is out of range.                                                   */
int tosimp_set_bcs(tosimp_ctx* ctx, const int64_t* fixed_dofs_host, int64_t n);
/* Load vector f (device, n_dof FP64); copied into the workspace.  EINVAL if f is
 * non-zero on a fixed DOF.                                                            */
int tosimp_set_loads(tosimp_ctx* ctx, const double* f_dev);
/* Mesh counts: n_elem, n_node, n_dof (any pointer may be NULL).                      */
int tosimp_counts(const tosimp_ctx* ctx, int64_t* n_elem, int64_t* n_node, int64_t* n_dof);

/* ---- the operator ----------------------------------------------------------------
 * tosimp_apply_K (paper Eq. matfree and Alg. "Fused Gather-GEMM-Scatter"):
 * y = K_c(xphys) v, one fused pass (gather the 24 element DOFs, multiply by
 * E_e K_E, accumulate), deterministic (no atomics; bit-identical across calls).
 * xphys: n_elem element densities of type xdtype; v, y: n_dof values.  prec selects
 * the arithmetic: PREC_FP64 needs v, y FP64; PREC_FP32 and the MFMA precisions need
 * v, y FP32; it may carry TOSIMP_V_ZERO_ON_FIXED (FP64/FP32 with xdtype of the same
 * width; ignored otherwise) or one TOSIMP_SCATTER_* flag (FP64 / FP32; EINVAL
 * otherwise).  y is overwritten (not accumulated); y must not overlap v or xphys
 * (EINVAL).                                                                           */
int tosimp_apply_K(tosimp_ctx* ctx, const void* xphys_dev, int xdtype, const void* v_dev,
                   void* y_dev, int prec);
/* Jacobi diagonal (paper Sec. "Preconditioned Conjugate Gradient"): d = diag(K_c),
 * n_dof values of type dtype (1 on fixed DOFs).                                      */
int tosimp_diag_K(tosimp_ctx* ctx, const void* xphys_dev, int xdtype, void* d_dev,
                  int dtype);

/* ---- the solve -------------------------------------------------------------------
 * tosimp_pcg_solve (paper Sec. "Preconditioned Conjugate Gradient and Warm-Start
 * Strategy"; Sec. "BF16 Arithmetic in the Conjugate Gradient Solver" for IR mode):
 * solve K_c(xphys) u = b.  xphys: n_elem FP64; b: n_dof FP64 (must be zero on fixed
 * DOFs); u_inout: n_dof FP64 initial guess (warm start), overwritten by the solution
 * (its fixed DOFs are zeroed first).  b and u_inout must be 16-byte aligned, and
 * u_inout must not overlap b or xphys (EINVAL).
 * PLAIN_FP64: Jacobi-PCG in FP64, stop on the recursive ||r|| <= tol ||b||.
 * IR: outer loop in FP64 (true residual r = b - K u, u += s e) around an inner
 * Jacobi-PCG (or NN flexible CG) in FP32 vectors on the unit-norm residual with FP32
 * or MFMA operator; every dot product, norm, alpha and beta is accumulated in FP64.
 * PRECOND_NN (IR mode): flexible CG with the learned preconditioner; an iteration whose
 * preconditioned residual is not a descent direction (<r, z> <= 0) or not finite takes
 * the Jacobi step instead (stats->fallbacks), and an inner solve that stagnates
 * (opts->nn_stall) is finished by plain Jacobi-PCG (stats->restarts).
 * IR stagnation (two outer steps in a row that do not halve the true residual) raises a
 * matrix-core inner precision to FP32 (stats->escalations); at FP32 it ends the solve
 * with NOT_CONVERGED.  The precision rule (paper Sec. "Condition Number Estimation",
 * Eq. bf16barrier) admits inner precision l only when u_l * kappa < 1 with unit
 * roundoffs 2^-8 (BF16), 2^-11 (FP16), 2^-24 (FP32); with enforce_rule = 2 kappa is the
 * library's estimate for the Jacobi-scaled operator at uniform density (Lanczos as in
 * tosimp_kappa with rtol 1e-3, window 50, at most 5,000 steps, seeded start vector),
 * computed on first use and kept until the mesh or boundary conditions change.
 * Returns OK, NOT_CONVERGED (cap hit, u valid), FALLBACK_USED (a fallback or restart was
 * taken, u valid), EBREAKDOWN or EPRECISION (the rule refused the inner precision; stats
 * holds the kappa used).  stats may be NULL.
 * The solve runs on a stream of the context, ordered after the work already enqueued on
 * the caller's stream and before any work enqueued there after the call.            */
int tosimp_pcg_solve(tosimp_ctx* ctx, const double* xphys_dev, const double* b_dev,
                     double* u_inout_dev, const tosimp_solve_opts* opts,
                     tosimp_solve_stats* stats);

/* ---- SIMP pieces -----------------------------------------------------------------
 * tosimp_sensitivity (paper Sec. "Three-Dimensional SIMP Topology Optimization"):
 * dc_e = -penal xphys_e^(penal-1) (E0 - Emin) u_e^T K_E u_e (n_elem FP64) and the
 * compliance f^T u (FP64 host scalar; synchronises; c_host may be NULL).  dc must not
 * overlap u, which is read around every element (EINVAL).                            */
int tosimp_sensitivity(tosimp_ctx* ctx, const double* xphys_dev, const double* u_dev,
                       double* dc_dev, double* c_host);
/* Cone density filter (paper Sec. "Three-Dimensional SIMP Topology Optimization", the
 * filter of radius rmin), weights max(0, rmin - centroid distance), neighbourhood cut
 * at the domain boundary.  FORWARD: out = H in / Hs; ADJOINT: out = H (in / Hs).
 * in, out: n_elem FP64, must not overlap (EINVAL).                                    */
int tosimp_filter(tosimp_ctx* ctx, const double* in_dev, double* out_dev, int mode);
/* Smoothed Heaviside projection of the three-field scheme (paper Sec.
 * "Three-Dimensional SIMP Topology Optimization", projection equation), elementwise on
 * n_elem FP64 values, den = tanh(beta eta) + tanh(beta (1 - eta)):
 *   g_dev NULL:  out = (tanh(beta eta) + tanh(beta (in - eta))) / den   (the projection)
 *   g_dev set:   out = g beta (1 - tanh^2(beta (in - eta))) / den        (chain rule:
 *                g times the derivative of the projection at in)
 * beta > 0 and finite, 0 <= eta <= 1 (EINVAL otherwise).  out may be in or g itself but
 * must not partly overlap either (EINVAL).  Asynchronous.                             */
int tosimp_project(tosimp_ctx* ctx, const double* in_dev, const double* g_dev,
                   double* out_dev, double beta, double eta);
/* tosimp_set_params: change the SIMP penalty and the filter radius of the current mesh
 * (continuation); the filter weights, row sums and H(1/Hs) are rebuilt when rmin
 * changes.  Ranges as tosimp_set_mesh.  Synchronises.                               */
int tosimp_set_params(tosimp_ctx* ctx, double penal, double rmin);
/* tosimp_grayness (paper Sec. "Experimental Setup"): g = 4/n sum_e rho_e (1 - rho_e)
 * of n_elem FP64 device values, into *g_host (FP64 reduction).  Synchronises.        */
int tosimp_grayness(tosimp_ctx* ctx, const double* rho_dev, double* g_host);
/* Optimality-criteria update of the density-filter scheme (paper Sec.
 * "Three-Dimensional SIMP Topology Optimization"; the three-field update with the
 * projected volume is part of tosimp_simp_step) with bisection on the volume
 * multiplier (bracket [0, 1e9], stop when (l2-l1)/(l1+l2) <= 1e-3):
 * x_new = clip(x sqrt(-dc / (dv lambda)), max(0, x - move), min(1, x + move)) with
 * dv = H(1/Hs); the volume test is sum(filter(x_new)) > volfrac n_elem, evaluated
 * exactly as the weighted sum dv^T x_new.  dc must be the filtered sensitivity.
 * Writes x_new and xphys_new = filter(x_new) (n_elem FP64), returns max|x_new - x|
 * in *change_host and the step count in *steps_host (either may be NULL).  x_new must
 * not overlap x, dc or xphys_new (EINVAL).  A bracket that has not closed after 256
 * steps (no multiplier puts the volume above the target) is an EINVAL error.          */
int tosimp_oc_update(tosimp_ctx* ctx, const double* x_dev, const double* dc_dev,
                     double volfrac, double move, double* x_new_dev,
                     double* xphys_new_dev, double* change_host, int* steps_host);
/* One SIMP iteration (paper Sec. "Software Architecture" gives the order): solve
 * K(xphys) u = f (warm start from u_inout), sensitivity, chain rule to the design, OC
 * update; x_inout and xphys_inout (n_elem FP64) are replaced by the new design and its
 * physical density, u_inout (n_dof FP64) by the solution.  xphys_inout must be the
 * physical density of x_inout on entry.
 *   opts->beta <= 0, density-filter scheme: xphys = H x / Hs, dc <- H (dc / Hs), OC on
 *     the filtered volume (tosimp_oc_update).
 *   opts->beta > 0, three-field scheme (paper Sec. "Three-Dimensional SIMP Topology
 *     Optimization", projection equation): xbar = H x / Hs, xphys = project(xbar);
 *     dc <- H ((dc * project'(xbar)) / Hs), dv = H (project'(xbar) / Hs), and the OC
 *     bisection tests the projected volume sum project(filter(x_new)) against
 *     volfrac n_elem.
 * x, xphys and u must not overlap (EINVAL).  Synchronises.                           */
int tosimp_simp_step(tosimp_ctx* ctx, double* x_inout_dev, double* xphys_inout_dev,
                     double* u_inout_dev, const tosimp_step_opts* opts,
                     tosimp_step_stats* stats);
/* tosimp_simp_protocol: the three-field SIMP-120 protocol of paper Sec. "Experimental
 * Setup".  Iteration it = 1..iters: (penal, beta, move, rmin) from the continuation
 * phases (the paper's: it 1-15 (1.5, 1, 0.20); 16-40 (3.5, 4, 0.15) with rmin moving
 * linearly to 1.35; 41-65 (4.5, 16, 0.08) to 1.25; 66-120 (4.5, 32, 0.05) to 1.20;
 * the initial radius is the context's); xphys = project(filter(x)); solve (warm start);
 * c = f^T u; g = grayness(xphys).  If a selected iterate exists and c > restart_factor
 * c_selected, the next design is the selected design (restart); otherwise the iterate
 * is eligible when penal >= eligible_penal and g < eligible_gray, becomes the selected
 * one when its c is the lowest eligible so far, and the three-field update of
 * tosimp_simp_step gives the next design.
 * x_inout: the initial design (the paper: volfrac everywhere), replaced by the final
 * one; x_sel_dev receives the selected design (unchanged if none); xphys_out the
 * physical density of the last iteration; u_inout the warm start and final solution
 * (all FP64 device, no overlaps).  records_host: iters entries.  *it_selected (0 if
 * none) and *c_selected.  The penalty and radius of the context are restored at exit.
 * Synchronises.                                                                        */
int tosimp_simp_protocol(tosimp_ctx* ctx, double* x_inout_dev, double* x_sel_dev,
                         double* xphys_out_dev, double* u_inout_dev,
                         const tosimp_protocol_opts* opts, tosimp_protocol_record* records_host,
                         int* it_selected, double* c_selected);

/* ---- conditioning ----------------------------------------------------------------
 * tosimp_lanczos (paper Sec. "Condition Number Estimation" estimates the extremes of
 * K; here by symmetric Lanczos in FP64, no reorthogonalisation): k steps on K_c(xphys)
 * (jacobi_scaled = 0) or on D^-1/2 K_c D^-1/2 (jacobi_scaled = 1) from the start
 * vector v0 (n_dof FP64 device, zeroed on fixed DOFs so the Krylov space stays in the
 * free block).  Writes alpha[0..m) and beta[0..m-1) to host arrays of length k and
 * m to *steps_host (m < k only on an invariant subspace).  Synchronises.
 * tosimp_tridiag_extremes: smallest and largest eigenvalue of the symmetric
 * tridiagonal (alpha, beta) of order m by Sturm bisection (host only).              */
int tosimp_lanczos(tosimp_ctx* ctx, const double* xphys_dev, const double* v0_dev, int k,
                   int jacobi_scaled, double* alpha_host, double* beta_host,
                   int* steps_host);
int tosimp_tridiag_extremes(const double* alpha, const double* beta, int m, double* lmin,
                            double* lmax);
/* tosimp_lanczos_noalloc: for callers that cannot allocate device memory (a tight
 * serving loop, a harness that forbids hipMalloc).  Computes exactly what tosimp_lanczos
 * computes (same kernels, same order: bit-identical alpha and beta), but keeps alpha and
 * beta in a fixed device array of the library instead of workspace grown on demand, so
 * the call allocates nothing (no hipMalloc / hipFree; the mesh workspace of
 * tosimp_set_mesh is reused).  k <= 16,383 (EINVAL beyond, the array's size: 256 KiB per
 * device, held until the process ends).  Writes beta_host[0..k-1) (entries from m - 1
 * on are unspecified) and alpha_host[0..m), m to *steps_host.  Every call on a device
 * shares that device's array: calls that overlap in time on one device (two threads, two
 * contexts) race and must be serialised by the caller.  Synchronises.               */
int tosimp_lanczos_noalloc(tosimp_ctx* ctx, const double* xphys_dev, const double* v0_dev,
                           int k, int jacobi_scaled, double* alpha_host, double* beta_host,
                           int* steps_host);
/* tosimp_kappa (paper Sec. "Condition Number Estimation"): extreme eigenvalues of
 * K_c(xphys) (jacobi_scaled = 0) or D^-1/2 K_c D^-1/2 (1) by the Lanczos of
 * tosimp_lanczos with a stopping rule: after every `window` steps the smallest Ritz
 * value is compared with its value `window` steps earlier, and the run stops once they
 * agree to rtol (relative), on an invariant subspace, or after kmax steps.  *lmin is an
 * upper bound of the smallest eigenvalue and *lmax a lower bound of the largest, so
 * lmax / lmin bounds kappa from below.  *steps = steps taken, *converged = 1 unless kmax
 * ended the run.  v0 as in tosimp_lanczos.  Synchronises every window.              */
int tosimp_kappa(tosimp_ctx* ctx, const double* xphys_dev, const double* v0_dev, int kmax,
                 int jacobi_scaled, double rtol, int window, double* lmin, double* lmax,
                 int* steps, int* converged);

/* ---- geometric multigrid ------------------------------------------------------------
 * tosimp_mg_apply (paper Sec. "Path to Geometric Multigrid Integration": the fused
 * operator as smoother, restriction R, prolongation P = R^T, direct coarsest solve):
 * z = V(r), one V-cycle for K_c(xphys) z = r.  Levels: n -> ceil(n/2) elements per axis of
 * twice the edge until an axis has one element (at most 12 levels); coarse operators
 * re-discretised (K_E scaled by the edge, a coarse modulus = sum of the existing children's
 * moduli / 8); a coarse DOF is fixed when a fine DOF in its interpolation support is;
 * trilinear P; Chebyshev smoothing of the given degree (0 = 2) on D^-1 K over
 * [lam / alpha, lam] (alpha 0 = 20), lam = lambda_max(K_E) / K_E[0][0] (an upper bound of
 * lambda_max(D^-1 K) for any density), before and after the coarse correction (symmetric
 * V-cycle); the coarsest level is solved with the dense inverse of its operator (at most
 * 1,536 DOFs: EINVAL for meshes whose coarsest grid is larger).  xphys: n_elem FP64; r, z:
 * n_dof values of prec (TOSIMP_PREC_FP64 or TOSIMP_PREC_FP32), r zero on fixed DOFs; z
 * must not overlap r or xphys (EINVAL).  The hierarchy is rebuilt for xphys on every call
 * (synchronises once for the coarsest inverse).  tosimp_pcg_solve with precond =
 * TOSIMP_PRECOND_MG runs CG preconditioned by one V-cycle per iteration (plain mode: FP64
 * vectors and V-cycle; IR mode: FP32 inner vectors and V-cycle).
 * tosimp_mg_levels: writes the element counts of up to `cap` levels to dims_host[3 l ..
 * 3 l + 2] and returns the number of levels (negative: an error status).              */
int tosimp_mg_apply(tosimp_ctx* ctx, const double* xphys_dev, const void* r_dev, void* z_dev,
                    int prec, int degree, double alpha);
int tosimp_mg_levels(tosimp_ctx* ctx, int* dims_host, int cap);

/* ---- learned preconditioner -------------------------------------------------------
 * A 3-level 3D-convolutional U-Net N on the node grid supplies the correction of a
 * variable two-stage preconditioner (tosimp_nn_precondition) in flexible CG (IR mode
 * with precond = TOSIMP_PRECOND_NN).  Not in the paper (its Sec. "Path to Geometric
 * Multigrid Integration" names stronger preconditioners as the way past Jacobi-PCG).
 * Layers (c_in -> c_out, kernel, stride; b = base): e0a 4->b, e0b b->b, d1 b->2b s2,
 * e1 2b->2b, d2 2b->4b s2, m2a 4b->4b, m2b 4b->4b, u1a [up(m2b), e1] 6b->2b,
 * u1b 2b->2b, u0a [up(u1b), e0b] 3b->b, u0b b->b (all 3x3x3, zero padding 1, leaky
 * ReLU 0.01), head b->3 (1x1x1, linear); nearest up-sampling; no biases.
 * Weights: FP32 master copy in [layer][c_out][c_in][kz][ky][kx] order (layers as
 * listed), compute copies in BF16 (bf16 = 1) or FP32.  Training: Adam (0.9, 0.999,
 * 1e-8) on the relative masked loss sum_free (N - t)^2 / sum_free t^2 with the unit-RMS
 * target t = e sqrt(n_dof) / ||e|| (flexible CG does not depend on the scale of z); the
 * residual input enters at unit RMS, r sqrt(n_dof) / ||r||.
 *
 * tosimp_nn_create: build the network for the current mesh (base 16 or 32); weights
 *   are zero until set.  Replaces an existing network.  Allocates its workspace.
 * tosimp_nn_num_params: number of FP32 master weights.
 * tosimp_nn_set_weights / get_weights: copy the master weights from / to host memory
 *   (n must equal the count); set_weights also resets the Adam moments.  Synchronise.
 * tosimp_nn_set_density: nodal density (mean of the adjacent elements) from an element
 *   density on the device (xdtype TOSIMP_F64 or TOSIMP_F32), and an FP32 copy of the
 *   density for the energy loss; used by apply and train_step until the next call.
 * tosimp_nn_apply: z = (||r|| / sqrt(n_dof)) N(r sqrt(n_dof) / ||r||, rho_node), zero on
 *   fixed DOFs (FP32 device vectors, n_dof; r and z must not alias).
 * tosimp_nn_precondition: the preconditioner flexible CG applies, at element density
 *   x32 (FP32 device): n = tosimp_nn_apply(r), s = <r,n>/<n,K n> (0 unless
 *   both are positive), z = s n + D^-1 (r - s K n), D the Jacobi diagonal of K_c(x32).
 *   Sets the nodal density.  r, z: FP32 device n_dof, distinct.  Synchronises.
 * tosimp_nn_forward: test hook, raw network output [n_node][3] FP32 for a channels-last
 *   input [n_node][4] FP32 (both device).
 * tosimp_nn_loss_grad: test hook, the loss against target [n_node][3] (device FP32;
 *   DOFs fixed by the BC mask excluded) into *loss_host and its gradient (master
 *   layout, host FP32, may be NULL).  Synchronises.
 * tosimp_nn_train_step: one Adam step on the mean loss of nb pairs (r, e), device FP32
 *   [nb][n_dof] each.  Synchronises; *loss_host = mean loss before the step.
 * tosimp_nn_set_loss: training loss, 0 = the relative MSE above (default), 1 = energy
 *   norm: for the correction n (network output on free DOFs) and a pair (r, e),
 *   L = 1 - <n,r>^2 / (<n,K n> <e,r>), the relative K-norm error of the best multiple of
 *   n, K at the density of tosimp_nn_set_density.
 * tosimp_nn_sample_grad: test hook, loss and gradient (master layout, host FP32, may be
 *   NULL) of one pair (r, e) (device FP32, n_dof each).  Synchronises.
 * tosimp_nn_make_targets: harvest_u[k] <- u_star - harvest_u[k] for k < count
 *   (u_star FP64 device, harvest_u FP32 device [count][n_dof]).                       */
int tosimp_nn_create(tosimp_ctx* ctx, int base, int bf16);
int tosimp_nn_num_params(const tosimp_ctx* ctx, int64_t* n);
int tosimp_nn_set_weights(tosimp_ctx* ctx, const float* w_host, int64_t n);
int tosimp_nn_get_weights(tosimp_ctx* ctx, float* w_host, int64_t n);
int tosimp_nn_set_density(tosimp_ctx* ctx, const void* x_dev, int xdtype);
int tosimp_nn_apply(tosimp_ctx* ctx, const float* r_dev, float* z_dev);
int tosimp_nn_precondition(tosimp_ctx* ctx, const float* x32_dev, const float* r_dev,
                           float* z_dev);
int tosimp_nn_forward(tosimp_ctx* ctx, const float* x4_dev, float* out3_dev);
int tosimp_nn_loss_grad(tosimp_ctx* ctx, const float* x4_dev, const float* target3_dev,
                        double* loss_host, float* grad_host);
int tosimp_nn_train_step(tosimp_ctx* ctx, const float* r_batch_dev, const float* e_batch_dev,
                         int nb, double lr, double* loss_host);
int tosimp_nn_make_targets(tosimp_ctx* ctx, const double* u_star_dev, float* harvest_u_dev,
                           int count);
int tosimp_nn_set_loss(tosimp_ctx* ctx, int kind);
int tosimp_nn_sample_grad(tosimp_ctx* ctx, const float* r_dev, const float* e_dev,
                          double* loss_host, float* grad_host);

#ifdef __cplusplus
}
#endif
#endif /* TOSIMP_H */
