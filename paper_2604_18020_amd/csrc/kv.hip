// Fused matrix-free operator y = K_c(x) v on the structured Q1 mesh (FP64 / FP32).
//
// Paper: Eq. (matfree) and Alg. "Fused Gather-GEMM-Scatter": one pass that gathers
// the 24 DOFs of each element, multiplies by E_e K_E and accumulates into y.  The
// paper uses one thread per element, K_E in shared memory and atomic scatter.
//
// gfx950 design (deterministic, no atomics, one launch):
//  * A block owns a 31 x 7 column of nodes and a chunk of node planes.  Its 256
//    threads are the 32 x 8 element columns that touch those nodes (one halo element
//    on the low side of each axis is recomputed by the neighbouring block); a row of 32
//    element columns lies in one wavefront.
//  * The block streams up the z axis.  Each step stages one node plane of v (33 x 9
//    nodes x 3 components) in LDS, one node per lane (a 12-byte FP32 / 24-byte FP64
//    buffer load; consecutive lanes take consecutive nodes of a row), issued ahead (two
//    planes in FP32, one in FP64), as 16- / 32-byte node records so that a corner is
//    one LDS read.
//    Each thread applies the element stiffness of its element column at the current
//    layer and keeps every partial result in registers in the 2D (x, y) Hadamard basis:
//    the forward transform of a plane is reused as the bottom face of the next layer,
//    and the top-face contributions of a layer are added to the bottom-face
//    contributions of the next before a single inverse transform.
//  * K_E is applied in factored form K_E = H^T S H / 64 (45 non-zeros in S, eight
//    distinct values, see common.h): about 150 VALU ops per element instead of 1,152.
//  * Each owned node sums the four element-column contributions around it in a fixed
//    order (the x pair by a DPP shift of the wave by one lane, the y pair through LDS)
//    and the owner stores its node straight from registers (one 12- / 24-byte store;
//    a wave's lanes write contiguous row segments), the plane's base in the scalar
//    buffer resource.  Fixed DOFs output y = v (a branch that only waves holding a
//    clamped node take).
//  * Operands known to be zero on fixed DOFs (all CG vectors) skip the BC bytes of the
//    loaded planes; only the owned node's BC byte is read.
//  * Block ids are remapped so that each XCD gets a contiguous range of tiles.
//  * Optionally the block's share of <v, y> (FP64) is stored per tile and a one-block
//    kernel finalises it (CG step length, Lanczos alpha).
#include <atomic>

#include "common.h"
#include "dev.h"

namespace tosimp {

constexpr int KBX = 32, KBY = 8;  // element columns per block (x, y)
static_assert(64 % KBX == 0 && KBX * KBY == 256, "a row of element columns lies in one wave");

template <typename T>
struct KvC {
  T ad, ao, cs, bd, bo, cd, co, hg;
};

enum KvFin { FIN_NONE = 0, FIN_ALPHA = 1, FIN_SCALAR = 2 };

template <typename T, typename XT>
struct KvArgs {
  const T* v;
  T* y;
  const XT* x;
  const uint8_t* mask;
  double* partials;   // one slot per tile when a dot is requested
  SolverState* st;    // FIN_ALPHA target
  double* out;        // FIN_SCALAR target
  int fin;
  int nx, ny, nz;
  int tiles_x, tiles_y, chunks_z, kz, ntiles, per_xcd;
  T E0mEmin, Emin;
  T penal;
  KvC<T> k;
  // Chebyshev epilogue of a multigrid smoothing step (EPI > 0): with t = K v at the owned
  // node, r = eb - t, d = ec2 r edinv (EPI 1) or ec1 edd + ec2 r edinv (EPI 2); edd <- d
  // and y <- v + d (y is the new iterate, never v itself).  EPI 3 is a visit's first two
  // steps from a zero iterate: the operand is formed while staging, v = ec0 (v_in
  // edinv) with v_in = eb, and the epilogue is EPI 2's with edd = v.
  const T* eb;
  T* edd;
  const T* edinv;  // per node
  T ec0, ec1, ec2;
};

// Element modulus from the element value xv.  PEN selects the law: kPenPow
// Emin + x^penal (E0 - Emin), kPenCube the same with penal = 3, kPenModulus: xv is the
// modulus itself (multigrid levels carry averaged moduli, not densities).
enum KvPen { kPenPow = 0, kPenCube = 1, kPenModulus = 2 };

template <typename T, typename XT, int PEN>
__device__ __forceinline__ T simp_E(XT xv, T Emin, T E0mEmin, T penal) {
  T x = static_cast<T>(xv);
  if constexpr (PEN == kPenModulus) return x;
  T xp;
  if constexpr (PEN == kPenCube) {
    xp = x * x * x;
  } else {
    xp = x > T(0) ? pow(x, penal) : T(0);
  }
  return Emin + xp * E0mEmin;
}

// ---------------------------------------------------------------- buffer access
// Raw buffer loads/stores: the per-lane offset is loop-invariant, the moving plane
// base lives in the (uniform) resource, and the hardware range check returns 0 for
// offsets past num_records and drops such stores; halo lanes and non-owner lanes use
// an offset beyond any buffer.
constexpr int kOOB = 0x7FFFFFF0;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, long long bytes) {
  const int n = bytes <= 0 ? 0 : (bytes >= 0x7FFFFFFF ? 0x7FFFFFFF : (int)bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, kRsrcWord3);
}

// For byte counts already known to be below 2^31 (the launcher's size limit).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc32(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kRsrcWord3);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, int off, int soff);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, int off, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, int off, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
__device__ __forceinline__ uint8_t buf_ld_u8(__amdgpu_buffer_rsrc_t r, int off, int soff) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, off, soff, 0);
}
// Stores take the whole offset in the VGPR and a zero soffset.  The compiler merges the
// three component stores of a node into one 16-byte (FP64) store; after a store wider
// than 8 bytes the data VGPRs must not be overwritten by the next VALU instruction, and
// the compiler inserts that wait state only when soffset is not an SGPR.  With the plane
// offset in an SGPR soffset the wait was omitted and the store occasionally wrote the
// value of the following instruction.  Out-of-range lanes keep an offset past
// num_records (the sum stays below 2^32 and the range check is unsigned).
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

// a if sel == 0 else b, as a bitwise blend (no branch around the computation of a).
__device__ __forceinline__ float bit_select(float a, float b, unsigned sel) {
  const unsigned m = 0u - sel;
  return __uint_as_float((__float_as_uint(a) & ~m) | (__float_as_uint(b) & m));
}
__device__ __forceinline__ double bit_select(double a, double b, unsigned sel) {
  const unsigned long long m = 0ull - (unsigned long long)sel;
  return __builtin_bit_cast(double, (__builtin_bit_cast(unsigned long long, a) & ~m) |
                                        (__builtin_bit_cast(unsigned long long, b) & m));
}

// The value of lane l + 1 in lane l (a DPP shift of the whole wave by one lane; lane 63
// reads 0).  The compiler folds the move into the instruction that consumes it.
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_next(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x130, 0xF, 0xF, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x130, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Node-wide buffer accesses: one lane moves the three components of a node (12 bytes in
// FP32, 24 in FP64).  Per-lane 4-byte accesses cap the memory pipeline far below HBM speed
// on this GPU; whole-node accesses keep the operator's loads and stores near streaming
// rates.
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Node3 {
  T c[3];
};

__device__ __forceinline__ Node3<float> buf_ld_node(const float*, __amdgpu_buffer_rsrc_t r,
                                                    int off, int soff) {
  const u32x3 w = __builtin_amdgcn_raw_buffer_load_b96(r, off, soff, 0);
  return {{__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z)}};
}
__device__ __forceinline__ Node3<double> buf_ld_node(const double*, __amdgpu_buffer_rsrc_t r,
                                                     int off, int soff) {
  // an offset past num_records (kOOB) stays past it after the + 16 (no wrap below 2^32)
  const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0);
  const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, (int)((unsigned)off + 16u), soff, 0);
  Node3<double> n;
  n.c[0] = __builtin_bit_cast(double, (unsigned long long)a.x | ((unsigned long long)a.y << 32));
  n.c[1] = __builtin_bit_cast(double, (unsigned long long)a.z | ((unsigned long long)a.w << 32));
  n.c[2] = __builtin_bit_cast(double, b);
  return n;
}
// Stores keep the whole offset in the VGPR and a zero soffset (see buf_st).
__device__ __forceinline__ void buf_st_node(const float* v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  const u32x3 w = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2])};
  __builtin_amdgcn_raw_buffer_store_b96(w, r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_st_node(const double* v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  const unsigned long long a = __builtin_bit_cast(unsigned long long, v[0]);
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v[1]);
  const u32x4 w = {(unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32)};
  __builtin_amdgcn_raw_buffer_store_b128(w, r, (int)off, 0, 0);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v[2]), r, (int)(off + 16u), 0, 0);
}

// PM: v is known to be zero on fixed DOFs (every vector the CG iterations apply K_c to
// is), so the plane's BC bytes are not loaded and v needs no masking; only the owned
// node's BC byte is read (fixed rows output y = v = 0).
template <typename T, typename XT, int PEN, bool DOT, bool PM, int D, int KZMAX, int EPI>
__device__ __forceinline__ void kv_body(const KvArgs<T, XT>& A) {
  // Multiply-adds are fused only within one expression, never across statements, so
  // every z step rounds identically whatever was folded away around it (a chunk's first
  // layer starts from zero accumulators): results do not depend on the chunk depth.
#pragma clang fp contract(on)
  static_assert(EPI == 0 || PM, "the smoothing epilogue needs v = 0 on fixed DOFs");
  constexpr int NXL = KBX + 1, NYL = KBY + 1, NPN = NXL * NYL;  // nodes of a plane window
  constexpr int NS = (NPN + 255) / 256;                          // node slots per thread
  constexpr int NE = KBX * KBY;
  static_assert(NS == 2, "two node slots per thread");
  // Node records of four values (the fourth unused) so that a corner is one LDS read.
  __shared__ __attribute__((aligned(16))) T sv[NPN][4];  // node plane window, masked
  __shared__ __attribute__((aligned(16))) T sr[PM ? 1 : NPN][4];  // unmasked (fixed rows: y = v)
  __shared__ T sb[3 * NE];        // lower-row corner pairs, [c][element column]
  __shared__ double sred[4];

  const int bid = blockIdx.x;
  const int t = (bid & 7) * A.per_xcd + (bid >> 3);
  if (t >= A.ntiles) return;  // whole block: padding of the XCD remap
  const int tx = t % A.tiles_x;
  const int rest = t / A.tiles_x;
  const int ty = rest % A.tiles_y;
  const int cz = rest / A.tiles_y;

  const int tid = threadIdx.x, lx = tid % KBX, ly = tid / KBX;
  const int ex0 = tx * (KBX - 1) - 1, ey0 = ty * (KBY - 1) - 1;
  const int k0 = cz * A.kz;
  const int k1 = min(k0 + A.kz, A.nz + 1);  // owned node planes [k0, k1)
  const int NX1 = A.nx + 1;
  const int plane = NX1 * (A.ny + 1);  // nodes per plane
  const int n_node = plane * (A.nz + 1);
  const int elayer = A.nx * A.ny;
  // One resource per array for the whole launch; planes move in the scalar offset.
  const auto rv = make_rsrc(A.v, 3LL * n_node * (long long)sizeof(T));
  const int ybytes = 3 * n_node * (int)sizeof(T);  // < 2^31 (launcher's node limit)
  const auto rm = make_rsrc(A.mask, n_node);
  const auto rx = make_rsrc(A.x, (long long)elayer * A.nz * (long long)sizeof(XT));
  const int vplane_bytes = 3 * plane * (int)sizeof(T);
  const auto reb = make_rsrc(A.eb, EPI ? 3LL * n_node * (long long)sizeof(T) : 0);
  const auto redd = make_rsrc(A.edd, EPI == 2 ? 3LL * n_node * (long long)sizeof(T) : 0);
  const auto redi = make_rsrc(A.edinv, EPI ? (long long)n_node * (long long)sizeof(T) : 0);

  // Plane-load slots: window node q = tid + 256 s, local (q % NXL, q / NXL).  Lanes of a
  // wave take consecutive nodes of a row, so a wave's loads cover contiguous segments.
  int voff[NS], moff[NS], doff[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int q = tid + 256 * s;
    const int jl = q / NXL, il = q - jl * NXL;
    const int i = ex0 + il, j = ey0 + jl;
    const bool ok = q < NPN && i >= 0 && i <= A.nx && j >= 0 && j <= A.ny;
    const int node = i + NX1 * j;
    voff[s] = ok ? 3 * node * (int)sizeof(T) : kOOB;
    moff[s] = ok ? node : kOOB;
    doff[s] = ok ? node * (int)sizeof(T) : kOOB;
  }
  // Element column of this thread.
  const int ex = ex0 + lx, ey = ey0 + ly;
  const bool exy_ok = ex >= 0 && ex < A.nx && ey >= 0 && ey < A.ny;
  const int xoff = exy_ok ? (ex + A.nx * ey) * (int)sizeof(XT) : kOOB;
  // Node owned by this thread in the output phase: local (lx+1, ly+1).
  const int ni = ex0 + lx + 1, nj = ey0 + ly + 1;
  const bool owner = lx < KBX - 1 && ly < KBY - 1 && ni <= A.nx && nj <= A.ny;
  const int qown = (ly + 1) * NXL + (lx + 1);  // this thread's owned node in sv / sr
  const int moffown = owner ? ni + NX1 * nj : kOOB;
  // Out-of-range lanes keep an offset past num_records (the sum stays below 2^32 and the
  // range check is unsigned).
  const unsigned yoffown = owner ? (unsigned)(3 * (ni + NX1 * nj) * (int)sizeof(T)) : (unsigned)kOOB;
  const int dioffown = owner ? (ni + NX1 * nj) * (int)sizeof(T) : kOOB;

  // Register ring of D planes in flight: the plane's node values and BC bytes, the owned
  // node's BC byte, and the density of the element layer below the plane.  The main
  // loop is branch-free so that every wait is for a load issued D steps earlier
  // (vmcnt waits are in order: any late load would drain the whole ring).  Planes
  // outside the mesh load a clamped plane with every DOF flagged fixed (zero).
  Node3<T> pv[D][NS];
  uint8_t pm[D][NS];
  uint8_t po[D];
  XT px[D];
  T pd[D][NS];  // EPI 3: per-node scale of the staged operand
  auto issue = [&](Node3<T>* v, uint8_t* m, uint8_t& mo, XT& xv, T* d, int k) {
    const int kc = min(max(k, 0), A.nz);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if constexpr (!PM) m[s] = buf_ld_u8(rm, moff[s], plane * kc);
      v[s] = buf_ld_node(A.v, rv, voff[s], vplane_bytes * kc);
      if constexpr (EPI == 3) d[s] = buf_ld<T>(redi, doff[s], plane * kc * (int)sizeof(T));
    }
    mo = buf_ld_u8(rm, moffown, plane * kc);
    const int ez = min(max(k - 1, 0), A.nz - 1);
    xv = buf_ld<XT>(rx, xoff, elayer * ez * (int)sizeof(XT));
  };

  T TA[12], TB[12];   // 2D-basis faces (ping-pong: bottom / top)
  T VA[3], VB[3];     // own node values (unmasked) of the matching planes
  uint8_t MA = 0, MB = 0;
  T acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    TA[i] = T(0);
    TB[i] = T(0);
    acc[i] = T(0);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) VA[c] = VB[c] = T(0);
  double dotacc = 0.0;

  T ya[3];  // upper-row corner pair of the owned node, kept across the barrier
  // One z step at node plane p: stage the plane, transform the top face, and (when
  // ELEM) apply element layer p-1 and (when OUT) emit node plane p-1.
  auto step = [&](int p, Node3<T>* v, uint8_t* m, uint8_t& mo, XT& xv, T* d, const T* tb,
                  T* tt, const T* vown, T* vnew, uint8_t mown, uint8_t& mnew, bool elem,
                  bool out, int refill) {
    // Keep each step's instructions inside its own region: the scheduler must not hoist
    // a later step's use of a ring slot above this step (that would wait on a fresh load).
    __builtin_amdgcn_sched_barrier(0);
    // A plane outside the mesh (p = -1 or nz + 1) was loaded clamped: zero it here.
    const int force = (p >= 0 && p <= A.nz) ? 0 : 7;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int q = tid + 256 * s;
      if (s > 0 && q >= NPN) continue;  // the second slot covers the window's last nodes
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (EPI == 3) {
          sv[q][c] = force ? T(0) : A.ec0 * (v[s].c[c] * d[s]);
        } else if constexpr (PM) {
          sv[q][c] = force ? T(0) : v[s].c[c];
        } else {
          sv[q][c] = (((m[s] | force) >> c) & 1) ? T(0) : v[s].c[c];
          sr[q][c] = v[s].c[c];
        }
      }
    }
    const XT xcur = xv;
    mnew = mo;
    __syncthreads();
    issue(v, m, mo, xv, d, refill);
    // Epilogue operands of the owned node of plane p-1 (stored at the end of this step).
    Node3<T> eb_n{}, edd_n{};
    T edi = T(0);
    if constexpr (EPI > 0) {
      if (elem && out) {
        eb_n = buf_ld_node(A.eb, reb, (int)yoffown, vplane_bytes * (p - 1));
        if constexpr (EPI == 2) edd_n = buf_ld_node(A.edd, redd, (int)yoffown, vplane_bytes * (p - 1));
        edi = buf_ld<T>(redi, dioffown, plane * (p - 1) * (int)sizeof(T));
      }
    }
    __builtin_amdgcn_sched_barrier(0);

    // Forward 2D transform of the top face (plane p) of this element column.
    {
      const int q00 = ly * NXL + lx;
      T v00[3], v10[3], v01[3], v11[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v00[c] = sv[q00][c];
        v10[c] = sv[q00 + 1][c];
        v01[c] = sv[q00 + NXL][c];
        v11[c] = sv[q00 + NXL + 1][c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T a0 = v00[c] + v10[c], a1 = v10[c] - v00[c];
        const T b0 = v01[c] + v11[c], b1 = v11[c] - v01[c];
        tt[0 * 3 + c] = a0 + b0;
        tt[1 * 3 + c] = a1 + b1;
        tt[2 * 3 + c] = b0 - a0;
        tt[3 * 3 + c] = b1 - a1;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) vnew[c] = PM ? sv[qown][c] : sr[qown][c];

    if (elem) {
      // ---- element layer ez = p - 1: bottom face tb, top face tt -------------
      const bool eok = exy_ok && p - 1 >= 0 && p - 1 < A.nz;
      const T E = eok ? simp_E<T, XT, PEN>(xcur, A.Emin, A.E0mEmin, A.penal) : T(0);
#define HB(m2, c) (tb[(m2) * 3 + (c)] + tt[(m2) * 3 + (c)])
#define HT(m2, c) (tt[(m2) * 3 + (c)] - tb[(m2) * 3 + (c)])
      const T h1x = HB(1, 0), h1y = HB(1, 1), h1z = HB(1, 2);
      const T h2x = HB(2, 0), h2y = HB(2, 1), h2z = HB(2, 2);
      const T h3x = HB(3, 0), h3y = HB(3, 1), h3z = HB(3, 2);
      const T h4x = HT(0, 0), h4y = HT(0, 1), h4z = HT(0, 2);
      const T h5x = HT(1, 0), h5y = HT(1, 1), h5z = HT(1, 2);
      const T h6x = HT(2, 0), h6y = HT(2, 1), h6z = HT(2, 2);
      const T h7x = HT(3, 0), h7y = HT(3, 1), h7z = HT(3, 2);
#undef HB
#undef HT
      const T kad = E * A.k.ad, kao = E * A.k.ao, kcs = E * A.k.cs, kbd = E * A.k.bd;
      const T kbo = E * A.k.bo, kcd = E * A.k.cd, kco = E * A.k.co, khg = E * A.k.hg;
      const T sA = kao * (h1x + h2y + h4z);
      const T g1x = kad * h1x + sA, g2y = kad * h2y + sA, g4z = kad * h4z + sA;
      const T s1 = kcs * (h1y + h2x), s2 = kcs * (h1z + h4x), s3 = kcs * (h2z + h4y);
      const T g1y = s1, g2x = s1, g1z = s2, g4x = s2, g2z = s3, g4y = s3;
      const T g3x = kbd * h3x + kbo * h6z, g6z = kbo * h3x + kbd * h6z;
      const T g3y = kbd * h3y + kbo * h5z, g5z = kbo * h3y + kbd * h5z;
      const T g5x = kbd * h5x + kbo * h6y, g6y = kbo * h5x + kbd * h6y;
      const T sC = kco * (h3z + h5y + h6x);
      const T g3z = kcd * h3z + sC, g5y = kcd * h5y + sC, g6x = kcd * h6x + sC;
      const T g7x = khg * h7x, g7y = khg * h7y, g7z = khg * h7z;

      // Inverse z stage: bottom face gets g[m2] - g[m2+4], top face g[m2] + g[m2+4].
      T R[12];
      R[0] = acc[0] - g4x;  R[1] = acc[1] - g4y;  R[2] = acc[2] - g4z;
      R[3] = acc[3] + (g1x - g5x);  R[4] = acc[4] + (g1y - g5y);  R[5] = acc[5] + (g1z - g5z);
      R[6] = acc[6] + (g2x - g6x);  R[7] = acc[7] + (g2y - g6y);  R[8] = acc[8] + (g2z - g6z);
      R[9] = acc[9] + (g3x - g7x);  R[10] = acc[10] + (g3y - g7y); R[11] = acc[11] + (g3z - g7z);
      acc[0] = g4x;  acc[1] = g4y;  acc[2] = g4z;
      acc[3] = g1x + g5x;  acc[4] = g1y + g5y;  acc[5] = g1z + g5z;
      acc[6] = g2x + g6x;  acc[7] = g2y + g6y;  acc[8] = g2z + g6z;
      acc[9] = g3x + g7x;  acc[10] = g3y + g7y; acc[11] = g3z + g7z;

      if (out) {
        // ---- node plane p-1 is complete in R: inverse 2D transform to corners --
        // The owned node (lx+1, ly+1) sums corner (1,1) of this column, (0,1) of column
        // lx+1, (1,0) of column (lx, ly+1) and (0,0) of (lx+1, ly+1).  The x neighbour
        // is the next lane (rows are 32 lanes, lane 31 owns no node), so the pairs
        // along x come from the next lane (lane_next); only the pair of the row below goes
        // through LDS.
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T u0 = R[0 * 3 + c] - R[2 * 3 + c], u1 = R[1 * 3 + c] - R[3 * 3 + c];
          const T w0 = R[0 * 3 + c] + R[2 * 3 + c], w1 = R[1 * 3 + c] + R[3 * 3 + c];
          const T c00 = u0 - u1, c10 = u0 + u1, c01 = w0 - w1, c11 = w0 + w1;
          const T n01 = lane_next(c01), n00 = lane_next(c00);
          ya[c] = c11 + n01;
          sb[c * NE + tid] = c10 + n00;
        }
      }
    }
    // Barrier: the corners are complete, and every read of the plane buffers is done
    // before the next step overwrites them.
    __syncthreads();
    if (elem && out) {
      // Node plane p-1: sum the four element columns around the owned node and store it
      // (consecutive lanes hold consecutive nodes of a row: contiguous segments).
      T yv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) yv[c] = ya[c] + sb[c * NE + tid + KBX];
      // Fixed rows are identity (y = v).  Only nodes on the clamped boundary have fixed
      // DOFs, so almost every wave skips this branch.
      if (mown) {
#pragma unroll
        for (int c = 0; c < 3; ++c) yv[c] = bit_select(yv[c], vown[c], (mown >> c) & 1);
      }
      const int qb = vplane_bytes * (p - 1);
      const auto ryq = make_rsrc32(reinterpret_cast<const char*>(A.y) + qb, ybytes - qb);
      if constexpr (EPI == 0) {
        buf_st_node(yv, ryq, yoffown);
      } else {
        T dv[3], xo[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T r = eb_n.c[c] - yv[c];
          const T dprev = EPI == 3 ? vown[c] : edd_n.c[c];
          const T d = EPI == 1 ? A.ec2 * (r * edi) : A.ec1 * dprev + A.ec2 * (r * edi);
          dv[c] = d;
          xo[c] = vown[c] + d;
        }
        if constexpr (DOT) {
#pragma unroll
          for (int c = 0; c < 3; ++c) dotacc += owner ? (double)eb_n.c[c] * (double)xo[c] : 0.0;
        }
        buf_st_node(xo, ryq, yoffown);
        const auto rddq = make_rsrc32(reinterpret_cast<const char*>(A.edd) + qb, ybytes - qb);
        buf_st_node(dv, rddq, yoffown);
      }
      if constexpr (DOT && EPI == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) dotacc += owner ? (double)vown[c] * (double)yv[c] : 0.0;
      }
    }
  };

  // Prologue: fill the ring with planes k0-1 .. k0+D-2.
#pragma unroll
  for (int s = 0; s < D; ++s) issue(pv[s], pm[s], po[s], px[s], pd[s], k0 - 1 + s);
  // Fully unrolled z sweep (no loop back-edge, so no register copies of in-flight
  // loads): step i handles plane k0-1+i; plane k0-1 only seeds the bottom face, plane
  // k0 applies layer k0-1 (plane k0-1 is not owned), later steps emit the plane below.
#pragma unroll
  for (int i = 0; i < KZMAX + 2; ++i) {
    const int p = k0 - 1 + i;
    if (p > k1) break;
    const int refill = min(p + D, k1);
    if (i % 2 == 0)
      step(p, pv[i % D], pm[i % D], po[i % D], px[i % D], pd[i % D], TA, TB, VA, VB, MA, MB,
           i >= 1, i >= 2, refill);
    else
      step(p, pv[i % D], pm[i % D], po[i % D], px[i % D], pd[i % D], TB, TA, VB, VA, MB, MA,
           i >= 1, i >= 2, refill);
  }

  if constexpr (DOT) {
    const double bsum = block_sum<256>(dotacc, sred);
    if (threadIdx.x == 0) A.partials[t] = bsum;  // one slot per tile
  }
}

// Finishes the fused <v, K v>: CG step length (FIN_ALPHA) or a plain scalar.
struct KvDotFin {
  SolverState* st;
  double* out;
  int fin;
  int guarded;
  __device__ void operator()(const double* t) const {
    if (guarded && st->done) return;
    const double tot = t[0];
    if (fin == FIN_ALPHA) {
      st->pq = tot;
      if (!(tot > 0.0) || !finite_val(tot)) {
        st->done = 3;  // breakdown
        st->alpha = 0.0;
      } else {
        st->alpha = st->rz / tot;
      }
    } else {
      *out = tot;
    }
  }
};

// Planes in flight per block, and the deepest z chunk a block sweeps (fully unrolled).
// A deeper register ring measured slower on MI355X: its registers cost occupancy, and
// more resident blocks hide the load latency better than deeper prefetch per block.
template <typename T>
constexpr int kv_depth() { return sizeof(T) == 8 ? 1 : 2; }
template <typename T>
constexpr int kv_kzmax() { return sizeof(T) == 8 ? 24 : 16; }

template <typename T, typename XT, int PEN, bool DOT, bool PM, int EPI = 0>
__global__ __launch_bounds__(256) void kv_stream(KvArgs<T, XT> A) {
  kv_body<T, XT, PEN, DOT, PM, kv_depth<T>(), kv_kzmax<T>(), EPI>(A);
}

// Solver variant: skips the whole operator once the solve has finished, so batches of
// iterations can be enqueued without a host round trip per iteration.
template <typename T, typename XT, int PEN, bool DOT, bool PM, int EPI = 0>
__global__ __launch_bounds__(256) void kv_stream_guarded(KvArgs<T, XT> A) {
  if (A.st->done) return;
  kv_body<T, XT, PEN, DOT, PM, kv_depth<T>(), kv_kzmax<T>(), EPI>(A);
}

// ------------------------------------------------------------------ host side
struct KvGeom {
  int tiles_x, tiles_y, chunks_z, kz, ntiles, per_xcd, grid;
};

// Tiling of the node grid: (KBX-1) x (KBY-1) = 31 x 7 node columns per block and `kz`
// node planes per chunk.  A chunk of kz planes costs kz + 2 plane loads, so deep chunks
// waste less; but the whole grid runs in ceil(ntiles / resident) rounds of equal blocks,
// so the chunk count is chosen to minimise rounds * (kz + 2) for the number of blocks
// the GPU keeps resident (occupancy x CUs).
static KvGeom kv_geom_for(int nx, int ny, int nz, int resident, int kzmax) {
  KvGeom g;
  g.tiles_x = (nx + 1 + KBX - 2) / (KBX - 1);
  g.tiles_y = (ny + 1 + KBY - 2) / (KBY - 1);
  const int cols = g.tiles_x * g.tiles_y;
  const int planes = nz + 1;
  if (resident < 1) resident = 1;
  double best = 1e300;
  int best_kz = kzmax < planes ? kzmax : planes;
  for (int chunks = 1; chunks <= planes; ++chunks) {
    const int kz = (planes + chunks - 1) / chunks;
    if (kz > kzmax) continue;
    const int nch = (planes + kz - 1) / kz;
    const long long n = (long long)cols * nch;
    const long long rounds = (n + resident - 1) / resident;
    // Fewer blocks than resident slots leave CUs idle: count the idle fraction.
    const double fill = n >= resident ? 1.0 : (double)n / resident;
    const double cost = (double)rounds * (kz + 2) / fill;
    if (cost < best - 1e-9) {
      best = cost;
      best_kz = kz;
    }
  }
  g.kz = best_kz;
  g.chunks_z = (planes + g.kz - 1) / g.kz;
  g.ntiles = cols * g.chunks_z;
  g.per_xcd = (g.ntiles + 7) / 8;
  g.grid = g.per_xcd * 8;
  return g;
}

static int num_cus(const tosimp_ctx* c) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
      n < 1)
    n = 256;
  return n;
}

// Upper bound on the blocks any operator launch uses (for sizing partial sums).
int kv_num_blocks(const tosimp_ctx* c) {
  const int tx = (c->nx + 1 + KBX - 2) / (KBX - 1);
  const int ty = (c->ny + 1 + KBY - 2) / (KBY - 1);
  return tx * ty * (c->nz + 1);
}

template <typename T>
static KvC<T> kv_consts(const tosimp_ctx* c) {
  KvC<T> k;
  k.ad = (T)c->hc.ad; k.ao = (T)c->hc.ao; k.cs = (T)c->hc.cs; k.bd = (T)c->hc.bd;
  k.bo = (T)c->hc.bo; k.cd = (T)c->hc.cd; k.co = (T)c->hc.co; k.hg = (T)c->hc.hg;
  return k;
}

template <typename K>
static int resident_blocks(const tosimp_ctx* c, K kernel) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * num_cus(c);
}

template <typename T, typename XT, int PEN, bool DOT, bool PM, int EPI = 0>
static hipError_t kv_launch_v(const tosimp_ctx* c, KvArgs<T, XT> A, bool guarded,
                              int* tiles_out = nullptr) {
  auto kern = guarded ? kv_stream_guarded<T, XT, PEN, DOT, PM, EPI>
                      : kv_stream<T, XT, PEN, DOT, PM, EPI>;
  // Resident blocks per device and kernel instance, computed once (concurrent first calls
  // compute the same value; devices beyond the table are queried every time).
  constexpr int kDevs = 64;
  static std::atomic<int> resident[kDevs][2];
  int res = 0;
  const bool cached = c->device >= 0 && c->device < kDevs;
  if (cached) res = resident[c->device][guarded ? 1 : 0].load(std::memory_order_relaxed);
  if (res == 0) {
    res = resident_blocks(c, kern);
    if (cached) resident[c->device][guarded ? 1 : 0].store(res, std::memory_order_relaxed);
  }
  const KvGeom g = kv_geom_for(A.nx, A.ny, A.nz, res, kv_kzmax<T>());
  A.tiles_x = g.tiles_x; A.tiles_y = g.tiles_y; A.chunks_z = g.chunks_z; A.kz = g.kz;
  A.ntiles = g.ntiles; A.per_xcd = g.per_xcd;
  if (DOT && g.ntiles > c->ws.kv_part_cap) return hipErrorInvalidValue;  // partial slots
  kern<<<dim3(g.grid), dim3(256), 0, c->stream>>>(A);
  if (tiles_out) *tiles_out = g.ntiles;
  if (!DOT || A.fin == FIN_NONE) return hipGetLastError();  // partials left to the caller
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize_sum<1>(c->stream, A.partials, g.ntiles,
                                KvDotFin{A.st, A.out, A.fin, guarded ? 1 : 0});
}

template <typename T, typename XT, bool PM>
static hipError_t kv_launch_t(const tosimp_ctx* c, const XT* x, const T* v, T* y,
                              double* partials, SolverState* st, double* out, int fin,
                              bool guarded) {
  KvArgs<T, XT> A;
  A.v = v; A.y = y; A.x = x; A.mask = c->ws.mask;
  A.partials = partials; A.st = st; A.out = out; A.fin = fin;
  A.nx = c->nx; A.ny = c->ny; A.nz = c->nz;
  A.E0mEmin = (T)(c->E0 - c->Emin); A.Emin = (T)c->Emin; A.penal = (T)c->penal;
  A.k = kv_consts<T>(c);
  const bool p3 = c->penal == 3.0;
  const bool dot = fin != FIN_NONE;
  if (p3 && dot) return kv_launch_v<T, XT, kPenCube, true, PM>(c, A, guarded);
  if (p3) return kv_launch_v<T, XT, kPenCube, false, PM>(c, A, guarded);
  if (dot) return kv_launch_v<T, XT, kPenPow, true, PM>(c, A, guarded);
  return kv_launch_v<T, XT, kPenPow, false, PM>(c, A, guarded);
}

hipError_t kv_launch(const tosimp_ctx* c, int prec, int xdtype, const void* x,
                     const void* v, void* y, double* partials, SolverState* st,
                     double* out, int fin, bool guarded, bool premasked) {
  if (prec == TOSIMP_PREC_FP64) {
    if (xdtype == TOSIMP_F64) {
      if (premasked)
        return kv_launch_t<double, double, true>(c, (const double*)x, (const double*)v,
                                                 (double*)y, partials, st, out, fin, guarded);
      return kv_launch_t<double, double, false>(c, (const double*)x, (const double*)v,
                                                (double*)y, partials, st, out, fin, guarded);
    }
    return kv_launch_t<double, float, false>(c, (const float*)x, (const double*)v, (double*)y,
                                             partials, st, out, fin, guarded);
  }
  if (xdtype == TOSIMP_F64)
    return kv_launch_t<float, double, false>(c, (const double*)x, (const float*)v, (float*)y,
                                             partials, st, out, fin, guarded);
  if (premasked)
    return kv_launch_t<float, float, true>(c, (const float*)x, (const float*)v, (float*)y,
                                           partials, st, out, fin, guarded);
  return kv_launch_t<float, float, false>(c, (const float*)x, (const float*)v, (float*)y,
                                          partials, st, out, fin, guarded);
}

// Operator on a grid of the multigrid hierarchy: element moduli E given (no SIMP law),
// element stiffness scaled by kscale (K_E of an element of edge kscale h), fixed DOFs
// from `mask`, v zero on fixed DOFs.  Same kernel as the fine-grid operator; with st the
// launch returns at once when the solve has finished (guarded).
template <typename T>
static hipError_t kv_level_t(const tosimp_ctx* c, const T* E, const T* v, T* y, int nx,
                             int ny, int nz, const uint8_t* mask, double kscale,
                             const SolverState* st, const KvCheb* ch) {
  KvArgs<T, T> A{};
  A.v = v; A.y = y; A.x = E; A.mask = mask;
  A.st = const_cast<SolverState*>(st);
  A.fin = FIN_NONE;
  A.nx = nx; A.ny = ny; A.nz = nz;
  A.E0mEmin = T(1); A.Emin = T(0); A.penal = T(1);
  KvC<T> k;
  k.ad = (T)(kscale * c->hc.ad); k.ao = (T)(kscale * c->hc.ao);
  k.cs = (T)(kscale * c->hc.cs); k.bd = (T)(kscale * c->hc.bd);
  k.bo = (T)(kscale * c->hc.bo); k.cd = (T)(kscale * c->hc.cd);
  k.co = (T)(kscale * c->hc.co); k.hg = (T)(kscale * c->hc.hg);
  A.k = k;
  if (!ch || ch->mode == 0) return kv_launch_v<T, T, kPenModulus, false, true>(c, A, st != nullptr);
  A.eb = (const T*)ch->b;
  A.edd = (T*)ch->dd;
  A.edinv = (const T*)ch->dinv;
  A.ec0 = (T)ch->c0;
  A.ec1 = (T)ch->c1;
  A.ec2 = (T)ch->c2;
  if (ch->dot && (ch->mode == 1 || ch->mode == 2)) {
    A.partials = ch->dot;
    if (ch->mode == 1)
      return kv_launch_v<T, T, kPenModulus, true, true, 1>(c, A, st != nullptr, ch->dot_tiles);
    return kv_launch_v<T, T, kPenModulus, true, true, 2>(c, A, st != nullptr, ch->dot_tiles);
  }
  if (ch->mode == 1) return kv_launch_v<T, T, kPenModulus, false, true, 1>(c, A, st != nullptr);
  if (ch->mode == 3) return kv_launch_v<T, T, kPenModulus, false, true, 3>(c, A, st != nullptr);
  return kv_launch_v<T, T, kPenModulus, false, true, 2>(c, A, st != nullptr);
}

hipError_t kv_level_launch(const tosimp_ctx* c, int prec, const void* E, const void* v,
                           void* y, int nx, int ny, int nz, const uint8_t* mask,
                           double kscale, const SolverState* st, const KvCheb* ch) {
  if (ch && ch->mode != 0 && (y == v || ch->dd == v || ch->dd == y)) return hipErrorInvalidValue;
  if (prec == TOSIMP_PREC_FP64)
    return kv_level_t<double>(c, (const double*)E, (const double*)v, (double*)y, nx, ny, nz,
                              mask, kscale, st, ch);
  return kv_level_t<float>(c, (const float*)E, (const float*)v, (float*)y, nx, ny, nz, mask,
                           kscale, st, ch);
}

// ------------------------------------------------------------ Jacobi diagonal
// Every diagonal entry of K_E is the same value kd, so diag(K)_(n,c) = kd * sum of E
// over the (at most eight) elements around node n, identical for the three components.
template <typename XT, int PEN>
__global__ __launch_bounds__(256) void diag_node_kernel(const XT* __restrict__ x, int nx,
                                                        int ny, int nz, double kd,
                                                        double Emin, double E0mEmin,
                                                        double penal, double* dinv64,
                                                        float* dinv32, double* dfull,
                                                        float* dfull32,
                                                        const uint8_t* mask) {
  const int64_t NX1 = nx + 1, NY1 = ny + 1;
  const int64_t n_node = NX1 * NY1 * (nz + 1);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < n_node;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % NX1);
    const int64_t r = n / NX1;
    const int j = (int)(r % NY1);
    const int k = (int)(r / NY1);
    double s = 0.0;
    for (int dz = -1; dz <= 0; ++dz)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dx = -1; dx <= 0; ++dx) {
          const int ex = i + dx, ey = j + dy, ez = k + dz;
          if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
          const double xv = (double)x[ex + (int64_t)nx * (ey + (int64_t)ny * ez)];
          if (PEN == kPenModulus) {
            s += xv;
          } else {
            const double xp = PEN == kPenCube ? xv * xv * xv : (xv > 0.0 ? pow(xv, penal) : 0.0);
            s += Emin + xp * E0mEmin;
          }
        }
    const double d = kd * s;
    if (dinv64) dinv64[n] = 1.0 / d;
    if (dinv32) dinv32[n] = (float)(1.0 / d);
    if (dfull || dfull32) {
      const uint8_t m = mask[n];
      for (int c = 0; c < 3; ++c) {
        const double dc = ((m >> c) & 1) ? 1.0 : d;
        if (dfull) dfull[3 * n + c] = dc;
        if (dfull32) dfull32[3 * n + c] = (float)dc;
      }
    }
  }
}

template <typename XT>
static hipError_t diag_launch(const tosimp_ctx* c, const XT* x, double* dinv64,
                              float* dinv32, double* dfull, float* dfull32) {
  const bool p3 = c->penal == 3.0;
  dim3 grid(2048), block(256);
  if (p3)
    diag_node_kernel<XT, kPenCube><<<grid, block, 0, c->stream>>>(
        x, c->nx, c->ny, c->nz, c->kd, c->Emin, c->E0 - c->Emin, c->penal, dinv64, dinv32,
        dfull, dfull32, c->ws.mask);
  else
    diag_node_kernel<XT, kPenPow><<<grid, block, 0, c->stream>>>(
        x, c->nx, c->ny, c->nz, c->kd, c->Emin, c->E0 - c->Emin, c->penal, dinv64, dinv32,
        dfull, dfull32, c->ws.mask);
  return hipGetLastError();
}

hipError_t launch_diag_inv(const tosimp_ctx* c, const double* xphys, double* dinv64,
                           float* dinv32) {
  return diag_launch<double>(c, xphys, dinv64, dinv32, nullptr, nullptr);
}

hipError_t launch_diag_inv32(const tosimp_ctx* c, const float* x32, float* dinv32) {
  return diag_launch<float>(c, x32, nullptr, dinv32, nullptr, nullptr);
}

// Inverse Jacobi diagonal per node of a multigrid level: 1 / (kd kscale sum of E around
// the node), FP64 and / or FP32 (either may be null).
hipError_t launch_diag_level(const tosimp_ctx* c, const double* E, int nx, int ny, int nz,
                             double kscale, double* dinv64, float* dinv32) {
  diag_node_kernel<double, kPenModulus><<<dim3(2048), dim3(256), 0, c->stream>>>(
      E, nx, ny, nz, c->kd * kscale, 0.0, 1.0, 1.0, dinv64, dinv32, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_diag_full(const tosimp_ctx* c, int xdtype, const void* x, int dtype,
                            void* d) {
  double* d64 = dtype == TOSIMP_F64 ? (double*)d : nullptr;
  float* d32 = dtype == TOSIMP_F32 ? (float*)d : nullptr;
  if (xdtype == TOSIMP_F64) return diag_launch<double>(c, (const double*)x, nullptr, nullptr, d64, d32);
  return diag_launch<float>(c, (const float*)x, nullptr, nullptr, d64, d32);
}

}  // namespace tosimp
