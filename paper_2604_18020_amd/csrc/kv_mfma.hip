// Low-precision MFMA variant of the fused operator: y = K_c(x) v with FP32 storage, the
// 24x24 element contraction on BF16 or FP16 matrix cores (v_mfma_f32_16x16x32_{bf16,f16})
// and FP32 accumulation.
//
// Paper: Sec. "BF16 WMMA Tensor-Core Variant": K_E zero-padded to 32x32, element DOF
// vectors as the columns of the second operand, the SIMP scale applied after the
// product in FP32.  On gfx950 one 16x16x32 MFMA covers the whole padded K = 24 -> 32
// reduction, so a 16-element group needs two MFMAs (output rows 0-15 and 16-31).
//
// Structure: the owner-computes z sweep of the FP32/FP64 kernel on 16 x 16 element-column
// tiles (15 x 15 owned nodes per block, one node plane staged per step), with the
// element stage replaced by
//   1. each wave gathers, for 4 groups of 16 element columns, the 24 masked DOFs of each
//      element from the two LDS node planes in the MFMA B-operand lane layout
//      (lane l: element l % 16 of the group, DOFs 8 (l / 16) .. + 7), converts them,
//   2. two MFMAs with K_E (held in registers in the A-operand layout) produce the 24
//      element forces, scaled by E_e (and, for FP16, by a per-element power of two that
//      keeps the inputs in range), written to LDS,
//   3. each element thread accumulates its bottom-face forces with the previous layer's
//      top-face forces (nodal basis) and the four element columns around each node are
//      summed in a fixed order, as in the FP32/FP64 kernel.
#include "common.h"
#include "dev.h"

namespace tosimp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int MBX = 16, MBY = 16;

struct KvMArgs {
  const float* v;
  float* y;
  const void* x;
  int x_is_f32;
  const uint8_t* mask;
  const uint16_t* ke;  // [2 row tiles][64 lanes][8]: K_E bits in the A-operand layout
  const SolverState* st;
  int nx, ny, nz, tiles_x, tiles_y, kz, ntiles, per_xcd;
  float Emin, E0mEmin, penal;
  int p3;
};

// Round-to-nearest-even FP32 -> BF16 bits (inputs are finite).
__device__ __forceinline__ unsigned short f2bf(float f) {
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <bool F16, bool GUARD>
__global__ __launch_bounds__(256) void kv_mfma_kernel(KvMArgs A) {
  constexpr int NXL = MBX + 1, NYL = MBY + 1, ROW = 3 * NXL, NPV = ROW * NYL;
  constexpr int NLD = (NPV + 255) / 256;
  constexpr int NE = MBX * MBY;
  __shared__ float sv[2][NLD * 256];
  __shared__ float sf[24 * NE];
  __shared__ float sc[12 * NE];
  __shared__ float sE[NE];

  if (GUARD && A.st->done) return;
  const int bid = blockIdx.x;
  const int t = (bid & 7) * A.per_xcd + (bid >> 3);
  if (t >= A.ntiles) return;
  const int tx = t % A.tiles_x;
  const int rest = t / A.tiles_x;
  const int ty = rest % A.tiles_y;
  const int cz = rest / A.tiles_y;
  const int tid = threadIdx.x, lx = tid % MBX, ly = tid / MBX;
  const int lane = tid & 63, wave = tid >> 6;
  const int ex0 = tx * (MBX - 1) - 1, ey0 = ty * (MBY - 1) - 1;
  const int k0 = cz * A.kz;
  const int k1 = min(k0 + A.kz, A.nz + 1);
  const int NX1 = A.nx + 1;
  const long long plane = (long long)NX1 * (A.ny + 1);

  // K_E in the A-operand layout (row tiles 0-15 and 16-31).
  u16x8 ka0 = *reinterpret_cast<const u16x8*>(A.ke + (0 * 64 + lane) * 8);
  u16x8 ka1 = *reinterpret_cast<const u16x8*>(A.ke + (1 * 64 + lane) * 8);

  // Plane-load slots (flat LDS index = contiguous row segments of the vector).
  long long goff[NLD];
  int gcomp[NLD];
  bool gok[NLD];
#pragma unroll
  for (int s = 0; s < NLD; ++s) {
    const int f = tid + 256 * s;
    const int jl = f / ROW, w = f - jl * ROW, il = w / 3, c = w - il * 3;
    const int i = ex0 + il, j = ey0 + jl;
    gok[s] = f < NPV && i >= 0 && i <= A.nx && j >= 0 && j <= A.ny;
    goff[s] = gok[s] ? (long long)i + (long long)NX1 * j : 0;
    gcomp[s] = c;
  }
  float pv[NLD];
  auto load_plane = [&](int k) {
    const bool kok = k >= 0 && k <= A.nz;
#pragma unroll
    for (int s = 0; s < NLD; ++s) {
      pv[s] = 0.0f;
      if (gok[s] && kok) {
        const long long n = goff[s] + plane * k;
        const uint8_t m = A.mask[n];
        pv[s] = ((m >> gcomp[s]) & 1) ? 0.0f : A.v[3 * n + gcomp[s]];
      }
    }
  };
  const int ex = ex0 + lx, ey = ey0 + ly;
  const bool exy_ok = ex >= 0 && ex < A.nx && ey >= 0 && ey < A.ny;
  const long long ebase = exy_ok ? (long long)ex + (long long)A.nx * ey : 0;
  const long long elayer = (long long)A.nx * A.ny;
  const int ni = ex0 + lx + 1, nj = ey0 + ly + 1;
  const bool owner = lx < MBX - 1 && ly < MBY - 1 && ni <= A.nx && nj <= A.ny;
  const long long nbase = (long long)ni + (long long)NX1 * nj;

  float acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = 0.0f;

  load_plane(k0 - 1);
  for (int p = k0 - 1; p <= k1; ++p) {
    float* cur = sv[p & 1];
    const float* bot = sv[(p + 1) & 1];
#pragma unroll
    for (int s = 0; s < NLD; ++s) cur[tid + 256 * s] = pv[s];
    // modulus of this thread's element column at layer p - 1
    {
      const int ez = p - 1;
      float E = 0.0f;
      if (exy_ok && ez >= 0 && ez < A.nz) {
        const long long e = ebase + elayer * ez;
        const float xv = A.x_is_f32 ? ((const float*)A.x)[e] : (float)((const double*)A.x)[e];
        const float xp = A.p3 ? xv * xv * xv : (xv > 0.0f ? powf(xv, A.penal) : 0.0f);
        E = A.Emin + xp * A.E0mEmin;
      }
      sE[tid] = E;
    }
    __syncthreads();
    if (p < k1) load_plane(p + 1);

    if (p >= k0) {
      // ---- element forces of layer p - 1 on the matrix cores ----------------------
      const int q = lane >> 4;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int e = wave * 64 + g * 16 + (lane & 15);
        const int elx = e % MBX, ely = e / MBX;
        float vals[8];
        float mx = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int J = 8 * q + j;
          float val = 0.0f;
          if (J < 24) {
            const int a = J / 3, c = J - 3 * (J / 3);
            const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
            const float* pl = az ? cur : bot;
            val = pl[(ely + ay) * ROW + (elx + ax) * 3 + c];
          }
          vals[j] = val;
          mx = fmaxf(mx, fabsf(val));
        }
        float scale = 1.0f, unscale = 1.0f;
        if (F16) {
          mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
          mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
          if (mx > 0.0f) {
            const int ex2 = ilogbf(mx);
            scale = ldexpf(1.0f, -ex2);
            unscale = ldexpf(1.0f, ex2);
          }
        }
        f32x4 d0 = {0.0f, 0.0f, 0.0f, 0.0f}, d1 = {0.0f, 0.0f, 0.0f, 0.0f};
        if (F16) {
          f16x8 b;
#pragma unroll
          for (int j = 0; j < 8; ++j) b[j] = (_Float16)(vals[j] * scale);
          d0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, ka0), b, d0, 0, 0, 0);
          d1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, ka1), b, d1, 0, 0, 0);
        } else {
          u16x8 bb;
#pragma unroll
          for (int j = 0; j < 8; ++j) bb[j] = f2bf(vals[j]);
          d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ka0),
                                                       __builtin_bit_cast(bf16x8, bb), d0, 0, 0, 0);
          d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ka1),
                                                       __builtin_bit_cast(bf16x8, bb), d1, 0, 0, 0);
        }
        const float Es = sE[e] * unscale;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          sf[(4 * q + j) * NE + e] = d0[j] * Es;          // rows 0..15
          const int r1 = 16 + 4 * q + j;                   // rows 16..31 (24.. padding)
          if (r1 < 24) sf[r1 * NE + e] = d1[j] * Es;
        }
      }
    }
    __syncthreads();
    if (p >= k0) {
      // bottom-face forces (nodes a = 0..3) plus the previous layer's top face
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        const float R = acc[i] + sf[i * NE + tid];
        acc[i] = sf[(12 + i) * NE + tid];
        sc[i * NE + tid] = R;  // corner (ax, ay) = i / 3, component i % 3
      }
    }
    __syncthreads();
    if (p - 1 >= k0 && owner) {
      const long long n = nbase + plane * (p - 1);
      const uint8_t m = A.mask[n];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float yv = (sc[(9 + c) * NE + tid] + sc[(6 + c) * NE + tid + 1]) +
                   (sc[(3 + c) * NE + tid + MBX] + sc[(0 + c) * NE + tid + MBX + 1]);
        if ((m >> c) & 1) yv = A.v[3 * n + c];
        A.y[3 * n + c] = yv;
      }
    }
  }
}

hipError_t kv_mfma_launch(const tosimp_ctx* c, int prec, int xdtype, const void* x,
                          const float* v, float* y, SolverState* st, bool guarded) {
  KvMArgs A;
  A.v = v; A.y = y; A.x = x; A.x_is_f32 = xdtype == TOSIMP_F32; A.mask = c->ws.mask;
  A.ke = c->ws.ke_mfma + (prec == TOSIMP_PREC_FP16_MFMA ? 2 * 64 * 8 : 0);
  A.st = st;
  A.nx = c->nx; A.ny = c->ny; A.nz = c->nz;
  A.tiles_x = (c->nx + 1 + MBX - 2) / (MBX - 1);
  A.tiles_y = (c->ny + 1 + MBY - 2) / (MBY - 1);
  A.kz = 12;
  const int chunks = (c->nz + 1 + A.kz - 1) / A.kz;
  A.ntiles = A.tiles_x * A.tiles_y * chunks;
  A.per_xcd = (A.ntiles + 7) / 8;
  A.Emin = (float)c->Emin; A.E0mEmin = (float)(c->E0 - c->Emin); A.penal = (float)c->penal;
  A.p3 = c->penal == 3.0;
  dim3 grid(A.per_xcd * 8), block(256);
  const bool f16 = prec == TOSIMP_PREC_FP16_MFMA;
  if (f16 && guarded) kv_mfma_kernel<true, true><<<grid, block, 0, c->stream>>>(A);
  else if (f16) kv_mfma_kernel<true, false><<<grid, block, 0, c->stream>>>(A);
  else if (guarded) kv_mfma_kernel<false, true><<<grid, block, 0, c->stream>>>(A);
  else kv_mfma_kernel<false, false><<<grid, block, 0, c->stream>>>(A);
  return hipGetLastError();
}

}  // namespace tosimp
