// Learned preconditioner: 3D-convolutional U-Net on the node grid, trained on the GPU.
//
// Not in the paper (its Sec. "Path to Geometric Multigrid Integration" names stronger
// preconditioning as the way past Jacobi-PCG).  The network: 3 levels with base, 2 base
// and 4 base channels, inputs (r_x, r_y, r_z, nodal density), output a 3-component
// correction, LeakyReLU, no biases, nearest up-sampling and concatenated skips.  The
// layer list is the same as the oracle's.
//
// Tensors are channels-last: [voxel][channel], voxel = x + X (y + Y z) on a level's grid.
// Convolutions run on the matrix cores:
//   forward      Y[o][co]  = sum_{t, ci} W[co][t][ci] X[nbr(o, t)][ci]
//   data grad    dX[i][ci] = sum_{t, co} W[co][t][ci] dZ[o(i, t)][co]   (W stored as WT)
//   weight grad  dW[co][t][ci] = sum_o dZ[o][co] X[nbr(o, t)][ci]
// with K cut into chunks of 32 (one v_mfma_f32_16x16x32_bf16, or eight
// v_mfma_f32_16x16x4f32 for FP32 storage).  BF16 3x3x3 layers run as sweeps up the z
// axis with operand planes in an LDS ring and the weights in registers (conv3z_kernel,
// conv3s2_kernel); the stride-2 data gradient visits each voxel's parity-class taps only
// (conv_tgrad_s2_kernel); the remaining shapes use the LDS brick kernel or the implicit
// GEMM that gathers operands from global memory.  dZ = dY * leaky'(a) is formed on load
// from the layer's stored activation a (leaky ReLU preserves the sign, so a determines
// the slope).  Weight gradients are reduced per voxel chunk and the chunks summed in a
// fixed order (deterministic).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "dev.h"

namespace tosimp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr float kLeak = 0.01f;

// ---------------------------------------------------------------- element types
struct bf16_t {
  unsigned short bits;
};

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(bf16_t v) { return __uint_as_float((unsigned)v.bits << 16); }
template <typename ST>
__device__ __forceinline__ ST from_f(float f);
template <>
__device__ __forceinline__ float from_f<float>(float f) { return f; }
template <>
__device__ __forceinline__ bf16_t from_f<bf16_t>(float f) {
  const unsigned u = __float_as_uint(f);
  bf16_t r;
  r.bits = (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  return r;
}

// Eight consecutive values of a row (16 bytes for bf16, 32 for fp32).
template <typename ST>
struct Pack8;
template <>
struct Pack8<bf16_t> {
  u16x8 v;
  __device__ __forceinline__ void load(const bf16_t* p) { v = *reinterpret_cast<const u16x8*>(p); }
  __device__ __forceinline__ void store(bf16_t* p) const { *reinterpret_cast<u16x8*>(p) = v; }
  __device__ __forceinline__ void zero() { v = (u16x8){0, 0, 0, 0, 0, 0, 0, 0}; }
  __device__ __forceinline__ float get(int j) const { return __uint_as_float((unsigned)v[j] << 16); }
  __device__ __forceinline__ void set(int j, float f) { v[j] = from_f<bf16_t>(f).bits; }
};
template <>
struct Pack8<float> {
  float v[8];
  __device__ __forceinline__ void load(const float* p) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    const float4 b = *reinterpret_cast<const float4*>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
  __device__ __forceinline__ void store(float* p) const {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<float4*>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = 0.0f;
  }
  __device__ __forceinline__ float get(int j) const { return v[j]; }
  __device__ __forceinline__ void set(int j, float f) { v[j] = f; }
};

// acc += A (16 x 32) * B (32 x 16): lane (m or n = l % 16, q = l / 16) supplies eight
// consecutive k of the chunk, k = 8 q + j (the same assignment in A and B).
__device__ __forceinline__ void mma32(f32x4& acc, const Pack8<bf16_t>& a, const Pack8<bf16_t>& b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a.v),
                                                __builtin_bit_cast(bf16x8, b.v), acc, 0, 0, 0);
}
__device__ __forceinline__ void mma32(f32x4& acc, const Pack8<float>& a, const Pack8<float>& b) {
#pragma unroll
  for (int j = 0; j < 8; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[j], b.v[j], acc, 0, 0, 0);
}

struct Grid3 {
  int X, Y, Z;
  __host__ __device__ int n() const { return X * Y * Z; }
};

// ------------------------------------------------------------- convolution kernels
struct ConvArgs {
  const void* in;      // FWD: X [Vin][cin]; BWD: dY [Vout][cout] (gradient wrt the output)
  const void* act;     // BWD: the layer's stored output a [Vout][cout] (null: no activation)
  const void* w;       // FWD: W [cout][taps][cin]; BWD: WT [cin][taps][cout]
  void* out;           // FWD: Y [Vout][cout]; BWD: dX [Vin][cin]
  Grid3 gin, gout;     // input / output grids of the forward convolution
  int cin, cout;       // channels (multiples of 8 / 16) of the forward convolution
  int ksize, stride;
  int apply_act;       // FWD: leaky ReLU on the output
  // z-sweep forward with the up-sampling concatenation read in place (c1 > 0): operand
  // channels [0, c1) are the nearest up-sampling of `in` [Vcoarse][c1] on grid gcoarse,
  // channels [c1, cin) are `skip` [Vout][cin - c1].
  const void* skip;
  Grid3 gcoarse;
  int c1;
  // z-sweep weight rows: channel stride per tap wk (0: the sweep's K channels) and first
  // channel wc0 (a pass over part of K); FP32 partial result of a two-pass layer.
  int wk, wc0;
  float* part;
  // channels per coarse voxel (0: c1) and the first one read (a pass over part of them)
  int cstr, cc0;
  // first layer reading the residual in place: `in` = r (FP32, 3 per node), `skip` = the
  // nodal density (FP32); ||r||^2 from the 512 block partials npart, stored into *nout
  const double* npart;
  double* nout;
};

// One wave: RT x 16 "row" voxels of the result x a group of up to 64 result channels
// (blockIdx.y selects the group).  FWD rows are output voxels, K = taps x cin, result
// channels cout; BWD rows are input voxels, K = taps x cout, result channels cin.  Each
// K chunk of 32 loads the RT gathered A tiles and the weight tiles once and issues
// RT x (channels / 16) matrix-core products.  RT = 4 (each weight tile serving four voxel
// tiles) measured slower than RT = 1 on MI355X, RT = 2 the same, and so did issuing the
// loads of two to four K chunks before their products (12-70% slower): the gathered
// activation loads need the latency hiding of more waves more than weight reuse or
// in-wave overlap, which cost registers and with them waves.
constexpr int kConvRT = 1;

// BF16: the accumulators are held in ordinary VGPRs (no AGPR split), which lets eight
// (forward) or seven (data gradient) waves share a SIMD instead of six or five; the
// loads are latency-bound, so the extra waves shorten a forward pass by ~6%.  FP32
// needs more registers than that bound allows and keeps the compiler's choice.
template <typename ST, bool BWD>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(ST) == 2 ? (BWD ? 7 : 8) : 1)))
void conv_igemm_kernel(ConvArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const Grid3 rg = BWD ? a.gin : a.gout;   // grid of the rows
  const Grid3 og = BWD ? a.gout : a.gin;   // grid the operand A is read from
  const int nrow = rg.n();
  const int v0 = wave * 16 * kConvRT;
  if (v0 >= nrow) return;
  const int kch = BWD ? a.cout : a.cin;    // channels along K
  const int nres = BWD ? a.cin : a.cout;   // result channels
  const int taps = a.ksize * a.ksize * a.ksize;
  const int K = taps * kch;
  const int m = lane & 15, q = lane >> 4;
  const int pad = a.ksize / 2;
  const ST* in = (const ST*)a.in;
  const ST* act = (const ST*)a.act;
  const ST* w = (const ST*)a.w;
  const int cg = blockIdx.y * 64;  // first result channel of this group
  const int nblk = min(4, (nres - cg) / 16);
  int vx[kConvRT], vy[kConvRT], vz[kConvRT];
  bool vok[kConvRT];
#pragma unroll
  for (int r = 0; r < kConvRT; ++r) {
    const int v = v0 + 16 * r + m;
    vok[r] = v < nrow;
    vx[r] = v % rg.X;
    vy[r] = (v / rg.X) % rg.Y;
    vz[r] = v / (rg.X * rg.Y);
  }
  f32x4 acc[kConvRT][4];
#pragma unroll
  for (int r = 0; r < kConvRT; ++r)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[r][b] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};

  for (int k0 = 0; k0 < K; k0 += 32) {
    const int k = k0 + 8 * q;
    const bool kok = k < K;
    const int t = kok ? k / kch : 0, c = kok ? k - t * kch : 0;
    const int tx = t % a.ksize, ty = (t / a.ksize) % a.ksize, tz = t / (a.ksize * a.ksize);
    Pack8<ST> B[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      B[b].zero();
      if (b < nblk && kok) B[b].load(w + (long long)(cg + b * 16 + m) * K + k);
    }
#pragma unroll
    for (int r = 0; r < kConvRT; ++r) {
      Pack8<ST> A;
      A.zero();
      if (vok[r] && kok) {
        int sx, sy, sz;
        bool ok;
        if (!BWD) {
          sx = vx[r] * a.stride + tx - pad;
          sy = vy[r] * a.stride + ty - pad;
          sz = vz[r] * a.stride + tz - pad;
          ok = sx >= 0 && sx < og.X && sy >= 0 && sy < og.Y && sz >= 0 && sz < og.Z;
        } else {
          const int ux = vx[r] + pad - tx, uy = vy[r] + pad - ty, uz = vz[r] + pad - tz;
          ok = ux >= 0 && uy >= 0 && uz >= 0 && ux % a.stride == 0 && uy % a.stride == 0 &&
               uz % a.stride == 0;
          sx = ux / a.stride;
          sy = uy / a.stride;
          sz = uz / a.stride;
          ok = ok && sx < og.X && sy < og.Y && sz < og.Z;
        }
        if (ok) {
          const long long s = (long long)sx + (long long)og.X * (sy + (long long)og.Y * sz);
          A.load(in + s * kch + c);
          if (BWD && act) {
            Pack8<ST> av;
            av.load(act + s * kch + c);
#pragma unroll
            for (int j = 0; j < 8; ++j) A.set(j, A.get(j) * (av.get(j) > 0.0f ? 1.0f : kLeak));
          }
        }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b < nblk) mma32(acc[r][b], A, B[b]);
    }
  }
  ST* out = (ST*)a.out;
#pragma unroll
  for (int r = 0; r < kConvRT; ++r) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b < nblk) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = v0 + 16 * r + 4 * q + j;
          if (row < nrow) {
            float val = acc[r][b][j];
            if (!BWD && a.apply_act) val = val > 0.0f ? val : kLeak * val;
            out[(long long)row * nres + cg + b * 16 + m] = from_f<ST>(val);
          }
        }
      }
    }
  }
}

// Data gradient of a stride-2 3x3x3 convolution (its transpose): an operand voxel i
// receives, per axis, the taps whose i + 1 - t is even, t = 1 for even i and t = 0, 2 for
// odd i, so a voxel has 1 to 8 taps instead of 27.  A wave holds 16 operand voxels of one
// parity class along a row (x = 2 (16 b + m) + px) and up to 64 result channels; its K
// runs over the class's taps only, in ascending tap order and the cout channels in chunks
// of 32 within a tap: the order in which the implicit GEMM meets the same non-zero terms
// (it adds zeros for the others), so the sums agree with it.
template <typename ST>
__global__ __launch_bounds__(256) void conv_tgrad_s2_kernel(ConvArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const Grid3 gi = a.gin, go = a.gout;
  const int nxb = ((gi.X + 1) / 2 + 15) / 16;  // 16-voxel blocks of one x parity per row
  const int xb = wave % nxb;
  int rr = wave / nxb;
  const int px = rr & 1;
  rr >>= 1;
  const int y = rr % gi.Y, z = rr / gi.Y;
  if (z >= gi.Z) return;  // whole wave
  const int m = lane & 15, q = lane >> 4;
  const int kch = a.cout, nres = a.cin;  // K channels (dY), result channels (dX)
  const int cg = blockIdx.y * 64;
  const int nblk = min(4, (nres - cg) / 16);
  const int x = 2 * (16 * xb + m) + px;  // this lane's operand-row voxel
  const ST* dY = (const ST*)a.in;
  const ST* act = (const ST*)a.act;
  const ST* wt = (const ST*)a.w;          // WT [cin][27][cout]
  f32x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
  const int py = y & 1, pz = z & 1;
  for (int iz = 0; iz < 1 + pz; ++iz) {
    const int tz = pz ? 2 * iz : 1;
    const int oz = (z + 1 - tz) / 2;
    if (oz >= go.Z) continue;
    for (int iy = 0; iy < 1 + py; ++iy) {
      const int ty = py ? 2 * iy : 1;
      const int oy = (y + 1 - ty) / 2;
      if (oy >= go.Y) continue;
      for (int ix = 0; ix < 1 + px; ++ix) {
        const int tx = px ? 2 * ix : 1;
        const int ox = (x + 1 - tx) / 2;
        const bool ok = x < gi.X && ox < go.X;
        const int t = tx + 3 * ty + 9 * tz;
        const long long o = (long long)ox + (long long)go.X * (oy + (long long)go.Y * oz);
        for (int cc = 0; cc < kch; cc += 32) {
          Pack8<ST> A;
          A.zero();
          if (ok) {
            A.load(dY + o * kch + cc + 8 * q);
            if (act) {
              Pack8<ST> av;
              av.load(act + o * kch + cc + 8 * q);
#pragma unroll
              for (int j = 0; j < 8; ++j) A.set(j, A.get(j) * (av.get(j) > 0.0f ? 1.0f : kLeak));
            }
          }
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if (b < nblk) {
              Pack8<ST> B;
              B.load(wt + (long long)(cg + 16 * b + m) * (27 * kch) + t * kch + cc + 8 * q);
              mma32(acc[b], A, B);
            }
          }
        }
      }
    }
  }
  ST* out = (ST*)a.out;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (b < nblk) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int xr = 2 * (16 * xb + 4 * q + j) + px;
        if (xr < gi.X)
          out[((long long)xr + (long long)gi.X * (y + (long long)gi.Y * z)) * nres + cg + 16 * b + m] =
              from_f<ST>(acc[b][j]);
      }
    }
  }
}

// Stride-1 3x3x3 convolutions (forward, and the data gradient as the convolution with
// mirrored taps), tiled through LDS.  A block owns an output brick of 16 x 8 x 4 voxels
// (x fastest) and a group of up to 32 result channels.  For each slice of CS channels
// along K (32 bytes per voxel: 16 BF16 / 8 FP32) it stages in LDS the halo'd brick of
// 18 x 10 x 6 operand voxels (zero outside the grid; for the data gradient
// dZ = dY leaky'(a) is formed while staging) and the group's weights of the slice (27
// taps x CS).  Wave w computes the 8 rows (y) of z layer w: for each tap pair (tz, tx)
// it holds the weight tiles of the three y taps in registers and walks the ten brick
// rows rho once; the operand tile of row rho (16 consecutive voxels x CS channels, one
// 8-byte LDS read per lane, conflict-free) feeds output rows rho - oy(ty) for all three
// y taps, so each operand tile read serves up to three matrix-core products.  Products
// are 16 x 16 x 16 (BF16) or two 16 x 16 x 4 (FP32).  Summation order: channel slice, tz,
// tx, row, ty (fixed: deterministic).
constexpr int kBrX = 16, kBrY = 4, kBrZ = 4;                      // output brick
constexpr int kHaX = kBrX + 2, kHaY = kBrY + 2, kHaZ = kBrZ + 2;  // staged brick
constexpr int kHaVox = kHaX * kHaY * kHaZ;                        // 1080
constexpr int kC3Group = 32;                                      // result channels per block
constexpr int kC3SliceBytes = 32;                                 // K channel bytes per voxel and slice
constexpr int kC3WPad = 8;                                        // weight row pad (elements)

typedef short s16x4 __attribute__((ext_vector_type(4)));

// Four BF16 / two FP32 consecutive channels (8 bytes) of a lane's share of a K step.
template <typename ST>
struct Pk4;
template <>
struct Pk4<bf16_t> {
  s16x4 v;
  __device__ __forceinline__ void load(const bf16_t* p) { v = *reinterpret_cast<const s16x4*>(p); }
};
template <>
struct Pk4<float> {
  float2 v;
  __device__ __forceinline__ void load(const float* p) { v = *reinterpret_cast<const float2*>(p); }
};
// acc += A (16 x K) B (K x 16) for one K step of CS channels: lane (m or n, q) supplies
// the channels 4q..4q+3 (BF16) or 2q, 2q+1 (FP32, one per 16 x 16 x 4 product).
__device__ __forceinline__ void mma16(f32x4& acc, const Pk4<bf16_t>& a, const Pk4<bf16_t>& b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.v, b.v, acc, 0, 0, 0);
}
__device__ __forceinline__ void mma16(f32x4& acc, const Pk4<float>& a, const Pk4<float>& b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v.x, b.v.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v.y, b.v.y, acc, 0, 0, 0);
}

template <typename ST>
constexpr int conv3_cs() { return kC3SliceBytes / (int)sizeof(ST); }  // 16 BF16, 8 FP32
template <typename ST>
constexpr int conv3_wrow() { return 27 * conv3_cs<ST>() + kC3WPad; }
template <typename ST>
constexpr int conv3_lds_bytes() {
  return (kHaVox * conv3_cs<ST>() + kC3Group * conv3_wrow<ST>()) * (int)sizeof(ST);
}

template <typename ST, bool BWD>
__global__ __launch_bounds__(256) void conv3_lds_kernel(ConvArgs a) {
  constexpr int CS = conv3_cs<ST>(), WROW = conv3_wrow<ST>();
  constexpr int PV = CS / 8;       // 8-element staging pieces per voxel slice
  constexpr int LQ = CS / 4;       // elements per lane and K step
  __shared__ __attribute__((aligned(16))) unsigned char smem[conv3_lds_bytes<ST>()];
  ST* brick = reinterpret_cast<ST*>(smem);   // [1080 voxels][CS]
  ST* ws = brick + kHaVox * CS;               // [32 channels][27 taps x CS (+ pad)]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const Grid3 g = a.gout;  // stride 1: input and output grids agree
  const int nbx = (g.X + kBrX - 1) / kBrX, nby = (g.Y + kBrY - 1) / kBrY;
  const int bx = blockIdx.x % nbx, rest = blockIdx.x / nbx;
  const int by = rest % nby, bz = rest / nby;
  const int x0 = bx * kBrX, y0 = by * kBrY, z0 = bz * kBrZ;
  const int kch = BWD ? a.cout : a.cin;   // channels along K
  const int nres = BWD ? a.cin : a.cout;  // result channels
  const int Kw = 27 * kch;                // weight row length in global memory
  const int cg = blockIdx.y * kC3Group;
  const int ng = min(kC3Group, nres - cg), nblk = ng / 16;
  const int m = lane & 15, q = lane >> 4;
  const ST* in = (const ST*)a.in;
  const ST* act = (const ST*)a.act;
  const ST* w = (const ST*)a.w;

  f32x4 acc[kBrY][2];
#pragma unroll
  for (int r = 0; r < kBrY; ++r)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[r][b] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};

  for (int cs0 = 0; cs0 < kch; cs0 += CS) {
    // ---- stage the brick's slice of channels [cs0, cs0 + CS) and the group's weights:
    // each batch of loads is issued before its LDS stores (one latency per batch).
    constexpr int NBP = (kHaVox * PV + 255) / 256;        // brick pieces per thread
    constexpr int NWP = (kC3Group * 27 * PV + 255) / 256;  // weight pieces per thread
    {
      Pack8<ST> pb[NBP], pa[BWD ? NBP : 1];
#pragma unroll
      for (int i = 0; i < NBP; ++i) {
        const int idx = tid + 256 * i;
        const int vb = idx / PV, pc = idx - vb * PV;
        const int hx = vb % kHaX, hr = vb / kHaX, hy = hr % kHaY, hz = hr / kHaY;
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
        pb[i].zero();
        if (BWD) pa[i].zero();
        if (idx < kHaVox * PV && gx >= 0 && gx < g.X && gy >= 0 && gy < g.Y && gz >= 0 &&
            gz < g.Z) {
          const long long o =
              ((long long)gx + (long long)g.X * (gy + (long long)g.Y * gz)) * kch + cs0 + 8 * pc;
          pb[i].load(in + o);
          if (BWD && act) pa[i].load(act + o);
        }
      }
#pragma unroll
      for (int i = 0; i < NBP; ++i) {
        const int idx = tid + 256 * i;
        if (idx < kHaVox * PV) {
          if (BWD && act) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
              pb[i].set(j, pb[i].get(j) * (pa[i].get(j) > 0.0f ? 1.0f : kLeak));
          }
          const int vb = idx / PV, pc = idx - vb * PV;
          pb[i].store(brick + vb * CS + 8 * pc);
        }
      }
    }
    {
      Pack8<ST> pw[NWP];
#pragma unroll
      for (int i = 0; i < NWP; ++i) {
        const int idx = tid + 256 * i;
        const int n = idx / (27 * PV), rr = idx - n * (27 * PV), t = rr / PV, pc = rr - t * PV;
        pw[i].zero();
        if (n < ng) pw[i].load(w + (long long)(cg + n) * Kw + t * kch + cs0 + 8 * pc);
      }
#pragma unroll
      for (int i = 0; i < NWP; ++i) {
        const int idx = tid + 256 * i;
        const int n = idx / (27 * PV), rr = idx - n * (27 * PV), t = rr / PV, pc = rr - t * PV;
        if (n < ng) pw[i].store(ws + n * WROW + t * CS + 8 * pc);
      }
    }
    __syncthreads();
    // ---- taps: for each (tz, tx) the three y taps share every operand row tile
    for (int tz = 0; tz < 3; ++tz) {
      const int oz = BWD ? 2 - tz : tz;
      for (int tx = 0; tx < 3; ++tx) {
        const int ox = BWD ? 2 - tx : tx;
        Pk4<ST> B[3][2];
#pragma unroll
        for (int ty = 0; ty < 3; ++ty)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            if (b < nblk) B[ty][b].load(ws + (b * 16 + m) * WROW + (tx + 3 * ty + 9 * tz) * CS + LQ * q);
        const ST* arow = brick + ((m + ox) + kHaX * kHaY * (wv + oz)) * CS + LQ * q;
#pragma unroll
        for (int rho = 0; rho < kHaY; ++rho) {
          Pk4<ST> A;
          A.load(arow + kHaX * rho * CS);
#pragma unroll
          for (int ty = 0; ty < 3; ++ty) {
            // forward: output row rho - ty reads tap ty; data gradient: rho - (2 - ty)
            const int r = rho - (BWD ? 2 - ty : ty);
            if (r >= 0 && r < kBrY) {
#pragma unroll
              for (int b = 0; b < 2; ++b)
                if (b < nblk) mma16(acc[r][b], A, B[ty][b]);
            }
          }
        }
      }
    }
    __syncthreads();  // the next slice overwrites the brick and the weights
  }
  ST* out = (ST*)a.out;
  const int gz = z0 + wv;
#pragma unroll
  for (int r = 0; r < kBrY; ++r) {
    const int gy = y0 + r;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (b < nblk && gy < g.Y && gz < g.Z) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gx = x0 + 4 * q + j;
          if (gx < g.X) {
            float val = acc[r][b][j];
            if (!BWD && a.apply_act) val = val > 0.0f ? val : kLeak * val;
            const long long o = (long long)gx + (long long)g.X * (gy + (long long)g.Y * gz);
            out[o * nres + cg + b * 16 + m] = from_f<ST>(val);
          }
        }
      }
    }
  }
}

template <typename ST, bool BWD>
hipError_t launch_conv3_lds(hipStream_t s, const ConvArgs& a) {
  const int kch = BWD ? a.cout : a.cin, nres = BWD ? a.cin : a.cout;
  if (kch % conv3_cs<ST>() || nres % 16) return hipErrorInvalidValue;
  const Grid3 g = a.gout;
  const int nb = ((g.X + kBrX - 1) / kBrX) * ((g.Y + kBrY - 1) / kBrY) * ((g.Z + kBrZ - 1) / kBrZ);
  conv3_lds_kernel<ST, BWD><<<dim3(nb, (nres + kC3Group - 1) / kC3Group), 256, 0, s>>>(a);
  return hipGetLastError();
}

// Stride-1 3x3x3 convolutions in BF16 as a sweep up the z axis (forward, and the data
// gradient as the convolution with mirrored taps).  A block owns a 16 x 8 column of
// result voxels (x fastest), a chunk of result planes and 16 result channels
// (blockIdx.y); wave w holds result rows 2w and 2w + 1.  Operand planes pass through a
// ring of four LDS slots, each an 18 x 10 voxel window with all KCH channels: while the
// block forms result plane z from the slots of planes z - 1, z, z + 1, the loads of
// plane z + 2 are in flight; they are stored into the fourth slot after the products, and
// one barrier per plane separates the steps.  For each y offset oy of the taps, K = the
// nine (oz, ox) offsets x KCH channels is cut into matrix-core steps of 32 (one
// v_mfma_f32_16x16x32_bf16; a lane's eight K values lie in one tap; the last step is
// padded with zero weights), so the operand row tile that a lane reads from LDS for a
// window row feeds the products of every result row that uses that row (up to three oy).
// The weight tiles of the whole K (3 x S tiles of 16 channels x 32) stay in registers
// for the sweep.  Summation order per result: step, then oy (fixed, deterministic).
constexpr int kZX = 16, kZRW = 2, kZY = 4 * kZRW;                  // result tile, rows per wave
constexpr int kZPX = kZX + 2, kZPY = kZY + 2, kZPlane = kZPX * kZPY;  // 18 x 10 window
constexpr int kZSlots = 4;

template <int KCH>
constexpr int conv3z_steps() { return (9 * KCH + 31) / 32; }
// LDS voxel pitch in elements: an odd number of 16-byte units, so the 16-byte operand
// reads of consecutive voxels (one per lane) fall in distinct banks.
template <int KCH>
constexpr int conv3z_vs() { return (KCH / 8) % 2 ? KCH : KCH + 8; }
template <int KCH>
constexpr int conv3z_lds_bytes() { return kZSlots * kZPlane * conv3z_vs<KCH>() * 2; }

struct Conv3zGeom {
  int tiles_x, tiles_y, kz, nblk, per_xcd;
};

// Weight piece of step s, y offset oy, result channel n and lane quarter q (8 K values):
// K index 32 s + 8 q within oy's group; zero past the nine (oz, ox) offsets.
template <int KCH, bool BWD>
__device__ __forceinline__ void conv3z_wload(Pack8<bf16_t>& B, const bf16_t* w, int row, int oy,
                                             int s, int q, int wk, int wc0);

// The block's weight tiles (16 result channels from row0, 3 oy x S steps) fetched once
// per block into the LDS area `stage` (before any operand plane is staged there), then
// into every wave's registers; the block's threads share the global loads.
template <int KCH, bool BWD, int NT>
__device__ __forceinline__ void conv3z_weights(Pack8<bf16_t> (&Bw)[3][conv3z_steps<KCH>()],
                                               const bf16_t* w, int row0, bf16_t* stage,
                                               int wk = KCH, int wc0 = 0) {
  constexpr int S = conv3z_steps<KCH>();
  constexpr int NW = 3 * S * 16 * 4;  // 16-byte pieces
  constexpr int NI = (NW + NT - 1) / NT;
  const int tid = threadIdx.x, m = tid & 15, q = (tid & 63) >> 4;
  Pack8<bf16_t> t[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int idx = tid + NT * i;
    const int qq = idx & 3, n = (idx >> 2) & 15, rs = idx >> 6;
    t[i].zero();
    if (idx < NW) conv3z_wload<KCH, BWD>(t[i], w, row0 + n, rs / S, rs % S, qq, wk, wc0);
  }
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int idx = tid + NT * i;
    if (idx < NW) t[i].store(stage + 8 * idx);  // piece idx = ((oy S + s) 16 + n) 4 + qq
  }
  __syncthreads();
#pragma unroll
  for (int oy = 0; oy < 3; ++oy)
#pragma unroll
    for (int s = 0; s < S; ++s) Bw[oy][s].load(stage + 8 * ((((oy * S + s) * 16 + m) << 2) + q));
  __syncthreads();  // the operand planes overwrite the staging area next
}

// Weight rows hold 27 taps of wk channels; the sweep's K channels start at wc0.
template <int KCH, bool BWD>
__device__ __forceinline__ void conv3z_wload(Pack8<bf16_t>& B, const bf16_t* w, int row, int oy,
                                             int s, int q, int wk, int wc0) {
  const int kk = 32 * s + 8 * q;
  const int c = kk / KCH, ch = kk - c * KCH;
  B.zero();
  if (c < 9) {
    const int oz = c / 3, ox = c - 3 * oz;
    const int t = ox + 3 * oy + 9 * oz;
    B.load(w + (long long)row * (27 * wk) + (BWD ? 26 - t : t) * wk + wc0 + ch);
  }
}

typedef unsigned int u32x4z __attribute__((ext_vector_type(4)));
constexpr int kZOOB = 0x7FFFFFF0;  // buffer offset past any range: loads return 0, stores drop

__device__ __forceinline__ __amdgpu_buffer_rsrc_t conv3z_rsrc(const void* base, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}

// Planes issued a whole step before they are stored into LDS (two register sets, steps in
// pairs), or at the start of the step that stores them.
template <int KCH>
constexpr bool conv3z_prefetch() { return KCH == 32; }

// Waves per SIMD the register budget is set for (forward KCH 16: 128 VGPRs, four waves;
// the data gradient also holds the stored activation of the planes in flight).
template <int KCH, bool BWD>
constexpr int conv3z_waves() {
  return KCH <= 8 ? 5 : KCH <= 16 ? (BWD ? 3 : 4) : KCH <= 48 ? 2 : 1;
}

// OUTM 0: BF16 result (with the activation); 1: FP32 partial sums into a.part (no
// activation); 2: the FP32 partial in a.part added first, then the activation and the
// BF16 result; 3: the partial added first and stored back (passes of a layer whose K is
// split, in a fixed order).
// INP: the first layer of the preconditioner, its operand (r at unit RMS per DOF, the
// nodal density, four zero channels) formed while staging from r and the density.
template <int KCH, bool BWD, int C1 = 0, int OUTM = 0, bool INP = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(conv3z_waves<KCH, BWD>())))
void conv3z_kernel(ConvArgs a, Conv3zGeom gm) {
  static_assert(C1 == 0 || (!BWD && C1 % 8 == 0 && C1 <= KCH), "concatenated operand: forward");
  static_assert(OUTM == 0 || !BWD, "split K: forward");
  static_assert(!INP || (KCH == 8 && !BWD && C1 == 0 && OUTM == 0), "input layer: 8 channels");
  constexpr int S = conv3z_steps<KCH>();
  constexpr int PV = KCH / 8;                     // 16-byte pieces per voxel
  constexpr int NP = (kZPlane * PV + 255) / 256;  // plane pieces per thread
  constexpr int VS = conv3z_vs<KCH>();
  extern __shared__ __attribute__((aligned(16))) unsigned char zsm[];
  bf16_t* planes = reinterpret_cast<bf16_t*>(zsm);   // [4 slots][180 voxels][VS]
  const int blin = (blockIdx.x & 7) * gm.per_xcd + (blockIdx.x >> 3);
  if (blin >= gm.nblk) return;  // whole block
  const Grid3 g = a.gout;       // stride 1: operand and result grids agree
  const int bx = blin % gm.tiles_x, rest = blin / gm.tiles_x;
  const int by = rest % gm.tiles_y, bz = rest / gm.tiles_y;
  const int x0 = bx * kZX, y0 = by * kZY;
  const int za = bz * gm.kz, zb = min(za + gm.kz, g.Z);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int nres = BWD ? a.cin : a.cout;
  const int cg = blockIdx.y * 16;
  const long long nvox = (long long)g.X * g.Y * g.Z;
  // Operand (and stored activation) and result tensors as buffer resources: lanes outside
  // the grid use an offset past the range, so loads return zeros and stores are dropped
  // without branches (the wait for a plane's loads then has a fixed count).
  constexpr int C2 = KCH - C1;  // channels read at the voxel itself
  const Grid3 gc = a.gcoarse;
  const int cstr = a.cstr ? a.cstr : C1;  // channels per coarse voxel
  const __amdgpu_buffer_rsrc_t rin =
      INP ? conv3z_rsrc(a.in, nvox * 12)
          : C1 ? conv3z_rsrc(a.in, (long long)gc.X * gc.Y * gc.Z * cstr * 2)
               : conv3z_rsrc(a.in, nvox * KCH * 2);
  const __amdgpu_buffer_rsrc_t ract = INP  ? conv3z_rsrc(a.skip, nvox * 4)
                                      : C1 ? conv3z_rsrc(a.skip, nvox * C2 * 2)
                                           : conv3z_rsrc(BWD ? a.act : a.in, nvox * KCH * 2);
  const __amdgpu_buffer_rsrc_t rout = conv3z_rsrc(a.out, nvox * nres * 2);
  const __amdgpu_buffer_rsrc_t rpart = conv3z_rsrc(a.part, OUTM ? nvox * nres * 4 : 0);
  const bf16_t* w = (const bf16_t*)a.w;

  // Plane pieces of this thread: window voxel and byte offset in the plane.  With C1 the
  // pieces of the up-sampled channels of every window voxel come first (NC of them, byte
  // offsets in the coarse plane), then those of the skipped channels, so only the one
  // register slot straddling the boundary needs both loads.
  constexpr int NC = kZPlane * C1 / 8;
  int pvox[NP], pgo[NP];
  bool pok[NP], pco[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int idx = tid + 256 * i;
    pco[i] = idx < NC;
    const int k = pco[i] ? idx : idx - NC;
    const int pw = pco[i] ? C1 / 8 : (C2 ? C2 / 8 : 1);  // pieces per voxel in this part
    const int vb = k / pw, pc = k - vb * pw;
    const int ch = pco[i] ? 8 * pc : C1 + 8 * pc;
    const int hx = vb % kZPX, hy = vb / kZPX;
    const int gx = x0 - 1 + hx, gy = y0 - 1 + hy;
    pok[i] = idx < kZPlane * PV && gx >= 0 && gx < g.X && gy >= 0 && gy < g.Y;
    pvox[i] = idx < kZPlane * PV ? vb * VS + ch : -1;
    if (INP)
      pgo[i] = gx + g.X * gy;  // node index in the plane
    else if (C1 == 0)
      pgo[i] = ((gx + g.X * gy) * KCH + ch) * 2;
    else if (pco[i])
      pgo[i] = (((gx >> 1) + gc.X * (gy >> 1)) * cstr + a.cc0 + ch) * 2;
    else
      pgo[i] = ((gx + g.X * gy) * C2 + ch - C1) * 2;
  }
  const int pstride = INP ? g.X * g.Y : g.X * g.Y * C2 * 2;  // bytes (INP: nodes) per plane
  const int cstride = gc.X * gc.Y * cstr * 2;      // bytes per coarse plane (C1 > 0)
  float inv = 0.0f;  // INP: sqrt(n_dof) / ||r||
  auto plane_load = [&](Pack8<bf16_t>* pb, Pack8<bf16_t>* pa, int gz) {
    const bool zok = gz >= 0 && gz < g.Z;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if constexpr (INP) {
        const bool ok = zok && pok[i];
        const int nd = pgo[i] + gz * pstride;
        const auto rv = __builtin_amdgcn_raw_buffer_load_b96(rin, ok ? 12 * nd : kZOOB, 0, 0);
        const unsigned dv = __builtin_amdgcn_raw_buffer_load_b32(ract, ok ? 4 * nd : kZOOB, 0, 0);
        pb[i].zero();
        pb[i].set(0, __uint_as_float(rv[0]) * inv);
        pb[i].set(1, __uint_as_float(rv[1]) * inv);
        pb[i].set(2, __uint_as_float(rv[2]) * inv);
        pb[i].set(3, __uint_as_float(dv));
      } else if constexpr (C1 == 0) {
        const int off = zok && pok[i] ? pgo[i] + gz * pstride : kZOOB;
        pb[i].v = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(rin, off, 0, 0));
        if (BWD)
          pa[i].v =
              __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(ract, off, 0, 0));
      } else if (256 * i + 255 < NC) {  // up-sampled channels only
        const int offc = zok && pok[i] ? pgo[i] + (gz >> 1) * cstride : kZOOB;
        pb[i].v = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(rin, offc, 0, 0));
      } else if (256 * i >= NC) {  // skipped channels only
        const int offs = zok && pok[i] ? pgo[i] + gz * pstride : kZOOB;
        pb[i].v = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(ract, offs, 0, 0));
      } else {  // both issued, the one not holding the piece out of range (it returns 0)
        const int offc = zok && pok[i] && pco[i] ? pgo[i] + (gz >> 1) * cstride : kZOOB;
        const int offs = zok && pok[i] && !pco[i] ? pgo[i] + gz * pstride : kZOOB;
        pb[i].v = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(rin, offc, 0, 0) |
                                                __builtin_amdgcn_raw_buffer_load_b128(ract, offs, 0, 0));
      }
    }
  };
  auto plane_store = [&](Pack8<bf16_t>* pb, Pack8<bf16_t>* pa, int gz) {
    bf16_t* dst = planes + ((gz + 4) & 3) * (kZPlane * VS);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (pvox[i] >= 0) {
        if (BWD) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            pb[i].set(j, pb[i].get(j) * (pa[i].get(j) > 0.0f ? 1.0f : kLeak));
        }
        pb[i].store(dst + pvox[i]);
      }
    }
  };

  // Weights: in registers for the sweep.
  static_assert(3 * S * 16 * 32 <= kZSlots * kZPlane * VS, "weight staging fits the slots");
  Pack8<bf16_t> Bw[3][S];
  conv3z_weights<KCH, BWD, 256>(Bw, w, cg, planes, a.wk ? a.wk : KCH, a.wc0);
  if constexpr (INP) {
    // ||r||^2 from its 512 block partials, added in one fixed order by every block (each
    // thread two, then a tree in LDS, in the plane slots before any plane is staged)
    double* red = reinterpret_cast<double*>(zsm);
    red[tid] = a.npart[2 * tid] + a.npart[2 * tid + 1];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    const double tot = red[0];
    if (blin == 0 && blockIdx.y == 0 && tid == 0) *a.nout = tot;
    inv = (float)(sqrt(3.0 * (double)nvox) / sqrt(fmax(tot, 1e-300)));
    __syncthreads();  // the planes overwrite the reduction area next
  }
  {  // planes za - 1, za, za + 1
    Pack8<bf16_t> p0[NP], a0[BWD ? NP : 1], p1[NP], a1[BWD ? NP : 1], p2[NP], a2[BWD ? NP : 1];
    plane_load(p0, a0, za - 1);
    plane_load(p1, a1, za);
    plane_load(p2, a2, za + 1);
    plane_store(p0, a0, za - 1);
    plane_store(p1, a1, za);
    plane_store(p2, a2, za + 1);
  }
  // With PF, two register sets for planes in flight: the loads of plane z + 3 are issued
  // at step z and stored into LDS at step z + 1, so each plane has a whole step to arrive.
  constexpr bool PF = conv3z_prefetch<KCH>();
  Pack8<bf16_t> r0[NP], ra0[BWD ? NP : 1], r1[PF ? NP : 1], ra1[PF && BWD ? NP : 1];
  if (PF) plane_load(r0, ra0, za + 2);
  __syncthreads();

  // Operand offset of this lane's window row 2 wv, voxel m, within a slot; per step s the
  // lane's (oz, ox, channel) follow from 32 s + 8 q (formed where used: few registers).
  const int lbase = ((kZRW * wv) * kZPX + m) * VS;
  // Result offset (bytes) of this lane's first voxel in a plane.
  const int gx0 = x0 + 4 * q, gy0 = y0 + kZRW * wv;
  const int obase = ((gx0 + g.X * gy0) * nres + cg + m) * 2;
  const int ostride = g.X * g.Y * nres * 2;  // bytes per result plane
  // Step z: issue plane z + 3 into `ld`, form result plane z, store plane z + 2 (issued
  // the step before, in `st`) into its slot, barrier.  Steps run in pairs; the second of
  // a pair past the chunk stores nothing.  Every load and store is issued unconditionally.
  auto step = [&](int z, Pack8<bf16_t>* ld, Pack8<bf16_t>* lda, Pack8<bf16_t>* st,
                  Pack8<bf16_t>* sta) {
    if (PF)
      plane_load(ld, lda, z + 3);
    else
      plane_load(st, sta, z + 2);
    const bool zin = z < zb;
    float pin[kZRW][4];  // the first pass's FP32 sums (OUTM 2), issued with the planes
    if constexpr (OUTM >= 2) {
#pragma unroll
      for (int r = 0; r < kZRW; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool ok = zin && gx0 + j < g.X && gy0 + r < g.Y;
          const int off = ok ? 2 * (obase + (j + g.X * r) * (nres * 2) + z * ostride) : kZOOB;
          pin[r][j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rpart, off, 0, 0));
        }
    }
    f32x4 acc[kZRW];
#pragma unroll
    for (int r = 0; r < kZRW; ++r) acc[r] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    const int sb0 = ((z + 3) & 3) * (kZPlane * VS), sb1 = ((z + 4) & 3) * (kZPlane * VS),
              sb2 = ((z + 5) & 3) * (kZPlane * VS);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int kk = 32 * s + 8 * q;
      int c = kk / KCH;
      const int ch = kk - c * KCH;
      if (c >= 9) c = 0;  // zero weights: any finite operand
      const int oz = c / 3, ox = c - 3 * oz;
      const bf16_t* ab = planes + (oz == 0 ? sb0 : oz == 1 ? sb1 : sb2) + lbase + ox * VS + ch;
#pragma unroll
      for (int rho = 0; rho < kZRW + 2; ++rho) {
        Pack8<bf16_t> A;
        A.load(ab + rho * (kZPX * VS));
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
          const int r = rho - oy;
          if (r >= 0 && r < kZRW) mma32(acc[r], A, Bw[oy][s]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kZRW; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = zin && gx0 + j < g.X && gy0 + r < g.Y;
        const int off = ok ? obase + (j + g.X * r) * (nres * 2) + z * ostride : kZOOB;
        if constexpr (OUTM == 1 || OUTM == 3) {
          const float v = OUTM == 3 ? pin[r][j] + acc[r][j] : acc[r][j];
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rpart, ok ? 2 * off : kZOOB,
                                                0, 0);
        } else {
          float val = OUTM == 2 ? pin[r][j] + acc[r][j] : acc[r][j];
          if (!BWD && a.apply_act) val = val > 0.0f ? val : kLeak * val;
          __builtin_amdgcn_raw_buffer_store_b16(from_f<bf16_t>(val).bits, rout, off, 0, 0);
        }
      }
    plane_store(st, sta, z + 2);
    __syncthreads();
  };
  if constexpr (PF) {
    for (int z = za; z < zb; z += 2) {  // in pairs: the register sets alternate
      step(z, r1, ra1, r0, ra0);
      step(z + 1, r0, ra0, r1, ra1);
    }
  } else {
    for (int z = za; z < zb; ++z) step(z, r0, ra0, r0, ra0);
  }
}

// Chunks of result planes: a chunk of kz planes loads stride (kz - 1) + 3 operand planes,
// and the grid runs in ceil(blocks / resident) rounds, so kz minimises rounds x planes
// loaded (idle slots of a partial first round counted as lost).  Result tiles tx x ty.
static Conv3zGeom conv3z_geom(const Grid3& g, int groups, int resident, int tx = kZX,
                              int ty = kZY, int stride = 1) {
  Conv3zGeom gm;
  gm.tiles_x = (g.X + tx - 1) / tx;
  gm.tiles_y = (g.Y + ty - 1) / ty;
  const long long cols = (long long)gm.tiles_x * gm.tiles_y * groups;
  if (resident < 1) resident = 1;
  double best = 1e300;
  int best_kz = g.Z;
  for (int chunks = 1; chunks <= g.Z; ++chunks) {
    const int kz = (g.Z + chunks - 1) / chunks;
    const int nch = (g.Z + kz - 1) / kz;
    const long long n = cols * nch;
    const long long rounds = (n + resident - 1) / resident;
    const double fill = n >= resident ? 1.0 : (double)n / resident;
    const double cost = (double)rounds * (stride * (kz - 1) + 3) / fill;
    if (cost < best - 1e-9) {
      best = cost;
      best_kz = kz;
    }
  }
  gm.kz = best_kz;
  gm.nblk = gm.tiles_x * gm.tiles_y * ((g.Z + gm.kz - 1) / gm.kz);
  gm.per_xcd = (gm.nblk + 7) / 8;
  return gm;
}

// Blocks per CU x CUs for a kernel instance with `smem` bytes of dynamic LDS (which it is
// allowed), computed once per instance (concurrent first calls compute the same value).
template <typename K>
static hipError_t conv_resident(K kern, int smem, std::atomic<int>& once, int* resident) {
  int r = once.load(std::memory_order_relaxed);
  if (r == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, smem);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, smem) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    r = per_cu * cus;
    once.store(r, std::memory_order_relaxed);
  }
  *resident = r;
  return hipSuccess;
}

template <int KCH, bool BWD, int C1 = 0, int OUTM = 0, bool INP = false>
hipError_t launch_conv3z_t(hipStream_t s, const ConvArgs& a) {
  constexpr int smem = conv3z_lds_bytes<KCH>();
  static_assert(!INP || smem >= 256 * 8, "the norm's reduction fits the plane slots");
  auto kern = conv3z_kernel<KCH, BWD, C1, OUTM, INP>;
  static std::atomic<int> once{0};
  int resident = 0;
  const hipError_t e = conv_resident(kern, smem, once, &resident);
  if (e != hipSuccess) return e;
  const int nres = BWD ? a.cin : a.cout;
  const Conv3zGeom gm = conv3z_geom(a.gout, nres / 16, resident);
  kern<<<dim3(8 * gm.per_xcd, nres / 16), 256, smem, s>>>(a, gm);
  return hipGetLastError();
}

// Stride-2 3x3x3 convolutions in BF16 (the encoder's down-sampling layers, forward) as a
// z-sweep: result plane z reads operand planes 2z - 1, 2z, 2z + 1.  A block owns a 16 x 4
// column of result voxels, a chunk of result planes and 16 result channels; wave w holds
// result row w.  Operand planes pass through a ring of five LDS slots (33 x 9 voxel
// windows with all KCH channels): step z issues the loads of planes 2z + 2 and 2z + 3,
// forms result plane z from the slots of planes 2z - 1 .. 2z + 1 (lane m reads window
// voxel 2m + ox), stores the two new planes into their slots and ends with one barrier.
// K steps and register-held weights as in the stride-1 sweep; one accumulator per y
// offset, added in the order oy = 0, 1, 2.
constexpr int kSX = 16, kSY = 4;                                                // result tile
constexpr int kSPX = 2 * kSX + 1, kSPY = 2 * kSY + 1, kSPlane = kSPX * kSPY;  // 33 x 9 window
constexpr int kSSlots = 5;

template <int KCH>
constexpr int conv3s2_lds_bytes() { return kSSlots * kSPlane * KCH * 2; }

template <int KCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KCH <= 16 ? 3 : 1)))
void conv3s2_kernel(ConvArgs a, Conv3zGeom gm) {
  constexpr int S = conv3z_steps<KCH>();
  constexpr int PV = KCH / 8;                      // 16-byte pieces per voxel
  constexpr int NP = (kSPlane * PV + 255) / 256;   // pieces per thread and plane
  constexpr int SLOT = kSPlane * KCH;              // elements per slot
  extern __shared__ __attribute__((aligned(16))) unsigned char zsm[];
  bf16_t* planes = reinterpret_cast<bf16_t*>(zsm);  // [5 slots][297 voxels][KCH]
  const int blin = (blockIdx.x & 7) * gm.per_xcd + (blockIdx.x >> 3);
  if (blin >= gm.nblk) return;  // whole block
  const Grid3 gi = a.gin, g = a.gout;
  const int bx = blin % gm.tiles_x, rest = blin / gm.tiles_x;
  const int by = rest % gm.tiles_y, bz = rest / gm.tiles_y;
  const int x0 = bx * kSX, y0 = by * kSY;
  const int za = bz * gm.kz, zb = min(za + gm.kz, g.Z);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int nres = a.cout;
  const int cg = blockIdx.y * 16;
  const __amdgpu_buffer_rsrc_t rin = conv3z_rsrc(a.in, (long long)gi.n() * KCH * 2);
  const __amdgpu_buffer_rsrc_t rout = conv3z_rsrc(a.out, (long long)g.n() * nres * 2);

  int pvox[NP], pgo[NP];
  bool pok[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int idx = tid + 256 * i;
    const int vb = idx / PV, pc = idx - vb * PV;
    const int hx = vb % kSPX, hy = vb / kSPX;
    const int gx = 2 * x0 - 1 + hx, gy = 2 * y0 - 1 + hy;
    pok[i] = idx < kSPlane * PV && gx >= 0 && gx < gi.X && gy >= 0 && gy < gi.Y;
    pvox[i] = idx < kSPlane * PV ? vb * KCH + 8 * pc : -1;
    pgo[i] = ((gx + gi.X * gy) * KCH + 8 * pc) * 2;
  }
  const int pstride = gi.X * gi.Y * KCH * 2;  // bytes per operand plane
  auto plane_load = [&](Pack8<bf16_t>* pb, int gz) {
    const bool zok = gz >= 0 && gz < gi.Z;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int off = zok && pok[i] ? pgo[i] + gz * pstride : kZOOB;
      pb[i].v = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(rin, off, 0, 0));
    }
  };
  auto plane_store = [&](const Pack8<bf16_t>* pb, int gz) {  // gz >= -1
    bf16_t* dst = planes + ((gz + kSSlots) % kSSlots) * SLOT;
#pragma unroll
    for (int i = 0; i < NP; ++i)
      if (pvox[i] >= 0) pb[i].store(dst + pvox[i]);
  };

  static_assert(3 * S * 16 * 32 <= kSSlots * SLOT, "weight staging fits the slots");
  Pack8<bf16_t> Bw[3][S];
  conv3z_weights<KCH, false, 256>(Bw, (const bf16_t*)a.w, cg, planes, KCH, 0);
  {  // planes 2 za - 1, 2 za, 2 za + 1
    Pack8<bf16_t> p0[NP], p1[NP], p2[NP];
    plane_load(p0, 2 * za - 1);
    plane_load(p1, 2 * za);
    plane_load(p2, 2 * za + 1);
    plane_store(p0, 2 * za - 1);
    plane_store(p1, 2 * za);
    plane_store(p2, 2 * za + 1);
  }
  __syncthreads();

  const int lbase = ((2 * wv) * kSPX + 2 * m) * KCH;  // window row 2 wv, voxel 2 m
  const int gx0 = x0 + 4 * q, gy = y0 + wv;
  const int obase = ((gx0 + g.X * gy) * nres + cg + m) * 2;
  const int ostride = g.X * g.Y * nres * 2;
  for (int z = za; z < zb; ++z) {
    Pack8<bf16_t> pa[NP], pb[NP];
    plane_load(pa, 2 * z + 2);
    plane_load(pb, 2 * z + 3);
    f32x4 acc[3];
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) acc[oy] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    const int sb0 = ((2 * z - 1 + kSSlots) % kSSlots) * SLOT;
    const int sb1 = ((2 * z + kSSlots) % kSSlots) * SLOT;
    const int sb2 = ((2 * z + 1 + kSSlots) % kSSlots) * SLOT;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int kk = 32 * s + 8 * q;
      int c = kk / KCH;
      const int ch = kk - c * KCH;
      if (c >= 9) c = 0;  // zero weights: any finite operand
      const int oz = c / 3, ox = c - 3 * oz;
      const bf16_t* ab = planes + (oz == 0 ? sb0 : oz == 1 ? sb1 : sb2) + lbase + ox * KCH + ch;
#pragma unroll
      for (int oy = 0; oy < 3; ++oy) {
        Pack8<bf16_t> A;
        A.load(ab + oy * (kSPX * KCH));
        mma32(acc[oy], A, Bw[oy][s]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float val = (acc[0][j] + acc[1][j]) + acc[2][j];
      if (a.apply_act) val = val > 0.0f ? val : kLeak * val;
      const bool ok = gx0 + j < g.X && gy < g.Y;
      const int off = ok ? obase + j * (nres * 2) + z * ostride : kZOOB;
      __builtin_amdgcn_raw_buffer_store_b16(from_f<bf16_t>(val).bits, rout, off, 0, 0);
    }
    plane_store(pa, 2 * z + 2);
    plane_store(pb, 2 * z + 3);
    __syncthreads();
  }
}

template <int KCH>
hipError_t launch_conv3s2_t(hipStream_t s, const ConvArgs& a) {
  constexpr int smem = conv3s2_lds_bytes<KCH>();
  auto kern = conv3s2_kernel<KCH>;
  static std::atomic<int> once{0};
  int resident = 0;
  const hipError_t e = conv_resident(kern, smem, once, &resident);
  if (e != hipSuccess) return e;
  const Conv3zGeom gm = conv3z_geom(a.gout, a.cout / 16, resident, kSX, kSY, 2);
  kern<<<dim3(8 * gm.per_xcd, a.cout / 16), 256, smem, s>>>(a, gm);
  return hipGetLastError();
}

// BF16 stride-2 3x3x3 forward with 16 or 32 operand channels on grids whose result is the
// operand's (n - 1) / 2 + 1 per axis; hipErrorNotSupported for the others.
hipError_t launch_conv3s2(hipStream_t s, const ConvArgs& a) {
  if (a.cout % 16 || a.gout.X != (a.gin.X - 1) / 2 + 1 || a.gout.Y != (a.gin.Y - 1) / 2 + 1 ||
      a.gout.Z != (a.gin.Z - 1) / 2 + 1 || 2LL * a.gin.n() * a.cin >= (1LL << 31) ||
      2LL * a.gout.n() * a.cout >= (1LL << 31))
    return hipErrorNotSupported;
  switch (a.cin) {
    case 16: return launch_conv3s2_t<16>(s, a);
    case 32: return launch_conv3s2_t<32>(s, a);
    default: return hipErrorNotSupported;
  }
}

// The up-sampling layers reading their concatenated operand in place (48 channels: 32
// up-sampled, 16 skipped; 96: 64 up-sampled, 32 skipped, in three passes through a.part);
// hipErrorNotSupported for other shapes.
hipError_t launch_conv3z_cat(hipStream_t s, const ConvArgs& a) {
  // every result voxel's coarse parent (x / 2, y / 2, z / 2) lies on the coarse grid
  if (a.cout % 16 || !a.skip || 4LL * a.gout.n() * (a.cin > a.cout ? a.cin : a.cout) >= (1LL << 31) ||
      a.gout.X > 2 * a.gcoarse.X || a.gout.Y > 2 * a.gcoarse.Y || a.gout.Z > 2 * a.gcoarse.Z)
    return hipErrorNotSupported;
  if (a.cin == 48 && a.c1 == 32) return launch_conv3z_t<48, false, 32>(s, a);
  if (a.cin == 96 && a.c1 == 64 && a.part) {
    // three passes over K, each with 32 channels: up-sampled channels 0-31 into the FP32
    // partial, 32-63 added to it, then the 32 skipped channels added with the activation
    // (weight rows of 27 x 96 channels)
    ConvArgs p = a;
    p.wk = 96;
    p.wc0 = 0;
    p.c1 = 32;
    p.cstr = 64;
    p.cc0 = 0;
    hipError_t e = launch_conv3z_t<32, false, 32, 1>(s, p);
    if (e != hipSuccess) return e;
    p.wc0 = 32;
    p.cc0 = 32;
    e = launch_conv3z_t<32, false, 32, 3>(s, p);
    if (e != hipSuccess) return e;
    ConvArgs q = a;
    q.in = a.skip;
    q.skip = nullptr;
    q.c1 = 0;
    q.wk = 96;
    q.wc0 = 64;
    return launch_conv3z_t<32, false, 0, 2>(s, q);
  }
  return hipErrorNotSupported;
}

// The preconditioner's first layer reading r and the density in place (8 operand channels,
// 16 results); hipErrorNotSupported for other shapes.
hipError_t launch_conv3z_input(hipStream_t s, const ConvArgs& a) {
  if (a.cin != 8 || a.cout % 16 || !a.in || !a.skip || !a.npart || !a.nout ||
      12LL * a.gout.n() >= (1LL << 31) || 2LL * a.gout.n() * a.cout >= (1LL << 31))
    return hipErrorNotSupported;
  return launch_conv3z_t<8, false, 0, 0, true>(s, a);
}

// BF16 stride-1 3x3x3 layers whose K channel count has a z-sweep instance (forward 8, 16,
// 32, 48, 64; data gradient 16, 32); returns hipErrorNotSupported for the others (the caller
// uses the brick kernel).
template <bool BWD>
hipError_t launch_conv3z(hipStream_t s, const ConvArgs& a) {
  const int kch = BWD ? a.cout : a.cin, nres = BWD ? a.cin : a.cout;
  // 32-bit byte offsets into the operand and result tensors; the data gradient forms
  // dY leaky'(a) from the stored activation.
  if (nres % 16 || 2LL * a.gout.n() * (kch > nres ? kch : nres) >= (1LL << 31) ||
      (BWD && !a.act))
    return hipErrorNotSupported;
  if constexpr (BWD) {
    switch (kch) {
      case 16: return launch_conv3z_t<16, true>(s, a);
      case 32: return launch_conv3z_t<32, true>(s, a);
      default: return hipErrorNotSupported;
    }
  } else {
    switch (kch) {
      case 8: return launch_conv3z_t<8, false>(s, a);
      case 16: return launch_conv3z_t<16, false>(s, a);
      case 32: return launch_conv3z_t<32, false>(s, a);
      case 48: return launch_conv3z_t<48, false>(s, a);
      case 64: return launch_conv3z_t<64, false>(s, a);
      default: return hipErrorNotSupported;
    }
  }
}

// Weight gradient, one block per (chunk of cvox output voxels, tap, group of up to 32
// (cout/16 x cin/16) tiles).  Per step of kc voxels (a multiple of 32 dividing cvox,
// as many as fit 32 KB of LDS) the block stages dZ = dY leaky'(a)
// and the tap's input rows X[nbr(o, t)] in LDS, both transposed to [channel][voxel], with
// coalesced 16-byte row loads; each lane's eight consecutive voxels of a channel are then
// one 16-byte LDS read, and each wave issues one matrix-core product per tile it owns
// (K = the chunk's voxels in order, 8 per lane group).  Partial sums go to
// part[chunk][cout][taps][cin]; conv_wgrad_reduce sums the chunks in index order.
// cvox is a multiple of 256, cout of 16, cin of 8.
constexpr int kWgPad = 8;           // LDS row pitch kc + 8 elements (rows stay 16-byte aligned)
constexpr int kWgTiles = 8;         // tiles per wave and block group
constexpr int kWgLds = 32768;       // LDS budget of the staged step

__device__ __forceinline__ void put_elem(bf16_t* p, const Pack8<bf16_t>& a, int j) {
  p->bits = a.v[j];
}
__device__ __forceinline__ void put_elem(float* p, const Pack8<float>& a, int j) { *p = a.v[j]; }

template <typename ST>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(ConvArgs a, float* part, int cvox,
                                                         int kc) {
  extern __shared__ __align__(16) unsigned char wg_smem[];
  const int cout = a.cout, cin = a.cin;
  const int pitch = kc + kWgPad;
  ST* sdz = reinterpret_cast<ST*>(wg_smem);    // [cout][pitch]
  ST* sxt = sdz + (size_t)cout * pitch;         // [cin][pitch]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int chunk = blockIdx.x, t = blockIdx.y;
  const int taps = a.ksize * a.ksize * a.ksize;
  const int pad = a.ksize / 2;
  const int tx = t % a.ksize, ty = (t / a.ksize) % a.ksize, tz = t / (a.ksize * a.ksize);
  const ST* X = (const ST*)a.in;   // layer input [Vin][cin]
  const ST* dY = (const ST*)a.out; // gradient wrt the layer output [Vout][cout]
  const ST* act = (const ST*)a.act;
  const int nci = (cin + 15) / 16;
  const int tile_end = min((cout / 16) * nci, (int)(blockIdx.z + 1) * 4 * kWgTiles);
  const int tile0 = blockIdx.z * 4 * kWgTiles + wv;  // this wave: tile0, tile0 + 4, ...
  const int m = lane & 15, q = lane >> 4;
  const int Vout = a.gout.n();
  const int c8o = cout / 8, c8i = cin / 8;
  f32x4 acc[kWgTiles];
#pragma unroll
  for (int j = 0; j < kWgTiles; ++j) acc[j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < cvox; k0 += kc) {
    __syncthreads();  // the previous stage's reads are done
    for (int idx = threadIdx.x; idx < kc * c8o; idx += 256) {
      const int v = idx / c8o, c8 = idx - v * c8o;
      const int o = chunk * cvox + k0 + v;
      Pack8<ST> d;
      d.zero();
      if (o < Vout) {
        d.load(dY + (long long)o * cout + 8 * c8);
        if (act) {
          Pack8<ST> av;
          av.load(act + (long long)o * cout + 8 * c8);
#pragma unroll
          for (int j = 0; j < 8; ++j) d.set(j, d.get(j) * (av.get(j) > 0.0f ? 1.0f : kLeak));
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) put_elem(sdz + (8 * c8 + j) * pitch + v, d, j);
    }
    for (int idx = threadIdx.x; idx < kc * c8i; idx += 256) {
      const int v = idx / c8i, c8 = idx - v * c8i;
      const int o = chunk * cvox + k0 + v;
      Pack8<ST> xv;
      xv.zero();
      if (o < Vout) {
        const int ox = o % a.gout.X, oy = (o / a.gout.X) % a.gout.Y, oz = o / (a.gout.X * a.gout.Y);
        const int sx = ox * a.stride + tx - pad, sy = oy * a.stride + ty - pad,
                  sz = oz * a.stride + tz - pad;
        if (sx >= 0 && sx < a.gin.X && sy >= 0 && sy < a.gin.Y && sz >= 0 && sz < a.gin.Z)
          xv.load(X + ((long long)sx + (long long)a.gin.X * (sy + (long long)a.gin.Y * sz)) * cin +
                  8 * c8);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) put_elem(sxt + (8 * c8 + j) * pitch + v, xv, j);
    }
    __syncthreads();
    for (int ks = 0; ks < kc; ks += 32) {
#pragma unroll
      for (int j = 0; j < kWgTiles; ++j) {
        const int tile = tile0 + 4 * j;
        if (tile < tile_end) {
          const int cb = tile / nci, ib = tile % nci;
          const int ci = ib * 16 + m;
          Pack8<ST> A, B;
          A.load(sdz + (cb * 16 + m) * pitch + ks + 8 * q);
          if (ci < cin) B.load(sxt + ci * pitch + ks + 8 * q); else B.zero();
          mma32(acc[j], A, B);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kWgTiles; ++j) {
    const int tile = tile0 + 4 * j;
    if (tile < tile_end) {
      const int cb = tile / nci, ib = tile % nci;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int orow = cb * 16 + 4 * q + jj;  // co
        const int ocol = ib * 16 + m;           // ci
        if (ocol < cin)
          part[(((long long)chunk * cout + orow) * taps + t) * cin + ocol] = acc[j][jj];
      }
    }
  }
}

// Sums the chunks in index order; the loads of 16 chunks are issued before their
// additions (one thread per weight, so a layer has only a few thousand threads and each
// would otherwise wait for nchunk load latencies in a row).
__global__ __launch_bounds__(256) void conv_wgrad_reduce(const float* part, int nchunk, int n,
                                                         float* grad, int accumulate) {
  constexpr int U = 16;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float s = 0.0f;
    int c = 0;
    for (; c + U <= nchunk; c += U) {
      float v[U];
#pragma unroll
      for (int j = 0; j < U; ++j) v[j] = part[(long long)(c + j) * n + i];
#pragma unroll
      for (int j = 0; j < U; ++j) s += v[j];
    }
    for (; c < nchunk; ++c) s += part[(long long)c * n + i];
    grad[i] = accumulate ? grad[i] + s : s;
  }
}

// ----------------------------------------------------------- elementwise kernels
// Network input: [v][0..2] = r / ||r|| (DOF vector is node-major, so already
// channels-last), [v][3] = nodal density, [v][4..7] = 0.
template <typename ST>
__global__ void build_input_kernel(const float* r, const double* rnorm2, const float* rho_node,
                                   ST* inp, int n_node) {
  // residual at unit RMS per DOF: r sqrt(n_dof) / ||r||
  const float inv = (float)(sqrt(3.0 * n_node) / sqrt(fmax(*rnorm2, 1e-300)));
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n_node; v += gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) inp[8 * v + c] = from_f<ST>(r[3 * v + c] * inv);
    inp[8 * v + 3] = from_f<ST>(rho_node[v]);
#pragma unroll
    for (int c = 4; c < 8; ++c) inp[8 * v + c] = from_f<ST>(0.0f);
  }
}

// The same from the 512 per-block partial sums of ||r||^2: every block adds them in one
// fixed order (each thread two, then a tree in LDS), so all blocks use the same value;
// block 0 also stores it into *rnorm2 (for the output scaling).
template <typename ST>
__global__ __launch_bounds__(256) void build_input_sum_kernel(const float* r, const double* partials,
                                                              double* rnorm2, const float* rho_node,
                                                              ST* inp, int n_node) {
  __shared__ double red[256];
  red[threadIdx.x] = partials[2 * threadIdx.x] + partials[2 * threadIdx.x + 1];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double tot = red[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) *rnorm2 = tot;
  const float inv = (float)(sqrt(3.0 * n_node) / sqrt(fmax(tot, 1e-300)));
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n_node; v += gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) inp[8 * v + c] = from_f<ST>(r[3 * v + c] * inv);
    inp[8 * v + 3] = from_f<ST>(rho_node[v]);
#pragma unroll
    for (int c = 4; c < 8; ++c) inp[8 * v + c] = from_f<ST>(0.0f);
  }
}

// Same from an FP32 channels-last [v][4] tensor (test hook / training input).
template <typename ST>
__global__ void pad_input_kernel(const float* x4, ST* inp, int n) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 4; ++c) inp[8 * v + c] = from_f<ST>(x4[4 * v + c]);
#pragma unroll
    for (int c = 4; c < 8; ++c) inp[8 * v + c] = from_f<ST>(0.0f);
  }
}

// Nodal density: mean of the (up to 8) elements around each node.
template <typename XT>
__global__ void node_density_kernel(const XT* x, int nx, int ny, int nz, float* rho) {
  const int n_node = (nx + 1) * (ny + 1) * (nz + 1);
  for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < n_node; n += gridDim.x * blockDim.x) {
    const int i = n % (nx + 1), j = (n / (nx + 1)) % (ny + 1), k = n / ((nx + 1) * (ny + 1));
    float s = 0.0f;
    int c = 0;
    for (int dz = -1; dz <= 0; ++dz)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dx = -1; dx <= 0; ++dx) {
          const int ex = i + dx, ey = j + dy, ez = k + dz;
          if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
          s += (float)x[ex + nx * (ey + ny * ez)];
          ++c;
        }
    rho[n] = s / (float)c;
  }
}

// [up(coarse) | skip] concatenation: dst[v][0..c1) = coarse[parent(v)], dst[v][c1..) = skip[v].
// One thread copies eight channels (16 B in BF16) of one voxel; c1 and c2 are multiples of
// 8 and n (c1 + c2) / 8 < 2^31 (at most 12 chunks per voxel at the largest mesh), so the
// index arithmetic is 32-bit.
template <typename ST>
__global__ __launch_bounds__(256) void upcat_kernel(const ST* coarse, Grid3 gc, int c1,
                                                    const ST* skip, int c2, ST* dst, Grid3 gf) {
  const unsigned ct8 = (unsigned)(c1 + c2) / 8, c18 = (unsigned)c1 / 8;
  const unsigned units = (unsigned)gf.n() * ct8;
  for (unsigned u = blockIdx.x * blockDim.x + threadIdx.x; u < units; u += gridDim.x * blockDim.x) {
    const unsigned v = u / ct8, c8 = u - v * ct8;
    Pack8<ST> p;
    if (c8 < c18) {
      const unsigned x = v % (unsigned)gf.X, y = (v / (unsigned)gf.X) % (unsigned)gf.Y,
                     z = v / ((unsigned)gf.X * (unsigned)gf.Y);
      const unsigned pv = (x / 2) + (unsigned)gc.X * ((y / 2) + (unsigned)gc.Y * (z / 2));
      p.load(coarse + (size_t)pv * c1 + 8 * c8);
    } else {
      p.load(skip + (size_t)v * c2 + 8 * (c8 - c18));
    }
    p.store(dst + (size_t)u * 8);
  }
}

// Adjoint of the up-sampling half of upcat: coarse[pv][c] = sum over children of g[v][c].
template <typename ST>
__global__ void upcat_adjoint_kernel(const ST* g, Grid3 gf, int ct, ST* coarse, Grid3 gc, int c1) {
  const int n = gc.n();
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (long long)n * c1;
       i += (long long)gridDim.x * blockDim.x) {
    const int pv = (int)(i / c1), c = (int)(i % c1);
    const int px = pv % gc.X, py = (pv / gc.X) % gc.Y, pz = pv / (gc.X * gc.Y);
    float s = 0.0f;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int x = 2 * px + dx, y = 2 * py + dy, z = 2 * pz + dz;
          if (x < gf.X && y < gf.Y && z < gf.Z)
            s += to_f(g[((long long)x + (long long)gf.X * (y + (long long)gf.Y * z)) * ct + c]);
        }
    coarse[i] = from_f<ST>(s);
  }
}

// dst[v][c] = a[v][c] + b[v][boff + c] (gradient of a tensor used by a conv and a skip).
template <typename ST>
__global__ void add_skip_kernel(ST* dst, const ST* a, const ST* b, int n, int c, int bct, int boff) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (long long)n * c;
       i += (long long)gridDim.x * blockDim.x) {
    const long long v = i / c;
    const int ch = (int)(i % c);
    dst[i] = from_f<ST>(to_f(a[i]) + to_f(b[v * bct + boff + ch]));
  }
}

// Relative masked MSE of the 3 output channels against target e (FP32 DOF layout):
// loss = sum(m (out - e)^2) / sum(m e^2); writes dLoss/dout into g [v][16] (padded).
template <typename ST>
__global__ __launch_bounds__(256) void loss_kernel(const ST* out, const float* e, const uint8_t* mask,
                                                   int n_node, double* partials) {
  __shared__ double sred[4];
  double num = 0.0, den = 0.0;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n_node; v += gridDim.x * blockDim.x) {
    const uint8_t mk = mask[v];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if ((mk >> c) & 1) continue;
      const double t = e[3 * v + c], d = (double)to_f(out[16 * v + c]) - t;
      num += d * d;
      den += t * t;
    }
  }
  const double v[2] = {num, den};
  store_block_sums<2>(v, partials, sred);
}

struct LossFin {
  double* den_num;
  __device__ void operator()(const double* t) const {
    den_num[0] = t[1];
    den_num[1] = t[0];
  }
};

// den_num[0] = sum m e^2, den_num[1] = sum m (out - e)^2.
template <typename ST>
hipError_t launch_loss(hipStream_t s, const ST* out, const float* e, const uint8_t* mask, int n,
                       double* partials, double* den_num) {
  loss_kernel<ST><<<1024, 256, 0, s>>>(out, e, mask, n, partials);
  return launch_finalize_sum<2>(s, partials, 1024, LossFin{den_num});
}

template <typename ST>
__global__ void loss_grad_kernel(const ST* out, const float* e, const uint8_t* mask, int n_node,
                                 const double* den_num, ST* g) {
  const float s = (float)(2.0 / fmax(den_num[0], 1e-300));
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n_node; v += gridDim.x * blockDim.x) {
    const uint8_t mk = mask[v];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float gv = 0.0f;
      if (c < 3 && !((mk >> c) & 1)) gv = s * (to_f(out[16 * v + c]) - e[3 * v + c]);
      g[16 * v + c] = from_f<ST>(gv);
    }
  }
}

// Network output to a DOF vector: z[3v + c] = scale * out[v][c], zero on fixed DOFs.
// The preconditioner's output with the 1x1 head fused in: z = ||r|| / sqrt(n_dof) *
// (W_head a) on free DOFs, 0 on fixed ones, from the last hidden layer's 16 channels a.
// The head's result is rounded to the storage type, as the head layer stores it.
template <typename ST>
__global__ __launch_bounds__(256) void head_output_kernel(const ST* a, const ST* wh, int cip,
                                                          const uint8_t* mask,
                                                          const double* rnorm2, float* z,
                                                          int n_node) {
  __shared__ float w[3][16];
  if (threadIdx.x < 48) w[threadIdx.x >> 4][threadIdx.x & 15] = to_f(wh[(threadIdx.x >> 4) * cip + (threadIdx.x & 15)]);
  __syncthreads();
  const float s = (float)(sqrt(*rnorm2) / sqrt(3.0 * n_node));  // ||r|| / sqrt(n_dof)
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n_node; v += gridDim.x * blockDim.x) {
    Pack8<ST> lo, hi;
    lo.load(a + 16 * (long long)v);
    hi.load(a + 16 * (long long)v + 8);
    const uint8_t mk = mask[v];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += w[c][j] * lo.get(j);
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += w[c][8 + j] * hi.get(j);
      z[3 * (long long)v + c] = ((mk >> c) & 1) ? 0.0f : s * to_f(from_f<ST>(acc));
    }
  }
}

// Adam on the FP32 master weights, then the compute copies: W [co][t][ci_pad] and the
// transposed WT [ci_pad][t][co] used by the data gradient (padding channels stay 0).
struct AdamArgs {
  float lr, b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
  float omb1, omb2;                // 1 - b1, 1 - b2 (rounded from FP64)
};

__global__ void adam_kernel(float* w, float* m, float* v, const float* g, int n, AdamArgs a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = a.b1 * m[i] + a.omb1 * gi;
    const float vi = a.b2 * v[i] + a.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
  }
}

// master layout [co][ci][taps] (as the oracle's W[o, i, a, b, c] flattened; taps ordered
// z, y, x) -> W [co_pad][taps][ci_pad] and WT [ci_pad][taps][co_pad].
template <typename ST>
__global__ void pack_weights_kernel(const float* master, int co, int ci, int taps, int cop, int cip,
                                    ST* W, ST* WT) {
  const int n = cop * taps * cip;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int c_i = i % cip, t = (i / cip) % taps, c_o = i / (cip * taps);
    const float val = (c_o < co && c_i < ci) ? master[((long long)c_o * ci + c_i) * taps + t] : 0.0f;
    W[i] = from_f<ST>(val);
    WT[((long long)c_i * taps + t) * cop + c_o] = from_f<ST>(val);
  }
}

// gradient [co][taps][ci_pad] -> master layout [co][ci][taps]
__global__ void unpack_grad_kernel(const float* g, int co, int ci, int taps, int cip, float* out) {
  const int n = co * ci * taps;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int t = i % taps, c_i = (i / taps) % ci, c_o = i / (taps * ci);
    out[i] = g[((long long)c_o * taps + t) * cip + c_i];
  }
}

// Small helpers of the training and test entry points.
__global__ void accum_kernel(float* acc, const float* g, int n, int add) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    acc[i] = add ? acc[i] + g[i] : g[i];
}

__global__ void scale_kernel(float* g, int n, float s) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) g[i] *= s;
}
__global__ void take3_bf16(const bf16_t* o, float* out, int n) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    for (int c = 0; c < 3; ++c) out[3 * v + c] = to_f(o[16 * v + c]);
}
__global__ void take3_f32(const float* o, float* out, int n) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    for (int c = 0; c < 3; ++c) out[3 * v + c] = o[16 * v + c];
}


// ------------------------------------------------------------ energy-norm loss
// Training loss of the correction n (head output on free DOFs, DOF layout) for a pair
// (r, e = K^-1 r): L = 1 - a^2 / (q c), a = <n, r>, q = <n, K n>, c = <e, r>, the relative
// energy-norm error of the best multiple of n; dL/dn = -(2a / (q c)) (r - (a/q) K n).
template <typename ST>
__global__ void head_to_dof_kernel(const ST* out, const uint8_t* mask, float* nd, int n_node) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n_node; v += gridDim.x * blockDim.x) {
    const uint8_t mk = mask[v];
#pragma unroll
    for (int c = 0; c < 3; ++c) nd[3 * v + c] = ((mk >> c) & 1) ? 0.0f : to_f(out[16 * v + c]);
  }
}

__global__ __launch_bounds__(256) void energy_dots_kernel(const float* __restrict__ nd,
                                                          const float* __restrict__ r,
                                                          const float* __restrict__ e, int n,
                                                          double* partials) {
  __shared__ double sred[4];
  double a = 0.0, c = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    a += (double)nd[i] * (double)r[i];
    c += (double)e[i] * (double)r[i];
  }
  const double v[2] = {a, c};
  store_block_sums<2>(v, partials, sred);
}

// scal[4] = q (from the operator's fused dot); sets scal[5] = a, scal[6] = c and the
// reported loss as scal[2] / scal[1].
struct EnergyFin {
  double* scal;
  __device__ void operator()(const double* t) const {
    const double a = t[0], c = t[1], q = scal[4];
    scal[5] = a;
    scal[6] = c;
    scal[1] = 1.0;
    scal[2] = (q > 0.0 && c > 0.0) ? 1.0 - a * a / (q * c) : 1.0;
  }
};

template <typename ST>
__global__ void energy_grad_kernel(const float* r, const float* Knd, const uint8_t* mask,
                                   const double* scal, ST* g, int n_node) {
  const double q = scal[4], a = scal[5], c = scal[6];
  const bool ok = q > 0.0 && c > 0.0;
  const float k1 = ok ? (float)(-2.0 * a / (q * c)) : 0.0f;
  const float sa = ok ? (float)(a / q) : 0.0f;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n_node; v += gridDim.x * blockDim.x) {
    const uint8_t mk = mask[v];
#pragma unroll
    for (int ch = 0; ch < 16; ++ch) {
      float gv = 0.0f;
      if (ch < 3 && !((mk >> ch) & 1)) gv = k1 * (r[3 * v + ch] - sa * Knd[3 * v + ch]);
      g[16 * v + ch] = from_f<ST>(gv);
    }
  }
}

// ------------------------------------------------------------------- flexible CG
// FCG(m) (flexible CG truncated to the m latest directions): z_k = M(r_k),
//   p_k = z_k + sum_j beta_j p_j,  beta_j = -<z_k, q_j> / <p_j, q_j>  (j: the window),
//   q_k = K p_k,  alpha_k = <r_k, z_k> / <p_k, q_k>.
// m = 1 is FCG(1); with a fixed SPD preconditioner every m gives PCG in exact arithmetic.
// A z that is not a descent direction (<r, z> <= 0 or non-finite) is replaced by the
// Jacobi step z = D^-1 r.  Directions and their images live in a ring of m slots; the
// host passes the window size and the slot of each enqueued iteration (kernels of a
// finished solve return at once, so the host's count equals the device's).
constexpr int kFcgMax = 16;

struct FcgWin {
  const float* P[kFcgMax];
  const float* Q[kFcgMax];
  int nw;  // directions in the window (slots 0 .. nw-1)
};

// <r, z> and <z, q_j> for the window; pass 1 runs only when a fallback is pending.
__global__ __launch_bounds__(256) void fcgm_dots_kernel(const float* __restrict__ r,
                                                        const float* __restrict__ z, FcgWin w,
                                                        int n, const SolverState* st, int pass,
                                                        double* partials) {
  __shared__ double sred[4];
  if (st->done || (pass == 1 && st->aux == 0.0)) return;
  double acc[1 + kFcgMax];
#pragma unroll
  for (int j = 0; j <= kFcgMax; ++j) acc[j] = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double zi = z[i];
    acc[0] += (double)r[i] * zi;
#pragma unroll
    for (int j = 0; j < kFcgMax; ++j)
      if (j < w.nw) acc[1 + j] += zi * (double)w.Q[j][i];
  }
  store_block_sums<1 + kFcgMax>(acc, partials, sred);
}

struct FcgmFin {
  SolverState* st;
  double* pq;    // <p_j, q_j> per slot
  double* coef;  // beta_j per slot (output)
  int nw;
  int pass;      // 0: check the network's z; 1: after the Jacobi replacement
  __device__ void operator()(const double* t) const {
    if (st->done || (pass == 1 && st->aux == 0.0)) return;
    const double RZ = t[0];
    bool ok = finite_val(RZ) && RZ > 0.0;
    for (int j = 0; j < kFcgMax; ++j) {
      const double b = j < nw ? -t[1 + j] / pq[j] : 0.0;
      coef[j] = b;
      ok = ok && finite_val(b);
    }
    if (pass == 0) {
      if (ok) {
        st->aux = 0.0;
        st->rz = RZ;
      } else {
        st->aux = 1.0;  // replace z by the Jacobi step
      }
    } else {
      st->rz = RZ;
      st->aux = 0.0;
      st->nfallback += 1;
      if (!ok) st->done = 3;
    }
  }
};

__global__ __launch_bounds__(256) void fcg_jacobi_z_kernel(const float* __restrict__ r,
                                                           float* __restrict__ z,
                                                           const float* __restrict__ dinv, int n,
                                                           const SolverState* st) {
  if (st->done || st->aux == 0.0) return;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    z[i] = r[i] * dinv[(unsigned)i / 3u];
}

// p_slot = z + sum_j beta_j p_j (the slot's old direction is read before it is replaced).
__global__ __launch_bounds__(256) void fcgm_direction_kernel(const float* __restrict__ z, FcgWin w,
                                                             const double* coef, float* pout,
                                                             int n, const SolverState* st) {
  if (st->done) return;
  float b[kFcgMax];
#pragma unroll
  for (int j = 0; j < kFcgMax; ++j) b[j] = j < w.nw ? (float)coef[j] : 0.0f;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    float v = z[i];
#pragma unroll
    for (int j = 0; j < kFcgMax; ++j)
      if (j < w.nw) v += b[j] * w.P[j][i];
    pout[i] = v;
  }
}

__global__ void fcg_store_pq_kernel(const SolverState* st, double* pq, int slot) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && !st->done) pq[slot] = st->pq;
}

// Stagnation guard of the learned solve: after each iteration, ||r||^2 either sets a new
// minimum or, once st->stall iterations have passed without one, the solve stops with
// done = 4 (the host then continues with plain Jacobi-PCG from the iterate).  init: the
// initial residual is the first minimum.
__global__ void fcg_stall_kernel(SolverState* st, int init) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || st->done || st->stall <= 0) return;
  if (init) {
    st->rmin = st->rr;
    st->kmin = 0;
  } else if (st->rr < st->rmin) {
    st->rmin = st->rr;
    st->kmin = st->iter;
  } else if (st->iter - st->kmin >= st->stall) {
    st->done = 4;
  }
}

// Two-stage preconditioner: n = network correction, then a Jacobi step on what remains,
//   s = <r, n> / <n, K n> (energy-optimal scale of n; 0 unless both are positive),
//   z = s n + D^-1 (r - s K n).
// With n = K^-1 r this returns K^-1 r; with n = 0 it is the Jacobi step.
__global__ __launch_bounds__(256) void dot_rn_kernel(const float* __restrict__ r,
                                                     const float* __restrict__ nv, int n,
                                                     const SolverState* st, double* partials) {
  __shared__ double sred[4];
  if (st->done) return;
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    s += (double)r[i] * (double)nv[i];
  const double v[1] = {s};
  store_block_sums<1>(v, partials, sred);
}

struct SetRn {
  SolverState* st;
  __device__ void operator()(const double* t) const {
    if (!st->done) st->s_rn = t[0];
  }
};

__global__ __launch_bounds__(256) void two_stage_kernel(const float* __restrict__ r,
                                                        const float* __restrict__ Kn,
                                                        const float* __restrict__ dinv,
                                                        float* __restrict__ z, int n,
                                                        const SolverState* st) {
  if (st->done) return;
  const double rn = st->s_rn, nkn = st->s_nkn;
  const float sc = (rn > 0.0 && nkn > 0.0 && finite_val(rn / nkn)) ? (float)(rn / nkn) : 0.0f;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float nv = z[i];  // z holds n on entry
    z[i] = sc * nv + dinv[(unsigned)i / 3u] * (r[i] - sc * Kn[i]);
  }
}

}  // namespace tosimp

// =========================================================================== host side
using namespace tosimp;

namespace {

struct Layer {
  const char* name;
  int ci, co, k, s;      // logical channels, kernel size, stride
  int cip, cop;          // padded channels (ci to 8, co to 16)
  int level_in, level_out;
  size_t moff, goff;     // offsets into the master / gradient arrays (floats)
  size_t woff;           // offset into the packed compute weights (elements)
};

struct NNState {
  int base = 16;
  int bf16 = 1;          // storage type of weights and activations
  size_t es = 2;         // element size
  std::vector<Layer> L;
  size_t nparam = 0, npacked = 0;
  Grid3 g[3];
  float* master = nullptr;     // FP32 weights [co][ci][taps] per layer
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;       // gradient in master layout
  float* gpack = nullptr;      // gradient per layer in [co][taps][ci_pad]
  void* W = nullptr;           // packed compute weights
  void* WT = nullptr;
  void* act[13] = {};          // per layer output (a), plus input at index 12
  void* cat1 = nullptr;        // [up(m2b) | s1] at level 1
  void* cat0 = nullptr;        // [up(u1b) | s0] at level 0
  float* u1part = nullptr;     // u1a's FP32 partial sums (BF16 forward in two passes)
  void* gbuf[6] = {};          // gradient scratch (largest level-0 sizes)
  float* gsum = nullptr;       // summed gradient of a training batch (master layout)
  float* x32 = nullptr;        // element density of the training pairs (FP32, for K n)
  float* fcgP = nullptr;       // flexible CG: direction ring [fcg_cap][n_dof] and images
  float* fcgQ = nullptr;
  int fcg_cap = 0;
  double* fpq = nullptr;       // <p_j, q_j> per ring slot
  double* fco = nullptr;       // direction coefficients per ring slot
  int loss_kind = 0;           // 0: relative MSE to the unit-RMS error; 1: energy norm
  float* wpart = nullptr;      // weight-gradient partials
  size_t wpart_cap = 0;
  float* rho_node = nullptr;
  double* scal = nullptr;      // device scalars: [0] ||r||^2, [1..2] den/num, [3] ||e||^2
  double* part = nullptr;
  int adam_t = 0;
};

NNState* nn_of(tosimp_ctx* c) { return (NNState*)c->nn; }

int ceil16(int c) { return (c + 15) / 16 * 16; }
int ceil8(int c) { return (c + 7) / 8 * 8; }

// Voxels per weight-gradient chunk: a multiple of 256 keeping the chunk count <= 512.
int wgrad_chunk(int nvox) {
  const int per = (nvox + 511) / 512;
  return std::max(256, (per + 255) / 256 * 256);
}

// With skip set (BF16 only), `in` is the coarse tensor of an up-sampling concatenation
// [up(in) | skip] that the z-sweep reads in place; hipErrorNotSupported if it cannot.
template <typename ST>
hipError_t conv_fwd(tosimp_ctx* c, NNState* S, const Layer& l, const void* in, void* out, int act,
                    const void* skip = nullptr, int c1 = 0, Grid3 gcoarse = {},
                    float* part = nullptr) {
  ConvArgs a{};
  a.in = in;
  a.w = (const char*)S->W + l.woff * S->es;
  a.out = out;
  a.gin = S->g[l.level_in];
  a.gout = S->g[l.level_out];
  a.cin = l.cip;
  a.cout = l.cop;
  a.ksize = l.k;
  a.stride = l.s;
  a.apply_act = act;
  if (skip) {
    if (sizeof(ST) != 2 || l.k != 3 || l.s != 1) return hipErrorNotSupported;
    a.skip = skip;
    a.c1 = c1;
    a.gcoarse = gcoarse;
    a.part = part;
    return launch_conv3z_cat(c->stream, a);
  }
  if constexpr (sizeof(ST) == 2) {
    if (l.k == 3 && (l.s == 1 || l.s == 2)) {
      const hipError_t e = l.s == 1 ? launch_conv3z<false>(c->stream, a)
                                    : launch_conv3s2(c->stream, a);
      if (e != hipErrorNotSupported) return e;
    }
  }
  if (l.k == 3 && l.s == 1 && a.cin % conv3_cs<ST>() == 0)
    return launch_conv3_lds<ST, false>(c->stream, a);
  const int waves = (a.gout.n() + 16 * kConvRT - 1) / (16 * kConvRT);
  conv_igemm_kernel<ST, false><<<dim3((waves + 3) / 4, (a.cout + 63) / 64), 256, 0, c->stream>>>(a);
  return hipGetLastError();
}

// dX (wrt this layer's input) from dY (wrt its activated output) and a (its output).
template <typename ST>
hipError_t conv_bwd(tosimp_ctx* c, NNState* S, const Layer& l, const void* dY, const void* a_out,
                    const void* x_in, void* dX, bool need_dx) {
  ConvArgs a{};
  a.gin = S->g[l.level_in];
  a.gout = S->g[l.level_out];
  a.cin = l.cip;
  a.cout = l.cop;
  a.ksize = l.k;
  a.stride = l.s;
  const int taps = l.k * l.k * l.k;
  // weight gradient
  {
    ConvArgs b = a;
    b.in = x_in;
    b.out = const_cast<void*>(dY);
    b.act = a_out;
    const int cvox = wgrad_chunk(a.gout.n());
    const int nchunk = (a.gout.n() + cvox - 1) / cvox;
    const size_t need = (size_t)nchunk * l.cop * taps * l.cip;
    if (need > S->wpart_cap) return hipErrorInvalidValue;
    const int ntile = (l.cop / 16) * ((l.cip + 15) / 16);
    const int ngroup = (ntile + 4 * kWgTiles - 1) / (4 * kWgTiles);
    int kc = 256;  // voxels per staged step: the largest power of two fitting the budget
    while (kc > 32 && (size_t)(l.cop + l.cip) * (kc + kWgPad) * S->es > (size_t)kWgLds) kc /= 2;
    const size_t smem = (size_t)(l.cop + l.cip) * (kc + kWgPad) * S->es;
    conv_wgrad_kernel<ST><<<dim3(nchunk, taps, ngroup), 256, smem, c->stream>>>(b, S->wpart,
                                                                                cvox, kc);
    const int n = l.cop * taps * l.cip;
    conv_wgrad_reduce<<<(n + 255) / 256, 256, 0, c->stream>>>(S->wpart, nchunk, n,
                                                              S->gpack + l.goff, 0);
  }
  if (need_dx) {
    a.in = dY;
    a.act = a_out;
    a.w = (const char*)S->WT + l.woff * S->es;
    a.out = dX;
    if constexpr (sizeof(ST) == 2) {
      if (l.k == 3 && l.s == 1) {
        const hipError_t e = launch_conv3z<true>(c->stream, a);
        if (e != hipErrorNotSupported) return e;
      }
    }
    if (l.k == 3 && l.s == 1 && a.cout % conv3_cs<ST>() == 0 && a.cin % 16 == 0)
      return launch_conv3_lds<ST, true>(c->stream, a);
    if (l.k == 3 && l.s == 2 && a.cout % 32 == 0 && a.cin % 16 == 0 &&
        a.gout.X == (a.gin.X - 1) / 2 + 1 && a.gout.Y == (a.gin.Y - 1) / 2 + 1 &&
        a.gout.Z == (a.gin.Z - 1) / 2 + 1) {
      const long long waves =
          (long long)(((a.gin.X + 1) / 2 + 15) / 16) * 2 * a.gin.Y * a.gin.Z;
      conv_tgrad_s2_kernel<ST><<<dim3((unsigned)((waves + 3) / 4), (a.cin + 63) / 64), 256, 0,
                                 c->stream>>>(a);
      return hipGetLastError();
    }
    const int waves = (a.gin.n() + 16 * kConvRT - 1) / (16 * kConvRT);
    conv_igemm_kernel<ST, true><<<dim3((waves + 3) / 4, (a.cin + 63) / 64), 256, 0, c->stream>>>(a);
  }
  return hipGetLastError();
}

}  // namespace

void tosimp::nn_release(tosimp_ctx* ctx) {
  NNState* S = ctx ? nn_of(ctx) : nullptr;
  if (!S) return;
  void* ptrs[] = {S->master, S->m,        S->v,    S->grad, S->gpack, S->W,   S->WT, S->cat1,
                  S->cat0,   S->wpart,    S->rho_node, S->scal, S->part, S->gsum, S->x32, S->u1part,
                  S->fcgP, S->fcgQ, S->fpq, S->fco};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (void* p : S->act)
    if (p) (void)hipFree(p);
  for (void* p : S->gbuf)
    if (p) (void)hipFree(p);
  delete S;
  ctx->nn = nullptr;
}


namespace {

hipError_t nn_alloc(void** p, size_t bytes) { return hipMalloc(p, bytes < 256 ? 256 : bytes); }

// Forward pass from the padded input tensor in act[12]; layer outputs in act[0..11].
// infer: the preconditioner's forward (no head: it is fused into the output kernel; in
// BF16 the up-sampling concatenations are read in place by u1a and u0a instead of being
// stored).
// r_in (BF16 inference): the first layer forms its operand from r (and the density) in
// place, the norm from the 512 partials in S->part; without it act[12] holds the input.
template <typename ST>
hipError_t nn_forward(tosimp_ctx* c, NNState* S, bool infer = false, const float* r_in = nullptr) {
  hipError_t e = hipSuccess;
  auto F = [&](int li, const void* in, int act) {
    if (e == hipSuccess) e = conv_fwd<ST>(c, S, S->L[li], in, S->act[li], act);
  };
  const int b = S->base;
  bool in_done = false;
  if (infer && sizeof(ST) == 2 && r_in) {
    const Layer& l0 = S->L[0];
    ConvArgs a0{};
    a0.in = r_in;
    a0.skip = S->rho_node;
    a0.npart = S->part;
    a0.nout = S->scal;
    a0.w = (const char*)S->W + l0.woff * S->es;
    a0.out = S->act[0];
    a0.gin = S->g[0];
    a0.gout = S->g[0];
    a0.cin = l0.cip;
    a0.cout = l0.cop;
    a0.ksize = 3;
    a0.stride = 1;
    a0.apply_act = 1;
    e = launch_conv3z_input(c->stream, a0);
    in_done = e == hipSuccess;
    if (e == hipErrorNotSupported) e = hipSuccess;
    if (e != hipSuccess) return e;
  }
  if (!in_done) {
    if (r_in)
      build_input_sum_kernel<ST><<<2048, 256, 0, c->stream>>>(r_in, S->part, S->scal, S->rho_node,
                                                            (ST*)S->act[12], (int)S->g[0].n());
    F(0, S->act[12], 1);               // e0a
  }
  F(1, S->act[0], 1);                  // e0b -> s0
  F(2, S->act[1], 1);                  // d1
  F(3, S->act[2], 1);                  // e1 -> s1
  F(4, S->act[3], 1);                  // d2
  F(5, S->act[4], 1);                  // m2a
  F(6, S->act[5], 1);                  // m2b
  if (e != hipSuccess) return e;
  bool cat1_done = false;
  if (infer && sizeof(ST) == 2) {      // u1a on [up(m2b) | s1] read in place, two passes
    e = conv_fwd<ST>(c, S, S->L[7], S->act[6], S->act[7], 1, S->act[3], 4 * b, S->g[2],
                     S->u1part);
    cat1_done = e == hipSuccess;
    if (e == hipErrorNotSupported) e = hipSuccess;
    if (e != hipSuccess) return e;
  }
  if (!cat1_done) {
    upcat_kernel<ST><<<2048, 256, 0, c->stream>>>((const ST*)S->act[6], S->g[2], 4 * b,
                                                 (const ST*)S->act[3], 2 * b, (ST*)S->cat1, S->g[1]);
    F(7, S->cat1, 1);                  // u1a
  }
  F(8, S->act[7], 1);                  // u1b
  if (e != hipSuccess) return e;
  bool cat0_done = false;
  if (infer && sizeof(ST) == 2) {      // u0a on [up(u1b) | s0] read in place
    e = conv_fwd<ST>(c, S, S->L[9], S->act[8], S->act[9], 1, S->act[1], 2 * b, S->g[1]);
    cat0_done = e == hipSuccess;
    if (e == hipErrorNotSupported) e = hipSuccess;
    if (e != hipSuccess) return e;
  }
  if (!cat0_done) {
    upcat_kernel<ST><<<2048, 256, 0, c->stream>>>((const ST*)S->act[8], S->g[1], 2 * b,
                                                 (const ST*)S->act[1], b, (ST*)S->cat0, S->g[0]);
    F(9, S->cat0, 1);                  // u0a
  }
  F(10, S->act[9], 1);                 // u0b
  if (!infer) F(11, S->act[10], 0);    // head (no activation)
  return e == hipSuccess ? hipGetLastError() : e;
}

// Backward pass from dLoss/d(head output) in gbuf[0] ([v0][16]); per-layer weight
// gradients land in gpack.  Buffer use (G = gbuf):
//   head: G0 -> G1; u0b: G1 -> G2; u0a: G2 -> G3 (= [up | s0] grad, kept);
//   up-adjoint G3 -> G4 (level 1); u1b: G4 -> G1; u1a: G1 -> G5 (= [up | s1], kept);
//   up-adjoint G5 -> G4 (level 2); m2b: G4 -> G1; m2a: G1 -> G2; d2: G2 -> G1;
//   G4 = G1 + skip(G5); e1: G4 -> G2; d1: G2 -> G1; G4 = G1 + skip(G3); e0b: G4 -> G2;
//   e0a: weight gradient only.
template <typename ST>
hipError_t nn_backward(tosimp_ctx* c, NNState* S) {
  void** G = S->gbuf;
  const int b = S->base;
  hipError_t e = hipSuccess;
  auto B = [&](int li, const void* dY, const void* aout, const void* xin, void* dX, bool ndx) {
    if (e == hipSuccess) e = conv_bwd<ST>(c, S, S->L[li], dY, aout, xin, dX, ndx);
  };
  B(11, G[0], nullptr, S->act[10], G[1], true);   // head (linear)
  B(10, G[1], S->act[10], S->act[9], G[2], true); // u0b
  B(9, G[2], S->act[9], S->cat0, G[3], true);     // u0a -> [2b up | b skip]
  if (e != hipSuccess) return e;
  upcat_adjoint_kernel<ST><<<2048, 256, 0, c->stream>>>((const ST*)G[3], S->g[0], 3 * b,
                                                       (ST*)G[4], S->g[1], 2 * b);
  B(8, G[4], S->act[8], S->act[7], G[1], true);   // u1b
  B(7, G[1], S->act[7], S->cat1, G[5], true);     // u1a -> [4b up | 2b skip]
  if (e != hipSuccess) return e;
  upcat_adjoint_kernel<ST><<<2048, 256, 0, c->stream>>>((const ST*)G[5], S->g[1], 6 * b,
                                                       (ST*)G[4], S->g[2], 4 * b);
  B(6, G[4], S->act[6], S->act[5], G[1], true);   // m2b
  B(5, G[1], S->act[5], S->act[4], G[2], true);   // m2a
  B(4, G[2], S->act[4], S->act[3], G[1], true);   // d2 -> grad wrt s1 (conv path)
  if (e != hipSuccess) return e;
  add_skip_kernel<ST><<<2048, 256, 0, c->stream>>>((ST*)G[4], (const ST*)G[1], (const ST*)G[5],
                                                  S->g[1].n(), 2 * b, 6 * b, 4 * b);
  B(3, G[4], S->act[3], S->act[2], G[2], true);   // e1
  B(2, G[2], S->act[2], S->act[1], G[1], true);   // d1 -> grad wrt s0 (conv path)
  if (e != hipSuccess) return e;
  add_skip_kernel<ST><<<2048, 256, 0, c->stream>>>((ST*)G[4], (const ST*)G[1], (const ST*)G[3],
                                                  S->g[0].n(), b, 3 * b, 2 * b);
  B(1, G[4], S->act[1], S->act[0], G[2], true);   // e0b
  B(0, G[2], S->act[0], S->act[12], nullptr, false);  // e0a
  if (e != hipSuccess) return e;
  for (const Layer& l : S->L) {
    const int taps = l.k * l.k * l.k;
    const int n = l.co * l.ci * taps;
    unpack_grad_kernel<<<(n + 255) / 256, 256, 0, c->stream>>>(S->gpack + l.goff, l.co, l.ci, taps,
                                                               l.cip, S->grad + l.moff);
  }
  return hipGetLastError();
}

template <typename ST>
hipError_t nn_pack(tosimp_ctx* c, NNState* S) {
  for (const Layer& l : S->L) {
    const int taps = l.k * l.k * l.k;
    const int n = l.cop * taps * l.cip;
    pack_weights_kernel<ST><<<(n + 255) / 256, 256, 0, c->stream>>>(
        S->master + l.moff, l.co, l.ci, taps, l.cop, l.cip, (ST*)S->W + l.woff,
        (ST*)S->WT + l.woff);
  }
  return hipGetLastError();
}

// ||r||^2 of an FP32 vector into *out (FP64, deterministic).
__global__ __launch_bounds__(256) void norm2f_kernel(const float* r, int n, double* partials) {
  __shared__ double sred[4];
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    s += (double)r[i] * (double)r[i];
  const double v[1] = {s};
  store_block_sums<1>(v, partials, sred);
}

struct SetScalar {
  double* out;
  __device__ void operator()(const double* t) const { *out = t[0]; }
};

// ||r||^2 into *out (two launches, deterministic).
hipError_t launch_norm2f(hipStream_t s, const float* r, int n, double* partials, double* out) {
  norm2f_kernel<<<1024, 256, 0, s>>>(r, n, partials);
  return launch_finalize_sum<1>(s, partials, 1024, SetScalar{out});
}

__global__ void scale_target_kernel(const float* e, const double* enorm2, float* out, int n) {
  const float inv = (float)(sqrt((double)n) / sqrt(fmax(*enorm2, 1e-300)));  // unit RMS
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = e[i] * inv;
}

__global__ void sub_targets_kernel(const double* ustar, float* hu, int n_dof, int count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (long long)n_dof * count;
       i += (long long)gridDim.x * blockDim.x)
    hu[i] = (float)(ustar[i % n_dof] - (double)hu[i]);
}

template <typename ST>
int nn_apply_t(tosimp_ctx* ctx, NNState* S, const float* r, float* z) {
  const int nn = (int)ctx->n_node;
  // ||r||^2 as 512 block partials, added by every block of the kernel that forms the
  // network's input (in BF16 the first convolution itself; no separate finalising launch)
  norm2f_kernel<<<512, 256, 0, ctx->stream>>>(r, (int)ctx->n_dof, S->part);
  TOSIMP_HIP(ctx, nn_forward<ST>(ctx, S, /*infer=*/true, r));
  const Layer& hl = S->L[11];
  head_output_kernel<ST><<<2048, 256, 0, ctx->stream>>>(
      (const ST*)S->act[10], (const ST*)((const char*)S->W + hl.woff * S->es), hl.cip,
      ctx->ws.mask, S->scal, z, nn);
  TOSIMP_HIP(ctx, hipGetLastError());
  return TOSIMP_OK;
}

// One sample: forward on (r, rho) with r at unit RMS, loss against e at unit RMS,
// backward; the sample's
// gradient is stored or added to gacc.
template <typename ST>
int nn_sample_grad(tosimp_ctx* ctx, NNState* S, const float* r, const float* e, float* tgt,
                   float* gacc, bool first, double* loss) {
  const int nn = (int)ctx->n_node;
  TOSIMP_HIP(ctx, launch_norm2f(ctx->stream, r, (int)ctx->n_dof, S->part, S->scal));
  build_input_kernel<ST><<<2048, 256, 0, ctx->stream>>>(r, S->scal, S->rho_node, (ST*)S->act[12], nn);
  TOSIMP_HIP(ctx, nn_forward<ST>(ctx, S));
  if (S->loss_kind == 1) {
    // energy norm: n on free DOFs, K n (FP32 operator at the pair's density), the dots
    float* nd = (float*)ctx->ws.w;
    float* Knd = ctx->ws.q32;
    const int n = (int)ctx->n_dof;
    const int vb = std::min(2048, (n + 255) / 256);
    head_to_dof_kernel<ST><<<2048, 256, 0, ctx->stream>>>((const ST*)S->act[11], ctx->ws.mask, nd, nn);
    TOSIMP_HIP(ctx, kv_launch(ctx, TOSIMP_PREC_FP32, TOSIMP_F32, S->x32, nd, Knd,
                              ctx->ws.partials + 2 * kMaxPartials, ctx->ws.st + 2, S->scal + 4,
                              2, false, true));
    energy_dots_kernel<<<vb, 256, 0, ctx->stream>>>(nd, r, e, n, S->part);
    TOSIMP_HIP(ctx, launch_finalize_sum<2>(ctx->stream, S->part, vb, EnergyFin{S->scal}));
    energy_grad_kernel<ST><<<2048, 256, 0, ctx->stream>>>(r, Knd, ctx->ws.mask, S->scal,
                                                          (ST*)S->gbuf[0], nn);
  } else {
    // Target e sqrt(n_dof) / ||e|| (unit RMS, the scale of the inputs): flexible CG does
    // not depend on the scale of z.
    TOSIMP_HIP(ctx, launch_norm2f(ctx->stream, e, (int)ctx->n_dof, S->part, S->scal + 3));
    scale_target_kernel<<<2048, 256, 0, ctx->stream>>>(e, S->scal + 3, tgt, (int)ctx->n_dof);
    TOSIMP_HIP(ctx, launch_loss<ST>(ctx->stream, (const ST*)S->act[11], tgt, ctx->ws.mask, nn,
                                     S->part, S->scal + 1));
    loss_grad_kernel<ST><<<2048, 256, 0, ctx->stream>>>((const ST*)S->act[11], tgt, ctx->ws.mask,
                                                        nn, S->scal + 1, (ST*)S->gbuf[0]);
  }
  TOSIMP_HIP(ctx, nn_backward<ST>(ctx, S));
  accum_kernel<<<(int)((S->nparam + 255) / 256), 256, 0, ctx->stream>>>(gacc, S->grad, (int)S->nparam,
                                                                       first ? 0 : 1);
  double dn[2];
  TOSIMP_HIP(ctx, hipMemcpyAsync(dn, S->scal + 1, sizeof(dn), hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *loss = dn[0] > 0 ? dn[1] / dn[0] : 0.0;
  return TOSIMP_OK;
}

}  // namespace


// The learned preconditioner z = M(r) on FP32 vectors: the network correction n
// (written to z), K n into Kn, the two scalars into st, then the Jacobi stage in place.
template <typename ST>
int nn_precond_t(tosimp_ctx* ctx, NNState* S, const float* x32, const float* r, float* z,
                 float* Kn, SolverState* st, double* part, double* kvpart) {
  const int n = (int)ctx->n_dof;
  const int vb = std::min(2048, (n + 255) / 256);
  int rc = nn_apply_t<ST>(ctx, S, r, z);
  if (rc) return rc;
  TOSIMP_HIP(ctx, kv_launch(ctx, TOSIMP_PREC_FP32, TOSIMP_F32, x32, z, Kn, kvpart, st,
                            &st->s_nkn, 2, true, true));
  dot_rn_kernel<<<vb, 256, 0, ctx->stream>>>(r, z, n, st, part);
  TOSIMP_HIP(ctx, launch_finalize_sum<1>(ctx->stream, part, vb, SetRn{st}));
  two_stage_kernel<<<vb, 256, 0, ctx->stream>>>(r, Kn, ctx->ws.dinv32, z, n, st);
  TOSIMP_HIP(ctx, hipGetLastError());
  return TOSIMP_OK;
}

// Flexible CG, FCG(m), with the learned preconditioner (see the FCG kernels above).
// Vectors: r in the FP32 workspace, z and K n in the FP64 scratch w (as floats), the m
// directions and their images in the network state; the iterate is e32.
int tosimp::nn_fcg_solve(tosimp_ctx* ctx, int prec, const float* x32, const float* b32,
                         float* e32, double tol, int maxit, int check_every, int window,
                         int stall, int* iters, int* fallbacks, int* done) {
  NNState* S = nn_of(ctx);
  if (!S) return tosimp_fail(ctx, TOSIMP_ESTATE, "NN preconditioner requested but no network");
  if (window < 1) window = 1;
  if (window > kFcgMax)
    return tosimp_fail(ctx, TOSIMP_EINVAL, "flexible CG window must be at most 16");
  Workspace& w = ctx->ws;
  const int n = (int)ctx->n_dof;
  if (S->fcg_cap < window) {  // direction ring, grown on demand
    if (S->fcgP) (void)hipFree(S->fcgP);
    if (S->fcgQ) (void)hipFree(S->fcgQ);
    S->fcgP = S->fcgQ = nullptr;
    S->fcg_cap = 0;
    if (nn_alloc((void**)&S->fcgP, (size_t)window * n * 4) != hipSuccess ||
        nn_alloc((void**)&S->fcgQ, (size_t)window * n * 4) != hipSuccess)
      return tosimp_fail(ctx, TOSIMP_ENOMEM, "flexible CG directions");
    S->fcg_cap = window;
  }
  float *r = w.r32, *z = (float*)w.w;
  float* Kn = z + n;
  SolverState* st = w.st + 1;
  SolverState* sh = w.st_host + 1;
  *sh = SolverState{};
  sh->aux = tol * tol;
  sh->maxit = maxit < 1 ? 1 : maxit;
  sh->stall = stall > 0 ? stall : 0;
  TOSIMP_HIP(ctx, hipMemcpyAsync(st, sh, sizeof(SolverState), hipMemcpyHostToDevice, ctx->stream));
  node_density_kernel<float><<<2048, 256, 0, ctx->stream>>>(x32, ctx->nx, ctx->ny, ctx->nz,
                                                           S->rho_node);
  TOSIMP_HIP(ctx, launch_fill_zero(ctx, e32, (int64_t)n * 4));
  double* part = w.partials;
  double* kvpart = w.partials + 2 * kMaxPartials;
  // r = b (masked), ||r||, ||b||, tolerance; the direction written here is not used
  TOSIMP_HIP(ctx, launch_pcg_init<float>(ctx, b32, nullptr, r, S->fcgP, w.dinv32, st, part, 0));
  fcg_stall_kernel<<<1, 64, 0, ctx->stream>>>(st, 1);
  const bool mfma = prec == TOSIMP_PREC_BF16_MFMA || prec == TOSIMP_PREC_FP16_MFMA;
  const int vb = std::min(2048, (n + 255) / 256);
  if (check_every < 1) check_every = 1;
  FcgWin win{};
  for (int j = 0; j < window; ++j) {
    win.P[j] = S->fcgP + (size_t)j * n;
    win.Q[j] = S->fcgQ + (size_t)j * n;
  }
  long long k = 0;  // iterations enqueued
  for (;;) {
    TOSIMP_HIP(ctx, hipMemcpyAsync(sh, st, sizeof(SolverState), hipMemcpyDeviceToHost, ctx->stream));
    TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (sh->done) break;
    for (int i = 0; i < check_every; ++i, ++k) {
      const int slot = (int)(k % window);
      win.nw = (int)std::min<long long>(k, window);
      float* P = S->fcgP + (size_t)slot * n;
      float* Q = S->fcgQ + (size_t)slot * n;
      int rc = S->bf16 ? nn_precond_t<bf16_t>(ctx, S, x32, r, z, Kn, st, part, kvpart)
                       : nn_precond_t<float>(ctx, S, x32, r, z, Kn, st, part, kvpart);
      if (rc) return rc;
      fcgm_dots_kernel<<<vb, 256, 0, ctx->stream>>>(r, z, win, n, st, 0, part);
      TOSIMP_HIP(ctx, launch_finalize_sum<1 + kFcgMax>(ctx->stream, part, vb,
                                                      FcgmFin{st, S->fpq, S->fco, win.nw, 0}));
      fcg_jacobi_z_kernel<<<vb, 256, 0, ctx->stream>>>(r, z, w.dinv32, n, st);
      fcgm_dots_kernel<<<vb, 256, 0, ctx->stream>>>(r, z, win, n, st, 1, part);
      TOSIMP_HIP(ctx, launch_finalize_sum<1 + kFcgMax>(ctx->stream, part, vb,
                                                      FcgmFin{st, S->fpq, S->fco, win.nw, 1}));
      fcgm_direction_kernel<<<vb, 256, 0, ctx->stream>>>(z, win, S->fco, P, n, st);
      TOSIMP_HIP(ctx, hipGetLastError());
      if (mfma) {
        TOSIMP_HIP(ctx, kv_mfma_launch(ctx, prec, TOSIMP_F32, x32, P, Q, st, true));
        TOSIMP_HIP(ctx, launch_alpha_from_dot32(ctx, P, Q, kvpart, st));
      } else {
        TOSIMP_HIP(ctx, kv_launch(ctx, TOSIMP_PREC_FP32, TOSIMP_F32, x32, P, Q, kvpart, st,
                                  nullptr, 1, true, true));
      }
      fcg_store_pq_kernel<<<1, 64, 0, ctx->stream>>>(st, S->fpq, slot);
      TOSIMP_HIP(ctx, launch_pcg_update<float>(ctx, e32, r, P, Q, w.dinv32, st, part));
      fcg_stall_kernel<<<1, 64, 0, ctx->stream>>>(st, 0);
    }
  }
  *iters = sh->iter;
  *fallbacks = sh->nfallback;
  *done = sh->done;
  return TOSIMP_OK;
}

#define NN_REQUIRE(cond, code, msg)                       \
  do {                                                    \
    if (!(cond)) return tosimp_fail(ctx, code, msg);      \
  } while (0)

extern "C" {

int tosimp_nn_create(tosimp_ctx* ctx, int base, int bf16) {
  if (!ctx) return TOSIMP_EINVAL;
  NN_REQUIRE(ctx->has_mesh, TOSIMP_ESTATE, "no mesh");
  NN_REQUIRE(base == 16 || base == 32, TOSIMP_EINVAL, "base channels must be 16 or 32");
  nn_release(ctx);
  NNState* S = new NNState();
  ctx->nn = S;
  S->base = base;
  S->bf16 = bf16 ? 1 : 0;
  S->es = bf16 ? 2 : 4;
  const int b = base;
  S->g[0] = {ctx->nx + 1, ctx->ny + 1, ctx->nz + 1};
  for (int lv = 1; lv < 3; ++lv)
    S->g[lv] = {(S->g[lv - 1].X - 1) / 2 + 1, (S->g[lv - 1].Y - 1) / 2 + 1, (S->g[lv - 1].Z - 1) / 2 + 1};
  struct D { const char* n; int ci, co, k, s, li, lo; };
  const D defs[12] = {{"e0a", 4, b, 3, 1, 0, 0},         {"e0b", b, b, 3, 1, 0, 0},
                      {"d1", b, 2 * b, 3, 2, 0, 1},      {"e1", 2 * b, 2 * b, 3, 1, 1, 1},
                      {"d2", 2 * b, 4 * b, 3, 2, 1, 2},  {"m2a", 4 * b, 4 * b, 3, 1, 2, 2},
                      {"m2b", 4 * b, 4 * b, 3, 1, 2, 2}, {"u1a", 6 * b, 2 * b, 3, 1, 1, 1},
                      {"u1b", 2 * b, 2 * b, 3, 1, 1, 1}, {"u0a", 3 * b, b, 3, 1, 0, 0},
                      {"u0b", b, b, 3, 1, 0, 0},         {"head", b, 3, 1, 1, 0, 0}};
  size_t mo = 0, wo = 0;
  size_t wpart = 0;
  for (const D& d : defs) {
    Layer l;
    l.name = d.n;
    l.ci = d.ci;
    l.co = d.co;
    l.k = d.k;
    l.s = d.s;
    l.cip = ceil8(d.ci);   // the 4 input channels are padded to 8, the rest are 16k
    l.cop = ceil16(d.co);  // the 3 head outputs are padded to 16
    l.level_in = d.li;
    l.level_out = d.lo;
    const int taps = d.k * d.k * d.k;
    l.moff = mo;
    l.goff = wo;
    l.woff = wo;
    mo += (size_t)d.co * d.ci * taps;
    wo += (size_t)l.cop * taps * l.cip;
    const int nvox = S->g[d.lo].n();
    const size_t nchunk = (nvox + wgrad_chunk(nvox) - 1) / wgrad_chunk(nvox);
    wpart = std::max(wpart, nchunk * l.cop * taps * l.cip);
    S->L.push_back(l);
  }
  S->nparam = mo;
  S->npacked = wo;
  S->wpart_cap = wpart;
  const size_t n0 = S->g[0].n(), n1 = S->g[1].n();
  hipError_t e = hipSuccess;
  auto A = [&](void** p, size_t bytes) { if (e == hipSuccess) e = nn_alloc(p, bytes); };
  A((void**)&S->master, mo * 4);
  A((void**)&S->m, mo * 4);
  A((void**)&S->v, mo * 4);
  A((void**)&S->grad, mo * 4);
  A((void**)&S->gsum, mo * 4);
  A((void**)&S->x32, (size_t)ctx->n_elem * 4);
  A((void**)&S->fpq, kFcgMax * 8);
  A((void**)&S->fco, kFcgMax * 8);
  A((void**)&S->gpack, wo * 4);
  A(&S->W, wo * S->es);
  A(&S->WT, wo * S->es);
  for (int i = 0; i < 12; ++i) {
    const Layer& l = S->L[i];
    A(&S->act[i], (size_t)S->g[l.level_out].n() * l.cop * S->es);
  }
  A(&S->act[12], n0 * 8 * S->es);
  A(&S->cat1, n1 * 6 * b * S->es);
  A(&S->cat0, n0 * 3 * b * S->es);
  if (S->es == 2) A((void**)&S->u1part, n1 * 2 * b * 4);
  const size_t gsz = std::max(n0 * 3 * b, n1 * 6 * b) * S->es;
  for (int i = 0; i < 6; ++i) A(&S->gbuf[i], gsz);
  A((void**)&S->wpart, wpart * 4);
  A((void**)&S->rho_node, n0 * 4);
  A((void**)&S->scal, 64 * 8);
  A((void**)&S->part, 4096 * 8);
  if (e != hipSuccess) {
    nn_release(ctx);
    return tosimp_fail(ctx, TOSIMP_ENOMEM, "network workspace");
  }
  TOSIMP_HIP(ctx, hipMemsetAsync(S->m, 0, mo * 4, ctx->stream));
  TOSIMP_HIP(ctx, hipMemsetAsync(S->v, 0, mo * 4, ctx->stream));
  TOSIMP_HIP(ctx, hipMemsetAsync(S->master, 0, mo * 4, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TOSIMP_OK;
}

int tosimp_nn_num_params(const tosimp_ctx* ctx, int64_t* n) {
  if (!ctx || !ctx->nn || !n) return TOSIMP_EINVAL;
  *n = (int64_t)((const NNState*)ctx->nn)->nparam;
  return TOSIMP_OK;
}

int tosimp_nn_set_weights(tosimp_ctx* ctx, const float* w_host, int64_t n) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S, TOSIMP_ESTATE, "no network");
  NN_REQUIRE(w_host && n == (int64_t)S->nparam, TOSIMP_EINVAL, "weight count mismatch");
  TOSIMP_HIP(ctx, hipMemcpyAsync(S->master, w_host, n * 4, hipMemcpyHostToDevice, ctx->stream));
  TOSIMP_HIP(ctx, hipMemsetAsync(S->m, 0, n * 4, ctx->stream));
  TOSIMP_HIP(ctx, hipMemsetAsync(S->v, 0, n * 4, ctx->stream));
  S->adam_t = 0;
  if (S->bf16) TOSIMP_HIP(ctx, nn_pack<bf16_t>(ctx, S));
  else TOSIMP_HIP(ctx, nn_pack<float>(ctx, S));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TOSIMP_OK;
}

int tosimp_nn_get_weights(tosimp_ctx* ctx, float* w_host, int64_t n) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S, TOSIMP_ESTATE, "no network");
  NN_REQUIRE(w_host && n == (int64_t)S->nparam, TOSIMP_EINVAL, "weight count mismatch");
  TOSIMP_HIP(ctx, hipMemcpyAsync(w_host, S->master, n * 4, hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TOSIMP_OK;
}

// Nodal density from the element density (FP64 or FP32); kept for the following calls.
int tosimp_nn_set_density(tosimp_ctx* ctx, const void* x, int xdtype) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S, TOSIMP_ESTATE, "no network");
  NN_REQUIRE(x && (xdtype == TOSIMP_F64 || xdtype == TOSIMP_F32), TOSIMP_EINVAL,
             "bad density pointer or dtype");
  if (xdtype == TOSIMP_F64) {
    node_density_kernel<double><<<2048, 256, 0, ctx->stream>>>((const double*)x, ctx->nx, ctx->ny,
                                                                ctx->nz, S->rho_node);
    TOSIMP_HIP(ctx, launch_copy_cast_x(ctx, (const double*)x, S->x32));
  } else {
    node_density_kernel<float><<<2048, 256, 0, ctx->stream>>>((const float*)x, ctx->nx, ctx->ny,
                                                               ctx->nz, S->rho_node);
    TOSIMP_HIP(ctx, hipMemcpyAsync(S->x32, x, (size_t)ctx->n_elem * 4, hipMemcpyDeviceToDevice,
                                   ctx->stream));
  }
  TOSIMP_HIP(ctx, hipGetLastError());
  return TOSIMP_OK;
}

// Loss used by tosimp_nn_train_step and tosimp_nn_sample_grad (0: relative MSE to the
// unit-RMS error, 1: energy norm of the best multiple of the correction).
int tosimp_nn_set_loss(tosimp_ctx* ctx, int kind) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S, TOSIMP_ESTATE, "no network");
  NN_REQUIRE(kind == 0 || kind == 1, TOSIMP_EINVAL, "loss kind must be 0 or 1");
  S->loss_kind = kind;
  return TOSIMP_OK;
}

// Test hook: loss and gradient (master layout, host) of one pair (r, e) at the density
// set by tosimp_nn_set_density.
int tosimp_nn_sample_grad(tosimp_ctx* ctx, const float* r, const float* e, double* loss_host,
                          float* grad_host) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S && r && e, TOSIMP_EINVAL, "bad arguments");
  float* tgt = (float*)ctx->ws.w + ctx->n_dof;  // second half: the energy loss uses the first
  double l = 0.0;
  int rc = S->bf16 ? nn_sample_grad<bf16_t>(ctx, S, r, e, tgt, S->gsum, true, &l)
                   : nn_sample_grad<float>(ctx, S, r, e, tgt, S->gsum, true, &l);
  if (rc) return rc;
  if (grad_host)
    TOSIMP_HIP(ctx, hipMemcpyAsync(grad_host, S->gsum, S->nparam * 4, hipMemcpyDeviceToHost,
                                   ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (loss_host) *loss_host = l;
  return TOSIMP_OK;
}

int tosimp_nn_apply(tosimp_ctx* ctx, const float* r, float* z) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S && r && z && r != (const float*)z, TOSIMP_EINVAL, "bad arguments");
  return S->bf16 ? nn_apply_t<bf16_t>(ctx, S, r, z) : nn_apply_t<float>(ctx, S, r, z);
}

// The full preconditioner of the flexible CG (network, then the Jacobi stage) at the
// element density x32 (FP32; also sets the nodal density and the FP32 Jacobi diagonal).
// r, z: FP32 n_dof, distinct.  Uses the FP64 scratch vector w and solver slot 2.
int tosimp_nn_precondition(tosimp_ctx* ctx, const float* x32, const float* r, float* z) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S && x32 && r && z && r != (const float*)z, TOSIMP_EINVAL, "bad arguments");
  Workspace& w = ctx->ws;
  SolverState* st = w.st + 2;
  w.st_host[2] = SolverState{};
  TOSIMP_HIP(ctx, hipMemcpyAsync(st, w.st_host + 2, sizeof(SolverState), hipMemcpyHostToDevice,
                                 ctx->stream));
  TOSIMP_HIP(ctx, launch_diag_inv32(ctx, x32, w.dinv32));
  node_density_kernel<float><<<2048, 256, 0, ctx->stream>>>(x32, ctx->nx, ctx->ny, ctx->nz,
                                                           S->rho_node);
  float* Kn = (float*)w.w;
  double* kvpart = w.partials + 2 * kMaxPartials;
  int rc = S->bf16 ? nn_precond_t<bf16_t>(ctx, S, x32, r, z, Kn, st, w.partials, kvpart)
                   : nn_precond_t<float>(ctx, S, x32, r, z, Kn, st, w.partials, kvpart);
  if (rc) return rc;
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return TOSIMP_OK;
}

// Test hook: raw network on an FP32 channels-last [v0][4] input; out [v0][3] FP32.
int tosimp_nn_forward(tosimp_ctx* ctx, const float* x4, float* out3) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S && x4 && out3, TOSIMP_EINVAL, "bad arguments");
  const int n0 = S->g[0].n();
  if (S->bf16) {
    pad_input_kernel<bf16_t><<<2048, 256, 0, ctx->stream>>>(x4, (bf16_t*)S->act[12], n0);
    TOSIMP_HIP(ctx, nn_forward<bf16_t>(ctx, S));
    take3_bf16<<<2048, 256, 0, ctx->stream>>>((const bf16_t*)S->act[11], out3, n0);
  } else {
    pad_input_kernel<float><<<2048, 256, 0, ctx->stream>>>(x4, (float*)S->act[12], n0);
    TOSIMP_HIP(ctx, nn_forward<float>(ctx, S));
    take3_f32<<<2048, 256, 0, ctx->stream>>>((const float*)S->act[11], out3, n0);
  }
  TOSIMP_HIP(ctx, hipGetLastError());
  return TOSIMP_OK;
}

// Test hook: loss and gradients (master layout, host) for one raw input [v0][4] and
// target [v0][3] (FP32, device); the mask is the context's BC mask.
int tosimp_nn_loss_grad(tosimp_ctx* ctx, const float* x4, const float* target3, double* loss_host,
                        float* grad_host) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S && x4 && target3, TOSIMP_EINVAL, "bad arguments");
  const int n0 = S->g[0].n();
  if (S->bf16) {
    pad_input_kernel<bf16_t><<<2048, 256, 0, ctx->stream>>>(x4, (bf16_t*)S->act[12], n0);
    TOSIMP_HIP(ctx, nn_forward<bf16_t>(ctx, S));
    TOSIMP_HIP(ctx, launch_loss<bf16_t>(ctx->stream, (const bf16_t*)S->act[11], target3,
                                        ctx->ws.mask, n0, S->part, S->scal + 1));
    loss_grad_kernel<bf16_t><<<2048, 256, 0, ctx->stream>>>((const bf16_t*)S->act[11], target3,
                                                            ctx->ws.mask, n0, S->scal + 1,
                                                            (bf16_t*)S->gbuf[0]);
    TOSIMP_HIP(ctx, nn_backward<bf16_t>(ctx, S));
  } else {
    pad_input_kernel<float><<<2048, 256, 0, ctx->stream>>>(x4, (float*)S->act[12], n0);
    TOSIMP_HIP(ctx, nn_forward<float>(ctx, S));
    TOSIMP_HIP(ctx, launch_loss<float>(ctx->stream, (const float*)S->act[11], target3,
                                       ctx->ws.mask, n0, S->part, S->scal + 1));
    loss_grad_kernel<float><<<2048, 256, 0, ctx->stream>>>((const float*)S->act[11], target3,
                                                           ctx->ws.mask, n0, S->scal + 1,
                                                           (float*)S->gbuf[0]);
    TOSIMP_HIP(ctx, nn_backward<float>(ctx, S));
  }
  double dn[2];
  TOSIMP_HIP(ctx, hipMemcpyAsync(dn, S->scal + 1, sizeof(dn), hipMemcpyDeviceToHost, ctx->stream));
  if (grad_host)
    TOSIMP_HIP(ctx, hipMemcpyAsync(grad_host, S->grad, S->nparam * 4, hipMemcpyDeviceToHost, ctx->stream));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (loss_host) *loss_host = dn[0] > 0 ? dn[1] / dn[0] : 0.0;
  return TOSIMP_OK;
}

// One Adam step on the summed gradient of nb (residual, error) pairs (device FP32, DOF
// layout, nb x n_dof each), with the nodal density set by tosimp_nn_set_density.
int tosimp_nn_train_step(tosimp_ctx* ctx, const float* r_batch, const float* e_batch, int nb,
                         double lr, double* loss_host) {
  if (!ctx) return TOSIMP_EINVAL;
  NNState* S = nn_of(ctx);
  NN_REQUIRE(S && r_batch && e_batch && nb >= 1 && lr > 0, TOSIMP_EINVAL, "bad arguments");
  float* tgt = (float*)ctx->ws.w + ctx->n_dof;  // scaled target (second half of the FP64 scratch)
  float* gsum = S->gsum;
  double tot = 0.0;
  for (int s = 0; s < nb; ++s) {
    double l = 0.0;
    const float* r = r_batch + (size_t)s * ctx->n_dof;
    const float* e = e_batch + (size_t)s * ctx->n_dof;
    int rc = S->bf16 ? nn_sample_grad<bf16_t>(ctx, S, r, e, tgt, gsum, s == 0, &l)
                     : nn_sample_grad<float>(ctx, S, r, e, tgt, gsum, s == 0, &l);
    if (rc) return rc;
    tot += l;
  }
  S->adam_t += 1;
  AdamArgs a;
  a.lr = (float)lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.c1 = (float)(1.0 - std::pow(0.9, S->adam_t));
  a.c2 = (float)(1.0 - std::pow(0.999, S->adam_t));
  a.omb1 = (float)(1.0 - 0.9);
  a.omb2 = (float)(1.0 - 0.999);
  // Adam step on the batch-mean gradient (the mean loss of the batch).
  scale_kernel<<<(int)((S->nparam + 255) / 256), 256, 0, ctx->stream>>>(gsum, (int)S->nparam,
                                                                       1.0f / (float)nb);
  adam_kernel<<<(int)((S->nparam + 255) / 256), 256, 0, ctx->stream>>>(S->master, S->m, S->v, gsum,
                                                                      (int)S->nparam, a);
  if (S->bf16) TOSIMP_HIP(ctx, nn_pack<bf16_t>(ctx, S));
  else TOSIMP_HIP(ctx, nn_pack<float>(ctx, S));
  TOSIMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (loss_host) *loss_host = tot / nb;
  return TOSIMP_OK;
}

// Harvested targets: hu[k] <- u_star - hu[k] for k < count (u_star FP64, hu FP32).
int tosimp_nn_make_targets(tosimp_ctx* ctx, const double* u_star, float* harvest_u, int count) {
  if (!ctx || !ctx->has_mesh) return TOSIMP_EINVAL;
  NN_REQUIRE(u_star && harvest_u && count >= 0, TOSIMP_EINVAL, "bad arguments");
  if (count == 0) return TOSIMP_OK;
  sub_targets_kernel<<<4096, 256, 0, ctx->stream>>>(u_star, harvest_u, (int)ctx->n_dof, count);
  TOSIMP_HIP(ctx, hipGetLastError());
  return TOSIMP_OK;
}

}  // extern "C"

