// The element product y_e = E_e K_E v_e of one hexahedron, element by element, in the
// exact Hadamard factorisation of K_E (the constants of common.h's HadConsts, scaled by
// the element edge).  Used where elements are handled one per thread: the atomic-scatter
// forms of the operator and the multigrid's smallest levels.
#pragma once

#include <hip/hip_runtime.h>

namespace tosimp {

template <typename T>
struct HexK {
  T ad, ao, cs, bd, bo, cd, co, hg;
};

// 24 element results from the 8 corner values of one element (corner q = cx + 2 cy +
// 4 cz).  Per axis the basis is {v0 + v1, v1 - v0}; mode m = mx + 2 my + 4 mz.  The
// forward transform takes (a, b) to (a + b, b - a) along each axis, the transposed one
// takes (g0, g1) back to (g0 - g1, g0 + g1); between them the 45 non-zeros of
// S = H K_E H^T / 64 (see the constants in common.h).
template <typename T>
__device__ __forceinline__ void hex_apply(T E, const HexK<T>& K, const T (&v)[8][3],
                                          T (&y)[8][3]) {
  T h[8][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int q = 0; q < 8; ++q) h[q][c] = v[q][c];
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (!(q & bit)) {
          const T a = h[q][c], b = h[q | bit][c];
          h[q][c] = a + b;
          h[q | bit][c] = b - a;
        }
  }
  const T kad = E * K.ad, kao = E * K.ao, kcs = E * K.cs, kbd = E * K.bd;
  const T kbo = E * K.bo, kcd = E * K.cd, kco = E * K.co, khg = E * K.hg;
  T g[8][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) g[0][c] = T(0);
  // normal block (1,x), (2,y), (4,z)
  const T sA = kao * (h[1][0] + h[2][1] + h[4][2]);
  g[1][0] = kad * h[1][0] + sA;
  g[2][1] = kad * h[2][1] + sA;
  g[4][2] = kad * h[4][2] + sA;
  // shear pairs
  const T s1 = kcs * (h[1][1] + h[2][0]), s2 = kcs * (h[1][2] + h[4][0]);
  const T s3 = kcs * (h[2][2] + h[4][1]);
  g[1][1] = s1; g[2][0] = s1;
  g[1][2] = s2; g[4][0] = s2;
  g[2][2] = s3; g[4][1] = s3;
  // bending pairs
  g[3][0] = kbd * h[3][0] + kbo * h[6][2];
  g[6][2] = kbo * h[3][0] + kbd * h[6][2];
  g[3][1] = kbd * h[3][1] + kbo * h[5][2];
  g[5][2] = kbo * h[3][1] + kbd * h[5][2];
  g[5][0] = kbd * h[5][0] + kbo * h[6][1];
  g[6][1] = kbo * h[5][0] + kbd * h[6][1];
  // twist block (3,z), (5,y), (6,x)
  const T sC = kco * (h[3][2] + h[5][1] + h[6][0]);
  g[3][2] = kcd * h[3][2] + sC;
  g[5][1] = kcd * h[5][1] + sC;
  g[6][0] = kcd * h[6][0] + sC;
  // hourglass
#pragma unroll
  for (int c = 0; c < 3; ++c) g[7][c] = khg * h[7][c];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int bit = 4; bit >= 1; bit >>= 1)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (!(q & bit)) {
          const T g0 = g[q][c], g1 = g[q | bit][c];
          g[q][c] = g0 - g1;
          g[q | bit][c] = g0 + g1;
        }
#pragma unroll
    for (int q = 0; q < 8; ++q) y[q][c] = g[q][c];
  }
}

}  // namespace tosimp
