// Device helpers of the 27-point stencil shared by the FE step kernel and the
// adjoint kernels: loading a 3x3 node neighbourhood of one layer and adding
// one z-slab of C_d (u_{i+d} - u_i) to the acceleration (Sec. 2, Eq.
// matrix_vector_form_with_dbcs with the lumped mass folded into C).
#pragma once
#include "osam_device.hpp"

namespace osam {

// Isotropic stencil on a box grid, interior node: the (p, q) block entry of
// offset d vanishes when p != q and d_p == 0 or d_q == 0 (mirror symmetry).
__host__ __device__ constexpr int d27_axis(int d27, int p) {
  return p == 0 ? d27 % 3 - 1 : (p == 1 ? (d27 % 9) / 3 - 1 : d27 / 9 - 1);
}
__host__ __device__ constexpr bool interior_zero(int d27, int p, int q) {
  return p != q && (d27_axis(d27, p) == 0 || d27_axis(d27, q) == 0);
}
// XCD-aware order: hardware hands workgroup i to XCD i % 8; give every XCD a
// contiguous range of logical blocks (chunk-major, i.e. neighbouring layers).
__device__ __forceinline__ int xcd_block(int bid, int n) {
  const int q = n >> 3, rem = n & 7, xcd = bid & 7, slot = bid >> 3;
  return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

// 3x3 neighbourhood of node layer L (SoA buffer P, component stride cs).
template <typename T, bool INTERIOR>
__device__ __forceinline__ void load_layer(T (&w)[9][3], const T *P, long long cs, int L, int npl,
                                           int nxp, int ix, int iy, int nx, int ny) {
#pragma unroll
  for (int n = 0; n < 9; ++n) {
    int jx = ix + n % 3 - 1, jy = iy + n / 3 - 1;
    if (!INTERIOR) {
      jx = jx < 0 ? 0 : (jx > nx ? nx : jx);
      jy = jy < 0 ? 0 : (jy > ny ? ny : jy);
    }
    const T *p = P + (long long)L * npl + (jx + nxp * jy);
#pragma unroll
    for (int c = 0; c < 3; ++c) w[n][c] = p[c * cs];
  }
}

// Contribution of one z-slab (dz = DZ) of the 27-point stencil to the node
// whose own value is ctr: acc += sum_n C_(dx,dy,DZ) (w[n] - ctr).
// ci: the interior case's block (kernel arguments: scalar loads), C: this node's case block.
template <typename T, bool INTERIOR, int DZ>
__device__ __forceinline__ void slab(const T *ci, const T *C, const T (&w)[9][3], const T (&ctr)[3],
                                     T (&acc)[3]) {
#pragma unroll
  for (int n = 0; n < 9; ++n) {
    const int d27 = (DZ + 1) * 9 + n;
    if (d27 == 13) continue;
    const int d26 = d27 < 13 ? d27 : d27 - 1;
    const T du[3] = {w[n][0] - ctr[0], w[n][1] - ctr[1], w[n][2] - ctr[2]};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (INTERIOR) {
          if (interior_zero(d27, p, q)) continue;
          acc[p] += ci[d26 * 9 + p * 3 + q] * du[q];
        } else {
          acc[p] += C[d26 * 9 + p * 3 + q] * du[q];
        }
      }
    }
  }
}

}  // namespace osam
