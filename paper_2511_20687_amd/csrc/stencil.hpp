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
__host__ __device__ constexpr int d27_nnz(int d27) {
  return (d27_axis(d27, 0) != 0) + (d27_axis(d27, 1) != 0) + (d27_axis(d27, 2) != 0);
}
// The mirror symmetries of a box element leave 27 distinct values in the
// interior node's 26 blocks: which of them entry (p, q) of offset d holds
// (-1: a structural zero), and with which sign.
//   face  (one axis a):        diagonal F[a][p]                    -> 3a + p
//   edge  (axes a, b; normal n): diagonal E[n][p]                    -> 9 + 3n + p
//                              (a, b) and (b, a): s_a s_b EO[n]     -> 18 + n
//   corner:                    diagonal V[p]                        -> 21 + p
//                              (p, q): s_p s_q VO[n], n = 3 - p - q -> 24 + n
__host__ __device__ constexpr int d27_face_axis(int d27) {   // the nonzero axis of a face offset
  return d27_axis(d27, 0) != 0 ? 0 : (d27_axis(d27, 1) != 0 ? 1 : 2);
}
__host__ __device__ constexpr int d27_edge_normal(int d27) {   // the zero axis of an edge offset
  return d27_axis(d27, 0) == 0 ? 0 : (d27_axis(d27, 1) == 0 ? 1 : 2);
}
__host__ __device__ constexpr int box_index(int d27, int p, int q) {
  return d27_nnz(d27) == 1   ? (p == q ? 3 * d27_face_axis(d27) + p : -1)
         : d27_nnz(d27) == 2 ? (p == q ? 9 + 3 * d27_edge_normal(d27) + p
                                       : (interior_zero(d27, p, q) ? -1 : 18 + (3 - p - q)))
                             : (p == q ? 21 + p : 24 + (3 - p - q));
}
__host__ __device__ constexpr int box_sign(int d27, int p, int q) {
  return p == q ? 1 : d27_axis(d27, p) * d27_axis(d27, q);
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

// Raw buffer access to one instance's [3][cs] field (gfx9-family resource,
// word 3 = 0x00020000): the resource and the byte offset soff are wave-uniform,
// only the per-lane byte offset voff lives in a vector register, so the
// addresses cost no vector arithmetic.  Instance spans stay below 2 GiB.
template <typename T>
struct Field {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ explicit Field(const T *base)
      : r(__builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, 0x7fffffff, 0x00020000)) {}
  __device__ __forceinline__ T ld(unsigned voff, unsigned soff) const {
    if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  }
  __device__ __forceinline__ void st(T x, unsigned voff, unsigned soff) const {
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, (int)voff, (int)soff, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, x), r,
                                            (int)voff, (int)soff, 0);
  }
};

// Byte strides of a [3][cs] field with npl nodes per layer (all below 2 GiB).
struct Strides {
  unsigned cs, npl, nxp;
};

// Interior node (1 <= ix < nx, 1 <= iy < ny): w[n][c] of layer L through a
// buffer resource; voff = (nid - nxp - 1) * sizeof(T) >= 0 is the only per-lane
// value, rows and components go into the uniform offset.
template <typename T>
__device__ __forceinline__ void load_layer_uniform(T (&w)[9][3], const T *P, const Strides &B, int L,
                                                   unsigned voff) {
  const Field<T> F(P);
  const unsigned lo = (unsigned)L * B.npl;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int ry = 0; ry < 3; ++ry) {
      const unsigned so = lo + c * B.cs + ry * B.nxp;
#pragma unroll
      for (int rx = 0; rx < 3; ++rx) w[3 * ry + rx][c] = F.ld(voff + rx * (unsigned)sizeof(T), so);
    }
}

// Interior rows shared across lanes: consecutive lanes hold consecutive nodes of
// a row, so each lane loads only the x-centred value of rows dy = -1, 0, 1 of
// layer L and takes its x-neighbours from the adjacent lanes.  voff = (nid -
// nxp) * sizeof(T) >= 0.  Every lane of the wave must take part; a lane whose
// adjacent lane is not its x-neighbour (lanes 0 and 63) must not use the result.
template <typename T>
__device__ __forceinline__ void load_layer_xshare(T (&w)[9][3], const T *P, const Strides &B, int L,
                                                  unsigned voff) {
  const Field<T> F(P);
  const unsigned lo = (unsigned)L * B.npl;
  T x[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int ry = 0; ry < 3; ++ry) x[ry][c] = F.ld(voff, lo + c * B.cs + ry * B.nxp);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int ry = 0; ry < 3; ++ry) {
      w[3 * ry + 1][c] = x[ry][c];
      w[3 * ry][c] = __shfl_up(x[ry][c], 1, 64);
      w[3 * ry + 2][c] = __shfl_down(x[ry][c], 1, 64);
    }
}

// Contribution of one z-slab (dz = DZ) of the 27-point stencil to the node
// whose own value is ctr: acc += sum_n C_(dx,dy,DZ) (w[n] - ctr).
// cb: the interior block's 27 distinct values (kernel arguments), C: this
// node's case block (memory), used when !INTERIOR.
template <typename T, bool INTERIOR, int DZ>
__device__ __forceinline__ void slab(const T *cb, const T *C, const T (&w)[9][3], const T (&ctr)[3],
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
          const int bi = box_index(d27, p, q);
          if (bi < 0) continue;
          if (box_sign(d27, p, q) > 0) acc[p] += cb[bi] * du[q];
          else acc[p] -= cb[bi] * du[q];
        } else {
          acc[p] += C[d26 * 9 + p * 3 + q] * du[q];
        }
      }
    }
  }
}

}  // namespace osam
