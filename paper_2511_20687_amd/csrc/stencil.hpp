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
// Row sums of the interior stencil along x: K = sum over the nine (dy, dz) of
// C_(dx,dy,dz) for dx = +1 or -1.  Its entry (p, q) collects, with signs, the
// box values listed below; kx_count returns the signed multiplicity of box value
// i in it.  Off the diagonal the signs cancel in pairs (edges and corners carry
// s_p s_q, odd in dy or dz), so K is diagonal: K_pp = F[0][p] + 2 E[2][p] +
// 2 E[1][p] + 4 V[p] (checked at compile time below).
__host__ __device__ constexpr int kx_count(int dx, int p, int q, int i) {
  int n = 0;
  for (int dz = 0; dz < 3; ++dz)
    for (int dy = 0; dy < 3; ++dy) {
      const int d27 = dz * 9 + dy * 3 + (dx + 1);
      if (box_index(d27, p, q) == i) n += box_sign(d27, p, q);
    }
  return n;
}
__host__ __device__ constexpr bool kx_is_diagonal_sum() {
  for (int dx = -1; dx <= 1; dx += 2)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q)
        for (int i = 0; i < 27; ++i) {
          int want = 0;
          if (p == q) want = (i == p) + 2 * (i == 15 + p) + 2 * (i == 12 + p) + 4 * (i == 21 + p);
          if (kx_count(dx, p, q, i) != want) return false;
        }
  return true;
}
static_assert(kx_is_diagonal_sum(), "x row sums of the interior stencil");

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

// load_layer of a boundary column on an x-face (ix = 0 or nx; FP32): the row's two
// x-positions of the node's own x-cell in one 8-byte load (4-byte alignment suffices),
// the clamped third position a copy of the face value, as load_layer would read it.
// Lanes of an x-face wave sit a row apart, so each lane's loads touch lines of their
// own: a third of the load instructions.  The 8 bytes are split by shifts (the FP32
// pair taken as the two elements of a vector load compiled to one 4-byte load).
typedef unsigned long long osam_u64_a4 __attribute__((aligned(4)));
__device__ __forceinline__ void load_layer_xface(float (&w)[9][3], const float *P, long long cs, int L, int npl,
                                                 int nxp, int ix, int iy, int nx, int ny) {
  const int j0 = ix == 0 ? 0 : nx - 1;   // x-positions j0, j0 + 1
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    int jy = iy + r - 1;
    jy = jy < 0 ? 0 : (jy > ny ? ny : jy);
    const float *p = P + (long long)L * npl + (j0 + nxp * jy);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned long long v = *reinterpret_cast<const osam_u64_a4 *>(p + c * cs);
      const float x0 = __builtin_bit_cast(float, (unsigned)v), x1 = __builtin_bit_cast(float, (unsigned)(v >> 32));
      w[3 * r][c] = x0;                      // x - 1 (clamped to 0 on the low face)
      w[3 * r + 1][c] = ix == 0 ? x0 : x1;   // the face
      w[3 * r + 2][c] = x1;                  // x + 1 (clamped to nx on the high face)
    }
  }
}

// load_layer of a boundary column on a y-face (iy = 0 or ny, 1 <= ix < nx; FP32): the
// two distinct rows (the face row and the row next to it; the clamped third is a copy of the
// face row), each component as one 8-byte load of x - 1, x and one 4-byte load of x + 1:
// 12 load instructions per layer instead of 27, the same values.
__device__ __forceinline__ void load_layer_yface(float (&w)[9][3], const float *P, long long cs, int L, int npl,
                                                 int nxp, int ix, int iy, int ny) {
  const int jin = iy == 0 ? 1 : ny - 1;   // the row next to the face
  float f[3][3], g[3][3];                  // [x - 1, x, x + 1][c] of the face row and of row jin
  const float *pf = P + (long long)L * npl + (ix - 1 + nxp * iy);
  const float *pg = P + (long long)L * npl + (ix - 1 + nxp * jin);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const unsigned long long a = *reinterpret_cast<const osam_u64_a4 *>(pf + c * cs);
    const unsigned long long b = *reinterpret_cast<const osam_u64_a4 *>(pg + c * cs);
    f[0][c] = __builtin_bit_cast(float, (unsigned)a);
    f[1][c] = __builtin_bit_cast(float, (unsigned)(a >> 32));
    f[2][c] = pf[c * cs + 2];
    g[0][c] = __builtin_bit_cast(float, (unsigned)b);
    g[1][c] = __builtin_bit_cast(float, (unsigned)(b >> 32));
    g[2][c] = pg[c * cs + 2];
  }
#pragma unroll
  for (int dx = 0; dx < 3; ++dx)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // rows dy = -1, 0, +1: on the low face -1 clamps to the face, on the high face +1 does
      w[dx][c] = iy == 0 ? f[dx][c] : g[dx][c];
      w[3 + dx][c] = f[dx][c];
      w[6 + dx][c] = iy == 0 ? g[dx][c] : f[dx][c];
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
// The x-centred values x[ry][c] of rows dy = ry - 1 of layer L at this lane's node.
template <typename T>
__device__ __forceinline__ void load_rows(T (&x)[3][3], const T *P, const Strides &B, int L, unsigned voff) {
  const Field<T> F(P);
  const unsigned lo = (unsigned)L * B.npl;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int ry = 0; ry < 3; ++ry) x[ry][c] = F.ld(voff, lo + c * B.cs + ry * B.nxp);
}

template <typename T>
__device__ __forceinline__ void load_layer_xshare(T (&w)[9][3], const T *P, const Strides &B, int L,
                                                  unsigned voff) {
  T x[3][3];
  load_rows<T>(x, P, B, L, voff);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int ry = 0; ry < 3; ++ry) {
      w[3 * ry + 1][c] = x[ry][c];
      w[3 * ry][c] = lane_prev(x[ry][c]);
      w[3 * ry + 2][c] = lane_next(x[ry][c]);
    }
}

// Interior nodes in x-resolved form.  With d = (dx, dy, dz) and u_{i+dx} the
// node of the same row at x offset dx, u_{i+d} - u_i = (u_{i+d} - u_{i+dx}) +
// (u_{i+dx} - u_i), so
//   sum_d C_d (u_{i+d} - u_i) = (S_0(i) + S_-1(i-1) + S_+1(i+1))
//                               + K ((u_{i-1} - u_i) + (u_{i+1} - u_i)),
// S_dx(j) = sum over the (dy, dz) rows of C_(dx,dy,dz) (u_row(j) - u(j)) formed
// at column j from its own values, K the x row sum of the blocks (diagonal:
// kx_is_diagonal_sum).  Every interior path adds in this order (rows in (dz, dy)
// order into S_-1, S_0, S_+1, then x_combine), so all layouts give the same bits;
// the x-shared one forms S_dx where the values are and moves only 3-vectors
// across lanes.
//
// s[p] += sum_q C_(d27)[p][q] d[q] over the box values (structural zeros skipped).
template <typename T>
__device__ __forceinline__ void xrow(const T *cb, int d27, const T (&d)[3], T (&s)[3]) {
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int bi = box_index(d27, p, q);
      if (bi < 0) continue;
      if (box_sign(d27, p, q) > 0) s[p] += cb[bi] * d[q];
      else s[p] -= cb[bi] * d[q];
    }
}
// Rows (dy = 0, 1, 2 - 1) of z-slab dz = DZ - 1 into S_-1 (sm), S_0 (s0), S_+1 (sp),
// from the slab's full 3x3 neighbourhood w and the centre slab wc (the three
// columns' own values wc[3], wc[4], wc[5]).
template <typename T>
__device__ __forceinline__ void xslab(const T *cb, int DZ, const T (&w)[9][3], const T (&wc)[9][3], T (&sm)[3],
                                      T (&s0)[3], T (&sp)[3]) {
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
    if (DZ == 1 && dy == 1) continue;   // the node's own row: u_row - u = 0
#pragma unroll
    for (int rx = 0; rx < 3; ++rx) {
      const T d[3] = {w[3 * dy + rx][0] - wc[3 + rx][0], w[3 * dy + rx][1] - wc[3 + rx][1],
                      w[3 * dy + rx][2] - wc[3 + rx][2]};
      xrow<T>(cb, DZ * 9 + dy * 3 + rx, d, rx == 0 ? sm : (rx == 1 ? s0 : sp));
    }
  }
}
// The x row sum K (diagonal entry p) and the final combination.
template <typename T>
__device__ __forceinline__ T kx_diag(const T *cb, int p) {
  return cb[p] + T(2) * (cb[15 + p] + cb[12 + p]) + T(4) * cb[21 + p];
}
template <typename T>
__device__ __forceinline__ T x_combine(T s0, T sm, T sp, T kx, T um, T u, T up) {
  return (s0 + sm + sp) + kx * ((um - u) + (up - u));
}

// Contribution of one z-slab (dz = DZ) of the 27-point stencil to a node of
// the boundary columns (interior nodes: xslab) whose own value is ctr:
// acc += sum_n C_(dx,dy,DZ) (w[n] - ctr), C the node's case block (memory).
template <typename T, int DZ>
__device__ __forceinline__ void slab(const T *C, const T (&w)[9][3], const T (&ctr)[3], T (&acc)[3],
                                     int skip = 0) {
  // skip (wave-uniform): components whose coefficient rows are zero (held lateral
  // components of the boundary cases); each acc[p] sums over n, q in the same order
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    if ((skip >> p) & 1) continue;
#pragma unroll
    for (int n = 0; n < 9; ++n) {
      const int d27 = (DZ + 1) * 9 + n;
      if (d27 == 13) continue;
      const int d26 = d27 < 13 ? d27 : d27 - 1;
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[p] += C[d26 * 9 + p * 3 + q] * (w[n][q] - ctr[q]);
    }
  }
}

}  // namespace osam
