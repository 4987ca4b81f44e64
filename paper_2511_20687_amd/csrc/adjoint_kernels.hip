// Kernels of the discrete adjoint of the coupled explicit rollout.
//
// With the explicit Newmark scheme (Sec. 4.1, beta = 0) every subdomain's
// displacement at t_k is its predictor, and the Schwarz data it passes on at
// t_k are built from those predictors; the accepted step (the Schwarz fixed
// point of Alg. 1) is therefore the explicit map
//   FOM:   u_k = u + dt v + dt^2/2 a,  a_k = C [u_k ; faces_k],  v_k = v + dt/2 (a + a_k)
//   OpInf: q_k = q + dt q' + dt^2/2 q'', q''_k = A q_k + H (q_k (x) q_k) + B g^_k + c,
//          q'_k = q' + dt/2 (q'' + q''_k)
// with faces_k from the sources' displacements at t_k (FOM layer copy, or
// Pi Phi q_k) and g^_k = Phi_S^T (FOM source layer) or T q_src,k (Sec. 4.2).
// These kernels evaluate that map again (checkpointed recomputation) and its
// transpose.  C = -M^-1 K with K symmetric, so C^T x = M C (M^-1 x): the
// transpose reuses the forward stencil on x / m and scales by m.
#include <hip/hip_runtime.h>

#include "adjoint.hpp"
#include "osam_device.hpp"
#include "stencil.hpp"

namespace osam {

__device__ __forceinline__ int node_case(int ix, int iy, int nx, int ny) {
  return (ix == 0 ? 0 : (ix == nx ? 2 : 1)) + 3 * (iy == 0 ? 0 : (iy == ny ? 2 : 1));
}

// out_j = s_j * sum_d C_d (in_{j+d} - in_j) on node layers k_lo..k_hi of the slab
// (s_j = mass of j's case when SCALED, else 1).  Face layers 0 and nzs take only
// the slab towards the interior (the input is zero on and beyond them).
template <typename T, bool SCALED>
__global__ void __launch_bounds__(256) stencil_kernel(SlabGeo<T> G, const T *__restrict__ in, T *__restrict__ out,
                                                      int k_lo, int k_hi) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = k_lo + blockIdx.y;
  if (col >= G.npl || k > k_hi) return;
  const int nxp = G.nx + 1, ix = col % nxp, iy = col / nxp;
  const int cse = node_case(ix, iy, G.nx, G.ny);
  const T *C = G.coef + cse * 234;
  T w[9][3], ctr[3], acc[3] = {T(0), T(0), T(0)};
  load_layer<T, false>(w, in, G.cs, k, G.npl, nxp, ix, iy, G.nx, G.ny);
#pragma unroll
  for (int c = 0; c < 3; ++c) ctr[c] = w[4][c];
  if (k > 0) {
    T wl[9][3];
    load_layer<T, false>(wl, in, G.cs, k - 1, G.npl, nxp, ix, iy, G.nx, G.ny);
    slab<T, -1>(C, wl, ctr, acc);
  }
  slab<T, 0>(C, w, ctr, acc);
  if (k < G.nzs) {
    T wh[9][3];
    load_layer<T, false>(wh, in, G.cs, k + 1, G.npl, nxp, ix, iy, G.nx, G.ny);
    slab<T, 1>(C, wh, ctr, acc);
  }
  const T sc = SCALED ? G.mass[cse] : T(1);
  const long long id = (long long)k * G.npl + col;
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c * G.cs + id] = sc * acc[c];
}

// Elementwise updates on the free layers 1..nzs-1 of [3][cs] fields.
//   mode 0: y = x0 + a1 x1 + a2 x2               (predictor)
//   mode 1: y = x0 + a1 (x1 + x2)                (velocity)
//   mode 2: y = x0 / mass (0 for held comps)     (adjoint: mu = lambda / m)
//   mode 3: y += x0                              (accumulate)
//   mode 4: x1 += a1 y ; x2 += a2 y  (y read)    (adjoint predictor: V += dt U, Aa' += h U)
//   mode 5: x0 += a1 x1 ; y = a1 x1              (adjoint velocity: Aa += g V, Aa' = g V)
//   mode 6: y = 0 on held comps                  (gradients: held components are not parameters)
template <typename T>
__global__ void __launch_bounds__(256) fom_elem_kernel(SlabGeo<T> G, int mode, T *y, T *x0, T *x1, T *x2, T a1,
                                                       T a2) {
  const long long nfree = (long long)G.npl * (G.nzs - 1);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * nfree) return;
  const int c = (int)(t / nfree);
  const long long r = t - (long long)c * nfree;
  const long long id = (long long)c * G.cs + G.npl + r;   // layer 1 onwards
  switch (mode) {
    case 0: y[id] = x0[id] + a1 * x1[id] + a2 * x2[id]; break;
    case 1: y[id] = x0[id] + a1 * (x1[id] + x2[id]); break;
    case 2:
    case 6: {
      const int col = (int)(r % G.npl), nxp = G.nx + 1, ix = col % nxp, iy = col / nxp;
      const int cse = node_case(ix, iy, G.nx, G.ny);
      const bool held = cse != 4 && ((G.held >> c) & 1);
      if (mode == 2) y[id] = held ? T(0) : x0[id] / G.mass[cse];
      else if (held) y[id] = T(0);
      break;
    }
    case 3: y[id] += x0[id]; break;
    case 4: {
      const T u = y[id];
      x1[id] += a1 * u;
      x2[id] += a2 * u;
      break;
    }
    case 5: {
      const T v = x1[id];
      x0[id] += a1 * v;
      y[id] = a1 * v;
      break;
    }
  }
}

// Misfit of one FOM slab at one observed step: U += u - obs on the free layers,
// obs in the free-DOF layout [3][free nodes]; per-workgroup FP64 partial of
// 1/2 ||u - obs||^2.
template <typename T>
__global__ void __launch_bounds__(256) fom_misfit_kernel(SlabGeo<T> G, T *U, const T *u, const T *obs,
                                                         double *partial) {
  const long long nfree = (long long)G.npl * (G.nzs - 1);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (t < 3 * nfree) {
    const int c = (int)(t / nfree);
    const long long r = t - (long long)c * nfree;
    const long long id = (long long)c * G.cs + G.npl + r;
    const T d = u[id] - obs[(long long)c * nfree + r];
    U[id] += d;
    e2 = 0.5 * (double)d * (double)d;
  }
  for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + (red[2] + red[3]));
}

// dst[c][nid] (+)= src[c][nid] for one node layer (offsets in elements).
template <typename T>
__global__ void layer_copy_kernel(T *dst, long long dst_cs, long long dst_off, const T *src, long long src_cs,
                                  long long src_off, int npl, int add) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * npl) return;
  const int c = t / npl, nid = t - c * npl;
  const T v = src[c * src_cs + src_off + nid];
  T &d = dst[c * dst_cs + dst_off + nid];
  d = add ? d + v : v;
}

// Face of a FOM slab from an OpInf source: dst = (Pi Phi) q (rows [r][3 npl]).
template <typename T>
__global__ void lift_face_kernel(const T *piphi, const T *q, int r, T *dst, long long dst_cs, long long dst_off,
                                 int npl) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = 3 * npl;
  if (m >= n) return;
  T s = T(0);
  for (int k = 0; k < r; ++k) s += piphi[(long long)k * n + m] * q[k];
  const int c = m / npl, nid = m - c * npl;
  dst[c * dst_cs + dst_off + nid] = s;
}

// y[k] += sum_m M[k][m] x[m]  (M [rows][n] column blocks of length n), one wave per row.
template <typename T>
__global__ void rows_dot_kernel(const T *M, int rows, int n, const T *x, long long x_cs, long long x_off, int npl,
                                T *y) {
  const int lane = threadIdx.x & 63, w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= rows) return;
  double s = 0.0;
  for (int m = lane; m < n; m += 64) {
    const int c = m / npl, nid = m - c * npl;
    s += (double)M[(long long)w * n + m] * (double)x[c * x_cs + x_off + nid];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[w] += (T)s;
}

// x[c][nid] += sum_k M[k][m] y[k] (transpose of rows_dot into a face layer).
template <typename T>
__global__ void rows_tdot_kernel(const T *M, int rows, int n, const T *y, T *x, long long x_cs, long long x_off,
                                 int npl) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  T s = T(0);
  for (int k = 0; k < rows; ++k) s += M[(long long)k * n + m] * y[k];
  const int c = m / npl, nid = m - c * npl;
  x[c * x_cs + x_off + nid] += s;
}

// Forward: q_k (predictor), q''_k = f(q_k, g^_k), q'_k; records the tape (mode 2: predictor only).
template <typename T>
__global__ void __launch_bounds__(256) rom_fwd_kernel(RomAdj<T> R) {
  extern __shared__ unsigned char smem_raw[];
  T *qk = reinterpret_cast<T *>(smem_raw);
  T *k2 = qk + R.r;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  for (int i = tid; i < R.r; i += blockDim.x) {
    qk[i] = R.q[i] + R.dt * R.qd[i] + R.h * R.qdd[i];
    R.tape_q[i] = qk[i];
  }
  if (R.mode == 2) return;   // predictor only
  for (int l = tid; l < R.rs; l += blockDim.x) R.tape_g[l] = R.gh[l];
  __syncthreads();
  if (R.r2 > 0) {
    for (int idx = tid; idx < R.r * R.r; idx += blockDim.x) {
      const int i = idx / R.r, j = idx - i * R.r;
      if (j >= i) k2[i * R.r - (i * (i - 1)) / 2 + (j - i)] = qk[i] * qk[j];
    }
    __syncthreads();
  }
  for (int i = wid; i < R.r; i += nw) {
    T s = T(0);
    for (int j = lane; j < R.r; j += 64) s += R.A[(long long)i * R.r + j] * qk[j];
    if (R.r2 > 0)
      for (int m = lane; m < R.r2; m += 64) s += R.H[(long long)i * R.r2 + m] * k2[m];
    for (int l = lane; l < R.rs; l += 64) s += R.B[(long long)i * R.rs + l] * R.gh[l];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) {
      const T an = s + (R.c ? R.c[i] : T(0));
      R.qd[i] = R.qd[i] + R.g * (R.qdd[i] + an);
      R.qdd[i] = an;
      R.q[i] = qk[i];
    }
  }
}

// Adjoint of one OpInf step (mode 0) or of q''_0 = f(q_0, g^_0) (mode 1):
//   Qdd += g Qd ; Qdd_prev = g Qd                         (velocity)
//   Q += q_k - obs                                        (misfit)
//   dA += Qdd q^T, dH += Qdd (q (x) q)^T, dB += Qdd g^T, dc += Qdd
//   Q += A^T Qdd + J_H(q)^T Qdd ; gbar = B^T Qdd          (acceleration)
// The predictor transpose (Qd += dt Q, Qdd_prev += h Q) follows in
// rom_adj_pred_kernel, after the FOM faces have added their part to Q.
template <typename T>
__global__ void __launch_bounds__(256) rom_adj_kernel(RomAdj<T> R) {
  extern __shared__ unsigned char smem_raw[];
  T *qk = reinterpret_cast<T *>(smem_raw);
  T *qdd = qk + R.r;
  T *k2 = qdd + R.r;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  double e2 = 0.0;
  for (int i = tid; i < R.r; i += blockDim.x) {
    qk[i] = R.tape_q[i];
    T a = R.Qdd[i];
    if (R.mode == 0) {
      a += R.g * R.Qd[i];
      R.Qdd_prev[i] = R.g * R.Qd[i];
    }
    qdd[i] = a;
    R.Qdd[i] = a;
    if (R.obs) {
      const T d = qk[i] - R.obs[i];
      R.Q[i] += d;
      e2 += 0.5 * (double)d * (double)d;
    }
  }
  for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o, 64);
  __shared__ double red[16];
  if (lane == 0) red[wid] = e2;
  __syncthreads();
  if (tid == 0 && R.partial) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    R.partial[0] = s;
  }
  if (R.r2 > 0) {
    for (int idx = tid; idx < R.r * R.r; idx += blockDim.x) {
      const int i = idx / R.r, j = idx - i * R.r;
      if (j >= i) k2[i * R.r - (i * (i - 1)) / 2 + (j - i)] = qk[i] * qk[j];
    }
  }
  __syncthreads();
  // gradients (rows i of the operators)
  for (int idx = tid; idx < R.r * R.r; idx += blockDim.x) {
    const int i = idx / R.r, j = idx - i * R.r;
    R.dA[idx] += (double)qdd[i] * (double)qk[j];
  }
  if (R.r2 > 0)
    for (long long idx = tid; idx < (long long)R.r * R.r2; idx += blockDim.x) {
      const int i = (int)(idx / R.r2);
      const int m = (int)(idx - (long long)i * R.r2);
      R.dH[idx] += (double)qdd[i] * (double)k2[m];
    }
  if (R.rs > 0)
    for (int idx = tid; idx < R.r * R.rs; idx += blockDim.x) {
      const int i = idx / R.rs, l = idx - i * R.rs;
      R.dB[idx] += (double)qdd[i] * (double)R.tape_g[l];
    }
  if (R.dc)
    for (int i = tid; i < R.r; i += blockDim.x) R.dc[i] += (double)qdd[i];
  // Q_j += sum_i Qdd_i (A_ij + dH(q)_i/dq_j); d(q_a q_b)/dq_j = q_b [a == j] + q_a [b == j]
  for (int j = wid; j < R.r; j += nw) {
    double s = 0.0;
    for (int i = lane; i < R.r; i += 64) {
      double t = (double)R.A[(long long)i * R.r + j];
      if (R.r2 > 0) {
        const T *Hr = R.H + (long long)i * R.r2;
        // entries (a, b) with a <= b containing j: (j, b >= j) and (a <= j, j)
        const int row_j = j * R.r - (j * (j - 1)) / 2;   // start of row a = j
        for (int b = j; b < R.r; ++b) t += (double)Hr[row_j + (b - j)] * (double)qk[b];
        for (int a = 0; a <= j; ++a) t += (double)Hr[a * R.r - (a * (a - 1)) / 2 + (j - a)] * (double)qk[a];
      }
      s += t * (double)qdd[i];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) R.Q[j] += (T)s;
  }
  // gbar = B^T Qdd
  for (int l = wid; l < R.rs; l += nw) {
    double s = 0.0;
    for (int i = lane; i < R.r; i += 64) s += (double)R.B[(long long)i * R.rs + l] * (double)qdd[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) R.gbar[l] = (T)s;
  }
}

template <typename T>
__global__ void rom_adj_pred_kernel(RomAdj<T> R) {
  for (int i = threadIdx.x; i < R.r; i += blockDim.x) {
    const T u = R.Q[i];
    R.Qd[i] += R.dt * u;
    R.Qdd_prev[i] += R.h * u;
  }
}

// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_stencil(const SlabGeo<T> &G, const T *in, T *out, int k_lo, int k_hi, bool scaled,
                          hipStream_t s) {
  const dim3 grid((G.npl + 255) / 256, k_hi - k_lo + 1);
  if (scaled) hipLaunchKernelGGL((stencil_kernel<T, true>), grid, dim3(256), 0, s, G, in, out, k_lo, k_hi);
  else hipLaunchKernelGGL((stencil_kernel<T, false>), grid, dim3(256), 0, s, G, in, out, k_lo, k_hi);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fom_elem(const SlabGeo<T> &G, int mode, T *y, T *x0, T *x1, T *x2, T a1, T a2, hipStream_t s) {
  const long long n = 3LL * G.npl * (G.nzs - 1);
  hipLaunchKernelGGL(fom_elem_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, mode, y, x0, x1,
                     x2, a1, a2);
  return hipGetLastError();
}
template <typename T>
int fom_misfit_blocks(const SlabGeo<T> &G) {
  return (int)((3LL * G.npl * (G.nzs - 1) + 255) / 256);
}
template <typename T>
hipError_t launch_fom_misfit(const SlabGeo<T> &G, T *U, const T *u, const T *obs, double *partial, hipStream_t s) {
  hipLaunchKernelGGL(fom_misfit_kernel<T>, dim3(fom_misfit_blocks(G)), dim3(256), 0, s, G, U, u, obs, partial);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_layer_copy(T *dst, long long dst_cs, long long dst_off, const T *src, long long src_cs,
                             long long src_off, int npl, int add, hipStream_t s) {
  hipLaunchKernelGGL(layer_copy_kernel<T>, dim3((3 * npl + 255) / 256), dim3(256), 0, s, dst, dst_cs, dst_off, src,
                     src_cs, src_off, npl, add);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_lift_face(const T *piphi, const T *q, int r, T *dst, long long dst_cs, long long dst_off, int npl,
                            hipStream_t s) {
  hipLaunchKernelGGL(lift_face_kernel<T>, dim3((3 * npl + 255) / 256), dim3(256), 0, s, piphi, q, r, dst, dst_cs,
                     dst_off, npl);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_rows_dot(const T *M, int rows, int n, const T *x, long long x_cs, long long x_off, int npl, T *y,
                           hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(rows_dot_kernel<T>, dim3((rows + 3) / 4), dim3(256), 0, s, M, rows, n, x, x_cs, x_off, npl, y);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_rows_tdot(const T *M, int rows, int n, const T *y, T *x, long long x_cs, long long x_off, int npl,
                            hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(rows_tdot_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, s, M, rows, n, y, x, x_cs, x_off,
                     npl);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_rom_fwd(const RomAdj<T> &R, hipStream_t s) {
  const size_t smem = sizeof(T) * (size_t)(R.r + (R.r2 > 0 ? R.r2 : 1));
  if (smem > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rom_fwd_kernel<T>, dim3(1), dim3(256), smem, s, R);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_rom_adj(const RomAdj<T> &R, hipStream_t s) {
  const size_t smem = sizeof(T) * (size_t)(2 * R.r + (R.r2 > 0 ? R.r2 : 1));
  if (smem > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rom_adj_kernel<T>, dim3(1), dim3(256), smem, s, R);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_rom_adj_pred(const RomAdj<T> &R, hipStream_t s) {
  hipLaunchKernelGGL(rom_adj_pred_kernel<T>, dim3(1), dim3(256), 0, s, R);
  return hipGetLastError();
}

#define OSAM_ADJ_INST(T)                                                                                      \
  template hipError_t launch_stencil<T>(const SlabGeo<T> &, const T *, T *, int, int, bool, hipStream_t);       \
  template hipError_t launch_fom_elem<T>(const SlabGeo<T> &, int, T *, T *, T *, T *, T, T, hipStream_t);      \
  template int fom_misfit_blocks<T>(const SlabGeo<T> &);                                                       \
  template hipError_t launch_fom_misfit<T>(const SlabGeo<T> &, T *, const T *, const T *, double *, hipStream_t); \
  template hipError_t launch_layer_copy<T>(T *, long long, long long, const T *, long long, long long, int, int, \
                                           hipStream_t);                                                      \
  template hipError_t launch_lift_face<T>(const T *, const T *, int, T *, long long, long long, int, hipStream_t); \
  template hipError_t launch_rows_dot<T>(const T *, int, int, const T *, long long, long long, int, T *,          \
                                         hipStream_t);                                                        \
  template hipError_t launch_rows_tdot<T>(const T *, int, int, const T *, T *, long long, long long, int,        \
                                          hipStream_t);                                                       \
  template hipError_t launch_rom_fwd<T>(const RomAdj<T> &, hipStream_t);                                        \
  template hipError_t launch_rom_adj<T>(const RomAdj<T> &, hipStream_t);                                        \
  template hipError_t launch_rom_adj_pred<T>(const RomAdj<T> &, hipStream_t);
OSAM_ADJ_INST(float)
OSAM_ADJ_INST(double)

}  // namespace osam
