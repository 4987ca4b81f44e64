// OpInf subdomain step (one workgroup per instance), fused with the Schwarz
// transfers that touch a reduced model.
//
// Method: Sec. 4.2, Eq. opinf_model_schwarz with the signs folded into the
// operators, q'' = A q + H (q (x) q) + B g^ + c, advanced by the same explicit
// Newmark-beta (beta = 0, gamma = 1/2) as the FOM (Eq. schwarz_opinf_discrete
// read as textbook Newmark).  Inputs on the overlap boundary (Sec. 4.2.2/4.2.3):
//   FOM neighbour:  g^ = Phi_S^T s, s = the face values the neighbour pushed
//   ROM neighbour:  g^ = (Phi_S^T Pi Phi_src) q_src (precomputed r_S x r_src)
// Output to FOM neighbours: (Pi Phi) q at the next step (the Newmark predictor),
// pushed into the neighbour's face layer; only the rows of Phi that the
// projection touches are kept.  The convergence sums use reduced coordinates
// (Phi has orthonormal columns).
//
// Fused path (small batches): A q + H (q (x) q) is evaluated with one wave per
// output row from the compressed quadratic vector staged in LDS.  Batched path
// (rom_pre_kernels.hip): f0 and the FOM-fed g^ arrive as partial sums.
#include <hip/hip_ext.h>

#include "rom_body.hpp"

namespace osam {

template <typename T, int V>
__global__ void __launch_bounds__(kRomThreads) rom_kernel(RomArgs<T> A) {
  rom_body<T, V>(A, blockIdx.x, StatusOf<T>{A});
}

template <typename T>
size_t rom_smem_bytes(int r, int rs, int r2) {
  return sizeof(T) * (size_t)(3 * r + (rs > 0 ? rs : 1) + (r2 > 0 ? r2 : 0));
}

template <typename T>
hipError_t launch_rom(const RomArgs<T> &A, int batch, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const size_t smem = rom_smem_bytes<T>(A.r, A.rs, A.r2);
  if (smem > 65536) return hipErrorInvalidValue;
  int rows = 0;
  for (int e = 0; e < A.nexp; ++e) rows = rows > 3 * A.ex[e].npl ? rows : 3 * A.ex[e].npl;
  const int G = rows > 0 ? (rows + kRomThreads - 1) / kRomThreads : 1;
  const dim3 grid(G, batch), block(kRomThreads);
  const int v = rom_variant(A);
  if constexpr (sizeof(T) == 8) {   // the batched parts are FP32 only
    if (v & kRomPre) return hipErrorInvalidValue;
    if (v == kRomNoPushRegs) hipExtLaunchKernelGGL((rom_kernel<T, kRomNoPushRegs>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
    else if (v == kRomWide) hipExtLaunchKernelGGL((rom_kernel<T, kRomWide>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
    else hipExtLaunchKernelGGL((rom_kernel<T, 0>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
  } else {
    if (v == 5) hipExtLaunchKernelGGL((rom_kernel<T, 5>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
    else if (v == 4) hipExtLaunchKernelGGL((rom_kernel<T, 4>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
    else if (v == 3) hipExtLaunchKernelGGL((rom_kernel<T, 3>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
    else if (v == 2) hipExtLaunchKernelGGL((rom_kernel<T, 2>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
    else if (v == 1) hipExtLaunchKernelGGL((rom_kernel<T, 1>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
    else hipExtLaunchKernelGGL((rom_kernel<T, 0>), grid, block, (uint32_t)smem, s, ev0, ev1, 0, A);
  }
  return hipGetLastError();
}
template hipError_t launch_rom<float>(const RomArgs<float> &, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_rom<double>(const RomArgs<double> &, int, hipStream_t, hipEvent_t, hipEvent_t);
template size_t rom_smem_bytes<float>(int, int, int);
template size_t rom_smem_bytes<double>(int, int, int);

// ---------------------------------------------------------------------------
// Initial reduced state: q0 = Phi^T u0, q'0 = Phi^T v0 (free DOFs), then
// q''0 = f(q0, g^0) with g^0 = Phi_S^T s0 from the IC on the Schwarz DOFs.
// Phi is column-major [r][n_free]; the free DOF vector [3][free nodes] is read
// straight from the subdomain-layout IC arrays (layers 1..nzs-1).
template <typename T>
__global__ void __launch_bounds__(256) project_kernel(const T *__restrict__ phi, long long nfree3,
                                                      long long nfree_nodes, const T *__restrict__ x,
                                                      long long x_cs, long long x_off,
                                                      double *__restrict__ partial, int nchunks) {
  // grid: (nchunks, r); partial[k][chunk]
  const int k = blockIdx.y;
  const long long per = (nfree3 + nchunks - 1) / nchunks;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < nfree3 ? lo + per : nfree3;
  double acc = 0.0;
  for (long long m = lo + threadIdx.x; m < hi; m += blockDim.x) {
    const long long c = m / nfree_nodes, fn = m - c * nfree_nodes;
    acc += (double)phi[(long long)k * nfree3 + m] * (double)x[c * x_cs + x_off + fn];
  }
  acc = wave_sum_d(acc);
  __shared__ double red[16];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    partial[(long long)k * nchunks + blockIdx.x] = s;
  }
}

template <typename T>
hipError_t launch_project(const T *phi, long long nfree3, long long nfree_nodes, const T *x,
                          long long x_cs, long long x_off, double *partial, int nchunks, int r,
                          hipStream_t s) {
  hipLaunchKernelGGL(project_kernel<T>, dim3(nchunks, r), dim3(256), 0, s, phi, nfree3, nfree_nodes,
                     x, x_cs, x_off, partial, nchunks);
  return hipGetLastError();
}
template hipError_t launch_project<float>(const float *, long long, long long, const float *, long long,
                                          long long, double *, int, int, hipStream_t);
template hipError_t launch_project<double>(const double *, long long, long long, const double *,
                                           long long, long long, double *, int, int, hipStream_t);

// Lift: u_free = Phi q for one instance into a [3][n_nodes] field (layers 1..nzs-1).
template <typename T>
__global__ void lift_kernel(const T *__restrict__ phi, long long nfree3, long long nfree_nodes, int r,
                            const T *__restrict__ q, T *__restrict__ out, long long out_cs,
                            long long out_off) {
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nfree3) return;
  T s = T(0);
  for (int k = 0; k < r; ++k) s += phi[(long long)k * nfree3 + m] * q[k];
  const long long c = m / nfree_nodes, fn = m - c * nfree_nodes;
  out[c * out_cs + out_off + fn] = s;
}

template <typename T>
hipError_t launch_lift(const T *phi, long long nfree3, long long nfree_nodes, int r, const T *q, T *out,
                       long long out_cs, long long out_off, hipStream_t s) {
  const int blocks = (int)((nfree3 + 255) / 256);
  hipLaunchKernelGGL(lift_kernel<T>, dim3(blocks), dim3(256), 0, s, phi, nfree3, nfree_nodes, r, q, out,
                     out_cs, out_off);
  return hipGetLastError();
}
template hipError_t launch_lift<float>(const float *, long long, long long, int, const float *, float *,
                                       long long, long long, hipStream_t);
template hipError_t launch_lift<double>(const double *, long long, long long, int, const double *,
                                        double *, long long, long long, hipStream_t);

}  // namespace osam
