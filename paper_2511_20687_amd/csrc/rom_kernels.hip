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
// This variant serves small batches: H (q (x) q) is evaluated with one wave per
// output row from the compressed quadratic vector staged in LDS.
#include "osam_device.hpp"

namespace osam {

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <typename T>
__global__ void __launch_bounds__(1024) rom_kernel(RomArgs<T> A) {
  const int b = blockIdx.x;
  Status *stp = A.status + b;
  if (stp->flags & kFinished) return;
  const long long step = stp->step;
  const int n_iter = stp->iter + 1;
  const int s2 = (int)(step % 2);
  const int r = A.r, rs = A.rs, r2 = A.r2;
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = bs >> 6;

  extern __shared__ unsigned char smem_raw[];
  T *q1s = reinterpret_cast<T *>(smem_raw);
  T *qdd1s = q1s + r;
  T *sh = qdd1s + r;
  T *k2 = sh + (rs > 0 ? rs : 1);
  __shared__ double red[2][16];

  const T *q0 = A.q[s2] + (long long)b * r;
  const T *qd0 = A.qd[s2] + (long long)b * r;
  const T *qdd0 = A.qdd[s2] + (long long)b * r;
  T *q1 = A.q[1 - s2] + (long long)b * r;
  T *qd1 = A.qd[1 - s2] + (long long)b * r;
  T *qdd1 = A.qdd[1 - s2] + (long long)b * r;

  // 1. displacement at t_k: Newmark predictor of the accepted state
  for (int i = tid; i < r; i += bs) q1s[i] = q0[i] + A.dt * qd0[i] + A.half_dt2 * qdd0[i];
  for (int k = tid; k < rs; k += bs) sh[k] = T(0);
  __syncthreads();

  // 2. reduced boundary input g^
  for (int fi = 0; fi < A.nfaces; ++fi) {
    const RomFaceIn<T> &f = A.fin[fi];
    const bool hold = n_iter == 1 && f.src_sd > A.sd && A.opts.guess == 0;
    if (f.type == kFaceFom) {
      // g^_k += sum_m Phi_S[m, k] s_m : one wave per mode k, lanes over the face DOFs
      const T *src = f.sface[hold ? (int)(step % 3) : (int)((step + 1) % 3)] + (long long)b * f.n;
      for (int k = wid; k < rs; k += nw) {
        const T *ph = f.phis + (long long)k * f.n;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
        int m = lane;
        for (; m + 192 < f.n; m += 256) {
          v0 += (double)(ph[m] * src[m]);
          v1 += (double)(ph[m + 64] * src[m + 64]);
          v2 += (double)(ph[m + 128] * src[m + 128]);
          v3 += (double)(ph[m + 192] * src[m + 192]);
        }
        for (; m < f.n; m += 64) v0 += (double)(ph[m] * src[m]);
        const double v = wave_sum_d((v0 + v1) + (v2 + v3));
        if (lane == 0) sh[k] += (T)v;
      }
      __syncthreads();
    } else {
      const T *qs = f.src_q[hold ? s2 : 1 - s2] + (long long)b * f.src_r;
      for (int k = wid; k < rs; k += nw) {
        double v = 0.0;
        for (int j = lane; j < f.src_r; j += 64) v += (double)(f.tm[(long long)k * f.src_r + j] * qs[j]);
        v = wave_sum_d(v);
        if (lane == 0) sh[k] += (T)v;
      }
      __syncthreads();
    }
  }

  // 3. compressed quadratic vector q_i q_j (i <= j), row by row
  if (r2 > 0) {
    for (int idx = tid; idx < r * r; idx += bs) {
      const int i = idx / r, j = idx - i * r;
      if (j >= i) k2[i * r - (i * (i - 1)) / 2 + (j - i)] = q1s[i] * q1s[j];
    }
    __syncthreads();
  }

  // 4. q''(t_k) = A q + H k2 + B g^ + c, one wave per row
  for (int i = wid; i < r; i += nw) {
    T s = T(0);
    const T *Ar = A.A + (long long)i * r;
    for (int j = lane; j < r; j += 64) s += Ar[j] * q1s[j];
    if (r2 > 0) {
      const T *Hr = A.H + (long long)i * r2;
      for (int j = lane; j < r2; j += 64) s += Hr[j] * k2[j];
    }
    if (A.B) {
      const T *Br = A.B + (long long)i * rs;
      for (int j = lane; j < rs; j += 64) s += Br[j] * sh[j];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) qdd1s[i] = s + (A.c ? A.c[i] : T(0));
  }
  __syncthreads();

  // 5. velocity, convergence sums, state
  double acc_abs = 0.0, acc_den = 0.0;
  for (int i = tid; i < r; i += bs) {
    const T qn = q1s[i], an = qdd1s[i];
    const T vn = qd0[i] + A.half_dt * (qdd0[i] + an);
    double d;
    if (n_iter >= 2)
      d = ((double)qn - (double)q1[i]) + (double)A.dt * ((double)vn - (double)qd1[i]);
    else
      d = ((double)qn - (double)q0[i]) + (double)A.dt * ((double)vn - (double)qd0[i]);
    acc_abs += d * d;
    const double e = (double)qn + (double)A.dt * (double)vn;
    acc_den += e * e;
    q1[i] = qn;
    qd1[i] = vn;
    qdd1[i] = an;
  }
  acc_abs = wave_sum_d(acc_abs);
  acc_den = wave_sum_d(acc_den);
  __syncthreads();
  if (lane == 0) {
    red[0][wid] = acc_abs;
    red[1][wid] = acc_den;
  }

  // 6. push the lifted displacement of the next step, (Pi Phi)(q + dt q' + dt^2/2 q''),
  //    into the FOM neighbours' faces (role of step k+1)
  if (A.nexp > 0) {
    __syncthreads();
    for (int i = tid; i < r; i += bs) qdd1s[i] = q1s[i] + A.dt * qd1[i] + A.half_dt2 * qdd1[i];
    __syncthreads();
    const int role = (int)((step + 2) % 3);
    for (int e = 0; e < A.nexp; ++e) {
      const RomExport<T> &ex = A.ex[e];
      const int n = 3 * ex.npl;
      T *dst = ex.role[role] + (long long)b * ex.is;
      for (int m = tid; m < n; m += bs) {
        T s = T(0);
        for (int k = 0; k < r; ++k) s += ex.piphi[(long long)k * n + m] * qdd1s[k];
        const int c = m / ex.npl, nid = m - c * ex.npl;
        dst[c * ex.cs + nid] = s;
      }
    }
  }
  // 7. record q at the recorded steps
  if (A.rec_q && A.rec_every > 0 && ((step + 1) % A.rec_every) == 0) {
    const long long col = (step + 1) / A.rec_every;
    if (col < A.rec_ncols)
      for (int i = tid; i < r; i += bs) A.rec_q[((long long)b * A.rec_ncols + col) * r + i] = q1s[i];
  }
  __syncthreads();
  if (tid == 0) {
    double ta = 0.0, td = 0.0;
    for (int i = 0; i < nw; ++i) {
      ta += red[0][i];
      td += red[1][i];
    }
    stp->sd_abs2[A.sd] = ta;
    stp->sd_den2[A.sd] = td;
    decide(*stp, A.sd, A.opts);
    __threadfence();
  }
}

template <typename T>
size_t rom_smem_bytes(int r, int rs, int r2) {
  return sizeof(T) * (size_t)(2 * r + (rs > 0 ? rs : 1) + (r2 > 0 ? r2 : 0));
}

template <typename T>
hipError_t launch_rom(const RomArgs<T> &A, int batch, hipStream_t s) {
  const size_t smem = rom_smem_bytes<T>(A.r, A.rs, A.r2);
  if (smem > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rom_kernel<T>, dim3(batch), dim3(1024), smem, s, A);
  return hipGetLastError();
}
template hipError_t launch_rom<float>(const RomArgs<float> &, int, hipStream_t);
template hipError_t launch_rom<double>(const RomArgs<double> &, int, hipStream_t);
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
